"""MI355X-native FIM black-oil hot path (paper arXiv 2406.10862, OpenCAEPoro).

The compute path lives in the HIP library ``libfim.so`` (see ``include/fim.h``);
``paper_2406_10862_amd.fim`` is its thin ctypes binding.  Importing the package
itself loads nothing, so the seeded input generators in ``reservoirs`` can be
used without a GPU.
"""
__all__ = ["reservoirs", "fim"]
