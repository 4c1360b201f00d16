"""FP64 CPU oracle for the FIM black-oil step.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py.  The product path never imports this package.
"""
