"""torch.autograd binding of the discrete adjoint (fim_adjoint_gradient).

`MismatchObjective(res, dt, q_obs)` is a callable taking the per-cell
log-permeability theta (a float64 CUDA tensor of ncells values) and
returning the production mismatch

    J(theta) = sum over the schedule steps s and the producers w of
               (q_o,w(x_s) - q_obs[s, w])^2

of a forward run from the reservoir's initial state, as a 0-d tensor whose
backward pass is the library's discrete adjoint: dJ/dtheta with theta_c =
ln k_c and the three permeabilities of cell c scaled together (kx = ky =
exp(theta), kz = exp(theta) * kz/kx of the reservoir).  The paper computes no
gradient; what is differentiated is the discrete backward-Euler system of
eqs. (1)-(2) with the fluxes and wells of Sec. 3.2.3-3.2.4 that the forward
steps solve.

Argument marshalling only: the permeabilities go to the library as device
tensors (fim_set_perm_dev), the forward run, the backward sweep and the
gradient are the library's kernels; the backward pass multiplies the
library's gradient by the incoming scalar, as the chain rule asks.
"""
from __future__ import annotations

import numpy as np

from . import fim, reservoirs as rv


class _Mismatch:
    """torch.autograd.Function subclass, built on first use (torch is
    imported lazily, like the rest of the binding)."""
    cls = None

    @classmethod
    def get(cls):
        if cls.cls is None:
            import torch

            class FimMismatch(torch.autograd.Function):
                @staticmethod
                def forward(ctx, theta, obj):
                    J, grad = obj._run(theta)
                    ctx.save_for_backward(grad)
                    return J

                @staticmethod
                def backward(ctx, gJ):
                    (grad,) = ctx.saved_tensors
                    return gJ * grad, None

            cls.cls = FimMismatch
        return cls.cls


class MismatchObjective:
    """J(theta) of a reservoir, a schedule dt[nsteps] (days) and observed
    producer oil rates q_obs[nsteps, nwells] (stb/d; entries of injectors are
    ignored), differentiable through torch.autograd.  checkpoint_every = k
    >= 1 keeps the state of every k-th schedule step during the forward run
    and recomputes segments in the backward sweep (0 keeps every sub-step).
    The last call's fim_adjoint_report is kept in `.report`."""

    def __init__(self, res: rv.Reservoir, dt, q_obs, options: rv.Options | None = None,
                 checkpoint_every: int = 5):
        import torch

        self.res = res
        self.dt = np.atleast_1d(np.asarray(dt, np.float64))
        self.q_obs = np.asarray(q_obs, np.float64).reshape(len(self.dt), len(res.wells))
        self.every = int(checkpoint_every)
        self.fim = fim.Fim(res, options=options)
        d = torch.device("cuda", self.fim.device)
        self.kv_ratio = torch.from_numpy(np.asarray(res.kz, np.float64) /
                                         np.asarray(res.kx, np.float64)).to(d)
        self.report = None

    def theta0(self):
        """ln k of the reservoir itself, as a CUDA tensor."""
        import torch

        return torch.from_numpy(np.log(np.asarray(self.res.kx, np.float64))).to(
            self.kv_ratio.device)

    def __call__(self, theta):
        return _Mismatch.get().apply(theta, self)

    def _run(self, theta):
        import torch

        fim._tensor_shape(theta, torch.float64, self.fim.n, "theta")
        fim._tensor_device(theta, "theta", self.fim.device)
        with torch.no_grad():
            kh = torch.exp(theta.detach()).contiguous()
            kz = (kh * self.kv_ratio).contiguous()
            torch.cuda.current_stream(theta.device).synchronize()
            self.fim.fim_set_perm_dev(kh, kh, kz)
            self.fim.set_initial_state()
            rc, grad, rep = self.fim.fim_adjoint_gradient(self.dt, self.q_obs, self.every)
        self.report = rep
        if rc != fim.FIM_OK:
            raise fim.FimError(f"fim_adjoint_gradient returned {rc}: "
                               f"{fim.lib().fim_last_error().decode()}")
        J = torch.tensor(rep.objective, dtype=torch.float64, device=theta.device)
        return J, torch.from_numpy(grad).to(theta.device)
