"""Discrete adjoint of the oracle's backward-Euler system: test
infrastructure, used only by tests/.

The paper computes no gradient.  What is differentiated here is the discrete
system the oracle solves: the backward-Euler residual of eqs. (1)-(2) with
the two-point fluxes and the Peaceman wells of Sec. 3.2.3-3.2.4,

    R_m(x_m, x_{m-1}; theta) = (A(x_m) - A(x_{m-1})) / dt_m + sum_faces F + sum_perf q,

for every accepted sub-step m, with theta_c = ln k_c (kx, ky and kz of cell c
scaled together; porosity fixed).  The objective is the production mismatch

    J = sum over schedule-step ends s, producers w of (q_o,w(x_s) - q_obs[s, w])^2.

With the Lagrangian J + sum_m lam_m^T R_m, stationarity in x_m gives

    J_m^T lam_m = -(dJ/dx_m)^T + (1/dt_{m+1}) (dA(x_m)/dx_m)^T lam_{m+1}

(J_m = dR_m/dx_m; no second term for the last sub-step, no first one away
from schedule-step ends), and dJ/dtheta = sum_m lam_m^T dR_m/dtheta + the
explicit dJ/dtheta of the well indices.  The theta dependence is written out
from the definitions: T_f = 0.001127 A / (h_K/k_K + h_L/k_L), so
dT_f/dtheta_K = T_f (h_K/k_K) / (h_K/k_K + h_L/k_L); a Peaceman WI scales with
sqrt(kx ky), so dWI/dtheta = WI (an explicit WI does not depend on k).  The
transposed systems are solved directly (scipy sparse LU).

Parity of this module is pinned by central differences of J itself
(tests/test_oracle_adjoint.py).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.fimref import OracleModel, prop_index

PROD, INJ_WATER, INJ_GAS = 0, 1, 2
RATE = 1


def _interior_faces(res):
    """Every interior face as (K, L, r_K, r_L) index/half-resistance arrays
    per axis (K < L neighbours along the axis, r = half-length / k)."""
    nx, ny, nz = res.nx, res.ny, res.nz
    c = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    i = c % nx
    j = (c // nx) % ny
    k = c // (nx * ny)
    out = []
    for axis, (perm, d, idx) in enumerate([(res.kx, res.dx, i), (res.ky, res.dy, j),
                                           (res.kz, res.dz, k)]):
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[2 - axis] = slice(None, -1)
        sl_hi[2 - axis] = slice(1, None)
        K = c[tuple(sl_lo)].ravel()
        L = c[tuple(sl_hi)].ravel()
        rK = 0.5 * np.asarray(d)[idx[tuple(sl_lo)].ravel()] / np.asarray(perm)[K]
        rL = 0.5 * np.asarray(d)[idx[tuple(sl_hi)].ravel()] / np.asarray(perm)[L]
        out.append((axis, K, L, rK, rL))
    return out


class AdjointOracle:
    """Forward run with every accepted sub-step state, then the backward sweep."""

    def __init__(self, res, opt_over=None):
        self.res = res
        self.o = OracleModel(res)
        self.nb = self.o.nb
        self.n = self.o.n
        self.nw = self.o.nw
        self.ix = prop_index(self.nb)
        self.st = self.o.static()
        self.faces = _interior_faces(res)
        self.opt = self.o.options(**(opt_over or {}))
        cells, wells, wi_dk = [], [], []
        for w, wl in enumerate(res.wells):
            cells += list(wl.cells)
            wells += [w] * len(wl.cells)
            wi_dk += [0.0 if wl.wi is not None else 1.0] * len(wl.cells)
        self.pcell = np.asarray(cells, int)
        self.pwell = np.asarray(wells, int)
        self.wi_dk = np.asarray(wi_dk)
        self.wi = self.st["wi"]

    # -- forward ----------------------------------------------------------------
    def forward(self, dts):
        """States after every accepted sub-step (index 0: the start), the
        sub-step lengths and, per state, the schedule step it ends (or -1)."""
        o = self.o
        states, hsub, send = [o.state()], [], [-1]
        for s, dt in enumerate(dts):
            start = o.state()
            st, rep = o.step(dt, self.opt)
            if st != 0:
                raise RuntimeError(f"oracle forward step {s} failed")
            subs = list(rep.dt_sub[: rep.nsub])
            o.set_state(**start)
            for h in subs:
                st, rep = o.step(h, self.opt)
                if st != 0 or rep.nsub != 1:
                    raise RuntimeError(f"oracle replay of sub-step {h} failed")
                states.append(o.state())
                hsub.append(h)
                send.append(-1)
            send[-1] = s
        return states, hsub, send

    # -- pieces ---------------------------------------------------------------------
    def _rec(self, x):
        return self.o.props(**x)

    def _perf_rates(self, x, rec):
        """Per perforation: the component rates q[p, i] (production positive)."""
        nb, ix = self.nb, self.ix
        P, pb = x["P"], x["pbhp"]
        q = np.zeros((len(self.pcell), nb))
        for p, (c, w) in enumerate(zip(self.pcell, self.pwell)):
            wl = self.res.wells[w]
            # flow out of the cell (a producer, or an injector perforation
            # below its cell's pressure) carries the cell's phases
            if wl.kind == PROD or pb[w] < P[c]:
                d = P[c] - pb[w]
                lam = [rec[ix[f"Lam_{ph}"], c] for ph in "wog"[:nb]]
                if nb == 3:
                    lam[2] += rec[ix["Lam_og"], c]
                q[p] = self.wi[p] * np.asarray(lam) * d
            else:
                i = 0 if wl.kind == INJ_WATER else 2
                if i < nb:
                    b = rec[ix[f"b_{'wog'[i]}"], c]
                    q[p, i] = -self.wi[p] * rec[ix["lam_t"], c] * b * (pb[w] - P[c])
        return q

    def _face_fluxes(self, x, rec, axis, K, L):
        """F[f, i] from K to L across the faces of one axis."""
        nb, ix = self.nb, self.ix
        T = self.st[("tx", "ty", "tz")[axis]][K]
        z = self.st["depth"]
        P = x["P"]
        F = np.zeros((len(K), nb))
        up_o = None
        for j, ph in enumerate("wog"[:nb]):
            gam = rec[ix[f"gam_{ph}"]]
            dphi = (P[K] - P[L]) - 0.5 * (gam[K] + gam[L]) * (z[K] - z[L])
            up = dphi >= 0.0
            lam = rec[ix[f"Lam_{ph}"]]
            F[:, j] = T * np.where(up, lam[K], lam[L]) * dphi
            if ph == "o":
                up_o, dphi_o = up, dphi
        if nb == 3:
            lam_og = rec[ix["Lam_og"]]
            F[:, 2] += T * np.where(up_o, lam_og[K], lam_og[L]) * dphi_o
        return F

    def dR_dtheta_T(self, x, lam, rec=None):
        """g[c] = lam^T dR/dtheta_c at state x (lam over all block rows)."""
        nb, n = self.nb, self.n
        rec = self._rec(x) if rec is None else rec
        lam = np.asarray(lam).reshape(-1, nb)
        g = np.zeros(n)
        for axis, K, L, rK, rL in self.faces:
            F = self._face_fluxes(x, rec, axis, K, L)
            d = np.einsum("fi,fi->f", lam[K] - lam[L], F)     # R_K += F, R_L -= F
            np.add.at(g, K, d * rK / (rK + rL))
            np.add.at(g, L, d * rL / (rK + rL))
        q = self._perf_rates(x, rec)
        for p, (c, w) in enumerate(zip(self.pcell, self.pwell)):
            wl = self.res.wells[w]
            t = lam[c] @ q[p]
            i = 2 if wl.kind == INJ_GAS else 0
            if wl.control == RATE and i < nb:
                t -= lam[n + w, 0] * q[p, i]              # R_w = -sum_p q_i - target
            g[c] += t * self.wi_dk[p]
        return g

    def objective_terms(self, x, qobs_row, rec=None):
        """J_s, dJ/dx (all block rows) and the explicit dJ/dtheta at state x."""
        nb, n, ix = self.nb, self.n, self.ix
        rec = self._rec(x) if rec is None else rec
        P, pb = x["P"], x["pbhp"]
        q = self._perf_rates(x, rec)
        Js = 0.0
        dJdx = np.zeros((n + self.nw, nb))
        dJdth = np.zeros(n)
        unk = ["P", "Sw", "X"][:nb]
        for w, wl in enumerate(self.res.wells):
            if wl.kind != PROD:
                continue
            ps = np.nonzero(self.pwell == w)[0]
            r = q[ps, 1].sum() - qobs_row[w]
            Js += r * r
            for p in ps:
                c = self.pcell[p]
                d = P[c] - pb[w]
                lam_o = rec[ix["Lam_o"], c]
                for u, name in enumerate(unk):
                    dl = rec[ix[f"dLam_o_d{name}"], c]
                    dJdx[c, u] += 2 * r * self.wi[p] * (dl * d + (lam_o if u == 0 else 0.0))
                dJdx[n + w, 0] += 2 * r * (-self.wi[p] * lam_o)
                dJdth[c] += 2 * r * q[p, 1] * self.wi_dk[p]
        return Js, dJdx.ravel(), dJdth

    def dA_dx_T(self, x, lam, rec=None):
        """(dA/dx)^T lam on the cell rows (zero on the well rows)."""
        nb, n, ix = self.nb, self.n, self.ix
        rec = self._rec(x) if rec is None else rec
        lam = np.asarray(lam).reshape(-1, nb)
        out = np.zeros((n + self.nw, nb))
        unk = ["P", "Sw", "X"][:nb]
        for i, ph in enumerate("wog"[:nb]):
            for u, name in enumerate(unk):
                out[:n, u] += rec[ix[f"dA_{ph}_d{name}"]] * lam[:n, i]
        return out.ravel()

    def jacobian(self, dt, x, xold):
        Aold = self.o.accum(**xold)
        R, val = self.o.assemble(dt, Aold, jacobian=True, **x)
        rowptr, colind = self.o.pattern()
        nb = self.nb
        J = sp.bsr_matrix((val.reshape(-1, nb, nb), colind, rowptr),
                          shape=(len(R), len(R)))
        return J

    # -- the gradient ---------------------------------------------------------------
    def gradient(self, dts, qobs):
        """(J, dJ/dtheta[n]) for the steps dts and observations qobs[s, w]."""
        qobs = np.asarray(qobs, float).reshape(len(dts), self.nw)
        states, hsub, send = self.forward(dts)
        M = len(hsub)
        grad = np.zeros(self.n)
        Jtot = 0.0
        lam_next = None
        for m in range(M, 0, -1):
            x, xold = states[m], states[m - 1]
            rec = self._rec(x)
            rhs = np.zeros((self.n + self.nw) * self.nb)
            if lam_next is not None:
                rhs += self.dA_dx_T(x, lam_next, rec) / hsub[m]
            s = send[m]
            if s >= 0:
                Js, dJdx, dJdth = self.objective_terms(x, qobs[s], rec)
                Jtot += Js
                rhs -= dJdx
                grad += dJdth
            Jm = self.jacobian(hsub[m - 1], x, xold)
            lam = spla.spsolve(Jm.T.tocsc(), rhs)
            grad += self.dR_dtheta_T(x, lam, rec)
            lam_next = lam
        return Jtot, grad

    def objective(self, dts, qobs):
        """J alone (a forward run): the quantity the gradient differentiates."""
        qobs = np.asarray(qobs, float).reshape(len(dts), self.nw)
        states, hsub, send = self.forward(dts)
        Jtot = 0.0
        for m in range(1, len(states)):
            if send[m] >= 0:
                Jtot += self.objective_terms(states[m], qobs[send[m]])[0]
        return Jtot
