// fim_phys.hip - cell, face and well kernels of the FIM black-oil step.
//
// Paper anchors: Sec. 2.1 eqs. (1)-(2) and the constraints below them
// (component conservation, Darcy flux with gravity, N_i = phi sum S_j xi_j
// x_ij, sum S_j = 1, black-oil closure); Secs. 3.2.3-3.2.4 (Bulk PVT/SAT/ROCK/ACCU,
// BulkConn, AllWells); Sec. 3.2.5 (one Newton iteration: assemble, solve
// and update, update properties, check convergence).
//
// All kernels are bound by HBM traffic: one thread owns one cell, state and
// property arrays are structure-of-arrays so a wave touches contiguous
// memory, and the PVT table is staged in LDS for the interval searches.
#include <math.h>

#include "fim_internal.h"
#include "fim_reduce.h"

namespace fim {

constexpr double kDarcy = 0.001127;     // mD*ft^2/(ft*cP) * psi -> rb/day
constexpr double kBbl = 5.615;          // ft3 per bbl
constexpr double kPsiFt = 144.0;        // (lb/ft3)*ft -> psi

// ---------------------------------------------------------------------------
// static precompute: volumes, centre depths, pore volumes, TPFA transmissibilities

__device__ inline double harmonic_T(double k1, double h1, double k2, double h2, double area) {
    // conductances k*A/h of the two half cells in series
    double g1 = k1 * area / h1, g2 = k2 * area / h2;
    if (!(g1 > 0.0) || !(g2 > 0.0)) return 0.0;
    return kDarcy * (g1 * g2) / (g1 + g2);
}

__global__ __launch_bounds__(kBlock) void k_static(Grid g, const double *dx, const double *dy,
                                                   const double *dz, double top,
                                                   const double *kx, const double *ky,
                                                   const double *kz, const double *poro,
                                                   double *vol, double *depth, double *pvref,
                                                   double *tx, double *ty, double *tz) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.n) return;
    int i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    double above = 0.0;
    for (int kk = 0; kk < k; ++kk) above += dz[kk];
    double v = dx[i] * dy[j] * dz[k];
    vol[c] = v;
    depth[c] = top + above + 0.5 * dz[k];
    pvref[c] = v * poro[c] / kBbl;
    int nxy = g.nx * g.ny;
    tx[c] = (i + 1 < g.nx)
                ? harmonic_T(kx[c], 0.5 * dx[i], kx[c + 1], 0.5 * dx[i + 1], dy[j] * dz[k])
                : 0.0;
    ty[c] = (j + 1 < g.ny) ? harmonic_T(ky[c], 0.5 * dy[j], ky[c + g.nx], 0.5 * dy[j + 1],
                                        dx[i] * dz[k])
                           : 0.0;
    tz[c] = (k + 1 < g.nz)
                ? harmonic_T(kz[c], 0.5 * dz[k], kz[c + nxy], 0.5 * dz[k + 1], dx[i] * dy[j])
                : 0.0;
}

// Peaceman well index with the anisotropic equivalent radius
__global__ void k_peaceman(Grid g, int nperf, const int *pcell, const int *pwell,
                           const double *dx, const double *dy, const double *dz,
                           const double *kx, const double *ky, const double *rw,
                           const double *skin, double *wi) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nperf || wi[p] > 0.0) return;
    int c = pcell[p], w = pwell[p];
    int i = c % g.nx, j = (c / g.nx) % g.ny, k = c / (g.nx * g.ny);
    double a = ky[c] / kx[c];                          // anisotropy ratio
    double num = sqrt(sqrt(a) * dx[i] * dx[i] + sqrt(1.0 / a) * dy[j] * dy[j]);
    double ro = 0.28 * num / (pow(a, 0.25) + pow(1.0 / a, 0.25));
    wi[p] = 2.0 * M_PI * kDarcy * sqrt(kx[c] * ky[c]) * dz[k] / (log(ro / rw[w]) + skin[w]);
}

// ---------------------------------------------------------------------------
// per-cell black-oil properties with derivatives

struct TabL {                       // PVT columns in LDS
    const double *p, *bo, *rs, *muo, *bg, *mug;
    int n;
};

__device__ inline void stage_table(const Phys &f, double *sm, TabL &t) {
    for (int e = threadIdx.x; e < 6 * f.nrows; e += blockDim.x) sm[e] = f.tab[e];
    t.n = f.nrows;
    t.p = sm;
    t.bo = sm + f.nrows;
    t.rs = sm + 2 * f.nrows;
    t.muo = sm + 3 * f.nrows;
    t.bg = sm + 4 * f.nrows;
    t.mug = sm + 5 * f.nrows;
    __syncthreads();
}

// largest i in [0, n-2] with t[i] <= v (0 when v is below the table)
__device__ inline int interval(const double *t, int n, double v) {
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (t[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline double lin(const double *t, const double *y, int i, double v, double &slope) {
    slope = (y[i + 1] - y[i]) / (t[i + 1] - t[i]);
    return y[i] + slope * (v - t[i]);
}

__device__ inline void corey(double num, double den, double kmax, double ex, double &kr,
                             double &dkr) {
    double s = num / den;
    if (s <= 0.0) {
        kr = 0.0;
        dkr = 0.0;
    } else if (s >= 1.0) {
        kr = kmax;
        dkr = 0.0;
    } else {
        double sp = pow(s, ex - 1.0);
        kr = kmax * sp * s;
        dkr = kmax * ex * sp / den;
    }
}

__device__ inline double rs_sat(const TabL &t, double P) {
    double s;
    return lin(t.p, t.rs, interval(t.p, t.n, P), P, s);
}

template <int NB>
__device__ void cell_props(const Phys &f, const TabL &t, double pvref, double P, double Sw,
                           double X, int flag, double (&r)[Rec<NB>::NREC]) {
    using RI = Rec<NB>;
    constexpr int G = RI::G;
#pragma unroll
    for (int q = 0; q < RI::NREC; ++q) r[q] = 0.0;

    const double bw = exp(f.cw * (P - f.pw_ref)) / f.bw_ref;
    const double dbw = f.cw * bw;
    double Rs = 0, dRsP = 0, dRsX = 0, Bo, dBoP, dBoX = 0, muo, dmuoP, dmuoX = 0;
    double Sg = 0, dSgX = 0, Bg = 1, dBgP = 0, mug = 1, dmugP = 0;
    const int ip = interval(t.p, t.n, P);
    if constexpr (NB == 2) {
        Bo = lin(t.p, t.bo, ip, P, dBoP);
        muo = lin(t.p, t.muo, ip, P, dmuoP);
    } else {
        Bg = lin(t.p, t.bg, ip, P, dBgP);
        mug = lin(t.p, t.mug, ip, P, dmugP);
        if (flag == kSat) {
            Rs = lin(t.p, t.rs, ip, P, dRsP);
            Bo = lin(t.p, t.bo, ip, P, dBoP);
            muo = lin(t.p, t.muo, ip, P, dmuoP);
            Sg = X;
            dSgX = 1.0;
        } else {
            // undersaturated: bubble point on the Rs column, saturated data at
            // Pb on the same interval, linear extension in P - Pb
            Rs = X;
            dRsX = 1.0;
            const int ir = interval(t.rs, t.n, Rs);
            const double dPb = (t.p[ir + 1] - t.p[ir]) / (t.rs[ir + 1] - t.rs[ir]);
            const double Pb = t.p[ir] + (Rs - t.rs[ir]) * dPb;
            double sB, sM;
            const double Bb = lin(t.p, t.bo, ir, Pb, sB);
            const double Mb = lin(t.p, t.muo, ir, Pb, sM);
            const double d = P - Pb;
            Bo = Bb * (1.0 - f.co_us * d);
            dBoP = -Bb * f.co_us;
            dBoX = (sB * (1.0 - f.co_us * d) + Bb * f.co_us) * dPb;
            muo = Mb * (1.0 + f.cmu_us * d);
            dmuoP = Mb * f.cmu_us;
            dmuoX = (sM * (1.0 + f.cmu_us * d) - Mb * f.cmu_us) * dPb;
        }
    }
    const double bo = 1.0 / Bo, dboP = -dBoP * bo * bo, dboX = -dBoX * bo * bo;
    const double bg = 1.0 / Bg, dbgP = -dBgP * bg * bg;

    // gravity gradients rho_j / 144
    const double mo = kBbl * f.rho_o + Rs * f.rho_g;        // lb per stb of oil + gas
    r[RI::GAM + 0 * G + 0] = f.rho_w * bw / kPsiFt;
    r[RI::GAM + 0 * G + 1] = f.rho_w * dbw / kPsiFt;
    r[RI::GAM + 1 * G + 0] = mo * bo / (kBbl * kPsiFt);
    r[RI::GAM + 1 * G + 1] = (dRsP * f.rho_g * bo + mo * dboP) / (kBbl * kPsiFt);
    if constexpr (NB == 3) {
        r[RI::GAM + 1 * G + 3] = (dRsX * f.rho_g * bo + mo * dboX) / (kBbl * kPsiFt);
        r[RI::GAM + 2 * G + 0] = f.rho_g * bg / (kBbl * kPsiFt);
        r[RI::GAM + 2 * G + 1] = f.rho_g * dbgP / (kBbl * kPsiFt);
    }

    // relative permeabilities
    const double So = 1.0 - Sw - Sg;
    const double Dgo = 1.0 - f.swc - f.sor - (NB == 3 ? f.sgc : 0.0);
    double krw, dkrw, kro, dkro, krg = 0, dkrg = 0;
    corey(Sw - f.swc, 1.0 - f.swc - f.sor, f.krw_max, f.nw, krw, dkrw);
    corey(So - f.sor, Dgo, f.kro_max, f.no, kro, dkro);
    if constexpr (NB == 3) corey(Sg - f.sgc, Dgo, f.krg_max, f.ng, krg, dkrg);
    const double dkroSw = -dkro, dkroX = -dkro * dSgX, dkrgX = dkrg * dSgX;

    // Lam_j = kr_j b_j / mu_j
    r[RI::LAM + 0] = krw * bw / f.muw;
    r[RI::LAM + 1] = krw * dbw / f.muw;
    r[RI::LAM + 2] = dkrw * bw / f.muw;
    const double bmo = bo / muo;
    const double dbmoP = (dboP - bmo * dmuoP) / muo;
    const double dbmoX = (dboX - bmo * dmuoX) / muo;
    const double lo = kro * bmo;
    r[RI::LAM + G + 0] = lo;
    r[RI::LAM + G + 1] = kro * dbmoP;
    r[RI::LAM + G + 2] = dkroSw * bmo;
    if constexpr (NB == 3) {
        const double dloX = dkroX * bmo + kro * dbmoX;
        r[RI::LAM + G + 3] = dloX;
        const double bmg = bg / mug;
        r[RI::LAM + 2 * G + 0] = krg * bmg;
        r[RI::LAM + 2 * G + 1] = krg * (dbgP - bmg * dmugP) / mug;
        r[RI::LAM + 2 * G + 3] = dkrgX * bmg;
        r[RI::LAMOG + 0] = Rs * lo;
        r[RI::LAMOG + 1] = dRsP * lo + Rs * r[RI::LAM + G + 1];
        r[RI::LAMOG + 2] = Rs * r[RI::LAM + G + 2];
        r[RI::LAMOG + 3] = dRsX * lo + Rs * dloX;
    }
    // total mobility sum_j kr_j / mu_j
    r[RI::LT + 0] = krw / f.muw + kro / muo + (NB == 3 ? krg / mug : 0.0);
    r[RI::LT + 1] = -kro * dmuoP / (muo * muo) - (NB == 3 ? krg * dmugP / (mug * mug) : 0.0);
    r[RI::LT + 2] = dkrw / f.muw + dkroSw / muo;
    if constexpr (NB == 3) r[RI::LT + 3] = dkroX / muo - kro * dmuoX / (muo * muo) + dkrgX / mug;

    // pore volume and accumulation N_i = PV sum_j S_j b_j x_ij
    const double pv = pvref * (1.0 + f.cr * (P - f.pref));
    const double dpv = pvref * f.cr;
    r[RI::PV] = pv;
    r[RI::B + 0] = bw;
    r[RI::B + 1] = bo;
    r[RI::DBP + 0] = dbw;
    r[RI::DBP + 1] = dboP;
    r[RI::ACC + 0] = pv * bw * Sw;
    r[RI::ACC + 1] = (dpv * bw + pv * dbw) * Sw;
    r[RI::ACC + 2] = pv * bw;
    r[RI::ACC + G + 0] = pv * bo * So;
    r[RI::ACC + G + 1] = (dpv * bo + pv * dboP) * So;
    r[RI::ACC + G + 2] = -pv * bo;
    if constexpr (NB == 3) {
        r[RI::B + 2] = bg;
        r[RI::DBP + 2] = dbgP;
        r[RI::ACC + G + 3] = pv * (dboX * So - bo * dSgX);
        const double gas = bg * Sg + Rs * bo * So;
        const double gP = dbgP * Sg + (dRsP * bo + Rs * dboP) * So;
        const double gX = bg * dSgX + (dRsX * bo + Rs * dboX) * So - Rs * bo * dSgX;
        r[RI::ACC + 2 * G + 0] = pv * gas;
        r[RI::ACC + 2 * G + 1] = dpv * gas + pv * gP;
        r[RI::ACC + 2 * G + 2] = -pv * Rs * bo;
        r[RI::ACC + 2 * G + 3] = pv * gX;
    }
}

template <int NB>
__device__ __forceinline__ void props_body(int bid, const Phys &f, int n,
                                           const double *__restrict__ pvref,
                                           const double *__restrict__ P,
                                           const double *__restrict__ Sw,
                                           const double *__restrict__ X,
                                           const int8_t *__restrict__ flag,
                                           double *__restrict__ rec, double *__restrict__ aold) {
    __shared__ double sm[6 * kMaxTableRows];
    TabL t;
    stage_table(f, sm, t);
    const int c = bid * blockDim.x + threadIdx.x;
    if (c >= n) return;
    using RI = Rec<NB>;
    double r[RI::NREC];
    cell_props<NB>(f, t, pvref[c], P[c], Sw[c], NB == 3 ? X[c] : 0.0, NB == 3 ? flag[c] : 0, r);
#pragma unroll
    for (int q = 0; q < RI::NREC; ++q) rec[(size_t)q * n + c] = r[q];
    if (aold)
#pragma unroll
        for (int i = 0; i < NB; ++i) aold[(size_t)i * n + c] = r[RI::ACC + i * RI::G];
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_props(Phys f, int n, const double *__restrict__ pvref,
                                                  const double *__restrict__ P,
                                                  const double *__restrict__ Sw,
                                                  const double *__restrict__ X,
                                                  const int8_t *__restrict__ flag,
                                                  double *__restrict__ rec,
                                                  double *__restrict__ aold) {
    props_body<NB>(blockIdx.x, f, n, pvref, P, Sw, X, flag, rec, aold);
}

// ---------------------------------------------------------------------------
// face fluxes and cell-centric assembly

template <int NB>
struct Side {                       // what a face needs from one cell
    double P, z;
    double lam[NB][NB + 1];
    double lamog[NB + 1];
    double gam[NB][NB + 1];
};

template <int NB>
__device__ inline void load_side(const double *__restrict__ rec, int n, int c,
                                 const double *__restrict__ P, const double *__restrict__ depth,
                                 Side<NB> &s) {
    using RI = Rec<NB>;
    s.P = P[c];
    s.z = depth[c];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int u = 0; u <= NB; ++u) {
            s.lam[j][u] = rec[(size_t)(RI::LAM + j * RI::G + u) * n + c];
            s.gam[j][u] = rec[(size_t)(RI::GAM + j * RI::G + u) * n + c];
        }
#pragma unroll
    for (int u = 0; u <= NB; ++u)
        s.lamog[u] = (NB == 3) ? rec[(size_t)(RI::LAMOG + u) * n + c] : 0.0;
}

// Flux of every component from K to L across a face of transmissibility T
// (phase-potential upstream weighting, arithmetic mean face density) and
// its derivatives w.r.t. the unknowns of K and of L.  Both cells of a face
// evaluate it with the same (K, L) order, so F_LK = -F_KL exactly.
template <int NB>
__device__ inline void face_flux(double T, const Side<NB> &K, const Side<NB> &L, double (&F)[NB],
                                 double (&dK)[NB][NB], double (&dL)[NB][NB]) {
    const double dz = K.z - L.z;
    double dphi[NB], gK[NB][NB], gL[NB][NB];
    bool up[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        dphi[j] = (K.P - L.P) - 0.5 * (K.gam[j][0] + L.gam[j][0]) * dz;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            gK[j][u] = (u == 0 ? 1.0 : 0.0) - 0.5 * K.gam[j][1 + u] * dz;
            gL[j][u] = (u == 0 ? -1.0 : 0.0) - 0.5 * L.gam[j][1 + u] * dz;
        }
        up[j] = dphi[j] >= 0.0;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const double c = up[i] ? K.lam[i][0] : L.lam[i][0];
        F[i] = T * c * dphi[i];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const double dcK = up[i] ? K.lam[i][1 + u] : 0.0;
            const double dcL = up[i] ? 0.0 : L.lam[i][1 + u];
            dK[i][u] = T * (dcK * dphi[i] + c * gK[i][u]);
            dL[i][u] = T * (dcL * dphi[i] + c * gL[i][u]);
        }
    }
    if constexpr (NB == 3) {        // gas dissolved in the oil phase
        const double c = up[1] ? K.lamog[0] : L.lamog[0];
        F[2] += T * c * dphi[1];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const double dcK = up[1] ? K.lamog[1 + u] : 0.0;
            const double dcL = up[1] ? 0.0 : L.lamog[1 + u];
            dK[2][u] += T * (dcK * dphi[1] + c * gK[1][u]);
            dL[2][u] += T * (dcL * dphi[1] + c * gL[1][u]);
        }
    }
}

template <int NB>
__device__ inline void store_block(double *__restrict__ val, int q, const double (&b)[NB][NB]) {
    double *dst = val + (size_t)q * NB * NB;
    if constexpr (NB == 2) {
        reinterpret_cast<double2 *>(dst)[0] = make_double2(b[0][0], b[0][1]);
        reinterpret_cast<double2 *>(dst)[1] = make_double2(b[1][0], b[1][1]);
    } else {
#pragma unroll
        for (int e = 0; e < NB; ++e)
#pragma unroll
            for (int u = 0; u < NB; ++u) dst[e * NB + u] = b[e][u];
    }
}

// Perforation rate of every component and its derivatives (production
// positive), weighted by the side the flow comes from: out of the cell
// (producers, and injector perforations whose cell pressure exceeds the
// BHP) WI*Lam_i*(P - Pbhp); into the cell, the injected pure water or free
// gas, -WI*lam_t*b_inj*(Pbhp - P).
template <int NB>
__device__ inline void perf_rate(int kind, double wi, double P, double pbhp,
                                 const double *__restrict__ rec, int n, int c, double (&q)[NB],
                                 double (&dq)[NB][NB], double (&dqb)[NB]) {
    using RI = Rec<NB>;
    auto R = [&](int k) { return rec[(size_t)k * n + c]; };
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        q[i] = 0.0;
        dqb[i] = 0.0;
#pragma unroll
        for (int u = 0; u < NB; ++u) dq[i][u] = 0.0;
    }
    if (kind == kProd || pbhp < P) {
        const double d = P - pbhp;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            double lam = R(RI::LAM + i * RI::G);
            if (NB == 3 && i == 2) lam += R(RI::LAMOG);
            q[i] = wi * lam * d;
            dqb[i] = -wi * lam;
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                double dl = R(RI::LAM + i * RI::G + 1 + u);
                if (NB == 3 && i == 2) dl += R(RI::LAMOG + 1 + u);
                dq[i][u] = wi * (dl * d + (u == 0 ? lam : 0.0));
            }
        }
    } else {
        const int i = (kind == kInjWater) ? 0 : 2;
        if (i >= NB) return;
        const double lt = R(RI::LT), b = R(RI::B + i), db = R(RI::DBP + i);
        const double d = pbhp - P;
        q[i] = -wi * lt * b * d;
        dqb[i] = -wi * lt * b;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const double dlt = R(RI::LT + 1 + u);
            dq[i][u] = -wi * ((dlt * b + (u == 0 ? lt * db : 0.0)) * d - (u == 0 ? lt * b : 0.0));
        }
    }
}

template <int NB>
__device__ __forceinline__ void assemble_cells_body(
    int bid, const Grid &g, const Wells &w, const Sys &sys, const double *__restrict__ depth,
    const double *__restrict__ tx, const double *__restrict__ ty, const double *__restrict__ tz,
    const double *__restrict__ P, const double *__restrict__ pbhp,
    const double *__restrict__ rec, const double *__restrict__ aold, double dt) {
    using RI = Rec<NB>;
    const int c = bid * blockDim.x + threadIdx.x;
    const int n = g.n;
    if (c >= n) return;
    const int nx = g.nx, nxy = g.nx * g.ny;
    const int i = c % nx, j = (c / nx) % g.ny, k = c / nxy;

    double R[NB], D[NB][NB];
    const double rdt = 1.0 / dt;
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        R[e] = (rec[(size_t)(RI::ACC + e * RI::G) * n + c] - aold[(size_t)e * n + c]) * rdt;
#pragma unroll
        for (int u = 0; u < NB; ++u) D[e][u] = rec[(size_t)(RI::ACC + e * RI::G + 1 + u) * n + c] * rdt;
    }
    Side<NB> me, nbr;
    load_side<NB>(rec, n, c, P, depth, me);
    const bool ex[6] = {k > 0, j > 0, i > 0, i + 1 < nx, j + 1 < g.ny, k + 1 < g.nz};
    const int q0 = sys.rowptr[c];
    const int qd = q0 + ex[0] + ex[1] + ex[2];
    int q = qd + 1 + ex[3] + ex[4] + ex[5];       // the first well column
    double F[NB], dK[NB][NB], dL[NB][NB], off[NB][NB];
    // 2x2 blocks: the off-diagonal blocks (-z, -y, -x, +x, +y, +z) are held
    // and stored with the diagonal one after the last face, so the row's
    // lines are written in one burst rather than piecemeal while the faces'
    // loads are in flight (3x3 blocks store each at once: held, they would
    // take the kernel to one wave per SIMD)
    constexpr bool kBurst = NB == 2;
    double OB[kBurst ? 6 : 1][NB][NB];
    int ql = q0, qu = qd + 1;
    auto put = [&](int d, int &qp) {
        if constexpr (kBurst) {
#pragma unroll
            for (int e = 0; e < NB; ++e)
#pragma unroll
                for (int u = 0; u < NB; ++u) OB[d][e][u] = off[e][u];
        } else {
            store_block<NB>(sys.val, qp++, off);
        }
    };

    // neighbour below in index order: it is the K side of the face
    auto lower = [&](int d, int cn, double T) {
        load_side<NB>(rec, n, cn, P, depth, nbr);
        face_flux<NB>(T, nbr, me, F, dK, dL);
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            R[e] -= F[e];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                D[e][u] -= dL[e][u];
                off[e][u] = -dK[e][u];
            }
        }
        put(d, ql);
    };
    // neighbour above in index order: this cell is the K side
    auto upper = [&](int d, int cn, double T) {
        load_side<NB>(rec, n, cn, P, depth, nbr);
        face_flux<NB>(T, me, nbr, F, dK, dL);
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            R[e] += F[e];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                D[e][u] += dK[e][u];
                off[e][u] = dL[e][u];
            }
        }
        put(d, qu);
    };
    if (ex[0]) lower(0, c - nxy, tz[c - nxy]);
    if (ex[1]) lower(1, c - nx, ty[c - nx]);
    if (ex[2]) lower(2, c - 1, tx[c - 1]);
    if (ex[3]) upper(3, c + 1, tx[c]);
    if (ex[4]) upper(4, c + nx, ty[c]);
    if (ex[5]) upper(5, c + nxy, tz[c]);

    // perforations of this cell, in ascending well order (well columns)
    for (int pp = w.cps[c]; pp < w.cps[c + 1]; ++pp) {
        const int p = w.cperf[pp];
        const int wl = w.pwell[p];
        double qr[NB], dq[NB][NB], dqb[NB];
        perf_rate<NB>(w.kind[wl], w.wi[p], me.P, pbhp[wl], rec, n, c, qr, dq, dqb);
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            R[e] += qr[e];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                D[e][u] += dq[e][u];
                off[e][u] = (u == 0) ? dqb[e] : 0.0;
            }
        }
        store_block<NB>(sys.val, q++, off);
    }
    if constexpr (kBurst) {
        int qs = q0;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (ex[d]) store_block<NB>(sys.val, qs++, OB[d]);
        store_block<NB>(sys.val, qs++, D);
#pragma unroll
        for (int d = 3; d < 6; ++d)
            if (ex[d]) store_block<NB>(sys.val, qs++, OB[d]);
    } else {
        store_block<NB>(sys.val, qd, D);
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) sys.R[(size_t)c * NB + e] = R[e];
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_assemble_cells(
    Grid g, Wells w, Sys sys, const double *__restrict__ depth, const double *__restrict__ tx,
    const double *__restrict__ ty, const double *__restrict__ tz, const double *__restrict__ P,
    const double *__restrict__ pbhp, const double *__restrict__ rec,
    const double *__restrict__ aold, double dt) {
    // each XCD takes one contiguous run of cells: the planes above and below a
    // cell, whose property records its faces read, are then read by blocks
    // of the same XCD around the same time and stay in that XCD's L2
    assemble_cells_body<NB>(xcd_block(blockIdx.x, gridDim.x), g, w, sys, depth, tx, ty, tz, P,
                            pbhp, rec, aold, dt);
}

// Well rows: one wave per well.  Rate rows sum the injected component over
// the perforations; BHP rows pin the bottom-hole pressure.  Slots >= 1 of a
// well row are identity rows.  wmeas[w] = |R_w| / |dR_w/dPbhp| (psi).
template <int NB>
__device__ __forceinline__ void assemble_wells_body(int wl, const Wells &w, const Sys &sys, int n,
                                                    const double *__restrict__ P,
                                                    const double *__restrict__ pbhp,
                                                    const double *__restrict__ rec,
                                                    double *__restrict__ wmeas) {
    const int lane = threadIdx.x;
    const int row = n + wl, base = sys.rowptr[row];
    const int p0 = w.wps[wl], np = w.wps[wl + 1] - p0;
    const bool rate = w.ctrl[wl] == kRate;
    const int kind = w.kind[wl];
    const int ii = (kind == kInjGas) ? 2 : 0;
    double s[2] = {0.0, 0.0};
    for (int p = lane; p < np; p += 64) {
        const int pid = p0 + p, c = w.pcell[pid];
        double blk[NB][NB];
#pragma unroll
        for (int e = 0; e < NB; ++e)
#pragma unroll
            for (int u = 0; u < NB; ++u) blk[e][u] = 0.0;
        if (rate && ii < NB) {
            double qr[NB], dq[NB][NB], dqb[NB];
            perf_rate<NB>(kind, w.wi[pid], P[c], pbhp[wl], rec, n, c, qr, dq, dqb);
            s[0] += qr[ii];
            s[1] += dqb[ii];
#pragma unroll
            for (int u = 0; u < NB; ++u) blk[0][u] = -dq[ii][u];
        }
        store_block<NB>(sys.val, base + p, blk);
    }
    const bool mx[2] = {false, false};
    wave_reduce<2>(s, mx);
    if (lane == 0) {
        double d[NB][NB];
#pragma unroll
        for (int e = 0; e < NB; ++e)
#pragma unroll
            for (int u = 0; u < NB; ++u) d[e][u] = (e == u && e > 0) ? 1.0 : 0.0;
        double r0;
        if (rate) {
            d[0][0] = -s[1];
            r0 = -s[0] - w.target[wl];
        } else {
            d[0][0] = 1.0;
            r0 = pbhp[wl] - w.target[wl];
        }
        store_block<NB>(sys.val, base + np, d);
        sys.R[(size_t)row * NB] = r0;
#pragma unroll
        for (int e = 1; e < NB; ++e) sys.R[(size_t)row * NB + e] = 0.0;
        wmeas[wl] = fabs(r0) / (d[0][0] != 0.0 ? fabs(d[0][0]) : 1.0);
    }
}

template <int NB>
__global__ __launch_bounds__(64) void k_assemble_wells(Wells w, Sys sys, int n,
                                                       const double *__restrict__ P,
                                                       const double *__restrict__ pbhp,
                                                       const double *__restrict__ rec,
                                                       double *__restrict__ wmeas) {
    assemble_wells_body<NB>(blockIdx.x, w, sys, n, P, pbhp, rec, wmeas);
}

// ---------------------------------------------------------------------------
// convergence measures: out = [max_c dt|R_ic|/(PV b_i)], [sum_c R_ic],
// [sum_c PV b_i], max well measure

template <int NB>
__device__ __forceinline__ void conv_body(int bid, int nblk, int n, int nw,
                                          const double *__restrict__ rec,
                                          const double *__restrict__ R,
                                          const double *__restrict__ wmeas, double dt,
                                          double *partials) {
    using RI = Rec<NB>;
    constexpr int K = 3 * NB + 1;
    double v[K];
    bool mx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = 0.0;
        mx[k] = (k < NB) || (k == 3 * NB);
    }
    for (int c = bid * blockDim.x + threadIdx.x; c < n; c += nblk * blockDim.x) {
        const double pv = rec[(size_t)RI::PV * n + c];
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const double r = R[(size_t)c * NB + e];
            const double scale = pv * rec[(size_t)(RI::B + e) * n + c];
            v[e] = rop(v[e], dt * fabs(r) / scale, true);
            v[NB + e] += r;
            v[2 * NB + e] += scale;
        }
    }
    if (bid == 0)
        for (int wl = threadIdx.x; wl < nw; wl += blockDim.x) v[3 * NB] = rop(v[3 * NB], wmeas[wl], true);
    block_partials<K>(v, mx, partials, bid, nblk);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_conv(int n, int nw, const double *__restrict__ rec,
                                                 const double *__restrict__ R,
                                                 const double *__restrict__ wmeas, double dt,
                                                 double *partials) {
    conv_body<NB>(blockIdx.x, gridDim.x, n, nw, rec, R, wmeas, dt, partials);
}

template <int NB>
__device__ __forceinline__ void conv_finish_body(int nparts, const double *partials, double *out) {
    constexpr int K = 3 * NB + 1;
    bool mx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) mx[k] = (k < NB) || (k == 3 * NB);
    double a[K];
    finish_partials<K>(nparts, mx, partials, a);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = a[k];
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_conv_finish(int nparts, const double *partials,
                                                        double *out) {
    conv_finish_body<NB>(nparts, partials, out);
}

// ---------------------------------------------------------------------------
// Newton update: delta = -y; per-cell saturation chop and pressure clip,
// three-phase variable switching; out = [max|dP| (cells and wells), max|dS|,
// largest distance of a saturation of the new iterate outside [0, 1]]

template <int NB>
__device__ __forceinline__ void newton_update_body(int bid, int nblk, const Phys &f, int n,
                                                   const double *__restrict__ y, double ds_max,
                                                   double dp_max, double *__restrict__ P,
                                                   double *__restrict__ Sw,
                                                   double *__restrict__ X,
                                                   int8_t *__restrict__ flag, double *partials) {
    __shared__ double sm[6 * kMaxTableRows];
    TabL t;
    stage_table(f, sm, t);
    double v[3] = {0.0, 0.0, 0.0};
    const bool mx[3] = {true, true, true};
    for (int c = bid * blockDim.x + threadIdx.x; c < n; c += nblk * blockDim.x) {
        double dP = -y[(size_t)c * NB];
        dP = fmin(fmax(dP, -dp_max), dp_max);
        double dS = -y[(size_t)c * NB + 1];
        double dX = (NB == 3) ? -y[(size_t)c * NB + 2] : 0.0;
        const bool sat = (NB == 3) && flag[c] == kSat;
        double m = fabs(dS);
        if (sat) m = fmax(m, fabs(dX));
        if (m > ds_max) {
            const double a = ds_max / m;
            dS *= a;
            if (sat) dX *= a;
        }
        const double p = P[c] + dP;
        const double sw = Sw[c] + dS;
        P[c] = p;
        Sw[c] = sw;
        v[0] = rop(v[0], fabs(dP), true);
        v[1] = rop(v[1], fabs(dS), true);
        double sg = 0.0;
        if constexpr (NB == 3) {
            if (sat) v[1] = rop(v[1], fabs(dX), true);
            const double x = X[c] + dX;
            if (sat && x < 0.0) {
                flag[c] = kUnsat;
                X[c] = rs_sat(t, p);
            } else if (!sat && x > rs_sat(t, p)) {
                flag[c] = kSat;
                X[c] = 0.0;
            } else {
                X[c] = x;
                if (sat) sg = x;
            }
        }
        // distance of the saturations (Sw, So, Sg) outside [0, 1]
        const double so = 1.0 - sw - sg;
        v[2] = rop(v[2], fmax(fmax(fmax(-sw, sw - 1.0), fmax(-so, so - 1.0)), fmax(-sg, sg - 1.0)),
                   true);
        if (dP != dP || dS != dS || dX != dX) v[0] = NAN;
    }
    block_partials<3>(v, mx, partials, bid, nblk);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_newton_update(Phys f, int n, int nw,
                                                          const double *__restrict__ y,
                                                          double ds_max, double dp_max,
                                                          double *__restrict__ P,
                                                          double *__restrict__ Sw,
                                                          double *__restrict__ X,
                                                          int8_t *__restrict__ flag,
                                                          double *partials) {
    (void)nw;
    newton_update_body<NB>(blockIdx.x, gridDim.x, f, n, y, ds_max, dp_max, P, Sw, X, flag,
                           partials);
}

// One block: combines the cell maxima and updates the well pressures (the
// BHP unknowns follow the cells in y), clipped like the cell pressures.
template <int NB>
__device__ __forceinline__ void newton_finish_body(int nparts, int n, int nw,
                                                   const double *__restrict__ y, double dp_max,
                                                   double *pbhp, const double *partials,
                                                   double *out) {
    const bool mx[3] = {true, true, true};
    double a[3];
    finish_partials<3>(nparts, mx, partials, a);
    if (threadIdx.x == 0) {
        double m = a[0];
        for (int wl = 0; wl < nw; ++wl) {
            double d = -y[(size_t)(n + wl) * NB];
            d = fmin(fmax(d, -dp_max), dp_max);
            pbhp[wl] += d;
            m = rop(m, fabs(d), true);
            if (d != d) m = NAN;
        }
        out[0] = m;
        out[1] = a[1];
        out[2] = a[2];
    }
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_newton_finish(int nparts, int n, int nw,
                                                          const double *__restrict__ y,
                                                          double dp_max, double *pbhp,
                                                          const double *partials, double *out) {
    newton_finish_body<NB>(nparts, n, nw, y, dp_max, pbhp, partials, out);
}

// Surface rates per well: q[w*3 + i], production positive.
template <int NB>
__global__ __launch_bounds__(64) void k_well_rates(Wells w, const double *__restrict__ P,
                                                   const double *__restrict__ pbhp,
                                                   const double *__restrict__ rec, int n,
                                                   double *__restrict__ qout) {
    const int wl = blockIdx.x, lane = threadIdx.x;
    const int p0 = w.wps[wl], np = w.wps[wl + 1] - p0;
    double s[3] = {0.0, 0.0, 0.0};
    for (int p = lane; p < np; p += 64) {
        const int pid = p0 + p, c = w.pcell[pid];
        double qr[NB], dq[NB][NB], dqb[NB];
        perf_rate<NB>(w.kind[wl], w.wi[pid], P[c], pbhp[wl], rec, n, c, qr, dq, dqb);
#pragma unroll
        for (int e = 0; e < NB; ++e) s[e] += qr[e];
    }
    const bool mx[3] = {false, false, false};
    wave_reduce<3>(s, mx);
    if (lane == 0)
        for (int e = 0; e < 3; ++e) qout[wl * 3 + e] = s[e];
}

// ---------------------------------------------------------------------------
// discrete adjoint of the backward-Euler system
//
// The parameter of cell c is theta_c = ln k_c, with kx, ky and kz of the
// cell scaled together.  The residual depends on it through the face
// transmissibilities (harmonic, so dT/dtheta_c = T g_o/(g_c + g_o) with g the
// half-cell conductances k A/h of the face's two cells) and through the
// Peaceman well indices (WI ~ sqrt(kx ky), so dWI/dtheta_c = WI; an explicit
// WI does not depend on k: wi_dk = 0).  The objective is the production
// mismatch J = sum over schedule-step ends and producers of
// (q_o,w - q_obs,w)^2, q_o,w the surface oil rate of the well.

// Objective terms at the end of a schedule step, one wave per well:
// r_w = q_o,w - qobs[w]; per perforation p of a producer
// objp[p][u] = 2 r_w dq_o,p/dx_u (u < NB) and objp[p][NB] = 2 r_w q_o,p wi_dk[p]
// (dJ/dtheta of its cell); per well objw[2w] = 2 r_w dq_o,w/dPbhp and
// objw[2w+1] = r_w^2.  Other wells get zeros.
template <int NB>
__global__ __launch_bounds__(64) void k_adj_objective(Wells w, int n,
                                                      const double *__restrict__ P,
                                                      const double *__restrict__ pbhp,
                                                      const double *__restrict__ rec,
                                                      const double *__restrict__ wi_dk,
                                                      const double *__restrict__ qobs,
                                                      double *__restrict__ objp,
                                                      double *__restrict__ objw) {
    const int wl = blockIdx.x, lane = threadIdx.x;
    const int p0 = w.wps[wl], np = w.wps[wl + 1] - p0;
    const bool prod = w.kind[wl] == kProd;
    double s[2] = {0.0, 0.0};
    if (prod)
        for (int p = lane; p < np; p += 64) {
            const int pid = p0 + p, c = w.pcell[pid];
            double qr[NB], dq[NB][NB], dqb[NB];
            perf_rate<NB>(kProd, w.wi[pid], P[c], pbhp[wl], rec, n, c, qr, dq, dqb);
            s[0] += qr[1];
            s[1] += dqb[1];
        }
    const bool mx[2] = {false, false};
    wave_reduce<2>(s, mx);
    const double r = prod ? s[0] - qobs[wl] : 0.0;
    for (int p = lane; p < np; p += 64) {
        const int pid = p0 + p, c = w.pcell[pid];
        double *o = objp + (size_t)pid * (NB + 1);
        double qr[NB], dq[NB][NB], dqb[NB];
        if (prod) perf_rate<NB>(kProd, w.wi[pid], P[c], pbhp[wl], rec, n, c, qr, dq, dqb);
#pragma unroll
        for (int u = 0; u < NB; ++u) o[u] = prod ? 2.0 * r * dq[1][u] : 0.0;
        o[NB] = prod ? 2.0 * r * qr[1] * wi_dk[pid] : 0.0;
    }
    if (lane == 0) {
        objw[2 * wl] = 2.0 * r * s[1];
        objw[2 * wl + 1] = r * r;
    }
}

// Right side of the adjoint system of a sub-step: on the cell rows
// (1/dt_next) (dA/dx)^T lam_next (lam_next null on the last sub-step), minus
// dJ/dx when the sub-step ends a schedule step (objp, objw non-null).
template <int NB>
__global__ __launch_bounds__(kBlock) void k_adj_rhs(Wells w, int n, int nw,
                                                    const double *__restrict__ rec,
                                                    const double *__restrict__ lam_next,
                                                    double rdt_next,
                                                    const double *__restrict__ objp,
                                                    const double *__restrict__ objw,
                                                    double *__restrict__ rhs) {
    using RI = Rec<NB>;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n + nw) return;
    double out[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) out[u] = 0.0;
    if (r < n) {
        if (lam_next) {
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                double a = 0.0;
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    a += rec[(size_t)(RI::ACC + i * RI::G + 1 + u) * n + r] * lam_next[(size_t)r * NB + i];
                out[u] = a * rdt_next;
            }
        }
        if (objp)
            for (int pp = w.cps[r]; pp < w.cps[r + 1]; ++pp) {
                const double *o = objp + (size_t)w.cperf[pp] * (NB + 1);
#pragma unroll
                for (int u = 0; u < NB; ++u) out[u] -= o[u];
            }
    } else if (objw) {
        out[0] = -objw[2 * (r - n)];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) rhs[(size_t)r * NB + u] = out[u];
}

// grad[c] += lam^T dR/dtheta_c (+ dJ/dtheta_c when objp is non-null) at
// the state of the sub-step, cell-centric: the faces of c, then its
// perforations (their own rows, and the well row of a rate-controlled well).
template <int NB>
__global__ __launch_bounds__(kBlock) void k_adj_grad(
    Grid g, Wells w, const double *__restrict__ depth, const double *__restrict__ tx,
    const double *__restrict__ ty, const double *__restrict__ tz, const double *__restrict__ kx,
    const double *__restrict__ ky, const double *__restrict__ kz, const double *__restrict__ dx,
    const double *__restrict__ dy, const double *__restrict__ dz, const double *__restrict__ P,
    const double *__restrict__ pbhp, const double *__restrict__ rec,
    const double *__restrict__ wi_dk, const double *__restrict__ lam,
    const double *__restrict__ objp, double *__restrict__ grad) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = g.n;
    if (c >= n) return;
    const int nx = g.nx, nxy = g.nx * g.ny;
    const int i = c % nx, j = (c / nx) % g.ny, k = c / nxy;
    Side<NB> me, nbr;
    load_side<NB>(rec, n, c, P, depth, me);
    double lc[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) lc[e] = lam[(size_t)c * NB + e];
    double acc = 0.0;
    // face to cell cn; rc = h/k of this cell's half, ro of the other's
    auto face = [&](int cn, double T, double rc, double ro, bool lower) {
        if (!(T > 0.0)) return;
        load_side<NB>(rec, n, cn, P, depth, nbr);
        double F[NB], dK[NB][NB], dL[NB][NB];
        double d = 0.0;
        if (lower) {            // flux from cn into c: R_cn += F, R_c -= F
            face_flux<NB>(T, nbr, me, F, dK, dL);
#pragma unroll
            for (int e = 0; e < NB; ++e) d += (lam[(size_t)cn * NB + e] - lc[e]) * F[e];
        } else {                // flux from c into cn: R_c += F, R_cn -= F
            face_flux<NB>(T, me, nbr, F, dK, dL);
#pragma unroll
            for (int e = 0; e < NB; ++e) d += (lc[e] - lam[(size_t)cn * NB + e]) * F[e];
        }
        acc += d * (rc / (rc + ro));
    };
    if (k > 0) face(c - nxy, tz[c - nxy], 0.5 * dz[k] / kz[c], 0.5 * dz[k - 1] / kz[c - nxy], true);
    if (j > 0) face(c - nx, ty[c - nx], 0.5 * dy[j] / ky[c], 0.5 * dy[j - 1] / ky[c - nx], true);
    if (i > 0) face(c - 1, tx[c - 1], 0.5 * dx[i] / kx[c], 0.5 * dx[i - 1] / kx[c - 1], true);
    if (i + 1 < nx) face(c + 1, tx[c], 0.5 * dx[i] / kx[c], 0.5 * dx[i + 1] / kx[c + 1], false);
    if (j + 1 < g.ny) face(c + nx, ty[c], 0.5 * dy[j] / ky[c], 0.5 * dy[j + 1] / ky[c + nx], false);
    if (k + 1 < g.nz) face(c + nxy, tz[c], 0.5 * dz[k] / kz[c], 0.5 * dz[k + 1] / kz[c + nxy], false);
    for (int pp = w.cps[c]; pp < w.cps[c + 1]; ++pp) {
        const int p = w.cperf[pp];
        const int wl = w.pwell[p];
        double qr[NB], dq[NB][NB], dqb[NB];
        perf_rate<NB>(w.kind[wl], w.wi[p], me.P, pbhp[wl], rec, n, c, qr, dq, dqb);
        double t = 0.0;
#pragma unroll
        for (int e = 0; e < NB; ++e) t += lc[e] * qr[e];
        const int ii = (w.kind[wl] == kInjGas) ? 2 : 0;        // the rate row's component
        if (w.ctrl[wl] == kRate && ii < NB) t -= lam[(size_t)(n + wl) * NB] * qr[ii];
        acc += t * wi_dk[p];
        if (objp) acc += objp[(size_t)p * (NB + 1) + NB];
    }
    grad[c] += acc;
}

// ---------------------------------------------------------------------------
// launchers

static inline int blocks_for(long n, int bs) { return (int)((n + bs - 1) / bs); }

void launch_static(hipStream_t s, Grid g, const double *dx, const double *dy, const double *dz,
                   double top, const double *kx, const double *ky, const double *kz,
                   const double *poro, double *vol, double *depth, double *pvref, double *tx,
                   double *ty, double *tz) {
    hipLaunchKernelGGL(k_static, dim3(blocks_for(g.n, kBlock)), dim3(kBlock), 0, s, g, dx, dy,
                       dz, top, kx, ky, kz, poro, vol, depth, pvref, tx, ty, tz);
}

void launch_peaceman(hipStream_t s, Grid g, int nperf, const int *pcell, const int *pwell,
                     const double *dx, const double *dy, const double *dz, const double *kx,
                     const double *ky, const double *rw, const double *skin, double *wi) {
    if (nperf == 0) return;
    hipLaunchKernelGGL(k_peaceman, dim3(blocks_for(nperf, 64)), dim3(64), 0, s, g, nperf, pcell,
                       pwell, dx, dy, dz, kx, ky, rw, skin, wi);
}

void launch_props(hipStream_t s, int nb, Phys f, int n, const double *pvref, const double *P,
                  const double *Sw, const double *X, const int8_t *flag, double *rec,
                  double *aold) {
    dim3 grid(blocks_for(n, kBlock)), block(kBlock);
    if (nb == 2)
        hipLaunchKernelGGL(k_props<2>, grid, block, 0, s, f, n, pvref, P, Sw, X, flag, rec, aold);
    else
        hipLaunchKernelGGL(k_props<3>, grid, block, 0, s, f, n, pvref, P, Sw, X, flag, rec, aold);
}

void launch_assemble(hipStream_t s, int nb, Grid g, Phys f, Wells w, Sys sys,
                     const double *depth, const double *tx, const double *ty, const double *tz,
                     const double *P, const double *pbhp, const double *rec, const double *aold,
                     double dt, double *wmeas) {
    (void)f;
    dim3 grid(blocks_for(g.n, kBlock)), block(kBlock);
    if (nb == 2) {
        hipLaunchKernelGGL(k_assemble_cells<2>, grid, block, 0, s, g, w, sys, depth, tx, ty, tz,
                           P, pbhp, rec, aold, dt);
        if (w.nw)
            hipLaunchKernelGGL(k_assemble_wells<2>, dim3(w.nw), dim3(64), 0, s, w, sys, g.n, P,
                               pbhp, rec, wmeas);
    } else {
        hipLaunchKernelGGL(k_assemble_cells<3>, grid, block, 0, s, g, w, sys, depth, tx, ty, tz,
                           P, pbhp, rec, aold, dt);
        if (w.nw)
            hipLaunchKernelGGL(k_assemble_wells<3>, dim3(w.nw), dim3(64), 0, s, w, sys, g.n, P,
                               pbhp, rec, wmeas);
    }
}

void launch_conv(hipStream_t s, int nb, int n, int nw, const double *rec, const double *R,
                 const double *wmeas, double dt, double *partials, int nblocks, double *out) {
    if (nb == 2) {
        hipLaunchKernelGGL(k_conv<2>, dim3(nblocks), dim3(kBlock), 0, s, n, nw, rec, R, wmeas, dt,
                           partials);
        hipLaunchKernelGGL(k_conv_finish<2>, dim3(1), dim3(kBlock), 0, s, nblocks, partials, out);
    } else {
        hipLaunchKernelGGL(k_conv<3>, dim3(nblocks), dim3(kBlock), 0, s, n, nw, rec, R, wmeas, dt,
                           partials);
        hipLaunchKernelGGL(k_conv_finish<3>, dim3(1), dim3(kBlock), 0, s, nblocks, partials, out);
    }
}

void launch_newton_update(hipStream_t s, int nb, Phys f, int n, int nw, const double *y,
                          double ds_max, double dp_max, double *P, double *Sw, double *X,
                          int8_t *flag, double *pbhp, double *partials, int nblocks,
                          double *out) {
    if (nb == 2) {
        hipLaunchKernelGGL(k_newton_update<2>, dim3(nblocks), dim3(kBlock), 0, s, f, n, nw, y,
                           ds_max, dp_max, P, Sw, X, flag, partials);
        hipLaunchKernelGGL(k_newton_finish<2>, dim3(1), dim3(kBlock), 0, s, nblocks, n, nw, y,
                           dp_max, pbhp, partials, out);
    } else {
        hipLaunchKernelGGL(k_newton_update<3>, dim3(nblocks), dim3(kBlock), 0, s, f, n, nw, y,
                           ds_max, dp_max, P, Sw, X, flag, partials);
        hipLaunchKernelGGL(k_newton_finish<3>, dim3(1), dim3(kBlock), 0, s, nblocks, n, nw, y,
                           dp_max, pbhp, partials, out);
    }
}

void launch_well_rates(hipStream_t s, int nb, Wells w, const double *P, const double *pbhp,
                       const double *rec, int n, double *q) {
    if (!w.nw) return;
    if (nb == 2)
        hipLaunchKernelGGL(k_well_rates<2>, dim3(w.nw), dim3(64), 0, s, w, P, pbhp, rec, n, q);
    else
        hipLaunchKernelGGL(k_well_rates<3>, dim3(w.nw), dim3(64), 0, s, w, P, pbhp, rec, n, q);
}

void launch_adj_objective(hipStream_t s, int nb, Wells w, int n, const double *P,
                          const double *pbhp, const double *rec, const double *wi_dk,
                          const double *qobs, double *objp, double *objw) {
    if (!w.nw) return;
    if (nb == 2)
        hipLaunchKernelGGL(k_adj_objective<2>, dim3(w.nw), dim3(64), 0, s, w, n, P, pbhp, rec,
                           wi_dk, qobs, objp, objw);
    else
        hipLaunchKernelGGL(k_adj_objective<3>, dim3(w.nw), dim3(64), 0, s, w, n, P, pbhp, rec,
                           wi_dk, qobs, objp, objw);
}

void launch_adj_rhs(hipStream_t s, int nb, Wells w, int n, const double *rec,
                    const double *lam_next, double rdt_next, const double *objp,
                    const double *objw, double *rhs) {
    dim3 grid(blocks_for((long)n + w.nw, kBlock)), block(kBlock);
    if (nb == 2)
        hipLaunchKernelGGL(k_adj_rhs<2>, grid, block, 0, s, w, n, w.nw, rec, lam_next, rdt_next,
                           objp, objw, rhs);
    else
        hipLaunchKernelGGL(k_adj_rhs<3>, grid, block, 0, s, w, n, w.nw, rec, lam_next, rdt_next,
                           objp, objw, rhs);
}

void launch_adj_grad(hipStream_t s, int nb, Grid g, Wells w, const double *depth,
                     const double *tx, const double *ty, const double *tz, const double *kx,
                     const double *ky, const double *kz, const double *dx, const double *dy,
                     const double *dz, const double *P, const double *pbhp, const double *rec,
                     const double *wi_dk, const double *lam, const double *objp, double *grad) {
    dim3 grid(blocks_for(g.n, kBlock)), block(kBlock);
    if (nb == 2)
        hipLaunchKernelGGL(k_adj_grad<2>, grid, block, 0, s, g, w, depth, tx, ty, tz, kx, ky, kz,
                           dx, dy, dz, P, pbhp, rec, wi_dk, lam, objp, grad);
    else
        hipLaunchKernelGGL(k_adj_grad<3>, grid, block, 0, s, g, w, depth, tx, ty, tz, kx, ky, kz,
                           dx, dy, dz, P, pbhp, rec, wi_dk, lam, objp, grad);
}

// ---------------------------------------------------------------------------
// batched launches over the members of an ensemble (each member's blocks run
// the bodies above on the member's own buffers)

template <int NB>
__global__ __launch_bounds__(kBlock) void kb_props(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    const bool ao = (B.flags[m] & kAold) != 0;
    props_body<NB>(b, M.f, M.n, M.pvref, M.P, M.Sw, M.X, M.flag, M.rec, ao ? M.aold : nullptr);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void kb_assemble_cells(const Member *__restrict__ mem, Batch B,
                                                            const double *__restrict__ dt) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    assemble_cells_body<NB>(b, M.g, M.wells, M.sys, M.depth, M.tx, M.ty, M.tz, M.P, M.pbhp, M.rec,
                            M.aold, dt[m]);
}

template <int NB>
__global__ __launch_bounds__(64) void kb_assemble_wells(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    assemble_wells_body<NB>(b, M.wells, M.sys, M.n, M.P, M.pbhp, M.rec, M.wmeas);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void kb_conv(const Member *__restrict__ mem, Batch B,
                                                  const double *__restrict__ dt) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    conv_body<NB>(b, nb, M.n, M.nw, M.rec, M.sys.R, M.wmeas, dt[m], M.partials);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void kb_conv_finish(const Member *__restrict__ mem, Batch B,
                                                         int slot) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    conv_finish_body<NB>(conv_blocks(M.n), M.partials, M.scal + slot);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void kb_newton_update(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    newton_update_body<NB>(b, nb, M.f, M.n, M.x, M.ds_max, M.dp_max, M.P, M.Sw, M.X, M.flag,
                           M.partials);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void kb_newton_finish(const Member *__restrict__ mem, Batch B,
                                                           int slot) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    newton_finish_body<NB>(update_blocks(M.n), M.n, M.nw, M.x, M.dp_max, M.pbhp, M.partials,
                           M.scal + slot);
}

// Copies of the state (P, Sw, X, flag over the cells, the BHP over the
// wells) between the live arrays and the save slots: to slot k when
// flags[m] has save_bit, back from slot k when it has restore_bit.
__global__ __launch_bounds__(kBlock) void kb_state_copy(const Member *__restrict__ mem,
                                                        const int *__restrict__ bstart,
                                                        const int *__restrict__ flags, int nm,
                                                        const StateSlots *__restrict__ slots,
                                                        int k, int save_bit, int restore_bit) {
    Batch B{bstart, flags, nm, save_bit | restore_bit};
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    const StateSlots &S = slots[m];
    const bool save = (flags[m] & save_bit) != 0;
    const int c = b * blockDim.x + threadIdx.x;
    if (c < M.n) {
        if (save) {
            S.P[k][c] = M.P[c];
            S.Sw[k][c] = M.Sw[c];
            S.X[k][c] = M.X[c];
            S.flag[k][c] = M.flag[c];
        } else {
            M.P[c] = S.P[k][c];
            M.Sw[c] = S.Sw[k][c];
            M.X[c] = S.X[k][c];
            M.flag[c] = S.flag[k][c];
        }
    }
    if (c < M.nw) {
        if (save) S.pbhp[k][c] = M.pbhp[c];
        else M.pbhp[c] = S.pbhp[k][c];
    }
}

// scal[first .. first + count) of every member that takes part, to
// packed[m * ld + e]
__global__ void kb_gather_scalars(const Member *__restrict__ mem, Batch B, int first, int count,
                                  double *__restrict__ packed, int ld) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    for (int e = threadIdx.x; e < count; e += blockDim.x) packed[(size_t)m * ld + e] = M.scal[first + e];
}

int blocks_for_cells(int n) { return blocks_for(n, kBlock); }

void launchb_props(hipStream_t s, int nb, const Member *mem, Batch B, int total) {
    if (total <= 0) return;
    if (nb == 2) hipLaunchKernelGGL(kb_props<2>, dim3(total), dim3(kBlock), 0, s, mem, B);
    else hipLaunchKernelGGL(kb_props<3>, dim3(total), dim3(kBlock), 0, s, mem, B);
}

void launchb_assemble(hipStream_t s, int nb, const Member *mem, Batch cells, int tcells,
                      Batch wells, int twells, const double *dt) {
    if (nb == 2) {
        if (tcells > 0)
            hipLaunchKernelGGL(kb_assemble_cells<2>, dim3(tcells), dim3(kBlock), 0, s, mem, cells, dt);
        if (twells > 0)
            hipLaunchKernelGGL(kb_assemble_wells<2>, dim3(twells), dim3(64), 0, s, mem, wells);
    } else {
        if (tcells > 0)
            hipLaunchKernelGGL(kb_assemble_cells<3>, dim3(tcells), dim3(kBlock), 0, s, mem, cells, dt);
        if (twells > 0)
            hipLaunchKernelGGL(kb_assemble_wells<3>, dim3(twells), dim3(64), 0, s, mem, wells);
    }
}

void launchb_conv(hipStream_t s, int nb, const Member *mem, Batch part, int tpart, Batch one,
                  int tone, const double *dt, int slot) {
    if (nb == 2) {
        hipLaunchKernelGGL(kb_conv<2>, dim3(tpart), dim3(kBlock), 0, s, mem, part, dt);
        hipLaunchKernelGGL(kb_conv_finish<2>, dim3(tone), dim3(kBlock), 0, s, mem, one, slot);
    } else {
        hipLaunchKernelGGL(kb_conv<3>, dim3(tpart), dim3(kBlock), 0, s, mem, part, dt);
        hipLaunchKernelGGL(kb_conv_finish<3>, dim3(tone), dim3(kBlock), 0, s, mem, one, slot);
    }
}

void launchb_newton_update(hipStream_t s, int nb, const Member *mem, Batch part, int tpart,
                           Batch one, int tone, int slot) {
    if (nb == 2) {
        hipLaunchKernelGGL(kb_newton_update<2>, dim3(tpart), dim3(kBlock), 0, s, mem, part);
        hipLaunchKernelGGL(kb_newton_finish<2>, dim3(tone), dim3(kBlock), 0, s, mem, one, slot);
    } else {
        hipLaunchKernelGGL(kb_newton_update<3>, dim3(tpart), dim3(kBlock), 0, s, mem, part);
        hipLaunchKernelGGL(kb_newton_finish<3>, dim3(tone), dim3(kBlock), 0, s, mem, one, slot);
    }
}

void launchb_state_copy(hipStream_t s, const Member *mem, const int *bstart, const int *flags,
                        int nm, int total, const StateSlots *slots, int k, int save_bit,
                        int restore_bit) {
    if (total > 0)
        hipLaunchKernelGGL(kb_state_copy, dim3(total), dim3(kBlock), 0, s, mem, bstart, flags, nm,
                           slots, k, save_bit, restore_bit);
}

void launchb_gather_scalars(hipStream_t s, const Member *mem, Batch one, int tone, int first,
                            int count, double *packed, int ld) {
    if (tone > 0)
        hipLaunchKernelGGL(kb_gather_scalars, dim3(tone), dim3(64), 0, s, mem, one, first, count,
                           packed, ld);
}

}  // namespace fim
