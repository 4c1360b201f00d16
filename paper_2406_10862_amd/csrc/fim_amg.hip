// fim_amg.hip - CPR two-stage preconditioner with an aggregation AMG on the
// pressure block (paper Sec. 5.1: CPR with AMG on pressure and block-Jacobi
// smoothing, inside FGMRES).
//
// Stage 1: quasi-IMPES decoupling.  For each cell the weights w_c solve
// D_c^T w_c = e_P (D_c the diagonal block), normalised by max|w_c|; the
// pressure matrix is A_p[c][d] = w_c^T A_cd e_P (well rows keep their BHP
// equation).  A_p is solved approximately by one V- or W-cycle.
// Stage 2: block Jacobi on the residual of the full system.
//
// The hierarchy exploits the Cartesian grid: aggregates are 2x2x2 boxes, so
// with piecewise-constant interpolation every Galerkin coarse operator is
// again a 7-point stencil (plus the well rows and columns, each well staying
// its own aggregate).  The smoother is red-black Gauss-Seidel.  Level data
// is stored colour-split (all red cells, then all black cells, the x
// dimension padded to even) so a colour sweep reads its coefficients
// contiguously; padded cells have a unit diagonal and no couplings.  The
// coarsest level is inverted densely once per setup.
#include <math.h>

#include "fim_internal.h"
#include "fim_reduce.h"

namespace fim {

// stencil slots: 0 diagonal, 1 -x, 2 +x, 3 -y, 4 +y, 5 -z, 6 +z
__device__ inline int split_of(const AmgLevel &L, int i, int j, int k) {
    const int c = i + L.nxp * (j + L.ny * k);
    return (((i + j + k) & 1) ? L.half : 0) + (c >> 1);
}

// n / d for n * d < 2^40, with m = ceil(2^40 / d) from the host: the
// rounding error of the product stays below 1/d, so the quotient is exact.
__device__ inline int fdiv(int n, unsigned long long m) {
    return (int)(((unsigned long long)(unsigned)n * m) >> 40);
}

// Grid position of split entry s: (i, j, k), padded natural index
// c = i + nxp*(j + ny*k) and colour (i + j + k) & 1.
struct Pos {
    int i, j, k, c, color;
};

__device__ inline Pos pos_of(const AmgLevel &L, int s) {
    Pos p;
    p.color = s >= L.half;
    const int c0 = 2 * (s - p.color * L.half);
    const int row = fdiv(c0, L.mnxp);
    p.k = fdiv(row, L.mny);
    p.j = row - p.k * L.ny;
    const int i0 = c0 - row * L.nxp;
    p.i = i0 + (((p.j + p.k) & 1) ^ p.color);
    p.c = c0 + (p.i - i0);
    return p;
}

// Position of the cell (i, j, k).
__device__ inline Pos pos_at(const AmgLevel &L, int i, int j, int k) {
    Pos p;
    p.i = i;
    p.j = j;
    p.k = k;
    p.c = i + L.nxp * (j + L.ny * k);
    p.color = (i + j + k) & 1;
    return p;
}

__device__ inline int split_pos(const AmgLevel &L, const Pos &p) {
    return (p.color ? L.half : 0) + (p.c >> 1);
}

// Neighbour d (stencil slot) of p: false outside the grid; otherwise its
// split index (the other colour) in ns.
__device__ inline bool nbr(const AmgLevel &L, const Pos &p, int d, int &ns) {
    int dc;
    bool in;
    switch (d) {
        case 1: in = p.i > 0; dc = -1; break;
        case 2: in = p.i + 1 < L.nx; dc = 1; break;
        case 3: in = p.j > 0; dc = -L.nxp; break;
        case 4: in = p.j + 1 < L.ny; dc = L.nxp; break;
        case 5: in = p.k > 0; dc = -L.nxp * L.ny; break;
        default: in = p.k + 1 < L.nz; dc = L.nxp * L.ny; break;
    }
    ns = (p.color ? 0 : L.half) + ((p.c + dc) >> 1);
    return in;
}

// coordinates of neighbour d of p
__device__ inline void nbr_ijk(const Pos &p, int d, int &ni, int &nj, int &nk) {
    ni = p.i + (d == 2) - (d == 1);
    nj = p.j + (d == 4) - (d == 3);
    nk = p.k + (d == 6) - (d == 5);
}

__device__ inline void cell_of(const AmgLevel &L, int s, int &i, int &j, int &k) {
    const Pos p = pos_of(L, s);
    i = p.i;
    j = p.j;
    k = p.k;
}

__device__ inline bool neighbour(const AmgLevel &L, int d, int i, int j, int k, int &ni, int &nj,
                                 int &nk) {
    ni = i;
    nj = j;
    nk = k;
    switch (d) {
        case 1: ni = i - 1; break;
        case 2: ni = i + 1; break;
        case 3: nj = j - 1; break;
        case 4: nj = j + 1; break;
        case 5: nk = k - 1; break;
        default: nk = k + 1; break;
    }
    return ni >= 0 && ni < L.nx && nj >= 0 && nj < L.ny && nk >= 0 && nk < L.nz;
}

// ---------------------------------------------------------------------------
// setup: pressure matrix from the Jacobian

template <int NB>
__device__ inline void qi_weights(const double *__restrict__ d, double (&w)[NB]) {
    // first row of D^-1 (adjugate row over the determinant), then scaled
    if constexpr (NB == 2) {
        const double det = d[0] * d[3] - d[1] * d[2];
        w[0] = d[3] / det;
        w[1] = -d[1] / det;
    } else {
        const double c0 = d[4] * d[8] - d[5] * d[7];
        const double c1 = -(d[1] * d[8] - d[2] * d[7]);
        const double c2 = d[1] * d[5] - d[2] * d[4];
        const double det = d[0] * c0 + d[3] * c1 + d[6] * c2;
        w[0] = c0 / det;
        w[1] = c1 / det;
        w[2] = c2 / det;
    }
    double m = 0.0;
#pragma unroll
    for (int e = 0; e < NB; ++e) m = fmax(m, fabs(w[e]));
    if (!(m > 0.0) || !isfinite(m)) {
#pragma unroll
        for (int e = 0; e < NB; ++e) w[e] = (e == 0) ? 1.0 : 0.0;
        return;
    }
#pragma unroll
    for (int e = 0; e < NB; ++e) w[e] /= m;
}

template <int NB>
__device__ inline double pcoef(const double *__restrict__ val, int q, const double (&w)[NB]) {
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < NB; ++e) s += w[e] * val[(size_t)q * NB * NB + e * NB];
    return s;
}

// Also copies the pressure column of every block of the row (rows of
// cells and wells) into ap[q][NB], the only part of A that the second CPR
// stage multiplies.
template <int NB, class LT>
__device__ __forceinline__ void amg_extract_body(int bid, int nblk, const AmgLevel &L,
                                                 const Grid &g, const Wells &wl, const Sys &sys,
                                                 double *__restrict__ wq, LT *__restrict__ ap) {
    // a group of 8 lanes per row, lane lg on the row's blocks lg, lg + 8, ...
    // (adjacent lanes read adjacent blocks); every lane forms the row's
    // weights from the diagonal block
    constexpr int G = 8;
    const int lg = threadIdx.x & (G - 1);
    const int t = (int)(((long)xcd_block(bid, nblk) * blockDim.x + threadIdx.x) / G);
    const int n = g.n;
    const int stride = 2 * L.half;
    if (t >= n + L.nw) return;
    const int q0 = sys.rowptr[t], q1 = sys.rowptr[t + 1];
    for (int q = q0 + lg; q < q1; q += G)
#pragma unroll
        for (int u = 0; u < NB; ++u) ap[(size_t)q * NB + u] = (LT)sys.val[(size_t)q * NB * NB + u * NB];
    if (t < n) {
        const int c = t, nx = g.nx, ny = g.ny, nxy = nx * ny;
        const int i = c % nx, j = (c / nx) % ny, k = c / nxy;
        double w[NB];
        qi_weights<NB>(sys.val + (size_t)sys.diagpos[c] * NB * NB, w);
        if (lg == 0)
#pragma unroll
            for (int e = 0; e < NB; ++e) wq[(size_t)c * NB + e] = w[e];
        const int s = split_of(L, i, j, k);
        // the row's 7-point blocks in their order -z, -y, -x, diagonal, +x,
        // +y, +z (those that exist), then its well columns
        const unsigned mask = (k > 0) | (j > 0) << 1 | (i > 0) << 2 | 1u << 3 | (i + 1 < nx) << 4 |
                              (j + 1 < ny) << 5 | (k + 1 < g.nz) << 6;
        if (lg < 7) {
            // slot lg holds stencil entry d of L.a (diagonal, -x, +x, -y, +y, -z, +z)
            const int d = (0x6420135 >> (4 * lg)) & 15;
            const int q = q0 + __popc(mask & ((1u << lg) - 1));
            L.a[(size_t)d * stride + s] = ((mask >> lg) & 1) ? pcoef<NB>(sys.val, q, w) : 0.0;
        } else {
            int q = q0 + __popc(mask);
            for (int pp = wl.cps[c]; pp < wl.cps[c + 1]; ++pp) L.acw[wl.cperf[pp]] = pcoef<NB>(sys.val, q++, w);
        }
    } else if (lg == 0) {
        const int wi = t - n;
        const int base = sys.rowptr[n + wi];
        const int p0 = L.sps[wi], np = L.sps[wi + 1] - p0;
        for (int p = 0; p < np; ++p) L.awc[p0 + p] = sys.val[(size_t)(base + p) * NB * NB];
        L.aww[wi] = sys.val[(size_t)(base + np) * NB * NB];
    }
}

template <int NB, class LT>
__global__ __launch_bounds__(kBlock) void k_amg_extract(AmgLevel L, Grid g, Wells wl, Sys sys,
                                                        double *__restrict__ wq,
                                                        LT *__restrict__ ap) {
    amg_extract_body<NB, LT>(blockIdx.x, gridDim.x, L, g, wl, sys, wq, ap);
}

// CPR for a transposed Jacobian (the adjoint systems).  With the forward
// quasi-IMPES weights W (rows of J combined) and the pressure injection P_p,
// the pressure operator of J is A_p = W^T J P_p; for J^T the first stage
// restricts the pressure component, solves A_p^T = P_p^T J^T W and prolongs
// with W.  From the blocks of J^T: A_p^T(c, c') = sum_i J^T(c, c')[0][i] w_i(c'),
// i.e. the first row of every block weighted by its column cell's weights
// (the BHP slot for a well column).  apT[q][u] = sum_i J^T_q[u][i] w_i(col q)
// gives J^T x1 for x1 = W mu in the fused second stage.
template <int NB>
__global__ __launch_bounds__(kBlock) void k_cprT_weights(int n, Sys sysT, double *__restrict__ wq) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double *dT = sysT.val + (size_t)sysT.diagpos[c] * NB * NB;
    double d[NB * NB], w[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e)
#pragma unroll
        for (int u = 0; u < NB; ++u) d[e * NB + u] = dT[u * NB + e];   // J's diagonal block
    qi_weights<NB>(d, w);
#pragma unroll
    for (int e = 0; e < NB; ++e) wq[(size_t)c * NB + e] = w[e];
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_cprT_extract(AmgLevel L, Grid g, Wells wl, Sys sysT,
                                                         const double *__restrict__ wq,
                                                         double *__restrict__ ap) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = g.n;
    if (t >= n + L.nw) return;
    for (int q = sysT.rowptr[t]; q < sysT.rowptr[t + 1]; ++q) {
        const int col = sysT.colind[q];
        double w[NB];
#pragma unroll
        for (int e = 0; e < NB; ++e) w[e] = col < n ? wq[(size_t)col * NB + e] : (e == 0 ? 1.0 : 0.0);
        const double *b = sysT.val + (size_t)q * NB * NB;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            double a = 0.0;
#pragma unroll
            for (int e = 0; e < NB; ++e) a += b[u * NB + e] * w[e];
            ap[(size_t)q * NB + u] = a;
        }
    }
    auto coef = [&](int q) { return ap[(size_t)q * NB]; };
    if (t < n) {
        const int c = t, nx = g.nx, ny = g.ny, nxy = nx * ny;
        const int i = c % nx, j = (c / nx) % ny, k = c / nxy;
        const int s = split_of(L, i, j, k);
        const int stride = 2 * L.half;
        int q = sysT.rowptr[c];
        double a[7];
        a[5] = (k > 0) ? coef(q++) : 0.0;
        a[3] = (j > 0) ? coef(q++) : 0.0;
        a[1] = (i > 0) ? coef(q++) : 0.0;
        a[0] = coef(q++);
        a[2] = (i + 1 < nx) ? coef(q++) : 0.0;
        a[4] = (j + 1 < ny) ? coef(q++) : 0.0;
        a[6] = (k + 1 < g.nz) ? coef(q++) : 0.0;
#pragma unroll
        for (int d = 0; d < 7; ++d) L.a[(size_t)d * stride + s] = a[d];
        for (int pp = wl.cps[c]; pp < wl.cps[c + 1]; ++pp) L.acw[wl.cperf[pp]] = coef(q++);
    } else {
        const int wi = t - n;
        const int base = sysT.rowptr[n + wi];
        const int p0 = L.sps[wi], np = L.sps[wi + 1] - p0;
        for (int p = 0; p < np; ++p) L.awc[p0 + p] = coef(base + p);
        L.aww[wi] = coef(base + np);
    }
}

// Galerkin coarsening with piecewise-constant aggregates: couplings inside an
// aggregate move to the coarse diagonal, couplings across an aggregate face
// add up on the coarse stencil slot of that face.
__device__ __forceinline__ void amg_coarsen_body(int bid, const AmgLevel &F, const AmgLevel &C,
                                                 const int *__restrict__ cfs_ptr,
                                                 const int *__restrict__ cfs_idx) {
    const int t = bid * blockDim.x + threadIdx.x;
    const int ncs = 2 * C.half;
    const int fstride = 2 * F.half;
    if (t < ncs) {
        int I, J, K;
        cell_of(C, t, I, J, K);
        if (I >= C.nx) return;                     // padded coarse cell: fixed at creation
        double a[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                    if (i >= F.nx || j >= F.ny || k >= F.nz) continue;
                    const int s = split_of(F, i, j, k);
                    a[0] += F.a[s];
#pragma unroll
                    for (int d = 1; d < 7; ++d) {
                        int ni, nj, nk;
                        if (!neighbour(F, d, i, j, k, ni, nj, nk)) continue;
                        const double v = F.a[(size_t)d * fstride + s];
                        if ((ni >> 1) == I && (nj >> 1) == J && (nk >> 1) == K) a[0] += v;
                        else a[d] += v;
                    }
                }
#pragma unroll
        for (int d = 0; d < 7; ++d) C.a[(size_t)d * ncs + t] = a[d];
    } else {
        const int cs = t - ncs;                     // coarse well slot
        if (cs < C.nslot) {
            double acw = 0.0, awc = 0.0;
            for (int q = cfs_ptr[cs]; q < cfs_ptr[cs + 1]; ++q) {
                acw += F.acw[cfs_idx[q]];
                awc += F.awc[cfs_idx[q]];
            }
            C.acw[cs] = acw;
            C.awc[cs] = awc;
        } else if (cs < C.nslot + C.nw) {
            C.aww[cs - C.nslot] = F.aww[cs - C.nslot];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_amg_coarsen(AmgLevel F, AmgLevel C,
                                                        const int *__restrict__ cfs_ptr,
                                                        const int *__restrict__ cfs_idx) {
    amg_coarsen_body(blockIdx.x, F, C, cfs_ptr, cfs_idx);
}

// dense matrix of the coarsest level: rows/cols are split indices, then wells
__device__ __forceinline__ void amg_dense_row(const AmgLevel &L, double *__restrict__ M, int t) {
    const int n = 2 * L.half + L.nw;
    if (t >= n) return;
    double *row = M + (size_t)t * n;
    for (int c = 0; c < n; ++c) row[c] = 0.0;
    if (t < 2 * L.half) {
        int i, j, k;
        cell_of(L, t, i, j, k);
        if (i >= L.nx) {
            row[t] = 1.0;
            return;
        }
        row[t] = L.a[t];
        for (int d = 1; d < 7; ++d) {
            int ni, nj, nk;
            if (neighbour(L, d, i, j, k, ni, nj, nk))
                row[split_of(L, ni, nj, nk)] += L.a[(size_t)d * 2 * L.half + t];
        }
        for (int q = L.cps[t]; q < L.cps[t + 1]; ++q) {
            const int sl = L.cslot[q];
            row[2 * L.half + L.swell[sl]] += L.acw[sl];
        }
    } else {
        const int w = t - 2 * L.half;
        row[t] = L.aww[w];
        for (int q = L.sps[w]; q < L.sps[w + 1]; ++q) row[L.scell[q]] += L.awc[q];
    }
}

__global__ void k_amg_dense(AmgLevel L, double *__restrict__ M) {
    amg_dense_row(L, M, blockIdx.x * blockDim.x + threadIdx.x);
}

// Gauss-Jordan inverse with partial pivoting by one workgroup; A is
// overwritten, Ainv receives the inverse transposed, *bad is set on a zero
// pivot.
__global__ __launch_bounds__(1024) void k_dense_invert(int n, double *__restrict__ A,
                                                       double *__restrict__ Ainv,
                                                       double *__restrict__ colk, int *bad) {
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    __shared__ int piv;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < n * n; e += nt) Ainv[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int bidx = k;
        for (int r = k + tid; r < n; r += nt) {
            const double v = fabs(A[(size_t)r * n + k]);
            if (v > best) {
                best = v;
                bidx = r;
            }
        }
        bv[tid] = best;
        bi[tid] = bidx;
        __syncthreads();
        for (int off = nt / 2; off > 0; off >>= 1) {
            if (tid < off) {
                const double o = bv[tid + off];
                const int oi = bi[tid + off];
                if (o > bv[tid] || (o == bv[tid] && oi < bi[tid])) {
                    bv[tid] = o;
                    bi[tid] = oi;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            piv = bi[0];
            if (!(bv[0] > 0.0)) *bad = 1;
        }
        __syncthreads();
        const int p = piv;
        if (p != k)
            for (int c = tid; c < n; c += nt) {
                double t1 = A[(size_t)k * n + c];
                A[(size_t)k * n + c] = A[(size_t)p * n + c];
                A[(size_t)p * n + c] = t1;
                t1 = Ainv[(size_t)k * n + c];
                Ainv[(size_t)k * n + c] = Ainv[(size_t)p * n + c];
                Ainv[(size_t)p * n + c] = t1;
            }
        __syncthreads();
        const double dk = A[(size_t)k * n + k];
        const double rdk = (dk != 0.0) ? 1.0 / dk : 0.0;
        for (int c = tid; c < n; c += nt) {
            A[(size_t)k * n + c] *= rdk;
            Ainv[(size_t)k * n + c] *= rdk;
        }
        for (int r = tid; r < n; r += nt) colk[r] = A[(size_t)r * n + k];
        __syncthreads();
        for (int e = tid; e < n * n; e += nt) {
            const int r = e / n, c = e % n;
            if (r == k) continue;
            const double f = colk[r];
            if (f == 0.0) continue;
            A[e] -= f * A[(size_t)k * n + c];
            Ainv[e] -= f * Ainv[(size_t)k * n + c];
        }
        __syncthreads();
    }
    // stored transposed (the coarse solve reads it by columns)
    for (int e = tid; e < n * n; e += nt) {
        const int r = e / n, c = e % n;
        if (r < c) {
            const double t = Ainv[e];
            Ainv[e] = Ainv[(size_t)c * n + r];
            Ainv[(size_t)c * n + r] = t;
        }
    }
}

// The same Gauss-Jordan elimination with [A | A^-1] in LDS (n <= kDenseLds):
// one wave finds the pivot with shuffles (largest magnitude, the smallest
// row on ties, as above), the workgroup updates, three barriers per pivot;
// the inverse is stored transposed, as above.
constexpr int kDenseLds = 96;
size_t dense_lds_bytes(int n) { return ((size_t)2 * n * n + n) * sizeof(double); }

__device__ __forceinline__ void dense_invert_lds_body(int n, const double *__restrict__ Ag,
                                                      double *__restrict__ Ainv, int *bad,
                                                      double *sm) {
    double *A = sm, *X = sm + (size_t)n * n, *colk = sm + (size_t)2 * n * n;
    __shared__ int piv;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < n * n; e += nt) {
        A[e] = Ag[e];
        X[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (tid < 64) {
            double best = -1.0;
            int bidx = k;
            for (int r = k + tid; r < n; r += 64) {
                const double v = fabs(A[(size_t)r * n + k]);
                if (v > best) {
                    best = v;
                    bidx = r;
                }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bidx, off, 64);
                if (ob > best || (ob == best && oi < bidx)) {
                    best = ob;
                    bidx = oi;
                }
            }
            if (tid == 0) {
                piv = bidx;
                if (!(best > 0.0)) *bad = 1;
            }
        }
        __syncthreads();
        const int p = piv;
        const double dk = A[(size_t)p * n + k];           // the pivot, before any write
        const double rdk = (dk != 0.0) ? 1.0 / dk : 0.0;
        // the pivot column after the swap of rows k and p, read before it changes
        for (int r = tid; r < n; r += nt) colk[r] = A[(size_t)((r == p) ? k : r) * n + k];
        __syncthreads();
        // row k <- row p scaled, row p <- old row k
        for (int c = tid; c < n; c += nt) {
            const double ak = A[(size_t)k * n + c], xk = X[(size_t)k * n + c];
            const double ap = A[(size_t)p * n + c], xp = X[(size_t)p * n + c];
            A[(size_t)k * n + c] = ap * rdk;
            X[(size_t)k * n + c] = xp * rdk;
            if (p != k) {
                A[(size_t)p * n + c] = ak;
                X[(size_t)p * n + c] = xk;
            }
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += nt) {
            const int r = e / n, c = e % n;
            if (r == k) continue;
            const double f = colk[r];
            if (f == 0.0) continue;
            A[e] -= f * A[(size_t)k * n + c];
            X[e] -= f * X[(size_t)k * n + c];
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += nt) Ainv[(size_t)(e % n) * n + e / n] = X[e];   // transposed
}

__global__ __launch_bounds__(1024) void k_dense_invert_lds(int n, const double *__restrict__ Ag,
                                                           double *__restrict__ Ainv, int *bad) {
    extern __shared__ double sm[];
    dense_invert_lds_body(n, Ag, Ainv, bad, sm);
}

// (Minv b)[row] by one thread, the columns in order; the inverse is stored
// transposed (MT[c * n + r] = Minv[r][c]), so the threads of consecutive
// rows read consecutive words
__device__ inline double dense_row(int n, const double *__restrict__ MT, const double *b,
                                   int row) {
    double s = 0.0;
    int c = 0;
    for (; c + 8 <= n; c += 8) {             // eight columns' loads in flight at once
        double m[8], v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            m[u] = MT[(size_t)(c + u) * n + row];
            v[u] = b[c + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s += m[u] * v[u];
    }
    for (; c < n; ++c) s += MT[(size_t)c * n + row] * b[c];
    return s;
}

// x = Minv b, one thread per row
__global__ __launch_bounds__(256) void k_dense_gemv(int n, const double *__restrict__ MT,
                                                    const double *__restrict__ b,
                                                    double *__restrict__ x) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row < n) x[row] = dense_row(n, MT, b, row);
}

// ---------------------------------------------------------------------------
// exact coarsest solve by slabs (the block-tridiagonal form of the level:
// slab b = the cells with coordinate b along the axis, in-slab position
// p = u + nu * v over the other two axes, then the slab's wells)

__device__ inline void slab_cell(const AmgExact &E, int b, int p, int &i, int &j, int &k) {
    const int u = p % E.nu, v = p / E.nu;
    if (E.axis == 0) {
        i = b; j = u; k = v;
    } else if (E.axis == 1) {
        i = u; j = b; k = v;
    } else {
        i = u; j = v; k = b;
    }
}

__device__ inline int slab_pos(const AmgExact &E, int i, int j, int k, int &b) {
    if (E.axis == 0) {
        b = i;
        return j + E.nu * k;
    }
    if (E.axis == 1) {
        b = j;
        return i + E.nu * k;
    }
    b = k;
    return i + E.nu * j;
}

// stencil entry d of the cell at slab b, position p
__device__ inline double slab_coef(const AmgLevel &L, const AmgExact &E, int b, int p, int d) {
    int i, j, k;
    slab_cell(E, b, p, i, j, k);
    return L.a[(size_t)d * 2 * L.half + split_of(L, i, j, k)];
}

// The block of slab b (m = ncs + its wells, row-major with stride m) into A.
__device__ void slab_block(const AmgLevel &L, const AmgExact &E, int b, int m, double *A) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < m * m; e += nt) A[e] = 0.0;
    __syncthreads();
    const int stride = 2 * L.half, w0 = E.swp[b];
    for (int p = tid; p < E.ncs; p += nt) {
        int i, j, k;
        slab_cell(E, b, p, i, j, k);
        const int s = split_of(L, i, j, k);
        A[(size_t)p * m + p] = L.a[s];
        const int u = p % E.nu, v = p / E.nu;
#pragma unroll
        for (int d = 1; d < 7; ++d) {
            const int ax = (d - 1) >> 1;
            if (ax == E.axis) continue;
            const int sgn = (d & 1) ? -1 : 1;
            // the first in-slab axis moves u, the second v
            const bool first = ax == (E.axis == 0 ? 1 : 0);
            const int nu = first ? u + sgn : u, nv = first ? v : v + sgn;
            if (nu < 0 || nu >= E.nu || nv < 0 || nv >= E.nv) continue;
            A[(size_t)p * m + nu + E.nu * nv] += L.a[(size_t)d * stride + s];
        }
        for (int q = L.cps[s]; q < L.cps[s + 1]; ++q) {
            const int sl = L.cslot[q];
            A[(size_t)p * m + E.ncs + E.wrank[L.swell[sl]]] += L.acw[sl];
        }
    }
    for (int e = tid; e < E.swp[b + 1] - w0; e += nt) {
        const int w = E.sw[w0 + e], row = E.ncs + e;
        A[(size_t)row * m + row] += L.aww[w];
        for (int q = L.sps[w]; q < L.sps[w + 1]; ++q) {
            const Pos ps = pos_of(L, L.scell[q]);
            int bb;
            const int pc = slab_pos(E, ps.i, ps.j, ps.k, bb);
            A[(size_t)row * m + pc] += L.awc[q];
        }
    }
    __syncthreads();
}

// a lane's double, read by every lane of the wave (l uniform)
__device__ inline double readlane_d(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

constexpr int kSlabRows = (kSlabMax + 15) / 16;    // rows of a slab block per wave

// Row of register slot i of a wave: rows in pairs (2p, 2p + 1), pair p held
// by wave p % 16.
__device__ inline int slab_row(int wave, int i) { return 32 * (i >> 1) + 2 * wave + (i & 1); }

// Gauss-Jordan inversion without pivoting (the pressure operator's Schur
// complements keep its diagonal dominance; a zero or non-finite pivot sets
// *bad) of the m x m block held in registers by a 1024-thread workgroup:
// slot i of wave w holds row slab_row(w, i), lane l columns l and l + 64.
// Pivots go in pairs k, k + 1: the wave holding both rows takes the two
// elimination steps on them (row k scaled, its pivot entry becoming
// 1 / pivot; row k + 1 eliminated with it and scaled; row k then eliminated
// with row k + 1) and passes them on through the buffers U ([2][2][ld], two
// so one barrier per pair); every other row r then takes a_r - a_rk u_k -
// a_r,k+1 u_k+1 with columns k and k + 1 entering as zero, which is the two
// steps at once.
__device__ __forceinline__ void gj_invert(double (&a)[kSlabRows][2], int lane, int wave, int m,
                                          double *U, int ld, int *bad) {
    // pair p = 16 j + ow: rows k = 32 j + 2 ow and k + 1 in slots 2 j and
    // 2 j + 1 of wave ow (j is a constant of the unrolled loop, so the
    // registers are indexed statically), their columns in slot h
#pragma unroll
    for (int j = 0; j < kSlabRows / 2; ++j) {
        const int h = j == 2 ? 1 : 0;
        for (int ow = 0; ow < 16; ++ow) {
            const int k = 32 * j + 2 * ow;
            if (k >= m) break;
            const bool two = k + 1 < m;
            const int lk = k - 64 * h;              // lane of column k (k + 1: lk + 1)
            double *U0 = U + (ow & 1) * 2 * ld, *U1 = U0 + ld;
            if (wave == ow) {
                const double piv = readlane_d(a[2 * j][h], lk);
                const double ip = 1.0 / piv;
                if (lane == 0 && !(fabs(piv) > 0.0 && isfinite(piv))) *bad = 1;
                double w[2] = {a[2 * j][0] * ip, a[2 * j][1] * ip};   // row k, step k
                if (lane == lk) w[h] = ip;
                double v[2] = {0.0, 0.0};
                if (two) {
                    double t2[2] = {a[2 * j + 1][0], a[2 * j + 1][1]};   // row k + 1
                    const double f1 = readlane_d(t2[h], lk);
                    if (lane == lk) t2[h] = 0.0;
                    t2[0] -= f1 * w[0];
                    t2[1] -= f1 * w[1];
                    const double piv1 = readlane_d(t2[h], lk + 1);
                    const double ip1 = 1.0 / piv1;
                    if (lane == 0 && !(fabs(piv1) > 0.0 && isfinite(piv1))) *bad = 1;
                    v[0] = t2[0] * ip1;
                    v[1] = t2[1] * ip1;
                    if (lane == lk + 1) v[h] = ip1;
                    const double g = readlane_d(w[h], lk + 1);        // row k, step k + 1
                    if (lane == lk + 1) w[h] = 0.0;
                    w[0] -= g * v[0];
                    w[1] -= g * v[1];
                }
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int q = lane + 64 * hh;
                    if (q < m) {
                        U0[q] = w[hh];
                        U1[q] = v[hh];
                    }
                }
            }
            lds_barrier();
            const double p0 = lane < m ? U0[lane] : 0.0, p1 = lane + 64 < m ? U0[lane + 64] : 0.0;
            const double q0 = lane < m ? U1[lane] : 0.0, q1 = lane + 64 < m ? U1[lane + 64] : 0.0;
#pragma unroll
            for (int i = 0; i < kSlabRows; ++i) {
                const int r = slab_row(wave, i);
                if (r >= m) continue;
                if (r == k) {
                    a[i][0] = p0;
                    a[i][1] = p1;
                    continue;
                }
                if (r == k + 1) {
                    a[i][0] = q0;
                    a[i][1] = q1;
                    continue;
                }
                const double f = readlane_d(a[i][h], lk);
                const double f1 = two ? readlane_d(a[i][h], lk + 1) : 0.0;
                double v0 = a[i][0], v1 = a[i][1];
                if (h == 0 && (lane == lk || lane == lk + 1)) v0 = 0.0;
                if (h == 1 && (lane == lk || lane == lk + 1)) v1 = 0.0;
                a[i][0] = v0 - f * p0 - f1 * q0;
                a[i][1] = v1 - f * p1 - f1 * q1;
            }
        }
    }
}

// Slab b's block minus its couplings through the inverse P (in registers,
// the layout of gj_invert) of the neighbouring slab b - dir: A_bb -
// diag(rowc) P diag(colc) on the cell rows and columns (a cell couples to
// the same position of the neighbouring slab), into the registers a.
__device__ inline void slab_schur_load(const double *A, int m, int ncs, bool couple,
                                       const double *rowc, const double *colc,
                                       double (&a)[kSlabRows][2], int lane, int wave) {
#pragma unroll
    for (int i = 0; i < kSlabRows; ++i) {
        const int r = slab_row(wave, i);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = lane + 64 * h;
            double v = 0.0;
            if (r < m && q < m) {
                v = A[(size_t)r * m + q];
                if (couple && r < ncs && q < ncs) v -= rowc[r] * a[i][h] * colc[q];
            }
            a[i][h] = v;
        }
    }
}

// Coupling coefficients of slab b with slab b - dir: rowc[p] of b's cell p
// towards b - dir, colc[p] of b - dir's cell p towards b.
__device__ inline void slab_couplings(const AmgLevel &L, const AmgExact &E, int b, int dir,
                                      double *rowc, double *colc) {
    const int dm = 2 * E.axis + 1, dp = 2 * E.axis + 2;
    for (int p = threadIdx.x; p < E.ncs; p += blockDim.x) {
        rowc[p] = slab_coef(L, E, b, p, dir > 0 ? dm : dp);
        colc[p] = slab_coef(L, E, b - dir, p, dir > 0 ? dp : dm);
    }
}

// One 1024-thread workgroup: the Schur complements of nsteps slabs from b0
// in direction dir (+1: D_b = A_bb - A_b,b-1 inv(D_b-1) A_b-1,b from the
// first slab up; -1: E_b = A_bb - A_b,b+1 inv(E_b+1) A_b+1,b from the last
// down), each inverted by gj_invert and stored to E.binv.  The inverse of
// one slab stays in the registers for the next slab's Schur complement.
__device__ void exact_factor_wg(const AmgLevel &L, const AmgExact &E, double *lds, int b0,
                                int nsteps, int dir) {
    const int tid = threadIdx.x;
    // (the wave index as a scalar, so the row tests branch uniformly)
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double *A = lds;                                  // [mmax * mmax], stride m
    double *U = lds + (size_t)E.mmax * E.mmax;        // [2][2][mmax] pivot row pairs
    double *rowc = U + 4 * E.mmax, *colc = rowc + E.mmax;
    double a[kSlabRows][2];
#pragma unroll
    for (int i = 0; i < kSlabRows; ++i) a[i][0] = a[i][1] = 0.0;
    for (int st = 0; st < nsteps; ++st) {
        const int b = b0 + dir * st;
        const int m = E.ncs + E.swp[b + 1] - E.swp[b];
        if (st > 0) slab_couplings(L, E, b, dir, rowc, colc);
        slab_block(L, E, b, m, A);                  // (ends with a barrier)
        slab_schur_load(A, m, E.ncs, st > 0, rowc, colc, a, lane, wave);
        gj_invert(a, lane, wave, m, U, E.mmax, E.bad);
        double *dst = E.binv + (size_t)b * E.mmax * E.mmax;
#pragma unroll
        for (int i = 0; i < kSlabRows; ++i) {
            const int r = slab_row(wave, i);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = lane + 64 * h;
                if (r < m && q < m) dst[(size_t)r * m + q] = a[i][h];
            }
        }
        // (the next slab's coefficients and block overwrite LDS only after
        // every thread has read this slab's: a barrier ends each pair)
        __syncthreads();
    }
}

// The twist slab t of the two-sided factorisation: T_t = A_tt - A_t,t-1
// inv(D_t-1) A_t-1,t - A_t,t+1 inv(E_t+1) A_t+1,t (either term absent at an
// end), inverted by gj_invert into E.binv; the two neighbours' inverses are
// read from E.binv.
__device__ void exact_twist_wg(const AmgLevel &L, const AmgExact &E, double *lds) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int t = E.twist;
    double *A = lds, *U = lds + (size_t)E.mmax * E.mmax;
    double *c0 = U + 4 * E.mmax, *c1 = c0 + E.mmax, *c2 = c1 + E.mmax, *c3 = c2 + E.mmax;
    const int m = E.ncs + E.swp[t + 1] - E.swp[t];
    const bool lo = t > 0, hi = t + 1 < E.nslab;
    if (lo) slab_couplings(L, E, t, 1, c0, c1);
    if (hi) slab_couplings(L, E, t, -1, c2, c3);
    slab_block(L, E, t, m, A);                      // (ends with a barrier)
    const size_t mm = (size_t)E.mmax * E.mmax;
    const int mlo = lo ? E.ncs + E.swp[t] - E.swp[t - 1] : 0;
    const int mhi = hi ? E.ncs + E.swp[t + 2] - E.swp[t + 1] : 0;
    double a[kSlabRows][2];
#pragma unroll
    for (int i = 0; i < kSlabRows; ++i) {
        const int r = slab_row(wave, i);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = lane + 64 * h;
            double v = 0.0;
            if (r < m && q < m) {
                v = A[(size_t)r * m + q];
                if (r < E.ncs && q < E.ncs) {
                    if (lo) v -= c0[r] * E.binv[(size_t)(t - 1) * mm + (size_t)r * mlo + q] * c1[q];
                    if (hi) v -= c2[r] * E.binv[(size_t)(t + 1) * mm + (size_t)r * mhi + q] * c3[q];
                }
            }
            a[i][h] = v;
        }
    }
    gj_invert(a, lane, wave, m, U, E.mmax, E.bad);
    double *dst = E.binv + (size_t)t * mm;
#pragma unroll
    for (int i = 0; i < kSlabRows; ++i) {
        const int r = slab_row(wave, i);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = lane + 64 * h;
            if (r < m && q < m) dst[(size_t)r * m + q] = a[i][h];
        }
    }
}

__global__ __launch_bounds__(1024) void k_amg_exact_factor(AmgLevel L, AmgExact E) {
    extern __shared__ double lds[];
    exact_factor_wg(L, E, lds, 0, E.nslab, 1);
}

// The two sides of the two-sided factorisation at once: workgroup 0 the
// slabs below the twist from the first up, workgroup 1 those above it from
// the last down.
__global__ __launch_bounds__(1024) void k_amg_exact_factor2(AmgLevel L, AmgExact E) {
    extern __shared__ double lds[];
    const bool up = blockIdx.x == 0;
    exact_factor_wg(L, E, lds, up ? 0 : E.nslab - 1, up ? E.twist : E.nslab - 1 - E.twist,
                    up ? 1 : -1);
}

__global__ __launch_bounds__(1024) void k_amg_exact_twist(AmgLevel L, AmgExact E) {
    extern __shared__ double lds[];
    exact_twist_wg(L, E, lds);
}

// The exact solve by the whole workgroup: x = A^-1 b of the level, through
// z (LDS, [nslab][mmax]) and t ([mmax]).  Forward: z_b = inv(D_b) (b_b -
// A_b,b-1 z_b-1); backward: x_b = z_b - inv(D_b) A_b,b+1 x_b+1.  A row of a
// block product is summed by 8 lanes (columns lane, lane + 8, ...) and a
// fixed shuffle tree.
__device__ void exact_solve_wg(const AmgLevel &L, const AmgExact &E, double *z) {
    const int tid = threadIdx.x, nt = blockDim.x;
    double *t = z + (size_t)E.nslab * E.mmax;
    // the cells' right-hand sides and couplings to the slabs before and
    // after, staged in slab order
    double *bb = t + E.mmax, *am = bb + (size_t)E.nslab * E.ncs, *apc = am + (size_t)E.nslab * E.ncs;
    int *sp = reinterpret_cast<int *>(apc + (size_t)E.nslab * E.ncs);   // slab -> wells
    const int mm = E.mmax * E.mmax, dm = 2 * E.axis + 1, dp = 2 * E.axis + 2;
    {
        // (the wells' right-hand sides go to their places in z, which the
        // forward step of their slab reads before it writes there)
        for (int e = tid; e <= E.nslab; e += nt) sp[e] = E.swp[e];
        for (int b = tid; b < E.nslab; b += nt)
            for (int q = E.swp[b]; q < E.swp[b + 1]; ++q)
                z[(size_t)b * E.mmax + E.ncs + (q - E.swp[b])] = L.b[2 * L.half + E.sw[q]];
        const int stride = 2 * L.half;
        for (int e = tid; e < stride; e += nt) {
            const Pos ps = pos_of(L, e);
            if (ps.i >= L.nx) continue;
            int b;
            const int idx = slab_pos(E, ps.i, ps.j, ps.k, b);
            const size_t o = (size_t)b * E.ncs + idx;
            bb[o] = L.b[e];
            am[o] = L.a[(size_t)dm * stride + e];
            apc[o] = L.a[(size_t)dp * stride + e];
        }
        __syncthreads();
    }
    // a block product y = B t: row r (r < kSlabMax) is summed by the 32-lane
    // group r % 32 in pass r / 32, lane l taking the columns l + 32 u; a
    // block's entries for a thread are kU values (a slot past the block
    // loads the block's first entry and is dropped)
    constexpr int kP = (kSlabMax + 31) / 32, kC = (kSlabMax + 31) / 32, kU = kP * kC;
    const int grp = tid >> 5, l32 = tid & 31;
    auto slab_m = [&](int b) { return E.ncs + sp[b + 1] - sp[b]; };
    auto fetch = [&](int b, double (&v)[kU]) {
        const int m = slab_m(b);
        const double *B = E.binv + (size_t)b * mm;
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            const int r = grp + 32 * p;
#pragma unroll
            for (int u = 0; u < kC; ++u) {
                const int c = l32 + 32 * u;
                v[p * kC + u] = B[(r < m && c < m) ? (size_t)r * m + c : 0];
            }
        }
    };
    auto product = [&](int b, const double (&v)[kU], bool sub) {
        const int m = slab_m(b);
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            const int r = grp + 32 * p;
            double acc = 0.0;
#pragma unroll
            for (int u = 0; u < kC; ++u) {
                const int c = l32 + 32 * u;
                const double tc = t[c < m ? c : 0];
                acc += c < m ? v[p * kC + u] * tc : 0.0;
            }
#pragma unroll
            for (int off = 16; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if (r < m && l32 == 0) {
                double &zr = z[(size_t)b * E.mmax + r];
                zr = sub ? zr - acc : acc;
            }
        }
    };
    // the sweep's steps: forward over the slabs, then backward from the
    // second last; the block of step i + 1 is loaded during step i into
    // the other register buffer (steps taken in pairs, so each buffer keeps
    // its role), and the barriers order LDS only, so those loads stay in
    // flight across them
    const int nstep = 2 * E.nslab - 1;
    auto slab_at = [&](int i) { return i < E.nslab ? i : 2 * E.nslab - 2 - i; };
    auto step = [&](int i, const double (&cur)[kU], double (&nxt)[kU]) {
        const int b = slab_at(i);
        const bool back = i >= E.nslab;
        const int m = slab_m(b);
        for (int p = tid; p < m; p += nt) {
            double v;
            if (p < E.ncs) {
                const size_t o = (size_t)b * E.ncs + p;
                if (back) {
                    v = apc[o] * z[(size_t)(b + 1) * E.mmax + p];
                } else {
                    v = bb[o];
                    if (b > 0) v -= am[o] * z[(size_t)(b - 1) * E.mmax + p];
                }
            } else {
                v = back ? 0.0 : z[(size_t)b * E.mmax + p];
            }
            t[p] = v;
        }
        if (i + 1 < nstep) fetch(slab_at(i + 1), nxt);
        lds_barrier();
        product(b, cur, back);
        lds_barrier();
    };
    double va[kU], vb[kU];
    fetch(0, va);
    for (int i = 0; i < nstep; i += 2) {
        step(i, va, vb);
        if (i + 1 < nstep) step(i + 1, vb, va);
    }
    for (int e = tid; e < 2 * L.half; e += nt) {
        const Pos ps = pos_of(L, e);
        double v = 0.0;                             // padded entries stay zero
        if (ps.i < L.nx) {
            int b;
            const int p = slab_pos(E, ps.i, ps.j, ps.k, b);
            v = z[(size_t)b * E.mmax + p];
        }
        L.x[e] = v;
    }
    for (int b = tid; b < E.nslab; b += nt)
        for (int q = E.swp[b]; q < E.swp[b + 1]; ++q)
            L.x[2 * L.half + E.sw[q]] = z[(size_t)b * E.mmax + E.ncs + (q - E.swp[b])];
}

__global__ __launch_bounds__(1024) void k_amg_exact_solve(AmgLevel L, AmgExact E) {
    extern __shared__ double lds[];
    exact_solve_wg(L, E, lds);
}

// Storage index (the level's split order; wells after the cells) of slab b,
// position p.
__device__ inline int slab_storage(const AmgLevel &L, const AmgExact &E, int b, int p) {
    if (p >= E.ncs) return 2 * L.half + E.sw[E.swp[b] + p - E.ncs];
    int i, j, k;
    slab_cell(E, b, p, i, j, k);
    return split_of(L, i, j, k);
}

// The level's inverse X = A^-1 from the two-sided slab factors, kInvCols
// columns per workgroup: the columns of positions p0 .. p0 + 9 of slab s
// (contiguous columns of X) solved with those unit right sides: from slab s
// towards the twist slab (z_s a column of the inverse held for slab s), the
// twist, then outward on both sides.  Thread (r, c) forms row r of column c
// from row r of the slab's inverse in eight chunks of 12 entries (immediate
// offsets; a chunk may run past the row, into the next one or the
// allocation's padding, where t is zero), two chunks in flight, the first
// loaded before the step's barrier.  Each step's result goes to its rows of
// X at once (the results towards the twist are read back by the same
// threads on the way out); the barriers order LDS only, so those loads and
// stores stay in flight.  Grid: nslab x ceil(mmax / kInvCols) workgroups of
// kInvCols * kSlabMax threads (252 for 28 slabs of 90: one round over the
// CUs).
constexpr int kInvCols = 10, kInvCh = 12, kInvChunks = kSlabMax / kInvCh;
__global__ __launch_bounds__(kInvCols * kSlabMax) void k_amg_exact_inverse(AmgLevel L, AmgExact E) {
    __shared__ double zx[kSlabMax][kInvCols], t[kSlabMax][kInvCols], xt[kSlabMax][kInvCols];
    const int groups = (E.mmax + kInvCols - 1) / kInvCols;
    const int s = blockIdx.x / groups, p0 = (blockIdx.x % groups) * kInvCols;
    const int ms = E.ncs + E.swp[s + 1] - E.swp[s];
    if (p0 >= ms) return;                                 // (uniform over the block)
    const int r = threadIdx.x / kInvCols, c = threadIdx.x % kInvCols;
    const bool con = p0 + c < ms;
    const size_t col = (size_t)s * E.ncs + E.swp[s] + p0 + c;
    const int dm = 2 * E.axis + 1, dp = 2 * E.axis + 2;
    const size_t mm = (size_t)E.mmax * E.mmax;
    auto slab_m = [&](int b) { return E.ncs + E.swp[b + 1] - E.swp[b]; };
    auto row_of = [&](int b, int m) { return E.binv + (size_t)b * mm + (size_t)(r < m ? r : 0) * m; };
    auto load_chunk = [&](const double *B, double (&v)[kInvCh]) {
#pragma unroll
        for (int u = 0; u < kInvCh; ++u) v[u] = B[u];
    };
    auto use_chunk = [&](const double (*tq)[kInvCols], const double (&v)[kInvCh], double (&acc)[4]) {
#pragma unroll
        for (int u = 0; u < kInvCh; ++u) acc[u & 3] += v[u] * tq[u][c];
    };
    double va[kInvCh], vb[kInvCh];
    auto product = [&](const double *B) {           // (va holds chunk 0)
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
        for (int ch = 0; ch < kInvChunks; ch += 2) {
            load_chunk(B + kInvCh * (ch + 1), vb);
            use_chunk(t + kInvCh * ch, va, acc);
            if (ch + 2 < kInvChunks) load_chunk(B + kInvCh * (ch + 2), va);
            use_chunk(t + kInvCh * (ch + 1), vb, acc);
        }
        return (acc[0] + acc[1]) + (acc[2] + acc[3]);
    };
    // the result of a step: to zx and to its rows of X
    auto put = [&](int b, int m, double v) {
        if (r < m) {
            zx[r][c] = v;
            if (con) E.X[(size_t)slab_storage(L, E, b, r) * E.ldx + col] = v;
        }
    };
    // a step b from a neighbour's result in zx: the right side -coef(d) zx
    // (cell rows; d towards that neighbour), then inv(.) of slab b times it
    auto step = [&](int b, int m, int d) {
        const double *B = row_of(b, m);
        load_chunk(B, va);
        t[r][c] = r < E.ncs && r < m ? -slab_coef(L, E, b, r, d) * zx[r][c] : 0.0;
        lds_barrier();
        const double v = product(B);
        lds_barrier();                                     // (t and zx read)
        return v;
    };
    const int t0 = E.twist;
    // towards the twist: below it z_b = inv(D_b)(e_p [b = s] - A_b,b-1 z_b-1),
    // above it z_b = inv(E_b)(e_p [b = s] - A_b,b+1 z_b+1)
    const int dir = s < t0 ? 1 : -1;
    for (int b = s; b != t0; b += dir) {
        const int m = slab_m(b);
        double z = 0.0;
        if (b == s) {
            if (r < m && con) z = row_of(b, m)[p0 + c];
        } else {
            z = step(b, m, dir > 0 ? dm : dp);
        }
        put(b, m, z);
        lds_barrier();
    }
    // the twist: x_t = inv(T_t)(e_p [t = s] - the coupling to the last z)
    {
        const int m = slab_m(t0);
        double x = 0.0;
        if (s == t0) {
            if (r < m && con) x = row_of(t0, m)[p0 + c];
        } else {
            x = step(t0, m, s < t0 ? dm : dp);
        }
        put(t0, m, x);
        if (r < m) xt[r][c] = x;
        lds_barrier();
    }
    // outward: below the twist x_b = z_b - inv(D_b) A_b,b+1 x_b+1, above it
    // x_b = z_b - inv(E_b) A_b,b-1 x_b-1, where z_b is stored for the slabs
    // between s and the twist and zero elsewhere
    for (int side = 0; side < 2; ++side) {
        const int od = side == 0 ? -1 : 1;
        if (side == 1) {
            zx[r][c] = xt[r][c];
            lds_barrier();
        }
        for (int b = t0 + od; b >= 0 && b < E.nslab; b += od) {
            const int m = slab_m(b);
            const bool stored = od < 0 ? (s < t0 && b >= s) : (s > t0 && b <= s);
            double zb = 0.0;
            if (r < m && stored && con) zb = E.X[(size_t)slab_storage(L, E, b, r) * E.ldx + col];
            // step() forms -coef * x of the neighbour: x_b = zb + inv(.) (that)
            const double v = step(b, m, od < 0 ? dp : dm);
            put(b, m, zb + v);
            lds_barrier();
        }
    }
}

// x = X b over the whole chip: a wave per row, its entries in chunks of 8
// 16-byte loads per lane (the first chunk issued before b is gathered into
// slab order in LDS by the workgroup, the next one before the current one is
// used), four partial sums and a fixed shuffle tree.  Grid: ceil(nst /
// kGemvRows) workgroups of 64 kGemvRows.  (Sixteen rows per workgroup
// spread the gather of b over more rows: 12.6 -> 11.2 us for 2469 rows
// against eight; chunks of 16 loads per lane were slower, 16.5 us.)
constexpr int kGemvRows = 16, kGemvCh = 8;
__global__ __launch_bounds__(64 * kGemvRows) void k_amg_exact_gemv(AmgLevel L, AmgExact E) {
    extern __shared__ double bs[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = min((int)blockIdx.x * kGemvRows + wave, E.nst - 1);   // (a spare wave
    const double2 *X = reinterpret_cast<const double2 *>(E.X + (size_t)row * E.ldx);   // repeats
    const double2 *B = reinterpret_cast<const double2 *>(bs);              // the last row)
    const int n2 = E.ldx / 2, nch = (n2 + 64 * kGemvCh - 1) / (64 * kGemvCh);
    auto load = [&](int ch, double2 (&v)[kGemvCh]) {
#pragma unroll
        for (int u = 0; u < kGemvCh; ++u) {
            const int f = 64 * (kGemvCh * ch + u) + lane;
            v[u] = f < n2 ? X[f] : make_double2(0.0, 0.0);
        }
    };
    double2 va[kGemvCh], vb[kGemvCh];
    load(0, va);
    for (int f = tid; f < E.ldx; f += blockDim.x) bs[f] = f < E.ncol ? L.b[E.cmap[f]] : 0.0;
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    auto use = [&](int ch, const double2 (&v)[kGemvCh]) {
#pragma unroll
        for (int u = 0; u < kGemvCh; ++u) {
            const int f = 64 * (kGemvCh * ch + u) + lane;
            const double2 bv = f < n2 ? B[f] : make_double2(0.0, 0.0);
            acc[u & 3] += v[u].x * bv.x + v[u].y * bv.y;
        }
    };
    for (int ch = 0; ch < nch; ch += 2) {
        if (ch + 1 < nch) load(ch + 1, vb);
        use(ch, va);
        if (ch + 1 >= nch) break;
        if (ch + 2 < nch) load(ch + 2, va);
        use(ch + 1, vb);
    }
    double v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0 && blockIdx.x * kGemvRows + wave < E.nst) L.x[row] = v;
}

// ---------------------------------------------------------------------------
// cycle kernels

// Value of neighbour d of p (ns its split index), or of p itself when the
// neighbour is outside the grid (in = false): the stencil coefficient of a
// missing neighbour is zero on every level, so the stencil loops multiply
// by it without a branch and their loads need no wait in between.
// M: the read mode as a constant (the sweeps' modes are fixed per launch or
// phase), or -1 to take it from mode.
template <int M>
__device__ inline double read_cell(const AmgLevel &L, const AmgLevel &C, int mode, int ns,
                                   const Pos &p, int d, bool in) {
    const int m = M >= 0 ? M : mode;
    if (m & kCellsZero) return 0.0;
    double v = L.x[ns];
    if (m & kCellsCorr) {
        int ni = p.i, nj = p.j, nk = p.k;
        if (in) nbr_ijk(p, d, ni, nj, nk);
        v += C.x[split_of(C, ni >> 1, nj >> 1, nk >> 1)];
    }
    return v;
}

template <int M>
__device__ inline double read_well(const AmgLevel &L, const AmgLevel &C, int mode, int w) {
    const int m = M >= 0 ? M : mode;
    if (m & kWellsSnap) return L.xs[w];
    if (m & kWellsZero) return 0.0;
    double v = L.x[2 * L.half + w];
    if (m & kWellsCorr) v += C.x[2 * C.half + w];
    return v;
}

// Gauss-Seidel value of cell h of one colour (cells of one colour are not
// coupled to each other, so a colour sweep is exact and order-free);
// padded cells get 0.
// (Early: the divisor is read with the stencil and the division is not
// behind a branch, which pays in the multi-block kernels that stream HBM;
// in the one-workgroup sub-cycle, issue-bound with its data in LDS, the
// padded lanes' extra division costs more.  Same value either way.)
template <int M, bool Early>
__device__ inline double sweep_value(const AmgLevel &L, const AmgLevel &C, int color, int mode,
                                     int h) {
    const int s = color * L.half + h;
    const Pos p = pos_of(L, s);
    const int stride = 2 * L.half;
    const bool pad = p.i >= L.nx;
    // (Early: a padded cell divides 0 by 1)
    const double dg = Early ? L.a[s] : 1.0;
    double acc = L.b[s];
#pragma unroll
    for (int d = 1; d < 7; ++d) {
        int ns;
        const bool in = nbr(L, p, d, ns);
        acc -= L.a[(size_t)d * stride + s] * read_cell<M>(L, C, mode, in ? ns : s, p, d, in);
    }
    for (int q = L.cps[s]; q < L.cps[s + 1]; ++q) {
        const int sl = L.cslot[q];
        acc -= L.acw[sl] * read_well<M>(L, C, mode, L.swell[sl]);
    }
    // a padded cell (its neighbours in the grid are valid entries) is
    // computed like the others and dropped here: no branch before the loads
    if (Early) return (pad ? 0.0 : acc) / (pad ? 1.0 : dg);
    return pad ? 0.0 : acc / L.a[s];
}

template <int M, bool Early = false>
__device__ inline void sweep_item(const AmgLevel &L, const AmgLevel &C, int color, int mode,
                                  int h) {
    L.x[color * L.half + h] = sweep_value<M, Early>(L, C, color, mode, h);
}

// The first pre-smoothing pair from a zero iterate (wells still zero) in
// one pass: red cell h gets b/a_0 (all its neighbours are zero), black cell
// h gets its Gauss-Seidel value from those red values, computed on the fly.
__device__ inline double red_from_zero(const AmgLevel &L, int s) { return L.b[s] / L.a[s]; }

// (red and black values of entry h; padded cells computed and dropped)
template <bool Early>
__device__ inline double presmooth_black(const AmgLevel &L, int h);

template <bool Early>
__device__ inline void presmooth_values(const AmgLevel &L, int h, double &red, double &black) {
    const double r0 = red_from_zero(L, h);
    red = (pos_of(L, h).i >= L.nx) ? 0.0 : r0;
    black = presmooth_black<Early>(L, h);
}

template <bool Early>
__device__ inline double presmooth_black(const AmgLevel &L, int h) {
    const int s = L.half + h;
    const Pos p = pos_of(L, s);
    const int stride = 2 * L.half;
    const bool pad = p.i >= L.nx;
    const double dg = Early ? L.a[s] : 1.0;     // (as in sweep_value)
    double acc = L.b[s];
#pragma unroll
    for (int d = 1; d < 7; ++d) {
        int ns;
        const bool in = nbr(L, p, d, ns);
        acc -= L.a[(size_t)d * stride + s] * red_from_zero(L, in ? ns : s);
    }
    for (int q = L.cps[s]; q < L.cps[s + 1]; ++q) acc -= L.acw[L.cslot[q]] * 0.0;
    return Early ? (pad ? 0.0 : acc) / (pad ? 1.0 : dg) : (pad ? 0.0 : acc / L.a[s]);
}

template <bool Early = false>
__device__ inline void presmooth_item(const AmgLevel &L, int h) {
    double red, black;
    presmooth_values<Early>(L, h, red, black);
    L.x[h] = red;
    L.x[L.half + h] = black;
}

// wells: one wave per well, lanes stride over its slots; xcell(s) gives
// the value of the cell with split index s
// (two slots of a lane at a time, both cell values formed before either is
// added: the sum runs in the same order as one slot at a time)
template <class XC>
__device__ inline double well_row_sum_of(const AmgLevel &L, int w, int lane, XC xcell) {
    double acc = 0.0;
    const int q1 = L.sps[w + 1];
    int q = L.sps[w] + lane;
    for (; q + 64 < q1; q += 128) {
        const double a0 = L.awc[q], a1 = L.awc[q + 64];
        const double x0 = xcell(L.scell[q]), x1 = xcell(L.scell[q + 64]);
        acc += a0 * x0;
        acc += a1 * x1;
    }
    if (q < q1) acc += L.awc[q] * xcell(L.scell[q]);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    return acc;
}

__device__ inline double well_row_sum(const AmgLevel &L, int w, int lane) {
    return well_row_sum_of(L, w, lane, [&](int s) { return L.x[s]; });
}

// The Gauss-Seidel value of well w from the cell values xcell.  (Every lane
// reads the row's b and diagonal with its slots and stores the same value,
// so no load waits behind the reduction and a lane-0 branch.)
template <class XC>
__device__ inline void well_sweep_of(const AmgLevel &L, int w, int lane, XC xcell) {
    const double bw = L.b[2 * L.half + w], aw = L.aww[w];
    const double sum = well_row_sum_of(L, w, lane, xcell);
    L.x[2 * L.half + w] = (bw - sum) / aw;
}

__device__ inline void well_sweep_item(const AmgLevel &L, int w, int lane) {
    well_sweep_of(L, w, lane, [&](int s) { return L.x[s]; });
}

// The launched smoothing folds each well sweep into the kernel before it:
// its first well_blocks blocks (dispatched first, so their chain of
// dependent loads overlaps the cells' work; a multiple of the XCD count, so
// the cell blocks keep their XCD mapping) take one wave per well and form
// the cell values of the well's slots themselves, exactly as the cell
// blocks compute them (a red value from the previous kernel, a black one
// recomputed), so the well's value is that of a separate well sweep after
// the kernel, bit for bit.  While the cell blocks run, the wells' old
// values must stay readable: a colour-1 sweep reads them from the snapshot
// L.xs that the colour-0 sweep before it wrote (kWellsSnap), and the first
// pre-smoothing reads none (its wells are zero).
__device__ inline int well_wave() { return ((int)blockIdx.x * kBlock + (int)threadIdx.x) >> 6; }

__global__ __launch_bounds__(kBlock) void k_amg_presmooth(AmgLevel L, int well_blocks) {
    if ((int)blockIdx.x >= well_blocks) {
        const int nb = (int)gridDim.x - well_blocks;
        const int h = xcd_block((int)blockIdx.x - well_blocks, nb) * blockDim.x + threadIdx.x;
        if (h < L.half) presmooth_item<true>(L, h);
        return;
    }
    const int w = well_wave();
    if (w < L.nw)
        well_sweep_of(L, w, threadIdx.x & 63, [&](int s) {
            if (s >= L.half) return presmooth_black<true>(L, s - L.half);
            return pos_of(L, s).i >= L.nx ? 0.0 : red_from_zero(L, s);
        });
}

// Colour 0 (its well blocks store the snapshot of the wells' values as
// read in mode) or colour 1 (mode includes kWellsSnap; its well blocks
// compute the wells' Gauss-Seidel values).
template <int M>
__global__ __launch_bounds__(kBlock) void k_amg_sweep(AmgLevel L, AmgLevel C, int color, int mode,
                                                      int well_blocks) {
    if ((int)blockIdx.x >= well_blocks) {
        const int nb = (int)gridDim.x - well_blocks;
        const int h = xcd_block((int)blockIdx.x - well_blocks, nb) * blockDim.x + threadIdx.x;
        if (h < L.half) sweep_item<M, true>(L, C, color, mode, h);
        return;
    }
    const int w = well_wave(), lane = threadIdx.x & 63;
    if (w >= L.nw) return;
    if (color == 0) {
        if (lane == 0) L.xs[w] = read_well<M>(L, C, mode, w);
        return;
    }
    well_sweep_of(L, w, lane, [&](int s) {
        if (s < L.half) return L.x[s];
        return sweep_value<M, true>(L, C, 1, mode, s - L.half);
    });
}

__device__ inline double cell_residual(const AmgLevel &L, int s, const Pos &p) {
    const int stride = 2 * L.half;
    double r = L.b[s] - L.a[s] * L.x[s];
#pragma unroll
    for (int d = 1; d < 7; ++d) {
        int ns;
        const bool in = nbr(L, p, d, ns);
        r -= L.a[(size_t)d * stride + s] * L.x[in ? ns : s];
    }
    for (int q = L.cps[s]; q < L.cps[s + 1]; ++q) {
        const int sl = L.cslot[q];
        r -= L.acw[sl] * L.x[2 * L.half + L.swell[sl]];
    }
    return r;
}

// Restriction (R = P^T): the coarse right-hand side of a coarse cell is
// the sum of the fine residuals r = b - A x over its 2x2x2 aggregate.  A
// group of 8 lanes takes one coarse cell (natural index t): lane q computes
// the residual of child (q & 1, (q >> 1) & 1, q >> 2) and the group's first
// lane adds the existing children in that (k, j, i) order.  Every lane of
// the wave must call it (shuffles); on = false marks lanes past the end.
__device__ inline double restrict_child(const AmgLevel &F, const AmgLevel &C, int t, int q,
                                        bool on, int &have) {
    // a missing child (or a lane past the end) computes the residual of a
    // cell that exists and drops it: no branch before the loads
    const int tc = on ? t : 0;
    const int JK = fdiv(tc, C.mnx), I = tc - JK * C.nx;
    const int K = fdiv(JK, C.mny), J = JK - K * C.ny;
    const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q >> 2);
    have = on && i < F.nx && j < F.ny && k < F.nz;
    const Pos p = pos_at(F, min(i, F.nx - 1), min(j, F.ny - 1), min(k, F.nz - 1));
    const double r = cell_residual(F, split_pos(F, p), p);
    return have ? r : 0.0;
}

__device__ inline void restrict_sum(const AmgLevel &C, int t, int q, bool on, double r,
                                    int have) {
    const int first = (threadIdx.x & 63) & ~7;
    double sum = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const double rc = __shfl(r, first + c, 64);
        if (__shfl(have, first + c, 64)) sum += rc;
    }
    if (on && q == 0) {
        const int JK = fdiv(t, C.mnx), I = t - JK * C.nx;
        const int K = fdiv(JK, C.mny), J = JK - K * C.ny;
        C.b[split_of(C, I, J, K)] = sum;
    }
}

__device__ inline void restrict_group(const AmgLevel &F, const AmgLevel &C, int t, int q,
                                      bool on) {
    int have;
    const double r = restrict_child(F, C, t, q, on, have);
    restrict_sum(C, t, q, on, r, have);
}

// a well is its own aggregate: its coarse right-hand side is its residual
// (b, the diagonal and x of the row are read with its slots and every lane
// stores the same value, as in well_sweep_item)
__device__ inline void restrict_well(const AmgLevel &F, const AmgLevel &C, int w, int lane) {
    const int f = 2 * F.half + w;
    const double bw = F.b[f], aw = F.aww[w], xw = F.x[f];
    const double sum = well_row_sum(F, w, lane);
    C.b[2 * C.half + w] = bw - aw * xw - sum;
}

// coarse cells (8 lanes each) then wells (one wave each)
__global__ __launch_bounds__(kBlock) void k_amg_restrict(AmgLevel F, AmgLevel C) {
    const int bx = xcd_block(blockIdx.x, gridDim.x);
    const long t8 = (long)bx * blockDim.x + threadIdx.x;
    const long n8 = 8L * C.nx * C.ny * C.nz;
    const int cell_blocks = (int)((n8 + kBlock - 1) / kBlock);
    if (bx < cell_blocks) {
        restrict_group(F, C, (int)(t8 >> 3), (int)(t8 & 7), t8 < n8);
    } else {
        const int w = ((bx - cell_blocks) * kBlock + threadIdx.x) >> 6;
        if (w < F.nw) restrict_well(F, C, w, threadIdx.x & 63);
    }
}

// Restriction on large levels, by row segments: a block takes up to kSegAgg
// aggregates along i of one coarse row (J, K).  Its four waves compute the
// residuals of the segment's fine cells, one fine row (j, k) each, so a
// wave's loads of a stencil array fall on two runs of consecutive entries
// (the two colours) rather than on eight half-lines; the residuals go to
// LDS and each aggregate then sums its existing children in the same
// (k, j, i) order as k_amg_restrict, so the sums are the same bit for bit.
constexpr int kSegAgg = 32;

__global__ __launch_bounds__(kBlock) void k_amg_restrict_rows(AmgLevel F, AmgLevel C, int nseg,
                                                              int cell_blocks) {
    const int bx = xcd_block(blockIdx.x, gridDim.x);
    if (bx >= cell_blocks) {
        const int w = ((bx - cell_blocks) * kBlock + threadIdx.x) >> 6;
        if (w < F.nw) restrict_well(F, C, w, threadIdx.x & 63);
        return;
    }
    __shared__ double rr[4][2 * kSegAgg];
    const int seg = bx % nseg, JK = bx / nseg;
    const int J = JK % C.ny, K = JK / C.ny;
    const int I0 = seg * kSegAgg;
    const int row = threadIdx.x >> 6, li = threadIdx.x & 63;
    const int i = 2 * I0 + li, j = 2 * J + (row & 1), k = 2 * K + (row >> 1);
    const bool have = i < F.nx && j < F.ny && k < F.nz;
    // a lane without a cell computes the residual of the segment's first
    // cell (which always exists) and stores nothing: no branch before the loads
    const Pos p = pos_at(F, have ? i : 2 * I0, have ? j : 2 * J, have ? k : 2 * K);
    const double r = cell_residual(F, split_pos(F, p), p);
    if (have) rr[row][li] = r;
    __syncthreads();
    const int I = I0 + (int)threadIdx.x;
    if (threadIdx.x < kSegAgg && I < C.nx) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int ci = 2 * I + (q & 1), cj = 2 * J + ((q >> 1) & 1), ck = 2 * K + (q >> 2);
            if (ci < F.nx && cj < F.ny && ck < F.nz) sum += rr[q >> 1][2 * threadIdx.x + (q & 1)];
        }
        C.b[split_of(C, I, J, K)] = sum;
    }
}

// x_fine += P x_coarse at fine entry t
__device__ inline void correct_item(const AmgLevel &F, const AmgLevel &C, int t) {
    if (t < 2 * F.half) {
        const Pos p = pos_of(F, t);
        if (p.i >= F.nx) return;
        F.x[t] += C.x[split_of(C, p.i >> 1, p.j >> 1, p.k >> 1)];
    } else if (t < 2 * F.half + F.nw) {
        const int w = t - 2 * F.half;
        F.x[t] += C.x[2 * C.half + w];
    }
}

__global__ __launch_bounds__(kBlock) void k_amg_correct(AmgLevel F, AmgLevel C) {
    correct_item(F, C, xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
}

// The coarse part of a cycle in one workgroup.  Below a few thousand cells
// a level's kernels are pure launch latency, and a W-cycle visits the
// coarse levels many times; here one workgroup walks the phase list the
// host recorded for the sub-cycle rooted at P.lv[0] (the same phases, in
// the same order, as the per-level launches, and the same per-entry
// arithmetic, so the result is bitwise that of the launched cycle).
// Iterates, right-hand sides and the well-slot structure of all its levels
// live in LDS (offsets from the host, per level; the phase list last); the
// root's right-hand side comes in from and its iterate goes back to HBM.
// The stencil coefficients stay in HBM and the L2.  Phases are separated
// by workgroup barriers.
template <class T>
__device__ inline void lds_copy(T *dst, const T *src, int n) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
}

// a colour sweep by the whole workgroup, two entries per thread at a time
// so their loads overlap
template <int M>
__device__ __forceinline__ void sweep_phase(const AmgLevel &F, const AmgLevel &C, int color,
                                            int mode) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int h = tid; h < F.half; h += 2 * nt) {
        const int h2 = h + nt;
        const double v1 = sweep_value<M, false>(F, C, color, mode, h);
        const double v2 = (h2 < F.half) ? sweep_value<M, false>(F, C, color, mode, h2) : 0.0;
        F.x[color * F.half + h] = v1;
        if (h2 < F.half) F.x[color * F.half + h2] = v2;
    }
}

// One phase of the sub-cycle on level F (coarser neighbour C) by the whole
// workgroup.  Inlined once with the coefficients of F in LDS and once with
// them in HBM, so every access has a known address space.
__device__ __forceinline__ void subcycle_phase(int op, const AmgLevel &F, const AmgLevel &C,
                                               const double *Minv, double *rbuf,
                                               const AmgExact *ex = nullptr,
                                               double *xs = nullptr) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nwaves = nt >> 6;
    const int kind = op & 15;
    if (kind == kOpPresmooth) {
        // (one entry per thread at a time: on one CU the clamped second
        // entry of a branch-free pair costs more issue slots than it saves)
        for (int h = tid; h < F.half; h += nt) presmooth_item(F, h);
    } else if (kind == kOpSweep) {
        const int color = (op >> 8) & 1, mode = (op >> 12) & 15;
        switch (mode) {
            case 0: sweep_phase<0>(F, C, color, mode); break;
            case kWellsCorr: sweep_phase<kWellsCorr>(F, C, color, mode); break;
            case kCellsCorr | kWellsCorr: sweep_phase<kCellsCorr | kWellsCorr>(F, C, color, mode); break;
            default: sweep_phase<-1>(F, C, color, mode);
        }
    } else if (kind == kOpWells) {
        for (int w = wave; w < F.nw; w += nwaves) well_sweep_item(F, w, lane);
    } else if (kind == kOpRestrict) {
        // The fine residuals in split order first (the stencil loads of a
        // wave are then contiguous; by aggregate every child's loads fall
        // on lines of their own), into rbuf; then every coarse cell sums
        // its children from there in the (k, j, i) order of the per-level
        // launch, so the sums are the same bit for bit.
        for (int s = tid; s < 2 * F.half; s += 2 * nt) {
            const int s2 = s + nt;
            const Pos p1 = pos_of(F, s);
            const double c1 = cell_residual(F, s, p1);
            double r2 = 0.0;
            if (s2 < 2 * F.half) {
                const Pos p2 = pos_of(F, s2);
                const double c2 = cell_residual(F, s2, p2);
                r2 = p2.i >= F.nx ? 0.0 : c2;
            }
            rbuf[s] = p1.i >= F.nx ? 0.0 : c1;
            if (s2 < 2 * F.half) rbuf[s2] = r2;
        }
        __syncthreads();
        const int nc = C.nx * C.ny * C.nz;
        for (int t = tid; t < nc; t += nt) {
            const int JK = fdiv(t, C.mnx), I = t - JK * C.nx;
            const int K = fdiv(JK, C.mny), J = JK - K * C.ny;
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i = 2 * I + (q & 1), j = 2 * J + ((q >> 1) & 1), k = 2 * K + (q >> 2);
                if (i < F.nx && j < F.ny && k < F.nz) sum += rbuf[split_pos(F, pos_at(F, i, j, k))];
            }
            C.b[split_of(C, I, J, K)] = sum;
        }
        for (int w = wave; w < F.nw; w += nwaves) restrict_well(F, C, w, lane);
    } else if (kind == kOpCorrect) {
        for (int t = tid; t < 2 * F.half + F.nw; t += nt) correct_item(F, C, t);
    } else if (ex) {
        exact_solve_wg(F, *ex, xs);
    } else {
        const int n = 2 * F.half + F.nw;
        for (int row = tid; row < n; row += nt) F.x[row] = dense_row(n, Minv, F.b, row);
    }
}

__global__ __launch_bounds__(kSubThreads) void k_amg_subcycle(AmgSub P) {
    extern __shared__ double lds[];
    int *ldi = reinterpret_cast<int *>(lds + P.ldoubles);
    const int tid = threadIdx.x;
    // Stage the image: the levels' iterates, right-hand sides (the root's
    // written there by the launch before, padded entries zero), well-slot
    // structure, the stencils and dense inverse that fit and the phase list
    // live in HBM laid out as here.  Every thread issues all its loads
    // before its first store.
    {
        constexpr int U = 8;
        uint4 *l16 = reinterpret_cast<uint4 *>(lds);
        const int nt = blockDim.x;
        for (int base = 0; base < P.img_n16; base += U * nt) {
            uint4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = base + u * nt + tid;
                v[u] = P.img[e < P.img_n16 ? e : 0];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = base + u * nt + tid;
                if (e < P.img_n16) l16[e] = v[u];
            }
        }
    }
    const int *ops = ldi + P.opsoff;
    double *rbuf = lds + P.rbufoff;                  // fine residuals of a restriction
    __syncthreads();
    auto level = [&](int k) {
        AmgLevel L = P.lv[k];
        L.x = lds + P.off[k][kSubX];
        L.b = lds + P.off[k][kSubB];
        L.acw = lds + P.off[k][kSubAcw];
        L.awc = lds + P.off[k][kSubAwc];
        L.cps = ldi + P.off[k][kSubCps];
        L.cslot = ldi + P.off[k][kSubCslot];
        L.swell = ldi + P.off[k][kSubSwell];
        L.scell = ldi + P.off[k][kSubScell];
        L.sps = ldi + P.off[k][kSubSps];
        return L;
    };
    for (int o = 0; o < P.nops; ++o) {
        const int op = __builtin_amdgcn_readfirstlane(ops[o]);
        const int l = (op >> 4) & 15;
        const AmgLevel C = level(l + 1);
        if ((op & 15) == kOpCoarse) {
            const AmgLevel F = level(l);
            if (P.minvoff >= 0) subcycle_phase(op, F, C, lds + P.minvoff, rbuf);
            else subcycle_phase(op, F, C, P.Minv, rbuf);
        } else if (P.off[l][kSubA] >= 0) {
            AmgLevel F = level(l);
            F.a = lds + P.off[l][kSubA];
            subcycle_phase(op, F, C, P.Minv, rbuf);
        } else {
            subcycle_phase(op, level(l), C, P.Minv, rbuf);
        }
        __syncthreads();
    }
    const AmgLevel &R = P.lv[0];
    for (int e = tid; e < 2 * R.half + R.nw; e += blockDim.x) R.x[e] = lds[P.off[0][kSubX] + e];
}

// ---------------------------------------------------------------------------
// CPR stage kernels

// v = w / h (the new Arnoldi vector; h = 1 without hptr; stored when v is
// given, in v's precision) and the pressure right-hand side b_p = W^T v of
// the first level.
template <int NB, class WT, class VT>
__device__ __forceinline__ void cpr_restrict_body(int bid, int n, int nw, const AmgLevel &L,
                                                  const int *__restrict__ split0,
                                                  const WT *__restrict__ w,
                                                  const double *__restrict__ hptr,
                                                  VT *__restrict__ v,
                                                  const double *__restrict__ wq) {
    const int r = bid * blockDim.x + threadIdx.x;
    if (r >= n + nw) return;
    // the weights and the split index are loaded with w (a well row loads
    // those of the last cell and does not use them: no branch before the
    // loads); n >= 1
    const int rc = r < n ? r : n - 1;
    double we[NB], q[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        we[e] = (double)w[(size_t)r * NB + e];
        q[e] = wq[(size_t)rc * NB + e];
    }
    const int sp = split0[rc];
    bool zero = false;
    double h = 1.0;
    if (hptr) {
        h = *hptr;
        zero = !(h > 0.0 && isfinite(h));
    }
    double a[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        a[e] = zero ? 0.0 : (hptr ? we[e] / h : we[e]);
        if (v) v[(size_t)r * NB + e] = (VT)a[e];
    }
    if (r < n) {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < NB; ++e) s += q[e] * a[e];
        L.b[sp] = s;
    } else {
        L.b[2 * L.half + (r - n)] = a[0];
    }
}

template <int NB, class WT, class VT>
__global__ __launch_bounds__(kBlock) void k_cpr_restrict(int n, int nw, AmgLevel L,
                                                         const int *__restrict__ split0,
                                                         const WT *__restrict__ w,
                                                         const double *__restrict__ hptr,
                                                         VT *__restrict__ v,
                                                         const double *__restrict__ wq) {
    cpr_restrict_body<NB, WT, VT>(blockIdx.x, n, nw, L, split0, w, hptr, v, wq);
}

// z = x1 + D^-1 (v - A x1), x1 = the pressure correction in the pressure
// slot of every row.  A x1 needs only the pressure column of each block,
// read from its compact copy ap[q][NB], with the column indices mapped to
// level-0 AMG entries (colsplit); a group of G lanes walks one block row as
// in the SpMV.
template <int NB, int G>
__global__ __launch_bounds__(kBlock) void k_cpr_finish(int n, int nw, AmgLevel L,
                                                       const int *__restrict__ split0,
                                                       const int *__restrict__ colsplit, Sys sys,
                                                       const double *__restrict__ ap,
                                                       const double *__restrict__ v,
                                                       const double *__restrict__ dinv,
                                                       double *__restrict__ z) {
    const int lg = threadIdx.x & (G - 1);
    const long blk = xcd_block(blockIdx.x, gridDim.x);
    const int r = (int)((blk * blockDim.x + threadIdx.x) / G);
    const int nrows = n + nw;
    auto xp = [&](int col) -> double {
        return col < n ? L.x[split0[col]] : L.x[2 * L.half + (col - n)];
    };
    double t[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) t[e] = 0.0;
    if (r < nrows) {
        const int b = sys.rowptr[r], e = sys.rowptr[r + 1];
        for (int q = b + lg; q < e; q += G) {
            const double p = L.x[__builtin_nontemporal_load(colsplit + q)];
            const double *col = ap + (size_t)q * NB;
#pragma unroll
            for (int u = 0; u < NB; ++u) t[u] += __builtin_nontemporal_load(col + u) * p;
        }
    }
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1)
#pragma unroll
        for (int u = 0; u < NB; ++u) t[u] += __shfl_xor(t[u], off, 64);
    if (r >= nrows || lg != 0) return;
    double res[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) res[u] = v[(size_t)r * NB + u] - t[u];
    const double *m = dinv + (size_t)r * NB * NB;
    const double pr = xp(r);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        double s = (u == 0) ? pr : 0.0;
#pragma unroll
        for (int e2 = 0; e2 < NB; ++e2) s += m[u * NB + e2] * res[e2];
        z[(size_t)r * NB + u] = s;
    }
}

// ---------------------------------------------------------------------------
// launchers

static inline dim3 grid_for(long n, int bs) { return dim3((unsigned)((n + bs - 1) / bs)); }

template <class LT>
static void extract_impl(hipStream_t s, int nb, const AmgLevel &L, Grid g, Wells w, Sys sys,
                         double *wq, LT *ap) {
    const long n = (long)g.n + L.nw;
    if (nb == 2)
        hipLaunchKernelGGL((k_amg_extract<2, LT>), grid_for(8 * n, kBlock), dim3(kBlock), 0, s, L, g,
                           w, sys, wq, ap);
    else
        hipLaunchKernelGGL((k_amg_extract<3, LT>), grid_for(8 * n, kBlock), dim3(kBlock), 0, s, L, g,
                           w, sys, wq, ap);
}

void launch_amg_extract(hipStream_t s, int nb, const AmgLevel &L, Grid g, Wells w, Sys sys,
                        double *wq, double *ap) {
    extract_impl(s, nb, L, g, w, sys, wq, ap);
}

void launch_cprT_extract(hipStream_t s, int nb, const AmgLevel &L, Grid g, Wells w, Sys sysT,
                         double *wq, double *ap) {
    const long n = (long)g.n + L.nw;
    if (nb == 2) {
        hipLaunchKernelGGL(k_cprT_weights<2>, grid_for(g.n, kBlock), dim3(kBlock), 0, s, g.n, sysT, wq);
        hipLaunchKernelGGL(k_cprT_extract<2>, grid_for(n, kBlock), dim3(kBlock), 0, s, L, g, w, sysT,
                           wq, ap);
    } else {
        hipLaunchKernelGGL(k_cprT_weights<3>, grid_for(g.n, kBlock), dim3(kBlock), 0, s, g.n, sysT, wq);
        hipLaunchKernelGGL(k_cprT_extract<3>, grid_for(n, kBlock), dim3(kBlock), 0, s, L, g, w, sysT,
                           wq, ap);
    }
}

void launch_amg_extract(hipStream_t s, int nb, const AmgLevel &L, Grid g, Wells w, Sys sys,
                        double *wq, float *ap) {
    extract_impl(s, nb, L, g, w, sys, wq, ap);
}

void launch_amg_coarsen(hipStream_t s, const AmgLevel &F, const AmgLevel &C, const int *cfs_ptr,
                        const int *cfs_idx) {
    const long n = 2L * C.half + C.nslot + C.nw;
    hipLaunchKernelGGL(k_amg_coarsen, grid_for(n, kBlock), dim3(kBlock), 0, s, F, C, cfs_ptr, cfs_idx);
}

void launch_amg_coarsest_setup(hipStream_t s, const AmgLevel &L, double *M, double *Minv,
                               double *colk, int *bad) {
    const int n = 2 * L.half + L.nw;
    hipLaunchKernelGGL(k_amg_dense, grid_for(n, 64), dim3(64), 0, s, L, M);
    if (n <= kDenseLds)
        hipLaunchKernelGGL(k_dense_invert_lds, dim3(1), dim3(1024), dense_lds_bytes(n), s, n, M, Minv,
                           bad);
    else
        hipLaunchKernelGGL(k_dense_invert, dim3(1), dim3(1024), 0, s, n, M, Minv, colk, bad);
}

hipError_t dense_allow_lds() {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_dense_invert_lds),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)dense_lds_bytes(kDenseLds));
}

void launch_amg_coarsest_solve(hipStream_t s, const AmgLevel &L, const double *Minv) {
    const int n = 2 * L.half + L.nw;
    hipLaunchKernelGGL(k_dense_gemv, grid_for((long)n, 256), dim3(256), 0, s, n, Minv, L.b, L.x);
}

// blocks of the wells (one wave each, rounded up to whole XCD rounds),
// then those of the cells
static inline int well_blocks_of(const AmgLevel &L) {
    const int wb = (int)((64L * L.nw + kBlock - 1) / kBlock);
    return (wb + kXcds - 1) / kXcds * kXcds;
}
static inline dim3 smooth_grid(const AmgLevel &L) {
    return dim3((unsigned)(well_blocks_of(L) + (L.half + kBlock - 1) / kBlock));
}

size_t exact_solve_lds(const AmgExact &E) {
    return ((size_t)E.nslab * E.mmax + E.mmax + 3 * (size_t)E.nslab * E.ncs + (E.nslab + 2) / 2) *
           sizeof(double);
}
size_t exact_factor_lds(const AmgExact &E) {
    return ((size_t)E.mmax * E.mmax + 8 * E.mmax) * sizeof(double);
}

// the largest LDS of a slab problem the plan admits (nslab * mmax <=
// kExactSlabDoubles, ncs <= mmax <= kSlabMax), which every context shares
static size_t exact_factor_lds_max() {
    return ((size_t)kSlabMax * kSlabMax + 8 * kSlabMax) * sizeof(double);
}
static size_t exact_solve_lds_max() {
    return ((size_t)4 * kExactSlabDoubles + kSlabMax + (kExactSlabDoubles + 2) / 2) * sizeof(double);
}

hipError_t exact_allow_lds() {
    for (const void *k : {reinterpret_cast<const void *>(&k_amg_exact_factor),
                          reinterpret_cast<const void *>(&k_amg_exact_factor2),
                          reinterpret_cast<const void *>(&k_amg_exact_twist)}) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)exact_factor_lds_max());
        if (e != hipSuccess) return e;
    }
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_amg_exact_solve),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)exact_solve_lds_max());
}

// One-sided (for the substitution, which reads inv(D_b) of every slab), or
// with X two-sided: both sides at once, then the twist.
void launch_amg_exact_factor(hipStream_t s, const AmgLevel &L, const AmgExact &E) {
    if (!E.X) {
        hipLaunchKernelGGL(k_amg_exact_factor, dim3(1), dim3(1024), exact_factor_lds(E), s, L, E);
        return;
    }
    hipLaunchKernelGGL(k_amg_exact_factor2, dim3(2), dim3(1024), exact_factor_lds(E), s, L, E);
    hipLaunchKernelGGL(k_amg_exact_twist, dim3(1), dim3(1024), exact_factor_lds(E), s, L, E);
}

void launch_amg_exact_solve(hipStream_t s, const AmgLevel &L, const AmgExact &E) {
    hipLaunchKernelGGL(k_amg_exact_solve, dim3(1), dim3(1024), exact_solve_lds(E), s, L, E);
}

void launch_amg_exact_inverse(hipStream_t s, const AmgLevel &L, const AmgExact &E) {
    const int groups = (E.mmax + kInvCols - 1) / kInvCols;
    hipLaunchKernelGGL(k_amg_exact_inverse, dim3((unsigned)(E.nslab * groups)),
                       dim3(kInvCols * kSlabMax), 0, s, L, E);
}

void launch_amg_exact_gemv(hipStream_t s, const AmgLevel &L, const AmgExact &E) {
    hipLaunchKernelGGL(k_amg_exact_gemv, dim3((unsigned)((E.nst + kGemvRows - 1) / kGemvRows)),
                       dim3(64 * kGemvRows), (size_t)E.ldx * sizeof(double), s, L, E);
}

void launch_amg_sweep(hipStream_t s, const AmgLevel &L, const AmgLevel &C, int color, int mode) {
    // colour 1 reads the wells from the snapshot the colour-0 sweep took
    if (color == 1) mode |= kWellsSnap;
    const dim3 grid = smooth_grid(L), block(kBlock);
    const int cb = well_blocks_of(L);
    switch (mode) {
        case kCellsCorr | kWellsCorr:
            hipLaunchKernelGGL(k_amg_sweep<kCellsCorr | kWellsCorr>, grid, block, 0, s, L, C,
                               color, mode, cb);
            break;
        case kWellsCorr | kWellsSnap:
            hipLaunchKernelGGL(k_amg_sweep<kWellsCorr | kWellsSnap>, grid, block, 0, s, L, C,
                               color, mode, cb);
            break;
        case 0:
            hipLaunchKernelGGL(k_amg_sweep<0>, grid, block, 0, s, L, C, color, mode, cb);
            break;
        case kWellsSnap:
            hipLaunchKernelGGL(k_amg_sweep<kWellsSnap>, grid, block, 0, s, L, C, color, mode, cb);
            break;
        default:
            hipLaunchKernelGGL(k_amg_sweep<-1>, grid, block, 0, s, L, C, color, mode, cb);
    }
}

void launch_amg_presmooth(hipStream_t s, const AmgLevel &L) {
    hipLaunchKernelGGL(k_amg_presmooth, smooth_grid(L), dim3(kBlock), 0, s, L, well_blocks_of(L));
}

void launch_amg_restrict(hipStream_t s, const AmgLevel &F, const AmgLevel &C, long seg_min) {
    if (seg_min > 0 && F.half >= seg_min) {
        const int nseg = (C.nx + kSegAgg - 1) / kSegAgg;
        const long cell_blocks = (long)nseg * C.ny * C.nz;
        const long well_blocks = (64L * F.nw + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_amg_restrict_rows, dim3((unsigned)(cell_blocks + well_blocks)),
                           dim3(kBlock), 0, s, F, C, nseg, (int)cell_blocks);
        return;
    }
    const long cell_blocks = (8L * C.nx * C.ny * C.nz + kBlock - 1) / kBlock;
    const long well_blocks = (64L * F.nw + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_amg_restrict, dim3((unsigned)(cell_blocks + well_blocks)), dim3(kBlock), 0,
                       s, F, C);
}

// rounded up to whole 16-byte units: the prologue stages the image in those
size_t amg_subcycle_lds(const AmgSub &P) {
    const size_t b = (size_t)P.ldoubles * sizeof(double) + ((size_t)P.opsoff + P.nops) * sizeof(int);
    return (b + 15) & ~(size_t)15;
}

hipError_t amg_subcycle_allow_lds(size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_amg_subcycle),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_amg_subcycle(hipStream_t s, const AmgSub &P) {
    hipLaunchKernelGGL(k_amg_subcycle, dim3(1), dim3(kSubThreads), amg_subcycle_lds(P), s, P);
}

void launch_amg_correct(hipStream_t s, const AmgLevel &F, const AmgLevel &C) {
    hipLaunchKernelGGL(k_amg_correct, grid_for(2L * F.half + F.nw, kBlock), dim3(kBlock), 0, s, F, C);
}

template <class WT, class VT>
static void restrict_impl(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                          const int *split0, const WT *w, const double *hptr, VT *v,
                          const double *wq) {
    const long rows = (long)n + nw;
    if (nb == 2)
        hipLaunchKernelGGL((k_cpr_restrict<2, WT, VT>), grid_for(rows, kBlock), dim3(kBlock), 0, s, n,
                           nw, L, split0, w, hptr, v, wq);
    else
        hipLaunchKernelGGL((k_cpr_restrict<3, WT, VT>), grid_for(rows, kBlock), dim3(kBlock), 0, s, n,
                           nw, L, split0, w, hptr, v, wq);
}

void launch_cpr_restrict(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                         const int *split0, const double *w, const double *hptr, double *v,
                         const double *wq) {
    restrict_impl(s, nb, n, nw, L, split0, w, hptr, v, wq);
}

void launch_cpr_restrict(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                         const int *split0, const double *w, const double *hptr, float *v,
                         const double *wq) {
    restrict_impl(s, nb, n, nw, L, split0, w, hptr, v, wq);
}

void launch_cpr_restrict(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                         const int *split0, const float *w, const double *hptr, float *v,
                         const double *wq) {
    restrict_impl(s, nb, n, nw, L, split0, w, hptr, v, wq);
}

void launch_cpr_finish(hipStream_t s, int nb, int n, int nw, const AmgLevel &L,
                       const int *split0, const int *colsplit, Sys sys, const double *ap,
                       const double *v, const double *dinv, double *z) {
    constexpr int G = 8;
    const long threads = ((long)n + nw) * G;
    if (nb == 2)
        hipLaunchKernelGGL((k_cpr_finish<2, G>), grid_for(threads, kBlock), dim3(kBlock), 0, s, n,
                           nw, L, split0, colsplit, sys, ap, v, dinv, z);
    else
        hipLaunchKernelGGL((k_cpr_finish<3, G>), grid_for(threads, kBlock), dim3(kBlock), 0, s, n,
                           nw, L, split0, colsplit, sys, ap, v, dinv, z);
}

// ---------------------------------------------------------------------------
// batched launches over the members of an ensemble

template <int NB>
__global__ __launch_bounds__(kBlock) void kb_amg_extract(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    amg_extract_body<NB, double>(b, nb, M.lv[0], M.g, M.wells, M.sys, M.wq, M.ap);
}

__global__ __launch_bounds__(kBlock) void kb_amg_coarsen(const Member *__restrict__ mem, Batch B,
                                                         int l) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    if (l >= M.nlev) return;
    amg_coarsen_body(b, M.lv[l - 1], M.lv[l], M.cfs_ptr[l], M.cfs_idx[l]);
}

// the dense matrix of the member's coarsest level and its inverse, by one
// workgroup (the rows by the threads, then the Gauss-Jordan elimination in
// LDS of the single-member launch)
__global__ __launch_bounds__(1024) void kb_amg_coarsest(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    const AmgLevel &L = M.lv[M.nlev - 1];
    extern __shared__ double sm[];
    if (M.exact) {
        exact_factor_wg(L, M.ex, sm, 0, M.ex.nslab, 1);
        return;
    }
    const int n = 2 * L.half + L.nw;
    for (int t = threadIdx.x; t < n; t += blockDim.x) amg_dense_row(L, M.Mden, t);
    __syncthreads();
    dense_invert_lds_body(n, M.Mden, M.Minv, M.amg_bad, sm);
}

// the first CPR stage's restriction: of the first vector of a restart
// cycle (j < 0: b / ||b|| in the first cycle, r / ||r|| after it) or of the
// new Arnoldi vector w / h_{j+1,j} (j >= 0), stored in V
template <int NB>
__global__ __launch_bounds__(kBlock) void kb_cpr_restrict(const Member *__restrict__ mem, Batch B,
                                                          int j, int first_bit, int s_norm,
                                                          int s_res) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    const double *w;
    const double *h;
    double *v;
    if (j < 0) {
        const bool first = (B.flags[m] & first_bit) != 0;
        w = first ? M.sys.R : M.r;
        h = M.scal + (first ? s_norm : s_res) + 1;
        v = M.V;
    } else {
        w = M.w;
        h = M.H + (size_t)j * (kMaxRestart + 2) + j + 1;
        v = M.V + (size_t)(j + 1) * M.nvec;
    }
    cpr_restrict_body<NB, double, double>(b, M.n, M.nw, M.lv[0], M.split0, w, h, v, M.wq);
}

// The member's whole AMG cycle by one workgroup, its phase list walked
// with every level's arrays in HBM (the phases and per-entry arithmetic of
// the per-level launches, so the result is bit for bit theirs).
__global__ __launch_bounds__(kSubThreads) void kb_amg_cycle(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    extern __shared__ double xs[];               // the slab solve's vectors
    for (int o = 0; o < M.nops; ++o) {
        const int op = __builtin_amdgcn_readfirstlane(M.ops[o]);
        const int l = (op >> 4) & 15;
        subcycle_phase(op, M.lv[l], M.lv[l + 1], M.Minv, M.rbuf, M.exact ? &M.ex : nullptr, xs);
        __syncthreads();
    }
}

void launchb_amg_extract(hipStream_t s, int nb, const Member *mem, Batch B, int total) {
    if (total <= 0) return;
    if (nb == 2) hipLaunchKernelGGL(kb_amg_extract<2>, dim3(total), dim3(kBlock), 0, s, mem, B);
    else hipLaunchKernelGGL(kb_amg_extract<3>, dim3(total), dim3(kBlock), 0, s, mem, B);
}

void launchb_amg_coarsen(hipStream_t s, const Member *mem, Batch B, int total, int level) {
    if (total > 0)
        hipLaunchKernelGGL(kb_amg_coarsen, dim3(total), dim3(kBlock), 0, s, mem, B, level);
}

void launchb_amg_coarsest(hipStream_t s, const Member *mem, Batch one, int tone, int nmax,
                          size_t exact_lds) {
    if (tone > 0)
        hipLaunchKernelGGL(kb_amg_coarsest, dim3(tone), dim3(1024),
                           std::max(dense_lds_bytes(nmax), exact_lds), s, mem, one);
}

hipError_t batch_allow_lds() {
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&kb_amg_coarsest), hipFuncAttributeMaxDynamicSharedMemorySize,
        (int)std::max(dense_lds_bytes(kDenseLds), exact_factor_lds_max()));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&kb_amg_cycle),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)exact_solve_lds_max());
}

int dense_lds_max() { return kDenseLds; }

void launchb_cpr_restrict(hipStream_t s, int nb, const Member *mem, Batch B, int total, int j,
                          int first_bit, int s_norm, int s_res) {
    if (total <= 0) return;
    if (nb == 2)
        hipLaunchKernelGGL(kb_cpr_restrict<2>, dim3(total), dim3(kBlock), 0, s, mem, B, j,
                           first_bit, s_norm, s_res);
    else
        hipLaunchKernelGGL(kb_cpr_restrict<3>, dim3(total), dim3(kBlock), 0, s, mem, B, j,
                           first_bit, s_norm, s_res);
}

void launchb_amg_cycle(hipStream_t s, const Member *mem, Batch one, int tone, size_t exact_lds) {
    if (tone > 0)
        hipLaunchKernelGGL(kb_amg_cycle, dim3(tone), dim3(kSubThreads), exact_lds, s, mem, one);
}

}  // namespace fim
