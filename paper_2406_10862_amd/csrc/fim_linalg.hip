// fim_linalg.hip - BSR SpMV, block-Jacobi preconditioner and the vector
// kernels of right-preconditioned GMRES (paper Sec. 5.1: FGMRES with
// block-Jacobi smoothing; Sec. 3.3.3: the solve returns the solution and
// the iteration count).
//
// Everything here streams HBM: SpMV assigns a group of G lanes to one block
// row so consecutive lanes read consecutive blocks (coalesced) while the
// matrix values and indices, read once, bypass the caches (non-temporal)
// and the gathered vector stays cached.  The orthogonalisation kernels read
// each basis vector once per pass with all dot products of a pass
// accumulated in registers.
#include <math.h>

#include <hip/hip_ext.h>

#include "fim_internal.h"
#include "fim_reduce.h"
#include "fim_block.h"

namespace fim {

typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kMaxDots = kMaxRestart + 1;   // basis vectors + the vector itself

// ---------------------------------------------------------------------------
// y = A x, canonical BSR.  A group of G lanes owns R block rows, spaced one
// wave's worth of groups apart so that, for each of its R rows, the lanes of
// a wave read one contiguous run of the value and index arrays; lane lg
// takes block rowptr[row] + lg.  The loads of all R rows are issued before
// any of them is used (row pointers, then indices and blocks, then x), so a
// wave keeps R times the bytes of a single row in flight through the same
// three dependent steps; rows with more than G blocks (well rows) finish in
// a second loop.  The matrix arrays use ordinary loads: between the Krylov
// steps of a restart cycle part of the matrix still sits in the MALL.
constexpr int kSpmvG = 8;
template <int NB> struct SpmvRows { static constexpr int R = NB == 2 ? 4 : 2; };

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <int NB, class MT>
__device__ inline void spmv_block(const MT *__restrict__ val, int q, double (&a)[NB * NB]) {
    if constexpr (NB == 2 && sizeof(MT) == 8) {
        const d2 *p = reinterpret_cast<const d2 *>(val + (size_t)q * 4);
        const d2 r0 = p[0], r1 = p[1];
        a[0] = r0.x;
        a[1] = r0.y;
        a[2] = r1.x;
        a[3] = r1.y;
    } else if constexpr (NB == 2) {
        const f4 b4 = *reinterpret_cast<const f4 *>(val + (size_t)q * 4);
        a[0] = b4.x;
        a[1] = b4.y;
        a[2] = b4.z;
        a[3] = b4.w;
    } else {
#pragma unroll
        for (int t = 0; t < NB * NB; ++t) a[t] = val[(size_t)q * NB * NB + t];
    }
}

template <int NB, class VT>
__device__ inline void spmv_x(const VT *__restrict__ x, int c, double (&xv)[NB]) {
    if constexpr (NB == 2 && sizeof(VT) == 8) {
        const d2 v2 = *reinterpret_cast<const d2 *>(x + (size_t)c * 2);
        xv[0] = v2.x;
        xv[1] = v2.y;
    } else if constexpr (NB == 2) {
        const f2 v2 = *reinterpret_cast<const f2 *>(x + (size_t)c * 2);
        xv[0] = v2.x;
        xv[1] = v2.y;
    } else {
#pragma unroll
        for (int t = 0; t < NB; ++t) xv[t] = x[(size_t)c * NB + t];
    }
}

template <int NB>
__device__ inline void spmv_fma(const double (&a)[NB * NB], const double (&xv)[NB],
                                double (&acc)[NB]) {
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        double sum = a[r * NB] * xv[0];
#pragma unroll
        for (int t = 1; t < NB; ++t) sum += a[r * NB + t] * xv[t];
        acc[r] += sum;
    }
}

// what a lane reads when no row of its range holds a block (x[0] is then
// read through column 0: every launch has at least one row)
__device__ __align__(16) double spmv_zero_blk[9] = {};
__device__ int spmv_zero_col[1] = {};

// rows covered by one workgroup
template <int NB, int G>
constexpr int spmv_rows_per_block() { return kBlock / G * SpmvRows<NB>::R; }

// MT / VT: element types of the matrix values and of x, y (double, or float
// for the inner solves of the mixed-precision mode); sums in double.
template <int NB, int G, class MT, class VT>
__global__ __launch_bounds__(kBlock) void k_spmv(int nrows, const int *__restrict__ rowptr,
                                                 const int *__restrict__ colind,
                                                 const MT *__restrict__ val,
                                                 const VT *__restrict__ x,
                                                 VT *__restrict__ y) {
    constexpr int R = SpmvRows<NB>::R;
    constexpr int GPW = 64 / G;             // lane groups per wave
    const int lg = threadIdx.x & (G - 1);
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long row0 = wave * (GPW * R) + ((threadIdx.x & 63) / G);
    // Every lane loads from an address inside the arrays (its own block,
    // else the last block of its row; a lane whose row range ends at 0 reads
    // a zero block of its own) and drops what it should not have read by a
    // select, so the loads are straight-line code with no wait between the
    // rows.  Rows past the end take the empty range at rowptr[nrows].
    int b[R], e[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const long row = row0 + k * GPW;
        const long rc = row < nrows ? row : nrows - 1;
        const int bb = __builtin_nontemporal_load(rowptr + rc);
        const int ee = __builtin_nontemporal_load(rowptr + rc + 1);
        b[k] = row < nrows ? bb : ee;
        e[k] = ee;
    }
    int col[R];
    double a[R][NB * NB];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int q = b[k] + lg;
        const int qs = q < e[k] ? q : e[k] - 1;
        const bool has = e[k] > 0;
        col[k] = *(has ? colind + qs : spmv_zero_col);
        spmv_block<NB>(has ? val : reinterpret_cast<const MT *>(spmv_zero_blk), has ? qs : 0,
                       a[k]);
    }
    double xv[R][NB];
#pragma unroll
    for (int k = 0; k < R; ++k) spmv_x<NB>(x, col[k], xv[k]);
    double acc[R][NB];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const bool ok = b[k] + lg < e[k];
#pragma unroll
        for (int t = 0; t < NB * NB; ++t) a[k][t] = ok ? a[k][t] : 0.0;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            xv[k][t] = ok ? xv[k][t] : 0.0;
            acc[k][t] = 0.0;
        }
        spmv_fma<NB>(a[k], xv[k], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        for (int q = b[k] + lg + G; q < e[k]; q += G) {
            double ab[NB * NB], xb[NB];
            spmv_block<NB>(val, q, ab);
            spmv_x<NB>(x, colind[q], xb);
            spmv_fma<NB>(ab, xb, acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
#pragma unroll
        for (int off = G / 2; off >= 1; off >>= 1)
#pragma unroll
            for (int t = 0; t < NB; ++t) acc[k][t] += __shfl_xor(acc[k][t], off, 64);
    }
    if (lg == 0) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const long row = row0 + k * GPW;
            if (row >= nrows) break;
            if constexpr (NB == 2 && sizeof(VT) == 8) {
                d2 o;
                o.x = acc[k][0];
                o.y = acc[k][1];
                *reinterpret_cast<d2 *>(y + (size_t)row * 2) = o;
            } else {
#pragma unroll
                for (int t = 0; t < NB; ++t) y[(size_t)row * NB + t] = (VT)acc[k][t];
            }
        }
    }
}

// With events e0/e1 the launch records the kernel's own start and end
// timestamps in them (no dispatch gap between a marker and the kernel).
template <class MT, class VT>
static void spmv_impl(hipStream_t s, int nb, int nrows, const int *rowptr, const int *colind,
                      const MT *val, const VT *x, VT *y, hipEvent_t e0, hipEvent_t e1) {
    constexpr int G = kSpmvG;
    const int per = nb == 2 ? spmv_rows_per_block<2, G>() : spmv_rows_per_block<3, G>();
    dim3 grid((unsigned)((nrows + per - 1) / per)), block(kBlock);
    if (e0 || e1) {
        if (nb == 2)
            hipExtLaunchKernelGGL((k_spmv<2, G, MT, VT>), grid, block, 0, s, e0, e1, 0, nrows,
                                  rowptr, colind, val, x, y);
        else
            hipExtLaunchKernelGGL((k_spmv<3, G, MT, VT>), grid, block, 0, s, e0, e1, 0, nrows,
                                  rowptr, colind, val, x, y);
    } else if (nb == 2) {
        hipLaunchKernelGGL((k_spmv<2, G, MT, VT>), grid, block, 0, s, nrows, rowptr, colind, val,
                           x, y);
    } else {
        hipLaunchKernelGGL((k_spmv<3, G, MT, VT>), grid, block, 0, s, nrows, rowptr, colind, val,
                           x, y);
    }
}

void launch_spmv(hipStream_t s, int nb, int nrows, const int *rowptr, const int *colind,
                 const double *val, const double *x, double *y, hipEvent_t e0, hipEvent_t e1) {
    spmv_impl(s, nb, nrows, rowptr, colind, val, x, y, e0, e1);
}

void launch_spmv(hipStream_t s, int nb, int nrows, const int *rowptr, const int *colind,
                 const float *val, const float *x, float *y, hipEvent_t e0, hipEvent_t e1) {
    spmv_impl(s, nb, nrows, rowptr, colind, val, x, y, e0, e1);
}

// ---------------------------------------------------------------------------
// J^T on J's (structurally symmetric) pattern: block q = (r, c) of J^T is
// the transpose of block tperm[q] = (c, r) of J.
template <int NB>
__global__ __launch_bounds__(kBlock) void k_bsr_transpose(long nnzb, const int *__restrict__ tperm,
                                                          const double *__restrict__ val,
                                                          double *__restrict__ valT) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnzb) return;
    const double *src = val + (size_t)tperm[q] * NB * NB;
    double *dst = valT + (size_t)q * NB * NB;
#pragma unroll
    for (int e = 0; e < NB; ++e)
#pragma unroll
        for (int u = 0; u < NB; ++u) dst[e * NB + u] = src[u * NB + e];
}

void launch_bsr_transpose(hipStream_t s, int nb, long nnzb, const int *tperm, const double *val,
                          double *valT) {
    if (nnzb <= 0) return;
    dim3 grid((unsigned)((nnzb + kBlock - 1) / kBlock)), block(kBlock);
    if (nb == 2)
        hipLaunchKernelGGL(k_bsr_transpose<2>, grid, block, 0, s, nnzb, tperm, val, valT);
    else
        hipLaunchKernelGGL(k_bsr_transpose<3>, grid, block, 0, s, nnzb, tperm, val, valT);
}

// ---------------------------------------------------------------------------
// block Jacobi: inverse of each diagonal block


template <int NB>
__global__ __launch_bounds__(kBlock) void k_bj_setup(int nrows, const int *__restrict__ diagpos,
                                                     const double *__restrict__ val,
                                                     double *__restrict__ dinv, int *bad) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double a[NB * NB], inv[NB * NB];
    const double *src = val + (size_t)diagpos[r] * NB * NB;
#pragma unroll
    for (int t = 0; t < NB * NB; ++t) a[t] = src[t];
    if (!invert_block<NB>(a, inv)) {
        atomicOr(bad, 1);
#pragma unroll
        for (int t = 0; t < NB * NB; ++t) inv[t] = (t % (NB + 1) == 0) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int t = 0; t < NB * NB; ++t) dinv[(size_t)r * NB * NB + t] = inv[t];
}

template <int NB>
__device__ inline void apply_block(const double *__restrict__ dinv, int r, const double (&v)[NB],
                                   double (&z)[NB]) {
    const double *m = dinv + (size_t)r * NB * NB;
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < NB; ++u) s += m[e * NB + u] * v[u];
        z[e] = s;
    }
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_bj_apply(int nrows, const double *__restrict__ dinv,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ y) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    double v[NB], z[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) v[e] = x[(size_t)r * NB + e];
    apply_block<NB>(dinv, r, v, z);
#pragma unroll
    for (int e = 0; e < NB; ++e) y[(size_t)r * NB + e] = z[e];
}

void launch_bj_setup(hipStream_t s, int nb, int nrows, const int *diagpos, const double *val,
                     double *dinv, int *bad) {
    dim3 grid((nrows + kBlock - 1) / kBlock), block(kBlock);
    if (nb == 2) hipLaunchKernelGGL(k_bj_setup<2>, grid, block, 0, s, nrows, diagpos, val, dinv, bad);
    else hipLaunchKernelGGL(k_bj_setup<3>, grid, block, 0, s, nrows, diagpos, val, dinv, bad);
}

void launch_bj_apply(hipStream_t s, int nb, int nrows, const double *dinv, const double *x,
                     double *y) {
    dim3 grid((nrows + kBlock - 1) / kBlock), block(kBlock);
    if (nb == 2) hipLaunchKernelGGL(k_bj_apply<2>, grid, block, 0, s, nrows, dinv, x, y);
    else hipLaunchKernelGGL(k_bj_apply<3>, grid, block, 0, s, nrows, dinv, x, y);
}

// ---------------------------------------------------------------------------
// Krylov vector kernels.  Grids are capped at 2048 blocks (8 per CU) so the
// per-block partials of a reduction stay few; every thread walks the vector
// with a grid stride.

int vec_blocks(long nvec) {
    long b = (nvec + kBlock - 1) / kBlock;
    return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

// out[0] = sum of the partials, out[1] = its square root (a norm finish)
__global__ __launch_bounds__(kBlock) void k_finish_norm(int nparts, const double *partials,
                                                        double *out) {
    const bool mx[1] = {false};
    double a[1];
    finish_partials<1>(nparts, mx, partials, a);
    if (threadIdx.x == 0) {
        out[0] = a[0];
        out[1] = sqrt(a[0]);
    }
}

// out[0] = ||x||^2, out[1] = ||x||
__global__ __launch_bounds__(kBlock) void k_norm2(long nvec, const double *__restrict__ x,
                                                  double *partials) {
    double v[1] = {0.0};
    const bool mx[1] = {false};
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nvec;
         i += (long)gridDim.x * blockDim.x) {
        const double a = x[i];
        v[0] += a * a;
    }
    block_partials<1>(v, mx, partials);
}

void launch_norm2(hipStream_t s, long nvec, const double *x, double *partials, double *out) {
    const int nblk = vec_blocks(nvec);
    hipLaunchKernelGGL(k_norm2, dim3(nblk), dim3(kBlock), 0, s, nvec, x, partials);
    hipLaunchKernelGGL(k_finish_norm, dim3(1), dim3(kBlock), 0, s, nblk, partials, out);
}

// v = w / h and z = M^-1 v (block Jacobi), one block row per thread.  h is
// read from device memory (h <= 0 or non-finite: zero vectors, the happy
// breakdown of the Arnoldi process).
template <int NB>
__global__ __launch_bounds__(kBlock) void k_normalize_precond(int nrows,
                                                              const double *__restrict__ w,
                                                              const double *__restrict__ hptr,
                                                              double *__restrict__ v,
                                                              double *__restrict__ z,
                                                              const double *__restrict__ dinv) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const double h = *hptr;
    const bool ok = h > 0.0 && isfinite(h);
    double a[NB], b[NB];
#pragma unroll
    for (int e = 0; e < NB; ++e) a[e] = ok ? w[(size_t)r * NB + e] / h : 0.0;
    apply_block<NB>(dinv, r, a, b);
#pragma unroll
    for (int e = 0; e < NB; ++e) {
        v[(size_t)r * NB + e] = a[e];
        z[(size_t)r * NB + e] = b[e];
    }
}

void launch_normalize_precond(hipStream_t s, int nb, int nrows, const double *w,
                              const double *hptr, double *v, double *z, const double *dinv) {
    dim3 grid((nrows + kBlock - 1) / kBlock), block(kBlock);
    if (nb == 2)
        hipLaunchKernelGGL(k_normalize_precond<2>, grid, block, 0, s, nrows, w, hptr, v, z, dinv);
    else
        hipLaunchKernelGGL(k_normalize_precond<3>, grid, block, 0, s, nrows, w, hptr, v, z, dinv);
}

// dst[i] = <V_i, w> for i < nv, dst[nv] = <w, w>, in two kernels.  The
// first runs a (column-block x vector-group) grid: each block accumulates
// kDotGroup dot products over its share of the rows (w is re-read once per
// group from cache) and writes one partial per product; the second sums the
// partials of each product in block order with one workgroup per product.
// Both are skipped when *gate == 0.
constexpr int kDotGroup = 8;
constexpr int kDotCols = 2048;

// The products of one group of NG vectors with w, and <w, w> when self: a
// thread takes U of its grid-stride elements at a time and issues all their
// loads before the first product (an element past the end re-reads the
// thread's first one and is dropped by a select), so even a group of one
// vector keeps several loads in flight.
template <class T, int NG>
__device__ inline void multidot_group(long nvec, const T *__restrict__ V, const T *__restrict__ w,
                                      bool self, double (&acc)[kDotGroup + 1]) {
    constexpr int U = NG <= 2 ? 4 : 2;
    const long S = (long)gridDim.x * blockDim.x;
    for (long e0 = (long)blockIdx.x * blockDim.x + threadIdx.x; e0 < nvec; e0 += U * S) {
        double we[U], v[U][NG];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long e = e0 + u * S < nvec ? e0 + u * S : e0;
            we[u] = (double)w[e];
#pragma unroll
            for (int i = 0; i < NG; ++i)
                v[u][i] = (double)__builtin_nontemporal_load(V + (size_t)i * nvec + e);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double wu = e0 + u * S < nvec ? we[u] : 0.0;
#pragma unroll
            for (int i = 0; i < NG; ++i) acc[i] += v[u][i] * wu;
            if (self) acc[kDotGroup] += wu * wu;
        }
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_multidot_part(long nvec, int nv,
                                                          const T *__restrict__ V,
                                                          const T *__restrict__ w,
                                                          double *__restrict__ partials,
                                                          const int *gate) {
    if (gate && *gate == 0) return;
    const int g0 = blockIdx.y * kDotGroup;
    const int ng = min(kDotGroup, nv - g0);
    double acc[kDotGroup + 1];
#pragma unroll
    for (int i = 0; i <= kDotGroup; ++i) acc[i] = 0.0;
    const bool self = blockIdx.y == 0;            // the first group also forms <w, w>
    const T *Vg = V + (size_t)g0 * nvec;
    switch (ng) {
    case 1: multidot_group<T, 1>(nvec, Vg, w, self, acc); break;
    case 2: multidot_group<T, 2>(nvec, Vg, w, self, acc); break;
    case 3: multidot_group<T, 3>(nvec, Vg, w, self, acc); break;
    case 4: multidot_group<T, 4>(nvec, Vg, w, self, acc); break;
    case 5: multidot_group<T, 5>(nvec, Vg, w, self, acc); break;
    case 6: multidot_group<T, 6>(nvec, Vg, w, self, acc); break;
    case 7: multidot_group<T, 7>(nvec, Vg, w, self, acc); break;
    default: multidot_group<T, kDotGroup>(nvec, Vg, w, self, acc); break;
    }
    __shared__ double sh[kDotGroup + 1][kWaves];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i <= kDotGroup; ++i) {
        if (i < ng || (i == kDotGroup && self)) {
            double a = acc[i];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
            if (lane == 0) sh[i][wid] = a;
        }
    }
    __syncthreads();
    if (threadIdx.x <= kDotGroup) {
        const int i = threadIdx.x;
        if ((i < kDotGroup && i < ng) || (i == kDotGroup && self)) {
            double a = sh[i][0];
            for (int w2 = 1; w2 < kWaves; ++w2) a += sh[i][w2];
            const int slot = (i < kDotGroup) ? g0 + i : nv;
            partials[(size_t)slot * gridDim.x + blockIdx.x] = a;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_multidot_sum(int ncols, const double *__restrict__ partials,
                                                         double *__restrict__ dst, const int *gate) {
    if (gate && *gate == 0) return;
    const int slot = blockIdx.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < ncols; b += blockDim.x) a += partials[(size_t)slot * ncols + b];
    __shared__ double sh[kWaves];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sh[0];
        for (int w2 = 1; w2 < kWaves; ++w2) t += sh[w2];
        dst[slot] = t;
    }
}

template <class T>
static void multidot_impl(hipStream_t s, long nvec, int nv, const T *V, const T *w,
                          double *partials, double *dst, const int *gate) {
    long cols = (nvec + kBlock - 1) / kBlock;
    cols = cols < kDotCols ? (cols > 0 ? cols : 1) : kDotCols;
    const int groups = (nv + kDotGroup - 1) / kDotGroup > 0 ? (nv + kDotGroup - 1) / kDotGroup : 1;
    hipLaunchKernelGGL(k_multidot_part<T>, dim3((unsigned)cols, groups), dim3(kBlock), 0, s, nvec,
                       nv, V, w, partials, gate);
    hipLaunchKernelGGL(k_multidot_sum, dim3(nv + 1), dim3(kBlock), 0, s, (int)cols, partials, dst,
                       gate);
}

void launch_multidot(hipStream_t s, long nvec, int nv, const double *V, const double *w,
                     double *partials, double *dst, const int *gate) {
    multidot_impl(s, nvec, nv, V, w, partials, dst, gate);
}

void launch_multidot(hipStream_t s, long nvec, int nv, const float *V, const float *w,
                     double *partials, double *dst, const int *gate) {
    multidot_impl(s, nvec, nv, V, w, partials, dst, gate);
}

// w -= sum_{i<nv} coef[i] V_i and the partials of ||w||^2.  The finishing
// kernel then sets hnext = ||w||; when hacc is set (second Gram-Schmidt
// pass) hacc[i] += coef[i]; when reorth is set (first pass) it becomes 1 if
// the norm dropped below a tenth of ||w_before|| = sqrt(coef[nv]) (a
// DGKS-type test for severe cancellation).  Both are skipped when
// *gate == 0.
template <class T>
__global__ __launch_bounds__(kBlock) void k_update_norm(long nvec, int nv,
                                                        const T *__restrict__ V,
                                                        const double *coef, T *w,
                                                        double *partials, const int *gate) {
    if (gate && *gate == 0) return;
    __shared__ double c[kMaxDots];
    for (int i = threadIdx.x; i <= nv; i += blockDim.x) c[i] = coef[i];
    __syncthreads();
    double v[1] = {0.0};
    const bool mx[1] = {false};
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nvec;
         e += (long)gridDim.x * blockDim.x) {
        double a = (double)w[e];
#pragma unroll 8
        for (int i = 0; i < nv; ++i)
            a -= c[i] * (double)__builtin_nontemporal_load(V + (size_t)i * nvec + e);
        const T at = (T)a;                         // the norm of what is stored
        w[e] = at;
        v[0] += (double)at * (double)at;
    }
    block_partials<1>(v, mx, partials);
}

__global__ __launch_bounds__(kBlock) void k_update_finish(int nparts, int nv, const double *coef,
                                                          const double *partials, double *hnext,
                                                          const int *gate, int *reorth,
                                                          double *hacc) {
    if (gate && *gate == 0) return;
    const bool mx[1] = {false};
    double a[1];
    finish_partials<1>(nparts, mx, partials, a);
    if (threadIdx.x == 0) {
        if (hacc)
            for (int i = 0; i < nv; ++i) hacc[i] += coef[i];
        if (reorth) *reorth = (a[0] < 1e-2 * coef[nv]) ? 1 : 0;
        *hnext = sqrt(a[0]);
    }
}

template <class T>
static void update_norm_impl(hipStream_t s, long nvec, int nv, const T *V, const double *coef,
                             T *w, double *partials, double *hnext, const int *gate, int *reorth,
                             double *hacc) {
    const int nblk = vec_blocks(nvec);
    hipLaunchKernelGGL(k_update_norm<T>, dim3(nblk), dim3(kBlock), 0, s, nvec, nv, V, coef, w,
                       partials, gate);
    hipLaunchKernelGGL(k_update_finish, dim3(1), dim3(kBlock), 0, s, nblk, nv, coef, partials,
                       hnext, gate, reorth, hacc);
}

void launch_update_norm(hipStream_t s, long nvec, int nv, const double *V, const double *coef,
                        double *w, double *partials, double *hnext, const int *gate, int *reorth,
                        double *hacc) {
    update_norm_impl(s, nvec, nv, V, coef, w, partials, hnext, gate, reorth, hacc);
}

void launch_update_norm(hipStream_t s, long nvec, int nv, const float *V, const double *coef,
                        float *w, double *partials, double *hnext, const int *gate, int *reorth,
                        double *hacc) {
    update_norm_impl(s, nvec, nv, V, coef, w, partials, hnext, gate, reorth, hacc);
}

// r = b - Ax; out[0] = ||r||^2, out[1] = ||r||
__global__ __launch_bounds__(kBlock) void k_residual(long nvec, const double *__restrict__ b,
                                                     const double *__restrict__ Ax,
                                                     double *__restrict__ r, double *partials) {
    double v[1] = {0.0};
    const bool mx[1] = {false};
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nvec;
         i += (long)gridDim.x * blockDim.x) {
        const double a = b[i] - Ax[i];
        r[i] = a;
        v[0] += a * a;
    }
    block_partials<1>(v, mx, partials);
}

void launch_residual(hipStream_t s, long nvec, const double *b, const double *Ax, double *r,
                     double *partials, double *out) {
    const int nblk = vec_blocks(nvec);
    hipLaunchKernelGGL(k_residual, dim3(nblk), dim3(kBlock), 0, s, nvec, b, Ax, r, partials);
    hipLaunchKernelGGL(k_finish_norm, dim3(1), dim3(kBlock), 0, s, nblk, partials, out);
}

// x += sum_{i<k} y_i Z_i (the flexible-GMRES update with stored
// preconditioned vectors)
template <class T>
__global__ __launch_bounds__(kBlock) void k_axpy_multi(long nvec, int k,
                                                       const T *__restrict__ Z,
                                                       const double *__restrict__ y,
                                                       double *__restrict__ x) {
    __shared__ double ys[kMaxRestart + 1];
    for (int i = threadIdx.x; i < k; i += blockDim.x) ys[i] = y[i];
    __syncthreads();
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nvec;
         e += (long)gridDim.x * blockDim.x) {
        double a = x[e];
        for (int i = 0; i < k; ++i) a += ys[i] * (double)Z[(size_t)i * nvec + e];
        x[e] = a;
    }
}

void launch_axpy_multi(hipStream_t s, long nvec, int k, const double *Z, const double *y,
                       double *x) {
    hipLaunchKernelGGL(k_axpy_multi<double>, dim3(vec_blocks(nvec)), dim3(kBlock), 0, s, nvec, k,
                       Z, y, x);
}

void launch_axpy_multi(hipStream_t s, long nvec, int k, const float *Z, const double *y,
                       double *x) {
    hipLaunchKernelGGL(k_axpy_multi<float>, dim3(vec_blocks(nvec)), dim3(kBlock), 0, s, nvec, k,
                       Z, y, x);
}

// y = (float) x, element by element (single-precision copies for the inner
// solves of the mixed-precision mode)
__global__ __launch_bounds__(kBlock) void k_to_float(long n, const double *__restrict__ x,
                                                     float *__restrict__ y) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}

void launch_to_float(hipStream_t s, long n, const double *x, float *y) {
    hipLaunchKernelGGL(k_to_float, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, x, y);
}

__global__ __launch_bounds__(kBlock) void k_to_double(long n, const float *__restrict__ x,
                                                      double *__restrict__ y) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

void launch_to_double(hipStream_t s, long n, const float *x, double *y) {
    hipLaunchKernelGGL(k_to_double, dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, x, y);
}

__global__ __launch_bounds__(kBlock) void k_scale_copy(long nvec, const double *__restrict__ x,
                                                       double a, double *__restrict__ y) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nvec;
         i += (long)gridDim.x * blockDim.x)
        y[i] = x ? a * x[i] : a;
}

// y = a*x, or y = a everywhere when x is null (a fill kernel, so nothing here
// records a memset node into a captured graph)
void launch_scale_copy(hipStream_t s, long nvec, const double *x, double a, double *y) {
    hipLaunchKernelGGL(k_scale_copy, dim3(vec_blocks(nvec)), dim3(kBlock), 0, s, nvec, x, a, y);
}

}  // namespace fim
