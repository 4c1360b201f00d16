// fim_linalg.hip - block transpose, block-Jacobi preconditioner and the
// vector kernels of right-preconditioned GMRES (paper Sec. 5.1: FGMRES with
// block-Jacobi smoothing; Sec. 3.3.3: the solve returns the solution and
// the iteration count).  The SpMV is in fim_spmv.hip.
//
// Everything here streams HBM.  The orthogonalisation kernels read each
// basis vector once per pass with the dot products of a group of vectors
// accumulated in registers.
#include <math.h>

#include "fim_internal.h"
#include "fim_reduce.h"
#include "fim_block.h"

namespace fim {

constexpr int kMaxDots = kMaxRestart + 1;   // basis vectors + the vector itself

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


// out[0] = sum of the partials, out[1] = its square root (a norm finish)
__device__ __forceinline__ void finish_norm_body(int nparts, const double *partials, double *out) {
    const bool mx[1] = {false};
    double a[1];
    finish_partials<1>(nparts, mx, partials, a);
    if (threadIdx.x == 0) {
        out[0] = a[0];
        out[1] = sqrt(a[0]);
    }
}

__global__ __launch_bounds__(kBlock) void k_finish_norm(int nparts, const double *partials,
                                                        double *out) {
    finish_norm_body(nparts, partials, out);
}

// out[0] = ||x||^2, out[1] = ||x||
__device__ __forceinline__ void norm2_body(int bid, int nblk, long nvec,
                                           const double *__restrict__ x, double *partials) {
    double v[1] = {0.0};
    const bool mx[1] = {false};
    for (long i = (long)bid * blockDim.x + threadIdx.x; i < nvec; i += (long)nblk * blockDim.x) {
        const double a = x[i];
        v[0] += a * a;
    }
    block_partials<1>(v, mx, partials, bid, nblk);
}

__global__ __launch_bounds__(kBlock) void k_norm2(long nvec, const double *__restrict__ x,
                                                  double *partials) {
    norm2_body(blockIdx.x, gridDim.x, nvec, x, partials);
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
__device__ inline void multidot_group(int bx, int nbx, long nvec, const T *__restrict__ V,
                                      const T *__restrict__ w, bool self,
                                      double (&acc)[kDotGroup + 1]) {
    constexpr int U = NG <= 2 ? 4 : 2;
    const long S = (long)nbx * blockDim.x;
    for (long e0 = (long)bx * blockDim.x + threadIdx.x; e0 < nvec; e0 += U * S) {
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

// The same over element pairs (16-byte loads of doubles), for vectors of
// even length whose rows start on a pair boundary: x then y of a pair.
template <class T, int NG>
__device__ inline void multidot_group2(int bx, int nbx, long nvec, const T *__restrict__ V,
                                       const T *__restrict__ w, bool self,
                                       double (&acc)[kDotGroup + 1]) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    constexpr int U = NG <= 2 ? 4 : 2;
    const long S = (long)nbx * blockDim.x, n2 = nvec >> 1;
    const T2 *w2 = reinterpret_cast<const T2 *>(w);
    for (long e0 = (long)bx * blockDim.x + threadIdx.x; e0 < n2; e0 += U * S) {
        T2 we[U], v[U][NG];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long e = e0 + u * S < n2 ? e0 + u * S : e0;
            we[u] = w2[e];
#pragma unroll
            for (int i = 0; i < NG; ++i)
                v[u][i] = __builtin_nontemporal_load(reinterpret_cast<const T2 *>(V + (size_t)i * nvec) + e);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool on = e0 + u * S < n2;
            const double wx = on ? (double)we[u].x : 0.0, wy = on ? (double)we[u].y : 0.0;
#pragma unroll
            for (int i = 0; i < NG; ++i) {
                acc[i] += (double)v[u][i].x * wx;
                acc[i] += (double)v[u][i].y * wy;
            }
            if (self) {
                acc[kDotGroup] += wx * wx;
                acc[kDotGroup] += wy * wy;
            }
        }
    }
}

// pairs of T can be read at V (rows of length nvec) and w
template <class T>
__device__ inline bool pair_aligned(long nvec, const T *V, const T *w) {
    return (nvec & 1) == 0 && (reinterpret_cast<uintptr_t>(V) & (2 * sizeof(T) - 1)) == 0 &&
           (reinterpret_cast<uintptr_t>(w) & (2 * sizeof(T) - 1)) == 0;
}

template <class T>
__device__ __forceinline__ void multidot_part_body(int bx, int nbx, int by, long nvec, int nv,
                                                   const T *__restrict__ V,
                                                   const T *__restrict__ w,
                                                   double *__restrict__ partials,
                                                   const int *gate) {
    if (gate && *gate == 0) return;
    const int g0 = by * kDotGroup;
    const int ng = min(kDotGroup, nv - g0);
    double acc[kDotGroup + 1];
#pragma unroll
    for (int i = 0; i <= kDotGroup; ++i) acc[i] = 0.0;
    const bool self = by == 0;                    // the first group also forms <w, w>
    const T *Vg = V + (size_t)g0 * nvec;
    if (pair_aligned(nvec, Vg, w)) {
        switch (ng) {
        case 1: multidot_group2<T, 1>(bx, nbx, nvec, Vg, w, self, acc); break;
        case 2: multidot_group2<T, 2>(bx, nbx, nvec, Vg, w, self, acc); break;
        case 3: multidot_group2<T, 3>(bx, nbx, nvec, Vg, w, self, acc); break;
        case 4: multidot_group2<T, 4>(bx, nbx, nvec, Vg, w, self, acc); break;
        case 5: multidot_group2<T, 5>(bx, nbx, nvec, Vg, w, self, acc); break;
        case 6: multidot_group2<T, 6>(bx, nbx, nvec, Vg, w, self, acc); break;
        case 7: multidot_group2<T, 7>(bx, nbx, nvec, Vg, w, self, acc); break;
        default: multidot_group2<T, kDotGroup>(bx, nbx, nvec, Vg, w, self, acc); break;
        }
    } else switch (ng) {
    case 1: multidot_group<T, 1>(bx, nbx, nvec, Vg, w, self, acc); break;
    case 2: multidot_group<T, 2>(bx, nbx, nvec, Vg, w, self, acc); break;
    case 3: multidot_group<T, 3>(bx, nbx, nvec, Vg, w, self, acc); break;
    case 4: multidot_group<T, 4>(bx, nbx, nvec, Vg, w, self, acc); break;
    case 5: multidot_group<T, 5>(bx, nbx, nvec, Vg, w, self, acc); break;
    case 6: multidot_group<T, 6>(bx, nbx, nvec, Vg, w, self, acc); break;
    case 7: multidot_group<T, 7>(bx, nbx, nvec, Vg, w, self, acc); break;
    default: multidot_group<T, kDotGroup>(bx, nbx, nvec, Vg, w, self, acc); break;
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
            partials[(size_t)slot * nbx + bx] = a;
        }
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_multidot_part(long nvec, int nv,
                                                          const T *__restrict__ V,
                                                          const T *__restrict__ w,
                                                          double *__restrict__ partials,
                                                          const int *gate) {
    multidot_part_body<T>(blockIdx.x, gridDim.x, blockIdx.y, nvec, nv, V, w, partials, gate);
}

__device__ __forceinline__ void multidot_sum_body(int slot, int ncols,
                                                  const double *__restrict__ partials,
                                                  double *__restrict__ dst, const int *gate) {
    if (gate && *gate == 0) return;
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

__global__ __launch_bounds__(kBlock) void k_multidot_sum(int ncols, const double *__restrict__ partials,
                                                         double *__restrict__ dst, const int *gate) {
    multidot_sum_body(blockIdx.x, ncols, partials, dst, gate);
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
__device__ __forceinline__ void update_norm_body(int bid, int nblk, long nvec, int nv,
                                                 const T *__restrict__ V, const double *coef,
                                                 T *w, double *partials, const int *gate) {
    if (gate && *gate == 0) return;
    __shared__ double c[kMaxDots];
    for (int i = threadIdx.x; i <= nv; i += blockDim.x) c[i] = coef[i];
    __syncthreads();
    double v[1] = {0.0};
    const bool mx[1] = {false};
    if (pair_aligned(nvec, V, w)) {
        // element pairs (16-byte loads of doubles), x then y
        typedef T T2 __attribute__((ext_vector_type(2)));
        T2 *w2 = reinterpret_cast<T2 *>(w);
        const long n2 = nvec >> 1;
        for (long e = (long)bid * blockDim.x + threadIdx.x; e < n2; e += (long)nblk * blockDim.x) {
            const T2 wv = w2[e];
            double a0 = (double)wv.x, a1 = (double)wv.y;
#pragma unroll 8
            for (int i = 0; i < nv; ++i) {
                const T2 vv = __builtin_nontemporal_load(reinterpret_cast<const T2 *>(V + (size_t)i * nvec) + e);
                a0 -= c[i] * (double)vv.x;
                a1 -= c[i] * (double)vv.y;
            }
            T2 at;
            at.x = (T)a0;
            at.y = (T)a1;
            w2[e] = at;
            v[0] += (double)at.x * (double)at.x;
            v[0] += (double)at.y * (double)at.y;
        }
    } else {
        for (long e = (long)bid * blockDim.x + threadIdx.x; e < nvec; e += (long)nblk * blockDim.x) {
            double a = (double)w[e];
#pragma unroll 8
            for (int i = 0; i < nv; ++i)
                a -= c[i] * (double)__builtin_nontemporal_load(V + (size_t)i * nvec + e);
            const T at = (T)a;                     // the norm of what is stored
            w[e] = at;
            v[0] += (double)at * (double)at;
        }
    }
    block_partials<1>(v, mx, partials, bid, nblk);
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_update_norm(long nvec, int nv,
                                                        const T *__restrict__ V,
                                                        const double *coef, T *w,
                                                        double *partials, const int *gate) {
    update_norm_body<T>(blockIdx.x, gridDim.x, nvec, nv, V, coef, w, partials, gate);
}

// With mirror set, the finished column (hacc, or coef in a first pass:
// nv coefficients and then hnext, which must follow them) is also stored
// there, in pinned host memory, for the host's Givens rotations.
__device__ __forceinline__ void update_finish_body(int nparts, int nv, const double *coef,
                                                   const double *partials, double *hnext,
                                                   const int *gate, int *reorth, double *hacc,
                                                   double *mirror = nullptr) {
    if (gate && *gate == 0) return;
    const bool mx[1] = {false};
    double a[1];
    finish_partials<1>(nparts, mx, partials, a);
    if (threadIdx.x == 0) {
        if (hacc)
            for (int i = 0; i < nv; ++i) hacc[i] += coef[i];
        if (reorth) *reorth = (a[0] < 1e-2 * coef[nv]) ? 1 : 0;
        *hnext = sqrt(a[0]);
        if (mirror) {
            const double *col = hacc ? hacc : coef;
            for (int i = 0; i <= nv; ++i) mirror[i] = col[i];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_update_finish(int nparts, int nv, const double *coef,
                                                          const double *partials, double *hnext,
                                                          const int *gate, int *reorth,
                                                          double *hacc, double *mirror) {
    update_finish_body(nparts, nv, coef, partials, hnext, gate, reorth, hacc, mirror);
}

template <class T>
static void update_norm_impl(hipStream_t s, long nvec, int nv, const T *V, const double *coef,
                             T *w, double *partials, double *hnext, const int *gate, int *reorth,
                             double *hacc, double *mirror) {
    const int nblk = vec_blocks(nvec);
    hipLaunchKernelGGL(k_update_norm<T>, dim3(nblk), dim3(kBlock), 0, s, nvec, nv, V, coef, w,
                       partials, gate);
    hipLaunchKernelGGL(k_update_finish, dim3(1), dim3(kBlock), 0, s, nblk, nv, coef, partials,
                       hnext, gate, reorth, hacc, mirror);
}

void launch_update_norm(hipStream_t s, long nvec, int nv, const double *V, const double *coef,
                        double *w, double *partials, double *hnext, const int *gate, int *reorth,
                        double *hacc, double *mirror) {
    update_norm_impl(s, nvec, nv, V, coef, w, partials, hnext, gate, reorth, hacc, mirror);
}

void launch_update_norm(hipStream_t s, long nvec, int nv, const float *V, const double *coef,
                        float *w, double *partials, double *hnext, const int *gate, int *reorth,
                        double *hacc, double *mirror) {
    update_norm_impl(s, nvec, nv, V, coef, w, partials, hnext, gate, reorth, hacc, mirror);
}

// r = b - Ax; out[0] = ||r||^2, out[1] = ||r||
__device__ __forceinline__ void residual_body(int bid, int nblk, long nvec,
                                              const double *__restrict__ b,
                                              const double *__restrict__ Ax,
                                              double *__restrict__ r, double *partials) {
    double v[1] = {0.0};
    const bool mx[1] = {false};
    for (long i = (long)bid * blockDim.x + threadIdx.x; i < nvec; i += (long)nblk * blockDim.x) {
        const double a = b[i] - Ax[i];
        r[i] = a;
        v[0] += a * a;
    }
    block_partials<1>(v, mx, partials, bid, nblk);
}

__global__ __launch_bounds__(kBlock) void k_residual(long nvec, const double *__restrict__ b,
                                                     const double *__restrict__ Ax,
                                                     double *__restrict__ r, double *partials) {
    residual_body(blockIdx.x, gridDim.x, nvec, b, Ax, r, partials);
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
__device__ __forceinline__ void axpy_multi_body(int bid, int nblk, long nvec, int k,
                                                const T *__restrict__ Z,
                                                const double *__restrict__ y,
                                                double *__restrict__ x) {
    __shared__ double ys[kMaxRestart + 1];
    for (int i = threadIdx.x; i < k; i += blockDim.x) ys[i] = y[i];
    __syncthreads();
    for (long e = (long)bid * blockDim.x + threadIdx.x; e < nvec; e += (long)nblk * blockDim.x) {
        double a = x[e];
        for (int i = 0; i < k; ++i) a += ys[i] * (double)Z[(size_t)i * nvec + e];
        x[e] = a;
    }
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_axpy_multi(long nvec, int k,
                                                       const T *__restrict__ Z,
                                                       const double *__restrict__ y,
                                                       double *__restrict__ x) {
    axpy_multi_body<T>(blockIdx.x, gridDim.x, nvec, k, Z, y, x);
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

__device__ __forceinline__ void scale_copy_body(int bid, int nblk, long nvec,
                                                const double *__restrict__ x, double a,
                                                double *__restrict__ y) {
    for (long i = (long)bid * blockDim.x + threadIdx.x; i < nvec; i += (long)nblk * blockDim.x)
        y[i] = x ? a * x[i] : a;
}

__global__ __launch_bounds__(kBlock) void k_scale_copy(long nvec, const double *__restrict__ x,
                                                       double a, double *__restrict__ y) {
    scale_copy_body(blockIdx.x, gridDim.x, nvec, x, a, y);
}

// y = a*x, or y = a everywhere when x is null (a fill kernel, so nothing here
// records a memset node into a captured graph)
void launch_scale_copy(hipStream_t s, long nvec, const double *x, double a, double *y) {
    hipLaunchKernelGGL(k_scale_copy, dim3(vec_blocks(nvec)), dim3(kBlock), 0, s, nvec, x, a, y);
}

// ---------------------------------------------------------------------------
// batched launches over the members of an ensemble (FP64 Krylov vectors of
// each member's context; the Hessenberg column of step j at H + j*LD)

constexpr int kLD = kMaxRestart + 2;

int dot_groups(int nv) { return (nv + kDotGroup - 1) / kDotGroup > 0 ? (nv + kDotGroup - 1) / kDotGroup : 1; }

__global__ __launch_bounds__(kBlock) void kb_scale_zero(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    scale_copy_body(b, nb, M.nvec, nullptr, 0.0, M.x);
}

__global__ __launch_bounds__(kBlock) void kb_norm_b(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    norm2_body(b, nb, M.nvec, M.sys.R, M.partials);
}

__global__ __launch_bounds__(kBlock) void kb_finish_norm(const Member *__restrict__ mem, Batch B,
                                                         int slot) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    finish_norm_body(vec_blocks(M.nvec), M.partials, M.scal + slot);
}

__global__ __launch_bounds__(kBlock) void kb_multidot_part(const Member *__restrict__ mem, Batch B,
                                                           int j, int second) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    const int cols = vec_blocks(M.nvec);
    multidot_part_body<double>(b % cols, cols, b / cols, M.nvec, j + 1, M.V, M.w, M.partials,
                               second ? M.reorth : nullptr);
}

__global__ __launch_bounds__(kBlock) void kb_multidot_sum(const Member *__restrict__ mem, Batch B,
                                                          int j, int second) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    multidot_sum_body(b, vec_blocks(M.nvec), M.partials, second ? M.tmp : M.H + (size_t)j * kLD,
                      second ? M.reorth : nullptr);
}

__global__ __launch_bounds__(kBlock) void kb_update_norm(const Member *__restrict__ mem, Batch B,
                                                         int j, int second) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    const double *col = M.H + (size_t)j * kLD;
    update_norm_body<double>(b, nb, M.nvec, j + 1, M.V, second ? M.tmp : col, M.w, M.partials,
                             second ? M.reorth : nullptr);
}

__global__ __launch_bounds__(kBlock) void kb_update_finish(const Member *__restrict__ mem, Batch B,
                                                           int j, int second) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    double *col = M.H + (size_t)j * kLD;
    if (second)
        update_finish_body(vec_blocks(M.nvec), j + 1, M.tmp, M.partials, col + j + 1, M.reorth,
                           nullptr, col);
    else
        update_finish_body(vec_blocks(M.nvec), j + 1, col, M.partials, col + j + 1, nullptr,
                           M.reorth, nullptr);
}

__global__ void kb_hcols(const Member *__restrict__ mem, Batch B, int j, double *__restrict__ packed,
                         int ld) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    for (int i = threadIdx.x; i < j + 2; i += blockDim.x)
        packed[(size_t)m * ld + i] = M.H[(size_t)j * kLD + i];
}

__global__ __launch_bounds__(kBlock) void kb_axpy(const Member *__restrict__ mem, Batch B,
                                                  const int *__restrict__ kcount,
                                                  const double *__restrict__ ypacked, int ld) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    axpy_multi_body<double>(b, nb, M.nvec, kcount[m], M.Z, ypacked + (size_t)m * ld, M.x);
}

__global__ __launch_bounds__(kBlock) void kb_residual(const Member *__restrict__ mem, Batch B) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    residual_body(b, nb, M.nvec, M.sys.R, M.t, M.r, M.partials);
}

void launchb_scale_zero(hipStream_t s, const Member *mem, Batch B, int total) {
    if (total > 0) hipLaunchKernelGGL(kb_scale_zero, dim3(total), dim3(kBlock), 0, s, mem, B);
}

void launchb_norm_b(hipStream_t s, const Member *mem, Batch part, int tpart, Batch one, int tone,
                    int slot) {
    if (tpart <= 0) return;
    hipLaunchKernelGGL(kb_norm_b, dim3(tpart), dim3(kBlock), 0, s, mem, part);
    hipLaunchKernelGGL(kb_finish_norm, dim3(tone), dim3(kBlock), 0, s, mem, one, slot);
}

void launchb_multidot(hipStream_t s, const Member *mem, Batch part, int tpart, Batch sum,
                      int tsum, int j, bool second) {
    if (tpart <= 0) return;
    hipLaunchKernelGGL(kb_multidot_part, dim3(tpart), dim3(kBlock), 0, s, mem, part, j, (int)second);
    hipLaunchKernelGGL(kb_multidot_sum, dim3(tsum), dim3(kBlock), 0, s, mem, sum, j, (int)second);
}

void launchb_update_norm(hipStream_t s, const Member *mem, Batch part, int tpart, Batch one,
                         int tone, int j, bool second) {
    if (tpart <= 0) return;
    hipLaunchKernelGGL(kb_update_norm, dim3(tpart), dim3(kBlock), 0, s, mem, part, j, (int)second);
    hipLaunchKernelGGL(kb_update_finish, dim3(tone), dim3(kBlock), 0, s, mem, one, j, (int)second);
}

void launchb_hcols(hipStream_t s, const Member *mem, Batch one, int tone, int j, double *packed,
                   int ld) {
    if (tone > 0) hipLaunchKernelGGL(kb_hcols, dim3(tone), dim3(64), 0, s, mem, one, j, packed, ld);
}

void launchb_axpy(hipStream_t s, const Member *mem, Batch B, int total, const int *kcount,
                  const double *ypacked, int ld) {
    if (total > 0)
        hipLaunchKernelGGL(kb_axpy, dim3(total), dim3(kBlock), 0, s, mem, B, kcount, ypacked, ld);
}

void launchb_residual(hipStream_t s, const Member *mem, Batch part, int tpart, Batch one, int tone,
                      int slot) {
    if (tpart <= 0) return;
    hipLaunchKernelGGL(kb_residual, dim3(tpart), dim3(kBlock), 0, s, mem, part);
    hipLaunchKernelGGL(kb_finish_norm, dim3(tone), dim3(kBlock), 0, s, mem, one, slot);
}

}  // namespace fim
