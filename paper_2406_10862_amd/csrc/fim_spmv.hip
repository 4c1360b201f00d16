// fim_spmv.hip - BSR SpMV y = A x, the GMRES operator (paper Sec. 5.1:
// FGMRES on the Jacobian of eqs. (1)-(2)).  It streams HBM: a group of G
// lanes reads consecutive blocks of one block row (coalesced), the matrix
// is read once per product and the gathered vector stays cached.
#include <hip/hip_ext.h>

#include "fim_internal.h"

namespace fim {

typedef double d2 __attribute__((ext_vector_type(2)));

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
__device__ __forceinline__ void spmv_body(int bid, int nrows, const int *__restrict__ rowptr,
                                          const int *__restrict__ colind,
                                          const MT *__restrict__ val, const VT *__restrict__ x,
                                          VT *__restrict__ y) {
    constexpr int R = SpmvRows<NB>::R;
    constexpr int GPW = 64 / G;             // lane groups per wave
    const int lg = threadIdx.x & (G - 1);
    const long wave = ((long)bid * blockDim.x + threadIdx.x) >> 6;
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

template <int NB, int G, class MT, class VT>
__global__ __launch_bounds__(kBlock) void k_spmv(int nrows, const int *__restrict__ rowptr,
                                                 const int *__restrict__ colind,
                                                 const MT *__restrict__ val,
                                                 const VT *__restrict__ x,
                                                 VT *__restrict__ y) {
    spmv_body<NB, G, MT, VT>(blockIdx.x, nrows, rowptr, colind, val, x, y);
}

// Batched over the members of an ensemble: y = J z_j into w (j >= 0) or
// y = J x into t (j < 0), each member with its own Jacobian.
template <int NB>
__global__ __launch_bounds__(kBlock) void kb_spmv(const Member *__restrict__ mem, Batch B, int j) {
    int m, b, nb;
    if (!batch_view(B, m, b, nb)) return;
    const Member &M = mem[m];
    const double *src = j >= 0 ? M.Z + (size_t)j * M.nvec : M.x;
    double *dst = j >= 0 ? M.w : M.t;
    spmv_body<NB, kSpmvG, double, double>(b, M.nrows, M.sys.rowptr, M.sys.colind, M.sys.val, src,
                                          dst);
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

int spmv_blocks(int nb, int nrows) {
    const int per = nb == 2 ? spmv_rows_per_block<2, kSpmvG>() : spmv_rows_per_block<3, kSpmvG>();
    return (nrows + per - 1) / per;
}

void launchb_spmv(hipStream_t s, int nb, const Member *mem, Batch B, int total, int j) {
    if (total <= 0) return;
    if (nb == 2) hipLaunchKernelGGL(kb_spmv<2>, dim3(total), dim3(kBlock), 0, s, mem, B, j);
    else hipLaunchKernelGGL(kb_spmv<3>, dim3(total), dim3(kBlock), 0, s, mem, B, j);
}

void launch_spmv(hipStream_t s, int nb, int nrows, const int *rowptr, const int *colind,
                 const double *val, const double *x, double *y, hipEvent_t e0, hipEvent_t e1) {
    spmv_impl(s, nb, nrows, rowptr, colind, val, x, y, e0, e1);
}

void launch_spmv(hipStream_t s, int nb, int nrows, const int *rowptr, const int *colind,
                 const float *val, const float *x, float *y, hipEvent_t e0, hipEvent_t e1) {
    spmv_impl(s, nb, nrows, rowptr, colind, val, x, y, e0, e1);
}

}  // namespace fim
