// fim_block.h - operations on one nb x nb block (nb = 2, 3) in registers.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace fim {

// Inverse of a row-major block; false when it is singular or not finite.
template <int NB>
__device__ inline bool invert_block(const double *a, double *inv) {
    if constexpr (NB == 2) {
        const double det = a[0] * a[3] - a[1] * a[2];
        if (!(det != 0.0) || !isfinite(det)) return false;
        const double r = 1.0 / det;
        inv[0] = a[3] * r;
        inv[1] = -a[1] * r;
        inv[2] = -a[2] * r;
        inv[3] = a[0] * r;
        return true;
    } else {
        // Gauss-Jordan elimination with row pivoting on [A | I]
        double m[NB][2 * NB];
#pragma unroll
        for (int r = 0; r < NB; ++r)
#pragma unroll
            for (int c = 0; c < 2 * NB; ++c) m[r][c] = c < NB ? a[r * NB + c] : (c - NB == r);
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            // pivot search and row swap with compile-time row indices only
            int p = c;
            double best = fabs(m[c][c]);
#pragma unroll
            for (int r = c + 1; r < NB; ++r)
                if (fabs(m[r][c]) > best) {
                    best = fabs(m[r][c]);
                    p = r;
                }
            if (!(best != 0.0)) return false;
#pragma unroll
            for (int r = c + 1; r < NB; ++r)
                if (r == p)
#pragma unroll
                    for (int k = 0; k < 2 * NB; ++k) {
                        const double t = m[c][k];
                        m[c][k] = m[r][k];
                        m[r][k] = t;
                    }
            const double d = 1.0 / m[c][c];
#pragma unroll
            for (int k = 0; k < 2 * NB; ++k) m[c][k] *= d;
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                if (r == c) continue;
                const double f = m[r][c];
#pragma unroll
                for (int k = 0; k < 2 * NB; ++k) m[r][k] -= f * m[c][k];
            }
        }
#pragma unroll
        for (int r = 0; r < NB; ++r)
#pragma unroll
            for (int c = 0; c < NB; ++c) inv[r * NB + c] = m[r][NB + c];
        return true;
    }
}

// C = A * B (row-major blocks)
template <int NB>
__device__ inline void block_mul(const double *A, const double *B, double *C) {
#pragma unroll
    for (int r = 0; r < NB; ++r)
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            double s = A[r * NB] * B[c];
#pragma unroll
            for (int k = 1; k < NB; ++k) s += A[r * NB + k] * B[k * NB + c];
            C[r * NB + c] = s;
        }
}

}  // namespace fim
