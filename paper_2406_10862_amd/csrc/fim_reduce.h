// fim_reduce.h - deterministic block and grid reductions for wave64.
//
// A grid reduction writes one partial per block, then the last block to
// arrive (ticket from a global counter) combines the partials in block order
// and resets the counter, so the result does not depend on scheduling and
// no second kernel launch is needed.
#pragma once
#include <hip/hip_runtime.h>

#include "fim_internal.h"

namespace fim {

constexpr int kWaves = kBlock / 64;

// sum, or a maximum that keeps NaN (a non-finite residual must not vanish)
__device__ inline double rop(double a, double b, bool mx) {
    return mx ? ((b > a || b != b) ? b : a) : a + b;
}

template <int K>
__device__ inline void wave_reduce(double (&v)[K], const bool (&mx)[K]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = rop(v[k], __shfl_xor(v[k], off, 64), mx[k]);
}

// Result valid in thread 0.  Every thread of the block must call it.
template <int K>
__device__ inline void block_reduce(double (&v)[K], const bool (&mx)[K], double (&sh)[K][kWaves]) {
    wave_reduce<K>(v, mx);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[k][wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double a = sh[k][0];
            for (int w = 1; w < kWaves; ++w) a = rop(a, sh[k][w], mx[k]);
            v[k] = a;
        }
    __syncthreads();
}

// Grid-wide reduction of K values per thread into out[K].  Returns true in
// the threads of the block that finished the reduction (the last block).
template <int K>
__device__ inline bool grid_reduce(double (&v)[K], const bool (&mx)[K], double *partials,
                                   unsigned *counter, double *out) {
    __shared__ double sh[K][kWaves];
    __shared__ int is_last;
    block_reduce<K>(v, mx, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) partials[(size_t)blockIdx.x * K + k] = v[k];
        __threadfence();
        unsigned t = atomicAdd(counter, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] = rop(a[k], partials[(size_t)b * K + k], mx[k]);
    block_reduce<K>(a, mx, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = a[k];
        atomicExch(counter, 0u);
    }
    return true;
}

}  // namespace fim
