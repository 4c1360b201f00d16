// fim_reduce.h - deterministic block and grid reductions for wave64.
//
// A grid reduction writes one partial per block; a one-block kernel then
// combines the partials in block order, so the result does not depend on
// scheduling.
#pragma once
#include <hip/hip_runtime.h>

#include "fim_internal.h"

namespace fim {

constexpr int kWaves = kBlock / 64;

// Workgroup barrier ordering LDS only.  __syncthreads() also orders global
// memory, so it waits for every load in flight, prefetches included; for
// phases that exchange values through LDS alone.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

// First half of a grid reduction: the block's K results go to
// partials[k * gridDim.x + blockIdx.x].  No fence or atomic: the kernel
// boundary makes them visible to the finishing kernel (a device-scope fence
// per block would write back the whole L2 of the block's XCD).
template <int K>
__device__ inline void block_partials(double (&v)[K], const bool (&mx)[K], double *partials,
                                      int bid, int nblk) {
    __shared__ double sh[K][kWaves];
    block_reduce<K>(v, mx, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) partials[(size_t)k * nblk + bid] = v[k];
}

template <int K>
__device__ inline void block_partials(double (&v)[K], const bool (&mx)[K], double *partials) {
    block_partials<K>(v, mx, partials, (int)blockIdx.x, (int)gridDim.x);
}

// Second half, run by a single block: combines nparts partials of each of
// the K slots in block order.  Result valid in thread 0.
template <int K>
__device__ inline void finish_partials(int nparts, const bool (&mx)[K], const double *partials,
                                       double (&a)[K]) {
    __shared__ double sh[K][kWaves];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = 0.0;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] = rop(a[k], partials[(size_t)k * nparts + b], mx[k]);
    block_reduce<K>(a, mx, sh);
}

}  // namespace fim
