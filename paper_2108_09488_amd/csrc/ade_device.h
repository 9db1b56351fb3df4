// ade_device.h -- device helpers shared by the kernels (gfx950, wave64).
#pragma once

#include "ade_internal.h"

namespace ade {

constexpr int kWave = 64;

// Workgroups of one launch are dispatched round-robin over the 8 XCDs of the
// chip (block b runs on XCD b % 8).  Give each XCD a contiguous range of tiles
// so that tiles sharing neighbour cells also share an L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n) {
    const uint32_t nx = 8;
    if (n < nx) return b;
    const uint32_t per = n / nx, rem = n % nx;
    const uint32_t x = b % nx, k = b / nx;
    return x * per + (x < rem ? x : rem) + k;
}

// Cell of a fixed-point position: rows of the (y[, z]) grid, x cells inside a row.
template <int DIM>
__device__ __forceinline__ uint32_t cell_key(const PlumeDev& P, uint32_t ux, uint32_t uy,
                                             uint32_t uz) {
    const uint32_t fx = __umulhi(ux, P.nfx);
    const uint32_t ry = __umulhi(uy, P.nr);
    const uint32_t rz = (DIM == 3) ? __umulhi(uz, P.nr) : 0u;
    return P.cbase + (rz * P.nr + ry) * P.nfx + fx;
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// Exclusive scan over the block (blockDim.x a multiple of 64, at most 1024).
// lds must hold blockDim.x / 64 elements; returns the block total in total.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds, T& total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    T x = wave_inclusive_scan(v);
    if (lane == kWave - 1) lds[w] = x;
    __syncthreads();
    T pre = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        T s = lds[i];
        pre += (i < w) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// Sum over the block in a fixed order (deterministic); result valid in all threads.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    T x = wave_sum(v);
    if (lane == 0) lds[w] = x;
    __syncthreads();
    T tot = 0;
    for (int i = 0; i < nw; ++i) tot += lds[i];
    __syncthreads();
    return tot;
}

}  // namespace ade
