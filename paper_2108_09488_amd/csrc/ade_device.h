// ade_device.h -- device helpers shared by the kernels (gfx950, wave64).
#pragma once

#include "ade_internal.h"

namespace ade {

constexpr int kWave = 64;

// Workgroups of one launch are dispatched round-robin over the 8 XCDs of the
// chip (workgroup b runs on XCD b % 8).  Items are dealt to the XCDs in turns
// of `group` consecutive items, so that neighbouring items (which share
// candidate cells) share an L2 while every XCD still gets an even share of
// every part of the item list (plumes of an ensemble differ in cost per item).
// A bijection of [0, n): the last incomplete round keeps the identity.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n, uint32_t group) {
    const uint32_t nx = 8, round = nx * group;
    const uint32_t full = n / round * round;
    if (b >= full) return b;
    const uint32_t g = b / round, r = b % round;
    return g * round + (r % nx) * group + r / nx;
}

// The m-th item (m = 0, 1, ...) that xcd_remap deals to XCD x, or n when
// XCD x has fewer than m + 1 items (the persistent grid walks this list).
__device__ __forceinline__ uint32_t xcd_item(uint32_t x, uint32_t m, uint32_t n, uint32_t group) {
    const uint32_t nx = 8, round = nx * group;
    const uint32_t full = n / round * round;
    const uint32_t per = full / nx;  // items of XCD x in complete rounds
    if (m < per) return (m / group) * round + x * group + m % group;
    const uint32_t t = full + x + (m - per) * nx;  // the identity tail, round-robin
    return t < n ? t : n;
}

// Cell of a fixed-point position: rows of the (y[, z]) grid, x cells inside a
// row, sub-rows (in y) inside an x cell; the position inside the row is the
// low word of uy * nr.
template <int DIM>
__device__ __forceinline__ uint32_t cell_key(const PlumeDev& P, uint32_t ux, uint32_t uy,
                                             uint32_t uz) {
    const uint32_t fx = __umulhi(ux, P.nfx);
    const uint32_t ry = __umulhi(uy, P.nr);
    const uint32_t rz = (DIM == 3) ? __umulhi(uz, P.nr) : 0u;
    const uint32_t sy = __umulhi(uy * P.nr, P.nsub);
    return P.cbase + ((rz * P.nr + ry) * P.nfx + fx) * P.nsub + sy;
}

// Counting pass: count the particle with this id in its cell and record the
// id in the cell's bucket, or past kBucket in the overflow list.
__device__ __forceinline__ void enlist(const CellLists& L, uint32_t key, uint32_t id) {
    const uint32_t t = atomicAdd(&L.count[key], 1u);
    if (t < kBucket) {
        L.bucket[(size_t)key * kBucket + t] = id;
    } else {
        const uint32_t p = atomicAdd(&L.ovf_count[0], 1u);
        L.ovf[p] = make_uint2(key, id);
    }
}

// Two particles of one cell counted with one atomic: their ids take
// consecutive slots of the cell's bucket (or the overflow list past kBucket).
// The order inside a cell's entries is free: placement ranks a cell's
// particles by id.
__device__ __forceinline__ void enlist2(const CellLists& L, uint32_t key, uint32_t id0, uint32_t id1) {
    const uint32_t t = atomicAdd(&L.count[key], 2u);
    const uint32_t ids[2] = {id0, id1};
#pragma unroll
    for (uint32_t q = 0; q < 2; ++q) {
        if (t + q < kBucket) {
            L.bucket[(size_t)key * kBucket + t + q] = ids[q];
        } else {
            const uint32_t p = atomicAdd(&L.ovf_count[0], 1u);
            L.ovf[p] = make_uint2(key, ids[q]);
        }
    }
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

// 16-byte record of a particle for the candidate loops: fixed-point position
// and concentration (2D: x, y, C[, C high word]; 3D FP32: x, y, z, C).  3D FP64
// does not fit and uses the structure-of-arrays state instead.
template <int DIM, typename real>
struct Rec {
    static constexpr bool kStageable = !(DIM == 3 && sizeof(real) == 8);
    static __device__ __forceinline__ uint4 pack(uint32_t x, uint32_t y, uint32_t z, real c) {
        uint4 r;
        r.x = x;
        r.y = y;
        if (sizeof(real) == 4) {
            const uint32_t cb = __float_as_uint((float)c);
            r.z = (DIM == 3) ? z : cb;
            r.w = (DIM == 3) ? cb : 0u;
        } else {
            const unsigned long long cb = (unsigned long long)__double_as_longlong((double)c);
            r.z = (uint32_t)cb;
            r.w = (uint32_t)(cb >> 32);
        }
        return r;
    }
    static __device__ __forceinline__ real conc(const uint4& r) {
        if (sizeof(real) == 4) return (real)__uint_as_float(DIM == 3 ? r.w : r.z);
        return (real)__longlong_as_double((long long)(((unsigned long long)r.w << 32) | r.z));
    }
};

}  // namespace ade
