// ade_geom.h -- neighbour-search geometry shared by the pair, adjoint and
// sensor kernels: targets in fixed point, the rows of cells around a target
// and the contiguous sorted-index ranges that hold its candidates.
#pragma once

#include "ade_device.h"

namespace ade {

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// r2 >= 1 in grid units, so the hardware reciprocal square root needs no
// denormal scaling
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }

template <typename real>
__device__ __forceinline__ real h2_of(const PlumeDev& P) {
    return sizeof(real) == 4 ? (real)P.H2f : (real)P.H2d;
}

constexpr int kMaxRowOffsets = 81;  // (2R+1)^2 for R <= 4
// candidate records each lane fetches together, ahead of their use
template <int LANES>
struct Batch {
    static constexpr int value = 4;
};

// A target particle: fixed-point position, its row and the fractional
// position inside the row (in row heights, from the low word of u * nr).
struct Target {
    uint32_t ux, uy, uz;
    int ry, rz;
    float fy, fz;
};

template <int DIM>
__device__ __forceinline__ Target make_target(const PlumeDev& P, uint32_t ux, uint32_t uy, uint32_t uz) {
    Target t;
    t.ux = ux;
    t.uy = uy;
    t.uz = uz;
    t.ry = (int)__umulhi(uy, P.nr);
    t.fy = (float)(uy * P.nr) * 2.3283064365386963e-10f;
    if (DIM == 3) {
        t.rz = (int)__umulhi(uz, P.nr);
        t.fz = (float)(uz * P.nr) * 2.3283064365386963e-10f;
    } else {
        t.rz = 0;
        t.fz = 0.f;
    }
    return t;
}

// Candidate cells of the neighbour row (oy, oz) of a target: the x window
// [x - w, x + w], w being (an upper bound of) the chord of the search radius
// at the row's nearest edge.  Returns false when the row lies beyond the
// search radius.  k0 .. k1 (inclusive) is the first cell range and k2 .. k3
// the second one, non-empty only when the window wraps around the periodic
// seam (k2 > k3 marks it empty).  The bounds are conservative: the float
// rounding of the distances is covered by relative slack on w^2 and an
// absolute slack of 64 grid units on w.
template <int DIM>
__device__ __forceinline__ bool row_cells(const PlumeDev& P, const Target& T, int oy, int oz,
                                          uint32_t& k0, uint32_t& k1, uint32_t& k2, uint32_t& k3) {
    float dy = 0.f, dz = 0.f;
    if (oy > 0) dy = (float)oy - T.fy;
    else if (oy < 0) dy = (float)(-oy - 1) + T.fy;
    if (DIM == 3) {
        if (oz > 0) dz = (float)oz - T.fz;
        else if (oz < 0) dz = (float)(-oz - 1) + T.fz;
    }
    const float d2 = (dy * dy + dz * dz) * P.rowh2f;
    uint32_t w = P.hx;
    if (d2 > 0.f) {
        const float w2 = P.Hc2f * 1.000001f - d2 * 0.999999f;
        if (w2 <= 0.f) return false;
        const float wf = __builtin_amdgcn_sqrtf(w2) * 1.000001f + 64.0f;
        w = wf < (float)P.hx ? (uint32_t)wf : P.hx;
    }
    const int nr = (int)P.nr;
    int yy = T.ry + oy;
    yy += (yy < 0) ? nr : 0;
    yy -= (yy >= nr) ? nr : 0;
    int zz = 0;
    if (DIM == 3) {
        zz = T.rz + oz;
        zz += (zz < 0) ? nr : 0;
        zz -= (zz >= nr) ? nr : 0;
    }
    const uint32_t nfx = P.nfx;
    const uint32_t row = P.cbase + ((uint32_t)zz * P.nr + (uint32_t)yy) * nfx;
    const uint32_t clo = __umulhi(T.ux - w, nfx);
    const uint32_t chi = __umulhi(T.ux + w, nfx);
    if (clo <= chi) {
        k0 = row + clo;
        k1 = row + chi;
        k2 = 1u;
        k3 = 0u;
    } else {
        k0 = row + clo;
        k1 = row + nfx - 1u;
        k2 = row;
        k3 = row + chi;
    }
    return true;
}

// Sorted-index ranges [s0, e0) and [s1, e1) of row number j (0 .. noff-1,
// oy fastest) of a target; all empty when the row is out of reach.
struct RowRanges {
    uint32_t s0, e0, s1, e1;
};

template <int DIM>
__device__ __forceinline__ RowRanges row_ranges(const PlumeDev& P, const uint32_t* __restrict__ cs,
                                                const Target& T, int j, int span) {
    RowRanges r{0u, 0u, 0u, 0u};
    const int R = P.R;
    const int oy = j % span - R, oz = (DIM == 3) ? j / span - R : 0;
    uint32_t k0, k1, k2, k3;
    if (row_cells<DIM>(P, T, oy, oz, k0, k1, k2, k3)) {
        r.s0 = cs[k0];
        r.e0 = cs[k1 + 1];
        if (k2 <= k3) {
            r.s1 = cs[k2];
            r.e1 = cs[k3 + 1];
        }
    }
    return r;
}

}  // namespace ade
