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

// x clamped to [0, 1] (NaN to 0): for FP32 the clamp bit of the instruction
// that forms x
__device__ __forceinline__ float clamp_unit(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ __forceinline__ double clamp_unit(double x) { return x > 0.0 ? (x < 1.0 ? x : 1.0) : 0.0; }
// max(x, 0) of an x <= 1 (1 - q with q >= 0; NaN to 0): for FP32 the clamp
// bit of the instruction that forms x, one compare and select for FP64
__device__ __forceinline__ float pos_unit(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ __forceinline__ double pos_unit(double x) { return x > 0.0 ? x : 0.0; }

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
    float xc;  // x in x cells of the plume (float; PlumeDev::cslack covers its rounding)
};

template <int DIM>
__device__ __forceinline__ Target make_target(const PlumeDev& P, uint32_t ux, uint32_t uy, uint32_t uz) {
    Target t;
    t.ux = ux;
    t.uy = uy;
    t.uz = uz;
    t.xc = (float)ux * P.cellx;
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

// Squared distance (grid units) from a target to the nearest edge of its
// neighbour row (oy, oz), without branches: along each axis the distance is
// oy - fy above the target's row, -oy - 1 + fy below it and 0 in it, which is
// the largest of the three.
template <int DIM>
__device__ __forceinline__ float row_edge_d2(const PlumeDev& P, const Target& T, int oy, int oz) {
    const float dy = fmaxf(fmaxf((float)oy - T.fy, (float)(-oy - 1) + T.fy), 0.f);
    float dz = 0.f;
    if (DIM == 3) dz = fmaxf(fmaxf((float)oz - T.fz, (float)(-oz - 1) + T.fz), 0.f);
    return (dy * dy + dz * dz) * P.rowh2f;
}

// Half-width of the x window of a target in its neighbour row (oy, oz), as a
// float in grid units: an upper bound of the chord of the search radius at
// the row's nearest edge (the search radius itself in the target's own row,
// where the bound exceeds hx and hx is taken); false when the row lies beyond
// the search radius.  The bound is conservative: the float rounding of the
// distances is covered by relative slack on w^2 and an absolute slack of 64
// grid units on w.
template <int DIM>
__device__ __forceinline__ bool row_halfwidth_f(const PlumeDev& P, const Target& T, int oy, int oz, float& w) {
    const float w2 = P.Hc2f * 1.000001f - row_edge_d2<DIM>(P, T, oy, oz) * 0.999999f;
    // (w is meaningless, and unused, when the row is out of reach)
    const float wf = __builtin_amdgcn_sqrtf(w2) * 1.000001f + 64.0f;
    w = fminf(wf, (float)P.hx);
    return w2 > 0.f;
}

// The same as a whole number of grid units (hx in the target's own row).
template <int DIM>
__device__ __forceinline__ bool row_halfwidth(const PlumeDev& P, const Target& T, int oy, int oz, uint32_t& w) {
    const float w2 = P.Hc2f * 1.000001f - row_edge_d2<DIM>(P, T, oy, oz) * 0.999999f;
    const float wf = __builtin_amdgcn_sqrtf(w2) * 1.000001f + 64.0f;
    w = wf < (float)P.hx ? (uint32_t)wf : P.hx;
    return w2 > 0.f;
}

// First cell of row (yy, zz) of a plume (row indices already wrapped; the
// plan keeps nr, nfx and nsub, the rows of a plume and the cells of a row
// below 2^24, so both products are 24-bit multiplies).
__device__ __forceinline__ uint32_t row_base(const PlumeDev& P, int yy, int zz) {
    return P.cbase + __umul24(__umul24((uint32_t)zz, P.nr) + (uint32_t)yy, P.nfx * P.nsub);
}

// y in -nr .. 2 nr - 1 wrapped into 0 .. nr - 1 (as unsigned values, the
// wrapped one is the smallest of y, y + nr and y - nr)
__device__ __forceinline__ int wrap_row(const PlumeDev& P, int y) {
    uint32_t u = (uint32_t)y;
    u = min(u, u + P.nr);
    u = min(u, u - P.nr);
    return (int)u;
}

// Sorted-index ranges of row number j (0 .. noff-1, oy fastest) of a target:
// [s0, e0) the cells of its x window, and when the window wraps around the
// periodic x seam [s1, e1) its low part at the start of the row ([s0, e0)
// then ends at the end of the row); all empty when the row is out of reach.
struct RowRanges {
    uint32_t s0, e0, s1, e1;
};

// Entry k of the cell-start table (tables are addressed with 32-bit byte
// offsets from the table's base: a context holds fewer than 2^30 cells).
__device__ __forceinline__ uint32_t cell_start_at(const uint32_t* __restrict__ cs, uint32_t k) {
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(cs) + (k << 2));
}

// Sorted-index ranges of the x cells floor(lo) .. floor(hi) of the row whose
// first cell is `row`, the window given in x cells (float, slack included,
// hi - lo < 2 nfx and -nfx <= lo, hi < 2 nfx: a window around a point of the
// box), taken around the periodic seam: [s0, e0) and, when the window wraps,
// its low part [s1, e1) at the start of the row; a window of a whole row or
// more takes the whole row.
__device__ __forceinline__ RowRanges window_ranges(const PlumeDev& P, const uint32_t* __restrict__ cs,
                                                   uint32_t row, float lo, float hi) {
    RowRanges r{0u, 0u, 0u, 0u};
    const int nfx = (int)P.nfx;
    const uint32_t ns = P.nsub;
    int clo = __float2int_rd(lo), chi = __float2int_rd(hi);
    if (chi < 0) {  // the whole window left of the seam
        clo += nfx;
        chi += nfx;
    } else if (clo >= nfx) {  // the whole window right of it
        clo -= nfx;
        chi -= nfx;
    }
    int hi2 = -1;  // the low part [0, hi2] of a window that wraps around the seam
    if (chi - clo + 1 >= nfx) {
        clo = 0;
        chi = nfx - 1;
    } else if (clo < 0) {
        hi2 = chi;
        clo += nfx;
        chi = nfx - 1;
    } else if (chi >= nfx) {
        hi2 = chi - nfx;
        chi = nfx - 1;
    }
    r.s0 = cell_start_at(cs, row + __umul24((uint32_t)clo, ns));
    r.e0 = cell_start_at(cs, row + __umul24((uint32_t)(chi + 1), ns));
    if (hi2 >= 0) {
        r.s1 = cell_start_at(cs, row);
        r.e1 = cell_start_at(cs, row + __umul24((uint32_t)(hi2 + 1), ns));
    }
    return r;
}

// Row (oy, oz) relative to the target's own row, |oy|, |oz| <= R.
template <int DIM>
__device__ __forceinline__ RowRanges row_ranges_at(const PlumeDev& P, const uint32_t* __restrict__ cs,
                                                   const Target& T, int oy, int oz) {
    RowRanges r{0u, 0u, 0u, 0u};
    float w;
    if (!row_halfwidth_f<DIM>(P, T, oy, oz, w)) return r;
    // the window [x - w, x + w] in x cells, widened by the slack: a superset
    // of the cells the exact window touches
    const float wc = fmar(w, P.cellx, P.cslack);
    const int yy = wrap_row(P, T.ry + oy);
    const int zz = (DIM == 3) ? wrap_row(P, T.rz + oz) : 0;
    return window_ranges(P, cs, row_base(P, yy, zz), T.xc - wc, T.xc + wc);
}

// Row number j (0 .. noff-1, oy fastest) of a target, span = 2R + 1.
template <int DIM>
__device__ __forceinline__ RowRanges row_ranges(const PlumeDev& P, const uint32_t* __restrict__ cs,
                                                const Target& T, int j, int span) {
    return row_ranges_at<DIM>(P, cs, T, j % span - P.R, (DIM == 3) ? j / span - P.R : 0);
}

// Steps a row offset (oy, oz) on by n rows in the order of row_ranges (oy
// fastest), for n <= 2 span.
__device__ __forceinline__ void next_row(int& oy, int& oz, int n, int R, int span) {
    oy += n;
    if (oy > R) {
        oy -= span;
        ++oz;
    }
    if (oy > R) {
        oy -= span;
        ++oz;
    }
}

}  // namespace ade
