// ade_walk.h -- a target's candidate list in LDS (the row windows of the
// cell order that can hold its neighbours), the lane cursor that walks it,
// and a generic batched walk; shared by the pair and adjoint kernels.
#pragma once

#include "ade_geom.h"

namespace ade {

// ---------------------------------------------------------------------------
// Candidate list of a target in LDS, in bytes of the 16-byte record array
// (a context holds fewer than 2^28 - 256 particles, so offsets fit 32 bits
// with room for a cursor step past the end).  Every stored range [s_k, e_k)
// of the sorted order is non-empty.  With one lane per target entry k holds
// (s_k, e_k); with several, (delta_k, e_k), delta_k = s_k - e_(k-1) (e_(-1) =
// 0), so that a lane's overshoot past one range carries into the next.  A
// sentinel closes the list; stepping into it puts the cursor at 2^31 or more
// with the end at 2^30, so no slot is valid after it and no further step is
// taken.  Entries of one target are `stride` apart (the targets of a
// workgroup interleaved), and list[0] is the target's first entry.
// ---------------------------------------------------------------------------
constexpr uint32_t kListEndStart = 0x80000000u, kListEndEnd = 0x40000000u;
constexpr uint32_t kRecBytes = 16;

template <int DIM, int LANES>
__device__ __forceinline__ uint32_t build_list(const PlumeDev& P, const uint32_t* __restrict__ cs,
                                               const Target& T, uint2* list, uint32_t stride) {
    const int span = 2 * P.R + 1;
    const int noff = (DIM == 3) ? span * span : span;
    uint32_t prev = 0, k = 0, total = 0;
    auto put = [&](uint32_t s, uint32_t e) {
        list[k * stride] = make_uint2(LANES == 1 ? s * kRecBytes : s * kRecBytes - prev, e * kRecBytes);
        total += e - s;
        prev = e * kRecBytes;
        ++k;
    };
    // four rows at a time: their cell-start loads are in flight together
    for (int j = 0; j < noff; j += 4) {
        RowRanges r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            r[q] = RowRanges{0u, 0u, 0u, 0u};
            if (j + q < noff) r[q] = row_ranges<DIM>(P, cs, T, j + q, span);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (r[q].e0 > r[q].s0) put(r[q].s0, r[q].e0);
            if (r[q].e1 > r[q].s1) put(r[q].s1, r[q].e1);
        }
    }
    list[k * stride] = make_uint2(LANES == 1 ? kListEndStart : kListEndStart - prev, kListEndEnd);
    return total;
}

// Lane cursor over the concatenated ranges: b is the byte offset of this
// lane's next record, e the end of its range; nx the entry after the current
// one (in flight from LDS).  A step advances b by LANES records.  With one
// lane a step lands exactly on the end of a range and the cursor moves to
// the next entry as it stands; with several, b - e < step exactly when the
// lane has run past the end of its range by less than one step, which is the
// overshoot carried into the next range (perhaps past it).
template <int LANES>
struct Cursor {
    static constexpr uint32_t kStep = LANES * kRecBytes;
    uint32_t b, e;
    uint2 nx;
    const uint2* lp;
    uint32_t stride;
    __device__ __forceinline__ void settle() {
        if (LANES == 1) {
            if (b == e) {
                b = nx.x;
                e = nx.y;
                lp += stride;
                nx = *lp;
            }
        } else {
            while (b - e < kStep) {
                b += nx.x;
                e = nx.y;
                lp += stride;
                nx = *lp;
            }
        }
    }
};

// A generic walk of a one-lane list: the lane evaluates every record of its
// ranges, fetched B at a time with the next batch in flight while the
// current one is evaluated; slots past the end of the list re-read record
// `self` and are passed to eval with keep = false.  The wavefront runs as
// many batches as its longest list needs.
template <int B, typename Fetch, typename Eval>
__device__ __forceinline__ void walk_stream(const uint2* list, uint32_t stride, uint32_t total, uint32_t self,
                                            Fetch&& fetch, Eval&& eval) {
    using CandT = decltype(fetch(0u));
    uint32_t share = total;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) share = max(share, (uint32_t)__shfl_xor((int)share, o, kWave));
    const uint32_t nb = __builtin_amdgcn_readfirstlane((share + B - 1) / B);
    if (nb == 0) return;
    Cursor<1> cur;
    cur.b = 0;
    cur.e = 0;
    cur.lp = list;
    cur.stride = stride;
    cur.nx = list[0];
    cur.settle();
    __builtin_amdgcn_s_waitcnt(0);
    CandT c0[B], c1[B];
    auto fill = [&](CandT(&c)[B]) {
        uint32_t idx[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
            idx[q] = cur.b < cur.e ? cur.b : self * kRecBytes;
            cur.b += Cursor<1>::kStep;
            cur.settle();
        }
#pragma unroll
        for (int q = 0; q < B; ++q) c[q] = fetch(idx[q]);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto run = [&](const CandT(&c)[B], uint32_t batch) {
#pragma unroll
        for (int q = 0; q < B; ++q) eval(c[q], batch * B + q < total);
    };
    fill(c0);
    for (uint32_t it = 1;; it += 2) {
        if (it >= nb) {
            run(c0, it - 1);
            break;
        }
        fill(c1);
        run(c0, it - 1);
        if (it + 1 >= nb) {
            run(c1, it);
            break;
        }
        fill(c0);
        run(c1, it);
    }
}

}  // namespace ade
