// ade_walk.h -- a target's candidate list in LDS (the row windows of the
// cell order that can hold its neighbours), the lane cursor that walks it,
// and a generic batched walk; shared by the pair and adjoint kernels.
#pragma once

#include "ade_geom.h"

namespace ade {

// ---------------------------------------------------------------------------
// Candidate list of a target in LDS (entry k at list[k * stride], a 24-bit
// multiply: both factors are below the LDS size): entries (s_k, e_k), in bytes of the
// 16-byte record array (a context holds fewer than 2^28 - 256 particles, so
// offsets fit 32 bits with room for a cursor step past the end), each a
// non-empty range [s_k, e_k) of the sorted order, touching ranges stored as
// one.  The rows are listed plane by plane (oz), in order of oy inside a
// plane, and a row whose window wraps around the periodic x seam gives its
// low part (at the start of the row) before its high part (which ends at the
// end of the row, where the next row of the plane begins).  A window narrows
// away from the target's own row, so the rows of a plane whose windows wrap
// are consecutive: each wrapped row's high part merges with the next wrapped
// row's low part, and a plane of n rows takes at most n + 1 entries, n + 2
// when the row index wraps around the box among them.  A sentinel closes the
// list; stepping into it puts the cursor at 2^31 or more with the end at
// 2^30, so no slot is valid after it and no further step is taken.  Entries
// of one target are `stride` apart (the targets of a workgroup interleaved),
// and list[0] is the target's first entry.
// ---------------------------------------------------------------------------
constexpr uint32_t kListEndStart = 0x80000000u, kListEndEnd = 0x40000000u;
constexpr uint32_t kRecBytes = 16;

// Appends ranges to a list, merging a range that starts where the pending
// one ends; flush() writes the pending range and the sentinel.
struct ListWriter {
    uint2* list;
    uint32_t stride, k = 0, total = 0, ps = 0, pe = 0;  // pe == 0: nothing pending
    __device__ __forceinline__ ListWriter(uint2* l, uint32_t s) : list(l), stride(s) {}
    __device__ __forceinline__ void put(uint32_t s, uint32_t e) {
        if (pe != 0u && s == pe) {
            pe = e;
            return;
        }
        if (pe != 0u) {
            list[__umul24(k, stride)] = make_uint2(ps * kRecBytes, pe * kRecBytes);
            total += pe - ps;
            ++k;
        }
        ps = s;
        pe = e;
    }
    __device__ __forceinline__ uint32_t flush() {
        if (pe != 0u) {
            list[__umul24(k, stride)] = make_uint2(ps * kRecBytes, pe * kRecBytes);
            total += pe - ps;
            ++k;
        }
        list[__umul24(k, stride)] = make_uint2(kListEndStart, kListEndEnd);
        return total;
    }
};

// Lane permutations inside a quad of lanes (full-rate DPP moves).  Every
// source lane is inside the quad, so with all lanes of the quad active no
// lane keeps its previous value (none is given).
template <int CTRL>
__device__ __forceinline__ uint32_t quad_perm(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

// The list as one lane builds it alone (every lane of a target builds the
// same list when LANES == 1).
template <int DIM>
__device__ __forceinline__ uint32_t build_list_lane(const PlumeDev& P, const uint32_t* __restrict__ cs,
                                                    const Target& T, uint2* list, uint32_t stride) {
    const int R = P.R, span = 2 * R + 1;
    const int noff = (DIM == 3) ? span * span : span;
    ListWriter w(list, stride);
    int oy = -R, oz = -R;  // row j of the loop below
    // four rows at a time: their cell-start loads are in flight together
    for (int j = 0; j < noff; j += 4) {
        RowRanges r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            r[q] = RowRanges{0u, 0u, 0u, 0u};
            if (j + q < noff) r[q] = row_ranges_at<DIM>(P, cs, T, oy, (DIM == 3) ? oz : 0);
            next_row(oy, oz, 1, R, span);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (r[q].e1 > r[q].s1) w.put(r[q].s1, r[q].e1);  // low part of a wrapped row first
            if (r[q].e0 > r[q].s0) w.put(r[q].s0, r[q].e0);
        }
    }
    return w.flush();
}

// The same ranges listed by the G lanes that serve one target (G = 2 or 4,
// consecutive lanes of a quad) together: lane g computes rows g, g + G, ...,
// and each round of G rows is written in row order at positions from a
// prefix count over the group.  A row's low part that starts where the
// previous row's range ends (a wrapped row after a wrapped row) extends that
// row's entry instead of taking its own, so the bound of n + 2 entries per
// plane of n rows holds as for ListWriter: in a run of wrapped rows, every
// pair of neighbouring rows either merges or has one of the two parts empty.
template <int DIM, int G>
__device__ __forceinline__ uint32_t build_list_group(const PlumeDev& P, const uint32_t* __restrict__ cs,
                                                     const Target& T, uint2* list, uint32_t stride) {
    // quad_perm controls: the previous lane of the group, the lane two back,
    // the group's last lane, and the two butterflies of a sum
    constexpr int kPrev = (G == 4) ? 0x90 : 0xA0;  // [0,0,1,2] / [0,0,2,2]
    constexpr int kPrev2 = 0x40;                    // [0,0,0,1]
    constexpr int kLast = (G == 4) ? 0xFF : 0xF5;  // [3,3,3,3] / [1,1,3,3]
    const uint32_t g = threadIdx.x & (G - 1);
    const int R = P.R, span = 2 * R + 1;
    const int noff = (DIM == 3) ? span * span : span;
    uint32_t base = 0, total = 0;
    uint32_t pS = 0, pE = 0;  // main range of the row before the round (end 0: none)
    // this lane's row j0 + g as offsets, stepped on by G rows a round (no
    // division by span per row)
    int oy = -R, oz = -R;
    next_row(oy, oz, (int)g, R, span);
    for (int j0 = 0; j0 < noff; j0 += G) {
        RowRanges r{0u, 0u, 0u, 0u};
        if (j0 + (int)g < noff) r = row_ranges_at<DIM>(P, cs, T, oy, (DIM == 3) ? oz : 0);
        next_row(oy, oz, G, R, span);
        const bool hasL = r.e1 > r.s1, hasH = r.e0 > r.s0;
        const uint32_t hS = hasH ? r.s0 : 0u, hE = hasH ? r.e0 : 0u;
        // main range of the previous row
        uint32_t qS = quad_perm<kPrev>(hS), qE = quad_perm<kPrev>(hE);
        if (g == 0) {
            qS = pS;
            qE = pE;
        }
        const bool mergeL = hasL && qE != 0u && qE == r.s1;
        const uint32_t cnt = ((hasL && !mergeL) ? 1u : 0u) + (hasH ? 1u : 0u);
        // inclusive prefix over the group; every lane takes part in the moves
        // (a move from a lane masked off by a branch would read nothing)
        uint32_t incl = cnt + (quad_perm<kPrev>(cnt) & (g >= 1 ? ~0u : 0u));
        if (G == 4) incl += quad_perm<kPrev2>(incl) & (g >= 2 ? ~0u : 0u);
        const uint32_t first = base + incl - cnt;
        uint32_t pos = first;
        if (hasL && !mergeL) {
            list[__umul24(pos, stride)] = make_uint2(r.s1 * kRecBytes, r.e1 * kRecBytes);
            ++pos;
        }
        if (hasH) list[__umul24(pos, stride)] = make_uint2(r.s0 * kRecBytes, r.e0 * kRecBytes);
        // the previous row's entry, extended by a merged low part, is
        // rewritten after the round's entries (the LDS writes of a wavefront
        // take effect in program order)
        asm volatile("" ::: "memory");
        if (mergeL) list[__umul24(first - 1u, stride)] = make_uint2(qS * kRecBytes, r.e1 * kRecBytes);
        total += (r.e1 - r.s1) + (r.e0 - r.s0);
        base += quad_perm<kLast>(incl);
        pS = quad_perm<kLast>(hS);
        pE = quad_perm<kLast>(hE);
    }
    list[__umul24(base, stride)] = make_uint2(kListEndStart, kListEndEnd);
    total += quad_perm<0xB1>(total);                // [1,0,3,2]
    if (G == 4) total += quad_perm<0x4E>(total);    // [2,3,0,1]
    return total;
}

// The same cooperative build over any block of ny x nz rows starting at row
// offsets (oy0, oz0) (oy fastest), the ranges of row (oy, oz) given by
// rows(oy, oz): for two neighbouring targets served by the four lanes of a
// quad, whose rows are union_row's arcs (G = 4).
template <typename RowFn>
__device__ __forceinline__ uint32_t build_rows_quad(RowFn&& rows, int ny, int nz, int oy0, int oz0, uint2* list,
                                                    uint32_t stride) {
    constexpr int G = 4;
    constexpr int kPrev = 0x90, kPrev2 = 0x40, kLast = 0xFF;  // as in build_list_group, G = 4
    const uint32_t g = threadIdx.x & (G - 1);
    const int nrows = ny * nz, oy1 = oy0 + ny - 1;
    auto step = [&](int& oy, int& oz, int n) {  // n <= 2 ny
        oy += n;
        if (oy > oy1) {
            oy -= ny;
            ++oz;
        }
        if (oy > oy1) {
            oy -= ny;
            ++oz;
        }
    };
    uint32_t base = 0, total = 0;
    uint32_t pS = 0, pE = 0;  // main range of the row before the round (end 0: none)
    int oy = oy0, oz = oz0;
    step(oy, oz, (int)g);
    for (int j0 = 0; j0 < nrows; j0 += G) {
        RowRanges r{0u, 0u, 0u, 0u};
        if (j0 + (int)g < nrows) r = rows(oy, oz);
        step(oy, oz, G);
        const bool hasL = r.e1 > r.s1, hasH = r.e0 > r.s0;
        const uint32_t hS = hasH ? r.s0 : 0u, hE = hasH ? r.e0 : 0u;
        uint32_t qS = quad_perm<kPrev>(hS), qE = quad_perm<kPrev>(hE);
        if (g == 0) {
            qS = pS;
            qE = pE;
        }
        const bool mergeL = hasL && qE != 0u && qE == r.s1;
        const uint32_t cnt = ((hasL && !mergeL) ? 1u : 0u) + (hasH ? 1u : 0u);
        uint32_t incl = cnt + (quad_perm<kPrev>(cnt) & (g >= 1 ? ~0u : 0u));
        incl += quad_perm<kPrev2>(incl) & (g >= 2 ? ~0u : 0u);
        const uint32_t first = base + incl - cnt;
        uint32_t pos = first;
        if (hasL && !mergeL) {
            list[__umul24(pos, stride)] = make_uint2(r.s1 * kRecBytes, r.e1 * kRecBytes);
            ++pos;
        }
        if (hasH) list[__umul24(pos, stride)] = make_uint2(r.s0 * kRecBytes, r.e0 * kRecBytes);
        asm volatile("" ::: "memory");
        if (mergeL) list[__umul24(first - 1u, stride)] = make_uint2(qS * kRecBytes, r.e1 * kRecBytes);
        total += (r.e1 - r.s1) + (r.e0 - r.s0);
        base += quad_perm<kLast>(incl);
        pS = quad_perm<kLast>(hS);
        pE = quad_perm<kLast>(hE);
    }
    list[__umul24(base, stride)] = make_uint2(kListEndStart, kListEndEnd);
    total += quad_perm<0xB1>(total);
    total += quad_perm<0x4E>(total);
    return total;
}

template <int DIM, int LANES>
__device__ __forceinline__ uint32_t build_list(const PlumeDev& P, const uint32_t* __restrict__ cs,
                                               const Target& T, uint2* list, uint32_t stride) {
    if (LANES == 2 || LANES == 4) return build_list_group<DIM, LANES>(P, cs, T, list, stride);
    return build_list_lane<DIM>(P, cs, T, list, stride);
}

// Lane cursor over the concatenated ranges: b is the byte offset of this
// lane's next record, e the end of its range; nx the entry after the current
// one (in flight from LDS).  A step advances b by LANES records.  With one
// lane a step lands exactly on the end of a range and the cursor moves to
// the next entry as it stands; with several, b - e < step exactly when the
// lane has run past the end of its range by less than one step, and that
// overshoot is carried into the next range (perhaps past it).
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
                b = nx.x + (b - e);
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
// many batches as its longest list needs; in the batches where every lane
// still has records, the slots need no end-of-list test and eval gets
// keep = true as a constant.
template <int B, typename Fetch, typename Eval>
__device__ __forceinline__ void walk_stream(const uint2* list, uint32_t stride, uint32_t total, uint32_t self,
                                            Fetch&& fetch, Eval&& eval) {
    using CandT = decltype(fetch(0u));
    uint32_t share = total, least = total;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        share = max(share, (uint32_t)__shfl_xor((int)share, o, kWave));
        least = min(least, (uint32_t)__shfl_xor((int)least, o, kWave));
    }
    const uint32_t nb = __builtin_amdgcn_readfirstlane((share + B - 1) / B);
    if (nb == 0) return;
    const uint32_t nfull = __builtin_amdgcn_readfirstlane(least / B);
    Cursor<1> cur;
    cur.b = 0;
    cur.e = 0;
    cur.lp = list;
    cur.stride = stride;
    cur.nx = list[0];
    cur.settle();
    __builtin_amdgcn_s_waitcnt(0);
    CandT c0[B], c1[B];
    auto fill = [&](CandT(&c)[B], uint32_t it) {
        uint32_t idx[B];
        if (it < nfull) {
#pragma unroll
            for (int q = 0; q < B; ++q) {
                idx[q] = cur.b;
                cur.b += Cursor<1>::kStep;
                cur.settle();
            }
        } else {
#pragma unroll
            for (int q = 0; q < B; ++q) {
                idx[q] = cur.b < cur.e ? cur.b : self * kRecBytes;
                cur.b += Cursor<1>::kStep;
                cur.settle();
            }
        }
#pragma unroll
        for (int q = 0; q < B; ++q) c[q] = fetch(idx[q]);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto run = [&](const CandT(&c)[B], uint32_t batch) {
        if (batch < nfull) {
#pragma unroll
            for (int q = 0; q < B; ++q) eval(c[q], true);
        } else {
#pragma unroll
            for (int q = 0; q < B; ++q) eval(c[q], batch * B + q < total);
        }
    };
    fill(c0, 0u);
    for (uint32_t it = 1;; it += 2) {
        if (it >= nb) {
            run(c0, it - 1);
            break;
        }
        fill(c1, it);
        run(c0, it - 1);
        if (it + 1 >= nb) {
            run(c1, it);
            break;
        }
        fill(c0, it + 1);
        run(c1, it);
    }
}

// Walk a target's list: every lane evaluates its share of the concatenated
// ranges in batches of B records.  The wavefront runs as many batches as its
// longest share needs (a uniform count, from the list totals); a slot past
// the end of a lane's share re-reads the target's own record (index self),
// which the predicate rejects (r2 = 0).  So every load is unconditional, and
// the loads of one batch stay in flight, in order, while the previous batch
// is evaluated.
template <int LANES, int B, typename Fetch, typename Eval>
__device__ __forceinline__ void walk_list_fn(uint32_t self, const uint2* list, uint32_t stride, uint32_t total,
                                             uint32_t lj, Fetch&& fetch, Eval&& evalrec) {
    using CandT = decltype(fetch(0u));
    // batches of the wavefront: the largest share of its lanes, in batches
    const uint32_t own = total > lj ? (total - lj + LANES - 1) / LANES : 0u;
    uint32_t share = own, least = own;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        share = max(share, (uint32_t)__shfl_xor((int)share, o, kWave));
        least = min(least, (uint32_t)__shfl_xor((int)least, o, kWave));
    }
    const uint32_t nb = __builtin_amdgcn_readfirstlane((share + B - 1) / B);
    if (nb == 0) return;
    // batches in which every lane of the wavefront still has records of its
    // own: their slots need no end-of-list test
    const uint32_t nfull = __builtin_amdgcn_readfirstlane(least / B);

    Cursor<LANES> cur;
    cur.b = lj * kRecBytes;
    cur.e = 0;
    cur.lp = list;
    cur.stride = stride;
    cur.nx = list[0];
    cur.settle();

    // nothing older than the first batch is in flight when the loop starts,
    // so both entries into the loop carry the same outstanding loads
    __builtin_amdgcn_s_waitcnt(0);
    CandT c0[B], c1[B];
    bool k0[B], k1[B];  // false: a padding slot
    // fill batch `it`: past the full batches a slot beyond the lane's share
    // re-reads the target's own record
    auto fill = [&](CandT(&c)[B], bool(&keep)[B], uint32_t it) {
        uint32_t idx[B];
        if (it < nfull) {
#pragma unroll
            for (int q = 0; q < B; ++q) {
                idx[q] = cur.b;
                keep[q] = true;
                cur.b += Cursor<LANES>::kStep;
                cur.settle();
            }
        } else {
#pragma unroll
            for (int q = 0; q < B; ++q) {
                keep[q] = cur.b < cur.e;
                idx[q] = keep[q] ? cur.b : self * kRecBytes;
                cur.b += Cursor<LANES>::kStep;
                cur.settle();
            }
        }
#pragma unroll
        for (int q = 0; q < B; ++q) c[q] = fetch(idx[q]);
        // keep the loads here, ahead of the evaluation they overlap with
        __builtin_amdgcn_sched_barrier(0);
    };
    auto eval = [&](const CandT(&c)[B], const bool(&keep)[B], uint32_t it) {
        if (it < nfull) {
#pragma unroll
            for (int q = 0; q < B; ++q) evalrec(c[q], true);
        } else {
#pragma unroll
            for (int q = 0; q < B; ++q) evalrec(c[q], keep[q]);
        }
    };
    fill(c0, k0, 0u);
    for (uint32_t it = 1;; it += 2) {
        if (it >= nb) {
            eval(c0, k0, it - 1);
            break;
        }
        fill(c1, k1, it);
        eval(c0, k0, it - 1);
        if (it + 1 >= nb) {
            eval(c1, k1, it);
            break;
        }
        fill(c0, k0, it + 1);
        eval(c1, k1, it);
    }
}

// ---------------------------------------------------------------------------
// Two neighbouring targets a and b of the cell order sharing one list: the
// rows that can hold a neighbour of either, each row's x window the
// smallest arc holding the windows of the targets that reach it.  Used by
// the uniform-flow and the velocity-field pair kernels.
// ---------------------------------------------------------------------------
// Whether a and b can share a list: their rows at most one apart per axis
// (dy, dz: b's row offsets from a's) and their separation small enough for
// b's separations to be formed from a's.
template <int DIM>
__device__ __forceinline__ bool pair_rows(const PlumeDev& P, const Target& A, const Target& B, int& dy, int& dz) {
    const int nr = (int)P.nr, span = 2 * P.R + 1;
    auto circ = [&](int d) {
        if (2 * d > nr) d -= nr;
        if (2 * d < -nr) d += nr;
        return d;
    };
    dy = circ(B.ry - A.ry);
    dz = (DIM == 3) ? circ(B.rz - A.rz) : 0;
    // |x_b - x_a| + H_u < 2^31 per axis: then for every neighbour c of b the
    // integer sum (x_b - x_a) + (x_a - x_c) does not wrap, and walk_pair's
    // separations of b are those of the minimum image
    auto near = [&](uint32_t ub, uint32_t ua) {
        const int32_t d = (int32_t)(ub - ua);
        return (uint32_t)(d < 0 ? -(int64_t)d : (int64_t)d) + P.hx < 0x80000000u;
    };
    const bool close = near(B.ux, A.ux) && near(B.uy, A.uy) && (DIM != 3 || near(B.uz, A.uz));
    return close && span + 1 <= nr && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
}

// Sorted-index ranges of the pair's row (oy, oz), offsets from a's row:
// (s1, e1) is the low part of a row cut by the seam (empty otherwise), (s0,
// e0) the rest.  The arc is the smallest one holding the windows of the
// targets that reach the row, taken in x cells in a's frame (b at A.xc +
// dxc, dxc = (x_b - x_a) in x cells), with the slack of row_ranges_at.
template <int DIM>
__device__ __forceinline__ RowRanges union_row(const PlumeDev& P, const uint32_t* __restrict__ cs, const Target& A,
                                               const Target& B, float dxc, int dy, int dz, int oy, int oz) {
    const int R = P.R;
    float wa = 0.f, wb = 0.f;
    const bool ra = abs(oy) <= R && abs(oz) <= R && row_halfwidth_f<DIM>(P, A, oy, oz, wa);
    const bool rb = abs(oy - dy) <= R && abs(oz - dz) <= R && row_halfwidth_f<DIM>(P, B, oy - dy, oz - dz, wb);
    if (!ra && !rb) return RowRanges{0u, 0u, 0u, 0u};
    const float wac = fmar(wa, P.cellx, P.cslack), wbc = fmar(wb, P.cellx, P.cslack);
    const float xb = A.xc + dxc;
    float lo = ra ? A.xc - wac : xb - wbc;
    float hi = ra ? A.xc + wac : xb + wbc;
    if (ra && rb) {
        lo = fminf(lo, xb - wbc);
        hi = fmaxf(hi, xb + wbc);
    }
    const int yy = wrap_row(P, A.ry + oy);
    const int zz = (DIM == 3) ? wrap_row(P, A.rz + oz) : 0;
    return window_ranges(P, cs, row_base(P, yy, zz), lo, hi);
}

}  // namespace ade
