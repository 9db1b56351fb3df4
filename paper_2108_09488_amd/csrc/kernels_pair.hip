// kernels_pair.hip -- the SPH pair sum of Eqs. (4)-(5) (Klapp et al.,
// arXiv:2108.09488, Section 2.2) on gfx950, fused with the explicit update of
// C and x and with the hashing of the moved particle for the next cell build.
//
// For a uniform flow the harmonic mean of Eq. (5) of two equal tensors is 2 D,
// so the pair term is
//     tau_ab = V [Gamma (x_ab^T D x_ab) / r^2 - tr D] (C_a - C_b) W'(r) / r,
// with V = m / rho and, for the Wendland kernels of Eq. (7) with support H,
//     C4: W'(r)/r = -(56/3) (B / H^2) (1 - q)^5 (1 + 5 q),
//     C2: W'(r)/r = -20 (B / H^2) (1 - q)^3,        q = r / H.
// With D from Eq. (3) the bracket is a0 + a1 (e . x_ab / r)^2, e = v / |v|,
// a0 = (Gamma - d)(alpha_T |v| + D_m) - (alpha_L - alpha_T)|v| and
// a1 = Gamma (alpha_L - alpha_T)|v|; |a1| is folded into the direction,
// E = sqrt|a1| e, so that the bracket is A0 +- (E . x_ab / r)^2 (see
// PlumeDev::dterm).  Separations are taken in grid units (L / 2^32) from the
// fixed-point positions; the bracket is scale free and the constant factor
// V (W'(r)/r)/f(q) is applied once per particle (PlumeDev::vphi).  For C4
// the kernel factor is evaluated as w^4 (w - 5/6 w^2) = (1 - q)^5 (1 + 5q) / 6
// (w = 1 - q), the 6 going with that constant factor.
//
// Neighbour predicate (the neighbour-list export applies it exactly): d =
// (int32)(u_a - u_b) per component (the two's-complement wrap is the minimum
// image), converted to the working precision, r2 = d_x d_x, r2 = fma(d_y,
// d_y, r2) [, r2 = fma(d_z, d_z, r2)], pair iff 0 < r2 <= H_u^2 (inclusive
// support).  The pair sum imposes r <= H through the kernel factor, which is
// 0 at q = 1 (clamp of 1 - q at 0), and r > 0 as PairTerm describes.
//
// Candidates: particles are sorted by (row, x cell), rows being a grid of
// height >= Hc / R in y (and z).  For each of the (2R+1)^(d-1) rows around a
// target, the x cells that can hold neighbours form one contiguous range of
// the sorted order (two at the periodic seam), cut to the chord of the
// search radius at the row's nearest edge.  A target's non-empty ranges are
// listed in LDS, in row order, and its LANES lanes walk the concatenation of
// the list as one stream (lane j takes elements j, j + LANES, ...): a lane
// crosses from one range into the next inside a batch, so candidates are
// fetched in batches of kBatch records with no per-row rounding and no
// pipeline drain at a row boundary.  The next batch is in flight while the
// current one is evaluated.
#include <hip/hip_ext.h>

#include "ade_walk.h"

namespace ade {

// One candidate: the pair term, evaluated without a branch (the lanes of a
// wavefront almost never all fail the predicate together); the kernel factor
// vanishes outside the support, and a candidate at r = 0 adds nothing.
// the constant the kernel factor of the pair term leaves out: its value at q = 0
template <int KERN>
constexpr double kPolyScale = (KERN == 4) ? 6.0 : 1.0;

// the bracket is A0 + S (E . x / r)^2 with S = +-1 (PlumeDev::dterm; in 2D
// S = +1 always).  The term forms S times it, (E . x / r)^2 + S A0, and
// finish_target multiplies the sum by S.
// ZC (zero separations): two distinct particles may share a position, so a
// candidate at r = 0 is cut by a select.  Without ZC the only candidate at
// r = 0 is the target's own record (a padding slot re-reads it): r^2 starts
// from a tiny offset (2^-40 in FP32), far below half a unit in the last place
// of any r^2 >= 1 (grid units), so it changes such an r^2 only where the
// exact sum sits on a rounding tie (then by one unit in the last place); it
// keeps the self term finite, and the self term is w (C_a - C_a) = 0 exactly.
template <typename real>
constexpr real kTinyR2 = sizeof(real) == 4 ? (real)9.094947017729282e-13 : (real)7.888609052210118e-31;  // 2^-40, 2^-100
template <int DIM, typename real, int KERN, bool ZC>
struct PairTerm {
    real invHu, a0s, ex, ey, ez;
    __device__ __forceinline__ void operator()(const Target& T, real Ca, uint32_t bx, uint32_t by,
                                               uint32_t bz, real Cb, real& acc) const {
        (*this)(T, Ca, bx, by, bz, Cb, true, acc);
    }
    // the same, added only if keep (a padding slot of a walk shared by two
    // targets)
    __device__ __forceinline__ void operator()(const Target& T, real Ca, uint32_t bx, uint32_t by,
                                               uint32_t bz, real Cb, bool keep, real& acc) const {
        const real dx = (real)(int32_t)(T.ux - bx);
        const real dy = (real)(int32_t)(T.uy - by);
        const real dz = (DIM == 3) ? (real)(int32_t)(T.uz - bz) : (real)0;
        sep(dx, dy, dz, Ca, Cb, keep, acc);
    }
    // the same from the separation (dx, dy, dz) = x_a - x_b in grid units
    __device__ __forceinline__ void sep(real dx, real dy, real dz, real Ca, real Cb, bool keep, real& acc) const {
        real r2 = ZC ? dx * dx : fmar(dx, dx, kTinyR2<real>);
        r2 = fmar(dy, dy, r2);
        if (DIM == 3) r2 = fmar(dz, dz, r2);
        // with ZC, r2 = 0 (the target itself, a padding slot, a coincident
        // particle) is cut by the select below; the support r <= H by the
        // clamp of 1 - q at 0, which zeroes the kernel factor outside it (W is
        // 0 at q = 1, so where the rounding of r puts 1 - q on the other side
        // of 0 the term is below 1e-28 of a typical one either way)
        const bool inside = ZC ? (keep && r2 > (real)0) : keep;
        const real rinv = rsqrt_r(r2);
        const real r = r2 * rinv;
        const real omq = clamp_unit(fmar(-r, invHu, (real)1));
        real f;
        if (KERN == 4) {  // (1 - q)^5 (1 + 5q) / 6
            const real o2 = omq * omq;
            f = (o2 * o2) * fmar((real)(-5.0 / 6.0), o2, omq);
        } else {
            f = omq * omq * omq;
        }
        real p = ex * dx;
        p = fmar(ey, dy, p);
        if (DIM == 3) p = fmar(ez, dz, p);
        const real pr = p * rinv;
        const real A = fmar(pr, pr, a0s);  // S times the bracket
        const real w = inside ? A * f : (real)0;
        acc = fmar(w, Ca - Cb, acc);
    }
};

// the constants come from the plume table as they are (FP32 copies for FP32),
// so they stay in scalar registers
template <int DIM, typename real, int KERN, bool ZC>
__device__ __forceinline__ PairTerm<DIM, real, KERN, ZC> make_term(const PlumeDev& P) {
    PairTerm<DIM, real, KERN, ZC> t;
    real c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = (sizeof(real) == 4) ? (real)P.fterm[k] : (real)P.dterm[k];
    t.invHu = c[1];
    t.a0s = c[3] * c[4];
    t.ex = c[5];
    t.ey = c[6];
    t.ez = c[7];
    return t;
}


template <typename real>
struct Cand {
    uint32_t x, y, z;
    real C;
};

template <int DIM, typename real>
__device__ __forceinline__ Cand<real> unpack(const uint4& r) {
    return Cand<real>{r.x, r.y, (DIM == 3) ? r.z : 0u, Rec<DIM, real>::conc(r)};
}

// Walk a target's list: every lane evaluates its share of the concatenated
// ranges in batches of B records.  The wavefront runs as many batches as its
// longest share needs (a uniform count, from the list totals); a slot past
// the end of a lane's share re-reads the target's own record (index self),
// which the predicate rejects (r2 = 0).  So every load is unconditional, and
// the loads of one batch stay in flight, in order, while the previous batch
// is evaluated.  (walk_list_fn is the same walk with any evaluation of a
// record.)
template <int LANES, typename Term, typename real, typename Fetch>
__device__ __forceinline__ void walk_list(const Term& term, const Target& T,
                                          real Ca, uint32_t self, const uint2* list, uint32_t stride,
                                          uint32_t total, uint32_t lj, Fetch&& fetch, real& acc) {
    walk_list_fn<LANES, Batch<LANES>::value>(self, list, stride, total, lj, fetch, [&](const Cand<real>& c, bool) {
        term(T, Ca, c.x, c.y, c.z, c.C, acc);
    });
}

// The end of a target's pair sum acc: rhs mode writes the right-hand side
// (vphi * acc) in id order; half mode the half-step concentration (and its
// candidate record); step mode updates C and x and returns the moved
// particle's cell key (its id in id), which the caller enters into the next
// build's cell lists (enlist).
template <int DIM, typename real, int KERN, int MODE>
__device__ __forceinline__ uint32_t finish_core(const PairLaunch& a, const PlumeDev& P, const Target& T, uint32_t i,
                                                real acc, uint32_t& id) {
    constexpr bool kRec = Rec<DIM, real>::kStageable;
    // the kernel factor's constant and the bracket's sign S (the pair term
    // sums S times the bracket)
    const double kS = kPolyScale<KERN> * P.dterm[4];
    id = 0u;
    if (MODE == kModeRhs) {
        static_cast<real*>(a.out)[a.sid[i]] = (real)(kS * P.vphi) * acc;
        return 0u;
    }
    const real sc = (real)(a.scale * P.dt * P.vphi * kS);
    const real Cb = static_cast<const real*>(a.Cbase)[i];
    if (MODE == kModeHalf) {
        const real Ch = fmar(sc, acc, Cb);
        static_cast<real*>(a.out)[i] = Ch;
        if (kRec) a.out_rec[i] = Rec<DIM, real>::pack(T.ux, T.uy, T.uz, Ch);
        return 0u;
    }
    // step: update C and x, key of the moved particle for the next build
    const int64_t k = *a.step;
    uint32_t u[3] = {T.ux, T.uy, T.uz};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double us = P.ushift[c];
        const int64_t s1 = (int64_t)rint((double)(k + 1) * us);
        const int64_t s0 = (int64_t)rint((double)k * us);
        u[c] += (uint32_t)(s1 - s0);
        a.upos[c][i] = u[c];
    }
    static_cast<real*>(a.uC)[i] = fmar(sc, acc, Cb);
    id = a.sid[i];
    a.uid[i] = id;
    const uint32_t key = cell_key<DIM>(P, u[0], u[1], u[2]);
    a.ukey[i] = key;
    return key;
}

// finish_core, and in step mode the moved particle entered into its cell.
template <int DIM, typename real, int KERN, int MODE>
__device__ __forceinline__ void finish_target(const PairLaunch& a, const PlumeDev& P, const Target& T, uint32_t i,
                                              real acc) {
    uint32_t id;
    const uint32_t key = finish_core<DIM, real, KERN, MODE>(a, P, T, i, acc, id);
    if (MODE == kModeStep) enlist(a.lists, key, id);
}

// One work item = `block / LANES` consecutive target particles of one tile.
// The plume and tile tables come in as read-only, non-aliased kernel
// arguments so that their workgroup-uniform reads go through the scalar unit.
template <int DIM, typename real, int KERN, int MODE, int LANES, bool ZC>
__device__ __forceinline__ void pair_item(const PairLaunch& a, const PlumeDev* __restrict__ plumes,
                                          const TileDev* __restrict__ tiles, uint32_t w,
                                          uint2* lds_list) {
    const uint32_t tpb = (uint32_t)a.block / LANES;  // targets per workgroup
    const uint32_t subs = kTile / tpb;
    const TileDev t = tiles[w / subs];
    const uint32_t i0 = t.start + (w % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = plumes[t.plume];
    const uint32_t lt = threadIdx.x / LANES, lj = threadIdx.x % LANES;
    // Lanes past the end of a ragged tile stay in the walk (the wavefront
    // reductions there need every lane) with an empty list and target i0.
    const bool active = i0 + lt < i1;
    const uint32_t i = active ? i0 + lt : i0;

    const uint32_t* __restrict__ px = a.spos[0];
    const uint32_t* __restrict__ py = a.spos[1];
    const uint32_t* __restrict__ pz = a.spos[2];
    const real* __restrict__ Cp = static_cast<const real*>(a.Cpair);
    const uint4* __restrict__ rec = a.rec;
    constexpr bool kRec = Rec<DIM, real>::kStageable;

    const Target T = make_target<DIM>(P, px[i], py[i], (DIM == 3) ? pz[i] : 0u);
    const real Ca = Cp[i];
    real acc = (real)0;

    // the lanes of a target list its rows together (build_list)
    uint2* list = lds_list + lt;
    uint32_t total = 0;
    if (active) total = build_list<DIM, LANES>(P, a.cell_start, T, list, tpb);
    else list[0] = make_uint2(kListEndStart, kListEndEnd);
    auto walk = [&](const auto& term) {
        if (kRec)
            walk_list<LANES>(term, T, Ca, i, list, tpb, total, lj,
                             [&](uint32_t k) {
                                 // 32-bit byte offset from a uniform base
                                 return unpack<DIM, real>(*reinterpret_cast<const uint4*>(
                                     reinterpret_cast<const char*>(rec) + k));
                             },
                             acc);
        else
            walk_list<LANES>(term, T, Ca, i, list, tpb, total, lj,
                             [&](uint32_t k) {
                                 k /= kRecBytes;
                                 return Cand<real>{px[k], py[k], (DIM == 3) ? pz[k] : 0u, Cp[k]};
                             },
                             acc);
    };
    walk(make_term<DIM, real, KERN, ZC>(P));

    // wavefront reduction over the lanes of a target (fixed order: deterministic)
    if (LANES >= 2) acc += __shfl_xor(acc, 1, kWave);
    if (LANES >= 4) acc += __shfl_xor(acc, 2, kWave);
    if (!active || lj != 0) return;
    finish_target<DIM, real, KERN, MODE>(a, P, T, i, acc);
}

// ---------------------------------------------------------------------------
// Two targets per lane.  A lane takes the consecutive sorted targets a and b
// of a work item (one tile, so one plume).  When their rows are at most one
// apart along y (and z), it visits each row that can hold a neighbour of
// either target once (span + 1 rows per axis at most), with the x window of
// the row widened to the smallest arc that holds the windows of the targets
// reaching it, and evaluates every record of that one list against both
// targets.  Each neighbour of a or b is listed exactly once, so the loads of
// the walk serve two pair sums.
//
// List capacity: the arcs shrink away from the pair (the windows of either
// target do, and the pair's rows are adjacent), so the rows whose arc crosses
// the periodic x seam are consecutive.  A split row is emitted low part
// first; its high part ends where the next row's low part begins, and
// touching ranges are stored as one, so a plane of n rows takes at most n + 2
// entries (one more than n + 1 for a wrap of the row index among the split
// rows).  A pair whose rows are further apart (sparse plumes) walks a's own
// list, then b's.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ uint32_t build_union(const PlumeDev& P, const uint32_t* __restrict__ cs, const Target& A,
                                                const Target& B, int dy, int dz, uint2* list, uint32_t stride) {
    const int R = P.R;
    const int ny = 2 * R + 1 + (dy != 0 ? 1 : 0);
    const int nz = (DIM == 3) ? 2 * R + 1 + (dz != 0 ? 1 : 0) : 1;
    const int nrows = ny * nz;
    const int oy0 = min(0, dy) - R, oy1 = oy0 + ny - 1;
    int oy = oy0, oz = (DIM == 3) ? min(0, dz) - R : 0;  // the row of j, stepped on (oy fastest)
    const float dxc = (float)(int32_t)(B.ux - A.ux) * P.cellx;
    ListWriter w(list, stride);
    // two rows at a time: their cell-start loads are in flight together
    for (int j = 0; j < nrows; j += 2) {
        RowRanges r[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            r[q] = RowRanges{0u, 0u, 0u, 0u};
            if (j + q < nrows) r[q] = union_row<DIM>(P, cs, A, B, dxc, dy, dz, oy, oz);
            if (++oy > oy1) {
                oy = oy0;
                ++oz;
            }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (r[q].e1 > r[q].s1) w.put(r[q].s1, r[q].e1);
            if (r[q].e0 > r[q].s0) w.put(r[q].s0, r[q].e0);
        }
    }
    return w.flush();
}

// The walk of one lane's list (walk_stream) for two targets: every record
// fetched is evaluated against TA and TB.  Padding slots re-read a's own
// record, which a's predicate rejects (r2 = 0); b's evaluation keeps only the
// slots below the lane's total.  Sums are added to accA and accB.  b's
// separation from a record is taken as (x_b - x_a) + (x_a - x_c) in the
// working precision, which saves its integer differences and conversions.
// pair_rows merges only pairs with |x_b - x_a| + H_u < 2^31 per axis, so for
// every neighbour of b the integer sum is its minimum-image separation; a
// record whose sum leaves [-2^31, 2^31) is then no neighbour of b, and the
// sum, at least 2^31 in magnitude, rejects it.  Exact in FP64; in FP32 one
// more rounding, which can move a candidate across r = H only within a
// rounding of it, where its term is below 1e-35 of a typical one (the
// neighbour-set export keeps the exact predicate).
template <int DIM, typename Term, typename real, typename Fetch>
__device__ __forceinline__ void walk_pair(const Term& term, const Target& TA, const Target& TB,
                                          real CA, real CB, uint32_t self, const uint2* list, uint32_t stride,
                                          uint32_t total, Fetch&& fetch, real& accA, real& accB) {
    const real bx = (real)(int32_t)(TB.ux - TA.ux);
    const real by = (real)(int32_t)(TB.uy - TA.uy);
    const real bz = (DIM == 3) ? (real)(int32_t)(TB.uz - TA.uz) : (real)0;
    walk_stream<Batch<1>::value>(list, stride, total, self, fetch, [&](const Cand<real>& c, bool keep) {
        const real dx = (real)(int32_t)(TA.ux - c.x);
        const real dy = (real)(int32_t)(TA.uy - c.y);
        const real dz = (DIM == 3) ? (real)(int32_t)(TA.uz - c.z) : (real)0;
        term.sep(dx, dy, dz, CA, c.C, true, accA);
        term.sep(dx + bx, dy + by, dz + bz, CB, c.C, keep, accB);
    });
}

// One work item = 2 * block consecutive target particles of one tile, two
// per lane.
template <int DIM, typename real, int KERN, int MODE, bool ZC>
__device__ __forceinline__ void pair_item2(const PairLaunch& a, const PlumeDev* __restrict__ plumes,
                                           const TileDev* __restrict__ tiles, uint32_t w, uint2* lds_list) {
    const uint32_t stride = (uint32_t)a.block;
    const uint32_t tpb = 2u * stride;  // targets per workgroup
    const uint32_t subs = kTile / tpb;
    const TileDev t = tiles[w / subs];
    const uint32_t i0 = t.start + (w % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = plumes[t.plume];
    // past the end of a ragged tile a lane keeps a copy of a valid target
    // (its sums are discarded)
    const uint32_t ia = i0 + 2u * threadIdx.x, ib = ia + 1u;
    const bool actA = ia < i1, actB = ib < i1;
    const uint32_t iA = actA ? ia : i0, iB = actB ? ib : iA;

    const uint32_t* __restrict__ px = a.spos[0];
    const uint32_t* __restrict__ py = a.spos[1];
    const uint32_t* __restrict__ pz = a.spos[2];
    const real* __restrict__ Cp = static_cast<const real*>(a.Cpair);
    const uint4* __restrict__ rec = a.rec;
    constexpr bool kRec = Rec<DIM, real>::kStageable;
    auto fetch = [&](uint32_t k) {
        if (kRec)  // 32-bit byte offset from a uniform base
            return unpack<DIM, real>(*reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(rec) + k));
        k /= kRecBytes;
        return Cand<real>{px[k], py[k], (DIM == 3) ? pz[k] : 0u, Cp[k]};
    };

    const Target TA = make_target<DIM>(P, px[iA], py[iA], (DIM == 3) ? pz[iA] : 0u);
    const Target TB = make_target<DIM>(P, px[iB], py[iB], (DIM == 3) ? pz[iB] : 0u);
    const real CA = Cp[iA], CB = Cp[iB];
    real accA = (real)0, accB = (real)0;

    uint2* list = lds_list + threadIdx.x;
    int dy = 0, dz = 0;
    const bool merged = actB && pair_rows<DIM>(P, TA, TB, dy, dz);
    uint32_t total = 0;
    if (merged) total = build_union<DIM>(P, a.cell_start, TA, TB, dy, dz, list, stride);
    else if (actA) total = build_list<DIM, 1>(P, a.cell_start, TA, list, stride);
    else list[0] = make_uint2(kListEndStart, kListEndEnd);
    const PairTerm<DIM, real, KERN, ZC> term = make_term<DIM, real, KERN, ZC>(P);
    walk_pair<DIM>(term, TA, TB, CA, CB, iA, list, stride, total, fetch, accA, accB);
    // the pair's moved particles: two of one cell are counted with one atomic
    uint32_t idA = 0u, idB = 0u, kA = 0u, kB = 0u;
    if (actA) kA = finish_core<DIM, real, KERN, MODE>(a, P, TA, iA, accA, idA);
    if (merged) kB = finish_core<DIM, real, KERN, MODE>(a, P, TB, iB, accB, idB);
    if (MODE == kModeStep) {
        if (merged && kA == kB) {
            enlist2(a.lists, kA, idA, idB);
        } else {
            if (actA) enlist(a.lists, kA, idA);
            if (merged) enlist(a.lists, kB, idB);
        }
    }

    // b of a pair that could not be merged walks its own list (a second walk
    // that only wavefronts holding such a pair enter)
    const bool alone = actB && !merged;
    if (__builtin_amdgcn_ballot_w64(alone) == 0ull) return;
    const Target T2 = make_target<DIM>(P, px[iB], py[iB], (DIM == 3) ? pz[iB] : 0u);
    const real C2 = Cp[iB];
    uint32_t total2 = 0;
    if (alone) total2 = build_list<DIM, 1>(P, a.cell_start, T2, list, stride);
    else list[0] = make_uint2(kListEndStart, kListEndEnd);
    real acc2 = (real)0;
    walk_list<1>(term, T2, C2, iB, list, stride, total2, 0u, fetch, acc2);
    if (alone) finish_target<DIM, real, KERN, MODE>(a, P, T2, iB, acc2);
}

// ---------------------------------------------------------------------------
// Two neighbouring targets served by the four lanes of a quad (3D FP32, no
// coincident particles).  The quad lists the union of the two targets' row
// windows together (build_rows_quad over union_row), its lanes walk the list
// as four lanes walk one target's (two records a lane a batch), and every
// record is evaluated for both targets, b's separation formed from a's as in
// walk_pair.  A wavefront holding a pair that pair_rows does not merge walks
// each target's own list instead, in two passes (the other target's offset
// then put 2^31 grid units away, so that its terms vanish), through the same
// walk.  Padding slots re-read a's record (the pass target's), which adds
// nothing for it; b keeps only the slots below the lane's share.
// ---------------------------------------------------------------------------
template <int DIM, typename real, int KERN, int MODE, bool ZC>
__device__ __forceinline__ void pair_item42(const PairLaunch& a, const PlumeDev* __restrict__ plumes,
                                            const TileDev* __restrict__ tiles, uint32_t w, uint2* lds_list) {
    const uint32_t nq = (uint32_t)a.block / 4u;  // quads (lists) per workgroup
    const uint32_t tpb = 2u * nq;                // targets per workgroup
    const uint32_t subs = kTile / tpb;
    const TileDev t = tiles[w / subs];
    const uint32_t i0 = t.start + (w % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = plumes[t.plume];
    const uint32_t lq = threadIdx.x / 4u, lj = threadIdx.x % 4u;
    // past the end of a ragged tile a quad keeps a copy of a valid target
    // (its sums are discarded)
    const uint32_t ia = i0 + 2u * lq, ib = ia + 1u;
    const bool actA = ia < i1, actB = ib < i1;
    const uint32_t iA = actA ? ia : i0, iB = actB ? ib : iA;

    const uint32_t* __restrict__ px = a.spos[0];
    const uint32_t* __restrict__ py = a.spos[1];
    const uint32_t* __restrict__ pz = a.spos[2];
    const real* __restrict__ Cp = static_cast<const real*>(a.Cpair);
    const uint4* __restrict__ rec = a.rec;
    auto fetch = [&](uint32_t k) {
        return unpack<DIM, real>(*reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(rec) + k));
    };
    auto target = [&](uint32_t k) { return make_target<DIM>(P, px[k], py[k], (DIM == 3) ? pz[k] : 0u); };
    int pry = 0, prz = 0;
    const bool close = pair_rows<DIM>(P, target(iA), target(iB), pry, prz);
    const bool merged = __builtin_amdgcn_ballot_w64(!close) == 0ull;  // the whole wavefront
    uint2* list = lds_list + lq;
    const PairTerm<DIM, real, KERN, ZC> term = make_term<DIM, real, KERN, ZC>(P);
    real accA = (real)0, accB = (real)0;
    const int npass = merged ? 1 : 2;
    for (int pass = 0; pass < npass; ++pass) {
        // the pass's pair: (a, b), or (a, a) and then (b, b), every step of
        // the walk the same; the targets are read per pass, so that no more
        // than their indices lives across the passes
        const bool second = pass == 1;
        const uint32_t k0 = second ? iB : iA, k1 = merged ? iB : k0;
        const Target T0 = target(k0), T1 = target(k1);
        const real C0 = Cp[k0], C1 = Cp[k1];
        const int ry = merged ? pry : 0, rz = merged ? prz : 0;
        const real bx = (real)(int32_t)(T1.ux - T0.ux);
        const real by = (real)(int32_t)(T1.uy - T0.uy);
        const real bz = (DIM == 3) ? (real)(int32_t)(T1.uz - T0.uz) : (real)0;
        uint32_t total = 0;
        if (actA && !(second && !actB)) {  // the same for the four lanes of a quad
            const int R = P.R;
            const int ny = 2 * R + 1 + (ry != 0 ? 1 : 0);
            const int nz = (DIM == 3) ? 2 * R + 1 + (rz != 0 ? 1 : 0) : 1;
            const float dxc = (float)(int32_t)(T1.ux - T0.ux) * P.cellx;
            total = build_rows_quad(
                [&](int oy, int oz) { return union_row<DIM>(P, a.cell_start, T0, T1, dxc, ry, rz, oy, oz); }, ny, nz,
                min(0, ry) - R, (DIM == 3) ? min(0, rz) - R : 0, list, nq);
        } else {
            list[0] = make_uint2(kListEndStart, kListEndEnd);
        }
        real acc0 = (real)0, acc1 = (real)0;
        walk_list_fn<4, 2>(k0, list, nq, total, lj, fetch, [&](const Cand<real>& c, bool keep) {
            const real dx = (real)(int32_t)(T0.ux - c.x);
            const real dy = (real)(int32_t)(T0.uy - c.y);
            const real dz = (DIM == 3) ? (real)(int32_t)(T0.uz - c.z) : (real)0;
            term.sep(dx, dy, dz, C0, c.C, true, acc0);
            term.sep(dx + bx, dy + by, dz + bz, C1, c.C, keep, acc1);
        });
        if (second) {
            accB = acc0;
        } else {
            accA = acc0;
            accB = acc1;
        }
    }
    // the quad's partial sums (fixed order: deterministic); lane 0 finishes
    // a, lane 1 b
    accA += __shfl_xor(accA, 1, kWave);
    accA += __shfl_xor(accA, 2, kWave);
    accB += __shfl_xor(accB, 1, kWave);
    accB += __shfl_xor(accB, 2, kWave);
    if (lj == 0 && actA) finish_target<DIM, real, KERN, MODE>(a, P, target(iA), iA, accA);
    if (lj == 1 && actB) finish_target<DIM, real, KERN, MODE>(a, P, target(iB), iB, accB);
}

// Six wavefronts per SIMD: at most 80 VGPRs (101 without the bound, four
// wavefronts).  A few addresses of the targets' state then spill to scratch
// outside the walk (72 bytes a lane, written and read once per work item).
template <int DIM, typename real, int KERN, int MODE, bool ZC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_pair42(PairLaunch a, const PlumeDev* __restrict__ plumes,
                                                const TileDev* __restrict__ tiles, uint32_t nwork) {
    extern __shared__ uint2 lds_list[];
    if (a.persistent == 0) {
        pair_item42<DIM, real, KERN, MODE, ZC>(a, plumes, tiles, xcd_remap(blockIdx.x, gridDim.x, a.xcd_group),
                                               lds_list);
        return;
    }
    const uint32_t nx = 8, x = blockIdx.x % nx, k = blockIdx.x / nx;
    const uint32_t per_x = (gridDim.x + nx - 1 - x) / nx;
    for (uint32_t m = k;; m += per_x) {
        const uint32_t w = xcd_item(x, m, nwork, a.xcd_group);
        if (w >= nwork) break;
        pair_item42<DIM, real, KERN, MODE, ZC>(a, plumes, tiles, w, lds_list);
    }
}

// Eight wavefronts per SIMD for the FP32 kernels: at most 64 VGPRs and 100
// SGPRs (kernel arguments are re-read from the argument segment rather than
// held across the candidate loop).
template <int DIM, typename real, int KERN, int MODE, int LANES, bool ZC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 && DIM == 2 ? 8 : 1)))
void k_pair(PairLaunch a, const PlumeDev* __restrict__ plumes,
                                              const TileDev* __restrict__ tiles, uint32_t nwork) {
    extern __shared__ uint2 lds_list[];
    if (a.persistent == 0) {
        pair_item<DIM, real, KERN, MODE, LANES, ZC>(a, plumes, tiles, xcd_remap(blockIdx.x, gridDim.x, a.xcd_group),
                                                    lds_list);
        return;
    }
    // persistent grid: the k-th of the workgroups on XCD x takes every
    // per_x-th of the items xcd_remap deals to that XCD (fixed assignment, no
    // queue); a target's list is written and read by the lanes of one
    // wavefront only, so consecutive items need no barrier
    const uint32_t nx = 8, x = blockIdx.x % nx, k = blockIdx.x / nx;
    const uint32_t per_x = (gridDim.x + nx - 1 - x) / nx;  // workgroups on this XCD
    for (uint32_t m = k;; m += per_x) {
        const uint32_t w = xcd_item(x, m, nwork, a.xcd_group);
        if (w >= nwork) break;
        pair_item<DIM, real, KERN, MODE, LANES, ZC>(a, plumes, tiles, w, lds_list);
    }
}

// Two targets per lane: at most 128 threads (a work item holds 2 * block
// targets of a 256-particle tile); six wavefronts per SIMD for 2D FP32 (the
// lane carries both targets through the walk).
template <int DIM, typename real, int KERN, int MODE, bool ZC>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 && DIM == 2 ? 6 : 1)))
void k_pair2(PairLaunch a, const PlumeDev* __restrict__ plumes, const TileDev* __restrict__ tiles, uint32_t nwork) {
    extern __shared__ uint2 lds_list[];
    if (a.persistent == 0) {
        pair_item2<DIM, real, KERN, MODE, ZC>(a, plumes, tiles, xcd_remap(blockIdx.x, gridDim.x, a.xcd_group), lds_list);
        return;
    }
    const uint32_t nx = 8, x = blockIdx.x % nx, k = blockIdx.x / nx;
    const uint32_t per_x = (gridDim.x + nx - 1 - x) / nx;
    for (uint32_t m = k;; m += per_x) {
        const uint32_t w = xcd_item(x, m, nwork, a.xcd_group);
        if (w >= nwork) break;
        pair_item2<DIM, real, KERN, MODE, ZC>(a, plumes, tiles, w, lds_list);
    }
}

// Neighbour-set export through the same candidate ranges and predicate:
// fill = 0 writes the count of particle id at offsets[id]; fill = 1 writes
// the ids from offsets[id] on.
template <int DIM, typename real>
__global__ __launch_bounds__(kTile) void k_nbr(const PlumeDev* __restrict__ plumes,
                                              const TileDev* __restrict__ tiles, StateArrays S,
                                              const uint32_t* __restrict__ cs, int fill,
                                              int64_t* __restrict__ offsets,
                                              int32_t* __restrict__ ids) {
    const TileDev t = tiles[blockIdx.x];
    const PlumeDev P = plumes[t.plume];
    const uint32_t i = t.start + threadIdx.x;
    if (i >= t.end) return;
    const uint32_t* px = S.pos[0];
    const uint32_t* py = S.pos[1];
    const uint32_t* pz = S.pos[2];
    const Target T = make_target<DIM>(P, px[i], py[i], (DIM == 3) ? pz[i] : 0u);
    const uint32_t me = S.id[i];
    const real H2 = h2_of<real>(P);
    const int span = 2 * P.R + 1, noff = (DIM == 3) ? span * span : span;
    int64_t k = fill ? offsets[me] : 0;
    auto walk = [&](uint32_t s, uint32_t e) {
        for (uint32_t b = s; b < e; ++b) {
            const real dx = (real)(int32_t)(T.ux - px[b]);
            const real dy = (real)(int32_t)(T.uy - py[b]);
            const real dz = (DIM == 3) ? (real)(int32_t)(T.uz - pz[b]) : (real)0;
            real r2 = dx * dx;
            r2 = fmar(dy, dy, r2);
            if (DIM == 3) r2 = fmar(dz, dz, r2);
            if (r2 > (real)0 && r2 <= H2) {
                if (fill) ids[k] = (int32_t)S.id[b];
                ++k;
            }
        }
    };
    for (int j = 0; j < noff; ++j) {
        const RowRanges r = row_ranges<DIM>(P, cs, T, j, span);
        walk(r.s0, r.e0);
        if (r.e1 > r.s1) walk(r.s1, r.e1);
    }
    if (!fill) offsets[me] = k;
}

template <int DIM, typename real, int KERN, int LANES, bool ZC>
static void launch_pair_l(int mode, const PairLaunch& a, hipStream_t s) {
    const uint32_t tpb = (uint32_t)a.block / LANES;
    const uint32_t nwork = a.ntiles * (kTile / tpb);
    PairLaunch c = a;
    if (nwork < 8) c.persistent = 0;  // a persistent grid needs a workgroup on every XCD
    const uint32_t grid = (c.persistent > 0) ? max(8u, min(nwork, (uint32_t)c.persistent)) : nwork;
    dim3 g(grid), b(a.block);
    const size_t shm = pair_lds_bytes(a.block, LANES, a.list_cap);
    auto kern = (mode == kModeStep)   ? k_pair<DIM, real, KERN, kModeStep, LANES, ZC>
                : (mode == kModeHalf) ? k_pair<DIM, real, KERN, kModeHalf, LANES, ZC>
                                      : k_pair<DIM, real, KERN, kModeRhs, LANES, ZC>;
    if (c.ev0)  // timed launch: the events carry the kernel's own start and end stamps
        hipExtLaunchKernelGGL(kern, g, b, (uint32_t)shm, s, c.ev0, c.ev1, 0u, c, c.plumes, c.tiles, nwork);
    else
        hipLaunchKernelGGL(kern, g, b, shm, s, c, c.plumes, c.tiles, nwork);
}

template <int DIM, typename real, int KERN, bool ZC>
static void launch_pair_2(int mode, const PairLaunch& a, hipStream_t s) {
    const uint32_t tpb = 2u * (uint32_t)a.block;
    const uint32_t nwork = a.ntiles * (kTile / tpb);
    PairLaunch c = a;
    if (nwork < 8) c.persistent = 0;
    const uint32_t grid = (c.persistent > 0) ? max(8u, min(nwork, (uint32_t)c.persistent)) : nwork;
    dim3 g(grid), b(a.block);
    const size_t shm = pair_lds_bytes(a.block, 1, a.list_cap);
    auto kern = (mode == kModeStep)   ? k_pair2<DIM, real, KERN, kModeStep, ZC>
                : (mode == kModeHalf) ? k_pair2<DIM, real, KERN, kModeHalf, ZC>
                                      : k_pair2<DIM, real, KERN, kModeRhs, ZC>;
    if (c.ev0)
        hipExtLaunchKernelGGL(kern, g, b, (uint32_t)shm, s, c.ev0, c.ev1, 0u, c, c.plumes, c.tiles, nwork);
    else
        hipLaunchKernelGGL(kern, g, b, shm, s, c, c.plumes, c.tiles, nwork);
}

template <int DIM, typename real, int KERN, bool ZC>
static void launch_pair_42(int mode, const PairLaunch& a, hipStream_t s) {
    const uint32_t tpb = (uint32_t)a.block / 2u;
    const uint32_t nwork = a.ntiles * (kTile / tpb);
    PairLaunch c = a;
    if (nwork < 8) c.persistent = 0;
    const uint32_t grid = (c.persistent > 0) ? max(8u, min(nwork, (uint32_t)c.persistent)) : nwork;
    dim3 g(grid), b(a.block);
    const size_t shm = pair_lds_bytes(a.block, 4, a.list_cap);
    auto kern = (mode == kModeStep)   ? k_pair42<DIM, real, KERN, kModeStep, ZC>
                : (mode == kModeHalf) ? k_pair42<DIM, real, KERN, kModeHalf, ZC>
                                      : k_pair42<DIM, real, KERN, kModeRhs, ZC>;
    if (c.ev0)
        hipExtLaunchKernelGGL(kern, g, b, (uint32_t)shm, s, c.ev0, c.ev1, 0u, c, c.plumes, c.tiles, nwork);
    else
        hipLaunchKernelGGL(kern, g, b, shm, s, c, c.plumes, c.tiles, nwork);
}

template <int DIM, typename real, int KERN, bool ZC>
static void launch_pair_z(int mode, const PairLaunch& a, hipStream_t s) {
    if (a.targets == 2 && a.lanes == 4) {
        // two targets a quad: FP32 without coincident particles, else one
        // target a quad
        if constexpr (sizeof(real) == 4 && !ZC) launch_pair_42<DIM, real, KERN, ZC>(mode, a, s);
        else launch_pair_l<DIM, real, KERN, 4, ZC>(mode, a, s);
    } else if (a.targets == 2) launch_pair_2<DIM, real, KERN, ZC>(mode, a, s);
    else if (a.lanes == 4) launch_pair_l<DIM, real, KERN, 4, ZC>(mode, a, s);
    else if (a.lanes == 2) launch_pair_l<DIM, real, KERN, 2, ZC>(mode, a, s);
    else launch_pair_l<DIM, real, KERN, 1, ZC>(mode, a, s);
}

// the kernels without the r > 0 test exist for FP32 and Wendland C4 (the
// FP32 problems); everything else tests every candidate
template <int DIM, typename real, int KERN>
static void launch_pair_t(int mode, const PairLaunch& a, hipStream_t s) {
    if constexpr (sizeof(real) == 4 && KERN == 4) {
        if (!a.zc) {
            launch_pair_z<DIM, real, KERN, false>(mode, a, s);
            return;
        }
    }
    launch_pair_z<DIM, real, KERN, true>(mode, a, s);
}

hipError_t launch_pair(int dim, int real_bytes, int kernel, int mode, const PairLaunch& a,
                       int block, hipStream_t s) {
    (void)block;
    if (a.block <= 0 || a.block > kTile || kTile % a.block != 0) return hipErrorInvalidValue;
    if (a.lanes != 1 && a.lanes != 2 && a.lanes != 4) return hipErrorInvalidValue;
    if (a.targets != 1 && (a.targets != 2 || !((a.lanes == 1 && 2 * a.block <= kTile) || a.lanes == 4)))
        return hipErrorInvalidValue;
    if (a.list_cap < 3 || pair_lds_bytes(a.block, a.lanes, a.list_cap) > kPairLdsMax) return hipErrorInvalidValue;
    if (dim == 2) {
        if (real_bytes == 4) {
            if (kernel == 4) launch_pair_t<2, float, 4>(mode, a, s);
            else launch_pair_t<2, float, 2>(mode, a, s);
        } else {
            if (kernel == 4) launch_pair_t<2, double, 4>(mode, a, s);
            else launch_pair_t<2, double, 2>(mode, a, s);
        }
    } else {
        if (real_bytes == 4) {
            if (kernel == 4) launch_pair_t<3, float, 4>(mode, a, s);
            else launch_pair_t<3, float, 2>(mode, a, s);
        } else {
            if (kernel == 4) launch_pair_t<3, double, 4>(mode, a, s);
            else launch_pair_t<3, double, 2>(mode, a, s);
        }
    }
    return hipGetLastError();
}

hipError_t launch_nbr(int dim, int real_bytes, int fill, const PlumeDev* plumes,
                      const TileDev* tiles, uint32_t ntiles, StateArrays S,
                      const uint32_t* cell_start, int64_t* offsets, int32_t* ids, hipStream_t s) {
    dim3 g(ntiles), b(kTile);
    if (dim == 2 && real_bytes == 4)
        hipLaunchKernelGGL((k_nbr<2, float>), g, b, 0, s, plumes, tiles, S, cell_start, fill, offsets, ids);
    else if (dim == 2)
        hipLaunchKernelGGL((k_nbr<2, double>), g, b, 0, s, plumes, tiles, S, cell_start, fill, offsets, ids);
    else if (real_bytes == 4)
        hipLaunchKernelGGL((k_nbr<3, float>), g, b, 0, s, plumes, tiles, S, cell_start, fill, offsets, ids);
    else
        hipLaunchKernelGGL((k_nbr<3, double>), g, b, 0, s, plumes, tiles, S, cell_start, fill, offsets, ids);
    return hipGetLastError();
}

}  // namespace ade
