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
// Separations are taken in grid units (L / 2^32) from the fixed-point
// positions; Gamma x^T D x / r^2 is scale free and the constant factor
// V (W'(r)/r)/f(q) is applied once per particle (PlumeDev::vphi).
//
// Neighbour predicate (shared with the neighbour-list export): d = (int32)
// (u_a - u_b) per component (the two's-complement wrap is the minimum image),
// converted to the working precision, r2 = d_x d_x, r2 = fma(d_y, d_y, r2)
// [, r2 = fma(d_z, d_z, r2)], pair iff 0 < r2 <= H_u^2 (inclusive support).
//
// Candidates: particles are sorted by (row, x cell), rows being a grid of
// height >= Hc / R in y (and z).  For each of the (2R+1)^(d-1) rows around a
// target, the x cells that can hold neighbours form one contiguous range of
// the sorted order (two at the periodic seam), cut to the chord of the
// search radius at the row's nearest edge.  Each lane walks its ranges in
// batches of kBatch candidate records, the next batch in flight while the
// current one is evaluated, and the cell-start bounds of the next row in
// flight while the current row is walked.  Optionally a workgroup first
// stages the union of its candidate ranges in LDS (coalesced reads) and the
// lanes walk the staged copy, falling back to global memory for a range
// outside it.
#include <hip/hip_ext.h>

#include "ade_geom.h"

namespace ade {

// One candidate: predicate and, if inside the support, the pair term.
template <int DIM, typename real, int KERN>
struct PairTerm {
    real H2, invHu, kxx, kyy, kzz, kxy, kxz, kyz, trD;
    __device__ __forceinline__ void operator()(const Target& T, real Ca, uint32_t bx, uint32_t by,
                                               uint32_t bz, real Cb, real& acc) const {
        const real dx = (real)(int32_t)(T.ux - bx);
        const real dy = (real)(int32_t)(T.uy - by);
        const real dz = (DIM == 3) ? (real)(int32_t)(T.uz - bz) : (real)0;
        const real dC = Ca - Cb;  // formed before the test: the whole record is fetched at once
        real r2 = dx * dx;
        r2 = fmar(dy, dy, r2);
        if (DIM == 3) r2 = fmar(dz, dz, r2);
        if (r2 > (real)0 && r2 <= H2) {
            const real rinv = rsqrt_r(r2);
            const real q = r2 * rinv * invHu;
            real omq = (real)1 - q;
            omq = omq > (real)0 ? omq : (real)0;
            real f;
            if (KERN == 4) {
                const real o2 = omq * omq;
                f = o2 * o2 * omq * fmar((real)5, q, (real)1);
            } else {
                f = omq * omq * omq;
            }
            real Q;
            if (DIM == 3)
                Q = dx * (kxx * dx + kxy * dy + kxz * dz) + dy * (kyy * dy + kyz * dz) + kzz * dz * dz;
            else
                Q = dx * (kxx * dx + kxy * dy) + kyy * dy * dy;
            const real A = Q * (rinv * rinv) - trD;
            acc = fmar(A * f, dC, acc);
        }
    }
};

template <typename real>
struct Cand {
    uint32_t x, y, z;
    real C;
};

template <int DIM, typename real>
__device__ __forceinline__ Cand<real> unpack(const uint4& r) {
    return Cand<real>{r.x, r.y, (DIM == 3) ? r.z : 0u, Rec<DIM, real>::conc(r)};
}

// Walk the candidates b = s + lane, s + lane + LANES, ... < e in batches of
// kBatch: the batch after the current one is fetched before the current one
// is evaluated.  Past the end of the range a batch is padded with a record
// half the box away from the target, which fails the predicate.
template <int DIM, typename real, int KERN, int LANES, typename Fetch>
__device__ __forceinline__ void walk_batched(const PairTerm<DIM, real, KERN>& term, const Target& T,
                                             real Ca, uint32_t s, uint32_t e, uint32_t lj,
                                             Fetch&& fetch, real& acc) {
    constexpr int kBatch = Batch<LANES>::value;
    uint32_t b = s + lj;
    if (b >= e) return;
    const Cand<real> pad{T.ux + 0x80000000u, T.uy, T.uz, Ca};
    Cand<real> cur[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
        const uint32_t bb = b + q * LANES;
        cur[q] = (bb < e) ? fetch(bb) : pad;
    }
    for (;;) {
        const uint32_t bn = b + kBatch * LANES;
        const bool more = bn < e;
        Cand<real> nxt[kBatch];
        if (more) {
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const uint32_t bb = bn + q * LANES;
                nxt[q] = (bb < e) ? fetch(bb) : pad;
            }
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) term(T, Ca, cur[q].x, cur[q].y, cur[q].z, cur[q].C, acc);
        if (!more) break;
#pragma unroll
        for (int q = 0; q < kBatch; ++q) cur[q] = nxt[q];
        b = bn;
    }
}

// One work item = `block / LANES` consecutive target particles of one tile.
template <int DIM, typename real, int KERN, int MODE, int LANES>
__device__ __forceinline__ void pair_item(const PairLaunch& a, uint32_t w, uint4* lds_rec,
                                          uint32_t* o_lo, uint32_t* o_hi, uint32_t* o_base) {
    const uint32_t tpb = (uint32_t)a.block / LANES;  // targets per workgroup
    const uint32_t subs = kTile / tpb;
    const TileDev t = a.tiles[w / subs];
    const uint32_t i0 = t.start + (w % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = a.plumes[t.plume];
    const uint32_t lt = threadIdx.x / LANES, lj = threadIdx.x % LANES;
    const uint32_t i = i0 + lt;
    const bool active = i < i1;

    const uint32_t* __restrict__ px = a.spos[0];
    const uint32_t* __restrict__ py = a.spos[1];
    const uint32_t* __restrict__ pz = a.spos[2];
    const real* __restrict__ Cp = static_cast<const real*>(a.Cpair);
    const uint4* __restrict__ rec = a.rec;
    const uint32_t* __restrict__ cs = a.cell_start;
    const int R = P.R;
    const int span = 2 * R + 1;
    const int noff = (DIM == 3) ? span * span : span;
    constexpr bool kRec = Rec<DIM, real>::kStageable;

    // ---- stage the union of the workgroup's candidate ranges in LDS ----------
    const bool stage = kRec && a.stage > 0;
    if (stage) {
        const uint32_t cap = (uint32_t)a.stage * (uint32_t)a.block;
        __syncthreads();  // the previous item of a persistent workgroup is done with LDS
        for (int o = threadIdx.x; o < noff; o += blockDim.x) {
            const int oy = o % span - R, oz = (DIM == 3) ? o / span - R : 0;
            const uint32_t fx = px[i0], lx = px[i1 - 1];
            const int fy = (int)__umulhi(py[i0], P.nr), ly = (int)__umulhi(py[i1 - 1], P.nr);
            const int fz = (DIM == 3) ? (int)__umulhi(pz[i0], P.nr) : 0;
            const int lz = (DIM == 3) ? (int)__umulhi(pz[i1 - 1], P.nr) : 0;
            const int nr = (int)P.nr;
            uint32_t lo = 0, hi = 0;
            const bool rows_ok = fz == lz && fy + oy >= 0 && ly + oy < nr &&
                                 (DIM == 2 || (fz + oz >= 0 && fz + oz < nr));
            const bool x_ok = fx >= P.hx && lx <= 0xffffffffu - P.hx;
            if (rows_ok && x_ok) {
                const int clo = (int)__umulhi(fx - P.hx, P.nfx) - 1;
                const int chi = (int)__umulhi(lx + P.hx, P.nfx) + 1;
                if (clo >= 0 && chi < (int)P.nfx) {
                    const uint32_t zrow = (DIM == 3) ? (uint32_t)(fz + oz) * P.nr : 0u;
                    const uint32_t klo = P.cbase + (zrow + (uint32_t)(fy + oy)) * P.nfx + (uint32_t)clo;
                    const uint32_t khi = P.cbase + (zrow + (uint32_t)(ly + oy)) * P.nfx + (uint32_t)chi;
                    if (klo <= khi) {
                        lo = cs[klo];
                        hi = cs[khi + 1];
                    }
                }
            }
            o_lo[o] = lo;
            o_hi[o] = hi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            for (int o = 0; o < noff; ++o) {
                const uint32_t n = o_hi[o] - o_lo[o];
                o_base[o] = run;
                if (run + n > cap) o_hi[o] = o_lo[o];  // does not fit: that row reads global memory
                else run += n;
            }
        }
        __syncthreads();
        for (int o = 0; o < noff; ++o) {
            const uint32_t lo = o_lo[o], n = o_hi[o] - lo, base = o_base[o];
            for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) lds_rec[base + j] = rec[lo + j];
        }
        __syncthreads();
    }
    if (!active) return;  // all LANES lanes of a target share `active`

    const Target T = make_target<DIM>(P, px[i], py[i], (DIM == 3) ? pz[i] : 0u);
    const real Ca = Cp[i];
    PairTerm<DIM, real, KERN> term;
    term.H2 = h2_of<real>(P);
    term.invHu = (real)P.invHu;
    term.kxx = (real)P.kg[0];
    term.kyy = (real)P.kg[1];
    term.kzz = (real)P.kg[2];
    term.kxy = (real)P.kg[3];
    term.kxz = (real)P.kg[4];
    term.kyz = (real)P.kg[5];
    term.trD = (real)P.trD;
    real acc = (real)0;

    auto walk = [&](int o, uint32_t s, uint32_t e) {
        if (kRec) {
            if (stage && s >= o_lo[o] && e <= o_hi[o]) {
                const uint32_t shift = o_base[o] - o_lo[o];
                walk_batched<DIM, real, KERN, LANES>(
                    term, T, Ca, s + shift, e + shift, lj,
                    [&](uint32_t k) { return unpack<DIM, real>(lds_rec[k]); }, acc);
            } else {
                walk_batched<DIM, real, KERN, LANES>(
                    term, T, Ca, s, e, lj, [&](uint32_t k) { return unpack<DIM, real>(rec[k]); }, acc);
            }
        } else {
            walk_batched<DIM, real, KERN, LANES>(
                term, T, Ca, s, e, lj,
                [&](uint32_t k) { return Cand<real>{px[k], py[k], (DIM == 3) ? pz[k] : 0u, Cp[k]}; },
                acc);
        }
    };

    // rows in order (oz major, oy minor); the cell-start bounds of the next
    // row are in flight while the current row is walked
    RowRanges cur = row_ranges<DIM>(P, cs, T, 0, span);
    for (int j = 0; j < noff; ++j) {
        RowRanges nxt{0u, 0u, 0u, 0u};
        if (j + 1 < noff) nxt = row_ranges<DIM>(P, cs, T, j + 1, span);
        walk(j, cur.s0, cur.e0);
        if (cur.e1 > cur.s1) walk(j, cur.s1, cur.e1);
        cur = nxt;
    }
    // wavefront reduction over the lanes of a target (fixed order: deterministic)
    if (LANES >= 2) acc += __shfl_xor(acc, 1, kWave);
    if (LANES >= 4) acc += __shfl_xor(acc, 2, kWave);
    if (lj != 0) return;

    if (MODE == kModeRhs) {
        static_cast<real*>(a.out)[a.sid[i]] = (real)P.vphi * acc;
        return;
    }
    const real sc = (real)(a.scale * P.dt * P.vphi);
    const real Cb = static_cast<const real*>(a.Cbase)[i];
    if (MODE == kModeHalf) {
        const real Ch = fmar(sc, acc, Cb);
        static_cast<real*>(a.out)[i] = Ch;
        if (kRec) a.out_rec[i] = Rec<DIM, real>::pack(T.ux, T.uy, T.uz, Ch);
        return;
    }
    // step: update C and x, hash the moved particle for the next build
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
    a.uid[i] = a.sid[i];
    const uint32_t key = cell_key<DIM>(P, u[0], u[1], u[2]);
    a.ukey[i] = key;
    a.utick[i] = atomicAdd(&a.count[key], 1u);
}

template <int DIM, typename real, int KERN, int MODE, int LANES>
__global__ __launch_bounds__(256) void k_pair(PairLaunch a, uint32_t nwork) {
    extern __shared__ uint4 lds_rec[];
    __shared__ uint32_t o_lo[kMaxRowOffsets], o_hi[kMaxRowOffsets], o_base[kMaxRowOffsets];
    if (a.persistent == 0) {
        pair_item<DIM, real, KERN, MODE, LANES>(a, xcd_remap(blockIdx.x, gridDim.x), lds_rec, o_lo,
                                                o_hi, o_base);
        return;
    }
    // persistent grid: each workgroup takes every per_x-th item of a
    // contiguous per-XCD share of the items (no queue, fixed assignment)
    const uint32_t nx = 8, x = blockIdx.x % nx, k = blockIdx.x / nx;
    const uint32_t per_x = (gridDim.x + nx - 1 - x) / nx;  // workgroups on this XCD
    const uint32_t lo = (uint32_t)(((uint64_t)nwork * x) / nx), hi = (uint32_t)(((uint64_t)nwork * (x + 1)) / nx);
    for (uint32_t w = lo + k; w < hi; w += per_x)
        pair_item<DIM, real, KERN, MODE, LANES>(a, w, lds_rec, o_lo, o_hi, o_base);
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

template <int DIM, typename real, int KERN, int LANES>
static void launch_pair_l(int mode, const PairLaunch& a, hipStream_t s) {
    const uint32_t tpb = (uint32_t)a.block / LANES;
    const uint32_t nwork = a.ntiles * (kTile / tpb);
    PairLaunch c = a;
    if (nwork < 8) c.persistent = 0;  // a persistent grid needs a workgroup on every XCD
    const uint32_t grid = (c.persistent > 0) ? max(8u, min(nwork, (uint32_t)c.persistent)) : nwork;
    dim3 g(grid), b(a.block);
    const size_t shm = (Rec<DIM, real>::kStageable && a.stage > 0)
                           ? sizeof(uint4) * (size_t)a.stage * (size_t)a.block : 0;
    auto kern = (mode == kModeStep)   ? k_pair<DIM, real, KERN, kModeStep, LANES>
                : (mode == kModeHalf) ? k_pair<DIM, real, KERN, kModeHalf, LANES>
                                      : k_pair<DIM, real, KERN, kModeRhs, LANES>;
    if (c.ev0)  // timed launch: the events carry the kernel's own start and end stamps
        hipExtLaunchKernelGGL(kern, g, b, (uint32_t)shm, s, c.ev0, c.ev1, 0u, c, nwork);
    else
        hipLaunchKernelGGL(kern, g, b, shm, s, c, nwork);
}

template <int DIM, typename real, int KERN>
static void launch_pair_t(int mode, const PairLaunch& a, hipStream_t s) {
    if (a.lanes == 4) launch_pair_l<DIM, real, KERN, 4>(mode, a, s);
    else if (a.lanes == 2) launch_pair_l<DIM, real, KERN, 2>(mode, a, s);
    else launch_pair_l<DIM, real, KERN, 1>(mode, a, s);
}

hipError_t launch_pair(int dim, int real_bytes, int kernel, int mode, const PairLaunch& a,
                       int block, hipStream_t s) {
    (void)block;
    if (a.block <= 0 || a.block > kTile || kTile % a.block != 0) return hipErrorInvalidValue;
    if (a.lanes != 1 && a.lanes != 2 && a.lanes != 4) return hipErrorInvalidValue;
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
