// kernels_general.hip -- the SPH pair sum of Eqs. (4)-(5) (Klapp et al.,
// arXiv:2108.09488, Section 2.2) for a velocity field: every particle has its
// own velocity v_a, hence its own dispersion tensor D_a (Eq. 3), so the pair
// term takes the elementwise harmonic mean of Eq. (5),
//     h_ij = 4 D_ij,a D_ij,b / (D_ij,a + D_ij,b)   (0 when D_ij,a D_ij,b <= 0),
//     Dcal_ab = sum_ij h_ij [Gamma x_i x_j / r^2 - delta_ij],
// and Eq. (4) gains its convective term,
//     (dC/dt)_a = 1/2 sum_b V Dcal_ab (C_a - C_b) W'(r)/r
//               + C_a sum_b V (v_a - v_b) . x_ab W'(r)/r,
// with V = m / rho for equal masses and densities.  Particles move by their
// own velocities, each on the exact fixed-point schedule of the uniform case
// (displacement rint((k+1) u_a) - rint(k u_a) at step k, u_a = dt v_a / L
// 2^32), and are hashed and counted into the next build's cells as there.
// One, two or four lanes per target walk the target's candidate list
// (ade_walk.h), or in 2D FP32 the four lanes of a quad walk the merged list of
// two neighbouring targets and evaluate every record for both.  Each
// particle carries the reciprocals of its tensor components, so a harmonic
// mean costs one add and one reciprocal; in 2D FP32 a candidate is one
// 32-byte record, elsewhere it is read from the structure-of-arrays state.
#include <hip/hip_ext.h>

#include "ade_walk.h"

namespace ade {

// candidate records per lane per batch of the walk (2: the kernel stays at
// 64 VGPRs; 4 measured about 13% slower in both update and rhs mode)
constexpr int kGenBatch = 2;

template <int DIM>
struct GenDims {
    static constexpr int kT = DIM == 2 ? 3 : 6;  // tensor components stored per particle
};
// whether stored component k is on the diagonal
template <int DIM>
__host__ __device__ constexpr bool is_diag(int k) {
    return DIM == 2 ? (k == 0 || k == 2) : (k == 0 || k == 3 || k == 5);
}

// Eq. (3) for velocity v: the stored components (2D: xx, xy, yy; 3D: xx,
// xy, xz, yy, yz, zz)
template <int DIM>
__host__ __device__ inline void tensor_of(double aL, double aT, double Dm, const double* v, double* Dt) {
    double s2 = 0.0;
    for (int c = 0; c < DIM; ++c) s2 += v[c] * v[c];
    const double sp = sqrt(s2);
    auto comp = [&](int i, int j) {
        double d = (i == j) ? aT * sp + Dm : 0.0;
        if (sp > 0.0) d += (aL - aT) * v[i] * v[j] / sp;
        return d;
    };
    if (DIM == 2) {
        Dt[0] = comp(0, 0);
        Dt[1] = comp(0, 1);
        Dt[2] = comp(1, 1);
    } else {
        Dt[0] = comp(0, 0);
        Dt[1] = comp(0, 1);
        Dt[2] = comp(0, 2);
        Dt[3] = comp(1, 1);
        Dt[4] = comp(1, 2);
        Dt[5] = comp(2, 2);
    }
}

// Velocities (double, SoA dim x N in id order) into the hashed buffer U,
// which after ade_init_particles holds particle a at index a, with the
// reciprocals of the tensor components they give (the pair term needs only
// those: see hmean).
template <int DIM, typename real>
__global__ __launch_bounds__(kTile) void k_setvel(const PlumeDev* __restrict__ plumes,
                                                 const TileDev* __restrict__ tiles,
                                                 const double* __restrict__ v, uint32_t N, StateArrays U) {
    const TileDev t = tiles[blockIdx.x];
    const uint32_t a = t.start + threadIdx.x;
    if (a >= t.end) return;
    const PlumeDev P = plumes[t.plume];
    double va[3] = {0.0, 0.0, 0.0}, Dt[6];
    for (int c = 0; c < DIM; ++c) {
        va[c] = v[(size_t)c * N + a];
        static_cast<real*>(U.vel[c])[a] = (real)va[c];
    }
    // the tensor of the velocity as stored (working precision), so that the
    // moves and the tensors see the same velocity
    for (int c = 0; c < DIM; ++c) va[c] = (double)(real)va[c];
    tensor_of<DIM>(P.aL, P.aT, P.Dm, va, Dt);
    for (int k = 0; k < GenDims<DIM>::kT; ++k) {
        // a diagonal component is at least min(alpha_L, alpha_T) |v| + D_m
        // >= 0; a rounding below 0 is taken as 0, so its reciprocal is
        // positive (or +inf)
        const double d = is_diag<DIM>(k) ? fmax(Dt[k], 0.0) : Dt[k];
        static_cast<real*>(U.rD[k])[a] = (real)(1.0 / d);
    }
}

// One particle as the pair term reads it: position, C, velocity and the
// reciprocals of its tensor components.
template <int DIM, typename real>
struct GPart {
    uint32_t x, y, z;
    real C;
    real v[DIM];
    real r[GenDims<DIM>::kT];
};

// 2D FP32 reads the particle's 32-byte record, the other cases the
// structure-of-arrays state.
template <int DIM, typename real>
__device__ __forceinline__ GPart<DIM, real> load_part(const StateArrays& S, uint32_t k) {
    GPart<DIM, real> p;
    if constexpr (DIM == 2 && sizeof(real) == 4) {
        // 32-bit byte offset from a uniform base (a velocity-field context in
        // 2D FP32 holds fewer than 2^27 particles)
        const char* base = reinterpret_cast<const char*>(S.grec) + (k << 5);
        const uint4 a = *reinterpret_cast<const uint4*>(base), b = *reinterpret_cast<const uint4*>(base + 16);
        p.x = a.x;
        p.y = a.y;
        p.z = 0u;
        p.C = __uint_as_float(a.z);
        p.v[0] = __uint_as_float(a.w);
        p.v[1] = __uint_as_float(b.x);
        p.r[0] = __uint_as_float(b.y);
        p.r[1] = __uint_as_float(b.z);
        p.r[2] = __uint_as_float(b.w);
    } else {
        p.x = S.pos[0][k];
        p.y = S.pos[1][k];
        p.z = (DIM == 3) ? S.pos[2][k] : 0u;
        p.C = static_cast<const real*>(S.C)[k];
#pragma unroll
        for (int d = 0; d < DIM; ++d) p.v[d] = static_cast<const real*>(S.vel[d])[k];
#pragma unroll
        for (int q = 0; q < GenDims<DIM>::kT; ++q) p.r[q] = static_cast<const real*>(S.rD[q])[k];
    }
    return p;
}

// A quarter of the harmonic mean of Eq. (5) from the reciprocals of the two
// components: 4 p q / (p + q) = 4 / (1/p + 1/q) when p q > 0, and 0 when
// p q <= 0 (a product of reciprocals has the sign of p q; a zero component
// has an infinite reciprocal, whose product is not positive against the other
// sign and whose sum gives 0 against the same sign).
__device__ __forceinline__ float hmean(float ra, float rb) {
    return ra * rb > 0.f ? __builtin_amdgcn_rcpf(ra + rb) : 0.f;
}
__device__ __forceinline__ double hmean(double ra, double rb) {
    return ra * rb > 0.0 ? 1.0 / (ra + rb) : 0.0;
}
// the same for diagonal components, whose reciprocals are positive or +inf:
// the sum is never NaN and 1 / inf = 0 covers a zero component
__device__ __forceinline__ float hmean_diag(float ra, float rb) { return __builtin_amdgcn_rcpf(ra + rb); }
__device__ __forceinline__ double hmean_diag(double ra, double rb) { return 1.0 / (ra + rb); }

// The walk of a target's list by its LANES lanes: lane lj evaluates records
// lj, lj + LANES, ... of the concatenated ranges, B at a time with the next
// batch in flight; slots past the end of its share re-read record `self`
// (the target's own: r2 = 0, rejected by the predicate).  The wavefront runs
// as many batches as its largest share needs.
template <int LANES, int B, typename Fetch, typename Eval>
__device__ __forceinline__ void walk_lanes(const uint2* list, uint32_t stride, uint32_t total, uint32_t lj,
                                           uint32_t self, Fetch&& fetch, Eval&& eval) {
    using CandT = decltype(fetch(0u));
    uint32_t share = total > lj ? (total - lj + LANES - 1) / LANES : 0u;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) share = max(share, (uint32_t)__shfl_xor((int)share, o, kWave));
    const uint32_t nb = __builtin_amdgcn_readfirstlane((share + B - 1) / B);
    if (nb == 0) return;
    Cursor<LANES> cur;
    cur.b = lj * kRecBytes;
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
            cur.b += Cursor<LANES>::kStep;
            cur.settle();
        }
#pragma unroll
        for (int q = 0; q < B; ++q) c[q] = fetch(idx[q]);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto run = [&](const CandT(&c)[B]) {
#pragma unroll
        for (int q = 0; q < B; ++q) eval(c[q], true);
    };
    fill(c0);
    for (uint32_t it = 1;; it += 2) {
        if (it >= nb) {
            run(c0);
            break;
        }
        fill(c1);
        run(c0);
        if (it + 1 >= nb) {
            run(c1);
            break;
        }
        fill(c0);
        run(c1);
    }
}

// The pair term of Eqs. (4)-(5) between target A and candidate c at the
// separation (dx, dy, dz) = x_a - x_c in grid units: disp gains Dcal_ac / 4
// f (C_a - C_c) and conv f (v_a - v_c) . x_ac, with f the kernel factor
// W'(r)/r short of its constant (keep false: the slot adds nothing).
template <int DIM, typename real, int KERN>
__device__ __forceinline__ void gen_term(const GPart<DIM, real>& A, const GPart<DIM, real>& c, real dx, real dy,
                                         real dz, bool keep, real invHu, real gam, real& disp, real& conv) {
    const real dx2 = dx * dx, dy2 = dy * dy;
    real r2 = dx2 + dy2;
    if (DIM == 3) r2 = fmar(dz, dz, r2);
    // the support is cut by the clamp of 1 - q at 0; r2 = 0 (the target
    // itself, a padding slot, a coincident particle) by the select below.
    // Two distinct positions are at least one grid unit apart, so the
    // clamp of r2 at 1 changes nothing else and keeps every factor finite.
    const bool in = keep && r2 > (real)0;
    const real rinv = rsqrt_r(r2 > (real)1 ? r2 : (real)1);
    real omq = fmar(-(r2 * rinv), invHu, (real)1);
    omq = pos_unit(omq);
    real f;
    if (KERN == 4) {  // (1 - q)^5 (1 + 5q) / 6
        const real o2 = omq * omq;
        f = (o2 * o2) * fmar((real)(-5.0 / 6.0), o2, omq);
    } else {
        f = omq * omq * omq;
    }
    f = in ? f : (real)0;
    const real ir2 = rinv * rinv;
    // the pair's harmonic-mean tensor h, divided by 4
    real quad, tr;
    if (DIM == 2) {
        const real hxx = hmean_diag(A.r[0], c.r[0]), hxy = hmean(A.r[1], c.r[1]);
        const real hyy = hmean_diag(A.r[2], c.r[2]);
        quad = fmar(hxx, dx2, fmar(hyy, dy2, (hxy + hxy) * (dx * dy)));
        tr = hxx + hyy;
    } else {
        const real hxx = hmean_diag(A.r[0], c.r[0]), hxy = hmean(A.r[1], c.r[1]), hxz = hmean(A.r[2], c.r[2]);
        const real hyy = hmean_diag(A.r[3], c.r[3]), hyz = hmean(A.r[4], c.r[4]);
        const real hzz = hmean_diag(A.r[5], c.r[5]);
        quad = hxx * dx2 + hyy * dy2 + hzz * dz * dz + (real)2 * (hxy * dx * dy + hxz * dx * dz + hyz * dy * dz);
        tr = hxx + hyy + hzz;
    }
    const real dcal = fmar(gam * quad, ir2, -tr);  // Dcal / 4
    disp = fmar(dcal * f, A.C - c.C, disp);
    real vx = (A.v[0] - c.v[0]) * dx;
    vx = fmar(A.v[1] - c.v[1], dy, vx);
    if (DIM == 3) vx = fmar(A.v[DIM - 1] - c.v[DIM - 1], dz, vx);
    conv = fmar(f, vx, conv);
}

// The end of target i's pair sums (disp: the Dcal / 4 terms, conv: the
// convective ones): rhs mode writes the right-hand side in id order; the
// other modes update C, move the particle on its own schedule and hash it
// into the next build's cell counts.
template <int DIM, typename real, int KERN, int MODE>
__device__ __forceinline__ void gen_finish(const GenLaunch& g, const PlumeDev& P, const Target& T,
                                           const GPart<DIM, real>& A, uint32_t i, real disp, real conv) {
    constexpr int NT = GenDims<DIM>::kT;
    const StateArrays& S = g.S;
    // 1/2 of the sum of Dcal terms = 2 disp (disp sums Dcal / 4); x_ab of the
    // convective term is in grid units, L / 2^32 each; the kernel factor f
    // left out its value at q = 0 (6 for C4)
    constexpr double kS = (KERN == 4) ? 6.0 : 1.0;
    const real rhs = (real)(kS * P.vphi) * fmar(A.C * (real)(P.L * (1.0 / 4294967296.0)), conv, (real)2 * disp);
    if (MODE == kModeRhs) {
        static_cast<real*>(g.out)[S.id[i]] = rhs;
        return;
    }
    // step (Euler), or the predictor-corrector's two stages (Eqs. 8-9, each
    // followed by a cell build): the predictor writes C^(1/2) = C + dt/2 rhs,
    // carries C^n and moves to x^(1/2); the corrector, evaluated there,
    // writes C^n + dt rhs and moves on to x^(n+1).  C, the move on the
    // particle's own schedule (from step k + f0 to k + f1), hashing and
    // counting
    const StateArrays& U = g.U;
    double f0 = 0.0, f1 = 1.0;
    if (MODE == kModeHalf) {
        static_cast<real*>(U.C)[i] = fmar((real)(0.5 * P.dt), rhs, A.C);
        static_cast<real*>(U.Cb)[i] = A.C;
        f1 = 0.5;
    } else if (MODE == kModeFull) {
        static_cast<real*>(U.C)[i] = fmar((real)P.dt, rhs, static_cast<const real*>(S.Cb)[i]);
        f0 = 0.5;
    } else {
        static_cast<real*>(U.C)[i] = fmar((real)P.dt, rhs, A.C);
    }
    const int64_t k = *g.step;
    uint32_t u[3] = {T.ux, T.uy, T.uz};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double us = (double)A.v[c] * P.dt / P.L * 4294967296.0;
        const int64_t s1 = (int64_t)rint(((double)k + f1) * us);
        const int64_t s0 = (int64_t)rint(((double)k + f0) * us);
        u[c] += (uint32_t)(s1 - s0);
        U.pos[c][i] = u[c];
        static_cast<real*>(U.vel[c])[i] = A.v[c];
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) static_cast<real*>(U.rD[q])[i] = A.r[q];
    const uint32_t id = S.id[i];
    U.id[i] = id;
    const uint32_t key = cell_key<DIM>(P, u[0], u[1], u[2]);
    U.key[i] = key;
    enlist(g.lists, key, id);
}

// A work item = blockDim.x / LANES consecutive targets of one tile, LANES
// lanes per target (the launch shape of the context's tuning).
template <int DIM, typename real, int KERN, int MODE, int LANES>
__global__ __launch_bounds__(256) void k_pair_gen(GenLaunch g) {
    extern __shared__ uint2 lds_list[];
    const uint32_t tpb = blockDim.x / LANES, subs = kTile / tpb;
    const TileDev t = g.tiles[blockIdx.x / subs];
    const uint32_t i0 = t.start + (blockIdx.x % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = g.plumes[t.plume];
    const uint32_t lt = threadIdx.x / LANES, lj = threadIdx.x % LANES;
    // lanes past the end of a ragged tile stay in the walk (the wavefront
    // reductions need every lane) with an empty list and target i0
    const bool active = i0 + lt < i1;
    const uint32_t i = active ? i0 + lt : i0;

    const StateArrays& S = g.S;
    const GPart<DIM, real> A = load_part<DIM, real>(S, i);
    const Target T = make_target<DIM>(P, A.x, A.y, A.z);

    // every lane of a target writes the same list
    uint2* list = lds_list + lt;
    uint32_t total = 0;
    if (active) total = build_list<DIM, LANES>(P, g.cell_start, T, list, tpb);
    else list[0] = make_uint2(kListEndStart, kListEndEnd);

    const real invHu = (real)P.invHu;
    const real gam = (real)(DIM + 2);
    real disp = 0, conv = 0;
    auto fetch = [&](uint32_t k) { return load_part<DIM, real>(S, k / kRecBytes); };
    auto eval = [&](const GPart<DIM, real>& c, bool keep) {
        const real dx = (real)(int32_t)(T.ux - c.x);
        const real dy = (real)(int32_t)(T.uy - c.y);
        const real dz = (DIM == 3) ? (real)(int32_t)(T.uz - c.z) : (real)0;
        gen_term<DIM, real, KERN>(A, c, dx, dy, dz, keep, invHu, gam, disp, conv);
    };
    walk_lanes<LANES, kGenBatch>(list, tpb, total, lj, i, fetch, eval);
    // the lanes of a target combine their sums (fixed order: deterministic)
    if (LANES >= 2) {
        disp += __shfl_xor(disp, 1, kWave);
        conv += __shfl_xor(conv, 1, kWave);
    }
    if (LANES >= 4) {
        disp += __shfl_xor(disp, 2, kWave);
        conv += __shfl_xor(conv, 2, kWave);
    }
    if (!active || lj != 0) return;
    gen_finish<DIM, real, KERN, MODE>(g, P, T, A, i, disp, conv);
}

// Two neighbouring targets a and b served by the four lanes of a quad (2D
// FP32), as the uniform-flow kernel's quads serve them: the quad lists the
// union of the two targets' row windows (build_rows_quad over union_row), its
// lanes walk that list two records a lane a batch, and every record is
// evaluated for both targets, b's separation formed from a's as
// (x_b - x_a) + (x_a - x_c).  Each fetched record and each step of the cursor
// serve two pair terms, and the two terms' reciprocal chains are independent.
// A wavefront holding a pair that pair_rows does not merge walks each
// target's own list, in two passes.  Padding slots re-read the pass target's
// own record (r2 = 0 for it); b keeps only the slots below the lane's share.
template <int DIM, typename real, int KERN, int MODE>
__global__ __launch_bounds__(256) void k_pair_gen42(GenLaunch g) {
    extern __shared__ uint2 lds_list[];
    const uint32_t nq = blockDim.x / 4u;  // quads (lists) per workgroup
    const uint32_t tpb = 2u * nq, subs = kTile / tpb;
    const TileDev t = g.tiles[blockIdx.x / subs];
    const uint32_t i0 = t.start + (blockIdx.x % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = g.plumes[t.plume];
    const uint32_t lq = threadIdx.x / 4u, lj = threadIdx.x % 4u;
    // past the end of a ragged tile a quad keeps a copy of a valid target
    // (its sums are discarded)
    const uint32_t ia = i0 + 2u * lq, ib = ia + 1u;
    const bool actA = ia < i1, actB = ib < i1;
    const uint32_t iA = actA ? ia : i0, iB = actB ? ib : iA;

    const StateArrays& S = g.S;
    auto target = [&](uint32_t k) {
        return make_target<DIM>(P, S.pos[0][k], S.pos[1][k], (DIM == 3) ? S.pos[2][k] : 0u);
    };
    int pry = 0, prz = 0;
    const bool close = pair_rows<DIM>(P, target(iA), target(iB), pry, prz);
    const bool merged = __builtin_amdgcn_ballot_w64(!close) == 0ull;  // the whole wavefront
    uint2* list = lds_list + lq;
    const real invHu = (real)P.invHu;
    const real gam = (real)(DIM + 2);
    auto fetch = [&](uint32_t k) { return load_part<DIM, real>(S, k / kRecBytes); };
    real dispA = 0, convA = 0, dispB = 0, convB = 0;
    const int npass = merged ? 1 : 2;
    for (int pass = 0; pass < npass; ++pass) {
        // the pass's pair: (a, b), or (a, a) and then (b, b)
        const bool second = pass == 1;
        const uint32_t k0 = second ? iB : iA, k1 = merged ? iB : k0;
        const GPart<DIM, real> A0 = load_part<DIM, real>(S, k0), A1 = load_part<DIM, real>(S, k1);
        const Target T0 = make_target<DIM>(P, A0.x, A0.y, A0.z), T1 = make_target<DIM>(P, A1.x, A1.y, A1.z);
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
                [&](int oy, int oz) { return union_row<DIM>(P, g.cell_start, T0, T1, dxc, ry, rz, oy, oz); }, ny,
                nz, min(0, ry) - R, (DIM == 3) ? min(0, rz) - R : 0, list, nq);
        } else {
            list[0] = make_uint2(kListEndStart, kListEndEnd);
        }
        real d0 = 0, c0 = 0, d1 = 0, c1 = 0;
        // one record a lane a batch: two targets' terms per record hold the
        // kernel at 83 VGPRs (five wavefronts per SIMD, no spill); two
        // records took 127 VGPRs and ran 2-4% slower
        walk_list_fn<4, 1>(k0, list, nq, total, lj, fetch, [&](const GPart<DIM, real>& c, bool keep) {
            const real dx = (real)(int32_t)(T0.ux - c.x);
            const real dy = (real)(int32_t)(T0.uy - c.y);
            const real dz = (DIM == 3) ? (real)(int32_t)(T0.uz - c.z) : (real)0;
            gen_term<DIM, real, KERN>(A0, c, dx, dy, dz, true, invHu, gam, d0, c0);
            gen_term<DIM, real, KERN>(A1, c, dx + bx, dy + by, dz + bz, keep, invHu, gam, d1, c1);
        });
        if (second) {
            dispB = d0;
            convB = c0;
        } else {
            dispA = d0;
            convA = c0;
            dispB = d1;
            convB = c1;
        }
    }
    // the quad's partial sums (fixed order: deterministic); lane 0 finishes
    // a, lane 1 b
    dispA += __shfl_xor(dispA, 1, kWave);
    dispA += __shfl_xor(dispA, 2, kWave);
    convA += __shfl_xor(convA, 1, kWave);
    convA += __shfl_xor(convA, 2, kWave);
    dispB += __shfl_xor(dispB, 1, kWave);
    dispB += __shfl_xor(dispB, 2, kWave);
    convB += __shfl_xor(convB, 1, kWave);
    convB += __shfl_xor(convB, 2, kWave);
    const bool fa = lj == 0 && actA, fb = lj == 1 && actB;
    if (!fa && !fb) return;
    const uint32_t i = fa ? iA : iB;
    const GPart<DIM, real> A = load_part<DIM, real>(S, i);
    gen_finish<DIM, real, KERN, MODE>(g, P, make_target<DIM>(P, A.x, A.y, A.z), A, i, fa ? dispA : dispB,
                                      fa ? convA : convB);
}

// dD/dtheta_k of Eq. (3) at velocity v, in the stored component order (k =
// 0: alpha_L, v v^T/|v|; 1: alpha_T, |v| I - v v^T/|v|; 2: D_m, I; the v v^T/|v|
// parts are 0 for v = 0)
template <int DIM, typename real>
__device__ __forceinline__ void tensor_derivs(const real* v, real (&dD)[3][GenDims<DIM>::kT]) {
    real s2 = v[0] * v[0];
#pragma unroll
    for (int c = 1; c < DIM; ++c) s2 = fmar(v[c], v[c], s2);
    const real sp = sqrt(s2);
    const real inv = sp > (real)0 ? (real)1 / sp : (real)0;
    // (i, j) of stored component q: 2D xx, xy, yy; 3D xx, xy, xz, yy, yz, zz
    constexpr int ci[6] = {0, 0, DIM == 2 ? 1 : 0, 1, 1, 2};
    constexpr int cj[6] = {0, 1, DIM == 2 ? 1 : 2, 1, 2, 2};
#pragma unroll
    for (int q = 0; q < GenDims<DIM>::kT; ++q) {
        const int i = ci[q], j = cj[q];
        const real vv = v[i] * v[j] * inv;
        const real id = (i == j) ? (real)1 : (real)0;
        dD[0][q] = vv;
        dD[1][q] = fmar(sp, id, -vv);
        dD[2][q] = id;
    }
}

// Adjoint pass of the velocity-field Euler step.  With equal particle volumes
// the dispersion weights w_ab of the pair sum are symmetric and the convective
// term of Eq. (4) is diagonal in C, so L^T = L and
//     lambda^n = lambda + dt L lambda
// is the forward pair sum applied to lambda.  The gradient gains
// dt lambda_a (L_k C)_a, where L_k has each pair's harmonic mean replaced by
// its derivative with respect to theta_k: with p = D_ij,a and q = D_ij,b,
//     d(h/4)_ij = (q^2 dp + p^2 dq) / (p + q)^2   (0 where p q <= 0),
// and no convective part (it does not depend on theta).  The tensors come
// from the stored reciprocals (1 / inf = 0 for a zero component).
template <int DIM, typename real, int KERN, int LANES, int AMODE>
__global__ __launch_bounds__(256) void k_adjoint_gen(AdjGenLaunch g) {
    extern __shared__ uint2 lds_list[];
    __shared__ double lds[kTile / kWave];
    constexpr int NT = GenDims<DIM>::kT;
    const uint32_t tpb = blockDim.x / LANES, subs = kTile / tpb;
    const TileDev t = g.tiles[blockIdx.x / subs];
    const uint32_t i0 = t.start + (blockIdx.x % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = g.plumes[t.plume];
    const uint32_t lt = threadIdx.x / LANES, lj = threadIdx.x % LANES;
    const bool active = i0 + lt < i1;
    const uint32_t i = active ? i0 + lt : i0;

    const StateArrays& S = g.S;
    const real* __restrict__ lam_s = static_cast<const real*>(g.lam_s);
    const GPart<DIM, real> A = load_part<DIM, real>(S, i);
    const real la = lam_s[i];
    const Target T = make_target<DIM>(P, A.x, A.y, A.z);
    real Da[NT], dA[3][NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) Da[q] = (real)1 / A.r[q];
    tensor_derivs<DIM, real>(A.v, dA);

    uint2* list = lds_list + lt;
    uint32_t total = 0;
    if (active) total = build_list<DIM, LANES>(P, g.cell_start, T, list, tpb);
    else list[0] = make_uint2(kListEndStart, kListEndEnd);

    const real H2 = h2_of<real>(P), invHu = (real)P.invHu;
    const real gam = (real)(DIM + 2);
    real al = 0, cv = 0, gk[3] = {0, 0, 0};
    struct Cand {
        GPart<DIM, real> p;
        real lam;
    };
    auto fetch = [&](uint32_t k) {
        k /= kRecBytes;
        return Cand{load_part<DIM, real>(S, k), lam_s[k]};
    };
    // the Dcal-type bracket Gamma x^T M x / r^2 - tr M of a symmetric tensor M
    // (stored components), times r^2 / r^2 in grid units
    auto bracket = [&](const real (&M)[NT], real dx, real dy, real dz, real ir2) {
        real quad, tr;
        if (DIM == 2) {
            quad = fmar(M[0] * dx, dx, fmar((real)2 * M[1] * dx, dy, M[2] * dy * dy));
            tr = M[0] + M[2];
        } else {
            quad = M[0] * dx * dx + M[3] * dy * dy + M[5] * dz * dz +
                   (real)2 * (M[1] * dx * dy + M[2] * dx * dz + M[4] * dy * dz);
            tr = M[0] + M[3] + M[5];
        }
        return fmar(gam * quad, ir2, -tr);
    };
    auto eval = [&](const Cand& cc, bool keep) {
        const GPart<DIM, real>& c = cc.p;
        const real dx = (real)(int32_t)(T.ux - c.x);
        const real dy = (real)(int32_t)(T.uy - c.y);
        const real dz = (DIM == 3) ? (real)(int32_t)(T.uz - c.z) : (real)0;
        real r2 = dx * dx;
        r2 = fmar(dy, dy, r2);
        if (DIM == 3) r2 = fmar(dz, dz, r2);
        const bool in = keep && r2 > (real)0 && r2 <= H2;
        const real rinv = rsqrt_r(r2);
        const real q = r2 * rinv * invHu;
        real omq = (real)1 - q;
        omq = pos_unit(omq);
        real f;
        if (KERN == 4) {
            const real o2 = omq * omq;
            f = o2 * o2 * omq * fmar((real)5, q, (real)1);
        } else {
            f = omq * omq * omq;
        }
        f = in ? f : (real)0;
        const real ir2 = in ? rinv * rinv : (real)0;
        real h[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) h[k] = is_diag<DIM>(k) ? hmean_diag(A.r[k], c.r[k]) : hmean(A.r[k], c.r[k]);
        al = fmar(bracket(h, dx, dy, dz, ir2) * f, la - cc.lam, al);
        real vx = (A.v[0] - c.v[0]) * dx;
        vx = fmar(A.v[1] - c.v[1], dy, vx);
        if (DIM == 3) vx = fmar(A.v[DIM - 1] - c.v[DIM - 1], dz, vx);
        cv = fmar(f, vx, cv);
        // derivative operators: d(h/4) = wa dD_a + wb dD_b per component
        real dB[3][NT], wa[NT], wb[NT];
        tensor_derivs<DIM, real>(c.v, dB);
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const real p = Da[k], qq = (real)1 / c.r[k];
            const real s = p + qq;
            const real inv2 = p * qq > (real)0 ? (real)1 / (s * s) : (real)0;
            wa[k] = qq * qq * inv2;
            wb[k] = p * p * inv2;
        }
        const real dC = (A.C - c.C) * f;
#pragma unroll
        for (int th = 0; th < 3; ++th) {
            real dh[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) dh[k] = fmar(wa[k], dA[th][k], wb[k] * dB[th][k]);
            gk[th] = fmar(bracket(dh, dx, dy, dz, ir2), dC, gk[th]);
        }
    };
    walk_lanes<LANES, kGenBatch>(list, tpb, total, lj, i, fetch, eval);
    // the lanes of a target combine their sums (fixed order: deterministic)
    real red[5] = {al, cv, gk[0], gk[1], gk[2]};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        if (LANES >= 2) red[k] += __shfl_xor(red[k], 1, kWave);
        if (LANES >= 4) red[k] += __shfl_xor(red[k], 2, kWave);
    }
    al = red[0];
    cv = red[1];
    gk[0] = red[2];
    gk[1] = red[3];
    gk[2] = red[4];

    const double sd = P.dt * P.vphi;
    // the gradient's multiplier of (L_k X)_a / vphi = 2 gk (gk sums Dcal_k / 4):
    // dt lambda_a (Euler and the corrector stage at x^(1/2)), dt^2/2 y_a (the
    // predictor stage at x^n)
    double m = 0.0;
    if (active && lj == 0) {
        // (L u)_a / vphi: 1/2 of the sum of Dcal terms = 2 al (al sums Dcal / 4)
        const real Lx = fmar(la * (real)(P.L * (1.0 / 4294967296.0)), cv, (real)2 * al);
        const uint32_t id = S.id[i];
        if (AMODE == kAdjGenEuler) {
            static_cast<real*>(g.lam_out)[id] = fmar((real)sd, Lx, la);
            m = 2.0 * sd * (double)la;
        } else if (AMODE == kAdjGenHalf) {
            static_cast<real*>(g.lam_out)[id] = (real)P.vphi * Lx;  // y = L lambda
            m = 2.0 * sd * (double)la;
        } else {
            // lambda + dt y + dt^2/2 L y, with la = y here
            const real lam = static_cast<const real*>(g.lam_id)[id];
            const real dt = (real)P.dt;
            static_cast<real*>(g.lam_out)[id] = fmar(dt, la, fmar((real)(0.5 * P.dt * sd), Lx, lam));
            m = P.dt * sd * (double)la;
        }
    }
#pragma unroll
    for (int th = 0; th < 3; ++th) {
        const double c = block_sum(m * (double)gk[th], lds);
        if (threadIdx.x == 0) g.gpart[3 * blockIdx.x + th] += c;
    }
}

// four lanes per target, block / 4 targets per workgroup; the gradient
// partials are indexed by workgroup (kTile / (block / 4) per tile)
template <int DIM, typename real, int KERN>
static hipError_t launch_adj_gen_t(int mode, const AdjGenLaunch& a, uint32_t block, hipStream_t s) {
    constexpr int L = 4;
    const uint32_t tpb = block / L;  // targets per workgroup
    const size_t shm = (size_t)tpb * (size_t)a.list_cap * 8u;
    if (shm > kPairLdsMax || block < 64 || block > 256 || kTile % tpb) return hipErrorInvalidValue;
    if (DIM == 2 && sizeof(real) == 4 && !a.S.grec) return hipErrorInvalidValue;
    if (mode == kAdjGenFull && !a.lam_id) return hipErrorInvalidValue;
    auto kern = (mode == kAdjGenEuler)  ? k_adjoint_gen<DIM, real, KERN, L, kAdjGenEuler>
                : (mode == kAdjGenHalf) ? k_adjoint_gen<DIM, real, KERN, L, kAdjGenHalf>
                                        : k_adjoint_gen<DIM, real, KERN, L, kAdjGenFull>;
    hipLaunchKernelGGL(kern, dim3(a.ntiles * (kTile / tpb)), dim3(block), shm, s, a);
    return hipGetLastError();
}

hipError_t launch_adjoint_gen(int dim, int real_bytes, int kernel, int mode, const AdjGenLaunch& a,
                              uint32_t block, hipStream_t s) {
    if (mode != kAdjGenEuler && mode != kAdjGenHalf && mode != kAdjGenFull) return hipErrorInvalidValue;
    if (dim == 2) {
        if (real_bytes == 4)
            return kernel == 4 ? launch_adj_gen_t<2, float, 4>(mode, a, block, s)
                               : launch_adj_gen_t<2, float, 2>(mode, a, block, s);
        return kernel == 4 ? launch_adj_gen_t<2, double, 4>(mode, a, block, s)
                           : launch_adj_gen_t<2, double, 2>(mode, a, block, s);
    }
    if (real_bytes == 4)
        return kernel == 4 ? launch_adj_gen_t<3, float, 4>(mode, a, block, s)
                           : launch_adj_gen_t<3, float, 2>(mode, a, block, s);
    return kernel == 4 ? launch_adj_gen_t<3, double, 4>(mode, a, block, s)
                       : launch_adj_gen_t<3, double, 2>(mode, a, block, s);
}

hipError_t launch_setvel(int dim, int real_bytes, const PlumeDev* plumes, const TileDev* tiles, uint32_t ntiles,
                         const double* v, uint32_t N, StateArrays U, hipStream_t s) {
    dim3 gr(ntiles), b(kTile);
    if (dim == 2 && real_bytes == 4) hipLaunchKernelGGL((k_setvel<2, float>), gr, b, 0, s, plumes, tiles, v, N, U);
    else if (dim == 2) hipLaunchKernelGGL((k_setvel<2, double>), gr, b, 0, s, plumes, tiles, v, N, U);
    else if (real_bytes == 4) hipLaunchKernelGGL((k_setvel<3, float>), gr, b, 0, s, plumes, tiles, v, N, U);
    else hipLaunchKernelGGL((k_setvel<3, double>), gr, b, 0, s, plumes, tiles, v, N, U);
    return hipGetLastError();
}

template <int DIM, typename real, int KERN, int LANES>
static hipError_t launch_gen_l(int mode, const GenLaunch& g, hipStream_t s) {
    const uint32_t block = (uint32_t)g.block;
    if (block != 64 && block != 128 && block != 256) return hipErrorInvalidValue;
    const size_t shm = (size_t)(block / LANES) * (size_t)g.list_cap * 8u;
    if (shm > kPairLdsMax) return hipErrorInvalidValue;
    if (DIM == 2 && sizeof(real) == 4 && !g.S.grec) return hipErrorInvalidValue;
    dim3 gr(g.ntiles * (kTile / (block / LANES))), b(block);
    auto kern = (mode == kModeStep)   ? k_pair_gen<DIM, real, KERN, kModeStep, LANES>
                : (mode == kModeHalf) ? k_pair_gen<DIM, real, KERN, kModeHalf, LANES>
                : (mode == kModeFull) ? k_pair_gen<DIM, real, KERN, kModeFull, LANES>
                                      : k_pair_gen<DIM, real, KERN, kModeRhs, LANES>;
    if (g.ev0)  // timed launch: the events carry the kernel's own start and end stamps
        hipExtLaunchKernelGGL(kern, gr, b, (uint32_t)shm, s, g.ev0, g.ev1, 0u, g);
    else
        hipLaunchKernelGGL(kern, gr, b, shm, s, g);
    return hipGetLastError();
}

// four lanes per two targets (2D FP32): a work item holds block / 2 targets
template <int DIM, typename real, int KERN>
static hipError_t launch_gen_42(int mode, const GenLaunch& g, hipStream_t s) {
    const uint32_t block = (uint32_t)g.block;
    if (block != 64 && block != 128 && block != 256) return hipErrorInvalidValue;
    const size_t shm = (size_t)(block / 4u) * (size_t)g.list_cap * 8u;
    if (shm > kPairLdsMax || !g.S.grec) return hipErrorInvalidValue;
    dim3 gr(g.ntiles * (kTile / (block / 2u))), b(block);
    auto kern = (mode == kModeStep)   ? k_pair_gen42<DIM, real, KERN, kModeStep>
                : (mode == kModeHalf) ? k_pair_gen42<DIM, real, KERN, kModeHalf>
                : (mode == kModeFull) ? k_pair_gen42<DIM, real, KERN, kModeFull>
                                      : k_pair_gen42<DIM, real, KERN, kModeRhs>;
    if (g.ev0)
        hipExtLaunchKernelGGL(kern, gr, b, (uint32_t)shm, s, g.ev0, g.ev1, 0u, g);
    else
        hipLaunchKernelGGL(kern, gr, b, shm, s, g);
    return hipGetLastError();
}

template <int DIM, typename real, int KERN>
static hipError_t launch_gen_t(int mode, const GenLaunch& g, hipStream_t s) {
    if (g.targets == 2) {
        if constexpr (DIM == 2 && sizeof(real) == 4) {
            if (g.lanes == 4) return launch_gen_42<DIM, real, KERN>(mode, g, s);
        }
        return hipErrorInvalidValue;
    }
    if (g.lanes == 4) return launch_gen_l<DIM, real, KERN, 4>(mode, g, s);
    if (g.lanes == 2) return launch_gen_l<DIM, real, KERN, 2>(mode, g, s);
    if (g.lanes == 1) return launch_gen_l<DIM, real, KERN, 1>(mode, g, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pair_gen(int dim, int real_bytes, int kernel, int mode, const GenLaunch& g, hipStream_t s) {
    if (mode != kModeStep && mode != kModeRhs && mode != kModeHalf && mode != kModeFull) return hipErrorInvalidValue;
    if ((mode == kModeHalf || mode == kModeFull) && (!g.U.Cb || !g.S.Cb)) return hipErrorInvalidValue;
    if (dim == 2) {
        if (real_bytes == 4) return kernel == 4 ? launch_gen_t<2, float, 4>(mode, g, s) : launch_gen_t<2, float, 2>(mode, g, s);
        return kernel == 4 ? launch_gen_t<2, double, 4>(mode, g, s) : launch_gen_t<2, double, 2>(mode, g, s);
    }
    if (real_bytes == 4) return kernel == 4 ? launch_gen_t<3, float, 4>(mode, g, s) : launch_gen_t<3, float, 2>(mode, g, s);
    return kernel == 4 ? launch_gen_t<3, double, 4>(mode, g, s) : launch_gen_t<3, double, 2>(mode, g, s);
}

}  // namespace ade
