// adjoint.hip -- sensor interpolation and the discrete adjoint of the explicit
// SPH advection-dispersion step (Klapp et al., arXiv:2108.09488, Eqs. 3-5),
// giving dJ/d(alpha_L, alpha_T, D_m) for the misfit J = sum_s (C_s - d_s)^2.
//
// With rhs = L C and the explicit step C^{n+1} = C^n + dt L^n C^n,
//     lambda^N = dJ/dC^N,  lambda^n = lambda^{n+1} + dt (L^n)^T lambda^{n+1},
//     dJ/dtheta_k = sum_n dt lambda^{n+1} . (dL^n/dtheta_k) C^n.
// For equal particle volumes and a uniform tensor the pair weights are
// symmetric (w_ab = w_ba), so (L^n)^T = L^n: the adjoint kernel applies the
// same pair sum to lambda.
// The predictor-corrector step (Eqs. 8-9) is C^{n+1} = (I + dt L + dt^2/2 L^2)
// C^n: a uniform flow moves every particle by the same displacement, so the
// operator of the corrector stage is that of the predictor.  Its adjoint is
// the same two stages applied to lambda,
//     mu = lambda + dt/2 L lambda,  lambda^n = lambda + dt L mu,
// and with C^h = C^n + dt/2 L C^n the gradient gains
//     dt [lambda . L_k C^h + (mu - lambda) . L_k C^n]
// (= dt lambda . L_k C^n + dt^2/2 (lambda . L_k L C^n + L lambda . L_k C^n)).
// kAdjHalf forms mu, C^h and the second term; kAdjFull forms lambda^n and
// the first.  L depends on theta only through D (Eq. 3), which
// is linear in theta: dD/dalpha_L = v v^T/|v|, dD/dalpha_T = |v| I - v v^T/|v|,
// dD/dD_m = I.  With p = (x_ab . v)^2 / (|v|^2 r^2) the factor
// A = Gamma x^T M x / r^2 - tr M of the pair term becomes
//     alpha_L: |v| (Gamma p - 1),  alpha_T: |v| (Gamma (1 - p) - (d - 1)),
//     D_m: Gamma - d.
// The forward states are recomputed from checkpoints segment by segment
// (the cell build and the pair sums are deterministic, so the recompute is
// bit-identical to the forward run), and the gradient is accumulated in FP64
// per workgroup in a fixed order.
//
// Sensors: Shepard interpolation C_s = sum_b W(r_sb) C_b / sum_b W(r_sb) with
// the kernel of Eq. (7) (its normalisation cancels); its transpose seeds
// lambda^N = sum_s 2 (C_s - d_s) W(r_sb) / sum_b' W(r_sb').
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "ade_walk.h"
#include "ctx.h"

namespace ade {

// Kernel shape of Eq. (7) without its normalisation, as a function of q = r / H.
template <typename real, int KERN>
__device__ __forceinline__ real kernel_shape(real q) {
    real omq = (real)1 - q;
    omq = pos_unit(omq);
    const real o2 = omq * omq;
    if (KERN == 4) return o2 * o2 * o2 * fmar(q, fmar((real)(35.0 / 3.0), q, (real)6), (real)1);
    return o2 * o2 * fmar((real)4, q, (real)1);
}

template <int DIM>
__device__ __forceinline__ uint32_t to_fixed(double x, double L) {
    return (uint32_t)(int64_t)rint((x / L) * 4294967296.0);
}

// ---------------------------------------------------------------------------
// sensors
// ---------------------------------------------------------------------------
template <int DIM, typename real, int KERN>
__global__ __launch_bounds__(256) void k_sensor_fwd(const PlumeDev* __restrict__ plumes,
                                                   const double* __restrict__ xs, int ns,
                                                   StateArrays S, const uint32_t* __restrict__ cs,
                                                   real* __restrict__ pred, real* __restrict__ den) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const PlumeDev P = plumes[0];
    uint32_t u[3] = {0u, 0u, 0u};
    for (int c = 0; c < DIM; ++c) u[c] = to_fixed<DIM>(xs[(size_t)c * ns + s], P.L);
    const Target T = make_target<DIM>(P, u[0], u[1], u[2]);
    const real H2 = h2_of<real>(P), invHu = (real)P.invHu;
    const uint32_t* px = S.pos[0];
    const uint32_t* py = S.pos[1];
    const uint32_t* pz = S.pos[2];
    const real* C = static_cast<const real*>(S.C);
    const int span = 2 * P.R + 1, noff = (DIM == 3) ? span * span : span;
    real num = 0, dsum = 0;
    for (int j = 0; j < noff; ++j) {
        const RowRanges r = row_ranges<DIM>(P, cs, T, j, span);
        for (int part = 0; part < 2; ++part) {
            const uint32_t b0 = part ? r.s1 : r.s0, b1 = part ? r.e1 : r.e0;
            for (uint32_t b = b0; b < b1; ++b) {
                const real dx = (real)(int32_t)(T.ux - px[b]);
                const real dy = (real)(int32_t)(T.uy - py[b]);
                const real dz = (DIM == 3) ? (real)(int32_t)(T.uz - pz[b]) : (real)0;
                real r2 = dx * dx;
                r2 = fmar(dy, dy, r2);
                if (DIM == 3) r2 = fmar(dz, dz, r2);
                if (r2 <= H2) {
                    const real w = kernel_shape<real, KERN>(sqrt(r2) * invHu);
                    num = fmar(w, C[b], num);
                    dsum += w;
                }
            }
        }
    }
    pred[s] = dsum > (real)0 ? num / dsum : (real)0;
    if (den) den[s] = dsum;
}

// residual weights r_s = 2 (C_s - d_s) / sum_b W_sb and J (FP64, fixed order)
template <typename real>
__global__ __launch_bounds__(256) void k_sensor_resid(int ns, const real* __restrict__ pred,
                                                     const real* __restrict__ den,
                                                     const real* __restrict__ obs,
                                                     real* __restrict__ rw, double* __restrict__ J) {
    __shared__ double lds[256 / kWave];
    double acc = 0.0;
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
        const double d = (double)pred[s] - (double)obs[s];
        acc += d * d;
        rw[s] = den[s] > (real)0 ? (real)(2.0 * d / (double)den[s]) : (real)0;
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) *J = acc;
}

// lambda^N[id_b] = sum_s r_s W(r_sb), sensors staged through LDS in chunks
template <int DIM, typename real, int KERN>
__global__ __launch_bounds__(256) void k_sensor_seed(const PlumeDev* __restrict__ plumes,
                                                    const double* __restrict__ xs, int ns,
                                                    const real* __restrict__ rw, StateArrays S,
                                                    uint32_t N, real* __restrict__ lam) {
    __shared__ uint32_t su[256][3];
    __shared__ real sr[256];
    const PlumeDev P = plumes[0];
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < N;
    uint32_t u[3] = {0u, 0u, 0u};
    if (active)
        for (int c = 0; c < DIM; ++c) u[c] = S.pos[c][i];
    const real H2 = h2_of<real>(P), invHu = (real)P.invHu;
    real acc = 0;
    for (int s0 = 0; s0 < ns; s0 += 256) {
        __syncthreads();
        const int s = s0 + threadIdx.x;
        if (s < ns) {
            for (int c = 0; c < DIM; ++c) su[threadIdx.x][c] = to_fixed<DIM>(xs[(size_t)c * ns + s], P.L);
            sr[threadIdx.x] = rw[s];
        }
        __syncthreads();
        const int cnt = min(256, ns - s0);
        if (active) {
            for (int k = 0; k < cnt; ++k) {
                // separation sensor - particle, as in the forward interpolation
                const real dx = (real)(int32_t)(su[k][0] - u[0]);
                const real dy = (real)(int32_t)(su[k][1] - u[1]);
                const real dz = (DIM == 3) ? (real)(int32_t)(su[k][2] - u[2]) : (real)0;
                real r2 = dx * dx;
                r2 = fmar(dy, dy, r2);
                if (DIM == 3) r2 = fmar(dz, dz, r2);
                if (r2 <= H2) acc = fmar(sr[k], kernel_shape<real, KERN>(sqrt(r2) * invHu), acc);
            }
        }
    }
    if (active) lam[S.id[i]] = acc;
}

// ---------------------------------------------------------------------------
// adjoint step
// ---------------------------------------------------------------------------
// The adjoint passes walk the candidate lists of the forward kernels (cell
// rows in LDS, one lane per target, batches of records in flight).  A
// candidate carries its position and the pass's two values: X (the state in
// the gradient terms) and u (the vector the operator is applied to).  In 2D
// FP32 they travel as one 16-byte record (x, y, X, u) written just before
// the pass; otherwise they are read from the arrays.
template <typename real>
struct ACand {
    uint32_t x, y, z;
    real X, u;
};

template <int DIM, typename real>
struct ARec {
    static constexpr bool kPacked = DIM == 2 && sizeof(real) == 4;
};

__device__ __forceinline__ uint32_t fbits(float v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ float bitsf(uint32_t v) { return __builtin_bit_cast(float, v); }

// lambda from id order into cell order (and the records (x, y, X, lambda))
template <int DIM, typename real>
__global__ __launch_bounds__(256) void k_adj_gather(StateArrays S, const real* __restrict__ lam_id,
                                                   const real* __restrict__ X, uint32_t N,
                                                   real* __restrict__ lam_s, uint4* __restrict__ arec) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const real l = lam_id[S.id[i]];
    lam_s[i] = l;
    if constexpr (ARec<DIM, real>::kPacked) arec[i] = make_uint4(S.pos[0][i], S.pos[1][i], fbits(X[i]), fbits(l));
}

struct AdjConst {
    double speed;    // |v|
};

// kAdjEuler: out = lambda^n (id order) = lam + dt L lam, gradient dt lam . L_k X.
// kAdjHalf:  out = mu (cell order) = lam + dt/2 L lam, xh_out = C^h (cell
//            order) = X + dt/2 L X, arec_out = their records, gradient
//            dt (mu - lam) . L_k X.
// kAdjFull:  out = lambda^n (id order) = lam + dt L u (u = mu), gradient
//            dt lam . L_k X (X = C^h).
// A workgroup takes blockDim.x consecutive targets of a tile; its gradient
// partials go to gpart[3 * blockIdx.x ..].
enum AdjMode { kAdjEuler = 0, kAdjHalf = 1, kAdjFull = 2 };

template <int DIM, typename real, int KERN, int AMODE>
__global__ __launch_bounds__(256) void k_adjoint(const PlumeDev* __restrict__ plumes,
                                                const TileDev* __restrict__ tiles, StateArrays S,
                                                const uint32_t* __restrict__ cs,
                                                const real* __restrict__ u_s,
                                                const real* __restrict__ lam_s,
                                                const real* __restrict__ X,
                                                const uint4* __restrict__ arec,
                                                real* __restrict__ lam_out, real* __restrict__ xh_out,
                                                uint4* __restrict__ arec_out, AdjConst ac,
                                                double* __restrict__ gpart) {
    extern __shared__ uint2 lds_list[];
    __shared__ double lds[kTile / kWave];
    constexpr bool kPacked = ARec<DIM, real>::kPacked;
    const uint32_t tpb = blockDim.x, subs = kTile / tpb;
    const TileDev t = tiles[blockIdx.x / subs];
    const uint32_t i0 = t.start + (blockIdx.x % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = plumes[t.plume];
    const bool active = i0 + threadIdx.x < i1;
    const uint32_t i = active ? i0 + threadIdx.x : i0;
    const uint32_t* __restrict__ px = S.pos[0];
    const uint32_t* __restrict__ py = S.pos[1];
    const uint32_t* __restrict__ pz = S.pos[2];
    const Target T = make_target<DIM>(P, px[i], py[i], (DIM == 3) ? pz[i] : 0u);
    const real Xi = X[i], ui = u_s[i], li = lam_s[i];
    const real H2 = h2_of<real>(P), invHu = (real)P.invHu;
    const real a0 = (real)P.a0, a1 = (real)P.a1;
    const real gam = (real)(DIM + 2), spd = (real)ac.speed;
    const real vx = (real)P.ehat[0], vy = (real)P.ehat[1], vz = (real)P.ehat[2];

    uint2* list = lds_list + threadIdx.x;
    uint32_t total = 0;
    if (active) total = build_list<DIM, 1>(P, cs, T, list, tpb);
    else list[0] = make_uint2(kListEndStart, kListEndEnd);

    real al = 0, cl = 0, g1 = 0, g2 = 0, g3 = 0;
    auto fetch = [&](uint32_t k) {
        if constexpr (kPacked) {
            const uint4 r = *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(arec) + k);
            return ACand<real>{r.x, r.y, 0u, (real)bitsf(r.z), (real)bitsf(r.w)};
        } else {
            k /= kRecBytes;
            return ACand<real>{px[k], py[k], (DIM == 3) ? pz[k] : 0u, X[k], u_s[k]};
        }
    };
    // branch-free: outside the support (and at r2 = 0, where 1/r is infinite)
    // f and p are replaced by 0, so every term is exactly 0
    auto eval = [&](const ACand<real>& c, bool keep) {
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
        // Gamma x^T D x / r^2 - tr D = a0 + a1 p, p = (e . x / r)^2
        const real xv = fmar(dz, vz, fmar(dy, vy, dx * vx));
        real p = xv * xv * (rinv * rinv);
        f = in ? f : (real)0;
        p = in ? p : (real)0;
        const real A = fmar(a1, p, a0);
        const real dCf = (Xi - c.X) * f;
        al = fmar(A * f, ui - c.u, al);
        if (AMODE == kAdjHalf) cl = fmar(A, dCf, cl);
        g1 = fmar(spd * fmar(gam, p, (real)-1), dCf, g1);
        g2 = fmar(spd * fmar(-gam, p, gam - (real)(DIM - 1)), dCf, g2);
        g3 = fmar(gam - (real)DIM, dCf, g3);
    };
    walk_stream<4>(list, tpb, total, i, fetch, eval);

    double mult = 0.0;  // the gradient's multiplier of this particle
    if (active) {
        const double sd = P.dt * P.vphi;
        if (AMODE == kAdjHalf) {
            const real h = (real)(0.5 * sd);
            const real mu = fmar(h, al, li), xh = fmar(h, cl, Xi);
            lam_out[i] = mu;
            xh_out[i] = xh;
            if constexpr (kPacked) arec_out[i] = make_uint4(T.ux, T.uy, fbits(xh), fbits(mu));
            mult = 0.5 * sd * (double)al;  // mu - lambda
        } else {
            lam_out[S.id[i]] = fmar((real)sd, al, li);
            mult = (double)li;
        }
    }
    // per-workgroup gradient partials, accumulated over the steps in FP64
    const double s = P.dt * P.vphi;
    const double c1 = block_sum(active ? s * mult * (double)g1 : 0.0, lds);
    const double c2 = block_sum(active ? s * mult * (double)g2 : 0.0, lds);
    const double c3 = block_sum(active ? s * mult * (double)g3 : 0.0, lds);
    if (threadIdx.x == 0) {
        gpart[3 * blockIdx.x + 0] += c1;
        gpart[3 * blockIdx.x + 1] += c2;
        gpart[3 * blockIdx.x + 2] += c3;
    }
}

__global__ __launch_bounds__(256) void k_grad_reduce(const double* __restrict__ gpart, uint32_t nb,
                                                    double* __restrict__ out) {
    __shared__ double lds[256 / kWave];
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) s += gpart[3 * b + k];
        s = block_sum(s, lds);
        if (threadIdx.x == 0) out[k] = s;
    }
}

// copy of a state snapshot: positions, C (as 32-bit words), ids, records,
// the cell table and the step counter
struct SnapCopy {
    uint32_t* dpos[3];
    const uint32_t* spos[3];
    uint32_t* dC;
    const uint32_t* sC;
    uint32_t* did;
    const uint32_t* sid;
    uint4* drec;
    const uint4* srec;
    uint32_t* dcs;
    const uint32_t* scs;
    int64_t* dstep;
    const int64_t* sstep;
    uint32_t n, ncs, cwords;
    // velocity field: the per-particle arrays (velocities, tensor reciprocals,
    // 2D FP32 records) as 32-bit words, xn[e] words each
    uint32_t* dx[10];
    const uint32_t* sx[10];
    uint32_t xn[10];
    int nx;
};

__global__ __launch_bounds__(256) void k_copy_snap(SnapCopy a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *a.dstep = *a.sstep;
    if (i < a.n * a.cwords) a.dC[i] = a.sC[i];
    if (i < a.ncs) a.dcs[i] = a.scs[i];
    if (i >= a.n) return;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (a.dpos[d]) a.dpos[d][i] = a.spos[d][i];
    a.did[i] = a.sid[i];
    if (a.drec) a.drec[i] = a.srec[i];
}

// the velocity-field arrays of a snapshot copy (a separate launch: the
// 32-byte records make them the largest arrays)
__global__ __launch_bounds__(256) void k_copy_snap_x(SnapCopy a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int e = 0; e < a.nx; ++e)
        if (i < a.xn[e]) a.dx[e][i] = a.sx[e][i];
}

namespace {

#define ADE_DISPATCH3(dim, rb, kern, CALL)                              \
    do {                                                                \
        if (dim == 2 && rb == 4 && kern == 4) { CALL(2, float, 4); }    \
        else if (dim == 2 && rb == 4) { CALL(2, float, 2); }            \
        else if (dim == 2 && kern == 4) { CALL(2, double, 4); }         \
        else if (dim == 2) { CALL(2, double, 2); }                      \
        else if (rb == 4 && kern == 4) { CALL(3, float, 4); }           \
        else if (rb == 4) { CALL(3, float, 2); }                        \
        else if (kern == 4) { CALL(3, double, 4); }                     \
        else { CALL(3, double, 2); }                                    \
    } while (0)

// One state snapshot: the sorted particle state and its cell table.
struct Snap {
    uint32_t* pos[3];
    void* C;
    uint32_t* id;
    uint4* rec;
    uint32_t* cs;
    int64_t* step;
    void* vel[3];  // velocity field only (null otherwise)
    void* rD[6];
    uint4* grec;
};

constexpr uint32_t kAdjMaxSubs = 4;  // workgroups per tile of the adjoint passes (64 threads)
// the velocity-field pass: 256 threads, four lanes per target, so 64 targets
// and kAdjMaxSubs workgroups per tile
constexpr uint32_t kGenAdjBlock = 256;

// threads per workgroup of the adjoint passes: the largest of 256, 128, 64
// whose candidate lists fit in 64 KiB of LDS
uint32_t adj_block(const Plan& pl) {
    for (uint32_t b = 256; b > 64; b /= 2)
        if ((size_t)b * (size_t)pl.list_cap * 8u <= kPairLdsMax) return b;
    return 64;
}

// count snapshots laid out one after the other, `stride` bytes apart (every
// snapshot of a context has the same size and starts 256-byte aligned)
struct SnapSeq {
    Snap first{};
    size_t stride = 0;
    size_t count = 0;
    Snap operator[](size_t k) const {
        Snap s = first;
        const size_t d = k * stride;
        auto shift = [d](auto*& p) {
            if (p) p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(reinterpret_cast<char*>(p) + d);
        };
        for (int i = 0; i < 3; ++i) shift(s.pos[i]);
        shift(s.C);
        shift(s.id);
        shift(s.rec);
        shift(s.cs);
        shift(s.step);
        for (int i = 0; i < 3; ++i) shift(s.vel[i]);
        for (int i = 0; i < 6; ++i) shift(s.rD[i]);
        shift(s.grec);
        return s;
    }
};

struct AdjLayout {
    size_t bytes = 0;
    SnapSeq ck;    // checkpoints (every K steps, plus the final state)
    SnapSeq seg;   // states of one segment
    SnapSeq segh;  // velocity field with the predictor-corrector: their half-step states
    void* y;                // ... and y = L lambda of the corrector stage (id order)
    void* lam[2];
    void* lam_s;
    void* mu_s;  // predictor-corrector: mu and C^h of the step (cell order)
    void* ch_s;
    uint4* arec;   // 2D FP32: candidate records of the pass (x, y, X, u)
    uint4* arec2;  // predictor-corrector: those of the second pass
    void* pred;
    void* den;
    void* rw;
    double* J;
    double* gpart;
    double* grad;
};

void take_snap(char* base, size_t& off, const ade_ctx* c, Snap& s) {
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~size_t(255);
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const Plan& pl = c->plan;
    const size_t N = (size_t)pl.N;
    for (int d = 0; d < 3; ++d) s.pos[d] = (d < pl.dim) ? (uint32_t*)take(N * 4) : nullptr;
    s.C = take(N * pl.real_bytes);
    s.id = (uint32_t*)take(N * 4);
    s.rec = c->S.rec ? (uint4*)take(N * 16) : nullptr;
    s.cs = (uint32_t*)take((pl.ncell + 1) * 4);
    s.step = (int64_t*)take(8);
    for (int d = 0; d < 3; ++d) s.vel[d] = c->S.vel[d] ? take(N * pl.real_bytes) : nullptr;
    for (int d = 0; d < 6; ++d) s.rD[d] = c->S.rD[d] ? take(N * pl.real_bytes) : nullptr;
    s.grec = c->S.grec ? (uint4*)take(N * 32) : nullptr;
}

void adj_layout(const ade_ctx* c, int64_t nsteps, int32_t K, int32_t ns, char* base, AdjLayout& L) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~size_t(255);
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const Plan& pl = c->plan;
    const int64_t nck = (nsteps + K - 1) / K + 1;
    // one snapshot's size, as take_snap lays it out from an aligned offset
    size_t snap_bytes = 0;
    {
        Snap probe;
        take_snap(nullptr, snap_bytes, c, probe);
        snap_bytes = (snap_bytes + 255) & ~size_t(255);
    }
    const bool gpc = pl.general && pl.integrator == ADE_PC;
    auto seq = [&](SnapSeq& q, size_t count) {
        q.count = count;
        q.stride = snap_bytes;
        off = (off + 255) & ~size_t(255);
        size_t o = off;
        if (count) take_snap(base, o, c, q.first);
        off += count * snap_bytes;
    };
    seq(L.ck, (size_t)nck);
    seq(L.seg, (size_t)K);
    seq(L.segh, gpc ? (size_t)K : 0);
    const size_t N = (size_t)pl.N, rb = (size_t)pl.real_bytes;
    L.lam[0] = take(N * rb);
    L.lam[1] = take(N * rb);
    L.lam_s = take(N * rb);
    L.y = gpc ? take(N * rb) : nullptr;
    const bool pc = pl.integrator == ADE_PC;
    const bool packed = pl.dim == 2 && pl.real_bytes == 4;
    L.mu_s = pc ? take(N * rb) : nullptr;
    L.ch_s = pc ? take(N * rb) : nullptr;
    L.arec = packed ? (uint4*)take(N * 16) : nullptr;
    L.arec2 = (packed && pc) ? (uint4*)take(N * 16) : nullptr;
    L.pred = take((size_t)ns * rb);
    L.den = take((size_t)ns * rb);
    L.rw = take((size_t)ns * rb);
    L.J = (double*)take(8);
    L.gpart = (double*)take((size_t)pl.ntiles * kAdjMaxSubs * 3 * 8);
    L.grad = (double*)take(3 * 8);
    L.bytes = off + 256;
}

// one launch per snapshot (the arrays are small for the adjoint's problem
// sizes, so separate copies would be launch-bound)
int copy_state(const ade_ctx* c, const Snap& dst, const Snap& src) {
    const Plan& pl = c->plan;
    const uint32_t N = (uint32_t)pl.N, nc = (uint32_t)pl.ncell + 1;
    const uint32_t words = (uint32_t)pl.real_bytes / 4;
    SnapCopy a;
    for (int d = 0; d < 3; ++d) {
        a.dpos[d] = (d < pl.dim) ? dst.pos[d] : nullptr;
        a.spos[d] = (d < pl.dim) ? src.pos[d] : nullptr;
    }
    a.dC = static_cast<uint32_t*>(dst.C);
    a.sC = static_cast<const uint32_t*>(src.C);
    a.did = dst.id;
    a.sid = src.id;
    a.drec = (dst.rec && src.rec) ? dst.rec : nullptr;
    a.srec = src.rec;
    a.dcs = dst.cs;
    a.scs = src.cs;
    a.dstep = dst.step;
    a.sstep = src.step;
    a.n = N;
    a.ncs = nc;
    a.cwords = words;
    const uint32_t items = std::max(N * words, nc);
    a.nx = 0;
    uint32_t xitems = 0;
    auto extra = [&](void* d, const void* s, uint32_t nw) {
        if (!d || !s) return;
        a.dx[a.nx] = static_cast<uint32_t*>(d);
        a.sx[a.nx] = static_cast<const uint32_t*>(s);
        a.xn[a.nx] = nw;
        ++a.nx;
        xitems = std::max(xitems, nw);
    };
    for (int d = 0; d < 3; ++d) extra(dst.vel[d], src.vel[d], N * words);
    for (int d = 0; d < 6; ++d) extra(dst.rD[d], src.rD[d], N * words);
    extra(dst.grec, src.grec, N * 8);
    hipLaunchKernelGGL(k_copy_snap, dim3((items + 255) / 256), dim3(256), 0, c->stream, a);
    HIPCHK(hipGetLastError());
    if (a.nx > 0) {
        hipLaunchKernelGGL(k_copy_snap_x, dim3((xitems + 255) / 256), dim3(256), 0, c->stream, a);
        HIPCHK(hipGetLastError());
    }
    return ADE_OK;
}

Snap live(ade_ctx* c) {
    Snap s;
    for (int d = 0; d < 3; ++d) s.pos[d] = c->S.pos[d];
    s.C = c->S.C;
    s.id = c->S.id;
    s.rec = c->S.rec;
    s.cs = c->cell_start;
    s.step = c->step;
    for (int d = 0; d < 3; ++d) s.vel[d] = c->S.vel[d];
    for (int d = 0; d < 6; ++d) s.rD[d] = c->S.rD[d];
    s.grec = c->S.grec;
    return s;
}

StateArrays snap_arrays(const ade_ctx* c, const Snap& s) {
    StateArrays a = c->S;
    for (int d = 0; d < 3; ++d) a.pos[d] = s.pos[d] ? s.pos[d] : s.pos[0];
    a.C = s.C;
    a.id = s.id;
    a.rec = s.rec;
    for (int d = 0; d < 3; ++d) a.vel[d] = s.vel[d];
    for (int d = 0; d < 6; ++d) a.rD[d] = s.rD[d];
    a.grec = s.grec;
    return a;
}

int check_sensor_args(const ade_ctx* c, const double* d_xs, int32_t ns) {
    if (!c) return fail(ADE_EINVAL, "null ctx");
    if (!d_xs || ns <= 0) return fail(ADE_EINVAL, "sensors: null positions or n_sensors <= 0");
    if (c->plan.P != 1) return fail(ADE_EINVAL, "sensors and the adjoint need a single-plume context");
    if (!c->built) return fail(ADE_ESTATE, "cells not built");
    return ADE_OK;
}

int launch_sensor_fwd(ade_ctx* c, const double* d_xs, int32_t ns, const StateArrays& S,
                      const uint32_t* cs, void* pred, void* den) {
    const Plan& pl = c->plan;
    dim3 g((ns + 255) / 256), b(256);
#define CALL(D, R, K)                                                                        \
    hipLaunchKernelGGL((k_sensor_fwd<D, R, K>), g, b, 0, c->stream, c->plumes, d_xs, ns, S, cs, \
                       (R*)pred, (R*)den)
    ADE_DISPATCH3(pl.dim, pl.real_bytes, pl.kernel, CALL);
#undef CALL
    HIPCHK(hipGetLastError());
    return ADE_OK;
}

}  // namespace
}  // namespace ade

using namespace ade;

extern "C" {

int ade_sensor_interp(ade_ctx* c, const double* d_xs, int32_t n_sensors, void* d_Cs) {
    int rc = check_sensor_args(c, d_xs, n_sensors);
    if (rc) return rc;
    if (!d_Cs) return fail(ADE_EINVAL, "null output");
    return launch_sensor_fwd(c, d_xs, n_sensors, c->S, c->cell_start, d_Cs, nullptr);
}

int ade_adjoint_workspace_bytes(const ade_ctx* c, int64_t nsteps, int32_t ckpt_every, int32_t n_sensors,
                                size_t* bytes) {
    if (!c || !bytes) return fail(ADE_EINVAL, "null argument");
    if (nsteps < 1 || ckpt_every < 1 || n_sensors < 1)
        return fail(ADE_EINVAL, "nsteps, ckpt_every and n_sensors must be positive");
    AdjLayout L;
    adj_layout(c, nsteps, ckpt_every, n_sensors, nullptr, L);
    *bytes = L.bytes;
    return ADE_OK;
}

}  // extern "C"

namespace {

// The adjoint run of ade_adjoint over a workspace of ws_bytes at d_ws
// (256-byte aligned; arguments checked by the caller).
int adjoint_run(ade_ctx* c, int64_t nsteps, int32_t K, const double* d_xs, int32_t ns, const void* d_obs,
                void* d_ws, size_t ws_bytes, double* h_J, double* h_grad) {
    int rc = ADE_OK;
    AdjLayout L;
    adj_layout(c, nsteps, K, ns, nullptr, L);
    if (ws_bytes < L.bytes) return fail(ADE_EWORKSPACE, "adjoint workspace too small: need %zu bytes", L.bytes);
    adj_layout(c, nsteps, K, ns, static_cast<char*>(d_ws), L);

    const Plan& pl = c->plan;
    const uint32_t N = (uint32_t)pl.N;
    hipStream_t st = c->stream;
    const Snap cur = live(c);
    const int64_t nck = (nsteps + K - 1) / K;

    // forward run with checkpoints
    for (int64_t n = 0; n < nsteps; ++n) {
        if (n % K == 0 && (rc = copy_state(c, L.ck[(size_t)(n / K)], cur))) return rc;
        if ((rc = enqueue_step(c))) return rc;
    }
    if ((rc = copy_state(c, L.ck[(size_t)nck], cur))) return rc;

    // misfit and the adjoint seed at step N
    if ((rc = launch_sensor_fwd(c, d_xs, ns, c->S, c->cell_start, L.pred, L.den))) return rc;
    if (pl.real_bytes == 4)
        hipLaunchKernelGGL((k_sensor_resid<float>), dim3(1), dim3(256), 0, st, ns, (const float*)L.pred,
                           (const float*)L.den, (const float*)d_obs, (float*)L.rw, L.J);
    else
        hipLaunchKernelGGL((k_sensor_resid<double>), dim3(1), dim3(256), 0, st, ns, (const double*)L.pred,
                           (const double*)L.den, (const double*)d_obs, (double*)L.rw, L.J);
    HIPCHK(hipGetLastError());
    {
        dim3 g((N + 255) / 256), b(256);
#define CALL(D, R, KK)                                                                             \
    hipLaunchKernelGGL((k_sensor_seed<D, R, KK>), g, b, 0, st, c->plumes, d_xs, ns, (const R*)L.rw, \
                       c->S, N, (R*)L.lam[0])
        ADE_DISPATCH3(pl.dim, pl.real_bytes, pl.kernel, CALL);
#undef CALL
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemsetAsync(L.gpart, 0, (size_t)pl.ntiles * kAdjMaxSubs * 3 * 8, st));
    const uint32_t ab = adj_block(pl), asubs = kTile / ab;
    const size_t ashm = (size_t)ab * (size_t)pl.list_cap * 8u;
    if (ashm > kPairLdsMax) return fail(ADE_EINVAL, "candidate lists of the adjoint do not fit in LDS");

    AdjConst ac{};
    {
        const PlumeDev& P = pl.plumes[0];
        double sp = 0;
        for (int k = 0; k < pl.dim; ++k) sp += P.vel[k] * P.vel[k];
        sp = std::sqrt(sp);
        ac.speed = sp;
    }

    // reverse sweep, segment by segment
    int li = 0;
    for (int64_t sgi = nck - 1; sgi >= 0; --sgi) {
        const int64_t n0 = sgi * K, n1 = std::min<int64_t>(n0 + K, nsteps);
        if ((rc = copy_state(c, cur, L.ck[(size_t)sgi]))) return rc;
        const bool gpc = pl.general && pl.integrator == ADE_PC;
        for (int64_t n = n0; n < n1; ++n) {
            if ((rc = copy_state(c, L.seg[(size_t)(n - n0)], cur))) return rc;
            if (gpc) {  // the step in its stages, keeping the half-step state
                if ((rc = run_gen(c, kModeHalf, nullptr)) || (rc = enqueue_build(c, 0))) return rc;
                if ((rc = copy_state(c, L.segh[(size_t)(n - n0)], cur))) return rc;
                if ((rc = run_gen(c, kModeFull, nullptr)) || (rc = enqueue_build(c, 1))) return rc;
            } else if ((rc = enqueue_step(c))) {
                return rc;
            }
        }
        for (int64_t n = n1 - 1; n >= n0; --n) {
            const Snap sn = L.seg[(size_t)(n - n0)];
            const StateArrays Sa = snap_arrays(c, sn);
            dim3 g((N + 255) / 256), b(256);
            const dim3 ag(pl.ntiles * asubs), abk(ab);
#define GATHER(D, R, KK)                                                                                   \
    hipLaunchKernelGGL((k_adj_gather<D, R>), g, b, 0, st, Sa, (const R*)L.lam[li], (const R*)sn.C, N,       \
                       (R*)L.lam_s, L.arec)
            ADE_DISPATCH3(pl.dim, pl.real_bytes, pl.kernel, GATHER);
#undef GATHER
#define LAUNCH(D, R, KK, MODE, U, X, REC, OUT, XH, RECOUT)                                                   \
    hipLaunchKernelGGL((k_adjoint<D, R, KK, MODE>), ag, abk, (uint32_t)ashm, st, c->plumes, c->tiles, Sa,     \
                       sn.cs, (const R*)(U), (const R*)L.lam_s, (const R*)(X), (const uint4*)(REC), (R*)(OUT), \
                       (R*)(XH), (uint4*)(RECOUT), ac, L.gpart)
            if (pl.general) {  // velocity field
                AdjGenLaunch ga;
                ga.plumes = c->plumes;
                ga.tiles = c->tiles;
                ga.ntiles = pl.ntiles;
                ga.list_cap = pl.list_cap;
                ga.S = Sa;
                ga.cell_start = sn.cs;
                ga.lam_s = L.lam_s;
                ga.lam_id = nullptr;
                ga.lam_out = L.lam[1 - li];
                ga.gpart = L.gpart;
                if (pl.integrator == ADE_PC) {
                    // y = L2 lambda at the half-step state (its own cells and
                    // order), then lambda^n = lambda + dt y + dt^2/2 L1 y here
                    const Snap sh = L.segh[(size_t)(n - n0)];
                    const StateArrays Sh = snap_arrays(c, sh);
#define GATHER_H(D, R, KK)                                                                                 \
    hipLaunchKernelGGL((k_adj_gather<D, R>), g, b, 0, st, Sh, (const R*)L.lam[li], (const R*)sh.C, N,       \
                       (R*)L.lam_s, L.arec)
                    ADE_DISPATCH3(pl.dim, pl.real_bytes, pl.kernel, GATHER_H);
#undef GATHER_H
                    AdjGenLaunch gh = ga;
                    gh.S = Sh;
                    gh.cell_start = sh.cs;
                    gh.lam_out = L.y;
                    HIPCHK(launch_adjoint_gen(pl.dim, pl.real_bytes, pl.kernel, kAdjGenHalf, gh, kGenAdjBlock, st));
#define GATHER_Y(D, R, KK)                                                                                 \
    hipLaunchKernelGGL((k_adj_gather<D, R>), g, b, 0, st, Sa, (const R*)L.y, (const R*)sn.C, N,             \
                       (R*)L.lam_s, L.arec)
                    ADE_DISPATCH3(pl.dim, pl.real_bytes, pl.kernel, GATHER_Y);
#undef GATHER_Y
                    ga.lam_id = L.lam[li];
                    HIPCHK(launch_adjoint_gen(pl.dim, pl.real_bytes, pl.kernel, kAdjGenFull, ga, kGenAdjBlock, st));
                } else {
                    HIPCHK(launch_adjoint_gen(pl.dim, pl.real_bytes, pl.kernel, kAdjGenEuler, ga, kGenAdjBlock, st));
                }
            } else if (pl.integrator == ADE_PC) {
#define CALL(D, R, KK)                                                                                    \
    LAUNCH(D, R, KK, kAdjHalf, L.lam_s, sn.C, L.arec, L.mu_s, L.ch_s, L.arec2);                              \
    LAUNCH(D, R, KK, kAdjFull, L.mu_s, L.ch_s, L.arec2, L.lam[1 - li], nullptr, nullptr)
                ADE_DISPATCH3(pl.dim, pl.real_bytes, pl.kernel, CALL);
#undef CALL
            } else {
#define CALL(D, R, KK) LAUNCH(D, R, KK, kAdjEuler, L.lam_s, sn.C, L.arec, L.lam[1 - li], nullptr, nullptr)
                ADE_DISPATCH3(pl.dim, pl.real_bytes, pl.kernel, CALL);
#undef CALL
            }
#undef LAUNCH
            HIPCHK(hipGetLastError());
            li = 1 - li;
        }
    }
    // leave the context at step nsteps
    if ((rc = copy_state(c, cur, L.ck[(size_t)nck]))) return rc;
    const uint32_t nparts = pl.ntiles * (pl.general ? kAdjMaxSubs : asubs);  // workgroups of the passes
    hipLaunchKernelGGL(k_grad_reduce, dim3(1), dim3(256), 0, st, L.gpart, nparts, L.grad);
    HIPCHK(hipGetLastError());
    double hostv[4];
    HIPCHK(hipMemcpyAsync(hostv, L.grad, 3 * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hostv + 3, L.J, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < 3; ++k) h_grad[k] = hostv[k];
    *h_J = hostv[3];
    return ADE_OK;
}

int check_adjoint_args(ade_ctx* c, int64_t nsteps, int32_t K, const double* d_xs, int32_t ns, const void* d_obs,
                       double* h_J, double* h_grad) {
    int rc = check_sensor_args(c, d_xs, ns);
    if (rc) return rc;
    if (!d_obs || !h_J || !h_grad) return fail(ADE_EINVAL, "null argument");
    if (nsteps < 1 || K < 1) return fail(ADE_EINVAL, "nsteps and ckpt_every must be positive");
    return ADE_OK;
}

// Adjoint workspace of the allocation-free entry point: a fixed array in the
// library's device memory (one copy per GPU, held until the process ends).
// Host code reaches it only through the address hipGetSymbolAddress gives
// on each device, never through the array's name.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// The scratch array's address on the device of stream st (looked up once per
// device, with that device current).
int scratch_on(hipStream_t st, void** out) {
    int cur = 0, dev = 0;
    HIPCHK(hipGetDevice(&cur));
    dev = cur;
    if (st) HIPCHK(hipStreamGetDevice(st, &dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(ADE_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        if (dev != cur) HIPCHK(hipSetDevice(dev));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return fail(ADE_EHIP, "hipGetSymbolAddress of the scratch array: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ADE_OK;
}

}  // namespace

extern "C" {

int ade_adjoint(ade_ctx* c, int64_t nsteps, int32_t K, const double* d_xs, int32_t ns, const void* d_obs,
                void* d_ws, size_t ws_bytes, double* h_J, double* h_grad) {
    int rc = check_adjoint_args(c, nsteps, K, d_xs, ns, d_obs, h_J, h_grad);
    if (rc) return rc;
    if (!d_ws) return fail(ADE_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(d_ws) & 255u) return fail(ADE_EINVAL, "workspace must be 256-byte aligned");
    return adjoint_run(c, nsteps, K, d_xs, ns, d_obs, d_ws, ws_bytes, h_J, h_grad);
}

int ade_adjoint_noalloc_max_bytes(size_t* bytes) {
    if (!bytes) return fail(ADE_EINVAL, "null argument");
    *bytes = kNoAllocScratchBytes;
    return ADE_OK;
}

int ade_adjoint_noalloc(ade_ctx* c, int64_t nsteps, int32_t K, const double* d_xs, int32_t ns, const void* d_obs,
                        double* h_J, double* h_grad) {
    int rc = check_adjoint_args(c, nsteps, K, d_xs, ns, d_obs, h_J, h_grad);
    if (rc) return rc;
    AdjLayout L;
    adj_layout(c, nsteps, K, ns, nullptr, L);
    if (L.bytes > kNoAllocScratchBytes)
        return fail(ADE_EWORKSPACE,
                    "ade_adjoint_noalloc: this run needs %zu bytes of adjoint workspace, above the %zu bytes of "
                    "the library's static scratch array; use ade_adjoint with a workspace",
                    L.bytes, kNoAllocScratchBytes);
    void* ws = nullptr;
    if ((rc = scratch_on(c->stream, &ws))) return rc;
    return adjoint_run(c, nsteps, K, d_xs, ns, d_obs, ws, kNoAllocScratchBytes, h_J, h_grad);
}

}  // extern "C"
