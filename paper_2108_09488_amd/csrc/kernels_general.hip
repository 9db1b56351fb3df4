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
// One lane per target walks the target's candidate list (ade_walk.h); the
// candidates are read from the structure-of-arrays state.
#include <hip/hip_ext.h>

#include "ade_walk.h"

namespace ade {

template <int DIM>
struct GenDims {
    static constexpr int kT = DIM == 2 ? 3 : 6;  // tensor components stored per particle
};

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
// tensors they give.
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
    for (int k = 0; k < GenDims<DIM>::kT; ++k) static_cast<real*>(U.Dt[k])[a] = (real)Dt[k];
}

template <int DIM, typename real>
struct GCand {
    uint32_t x, y, z;
    real C;
    real v[DIM];
    real D[GenDims<DIM>::kT];
};

__device__ __forceinline__ float harm4(float p, float q) {
    const float pq = p * q;
    return pq > 0.f ? 4.f * pq / (p + q) : 0.f;
}
__device__ __forceinline__ double harm4(double p, double q) {
    const double pq = p * q;
    return pq > 0.0 ? 4.0 * pq / (p + q) : 0.0;
}

// A work item = blockDim.x consecutive targets of one tile (blockDim.x a
// divisor of the tile, chosen so the candidate lists fit in LDS).
template <int DIM, typename real, int KERN, int MODE>
__global__ __launch_bounds__(256) void k_pair_gen(GenLaunch g) {
    extern __shared__ uint2 lds_list[];
    constexpr int NT = GenDims<DIM>::kT;
    const uint32_t tpb = blockDim.x, subs = kTile / tpb;
    const TileDev t = g.tiles[blockIdx.x / subs];
    const uint32_t i0 = t.start + (blockIdx.x % subs) * tpb;
    if (i0 >= t.end) return;  // whole workgroup: ragged last tile
    const uint32_t i1 = min(t.end, i0 + tpb);
    const PlumeDev P = g.plumes[t.plume];
    const bool active = i0 + threadIdx.x < i1;
    const uint32_t i = active ? i0 + threadIdx.x : i0;

    const StateArrays& S = g.S;
    const uint32_t* __restrict__ px = S.pos[0];
    const uint32_t* __restrict__ py = S.pos[1];
    const uint32_t* __restrict__ pz = S.pos[2];
    const real* __restrict__ C = static_cast<const real*>(S.C);
    const Target T = make_target<DIM>(P, px[i], py[i], (DIM == 3) ? pz[i] : 0u);
    const real Ca = C[i];
    real va[DIM], Da[NT];
#pragma unroll
    for (int c = 0; c < DIM; ++c) va[c] = static_cast<const real*>(S.vel[c])[i];
#pragma unroll
    for (int k = 0; k < NT; ++k) Da[k] = static_cast<const real*>(S.Dt[k])[i];

    uint2* list = lds_list + threadIdx.x;
    uint32_t total = 0;
    if (active) total = build_list<DIM, 1>(P, g.cell_start, T, list, tpb);
    else list[0] = make_uint2(kListEndStart, kListEndEnd);

    const real H2 = h2_of<real>(P), invHu = (real)P.invHu;
    const real gam = (real)(DIM + 2);
    real disp = 0, conv = 0;
    auto fetch = [&](uint32_t k) {
        k /= kRecBytes;
        GCand<DIM, real> c;
        c.x = px[k];
        c.y = py[k];
        c.z = (DIM == 3) ? pz[k] : 0u;
        c.C = C[k];
#pragma unroll
        for (int d = 0; d < DIM; ++d) c.v[d] = static_cast<const real*>(S.vel[d])[k];
#pragma unroll
        for (int q = 0; q < NT; ++q) c.D[q] = static_cast<const real*>(S.Dt[q])[k];
        return c;
    };
    auto eval = [&](const GCand<DIM, real>& c, bool keep) {
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
        omq = omq > (real)0 ? omq : (real)0;
        real f;
        if (KERN == 4) {
            const real o2 = omq * omq;
            f = o2 * o2 * omq * fmar((real)5, q, (real)1);
        } else {
            f = omq * omq * omq;
        }
        // outside the support (and at r2 = 0) every factor below is finite
        // and f = 0, so the terms vanish
        f = in ? f : (real)0;
        const real ir2 = in ? rinv * rinv : (real)0;
        real quad, tr;
        if (DIM == 2) {
            const real hxx = harm4(Da[0], c.D[0]), hxy = harm4(Da[1], c.D[1]), hyy = harm4(Da[2], c.D[2]);
            quad = fmar(hxx * dx, dx, fmar((real)2 * hxy * dx, dy, hyy * dy * dy));
            tr = hxx + hyy;
        } else {
            const real hxx = harm4(Da[0], c.D[0]), hxy = harm4(Da[1], c.D[1]), hxz = harm4(Da[2], c.D[2]);
            const real hyy = harm4(Da[3], c.D[3]), hyz = harm4(Da[4], c.D[4]), hzz = harm4(Da[5], c.D[5]);
            quad = hxx * dx * dx + hyy * dy * dy + hzz * dz * dz +
                   (real)2 * (hxy * dx * dy + hxz * dx * dz + hyz * dy * dz);
            tr = hxx + hyy + hzz;
        }
        const real dcal = fmar(gam * quad, ir2, -tr);
        disp = fmar((real)0.5 * dcal * f, Ca - c.C, disp);
        real vx = (va[0] - c.v[0]) * dx + (va[1] - c.v[1]) * dy;
        if (DIM == 3) vx = fmar(va[DIM - 1] - c.v[DIM - 1], dz, vx);
        conv = fmar(f, vx, conv);
    };
    walk_stream<4>(list, tpb, total, i, fetch, eval);
    if (!active) return;

    // x_ab of the convective term in grid units: L / 2^32 per unit
    const real rhs = (real)P.vphi * fmar(Ca * (real)(P.L * (1.0 / 4294967296.0)), conv, disp);
    if (MODE == kModeRhs) {
        static_cast<real*>(g.out)[S.id[i]] = rhs;
        return;
    }
    // step: C, the move on the particle's own schedule, hashing and counting
    const StateArrays& U = g.U;
    static_cast<real*>(U.C)[i] = fmar((real)P.dt, rhs, Ca);
    const int64_t k = *g.step;
    uint32_t u[3] = {T.ux, T.uy, T.uz};
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const double us = (double)va[c] * P.dt / P.L * 4294967296.0;
        const int64_t s1 = (int64_t)rint((double)(k + 1) * us);
        const int64_t s0 = (int64_t)rint((double)k * us);
        u[c] += (uint32_t)(s1 - s0);
        U.pos[c][i] = u[c];
        static_cast<real*>(U.vel[c])[i] = va[c];
    }
#pragma unroll
    for (int q = 0; q < NT; ++q) static_cast<real*>(U.Dt[q])[i] = Da[q];
    const uint32_t id = S.id[i];
    U.id[i] = id;
    const uint32_t key = cell_key<DIM>(P, u[0], u[1], u[2]);
    U.key[i] = key;
    enlist(g.lists, key, id);
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

template <int DIM, typename real, int KERN>
static hipError_t launch_gen_t(int mode, const GenLaunch& g, hipStream_t s) {
    uint32_t block = 256;  // the largest divisor of the tile whose lists fit in LDS
    while (block > 64 && (size_t)block * (size_t)g.list_cap * 8u > kPairLdsMax) block /= 2;
    const size_t shm = (size_t)block * (size_t)g.list_cap * 8u;
    if (shm > kPairLdsMax) return hipErrorInvalidValue;
    dim3 gr(g.ntiles * (kTile / block)), b(block);
    auto kern = (mode == kModeStep) ? k_pair_gen<DIM, real, KERN, kModeStep> : k_pair_gen<DIM, real, KERN, kModeRhs>;
    if (g.ev0)  // timed launch: the events carry the kernel's own start and end stamps
        hipExtLaunchKernelGGL(kern, gr, b, (uint32_t)shm, s, g.ev0, g.ev1, 0u, g);
    else
        hipLaunchKernelGGL(kern, gr, b, shm, s, g);
    return hipGetLastError();
}

hipError_t launch_pair_gen(int dim, int real_bytes, int kernel, int mode, const GenLaunch& g, hipStream_t s) {
    if (mode != kModeStep && mode != kModeRhs) return hipErrorInvalidValue;
    if (dim == 2) {
        if (real_bytes == 4) return kernel == 4 ? launch_gen_t<2, float, 4>(mode, g, s) : launch_gen_t<2, float, 2>(mode, g, s);
        return kernel == 4 ? launch_gen_t<2, double, 4>(mode, g, s) : launch_gen_t<2, double, 2>(mode, g, s);
    }
    if (real_bytes == 4) return kernel == 4 ? launch_gen_t<3, float, 4>(mode, g, s) : launch_gen_t<3, float, 2>(mode, g, s);
    return kernel == 4 ? launch_gen_t<3, double, 4>(mode, g, s) : launch_gen_t<3, double, 2>(mode, g, s);
}

}  // namespace ade
