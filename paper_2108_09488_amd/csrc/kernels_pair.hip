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
#include "ade_device.h"

namespace ade {

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float rsqrt_r(float x) { return rsqrtf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }

template <typename real>
__device__ __forceinline__ real h2_of(const PlumeDev& P) {
    return sizeof(real) == 4 ? (real)P.H2f : (real)P.H2d;
}

// Visit every particle b (sorted index) of the plume with 0 < r2 <= H_u^2
// around the fixed-point position (ux, uy, uz).  Candidates: the rows within
// R rows (y, and z in 3D) of the target's row, and in each row the x cells
// covering [x - hx, x + hx]; each such cell range is contiguous in the sorted
// order, so a row costs two loads of the cell-start table.
template <int DIM, typename real, typename F>
__device__ __forceinline__ void for_each_neighbour(const PlumeDev& P,
                                                   const uint32_t* __restrict__ cs,
                                                   const uint32_t* __restrict__ px,
                                                   const uint32_t* __restrict__ py,
                                                   const uint32_t* __restrict__ pz,
                                                   uint32_t ux, uint32_t uy, uint32_t uz,
                                                   F&& visit) {
    const real H2 = h2_of<real>(P);
    const int R = P.R;
    const int nr = (int)P.nr;
    const uint32_t nfx = P.nfx;
    const int ry = (int)__umulhi(uy, P.nr);
    const int rz = (DIM == 3) ? (int)__umulhi(uz, P.nr) : 0;
    const uint32_t clo = __umulhi(ux - P.hx, nfx);
    const uint32_t chi = __umulhi(ux + P.hx, nfx);
    const bool wrapx = clo > chi;

    auto scan = [&](uint32_t s, uint32_t e) {
        for (uint32_t b = s; b < e; ++b) {
            const real dx = (real)(int32_t)(ux - px[b]);
            const real dy = (real)(int32_t)(uy - py[b]);
            const real dz = (DIM == 3) ? (real)(int32_t)(uz - pz[b]) : (real)0;
            real r2 = dx * dx;
            r2 = fmar(dy, dy, r2);
            if (DIM == 3) r2 = fmar(dz, dz, r2);
            if (r2 > (real)0 && r2 <= H2) visit(b, dx, dy, dz, r2);
        }
    };

    const int zlo = (DIM == 3) ? -R : 0, zhi = (DIM == 3) ? R : 0;
    for (int oz = zlo; oz <= zhi; ++oz) {
        int zz = rz + oz;
        zz += (zz < 0) ? nr : 0;
        zz -= (zz >= nr) ? nr : 0;
        for (int oy = -R; oy <= R; ++oy) {
            int yy = ry + oy;
            yy += (yy < 0) ? nr : 0;
            yy -= (yy >= nr) ? nr : 0;
            const uint32_t row = P.cbase + ((uint32_t)zz * P.nr + (uint32_t)yy) * nfx;
            const uint32_t s0 = cs[row + clo];
            const uint32_t e0 = wrapx ? cs[row + nfx] : cs[row + chi + 1];
            scan(s0, e0);
            if (wrapx) scan(cs[row], cs[row + chi + 1]);
        }
    }
}

template <int DIM, typename real, int KERN, int MODE>
__global__ __launch_bounds__(kTile) void k_pair(PairLaunch a) {
    const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
    const TileDev t = a.tiles[tile];
    const PlumeDev& P = a.plumes[t.plume];
    const uint32_t i = t.start + threadIdx.x;
    if (i >= t.end) return;

    const uint32_t* __restrict__ px = a.spos[0];
    const uint32_t* __restrict__ py = a.spos[1];
    const uint32_t* __restrict__ pz = a.spos[2];
    const real* __restrict__ Cp = static_cast<const real*>(a.Cpair);

    const uint32_t ux = px[i], uy = py[i], uz = (DIM == 3) ? pz[i] : 0u;
    const real Ca = Cp[i];
    const real invHu = (real)P.invHu;
    const real kxx = (real)P.kg[0], kyy = (real)P.kg[1], kzz = (real)P.kg[2];
    const real kxy = (real)P.kg[3], kxz = (real)P.kg[4], kyz = (real)P.kg[5];
    const real trD = (real)P.trD;
    real acc = (real)0;

    for_each_neighbour<DIM, real>(
        P, a.cell_start, px, py, pz, ux, uy, uz,
        [&](uint32_t b, real dx, real dy, real dz, real r2) {
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
            acc = fmar(A * f, Ca - Cp[b], acc);
        });

    if (MODE == kModeRhs) {
        static_cast<real*>(a.out)[a.sid[i]] = (real)P.vphi * acc;
        return;
    }
    const real sc = (real)(a.scale * P.dt * P.vphi);
    const real Cb = static_cast<const real*>(a.Cbase)[i];
    if (MODE == kModeHalf) {
        static_cast<real*>(a.out)[i] = fmar(sc, acc, Cb);
        return;
    }
    // step: update C and x, hash the moved particle for the next build
    const int64_t k = *a.step;
    uint32_t u[3] = {ux, uy, uz};
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

// Neighbour-set export: fill = 0 writes the count of particle id at
// offsets[id]; fill = 1 writes the ids from offsets[id] on.
template <int DIM, typename real>
__global__ __launch_bounds__(kTile) void k_nbr(const PlumeDev* __restrict__ plumes,
                                              const TileDev* __restrict__ tiles, StateArrays S,
                                              const uint32_t* __restrict__ cs, int fill,
                                              int64_t* __restrict__ offsets,
                                              int32_t* __restrict__ ids) {
    const TileDev t = tiles[blockIdx.x];
    const PlumeDev& P = plumes[t.plume];
    const uint32_t i = t.start + threadIdx.x;
    if (i >= t.end) return;
    const uint32_t* px = S.pos[0];
    const uint32_t* py = S.pos[1];
    const uint32_t* pz = S.pos[2];
    const uint32_t ux = px[i], uy = py[i], uz = (DIM == 3) ? pz[i] : 0u;
    const uint32_t me = S.id[i];
    int64_t k = fill ? offsets[me] : 0;
    for_each_neighbour<DIM, real>(P, cs, px, py, pz, ux, uy, uz,
                                  [&](uint32_t b, real, real, real, real) {
                                      if (fill) ids[k] = (int32_t)S.id[b];
                                      ++k;
                                  });
    if (!fill) offsets[me] = k;
}

template <int DIM, typename real, int KERN>
static void launch_pair_t(int mode, const PairLaunch& a, int block, hipStream_t s) {
    (void)block;
    dim3 g(a.ntiles), b(kTile);
    if (mode == kModeStep) hipLaunchKernelGGL((k_pair<DIM, real, KERN, kModeStep>), g, b, 0, s, a);
    else if (mode == kModeHalf) hipLaunchKernelGGL((k_pair<DIM, real, KERN, kModeHalf>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_pair<DIM, real, KERN, kModeRhs>), g, b, 0, s, a);
}

hipError_t launch_pair(int dim, int real_bytes, int kernel, int mode, const PairLaunch& a,
                       int block, hipStream_t s) {
    if (dim == 2) {
        if (real_bytes == 4) {
            if (kernel == 4) launch_pair_t<2, float, 4>(mode, a, block, s);
            else launch_pair_t<2, float, 2>(mode, a, block, s);
        } else {
            if (kernel == 4) launch_pair_t<2, double, 4>(mode, a, block, s);
            else launch_pair_t<2, double, 2>(mode, a, block, s);
        }
    } else {
        if (real_bytes == 4) {
            if (kernel == 4) launch_pair_t<3, float, 4>(mode, a, block, s);
            else launch_pair_t<3, float, 2>(mode, a, block, s);
        } else {
            if (kernel == 4) launch_pair_t<3, double, 4>(mode, a, block, s);
            else launch_pair_t<3, double, 2>(mode, a, block, s);
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
