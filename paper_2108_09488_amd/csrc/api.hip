// api.hip -- the C ABI declared in include/adesph.h: parameter validation,
// workspace layout (the caller owns all device memory), per-plume constants
// and the launch sequence of one step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

using namespace ade;

namespace ade {

namespace {
thread_local std::string g_err;
}

const char* last_error() { return g_err.c_str(); }

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int targets_of(const ade_tuning& t) { return t.targets == 2 ? 2 : 1; }
// two targets per lane: the merged list, or the single-target list of the
// second target of a pair that could not be merged, whichever is longer
int tuning_list_cap(const Plan& pl, const ade_tuning& t) {
    return targets_of(t) == 2 ? std::max(pl.list_cap_pair, pl.list_cap) : pl.list_cap;
}

// launch shapes of the velocity-field kernel: one target per group of
// lanes, or in 2D FP32 two targets per quad; no persistent grid
bool gen_tuning_fits(const Plan& pl, const ade_tuning& t) {
    if (t.block != 64 && t.block != 128 && t.block != 256) return false;
    if (t.lanes != 1 && t.lanes != 2 && t.lanes != 4) return false;
    if (t.targets < 0 || t.targets > 2 || t.persistent != 0) return false;
    if (targets_of(t) == 2 && !(t.lanes == 4 && pl.dim == 2 && pl.real_bytes == 4)) return false;
    return pair_lds_bytes(t.block, t.lanes, tuning_list_cap(pl, t)) <= kPairLdsMax;
}

bool tuning_fits(const Plan& pl, const ade_tuning& t) {
    if (t.block != 64 && t.block != 128 && t.block != 256) return false;
    if (t.lanes != 1 && t.lanes != 2 && t.lanes != 4) return false;
    if (t.targets != 0 && t.targets != 1 && t.targets != 2) return false;
    // two targets: a lane each (block <= 128), or a quad each (FP32)
    if (targets_of(t) == 2 && !((t.lanes == 1 && 2 * t.block <= kTile) || (t.lanes == 4 && pl.real_bytes == 4)))
        return false;
    return pair_lds_bytes(t.block, t.lanes, tuning_list_cap(pl, t)) <= kPairLdsMax;
}

double trace_D(int dim, double aL, double aT, double Dm, const double* v, double D[9]) {
    double s2 = 0;
    for (int i = 0; i < dim; ++i) s2 += v[i] * v[i];
    const double sp = std::sqrt(s2);
    double tr = 0;
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double d = (i == j) ? aT * sp + Dm : 0.0;
            if (sp > 0) d += (aL - aT) * v[i] * v[j] / sp;
            D[i * 3 + j] = d;
            if (i == j) tr += d;
        }
    return tr;
}

}  // namespace ade

namespace {



constexpr double kTwo32 = 4294967296.0;
constexpr double kPi = 3.14159265358979323846;

// Bump allocator over the caller's workspace (base == nullptr: size only).
struct Bump {
    char* base;
    size_t off = 0;
    explicit Bump(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    void* take_bytes(size_t bytes) { return take<char>(bytes); }
};



// Kernel normalisation B and the prefactor of W'(r)/r (Eq. 7 and its C2 sibling).
double kernel_phi_prefactor(int kernel, int dim, double H) {
    double B;
    if (kernel == ADE_WENDLAND_C4)
        B = (dim == 2) ? 9.0 / (kPi * H * H) : 495.0 / (32.0 * kPi * H * H * H);
    else
        B = (dim == 2) ? 7.0 / (kPi * H * H) : 21.0 / (2.0 * kPi * H * H * H);
    return (kernel == ADE_WENDLAND_C4) ? -(56.0 / 3.0) * B / (H * H) : -20.0 * B / (H * H);
}

int plan_grid(const ade_params* params, const int64_t* counts, int32_t nplumes, Plan& pl, int auto_xsub) {
    if (!params || !counts) return fail(ADE_EINVAL, "null params or counts");
    if (nplumes <= 0) return fail(ADE_EINVAL, "nplumes must be positive");
    const ade_params& p0 = params[0];
    pl.dim = p0.dim;
    pl.real_bytes = p0.real_bytes;
    pl.kernel = p0.kernel;
    pl.integrator = p0.integrator;
    pl.general = (p0.flags & ADE_VELOCITY_FIELD) != 0;
    pl.check_finite = false;
    for (int p = 0; p < nplumes; ++p) pl.check_finite = pl.check_finite || (params[p].flags & ADE_CHECK_FINITE);
    pl.P = nplumes;
    if (pl.dim != 2 && pl.dim != 3) return fail(ADE_EINVAL, "dim must be 2 or 3 (got %d)", pl.dim);
    if (pl.real_bytes != 4 && pl.real_bytes != 8) return fail(ADE_EINVAL, "real_bytes must be 4 or 8");
    if (pl.kernel != ADE_WENDLAND_C2 && pl.kernel != ADE_WENDLAND_C4)
        return fail(ADE_EINVAL, "kernel must be ADE_WENDLAND_C2 or ADE_WENDLAND_C4");
    if (pl.integrator != ADE_EULER && pl.integrator != ADE_PC)
        return fail(ADE_EINVAL, "integrator must be ADE_EULER or ADE_PC");
    pl.plumes.clear();
    pl.tiles.clear();
    pl.list_cap = pl.list_cap_pair = 0;
    pl.nbar_max = 0.0;
    uint64_t N = 0, cbase = 0;
    for (int p = 0; p < nplumes; ++p) {
        const ade_params& q = params[p];
        if (q.dim != pl.dim || q.real_bytes != pl.real_bytes || q.kernel != pl.kernel ||
            q.integrator != pl.integrator)
            return fail(ADE_EINVAL, "plume %d: dim, real_bytes, kernel and integrator must match plume 0", p);
        if (q.reserved != 0) return fail(ADE_EINVAL, "plume %d: reserved must be 0", p);
        if (((q.flags & ADE_VELOCITY_FIELD) != 0) != pl.general)
            return fail(ADE_EINVAL, "plume %d: ADE_VELOCITY_FIELD must match plume 0", p);
        if (q.flags & ~(uint32_t)(ADE_STRICT_DT | ADE_CHECK_FINITE | ADE_VELOCITY_FIELD))
            return fail(ADE_EINVAL, "plume %d: unknown flags", p);
        if (pl.general && !(q.dt > 0))
            return fail(ADE_EINVAL, "plume %d: a velocity field needs dt > 0", p);
        if (counts[p] <= 0) return fail(ADE_EINVAL, "plume %d: count must be positive", p);
        const double vals[] = {q.H, q.L, q.alpha_L, q.alpha_T, q.D_m, q.v[0], q.v[1], q.v[2], q.dt, q.rho0, q.mass};
        for (double v : vals)
            if (!std::isfinite(v)) return fail(ADE_EINVAL, "plume %d: non-finite parameter", p);
        if (!(q.L > 0) || !(q.H > 0)) return fail(ADE_EINVAL, "plume %d: H and L must be positive", p);
        if (q.H * 3.0 > q.L) return fail(ADE_EINVAL, "plume %d: support H must be at most L/3", p);
        if (q.alpha_L < 0 || q.alpha_T < 0 || q.D_m < 0)
            return fail(ADE_EINVAL, "plume %d: dispersivities and D_m must be >= 0", p);
        if (!(q.rho0 > 0) || !(q.mass > 0)) return fail(ADE_EINVAL, "plume %d: rho0 and mass must be positive", p);
        if (q.cell_rows < 0 || q.cell_rows > 4 || q.cell_xsub < 0 || q.cell_xsub > 32)
            return fail(ADE_EINVAL, "plume %d: cell_rows in 0..4, cell_xsub in 0..32", p);

        PlumeDev d;
        std::memset(&d, 0, sizeof d);
        d.poff = (uint32_t)N;
        d.n = (uint32_t)counts[p];
        N += (uint64_t)counts[p];
        if (N > 0x0fffff00ull) return fail(ADE_EINVAL, "at most 2^28 - 256 particles per context");

        // cell grid in grid units: rows of height >= Hc / rows_per_H, x cells of width >= Hc / xsub
        const double Hu = q.H / q.L * kTwo32;
        const double Hc = Hu * (1.0 + 1.0 / 65536.0) + 2.0;
        // expected neighbours per particle (support volume over particle volume)
        const double nbar = (double)counts[p] *
                            (pl.dim == 2 ? kPi * q.H * q.H : 4.0 / 3.0 * kPi * q.H * q.H * q.H) /
                            std::pow(q.L, pl.dim);
        // rows of H/2, or H/4 for thousands of neighbours per particle, where
        // the tighter row windows (fewer candidates per neighbour) outweigh
        // the row work (measured: -6% and -8.5% on the 10^6 and 4x10^6
        // paper-scale problems)
        const int rsub = q.cell_rows ? q.cell_rows : (nbar > 2000.0 ? 4 : 2);
        // a plume of many neighbours does enough pair work per cell that
        // narrower x cells (fewer candidates per neighbour) outweigh the
        // extra cells when the tables fit.  2D: H/12 from 80 expected
        // neighbours (measured on the sweep: its h/dp = 3 plumes, 111
        // neighbours, take the pair kernel from 115 to 108.6 us; at 46
        // neighbours H/12 is slower).  3D: H/28 from 200 (the 128^3 plume, 256
        // neighbours: 1.00 -> 0.99 ms per graph-replayed step, 2% off the pair
        // kernel; 137 neighbours even at best, 74 slower), H/16 below.
        int xsub = q.cell_xsub;
        if (!xsub) {
            xsub = auto_xsub;
            if (pl.dim == 2 && auto_xsub == 8 && nbar >= 80.0) xsub = 12;
            if (pl.dim == 3 && auto_xsub == 28 && nbar < 200.0) xsub = 16;
        }
        const double cap = std::max(8.0 * (double)counts[p], 4096.0);
        double nr = std::floor(kTwo32 * rsub / Hc);
        double nfx = std::floor(kTwo32 * xsub / Hc);
        while (std::pow(nr, pl.dim - 1) * nfx > cap && (nr > 3 || nfx > 3)) {
            if (nfx > 3 && nfx >= nr) nfx = std::max(3.0, std::floor(nfx / 2));
            else nr = std::max(3.0, std::floor(nr / 2));
        }
        if (nr < 3 || nfx < 3) return fail(ADE_EINVAL, "plume %d: box holds fewer than 3 cells", p);
        int R = (int)std::ceil(Hc * nr / kTwo32);
        if (2 * R + 1 > nr) return fail(ADE_EINVAL, "plume %d: cell rows overlap (H too large)", p);
        // A support radius holding thousands of particles leaves these cells
        // with hundreds each, far past their buckets.  Then (2D) the x cells
        // are narrowed and every row is split into sub-rows, to near-square
        // cells of about two particles, so that a lattice puts one or two of
        // its rows and columns in a cell.  Candidate windows still take whole
        // x cells, so the candidates of a row stay one contiguous range.
        double nsub = 1.0;
        if (pl.dim == 2 && (double)counts[p] / (nr * nfx) > 4.0) {
            const double side = std::sqrt(2.0 / (double)counts[p]);  // of a two-particle cell, in box units
            nfx = std::max(nfx, std::floor(1.0 / side));
            nsub = std::max(1.0, std::floor(1.0 / nr / side));
        }
        // the kernels index x cells, sub-rows and rows with 24-bit multiplies
        if (nfx >= 16777216.0 || nsub >= 16777216.0 || nr >= 16777216.0)
            return fail(ADE_EINVAL, "plume %d: more than 2^24 cells along an axis", p);
        if (nfx * nsub >= 16777216.0 || std::pow(nr, pl.dim - 1) >= 16777216.0)
            return fail(ADE_EINVAL, "plume %d: more than 2^24 cells in a row or rows in the plume", p);
        d.nr = (uint32_t)nr;
        d.nfx = (uint32_t)nfx;
        d.nsub = (uint32_t)nsub;
        d.R = R;
        d.hx = (uint32_t)std::ceil(Hc) + 1u;
        d.ncell = (uint32_t)(std::pow(nr, pl.dim - 1) * nfx * nsub);
        d.cbase = (uint32_t)cbase;
        cbase += d.ncell;
        // cell tables are addressed with 32-bit byte offsets
        if (cell_pad(cbase) >= (1ull << 30)) return fail(ADE_EINVAL, "too many cells (at most 2^30 per context)");
        d.Hu = Hu;
        d.H2d = Hu * Hu;
        d.H2f = (float)d.H2d;
        d.invHu = 1.0 / Hu;
        d.Hc2f = (float)(Hc * Hc);
        d.rowh2f = (float)((kTwo32 / nr) * (kTwo32 / nr));
        // candidate windows are cut in x cells in float arithmetic: positions
        // in cells carry a rounding of up to ~nfx 2^-23 cells, covered by the slack
        d.cellx = (float)(nfx / kTwo32);
        d.cslack = (float)(1.0 / 128.0 + nfx * std::ldexp(1.0, -20));

        double D[9];
        const double trD = trace_D(pl.dim, q.alpha_L, q.alpha_T, q.D_m, q.v, D);
        const double gamma = pl.dim + 2.0;
        double s2 = 0.0;
        for (int c = 0; c < pl.dim; ++c) s2 += q.v[c] * q.v[c];
        const double sp = std::sqrt(s2);
        // Gamma x^T D x / r^2 - tr D for the tensor of Eq. (3) split into its
        // isotropic part and the part along the flow direction e
        d.a0 = (gamma - pl.dim) * (q.alpha_T * sp + q.D_m) - (q.alpha_L - q.alpha_T) * sp;
        d.a1 = gamma * (q.alpha_L - q.alpha_T) * sp;
        for (int c = 0; c < 3; ++c) d.ehat[c] = (sp > 0) ? ((c < pl.dim) ? q.v[c] / sp : 0.0) : (c == 0 ? 1.0 : 0.0);
        {
            // the bracket a0 + a1 (e.n)^2 as A0 + S (E.n)^2, S = +-1, with
            // E = sqrt|a1| e; in 2D a negative a1 is turned into S = +1 by
            // (e.n)^2 + (e_perp.n)^2 = 1: A0 = a0 + a1, E = sqrt(-a1) e_perp
            const double sa = std::sqrt(std::fabs(d.a1));
            double A0 = d.a0, S = 1.0, E[3] = {sa * d.ehat[0], sa * d.ehat[1], sa * d.ehat[2]};
            if (d.a1 < 0) {
                if (pl.dim == 2) {
                    A0 = d.a0 + d.a1;
                    E[0] = -sa * d.ehat[1];
                    E[1] = sa * d.ehat[0];
                } else {
                    S = -1.0;
                }
            }
            if (pl.dim == 2) E[2] = 0.0;
            const double t[8] = {Hu * Hu, 1.0 / Hu, 5.0 / Hu, A0, S, E[0], E[1], E[2]};
            for (int k = 0; k < 8; ++k) {
                d.dterm[k] = t[k];
                d.fterm[k] = (float)t[k];
            }
        }
        d.trD = trD;
        const double V = q.mass / q.rho0;
        d.vphi = V * kernel_phi_prefactor(pl.kernel, pl.dim, q.H);
        double dt = q.dt;
        const double hs = 0.5 * q.H;
        if (dt <= 0) {
            if (!(trD > 0)) return fail(ADE_EINVAL, "plume %d: Eq. (10) needs tr D > 0", p);
            dt = 0.1 * hs * hs / trD;
        } else if ((q.flags & ADE_STRICT_DT) && trD > 0 && dt > 10.0 * 0.1 * hs * hs / trD) {
            return fail(ADE_EUNSTABLE, "plume %d: dt %g exceeds 10x the Eq. (10) bound %g", p, dt,
                        0.1 * hs * hs / trD);
        }
        d.dt = dt;
        for (int c = 0; c < 3; ++c) {
            d.ushift[c] = (c < pl.dim) ? dt * q.v[c] / q.L * kTwo32 : 0.0;
            d.vel[c] = (c < pl.dim) ? q.v[c] : 0.0;
        }
        d.mass = q.mass;
        d.L = q.L;
        d.aL = q.alpha_L;
        d.aT = q.alpha_T;
        d.Dm = q.D_m;
        d.tfirst = (uint32_t)pl.tiles.size();
        for (uint32_t s = 0; s < d.n; s += kTile) {
            TileDev t;
            t.plume = (uint32_t)p;
            t.start = d.poff + s;
            t.end = d.poff + std::min<uint32_t>(d.n, s + kTile);
            t.pad = 0;
            pl.tiles.push_back(t);
        }
        d.tcount = (uint32_t)pl.tiles.size() - d.tfirst;
        const int span = 2 * R + 1;
        pl.list_cap = std::max(pl.list_cap, list_cap_for(pl.dim, span));
        pl.list_cap_pair = std::max(pl.list_cap_pair, list_cap_pair_for(pl.dim, span));
        pl.plumes.push_back(d);
    }
    pl.N = (int64_t)N;
    pl.ncell = cbase;
    pl.ntiles = (uint32_t)pl.tiles.size();
    // The pair kernel takes the plumes in decreasing order of their expected
    // neighbours per particle (support volume over particle volume), so that
    // the cheapest work items come last and fill the end of the launch.
    {
        std::vector<std::pair<double, int>> cost;
        for (int p = 0; p < nplumes; ++p) {
            const ade_params& q = params[p];
            const double vol = (pl.dim == 2) ? kPi * q.H * q.H : 4.0 / 3.0 * kPi * q.H * q.H * q.H;
            cost.emplace_back(-(double)counts[p] * vol / std::pow(q.L, pl.dim), p);
            pl.nbar_max = std::max(pl.nbar_max, -cost.back().first);
        }
        std::stable_sort(cost.begin(), cost.end());
        pl.pair_tiles.clear();
        for (const auto& c : cost) {
            const PlumeDev& d = pl.plumes[c.second];
            pl.pair_tiles.insert(pl.pair_tiles.end(), pl.tiles.begin() + d.tfirst,
                                 pl.tiles.begin() + d.tfirst + d.tcount);
        }
    }
    pl.nscan = (uint32_t)std::max<uint64_t>(cell_pad(pl.ncell) / kCellChunk,
                                            ((uint64_t)N + 1 + kScanChunk - 1) / kScanChunk);
    return ADE_OK;
}

// Default x cells per support radius: 8 in 2D, 16 in 3D, where the pencil
// windows gain more from the narrower cells (the 128^3 plume: 1.19 ms per
// step against 1.22 at H/8), and narrower still for plumes of many
// neighbours (plan_grid).  A context's cell tables (count, start and an
// 8-id bucket: 40 bytes per cell) are read and written by every build pass.
// Past the chip's 256 MB last-level cache (the Infinity Cache) they go to
// HBM on every pass, so the default x cells of a context whose tables would
// exceed kCellTableBudget are coarsened step by step until they fit; a
// plume's explicit cell_xsub is kept.  Measured on the 256-plume 2D
// ensemble (5.4M particles, 9.6M cells at H/8): 465 us per step at H/8, 376
// at H/4, 355 at H/3, 480 at H/2; plumes whose tables fit run best at H/8.
constexpr double kCellTableBudget = 160.0 * 1048576.0;

int plan_build(const ade_params* params, const int64_t* counts, int32_t nplumes, Plan& pl) {
    // 3D: H/28 for plumes of 200 or more expected neighbours and H/16 for
    // the rest, then all at H/16, H/12, ... while the tables do not fit
    static const int k2d[] = {8, 6, 4, 3}, k3d[] = {28, 16, 12, 8, 6, 4, 3};
    const bool three = params && nplumes > 0 && params[0].dim == 3;
    const int* xs = three ? k3d : k2d;
    const int nxs = three ? 7 : 4;
    int rc = plan_grid(params, counts, nplumes, pl, xs[0]);
    bool any_auto = false;
    for (int p = 0; !rc && p < nplumes; ++p) any_auto = any_auto || params[p].cell_xsub == 0;
    for (int k = 1; k < nxs; ++k) {
        if (rc || !any_auto || (double)pl.ncell * (8.0 + 4.0 * kBucket) <= kCellTableBudget) break;
        rc = plan_grid(params, counts, nplumes, pl, xs[k]);
    }
    return rc;
}

}  // namespace

namespace {

void layout(Bump& b, ade_ctx* c, const Plan& pl) {
    const size_t N = (size_t)pl.N;
    const size_t rb = (size_t)pl.real_bytes;
    c->plumes = b.take<PlumeDev>(pl.P);
    c->tiles = b.take<TileDev>(pl.ntiles);
    c->pair_tiles = b.take<TileDev>(pl.ntiles);
    StateArrays* bufs[2] = {&c->S, &c->U};
    for (int k = 0; k < 2; ++k) {
        StateArrays& s = *bufs[k];
        for (int d = 0; d < 3; ++d) s.pos[d] = (d < pl.dim) ? b.take<uint32_t>(N) : nullptr;
        s.rec = (k == 0 && !(pl.dim == 3 && pl.real_bytes == 8)) ? b.take<uint4>(N) : nullptr;
        s.C = b.take_bytes(N * rb);
        s.id = b.take<uint32_t>(N);
        s.key = (k == 1) ? b.take<uint32_t>(N) : nullptr;
        for (int d = 0; d < 3; ++d) s.vel[d] = (pl.general && d < pl.dim) ? b.take_bytes(N * rb) : nullptr;
        for (int d = 0; d < 6; ++d) s.rD[d] = (pl.general && d < (pl.dim == 2 ? 3 : 6)) ? b.take_bytes(N * rb) : nullptr;
        s.grec = (k == 0 && pl.general && pl.dim == 2 && pl.real_bytes == 4) ? b.take<uint4>(2 * N) : nullptr;
        s.Cb = (pl.general && pl.integrator == ADE_PC) ? b.take_bytes(N * rb) : nullptr;
    }
    if (pl.dim == 2) {  // never read in 2D, but keep the pointers valid
        c->S.pos[2] = c->S.pos[0];
        c->U.pos[2] = c->U.pos[0];
    }
    c->count = b.take<uint32_t>(cell_pad(pl.ncell));
    c->lists.count = c->count;
    c->lists.bucket = b.take<uint32_t>(cell_pad(pl.ncell) * kBucket);
    c->lists.ovf = b.take<uint2>(N);
    c->lists.ovf_count = b.take<uint32_t>(2);
    c->cell_start = b.take<uint32_t>(cell_pad(pl.ncell));
    c->scan_partial = b.take_bytes((size_t)pl.nscan * 8);
    c->aux = b.take_bytes(N * rb);
    c->aux_rec = (pl.dim == 3 && pl.real_bytes == 8) ? nullptr : b.take<uint4>(N);
    c->mass_partial = b.take<double>(pl.ntiles);
    c->range_partial = b.take<double>(2 * (size_t)pl.ntiles);
    c->step = b.take<int64_t>(1);
    c->nonfinite = b.take<uint32_t>(1);
}

// smallest and largest C of a tile, then of each plume (FP64; NaNs are
// skipped by fmin / fmax)
__device__ __forceinline__ void block_minmax(double& lo, double& hi, double* lds) {
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64, nw = blockDim.x / 64;
    if (lane == 0) {
        lds[2 * w] = lo;
        lds[2 * w + 1] = hi;
    }
    __syncthreads();
    for (int k = 0; k < nw; ++k) {
        lo = fmin(lo, lds[2 * k]);
        hi = fmax(hi, lds[2 * k + 1]);
    }
}

template <typename real>
__global__ __launch_bounds__(kTile) void k_range_tiles(const TileDev* __restrict__ tiles, const real* __restrict__ C,
                                                      double* __restrict__ partial) {
    __shared__ double lds[2 * kTile / 64];
    const TileDev t = tiles[blockIdx.x];
    const uint32_t i = t.start + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (i < t.end) lo = hi = (double)C[i];
    block_minmax(lo, hi, lds);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = lo;
        partial[2 * blockIdx.x + 1] = hi;
    }
}

__global__ __launch_bounds__(256) void k_range_plumes(const PlumeDev* __restrict__ plumes,
                                                     const double* __restrict__ partial, double* __restrict__ out) {
    __shared__ double lds[2 * 256 / 64];
    const PlumeDev& P = plumes[blockIdx.x];
    double lo = INFINITY, hi = -INFINITY;
    for (uint32_t k = threadIdx.x; k < P.tcount; k += blockDim.x) {
        lo = fmin(lo, partial[2 * (P.tfirst + k)]);
        hi = fmax(hi, partial[2 * (P.tfirst + k) + 1]);
    }
    block_minmax(lo, hi, lds);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = lo;
        out[2 * blockIdx.x + 1] = hi;
    }
}

// finite check of the sorted concentrations: any NaN or infinity sets *flag
// (vector stores of the same value, order-free)
template <typename real>
__global__ __launch_bounds__(256) void k_check_finite(const real* __restrict__ C, uint32_t N,
                                                     uint32_t* __restrict__ flag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N && !isfinite(C[i])) *flag = 1u;
}

// Sum the recorded event pairs into the totals and recycle the events.
int flush_events(ade_ctx* c) {
    if (c->ev_used == 0) return ADE_OK;
    HIPCHK(hipEventSynchronize(c->events[c->ev_used - 1]));
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->events[k], c->events[k + 1]));
        c->timed_ms += ms;
        c->timed_launches += 1;
    }
    c->ev_used = 0;
    return ADE_OK;
}

}  // namespace

namespace ade {

// a pair of timing events from the context's pool into e0, e1; they are left
// as they are when timing is off (or a graph is being captured)
static int take_events(ade_ctx* c, hipEvent_t& e0, hipEvent_t& e1) {
    if (!c->timing || c->capturing) return ADE_OK;
    if (c->ev_used + 2 > c->events.size()) {
        if (c->events.size() < 4096) {
            size_t old = c->events.size();
            c->events.resize(old + 512);
            for (size_t k = old; k < c->events.size(); ++k) HIPCHK(hipEventCreate(&c->events[k]));
        } else {
            int rc = flush_events(c);
            if (rc) return rc;
        }
    }
    e0 = c->events[c->ev_used++];
    e1 = c->events[c->ev_used++];
    return ADE_OK;
}

// launch a pair kernel; when timing is on, events stamped with the kernel's
// own start and end times are attached to the launch
int run_pair(ade_ctx* c, int mode, const PairLaunch& a) {
    const Plan& pl = c->plan;
    PairLaunch b = a;
    b.ev0 = b.ev1 = nullptr;
    int rc = take_events(c, b.ev0, b.ev1);
    if (rc) return rc;
    HIPCHK(launch_pair(pl.dim, pl.real_bytes, pl.kernel, mode, b, c->tuning.block, c->stream));
    return ADE_OK;
}

// the same for the velocity-field pair kernel
int run_gen(ade_ctx* c, int mode, void* out) {
    const Plan& pl = c->plan;
    GenLaunch g = gen_args(c, out);
    int rc = take_events(c, g.ev0, g.ev1);
    if (rc) return rc;
    HIPCHK(launch_pair_gen(pl.dim, pl.real_bytes, pl.kernel, mode, g, c->stream));
    return ADE_OK;
}

PairLaunch pair_args(ade_ctx* c, int mode, const void* Cpair, const void* Cbase, double scale, void* out) {
    PairLaunch a;
    std::memset(&a, 0, sizeof a);
    a.plumes = c->plumes;
    a.tiles = c->pair_tiles;
    a.ntiles = c->plan.ntiles;
    a.block = c->tuning.block;
    a.lanes = c->tuning.lanes;
    a.targets = targets_of(c->tuning);
    a.list_cap = tuning_list_cap(c->plan, c->tuning);
    a.persistent = c->tuning.persistent;
    a.xcd_group = c->tuning.xcd_group > 0 ? (uint32_t)c->tuning.xcd_group : 32u;
    a.zc = c->coincident ? 1 : 0;
    // candidate records carrying the concentrations the pair sum reads
    a.rec = (Cpair == c->aux) ? c->aux_rec : c->S.rec;
    a.out_rec = c->aux_rec;
    for (int d = 0; d < 3; ++d) {
        a.spos[d] = c->S.pos[d];
        a.upos[d] = c->U.pos[d];
    }
    a.sid = c->S.id;
    a.Cpair = Cpair;
    a.Cbase = Cbase;
    a.cell_start = c->cell_start;
    a.uC = c->U.C;
    a.uid = c->U.id;
    a.ukey = c->U.key;
    a.lists = c->lists;
    a.step = c->step;
    a.scale = scale;
    a.out = out;
    (void)mode;
    return a;
}

// counting sort of the hashed U buffer into S (cell order) and cell_start
int enqueue_build(ade_ctx* c, int inc_step) {
    const Plan& pl = c->plan;
    HIPCHK(launch_scan(c->lists, c->cell_start, (uint32_t*)c->scan_partial, (uint32_t)pl.ncell, c->stream));
    HIPCHK(launch_place(pl.dim, pl.real_bytes, c->U, c->S, c->lists, c->cell_start, (uint32_t)pl.N, c->step,
                        inc_step, c->stream));
    return ADE_OK;
}

GenLaunch gen_args(ade_ctx* c, void* out) {
    GenLaunch g;
    std::memset(&g, 0, sizeof g);
    g.plumes = c->plumes;
    g.tiles = c->pair_tiles;
    g.ntiles = c->plan.ntiles;
    g.list_cap = tuning_list_cap(c->plan, c->tuning);
    g.lanes = c->tuning.lanes;
    g.targets = targets_of(c->tuning);
    g.block = c->tuning.block;
    g.S = c->S;
    g.U = c->U;
    g.cell_start = c->cell_start;
    g.lists = c->lists;
    g.step = c->step;
    g.out = out;
    return g;
}

int enqueue_step(ade_ctx* c) {
    const Plan& pl = c->plan;
    int rc;
    if (pl.general && pl.integrator == ADE_PC) {
        // velocity field, predictor-corrector: the corrector's positions
        // x^(1/2) have their own relative geometry, so they get a cell build
        if ((rc = run_gen(c, kModeHalf, nullptr))) return rc;
        if ((rc = enqueue_build(c, 0))) return rc;
        if ((rc = run_gen(c, kModeFull, nullptr))) return rc;
    } else if (pl.general) {  // velocity field: explicit Euler
        if ((rc = run_gen(c, kModeStep, nullptr))) return rc;
    } else if (pl.integrator == ADE_PC) {
        PairLaunch h = pair_args(c, kModeHalf, c->S.C, c->S.C, 0.5, c->aux);
        if ((rc = run_pair(c, kModeHalf, h))) return rc;
        PairLaunch f = pair_args(c, kModeStep, c->aux, c->S.C, 1.0, nullptr);
        if ((rc = run_pair(c, kModeStep, f))) return rc;
    } else {
        PairLaunch f = pair_args(c, kModeStep, c->S.C, c->S.C, 1.0, nullptr);
        if ((rc = run_pair(c, kModeStep, f))) return rc;
    }
    return enqueue_build(c, 1);
}

}  // namespace ade

namespace {

void drop_events(ade_ctx* c) {
    for (hipEvent_t e : c->events) hipEventDestroy(e);
    c->events.clear();
    c->ev_used = 0;
}

void drop_graph(ade_ctx* c) {
    if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

}  // namespace

extern "C" {

int ade_workspace_bytes(const ade_params* params, const int64_t* counts, int32_t nplumes, size_t* bytes) {
    if (!bytes) return fail(ADE_EINVAL, "null bytes");
    Plan pl;
    int rc = plan_build(params, counts, nplumes, pl);
    if (rc) return rc;
    Bump b(nullptr);
    ade_ctx tmp;
    layout(b, &tmp, pl);
    *bytes = b.off + 256;
    return ADE_OK;
}

int ade_create(const ade_params* params, const int64_t* counts, int32_t nplumes, void* d_ws,
               size_t ws_bytes, void* stream, ade_ctx** out) {
    if (!out) return fail(ADE_EINVAL, "null out");
    *out = nullptr;
    if (!d_ws) return fail(ADE_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(d_ws) & 255u) return fail(ADE_EINVAL, "workspace must be 256-byte aligned");
    ade_ctx* c = new (std::nothrow) ade_ctx();
    if (!c) return fail(ADE_EINVAL, "out of host memory");
    int rc = plan_build(params, counts, nplumes, c->plan);
    if (rc) {
        delete c;
        return rc;
    }
    // the velocity-field kernel's lists (one target per lane, at least 64 per workgroup)
    if (c->plan.general && (size_t)64 * (size_t)c->plan.list_cap * 8u > kPairLdsMax) {
        delete c;
        return fail(ADE_EINVAL, "too many neighbour rows: the candidate lists do not fit in LDS");
    }
    // its 32-byte candidate records (2D FP32) are addressed with 32-bit byte offsets
    if (c->plan.general && c->plan.dim == 2 && c->plan.real_bytes == 4 && c->plan.N > 0x07ffff00) {
        delete c;
        return fail(ADE_EINVAL, "a 2D FP32 velocity-field context holds at most 2^27 - 256 particles");
    }
    // default launch shape: the fewest lanes per particle that still give
    // the chip about 4 wavefronts per SIMD (4096 wavefronts of 64 lanes, i.e.
    // 2^18 lanes): two targets per lane from 2^19 particles on (the fastest
    // shape on the 2D sweep), one lane per target from 2^18, two lanes from
    // 2^17, else four; then the next shapes whose candidate lists fit in LDS.
    // Plumes of thousands of neighbours per particle, and 3D plumes, take
    // four lanes per target, or in FP32 four lanes per two neighbouring
    // targets: the targets of a wavefront then walk nearly the same candidate
    // ranges and share their cache lines, and a pair of targets shares every
    // record it fetches (the autotuner's choice on the 10^6-particle,
    // 31k-neighbour problem: 19.3 ms per pair launch against 22.8 ms for one
    // target a quad; on the 128^3 plume 0.88-0.90 ms against 0.90-0.92).
    {
        const int64_t N = c->plan.N;
        const bool quads = c->plan.nbar_max > 2000.0 || c->plan.dim == 3;
        const int qtargets = c->plan.real_bytes == 4 ? 2 : 1;
        const ade_tuning first = quads ? ade_tuning{c->plan.dim == 3 ? 64 : 128, 4, 128, 0, qtargets}
                                 : N >= (1 << 19) ? ade_tuning{64, 1, 0, 0, 2}
                                 : N >= (1 << 18) ? ade_tuning{256, 1, 0, 0, 1}
                                 : N >= (1 << 17) ? ade_tuning{256, 2, 0, 0, 1}
                                                  : ade_tuning{256, 4, 0, 0, 1};
        const ade_tuning defaults[6] = {first, {256, 2, 0, 0, 1}, {256, 4, 0, 0, 1}, {128, 4, 0, 0, 1},
                                        {64, 4, 0, 0, 1}, {64, 1, 0, 0, 2}};
        bool ok = false;
        for (const ade_tuning& t : defaults)
            if (!ok && tuning_fits(c->plan, t)) {
                c->tuning = t;
                ok = true;
            }
        if (!ok) {
            delete c;
            return fail(ADE_EINVAL, "too many neighbour rows: the candidate lists do not fit in LDS");
        }
        // a velocity field: four lanes per target in the largest workgroup
        // whose lists fit, or in 2D FP32 for plumes of thousands of
        // neighbours four lanes per two targets, block 128 (10^6 particles,
        // 31k neighbours: 44 against 64 ms per update launch; on the 512^2
        // plumes of 46 and 111 neighbours the same as, or 3% slower than,
        // one target a quad).  Its autotuner may choose otherwise.
        if (c->plan.general) {
            for (int bb : {64, 128, 256})
                if (gen_tuning_fits(c->plan, ade_tuning{bb, 4, 0, 0, 1})) c->tuning = ade_tuning{bb, 4, 0, 0, 1};
            const ade_tuning q{128, 4, 0, 0, 2};
            if (c->plan.nbar_max > 2000.0 && gen_tuning_fits(c->plan, q)) c->tuning = q;
        }
    }
    Bump b(d_ws);
    layout(b, c, c->plan);
    if (b.off + 256 > ws_bytes) {
        delete c;
        return fail(ADE_EWORKSPACE, "workspace too small: need %zu bytes", b.off + 256);
    }
    c->stream = static_cast<hipStream_t>(stream);
    const Plan& pl = c->plan;
    c->h_total = (uint32_t)pl.N;
    auto cleanup = [&](int code) {
        delete c;
        return code;
    };
    if (hipMemcpyAsync(c->plumes, pl.plumes.data(), sizeof(PlumeDev) * pl.P, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->tiles, pl.tiles.data(), sizeof(TileDev) * pl.ntiles, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->pair_tiles, pl.pair_tiles.data(), sizeof(TileDev) * pl.ntiles, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->cell_start + pl.ncell, &c->h_total, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemsetAsync(c->count, 0, sizeof(uint32_t) * cell_pad(pl.ncell), c->stream) != hipSuccess ||
        hipMemsetAsync(c->step, 0, sizeof(int64_t), c->stream) != hipSuccess ||
        hipMemsetAsync(c->lists.ovf_count, 0, 2 * sizeof(uint32_t), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return cleanup(fail(ADE_EHIP, "uploading the plume tables failed"));
    *out = c;
    return ADE_OK;
}

int ade_init_particles(ade_ctx* c, const double* d_x, const void* d_C) {
    if (!c || !d_x || !d_C) return fail(ADE_EINVAL, "null argument");
    const Plan& pl = c->plan;
    HIPCHK(hipMemsetAsync(c->count, 0, sizeof(uint32_t) * cell_pad(pl.ncell), c->stream));
    HIPCHK(hipMemsetAsync(c->lists.ovf_count, 0, 2 * sizeof(uint32_t), c->stream));
    HIPCHK(hipMemsetAsync(c->step, 0, sizeof(int64_t), c->stream));
    HIPCHK(launch_init(pl.dim, pl.real_bytes, c->plumes, c->tiles, pl.ntiles, d_x, d_C, (uint32_t)pl.N,
                       c->U, c->lists, c->stream));
    c->initialized = true;
    c->built = false;
    c->vel_set = false;
    if (!c->coincident) drop_graph(c);
    c->coincident = true;  // until the cell build checks the new positions
    return ADE_OK;
}

int ade_set_velocities(ade_ctx* c, const double* d_v) {
    if (!c || !d_v) return fail(ADE_EINVAL, "null argument");
    const Plan& pl = c->plan;
    if (!pl.general) return fail(ADE_EINVAL, "context created without ADE_VELOCITY_FIELD");
    if (!c->initialized || c->built)
        return fail(ADE_ESTATE, "ade_set_velocities belongs between ade_init_particles and ade_build_cells");
    HIPCHK(launch_setvel(pl.dim, pl.real_bytes, c->plumes, c->tiles, pl.ntiles, d_v, (uint32_t)pl.N, c->U,
                         c->stream));
    c->vel_set = true;
    return ADE_OK;
}

// Whether two particles of a plume share a position, from the built cells
// (synchronises the stream).  With a uniform flow every particle of a plume
// moves by the same displacement, so the answer holds for the whole run; a
// velocity-field context keeps its own kernels and is not checked.
static int check_coincident(ade_ctx* c) {
    const Plan& pl = c->plan;
    bool found = true;
    if (!pl.general) {
        uint32_t h = 0;
        HIPCHK(hipMemsetAsync(c->nonfinite, 0, sizeof(uint32_t), c->stream));
        HIPCHK(launch_coincident(pl.dim, c->plumes, c->tiles, pl.ntiles, c->S, c->cell_start, c->nonfinite,
                                 c->stream));
        HIPCHK(hipMemcpyAsync(&h, c->nonfinite, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        found = h != 0;
    }
    if (found != c->coincident) drop_graph(c);  // a captured step holds the other kernels
    c->coincident = found;
    return ADE_OK;
}

int ade_build_cells(ade_ctx* c) {
    if (!c) return fail(ADE_EINVAL, "null ctx");
    if (!c->initialized) return fail(ADE_ESTATE, "ade_build_cells before ade_init_particles");
    if (c->plan.general && !c->vel_set && !c->built)
        return fail(ADE_ESTATE, "ade_build_cells before ade_set_velocities (ADE_VELOCITY_FIELD)");
    if (c->built) return ADE_OK;  // every step already leaves the cells built
    int rc = enqueue_build(c, 0);
    if (rc) return rc;
    c->built = true;
    return check_coincident(c);
}

int ade_coincident(const ade_ctx* c, int32_t* out) {
    if (!c || !out) return fail(ADE_EINVAL, "null argument");
    *out = c->coincident ? 1 : 0;
    return ADE_OK;
}

// ADE_CHECK_FINITE: after a call's steps, every concentration must be finite
// (synchronises the stream)
static int check_finite(ade_ctx* c) {
    const Plan& pl = c->plan;
    if (!pl.check_finite) return ADE_OK;
    uint32_t h = 0;
    HIPCHK(hipMemsetAsync(c->nonfinite, 0, sizeof(uint32_t), c->stream));
    const uint32_t N = (uint32_t)pl.N;
    if (pl.real_bytes == 4)
        hipLaunchKernelGGL((k_check_finite<float>), dim3((N + 255) / 256), dim3(256), 0, c->stream,
                           (const float*)c->S.C, N, c->nonfinite);
    else
        hipLaunchKernelGGL((k_check_finite<double>), dim3((N + 255) / 256), dim3(256), 0, c->stream,
                           (const double*)c->S.C, N, c->nonfinite);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&h, c->nonfinite, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (h) return fail(ADE_ENONFINITE, "a concentration is not finite after the step (ADE_CHECK_FINITE)");
    return ADE_OK;
}

int ade_step(ade_ctx* c, int64_t nsteps) {
    if (!c) return fail(ADE_EINVAL, "null ctx");
    if (nsteps < 0) return fail(ADE_EINVAL, "nsteps must be >= 0");
    if (!c->built) return fail(ADE_ESTATE, "ade_step before ade_build_cells");
    for (int64_t s = 0; s < nsteps; ++s) {
        int rc = enqueue_step(c);
        if (rc) return rc;
    }
    return nsteps > 0 ? check_finite(c) : ADE_OK;
}

int ade_step_graph(ade_ctx* c, int64_t nsteps) {
    if (!c) return fail(ADE_EINVAL, "null ctx");
    if (nsteps < 0) return fail(ADE_EINVAL, "nsteps must be >= 0");
    if (!c->built) return fail(ADE_ESTATE, "ade_step_graph before ade_build_cells");
    if (!c->stream) return fail(ADE_EINVAL, "graph capture needs a non-default stream");
    if (!c->graph_exec) {
        HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        c->capturing = true;
        int rc = enqueue_step(c);
        c->capturing = false;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(ADE_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        c->graph = g;
        e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(c);
            return fail(ADE_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    for (int64_t s = 0; s < nsteps; ++s) HIPCHK(hipGraphLaunch(c->graph_exec, c->stream));
    return nsteps > 0 ? check_finite(c) : ADE_OK;
}

int ade_rhs(ade_ctx* c, void* d_rhs) {
    if (!c || !d_rhs) return fail(ADE_EINVAL, "null argument");
    if (!c->built) return fail(ADE_ESTATE, "ade_rhs before ade_build_cells");
    const Plan& pl = c->plan;
    if (pl.general) return run_gen(c, kModeRhs, d_rhs);
    PairLaunch a = pair_args(c, kModeRhs, c->S.C, c->S.C, 1.0, d_rhs);
    return run_pair(c, kModeRhs, a);
}

int ade_read_C(const ade_ctx* c, void* d_C_out) {
    if (!c || !d_C_out) return fail(ADE_EINVAL, "null argument");
    if (!c->built) return fail(ADE_ESTATE, "ade_read_C before ade_build_cells");
    HIPCHK(launch_read_C(c->plan.real_bytes, c->S, (uint32_t)c->plan.N, d_C_out, c->stream));
    return ADE_OK;
}

int ade_read_x(const ade_ctx* c, double* d_x_out) {
    if (!c || !d_x_out) return fail(ADE_EINVAL, "null argument");
    if (!c->built) return fail(ADE_ESTATE, "ade_read_x before ade_build_cells");
    HIPCHK(launch_read_x(c->plan.dim, c->plumes, c->tiles, c->plan.ntiles, c->S, (uint32_t)c->plan.N,
                         d_x_out, c->stream));
    return ADE_OK;
}

int ade_mass(const ade_ctx* c, double* d_out) {
    if (!c || !d_out) return fail(ADE_EINVAL, "null argument");
    if (!c->built) return fail(ADE_ESTATE, "ade_mass before ade_build_cells");
    HIPCHK(launch_mass(c->plan.real_bytes, c->plumes, c->plan.P, c->tiles, c->plan.ntiles, c->S,
                       c->mass_partial, d_out, c->stream));
    return ADE_OK;
}

int ade_conc_range(const ade_ctx* c, double* d_out) {
    if (!c || !d_out) return fail(ADE_EINVAL, "null argument");
    if (!c->built) return fail(ADE_ESTATE, "ade_conc_range before ade_build_cells");
    const Plan& pl = c->plan;
    if (pl.real_bytes == 4)
        hipLaunchKernelGGL((k_range_tiles<float>), dim3(pl.ntiles), dim3(kTile), 0, c->stream, c->tiles,
                           (const float*)c->S.C, c->range_partial);
    else
        hipLaunchKernelGGL((k_range_tiles<double>), dim3(pl.ntiles), dim3(kTile), 0, c->stream, c->tiles,
                           (const double*)c->S.C, c->range_partial);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_range_plumes, dim3(pl.P), dim3(256), 0, c->stream, c->plumes, c->range_partial, d_out);
    HIPCHK(hipGetLastError());
    return ADE_OK;
}

int ade_neighbours(ade_ctx* c, int64_t* d_offsets, int32_t* d_ids, int64_t cap, int64_t* h_needed) {
    if (!c || !d_offsets || !h_needed) return fail(ADE_EINVAL, "null argument");
    if (!c->built) return fail(ADE_ESTATE, "ade_neighbours before ade_build_cells");
    const Plan& pl = c->plan;
    HIPCHK(launch_nbr(pl.dim, pl.real_bytes, 0, c->plumes, c->tiles, pl.ntiles, c->S, c->cell_start,
                      d_offsets, nullptr, c->stream));
    HIPCHK(launch_scan64(d_offsets, (uint32_t)pl.N, (int64_t*)c->scan_partial, c->stream));
    int64_t total = 0;
    HIPCHK(hipMemcpyAsync(&total, d_offsets + pl.N, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *h_needed = total;
    if (d_ids && cap >= total)
        HIPCHK(launch_nbr(pl.dim, pl.real_bytes, 1, c->plumes, c->tiles, pl.ntiles, c->S, c->cell_start,
                          d_offsets, d_ids, c->stream));
    return ADE_OK;
}

int ade_kernel_timing(ade_ctx* c, int32_t mode, double* h_ms, int64_t* h_count) {
    if (!c) return fail(ADE_EINVAL, "null ctx");
    if (mode == 1) {
        int rc = flush_events(c);
        if (rc) return rc;
        c->timed_ms = 0.0;
        c->timed_launches = 0;
        c->timing = true;
        return ADE_OK;
    }
    if (mode != 0) return fail(ADE_EINVAL, "mode must be 0 or 1");
    int rc = flush_events(c);
    if (rc) return rc;
    c->timing = false;
    if (h_ms) *h_ms = c->timed_ms;
    if (h_count) *h_count = c->timed_launches;
    return ADE_OK;
}

// cell counts and overflow count of the next build back to zero (as every
// build leaves them)
static int clear_counts(ade_ctx* c) {
    HIPCHK(hipMemsetAsync(c->count, 0, sizeof(uint32_t) * cell_pad(c->plan.ncell), c->stream));
    HIPCHK(hipMemsetAsync(c->lists.ovf_count, 0, 2 * sizeof(uint32_t), c->stream));
    return ADE_OK;
}

// Times the candidate launch shapes of a tuner: `launch(k)` enqueues
// candidate k's step-mode kernel with the events around it (and clears the
// cell counts it leaves).  The clocks of the GPU rise only under sustained
// load and fall again within seconds of idling (a context timed back to back
// ran 10% faster from its second timing on; with 2 s idle between timings it
// never did), so the GPU is first kept busy for ~50 ms with the first
// candidate, and every round then times each candidate once (round 0
// untimed), so that a drift of the clocks weighs on all candidates alike.
static int time_candidates(ade_ctx* c, int ncand, int32_t reps, hipEvent_t e0, hipEvent_t e1,
                           const std::function<hipError_t(int)>& launch, int* best) {
    auto timed = [&](int k, float* ms) -> int {
        if (launch(k) != hipSuccess) return fail(ADE_EHIP, "autotune launch");
        int rc = clear_counts(c);
        if (rc) return rc;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return fail(ADE_EHIP, "event synchronise");
        return ADE_OK;
    };
    float one = 0.f;
    int rc = timed(0, &one);
    const int warm = std::min(4000, (int)std::ceil(50.0 / std::max(one, 0.01f)));
    for (int k = 0; !rc && k < warm; ++k) {
        if (launch(0) != hipSuccess) rc = fail(ADE_EHIP, "autotune launch");
        else rc = clear_counts(c);
    }
    std::vector<float> tot((size_t)ncand, 0.f);
    for (int r = 0; !rc && r <= reps; ++r)
        for (int k = 0; !rc && k < ncand; ++k) {
            rc = timed(k, &one);
            if (r > 0) tot[(size_t)k] += one;
        }
    if (rc) return rc;
    *best = (int)(std::min_element(tot.begin(), tot.end()) - tot.begin());
    return ADE_OK;
}

// The velocity-field kernel's autotuner: block x (lanes, targets), the step-mode kernel
// timed as ade_autotune times the uniform-flow one.
static int autotune_gen(ade_ctx* c, int32_t reps, int32_t flags, ade_tuning* best) {
    const Plan& pl = c->plan;
    const ade_tuning start = c->tuning;
    std::vector<ade_tuning> cands;
    const int shapes[4][2] = {{1, 1}, {2, 1}, {4, 1}, {4, 2}};  // lanes, targets
    for (const auto& sh : shapes) {
        if ((flags & ADE_TUNE_KEEP_LANES) && (sh[0] != start.lanes || sh[1] != targets_of(start))) continue;
        for (int bb : {64, 128, 256}) {
            const ade_tuning cand{bb, sh[0], 0, 0, sh[1]};
            if (gen_tuning_fits(pl, cand)) cands.push_back(cand);
        }
    }
    if (cands.empty()) return fail(ADE_EINVAL, "no launch shape fits");
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int kbest = 0;
    int rc = time_candidates(c, (int)cands.size(), reps, e0, e1,
                             [&](int k) {
                                 c->tuning = cands[(size_t)k];
                                 GenLaunch g = gen_args(c, nullptr);
                                 g.ev0 = e0;
                                 g.ev1 = e1;
                                 return launch_pair_gen(pl.dim, pl.real_bytes, pl.kernel, kModeStep, g, c->stream);
                             },
                             &kbest);
    const int rc_clear = clear_counts(c);
    if (!rc) rc = rc_clear;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->tuning = rc ? start : cands[(size_t)kbest];
    drop_graph(c);
    if (rc) return rc;
    if (best) *best = c->tuning;
    return ADE_OK;
}

int ade_autotune(ade_ctx* c, int32_t reps, int32_t flags, ade_tuning* best) {
    if (!c) return fail(ADE_EINVAL, "null ctx");
    if (reps < 1) return fail(ADE_EINVAL, "reps must be positive");
    if (!c->built) return fail(ADE_ESTATE, "ade_autotune before ade_build_cells");
    if (c->plan.general) return autotune_gen(c, reps, flags, best);
    const Plan& pl = c->plan;
    const ade_tuning start = c->tuning;
    const int blocks[3] = {64, 128, 256}, pers[2] = {0, 2048}, groups[3] = {8, 32, 128};
    // (lanes, targets): one lane per two targets, 1, 2, 4 lanes per target, or
    // four lanes per two targets (FP32; tuning_fits drops it for FP64)
    const int shapes[5][2] = {{1, 2}, {1, 1}, {2, 1}, {4, 1}, {4, 2}};
    std::vector<ade_tuning> cands;
    for (const auto& sh : shapes) {
        const int lb = sh[0], tg = sh[1];
        if ((flags & ADE_TUNE_KEEP_LANES) && (lb != start.lanes || tg != targets_of(start))) continue;
        for (int bb : blocks)
            for (int xg : groups)
                for (int pp : pers) {
                    const ade_tuning cand{bb, lb, xg, pp, tg};
                    if (tuning_fits(pl, cand)) cands.push_back(cand);
                }
    }
    if (cands.empty()) return fail(ADE_EINVAL, "no launch shape fits");
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int kbest = 0;
    // the step-mode kernel, as a step runs it; its outputs go to the hashed
    // buffer U and the cell counts of the next build, which are cleared again
    // after every launch
    int rc = time_candidates(c, (int)cands.size(), reps, e0, e1,
                             [&](int k) {
                                 c->tuning = cands[(size_t)k];
                                 PairLaunch a = pair_args(c, kModeStep, c->S.C, c->S.C, 1.0, nullptr);
                                 a.ev0 = e0;
                                 a.ev1 = e1;
                                 return launch_pair(pl.dim, pl.real_bytes, pl.kernel, kModeStep, a, a.block,
                                                    c->stream);
                             },
                             &kbest);
    const int rc_clear = clear_counts(c);  // also after a failed launch
    if (!rc) rc = rc_clear;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->tuning = rc ? start : cands[(size_t)kbest];
    drop_graph(c);
    if (rc) return rc;
    if (best) *best = c->tuning;
    return ADE_OK;
}

int ade_set_tuning(ade_ctx* c, const ade_tuning* t) {
    if (!c || !t) return fail(ADE_EINVAL, "null argument");
    if (c->plan.general) {
        if (!gen_tuning_fits(c->plan, *t))
            return fail(ADE_EINVAL, "a velocity-field context takes block 64, 128 or 256, lanes 1, 2 or 4, one "
                                    "target per lane group (or two per quad in 2D FP32), no persistent grid, "
                                    "and lists that fit in LDS");
        c->tuning = *t;
        c->tuning.targets = targets_of(*t);
        drop_graph(c);
        return ADE_OK;
    }
    if (t->block != 64 && t->block != 128 && t->block != 256)
        return fail(ADE_EINVAL, "block must be 64, 128 or 256");
    if (t->lanes != 1 && t->lanes != 2 && t->lanes != 4) return fail(ADE_EINVAL, "lanes must be 1, 2 or 4");
    if (t->targets < 0 || t->targets > 2) return fail(ADE_EINVAL, "targets must be 0, 1 or 2");
    if (targets_of(*t) == 2 && !((t->lanes == 1 && t->block <= 128) || (t->lanes == 4 && c->plan.real_bytes == 4)))
        return fail(ADE_EINVAL, "two targets need lanes = 1 and block <= 128, or lanes = 4 in FP32");
    if (t->xcd_group < 0 || t->xcd_group > 4096) return fail(ADE_EINVAL, "xcd_group in 0..4096");
    if (!tuning_fits(c->plan, *t))
        return fail(ADE_EINVAL, "candidate lists of %d lists per workgroup need %zu bytes of LDS (max %zu)",
                    t->block / t->lanes, pair_lds_bytes(t->block, t->lanes, tuning_list_cap(c->plan, *t)),
                    kPairLdsMax);
    if (t->persistent < 0 || t->persistent > 65536) return fail(ADE_EINVAL, "persistent in 0..65536");
    c->tuning = *t;
    drop_graph(c);
    return ADE_OK;
}

int ade_get_tuning(const ade_ctx* c, ade_tuning* t) {
    if (!c || !t) return fail(ADE_EINVAL, "null argument");
    *t = c->tuning;
    return ADE_OK;
}

int ade_info(const ade_ctx* c, int32_t plume, int64_t* n_total, int64_t* n_cells, int64_t* n_tiles,
             double* dt, int64_t* step) {
    if (!c) return fail(ADE_EINVAL, "null ctx");
    if (plume < 0 || plume >= c->plan.P) return fail(ADE_EINVAL, "plume out of range");
    if (n_total) *n_total = c->plan.N;
    if (n_cells) *n_cells = (int64_t)c->plan.ncell;
    if (n_tiles) *n_tiles = c->plan.ntiles;
    if (dt) *dt = c->plan.plumes[plume].dt;
    if (step) {
        int64_t v = 0;
        HIPCHK(hipMemcpyAsync(&v, c->step, sizeof v, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        *step = v;
    }
    return ADE_OK;
}

}  // extern "C"

namespace {

// A saved state: this header, then the sorted particle state as the device
// holds it (positions, C, ids, candidate records, the velocity-field arrays),
// the cell-start table (with its sentinel) and the step counter: everything
// the next step reads, so a loaded state continues bit-identically.
struct StateHeader {
    uint64_t magic;
    uint32_t dim, real_bytes, general, integrator;
    uint64_t N, ncell, bytes;
    uint64_t layout;  // layout_hash of the saving context
};
constexpr uint64_t kStateMagic = 0x3154415453454441ull;  // "ADESTAT1"

// FNV-1a over what places the saved arrays: each plume's particle range and
// cell grid.  Two contexts of equal N and cell count but another split of
// either into plumes do not share a state.
uint64_t layout_hash(const Plan& pl) {
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&](uint32_t w) {
        for (int b = 0; b < 4; ++b) {
            h ^= (w >> (8 * b)) & 0xffu;
            h *= 0x100000001b3ull;
        }
    };
    mix((uint32_t)pl.plumes.size());
    for (const PlumeDev& q : pl.plumes) {
        mix(q.poff);
        mix(q.n);
        mix(q.cbase);
        mix(q.ncell);
        mix(q.nfx);
        mix(q.nr);
        mix(q.nsub);
    }
    return h;
}

struct Section {
    void* dev;
    size_t bytes;
};

std::vector<Section> state_sections(const ade_ctx* c) {
    const Plan& pl = c->plan;
    const size_t N = (size_t)pl.N, rb = (size_t)pl.real_bytes;
    const StateArrays& S = c->S;
    std::vector<Section> v;
    for (int d = 0; d < pl.dim; ++d) v.push_back({S.pos[d], N * 4});
    v.push_back({S.C, N * rb});
    v.push_back({S.id, N * 4});
    if (S.rec) v.push_back({S.rec, N * 16});
    for (int d = 0; d < 3; ++d)
        if (S.vel[d]) v.push_back({S.vel[d], N * rb});
    for (int d = 0; d < 6; ++d)
        if (S.rD[d]) v.push_back({S.rD[d], N * rb});
    if (S.grec) v.push_back({S.grec, N * 32});
    v.push_back({c->cell_start, ((size_t)pl.ncell + 1) * 4});
    v.push_back({c->step, 8});
    return v;
}

size_t state_size(const ade_ctx* c) {
    size_t b = sizeof(StateHeader);
    for (const Section& s : state_sections(c)) b += s.bytes;
    return b;
}

}  // namespace

extern "C" {

int ade_state_bytes(const ade_ctx* c, size_t* bytes) {
    if (!c || !bytes) return fail(ADE_EINVAL, "null argument");
    *bytes = state_size(c);
    return ADE_OK;
}

int ade_save_state(const ade_ctx* c, void* h_buf, size_t bytes) {
    if (!c || !h_buf) return fail(ADE_EINVAL, "null argument");
    if (!c->built) return fail(ADE_ESTATE, "ade_save_state before ade_build_cells");
    const size_t need = state_size(c);
    if (bytes < need) return fail(ADE_EINVAL, "state buffer too small: need %zu bytes", need);
    const Plan& pl = c->plan;
    StateHeader h{kStateMagic, (uint32_t)pl.dim, (uint32_t)pl.real_bytes, pl.general ? 1u : 0u,
                  (uint32_t)pl.integrator, (uint64_t)pl.N, (uint64_t)pl.ncell, (uint64_t)need,
                  layout_hash(pl)};
    char* p = static_cast<char*>(h_buf);
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    for (const Section& s : state_sections(c)) {
        HIPCHK(hipMemcpyAsync(p, s.dev, s.bytes, hipMemcpyDeviceToHost, c->stream));
        p += s.bytes;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return ADE_OK;
}

int ade_load_state(ade_ctx* c, const void* h_buf, size_t bytes) {
    if (!c || !h_buf) return fail(ADE_EINVAL, "null argument");
    const Plan& pl = c->plan;
    StateHeader h;
    if (bytes < sizeof h) return fail(ADE_EINVAL, "state buffer too small");
    std::memcpy(&h, h_buf, sizeof h);
    const size_t need = state_size(c);
    if (h.magic != kStateMagic || h.dim != (uint32_t)pl.dim || h.real_bytes != (uint32_t)pl.real_bytes ||
        h.general != (pl.general ? 1u : 0u) || h.integrator != (uint32_t)pl.integrator ||
        h.N != (uint64_t)pl.N || h.ncell != (uint64_t)pl.ncell || h.bytes != need ||
        h.layout != layout_hash(pl))
        return fail(ADE_EINVAL, "saved state does not belong to a context of these parameters");
    if (bytes < need) return fail(ADE_EINVAL, "state buffer too small: need %zu bytes", need);
    const char* p = static_cast<const char*>(h_buf) + sizeof h;
    for (const Section& s : state_sections(c)) {
        HIPCHK(hipMemcpyAsync(s.dev, p, s.bytes, hipMemcpyHostToDevice, c->stream));
        p += s.bytes;
    }
    // the next step's counting pass starts from empty cells
    HIPCHK(hipMemsetAsync(c->count, 0, sizeof(uint32_t) * cell_pad(pl.ncell), c->stream));
    HIPCHK(hipMemsetAsync(c->lists.ovf_count, 0, 2 * sizeof(uint32_t), c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->initialized = true;
    c->built = true;
    c->vel_set = true;
    return check_coincident(c);
}

int ade_destroy(ade_ctx* c) {
    if (!c) return ADE_OK;
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    drop_graph(c);
    drop_events(c);
    delete c;
    return ADE_OK;
}

const char* ade_last_error(void) { return ade::last_error(); }

const char* ade_version(void) { return "adesph 0.1 (gfx950)"; }

}  // extern "C"
