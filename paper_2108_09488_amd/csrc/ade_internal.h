// ade_internal.h -- device-side tables and kernel launch declarations shared
// by the kernels and the C-ABI host code of the SPH advection-dispersion
// library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ade {

constexpr int kTile = 256;          // particles per tile (a tile never spans two plumes)
constexpr int kScanPerThread = 16;  // counting-sort scan: elements per thread
constexpr int kScanBlock = 256;
constexpr int kScanChunk = kScanPerThread * kScanBlock;
constexpr int kCellChunk = 1024;    // cell-count scan: 256 threads x 4 counts per workgroup

// cell tables are padded to a whole number of scan chunks (plus the sentinel)
inline uint64_t cell_pad(uint64_t ncell) { return (ncell + 1 + kCellChunk - 1) / kCellChunk * kCellChunk; }

// Per-plume constants.  Positions are uint32 fractions of the box, so all
// lengths below are in grid units (L / 2^32).
struct PlumeDev {
    uint32_t poff, n;       // particles [poff, poff + n) in the concatenated order
    uint32_t cbase, ncell;  // cells [cbase, cbase + ncell) of the global cell table
    uint32_t nfx, nr;       // cells per row along x; rows per side in y (and z)
    int32_t R;              // rows to each side that can hold neighbours
    uint32_t hx;            // half-width of the x search window (>= H_u (1 + 2^-16))
    uint32_t tfirst, tcount;// tiles of this plume
    uint32_t nsub;          // sub-rows per row (cells of a row: nfx x-cells of nsub sub-rows each)
    uint32_t pad1;
    double Hu;              // support radius in grid units
    double H2d;             // Hu^2 (double)
    float H2f;              // Hu^2 rounded to float
    float cellx;            // x cells per grid unit, nfx * 2^-32 (float)
    double invHu;
    float Hc2f;             // square of the search radius Hc = H_u (1 + 2^-16) + 2
    float rowh2f;           // square of the row height in grid units, (2^32 / nr)^2
    float cslack;           // slack of a candidate window in x cells (covers float rounding)
    float pad4;
    double a0, a1;          // Gamma x^T D x / r^2 - tr D = a0 + a1 (e . x / r)^2 (Eq. 3 tensor)
    double ehat[3];         // unit flow direction e (x axis when |v| = 0)
    double pad3;
    // pair-term constants as the pair kernel uses them: Hu^2, 1/Hu, 5/Hu,
    // A0, S, E_x, E_y, E_z with the bracket A = A0 + S (E . x / r)^2,
    // E = sqrt|a1| e, S = sign of a1 (in 2D always +1: a negative a1 is
    // folded into A0 and E normal to the flow)
    double dterm[8];
    float fterm[8];         // the same in FP32
    double trD;             // trace of D
    double vphi;            // V * (kernel derivative prefactor): rhs = vphi * sum
    double dt;
    double ushift[3];       // displacement per step in grid units
    double vel[3];          // flow velocity (physical units)
    double mass;            // particle mass
    double L;
    double aL, aT, Dm;      // alpha_L, alpha_T, D_m (per-particle tensors of a velocity field)
};

struct TileDev {
    uint32_t plume, start, end, pad;
};

// Particle state in structure-of-arrays form.
struct StateArrays {
    uint32_t* pos[3];
    uint4* rec;      // 16-byte candidate records (sorted buffer S only; null if unused)
    void* C;
    uint32_t* id;
    uint32_t* key;   // cell key (hashed buffer U only)
    // velocity field only (null otherwise): per-particle velocity (DIM
    // components) and the reciprocals of the components of the dispersion
    // tensor of Eq. (3) it gives (2D: xx, xy, yy; 3D: xx, xy, xz, yy, yz, zz;
    // 1/0 = inf), in the working precision
    void* vel[3];
    void* rD[6];
    // velocity field with the predictor-corrector: C^n carried through the
    // predictor's build (null otherwise)
    void* Cb;
    // velocity field in 2D FP32, sorted buffer S only (null otherwise): a
    // 32-byte record per particle, {x, y, C, v_x} {v_y, 1/D_xx, 1/D_xy, 1/D_yy}
    uint4* grec;
};

// Counting pass of the cell build: the number of particles per cell and
// their ids -- the first kBucket of a cell in its bucket, any further ones in
// an overflow list of (key, id) pairs.
constexpr uint32_t kBucket = 8;
struct CellLists {
    uint32_t* count;      // per cell (cleared by the scan)
    uint32_t* bucket;     // kBucket entries per cell: particle ids
    uint2* ovf;           // overflow pairs (key, id), up to N
    uint32_t* ovf_count;  // [0] pairs added since the last scan, [1] pairs of the current build
};

// kModeFull: the corrector of the velocity-field predictor-corrector step
enum PairMode { kModeStep = 0, kModeHalf = 1, kModeRhs = 2, kModeFull = 3 };

struct PairLaunch {
    const PlumeDev* plumes;
    const TileDev* tiles;
    uint32_t ntiles;
    int block;              // threads per workgroup
    int lanes;              // lanes per target particle (1, 2 or 4)
    int targets;            // target particles per lane: 1, or 2 (one lane, block <= 128)
    int list_cap;           // candidate-list entries per target in LDS (list_cap_for)
    int persistent;         // 0: one workgroup per work item; > 0: that many workgroups loop
    uint32_t xcd_group;     // consecutive work items an XCD takes in turn (>= 1)
    int zc;                 // 1: two distinct particles may share a position, so every
                            // candidate is tested for r > 0; 0: the only candidate at
                            // r = 0 is the target's own record (FP32 C4 kernels skip the test)
    const uint4* rec;       // candidate records (position + C of Cpair), or null: SoA reads
    const uint32_t* spos[3];
    const uint32_t* sid;
    const void* Cpair;      // concentrations entering C_a - C_b
    const void* Cbase;      // concentrations updated (step mode)
    const uint32_t* cell_start;
    // step mode outputs
    uint32_t* upos[3];
    void* uC;
    uint32_t* uid;
    uint32_t* ukey;
    CellLists lists;
    const int64_t* step;
    double scale;           // fraction of the plume's dt: step 1, half 0.5 (unused for rhs)
    void* out;              // half: S-order output; rhs: id-order output
    uint4* out_rec;         // half: candidate records with the half-step C (S order)
    hipEvent_t ev0, ev1;    // if set: events stamped at the kernel's start and end
};

// candidate-list capacity per target for plumes of span = 2R + 1 neighbour
// rows per axis: span + 2 entries per plane of rows (see build_list), plus a
// sentinel and one entry read past it
inline int list_cap_for(int dim, int span) { return (dim == 3 ? span : 1) * (span + 2) + 2; }
// the same for the merged list of a lane's two targets (span + 1 rows per
// plane, span + 1 planes in 3D; n + 2 ranges per plane of n rows)
inline int list_cap_pair_for(int dim, int span) { return (dim == 3 ? span + 1 : 1) * (span + 3) + 2; }
// LDS bytes of the pair kernel's candidate lists for a workgroup
inline size_t pair_lds_bytes(int block, int lanes, int list_cap) {
    return (size_t)(block / lanes) * (size_t)list_cap * 8u;
}
constexpr size_t kPairLdsMax = 65536;

// kernel launchers (kernels_*.hip); all return hipError_t of the launch
hipError_t launch_init(int dim, int real_bytes, const PlumeDev* plumes, const TileDev* tiles,
                       uint32_t ntiles, const double* x, const void* C, uint32_t N,
                       StateArrays U, CellLists lists, hipStream_t s);
hipError_t launch_scan(CellLists lists, uint32_t* cell_start, uint32_t* partial, uint32_t ncell,
                       hipStream_t s);
hipError_t launch_place(int dim, int real_bytes, StateArrays U, StateArrays S, CellLists lists,
                        const uint32_t* cell_start, uint32_t N, int64_t* step, int inc_step,
                        hipStream_t s);
// Velocity field (per-particle velocities, general Eq. 4): the pair sum with
// per-pair harmonic means and the convective term, one lane per target.
struct GenLaunch {
    const PlumeDev* plumes;
    const TileDev* tiles;
    uint32_t ntiles;
    int list_cap;
    int lanes;              // lanes per target particle: 1, 2 or 4 (per two targets: 4)
    int targets;            // targets per group of lanes: 1, or 2 (four lanes, 2D FP32)
    int block;              // threads per workgroup: 64, 128 or 256 (its lists fit in LDS)
    StateArrays S, U;
    const uint32_t* cell_start;
    CellLists lists;
    const int64_t* step;
    void* out;              // rhs mode: id-order output
    hipEvent_t ev0, ev1;    // if set: events stamped at the kernel's start and end
};
hipError_t launch_setvel(int dim, int real_bytes, const PlumeDev* plumes, const TileDev* tiles, uint32_t ntiles,
                         const double* v, uint32_t N, StateArrays U, hipStream_t s);
// Adjoint pass of the velocity-field Euler step over a state snapshot S:
// lam_out (id order) = lambda + dt L^T lambda, gradient partials per
// workgroup added to gpart[3 * workgroup + k].
struct AdjGenLaunch {
    const PlumeDev* plumes;
    const TileDev* tiles;
    uint32_t ntiles;
    int list_cap;
    StateArrays S;
    const uint32_t* cell_start;
    const void* lam_s;  // the vector the pass applies the operator to, in the snapshot's cell order
    const void* lam_id; // corrector pass: lambda^(n+1) in id order
    void* lam_out;      // the pass's output in id order
    double* gpart;
};
// passes: Euler (lambda + dt L lambda), and the predictor-corrector's two:
// at the half-step snapshot y = L lambda, at the step's snapshot
// lambda + dt y + dt^2/2 L y
enum AdjGenMode { kAdjGenEuler = 0, kAdjGenHalf = 1, kAdjGenFull = 2 };
hipError_t launch_adjoint_gen(int dim, int real_bytes, int kernel, int mode, const AdjGenLaunch& a,
                              uint32_t block, hipStream_t s);
hipError_t launch_pair_gen(int dim, int real_bytes, int kernel, int mode, const GenLaunch& g, hipStream_t s);
hipError_t launch_pair(int dim, int real_bytes, int kernel, int mode, const PairLaunch& a,
                       int block, hipStream_t s);
hipError_t launch_read_C(int real_bytes, StateArrays S, uint32_t N, void* out, hipStream_t s);
hipError_t launch_coincident(int dim, const PlumeDev* plumes, const TileDev* tiles, uint32_t ntiles,
                             StateArrays S, const uint32_t* cell_start, uint32_t* flag, hipStream_t s);
hipError_t launch_read_x(int dim, const PlumeDev* plumes, const TileDev* tiles, uint32_t ntiles,
                         StateArrays S, uint32_t N, double* out, hipStream_t s);
hipError_t launch_mass(int real_bytes, const PlumeDev* plumes, int nplumes, const TileDev* tiles,
                       uint32_t ntiles, StateArrays S, double* partial, double* out,
                       hipStream_t s);
hipError_t launch_nbr(int dim, int real_bytes, int fill, const PlumeDev* plumes,
                      const TileDev* tiles, uint32_t ntiles, StateArrays S,
                      const uint32_t* cell_start, int64_t* offsets, int32_t* ids, hipStream_t s);
hipError_t launch_scan64(int64_t* data, uint32_t n, int64_t* partial, hipStream_t s);

}  // namespace ade
