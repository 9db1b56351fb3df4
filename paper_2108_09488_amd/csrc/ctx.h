// ctx.h -- host-side context of the C ABI shared by the API translation
// units: the plan of a context (per-plume tables), the context itself and the
// launch sequences every entry point builds on.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/adesph.h"
#include "ade_internal.h"

namespace ade {

// records a thread-local error message and returns code
int fail(int code, const char* fmt, ...);

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ADE_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

struct Plan {
    int dim = 0, real_bytes = 0, kernel = 0, integrator = 0, P = 0;
    int64_t N = 0;
    uint64_t ncell = 0;
    uint32_t ntiles = 0, nscan = 0;
    int list_cap = 0;       // candidate-list entries per target (largest plume)
    int list_cap_pair = 0;  // the same for a lane's merged list of two targets
    double nbar_max = 0.0;  // largest expected neighbours per particle of a plume
    bool general = false;   // velocity field: per-particle velocities (ADE_VELOCITY_FIELD)
    bool check_finite = false;  // ADE_CHECK_FINITE on any plume
    std::vector<PlumeDev> plumes;
    std::vector<TileDev> tiles;
    std::vector<TileDev> pair_tiles;  // the tiles in the pair kernel's order (costliest plumes first)
};

// whether a launch shape fits the plan (LDS of the candidate lists)
bool tuning_fits(const Plan& pl, const ade_tuning& t);

// D of Eq. (3) for a uniform flow (row stride 3); returns its trace.
double trace_D(int dim, double aL, double aT, double Dm, const double* v, double D[9]);

}  // namespace ade

struct ade_ctx {
    ade::Plan plan;
    hipStream_t stream = nullptr;
    ade_tuning tuning{256, 2, 0, 0};
    ade::PlumeDev* plumes = nullptr;
    ade::TileDev* tiles = nullptr;
    ade::TileDev* pair_tiles = nullptr;
    ade::StateArrays S{}, U{};
    ade::CellLists lists{};
    uint32_t* count = nullptr;
    uint32_t* cell_start = nullptr;
    void* scan_partial = nullptr;
    void* aux = nullptr;
    uint4* aux_rec = nullptr;
    double* mass_partial = nullptr;
    double* range_partial = nullptr;  // per tile: min and max of C
    int64_t* step = nullptr;
    uint32_t* nonfinite = nullptr;  // finite check: set when a concentration is not finite
    uint32_t h_total = 0;  // host copy of N for the cell-start sentinel
    bool initialized = false, built = false;
    // two particles of a plume share a position (the pair kernels then test
    // every candidate for r > 0); true until a cell build has checked
    bool coincident = true;
    bool vel_set = false;  // velocity field: ade_set_velocities called since init
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool capturing = false;
    // pair-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t ev_used = 0;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
};

namespace ade {

// enqueue a pair kernel (timed when timing is on)
int run_pair(ade_ctx* c, int mode, const PairLaunch& a);
// launch arguments of a pair kernel over the sorted state of c
PairLaunch pair_args(ade_ctx* c, int mode, const void* Cpair, const void* Cbase, double scale, void* out);
// counting sort of the hashed U buffer into S and the cell-start table
int enqueue_build(ade_ctx* c, int inc_step);
// one explicit step (pair sum, update, rebuild)
int enqueue_step(ade_ctx* c);
// launch arguments of the velocity-field pair kernel over the sorted state of c
GenLaunch gen_args(ade_ctx* c, void* out);
// enqueue the velocity-field pair kernel (timed when timing is on)
int run_gen(ade_ctx* c, int mode, void* out);

}  // namespace ade
