/*
 * adesph.h -- C ABI of the MI355X (gfx950) SPH advection-dispersion library.
 *
 * The library advances the concentration C of Lagrangian particles under
 *     dC/dt = div(D grad C) - C div v,   dx/dt = v                 (Eqs. 1-2)
 * with the dispersion tensor of Eq. (3),
 *     D_ij = (alpha_T |v| + D_m) delta_ij + (alpha_L - alpha_T) v_i v_j / |v|,
 * discretised by the consistent SPH operator of Eqs. (4)-(5),
 *     (dC/dt)_a = 1/2 sum_b (m_b / rhobar_ab) Dcal_ab (C_a - C_b) x_ab . grad_a W_ab / |x_ab|^2,
 *     Dcal_ab   = sum_ij 4 D_ij,a D_ij,b / (D_ij,a + D_ij,b) [Gamma x_i x_j / |x_ab|^2 - delta_ij],
 * with the Wendland kernel of Eq. (7) (support radius H), Gamma = d + 2
 * (= 4 in 2D as in Eq. 5), in a periodic box, for a uniform flow v (so the
 * convective term of Eq. 4 vanishes and D is the same for every particle),
 * all particles of a plume having equal mass and density.  Time stepping is
 * explicit Euler, or the predictor-corrector of Eqs. (8)-(9).
 * A context created with ADE_VELOCITY_FIELD takes a velocity per particle
 * instead (ade_set_velocities): each particle then has its own tensor D_a,
 * the pair term takes the harmonic mean of Eq. (5) per component, and the
 * convective term of Eq. (4),
 *     + C_a sum_b (m_b / rhobar_ab) (v_a - v_b) . grad_a W_ab,
 * is added; particles move with their own velocities (explicit Euler, or
 * the predictor-corrector with a cell build at the half-step positions).
 * Reference: Klapp, Sigalotti, Alvarado-Rodriguez & Rendon, "Consistent SPH
 * simulations of the anisotropic dispersion of a contaminant plume",
 * arXiv:2108.09488, Sections 2.1-2.4.
 *
 * Conventions (every entry point):
 *  - Returns an int status: ADE_OK (0) or a negative ADE_E* code; never aborts.
 *    ade_last_error() returns a thread-local message for the last failure.
 *  - Pointers named d_* are device pointers, h_* host pointers.  The caller
 *    owns every buffer; the library never allocates device memory.  Device
 *    buffers passed to ade_create must stay valid until ade_destroy.
 *  - All device work is enqueued on the HIP stream given to ade_create and is
 *    asynchronous, except where a host output (h_*, a saved state), the
 *    finite check of ADE_CHECK_FINITE or the coincidence check of
 *    ade_build_cells and ade_load_state forces a synchronisation.
 *  - Positions are SoA doubles, x[c * n + a] for component c of particle a.
 *    The library stores them as 32-bit fixed-point fractions of the box,
 *    u = round(x / L * 2^32) mod 2^32 (resolution L / 2^32): positions are
 *    periodic by construction, and in a uniform flow every particle of a
 *    plume moves by exactly the same displacement each step.
 *  - Several plumes ("an ensemble") can share one context; their particles
 *    are concatenated in plume order in every per-particle array.
 */
#ifndef ADESPH_H
#define ADESPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ade_ctx ade_ctx;

enum {
    ADE_OK = 0,
    ADE_EINVAL = -1,      /* invalid argument (value, size or null pointer) */
    ADE_EWORKSPACE = -2,  /* workspace smaller than ade_workspace_bytes()  */
    ADE_EHIP = -3,        /* a HIP runtime call failed                      */
    ADE_EUNSTABLE = -4,   /* dt above 10x the Eq. (10) bound (ADE_STRICT_DT) */
    ADE_ENONFINITE = -5,  /* non-finite concentration (ADE_CHECK_FINITE)    */
    ADE_ESTATE = -6       /* call out of order (e.g. step before init)      */
};

enum { ADE_WENDLAND_C2 = 2, ADE_WENDLAND_C4 = 4 };
enum { ADE_EULER = 1, ADE_PC = 2 };
enum { ADE_STRICT_DT = 1u, ADE_CHECK_FINITE = 2u, ADE_VELOCITY_FIELD = 4u };

/* One plume: kernel, box, dispersion parameters (Eq. 3), flow and time step.
 * All plumes of a context must share dim, real_bytes, kernel and integrator. */
typedef struct {
    int32_t dim;        /* 2 or 3 */
    int32_t real_bytes; /* 4: FP32 concentration and arithmetic, 8: FP64     */
    int32_t kernel;     /* ADE_WENDLAND_C2 or ADE_WENDLAND_C4 (Eq. 7)        */
    int32_t integrator; /* ADE_EULER or ADE_PC (Eqs. 8-9)                    */
    double H;           /* support radius: W(r) = 0 for r > H (> 0, <= L/3)  */
    double L;           /* side of the periodic box [0, L)^dim (> 0)         */
    double alpha_L;     /* longitudinal dispersivity (>= 0)                  */
    double alpha_T;     /* transverse dispersivity (>= 0)                    */
    double D_m;         /* molecular diffusion coefficient (>= 0)            */
    double v[3];        /* uniform flow velocity (v[2] ignored in 2D; ignored
                           with ADE_VELOCITY_FIELD)                         */
    double dt;          /* time step; <= 0 selects Eq. (10): 0.1 (H/2)^2 / tr D */
    double rho0;        /* density of every particle (> 0)                   */
    double mass;        /* mass of every particle (> 0)                      */
    uint32_t flags;     /* ADE_STRICT_DT | ADE_CHECK_FINITE |
                           ADE_VELOCITY_FIELD (per-particle velocities; the
                           same on every plume of a context; dt > 0)         */
    int32_t cell_rows;  /* cell grid: rows per support radius in y (and z),
                           1..4; 0 = default (2, or 4 for more than 2000
                           expected neighbours per particle)                */
    int32_t cell_xsub;  /* cell grid: cells per support radius along x,
                           1..32; 0 = default (8 in 2D, 12 for a 2D plume
                           of 80 or more expected neighbours, 16 in 3D, 28
                           for a 3D plume of 200 or more; fewer, down to 3,
                           when a context's cell tables would pass 160 MiB
                           at 40 bytes per cell)                            */
    int32_t reserved;   /* must be 0                                         */
} ade_params;

/* Launch shape of the pair kernel (chosen by the autotuner, or defaults).
 * lanes sets how many lanes of a wavefront share one target particle (its
 * candidates are interleaved over them and the partial sums are combined by
 * a wavefront reduction); with N particles the kernel runs N*lanes/64
 * wavefronts, so lanes is the waves-per-CU knob.  Each target keeps the list
 * of its candidate ranges in LDS: 8 * (P * (S + 2) + 2) bytes per target,
 * S = 2R+1 neighbour rows per axis of the plume with the most and P = 1 (2D)
 * or S (3D) planes of rows, and block / lanes targets per workgroup must fit
 * in 64 KiB (ADE_EINVAL otherwise).
 * targets = 2 (with lanes = 1 and block <= 128) gives each lane two
 * consecutive target particles of the cell order: the lane walks one list
 * holding the candidates of both, 8 * (P * (S + 3) + 2) bytes per lane with
 * S = 2R+1 rows and P = 1 (2D) or S + 1 (3D) planes, and evaluates every
 * candidate it loads for both targets, halving the candidate loads per pair
 * evaluated.  In FP32, targets = 2 with lanes = 4 gives the four lanes of a
 * quad two consecutive targets: they list the candidates of both together
 * (the same bytes per quad as a lane's two-target list) and evaluate every
 * candidate for both.  The summation order, and so the last bits of the
 * result, depend on lanes and targets and on nothing else here.  A new
 * context starts with the fewest lanes per particle that keep about 4
 * wavefronts per SIMD: block 64 with two targets per lane from 2^19
 * particles on, else 256 threads with 1 (from 2^18), 2 (from 2^17) or 4
 * lanes per target; a 3D context, or one with a plume of more than 2000
 * expected neighbours per particle, starts with 4 lanes per two targets in
 * FP32 (block 64 in 3D, 128 in 2D) or per target in FP64, xcd_group 128;
 * when the lists do not fit, the first of {256,2}, {256,4}, {128,4}, {64,4}
 * lanes per target, or block 64 with two targets per lane, that does. */
typedef struct {
    int32_t block;          /* threads per workgroup: 64, 128 or 256          */
    int32_t lanes;          /* lanes per target particle: 1, 2 or 4           */
    int32_t xcd_group;      /* work items (tiles or parts of tiles) each XCD
                               takes in turn, so that neighbouring items
                               share an L2 while the XCDs share every part
                               of the work evenly; 0 = default (32)          */
    int32_t persistent;     /* 0: one workgroup per work item; > 0: a grid of
                               that many workgroups loops over the items     */
    int32_t targets;        /* target particles per lane: 1 (0 = 1) or 2      */
} ade_tuning;

/* Bytes of device workspace needed for nplumes plumes with counts[p]
 * particles each (host-only, pure). */
int ade_workspace_bytes(const ade_params *params, const int64_t *counts, int32_t nplumes,
                        size_t *bytes);

/* Validates the parameters and lays out the caller's workspace d_ws
 * (ws_bytes >= ade_workspace_bytes, 256-byte aligned); stream is a
 * hipStream_t (NULL: the default stream).  *out receives the context.  A
 * context holds at most 2^28 - 256 particles in total (candidate records are
 * addressed with 32-bit byte offsets); larger ensembles take several
 * contexts.  A plume of a multi-plume context evolves bit for bit as it does
 * alone when both runs have the same cell grid (cell_rows, and cell_xsub
 * where the context's cell tables would pass the 160 MiB budget, since the
 * default x cells then widen for the whole context) and the same lanes and
 * targets: the grid fixes the candidate order of every sum. */
int ade_create(const ade_params *params, const int64_t *counts, int32_t nplumes, void *d_ws,
               size_t ws_bytes, void *stream, ade_ctx **out);

/* Loads positions d_x (double, SoA dim x N, N = sum of counts, plumes
 * concatenated) and concentrations d_C (N reals of real_bytes) and resets
 * the step counter.  The ids of the particles are their indices in d_x. */
int ade_init_particles(ade_ctx *ctx, const double *d_x, const void *d_C);

/* Velocity field (contexts created with ADE_VELOCITY_FIELD): d_v holds the
 * velocity of every particle (double, SoA dim x N in id order, the layout of
 * d_x).  Call after ade_init_particles and before ade_build_cells (ADE_ESTATE
 * otherwise; ADE_EINVAL for a context without the flag); init clears it.
 * Each particle keeps its velocity, stored in the working precision, for
 * the whole run; its tensor D_a (Eq. 3) is formed from the stored value.
 * Every step, particle a moves by rint((k + 1) u_a) - rint(k u_a) grid
 * units (u_a = dt v_a / L * 2^32, k the step index), so the displacement
 * after k steps is rint(k u_a): exact when u_a is an integer.  With ADE_PC
 * the predictor moves it to x + rint((k + 1/2) u_a) - rint(k u_a), the cells
 * are rebuilt there for the corrector, and the corrector completes the step.
 * The pair sum
 * takes the launch shapes block {64, 128, 256} x lanes {1, 2, 4} with one
 * target per group of lanes, and in 2D FP32 also four lanes per two targets
 * (targets = 2), no persistent grid, through ade_set_tuning or ade_autotune.
 * A new context starts with 4 lanes per target in the largest block whose
 * lists fit, or in 2D FP32 with a plume of more than 2000 expected
 * neighbours per particle with block 128 and four lanes per two targets.  A 2D FP32 velocity-field context holds at most 2^27 - 256
 * particles (its 32-byte candidate records take 32-bit byte offsets).
 * ade_adjoint takes it
 * (Euler or ADE_PC): its checkpoints then hold the velocities and tensors
 * too, the recompute keeps every step's half-step state for the
 * predictor-corrector, and the gradient differentiates every pair's
 * harmonic mean. */
int ade_set_velocities(ade_ctx *ctx, const double *d_v);

/* Cell-linked list: cell hash, counting sort by cell (stable, ordered by
 * particle id within a cell) and the cell-start table, then the particle
 * state is gathered into cell order.  Needed once after init; every step
 * rebuilds it.  For a uniform flow it also checks whether two particles of
 * a plume share a position (and synchronises the stream for that): the sum
 * of Eq. (4) leaves out pairs at r = 0, and when no two particles coincide
 * the only candidate at r = 0 is a target's own record, whose term is zero,
 * so the FP32 Wendland C4 pair kernels skip the test (the same sums but for
 * a rounding of r^2 where it sits on a tie; every step keeps the relative
 * positions of a plume's particles, so the check holds for the run).
 * ade_load_state repeats the check. */
int ade_build_cells(ade_ctx *ctx);

/* *out = 1 when two particles of a plume share a position (or the context
 * has not been checked: before ade_build_cells, and always for
 * ADE_VELOCITY_FIELD contexts), else 0. */
int ade_coincident(const ade_ctx *ctx, int32_t *out);

/* nsteps explicit steps (pair sum of Eqs. 4-5, update of C and x, rebuild).
 * With ADE_CHECK_FINITE on any plume of the context, the concentrations are
 * checked after the last step (the stream is synchronised) and a NaN or an
 * infinity returns ADE_ENONFINITE (the steps have run). */
int ade_step(ade_ctx *ctx, int64_t nsteps);

/* The same steps replayed from a HIP graph holding one captured step (the
 * finite check as for ade_step, after the replays). */
int ade_step_graph(ade_ctx *ctx, int64_t nsteps);

/* rhs of Eq. (4) at the current state, written in particle-id order to
 * d_rhs (N reals). */
int ade_rhs(ade_ctx *ctx, void *d_rhs);

/* Current concentrations / positions in particle-id order. */
int ade_read_C(const ade_ctx *ctx, void *d_C_out);
int ade_read_x(const ade_ctx *ctx, double *d_x_out);

/* Solute mass sum_a m_a C_a of each plume, accumulated in FP64 in a fixed
 * order, to d_out[nplumes] (device). */
int ade_mass(const ade_ctx *ctx, double *d_out);

/* Smallest and largest concentration of each plume (the paper's
 * negative-concentration diagnostic, Section 4), in FP64, to
 * d_out[2 * plume] (min) and d_out[2 * plume + 1] (max) (device); NaNs are
 * skipped (see ADE_CHECK_FINITE). */
int ade_conc_range(const ade_ctx *ctx, double *d_out);

/* Neighbour sets as used by the pair sum: for particle a (id order), the
 * ids of all b != a with 0 < |x_ab| <= H, in d_ids[d_offsets[a] ..
 * d_offsets[a+1]) (unordered within a particle).  d_offsets has N+1
 * entries.  *h_needed receives the total; ids are written only if
 * cap >= total.  Synchronises the stream. */
int ade_neighbours(ade_ctx *ctx, int64_t *d_offsets, int32_t *d_ids, int64_t cap,
                   int64_t *h_needed);

/* Shepard interpolation C_s = sum_b W_sb C_b / sum_b W_sb at n_sensors points
 * d_xs (double, SoA dim x S) of plume 0, to d_Cs (S reals). */
int ade_sensor_interp(ade_ctx *ctx, const double *d_xs, int32_t n_sensors, void *d_Cs);

/* Workspace for ade_adjoint (device bytes). */
int ade_adjoint_workspace_bytes(const ade_ctx *ctx, int64_t nsteps, int32_t ckpt_every,
                                int32_t n_sensors, size_t *bytes);

/* Misfit and gradient of J = sum_s (C_s(T) - d_s)^2 after nsteps steps of the
 * context's integrator (explicit Euler, or the predictor-corrector of Eqs.
 * 8-9: its step is C <- (I + dt L + dt^2/2 L^2) C for a uniform flow, and the
 * adjoint applies the same two stages to lambda) from the current state,
 * w.r.t. (alpha_L, alpha_T, D_m) of plume 0, by a discrete adjoint with a
 * checkpoint every ckpt_every steps and recompute.  For a velocity field
 * (ADE_VELOCITY_FIELD, explicit Euler) the operator is again its own
 * transpose (symmetric pair weights, a convective term diagonal in C) and
 * the gradient takes d(h/4)_ij = (q^2 dp + p^2 dq) / (p + q)^2 per pair and
 * component (p, q the two particles' tensor components); with ADE_PC the
 * corrector's operator L2 lives at the half-step positions, so a reverse
 * step is y = L2 lambda there and lambda + dt y + dt^2/2 L1 y at x^n.
 * d_obs holds S reals.  On return the context holds the state at step
 * nsteps.  h_grad receives 3 doubles; synchronises the stream. */
int ade_adjoint(ade_ctx *ctx, int64_t nsteps, int32_t ckpt_every, const double *d_xs,
                int32_t n_sensors, const void *d_obs, void *d_adj_ws, size_t adj_ws_bytes,
                double *h_J, double *h_grad);

/* The same as ade_adjoint, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the adjoint workspace is a fixed array of the library's own
 * device memory instead of a caller's buffer, so the call allocates nothing
 * (no hipMalloc, no hipFree, no allocating library routine).  The array
 * holds ade_adjoint_noalloc_max_bytes() bytes (64 MiB); a run whose adjoint
 * workspace (ade_adjoint_workspace_bytes) is larger returns ADE_EWORKSPACE
 * and changes nothing.  Each GPU the library runs on holds one such array
 * from the first call on it until the process ends, and every call on that
 * GPU uses it: calls that overlap on one GPU (other threads, other streams)
 * race and must not be made.  Results are those of ade_adjoint (the same
 * kernels in the same order); arguments, errors and synchronisation as for
 * ade_adjoint. */
int ade_adjoint_noalloc(ade_ctx *ctx, int64_t nsteps, int32_t ckpt_every, const double *d_xs,
                        int32_t n_sensors, const void *d_obs, double *h_J, double *h_grad);
int ade_adjoint_noalloc_max_bytes(size_t *bytes);

/* HIP-event timing of the pair kernel launches on the context's stream.
 * mode 1: start (clears the totals; events are recorded around every pair
 * kernel launched eagerly by ade_step / ade_rhs).  mode 0: stop, synchronise
 * and return the summed kernel time in *h_ms and the number of launches in
 * *h_count (either may be NULL). */
int ade_kernel_timing(ade_ctx *ctx, int32_t mode, double *h_ms, int64_t *h_count);

/* Autotuner: times the pair kernel as a step launches it (update mode; reps
 * launches each plus one warm-up, each timed by HIP events stamped with the
 * kernel's own start and end on the context's stream; the kernel's outputs
 * go to the step's scratch buffers and the next build's cell counts, which
 * are cleared after every launch) over the launch shapes block {64,128,256} x (lanes,
 * targets) {(1,2), (1,1), (2,1), (4,1), (4,2)} x persistent {0, 8 workgroups
 * per CU} x xcd_group {8, 32, 128} that are valid and fit the LDS limit (a
 * velocity-field context: block x (lanes, targets) only), keeps the
 * fastest in the context and returns it in *best (may be NULL).  With
 * ADE_TUNE_KEEP_LANES the current lanes and targets are kept, so results stay
 * bitwise identical to the untuned context.  Needs built cells; does not
 * change the particle state.  Synchronises the stream. */
enum { ADE_TUNE_KEEP_LANES = 1 };
int ade_autotune(ade_ctx *ctx, int32_t reps, int32_t flags, ade_tuning *best);

int ade_set_tuning(ade_ctx *ctx, const ade_tuning *t);
int ade_get_tuning(const ade_ctx *ctx, ade_tuning *t);

/* Scalar facts about a context: number of particles, cells, tiles, the time
 * step of plume p actually used, and the step counter. */
int ade_info(const ade_ctx *ctx, int32_t plume, int64_t *n_total, int64_t *n_cells,
             int64_t *n_tiles, double *dt, int64_t *step);

/* Checkpoint and resume.  ade_state_bytes gives the size of a saved state
 * (host-only).  ade_save_state copies the context's state (the sorted
 * particle state with its candidate records and velocity-field arrays, the
 * cell table and the step counter; after ade_build_cells) into the caller's
 * host buffer h_buf of at least that many bytes, synchronising the stream.
 * ade_load_state puts such a state into a context created with the same
 * parameters and counts: the context then continues bit-identically to the
 * one saved, as if built.  It checks the dimension, precision, integrator,
 * flow kind, and each plume's particle range and cell grid (ADE_EINVAL when
 * any differs, or for a short buffer).  The state holds no other plume
 * parameter: a uniform-flow context steps with its own dispersivities and dt,
 * a velocity-field context with the velocities and tensors saved. */
int ade_state_bytes(const ade_ctx *ctx, size_t *bytes);
int ade_save_state(const ade_ctx *ctx, void *h_buf, size_t bytes);
int ade_load_state(ade_ctx *ctx, const void *h_buf, size_t bytes);

int ade_destroy(ade_ctx *ctx);

const char *ade_last_error(void);
const char *ade_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ADESPH_H */
