/*
 * adiwave.h -- C ABI of the MI355X (gfx950) ADI solver for the implicit
 * finite-difference 2-D acoustic wave equation.
 *
 * Method (Altybay, Ruzhansky, Tokmagambetov, "A parallel hybrid implementation
 * of the 2D acoustic wave equation", Sec. 2):
 *   u_tt - kappa(x, y) (u_xx + u_yy) = f on the unit square, zero Dirichlet
 *   walls (eqs. (f1)-(f5)); kappa is the paper's coefficient c of eq. (f1),
 *   taken here time-independent and per cell, and supplied either as a wave
 *   speed (kappa = speed^2) or directly.
 *   Time discretisation: the three-level implicit scheme of eq. (CN1) with
 *   weights 1/2 on levels k+1 and k-1, factored in the alternating-direction
 *   way of eqs. (fr1)-(fr2): first an implicit solve along every x-line, then
 *   along every y-line.  With beta = dt^2/2 and r = beta kappa / h^2, one step
 *   n -> n+1 is
 *     rho   = dt^2 (kappa Lap_h u^n + f^n)               (5-point Laplacian)
 *           = 2 r (u_W + u_E + u_S + u_N - 4 u_C) + dt^2 f^n
 *     (I - beta K Lxx) w = rho      x-lines: -r w_{i-1} + (1+2r) w_i - r w_{i+1}
 *     (I - beta K Lyy) d = w        y-lines: same coefficients along j
 *     u^{n+1} = 2 u^n - u^{n-1} + d
 *   The paper solves the line systems by cyclic reduction (Sec. 3.1); this
 *   library solves them by an exact partition (sub-structuring) method, which
 *   reaches the same solution up to rounding.
 *
 * Grids and layout: nx x ny interior nodes, spacing h (the walls are not
 * stored); every field is row-major, node (i, j) at offset j*nx + i, x fastest.
 * All field pointers are DEVICE pointers of the handle's element type
 * (float for ADI_F32, double for ADI_F64), owned by the caller, contiguous,
 * and must stay valid until the work queued on the handle's stream is done.
 * Index arrays are device int32 arrays of flat node offsets j*nx + i.
 *
 * Ownership: the library owns the handle and its device workspace
 * (coefficient field r, the x-sweep result w, chunk summaries of the y-line
 * partition, reduced-system solution).  They are allocated by the create call
 * and freed by the destroy call; stepping allocates nothing.
 *
 * Streams: every call queues work on the HIP stream bound to the handle (or
 * passed explicitly) and returns without synchronising, except where stated.
 *
 * Errors: every entry point returns an adi_status.  Arguments are validated
 * before anything is queued; on error nothing is written to the outputs and
 * adi_last_error() returns a message (per host thread).  HIP runtime failures
 * map to ADI_EHIP with the runtime's error string.
 */
#ifndef ADIWAVE_H
#define ADIWAVE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adi_wave_s* adi_wave_t;          /* opaque; owned by the library */

typedef enum { ADI_F32 = 0, ADI_F64 = 1 } adi_dtype;

typedef enum {
    ADI_OK = 0,
    ADI_EINVAL = -1,          /* bad argument, detected before any work is queued */
    ADI_ENOMEM = -2,          /* device allocation failed (create only) */
    ADI_EHIP = -3,            /* HIP runtime error */
    ADI_EUNSUPPORTED = -4     /* valid but outside what the kernels handle (sizes) */
} adi_status;

typedef enum {
    ADI_START_PAPER = 0,      /* u^1 = u^0 + dt psi, eq. (CN2): first order in time */
    ADI_START_GHOST = 1       /* scheme at n = 0 with ghost level u^{-1} = u^1 - 2 dt psi */
} adi_start_mode;

/* Point sources: f^n is zero except at `count` nodes, where it takes the values
 * amp[k*count + s] for the k-th step of the call (the level n whose right-hand
 * side is being built, eq. (CN1) uses f^k).  A discrete delta of strength s(t)
 * is f = s(t)/h^2 at its node.  count may be 0 (idx/amp ignored).  At most
 * ADI_MAX_SOURCES sources per call.  Offsets outside [0, nx*ny) are ignored. */
#define ADI_MAX_SOURCES 1024
typedef struct {
    int count;
    const int* idx;           /* device, count node offsets */
    const void* amp;          /* device, nsteps x count values of the handle's type */
} adi_source;

/* Receivers: after step k of a call, u^{n+1} at node idx[r] is written to
 * traces[k*count + r].  count may be 0.  An offset outside [0, nx*ny) records NaN. */
typedef struct {
    int count;
    const int* idx;           /* device, count node offsets */
    void* traces;             /* device, nsteps x count values of the handle's type */
} adi_receivers;

/* ---------------------------------------------------------------- handle ---- */

/* Create a solver for an nx x ny interior grid with spacing h and time step dt:
 * the uniform grid of Sec. 2, eq. (f6) (nodes (i+1) h, (j+1) h; h = 1/(N+1) for
 * N interior nodes on the unit square), and the coefficient of the line systems
 * of eq. (CN1) in the split of eqs. (fr1)-(fr2), r = beta kappa / h^2.
 * speed: device field (nx*ny, handle type) of wave speeds (kappa = speed^2),
 *        or NULL to use the constant speed_scalar.  Speeds must be > 0.
 * The per-node coefficient r = dt^2 speed^2 / (2 h^2) is computed on the
 * device in the handle's type and kept in the workspace.
 * hip_stream: hipStream_t the handle queues on (NULL = default stream).
 * Limits: 1 <= nx <= 8192, 1 <= ny <= 16384.
 * Synchronises the stream before returning (the workspace is ready). */
adi_status adi_wave_create(adi_wave_t* out, int nx, int ny, double h, double dt,
                           const void* speed, double speed_scalar, adi_dtype dtype,
                           void* hip_stream);

/* Replace the coefficient by kappa directly (device field of the handle's
 * type, or NULL to use kappa_scalar).  Queued on the handle's stream. */
adi_status adi_wave_set_kappa(adi_wave_t w, const void* kappa, double kappa_scalar);

/* Rebind the handle to another HIP stream. */
adi_status adi_wave_set_stream(adi_wave_t w, void* hip_stream);

/* Level u^1 from u^0 (Sec. 2, eq. (CN2) for ADI_START_PAPER; the second-order
 * ghost-level start for ADI_START_GHOST).  psi: device field or NULL (zero
 * initial velocity).  f0: sources of level 0 (amp holds 1 x count values) or
 * NULL.  u1 must not alias u0 or psi. */
adi_status adi_wave_start(adi_wave_t w, const void* u0, const void* psi,
                          const adi_source* f0, int mode, void* u1);

/* nsteps ADI steps (Sec. 2 scheme, Sec. 3 Algorithm 1 time loop).
 * On entry *u_prev, *u_curr point to u^{n-1}, u^n.  Each step writes u^{n+1}
 * over u^{n-1} and swaps the two pointers, so on return *u_curr points to
 * u^{n+nsteps} and *u_prev to u^{n+nsteps-1} (the roles rotate as the
 * paper's swap of level matrices).  f, rec: may be NULL.  nsteps >= 0. */
adi_status adi_wave_step(adi_wave_t w, void** u_prev, void** u_curr,
                         const adi_source* f, const adi_receivers* rec, int nsteps);

/* Free the handle and its workspace (synchronises the handle's stream). */
adi_status adi_wave_destroy(adi_wave_t w);

/* ----------------------------------------------------------------- adjoint -- */

/* Gradients of a scalar function J of the receiver traces with respect to
 * the per-node coefficient kappa (and the source values), by the discrete
 * adjoint of the step above run backwards in time (not in the paper).
 * With lambda^m = dJ/du^m, A_x = I - beta K Lxx, A_y = I - beta K Lyy:
 *   nu = A_y^{-T} lambda^{k+1}, mu = A_x^{-T} nu,
 *   dJ/dkappa += dt^2 mu Lap(u^k) + beta (mu Lxx w^k + nu Lyy d^k),
 *   dJ/df^k = dt^2 mu at the source nodes,
 *   lambda^k = g^k + 2 lambda^{k+1} - lambda^{k+2} + dt^2 Lap(kappa mu),
 * with d^k = u^{k+1} - 2u^k + u^{k-1} and w^k = A_y d^k formed from the levels.
 * The initial levels are treated as independent of kappa.  Where the forward
 * run takes the one-pass step, the reverse pass works on the exact step's levels
 * recomputed from its checkpoints (the two steps differ by at most the one-pass
 * bound, half an ulp per step), so the gradient then depends on
 * checkpoint_every only at that level; after exact steps it does not at all. */

/* Forward run of nsteps steps from (u_prev, u_curr) (not modified) with
 * sources and receivers exactly as adi_wave_step (the handle's step: the
 * one-pass step where it is allowed, else the exact two-pass step; never cyclic
 * reduction), keeping the level pair every checkpoint_every steps in
 * handle-owned device memory (allocated here on first use or growth:
 * 2 * ceil(nsteps / checkpoint_every) + 6 fields).
 * The handle keeps ONE forward record: this call replaces the previous one,
 * and a coefficient change (adi_wave_set_kappa, adi_wave_step_tdc) discards it.
 * record (may be NULL) receives the id of the new record (never 0). */
adi_status adi_adjoint_forward(adi_wave_t w, const void* u_prev, const void* u_curr,
                               const adi_source* f, const adi_receivers* rec, int nsteps,
                               int checkpoint_every, unsigned long long* record);

/* Reverse pass of the stored forward record (same f and rec as that run).
 * record: the id adi_adjoint_forward returned, or 0 for whatever record is
 * stored; ADI_EINVAL when no record is stored, when the coefficient changed
 * since the forward run, or when record names a run that a later forward run
 * replaced (nothing is written then).
 * grad_traces: device, nsteps x rec->count values of dJ/d(trace).
 * grad_kappa: device nx*ny, overwritten with dJ/dkappa.
 * grad_amp: device nsteps x f->count, overwritten with dJ/d(source value),
 * or NULL.  Each segment between checkpoints is recomputed once, with the
 * exact two-pass step, on a second stream the library creates for the handle,
 * overlapping the reverse pass of the segment after it (allocates
 * 2 * checkpoint_every fields and a copy of the y-chunk planes on first use or
 * growth); the call returns with all its work ordered on the handle's stream. */
adi_status adi_adjoint_backward(adi_wave_t w, unsigned long long record, const adi_source* f,
                                const adi_receivers* rec, const void* grad_traces,
                                void* grad_kappa, void* grad_amp);

/* One step of eq. (CN1) with a coefficient that changes in time (Sec. 2: the
 * c^{k+1} and c^{k-1} of the scheme).  kappa_prev multiplies the Laplacian of
 * u^{n-1} and kappa_next that of u^{n+1} (device nx*ny fields of the handle's
 * dtype, the coefficient kappa = c^2 itself; NULL = the handle's current
 * coefficient).  In delta form the step solves
 *   (I - beta K^{n+1} Lxx)(I - beta K^{n+1} Lyy) delta
 *       = dt^2 f + beta (2 K^{n+1} Lap u^n + (K^{n-1} - K^{n+1}) Lap u^{n-1}),
 * beta = dt^2 / 2, and u^{n+1} = 2u^n - u^{n-1} + delta is written over u^{n-1};
 * the pointers rotate as in adi_wave_step (one step).  f: this step's source
 * values (count values, already divided by h^2); rec: traces of u^{n+1} (count
 * values).  kappa_next becomes the handle's coefficient (its pivots and chunk
 * planes are rebuilt on the stream); the one-pass step stays off until the next
 * adi_wave_set_kappa, which measures the coefficient again.  Uses the exact
 * two-pass kernels; the first call allocates two nx*ny fields of workspace. */
adi_status adi_wave_step_tdc(adi_wave_t w, void** u_prev, void** u_curr, const void* kappa_prev,
                             const void* kappa_next, const adi_source* f, const adi_receivers* rec);

/* Paper-fidelity modes: one pair of sub-steps of the ADI split exactly as
 * printed.  Levels sit on half steps; the x-sub-step takes (u^{k-1/2}, u^k) to
 * u^{k+1/2} and the y-sub-step (u^k, u^{k+1/2}) to u^{k+1}, each a three-level
 * scheme with the tau^2 denominator and one direction's second difference:
 *   ADI_SPLIT_FR      eqs. (fr1)-(fr2) of Sec. 2: weights 1/2 on the new and the
 *                     oldest level of each sub-step;
 *   ADI_SPLIT_THETA1  the line systems of Listing 1 (Sec. 3.2: a = c = tau^2,
 *                     b = 2 tau^2 + h^2): weight 1 on the new level, a right-hand
 *                     side from the two older levels only (kappa and f enter as
 *                     kappa tau^2 on the second difference and tau^2 f).
 * u_half: device nx*ny, u^{k-1/2} on entry and u^{k+1/2} on return; u_curr: u^k
 * on entry and u^{k+1} on return (distinct buffers of the handle's dtype; no
 * pointer rotation).  f: sources of f^k for the x-sub-step, f_half: of
 * f^{k+1/2} for the y-sub-step (count values each, already divided by h^2, or
 * NULL); rec: receivers sampled from u^{k+1} (count values).  The lines are
 * solved by cyclic reduction, one launch per level (the first call allocates
 * 3 nx*ny values).  Neither mode is the scheme of adi_wave_step: the printed
 * split moves waves sqrt(2) times too fast and Listing 1's system is first
 * order and dissipative; they reproduce the paper's formulas for comparison. */
typedef enum {
    ADI_SPLIT_FR = 1,
    ADI_SPLIT_THETA1 = 2
} adi_split_mode;
adi_status adi_wave_step_split(adi_wave_t w, int mode, void* u_half, void* u_curr, const adi_source* f,
                               const adi_source* f_half, const adi_receivers* rec);

/* ------------------------------------------------------ batched simulations -- */

/* Many independent simulations of uneven grid sizes advanced together: each
 * step of the batch advances every simulation by one ADI step (the scheme of
 * Sec. 2, eq. (CN1) split as eqs. (fr1)-(fr2), on its own grid of eq. (f6),
 * spacing, time step and coefficient; the batching itself is not in the
 * paper), with one
 * launch per kernel for the whole batch over a work list of (simulation,
 * tile) items.  No sources or receivers. */
typedef struct adi_batch_s* adi_batch_t;

/* count simulations; nx, ny, h, dt: host arrays of count entries.
 * speed: host array of count device pointers to speed fields (nx[s]*ny[s]
 * values) with NULL entries meaning "use speed_scalar[s]"; speed may be NULL
 * (then speed_scalar is required).  Limits as for adi_wave_create, and the
 * widest grid fixes the launch plan.  Synchronises the stream. */
adi_status adi_batch_create(adi_batch_t* out, int count, const int* nx, const int* ny,
                            const double* h, const double* dt, const void* const* speed,
                            const double* speed_scalar, adi_dtype dtype, void* hip_stream);

/* Bind the two time levels of every simulation (host arrays of count device
 * pointers, u^{n-1} and u^n); uploads the descriptor table and synchronises
 * the stream.  Resets the step parity and drops a captured graph. */
adi_status adi_batch_bind(adi_batch_t b, void* const* u_prev, void* const* u_curr);

/* u^1 from u^0 for every simulation (psi = 0): reads the bound u_prev[s]
 * as u^0 and writes u_curr[s].  Only before the first step after a bind. */
adi_status adi_batch_start(adi_batch_t b, int mode);

/* nsteps steps of every simulation; the roles of the two bound levels rotate
 * (adi_batch_levels reports them).  Replays the captured graph when present. */
adi_status adi_batch_step(adi_batch_t b, int nsteps);

/* Current roles after the steps so far: fills u_prev[s], u_curr[s]. */
adi_status adi_batch_levels(adi_batch_t b, void** u_prev, void** u_curr);

/* enable = 1: capture two steps (both level parities) in a hipGraph that
 * adi_batch_step replays; enable = 0: drop it. */
adi_status adi_batch_graph(adi_batch_t b, int enable);

typedef struct {
    int x_threads_per_line;   /* line-group width of the x-sweep */
    int x_grid;               /* workgroups of each persistent launch (0 = one per work unit) */
    int yscan_grid;
    int ysolve_grid;
    int graph;                /* 1 if a captured graph is replayed (read-only) */
    int count;                /* simulations (read-only) */
    long long nodes;          /* total grid nodes (read-only) */
    size_t workspace_bytes;   /* device bytes owned by the batch (read-only) */
    int x_items, yscan_items, ysolve_items;   /* work-list lengths (read-only) */
    int fused_step;           /* 1: one-pass step for every simulation (FP32, when each
                                 simulation's truncation bound holds; the default then),
                                 2 (set only): exact two-pass step, 0 (set): keep */
    int fused_allowed;        /* read-only: the one-pass step is allowed for the batch */
    int fused_items;          /* read-only: one-pass work items (tiles or strip segments)
                                 over all simulations */
    int fused_lane_nodes;     /* one-pass tiles: x-line nodes per lane, 8 (default) or 4
                                 (narrower tiles with r kept in LDS), 0 (set) = keep */
    int fused_strips;         /* 1: the one-pass step on column strips instead of tiles
                                 (each simulation's fewest strips of at most 240 columns, of
                                 one width, in segments of at most 1024 rows), 0 (get): on
                                 tiles; set: 1 = strips, 2 = tiles, 0 = keep.  The
                                 autotuner times both tile kinds and the strips */
} adi_batch_plan;
adi_status adi_batch_get_plan(adi_batch_t b, adi_batch_plan* p);
adi_status adi_batch_set_plan(adi_batch_t b, const adi_batch_plan* p);

/* Autotuner: times candidate plans (line-group width, then each launch's
 * persistent grid size) for trial_steps steps on scratch levels it allocates
 * and frees, keeps the fastest plan and returns its milliseconds per step.
 * The bound levels are not touched.  Synchronises the stream. */
adi_status adi_batch_autotune(adi_batch_t b, int trial_steps, double* best_ms_per_step);

adi_status adi_batch_destroy(adi_batch_t b);

/* ------------------------------------------------------- batched line solve -- */

/* Solve `batch` independent tridiagonal systems of size n: the batched line
 * solve of Sec. 3.1 (Algorithm 1 solves one such system per grid line, by cyclic
 * reduction; here any strictly diagonally dominant systems, in any of the
 * layouts below):
 *   a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k],  k = 0..n-1
 * (a[0] and c[n-1] are ignored).  Element k of system s is at offset
 * s*sys_stride + k*elem_stride (in elements) in each of a, b, c, d (device,
 * dtype).  The solution overwrites d; a, b, c are not modified.  No pivoting:
 * the systems must be solvable by Gaussian elimination without pivoting
 * (e.g. strictly diagonally dominant), as the paper's line systems are.
 * Contiguous systems (elem_stride == 1, n <= 16384 / 8192 for f64) are solved
 * one per workgroup on chip.  Other layouts take a partition solve in three
 * launches (chunks of 32 rows for f32, 16 for f64, eliminated onto their last
 * row; the chunk-boundary system, solved by a second partition level with up to
 * 64 threads per system, or by one thread per system when it has more than 1024
 * rows; then the chunks again),
 * with a library workspace of 6*ceil(n/chunk)*batch values allocated on first
 * use (or growth) and kept; a call that needs more synchronises the stream
 * before it replaces the workspace, and ADI_ENOMEM if that allocation fails.
 * hip_stream: stream to queue on (NULL = default). */
adi_status tridiag_solve_batched(adi_dtype dtype, int n, int batch, const void* a,
                                 const void* b, const void* c, void* d,
                                 long long sys_stride, long long elem_stride,
                                 void* hip_stream);

/* The same solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): identical
 * arguments, kernels and results, but no allocation ever.  Where the partition
 * solve needs its workspace, it uses a fixed device array of 64 MiB built into
 * the library (one copy per device, held until the process ends) instead of
 * allocating one: a layout that needs more (6*ceil(n/chunk)*batch values) is
 * rejected with ADI_EINVAL before anything is queued.  Every call on a device
 * shares that device's array, so calls that overlap in time on one device
 * (different streams or host threads) race and must be serialised by the
 * caller; calls queued on one stream are ordered and safe.  The first call on
 * a device looks the array's address up (no allocation). */
adi_status tridiag_solve_batched_noalloc(adi_dtype dtype, int n, int batch, const void* a,
                                         const void* b, const void* c, void* d,
                                         long long sys_stride, long long elem_stride,
                                         void* hip_stream);

/* ------------------------------------------------------ introspection/timing -- */

typedef struct {
    int nx, ny;
    int dtype;
    int x_threads_per_line;   /* x-sweep: threads cooperating on one x-line (8 nodes each) */
    int x_rows_per_strip;     /* x-sweep: consecutive rows per thread group */
    int y_fused;              /* 1: y-chunk elimination fused into the x-sweep */
    int y_chunk_rows;         /* y-lines are split in chunks of this many rows */
    int y_chunks;             /* number of chunks per y-line */
    int kernels_per_step;     /* launches queued per ADI step */
    size_t workspace_bytes;   /* device bytes owned by the handle */
    int fused_step;           /* 1: adi_wave_step runs the one-pass step */
    int fused_allowed;        /* 1: the one-pass step's truncation bound holds (FP32:
                                 r_max <= 0.18 and nx % 4 == 0; FP64: r_max <= 0.13 and nx
                                 even) */
    double r_max;             /* largest r = dt^2 kappa / (2 h^2) */
    int line_solver;          /* 1: partition / scan solvers, 2: cyclic-reduction baseline */
    int fused_tile_cols;      /* one-pass step: output columns per tile (64 rows each) or per
                                 column strip; chosen for the device's compute units unless
                                 set through adi_wave_set_tuning */
    int fused_tiles;          /* one-pass step: tiles, or strip segments, per step (one
                                 workgroup each) */
    int fused_lane_nodes;     /* one-pass step: x-line nodes per lane (8, or 4 on tiles of at
                                 most 240 columns whose r stays in LDS for the y-lines) */
    int fused_segment_rows;   /* one-pass step on column strips (chosen where every compute
                                 unit gets a segment of >= 256 rows): output rows per strip
                                 segment (fused_tile_cols wide, four nodes per lane);
                                 0 when the step runs on 64-row tiles */
    int fused_strips_wide;    /* column strips: the first this many are fused_tile_cols wide,
                                 the others 8 columns narrower (the automatic plan mixes the
                                 two widths to cover nx evenly) */
} adi_wave_info;

adi_status adi_wave_get_info(adi_wave_t w, adi_wave_info* info);

/* Override the launch configuration chosen at create (for the autotuner).
 * Any field <= 0 keeps the current value.  Reallocates chunk workspace if the
 * chunk size changes (synchronises the stream). */
typedef struct {
    int x_threads_per_line;   /* 64, 128, 256 or 1024, with 8 * threads >= nx */
    int x_rows_per_strip;     /* >= 1 (unfused plans; a fused strip is one y-chunk) */
    int y_fused;              /* 1 = fuse the y-chunk elimination into the x-sweep, 2 = separate */
    int y_chunk_rows;         /* 16 or 32 */
    int fused_step;           /* 1 = one-pass step when allowed (else ADI_EUNSUPPORTED),
                                 2 = exact two-pass step, 0 = keep */
    int line_solver;          /* 1 = partition / scan line solvers (default),
                                 2 = cyclic reduction, one launch per level for all lines
                                 of a sweep (the paper's Sec. 3.1 solver, as a same-GPU
                                 baseline; allocates 3 nx*ny values), 0 = keep */
    int fused_tile_cols;      /* one-pass tile width: a multiple of 8, at most 496 (240 with 4
                                 nodes per lane; FP64 column strips: at most 64); -1 = back
                                 to the automatic choice, 0 = keep */
    int fused_lane_nodes;     /* one-pass x-line nodes per lane: 8 or 4; -1 = back to the
                                 automatic choice (4 where the tiles come out narrow), 0 = keep */
    int fused_segment_rows;   /* one-pass step on column strips (at most 240 columns, four
                                 nodes per lane) with this many output rows per segment (>= 8),
                                 -2 = on 64-row tiles, -1 = back to the automatic choice, 0 = keep */
} adi_tuning;
adi_status adi_wave_set_tuning(adi_wave_t w, const adi_tuning* t);

/* Run nsteps steps exactly as adi_wave_step does, with HIP events around every
 * launch; on return (the stream is synchronised) ms_per_kernel[k] holds the
 * mean duration in milliseconds of launch kind k over the steps and names[k]
 * its name, for k < *nkinds (at most 8). */
adi_status adi_wave_profile(adi_wave_t w, void** u_prev, void** u_curr,
                            const adi_source* f, int nsteps, double* ms_per_kernel,
                            const char** names, int* nkinds);

/* Plain device copy kernel of `bytes` bytes (a multiple of 16, 16-byte aligned
 * pointers), for measuring achievable HBM bandwidth next to the solver. */
adi_status adi_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Message for the last non-OK status returned on this host thread. */
const char* adi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ADIWAVE_H */
