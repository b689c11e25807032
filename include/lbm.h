/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 multi-relaxation-time lattice
 * Boltzmann library.
 *
 * The scheme is the standard D2Q9 MRT model of Xu & Sagaut, "Optimal
 * low-dispersion low-dissipation LBM schemes for computational
 * aeroacoustics":
 *   evolution      f_i(x + v_i, t + 1) = f_i + Lambda_ij (f^eq_j - f_j)     (Sec. 2.1, Eq. blbs)
 *   relaxation     Lambda = M^{-1} S M, S = diag(0,0,0,s_e,s_eps,s_q,s_q,s_nu,s_nu)
 *                                                                         (Sec. 2.1; Sec. 2.3)
 *   equilibrium    m^eq = (rho, jx, jy, -2rho + 3|j|^2/rho, rho - 3|j|^2/rho,
 *                          -jx, -jy, (jx^2 - jy^2)/rho, jx jy/rho)         (Sec. 2.3)
 *   lattice        periodic nx x ny, unit spacing and time step             (Sec. 2.1; Sec. 5)
 *
 * Velocity order (fixes every population layout below):
 *   v_0=(0,0) v_1=(1,0) v_2=(0,1) v_3=(-1,0) v_4=(0,-1)
 *   v_5=(1,1) v_6=(-1,1) v_7=(-1,-1) v_8=(1,-1).
 *
 * Conventions that hold for every function:
 *   - Every function returns lbm_status (0 == LBM_OK) unless stated; nothing
 *     throws across the ABI.  On failure lbm_last_error() describes it.
 *   - "device pointer" = memory on the GPU the lattice lives on, "host
 *     pointer" = ordinary CPU memory.  Field arrays are contiguous, row-major
 *     [ny][nx] (x fastest) in IEEE double; population arrays are [9][ny][nx].
 *   - The caller owns every buffer, including the device workspace and the
 *     stream; the library owns only its host-side handle objects.
 *   - Functions marked "enqueued" only enqueue GPU work on the lattice's
 *     stream and return; functions marked "syncs" wait for that stream.
 *   - A handle is used from one host thread at a time.
 *   - The logical state at integer t is the pre-collision f(t).
 */
#ifndef LBM_H_
#define LBM_H_

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define LBM_API __attribute__((visibility("default")))
#else
#define LBM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK            0
#define LBM_E_INVAL      (-1)  /* invalid argument or descriptor                 */
#define LBM_E_NOMEM      (-2)  /* workspace too small / capacity exceeded         */
#define LBM_E_HIP        (-3)  /* a HIP runtime call failed                       */
#define LBM_E_NONFINITE  (-4)  /* diagnostics found non-finite populations        */
#define LBM_E_STATE      (-5)  /* call out of order (e.g. step before init)       */

/* Storage type of the population deviations held in HBM. */
#define LBM_STORE_F64   0
#define LBM_STORE_F32   1
#define LBM_STORE_F16   2
#define LBM_STORE_BF16  3
/* Arithmetic type of the collision. */
#define LBM_COMPUTE_F64 0
#define LBM_COMPUTE_F32 1

/* scale_exp value asking lbm_init_equilibrium to choose the storage scale. */
#define LBM_SCALE_AUTO  INT32_MIN

/*
 * Lattice descriptor.
 *   nx, ny      lattice size, >= 1 each; with pitch = nx rounded up to 64,
 *               pitch * ny < 2^31 and pitch * ny * sizeof(storage) < 2^32
 *               (one population plane below 4 GiB).
 *   storage     LBM_STORE_*.  The library stores the deviation
 *               g_i = (f_i - f^eq_i(rho0, u0)) * 2^scale_exp, i.e. the
 *               fluctuating part about the uniform state (Sec. 4.1, Eq.
 *               perturb-f), rounded to nearest even.
 *   compute     LBM_COMPUTE_*.  Allowed pairs: (F64,F64), (F64,F32),
 *               (F32,F32), (F16,F32), (BF16,F32).  With F64 storage and F32
 *               compute the increment of the collision is evaluated in F32
 *               and added to the stored value in F64.
 *   s_e, s_eps, s_q, s_nu
 *               relaxation rates, each in (0, 2]  (Sec. 2.1 stability range,
 *               widened to include 2 as in Sec. 3.2 and Table 4).
 *   rho0 > 0, u0x, u0y
 *               uniform base state of the deviation storage; any finite value
 *               is correct, values near the flow's mean minimise rounding.
 *   scale_exp   p in [-60, 60], or LBM_SCALE_AUTO (F16/BF16: chosen at init
 *               so that max|g| * 2^p is about 2^13; F64/F32: 0).
 *   flags       reserved, must be 0.
 */
typedef struct lbm_desc {
    int32_t nx, ny;
    int32_t storage;
    int32_t compute;
    double s_e, s_eps, s_q, s_nu;
    double rho0, u0x, u0y;
    int32_t scale_exp;
    int32_t flags;
} lbm_desc;

typedef struct lbm_lattice lbm_lattice;

/* Launch shape of the fused step kernel (chosen by lbm_tune or set by hand;
 * a new lattice of at least 2^19 cells starts with a several-steps shape by
 * storage type: FP32
 * {13, 64, 4, R, 1, 32}, FP16 {12, 64, 4, R, 1, 34}, BF16 {12, 64, 4, R, 1,
 * 40}, FP64 {13, 64, 4, R, 1, 32} (workgroup-shared halo, R chosen from the
 * lattice size so that three (FP32), four (FP16, BF16) or two (FP64)
 * workgroups per compute unit cover the lattice in one round, at least 8:
 * 92, 69, 69, 137 rows on 4096^2); a smaller one with {0, 64, 4, 1, 1, 0}).
 *   variant   0 = one cell per lane (nine direct loads),
 *             1, 2, 3 = 2, 4, 8 consecutive cells per lane (aligned vector
 *             loads, x-shift by cross-lane exchange; needs nx % 2^variant == 0
 *             and block_x % 64 == 0),
 *             4 = one cell per lane, each workgroup walks whole rows in chunks
 *             of block_x cells (row strips),
 *             5, 6, 7 = 2, 4, 8 consecutive cells per lane, x-shifted values
 *             taken from overlapping aligned vector loads (needs
 *             nx % 2^(variant-4) == 0)
 *             8 .. 13 = T = 2 .. 7 steps per launch (temporal blocking in
 *             registers): each wave of 64 lanes owns a strip of 64 - 2(T-1)
 *             columns, rounded down to whole 32-byte (else 16-byte) pieces
 *             of a stored row where that drops at most two columns, and a segment of
 *             `rows` rows; T = 5, 6 and 7 take no non-temporal loads, T = 7 no
 *             skewed pipeline; block_x must be 64,
 *             block_y (waves per workgroup) 1..4, rows 1..4096.  lbm_step(n)
 *             then makes n / T such launches and takes the remaining steps
 *             as described there (one-step launches use the one-step shape
 *             last set or found by lbm_tune).
 *   block_x   lanes along x per workgroup, block_y rows per workgroup pass;
 *             64 <= block_x * block_y <= 1024
 *   rows      rows each lane processes, 1..64 (tile height = block_y * rows)
 *   xcd_remap 1 = renumber workgroups so that neighbouring tiles run on the
 *             same XCD (shared L2), 0 = hardware order
 *   flags     bit 0: non-temporal loads; bit 1: issue the next row's (variants
 *             0 and 8-13) or next chunk's (variant 4) loads before colliding
 *             the current cells (variants 0, 4, 8-13 only); bit 2
 *             (variants 8-13 only): move values between neighbouring
 *             lanes with DPP whole-wave shifts instead of LDS shuffles; bit 3
 *             (variants 8-13 only, not with bit 1): issue the loads two
 *             rows ahead; bit 4 (variants 9-12 only, not with bit 0):
 *             skewed pipeline, in which stage p works two rows behind stage
 *             p-1 instead of one, so that the T collisions of a row
 *             iteration do not depend on each other; bit 5 (variants
 *             10-13 with flags 32, 34, 40, or with bit 4 set, 48, 50, 56;
 *             FP64 storage: variants 12-13, flags 32, 34, 40):
 *             workgroup-shared halo -- the block_y waves of a workgroup
 *             own one strip of 64 block_y - 2(T-1) columns (rounded as
 *             above) and pass the values a stage takes from the
 *             neighbouring column through LDS (with a workgroup barrier per
 *             stage; with bit 4, one per row through two alternating
 *             buffers), so that only the workgroup's outer edges recompute
 *             a halo.
 * Every shape produces bit-identical results. */
typedef struct lbm_launch {
    int32_t variant;
    int32_t block_x;
    int32_t block_y;
    int32_t rows;
    int32_t xcd_remap;
    int32_t flags;
} lbm_launch;

/* ---- status and helpers ------------------------------------------------ */

/* Static text for a status code; never NULL. */
LBM_API const char *lbm_status_string(lbm_status s);
/* Message of the most recent failure on the calling thread ("" if none). */
LBM_API const char *lbm_last_error(void);
/* s_nu = 1 / (3 nu + 1/2): sigma = 1/s - 1/2 (Sec. 2.3) and nu = sigma_nu / 3
 * (first-order dissipation matrix, Sec. 2.3.1; Table 4 prints both).
 * Returns NaN for nu outside [0, inf). */
LBM_API double lbm_s_from_nu(double nu);

/* ---- single lattice ---------------------------------------------------- */

/* Device workspace bytes a lattice with this descriptor needs: two
 * population buffers [9][ny][pitch] of the storage type (pitch = nx rounded
 * up to 64 elements), reduction scratch and padding.  0 if invalid. */
LBM_API size_t lbm_workspace_bytes(const lbm_desc *desc);

/* Creates a lattice handle on the current HIP device.
 *   dev_ws    device pointer, 256-byte aligned, >= lbm_workspace_bytes(desc)
 *             bytes, owned by the caller and not freed by lbm_destroy.
 *   stream    hipStream_t to enqueue on (NULL = the null stream).
 *   out       receives the handle.
 * Errors: LBM_E_INVAL (descriptor, alignment), LBM_E_NOMEM (ws_bytes). */
LBM_API lbm_status lbm_create(const lbm_desc *desc, void *dev_ws, size_t ws_bytes, void *stream,
                      lbm_lattice **out);
/* Releases the handle (not the workspace).  Does not wait for the stream. */
LBM_API lbm_status lbm_destroy(lbm_lattice *lat);
/* Replaces the stream used by later calls. */
LBM_API lbm_status lbm_set_stream(lbm_lattice *lat, void *stream);
/* Copies the descriptor, with scale_exp resolved once init has run. */
LBM_API lbm_status lbm_get_desc(const lbm_lattice *lat, lbm_desc *out);

/* Equilibrium initialisation from macroscopic fields (Sec. 5.2 initial
 * condition): f(x, 0) = M^{-1} m^eq(rho, rho u).  rho, ux, uy: device
 * pointers [ny][nx] FP64; rho must be > 0 and all values finite (not checked
 * on the device; non-finite input shows up in lbm_diagnostics).  Sets t = 0.
 * Enqueued; syncs once when scale_exp is LBM_SCALE_AUTO. */
LBM_API lbm_status lbm_init_equilibrium(lbm_lattice *lat, const double *rho, const double *ux,
                                const double *uy);

/* Advances n >= 0 steps of the fused collide-and-pull-stream update
 * (Sec. 2.1, Eq. blbs with Lambda = M^{-1} S M; pull form of Sec. 2.2, Eq.
 * l-mrt-lbs).  Enqueued.  LBM_E_STATE before init.  With a shape of T > 1
 * steps per launch: n / T launches of it, then the r = n % T remaining
 * steps in one launch of the same shape with r steps per pass (variant
 * 6 + r) when r >= 2 and that shape is supported (for a shared-halo shape
 * with r < 4: the same with one wave per strip and flags 2), else r one-step
 * launches; every split gives bit-identical results. */
LBM_API lbm_status lbm_step(lbm_lattice *lat, int64_t n);
/* Kernel launches lbm_step(lat, n) makes with the current shapes; -1 if
 * lat is NULL or n < 0. */
LBM_API int64_t lbm_step_launches(const lbm_lattice *lat, int64_t n);

/* Macroscopic fields of the current state (Sec. 2.1, Eq. q-macro):
 * rho = sum_i f_i, u = (sum_i v_i f_i) / rho, evaluated in FP64.
 * rho, ux, uy: device pointers [ny][nx] FP64.  Enqueued. */
LBM_API lbm_status lbm_read_moments(lbm_lattice *lat, double *rho, double *ux, double *uy);

/* Global FP64 diagnostics of the current state (host pointer out[4]):
 *   out[0] = sum_x (rho - rho0), out[1] = sum_x (jx - rho0 u0x),
 *   out[2] = sum_x (jy - rho0 u0y)   (the collision invariants of Sec. 2.1,
 *   Eq. eq_conservative; constant in exact arithmetic),
 *   out[3] = number of non-finite stored values.
 * Syncs.  Returns LBM_E_NONFINITE when out[3] > 0 (out is still filled). */
LBM_API lbm_status lbm_diagnostics(lbm_lattice *lat, double out[4]);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops): the diagnostics of lbm_diagnostics for a raw state held by
 * the caller, with no lattice handle and no workspace.
 *   desc       describes the state's lattice (validated as by lbm_create, so
 *              lattices beyond the library's size limits are rejected with
 *              LBM_E_INVAL); for F16/BF16 storage scale_exp must be the
 *              state's explicit scale (lbm_get_desc of the lattice it came
 *              from), LBM_SCALE_AUTO is rejected.
 *   dev_state  device pointer to the raw state in the layout lbm_save_state
 *              writes: [9][ny][pitch] values of the storage type, pitch = nx
 *              rounded up to 64 (columns nx..pitch-1 are not read).
 *   dev_out    device pointer to 4 doubles, filled as out[] of
 *              lbm_diagnostics.
 *   stream     hipStream_t of the current device (NULL = null stream).
 * Enqueued; never waits, allocates nothing (no hipMalloc, no workspace).
 * The reduction's partial sums live in a library-owned static device array
 * of 82,432 bytes per GPU (LBM_NOALLOC_SCRATCH_BYTES), held until the
 * process ends; its need does not grow with the lattice.  Every call on one
 * GPU shares that array: calls that overlap on one GPU (different streams
 * without ordering) race and give wrong sums.  Each call rewrites every
 * partial it reads, so nothing carries over from an earlier call. */
#define LBM_NOALLOC_SCRATCH_BYTES 82432
LBM_API lbm_status lbm_diagnostics_noalloc(const lbm_desc *desc, const void *dev_state, double *dev_out,
                                           void *stream);

/* FP64 Fourier projection of the population deviations onto the lattice mode
 * k = 2 pi (mx / nx, my / ny), the plane-wave amplitudes of the von Neumann
 * analysis (Sec. 4.1, Eq. perturb-w-f):
 *   dev_out[2i] + I dev_out[2i+1] = sum_x (f_i(x,t) - f^eq_i(rho0,u0)) e^{-I k.x},
 * i = 0..8 (18 doubles, device pointer).  Enqueued. */
LBM_API lbm_status lbm_project(lbm_lattice *lat, int32_t mx, int32_t my, double *dev_out);

/* Pre-collision populations f(t) as FP64, device pointer [9][ny][nx].  Enqueued. */
LBM_API lbm_status lbm_read_populations(lbm_lattice *lat, double *dev_f);
/* Replaces the state by FP64 populations (rounded to the storage type);
 * t is left unchanged.  Enqueued. */
LBM_API lbm_status lbm_write_populations(lbm_lattice *lat, const double *dev_f);

/* Imposes the equilibrium f(x, y, t) = f^eq(rho, rho u) on one node of the
 * current (pre-collision) state: the point source of Sec. 5.1 prescribes the
 * density of a node every step with zero velocity.  Call it after each
 * lbm_step.  rho > 0, all finite, 0 <= x < nx, 0 <= y < ny.  Enqueued. */
LBM_API lbm_status lbm_set_node_equilibrium(lbm_lattice *lat, int32_t x, int32_t y, double rho, double ux,
                                            double uy);

/* Bytes of the raw state: the current buffer in its storage type, laid out
 * [9][ny][pitch] with pitch = nx rounded up to 64 elements (the values of
 * columns nx..pitch-1 are unspecified). */
LBM_API size_t lbm_state_bytes(const lbm_lattice *lat);
/* Bitwise checkpoint of the raw state into / from a device buffer of
 * lbm_state_bytes bytes; load also sets t.  Enqueued. */
LBM_API lbm_status lbm_save_state(lbm_lattice *lat, void *dev_dst);
LBM_API lbm_status lbm_load_state(lbm_lattice *lat, const void *dev_src, int64_t t);

/* Steps taken since init (or the t given to lbm_load_state). */
LBM_API int64_t lbm_time(const lbm_lattice *lat);

/* Launch shape of the step kernel for this lattice. */
LBM_API lbm_status lbm_get_launch(const lbm_lattice *lat, lbm_launch *out);
/* LBM_E_INVAL if the shape is not supported for this lattice. */
LBM_API lbm_status lbm_set_launch(lbm_lattice *lat, const lbm_launch *cfg);
/* Times the supported launch shapes on this lattice (reps launches each,
 * the state is left unchanged) and selects the one with the least time per
 * step; the fastest one-step shape is kept for a single left-over step
 * (see lbm_step for the rest).  best_us
 * receives microseconds per step.  best/best_us may be NULL.  Syncs. */
LBM_API lbm_status lbm_tune(lbm_lattice *lat, int32_t reps, lbm_launch *best, double *best_us);
/* Times n launches of the current shape (state unchanged; syncs); avg_us is
 * per launch, which covers lbm_steps_per_launch steps. */
LBM_API lbm_status lbm_time_launches(lbm_lattice *lat, int32_t n, double *avg_us);
/* Steps one launch of this shape advances (1, or T for variants 8-13);
 * 0 if cfg is NULL.  Does not validate the shape. */
LBM_API int32_t lbm_steps_per_launch(const lbm_launch *cfg);

/* ---- pools: many lattices advanced together ------------------------------
 *
 * A pool advances its members (lattices of any size, rates and storage)
 * with persistent launches per storage class: with steps_per_launch T > 1
 * one launch advances every member by T steps (strip tasks of the
 * several-steps-per-pass kernel, see lbm_launch variants 8-13) and a member
 * whose remaining count is not a multiple of T takes its last steps in
 * one-step launches; step loops of T 2^m steps up to graph_steps (at the
 * end of a run, the r < T remaining steps as one pass of r steps), each with
 * as many one-step launches as its members need, are recorded once as HIP
 * graphs and replayed (lbm_pool_step(n) runs n steps as a few such replays).
 * The members of a class are split into two groups of about equal cell
 * counts whose launches form independent chains in the recorded loop
 * (members never read each other's state), so the end of one group's
 * launch overlaps the next launch of the other.  Each
 * member carries its own step count: a member added with nsteps stops after
 * exactly nsteps steps, independently of the others, and is then returned by
 * lbm_pool_poll.  Members join and leave between lbm_pool_step calls
 * (continuous batching).  A lattice gives bit-identical results alone or in
 * a pool (same per-cell arithmetic).
 *
 * While a lattice is in a pool, every lattice call that reads or changes its
 * state returns LBM_E_STATE.  Ordering: lbm_pool_add makes the pool's stream
 * wait for work already enqueued on the lattice's stream; lbm_pool_poll and
 * lbm_pool_remove make the lattice's stream wait for the pool's stream, so
 * readback enqueued afterwards on the lattice's stream sees the final state. */

typedef struct lbm_pool lbm_pool;

/* Launch shape of a pool.
 *   tile_cells   target cells per tile of the one-step launch (a tile is
 *                whole rows of one member: max(1, tile_cells / nx) rows),
 *                64 .. 2^22
 *   block        threads per workgroup of the one-step launch, multiple of
 *                64, 64 .. 1024
 *   grid         workgroups of a persistent launch (both kinds), 1 .. 2^20
 *   graph_steps  longest recorded step loop (a loop is T 2^m steps, or
 *                fewer than T), 1 .. 1024
 *   steps_per_launch  T = 1, 2, 4, 5, 6 or 7; T > 1 adds strip tasks (columns
 *                as for lbm_launch variants 8-13) of seg_rows rows, one wave
 *                each
 *   seg_rows     rows of a strip task, 1 .. 4096: each member's ny rows are
 *                cut into max(1, round(ny / seg_rows)) segments of nearly
 *                equal height (they differ by at most one row)
 *   waves        waves per workgroup of the T-step launch, 1 .. 4
 *   flags        T-step kernel flags as in lbm_launch: 0, 2, 4 or 12 (one
 *                wave per strip task); or 32 or 34 (waves must be 4): one
 *                workgroup per strip task, its waves sharing the halo
 *                columns through LDS as for lbm_launch variants 10-13 with
 *                flag 32 (34 also loads one row ahead): four-wave strips of
 *                64 * 4 - 2(T-1) columns (rounded as there) from column 0,
 *                and the columns left over in one more, narrower,
 *                four-wave strip; or 96 or 98 (32 or 34 plus bit 6): the
 *                same, except that left-over columns that fit one
 *                two-wave strip (64 * 2 - 2(T-1) columns, rounded alike)
 *                go to one, run as a second launch beside the first.
 * The tile table holds the one-step tiles and, for T > 1, the strip tasks
 * of every unfinished member. */
typedef struct lbm_pool_shape {
    int32_t tile_cells;
    int32_t block;
    int32_t grid;
    int32_t graph_steps;
    int32_t steps_per_launch;
    int32_t seg_rows;
    int32_t waves;
    int32_t flags;
} lbm_pool_shape;

/* Device bytes of a pool's member and tile tables; 0 if out of range
 * (max_members in [1, 2^20], max_tiles in [1, 2^26]). */
LBM_API size_t lbm_pool_workspace_bytes(int32_t max_members, int32_t max_tiles);
/* Creates a pool.  dev_ws: device pointer, 256-byte aligned, at least
 * lbm_pool_workspace_bytes bytes, owned by the caller; stream: the pool's
 * hipStream_t.  Allocates pinned host staging for the tables.  Initial
 * shape {256, 512, 4096, 256, 7, 96, 4, 32} (seven steps per launch, one
 * workgroup of four waves per strip task). */
LBM_API lbm_status lbm_pool_create(void *dev_ws, size_t ws_bytes, void *stream, int32_t max_members,
                                   int32_t max_tiles, lbm_pool **out);
/* Returns every member to its lattice (as lbm_pool_remove) and frees the
 * handle; does not free dev_ws. */
LBM_API lbm_status lbm_pool_destroy(lbm_pool *pool);
/* Adds an initialised lattice that will advance nsteps >= 0 more steps.
 * LBM_E_NOMEM when the member or tile table is full. */
LBM_API lbm_status lbm_pool_add(lbm_pool *pool, lbm_lattice *lat, int64_t nsteps);
/* Takes a member out before it is done; its time is the steps taken so far. */
LBM_API lbm_status lbm_pool_remove(lbm_pool *pool, lbm_lattice *lat);
/* Advances every member by min(nsteps, its remaining steps).  Enqueued. */
LBM_API lbm_status lbm_pool_step(lbm_pool *pool, int64_t nsteps);
/* Returns up to cap members whose steps are done and whose last step has
 * completed on the device; they leave the pool.  wait != 0 blocks until at
 * least the oldest finished member has completed (if there is one). */
LBM_API lbm_status lbm_pool_poll(lbm_pool *pool, lbm_lattice **done, int32_t cap, int32_t wait,
                                 int32_t *ndone);
/* Members currently held (including finished ones not yet polled). */
LBM_API int32_t lbm_pool_members(const lbm_pool *pool);
/* Steps a member still has to take, or -1 if it is not in the pool. */
LBM_API int64_t lbm_pool_remaining(const lbm_pool *pool, const lbm_lattice *lat);
LBM_API lbm_status lbm_pool_get_shape(const lbm_pool *pool, lbm_pool_shape *out);
/* LBM_E_INVAL for an invalid shape, LBM_E_NOMEM if the tiles would not fit. */
LBM_API lbm_status lbm_pool_set_shape(lbm_pool *pool, const lbm_pool_shape *shape);
/* Times reps launches that advance every member by one launch's worth of
 * steps (steps_per_launch; states unchanged; syncs); avg_us per launch. */
LBM_API lbm_status lbm_pool_time_launches(lbm_pool *pool, int32_t reps, double *avg_us);
/* Times tile sizes, workgroup sizes, grid sizes and T-step strip shapes on
 * the current members, keeps the one with the least time per step (states
 * unchanged; syncs); best_us is per step. */
LBM_API lbm_status lbm_pool_tune(lbm_pool *pool, int32_t reps, lbm_pool_shape *best, double *best_us);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H_ */
