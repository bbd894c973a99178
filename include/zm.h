/*
 * zm.h -- C ABI of the MI355X Z-Model high-order step library (libzm.so).
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the hot path of
 * the Z-Model Rayleigh-Taylor interface solver that the Beatnik
 * mini-application is built on (Stewart & Bridges, 2024):
 *
 *   state      per mesh point a position z = (z1, z2, z3) and two vorticity
 *              components w = (w1, w2) on a regular n1 x n2 mesh
 *              (sec. 2, SurfaceMesh; sec. 3.1, ProblemManager);
 *   BR velocity  the Birkhoff-Rott velocity of every point from the position
 *              and vorticity of every point (sec. 2, BRSolver), evaluated by
 *              brute force over all pairs (sec. 3.2.1, exact integral);
 *   derivatives  surface tangents and Laplacians by two-node-deep stencils
 *              with periodic coordinate correction (sec. 3.1, SurfaceMesh
 *              and BoundaryCondition), and the position/vorticity time
 *              derivatives (sec. 2, ZModel);
 *   step       third-order Runge-Kutta, three derivative evaluations per
 *              step (sec. 3.1, TimeIntegrator).
 *
 * The paper prints no equations.  The library implements this reading:
 *   mesh       doubly periodic, period L_a, spacing h_a = L_a / n_a,
 *              point index p = i2 * n1 + i1;
 *   D_a f      [8 (f(i+1) - f(i-1)) - (f(i+2) - f(i-2))] / (12 h_a), indices
 *              periodic, z1 (z2) gains +-L1 (+-L2) when the stencil crosses
 *              the seam along axis 1 (2);
 *   gamma      w1 T2 - w2 T1 with T_a = D_a z (BR source strength);
 *   u_i        -(h1 h2 / 4 pi) sum_j sum_images c (r x gamma_j) /
 *              (|r|^2 + eps^2)^(3/2),  r = z_i - z_j - (s1 L1, s2 L2, 0),
 *              image chosen by the index offset j_a - i_a reduced into the
 *              period cell centred on i; when n_a is even and the offset is
 *              exactly n_a/2 both end images count with weight 1/2; with
 *              image_layers = K > 0 the shifts (s1+m1, s2+m2),
 *              m in [-K, K]^2, are all summed;
 *   cutoff     with cutoff = rc > 0 (sec. 3.2.2, cutoff-based approximate
 *              integral) the same sum runs only over the sources whose
 *              nearest periodic image (per axis the integer S_a nearest to
 *              (z_i,a - z_j,a) / L_a) lies within the 3D distance rc:
 *              r_a = (z_i,a - z_j,a) - S_a L_a, included iff
 *              r1*r1 + r2*r2 + r3*r3 < rc*rc (evaluated in that order in
 *              double), weight 1, no ties, rc <= 0.45 min(L1, L2), K = 0;
 *              on a free sheet S_a = 0 (r = z_i - z_j) and any rc > 0;
 *   free sheet with boundary = ZM_BOUNDARY_FREE (sec. 3.1, BoundaryCondition:
 *              non-periodic values are extrapolated into the boundary cells)
 *              the stencils take ghost values from a cubic extrapolation,
 *              g(-1) = 4 g0 - 6 g1 + 4 g2 - g3, g(-2) = 10 g0 - 20 g1 + 15 g2
 *              - 4 g3 (and mirrored at the far end), for z, w and V, and
 *              the BR sum has no images and no ties (r = z_i - z_j),
 *              exact or with a cutoff;
 *   low order  with model = ZM_MODEL_LOW the BR sum is replaced by its
 *              flat-sheet approximation (sec. 2: the low-order solver uses
 *              FFTs for the BR integral): u = 1/2 (R1 w1 + R2 w2) n^ with
 *              n^ = T1 x T2 / |T1 x T2| and R_a the Riesz transform over the
 *              periodic mesh, symbol i k_a / |k| on exp(i k.alpha),
 *              k_a = 2 pi m_a / L_a, zero at k = 0 and, along axis a, at the
 *              unpaired mode m_a = n_a / 2;
 *   medium     with model = ZM_MODEL_MEDIUM (sec. 2: the medium order
 *              couples the FFT solver with the BR solver; sec. 6: it uses
 *              the FFTs for the change in vorticity) z_t = u is the BR
 *              velocity (exact or cutoff) and the |u|^2 of V is that of the
 *              low-order FFT velocity; periodic sheets, sides powers of two
 *              <= 4096; zm_br_velocity returns the BR velocity;
 *   q          |gamma|^2 / |T1 x T2|^2;
 *   V          A (|u|^2 - q/4 - 2 g z3);
 *   F(z, w)    z_t = u,  w_t = (D_1 V, D_2 V) + nu Lap(w);
 *   RK3        y1 = y0 + dt F(y0); y2 = 3/4 y0 + 1/4 (y1 + dt F(y1));
 *              y3 = 1/3 y0 + 2/3 (y2 + dt F(y2))  (Shu-Osher SSP-RK3).
 *
 * Conventions for every entry point
 *   - Device pointers (d_*) are caller-owned device memory on the device
 *     current when the context was created, float64, 256-byte aligned,
 *     structure-of-arrays planes: z is 3 planes of N = n1*n2 doubles
 *     (z1 plane, z2 plane, z3 plane), w is 2 planes, u is 3 planes.
 *   - The library never allocates device memory.  All scratch lives in the
 *     caller's workspace of zm_workspace_bytes() bytes, except that of
 *     zm_br_velocity_noalloc, which lives in a static device array.
 *   - Work is enqueued asynchronously on the stream given to zm_create (a
 *     hipStream_t, or NULL for the null stream).  Results are visible after
 *     that stream is synchronised.
 *   - Arguments are validated before anything is enqueued; a rejected call
 *     has no side effects.  No C++ exception crosses this interface.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef ZM_H
#define ZM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
typedef int32_t zm_status;
#define ZM_OK               0
#define ZM_ERR_INVALID_ARG (-1)  /* bad parameter or pointer                    */
#define ZM_ERR_UNSUPPORTED (-2)  /* valid request this build does not provide   */
#define ZM_ERR_WORKSPACE   (-3)  /* workspace missing, too small or misaligned  */
#define ZM_ERR_HIP         (-4)  /* a HIP runtime call or kernel launch failed  */
#define ZM_ERR_NONFINITE   (-5)  /* state became non-finite (check-finite flag) */
#define ZM_ERR_CAPACITY    (-6)  /* request exceeds a fixed capacity            */

/* ---- precision of the pair interactions ---------------------------------- */
#define ZM_FP64        0  /* all arithmetic in float64                          */
#define ZM_FP32_PAIRS  1  /* pair terms in float32 on tile-relative coordinates;
                             per-target sums, state, ties and RK3 in float64   */

/* ---- model order ----------------------------------------------------------- */
#define ZM_MODEL_HIGH  0  /* u from the Birkhoff-Rott sum (exact or cutoff)      */
#define ZM_MODEL_LOW   1  /* u = 1/2 (R1 w1 + R2 w2) n^ by FFT (low order)       */
#define ZM_MODEL_MEDIUM 2 /* z_t from the BR sum, |u|^2 in V from the FFT one   */

/* ---- boundary of the sheet -------------------------------------------------- */
#define ZM_BOUNDARY_PERIODIC 0  /* doubly periodic (images, seam correction)    */
#define ZM_BOUNDARY_FREE     1  /* non-periodic: ghosts extrapolated, no images */

/* ---- flags ---------------------------------------------------------------- */
#define ZM_FLAG_CHECK_FINITE 0x1u /* zm_step checks the state after each call
                                     and returns ZM_ERR_NONFINITE (this makes
                                     zm_step wait for its own work)            */
#define ZM_FLAG_GRAPH        0x2u /* zm_step captures one RK3 step into a HIP
                                     graph on first use and replays it (per-
                                     kernel timing, when enabled, uses the
                                     direct launches instead)                  */

/* ---- parameters ------------------------------------------------------------ */
typedef struct zm_params {
    int32_t  n1, n2;           /* mesh points per axis, 8 <= n_a <= 8192        */
    double   period1, period2; /* L1, L2 > 0 (parameter and x / y period)       */
    double   atwood;           /* A = (rho+ - rho-) / (rho+ + rho-)             */
    double   gravity;          /* g (acceleration -g e3)                        */
    double   eps;              /* desingularisation length, > 0                 */
    double   nu;               /* optional viscosity on w (0 = none), >= 0      */
    double   dt;               /* time step, > 0 (zm_step only)                 */
    int32_t  precision;        /* ZM_FP64 or ZM_FP32_PAIRS                      */
    int32_t  image_layers;     /* K >= 0 extra periodic image layers            */
    uint32_t flags;            /* ZM_FLAG_*                                     */
    int32_t  model;            /* ZM_MODEL_HIGH, ZM_MODEL_LOW (FP64, no cutoff,
                                  K = 0; sides powers of two <= 4096; single
                                  contexts only) or ZM_MODEL_MEDIUM (periodic,
                                  sides powers of two <= 4096; single contexts
                                  only)                                        */
    double   cutoff;           /* 0: exact all-pairs BR; > 0: cutoff BR with
                                  this 3D distance (FP64 only, K = 0; on a
                                  periodic sheet <= 0.45 min(L1, L2); single
                                  contexts only)                               */
    int32_t  boundary;         /* ZM_BOUNDARY_PERIODIC or ZM_BOUNDARY_FREE (free:
                                  high order, K = 0; single contexts only)     */
    int32_t  reserved;         /* must be 0                                     */
} zm_params;

typedef struct zm_ctx zm_ctx;  /* opaque */

/* Bytes of device workspace a context with these parameters needs (0 if the
 * parameters are invalid or the configuration is one zm_create refuses with
 * ZM_ERR_UNSUPPORTED).  Pure host function. */
size_t zm_workspace_bytes(const zm_params *params);

/* Create a context on the current device.  d_workspace: caller-owned device
 * memory of at least zm_workspace_bytes(params) bytes, 256-byte aligned, kept
 * alive and unused by the caller until zm_destroy.  hip_stream: the
 * hipStream_t all work is enqueued on (NULL = null stream).  On success *out
 * receives the context; on failure *out is set to NULL.
 * ZM_ERR_UNSUPPORTED for valid requests this library does not serve: FP32
 * cutoff; low order on sides that are not powers of two <= 4096 (also
 * medium order); and the FP32 pair form on meshes so anisotropic that a
 * pair patch spans more than 128 finest mesh spacings (its FP32
 * patch-relative coordinates would lose the 1e-5 bound there; FP64 serves
 * them). */
zm_status zm_create(zm_ctx **out, const zm_params *params,
                    void *d_workspace, size_t workspace_bytes, void *hip_stream);

/* Copy (d_z: 3 planes, d_w: 2 planes) into the context's state.  The inputs
 * may be freed or reused once the stream has passed this call. */
zm_status zm_init_state(zm_ctx *ctx, const double *d_z, const double *d_w);

/* One Birkhoff-Rott evaluation (pure function of its inputs, including the
 * tangents behind the source strength): d_u (3 planes) = u(d_z, d_w).
 * d_u must not overlap d_z or d_w.  The context state is not touched. */
zm_status zm_br_velocity(zm_ctx *ctx, const double *d_z, const double *d_w, double *d_u);

/* One evaluation of F: d_zt (3 planes) = u, d_wt (2 planes) = D V + nu Lap w.
 * Outputs must not overlap inputs.  The context state is not touched. */
zm_status zm_rhs(zm_ctx *ctx, const double *d_z, const double *d_w,
                 double *d_zt, double *d_wt);

/* Advance the context state by nsteps >= 0 RK3 steps of size params.dt. */
zm_status zm_step(zm_ctx *ctx, int32_t nsteps);

/* Copy the context state out (d_z: 3 planes, d_w: 2 planes). */
zm_status zm_get_state(zm_ctx *ctx, double *d_z, double *d_w);

/* Wait for the context's outstanding work and release its host resources.
 * The workspace may be freed afterwards.  NULL is accepted. */
zm_status zm_destroy(zm_ctx *ctx);

/* Static description of a status code. */
const char *zm_status_string(zm_status status);

/* Message of the last error on this context ("" if none; NULL ctx: the last
 * error of a failed zm_create or zm_br_velocity_noalloc on this thread). */
const char *zm_last_error(const zm_ctx *ctx);

/* ---- launch configuration and per-kernel timing ------------------------- */

typedef struct zm_launch_info {
    int32_t targets_per_lane;   /* register-blocked targets per thread       */
    int32_t patch_cols;         /* target patch: columns (axis 1)            */
    int32_t patch_rows;         /* target patch: rows (axis 2)               */
    int32_t source_splits;      /* source row ranges summed separately       */
    int32_t workgroups;         /* pair-kernel workgroups per evaluation     */
    int32_t threads_per_group;  /* 256                                        */
    int64_t pairs_per_eval;     /* N^2 (2K+1)^2: algorithmic pair count      */
} zm_launch_info;

/* Launch shape the pair kernel uses for this context (depends on n1, n2, K
 * and precision only).  For a cutoff context: one target per thread, target
 * blocks of patch_cols x patch_rows cells, source_splits = partial sums per
 * target (zm_cutoff_info.slots); pairs_per_eval stays N^2, the all-pairs
 * count. */
zm_status zm_get_launch_info(const zm_ctx *ctx, zm_launch_info *out);

#define ZM_KERNEL_SURFACE 0  /* tangents, source strength, q        */
#define ZM_KERNEL_PAIRS   1  /* all-pairs BR sweep                   */
#define ZM_KERNEL_TIES    2  /* split-tie correction (even n_a)      */
#define ZM_KERNEL_REDUCE  3  /* sum of source splits, V              */
#define ZM_KERNEL_UPDATE  4  /* D V, RK3 stage combination           */
#define ZM_KERNEL_CELLS   5  /* cutoff BR: cell binning and sorting  */
#define ZM_KERNEL_FFT     6  /* low order: FFT velocity and V        */
#define ZM_KERNEL_COUNT   7

typedef struct zm_kernel_stats {
    int64_t launches;           /* launches timed since the last read        */
    double  total_ms;           /* summed duration from HIP events           */
} zm_kernel_stats;

/* Enable (on != 0) or disable per-kernel timing: each launch is bracketed by
 * HIP events recorded on the context stream. */
zm_status zm_profile_enable(zm_ctx *ctx, int32_t on);

/* Wait for the timed launches, write ZM_KERNEL_COUNT entries to out (indexed
 * by ZM_KERNEL_*) and reset the counters. */
zm_status zm_profile_read(zm_ctx *ctx, zm_kernel_stats *out);

/* ---- cutoff solver ---------------------------------------------------------- */
/*
 * A context with params.cutoff = rc > 0 evaluates the BR velocity with the
 * cutoff solver (sec. 3.2.2: only sources within rc of a target contribute;
 * a pair is in when r1^2 + r2^2 + r3^2 < rc^2 for its image-shifted r).  The
 * device chooses the path per evaluation from the sheet's tangent map:
 *  - index window, when the horizontal map alpha -> (x, y) keeps one
 *    orientation and, on a periodic sheet, has sigma_min(J2) > 0, or, on a
 *    free sheet, stays within ||J2 - I|| < 1/2 of the identity: every source
 *    within rc then lies within an index disc around its target, which is
 *    walked per target (stencil) or, for windows too large for that on a
 *    periodic sheet, per 8 x 8 patch;
 *  - cell grid otherwise (folded, overturned or strongly stretched sheets):
 *    points are binned into cells of side >= rc / cells_per_cutoff in x and
 *    y over the period cell [-L_a/2, L_a/2) (z unbinned; periodic sheet:
 *    coordinates wrap; free sheet: cells clamp to the box, so points that
 *    left it fill the edge cells), sorted by cell (stable), and each target
 *    visits the cells within cells_per_cutoff of its own.
 * Every path sums each target's sources in a fixed order into `slots`
 * partial sums reduced in order, so results are deterministic.  With timing
 * enabled (zm_profile_enable) the pair kernels also count the pairs they
 * tested and the pairs within rc, and record the paths taken.
 */
#define ZM_CUT_PATH_CELLS   1  /* cell grid                                    */
#define ZM_CUT_PATH_WINDOW  2  /* index window per 8 x 8 patch                 */
#define ZM_CUT_PATH_STENCIL 4  /* index window per target                      */

typedef struct zm_cutoff_info {
    int32_t cells1, cells2;      /* cell grid along x / y                     */
    int32_t cells_per_cutoff;    /* neighbour reach in cells                  */
    int32_t block_cells;         /* target block side in cells                */
    int32_t slots;               /* partial sums per target (reduced in order)*/
    int32_t paths;               /* ZM_CUT_PATH_* bits of the timed evaluations */
    int64_t pairs_tested;        /* pair evaluations, see below               */
    int64_t pairs_accepted;      /* of those, pairs with |r| < rc             */
} zm_cutoff_info;

/* Cell grid of a cutoff context, and the pair counts and paths of the timed
 * evaluations (zm_profile_enable on) since timing was switched on or since
 * the previous call, which this call resets.  Waits for the context
 * stream.  ZM_ERR_UNSUPPORTED for an exact (cutoff = 0) context. */
zm_status zm_cutoff_info_get(zm_ctx *ctx, zm_cutoff_info *out);

/* ---- launch-shape tuning --------------------------------------------------- */
/*
 * The pair kernel's launch shape (targets per lane, number of source ranges
 * summed separately) is looked up per (n1, n2, precision) in a process-wide
 * table when a context or batch is created; sizes without an entry use a
 * built-in default.  The number of source ranges changes the order of the
 * per-target sums, so contexts and batch members of one size created after
 * the same tuning give bitwise-identical results.  The table is thread-safe.
 */
typedef struct zm_pair_tuning {
    int32_t targets_per_lane;   /* 1, 2 or 4                                  */
    int32_t source_splits;      /* >= 1 (clamped to n2)                       */
} zm_pair_tuning;

/* Set (t != NULL) or remove (t == NULL) the entry for (n1, n2, precision). */
zm_status zm_tuning_set(int32_t n1, int32_t n2, int32_t precision, const zm_pair_tuning *t);

/* The shape a new context of this size would use (entry or default). */
zm_status zm_tuning_get(int32_t n1, int32_t n2, int32_t precision, zm_pair_tuning *out);

/* Workspace bytes zm_autotune needs for these parameters (0 if invalid, or
 * if the FP32 pair form is refused on this mesh: see zm_create). */
size_t zm_autotune_workspace_bytes(const zm_params *params);

/* Time the pair kernel on synthetic data of this mesh size for every
 * candidate shape (targets per lane 1, 2, 4 x source splits from a quarter
 * to eight times the count that gives >= 2048 workgroups, plus the default
 * shape; for FP32 only the shapes the FP32 form accepts on this mesh,
 * ZM_ERR_UNSUPPORTED if none), store the fastest in the table and return it (best, and its
 * time per launch in best_ms; either may be NULL).  Synchronous: waits for
 * its own work on hip_stream.  Uses only the caller's workspace. */
zm_status zm_autotune(const zm_params *params, void *d_workspace, size_t workspace_bytes,
                      void *hip_stream, zm_pair_tuning *best, double *best_ms);

/* Workspace bytes zm_batch_autotune needs for this set of members (0 if an
 * entry is invalid, or one a batch refuses: see zm_batch_create). */
size_t zm_batch_autotune_workspace_bytes(const zm_params *params, int32_t count);

/* Choose the pair-kernel shape of every mesh size in a batch by timing the
 * batched persistent pair sweep itself (zm_batch_create below), not solo
 * launches: inside a batch the other members keep the device busy, so a
 * size's best split count can differ from its solo one.  On synthetic data
 * of the members' sizes, starting from the shapes new contexts would take,
 * every size (largest total pair work first) tries each candidate (targets
 * per lane 1, 2, 4 x source splits 1, 2, 4, ... up to n2 and the solo
 * candidates; for FP32 only shapes the form accepts) with the other sizes
 * fixed, keeping the fastest.  The chosen shapes go into the process-wide
 * table, so batches, pools and contexts created afterwards use them (and
 * stay bitwise identical to each other).  best: `count` entries (one per
 * member) or NULL; best_ms: time of one batched pair sweep with the chosen
 * shapes, or NULL.  Synchronous; uses only the caller's workspace. */
zm_status zm_batch_autotune(const zm_params *params, int32_t count, void *d_workspace,
                            size_t workspace_bytes, void *hip_stream, zm_pair_tuning *best,
                            double *best_ms);

/* ---- batched ensemble ---------------------------------------------------- */
/*
 * A batch advances `count` independent instances (each with its own mesh
 * size and parameters, one entry of `params`) with one set of launches per
 * RK3 stage: point kernels over all instances' points, and one persistent
 * pair launch per precision whose workgroups take (instance, target patch,
 * source split) items from a device work list ordered longest first.  Each
 * item runs exactly the arithmetic of the single-instance context with the
 * same parameters, so every instance's result is bitwise identical to a solo
 * zm_step.  Same ownership rules as the single-instance API: the caller
 * provides the workspace, the library never allocates device memory.
 */
typedef struct zm_batch zm_batch;  /* opaque */

typedef struct zm_batch_info {
    int32_t count;              /* instances                                   */
    int32_t work_items[2];      /* pair work items: [0] FP64, [1] FP32 pairs   */
    int32_t persistent_groups;  /* workgroups of one persistent pair launch    */
    int64_t pairs_per_step;     /* sum over instances of 3 N^2 (2K+1)^2        */
} zm_batch_info;

/* Workspace bytes for a batch of `count` instances (0 if any entry of params
 * is invalid or count < 1). */
size_t zm_batch_workspace_bytes(const zm_params *params, int32_t count);

/* Create a batch on the current device.  params: `count` parameter sets
 * (copied; exact BR only: cutoff = 0, else ZM_ERR_UNSUPPORTED).  batch_flags:
 * ZM_FLAG_GRAPH and/or ZM_FLAG_CHECK_FINITE (the per-instance params.flags
 * must be 0).  Workspace and stream as for
 * zm_create.  Uploads the descriptor table and work list (waits for the
 * stream once).  On failure *out is NULL and zm_batch_last_error(NULL) says
 * why. */
zm_status zm_batch_create(zm_batch **out, const zm_params *params, int32_t count,
                          uint32_t batch_flags, void *d_workspace, size_t workspace_bytes,
                          void *hip_stream);

/* Copy a state into / out of instance `index` (0 <= index < count); planes
 * of that instance's N points, as for zm_init_state / zm_get_state. */
zm_status zm_batch_init_state(zm_batch *b, int32_t index, const double *d_z, const double *d_w);
zm_status zm_batch_get_state(zm_batch *b, int32_t index, double *d_z, double *d_w);

/* Advance every instance by nsteps >= 0 RK3 steps. */
zm_status zm_batch_step(zm_batch *b, int32_t nsteps);

zm_status zm_batch_get_info(const zm_batch *b, zm_batch_info *out);

/* Wait for outstanding work and release host resources (NULL accepted). */
zm_status zm_batch_destroy(zm_batch *b);

/* Last error of this batch ("" if none; NULL: last failed zm_batch_create
 * on this thread). */
const char *zm_batch_last_error(const zm_batch *b);

/* ---- serving pool ----------------------------------------------------------- */
/*
 * Continuous batching of simulation requests of different mesh sizes.  The
 * caller gives the pool a device budget; requests are admitted first-in
 * first-out as soon as their footprint (zm_pool_request_bytes) fits in the
 * free budget, keep their state resident in the pool, and every call of
 * zm_pool_iterate advances all live requests by one RK3 step with one set
 * of batched launches (the same arithmetic as a solo context: each request's
 * trajectory is bitwise identical alone and in the mix).  Membership changes
 * (admissions, completions, cancellations, failures) take effect between
 * iterations.  The pool never allocates device memory.
 */
typedef struct zm_pool zm_pool;  /* opaque */

#define ZM_REQ_UNKNOWN   (-1)
#define ZM_REQ_QUEUED      0   /* waiting for budget                            */
#define ZM_REQ_LIVE        1   /* resident, advanced by every iteration          */
#define ZM_REQ_FINISHED    2   /* all steps done; state kept until released      */
#define ZM_REQ_FAILED      3   /* state became non-finite (check-finite pools);
                                  evicted alone, memory returned                 */

typedef struct zm_step_record {
    int64_t id;             /* request advanced by the iteration              */
    int32_t steps_done;     /* its completed RK3 steps after the iteration    */
    int32_t state;          /* ZM_REQ_* after the iteration                   */
    double  iteration_ms;   /* device time of the whole batched iteration     */
} zm_step_record;

typedef struct zm_pool_stats {
    int32_t queued, live, finished;
    int32_t iterations;      /* iterations run so far                          */
    int64_t used_bytes;      /* budget held by live and finished requests      */
    int64_t budget_bytes;
    int64_t pairs_done;      /* pair interactions evaluated so far             */
} zm_pool_stats;

/* Workspace bytes for a pool with this request budget (budget + tables). */
size_t zm_pool_workspace_bytes(size_t budget_bytes);

/* Budget bytes one request with these parameters occupies (0 if invalid). */
size_t zm_pool_request_bytes(const zm_params *params);

/* Create a pool on the current device.  flags: 0 or ZM_FLAG_CHECK_FINITE.
 * Workspace: at least zm_pool_workspace_bytes(budget_bytes), 256-byte
 * aligned, caller-owned. */
zm_status zm_pool_create(zm_pool **out, size_t budget_bytes, uint32_t flags, void *d_workspace,
                         size_t workspace_bytes, void *hip_stream);

/* Queue a request: params (params.flags must be 0, cutoff 0), initial state d_z (3
 * planes) / d_w (2 planes), steps >= 1.  The state is copied when the request
 * is admitted, so d_z / d_w must stay valid and unchanged until
 * zm_pool_query reports it no longer queued.  A request larger than the whole
 * budget is refused with ZM_ERR_CAPACITY. */
zm_status zm_pool_submit(zm_pool *pool, const zm_params *params, const double *d_z,
                         const double *d_w, int32_t steps, int64_t *id);

/* One iteration: retire/admit, then one RK3 step of every live request.
 * Writes up to `capacity` records (one per advanced request) and their
 * number to *count.  Waits for its own work (the iteration time is measured
 * with HIP events on the pool stream). */
zm_status zm_pool_iterate(zm_pool *pool, zm_step_record *records, int32_t capacity,
                          int32_t *count);

/* State (ZM_REQ_*) and completed steps of a request (ZM_REQ_UNKNOWN for ids
 * never issued or already released). */
zm_status zm_pool_query(const zm_pool *pool, int64_t id, int32_t *state, int32_t *steps_done);

/* Copy a live or finished request's current state out. */
zm_status zm_pool_fetch(zm_pool *pool, int64_t id, double *d_z, double *d_w);

/* Forget a finished or failed request and return its budget. */
zm_status zm_pool_release(zm_pool *pool, int64_t id);

/* Drop a queued or live request (its budget returns at once). */
zm_status zm_pool_cancel(zm_pool *pool, int64_t id);

zm_status zm_pool_get_stats(const zm_pool *pool, zm_pool_stats *out);

/* Wait for outstanding work and release host resources (NULL accepted). */
zm_status zm_pool_destroy(zm_pool *pool);

const char *zm_pool_last_error(const zm_pool *pool);

/* ---- allocation-free evaluation ------------------------------------------ */
/*
 * For callers that cannot allocate device memory at all: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 *
 * zm_br_velocity_noalloc computes what zm_br_velocity computes on a context
 * created with *params -- d_u (3 planes) = u(d_z, d_w) -- without a context
 * or a workspace: its scratch (source strengths, q, tie corrections and
 * per-source-range partial sums) lives in one static device array of
 * ZM_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends.  The call allocates nothing (no device or host
 * allocation); the caller passes the inputs and the output, all as for
 * zm_br_velocity (float64 planes, 256-byte aligned, d_u not overlapping an
 * input), and the stream the kernels are enqueued on (a hipStream_t, NULL =
 * null stream; asynchronous like every other call).
 *
 * Scope: exact BR sums (cutoff = 0) of the high- or medium-order model,
 * either pair form, any image_layers and boundary.  The pair kernel takes
 * the shape a context of this size would use when its partial sums fit the
 * scratch (then the result is bitwise that of zm_br_velocity); otherwise as
 * many source ranges as fit (the same sums in another order).  Meshes whose
 * scratch exceeds the array even with one source range -- about 645,000
 * points with an even side, 1.19 million with both sides odd or on a free
 * sheet -- are refused with ZM_ERR_CAPACITY.  Other errors as for zm_create
 * and zm_br_velocity; zm_last_error(NULL) gives the message.
 *
 * Every call on one device shares that device's array and leaves it holding
 * its scratch.  Calls that may overlap on one device (different streams,
 * different host threads) race on it: order them, e.g. on one stream.
 */
#define ZM_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

zm_status zm_br_velocity_noalloc(const zm_params *params, const double *d_z, const double *d_w,
                                 double *d_u, void *hip_stream);

/* Interface version (incremented on any ABI change). */
int32_t zm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ZM_H */
