/*
 * ecmg.h - C interface of the MI355X (gfx950) ECMG_jcg library.
 *
 * ECMG_jcg (Pan, He & Hu, arXiv 1506.02983, Algorithm 4) solves
 *     -div(beta grad u) = f  in a box,  u = g_D on Dirichlet faces,
 *     alpha u + beta du/dn = g_R on Robin faces            (Section 1, eq. bvp)
 * with trilinear (Q1) hexahedral finite elements on a hierarchy of uniform
 * grids (Section 2): the two coarsest grids are solved directly, every finer
 * grid starts Jacobi-preconditioned CG (JCG) from an extrapolated and
 * interpolated initial guess (EXP_finite, Sections 4.2.2-4.3) and iterates while
 * ||A u - f||_2 > eps ||f||_2, and a fourth-order extrapolation (EXP_true,
 * Section 4.2.1) combines the two finest solutions.
 *
 * Conventions shared by every call:
 *  - Level l (0-based) has n0[d] * 2^l elements on axis d; "levels" counts all
 *    grids, so levels - 2 grids are solved by JCG (Algorithm 4).
 *  - A node vector of level l has (nx+1)(ny+1)(nz+1) doubles, node (i,j,k) at
 *    index i + (nx+1)*(j + (ny+1)*k): x fastest, each z-plane contiguous.
 *  - Faces are numbered 0..5 = x-lo, x-hi, y-lo, y-hi, z-lo, z-hi.  A node on
 *    any Dirichlet face is a Dirichlet node (Dirichlet wins on shared edges).
 *  - The library owns all device memory it allocates; the caller owns every
 *    host buffer it passes.  Host buffers are read or written only during the
 *    call.  Nothing here allocates or frees caller memory.
 *  - Every function returns ECMG_OK (0) or a negative status; the message of
 *    the last failure is available from ecmg_last_error.  No C++ exception
 *    crosses this interface.  A context is not thread-safe: calls on one
 *    context must not overlap.
 *  - All arithmetic on the device is IEEE FP64 unless a call says otherwise.
 */
#ifndef ECMG_H
#define ECMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ECMG_OK           0
#define ECMG_EINVAL      -1   /* invalid argument or problem data                  */
#define ECMG_ENOMEM      -2   /* device or host allocation failed                  */
#define ECMG_ENOTCONV    -3   /* JCG reached max_iter; the iterate is kept         */
#define ECMG_EBREAKDOWN  -4   /* p.q <= 0 or not finite inside JCG                 */
#define ECMG_EDEVICE     -5   /* a HIP runtime call failed                         */
#define ECMG_ESTATE      -6   /* call out of order (e.g. solve before setup)       */
#define ECMG_ECALLBACK   -7   /* a field callback returned nonzero                 */
#define ECMG_ENOENT      -8   /* no tuning cache file, or no entry for the level   */

/* ---- face types (Section 1: Neumann is Robin with alpha = 0) ---------- */
#define ECMG_DIRICHLET 0
#define ECMG_ROBIN     1

/* ---- precision of the JCG iterations ---------------------------------- */
#define ECMG_FP64  0   /* everything in FP64                                          */
#define ECMG_MIXED 1   /* FP32 stencil and CG vectors inside an FP64 residual /
                          iterative-refinement loop; dots, stopping test, DSOLVE,
                          EXP_finite and EXP_true stay FP64.  Per JCG level solved
                          by the tiled kernels: r = F - A x in FP64 (the stop
                          test of Algorithm 4 is taken on it), FP32 JCG on
                          A d = r / ||r|| from d = 0 until its residual falls by
                          max(inner_tol, eps ||f_h|| / (2 ||r||)), x += ||r|| d in
                          FP64, repeated.  Small levels run in FP64: those the
                          persistent kernel solves and, on the tiled kernels,
                          those of at most persistent_nodes nodes (8,388,608,
                          the levels whose passes fold their scalar steps, when
                          persistent_nodes is -1).                                  */

/* ---- EXP_finite interpolation (Section 4.3) --------------------------- */
#define ECMG_SERENDIPITY20 0   /* 8 corners (eq. jiedian) + 12 mid-edges (eq. zhongdian)
                                  and 20-node tri-quadratic serendipity (eq. inter)   */
#define ECMG_LAGRANGE27    1   /* the Remark after eq. inter: face and body centres as
                                  means of eq. zhongdian along diagonals, then 27-node
                                  tri-quadratic Lagrange interpolation                 */

/* ---- iteration on the levels above the two DSOLVE grids (Section 4.1) --- */
#define ECMG_JCG 0   /* ECMG_jcg: CG preconditioned with M = diag(A) (Algorithm 4)   */
#define ECMG_CG  1   /* ECMG_cg: Algorithm 4 with plain CG (M = I on free nodes), the
                        variant Section 4.1 compares against; with ecmg_solve_fixed
                        and ecmg_cascadic_schedule it is the original ECMG of
                        Algorithm 3 (eq. ee)                                         */

/* ---- vectors of a level (ecmg_get / ecmg_set / ecmg_device_view) ------ */
#define ECMG_VEC_U      0   /* u_l: DSOLVE or JCG solution (g_D on Dirichlet nodes)    */
#define ECMG_VEC_W      1   /* W_l: EXP_finite output on every node, before g_D is
                               imposed (kept only with options.keep_w)                  */
#define ECMG_VEC_UTILDE 2   /* U~_l: EXP_true output (after ecmg_extrapolate)          */
#define ECMG_VEC_F      3   /* load vector F = int f phi + int_R g_R phi (Section 2)   */
#define ECMG_VEC_DINV   4   /* M^-1 on free nodes (1/diag(A); 1 with ECMG_CG), 0 on
                               Dirichlet nodes                                            */
#define ECMG_VEC_NONE  -1

/* ecmg_level_info.path: the kernels a level ran on.  DENSE: DSOLVE by the
 * explicit inverse (a GEMV); PERSISTENT: the whole JCG in one cooperative
 * launch; TILED: tiled stencil passes with the scalar steps folded into them;
 * TILED_UNFOLDED: tiled passes with one-block finishing kernels; COLUMN:
 * column kernels for init and the stencil of pass A (finishing kernels);
 * GATHER: one thread per node for init and the stencil of pass A (folded
 * scalars); MIXED: FP32 JCG inside FP64 refinement; QUEUE: the batched queue
 * kernel (ecmg_solve_batch, the serving loop). */
#define ECMG_PATH_DENSE          0
#define ECMG_PATH_PERSISTENT     1
#define ECMG_PATH_TILED          2
#define ECMG_PATH_TILED_UNFOLDED 3
#define ECMG_PATH_COLUMN         4
#define ECMG_PATH_GATHER         5
#define ECMG_PATH_MIXED          6
#define ECMG_PATH_QUEUE          7

/* Field sampled on a tensor product of coordinates.  The library asks for
 * out[(k*ny + j)*nx + i] = value at (x[i], y[j], z[k]).  face = -1 for points
 * inside the box, 0..5 when every point lies on that face (Robin data needs the
 * outward normal).  Return 0 on success; nonzero aborts setup with
 * ECMG_ECALLBACK.  Host version: x, y, z, out are host pointers. */
typedef int (*ecmg_host_fn)(int32_t face, int64_t nx, int64_t ny, int64_t nz,
                            const double *x, const double *y, const double *z,
                            double *out, void *user);
/* Device version: x, y, z, out are device pointers; work must be ordered on
 * the given HIP stream (hipStream_t passed as void*). */
typedef int (*ecmg_device_fn)(int32_t face, int64_t nx, int64_t ny, int64_t nz,
                              const double *x, const double *y, const double *z,
                              double *out, void *hip_stream, void *user);

/* A coefficient or data field: device callback if set, else host callback if
 * set, else the constant `value`. */
typedef struct {
    double value;
    ecmg_host_fn host;
    ecmg_device_fn device;
    void *user;
} ecmg_field;

/* The boundary value problem of Section 1 (eq. bvp) and its grid hierarchy. */
typedef struct {
    double lo[3], hi[3];       /* the box, lo < hi                                  */
    int32_t n0[3];             /* coarsest elements per axis, >= 1                  */
    int32_t levels;            /* number of grids, >= 2 (levels 0 and 1 are DSOLVE) */
    int32_t face_type[6];      /* ECMG_DIRICHLET or ECMG_ROBIN per face             */
    ecmg_field beta;           /* diffusion coefficient, > 0, sampled at element centroids */
    ecmg_field f;              /* right-hand side, sampled at 2x2x2 Gauss points     */
    ecmg_field g_D;            /* Dirichlet data, sampled at Dirichlet nodes         */
    ecmg_field alpha;          /* Robin coefficient, >= 0, at Robin face-element centroids */
    ecmg_field g_R;            /* Robin data, sampled at 2x2 Gauss points of Robin faces */
} ecmg_problem;

typedef struct {
    int32_t precision;         /* ECMG_FP64 (default) or ECMG_MIXED                      */
    int32_t max_iter;          /* JCG iteration cap per level (default 20000)            */
    int32_t interp;            /* ECMG_SERENDIPITY20 (default) or ECMG_LAGRANGE27        */
    int32_t keep_w;            /* keep W_l of every level for diagnostics (default 1)    */
    double inner_tol;          /* ECMG_MIXED: inner FP32 JCG relative reduction (1e-4)   */
    double dsolve_tol;         /* DSOLVE as FP64 JCG to this relative residual (1e-14)   */
    int32_t chunk;             /* JCG iterations between host status reads (0 = auto)    */
    int32_t timing;            /* 1 = time kernels with HIP events (ecmg_kernel_times)   */
    void *hip_stream;          /* hipStream_t to order all work on; NULL = own stream    */
    int64_t persistent_nodes;  /* grids of at most this many nodes run the whole JCG loop
                                  in one persistent launch; 0 = never, -1 = default
                                  (20,000; 2,400,000 in the serving loop)              */
    int64_t dsolve_dense_max;  /* ecmg_solve: DSOLVE levels with at most this many free
                                  nodes (capped at 8192) are solved with an explicit
                                  inverse of A_FF, built by ecmg_setup (Cholesky and
                                  inverse, rocSOLVER) and applied as one matrix-vector
                                  product per solve; larger ones, and 0, use FP64 JCG
                                  to dsolve_tol (default 8192).  The batched form and
                                  the server always use FP64 JCG, so their contexts
                                  are best created with 0 (no factorisation at setup) */
    int32_t autotune;          /* 0 (default): built-in JCG configuration per level; 1:
                                  ecmg_setup applies the choices the tuning cache holds
                                  for the hierarchy's JCG levels (a missing file or
                                  entry leaves the built-in choice)                     */
    const char *tune_cache;    /* JSON tuning cache path (see ecmg_autotune); NULL = the
                                  ECMG_TUNE_CACHE environment variable, if set; the
                                  string is read during ecmg_create only                */
    int32_t method;            /* ECMG_JCG (default) or ECMG_CG                          */
    int32_t speculate;         /* 1 (default): in ecmg_solve / ecmg_solve_levels, a tiled
                                  JCG level whose last two solves converged in the same
                                  number of iterations enqueues that many iterations and
                                  no status read, so the host does not wait between
                                  levels; if it then falls short of the tolerance, that
                                  level and every finer one are solved again from their
                                  EXP_finite start with status reads (same results as
                                  speculate = 0, at the cost of the repeated work).  On
                                  the levels with one-block finishing kernels the
                                  expected last pass B stores no residual (only the
                                  stop test reads it)                                   */
    int32_t fold_blocks;       /* tiled JCG levels whose two passes have at most this many
                                  blocks each take the CG scalar steps inside the passes
                                  (every block sums the previous pass's partials in one
                                  fixed order); larger levels run a one-block finishing
                                  kernel after each pass.  -1 = default (4096, also the
                                  largest value honoured), 0 = never.  Both forms compute
                                  the same recurrence; only the summation order differs */
    int32_t true_residual;     /* 1: after each JCG level, recompute ||F - A u||_2 on the
                                  free nodes from the final iterate (one more stencil
                                  pass per level) and report it as info.rre_true; 0
                                  (default): rre_true = -1                              */
    int32_t batch_graph;       /* ecmg_solve_batch (options of ctxs[0]): 1 (default) =
                                  the whole batched cascade as one launch, captured
                                  into a HIP graph on the first solve of a set of boxes
                                  and tolerance and replayed on later ones (level by
                                  level if the runtime cannot capture it); 0 = level by
                                  level, launch by launch.  Same results either way    */
    int32_t columns;           /* JCG levels that run one-block finishing kernels (those
                                  above fold_blocks): 1 (default) = JCG init and the
                                  stencil of pass A by the column kernels (a wavefront
                                  marches a column of nodes with its planes in
                                  registers), pass A of iterations >= 1 as a node-wise
                                  p / x update followed by that stencil; 0 = the tiled
                                  kernels (LDS plane tiles, pass A fused).  The same
                                  recurrence; only the summation order differs         */
    int64_t gather_nodes;      /* JCG levels of at most this many nodes whose passes fit
                                  folded scalar steps (at most fold_blocks blocks of
                                  256 nodes) run init and the stencil of pass A one
                                  thread per node, reading each node's 27-point row
                                  from the caches, after a node-wise p / x update that
                                  takes the scalar step (three launches per iteration
                                  instead of a tiled pass A's plane-by-plane march);
                                  -1 = default (1,048,576), 0 = never.  A tuned choice
                                  (autotune) takes precedence.  The same recurrence   */
    /* Device allocator hook (NULL = hipMalloc / hipFree).  alloc returns `bytes` of
     * device memory usable on hip_stream (the library's stream; hipStream_t as
     * void*), or NULL on failure (ECMG_ENOMEM); free releases a pointer alloc
     * returned, after every use of it enqueued on that stream so far.  Lets a
     * caching allocator (e.g. PyTorch's) back the hierarchy.  Both or neither. */
    void *(*alloc)(size_t bytes, void *hip_stream, void *user);
    void (*free)(void *ptr, void *hip_stream, void *user);
    void *alloc_user;
} ecmg_options;

/* One JCG level's configuration chosen by the autotuner. */
typedef struct {
    int32_t level;             /* level (>= 2); -1 from ecmg_tune_lookup                */
    int32_t path;              /* 0: tiled passes, 1: persistent kernel, 3: gather
                                  stencil (options.gather_nodes)                        */
    int32_t kz;                /* tiled: planes per z-chunk of a stencil block           */
    int32_t seg;               /* persistent: nodes per thread segment (1, 2 or 4)       */
    int32_t nwg;               /* persistent: most workgroups                            */
    int32_t candidates;        /* configurations timed                                   */
    double us_default;         /* microseconds per JCG iteration, built-in configuration */
    double us_best;            /* microseconds per JCG iteration, chosen configuration   */
} ecmg_tune_result;

/* Per-level report (Algorithm 4 and the "Iters"/"RRe" columns of Section 5). */
typedef struct {
    int32_t level, nx, ny, nz; /* level index and elements per axis                    */
    int32_t iters;             /* JCG iterations (DSOLVE levels: JCG iterations used, 0
                                  for the dense direct solve)                           */
    int32_t outer_steps;       /* ECMG_MIXED: FP64 refinement steps; else 0            */
    int32_t status;            /* ECMG_OK, ECMG_ENOTCONV or ECMG_EBREAKDOWN            */
    int32_t path;              /* how the level ran (ECMG_PATH_*)                        */
    double rre;                /* ||r||_2 / ||f_h||_2 at exit (recurrence residual)     */
    double nf;                 /* ||f_h||_2 of the stopping test                        */
    double ms;                 /* wall time of the level on the device stream          */
    double rre_true;           /* ||F - A u||_2 / ||f_h||_2 over the free nodes from the
                                  final iterate (options.true_residual = 1; else -1);
                                  rounding in the recurrence makes it differ from rre */
} ecmg_level_info;

typedef struct ecmg_ctx ecmg_ctx;

/* Fill *opt with the defaults listed above. */
void ecmg_default_options(ecmg_options *opt);

/* Create a context on the current HIP device.  opt may be NULL (defaults).
 * Fails with ECMG_EDEVICE when no gfx950 device is present. */
int ecmg_create(const ecmg_options *opt, ecmg_ctx **out);

/* Discretise every level (Section 2): beta at element centroids, alpha at
 * Robin face-element centroids, the load vector F by 2x2x2 Gauss per element
 * and 2x2 Gauss per Robin face element, g_D at Dirichlet nodes, the Jacobi
 * diagonal, and ||f_h||_2 = ||(F - A_FD g_D on free nodes, g_D on Dirichlet
 * nodes)||_2.  Validates the problem: ECMG_EINVAL for lo >= hi, n0 < 1,
 * levels < 2, a bad face type, beta <= 0, alpha < 0, non-finite samples, or a
 * singular system (no Dirichlet face and alpha == 0 everywhere).  Also builds
 * the direct DSOLVE of levels 0 and 1 (options.dsolve_dense_max).  May be
 * called again; it frees the previous hierarchy first. */
int ecmg_setup(ecmg_ctx *ctx, const ecmg_problem *problem);

/* Algorithm 4: DSOLVE on levels 0 and 1 (the explicit inverse of A_FF that
 * ecmg_setup built, or FP64 JCG to options.dsolve_tol; see dsolve_dense_max),
 * then for each finer level W = EXP_finite(u_{l-1}, u_{l-2}), JCG from W (with
 * g_D imposed) while ||r||_2 > rel_tol ||f_h||_2.  info: NULL or an array of
 * `levels` entries.  Returns ECMG_ENOTCONV / ECMG_EBREAKDOWN if any level
 * failed (all levels still run; each entry has its own status). */
int ecmg_solve(ecmg_ctx *ctx, double rel_tol, ecmg_level_info *info);

/* Algorithm 4 in full: ecmg_solve, then EXP_true on the finest level, enqueued
 * behind the cascade so that the call waits for the device once (U~ of the
 * finest level as ecmg_extrapolate(ctx, -1, NULL) leaves it: read it with
 * ecmg_get / ecmg_device_view / ecmg_norms).  Same arguments, results and
 * errors as ecmg_solve. */
int ecmg_solve_extrapolated(ecmg_ctx *ctx, double rel_tol, ecmg_level_info *info);

/* As ecmg_solve, but JCG on level l >= 2 runs exactly iters[l] iterations
 * (iters has `levels` entries; entries 0 and 1 are ignored). */
int ecmg_solve_fixed(ecmg_ctx *ctx, const int32_t *iters, ecmg_level_info *info);

/* As ecmg_solve with a tolerance per level: JCG on level l >= 2 stops when
 * ||r||_2 <= rel_tol[l] ||f_h||_2 (rel_tol has `levels` entries, each >= 0;
 * entries 0 and 1 are ignored).  Section 5 notes that a uniform tolerance lets
 * U~ lose fourth order on fine grids, since it combines two second-order
 * solutions that must both be accurate; a schedule tightened towards the finest
 * grid (ecmg_tolerance_schedule) keeps the coarse levels cheap. */
int ecmg_solve_levels(ecmg_ctx *ctx, const double *rel_tol, ecmg_level_info *info);

/* Host only: rel_tol[l] = min(1, eps_finest * ratio^(levels - 1 - l)) for
 * l >= 2 (repeated products), 0 for the two DSOLVE grids; ratio 1 is the
 * uniform tolerance, ratio 16 loosens each coarser grid by the factor its h^4
 * grows.  ECMG_EINVAL for levels < 3, eps_finest <= 0 or ratio < 1. */
int ecmg_tolerance_schedule(int32_t levels, double eps_finest, double ratio, double *rel_tol);

/* EXP_true (Section 4.2.1, eqs. t1 and chenlin; face and body centres as the
 * mean along their diagonals): U~_l from u_l and u_{l-1}, for 1 <= level <
 * levels (-1 = finest).  host_out: NULL (the call returns once the work is
 * enqueued on the library stream; later calls on the context are ordered
 * after it), or a node array of the level that receives U~_l (the call
 * returns when it is filled). */
int ecmg_extrapolate(ecmg_ctx *ctx, int32_t level, double *host_out);

/* Algorithm 4 for n independent problems at once (each context set up with
 * its own problem, all on one device, none repeated).  With options.batch_graph
 * (of ctxs[0], the default) the whole cascade of every box is one cooperative
 * launch of the queue kernel: each box's level is a task (DSOLVE levels from
 * zero, finer levels building their x = W by EXP_finite first) that waits for
 * the box's coarser levels to finish, so boxes move through their levels
 * independently; that launch is captured into a HIP graph on the first call for
 * a set of contexts and rel_tol and replayed by later calls (a new setup,
 * tuning or tolerance captures again).  Without it (or if the runtime cannot
 * capture), level by level: EXP_finite of every box, then the JCG of every box
 * on that level in one launch, with per-level device times.  Either way a
 * box's level runs on a few workgroups (about options' batched nodes per
 * workgroup), boxes with more nodes first, and the call waits once.
 * Per box the arithmetic is that of ecmg_solve with the persistent kernel, so
 * a box's result does not depend on the other boxes of the batch or on the
 * launch form (it equals a batch of that box alone bit for bit).  Work runs on
 * ctxs[0]'s stream (the other contexts' streams are synchronised first).
 * infos: NULL, or sum(levels of ctxs[i]) entries, box after box in input
 * order.  FP64 only (options.precision is ignored).  Returns ECMG_ENOTCONV /
 * ECMG_EBREAKDOWN if some box failed (all boxes still run; see infos). */
int ecmg_solve_batch(ecmg_ctx *const *ctxs, int32_t n, double rel_tol, ecmg_level_info *infos);

/* EXP_true on the finest level of n contexts, enqueued on ctxs[0]'s stream
 * without a host round trip per box; returns when all are done. */
int ecmg_extrapolate_batch(ecmg_ctx *const *ctxs, int32_t n);

/* ---- serving: continuous batching of independent requests ----------------
 * A server solves requests (each a problem of eq. bvp run through Algorithm 4
 * and EXP_true on its finest level) as they arrive.  The caller drives it:
 * A set-up thread of the server admits queued requests first come first
 * served while the device bytes of their hierarchies (ecmg_plan_bytes) fit the
 * budget and discretises them (Section 2) on a stream of its own, so the field
 * callbacks of a request run on that thread, concurrently with the caller's
 * thread.  ecmg_server_step moves the requests whose set-up has completed into
 * the active set, then advances every active request by one level: the levels
 * small enough for the persistent kernel of all requests share one launch (one
 * workgroup range per request), larger levels run the tiled kernels; finished
 * requests get EXP_true, their U~ copied to the caller's buffer and their
 * device memory kept for the next request with the same grids (a few contexts
 * per grid shape, counted in the budget and given up when a request needs the
 * room) or freed.  A request's result does not depend on which other requests
 * share its steps, on when its set-up ran or on which context it reused.
 * FP64 only. */
typedef struct ecmg_server ecmg_server;

/* opt: NULL = defaults (precision must be ECMG_FP64); the server's work runs
 * on opt->hip_stream or a stream of its own. */
int ecmg_server_create(const ecmg_options *opt, size_t hbm_budget_bytes, ecmg_server **out);

/* Queue a request.  problem and everything it points to (callbacks and their
 * user data) must stay valid until the request's state is 1 or later (set up);
 * the callbacks are called on the server's set-up thread.  host_out (NULL or
 * a dense array of the finest level's nodes, caller-owned) receives U~ and must
 * stay valid until the request is done.  ECMG_ENOMEM if its hierarchy alone
 * exceeds the budget. */
int ecmg_server_submit(ecmg_server *srv, const ecmg_problem *problem, double rel_tol, double *host_out,
                       uint64_t *ticket);

/* Take in the requests set up since the last step, run one level of every
 * active request, finish completed ones.  With no active request but some
 * queued or in set-up, first waits up to 2 ms for one to become ready.
 * n_done: NULL or the number completed in this step. */
int ecmg_server_step(ecmg_server *srv, int32_t *n_done);

/* state: 0 queued or in set-up, 1 set up (running), 2 done, < 0 the error
 * status of a failed request;
 * info (NULL or `levels` entries) is filled once done. */
int ecmg_server_poll(ecmg_server *srv, uint64_t ticket, int32_t *state, ecmg_level_info *info);

/* Latency from submit to U~ on the host over completed requests (p50, p99, in
 * ms), completed requests per second since creation or the last reset. */
int ecmg_server_stats(ecmg_server *srv, double *p50_ms, double *p99_ms, double *solves_per_s, int64_t *done);
/* Drain the tickets of requests that finished (done or failed) since the last
 * call, in the order they finished: up to cap of them into tickets (caller-
 * owned), their number into *n.  A caller that polls only these tickets does
 * not scan every pending request after each step. */
int ecmg_server_completed(ecmg_server *srv, uint64_t *tickets, int32_t cap, int32_t *n);
/* Host time (ms) since creation or the last reset: set-up of requests on the
 * set-up thread (discretisation with the field callbacks, allocation), level
 * work of the steps and finishing of requests (EXP_true, copy of U~) on the
 * calling thread.  Any argument may be NULL. */
int ecmg_server_times(ecmg_server *srv, double *setup_ms, double *step_ms, double *finish_ms);
/* Clears the latency statistics and the host times. */
int ecmg_server_reset_stats(ecmg_server *srv);
void ecmg_server_destroy(ecmg_server *srv);

/* EXP_finite alone: W_l from the current u_{l-1} and u_{l-2} (2 <= level);
 * writes W_l into u_l on free nodes (Dirichlet nodes keep g_D) and into the W
 * vector when kept.  Used for testing and for resuming a cascade. */
int ecmg_prolongate(ecmg_ctx *ctx, int32_t level);

/* JCG on one level from the current u_l: while ||r|| > rel_tol ||f_h|| (or
 * exactly fixed_iters iterations when fixed_iters >= 0). */
int ecmg_jcg(ecmg_ctx *ctx, int32_t level, double rel_tol, int32_t fixed_iters, ecmg_level_info *info);

/* q = A v on free rows of level `level`, 0 on Dirichlet rows (every column is
 * used, so v may carry g_D on Dirichlet nodes).  host_in, host_out: node
 * arrays.  This is the matrix-free operator of Section 2. */
int ecmg_apply(ecmg_ctx *ctx, int32_t level, const double *host_in, double *host_out);

/* Copy a vector of a level to / from a host node array (ECMG_VEC_*). */
int ecmg_get(ecmg_ctx *ctx, int32_t level, int32_t which, double *host_out);
int ecmg_set(ecmg_ctx *ctx, int32_t level, int32_t which, const double *host_in);

/* Device pointer of a vector (FP64) for zero-copy use.  On the device, rows
 * are padded: node (i,j,k) is at i + row_pitch*(j + (ny+1)*k) with row_pitch
 * >= nx+1 (a multiple of 16, so rows start on 128-byte lines); padding entries
 * are zero.  dims receives (nx+1, ny+1, nz+1), *row_pitch (if not NULL) the
 * pitch in elements.  The pointer stays valid until the next ecmg_setup or
 * ecmg_destroy. */
int ecmg_device_view(ecmg_ctx *ctx, int32_t level, int32_t which, void **dptr, int64_t dims[3],
                     int64_t *row_pitch);

/* Error norms of the tables of Section 5 on a level: v = vec[which]
 * - vec[minus_which] (ECMG_VEC_NONE = 0) - minus (NULL = 0), where minus is a
 * node array in host memory, or in device memory when minus_on_device != 0;
 * out[0] = max |v|, out[1] = (sum v^2 / N)^(1/2) over all N nodes (the tables'
 * L2 norm). */
int ecmg_norms(ecmg_ctx *ctx, int32_t level, int32_t which, int32_t minus_which,
               const double *minus, int32_t minus_on_device, double out[2]);

/* ecmg_norms without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that forbid hipMalloc):
 * out[0] = max |v|, out[1] = (sum v^2 / N)^(1/2) for v = vec[which] -
 * vec[minus_which] (ECMG_VEC_NONE = 0), the same kernel and summation order
 * as ecmg_norms, so the same results bit for bit.  The reduction's block
 * partials, arrival counter and totals (at most 2,048 blocks: 33 KB) live in
 * a static device array of the library, one per GPU, held until the process
 * ends; a level that needs more blocks is rejected with ECMG_EINVAL.  Every
 * call on a GPU shares that GPU's array, so calls that overlap on one GPU
 * (from several threads or contexts) race; calls on one context are ordered.
 * Makes no hipMalloc, hipFree or other allocating call; waits for the result. */
int ecmg_norms_noalloc(ecmg_ctx *ctx, int32_t level, int32_t which, int32_t minus_which, double out[2]);

/* Elements per axis of a level. */
int ecmg_level_dims(ecmg_ctx *ctx, int32_t level, int64_t n[3]);

/* Host only (no device needed): the per-level iteration counts of the
 * original ECMG (Algorithm 3, eq. ee) for ecmg_solve_fixed.  iters[0] =
 * iters[1] = 0 (the DSOLVE grids); fine grid j = 1 .. L (L = levels - 2, level
 * j + 1) runs ceil(m_L * beta^(L - j)), so the finest runs m_L; e.g. m_L = 4,
 * beta = 4 gives 4 * 4^(L - j).  iters: `levels` entries, caller-owned.
 * ECMG_EINVAL for levels < 3, m_L < 1, beta < 1 (or not finite), or a count
 * above 2^31 - 1. */
int ecmg_cascadic_schedule(int32_t levels, int32_t m_L, double beta, int32_t *iters);

/* Device bytes the hierarchy of `problem` needs at `precision` (no device
 * needed). */
int ecmg_plan_bytes(const ecmg_problem *problem, int32_t precision, size_t *bytes);

/* Kernel timing (options.timing = 1): for level `level` and kernel class k
 * (0 = JCG pass A, 1 = JCG pass B, 2 = JCG init, 3 = EXP_finite, 4 = EXP_true,
 * 5 = mixed-precision pass A, 6 = mixed-precision pass B, 7 = whole-level
 * persistent JCG used for small grids, 8 = mixed-precision start (r / ||r||
 * to FP32), 9 = mixed-precision update x += ||r|| d, 10 = JCG pass A of
 * iteration 0, which reads the p_0 that init stored; class 0 counts the later
 * iterations, 11 = JCG pass A of iterations >= 1 on the levels that run the
 * column or the gather kernels (ecmg_level_info.path): the node-wise p and x
 * update, then the stencil, timed from the start of the first kernel to the
 * end of the second (on the gather levels class 10 is timed the same way), 12 =
 * the JCG pass B a level solved without status reads expects to be its
 * last (options.speculate): it takes the stop test without storing r or
 * forming r.z, since nothing reads them if the test passes and the level is
 * solved again if it fails; class 1 counts the other pass B launches),
 * out[0] = total milliseconds and out[1] = launches that did work since the
 * last ecmg_reset_kernel_times.  Measured with HIP events on the library's
 * stream around each launch; both calls wait for the stream to finish the
 * launches they account. */
int ecmg_kernel_times(ecmg_ctx *ctx, int32_t level, int32_t k, double out[2]);
int ecmg_reset_kernel_times(ecmg_ctx *ctx);

/* The kernel classes timed from now on: bit k = class k of ecmg_kernel_times,
 * 0 = none, -1 = all (options.timing = 1 starts with all).  Records already
 * made still count.  Timing a class records two HIP events around each of its
 * launches, which lengthens launch-bound levels (the JCG passes of small
 * grids); to measure a step's time, time only the classes needed. */
int ecmg_set_timing(ecmg_ctx *ctx, int32_t mask);

/* Autotuner of the JCG configuration (how the loop of Algorithm 4 runs on each
 * level; the iterates are those of the same recurrence whatever is chosen, up
 * to summation order).  After ecmg_setup: for every JCG level (>= 2), times
 * `iters` fixed JCG iterations (<= 0: the level's iteration count in the last
 * converged solve on ctx, capped at 4000, or 8 before any) from the level's
 * current iterate,
 * which is restored, under the built-in configuration and each candidate
 * (tiled passes with z-chunks of 1, 2, 4, 8, 16, 32 or 64 planes; the persistent
 * kernel with segments of 2 or 4 nodes and at most 32, 64, 128 or 256 workgroups, for
 * grids of at most 20,000,000 nodes; the gather path of options.gather_nodes
 * where its passes fit folded scalar steps), keeps the fastest for later solves on
 * ctx and, if cache_path (or options.tune_cache, or $ECMG_TUNE_CACHE) names a
 * file, merges the choices into that JSON cache keyed by precision and
 * elements per axis (the file is replaced atomically).  out: NULL or
 * levels - 2 entries.  Allocates one scratch array of the largest JCG level
 * for the duration of the call; synchronous. */
int ecmg_autotune(ecmg_ctx *ctx, int32_t iters, const char *cache_path, ecmg_tune_result *out);

/* Autotuner of the batched form (ecmg_solve_batch): times a batch solve of the
 * n set-up contexts (rel_tol as in ecmg_solve_batch; the solutions are those of
 * the last candidate's solve) under their current configuration and under each
 * candidate -- about 2048, 4096, 8192, 16384 or 32768 nodes per workgroup of a
 * box (at most 16 workgroups) with segments of 2 or 4 nodes -- and gives every
 * context the fastest.  If cache_path (or ctxs[0]'s options.tune_cache) names a
 * file, the choice is merged into it under "batch <precision>", and a context
 * created with options.autotune = 1 takes it at setup.  out: NULL or one entry
 * (level -1, path 2, seg, nwg = nodes per workgroup).  Synchronous. */
int ecmg_autotune_batch(ecmg_ctx *const *ctxs, int32_t n, double rel_tol, const char *cache_path,
                        ecmg_tune_result *out);

/* Host only (no device needed): the choice the tuning cache at `path` holds for
 * a JCG level of nx x ny x nz elements at `precision`.  ECMG_ENOENT if the file
 * or the entry does not exist, ECMG_EINVAL if the file is not a tuning cache. */
int ecmg_tune_lookup(const char *path, int32_t precision, int32_t nx, int32_t ny, int32_t nz,
                     ecmg_tune_result *out);

/* The last error message of ctx (or of the calling thread when ctx is NULL). */
const char *ecmg_last_error(const ecmg_ctx *ctx);

/* Release every device allocation of ctx and the context itself. */
void ecmg_destroy(ecmg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ECMG_H */
