/*
 * wos.h -- C ABI of libwos: Walk-on-Spheres estimates of the screened Poisson
 * potential field and its gradient on MI355X (gfx950).
 *
 * The problem follows Muchacho & Pokorny, "Walk on Spheres for PDE-based Path
 * Planning":
 *   - PDE (Sec. III, eq. screened_poisson_wos, c = 1/t; here sigma = c):
 *         Laplacian(u) - sigma u = 0 in Omega,   u = g on the boundary.
 *   - Omega is the outer box minus obstacles, given through the distance to its
 *     boundary (Sec. V); the goal set is part of the boundary with g = g_goal
 *     (Sec. III, eq. screened_potential_field), obstacles and the outer box
 *     carry g_obstacle and g_outer (0 in the planning workloads).
 *   - Estimator (Sec. IV-A): mean over n walks of the one-point estimates
 *     u_hat(x_0) = prod_k C(R_k) g(xbar_K), with R_k the largest empty ball
 *     around x_k, x_{k+1} uniform on its sphere, and absorption in the
 *     eps-shell (Fig. 2); C(R) = 1 / 0F1(; d/2; sigma R^2 / 4).
 *   - Gradient (Sec. IV-A, first-sphere estimator):
 *         grad_hat u(x_0) = (d / R_0) C1(R_0) u_hat(x_1) v_0,
 *     C1(R) = 1 / 0F1(; d/2 + 1; sigma R^2 / 4)  (equal to the printed d/R
 *     form at sigma = 0).
 *
 * Conventions for every call:
 *   - Return 0 on success, a negative WOS_E* code on error; wos_last_error()
 *     then returns a message (thread-local).  Nothing is launched on error.
 *   - "host" pointers are read during the call only and may be freed after it
 *     returns.  "device" pointers are caller-owned device memory on the current
 *     HIP device; the call enqueues work on `stream` (a hipStream_t, NULL for the
 *     default stream) and returns without synchronising: device outputs are
 *     valid once the stream has reached that point.  Outputs are overwritten,
 *     never accumulated.
 *   - Matrices are row-major: queries Q x d, gradients Q x d.  The floating
 *     type of queries and of u / gradient outputs is float (WOS_FP32) or double
 *     (WOS_FP64); statistics and sensitivities are always double.
 *   - Random numbers: Philox4x32-10 with key = seed and counter
 *     (2k + j, walk, query, env_id) for step k; the walks of a query depend only
 *     on that identity, so estimates are reproducible and the batched, plain,
 *     forward and backward paths regenerate identical walks.
 *   - Queries outside Omega or within eps of its boundary are not errors: all
 *     their walks stop at once with u_hat = g of the nearest component and a
 *     zero gradient ("degenerate", counted in the statistics).
 *   - A walk that makes max_steps distance evaluations without reaching the
 *     eps-shell is truncated: it contributes 0 and is counted.
 */
#ifndef WOS_H
#define WOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WOS_OK 0
#define WOS_EINVAL (-1)  /* bad argument: NULL, NaN/Inf, eps <= 0, sigma < 0, n_walks < 1 ... */
#define WOS_EDIM (-2)    /* d outside [2, 8] */
#define WOS_ENOMEM (-3)  /* device or host allocation failed */
#define WOS_EHIP (-4)    /* HIP runtime or launch error */
#define WOS_ENOTSUP (-5) /* unsupported combination (see each call) */

#define WOS_MIN_DIM 2
#define WOS_MAX_DIM 8
#define WOS_BATCH_STRIDE 8 /* row stride of batched query / gradient arrays */
#define WOS_BATCH_STATS 16 /* columns of a batched stats row */

/* flags */
#define WOS_FP32 0u
#define WOS_FP64 1u
#define WOS_FULL_SCAN 2u /* scan every obstacle each step (no cluster culling);
                            same walks and results, more work: for testing */
#define WOS_SCALAR_CULL 4u /* FP32: cluster tests on the vector ALUs instead of the
                              matrix cores; same walks and results */
#define WOS_WAVE_SCAN 8u   /* FP32: every lane scans the members of every cluster
                              some lane of its wave needs, instead of queuing the
                              needed (walker, cluster) pairs; same walks */
#define WOS_OUT_FP64 16u   /* wos_estimate with FP32 walks: out_u and out_grad are
                              double, the FP64 walk sums without rounding to FP32
                              (means below FP32's range stay); other calls reject it */
#define WOS_NO_BOX_TEST 32u /* FP32 pair scan: every (walker, cluster) pair the
                               cluster bound keeps has its members scanned, without
                               the bounding-box test; same walks.  By default the
                               box test runs where the obstacles depend on 6 or
                               more coordinates (it culls little below that) */
#define WOS_BOX_TEST 64u    /* FP32 pair scan: the bounding-box test in every
                               dimension; same walks (not with WOS_NO_BOX_TEST) */

/* boundary-data modes */
#define WOS_BDATA_CLASS 0  /* g_goal / g_obstacle / g_outer per component */
#define WOS_BDATA_AFFINE 1 /* g(y) = a.y + b on every component; needs sigma = 0 */
#define WOS_BDATA_PLANE 2  /* g(y) = exp(k.y) on every component; needs |k|^2 = sigma */

/* outer boundary kinds */
#define WOS_OUTER_BOX 0  /* [lo, hi] */
#define WOS_OUTER_BALL 1 /* ball (center, radius) */

typedef struct wos_domain wos_domain; /* opaque, library-owned, immutable */
typedef struct wos_plan wos_plan;     /* opaque planning loop (captured HIP graph) */

typedef struct {
    int64_t n;               /* number of sphere obstacles (may be 0) */
    const double* centers;   /* host, n x d */
    const double* radii;     /* host, n, each >= 0 (0: point obstacle) */
} wos_spheres;

typedef struct {
    int64_t n;                 /* number of axis-aligned box obstacles (may be 0) */
    const double* centers;     /* host, n x d */
    const double* half_widths; /* host, n x d, each >= 0 */
} wos_boxes;

typedef struct {
    const double* center; /* host, d */
    double radius;        /* > 0 */
} wos_ball;

typedef struct {
    int kind;              /* WOS_OUTER_BOX or WOS_OUTER_BALL */
    const double* lo;      /* host, d (box) */
    const double* hi;      /* host, d (box), hi > lo */
    const double* center;  /* host, d (ball) */
    double radius;         /* ball radius > 0 */
    int geom_d;            /* 0 or d: the full space.  1 <= geom_d < d: extruded
                              geometry (Sec. VI): the outer boundary and every
                              obstacle depend on the first geom_d coordinates only
                              and the remaining ones are unbounded; only the first
                              geom_d entries of lo, hi, center and of the sphere
                              centres are read.  The goal ball and the point
                              source stay d-dimensional.  Box obstacles need the
                              full space. */
} wos_outer;

typedef struct {
    int mode;            /* WOS_BDATA_* */
    double g_goal;       /* class mode: value on the goal sphere (1 for planning) */
    double g_obstacle;   /* class mode: value on obstacles (0 for planning) */
    double g_outer;      /* class mode: value on the outer boundary (0) */
    const double* a_or_k;/* host, d: affine slope a or plane-wave vector k */
    double b;            /* affine offset */
} wos_bdata;

/* Planar serial arm with revolute joints (Sec. V-A): the walk coordinates are
 * the d joint angles, link i (length l_i) points along q_1 + ... + q_i in the
 * task plane, and the base joint sits at the plane's origin.  Obstacle points
 * in the task plane make the configurations that put a link on a point the
 * arm's part of the boundary.  The walk uses the lower bound d_tau(q) / K of
 * the joint-space distance to it: d_tau the planar distance between the
 * points and the links (segments), K = sqrt(sum_n (l_n + ... + l_d)^2), which
 * bounds how fast any point of the arm moves per unit of joint motion (the
 * printed sum over the first n links agrees for equal links).  A walk
 * absorbed there takes g_obstacle. */
typedef struct {
    const double* lengths;  /* host, d: link lengths >= 0, not all 0 */
    int64_t n_points;       /* obstacle points in the task plane, >= 1 */
    const double* points;   /* host, n_points x 2 */
} wos_arm;

/* Point source f = amplitude * delta_z (Sec. VI and VII: a unit impulse at the
 * goal point, with zero boundary data).  A walk step whose largest empty ball
 * holds z adds amplitude G_B(x_k, z), weighted by the step's screening
 * product, where G_B is the Green's function of (-Laplacian + sigma) on that
 * ball with zero data on its sphere (Sec. IV-A, the |B| f G_c term); the
 * first step adds c_imp * amplitude * grad_x G_B(x_0, z) to the gradient
 * estimate (the c_imp grad G_c term; c_imp = 1 is the unbiased weight). */
typedef struct {
    const double* z;     /* host, d: the source point (inside Omega) */
    double amplitude;    /* finite */
    double c_imp;        /* finite, >= 0 */
} wos_source;

typedef struct {
    uint32_t flags;     /* WOS_FP32 (default) or WOS_FP64, optionally | WOS_FULL_SCAN, WOS_SCALAR_CULL */
    uint32_t env_id;    /* counter word 3 of the RNG (default 0) */
    uint32_t max_steps; /* distance evaluations per walk before truncation; 0 -> 65536 */
    uint32_t reserved;  /* must be 0 */
} wos_options;

/*
 * wos_create_domain -- copy a domain description to the current device.
 * Omega = outer \ (goal ball U spheres U boxes U arm collisions) (Sec. V:
 * the walk only needs the distance to the boundary, or a lower bound of it;
 * here exact signed distances of the components, the arm's Lipschitz bound,
 * and their minimum).  goal may be NULL (no goal set); spheres, boxes and
 * arm may be NULL (none).  Ties resolve to the goal, then spheres by index,
 * then boxes, then the arm, then the outer boundary.  With 64 or more spheres
 * (boxes) the domain also keeps them grouped in clusters of 8 with bounding
 * spheres; the walk kernels skip a cluster that provably holds no nearer
 * obstacle, which changes the work done, never a distance or a walk.
 * source may be NULL (no volume source, the boundary-data problem).
 * Errors: WOS_EDIM, WOS_EINVAL (NULL out/outer/bdata, non-finite values,
 * negative radii, empty box, bad source, geom_d outside [0, d], boxes or an
 * arm with geom_d < d, bad arm), WOS_ENOTSUP (an arm with affine or
 * plane-wave data), WOS_ENOMEM, WOS_EHIP.
 */
int wos_create_domain(int d, const wos_spheres* spheres, const wos_boxes* boxes, const wos_arm* arm,
                      const wos_ball* goal, const wos_outer* outer, const wos_bdata* bdata,
                      const wos_source* source, wos_domain** out);

/* wos_destroy_domain -- free a domain (NULL is ignored).  The caller ensures no
 * enqueued work still uses it. */
void wos_destroy_domain(wos_domain* dom);

/* wos_domain_dim -- dimension d of a domain (or WOS_EINVAL for NULL). */
int wos_domain_dim(const wos_domain* dom);

/*
 * wos_estimate -- u(x_q) and grad u(x_q) for Q query points (Sec. IV-A).
 *   queries   device, Q x d (float or double per opt->flags)
 *   n_walks   walks per query, >= 1
 *   sigma     screening coefficient c = 1/t >= 0
 *   eps       absorption shell width > 0
 *   seed      Philox key
 *   out_u     device, Q (same type as queries; double with WOS_OUT_FP64)
 *   out_grad  device, Q x d, or NULL (same type as out_u)
 *   out_stats device double, Q x (d + 4), or NULL: per query
 *             [se_u, se_grad[0..d-1], mean_steps, n_truncated, n_degenerate],
 *             se = sample standard deviation / sqrt(n_walks)
 *   opt       NULL for defaults
 * Plain form: one walk per lane, lanes idle once their walk ends (about half
 * the lanes on 7-D workloads); for throughput in FP32 prefer
 * wos_estimate_batch, also with a single environment, whose lanes refill.
 * FP32 walks keep the weight product's binary exponent apart and sum in FP64,
 * so walks whose weight is below FP32's range still count; a mean below it
 * reads as 0 in FP32 out_u / out_grad (out_stats are FP64) unless WOS_OUT_FP64
 * asks for double outputs.
 * Errors: WOS_EINVAL, WOS_ENOTSUP (affine data with sigma != 0; plane wave
 * with |k|^2 != sigma; sigma R^2 too large for the weight series), WOS_EHIP.
 */
int wos_estimate(const wos_domain* dom, const void* queries, int64_t n_queries,
                 int64_t n_walks, double sigma, double eps, uint64_t seed, void* out_u,
                 void* out_grad, double* out_stats, const wos_options* opt, void* stream);

/*
 * wos_backward -- vector-Jacobian product of u with respect to the query
 * points, sigma and g_goal for upstream weights grad_u (device, Q, same type
 * as queries), regenerating the forward walks from (seed, walk, query,
 * env_id) instead of storing them:
 *   out_dx[q]   = grad_u[q] * grad_hat u(x_q)              (device, Q x d)
 *   out_dsigma  = sum_q grad_u[q] mean_w[d u_hat / d sigma] (device double scalar)
 *   out_dg_goal = sum_q grad_u[q] mean_w[W 1{goal}]        (device double scalar)
 *   out_dq      device double Q x 2 or NULL: per query (du/dsigma, du/dg_goal)
 * with d u_hat / d sigma = (W g) S, S = sum over weighted steps of
 * d ln C(R_k)/d sigma (the walk law does not depend on sigma, so this
 * pathwise derivative is exact), W the product of weights; with a point
 * source each source term W_k G_B adds W_k (S_k G_B + d G_B / d sigma).  In
 * the affine / plane-wave modes dg_goal is the sensitivity to a constant
 * added to the data on the goal sphere.
 * Errors: as wos_estimate; WOS_ENOTSUP for a point source at sigma = 0 (the
 * sigma derivative of the Laplace Green's function is not provided).
 */
int wos_backward(const wos_domain* dom, const void* queries, int64_t n_queries, int64_t n_walks,
                 double sigma, double eps, uint64_t seed, const void* grad_u, void* out_dx,
                 double* out_dsigma, double* out_dg_goal, double* out_dq,
                 const wos_options* opt, void* stream);

/*
 * wos_estimate_batch -- forward (grad_u == NULL) or fused forward + backward
 * over a ragged batch of environments in ONE persistent launch: a wave takes
 * a work unit (env, query, walk range) from a device counter and refills its
 * lanes with the next walk of the unit as soon as a walk ends.  FP32 only.
 *   envs       host array of n_envs domains (any mix of d)
 *   queries    device float, (sum Q) x 8: env e's queries are rows
 *              q_offsets[e] .. q_offsets[e+1]-1, first d_e columns used
 *   q_offsets  host, n_envs + 1, non-decreasing, q_offsets[0] = 0
 *   sigma, eps host, n_envs each
 *   n_walks    host, n_envs: walks per query of each env
 *   seed       Philox key; env e uses env_id = e
 *   out_u      device float, sum Q
 *   out_grad   device float, (sum Q) x 8, or NULL
 *   out_stats  device double, (sum Q) x WOS_BATCH_STATS, or NULL: columns
 *              0..11 as wos_estimate with d = 8 columns reserved for
 *              se_grad, then
 *              [12] sphere distances evaluated per walk (mean),
 *              [13] box distances evaluated per walk (mean),
 *              [14] cluster bounds evaluated per walk (mean),
 *              [15] cluster bounding boxes tested per walk (mean); these
 *              count the work the obstacle scan did after culling (per walk
 *              they wrap modulo 2^32)
 *   grad_u     device float, sum Q, or NULL for forward only
 *   out_dx     device float, (sum Q) x 8 (required with grad_u)
 *   out_dsigma device double, n_envs (required with grad_u)
 *   out_dg     device double, n_envs (required with grad_u)
 * Walk identities match wos_estimate / wos_backward called per env with
 * env_id = e, so results agree with those calls up to summation order.
 * Errors: as wos_estimate; WOS_ENOTSUP for WOS_FP64, and with grad_u for an
 * env with a point source at sigma = 0 (as wos_backward); WOS_EINVAL for an
 * env with more than 2^31 - 1 queries or a batch of 2^32 - 1 or more work
 * units (each at least 64 walks).
 */
int wos_estimate_batch(const wos_domain* const* envs, int n_envs, const float* queries,
                       const int64_t* q_offsets, const double* sigma, const double* eps,
                       const int64_t* n_walks, uint64_t seed, float* out_u, float* out_grad,
                       double* out_stats, const float* grad_u, float* out_dx,
                       double* out_dsigma, double* out_dg, const wos_options* opt,
                       void* stream);

/*
 * wos_estimate_batch_noalloc -- wos_estimate_batch for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, kernels, walks and
 * results, but its tables, work-unit counter and partial sums live in a
 * fixed device array of WOS_NOALLOC_SCRATCH_BYTES per device, reserved when
 * the library's device code loads on that device and held until the process
 * ends.  The call makes no device or pinned-host allocation; it copies
 * about (sizeof env table) x n_envs bytes from static host staging and clears
 * the counter with a fill kernel.
 * Limits: at most WOS_NOALLOC_MAX_ENVS environments, and 256-byte-aligned
 * [counter | tables | 208 bytes per work unit] within the array; a work unit
 * is one (query, walk range), so a batch needs about 208 bytes per query
 * when its queries take a few thousand walks (the full 512-env ragged batch,
 * 266081 queries x 2048 walks, needs 56 MB).  A batch beyond either limit
 * returns WOS_EINVAL before anything is launched.
 * Concurrency: every call on a device uses that device's one array, which
 * keeps the last call's contents.  Host threads are serialised by the
 * library, but calls whose work overlaps on the device (different streams
 * without ordering between them) race on the array: order them on one
 * stream or synchronise between them.
 * Errors: as wos_estimate_batch; WOS_EINVAL for a batch beyond the limits;
 * WOS_EHIP if the array's address cannot be resolved on the device.
 */
#define WOS_NOALLOC_SCRATCH_BYTES 67108864u /* 64 MiB */
#define WOS_NOALLOC_MAX_ENVS 1024
int wos_estimate_batch_noalloc(const wos_domain* const* envs, int n_envs, const float* queries,
                               const int64_t* q_offsets, const double* sigma, const double* eps,
                               const int64_t* n_walks, uint64_t seed, float* out_u, float* out_grad,
                               double* out_stats, const float* grad_u, float* out_dx,
                               double* out_dsigma, double* out_dg, const wos_options* opt,
                               void* stream);

/*
 * wos_plan_create -- gradient-ascent planning loop (Sec. III, screened-harmonic
 * paths; Sec. VII step rule s = min(s_ub, d(x)/2)) captured once as a HIP graph
 * of [fused forward + backward walk kernel, finalize, update] on `stream`.
 *   x      device float, S x d start points, updated in place each step
 *   Step t uses key seed + t (t kept on the device, so replays need no host
 *   work); start s is query s of the walks.  The step direction is the unit
 *   vector of the gradient's FP64 walk sums, so it exists even where the mean
 *   gradient is below FP32's range (long distances at large sigma).  A start
 *   whose estimated gradient is exactly zero does not move (a stall is
 *   counted); a start within eps of the boundary stops (status 1 at the goal,
 *   2 elsewhere).
 * The plan owns its scratch buffers; x must outlive the plan.
 * Errors: WOS_EINVAL (NULL pointers, n_starts outside [1, 2^24], n_walks
 * outside [1, 2^31], s_ub not finite and > 0, 2^32 - 1 or more work units),
 * WOS_ENOTSUP (WOS_FP64, WOS_OUT_FP64), WOS_EHIP / WOS_ENOMEM (set-up or
 * graph capture).
 */
int wos_plan_create(const wos_domain* dom, float* x, int64_t n_starts, int64_t n_walks,
                    double sigma, double eps, double s_ub, uint64_t seed,
                    const wos_options* opt, void* stream, wos_plan** out);

/* wos_plan_step -- replay the captured step n_steps times on the plan's stream. */
int wos_plan_step(wos_plan* plan, int n_steps);

/*
 * wos_plan_buffers -- device pointers owned by the plan (valid until destroy):
 *   u [S] float, grad [S x 8] float (last step's estimates, first d columns;
 *   values below FP32's range read as 0), path_len [S] double (sum of step
 *   lengths), stalls [S] int32, status [S] int32, step [1] uint64 (steps
 *   taken).  Any output pointer may be NULL.
 */
int wos_plan_buffers(wos_plan* plan, float** u, float** grad, double** path_len,
                     int32_t** stalls, int32_t** status, uint64_t** step);

/*
 * wos_plan_read -- synchronise the plan's stream and copy its state to host
 * arrays (any may be NULL): u [S] float, grad [S x 8] float, path_len [S]
 * double, stalls [S] int32, status [S] int32, step [1] uint64.
 */
int wos_plan_read(wos_plan* plan, float* u, float* grad, double* path_len, int32_t* stalls,
                  int32_t* status, uint64_t* step);

/* wos_plan_destroy -- synchronise the plan's stream and free it (NULL ignored). */
void wos_plan_destroy(wos_plan* plan);

/*
 * Launch shape of the persistent batched kernel, as searched by the
 * autotuner (no passage of the paper: the launch layout is this library's).
 */
typedef struct {
    int waves_per_block;  /* 1, 2 or 4: blocks of 64, 128 or 256 threads */
    int units_per_wave;   /* work units (query, walk range) per resident wave */
    int grid_mult;        /* grid = grid_mult x the resident blocks of the device */
    int walks_per_lane;   /* least walks each walk-carrying lane takes from a work unit */
    int lanes_per_walker; /* G = 1, 2, 4, ..., 64: a wave carries 64 / G walks at once;
                             all 64 lanes share those walks' member scans */
    double ms_default;    /* launch time with the built-in shape (4, 4, 1, 2, 1) */
    double ms_best;       /* launch time with the chosen shape */
    int tried;            /* shapes timed */
} wos_tune_result;

/*
 * wos_autotune_batch -- time the persistent launch of the caller's own batch
 * (arguments as wos_estimate_batch; fused != 0: forward + backward with
 * u-bar = 1, else forward only) for launch shapes reached by coordinate
 * descent from the built-in one: waves per block {1, 2, 4}, units per wave
 * {1, 2, 4, 8, 16}, grid multiple {1, 2}, walks per lane {1, 2, 4}, one
 * parameter at a time with the others held, then lanes per walker G (fewer
 * walks per wave, more waves, when the batch has too few walks to fill the
 * device) doubled from the current value up to 64 while the launch gets
 * faster, then halved likewise; a shape must beat the best by more than
 * 0.5 % to replace it.  The best shape is recorded for this batch
 * mix (the multiset of its environments' dimension and log2 buckets of
 * obstacle, query and walk counts), in memory for the batched calls of this
 * process and, when cache_path is not NULL, in that JSON file (created or
 * updated).  out (nullable) receives the shape and the two launch times.
 * Blocks the calling thread; allocates its own output buffers.
 * Errors: as wos_estimate_batch; WOS_EINVAL without queries.
 */
int wos_autotune_batch(const wos_domain* const* envs, int n_envs, const float* queries,
                       const int64_t* q_offsets, const double* sigma, const double* eps,
                       const int64_t* n_walks, uint64_t seed, int fused, const char* cache_path,
                       wos_tune_result* out);

/*
 * wos_autotune -- the same search on a synthetic scene of dimension d with
 * M sphere obstacles and Q queries (fused forward + backward), recorded in
 * the cache file (JSON, created or updated) under the bucket of (d, M, Q).
 * Batched launches look up their batch mix first, then the bucket of their
 * heaviest environment, else use the built-in shape; the cache is read from
 * cache_path (or $WOS_AUTOTUNE_CACHE when wos_set_autotune_cache was not
 * called).  Blocks the calling thread (synchronises the device).
 */
int wos_autotune(int d, int64_t n_obstacles, int64_t n_queries, int64_t n_walks,
                 const char* cache_path);

/* wos_set_autotune_cache -- load (or reset with NULL) the autotune cache. */
int wos_set_autotune_cache(const char* cache_path);

/*
 * wos_varadhan -- the Varadhan read-out of an estimate (Sec. III, eq.
 * transformation_varadhan): w = -sqrt(t) ln u with t = 1 / sigma, a distance
 * to the goal set that tends to the geodesic one as t -> 0, and
 * grad w = -sqrt(t) grad u / u (parallel to grad u, Sec. III).
 *   u          device, n (float or double per opt->flags)
 *   grad_u     device, n x stride (first d columns used), or NULL
 *   sigma      the screening coefficient the estimate was made with, > 0
 *   out_w      device, n; +inf where u <= 0 (no walk reached the goal)
 *   out_grad_w device, n x stride, or NULL (with grad_u); 0 where u <= 0
 * Asynchronous on stream.  Errors: WOS_EINVAL (sigma <= 0, NULL u / out_w,
 * grad_u without out_grad_w, stride < d), WOS_EDIM, WOS_EHIP.
 */
int wos_varadhan(const void* u, const void* grad_u, int64_t n, int d, int stride, double sigma,
                 void* out_w, void* out_grad_w, const wos_options* opt, void* stream);

/*
 * wos_debug_walks -- per-walk records of walks w0 .. w0+n-1 of one query, for
 * diagnostics and walk-level parity checks.  query is a host double array of
 * d values (cast to the compute type); q_index is the query's RNG index.
 * out_records (host double, n x (d + 7)): [u_hat, grad_hat[d], S, goal_w,
 * steps, status (0 absorbed, 1 degenerate, 2 truncated), class (0 goal,
 * 1 sphere, 2 box, 3 outer, 4 arm), d u_hat / d sigma].  Synchronous.
 */
int wos_debug_walks(const wos_domain* dom, const double* query, uint32_t q_index, int64_t w0,
                    int64_t n, double sigma, double eps, uint64_t seed, const wos_options* opt,
                    double* out_records);

/*
 * wos_debug_clusters -- host only, no device: the obstacle clusters that
 * wos_create_domain builds for this obstacle set (empty below 64 obstacles),
 * WOS_CLUSTER_ROWS obstacle rows per cluster.
 *   spheres, boxes   as wos_create_domain (either may be NULL)
 *   fp64             0: the FP32 tables, 1: the FP64 tables
 *   out_n_cl         host int64[2]: sphere clusters, box clusters
 *   order_sph        host int64, capacity n_cl_sph * WOS_CLUSTER_ROWS (may be NULL): caller
 *                    index of each clustered sphere row, -1 for padding
 *   bnd_sph          host double, capacity n_cl_sph * (d + 1) (may be NULL):
 *                    bounding sphere (centre, enlarged radius) per cluster,
 *                    as stored in the device table
 *   order_box, bnd_box  the same for boxes
 * Capacities are taken from the counts this call computes: call once with
 * NULL arrays to learn them.  Errors: WOS_EDIM, WOS_EINVAL.
 */
#define WOS_CLUSTER_ROWS 8
int wos_debug_clusters(int d, const wos_spheres* spheres, const wos_boxes* boxes, int fp64,
                       int64_t* out_n_cl, int64_t* order_sph, double* bnd_sph, int64_t* order_box,
                       double* bnd_box);

/*
 * wos_debug_cluster_boxes -- host only, no device: the bounding boxes that
 * the FP32 kernels test the (walker, cluster) pairs kept by the cluster
 * bound against, one per cluster of wos_debug_clusters (same cluster order).
 * Like the clusters, they only speed up the distance to the boundary that
 * every walk step queries (Sec. IV-A); the paper has no such structure.
 *   spheres, boxes   as wos_create_domain (either may be NULL)
 *   out_n_cl         host int64[2]: sphere clusters, box clusters
 *   box_sph          host double, capacity n_cl_sph * 2 d (may be NULL): per
 *                    cluster lo[d] then hi[d], the FP32 values of the device
 *                    table (the members' box enlarged by 2^-16 of its
 *                    diagonal on every side, rounded outwards)
 *   box_box          the same for box obstacles
 * Capacities are taken from the counts this call computes: call once with
 * NULL arrays to learn them.  Errors: WOS_EDIM, WOS_EINVAL.
 */
int wos_debug_cluster_boxes(int d, const wos_spheres* spheres, const wos_boxes* boxes, int64_t* out_n_cl,
                            double* box_sph, double* box_box);

/*
 * wos_microbench -- issue-rate microbenchmark on the current device, used as
 * the measured roofline ceiling of the walk kernels.  which: 0 FP32 fused
 * multiply-add (out_rate in FLOP/s, 2 per FMA), 1 FP32 square root
 * (operations/s), 2 the 7-D sphere-distance loop of the walk kernels (sphere
 * evaluations/s).  out_ms (nullable): kernel time.  Synchronous.
 * Errors: WOS_EINVAL (bad which / NULL out_rate), WOS_EHIP.
 */
int wos_microbench(int which, double* out_rate, double* out_ms);

/* wos_last_error -- message for the last failing call on this thread. */
const char* wos_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WOS_H */
