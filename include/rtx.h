/*
 * rtx.h -- C ABI of the MI355X (gfx950) library for two-point ray tracing of
 * every emitter/receiver pair of a ring array through a gridded sound-speed map
 * (arXiv 2511.18511: Sec. 3.2 ray tracing by the shooting method, Sec. 3.3
 * bilinear grid-to-ray interpolation, Sec. 3.4 ray linking, Sec. 3.1 system
 * matrix, Sec. 4.2 trapezoid accumulation along the ray, Appendix: the travel
 * time obeys the Eikonal equation grad T . grad T = 1/c^2).
 *
 * Conventions shared by every call
 *  - Grid: node (ix, iy) of an nx-by-ny grid with spacing h (metres) sits at
 *    x = (ix - (nx-1)/2) h, y = (iy - (ny-1)/2) h.  Node arrays are row-major
 *    [ny][nx] (index iy * nx + ix).  The ring is centred on the grid centre.
 *  - Ring: element k sits at radius `radius` (metres) and angle
 *    phi0 + 2 pi k / n_elem.  A pair is (emitter e, receiver r), e != r.  With
 *    pairs == NULL every ordered pair is traced, pair i being
 *    e = i / (n_elem - 1), k = i % (n_elem - 1), r = k < e ? k : k + 1.
 *  - theta: launch angle of a pair's ray relative to the inward normal at the
 *    emitter (radians, counter-clockwise positive, |theta| < pi/2).
 *  - Ray march: arc-length steps of ds_px pixels of dx/ds = d,
 *    dd/ds = -(G - (G.d) d) / c with G the per-pixel gradient of c, both taken
 *    by bilinear interpolation of node values (the node gradient by second-order
 *    central differences, second-order one-sided at the edges); classic RK4 or
 *    Heun; d renormalised after every step.  The step that crosses the ring is cut
 *    at the crossing (segment/circle intersection), giving a partial step ds'.
 *  - Travel time T = h sum_m w_m / c(p_m) and length L = h ((M-1) ds + ds') with
 *    trapezoid weights w_0 = ds/2, w_m = ds, w_{M-1} = (ds + ds')/2, w_M = ds'/2
 *    over the step points p_0..p_M (p_M = interception point).
 *  - Linking: misfit g = mod(phi_hit - phi_e, 2pi) - mod(phi_r - phi_e, 2pi),
 *    miss_px = |g| radius / h.  Start from the straight-ray angle (or theta on
 *    RTX_WARM_START), second point theta - g/2, then the secant through the two
 *    latest rays that hit, safeguarded by the latest sign bracket of g, by the
 *    angle limits +-(pi/2 - 1e-6) and by halving toward the last hitting angle
 *    after a ray that never reached the ring.  Stops at miss_px <= tol_px
 *    (LINKED) or after max_marches rays (NOT_CONVERGED, best ray returned).
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller unless
 * marked (host).  Calls enqueue work on `stream` (a hipStream_t; NULL = the
 * null stream) and return without waiting; outputs are valid once the stream
 * reaches that point.  The library keeps no reference to caller memory after a
 * call returns.  A plan owns device workspace (the packed medium) and must not
 * be used by two streams at once.
 *
 * Errors: every call returns RTX_OK or a negative RTX_E_* code and then leaves a
 * message for rtx_last_error() (per thread).  Host-detectable argument errors
 * return RTX_E_ARG and enqueue nothing.  Per-ray problems never fail the call:
 * they are reported in the int8 status of each pair (RTX_RAY_*): e == r or an
 * element index out of range -> BAD_INPUT; a non-positive or NaN sound speed met
 * at a ray point -> BAD_INPUT; no crossing within max_steps steps -> NO_HIT.
 */
#ifndef RTX_H
#define RTX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtx_plan_s *rtx_plan;

enum rtx_status {
    RTX_OK = 0,
    RTX_E_ARG = -1,          /* invalid argument (nothing enqueued) */
    RTX_E_HIP = -2,          /* a HIP runtime call or kernel launch failed */
    RTX_E_NOMEM = -3,        /* device allocation failed */
    RTX_E_UNSUPPORTED = -4,  /* option combination not implemented */
    RTX_E_CAPACITY = -5      /* nnz_cap smaller than the number of weights */
};
enum rtx_precision {
    RTX_F64 = 0,  /* every step in FP64 */
    RTX_F32C = 1  /* FP32 march with compensated (2Sum) position, direction and
                     travel-time accumulation; FP64 interception, misfit and
                     secant update */
};
enum rtx_integrator { RTX_HEUN = 2, RTX_RK4 = 4 };
enum rtx_flags {
    RTX_WARM_START = 1u,  /* start linking from the given theta */
    RTX_FIXED_ANGLE = 2u, /* trace once at the given theta, no linking */
    RTX_FAN_START = 4u,   /* cold start seeded from the emitter's fan of straight rays
                             (all ordered pairs only, pairs == NULL): every pair's
                             straight ray is first traced at a coarser step (a
                             seed, not counted); the nearest sign change of the
                             misfit over the rays of neighbouring receivers of
                             the same emitter seeds the secant, with a cubic
                             (first ray) and a quintic (second ray) inverse
                             interpolation of the fan samples; the linking then
                             runs in rounds of two rays (n_marches counts rays,
                             max_marches bounds the rounds).  The plan keeps a
                             mid-path checkpoint of every pair's linked ray
                             (2 x (44 or 84) + 16 bytes per pair of max_pairs),
                             which the all-pairs adjoint uses; see
                             rtx_tof_adjoint */
    RTX_INTERP_BSPLINE = 8u /* plan-wide (set at rtx_plan_create, fixed after):
                               interpolate c and its gradient with the
                               interpolating cubic B-spline of the node values
                               (Sec. 3.3; mirror extension at the grid edges)
                               instead of bilinearly.  Tracing and forward calls
                               only: adjoint, path weights and batches return
                               RTX_E_UNSUPPORTED on such a plan */
};
enum rtx_weight { RTX_W_LENGTH = 0, RTX_W_DTDC = 1 };
enum rtx_resid_kind { RTX_RESID_REAL = 0, RTX_RESID_RAYBORN_C64 = 1 };
enum rtx_ray_status {
    RTX_RAY_LINKED = 0,         /* miss <= tol (FIXED_ANGLE: the ray hit the ring) */
    RTX_RAY_NOT_CONVERGED = 1,  /* max_marches rays, best one returned */
    RTX_RAY_NO_HIT = 2,         /* no traced ray reached the ring */
    RTX_RAY_BAD_INPUT = 3       /* bad pair or bad sound speed on the path */
};

typedef struct {
    int32_t nx, ny; /* nodes; both >= 4 */
    double h;       /* node spacing, metres, > 0 */
} rtx_grid;

typedef struct {
    int32_t n_elem; /* >= 2 */
    double radius;  /* metres; radius/h + max(1, ds_px) <= (min(nx,ny) - 1)/2 */
    double phi0;    /* angle of element 0, radians */
} rtx_ring;

typedef struct {
    int32_t prec;        /* rtx_precision */
    int32_t integ;       /* rtx_integrator */
    double ds_px;        /* step in pixels, 0 < ds_px <= 2 */
    double tol_px;       /* linking tolerance on the miss, pixels, >= 0 */
    int32_t max_marches; /* traced rays per pair, >= 1 (30 is the usual value) */
    int32_t max_steps;   /* steps per ray; 0 = ceil(8 radius / (h ds_px)) */
    uint32_t flags;      /* rtx_flags */
} rtx_opts;

/* Creates a plan: validates grid/ring/opts and allocates device workspace for
   the packed medium (12 coefficients per grid cell in the plan's precision; 16
   with RTX_INTERP_BSPLINE, plus an FP64 [ny][nx] coefficient grid) and for up
   to max_pairs pairs per call.  *out receives the plan (host object). */
int rtx_plan_create(rtx_plan *out, const rtx_grid *grid, const rtx_ring *ring, const rtx_opts *opts,
                    int64_t max_pairs);

/* Frees the plan's device memory (synchronises the device first). */
int rtx_plan_destroy(rtx_plan plan);

/* Changes the per-call options (precision and RTX_INTERP_BSPLINE must not
   change: RTX_E_ARG). */
int rtx_plan_set_opts(rtx_plan plan, const rtx_opts *opts);

/* Packs the medium: c (device, float64 [ny][nx], m/s) -> node gradient and
   per-cell bilinear coefficients of (c, dc/dx, dc/dy) in the plan's precision
   (Sec. 3.3); on an RTX_INTERP_BSPLINE plan, the interpolating cubic B-spline
   coefficients (recursive prefilter in FP64, mirror extension) and each cell's
   4 x 4 stencil of them.  Later calls may pass c == NULL to reuse it. */
int rtx_set_medium(rtx_plan plan, const double *c, void *stream);

/* Linked ray tracing of n_pairs pairs (Sec. 3.2, 3.4): for each pair
     theta     [n] in/out: start (RTX_WARM_START) or fixed angle (RTX_FIXED_ANGLE)
                    on input; the linked (or best) launch angle on output;
     tof       [n] travel time, seconds       (may be NULL)
     len       [n] path length, metres        (may be NULL)
     miss_px   [n] final miss, pixels         (may be NULL)
     n_marches [n] rays traced                (may be NULL)
     status    [n] rtx_ray_status             (required)
   c: float64 [ny][nx] sound speed, or NULL for the medium of rtx_set_medium.
   pairs: int32 [n][2] (emitter, receiver) or NULL for all ordered pairs.
   Path weights (Sec. 3.1): when w_rowptr != NULL the rows
   W_ij = h sum_m w_m phi_j(p_m) of the linked rays are emitted as CSR: with
   w_col == NULL only w_rowptr [n+1] is written (count pass); otherwise w_col
   (int32 node index iy*nx+ix, ascending, unique per row) and w_val (float or
   double per precision, metres) are filled for nnz <= nnz_cap, else
   RTX_E_CAPACITY, with w_rowptr written all the same (so a caller can size
   the buffers from it and call again).  Rows of pairs whose status is NO_HIT
   or BAD_INPUT are empty.  The weights pass synchronises `stream` before
   returning; its scratch (4 n + 1 int64, and the row entries before they are
   merged, as int32 + value) is plan-owned and grown when a larger W
   arrives. */
int rtx_trace_rays(rtx_plan plan, const double *c, const int32_t *pairs, int64_t n_pairs, double *theta,
                   double *tof, double *len, double *miss_px, int32_t *n_marches, int8_t *status,
                   int64_t *w_rowptr, int32_t *w_col, void *w_val, int64_t nnz_cap, void *stream);

/* Forward travel time only (the operator of the ToF inversion, Sec. 3.1):
   same as rtx_trace_rays with len, miss, n_marches and weights omitted. */
int rtx_tof_forward(rtx_plan plan, const double *c, const int32_t *pairs, int64_t n_pairs, double *theta,
                    double *tof, int8_t *status, void *stream);

/* SART (Sec. 3.1: the default solver of the linearised ToF subproblem; the
   simultaneous algebraic reconstruction technique of Andersen and Kak) on the
   system matrix W of rtx_trace_rays: n_iter iterations of
     x_j <- x_j + lambda / V_j * sum_i W_ij (b_i - sum_l W_il x_l) / M_i
   with row sums M_i and column sums V_j of W, all columns updated from the
   previous iterate; rows with M_i == 0 (empty rows) and columns with V_j == 0
   (nodes no ray touches) take no part.
     w_rowptr [n_rows + 1] int64, w_col [nnz] int32, w_val [nnz] float
              (RTX_F32C plans) or double (RTX_F64): CSR as emitted by
              rtx_trace_rays (device); entries k outside [0, nnz) and columns
              outside [0, nx * ny) are left out
     b        [n_rows] float64 (device): data, e.g. travel-time residuals (s)
     x        [ny * nx] float64 (device, in/out): start and result, e.g. the
              slowness update (s/m); column index = iy * nx + ix
   The call transposes W once (CSC, built on the device by a stable radix
   sort of the entries by column, so rows stay ascending inside a column and
   the result is the same on every run) and then streams W by rows and by
   columns each iteration; arithmetic is FP64.  w_rowptr must be
   non-decreasing (otherwise the result is undefined; memory accesses stay in
   bounds).  Plan-owned scratch: about (2 max_pairs + 2 nx ny) x 8 bytes on
   first use, and about 2 (8 + entry size) x nnz bytes for the transpose and
   the sort (entry size 8 for float, 16 for double), grown when a larger W
   arrives (a call that grows it frees and allocates).
   Errors: n_rows < 0 or > max_pairs, nnz < 0, n_iter < 0, lambda outside
   (0, 2), missing buffers -> RTX_E_ARG (nothing enqueued); RTX_E_NOMEM.
   n_rows == 0 or n_iter == 0 leaves x unchanged. */
int rtx_sart(rtx_plan plan, int64_t n_rows, int64_t nnz, const int64_t *w_rowptr, const int32_t *w_col,
             const void *w_val, const double *b, double *x, int32_t n_iter, double lambda, void *stream);

/* Paraxial ray (Sec. 3.5: the default way to the ray Jacobian that the
   geometric spreading of the ray-Born Green's functions needs) along the rays
   traced at the given launch angles, typically the linked ones.  The
   first-order perturbation (dx, dd) of position and direction per unit change
   of the launch angle is integrated with the ray by the same Runge-Kutta
   scheme (the standard variational equations of the ray equations of Sec. 3.2;
   the paper cites them only).  Per pair (each output may be NULL except status):
     dgdth  [n] float64: derivative of the interception angle, and so of the
                misfit g, with respect to the launch angle
     jac    [n] float64: ray Jacobian at the interception, u x dx with u the
                direction of the crossing step, metres per radian (the width
                of the ray tube; its sign flips at each caustic)
     amp    [n] float64: geometric-spreading amplitude sqrt(c(x_r) /
                (c(x_e) |jac|)), 1/sqrt(m): the 2-D transport-equation solution
                normalised to the point-source far field (1/sqrt(distance) in a
                homogeneous medium)
     kmah   [n] int32: sign changes of the Jacobian along the ray (caustics)
     status [n] int8: rtx_ray_status of the traced ray; outputs are NaN / -1
                unless LINKED
   theta [n] float64 launch angles (as rtx_trace_rays); pairs and c as in
   rtx_trace_rays; the plan's precision, integrator, step, step limit and
   interpolation apply.  Errors as rtx_trace_rays (RTX_E_ARG, nothing
   enqueued). */
int rtx_paraxial(rtx_plan plan, const double *c, const int32_t *pairs, int64_t n_pairs, const double *theta,
                 double *dgdth, double *jac, double *amp, int32_t *kmah, int8_t *status, void *stream);

/* Free march without a ring: the ray equations of Sec. 3.2 followed for a
   fixed number of steps, as in the trajectory (radius) experiment of Sec. 4.1.
     x0   [n_rays][2] float64, device: start points, metres from the grid centre
     d0   [n_rays][2] float64, device: start directions (normalised on the device)
     pts  [n_rays][n_steps + 1][2] float64, device, caller-owned: the start
          point and the end point of every step, metres from the grid centre
   The plan's step ds_px, integrator, precision and interpolation apply; the
   ring plays no part.  From the first point outside the node rectangle on (and
   for a zero or non-finite direction) the points are NaN.  Near the edges the
   stage points of a step sample the field of the nearest cell.
   c: as in rtx_trace_rays.  Errors: n_rays < 0 or >= 2^31 - 256, n_steps < 0
   or >= 2^30, missing buffers -> RTX_E_ARG (nothing enqueued); n_rays == 0
   only packs c. */
int rtx_march_free(rtx_plan plan, const double *c, int64_t n_rays, const double *x0, const double *d0,
                   int32_t n_steps, double *pts, void *stream);

/* Adjoint of the path weights along the rays traced at the given theta:
     grad_j += sum_i rho_i sum_m w_m h kappa_m phi_j(p_m)
   kappa = 1 (RTX_W_LENGTH: transpose of the system matrix) or
   kappa = -1/c(p_m)^2 (RTX_W_DTDC: frozen-path derivative of T with respect to
   the node sound speeds, i.e. the travel-time gradient).
   rho = resid (RTX_RESID_REAL: float64 [n]) or, for RTX_RESID_RAYBORN_C64,
   rho_i = sum_k w_k Im(exp(-i w_k T_i) r_ik) with w_k = 2 pi freqs_hz[k]
   (freqs_hz host [n_freq]), r complex64 [n][n_freq] interleaved (re, im) and
   T = tof (float64 [n], required for this kind): the adjoint of phase-only data
   exp(i w T).  status (required, int8 [n], as returned by the forward call)
   selects the pairs used: those whose status is LINKED or NOT_CONVERGED, i.e.
   whose theta is a traced ray that reached the ring; others are skipped.  grad: [ny][nx] float (RTX_F32C) or double
   (RTX_F64), accumulated into (the caller zeroes it).  Accumulation uses
   atomics, so the FP32 result depends on summation order at rounding level.
   The updates first go to zeroed copies of the grid that the plan allocates on
   its first adjoint call (as many as fit in 64 MiB, at most 8; with room for
   fewer than two they go to grad directly), and a final kernel adds the copies
   into grad and zeroes them again.
   All pairs (pairs == NULL) after an RTX_FAN_START trace on the same plan,
   with the same medium and path options (ds_px, integrator, max_steps) since:
   a pair whose theta equals the angle that trace linked is marched as two
   halves, the second starting from the trace's mid-path checkpoint (the same
   samples as marching on, so the result is the same up to summation order);
   any other pair is marched whole.
   Node updates pass through a bounded queue in on-chip memory; if one of its
   waits ever hits its bound, the gradient is incomplete and the next
   rtx_plan_stats call on the plan returns RTX_E_HIP. */
int rtx_tof_adjoint(rtx_plan plan, const double *c, const int32_t *pairs, int64_t n_pairs,
                    const double *theta, const int8_t *status, const double *tof, const void *resid,
                    int32_t resid_kind, const double *freqs_hz, int32_t n_freq, int32_t weight, void *grad,
                    void *stream);

/* Work counters of the last trace / adjoint call on this plan (synchronises the
   device): total RK steps marched and rays traced (both trace passes of a fan
   start), and adjoint steps.  Returns RTX_E_HIP (and still fills the counters)
   if an adjoint of this plan reported an incomplete gradient. */
int rtx_plan_stats(rtx_plan plan, int64_t *trace_steps, int64_t *trace_rays, int64_t *adjoint_steps);

/* Work counters of one kernel launch of the last call: region 0 = the trace
   kernel (the fixed straight-ray pass under RTX_FAN_START), 1 = the linking pass
   of a fan start, 2 = the adjoint. */
int rtx_plan_region_stats(rtx_plan plan, int32_t region, int64_t *steps, int64_t *rays);

/* Per-kernel timing: while enabled, every kernel the plan launches is bracketed
   by HIP events recorded on its launch stream.  rtx_plan_timing(plan, 1) starts
   (and resets) it, 0 stops it; rtx_plan_timings (synchronises the device)
   returns per slot (host arrays of RTX_NUM_SLOTS) the summed milliseconds and
   the number of launches since the reset. */
enum rtx_slot { RTX_SLOT_PACK = 0, RTX_SLOT_TRACE = 1, RTX_SLOT_FAN_SEED = 2, RTX_SLOT_FAN_LINK = 3,
                RTX_SLOT_ADJOINT = 4, RTX_NUM_SLOTS = 5 };
int rtx_plan_timing(rtx_plan plan, int32_t enable);
int rtx_plan_timings(rtx_plan plan, double *total_ms, int32_t *count);

/* Launch shape of the plan's persistent kernels: rays (threads) per block,
   64, 128 or 256 (default 256).  Results do not depend on it; the autotuner
   in the Python package picks it per workload. */
int rtx_plan_set_launch(rtx_plan plan, int32_t rays_per_block);

/* ---- batched independent instances (one launch graph) ---------------------
   Many (medium, ring, pairs) problems traced by one persistent kernel over the
   concatenated pair space, optionally followed by one adjoint kernel; the whole
   run (counter reset, medium packing of every instance, trace, adjoint) is
   captured into a HIP graph on the first rtx_batch_run and replayed after.
   Every instance shares the batch's rtx_opts (precision, integrator, step,
   tolerance, limits, flags).  All arrays are caller-owned device memory that
   must stay valid for the batch's lifetime (the graph keeps the pointers). */
typedef struct {
    rtx_grid grid;
    rtx_ring ring;
    const double *c;        /* float64 [ny][nx] sound speed */
    const int32_t *pairs;   /* int32 [n][2] or NULL = all ordered pairs */
    int64_t n_pairs;        /* >= 1; n_elem (n_elem - 1) when pairs == NULL */
    double *theta;          /* [n] in/out, as in rtx_trace_rays (required) */
    double *tof, *len, *miss_px; /* [n] outputs (may be NULL) */
    int32_t *n_marches;     /* [n] (may be NULL) */
    int8_t *status;         /* [n] (required) */
    const double *resid;    /* float64 [n] adjoint residual rho, or NULL (then for every instance) */
    void *grad;             /* [ny][nx] float/double per precision, accumulated into (with resid) */
} rtx_instance;

typedef struct rtx_batch_s *rtx_batch;

/* Validates every instance (as rtx_plan_create does), allocates the packed
   tables and per-instance descriptors.  weight: rtx_weight of the adjoint.
   rays_per_block: 0 (default 256), 64, 128 or 256.  inst is (host) [n_inst].
   A batch holds at most 255 instances (else RTX_E_UNSUPPORTED) whose grids
   hold at most 2^24 nodes each (else RTX_E_ARG): the adjoint tags each node
   update with its instance in 8 bits. */
int rtx_batch_create(rtx_batch *out, const rtx_opts *opts, int32_t weight, int32_t rays_per_block,
                     int32_t n_inst, const rtx_instance *inst);

/* Enqueues one run of the batch graph on stream. */
int rtx_batch_run(rtx_batch batch, void *stream);

/* Per-instance completion of the last run (synchronises the device), in ms from
   the start of the run, from the device wall clock: fwd_ms when the instance's
   last pair was linked, done_ms when its last adjoint ray finished (= fwd_ms
   without adjoint).  Both (host) [n_inst], either may be NULL.  Returns
   RTX_E_HIP if the batch's adjoint reported incomplete gradients. */
int rtx_batch_times(rtx_batch batch, double *fwd_ms, double *done_ms);

/* Frees the batch (synchronises the device first). */
int rtx_batch_destroy(rtx_batch batch);

/* Message of the last failed call on this thread ("" if none). */
const char *rtx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RTX_H */
