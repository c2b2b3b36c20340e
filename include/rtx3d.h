/* rtx3d.h -- C ABI of the 3-D two-point ray tracer (HIP, gfx950).
 *
 * Ray tracing between point transducers on a sphere (hemispherical arrays,
 * arXiv 2511.18511 Sec. 3: the ToF method extended to 3-D acquisition
 * geometries) through a gridded sound-speed volume, with the Broyden-like
 * ray linking of Sec. 3.4 for 3-D configurations: the launch direction has two
 * angular parameters and every update traces one ray, the Jacobian estimate
 * being updated from the two most recent iterates.  Travel time and path length
 * follow Sec. 4.2's trapezoid rule.  Options, flags, precisions and statuses
 * are those of rtx.h.
 *
 * Conventions (the same as the CPU oracle's, which is independent code):
 *  - Volume c [nz][ny][nx] float64 in m/s on the device; node (ix, iy, iz) at
 *    ((ix - (nx-1)/2) h, (iy - (ny-1)/2) h, (iz - (nz-1)/2) h) metres.  The
 *    field and its node gradient (second-order central differences, one-sided
 *    at the faces) are interpolated trilinearly from the 8 vertices of the
 *    enclosing cell (Sec. 3.3 in 3-D).
 *  - Elements: host array elem [n_elem][3] (metres from the grid centre), all
 *    on one sphere |x| = R, which is also the interception boundary.
 *  - Launch parameters u = (u1, u2) per pair: the direction is
 *    normalize(n + u1 a1 + u2 a2) with n the inward normal at the emitter and
 *    (a1, a2) its tangent basis: a1 = normalize(k x n), a2 = n x a1, with
 *    k = (0, 0, 1), or (1, 0, 0) when |n_z| > 0.9.
 *  - Misfit g = (b1 . (q - r), b2 . (q - r)) / R with (b1, b2) the receiver's
 *    tangent basis built the same way, q the interception; miss = |q - r|
 *    (pixels, compared with tol_px).
 *  - Linking: start at the straight ray to the receiver (or the given u with
 *    RTX_WARM_START) with the homogeneous-medium Jacobian there; after each
 *    ray that hits, Broyden's rank-one update J += (dg - J du) du^T / |du|^2
 *    from the two latest hitting iterates and the step u -= J^-1 g, capped at
 *    length 0.5; a near-singular J (|det| <= 1e-12 (sum |J_ij|)^2) is replaced
 *    by the homogeneous Jacobian at the current u; a ray that does not reach
 *    the sphere within max_steps steps backs off to the midpoint with the
 *    latest hitting iterate (or halves u); at most max_marches rays, else the
 *    ray of smallest miss (NOT_CONVERGED).  RTX_FIXED_ANGLE traces one ray at
 *    the given u.  RTX_FAN_START and RTX_INTERP_BSPLINE are not supported here.
 *
 * Errors: every call returns an rtx_status; rtx3_last_error() describes the
 * last failure of this thread's 3-D calls.  Device pointers stay owned by the
 * caller; calls are enqueued on `stream` (a hipStream_t) and return without
 * waiting unless stated.
 */
#ifndef RTX3D_H
#define RTX3D_H

#include <stdint.h>

#include "rtx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtx3_plan_s *rtx3_plan;

typedef struct {
    int32_t nx, ny, nz; /* nodes per axis, >= 4 each, nx ny nz <= 2^28 */
    double h;           /* node spacing, metres */
} rtx3_grid;

/* Creates a plan: validates the grid, the options and the elements (n_elem >=
   2, all at distance R from the centre to 1e-9 relative, the sphere inside the
   grid with a margin of max(1, ds_px) pixels), copies the elements to the
   device and allocates the node table (4 values per node in the plan's
   precision) for up to max_pairs pairs per call. */
int rtx3_plan_create(rtx3_plan *out, const rtx3_grid *grid, int32_t n_elem, const double *elem, const rtx_opts *opts,
                     int64_t max_pairs);

/* Frees the plan's device memory (synchronises the device first). */
int rtx3_plan_destroy(rtx3_plan plan);

/* Changes the per-call options (precision must not change). */
int rtx3_plan_set_opts(rtx3_plan plan, const rtx_opts *opts);

/* Packs the volume c (device, float64 [nz][ny][nx], m/s) into the node table
   (c and its per-pixel node gradient).  Later calls may pass c == NULL. */
int rtx3_set_medium(rtx3_plan plan, const double *c, void *stream);

/* Linked (Broyden-like, Sec. 3.4) or fixed-direction tracing of n_pairs pairs:
     u         [n][2] float64 in/out: start (RTX_WARM_START) or fixed
                      (RTX_FIXED_ANGLE) parameters on input; the linked (or best)
                      ones on output
     tof       [n] travel time, s          (may be NULL)
     len       [n] path length, m          (may be NULL)
     miss_px   [n] final miss, pixels      (may be NULL)
     n_marches [n] rays traced             (may be NULL)
     status    [n] rtx_ray_status          (required)
   pairs: int32 [n][2] (emitter, receiver) device, or NULL for all ordered
   pairs e (n_elem - 1) + (r < e ? r : r - 1).  c as rtx3_set_medium (NULL:
   the packed one).  Errors: RTX_E_ARG (bad sizes, n > max_pairs, missing
   buffers), RTX_E_UNSUPPORTED (fan start, B-spline), RTX_E_HIP. */
int rtx3_trace_rays(rtx3_plan plan, const double *c, const int32_t *pairs, int64_t n_pairs, double *u, double *tof,
                    double *len, double *miss_px, int32_t *n_marches, int8_t *status, void *stream);

/* Free march (the trajectory experiment of Sec. 4.1 in 3-D): ray i from x0[i]
   (metres from the grid centre, float64 [n][3], device) along d0[i] (any
   non-zero length) for n_steps steps; pts [n][n_steps + 1][3] float64 (device)
   receives the start and every step's end point in metres, NaN from the first
   point outside the node box on.  Errors as rtx_march_free. */
int rtx3_march_free(rtx3_plan plan, const double *c, int64_t n_rays, const double *x0, const double *d0,
                    int32_t n_steps, double *pts, void *stream);

/* Steps and rays of the last rtx3_trace_rays call (synchronises the device). */
int rtx3_plan_stats(rtx3_plan plan, int64_t *steps, int64_t *rays);

/* Text of this thread's last 3-D error ("" if none). */
const char *rtx3_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RTX3D_H */
