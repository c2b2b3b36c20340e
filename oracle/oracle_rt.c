/*
 * oracle_rt.c -- plain, slow FP64 CPU oracle for two-point (shooting) ray tracing
 * through a gridded sound-speed map, with ray linking, travel time, path length,
 * sparse ray-to-grid weights and their adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP path.
 *
 * What it follows (arXiv 2511.18511):
 *   - Sec. 3.2 (ray tracing): shooting method, an initial-value problem per ray in
 *     the position x and unit direction d, driven by the medium and its gradient.
 *   - Sec. 3.3 (grid-to-ray interpolation): bilinear interpolation of the field
 *     and of its gradient, the gradient being taken from values on grid nodes,
 *     using only the vertices of the enclosing cell.
 *   - Sec. 3.4 (ray linking): misfit = angular discrepancy between the ray's
 *     interception with the boundary and the receiver; secant update of the launch
 *     angle (default), regula-falsi style bracketing; straight-ray initial guess
 *     for a homogeneous start, warm start from previous launch angles.
 *   - Sec. 3.1 (linearisation): a system-matrix row holds the interpolation
 *     coefficients of the sampled ray points, accumulated per grid node.
 *   - Sec. 4.2, trapezoid rule for the accumulated length with a partial last
 *     step ds' whose end point is replaced by the interception point.
 *   - Appendix: travel time obeys grad T . grad T = 1/c^2, T = integral ds / c.
 *
 * Readings where the paper is silent (the same list is kept with the design
 * notes): c itself is interpolated and T integrates 1/c; the node gradient is
 * second-order central differences, second-order one-sided at the grid edges;
 * the ray ODE is dx/ds = d, dd/ds = -(G - (G.d) d)/c in pixel units
 * (G = per-pixel gradient of c), integrated by classic RK4 or Heun, with d
 * renormalised after every step; the last step is cut at the ring by a
 * segment/circle intersection; the same trapezoid weights serve T, L and the
 * weights; the misfit is the emitter-relative unwrapped angle; the secant is
 * safeguarded by a sign bracket and by angle limits (details at link_pair).
 *
 * Units: positions in pixels relative to the grid centre (= ring centre), grid
 * node (ix, iy) at pixel (ix - (nx-1)/2, iy - (ny-1)/2); c in m/s; h in metres.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_GRID 0
#define OR_FISHEYE 1 /* analytic c = c0 (1 + |x|^2 / R^2), params {c0, R} */
#define OR_LINEAR 2  /* analytic c = c0 + ax x + ay y,   params {c0, ax, ay} */
#define OR_BSPLINE 3 /* grid, cubic B-spline interpolation of c (gradient analytic) */

#define ST_LINKED 0
#define ST_NOT_CONVERGED 1
#define ST_NO_HIT 2
#define ST_BAD_INPUT 3

#define OPT_WARM 1
#define OPT_FIXED 2
#define OPT_FAN 4

static const double PI = 3.14159265358979323846;

typedef struct {
    int kind;
    int nx, ny;
    double h;
    const double *c; /* [ny][nx] */
    double *gx, *gy; /* per-pixel gradient of c on nodes */
    double *bs;      /* cubic B-spline coefficients of c (OR_BSPLINE) */
    double p[4];
} Medium;

typedef struct {
    int n_elem;
    double radius_px;
    double phi0;
} Ring;

typedef struct {
    int integ; /* 2 = Heun, 4 = RK4 */
    double ds;  /* step, pixels */
    double tol; /* linking tolerance on the miss, pixels */
    int max_marches;
    int max_steps;
    int flags;
} Opts;

/* ---------------------------------------------------------------- gradient -- */
/* Second-order finite differences in index units along x (axis of ix) and y.
   Interior: (f[i+1] - f[i-1]) / 2.  Edges: (-3 f0 + 4 f1 - f2) / 2 and
   (3 f[n-1] - 4 f[n-2] + f[n-3]) / 2.  Needs n >= 3 along both axes. */
int or_gradient(int nx, int ny, const double *c, double *gx, double *gy)
{
    if (nx < 3 || ny < 3) return -1;
    for (int iy = 0; iy < ny; iy++) {
        for (int ix = 0; ix < nx; ix++) {
            double d;
            if (ix == 0)
                d = (-3.0 * c[iy * nx + 0] + 4.0 * c[iy * nx + 1] - c[iy * nx + 2]) / 2.0;
            else if (ix == nx - 1)
                d = (3.0 * c[iy * nx + nx - 1] - 4.0 * c[iy * nx + nx - 2] + c[iy * nx + nx - 3]) / 2.0;
            else
                d = (c[iy * nx + ix + 1] - c[iy * nx + ix - 1]) / 2.0;
            gx[iy * nx + ix] = d;
        }
    }
    for (int iy = 0; iy < ny; iy++) {
        for (int ix = 0; ix < nx; ix++) {
            double d;
            if (iy == 0)
                d = (-3.0 * c[0 * nx + ix] + 4.0 * c[1 * nx + ix] - c[2 * nx + ix]) / 2.0;
            else if (iy == ny - 1)
                d = (3.0 * c[(ny - 1) * nx + ix] - 4.0 * c[(ny - 2) * nx + ix] + c[(ny - 3) * nx + ix]) / 2.0;
            else
                d = (c[(iy + 1) * nx + ix] - c[(iy - 1) * nx + ix]) / 2.0;
            gy[iy * nx + ix] = d;
        }
    }
    return 0;
}

/* ------------------------------------------------------------- bilinear cell -- */
/* Enclosing cell of pixel position (px, py): lower-left node (ix, iy) and local
   coordinates (t, s) in [0,1].  The cell index is clamped to the grid and the
   local coordinates to [0,1].  Returns 0 on a NaN position. */
static int locate(const Medium *m, double px, double py, int *ix, int *iy, double *t, double *s)
{
    double u = px + 0.5 * (m->nx - 1);
    double v = py + 0.5 * (m->ny - 1);
    if (!(u == u) || !(v == v)) return 0;
    double fu = floor(u), fv = floor(v);
    if (fu < 0) fu = 0;
    if (fu > m->nx - 2) fu = m->nx - 2;
    if (fv < 0) fv = 0;
    if (fv > m->ny - 2) fv = m->ny - 2;
    double tt = u - fu, ss = v - fv;
    if (tt < 0) tt = 0;
    if (tt > 1) tt = 1;
    if (ss < 0) ss = 0;
    if (ss > 1) ss = 1;
    *ix = (int)fu;
    *iy = (int)fv;
    *t = tt;
    *s = ss;
    return 1;
}

/* Bilinear hat weights of the four cell corners, order (ix,iy), (ix+1,iy),
   (ix,iy+1), (ix+1,iy+1). */
static void hat4(double t, double s, double w[4])
{
    w[0] = (1.0 - t) * (1.0 - s);
    w[1] = t * (1.0 - s);
    w[2] = (1.0 - t) * s;
    w[3] = t * s;
}

/* ----------------------------------------------------------- cubic B-spline -- */
/* Sec. 3.3: cubic B-spline interpolation, control points at the grid nodes, C2
   field, first derivatives analytic, 4-node stencil per axis.  Reading: the
   interpolating spline (its coefficients solve sum_k b(k - j) coef_k = c_j with
   the centred cubic B-spline b, so the spline passes through the node values),
   mirror-symmetric extension at the grid edges.  The coefficients come from the
   standard two-pass recursive filter with pole z = sqrt(3) - 2 (causal then
   anti-causal, gain 6), applied along x then along y. */
static void bspline_filter_line(double *v, int n, int stride)
{
    const double z = sqrt(3.0) - 2.0;
    /* causal initialisation: sum over the mirror-extended signal of v[k] z^k,
       in closed form for the period-2(n-1) extension */
    double zn = z, iz = 1.0 / z, z2n = pow(z, (double)(n - 1));
    double sum = v[0] + z2n * v[(n - 1) * stride];
    z2n *= z2n * iz;
    for (int k = 1; k <= n - 2; k++) {
        sum += (zn + z2n) * v[k * stride];
        zn *= z;
        z2n *= iz;
    }
    v[0] = sum / (1.0 - zn * zn);
    for (int k = 1; k < n; k++) v[k * stride] += z * v[(k - 1) * stride];
    /* anti-causal initialisation for the mirror boundary */
    v[(n - 1) * stride] = (z / (z * z - 1.0)) * (v[(n - 1) * stride] + z * v[(n - 2) * stride]);
    for (int k = n - 2; k >= 0; k--) v[k * stride] = z * (v[(k + 1) * stride] - v[k * stride]);
    for (int k = 0; k < n; k++) v[k * stride] *= 6.0;
}

/* centred cubic B-spline weights of the nodes at offsets -1, 0, 1, 2 from the
   cell's lower node, local coordinate t in [0, 1], and their derivatives */
static void bspline_w(double t, double w[4], double dw[4])
{
    double u = 1.0 - t;
    w[0] = u * u * u / 6.0;
    w[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    w[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    w[3] = t * t * t / 6.0;
    dw[0] = -u * u / 2.0;
    dw[1] = (3.0 * t * t - 4.0 * t) / 2.0;
    dw[2] = (-3.0 * t * t + 2.0 * t + 1.0) / 2.0;
    dw[3] = t * t / 2.0;
}

static int mirror(int i, int n)
{
    if (i < 0) return -i;
    if (i > n - 1) return 2 * (n - 1) - i;
    return i;
}

/* c (m/s) and its per-pixel gradient at pixel position (px, py). */
static void medium_eval(const Medium *m, double px, double py, double *c, double *gx, double *gy)
{
    if (m->kind == OR_BSPLINE) {
        int ix, iy;
        double t, s, wx[4], dwx[4], wy[4], dwy[4];
        if (!locate(m, px, py, &ix, &iy, &t, &s)) {
            *c = *gx = *gy = NAN;
            return;
        }
        bspline_w(t, wx, dwx);
        bspline_w(s, wy, dwy);
        double v = 0, vx = 0, vy = 0;
        for (int b = 0; b < 4; b++) {
            int jy = mirror(iy - 1 + b, m->ny);
            for (int a = 0; a < 4; a++) {
                int jx = mirror(ix - 1 + a, m->nx);
                double cf = m->bs[jy * m->nx + jx];
                v += cf * wx[a] * wy[b];
                vx += cf * dwx[a] * wy[b];
                vy += cf * wx[a] * dwy[b];
            }
        }
        *c = v;
        *gx = vx;
        *gy = vy;
        return;
    }
    if (m->kind == OR_FISHEYE) {
        double x = px * m->h, y = py * m->h, c0 = m->p[0], R = m->p[1];
        *c = c0 * (1.0 + (x * x + y * y) / (R * R));
        *gx = c0 * 2.0 * x / (R * R) * m->h;
        *gy = c0 * 2.0 * y / (R * R) * m->h;
        return;
    }
    if (m->kind == OR_LINEAR) {
        double x = px * m->h, y = py * m->h;
        *c = m->p[0] + m->p[1] * x + m->p[2] * y;
        *gx = m->p[1] * m->h;
        *gy = m->p[2] * m->h;
        return;
    }
    int ix, iy;
    double t, s, w[4];
    if (!locate(m, px, py, &ix, &iy, &t, &s)) {
        *c = NAN;
        *gx = NAN;
        *gy = NAN;
        return;
    }
    hat4(t, s, w);
    int n0 = iy * m->nx + ix, n1 = n0 + 1, n2 = n0 + m->nx, n3 = n2 + 1;
    *c = w[0] * m->c[n0] + w[1] * m->c[n1] + w[2] * m->c[n2] + w[3] * m->c[n3];
    *gx = w[0] * m->gx[n0] + w[1] * m->gx[n1] + w[2] * m->gx[n2] + w[3] * m->gx[n3];
    *gy = w[0] * m->gy[n0] + w[1] * m->gy[n1] + w[2] * m->gy[n2] + w[3] * m->gy[n3];
}

/* ---------------------------------------------------------------- ray ODE -- */
/* State y = (x1, x2, d1, d2).  dx/ds = d; dd/ds = -(G - (G.d) d) / c. */
static void rhs(const Medium *m, const double y[4], double k[4])
{
    double c, gx, gy;
    medium_eval(m, y[0], y[1], &c, &gx, &gy);
    double gd = gx * y[2] + gy * y[3];
    k[0] = y[2];
    k[1] = y[3];
    k[2] = -(gx - gd * y[2]) / c;
    k[3] = -(gy - gd * y[3]) / c;
}

/* One step of length ds; the direction is renormalised afterwards. */
static void step(const Medium *m, int integ, double ds, const double y[4], double out[4])
{
    double k1[4], k2[4], k3[4], k4[4], tmp[4];
    if (integ == 2) { /* Heun: explicit trapezoid RK2 */
        rhs(m, y, k1);
        for (int i = 0; i < 4; i++) tmp[i] = y[i] + ds * k1[i];
        rhs(m, tmp, k2);
        for (int i = 0; i < 4; i++) out[i] = y[i] + ds / 2.0 * (k1[i] + k2[i]);
    } else { /* classic fourth-order Runge-Kutta */
        rhs(m, y, k1);
        for (int i = 0; i < 4; i++) tmp[i] = y[i] + ds / 2.0 * k1[i];
        rhs(m, tmp, k2);
        for (int i = 0; i < 4; i++) tmp[i] = y[i] + ds / 2.0 * k2[i];
        rhs(m, tmp, k3);
        for (int i = 0; i < 4; i++) tmp[i] = y[i] + ds * k3[i];
        rhs(m, tmp, k4);
        for (int i = 0; i < 4; i++) out[i] = y[i] + ds / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    double nrm = sqrt(out[2] * out[2] + out[3] * out[3]);
    out[2] /= nrm;
    out[3] /= nrm;
}

/* --------------------------------------------------------------- one march -- */
typedef struct {
    int status;   /* ST_LINKED here means "hit the ring" */
    int M;        /* index of the last sample (the interception point) */
    double dsp;   /* partial last step, pixels */
    double qx, qy;
    double *pts;  /* samples p_0..p_M, [M+1][2] pixels (owned, malloc) */
} March;

static double mod2pi(double a)
{
    double r = fmod(a, 2.0 * PI);
    if (r < 0) r += 2.0 * PI;
    return r;
}

/* Traces one ray from pixel point (ex, ey) with initial direction angle psi0
   until it crosses the ring |x| = R.  Samples p_m are the accepted step points;
   the crossing step m is cut at the larger root t in (0,1] of
   |p_{m-1} + t (p_m - p_{m-1})|^2 = R^2, the interception q replaces p_m and
   ds' = t ds.  More than max_steps steps without a crossing -> ST_NO_HIT.  A
   non-positive or NaN sound speed at a sample -> ST_BAD_INPUT. */
static void march(const Medium *m, const Ring *ring, const Opts *o, double ex, double ey, double psi0, March *r)
{
    int cap = 1024, n = 1;
    double *pts = (double *)malloc(sizeof(double) * 2 * cap);
    double y[4] = {ex, ey, cos(psi0), sin(psi0)}, yn[4];
    double R = ring->radius_px;
    pts[0] = ex;
    pts[1] = ey;
    r->status = ST_NO_HIT;
    r->M = 0;
    r->dsp = 0;
    r->qx = r->qy = NAN;
    for (int mstep = 1; mstep <= o->max_steps; mstep++) {
        double c, gx, gy;
        medium_eval(m, y[0], y[1], &c, &gx, &gy);
        if (!(c > 0.0)) {
            r->status = ST_BAD_INPUT;
            break;
        }
        step(m, o->integ, o->ds, y, yn);
        if (n + 1 > cap) {
            cap *= 2;
            pts = (double *)realloc(pts, sizeof(double) * 2 * cap);
        }
        if (yn[0] * yn[0] + yn[1] * yn[1] >= R * R) {
            double ax = yn[0] - y[0], ay = yn[1] - y[1];
            double A = ax * ax + ay * ay;
            double B = 2.0 * (y[0] * ax + y[1] * ay);
            double C = y[0] * y[0] + y[1] * y[1] - R * R;
            double D = B * B - 4.0 * A * C;
            if (D < 0) D = 0;
            double t = (B >= 0) ? (-2.0 * C) / (B + sqrt(D)) : (-B + sqrt(D)) / (2.0 * A);
            if (t > 1.0) t = 1.0;
            if (t < 0.0) t = 0.0;
            r->qx = y[0] + t * ax;
            r->qy = y[1] + t * ay;
            r->dsp = t * o->ds;
            pts[2 * n] = r->qx;
            pts[2 * n + 1] = r->qy;
            r->M = n;
            n++;
            double cq, gqx, gqy;
            medium_eval(m, r->qx, r->qy, &cq, &gqx, &gqy);
            r->status = (cq > 0.0) ? ST_LINKED : ST_BAD_INPUT;
            break;
        }
        for (int i = 0; i < 4; i++) y[i] = yn[i];
        pts[2 * n] = y[0];
        pts[2 * n + 1] = y[1];
        n++;
        r->M = n - 1;
    }
    r->pts = pts;
}

/* Trapezoid weights (pixels) of samples 0..M with partial last step dsp:
   w0 = ds/2, wm = ds (1 <= m <= M-2), w_{M-1} = (ds + ds')/2, w_M = ds'/2;
   M = 1: w0 = w1 = ds'/2. */
static double trap_weight(int mi, int M, double ds, double dsp)
{
    if (M == 1) return dsp / 2.0;
    if (mi == 0) return ds / 2.0;
    if (mi == M) return dsp / 2.0;
    if (mi == M - 1) return (ds + dsp) / 2.0;
    return ds;
}

/* T = sum w_m h / c(p_m) (seconds), L = ((M-1) ds + ds') h (metres). */
static void quadrature(const Medium *m, const March *r, double ds, double *T, double *L)
{
    double acc = 0.0;
    for (int i = 0; i <= r->M; i++) {
        double c, gx, gy;
        medium_eval(m, r->pts[2 * i], r->pts[2 * i + 1], &c, &gx, &gy);
        acc += trap_weight(i, r->M, ds, r->dsp) * m->h / c;
    }
    *T = acc;
    *L = ((r->M - 1) * ds + r->dsp) * m->h;
}

/* ---------------------------------------------------------------- geometry -- */
static double elem_angle(const Ring *ring, int k)
{
    return ring->phi0 + 2.0 * PI * k / ring->n_elem;
}

/* Emitter-relative unwrapped angular misfit of an interception point. */
static double misfit(const Ring *ring, int e, int rcv, double qx, double qy)
{
    double pe = elem_angle(ring, e), pr = elem_angle(ring, rcv);
    return mod2pi(atan2(qy, qx) - pe) - mod2pi(pr - pe);
}

static double straight_angle(const Ring *ring, int e, int rcv)
{
    return (mod2pi(elem_angle(ring, rcv) - elem_angle(ring, e)) - PI) / 2.0;
}

/* ------------------------------------------------------------------ linking -- */
typedef struct {
    double theta, T, L, miss;
    int n_marches, status;
} LinkOut;

/* Traces one ray of pair (e, rcv) at launch angle theta (relative to the inward
   normal at e) and returns status, misfit g and T, L of the march. */
static int trace_at(const Medium *m, const Ring *ring, const Opts *o, int e, int rcv, double theta,
                    double *g, double *T, double *L, March *keep)
{
    double pe = elem_angle(ring, e);
    double ex = ring->radius_px * cos(pe), ey = ring->radius_px * sin(pe);
    March r;
    march(m, ring, o, ex, ey, pe + PI + theta, &r);
    int st = r.status;
    if (st == ST_LINKED) {
        *g = misfit(ring, e, rcv, r.qx, r.qy);
        quadrature(m, &r, o->ds, T, L);
    } else {
        *g = NAN;
        *T = NAN;
        *L = NAN;
    }
    if (keep)
        *keep = r;
    else
        free(r.pts);
    return st;
}

/* Two-point linking of one pair by the safeguarded secant on the launch angle.
 *   theta_0: straight-ray angle (homogeneous start) or the warm-start value.
 *   second point: theta_1 = theta_0 - g_0 / 2, the homogeneous-medium Newton step
 *     (there dg/dtheta = 2); used only to obtain a second point, since a focusing
 *     medium can reverse the sign of dg/dtheta.
 *   then secant through the two latest traced angles that hit the ring.
 * Safeguards:
 *   (a) theta_neg / theta_pos = latest traced angles with g < 0 / g > 0.  Once
 *       both exist, a secant iterate outside the open interval between them, or
 *       a zero secant denominator, is replaced by their midpoint.
 *   (b) before such a bracket exists, an iterate at or beyond the limits
 *       +-(pi/2 - 1e-6) is replaced by the midpoint between the current angle
 *       and that limit; a zero secant denominator falls back to the Newton step.
 *   (c) a march with no interception (trapped ray) yields no g: the next angle is
 *       the midpoint with the latest angle that did hit, or half the angle if
 *       none did.
 *   (d) the limits +-pi/2 are never assumed to have a known misfit sign.
 * Stops when miss = |g| R <= tol (LINKED) or after max_marches traced rays
 * (NOT_CONVERGED, returning the traced ray of smallest miss). */
typedef struct {
    double th0; /* start angle, returned when no ray hits */
    double tha, ga, thb, gb, th_neg, th_pos;
    int nvalid, have_neg, have_pos;
    double best_miss, best_th, best_T, best_L;
} LinkState;

static void link_init(LinkState *s, double th0)
{
    memset(s, 0, sizeof(*s));
    s->th0 = th0;
    s->best_miss = INFINITY;
    s->best_th = th0;
    s->best_T = s->best_L = NAN;
}

/* Next angle after a ray at th that hit with misfit g (secant step + (a), (b)). */
static double link_after_hit(LinkState *s, double th, double g)
{
    const double lim = PI / 2.0 - 1e-6;
    double th_next;
    if (g < 0) {
        s->have_neg = 1;
        s->th_neg = th;
    }
    if (g > 0) {
        s->have_pos = 1;
        s->th_pos = th;
    }
    s->tha = s->thb;
    s->ga = s->gb;
    s->thb = th;
    s->gb = g;
    s->nvalid++;
    int den_zero = 0;
    if (s->nvalid == 1) {
        th_next = th - g / 2.0;
    } else if (s->gb - s->ga == 0.0) {
        den_zero = 1;
        th_next = th - g / 2.0;
    } else {
        th_next = s->thb - s->gb * (s->thb - s->tha) / (s->gb - s->ga);
    }
    if (s->have_neg && s->have_pos) {
        double lo = s->th_neg < s->th_pos ? s->th_neg : s->th_pos;
        double hi = s->th_neg < s->th_pos ? s->th_pos : s->th_neg;
        if (den_zero || !(th_next > lo && th_next < hi)) th_next = 0.5 * (s->th_neg + s->th_pos);
    } else {
        if (!(th_next < lim) && th_next == th_next) th_next = 0.5 * (th + lim);
        if (!(th_next > -lim) && th_next == th_next) th_next = 0.5 * (th - lim);
        if (!(th_next == th_next)) th_next = 0.5 * th;
    }
    return th_next;
}

/* Next angle after a ray at th that never reached the ring (c). */
static double link_after_miss(const LinkState *s, double th)
{
    return (s->nvalid > 0) ? 0.5 * (th + s->thb) : 0.5 * th;
}

static void link_best(LinkState *s, double th, double miss, double T, double L)
{
    if (miss < s->best_miss) {
        s->best_miss = miss;
        s->best_th = th;
        s->best_T = T;
        s->best_L = L;
    }
}

/* Runs the linking loop from angle th with state s and `done` rays already
   traced for this pair. */
static void link_run(const Medium *m, const Ring *ring, const Opts *o, int e, int rcv, LinkState *s, double th,
                     int done, LinkOut *out)
{
    out->n_marches = done;
    for (int k = done; k < o->max_marches; k++) {
        double g, T, L;
        int st = trace_at(m, ring, o, e, rcv, th, &g, &T, &L, NULL);
        out->n_marches++;
        if (st == ST_BAD_INPUT) {
            out->theta = s->th0;
            out->T = out->L = out->miss = NAN;
            out->status = ST_BAD_INPUT;
            return;
        }
        if (st == ST_LINKED) {
            double miss = fabs(g) * ring->radius_px;
            link_best(s, th, miss, T, L);
            if (miss <= o->tol) {
                out->theta = th;
                out->T = T;
                out->L = L;
                out->miss = miss;
                out->status = ST_LINKED;
                return;
            }
            th = link_after_hit(s, th, g);
        } else {
            th = link_after_miss(s, th);
        }
    }
    if (s->best_miss < INFINITY) {
        out->theta = s->best_th;
        out->T = s->best_T;
        out->L = s->best_L;
        out->miss = s->best_miss;
        out->status = ST_NOT_CONVERGED;
    } else {
        out->theta = s->th0;
        out->T = out->L = out->miss = NAN;
        out->status = ST_NO_HIT;
    }
}

static void link_pair(const Medium *m, const Ring *ring, const Opts *o, int e, int rcv, double theta0, LinkOut *out)
{
    LinkState s;
    link_init(&s, theta0);
    link_run(m, ring, o, e, rcv, &s, theta0, 0, out);
}

/* Fan start (an initial-guess option; the secant and its safeguards are
 * unchanged).  The straight-ray rays of all receivers of one emitter sample the
 * same function: the hit angle H(theta) = mod(phi_hit - phi_e, 2 pi) of a ray
 * launched at theta.  These fan rays only seed the linking, so they are traced
 * with a coarser step (fan_step: four tracing steps, at most a pixel) and are
 * not counted among the pair's rays.  For receiver r with target
 * D_r = mod(phi_r - phi_e, 2 pi) the samples give G_j = H_j - D_r at the
 * straight angles theta_j of the receivers at offsets j = 1..n-1 (increasing in
 * j); the linking of r then traces at the full resolution:
 *   - the sign change of G over consecutive samples (j, j+1) nearest to r's own
 *     offset (searching j = own, own+1, own-1-1, ... outward) seeds the secant:
 *     the end with the larger |G| then the one with the smaller |G| are fed to
 *     the state machine as hitting rays, whose next angle is their secant
 *     (linear) interpolation inside the bracket they form, or the cubic
 *     refinement below;
 *   - with no such bracket, the own fan sample is fed alone (homogeneous Newton
 *     second point); if it did not hit, the trapped-ray back-off applies; if it
 *     met bad input, the straight angle itself is traced;
 *   - the fed samples enter the secant's two latest points but not its sign
 *     bracket, which only full-resolution rays establish.
 * Only rays traced for this pair at the full resolution enter its best-ray
 * record and its ray count. */
typedef struct {
    double g, T, L; /* own straight ray: misfit (own receiver), time, length */
    int st;
} FanSample;

/* Cubic refinement of the fan seed: with the bracket (a, a+1) and both of its
   outer neighbours sampled, and G strictly monotone over the four samples
   a-1..a+2, the first linking angle is the value at G = 0 of the cubic that
   interpolates theta as a function of G through those samples (inverse
   Lagrange interpolation), if it lies strictly inside the bracket.  Otherwise
   (returns 0) the secant's own linear interpolation of the bracket stands. */
static int fan_cubic(const double *G, const double *TH, int m, int a, double *th)
{
    if (a < 1 || a + 2 > m - 1) return 0;
    const double *g = G + a - 1, *t = TH + a - 1;
    for (int i = 0; i < 4; i++)
        if (!(g[i] == g[i])) return 0;
    int up = g[1] > g[0];
    for (int i = 0; i < 3; i++)
        if (up ? !(g[i + 1] > g[i]) : !(g[i + 1] < g[i])) return 0;
    double v = 0.0;
    for (int i = 0; i < 4; i++) {
        double w = 1.0;
        for (int k = 0; k < 4; k++)
            if (k != i) w *= (0.0 - g[k]) / (g[i] - g[k]);
        v += w * t[i];
    }
    double lo = t[1] < t[2] ? t[1] : t[2], hi = t[1] < t[2] ? t[2] : t[1];
    if (!(v > lo && v < hi)) return 0;
    *th = v;
    return 1;
}

/* Quintic refinement of the fan seed, the second ray of the first round: with
   the bracket (a, a+1) and two samples on each side of it sampled and G strictly
   monotone over the six samples a-2..a+3, the value at G = 0 of the quintic
   that interpolates theta as a function of G through them, if it lies strictly
   inside the bracket (returns 1); otherwise 0. */
static int fan_quintic(const double *G, const double *TH, int m, int a, double *th)
{
    if (a < 2 || a + 3 > m - 1) return 0;
    const double *g = G + a - 2, *t = TH + a - 2;
    for (int i = 0; i < 6; i++)
        if (!(g[i] == g[i])) return 0;
    int up = g[1] > g[0];
    for (int i = 0; i < 5; i++)
        if (up ? !(g[i + 1] > g[i]) : !(g[i + 1] < g[i])) return 0;
    double v = 0.0;
    for (int i = 0; i < 6; i++) {
        double w = 1.0;
        for (int l = 0; l < 6; l++)
            if (l != i) w *= (0.0 - g[l]) / (g[i] - g[l]);
        v += w * t[i];
    }
    double lo = t[2] < t[3] ? t[2] : t[3], hi = t[2] < t[3] ? t[3] : t[2];
    if (!(v > lo && v < hi)) return 0;
    *th = v;
    return 1;
}

/* The four samples of smallest |g| seen by a fan-started pair: its fan seed
 * samples (bracket and outer neighbours, in order) and then every hitting ray
 * it traced (round by round, ray 0 first).  A new sample replaces the kept one
 * of largest |g| (the later of equal ones) when its |g| is strictly smaller. */
typedef struct {
    double th[4], g[4];
    int id[4], n, next;
} Top4;

static void top4_push(Top4 *t, double th, double g)
{
    int id = t->next++;
    if (t->n < 4) {
        t->th[t->n] = th;
        t->g[t->n] = g;
        t->id[t->n] = id;
        t->n++;
        return;
    }
    int w = 0;
    for (int k = 1; k < 4; k++)
        if (fabs(t->g[k]) > fabs(t->g[w]) || (fabs(t->g[k]) == fabs(t->g[w]) && t->id[k] > t->id[w])) w = k;
    if (fabs(g) < fabs(t->g[w])) {
        t->th[w] = th;
        t->g[w] = g;
        t->id[w] = id;
    }
}

/* Inverse cubic through the four kept samples: ordered by angle they must be
 * strictly increasing in angle and strictly monotone in g; the zero of the
 * cubic interpolating theta as a function of g is accepted if it lies strictly
 * between the outer two angles and inside the sign bracket of the traced rays,
 * when there is one (returns 1 and the angle). */
static int top4_estimate(const Top4 *t, const LinkState *s, double *th)
{
    if (t->n < 4) return 0;
    double a[4], g[4];
    for (int i = 0; i < 4; i++) {
        a[i] = t->th[i];
        g[i] = t->g[i];
    }
    for (int i = 1; i < 4; i++) /* insertion sort by angle */
        for (int j = i; j > 0 && a[j] < a[j - 1]; j--) {
            double x = a[j];
            a[j] = a[j - 1];
            a[j - 1] = x;
            x = g[j];
            g[j] = g[j - 1];
            g[j - 1] = x;
        }
    int up = g[1] > g[0];
    for (int i = 0; i < 3; i++) {
        if (!(a[i + 1] > a[i])) return 0;
        if (up ? !(g[i + 1] > g[i]) : !(g[i + 1] < g[i])) return 0;
    }
    double v = 0.0;
    for (int i = 0; i < 4; i++) {
        double w = 1.0;
        for (int q = 0; q < 4; q++)
            if (q != i) w *= -g[q] / (g[i] - g[q]);
        v += w * a[i];
    }
    if (!(v > a[0] && v < a[3])) return 0;
    if (s->have_neg && s->have_pos) {
        double lo = s->th_neg < s->th_pos ? s->th_neg : s->th_pos;
        double hi = s->th_neg < s->th_pos ? s->th_pos : s->th_neg;
        if (!(v > lo && v < hi)) return 0;
    }
    *th = v;
    return 1;
}

/* Linking in rounds of two rays (the fan start's iteration).  A round traces
 * the primary angle c0 and a hedge c1 = c0 - (c0 - ref) / 10, a tenth of the way
 * back towards the latest fed sample ref (or the start angle), so that a round
 * that does not link leaves two close samples, i.e. a local derivative, for the
 * next secant step; in the first round the hedge is the fan seed's quintic
 * estimate instead (fan_quintic; have_q), when there is one and it differs
 * from c0: the cubic and the quintic interpolant bracket most of the seed's
 * interpolation error between them.  After a round: a ray with bad input ends the pair (BAD);
 * every hitting ray enters the best-ray record (ray 0 first); the hitting ray of
 * smallest miss within the tolerance is the result; after max_marches rounds
 * (2 max_marches rays: the rounds, not the rays, are sequential) the best ray
 * is returned (NOT_CONVERGED), or NO_HIT; otherwise the hitting rays
 * are fed to the secant state machine in order of decreasing |g| (ray 0 first on
 * a tie), the last feed giving the next primary angle, or, when neither hit, the
 * trapped-ray back-off from c0 gives it; after the first two rounds, when a
 * ray hit, the inverse cubic through the four samples of smallest |g|
 * (top4_estimate) replaces the secant's angle where it is defined (later rounds
 * keep the safeguarded secant alone, whose bracket halving does not stall on a
 * misfit that jumps).  Both rays count as traced rays. */
static void link_pairs(const Medium *m, const Ring *ring, const Opts *o, int e, int rcv, LinkState *s, Top4 *t4,
                       double th, int have_q, double thq, LinkOut *out)
{
    out->n_marches = 0;
    for (;;) {
        double ref = s->nvalid > 0 ? s->thb : s->th0;
        double c[2] = {th, th == ref ? th + 1e-4 : th - 0.1 * (th - ref)};
        if (out->n_marches == 0 && have_q && thq != th) c[1] = thq;
        double g[2], T[2], L[2];
        int st[2];
        for (int j = 0; j < 2; j++) st[j] = trace_at(m, ring, o, e, rcv, c[j], &g[j], &T[j], &L[j], NULL);
        out->n_marches += 2;
        if (st[0] == ST_BAD_INPUT || st[1] == ST_BAD_INPUT) {
            out->theta = s->th0;
            out->T = out->L = out->miss = NAN;
            out->status = ST_BAD_INPUT;
            return;
        }
        int lk = -1;
        double lmiss = INFINITY;
        for (int j = 0; j < 2; j++) {
            if (st[j] != ST_LINKED) continue;
            double miss = fabs(g[j]) * ring->radius_px;
            link_best(s, c[j], miss, T[j], L[j]);
            if (miss <= o->tol && miss < lmiss) {
                lk = j;
                lmiss = miss;
            }
        }
        if (lk >= 0) {
            out->theta = c[lk];
            out->T = T[lk];
            out->L = L[lk];
            out->miss = lmiss;
            out->status = ST_LINKED;
            return;
        }
        if (out->n_marches >= 2 * o->max_marches) break; /* max_marches rounds */
        int hit0 = st[0] == ST_LINKED, hit1 = st[1] == ST_LINKED;
        for (int j = 0; j < 2; j++)
            if (st[j] == ST_LINKED) top4_push(t4, c[j], g[j]);
        if (hit0 && hit1) {
            int first = fabs(g[0]) >= fabs(g[1]) ? 0 : 1;
            link_after_hit(s, c[first], g[first]);
            th = link_after_hit(s, c[1 - first], g[1 - first]);
        } else if (hit0 || hit1) {
            int j = hit0 ? 0 : 1;
            th = link_after_hit(s, c[j], g[j]);
        } else {
            th = link_after_miss(s, c[0]);
        }
        double v;
        if ((hit0 || hit1) && out->n_marches <= 4 && top4_estimate(t4, s, &v)) th = v;
    }
    if (s->best_miss < INFINITY) {
        out->theta = s->best_th;
        out->T = s->best_T;
        out->L = s->best_L;
        out->miss = s->best_miss;
        out->status = ST_NOT_CONVERGED;
    } else {
        out->theta = s->th0;
        out->T = out->L = out->miss = NAN;
        out->status = ST_NO_HIT;
    }
}

static void link_fan(const Medium *m, const Ring *ring, const Opts *o, int e, int rcv, const FanSample *row,
                     LinkOut *out)
{
    const int n = ring->n_elem;
    const int jr = ((rcv - e) % n + n) % n; /* own offset, 1..n-1 */
    double pe = elem_angle(ring, e);
    double Dr = mod2pi(elem_angle(ring, rcv) - pe);
    double th_own = straight_angle(ring, e, rcv);
    const FanSample *own = &row[jr - 1];
    LinkState s;
    link_init(&s, th_own);
    Top4 t4;
    memset(&t4, 0, sizeof t4);
    /* G_j relative to this receiver, NaN where the sample did not hit */
    double *G = (double *)malloc(sizeof(double) * (n - 1));
    double *TH = (double *)malloc(sizeof(double) * (n - 1));
    for (int j = 1; j < n; j++) {
        int k = (e + j) % n;
        double Dj = mod2pi(elem_angle(ring, k) - pe);
        G[j - 1] = row[j - 1].st == ST_LINKED ? (row[j - 1].g + Dj) - Dr : NAN;
        TH[j - 1] = straight_angle(ring, e, k);
    }
    int found = -1, have_q = 0;
    double thq = 0.0;
    for (int d = 0; d < n && found < 0; d++) {
        int cand[2] = {jr - 1 + d, jr - 1 - d - 1};
        for (int c = 0; c < 2; c++) {
            int a = cand[c];
            if (a < 0 || a + 1 > n - 2) continue;
            if (G[a] == G[a] && G[a + 1] == G[a + 1] && G[a] * G[a + 1] <= 0.0) {
                found = a;
                break;
            }
        }
    }
    double th;
    if (found >= 0) {
        int near = fabs(G[found]) <= fabs(G[found + 1]) ? found : found + 1;
        int far = near == found ? found + 1 : found;
        link_after_hit(&s, TH[far], G[far]);
        th = link_after_hit(&s, TH[near], G[near]);
        double thc;
        if (fan_cubic(G, TH, n - 1, found, &thc)) th = thc;
        have_q = fan_quintic(G, TH, n - 1, found, &thq);
        for (int i = found - 1; i <= found + 2; i++)
            if (i >= 0 && i <= n - 2 && G[i] == G[i]) top4_push(&t4, TH[i], G[i]);
    } else if (own->st == ST_LINKED) {
        th = link_after_hit(&s, th_own, own->g);
    } else if (own->st == ST_NO_HIT) {
        th = link_after_miss(&s, th_own);
    } else {
        th = th_own;
    }
    /* the coarse samples steer the secant but do not bound it: only rays traced
       at the full resolution establish the sign bracket */
    s.have_neg = s.have_pos = 0;
    free(G);
    free(TH);
    link_pairs(m, ring, o, e, rcv, &s, &t4, th, have_q, thq, out);
}

/* Step of the fan rays: four times the tracing step, at most one pixel (and
   never below the tracing step); the step limit scales with it. */
static double fan_step(double ds) { return fmax(ds, fmin(4.0 * ds, 1.0)); }

/* --------------------------------------------------------------- exported -- */
static int setup(int kind, int nx, int ny, double h, const double *c, const double *mpar, int n_elem,
                 double radius, double phi0, int integ, double ds_px, double tol_px, int max_marches,
                 int max_steps, int flags, Medium *m, Ring *ring, Opts *o)
{
    memset(m, 0, sizeof(*m));
    m->kind = kind;
    m->nx = nx;
    m->ny = ny;
    m->h = h;
    m->c = c;
    for (int i = 0; i < 4; i++) m->p[i] = mpar ? mpar[i] : 0.0;
    if (kind == OR_GRID) {
        if (nx < 4 || ny < 4 || !c) return -1;
        m->gx = (double *)malloc(sizeof(double) * nx * ny);
        m->gy = (double *)malloc(sizeof(double) * nx * ny);
        or_gradient(nx, ny, c, m->gx, m->gy);
    }
    if (kind == OR_BSPLINE) {
        if (nx < 4 || ny < 4 || !c) return -1;
        m->bs = (double *)malloc(sizeof(double) * nx * ny);
        memcpy(m->bs, c, sizeof(double) * nx * ny);
        for (int iy = 0; iy < ny; iy++) bspline_filter_line(m->bs + (size_t)iy * nx, nx, 1);
        for (int ix = 0; ix < nx; ix++) bspline_filter_line(m->bs + ix, ny, nx);
    }
    ring->n_elem = n_elem;
    ring->radius_px = radius / h;
    ring->phi0 = phi0;
    o->integ = integ;
    o->ds = ds_px;
    o->tol = tol_px;
    o->max_marches = max_marches;
    o->max_steps = max_steps > 0 ? max_steps : (int)ceil(8.0 * ring->radius_px / ds_px);
    o->flags = flags;
    return 0;
}

static void teardown(Medium *m)
{
    free(m->gx);
    free(m->gy);
    free(m->bs);
}

/* Per pair (e, r): theta [in: warm start / fixed angle | out: linked angle],
   T (s), L (m), miss (pixels), number of traced rays and status.
   flags & OPT_FIXED: trace once at the given theta, no linking (status LINKED
   means "hit the ring"; miss is then the miss of that ray).
   flags & OPT_WARM: start linking from the given theta instead of the straight
   ray.  flags & OPT_FAN: fan start (see link_fan); needs every ordered pair in
   canonical order (returns -2 otherwise).  Pairs with e == r or an index outside
   [0, n_elem) get ST_BAD_INPUT. */
int or_trace(int kind, int nx, int ny, double h, const double *c, const double *mpar, int n_elem,
             double radius, double phi0, int integ, double ds_px, double tol_px, int max_marches,
             int max_steps, int flags, int n_pairs, const int32_t *pairs, double *theta, double *T,
             double *L, double *miss, int32_t *n_marches, int8_t *status)
{
    Medium m;
    Ring ring;
    Opts o;
    if (setup(kind, nx, ny, h, c, mpar, n_elem, radius, phi0, integ, ds_px, tol_px, max_marches, max_steps,
              flags, &m, &ring, &o))
        return -1;
    if (flags & OPT_FAN) {
        /* all ordered pairs in canonical order: row e holds receivers e+1..e+n-1 */
        int n = n_elem;
        if (n_pairs != n * (n - 1)) {
            teardown(&m);
            return -2;
        }
        for (int i = 0; i < n_pairs; i++) {
            int e = i / (n - 1), k = i % (n - 1);
            if (pairs[2 * i] != e || pairs[2 * i + 1] != (k < e ? k : k + 1)) {
                teardown(&m);
                return -2;
            }
        }
        FanSample *row = (FanSample *)malloc(sizeof(FanSample) * (n - 1));
        Opts of = o; /* the fan's coarse rays */
        of.ds = fan_step(o.ds);
        of.max_steps = (int)ceil(o.max_steps * o.ds / of.ds);
        for (int e = 0; e < n; e++) {
            for (int j = 1; j < n; j++) { /* straight rays of emitter e, by offset */
                int k = (e + j) % n;
                FanSample *f = &row[j - 1];
                f->st = trace_at(&m, &ring, &of, e, k, straight_angle(&ring, e, k), &f->g, &f->T, &f->L, NULL);
            }
            for (int j = 1; j < n; j++) {
                int r = (e + j) % n;
                int i = e * (n - 1) + (r < e ? r : r - 1);
                LinkOut lo;
                link_fan(&m, &ring, &o, e, r, row, &lo);
                theta[i] = lo.theta;
                T[i] = lo.T;
                L[i] = lo.L;
                miss[i] = lo.miss;
                n_marches[i] = lo.n_marches;
                status[i] = (int8_t)lo.status;
            }
        }
        free(row);
        teardown(&m);
        return 0;
    }
    for (int i = 0; i < n_pairs; i++) {
        int e = pairs[2 * i], r = pairs[2 * i + 1];
        if (e == r || e < 0 || r < 0 || e >= n_elem || r >= n_elem) {
            T[i] = L[i] = miss[i] = NAN;
            n_marches[i] = 0;
            status[i] = ST_BAD_INPUT;
            continue;
        }
        if (flags & OPT_FIXED) {
            double g, Ti, Li;
            int st = trace_at(&m, &ring, &o, e, r, theta[i], &g, &Ti, &Li, NULL);
            T[i] = Ti;
            L[i] = Li;
            miss[i] = fabs(g) * ring.radius_px;
            n_marches[i] = 1;
            status[i] = (int8_t)st;
            continue;
        }
        double th0 = (flags & OPT_WARM) ? theta[i] : straight_angle(&ring, e, r);
        LinkOut lo;
        link_pair(&m, &ring, &o, e, r, th0, &lo);
        theta[i] = lo.theta;
        T[i] = lo.T;
        L[i] = lo.L;
        miss[i] = lo.miss;
        n_marches[i] = lo.n_marches;
        status[i] = (int8_t)lo.status;
    }
    teardown(&m);
    return 0;
}

/* Samples of one fixed-angle march of pair (e, r): writes up to cap points
   [cap][2] (pixels), the partial step and the misfit; returns M + 1 (number of
   samples) or -status - 1 when the ray did not hit the ring. */
int or_march_points(int kind, int nx, int ny, double h, const double *c, const double *mpar, int n_elem,
                    double radius, double phi0, int integ, double ds_px, int max_steps, int e, int rcv,
                    double theta, double *pts, int cap, double *dsp, double *g)
{
    Medium m;
    Ring ring;
    Opts o;
    if (setup(kind, nx, ny, h, c, mpar, n_elem, radius, phi0, integ, ds_px, 1.0, 1, max_steps, OPT_FIXED, &m,
              &ring, &o))
        return -100;
    double Ti, Li;
    March r;
    int st = trace_at(&m, &ring, &o, e, rcv, theta, g, &Ti, &Li, &r);
    int n = r.M + 1;
    for (int i = 0; i < n && i < cap; i++) {
        pts[2 * i] = r.pts[2 * i];
        pts[2 * i + 1] = r.pts[2 * i + 1];
    }
    *dsp = r.dsp;
    free(r.pts);
    teardown(&m);
    return st == ST_LINKED ? n : -st - 1;
}

/* Free march (no ring): n_steps steps from pixel point x0 with direction d0,
   writing the n_steps + 1 points (pixels) into pts.  Used for the fish-eye
   trajectory experiments, where rays are followed over a full circle. */
int or_march_free(int kind, int nx, int ny, double h, const double *c, const double *mpar, int integ,
                  double ds_px, const double *x0, const double *d0, int n_steps, double *pts)
{
    Medium m;
    Ring ring;
    Opts o;
    if (setup(kind, nx, ny, h, c, mpar, 4, 1.0 * h, 0.0, integ, ds_px, 1.0, 1, 1, 0, &m, &ring, &o)) return -1;
    double y[4] = {x0[0], x0[1], d0[0], d0[1]}, yn[4];
    double nrm = sqrt(y[2] * y[2] + y[3] * y[3]);
    y[2] /= nrm;
    y[3] /= nrm;
    pts[0] = y[0];
    pts[1] = y[1];
    for (int i = 1; i <= n_steps; i++) {
        step(&m, integ, ds_px, y, yn);
        for (int j = 0; j < 4; j++) y[j] = yn[j];
        pts[2 * i] = y[0];
        pts[2 * i + 1] = y[1];
    }
    teardown(&m);
    return 0;
}

/* Interpolated c and per-pixel gradient at n pixel points. */
int or_interp(int kind, int nx, int ny, double h, const double *c, const double *mpar, int n, const double *pts,
              double *cv, double *gxv, double *gyv)
{
    Medium m;
    Ring ring;
    Opts o;
    if (setup(kind, nx, ny, h, c, mpar, 4, 1.0 * h, 0.0, 4, 0.25, 1.0, 1, 1, 0, &m, &ring, &o)) return -1;
    for (int i = 0; i < n; i++) medium_eval(&m, pts[2 * i], pts[2 * i + 1], &cv[i], &gxv[i], &gyv[i]);
    teardown(&m);
    return 0;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* One system-matrix row of pair (e, r) traced at the fixed angle theta:
   W_j = sum_m w_m h phi_j(p_m) (metres), merged per node and sorted by node
   index j = iy * nx + ix.  Grid media only.  Returns the number of nonzeros
   (written only when <= cap), or a negative value if the ray did not hit. */
long or_weights_row(int nx, int ny, double h, const double *c, int n_elem, double radius, double phi0, int integ,
                    double ds_px, int max_steps, int e, int rcv, double theta, int32_t *cols, double *vals,
                    long cap)
{
    Medium m;
    Ring ring;
    Opts o;
    if (setup(OR_GRID, nx, ny, h, c, NULL, n_elem, radius, phi0, integ, ds_px, 1.0, 1, max_steps, OPT_FIXED, &m,
              &ring, &o))
        return -100;
    double g, Ti, Li;
    March r;
    int st = trace_at(&m, &ring, &o, e, rcv, theta, &g, &Ti, &Li, &r);
    if (st != ST_LINKED) {
        free(r.pts);
        teardown(&m);
        return -1 - st;
    }
    double *dense = (double *)calloc((size_t)nx * ny, sizeof(double));
    int *touched = (int *)malloc(sizeof(int) * 4 * (r.M + 1));
    char *mark = (char *)calloc((size_t)nx * ny, 1);
    int nt = 0;
    for (int i = 0; i <= r.M; i++) {
        int ix, iy;
        double t, s, w[4];
        locate(&m, r.pts[2 * i], r.pts[2 * i + 1], &ix, &iy, &t, &s);
        hat4(t, s, w);
        int nodes[4] = {iy * nx + ix, iy * nx + ix + 1, (iy + 1) * nx + ix, (iy + 1) * nx + ix + 1};
        double wm = trap_weight(i, r.M, ds_px, r.dsp) * h;
        for (int k = 0; k < 4; k++) {
            if (w[k] == 0.0) continue;
            dense[nodes[k]] += wm * w[k];
            if (!mark[nodes[k]]) {
                mark[nodes[k]] = 1;
                touched[nt++] = nodes[k];
            }
        }
    }
    qsort(touched, nt, sizeof(int), cmp_int);
    if (nt <= cap) {
        for (int k = 0; k < nt; k++) {
            cols[k] = touched[k];
            vals[k] = dense[touched[k]];
        }
    }
    free(dense);
    free(touched);
    free(mark);
    free(r.pts);
    teardown(&m);
    return nt;
}

/* Adjoint of the path weights: grad_j += sum_i rho_i sum_m w_m h kappa_m phi_j(p_m)
   with kappa = 1 (weight_mode 0: transpose of the system matrix) or
   kappa = -1 / c(p_m)^2 (weight_mode 1: frozen-path derivative of T with respect
   to the node sound speeds).  Each pair is traced once at its fixed theta.
   Pairs whose ray does not hit the ring contribute nothing, and so do pairs
   whose status (if given) is neither LINKED nor NOT_CONVERGED -- the two cases
   where theta is a traced ray that hit.  Summed in FP64 in pair order. */
int or_adjoint(int nx, int ny, double h, const double *c, int n_elem, double radius, double phi0, int integ,
               double ds_px, int max_steps, int n_pairs, const int32_t *pairs, const double *theta,
               const int8_t *status, const double *rho, int weight_mode, double *grad)
{
    Medium m;
    Ring ring;
    Opts o;
    if (setup(OR_GRID, nx, ny, h, c, NULL, n_elem, radius, phi0, integ, ds_px, 1.0, 1, max_steps, OPT_FIXED, &m,
              &ring, &o))
        return -1;
    for (int p = 0; p < n_pairs; p++) {
        int e = pairs[2 * p], rc = pairs[2 * p + 1];
        if (e == rc || e < 0 || rc < 0 || e >= n_elem || rc >= n_elem) continue;
        if (status && status[p] != ST_LINKED && status[p] != ST_NOT_CONVERGED) continue;
        double g, Ti, Li;
        March r;
        int st = trace_at(&m, &ring, &o, e, rc, theta[p], &g, &Ti, &Li, &r);
        if (st == ST_LINKED) {
            for (int i = 0; i <= r.M; i++) {
                int ix, iy;
                double t, s, w[4];
                locate(&m, r.pts[2 * i], r.pts[2 * i + 1], &ix, &iy, &t, &s);
                hat4(t, s, w);
                double kappa = 1.0;
                if (weight_mode == 1) {
                    double cc, gx, gy;
                    medium_eval(&m, r.pts[2 * i], r.pts[2 * i + 1], &cc, &gx, &gy);
                    kappa = -1.0 / (cc * cc);
                }
                double a = rho[p] * trap_weight(i, r.M, ds_px, r.dsp) * h * kappa;
                grad[iy * nx + ix] += a * w[0];
                grad[iy * nx + ix + 1] += a * w[1];
                grad[(iy + 1) * nx + ix] += a * w[2];
                grad[(iy + 1) * nx + ix + 1] += a * w[3];
            }
        }
        free(r.pts);
    }
    teardown(&m);
    return 0;
}

/* Ray-Born-style residual reduction for phase-linearised data d_k = exp(i w_k T):
   the adjoint of dd_k = i w_k exp(i w_k T) dT applied to residuals r_k is
   rho = sum_k Re[ conj(i w_k exp(i w_k T)) r_k ] = sum_k w_k Im(exp(-i w_k T) r_k),
   w_k = 2 pi f_k.  resid is interleaved (re, im) [n][n_freq][2]. */
int or_rayborn_rho(int n, int n_freq, const double *T, const double *freqs, const double *resid, double *rho)
{
    for (int i = 0; i < n; i++) {
        double acc = 0.0;
        for (int k = 0; k < n_freq; k++) {
            double w = 2.0 * PI * freqs[k];
            double ph = fmod(w * T[i], 2.0 * PI);
            double re = resid[2 * ((size_t)i * n_freq + k)], im = resid[2 * ((size_t)i * n_freq + k) + 1];
            /* exp(-i ph) (re + i im) = (re cos ph + im sin ph) + i (im cos ph - re sin ph) */
            acc += w * (im * cos(ph) - re * sin(ph));
        }
        rho[i] = acc;
    }
    return 0;
}

/* The fan start's cubic refinement on its own (samples G[0..m-1], TH[0..m-1],
   bracket (a, a+1)): returns 1 and the angle, or 0 when the linear seed stands. */
int or_fan_cubic(const double *G, const double *TH, int m, int a, double *th)
{
    return fan_cubic(G, TH, m, a, th);
}

/* The first round's quintic hedge on its own (same arguments). */
int or_fan_quintic(const double *G, const double *TH, int m, int a, double *th)
{
    return fan_quintic(G, TH, m, a, th);
}

/* SART, the default solver of the linearised ToF subproblem (Sec. 3.1; the
   simultaneous algebraic reconstruction technique of Andersen and Kak).  With
   the system matrix W (CSR, n_rows x n_cols), its row sums M_i = sum_j W_ij and
   column sums V_j = sum_i W_ij, each of the n_iter iterations sets
     x_j <- x_j + lambda / V_j * sum_i W_ij (b_i - sum_l W_il x_l) / M_i
   for every column with V_j != 0, all from the x of the previous iteration
   (the simultaneous update); rows with M_i == 0 take no part.  x is updated in
   place.  Returns -1 on a column index out of range. */
int or_sart(int n_rows, int n_cols, const int64_t *rowptr, const int32_t *col, const double *val, const double *b,
            double *x, int n_iter, double lambda)
{
    double *M = (double *)calloc((size_t)n_rows, sizeof(double));
    double *V = (double *)calloc((size_t)n_cols, sizeof(double));
    double *upd = (double *)malloc(sizeof(double) * (size_t)n_cols);
    int rc = 0;
    for (int i = 0; i < n_rows && !rc; i++)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) {
            if (col[k] < 0 || col[k] >= n_cols) {
                rc = -1;
                break;
            }
            M[i] += val[k];
            V[col[k]] += val[k];
        }
    for (int it = 0; it < n_iter && !rc; it++) {
        for (int j = 0; j < n_cols; j++) upd[j] = 0.0;
        for (int i = 0; i < n_rows; i++) {
            if (M[i] == 0.0) continue;
            double proj = 0.0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) proj += val[k] * x[col[k]];
            double r = (b[i] - proj) / M[i];
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; k++) upd[col[k]] += val[k] * r;
        }
        for (int j = 0; j < n_cols; j++)
            if (V[j] != 0.0) x[j] += lambda * upd[j] / V[j];
    }
    free(M);
    free(V);
    free(upd);
    return rc;
}

/* ------------------------------------------------------------ paraxial ray -- */
/* The paraxial ray (Sec. 3.5, the default way to the ray Jacobian): the
   first-order perturbation (dx, dd) of a ray's position and direction caused by
   a perturbation of its launch angle obeys the variational equations of the ray
   ODE x' = d, d' = K(x, d) = -(G - (G.d) d) / c:
     (dx)' = dd,
     (dd)' = dK/dx dx + dK/dd dd,
     dK/dd dd = ((G.dd) d + (G.d) dd) / c,
     dK/dx dx = -(H dx - ((H dx).d) d) / c + (G - (G.d) d) (grad c . dx) / c^2,
   with grad c the gradient of the interpolated c and H_ab = dG_a/dx_b the
   derivative of the interpolated G (for the bilinear field: the derivatives of
   the two separately interpolated fields).  The paper cites the system only;
   this is its standard linearisation.  It is integrated with the ray by the
   same Runge-Kutta scheme on the 8-component state, and the renormalisation of
   d is linearised too: dd <- (dd - (n.dd) n) / |d|, n = d / |d|. */

/* c, per-pixel G, grad c and H (row-major dG_a/dx_b) at pixel position (px, py). */
static void medium_eval2(const Medium *m, double px, double py, double *c, double G[2], double dc[2], double H[4])
{
    if (m->kind == OR_FISHEYE) {
        double k = m->p[0] * 2.0 * m->h * m->h / (m->p[1] * m->p[1]);
        medium_eval(m, px, py, c, &G[0], &G[1]);
        dc[0] = G[0];
        dc[1] = G[1];
        H[0] = k;
        H[1] = H[2] = 0.0;
        H[3] = k;
        return;
    }
    if (m->kind == OR_LINEAR) {
        medium_eval(m, px, py, c, &G[0], &G[1]);
        dc[0] = G[0];
        dc[1] = G[1];
        H[0] = H[1] = H[2] = H[3] = 0.0;
        return;
    }
    int ix, iy;
    double t, s;
    if (!locate(m, px, py, &ix, &iy, &t, &s)) {
        *c = G[0] = G[1] = dc[0] = dc[1] = NAN;
        H[0] = H[1] = H[2] = H[3] = NAN;
        return;
    }
    if (m->kind == OR_BSPLINE) {
        double wx[4], dwx[4], wy[4], dwy[4];
        double ddwx[4] = {1.0 - t, 3.0 * t - 2.0, 1.0 - 3.0 * t, t};
        double ddwy[4] = {1.0 - s, 3.0 * s - 2.0, 1.0 - 3.0 * s, s};
        bspline_w(t, wx, dwx);
        bspline_w(s, wy, dwy);
        double v = 0, vx = 0, vy = 0, vxx = 0, vxy = 0, vyy = 0;
        for (int b = 0; b < 4; b++) {
            int jy = mirror(iy - 1 + b, m->ny);
            for (int a = 0; a < 4; a++) {
                double cf = m->bs[jy * m->nx + mirror(ix - 1 + a, m->nx)];
                v += cf * wx[a] * wy[b];
                vx += cf * dwx[a] * wy[b];
                vy += cf * wx[a] * dwy[b];
                vxx += cf * ddwx[a] * wy[b];
                vxy += cf * dwx[a] * dwy[b];
                vyy += cf * wx[a] * ddwy[b];
            }
        }
        *c = v;
        G[0] = dc[0] = vx;
        G[1] = dc[1] = vy;
        H[0] = vxx;
        H[1] = H[2] = vxy;
        H[3] = vyy;
        return;
    }
    /* bilinear: value weights and their t- and s-derivatives, corners
       (ix,iy), (ix+1,iy), (ix,iy+1), (ix+1,iy+1) */
    double w[4], wt[4] = {-(1.0 - s), 1.0 - s, -s, s}, ws[4] = {-(1.0 - t), -t, 1.0 - t, t};
    hat4(t, s, w);
    int n[4] = {iy * m->nx + ix, iy * m->nx + ix + 1, (iy + 1) * m->nx + ix, (iy + 1) * m->nx + ix + 1};
    *c = G[0] = G[1] = dc[0] = dc[1] = H[0] = H[1] = H[2] = H[3] = 0.0;
    for (int k = 0; k < 4; k++) {
        *c += w[k] * m->c[n[k]];
        G[0] += w[k] * m->gx[n[k]];
        G[1] += w[k] * m->gy[n[k]];
        dc[0] += wt[k] * m->c[n[k]];
        dc[1] += ws[k] * m->c[n[k]];
        H[0] += wt[k] * m->gx[n[k]];
        H[1] += ws[k] * m->gx[n[k]];
        H[2] += wt[k] * m->gy[n[k]];
        H[3] += ws[k] * m->gy[n[k]];
    }
}

/* y = (x1, x2, d1, d2, dx1, dx2, dd1, dd2) */
static void rhs8(const Medium *m, const double y[8], double k[8])
{
    double c, G[2], dc[2], H[4];
    medium_eval2(m, y[0], y[1], &c, G, dc, H);
    const double *d = y + 2, *q = y + 4, *p = y + 6;
    double gd = G[0] * d[0] + G[1] * d[1];
    double Hq[2] = {H[0] * q[0] + H[1] * q[1], H[2] * q[0] + H[3] * q[1]};
    double hqd = Hq[0] * d[0] + Hq[1] * d[1];
    double dcq = dc[0] * q[0] + dc[1] * q[1];
    double gp = G[0] * p[0] + G[1] * p[1];
    k[0] = d[0];
    k[1] = d[1];
    for (int a = 0; a < 2; a++) {
        k[2 + a] = -(G[a] - gd * d[a]) / c;
        k[4 + a] = p[a];
        k[6 + a] = -(Hq[a] - hqd * d[a]) / c + (G[a] - gd * d[a]) * dcq / (c * c) + (gp * d[a] + gd * p[a]) / c;
    }
}

static void step8(const Medium *m, int integ, double ds, const double y[8], double out[8])
{
    double k1[8], k2[8], k3[8], k4[8], tmp[8];
    if (integ == 2) {
        rhs8(m, y, k1);
        for (int i = 0; i < 8; i++) tmp[i] = y[i] + ds * k1[i];
        rhs8(m, tmp, k2);
        for (int i = 0; i < 8; i++) out[i] = y[i] + ds / 2.0 * (k1[i] + k2[i]);
    } else {
        rhs8(m, y, k1);
        for (int i = 0; i < 8; i++) tmp[i] = y[i] + ds / 2.0 * k1[i];
        rhs8(m, tmp, k2);
        for (int i = 0; i < 8; i++) tmp[i] = y[i] + ds / 2.0 * k2[i];
        rhs8(m, tmp, k3);
        for (int i = 0; i < 8; i++) tmp[i] = y[i] + ds * k3[i];
        rhs8(m, tmp, k4);
        for (int i = 0; i < 8; i++) out[i] = y[i] + ds / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    double nrm = sqrt(out[2] * out[2] + out[3] * out[3]);
    double n0 = out[2] / nrm, n1 = out[3] / nrm;
    double np = n0 * out[6] + n1 * out[7];
    out[6] = (out[6] - np * n0) / nrm;
    out[7] = (out[7] - np * n1) / nrm;
    out[2] = n0;
    out[3] = n1;
}

/* Paraxial quantities of the rays of pairs (e, r) at fixed launch angles:
     dgdth: derivative of the interception angle (and so of the misfit g) with
            respect to the launch angle;
     jac:   ray Jacobian at the interception, u x dx (u the direction of the
            crossing chord), in metres per radian: the ray-tube width;
     amp:   sqrt(c(q) / (c(x_e) |jac|)), the 2-D transport-equation amplitude
            normalised to the point-source far field (1/sqrt(distance) in a
            homogeneous medium); in 1/sqrt(m);
     kmah:  number of sign changes of the Jacobian d x dx over the accepted
            step points and the interception (caustics crossed).
   The interception point is q = p + t (p' - p) on the crossing chord; its
   perturbation is dp + t (dp' - dp) + dt (p' - p) with dt keeping |q| = R.
   status as in or_trace's fixed-angle mode; outputs NaN / -1 off LINKED. */
int or_paraxial(int kind, int nx, int ny, double h, const double *c, const double *mpar, int n_elem, double radius,
                double phi0, int integ, double ds_px, int max_steps, int n_pairs, const int32_t *pairs,
                const double *theta, double *dgdth, double *jac, double *amp, int32_t *kmah, int8_t *status)
{
    Medium m;
    Ring ring;
    Opts o;
    if (setup(kind, nx, ny, h, c, mpar, n_elem, radius, phi0, integ, ds_px, 1.0, 1, max_steps, OPT_FIXED, &m, &ring,
              &o))
        return -1;
    const double R = ring.radius_px;
    for (int i = 0; i < n_pairs; i++) {
        int e = pairs[2 * i], r = pairs[2 * i + 1];
        dgdth[i] = jac[i] = amp[i] = NAN;
        kmah[i] = -1;
        if (e == r || e < 0 || r < 0 || e >= n_elem || r >= n_elem) {
            status[i] = ST_BAD_INPUT;
            continue;
        }
        double pe = elem_angle(&ring, e), psi = pe + PI + theta[i];
        double y[8] = {R * cos(pe), R * sin(pe), cos(psi), sin(psi), 0.0, 0.0, -sin(psi), cos(psi)}, yn[8];
        double ce, ge[2], dce[2], He[4];
        medium_eval2(&m, y[0], y[1], &ce, ge, dce, He);
        int st = ST_NO_HIT, changes = 0;
        double jprev = 0.0;
        for (int k = 1; k <= o.max_steps; k++) {
            double cc, g2[2], d2[2], h4[4];
            medium_eval2(&m, y[0], y[1], &cc, g2, d2, h4);
            if (!(cc > 0.0)) {
                st = ST_BAD_INPUT;
                break;
            }
            step8(&m, o.integ, o.ds, y, yn);
            if (yn[0] * yn[0] + yn[1] * yn[1] >= R * R) {
                double ax = yn[0] - y[0], ay = yn[1] - y[1];
                double A = ax * ax + ay * ay, B = 2.0 * (y[0] * ax + y[1] * ay), C = y[0] * y[0] + y[1] * y[1] - R * R;
                double D = B * B - 4.0 * A * C;
                if (D < 0) D = 0;
                double t = (B >= 0) ? (-2.0 * C) / (B + sqrt(D)) : (-B + sqrt(D)) / (2.0 * A);
                if (t > 1.0) t = 1.0;
                if (t < 0.0) t = 0.0;
                double qx = y[0] + t * ax, qy = y[1] + t * ay;
                double dqx = y[4] + t * (yn[4] - y[4]), dqy = y[5] + t * (yn[5] - y[5]);
                double dt = -(qx * dqx + qy * dqy) / (qx * ax + qy * ay);
                dqx += dt * ax;
                dqy += dt * ay;
                double la = sqrt(A), ux = ax / la, uy = ay / la;
                double jq = ux * dqy - uy * dqx;
                if (jq * jprev < 0) changes++;
                double cq, gq[2], dcq[2], hq[4];
                medium_eval2(&m, qx, qy, &cq, gq, dcq, hq);
                st = (cq > 0.0) ? ST_LINKED : ST_BAD_INPUT;
                if (st == ST_LINKED) {
                    dgdth[i] = (qx * dqy - qy * dqx) / (R * R);
                    jac[i] = jq * h;
                    amp[i] = sqrt(cq / (ce * fabs(jq * h)));
                    kmah[i] = changes;
                }
                break;
            }
            for (int j = 0; j < 8; j++) y[j] = yn[j];
            double jn = y[2] * y[5] - y[3] * y[4];
            if (jn * jprev < 0) changes++;
            if (jn != 0.0) jprev = jn;
        }
        status[i] = (int8_t)st;
    }
    teardown(&m);
    return 0;
}
