/*
 * oracle_rt3.c -- plain, slow FP64 CPU oracle for two-point ray tracing in 3-D:
 * arrays of point transducers on a sphere (hemispherical arrays), a gridded
 * sound-speed volume, Broyden-like ray linking, travel time and path length.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP path.
 *
 * What it follows (arXiv 2511.18511):
 *   - Sec. 3 (software description): ToF inversion extended to 3-D acquisition
 *     geometries such as hemispherical arrays.
 *   - Sec. 3.2: the ray equations in the position x and unit direction d hold in
 *     any dimension.
 *   - Sec. 3.3: the field and its node gradient are interpolated from the
 *     vertices of the enclosing cell (in 3-D: trilinearly from 8 vertices).
 *   - Sec. 3.4 (3-D configurations): the misfit is the discrepancy between the
 *     interception of the ray by the boundary and the receiver, parameterised in
 *     the angular domain; the Broyden-like method updates the initial direction
 *     with one traced ray per update, its Jacobian estimate being updated from
 *     the two most recent iterates instead of being recomputed by finite
 *     differences (Newton, >= 3 rays per update).
 *   - Sec. 4.2: trapezoid rule with the last point replaced by the interception.
 *   - Sec. 4: Maxwell's fish-eye lens for dim = 3.
 *
 * Readings where the paper is silent (kept with the design notes):
 *   - grid node (ix, iy, iz) at pixel (ix - (nx-1)/2, iy - (ny-1)/2, iz - (nz-1)/2);
 *     the elements lie on a sphere of radius R about the grid centre, which is
 *     also the interception boundary;
 *   - node gradient: second-order central differences, one-sided at the edges;
 *     trilinear interpolation of c and of the gradient; ray ODE and integrators
 *     as in 2-D (x' = d, d' = -(G - (G.d) d)/c, classic RK4 or Heun, d
 *     renormalised after each step); the last step is cut at the sphere;
 *   - angular parameters: u = (u1, u2) in the emitter's tangent plane,
 *     d = normalize(n + u1 a1 + u2 a2) with n the inward normal and (a1, a2) a
 *     fixed orthonormal tangent basis; misfit g = (b1.(q - r), b2.(q - r)) / R
 *     in the receiver's tangent basis; miss = |q - r| (pixels);
 *   - Broyden-like update: start at the straight ray (or a warm start) with the
 *     Jacobian of the homogeneous medium there (closed form); after each ray
 *     that hits, Broyden's rank-one update J += (dg - J du) du^T / |du|^2 from
 *     the two most recent hitting iterates, then u <- u - J^-1 g with the step
 *     length capped at 0.5; a near-singular J is replaced by the homogeneous
 *     Jacobian at the current u; a ray that never reaches the sphere backs off
 *     to the midpoint with the latest hitting iterate (or halves u); at most
 *     max_marches rays, the ray of smallest miss returned otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define K3_GRID 0
#define K3_FISHEYE 1 /* c = c0 (1 + |x|^2 / R^2), params {c0, R} */
#define K3_LINEAR 2  /* c = c0 + a . x, params {c0, ax, ay, az} */
#define S3_LINKED 0
#define S3_NOT_CONVERGED 1
#define S3_NO_HIT 2
#define S3_BAD_INPUT 3
#define F3_WARM 1
#define F3_FIXED 2

typedef struct {
    int kind, nx, ny, nz;
    double h;
    const double *c; /* [nz][ny][nx] */
    double *g;       /* [3][nz][ny][nx] per-pixel node gradient */
    double p[4];
} Med3;

static size_t idx3(const Med3 *m, int ix, int iy, int iz) { return ((size_t)iz * m->ny + iy) * m->nx + ix; }

/* second-order differences along one axis (stride st, length n, index i) */
static double diff1(const double *c, size_t base, size_t st, int i, int n)
{
    if (i == 0) return (-3.0 * c[base] + 4.0 * c[base + st] - c[base + 2 * st]) / 2.0;
    if (i == n - 1) return (3.0 * c[base + (size_t)i * st] - 4.0 * c[base + (size_t)(i - 1) * st] +
                            c[base + (size_t)(i - 2) * st]) / 2.0;
    return (c[base + (size_t)(i + 1) * st] - c[base + (size_t)(i - 1) * st]) / 2.0;
}

static void grad3(Med3 *m)
{
    size_t n = (size_t)m->nx * m->ny * m->nz;
    m->g = (double *)malloc(sizeof(double) * 3 * n);
    for (int iz = 0; iz < m->nz; iz++)
        for (int iy = 0; iy < m->ny; iy++)
            for (int ix = 0; ix < m->nx; ix++) {
                size_t k = idx3(m, ix, iy, iz);
                m->g[k] = diff1(m->c, idx3(m, 0, iy, iz), 1, ix, m->nx);
                m->g[n + k] = diff1(m->c, idx3(m, ix, 0, iz), (size_t)m->nx, iy, m->ny);
                m->g[2 * n + k] = diff1(m->c, idx3(m, ix, iy, 0), (size_t)m->nx * m->ny, iz, m->nz);
            }
}

/* c and per-pixel gradient at pixel point x (grid-centred); NaN off a finite point */
static void eval3(const Med3 *m, const double x[3], double *c, double G[3])
{
    if (m->kind == K3_FISHEYE) {
        double h = m->h, c0 = m->p[0], R = m->p[1];
        double r2 = (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) * h * h;
        *c = c0 * (1.0 + r2 / (R * R));
        for (int a = 0; a < 3; a++) G[a] = c0 * 2.0 * x[a] * h / (R * R) * h;
        return;
    }
    if (m->kind == K3_LINEAR) {
        *c = m->p[0];
        for (int a = 0; a < 3; a++) {
            *c += m->p[1 + a] * x[a] * m->h;
            G[a] = m->p[1 + a] * m->h;
        }
        return;
    }
    int n3[3] = {m->nx, m->ny, m->nz}, i[3];
    double f[3];
    for (int a = 0; a < 3; a++) {
        double u = x[a] + 0.5 * (n3[a] - 1);
        if (!(u == u)) {
            *c = G[0] = G[1] = G[2] = NAN;
            return;
        }
        double fu = floor(u);
        if (fu < 0) fu = 0;
        if (fu > n3[a] - 2) fu = n3[a] - 2;
        double t = u - fu;
        if (t < 0) t = 0;
        if (t > 1) t = 1;
        i[a] = (int)fu;
        f[a] = t;
    }
    size_t n = (size_t)m->nx * m->ny * m->nz;
    *c = G[0] = G[1] = G[2] = 0.0;
    for (int k = 0; k < 8; k++) {
        int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
        double w = (bx ? f[0] : 1.0 - f[0]) * (by ? f[1] : 1.0 - f[1]) * (bz ? f[2] : 1.0 - f[2]);
        size_t q = idx3(m, i[0] + bx, i[1] + by, i[2] + bz);
        *c += w * m->c[q];
        for (int a = 0; a < 3; a++) G[a] += w * m->g[a * n + q];
    }
}

/* y = (x1, x2, x3, d1, d2, d3) */
static void rhs3(const Med3 *m, const double y[6], double k[6])
{
    double c, G[3];
    eval3(m, y, &c, G);
    double gd = G[0] * y[3] + G[1] * y[4] + G[2] * y[5];
    for (int a = 0; a < 3; a++) {
        k[a] = y[3 + a];
        k[3 + a] = -(G[a] - gd * y[3 + a]) / c;
    }
}

static void step3(const Med3 *m, int integ, double ds, const double y[6], double out[6])
{
    double k1[6], k2[6], k3[6], k4[6], t[6];
    if (integ == 2) {
        rhs3(m, y, k1);
        for (int i = 0; i < 6; i++) t[i] = y[i] + ds * k1[i];
        rhs3(m, t, k2);
        for (int i = 0; i < 6; i++) out[i] = y[i] + ds / 2.0 * (k1[i] + k2[i]);
    } else {
        rhs3(m, y, k1);
        for (int i = 0; i < 6; i++) t[i] = y[i] + ds / 2.0 * k1[i];
        rhs3(m, t, k2);
        for (int i = 0; i < 6; i++) t[i] = y[i] + ds / 2.0 * k2[i];
        rhs3(m, t, k3);
        for (int i = 0; i < 6; i++) t[i] = y[i] + ds * k3[i];
        rhs3(m, t, k4);
        for (int i = 0; i < 6; i++) out[i] = y[i] + ds / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    double nrm = sqrt(out[3] * out[3] + out[4] * out[4] + out[5] * out[5]);
    for (int a = 3; a < 6; a++) out[a] /= nrm;
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* One march from E (pixels, on the sphere |x| = R) along d0 until it crosses
   the sphere: status, interception q, T (s) and L (m) by the trapezoid rule with
   the last point replaced by q (the 2-D rules, Sec. 4.2). */
typedef struct {
    int status;
    double q[3], T, L;
} Hit3;

static Hit3 march3(const Med3 *m, double R, int integ, double ds, int max_steps, const double E[3], const double d0[3])
{
    Hit3 o;
    o.status = S3_NO_HIT;
    o.q[0] = o.q[1] = o.q[2] = o.T = o.L = NAN;
    double y[6] = {E[0], E[1], E[2], d0[0], d0[1], d0[2]}, yn[6];
    double nrm = sqrt(dot3(d0, d0));
    for (int a = 3; a < 6; a++) y[a] /= nrm;
    double acc = 0.0;
    for (int k = 1; k <= max_steps; k++) {
        double c, G[3];
        eval3(m, y, &c, G);
        if (!(c > 0.0)) {
            o.status = S3_BAD_INPUT;
            return o;
        }
        step3(m, integ, ds, y, yn);
        if (dot3(yn, yn) >= R * R) {
            double a[3] = {yn[0] - y[0], yn[1] - y[1], yn[2] - y[2]};
            double A = dot3(a, a), B = 2.0 * dot3(y, a), C = dot3(y, y) - R * R;
            double D = B * B - 4.0 * A * C;
            if (D < 0) D = 0;
            double t = (B >= 0) ? (-2.0 * C) / (B + sqrt(D)) : (-B + sqrt(D)) / (2.0 * A);
            if (t > 1.0) t = 1.0;
            if (t < 0.0) t = 0.0;
            for (int i = 0; i < 3; i++) o.q[i] = y[i] + t * a[i];
            double dsp = t * ds, cq, Gq[3];
            eval3(m, o.q, &cq, Gq);
            if (!(cq > 0.0)) {
                o.status = S3_BAD_INPUT;
                return o;
            }
            /* samples p_0..p_{M-1} (the accepted points, p_{M-1} = y) and p_M = q;
               p_0..p_{M-2} already carry ds/2 (p_0) or ds */
            int M = k;
            if (M == 1)
                acc = dsp / 2.0 / c + dsp / 2.0 / cq;
            else
                acc += (ds + dsp) / 2.0 / c + dsp / 2.0 / cq;
            o.T = acc * m->h;
            o.L = ((M - 1) * ds + dsp) * m->h;
            o.status = S3_LINKED;
            return o;
        }
        /* the start point of this step enters with weight ds/2 (first) or ds;
           its final weight is fixed once the crossing step is known */
        acc += (k == 1 ? ds / 2.0 : ds) / c;
        for (int i = 0; i < 6; i++) y[i] = yn[i];
    }
    return o;
}

/* inward normal and a fixed tangent basis at sphere point P */
static void frame(const double P[3], double n[3], double a1[3], double a2[3])
{
    double r = sqrt(dot3(P, P));
    for (int i = 0; i < 3; i++) n[i] = -P[i] / r;
    double hlp[3] = {0.0, 0.0, 1.0};
    if (fabs(n[2]) > 0.9) {
        hlp[0] = 1.0;
        hlp[2] = 0.0;
    }
    double c[3] = {hlp[1] * n[2] - hlp[2] * n[1], hlp[2] * n[0] - hlp[0] * n[2], hlp[0] * n[1] - hlp[1] * n[0]};
    double cn = sqrt(dot3(c, c));
    for (int i = 0; i < 3; i++) a1[i] = c[i] / cn;
    a2[0] = n[1] * a1[2] - n[2] * a1[1];
    a2[1] = n[2] * a1[0] - n[0] * a1[2];
    a2[2] = n[0] * a1[1] - n[1] * a1[0];
}

static void dir_of(const double u[2], const double n[3], const double a1[3], const double a2[3], double d[3])
{
    for (int i = 0; i < 3; i++) d[i] = n[i] + u[0] * a1[i] + u[1] * a2[i];
    double s = sqrt(dot3(d, d));
    for (int i = 0; i < 3; i++) d[i] /= s;
}

static void misfit3(const double q[3], const double Rc[3], const double b1[3], const double b2[3], double R,
                    double g[2])
{
    double e[3] = {q[0] - Rc[0], q[1] - Rc[1], q[2] - Rc[2]};
    g[0] = dot3(b1, e) / R;
    g[1] = dot3(b2, e) / R;
}

/* Jacobian dg/du of the straight-ray map at u (homogeneous medium): the chord
   from E along d meets the sphere at q = E + L d with L = -2 E.d, so
   dq = L dd - 2 d (E.dd), and dd/du_j = (a_j - d (d.a_j)) / |n + u.a|. */
static void jac0(const double E[3], const double u[2], const double n[3], const double a1[3], const double a2[3],
                 const double b1[3], const double b2[3], double R, double J[4])
{
    double v[3], d[3];
    for (int i = 0; i < 3; i++) v[i] = n[i] + u[0] * a1[i] + u[1] * a2[i];
    double nv = sqrt(dot3(v, v));
    for (int i = 0; i < 3; i++) d[i] = v[i] / nv;
    double L = -2.0 * dot3(E, d);
    const double *aj[2] = {a1, a2};
    for (int j = 0; j < 2; j++) {
        double da = dot3(d, aj[j]), dd[3], dq[3];
        for (int i = 0; i < 3; i++) dd[i] = (aj[j][i] - d[i] * da) / nv;
        double ed = dot3(E, dd);
        for (int i = 0; i < 3; i++) dq[i] = L * dd[i] - 2.0 * d[i] * ed;
        J[0 * 2 + j] = dot3(b1, dq) / R;
        J[1 * 2 + j] = dot3(b2, dq) / R;
    }
}

typedef struct {
    double u[2], T, L, miss;
    int n_marches, status;
} Link3;

static void link3(const Med3 *m, double R, int integ, double ds, double tol, int max_marches, int max_steps,
                  const double E[3], const double Rc[3], const double u0[2], int fixed, Link3 *out)
{
    double n[3], a1[3], a2[3], nr[3], b1[3], b2[3];
    frame(E, n, a1, a2);
    frame(Rc, nr, b1, b2);
    double u[2] = {u0[0], u0[1]}, J[4];
    jac0(E, u, n, a1, a2, b1, b2, R, J);
    double up[2] = {0, 0}, gp[2] = {0, 0};
    int have_prev = 0;
    double best = INFINITY;
    out->u[0] = u0[0];
    out->u[1] = u0[1];
    out->T = out->L = out->miss = NAN;
    out->n_marches = 0;
    out->status = S3_NO_HIT;
    for (int k = 0; k < (fixed ? 1 : max_marches); k++) {
        double d[3];
        dir_of(u, n, a1, a2, d);
        Hit3 h = march3(m, R, integ, ds, max_steps, E, d);
        out->n_marches++;
        if (h.status == S3_BAD_INPUT) {
            out->u[0] = u0[0];
            out->u[1] = u0[1];
            out->T = out->L = out->miss = NAN;
            out->status = S3_BAD_INPUT;
            return;
        }
        if (h.status != S3_LINKED) {
            if (fixed) {
                out->status = S3_NO_HIT;
                return;
            }
            for (int i = 0; i < 2; i++) u[i] = have_prev ? 0.5 * (u[i] + up[i]) : 0.5 * u[i];
            continue;
        }
        double g[2], e[3] = {h.q[0] - Rc[0], h.q[1] - Rc[1], h.q[2] - Rc[2]};
        misfit3(h.q, Rc, b1, b2, R, g);
        double miss = sqrt(dot3(e, e));
        if (miss < best) {
            best = miss;
            out->u[0] = u[0];
            out->u[1] = u[1];
            out->T = h.T;
            out->L = h.L;
            out->miss = miss;
        }
        if (fixed) {
            out->status = S3_LINKED;
            return;
        }
        if (miss <= tol) {
            out->status = S3_LINKED;
            return;
        }
        if (have_prev) {
            double du[2] = {u[0] - up[0], u[1] - up[1]}, dg[2] = {g[0] - gp[0], g[1] - gp[1]};
            double uu = du[0] * du[0] + du[1] * du[1];
            if (uu > 0.0) {
                double r0 = dg[0] - (J[0] * du[0] + J[1] * du[1]);
                double r1 = dg[1] - (J[2] * du[0] + J[3] * du[1]);
                J[0] += r0 * du[0] / uu;
                J[1] += r0 * du[1] / uu;
                J[2] += r1 * du[0] / uu;
                J[3] += r1 * du[1] / uu;
            }
        }
        double det = J[0] * J[3] - J[1] * J[2];
        double scale = fabs(J[0]) + fabs(J[1]) + fabs(J[2]) + fabs(J[3]);
        if (!(fabs(det) > 1e-12 * scale * scale)) {
            jac0(E, u, n, a1, a2, b1, b2, R, J);
            det = J[0] * J[3] - J[1] * J[2];
        }
        double s0 = -(J[3] * g[0] - J[1] * g[1]) / det, s1 = -(-J[2] * g[0] + J[0] * g[1]) / det;
        double sl = sqrt(s0 * s0 + s1 * s1);
        if (sl > 0.5) {
            s0 *= 0.5 / sl;
            s1 *= 0.5 / sl;
        }
        up[0] = u[0];
        up[1] = u[1];
        gp[0] = g[0];
        gp[1] = g[1];
        have_prev = 1;
        u[0] += s0;
        u[1] += s1;
    }
    out->status = best < INFINITY ? S3_NOT_CONVERGED : S3_NO_HIT;
    if (out->status == S3_NO_HIT) {
        out->u[0] = u0[0];
        out->u[1] = u0[1];
    }
}

static int setup3(int kind, int nx, int ny, int nz, double h, const double *c, const double *par, Med3 *m)
{
    memset(m, 0, sizeof(*m));
    m->kind = kind;
    m->nx = nx;
    m->ny = ny;
    m->nz = nz;
    m->h = h;
    m->c = c;
    for (int i = 0; i < 4; i++) m->p[i] = par ? par[i] : 0.0;
    if (kind == K3_GRID) {
        if (nx < 4 || ny < 4 || nz < 4 || !c) return -1;
        grad3(m);
    }
    return 0;
}

/* Straight-ray start: u of the direction from E towards Rc. */
static void straight_u(const double E[3], const double Rc[3], double u[2])
{
    double n[3], a1[3], a2[3], d[3] = {Rc[0] - E[0], Rc[1] - E[1], Rc[2] - E[2]};
    frame(E, n, a1, a2);
    double dn = dot3(d, n);
    u[0] = dot3(d, a1) / dn;
    u[1] = dot3(d, a2) / dn;
}

/* Linked (or warm-started, or fixed-direction) tracing of pairs (e, r) between
   elements at elem [n_elem][3] (metres from the grid centre, on one sphere). */
int or3_trace(int kind, int nx, int ny, int nz, double h, const double *c, const double *par, int n_elem,
              const double *elem, int integ, double ds_px, double tol_px, int max_marches, int max_steps, int flags,
              int n_pairs, const int32_t *pairs, double *u, double *T, double *L, double *miss, int32_t *n_marches,
              int8_t *status)
{
    Med3 m;
    if (setup3(kind, nx, ny, nz, h, c, par, &m)) return -1;
    double R = sqrt(dot3(elem, elem)) / h;
    if (max_steps <= 0) max_steps = (int)ceil(8.0 * R / ds_px);
    for (int i = 0; i < n_pairs; i++) {
        int e = pairs[2 * i], r = pairs[2 * i + 1];
        if (e == r || e < 0 || r < 0 || e >= n_elem || r >= n_elem) {
            T[i] = L[i] = miss[i] = NAN;
            n_marches[i] = 0;
            status[i] = S3_BAD_INPUT;
            continue;
        }
        double E[3], Rc[3], u0[2];
        for (int a = 0; a < 3; a++) {
            E[a] = elem[3 * e + a] / h;
            Rc[a] = elem[3 * r + a] / h;
        }
        if (flags & (F3_WARM | F3_FIXED)) {
            u0[0] = u[2 * i];
            u0[1] = u[2 * i + 1];
        } else {
            straight_u(E, Rc, u0);
        }
        Link3 o;
        link3(&m, R, integ, ds_px, tol_px, max_marches, max_steps, E, Rc, u0, (flags & F3_FIXED) != 0, &o);
        u[2 * i] = o.u[0];
        u[2 * i + 1] = o.u[1];
        T[i] = o.T;
        L[i] = o.L;
        miss[i] = o.miss;
        n_marches[i] = o.n_marches;
        status[i] = (int8_t)o.status;
    }
    free(m.g);
    return 0;
}

/* n_steps free steps from pixel point x0 along d0: points [n+1][3] (pixels). */
int or3_march_free(int kind, int nx, int ny, int nz, double h, const double *c, const double *par, int integ,
                   double ds_px, const double *x0, const double *d0, int n_steps, double *pts)
{
    Med3 m;
    if (setup3(kind, nx, ny, nz, h, c, par, &m)) return -1;
    double y[6] = {x0[0], x0[1], x0[2], d0[0], d0[1], d0[2]}, yn[6];
    double nrm = sqrt(dot3(d0, d0));
    for (int a = 3; a < 6; a++) y[a] /= nrm;
    for (int a = 0; a < 3; a++) pts[a] = y[a];
    for (int k = 1; k <= n_steps; k++) {
        step3(&m, integ, ds_px, y, yn);
        for (int i = 0; i < 6; i++) y[i] = yn[i];
        for (int a = 0; a < 3; a++) pts[3 * k + a] = y[a];
    }
    free(m.g);
    return 0;
}

/* The homogeneous Jacobian and the frames, for the tests: for pair (e, r) at u,
   J [2][2] and the emitter-frame direction d [3]. */
int or3_jac0(int n_elem, const double *elem, double h, int e, int r, const double *u, double *J, double *d)
{
    if (e < 0 || r < 0 || e >= n_elem || r >= n_elem) return -1;
    double E[3], Rc[3], n[3], a1[3], a2[3], nr[3], b1[3], b2[3];
    for (int a = 0; a < 3; a++) {
        E[a] = elem[3 * e + a] / h;
        Rc[a] = elem[3 * r + a] / h;
    }
    double R = sqrt(dot3(E, E));
    frame(E, n, a1, a2);
    frame(Rc, nr, b1, b2);
    jac0(E, u, n, a1, a2, b1, b2, R, J);
    dir_of(u, n, a1, a2, d);
    return 0;
}

/* c and per-pixel gradient at pixel points [n][3]. */
int or3_interp(int kind, int nx, int ny, int nz, double h, const double *c, const double *par, int n,
               const double *pts, double *cv, double *G)
{
    Med3 m;
    if (setup3(kind, nx, ny, nz, h, c, par, &m)) return -1;
    for (int i = 0; i < n; i++) eval3(&m, pts + 3 * i, &cv[i], G + 3 * i);
    free(m.g);
    return 0;
}

/* One fixed-direction ray of pair (e, r) at u: the misfit g [2] and the
   interception q [3] (pixels); returns the status. */
int or3_misfit(int kind, int nx, int ny, int nz, double h, const double *c, const double *par, int n_elem,
               const double *elem, int integ, double ds_px, int e, int r, const double *u, double *g, double *q)
{
    Med3 m;
    if (e < 0 || r < 0 || e >= n_elem || r >= n_elem || setup3(kind, nx, ny, nz, h, c, par, &m)) return -1;
    double E[3], Rc[3], n[3], a1[3], a2[3], nr[3], b1[3], b2[3], d[3];
    for (int a = 0; a < 3; a++) {
        E[a] = elem[3 * e + a] / h;
        Rc[a] = elem[3 * r + a] / h;
    }
    double R = sqrt(dot3(E, E));
    frame(E, n, a1, a2);
    frame(Rc, nr, b1, b2);
    dir_of(u, n, a1, a2, d);
    Hit3 hh = march3(&m, R, integ, ds_px, (int)ceil(8.0 * R / ds_px), E, d);
    for (int a = 0; a < 3; a++) q[a] = hh.q[a];
    misfit3(hh.q, Rc, b1, b2, R, g);
    free(m.g);
    return hh.status;
}
