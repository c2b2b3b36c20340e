// rtx3d.hip -- gfx950 (MI355X) kernels and C ABI for two-point ray tracing in
// 3-D between point transducers on a sphere (hemispherical arrays; arXiv
// 2511.18511 Sec. 3, 3.2-3.4) with the Broyden-like linking the paper proposes
// for 3-D configurations.  The C ABI and its conventions are declared in
// include/rtx3d.h.
//
// Design (one GPU, HIP only):
//  * The volume is packed into one record per node, (c, dc/dx, dc/dy, dc/dz) in
//    the plan's precision (16 B in FP32): a sample reads the 8 records of its
//    cell (eight 16-byte loads) and blends them trilinearly.  Per-node records
//    keep a 128^3 volume at 34 MB (MALL-resident), where per-cell trilinear
//    coefficients would take eight times that.
//  * One lane owns one pair and runs a flat loop whose body is one
//    integration step; at the sphere it does the interception, misfit, Broyden
//    update and the next ray's start in FP64, in the same loop.
//  * FP32-compensated precision as in 2-D: position, direction and the
//    travel-time sum as (hi, lo) pairs with error-free sums; FP64 for the
//    interception, misfit and the linking arithmetic.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rtx3d.h"

namespace {

constexpr int kB3 = 256;
thread_local std::string g3_err;

int fail3(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail3(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g3_err = buf;
    return code;
}

#define HIP3_TRY(expr)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail3(RTX_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------- arithmetic --
__device__ __forceinline__ float rcp3(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp3(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

template <class R>
__device__ __forceinline__ void tsum(R a, R b, R &s, R &e)  // Knuth: a + b = s + e
{
    s = a + b;
    R bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <class R>
__device__ __forceinline__ void ftsum(R a, R b, R &s, R &e)  // Dekker, |a| >= |b|
{
    s = a + b;
    e = b - (s - a);
}

// ----------------------------------------------------------------- packing --
// One thread per node: c and its per-pixel gradient, second-order central
// differences, second-order one-sided at the faces.
__device__ __forceinline__ double diff_axis(const double *c, size_t base, size_t st, int i, int n)
{
    if (i == 0) return (-3.0 * c[base] + 4.0 * c[base + st] - c[base + 2 * st]) * 0.5;
    if (i == n - 1)
        return (3.0 * c[base + (size_t)i * st] - 4.0 * c[base + (size_t)(i - 1) * st] +
                c[base + (size_t)(i - 2) * st]) *
               0.5;
    return (c[base + (size_t)(i + 1) * st] - c[base + (size_t)(i - 1) * st]) * 0.5;
}

template <class R>
__global__ void __launch_bounds__(kB3) k3_pack(const double *__restrict__ c, int nx, int ny, int nz,
                                               R *__restrict__ node)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)nx * ny * nz;
    if (k >= n) return;
    const int ix = (int)(k % nx), iy = (int)((k / nx) % ny), iz = (int)(k / ((int64_t)nx * ny));
    const size_t sxy = (size_t)nx * ny;
    R *o = node + 4 * k;
    o[0] = (R)c[k];
    o[1] = (R)diff_axis(c, (size_t)iz * sxy + (size_t)iy * nx, 1, ix, nx);
    o[2] = (R)diff_axis(c, (size_t)iz * sxy + ix, (size_t)nx, iy, ny);
    o[3] = (R)diff_axis(c, (size_t)iy * nx + ix, sxy, iz, nz);
}

// ------------------------------------------------------------------ lookup --
template <class R>
struct Vol {
    const R *node;  // [nz][ny][nx][4]
    int nx, ny, nz;
};

template <class R>
struct S3 {
    R c, gx, gy, gz;
};

__device__ __forceinline__ void load_node(const float *node, size_t k, float (&v)[4])
{
    const float4 a = *(const float4 *)(node + 4 * k);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
}

__device__ __forceinline__ void load_node(const double *node, size_t k, double (&v)[4])
{
    const double2 a = *(const double2 *)(node + 4 * k), b = *(const double2 *)(node + 4 * k + 2);
    v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y;
}

template <class R>
__device__ __forceinline__ R lerp3(R a, R b, R t)
{
    return fma(t, b - a, a);
}

// Sample at grid coordinate (uh + du, vh + dv, wh + dw); the cell index is
// clamped into the volume and the local coordinates to [0, 1].
template <class R>
__device__ __forceinline__ S3<R> lookup3(const Vol<R> &M, R uh, R du, R vh, R dv, R wh, R dw)
{
    const int ix = min(max((int)(uh + du), 0), M.nx - 2);
    const int iy = min(max((int)(vh + dv), 0), M.ny - 2);
    const int iz = min(max((int)(wh + dw), 0), M.nz - 2);
    const R t = fmin(fmax((uh - (R)ix) + du, (R)0), (R)1);
    const R s = fmin(fmax((vh - (R)iy) + dv, (R)0), (R)1);
    const R w = fmin(fmax((wh - (R)iz) + dw, (R)0), (R)1);
    const size_t sy = (size_t)M.nx, sz = (size_t)M.nx * M.ny;
    const size_t b = (size_t)iz * sz + (size_t)iy * sy + ix;
    R v[8][4];
    load_node(M.node, b, v[0]);
    load_node(M.node, b + 1, v[1]);
    load_node(M.node, b + sy, v[2]);
    load_node(M.node, b + sy + 1, v[3]);
    load_node(M.node, b + sz, v[4]);
    load_node(M.node, b + sz + 1, v[5]);
    load_node(M.node, b + sz + sy, v[6]);
    load_node(M.node, b + sz + sy + 1, v[7]);
    R f[4];
    for (int q = 0; q < 4; q++) {
        const R a0 = lerp3(v[0][q], v[1][q], t), a1 = lerp3(v[2][q], v[3][q], t);
        const R a2 = lerp3(v[4][q], v[5][q], t), a3 = lerp3(v[6][q], v[7][q], t);
        f[q] = lerp3(lerp3(a0, a1, s), lerp3(a2, a3, s), w);
    }
    return S3<R>{f[0], f[1], f[2], f[3]};
}

// --------------------------------------------------------------- ray state --
template <class R>
struct Ray3 {
    R ph[3], pl[3];  // grid coordinates, hi + lo
    R dh[3], dl[3];  // direction, hi + lo
    R Th, Tl;        // running trapezoid sum of w / c (pixels * s/m)
    int m;           // steps in this ray
};

// d' = -(G - (G.d) d) / c
template <class R>
__device__ __forceinline__ void curv3(const S3<R> &S, R ic, const R (&d)[3], R (&k)[3])
{
    const R gd = S.gx * d[0] + S.gy * d[1] + S.gz * d[2];
    k[0] = (gd * d[0] - S.gx) * ic;
    k[1] = (gd * d[1] - S.gy) * ic;
    k[2] = (gd * d[2] - S.gz) * ic;
}

template <class R>
__device__ __forceinline__ S3<R> sample_at(const Vol<R> &M, const Ray3<R> &y, const R (&off)[3])
{
    return lookup3(M, y.ph[0], y.pl[0] + off[0], y.ph[1], y.pl[1] + off[1], y.ph[2], y.pl[2] + off[2]);
}

// One step: the new state in nxt; returns the start sample (its c gives the
// quadrature term).  RK4 in the form x+ = x + ds d1 + ds^2/6 (k1 + k2 + k3),
// d+ = d1 + ds/6 (k1 + 2 k2 + 2 k3 + k4); Heun x+ = x + ds d1 + ds^2/2 k1,
// d+ = d1 + ds/2 (k1 + k2).
template <class R, bool COMP, int INTEG>
__device__ __forceinline__ S3<R> step3(const Vol<R> &M, const Ray3<R> &y, Ray3<R> &nxt, R ds, R &ic1)
{
    R d1[3], inc[3], idd[3];
    for (int a = 0; a < 3; a++) d1[a] = y.dh[a] + y.dl[a];
    const R zero[3] = {(R)0, (R)0, (R)0};
    const S3<R> s1 = sample_at(M, y, zero);
    ic1 = rcp3(s1.c);
    R k1[3];
    curv3(s1, ic1, d1, k1);
    if (INTEG == 4) {
        const R h2 = ds * (R)0.5;
        R o2[3], d2[3], k2[3], o3[3], d3[3], k3[3], o4[3], d4[3], k4[3];
        for (int a = 0; a < 3; a++) o2[a] = h2 * d1[a];
        const S3<R> s2 = sample_at(M, y, o2);
        for (int a = 0; a < 3; a++) d2[a] = fma(h2, k1[a], d1[a]);
        curv3(s2, rcp3(s2.c), d2, k2);
        for (int a = 0; a < 3; a++) {
            d3[a] = fma(h2, k2[a], d1[a]);
            o3[a] = h2 * d2[a];
        }
        const S3<R> s3 = sample_at(M, y, o3);
        curv3(s3, rcp3(s3.c), d3, k3);
        for (int a = 0; a < 3; a++) {
            d4[a] = fma(ds, k3[a], d1[a]);
            o4[a] = ds * d3[a];
        }
        const S3<R> s4 = sample_at(M, y, o4);
        curv3(s4, rcp3(s4.c), d4, k4);
        const R c6 = ds * ds * (R)(1.0 / 6.0), s6 = ds * (R)(1.0 / 6.0);
        for (int a = 0; a < 3; a++) {
            inc[a] = fma(c6, k1[a] + k2[a] + k3[a], ds * d1[a]);
            idd[a] = s6 * (k1[a] + (R)2 * (k2[a] + k3[a]) + k4[a]);
        }
    } else {
        R o2[3], d2[3], k2[3];
        for (int a = 0; a < 3; a++) o2[a] = ds * d1[a];
        const S3<R> s2 = sample_at(M, y, o2);
        for (int a = 0; a < 3; a++) d2[a] = fma(ds, k1[a], d1[a]);
        curv3(s2, rcp3(s2.c), d2, k2);
        for (int a = 0; a < 3; a++) {
            inc[a] = fma(ds * ds * (R)0.5, k1[a], ds * d1[a]);
            idd[a] = ds * (R)0.5 * (k1[a] + k2[a]);
        }
    }
    if (COMP) {
        R p[3], e[3], dd[3], dlo[3];
        for (int a = 0; a < 3; a++) {
            R s, er;
            ftsum(y.ph[a], inc[a], s, er);
            nxt.ph[a] = s;
            nxt.pl[a] = y.pl[a] + er;
            tsum(y.dh[a], idd[a], s, er);
            dd[a] = s;
            dlo[a] = y.dl[a] + er;
            p[a] = s * s;
            e[a] = fma(s, s, -p[a]);
        }
        // renormalise: eta = |d|^2 - 1 from exact squares of the hi parts, summed
        // largest first so that the 1 cancels exactly
        const R big = fmax(p[0], fmax(p[1], p[2])), sml = fmin(p[0], fmin(p[1], p[2]));
        const R mid = (p[0] + p[1] + p[2]) - big - sml;
        const R eta = (((big - (R)1) + mid) + sml) +
                      (e[0] + e[1] + e[2] + (R)2 * (dd[0] * dlo[0] + dd[1] * dlo[1] + dd[2] * dlo[2]));
        const R f = (R)-0.5 * eta;
        for (int a = 0; a < 3; a++) {
            nxt.dh[a] = dd[a];
            nxt.dl[a] = fma(dd[a], f, dlo[a]);
        }
    } else {
        R d[3];
        for (int a = 0; a < 3; a++) {
            nxt.ph[a] = y.ph[a] + inc[a];
            nxt.pl[a] = (R)0;
            d[a] = y.dh[a] + idd[a];
        }
        const R nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int a = 0; a < 3; a++) {
            nxt.dh[a] = d[a] / nrm;
            nxt.dl[a] = (R)0;
        }
    }
    return s1;
}

// ---------------------------------------------------------- geometry (FP64) --
struct Geo3 {
    int nx, ny, nz, n_elem;
    double c0[3];        // grid coordinate of the sphere centre
    double R;            // sphere radius, pixels
    double h, ds;
    const double *elem;  // [n_elem][3] pixels from the centre
};

__device__ __forceinline__ double dot(const double (&a)[3], const double (&b)[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// inward normal and tangent basis at sphere point P (the documented convention)
__device__ __forceinline__ void frame3(const double (&P)[3], double (&n)[3], double (&a1)[3], double (&a2)[3])
{
    const double r = sqrt(dot(P, P));
    for (int i = 0; i < 3; i++) n[i] = -P[i] / r;
    const bool alt = fabs(n[2]) > 0.9;
    const double k[3] = {alt ? 1.0 : 0.0, 0.0, alt ? 0.0 : 1.0};
    double c[3] = {k[1] * n[2] - k[2] * n[1], k[2] * n[0] - k[0] * n[2], k[0] * n[1] - k[1] * n[0]};
    const double cn = sqrt(dot(c, c));
    for (int i = 0; i < 3; i++) a1[i] = c[i] / cn;
    a2[0] = n[1] * a1[2] - n[2] * a1[1];
    a2[1] = n[2] * a1[0] - n[0] * a1[2];
    a2[2] = n[0] * a1[1] - n[1] * a1[0];
}

__device__ __forceinline__ void direction(const double (&u)[2], const double (&n)[3], const double (&a1)[3],
                                          const double (&a2)[3], double (&d)[3])
{
    for (int i = 0; i < 3; i++) d[i] = n[i] + u[0] * a1[i] + u[1] * a2[i];
    const double s = sqrt(dot(d, d));
    for (int i = 0; i < 3; i++) d[i] /= s;
}

// dg/du of the straight chord from E: q = E + L d, L = -2 E.d, so
// dq = L dd - 2 d (E.dd), dd/du_j = (a_j - d (d.a_j)) / |n + u.a|.
__device__ void jac_homog(const double (&E)[3], const double (&u)[2], const double (&n)[3], const double (&a1)[3],
                          const double (&a2)[3], const double (&b1)[3], const double (&b2)[3], double R,
                          double (&J)[4])
{
    double v[3], d[3];
    for (int i = 0; i < 3; i++) v[i] = n[i] + u[0] * a1[i] + u[1] * a2[i];
    const double nv = sqrt(dot(v, v));
    for (int i = 0; i < 3; i++) d[i] = v[i] / nv;
    const double L = -2.0 * dot(E, d);
    for (int j = 0; j < 2; j++) {
        const double(&aj)[3] = j ? a2 : a1;
        const double da = dot(d, aj);
        double dd[3], dq[3];
        for (int i = 0; i < 3; i++) dd[i] = (aj[i] - d[i] * da) / nv;
        const double ed = dot(E, dd);
        for (int i = 0; i < 3; i++) dq[i] = L * dd[i] - 2.0 * d[i] * ed;
        J[j] = dot(b1, dq) / R;
        J[2 + j] = dot(b2, dq) / R;
    }
}

template <class R, bool COMP>
__device__ __forceinline__ void ray3_start(Ray3<R> &ray, const Geo3 &g, const double (&E)[3], const double (&d)[3])
{
    for (int a = 0; a < 3; a++) {
        const double p = E[a] + g.c0[a];
        ray.ph[a] = (R)p;
        ray.pl[a] = COMP ? (R)(p - (double)ray.ph[a]) : (R)0;
        ray.dh[a] = (R)d[a];
        ray.dl[a] = COMP ? (R)(d[a] - (double)ray.dh[a]) : (R)0;
    }
    ray.Th = ray.Tl = (R)0;
    ray.m = 0;
}

template <class R>
__device__ __forceinline__ double pos(const Ray3<R> &y, const Geo3 &g, int a)
{
    return ((double)y.ph[a] - g.c0[a]) + (double)y.pl[a];
}

// ----------------------------------------------------------------- tracing --
struct Trace3Args {
    const int32_t *pairs;
    int64_t n_pairs;
    double *u, *tof, *len, *miss;
    int32_t *n_marches;
    int8_t *status;
    int max_marches, max_steps, flags;
    double tol;
    unsigned long long *stats;  // [2 * blocks]: steps, rays
};

__device__ __forceinline__ bool pair3(const Trace3Args &A, const Geo3 &g, int64_t p, int &e, int &r)
{
    if (A.pairs) {
        e = A.pairs[2 * p];
        r = A.pairs[2 * p + 1];
    } else {
        const int64_t k = p % (g.n_elem - 1);
        e = (int)(p / (g.n_elem - 1));
        r = (int)(k < e ? k : k + 1);
    }
    return e != r && e >= 0 && r >= 0 && e < g.n_elem && r < g.n_elem;
}

struct Link3 {
    double E[3], Rc[3], u[2], u0[2], J[4], up[2], gp[2];
    double best_miss, best_u[2], best_T, best_L;
    int have_prev, n_marches;
};

template <class R, bool COMP, int INTEG>
__global__ void __launch_bounds__(kB3) k3_trace(Vol<R> M, Geo3 g, Trace3Args A)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const R ds = (R)g.ds, R2 = (R)(g.R * g.R);
    const bool fixed = (A.flags & RTX_FIXED_ANGLE) != 0, warm = (A.flags & RTX_WARM_START) != 0;
    unsigned long long n_steps = 0, n_rays = 0;
    Ray3<R> ray;
    Link3 L;
    bool active = false;

    auto finish = [&](int st) {
        const bool has = L.best_miss < INFINITY;
        if (st == RTX_RAY_BAD_INPUT || (st == RTX_RAY_NO_HIT && !has)) {
            A.u[2 * p] = L.u0[0];
            A.u[2 * p + 1] = L.u0[1];
            if (A.tof) A.tof[p] = NAN;
            if (A.len) A.len[p] = NAN;
            if (A.miss) A.miss[p] = NAN;
        } else {
            A.u[2 * p] = L.best_u[0];
            A.u[2 * p + 1] = L.best_u[1];
            if (A.tof) A.tof[p] = L.best_T;
            if (A.len) A.len[p] = L.best_L;
            if (A.miss) A.miss[p] = L.best_miss;
        }
        if (A.n_marches) A.n_marches[p] = L.n_marches;
        A.status[p] = (int8_t)st;
    };
    auto start = [&]() {
        double n[3], a1[3], a2[3], d[3];
        frame3(L.E, n, a1, a2);
        direction(L.u, n, a1, a2, d);
        ray3_start<R, COMP>(ray, g, L.E, d);
    };
    auto next_pair = [&]() {
        while (p < A.n_pairs) {
            int e, r;
            if (!pair3(A, g, p, e, r)) {
                L.u0[0] = A.u[2 * p];
                L.u0[1] = A.u[2 * p + 1];
                L.best_miss = INFINITY;
                L.n_marches = 0;
                finish(RTX_RAY_BAD_INPUT);
                p += stride;
                continue;
            }
            for (int a = 0; a < 3; a++) {
                L.E[a] = g.elem[3 * e + a];
                L.Rc[a] = g.elem[3 * r + a];
            }
            double n[3], a1[3], a2[3], nr[3], b1[3], b2[3];
            frame3(L.E, n, a1, a2);
            frame3(L.Rc, nr, b1, b2);
            if (fixed || warm) {
                L.u[0] = A.u[2 * p];
                L.u[1] = A.u[2 * p + 1];
            } else {  // straight ray to the receiver
                double d[3] = {L.Rc[0] - L.E[0], L.Rc[1] - L.E[1], L.Rc[2] - L.E[2]};
                const double dn = dot(d, n);
                L.u[0] = dot(d, a1) / dn;
                L.u[1] = dot(d, a2) / dn;
            }
            L.u0[0] = L.u[0];
            L.u0[1] = L.u[1];
            jac_homog(L.E, L.u, n, a1, a2, b1, b2, g.R, L.J);
            L.have_prev = 0;
            L.n_marches = 0;
            L.best_miss = INFINITY;
            L.best_u[0] = L.u[0];
            L.best_u[1] = L.u[1];
            L.best_T = L.best_L = NAN;
            start();
            active = true;
            return;
        }
        active = false;
    };
    next_pair();

    while (active) {
        Ray3<R> nxt;
        R ic1;
        const S3<R> s1 = step3<R, COMP, INTEG>(M, ray, nxt, ds, ic1);
        n_steps++;
        const bool bad = !(s1.c > (R)0) || !(ray.ph[0] == ray.ph[0]) || !(ray.ph[1] == ray.ph[1]) ||
                         !(ray.ph[2] == ray.ph[2]);
        R q2 = (R)0;
        for (int a = 0; a < 3; a++) {
            const R v = (nxt.ph[a] - (R)g.c0[a]) + nxt.pl[a];
            q2 = fma(v, v, q2);
        }
        const bool crossed = !bad && q2 >= R2;
        const bool exhausted = !bad && !crossed && ray.m + 1 >= A.max_steps;
        if (!(bad || crossed || exhausted)) {
            const R term = (ray.m == 0 ? ds * (R)0.5 : ds) * ic1;
            if (COMP) {
                R s, e;
                ftsum(ray.Th, term, s, e);
                nxt.Th = s;
                nxt.Tl = ray.Tl + e;
            } else {
                nxt.Th = ray.Th + term;
                nxt.Tl = (R)0;
            }
            nxt.m = ray.m + 1;
            ray = nxt;
            continue;
        }
        // ---- end of a ray (rare, divergent, FP64)
        n_rays++;
        L.n_marches++;
        if (bad) {
            finish(RTX_RAY_BAD_INPUT);
            p += stride;
            next_pair();
            continue;
        }
        bool hit = false;
        double g2[2] = {0, 0}, miss = INFINITY;
        if (crossed) {
            double P[3], Q[3], a[3];
            for (int k = 0; k < 3; k++) {
                P[k] = pos(ray, g, k);
                Q[k] = pos(nxt, g, k);
                a[k] = Q[k] - P[k];
            }
            const double A2 = dot(a, a), B = 2.0 * dot(P, a), C = dot(P, P) - g.R * g.R;
            const double D = fmax(B * B - 4.0 * A2 * C, 0.0);
            double t = (B >= 0) ? (-2.0 * C) / (B + sqrt(D)) : (-B + sqrt(D)) / (2.0 * A2);
            t = fmin(fmax(t, 0.0), 1.0);
            double q[3];
            for (int k = 0; k < 3; k++) q[k] = P[k] + t * a[k];
            const double dsp = t * g.ds;
            R uq[3], lq[3];
            for (int k = 0; k < 3; k++) {
                const double v = q[k] + g.c0[k];
                uq[k] = (R)v;
                lq[k] = COMP ? (R)(v - (double)uq[k]) : (R)0;
            }
            const double cq = (double)lookup3(M, uq[0], lq[0], uq[1], lq[1], uq[2], lq[2]).c;
            if (!(cq > 0.0)) {
                finish(RTX_RAY_BAD_INPUT);
                p += stride;
                next_pair();
                continue;
            }
            // trapezoid with the interception as the last point: the start of this
            // step gets (ds + ds')/2 (ds'/2 when it is the emitter), q gets ds'/2
            const double acc = ray.m == 0 ? (0.5 * dsp) * (double)ic1 + (0.5 * dsp) / cq
                                          : ((double)ray.Th + (double)ray.Tl) + (0.5 * (g.ds + dsp)) * (double)ic1 +
                                                (0.5 * dsp) / cq;
            const double T = acc * g.h, Lm = (ray.m * g.ds + dsp) * g.h;
            double nr[3], b1[3], b2[3], e[3];
            frame3(L.Rc, nr, b1, b2);
            for (int k = 0; k < 3; k++) e[k] = q[k] - L.Rc[k];
            g2[0] = dot(b1, e) / g.R;
            g2[1] = dot(b2, e) / g.R;
            miss = sqrt(dot(e, e));
            hit = true;
            if (miss < L.best_miss) {
                L.best_miss = miss;
                L.best_u[0] = L.u[0];
                L.best_u[1] = L.u[1];
                L.best_T = T;
                L.best_L = Lm;
            }
        }
        if (fixed) {
            finish(hit ? RTX_RAY_LINKED : RTX_RAY_NO_HIT);
            p += stride;
            next_pair();
            continue;
        }
        if (hit && miss <= A.tol) {
            finish(RTX_RAY_LINKED);
            p += stride;
            next_pair();
            continue;
        }
        if (L.n_marches >= A.max_marches) {
            finish(L.best_miss < INFINITY ? RTX_RAY_NOT_CONVERGED : RTX_RAY_NO_HIT);
            p += stride;
            next_pair();
            continue;
        }
        if (hit) {  // Broyden-like update and step
            if (L.have_prev) {
                const double du0 = L.u[0] - L.up[0], du1 = L.u[1] - L.up[1];
                const double dg0 = g2[0] - L.gp[0], dg1 = g2[1] - L.gp[1];
                const double uu = du0 * du0 + du1 * du1;
                if (uu > 0.0) {
                    const double r0 = dg0 - (L.J[0] * du0 + L.J[1] * du1);
                    const double r1 = dg1 - (L.J[2] * du0 + L.J[3] * du1);
                    L.J[0] += r0 * du0 / uu;
                    L.J[1] += r0 * du1 / uu;
                    L.J[2] += r1 * du0 / uu;
                    L.J[3] += r1 * du1 / uu;
                }
            }
            double det = L.J[0] * L.J[3] - L.J[1] * L.J[2];
            const double sc = fabs(L.J[0]) + fabs(L.J[1]) + fabs(L.J[2]) + fabs(L.J[3]);
            if (!(fabs(det) > 1e-12 * sc * sc)) {
                double n[3], a1[3], a2[3], nr[3], b1[3], b2[3];
                frame3(L.E, n, a1, a2);
                frame3(L.Rc, nr, b1, b2);
                jac_homog(L.E, L.u, n, a1, a2, b1, b2, g.R, L.J);
                det = L.J[0] * L.J[3] - L.J[1] * L.J[2];
            }
            double s0 = -(L.J[3] * g2[0] - L.J[1] * g2[1]) / det, s1v = -(-L.J[2] * g2[0] + L.J[0] * g2[1]) / det;
            const double sl = sqrt(s0 * s0 + s1v * s1v);
            if (sl > 0.5) {
                s0 *= 0.5 / sl;
                s1v *= 0.5 / sl;
            }
            L.up[0] = L.u[0];
            L.up[1] = L.u[1];
            L.gp[0] = g2[0];
            L.gp[1] = g2[1];
            L.have_prev = 1;
            L.u[0] += s0;
            L.u[1] += s1v;
        } else {  // the ray never reached the sphere: back off
            for (int k = 0; k < 2; k++) L.u[k] = L.have_prev ? 0.5 * (L.u[k] + L.up[k]) : 0.5 * L.u[k];
        }
        start();
    }
    // per-block counters
    __shared__ unsigned long long sa[kB3 / 64], sb[kB3 / 64];
    for (int o = 32; o > 0; o >>= 1) {
        n_steps += __shfl_xor(n_steps, o);
        n_rays += __shfl_xor(n_rays, o);
    }
    if ((threadIdx.x & 63) == 0) {
        sa[threadIdx.x >> 6] = n_steps;
        sb[threadIdx.x >> 6] = n_rays;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long ta = 0, tb = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) {
            ta += sa[k];
            tb += sb[k];
        }
        A.stats[2 * blockIdx.x] = ta;
        A.stats[2 * blockIdx.x + 1] = tb;
    }
}

// Free march: ray i from x0[i] (metres) along d0[i]; positions in metres, NaN
// from the first point outside the node box.
template <class R, bool COMP, int INTEG>
__global__ void __launch_bounds__(kB3) k3_march(Vol<R> M, Geo3 g, int64_t n_rays, const double *__restrict__ x0,
                                                const double *__restrict__ d0, int n_steps, double *__restrict__ pts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rays) return;
    double E[3], d[3];
    for (int a = 0; a < 3; a++) {
        E[a] = x0[3 * i + a] / g.h;
        d[a] = d0[3 * i + a];
    }
    const double nrm = sqrt(dot(d, d));
    for (int a = 0; a < 3; a++) d[a] /= nrm;
    Ray3<R> ray;
    ray3_start<R, COMP>(ray, g, E, d);
    double *o = pts + (size_t)i * (size_t)(n_steps + 1) * 3;
    const int nn[3] = {g.nx, g.ny, g.nz};
    bool out = false;
    for (int k = 0; k <= n_steps; k++) {
        if (k > 0 && !out) {
            Ray3<R> nxt;
            R ic;
            (void)step3<R, COMP, INTEG>(M, ray, nxt, (R)g.ds, ic);
            ray = nxt;
        }
        double v[3];
        for (int a = 0; a < 3; a++) {
            v[a] = (double)ray.ph[a] + (double)ray.pl[a];
            out = out || !(v[a] >= 0.0 && v[a] <= nn[a] - 1.0);
        }
        out = out || !(ray.dh[0] == ray.dh[0]);
        for (int a = 0; a < 3; a++) o[3 * k + a] = out ? (double)NAN : (v[a] - g.c0[a]) * g.h;
    }
}

}  // namespace

// ==================================================================== plan ==
struct rtx3_plan_s {
    rtx3_grid grid;
    rtx_opts opts;
    int n_elem;
    double R_px;
    int64_t max_pairs;
    double *elem = nullptr;  // device [n_elem][3] pixels
    void *node = nullptr;    // [nz][ny][nx][4]
    bool have_medium = false;
    unsigned long long *stats = nullptr;
    int stat_blocks = 0;
};

namespace {

constexpr int kMaxBlocks3 = 4096;

int check3_opts(const rtx3_plan_s *P, const rtx_opts *o)
{
    if (o->prec != RTX_F64 && o->prec != RTX_F32C) return fail3(RTX_E_ARG, "unknown precision %d", o->prec);
    if (o->integ != RTX_RK4 && o->integ != RTX_HEUN) return fail3(RTX_E_ARG, "unknown integrator %d", o->integ);
    if (!(o->ds_px > 0 && o->ds_px <= 2)) return fail3(RTX_E_ARG, "ds_px must be in (0, 2]");
    if (!(o->tol_px >= 0)) return fail3(RTX_E_ARG, "tol_px must be >= 0");
    if (o->max_marches < 1 || o->max_marches > 1000) return fail3(RTX_E_ARG, "max_marches must be in [1, 1000]");
    if (o->max_steps < 0) return fail3(RTX_E_ARG, "max_steps < 0");
    if (o->flags & (RTX_FAN_START | RTX_INTERP_BSPLINE))
        return fail3(RTX_E_UNSUPPORTED, "the 3-D tracer has neither the fan start nor the B-spline medium");
    const double half = 0.5 * (std::min(P->grid.nx, std::min(P->grid.ny, P->grid.nz)) - 1);
    if (P->R_px + std::max(1.0, o->ds_px) > half)
        return fail3(RTX_E_ARG, "the element sphere (R = %.2f px) does not fit the grid with a margin", P->R_px);
    return RTX_OK;
}

int pack3(rtx3_plan_s *P, const double *c, hipStream_t s)
{
    if (!c) return P->have_medium ? RTX_OK : fail3(RTX_E_ARG, "c is NULL and no medium was set");
    const int64_t n = (int64_t)P->grid.nx * P->grid.ny * P->grid.nz;
    const unsigned blocks = (unsigned)((n + kB3 - 1) / kB3);
    if (P->opts.prec == RTX_F32C)
        hipLaunchKernelGGL(k3_pack<float>, dim3(blocks), dim3(kB3), 0, s, c, P->grid.nx, P->grid.ny, P->grid.nz,
                           (float *)P->node);
    else
        hipLaunchKernelGGL(k3_pack<double>, dim3(blocks), dim3(kB3), 0, s, c, P->grid.nx, P->grid.ny, P->grid.nz,
                           (double *)P->node);
    HIP3_TRY(hipGetLastError());
    P->have_medium = true;
    return RTX_OK;
}

Geo3 geo3(const rtx3_plan_s *P)
{
    Geo3 g;
    g.nx = P->grid.nx;
    g.ny = P->grid.ny;
    g.nz = P->grid.nz;
    g.n_elem = P->n_elem;
    g.c0[0] = 0.5 * (P->grid.nx - 1);
    g.c0[1] = 0.5 * (P->grid.ny - 1);
    g.c0[2] = 0.5 * (P->grid.nz - 1);
    g.R = P->R_px;
    g.h = P->grid.h;
    g.ds = P->opts.ds_px;
    g.elem = P->elem;
    return g;
}

template <class R, bool COMP>
int launch3(rtx3_plan_s *P, const Trace3Args &A, hipStream_t s)
{
    Vol<R> M{(const R *)P->node, P->grid.nx, P->grid.ny, P->grid.nz};
    const Geo3 g = geo3(P);
    auto kern = P->opts.integ == RTX_RK4 ? k3_trace<R, COMP, 4> : k3_trace<R, COMP, 2>;
    int blocks = (int)std::min<int64_t>((A.n_pairs + kB3 - 1) / kB3, kMaxBlocks3);
    P->stat_blocks = blocks;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kB3), 0, s, M, g, A);
    HIP3_TRY(hipGetLastError());
    return RTX_OK;
}

template <class R, bool COMP>
int launch3_march(rtx3_plan_s *P, int64_t n, const double *x0, const double *d0, int n_steps, double *pts,
                  hipStream_t s)
{
    Vol<R> M{(const R *)P->node, P->grid.nx, P->grid.ny, P->grid.nz};
    const Geo3 g = geo3(P);
    auto kern = P->opts.integ == RTX_RK4 ? k3_march<R, COMP, 4> : k3_march<R, COMP, 2>;
    hipLaunchKernelGGL(kern, dim3((unsigned)((n + kB3 - 1) / kB3)), dim3(kB3), 0, s, M, g, n, x0, d0, n_steps, pts);
    HIP3_TRY(hipGetLastError());
    return RTX_OK;
}

}  // namespace

extern "C" {

const char *rtx3_last_error(void) { return g3_err.c_str(); }

int rtx3_plan_create(rtx3_plan *out, const rtx3_grid *grid, int32_t n_elem, const double *elem, const rtx_opts *opts,
                     int64_t max_pairs)
{
    g3_err.clear();
    if (!out || !grid || !elem || !opts) return fail3(RTX_E_ARG, "null argument");
    *out = nullptr;
    if (grid->nx < 4 || grid->ny < 4 || grid->nz < 4) return fail3(RTX_E_ARG, "grid needs >= 4 nodes per axis");
    if ((int64_t)grid->nx * grid->ny * grid->nz > ((int64_t)1 << 28)) return fail3(RTX_E_ARG, "grid too large");
    if (!(grid->h > 0)) return fail3(RTX_E_ARG, "h must be > 0");
    if (n_elem < 2) return fail3(RTX_E_ARG, "need at least two elements");
    if (max_pairs < 1 || max_pairs > ((int64_t)1 << 31)) return fail3(RTX_E_ARG, "bad max_pairs");
    const double R = sqrt(elem[0] * elem[0] + elem[1] * elem[1] + elem[2] * elem[2]);
    if (!(R > 0)) return fail3(RTX_E_ARG, "element 0 is at the centre");
    std::vector<double> px(3 * (size_t)n_elem);
    for (int k = 0; k < n_elem; k++) {
        const double *x = elem + 3 * k;
        const double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        if (!(fabs(r - R) <= 1e-9 * R)) return fail3(RTX_E_ARG, "element %d is not on the sphere of element 0", k);
        for (int a = 0; a < 3; a++) px[3 * k + a] = x[a] / grid->h;
    }
    rtx3_plan_s *P = new rtx3_plan_s();
    P->grid = *grid;
    P->opts = *opts;
    P->n_elem = n_elem;
    P->R_px = R / grid->h;
    P->max_pairs = max_pairs;
    if (int rc = check3_opts(P, opts)) {
        delete P;
        return rc;
    }
    const size_t esz = opts->prec == RTX_F32C ? sizeof(float) : sizeof(double);
    const size_t nodes = (size_t)grid->nx * grid->ny * grid->nz;
    if (hipMalloc((void **)&P->elem, sizeof(double) * px.size()) != hipSuccess ||
        hipMalloc(&P->node, 4 * esz * nodes) != hipSuccess ||
        hipMalloc((void **)&P->stats, sizeof(unsigned long long) * 2 * kMaxBlocks3) != hipSuccess) {
        rtx3_plan_destroy(P);
        return fail3(RTX_E_NOMEM, "device allocation failed");
    }
    if (hipMemcpy(P->elem, px.data(), sizeof(double) * px.size(), hipMemcpyHostToDevice) != hipSuccess) {
        rtx3_plan_destroy(P);
        return fail3(RTX_E_HIP, "copying the elements failed");
    }
    *out = P;
    return RTX_OK;
}

int rtx3_plan_destroy(rtx3_plan P)
{
    if (!P) return RTX_OK;
    (void)hipDeviceSynchronize();
    if (P->elem) (void)hipFree(P->elem);
    if (P->node) (void)hipFree(P->node);
    if (P->stats) (void)hipFree(P->stats);
    delete P;
    return RTX_OK;
}

int rtx3_plan_set_opts(rtx3_plan P, const rtx_opts *opts)
{
    g3_err.clear();
    if (!P || !opts) return fail3(RTX_E_ARG, "null plan/opts");
    if (opts->prec != P->opts.prec) return fail3(RTX_E_ARG, "precision of a plan cannot change");
    if (int rc = check3_opts(P, opts)) return rc;
    P->opts = *opts;
    return RTX_OK;
}

int rtx3_set_medium(rtx3_plan P, const double *c, void *stream)
{
    g3_err.clear();
    if (!P) return fail3(RTX_E_ARG, "null plan");
    if (!c) return fail3(RTX_E_ARG, "c is NULL");
    return pack3(P, c, (hipStream_t)stream);
}

int rtx3_trace_rays(rtx3_plan P, const double *c, const int32_t *pairs, int64_t n_pairs, double *u, double *tof,
                    double *len, double *miss_px, int32_t *n_marches, int8_t *status, void *stream)
{
    g3_err.clear();
    if (!P) return fail3(RTX_E_ARG, "null plan");
    if (n_pairs < 0 || n_pairs > P->max_pairs) return fail3(RTX_E_ARG, "n_pairs outside [0, max_pairs]");
    if (!pairs && n_pairs != 0 && n_pairs != (int64_t)P->n_elem * (P->n_elem - 1))
        return fail3(RTX_E_ARG, "pairs == NULL requires n_pairs = n_elem (n_elem - 1)");
    if (n_pairs > 0 && (!u || !status)) return fail3(RTX_E_ARG, "u and status are required");
    hipStream_t s = (hipStream_t)stream;
    if (int rc = pack3(P, c, s)) return rc;
    if (n_pairs == 0) return RTX_OK;
    Trace3Args A;
    A.pairs = pairs;
    A.n_pairs = n_pairs;
    A.u = u;
    A.tof = tof;
    A.len = len;
    A.miss = miss_px;
    A.n_marches = n_marches;
    A.status = status;
    A.max_marches = P->opts.max_marches;
    A.max_steps = P->opts.max_steps > 0 ? P->opts.max_steps : (int)ceil(8.0 * P->R_px / P->opts.ds_px);
    A.flags = P->opts.flags;
    A.tol = P->opts.tol_px;
    A.stats = P->stats;
    return P->opts.prec == RTX_F32C ? launch3<float, true>(P, A, s) : launch3<double, false>(P, A, s);
}

int rtx3_march_free(rtx3_plan P, const double *c, int64_t n_rays, const double *x0, const double *d0,
                    int32_t n_steps, double *pts, void *stream)
{
    g3_err.clear();
    if (!P) return fail3(RTX_E_ARG, "null plan");
    if (n_rays < 0 || n_rays > ((int64_t)1 << 31) - kB3) return fail3(RTX_E_ARG, "bad n_rays");
    if (n_steps < 0 || n_steps >= (1 << 30)) return fail3(RTX_E_ARG, "bad n_steps");
    if (n_rays > 0 && (!x0 || !d0 || !pts)) return fail3(RTX_E_ARG, "x0, d0 and pts are required");
    hipStream_t s = (hipStream_t)stream;
    if (int rc = pack3(P, c, s)) return rc;
    if (n_rays == 0) return RTX_OK;
    return P->opts.prec == RTX_F32C ? launch3_march<float, true>(P, n_rays, x0, d0, n_steps, pts, s)
                                    : launch3_march<double, false>(P, n_rays, x0, d0, n_steps, pts, s);
}

int rtx3_plan_stats(rtx3_plan P, int64_t *steps, int64_t *rays)
{
    g3_err.clear();
    if (!P) return fail3(RTX_E_ARG, "null plan");
    HIP3_TRY(hipDeviceSynchronize());
    std::vector<unsigned long long> h(2 * (size_t)std::max(P->stat_blocks, 1));
    if (P->stat_blocks)
        HIP3_TRY(hipMemcpy(h.data(), P->stats, sizeof(unsigned long long) * 2 * P->stat_blocks,
                           hipMemcpyDeviceToHost));
    unsigned long long a = 0, b = 0;
    for (int k = 0; k < P->stat_blocks; k++) {
        a += h[2 * k];
        b += h[2 * k + 1];
    }
    if (steps) *steps = (int64_t)a;
    if (rays) *rays = (int64_t)b;
    return RTX_OK;
}

}  // extern "C"
