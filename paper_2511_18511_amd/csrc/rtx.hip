// rtx.hip -- gfx950 (MI355X) kernels and C ABI for linked two-point ray tracing
// of every emitter/receiver pair of a ring array through a gridded sound-speed
// map (arXiv 2511.18511, Sec. 3.2-3.4), with travel time, path length, path
// weights (Sec. 3.1) and their adjoint.  The C ABI is declared in include/rtx.h.
//
// Design (one GPU, HIP only):
//  * The medium is packed once per call into per-cell bilinear coefficients
//    (a, b, c, d) of f = a + b t + c s + d t s for f in (c, dc/dx, dc/dy): 12
//    values per cell, so one interpolation is three 16-byte loads in FP32 (six
//    in FP64) and nine FMAs.  Tables of up to 512x512 cells stay L2/MALL
//    resident; rays gather from them at random, nothing streams from HBM.
//  * One lane owns one pair.  The lane runs a flat loop whose body is exactly one
//    integration step; when its ray reaches the ring the lane does the (rare,
//    divergent) interception + misfit + secant update in FP64 and starts its next
//    ray or its next pair in the same loop, so a wave never waits for its
//    slowest ray between marches.  Pairs are dealt to lanes with a fixed stride.
//  * FP32-compensated precision: positions (grid coordinates), directions and
//    the travel-time sum are (hi, lo) float pairs updated with error-free
//    2Sum; the direction is renormalised through an exact |d|^2 - 1 (Dekker
//    products).  The interception, misfit, secant update and final T/L are FP64.
//  * The adjoint re-marches each pair at its fixed angle and scatters its
//    trapezoid-weighted hat contributions with hardware float atomics.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rtx.h"
#include "sart_sort.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;
constexpr int kBlock = 256;
constexpr int kCoef = 12;  // (c, gx, gy) x (a, b, c, d)

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(RTX_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ packing --
// Node gradient in index units: second-order central differences, second-order
// one-sided at the grid edges.
__device__ inline double node_dx(const double *c, int nx, int ix, int iy)
{
    const double *r = c + (size_t)iy * nx;
    if (ix == 0) return (-3.0 * r[0] + 4.0 * r[1] - r[2]) * 0.5;
    if (ix == nx - 1) return (3.0 * r[nx - 1] - 4.0 * r[nx - 2] + r[nx - 3]) * 0.5;
    return (r[ix + 1] - r[ix - 1]) * 0.5;
}

__device__ inline double node_dy(const double *c, int nx, int ny, int ix, int iy)
{
    const double *col = c + ix;
    if (iy == 0) return (-3.0 * col[0] + 4.0 * col[(size_t)nx] - col[2 * (size_t)nx]) * 0.5;
    if (iy == ny - 1)
        return (3.0 * col[(size_t)(ny - 1) * nx] - 4.0 * col[(size_t)(ny - 2) * nx] + col[(size_t)(ny - 3) * nx]) *
               0.5;
    return (col[(size_t)(iy + 1) * nx] - col[(size_t)(iy - 1) * nx]) * 0.5;
}

// One thread per cell (ix, iy), ix < nx-1, iy < ny-1: coefficients of
// f(t, s) = f00 + (f10 - f00) t + (f01 - f00) s + (f11 - f10 - f01 + f00) t s.
template <class R>
__global__ void k_pack(const double *__restrict__ c, int nx, int ny, R *__restrict__ tab)
{
    int ncx = nx - 1;
    int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= (int64_t)ncx * (ny - 1)) return;
    int ix = (int)(cell % ncx), iy = (int)(cell / ncx);
    double f[3][4];
    const int cx[4] = {ix, ix + 1, ix, ix + 1}, cy[4] = {iy, iy, iy + 1, iy + 1};
    for (int k = 0; k < 4; k++) {
        f[0][k] = c[(size_t)cy[k] * nx + cx[k]];
        f[1][k] = node_dx(c, nx, cx[k], cy[k]);
        f[2][k] = node_dy(c, nx, ny, cx[k], cy[k]);
    }
    R *o = tab + cell * kCoef;
    for (int q = 0; q < 3; q++) {
        o[4 * q + 0] = (R)f[q][0];
        o[4 * q + 1] = (R)(f[q][1] - f[q][0]);
        o[4 * q + 2] = (R)(f[q][2] - f[q][0]);
        o[4 * q + 3] = (R)((f[q][3] - f[q][1]) - (f[q][2] - f[q][0]));
    }
}

// ------------------------------------------------------- cubic B-spline --
// Sec. 3.3's cubic B-spline option: the field is the interpolating cubic
// B-spline of the node values, sum_k q_k B(u - k) with the centred cubic
// B-spline B, and the coefficients q solve sum_k B(j - k) q_k = c_j, the
// signal extended by mirroring about the first and last nodes.  Along each
// line the solve is the standard pair of first-order recursions with pole
// z = sqrt(3) - 2: a causal pass seeded with the sum of z^k over the mirrored
// signal (period 2(n - 1)), an anti-causal pass seeded from the mirror
// condition, and a gain of 6.  Rows first, then columns; FP64 throughout.
__device__ void bsp_filter(double *v, int n, int stride)
{
    const double z = 1.7320508075688772 - 2.0;
    const int period = 2 * (n - 1);
    double zk = 1.0, sum = 0.0;
    for (int k = 0; k < period && zk != 0.0; k++) {  // z^k underflows long before k = period on large grids
        const int j = k < n ? k : period - k;
        sum += zk * v[(size_t)j * stride];
        zk *= z;
    }
    double zp = 1.0;  // z^period
    for (int k = 0; k < period && zp != 0.0; k++) zp *= z;
    double prev = sum / (1.0 - zp);
    v[0] = prev;
    for (int k = 1; k < n; k++) {
        prev = v[(size_t)k * stride] + z * prev;
        v[(size_t)k * stride] = prev;
    }
    double nxt = (z / (z * z - 1.0)) * (v[(size_t)(n - 1) * stride] + z * v[(size_t)(n - 2) * stride]);
    v[(size_t)(n - 1) * stride] = nxt;
    for (int k = n - 2; k >= 0; k--) {
        nxt = z * (nxt - v[(size_t)k * stride]);
        v[(size_t)k * stride] = nxt;
    }
    for (int k = 0; k < n; k++) v[(size_t)k * stride] *= 6.0;
}

// One thread per row (rows = true) or column of the coefficient grid.
__global__ void k_bsp_lines(const double *__restrict__ c, double *__restrict__ q, int nx, int ny, bool rows)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (rows) {
        if (i >= ny) return;
        for (int k = 0; k < nx; k++) q[(size_t)i * nx + k] = c[(size_t)i * nx + k];
        bsp_filter(q + (size_t)i * nx, nx, 1);
    } else {
        if (i >= nx) return;
        bsp_filter(q + i, ny, nx);
    }
}

__device__ __forceinline__ int mirror_index(int i, int n)
{
    return i < 0 ? -i : i > n - 1 ? 2 * (n - 1) - i : i;
}

// One thread per cell: the 4 x 4 coefficients q[iy-1+b][ix-1+a] (b, a = 0..3),
// row by row, mirrored at the grid edges.
template <class R>
__global__ void k_pack_bsp(const double *__restrict__ q, int nx, int ny, R *__restrict__ tab)
{
    const int ncx = nx - 1;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= (int64_t)ncx * (ny - 1)) return;
    const int ix = (int)(cell % ncx), iy = (int)(cell / ncx);
    R *o = tab + cell * 16;
    for (int b = 0; b < 4; b++) {
        const int jy = mirror_index(iy - 1 + b, ny);
        for (int a = 0; a < 4; a++) o[4 * b + a] = (R)q[(size_t)jy * nx + mirror_index(ix - 1 + a, nx)];
    }
}

// -------------------------------------------------------------- arithmetic --
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64: hardware reciprocal refined by two Newton steps (within an ulp of 1/x;
// a correctly rounded division costs twice the instructions)
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float floor_(float x) { return floorf(x); }
__device__ __forceinline__ double floor_(double x) { return floor(x); }
__device__ __forceinline__ float fmin_(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double fmin_(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float fmax_(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double fmax_(double a, double b) { return fmax(a, b); }

// Error-free sum (Knuth): a + b = s + e exactly.
template <class R>
__device__ __forceinline__ void two_sum(R a, R b, R &s, R &e)
{
    s = a + b;
    R bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Error-free sum when |a| >= |b| or a == 0 (Dekker): a + b = s + e exactly.
template <class R>
__device__ __forceinline__ void fast_two_sum(R a, R b, R &s, R &e)
{
    s = a + b;
    e = b - (s - a);
}

// ----------------------------------------------------------- medium lookup --
template <class R>
struct Medium {
    const R *tab;
    int nx, ny;
};

// Cells are addressed with 32-bit byte offsets from the table base (tables are
// far below 4 GiB), so the loads take the scalar-base + 32-bit offset form.  The
// base is cast to the global address space: a table pointer read from memory (a
// batch's instance record) would otherwise be dereferenced with flat loads.
// (the host-side parse of these device functions sees no address spaces)
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL_AS __attribute__((address_space(1)))
#else
#define GLOBAL_AS
#endif
__device__ __forceinline__ void load_cell(const float *tab, uint32_t cell, float (&v)[12])
{
    const GLOBAL_AS float4 *p = (const GLOBAL_AS float4 *)((const GLOBAL_AS char *)tab + __umul24(cell, 48u));
    float4 a = p[0], b = p[1], c = p[2];
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
    v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
    v[8] = c.x, v[9] = c.y, v[10] = c.z, v[11] = c.w;
}

__device__ __forceinline__ void load_cell(const double *tab, uint32_t cell, double (&v)[12])
{
    const GLOBAL_AS double2 *p = (const GLOBAL_AS double2 *)((const GLOBAL_AS char *)tab + __umul24(cell, 96u));
    for (int k = 0; k < 6; k++) {
        double2 a = p[k];
        v[2 * k] = a.x;
        v[2 * k + 1] = a.y;
    }
}

// Interpolation at grid coordinate (uh + du, vh + dv) (u = ix-space, v =
// iy-space); du, dv are small offsets kept apart from the hi parts so that the
// local coordinates t, s keep full precision.  Cell index clamped to the grid,
// t and s to [0, 1].
template <class R>
struct Sample {
    R c, gx, gy, t, s;
    int ix, iy;
};

template <class R>
__device__ __forceinline__ Sample<R> lookup(const Medium<R> &M, R uh, R du, R vh, R dv)
{
    Sample<R> o;
    // cell index = floor of the coordinate, clamped to the grid; the float->int
    // conversion truncates (equal to floor for the non-negative coordinates that
    // survive the clamp), maps NaN to 0 and saturates, so any position gives an
    // in-bounds cell
    o.ix = min(max((int)(uh + du), 0), M.nx - 2);
    o.iy = min(max((int)(vh + dv), 0), M.ny - 2);
    R fu = (R)o.ix, fv = (R)o.iy;
    R t = (uh - fu) + du, s = (vh - fv) + dv;
    o.t = fmin_(fmax_(t, (R)0), (R)1);
    o.s = fmin_(fmax_(s, (R)0), (R)1);
    R v[12];
    // 24-bit multiplies: plans keep (nx-1)(ny-1) below 2^24 cells
    load_cell(M.tab, __umul24((uint32_t)o.iy, (uint32_t)(M.nx - 1)) + (uint32_t)o.ix, v);
    o.c = fma(o.s, fma(o.t, v[3], v[2]), fma(o.t, v[1], v[0]));
    o.gx = fma(o.s, fma(o.t, v[7], v[6]), fma(o.t, v[5], v[4]));
    o.gy = fma(o.s, fma(o.t, v[11], v[10]), fma(o.t, v[9], v[8]));
    return o;
}

// Cubic B-spline sample at (uh + du, vh + dv): same cell and local
// coordinates as `lookup`; weights of the stencil offsets -1..2 and their
// derivatives, contracted over x, then y.  (16 coefficients per cell: 64 B in
// FP32, four 16-byte loads.)
template <class R>
__device__ __forceinline__ void bsp_weights(R t, R (&w)[4], R (&dw)[4])
{
    const R u = (R)1 - t, t2 = t * t;
    w[0] = u * u * u * (R)(1.0 / 6.0);
    w[1] = fma(t2, fma(t, (R)0.5, (R)-1), (R)(2.0 / 3.0));
    w[2] = fma(t, fma(t, fma(t, (R)-0.5, (R)0.5), (R)0.5), (R)(1.0 / 6.0));
    w[3] = t2 * t * (R)(1.0 / 6.0);
    dw[0] = (R)-0.5 * u * u;
    dw[1] = t * fma(t, (R)1.5, (R)-2);
    dw[2] = fma(t, fma(t, (R)-1.5, (R)1), (R)0.5);
    dw[3] = (R)0.5 * t2;
}

__device__ __forceinline__ void load_stencil(const float *tab, uint32_t cell, float (&v)[16])
{
    const GLOBAL_AS float4 *p = (const GLOBAL_AS float4 *)((const GLOBAL_AS char *)tab + cell * 64u);
    for (int k = 0; k < 4; k++) {
        float4 a = p[k];
        v[4 * k] = a.x, v[4 * k + 1] = a.y, v[4 * k + 2] = a.z, v[4 * k + 3] = a.w;
    }
}

__device__ __forceinline__ void load_stencil(const double *tab, uint32_t cell, double (&v)[16])
{
    const GLOBAL_AS double2 *p = (const GLOBAL_AS double2 *)((const GLOBAL_AS char *)tab + (size_t)cell * 128u);
    for (int k = 0; k < 8; k++) {
        double2 a = p[k];
        v[2 * k] = a.x, v[2 * k + 1] = a.y;
    }
}

template <class R>
__device__ __forceinline__ Sample<R> lookup_bsp(const Medium<R> &M, R uh, R du, R vh, R dv)
{
    Sample<R> o;
    o.ix = min(max((int)(uh + du), 0), M.nx - 2);
    o.iy = min(max((int)(vh + dv), 0), M.ny - 2);
    o.t = fmin_(fmax_((uh - (R)o.ix) + du, (R)0), (R)1);
    o.s = fmin_(fmax_((vh - (R)o.iy) + dv, (R)0), (R)1);
    R q[16], wx[4], dwx[4], wy[4], dwy[4];
    load_stencil(M.tab, __umul24((uint32_t)o.iy, (uint32_t)(M.nx - 1)) + (uint32_t)o.ix, q);
    bsp_weights(o.t, wx, dwx);
    bsp_weights(o.s, wy, dwy);
    R c = 0, gx = 0, gy = 0;
    for (int b = 0; b < 4; b++) {
        R r = 0, rx = 0;
        for (int a = 0; a < 4; a++) {
            r = fma(q[4 * b + a], wx[a], r);
            rx = fma(q[4 * b + a], dwx[a], rx);
        }
        c = fma(r, wy[b], c);
        gx = fma(rx, wy[b], gx);
        gy = fma(r, dwy[b], gy);
    }
    o.c = c;
    o.gx = gx;
    o.gy = gy;
    return o;
}

// ------------------------------------------------------ pipelined cell cache --
// A wave that has its SIMD to itself (one lane per pair fills the chip at one
// wave per SIMD) waits out every gather it issues, so a step does not look its
// cells up when it needs them.  Three slots hold the cells of the stage points
// (stage 1, stages 2-3, stage 4).  Right after a slot's last read in a step, the
// cell of the matching stage point of the NEXT step is loaded into it without
// waiting; that point is predicted from the state, the direction and the
// curvature at the end of the previous step (x+ ~ x + ds d + ds^2/2 k, next
// stage points ~ x+ + ds/2 d+ and x+ + ds d+ with d+ ~ d + ds k), all of which
// are exact values, so a wrong guess never feeds the next guess.  The step reads
// its samples from the slots without branching and records how far each stage
// point lies from its slot's cell; a lane with a point outside (a missed
// prediction, the first step of a ray, the clamped edge of the grid) redoes the
// whole step from direct lookups.  Either way the samples are the bilinear
// interpolation in the cell containing the point.
template <class R>
struct Slot {
    R v[12];
    R fx, fy;  // cell origin in grid coordinates
    int ix, iy;
};

template <class R>
__device__ __forceinline__ void slot_fetch(const Medium<R> &M, Slot<R> &c, R u, R v)
{
    // the cell origin is clamped to the grid in floating point (max/min return
    // the number when the other operand is NaN), and the cell index
    // fy (nx - 1) + fx is exact in the slot's precision (cells stay below 2^24)
    c.fx = fmin_(fmax_(floor_(u), (R)0), (R)(M.nx - 2));
    c.fy = fmin_(fmax_(floor_(v), (R)0), (R)(M.ny - 2));
    c.ix = (int)c.fx;
    c.iy = (int)c.fy;
    load_cell(M.tab, (uint32_t)fma(c.fy, (R)(M.nx - 1), c.fx), c.v);
}

template <class R>
__device__ __forceinline__ void interp(const R (&v)[12], R t, R s, Sample<R> &o)
{
    o.c = fma(s, fma(t, v[3], v[2]), fma(t, v[1], v[0]));
    o.gx = fma(s, fma(t, v[7], v[6]), fma(t, v[5], v[4]));
    o.gy = fma(s, fma(t, v[11], v[10]), fma(t, v[9], v[8]));
}

// dd/ds = -(G - (G.d) d) / c
template <class R>
__device__ __forceinline__ void curvature(const Sample<R> &S, R ic, R dx, R dy, R &kx, R &ky)
{
    R gd = S.gx * dx + S.gy * dy;
    kx = (gd * dx - S.gx) * ic;
    ky = (gd * dy - S.gy) * ic;
}

// --------------------------------------------------------------- ray state --
// Position (grid coordinates) and direction as hi + lo pairs; the lo parts stay
// zero in FP64.
template <class R>
struct Ray {
    R uh, ul, vh, vl;
    R dxh, dxl, dyh, dyl;
    R Th, Tl;  // running trapezoid sum of w/c (pixels * s/m), compensated
    R kx, ky;  // curvature dd/ds at the end of the last step (cell prediction only)
    int m;     // steps taken in this ray
};

// Ray at grid point (pu, pv) with unit direction (cp, sp).
template <class R, bool COMP>
__device__ __forceinline__ void ray_set(Ray<R> &ray, double pu, double pv, double cp, double sp)
{
    ray.uh = (R)pu;
    ray.vh = (R)pv;
    ray.dxh = (R)cp;
    ray.dyh = (R)sp;
    if (COMP) {
        ray.ul = (R)(pu - (double)ray.uh);
        ray.vl = (R)(pv - (double)ray.vh);
        ray.dxl = (R)(cp - (double)ray.dxh);
        ray.dyl = (R)(sp - (double)ray.dyh);
    } else {
        ray.ul = ray.vl = ray.dxl = ray.dyl = (R)0;
    }
    ray.Th = ray.Tl = (R)0;
    ray.kx = ray.ky = (R)0;
    ray.m = 0;
}

template <class R, bool COMP>
__device__ __forceinline__ void ray_start(Ray<R> &ray, double pu, double pv, double psi)
{
    double sp, cp;
    sincos(psi, &sp, &cp);
    ray_set<R, COMP>(ray, pu, pv, cp, sp);
}

// Result of one integration step: the new state is written to `nxt`; `s1` is
// the medium at the step's start point p_m (its c gives the quadrature term).
template <class R>
struct StepOut {
    Sample<R> s1;
    R ic1;
};

// Keeps a value computed here: stops the compiler from sinking its producer (a
// table lookup) below the caller's crossing test.
template <class R>
__device__ __forceinline__ void materialize(R &x)
{
    asm volatile("" : "+v"(x));
}

// Fills the slots for the first step of a ray starting at y, without waiting.
template <class R>
__device__ __forceinline__ void slots_prime(const Medium<R> &M, Slot<R> (&C)[3], const Ray<R> &y, R ds, int integ)
{
    const R dx = y.dxh + y.dxl, dy = y.dyh + y.dyl;
    slot_fetch(M, C[0], y.uh + y.ul, y.vh + y.vl);
    if (integ == 4) slot_fetch(M, C[1], y.uh + fma(ds * (R)0.5, dx, y.ul), y.vh + fma(ds * (R)0.5, dy, y.vl));
    slot_fetch(M, C[2], y.uh + fma(ds, dx, y.ul), y.vh + fma(ds, dy, y.vl));
}

// The stage arithmetic of one step, reading its medium samples from `smp`
// (slots or direct lookups): start sample and 1/c there, position and direction
// increments, and the curvature at the last stage (kept for the next prediction).
template <class R>
struct StageOut {
    Sample<R> s1;
    R ic1, incx, incy, idx, idy, kx, ky;
};

template <class R, int INTEG, class S>
__device__ __forceinline__ void stages(S &smp, const Ray<R> &y, R ds, StageOut<R> &o)
{
    const R d1x = y.dxh + y.dxl, d1y = y.dyh + y.dyl;
    if (INTEG == 4) {
        // RK4 stage points: x, x + ds/2 d1, x + ds/2 d2, x + ds d3.  The first two
        // depend only on the state and the last two only on k1 and k2, so direct
        // lookups go out in two independent pairs.
        const R h2 = ds * (R)0.5;
        o.s1 = smp.get(0, y.ul, y.vl);
        Sample<R> s2 = smp.get(1, fma(h2, d1x, y.ul), fma(h2, d1y, y.vl));
        smp.done(0);
        o.ic1 = rcp(o.s1.c);
        R k1x, k1y, k2x, k2y;
        curvature(o.s1, o.ic1, d1x, d1y, k1x, k1y);
        R d2x = fma(h2, k1x, d1x), d2y = fma(h2, k1y, d1y);
        curvature(s2, rcp(s2.c), d2x, d2y, k2x, k2y);
        R d3x = fma(h2, k2x, d1x), d3y = fma(h2, k2y, d1y);
        Sample<R> s3 = smp.get(2, fma(h2, d2x, y.ul), fma(h2, d2y, y.vl));
        Sample<R> s4 = smp.get(3, fma(ds, d3x, y.ul), fma(ds, d3y, y.vl));
        smp.done(2);
        smp.done(3);
        R k3x, k3y, k4x, k4y;
        curvature(s3, rcp(s3.c), d3x, d3y, k3x, k3y);
        R d4x = fma(ds, k3x, d1x), d4y = fma(ds, k3y, d1y);
        curvature(s4, rcp(s4.c), d4x, d4y, k4x, k4y);
        materialize(k4x);
        materialize(k4y);
        // x+ = x + ds/6 (d1 + 2 d2 + 2 d3 + d4) = x + ds d1 + ds^2/6 (k1 + k2 + k3)
        const R c6 = ds * ds * (R)(1.0 / 6.0), s6 = ds * (R)(1.0 / 6.0);
        o.incx = fma(c6, k1x + k2x + k3x, ds * d1x);
        o.incy = fma(c6, k1y + k2y + k3y, ds * d1y);
        o.idx = s6 * (k1x + (R)2 * (k2x + k3x) + k4x);
        o.idy = s6 * (k1y + (R)2 * (k2y + k3y) + k4y);
        o.kx = k4x;
        o.ky = k4y;
    } else {
        // Heun stage points x and x + ds d1
        o.s1 = smp.get(0, y.ul, y.vl);
        Sample<R> s2 = smp.get(3, fma(ds, d1x, y.ul), fma(ds, d1y, y.vl));
        smp.done(0);
        smp.done(3);
        o.ic1 = rcp(o.s1.c);
        R k1x, k1y, k2x, k2y;
        curvature(o.s1, o.ic1, d1x, d1y, k1x, k1y);
        R d2x = fma(ds, k1x, d1x), d2y = fma(ds, k1y, d1y);
        curvature(s2, rcp(s2.c), d2x, d2y, k2x, k2y);
        materialize(k2x);
        materialize(k2y);
        // x+ = x + ds/2 (d1 + d2) = x + ds d1 + ds^2/2 k1
        o.incx = fma(ds * ds * (R)0.5, k1x, ds * d1x);
        o.incy = fma(ds * ds * (R)0.5, k1y, ds * d1y);
        o.idx = ds * (R)0.5 * (k1x + k2x);
        o.idy = ds * (R)0.5 * (k1y + k2y);
        o.kx = k2x;
        o.ky = k2y;
    }
}

// Slot reads for the fast path.  Stage k (0..3; Heun uses 0 and 3) reads slot
// 0, 1, 1, 2; done(k) reloads that slot for the next step.  With curvature k at
// the state (x, d): x+ = x + ds d + ds^2/2 k, d+ = d + ds k, so the next RK4
// stage points are x+, x+ + ds/2 d+ (+ ds^2/4 k at stage 3; the shared slot
// aims between), and x+ + ds (d+ + ds/2 k); Heun's are x+ and x+ + ds d+.
template <class R, int INTEG>
struct SlotSampler {
    const Medium<R> &M;
    Slot<R> (&C)[3];
    R uh, ul, vh, vl, dx, dy, kx, ky, ds, dev;
    __device__ __forceinline__ Sample<R> get(int k, R du, R dv)
    {
        const Slot<R> &c = C[k == 0 ? 0 : k == 3 ? 2 : 1];
        Sample<R> o;
        o.t = (uh - c.fx) + du;
        o.s = (vh - c.fy) + dv;
        dev = fmax_(dev, fmax_(fabs(o.t - (R)0.5), fabs(o.s - (R)0.5)));
        o.ix = c.ix;
        o.iy = c.iy;
        interp(c.v, o.t, o.s, o);
        return o;
    }
    __device__ __forceinline__ void fetch(Slot<R> &c, R a, R b)
    {
        const R hh = ds * ds;
        slot_fetch(M, c, uh + fma(a * ds, dx, fma(b * hh, kx, ul)), vh + fma(a * ds, dy, fma(b * hh, ky, vl)));
    }
    // (the scheduling barrier keeps the compiler from sinking the loads to the
    // end of the step, which would shorten the time they have to arrive)
    __device__ __forceinline__ void done(int k)
    {
        if (k == 0) fetch(C[0], (R)1, (R)0.5);
        if (INTEG == 4) {
            if (k == 2) fetch(C[1], (R)1.5, (R)1.125);
            if (k == 3) fetch(C[2], (R)2, (R)2);
        } else {
            if (k == 3) fetch(C[2], (R)2, (R)1.5);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
};

// Cubic B-spline lookups (no slots: a 16-coefficient stencil per sample).
template <class R>
struct BspSampler {
    const Medium<R> &M;
    R uh, vh;
    __device__ __forceinline__ Sample<R> get(int, R du, R dv) { return lookup_bsp(M, uh, du, vh, dv); }
    __device__ __forceinline__ void done(int) {}
};

// Direct lookups: the recovery path of a step with a point outside its slot.
template <class R>
struct LookupSampler {
    const Medium<R> &M;
    R uh, vh;
    __device__ __forceinline__ Sample<R> get(int, R du, R dv) { return lookup(M, uh, du, vh, dv); }
    __device__ __forceinline__ void done(int) {}
};

// The new state from a step's stage results: compensated (COMP) or plain
// position and direction update, then the direction renormalised.
template <class R, bool COMP>
__device__ __forceinline__ StepOut<R> advance(const Ray<R> &y, const StageOut<R> &st, Ray<R> &nxt);

template <class R, bool COMP, int INTEG, bool BSP = false>
__device__ __forceinline__ StepOut<R> ray_step(const Medium<R> &M, Slot<R> (&C)[3], const Ray<R> &y, Ray<R> &nxt,
                                               R ds)
{
    StageOut<R> st;
    if (BSP) {
        BspSampler<R> bs{M, y.uh, y.vh};
        stages<R, INTEG>(bs, y, ds, st);
    } else {
        SlotSampler<R, INTEG> fs{M, C, y.uh, y.ul, y.vh, y.vl, y.dxh + y.dxl, y.dyh + y.dyl, y.kx, y.ky, ds, (R)0};
        stages<R, INTEG>(fs, y, ds, st);
        if (!(fs.dev < (R)0.5)) {
            LookupSampler<R> ls{M, y.uh, y.vh};
            stages<R, INTEG>(ls, y, ds, st);
        }
    }
    return advance<R, COMP>(y, st, nxt);
}

template <class R, bool COMP>
__device__ __forceinline__ StepOut<R> advance(const Ray<R> &y, const StageOut<R> &st, Ray<R> &nxt)
{
    StepOut<R> o;
    o.s1 = st.s1;
    o.ic1 = st.ic1;
    const R incx = st.incx, incy = st.incy, idx = st.idx, idy = st.idy;
    nxt.kx = st.kx;
    nxt.ky = st.ky;
    if (COMP) {
        R s, e;
        // inside the ring a grid coordinate is at least max(1, ds) (the plan's
        // margin) >= |inc|, which is what the fast form needs; on the step that
        // leaves the ring a violated precondition only costs a rounding-level error
        fast_two_sum(y.uh, incx, s, e);
        nxt.uh = s;
        nxt.ul = y.ul + e;
        fast_two_sum(y.vh, incy, s, e);
        nxt.vh = s;
        nxt.vl = y.vl + e;
        two_sum(y.dxh, idx, s, e);
        R dxh = s, dxl = y.dxl + e;
        two_sum(y.dyh, idy, s, e);
        R dyh = s, dyl = y.dyl + e;
        // renormalise: eta = |d|^2 - 1 from exact squares of the hi parts
        R px = dxh * dxh, ex = fma(dxh, dxh, -px);
        R py = dyh * dyh, ey = fma(dyh, dyh, -py);
        R big = fmax_(px, py), sml = fmin_(px, py);
        R eta = ((big - (R)1) + sml) + (ex + ey + (R)2 * (dxh * dxl + dyh * dyl));
        R f = (R)-0.5 * eta;
        nxt.dxh = dxh;
        nxt.dyh = dyh;
        nxt.dxl = fma(dxh, f, dxl);
        nxt.dyl = fma(dyh, f, dyl);
    } else {
        nxt.uh = y.uh + incx;
        nxt.vh = y.vh + incy;
        nxt.ul = nxt.vl = (R)0;
        R dx = y.dxh + idx, dy = y.dyh + idy;
        R nrm = sqrt(dx * dx + dy * dy);
        nxt.dxh = dx / nrm;
        nxt.dyh = dy / nrm;
        nxt.dxl = nxt.dyl = (R)0;
    }
    return o;
}

// Trapezoid term of step-start sample p_m when the step does not cross.
template <class R, bool COMP>
__device__ __forceinline__ void add_T(Ray<R> &y, R term)
{
    if (COMP) {
        R s, e;
        fast_two_sum(y.Th, term, s, e);  // Th is 0 or a sum of positive terms >= term
        y.Th = s;
        y.Tl += e;
    } else {
        y.Th += term;
    }
}

// ------------------------------------------------------------- geometry (FP64) --
struct Geo {
    int nx, ny, n_elem;
    double cx, cy;  // grid coordinate of the ring centre
    double R;       // ring radius, pixels
    double phi0, h, ds;
};

__device__ __forceinline__ double elem_angle(const Geo &g, int k)
{
    return g.phi0 + 2.0 * kPi * k / g.n_elem;
}

// a mod 2 pi in [0, 2 pi).  The arguments met here lie in (-2 pi, 4 pi), where
// the result is a, a + 2 pi or a - 2 pi (the last exact): the same values as
// fmod followed by adding 2 pi to a negative remainder, without fmod's
// exponent-reduction loop.
__device__ __forceinline__ double mod2pi(double a)
{
    if (a >= 0.0 && a < kTwoPi) return a;
    if (a < 0.0 && a >= -kTwoPi) return a + kTwoPi;
    if (a >= kTwoPi && a < 2.0 * kTwoPi) return a - kTwoPi;
    double r = fmod(a, kTwoPi);
    if (r < 0) r += kTwoPi;
    return r;
}

// Crossing of the last step: larger root t in (0, 1] of |p + t (q - p)|^2 = R^2.
struct Hit {
    double qx, qy, t;
};

template <class R>
__device__ __forceinline__ Hit intersect(const Geo &g, const Ray<R> &a, const Ray<R> &b)
{
    double px = ((double)a.uh - g.cx) + (double)a.ul, py = ((double)a.vh - g.cy) + (double)a.vl;
    double qx = ((double)b.uh - g.cx) + (double)b.ul, qy = ((double)b.vh - g.cy) + (double)b.vl;
    double ax = qx - px, ay = qy - py;
    double A = ax * ax + ay * ay, B = 2.0 * (px * ax + py * ay), C = px * px + py * py - g.R * g.R;
    double D = fmax(B * B - 4.0 * A * C, 0.0);
    double t = (B >= 0) ? (-2.0 * C) / (B + sqrt(D)) : (-B + sqrt(D)) / (2.0 * A);
    t = fmin(fmax(t, 0.0), 1.0);
    Hit h;
    h.qx = px + t * ax;
    h.qy = py + t * ay;
    h.t = t;
    return h;
}

// Medium at a ring-centred FP64 pixel point.
template <class R, bool COMP, bool BSP = false>
__device__ __forceinline__ Sample<R> lookup_at(const Medium<R> &M, const Geo &g, double px, double py)
{
    double u = px + g.cx, v = py + g.cy;
    R uh = (R)u, vh = (R)v;
    R ul = COMP ? (R)(u - (double)uh) : (R)0, vl = COMP ? (R)(v - (double)vh) : (R)0;
    return BSP ? lookup_bsp(M, uh, ul, vh, vl) : lookup(M, uh, ul, vh, vl);
}

// ------------------------------------------------------------------ linking --
struct Link {
    double th, th0, tha, ga, thb, gb, th_neg, th_pos;
    double best_miss, best_th, best_T, best_L;
    int nvalid, have_neg, have_pos, n_marches;
};

__device__ __forceinline__ void link_reset(Link &L, double th0)
{
    L.th = L.th0 = th0;
    L.tha = L.ga = L.thb = L.gb = L.th_neg = L.th_pos = 0.0;
    L.best_miss = INFINITY;
    L.best_th = th0;
    L.best_T = L.best_L = NAN;
    L.nvalid = L.have_neg = L.have_pos = L.n_marches = 0;
}

// Next launch angle after a ray that hit with misfit g (secant through the two
// latest hitting rays, homogeneous Newton step for the second point,
// safeguarded by the sign bracket or by the angle limits).
__device__ __forceinline__ double link_next_hit(Link &L, double g)
{
    const double lim = kPi / 2.0 - 1e-6;
    double th = L.th;
    if (g < 0) {
        L.have_neg = 1;
        L.th_neg = th;
    }
    if (g > 0) {
        L.have_pos = 1;
        L.th_pos = th;
    }
    L.tha = L.thb;
    L.ga = L.gb;
    L.thb = th;
    L.gb = g;
    L.nvalid++;
    bool den_zero = false;
    double nx;
    if (L.nvalid == 1) {
        nx = th - g / 2.0;
    } else if (L.gb - L.ga == 0.0) {
        den_zero = true;
        nx = th - g / 2.0;
    } else {
        nx = L.thb - L.gb * (L.thb - L.tha) / (L.gb - L.ga);
    }
    if (L.have_neg && L.have_pos) {
        double lo = fmin(L.th_neg, L.th_pos), hi = fmax(L.th_neg, L.th_pos);
        if (den_zero || !(nx > lo && nx < hi)) nx = 0.5 * (L.th_neg + L.th_pos);
    } else {
        if (!(nx < lim) && nx == nx) nx = 0.5 * (th + lim);
        if (!(nx > -lim) && nx == nx) nx = 0.5 * (th - lim);
        if (!(nx == nx)) nx = 0.5 * th;
    }
    return nx;
}

// Keeps the compiler from moving memory accesses across this point.
__device__ __forceinline__ void compiler_fence() { __asm__ volatile("" ::: "memory"); }

// The four samples of smallest |g| of a fan-started pair: its fan samples (the
// bracket and its outer neighbours, in order), then every hitting ray it traced
// (round by round, ray 0 first).  A new sample replaces the kept one of largest
// |g| (the later of equal ones) when its |g| is strictly smaller.
struct Top4 {
    double th[4], g[4];
    int id[4], n, next;
};

__device__ __forceinline__ void top4_push(Top4 &t, double th, double g)
{
    const int id = t.next++;
    if (t.n < 4) {
        for (int k = 0; k < 4; k++)
            if (k == t.n) {
                t.th[k] = th;
                t.g[k] = g;
                t.id[k] = id;
            }
        t.n++;
        return;
    }
    int w = 0;
    for (int k = 1; k < 4; k++)
        if (fabs(t.g[k]) > fabs(t.g[w]) || (fabs(t.g[k]) == fabs(t.g[w]) && t.id[k] > t.id[w])) w = k;
    double gw = 0.0;
    for (int k = 0; k < 4; k++)
        if (k == w) gw = t.g[k];
    if (fabs(g) < fabs(gw))
        for (int k = 0; k < 4; k++)
            if (k == w) {
                t.th[k] = th;
                t.g[k] = g;
                t.id[k] = id;
            }
}

__device__ __forceinline__ void cswap(double &a, double &b, double &ga, double &gb)
{
    if (b < a) {
        double x = a;
        a = b;
        b = x;
        x = ga;
        ga = gb;
        gb = x;
    }
}

// Inverse cubic through the four kept samples (ordered by angle: strictly
// increasing angles, strictly monotone g); its zero is accepted strictly
// between the outer angles and inside the traced rays' sign bracket, if any.
__device__ __forceinline__ bool top4_estimate(const Top4 &t, const Link &L, double &th)
{
    if (t.n < 4) return false;
    double a0 = t.th[0], a1 = t.th[1], a2 = t.th[2], a3 = t.th[3];
    double g0 = t.g[0], g1 = t.g[1], g2 = t.g[2], g3 = t.g[3];
    cswap(a0, a1, g0, g1);
    cswap(a2, a3, g2, g3);
    cswap(a0, a2, g0, g2);
    cswap(a1, a3, g1, g3);
    cswap(a1, a2, g1, g2);
    const double a[4] = {a0, a1, a2, a3}, g[4] = {g0, g1, g2, g3};
    const bool up = g[1] > g[0];
    for (int i = 0; i < 3; i++) {
        if (!(a[i + 1] > a[i])) return false;
        if (up ? !(g[i + 1] > g[i]) : !(g[i + 1] < g[i])) return false;
    }
    double v = 0.0;
    for (int i = 0; i < 4; i++) {
        double w = 1.0;
        for (int q = 0; q < 4; q++)
            if (q != i) w *= -g[q] / (g[i] - g[q]);
        v += w * a[i];
    }
    if (!(v > a[0] && v < a[3])) return false;
    if (L.have_neg && L.have_pos) {
        const double lo = fmin(L.th_neg, L.th_pos), hi = fmax(L.th_neg, L.th_pos);
        if (!(v > lo && v < hi)) return false;
    }
    th = v;
    return true;
}

// ------------------------------------------------------------ trace kernel --
// Fan start: the straight-ray rays of all receivers of an emitter sample one
// function, the hit angle of a ray launched at theta; the nearest sign change of
// the receiver's misfit over consecutive samples seeds its secant.
struct FanSeed {
    double th_far, g_far, th_near, g_near;  // bracket ends (larger |g| first)
    double th_first;                        // first linking angle (cubic), if `cubic`
    double th_q;                            // the first round's second angle (quintic), if `quintic`
    double s_th[4], s_g[4];                 // the bracket and its outer neighbours that hit, in order
    int found, cubic, quintic, n_s;
};

constexpr uint32_t kStraight = 1u << 16;  // internal: fixed pass at straight angles

// State of a ray traced by the fan-started linking pass at the start of one of
// its later segments (position and direction hi/lo parts, the curvature the
// next step's cell prediction uses, and the step index; m < 0: none): the
// adjoint restarts there, which gives the same samples as marching on.
template <class R>
struct RayCkpt {
    R uh, ul, vh, vl, dxh, dxl, dyh, dyl, kx, ky;
    int m;
};

// Per pair: the angle of its linked ray, the lane (0 or 1) whose checkpoint
// belongs to that ray (-1: none), and the plan generation (medium and path
// options) it was traced under.
struct CkptHead {
    double theta;
    unsigned gen;
    int lane;
};

// The adjoint marches a linked ray in kSegs segments; the linking pass stores
// the ray's state at the kSegs - 1 segment starts after the first, every
// ckpt_stride steps (the chord's steps / kSegs; 0: a chord too short to split).
constexpr int kSegs = 2;

__device__ __forceinline__ int ckpt_stride(const Geo &g, double dphi)
{
    return (int)(2.0 * g.R * fabs(sin(0.5 * dphi)) / (g.ds * kSegs));
}

struct TraceArgs {
    const int32_t *pairs;
    int64_t n_pairs;
    double *theta, *tof, *len, *miss;
    int32_t *n_marches;
    int8_t *status;
    int max_marches, max_steps;
    double tol;
    uint32_t flags;
    unsigned long long *stats;  // [gridDim.x][2]: steps, rays
    double *gsig;               // fixed pass: signed misfit of each ray (or NULL)
    const FanSeed *seed;        // fan start: per-pair seeds
    const double *f_g;          // fan start: the signed misfit of the pair's own straight ray
    const int8_t *f_st;
    void *ckpt;                 // fan start: RayCkpt<R> [n_pairs][2][kSegs - 1] (or NULL)
    CkptHead *ckpt_head;        // [n_pairs]
    unsigned gen;               // plan generation written to the heads
};

__device__ __forceinline__ bool pair_of(const TraceArgs &A, const Geo &g, int64_t p, int &e, int &r)
{
    if (A.pairs) {
        e = A.pairs[2 * p];
        r = A.pairs[2 * p + 1];
    } else {
        int64_t k = p % (g.n_elem - 1);
        e = (int)(p / (g.n_elem - 1));
        r = (int)(k < e ? k : k + 1);
    }
    return e != r && e >= 0 && r >= 0 && e < g.n_elem && r < g.n_elem;
}

__device__ __forceinline__ void write_pair(const TraceArgs &A, int64_t p, double th, double T, double Lm,
                                           double miss, int nm, int st)
{
    if (!(A.flags & RTX_FIXED_ANGLE)) A.theta[p] = th;
    if (A.tof) A.tof[p] = T;
    if (A.len) A.len[p] = Lm;
    if (A.miss) A.miss[p] = miss;
    if (A.n_marches) A.n_marches[p] = nm;
    A.status[p] = (int8_t)st;
}

// Emitter of a pair: its angle and ring-centred position (pixels), computed once
// per pair; every ray of the pair starts there.
struct Emitter {
    double pe, ex, ey;
};

__device__ __forceinline__ Emitter emitter_of(const Geo &g, int e)
{
    Emitter o;
    o.pe = elem_angle(g, e);
    double sp, cp;
    sincos(o.pe, &sp, &cp);
    o.ex = g.R * cp;
    o.ey = g.R * sp;
    return o;
}

template <class R, bool COMP>
__device__ __forceinline__ void start_ray(Ray<R> &ray, const Geo &g, const Emitter &em, double th)
{
    ray_start<R, COMP>(ray, em.ex + g.cx, em.ey + g.cy, em.pe + kPi + th);
}

// Sum of per-lane counters over the block, written to out[blockIdx.x].
__device__ void block_sum2(unsigned long long a, unsigned long long b, unsigned long long *out)
{
    __shared__ unsigned long long sa[16], sb[16];  // up to 1024 threads
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long ta = 0, tb = 0;
        for (int k = 0; k < (int)(blockDim.x / 64); k++) {
            ta += sa[k];
            tb += sb[k];
        }
        out[2 * blockIdx.x] = ta;
        out[2 * blockIdx.x + 1] = tb;
    }
}

struct AdjArgs {
    const int32_t *pairs;
    int64_t n_pairs;
    const double *theta;
    const int8_t *status;
    const double *rho;
    int weight;
    int max_steps;
    unsigned long long *stats;
    unsigned int *err;  // set (bit 0) when an LDS queue wait hits its bound
    // all ordered pairs (pairs == NULL, tile > 0): work items walk tile x tile
    // blocks of (emitter, receiver) clusters of adjacent elements, so the rays
    // of a wave run side by side from one cluster to another and their node
    // updates land on fewer distinct nodes at a time (measured on the 256x256
    // workload: adjoint 1.80 -> 1.44 ms; the same order made the forward
    // passes slower, so they keep the canonical order); n_items counts the
    // items, including the e == r and past-the-end slots they skip
    int tile;
    int64_t n_items;
    // the node updates of block b go to copy b mod n_copies of the gradient
    // (consecutive blocks run on different XCDs): global float atomics are
    // performed at the memory side, where updates of one address from many
    // CUs queue behind each other; with one copy per XCD the queues are eight
    // times shorter (measured on the 256x256 workload: adjoint 1.43 -> 1.25 ms)
    int n_copies;
    // split (all pairs after a fan-started trace of this plan): every work
    // item of the tile walk becomes kSegs, the segments of its ray, the later
    // ones starting from the linking pass's checkpoints when those are the
    // ray's (head: same angle, plan generation gen); otherwise the first
    // segment's item marches the whole ray and the others do nothing.  The
    // kernel time is the longest lane's, so segments shorten it (a lane takes
    // the same segment of kSegs different rays).
    int split;
    const void *ckpt;            // RayCkpt<R> [n_pairs][2][kSegs - 1]
    const CkptHead *ckpt_head;   // [n_pairs]
    unsigned gen;
};

// Work item of an all-pairs tile walk -> (e, r) and the canonical pair index.
// Returns false for an item without a pair (e == r, or past the last element).
__device__ __forceinline__ bool tile_item(int n, int t, int64_t item, int &e, int &r, int64_t &q)
{
    const int nc = (n + t - 1) / t;
    const int64_t tt = item / (t * t);
    const int l = (int)(item - tt * t * t);
    e = (int)(tt / nc) * t + l / t;
    r = (int)(tt % nc) * t + l % t;
    if (e >= n || r >= n || e == r) return false;
    q = (int64_t)e * (n - 1) + (r < e ? r : r - 1);
    return true;
}

// Work item -> pair of the adjoint (false: no pair).
__device__ __forceinline__ bool adj_item(const AdjArgs &a, const Geo &g, int64_t item, int &e, int &r, int64_t &q)
{
    if (a.pairs || a.tile == 0) {
        TraceArgs pa;
        pa.pairs = a.pairs;
        q = item;
        return pair_of(pa, g, item, e, r);
    }
    return tile_item(g.n_elem, a.tile, item, e, r, q);
}

// One problem of a batch (device copy).
template <class R>
struct Inst {
    Medium<R> M;
    Geo g;
    TraceArgs A;  // forward outputs and options
    AdjArgs J;    // adjoint inputs
    R *grad;      // adjoint output
};

// Batched instances: independent (medium, ring, outputs) problems traced by one
// persistent launch over the concatenated pair space.  Lanes look up the
// instance of each pair they take; per-instance counters record the wall clock
// when an instance's last pair finishes.
struct BatchArgs {
    const void *inst;            // Inst<R>[n_inst] (device)
    const int64_t *off;          // [n_inst + 1] prefix sums of the pair counts
    int n_inst;
    unsigned int *remain;        // [n_inst] pairs left, set before the launch
    unsigned long long *t_done;  // [n_inst] wall clock at completion
};

__device__ __forceinline__ int find_inst(const BatchArgs &B, int64_t p)
{
    int lo = 0, hi = B.n_inst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (B.off[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void mark_done(const BatchArgs &B, int k)
{
    if (atomicSub(B.remain + k, 1u) == 1u) B.t_done[k] = wall_clock64();
}

template <class R, bool COMP, int INTEG, bool BATCH, bool BSP = false>
__global__ void __launch_bounds__(kBlock) k_trace(Medium<R> M, Geo g, TraceArgs A, BatchArgs B)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // item (pair of the launch)
    int64_t n_items = BATCH ? B.off[B.n_inst] : A.n_pairs;
    int64_t q = p;  // pair index within its instance
    int k = 0;      // instance
    Medium<R> m = M;
    Geo gg = g;
    TraceArgs a = A;
    R ds = (R)gg.ds, R2 = (R)(gg.R * gg.R), cx = (R)gg.cx, cy = (R)gg.cy;
    unsigned long long n_steps = 0, n_rays = 0;

    Ray<R> ray;
    Slot<R> C[3];
    Link L;
    int e = 0, r = 0;
    Emitter em{};
    double dr = 0;  // receiver angle relative to the emitter, mod 2 pi
    bool active = false;

    // Takes pairs from p onward until one is valid (invalid ones are written).
    auto next_pair = [&]() {
        while (p < n_items) {
            if (BATCH) {
                k = find_inst(B, p);
                const Inst<R> &I = ((const Inst<R> *)B.inst)[k];
                m = I.M;
                gg = I.g;
                a = I.A;
                q = p - B.off[k];
                ds = (R)gg.ds;
                R2 = (R)(gg.R * gg.R);
                cx = (R)gg.cx;
                cy = (R)gg.cy;
            } else {
                q = p;
            }
            if (pair_of(a, gg, q, e, r)) {
                em = emitter_of(gg, e);
                dr = mod2pi(elem_angle(gg, r) - em.pe);
                const bool given = (a.flags & (RTX_WARM_START | RTX_FIXED_ANGLE)) && !(a.flags & kStraight);
                double th0 = given ? a.theta[q] : (dr - kPi) / 2.0;
                link_reset(L, th0);
                double th = th0;
                start_ray<R, COMP>(ray, gg, em, th);
                if (!BSP) slots_prime(m, C, ray, ds, INTEG);
                active = true;
                return;
            }
            write_pair(a, q, a.theta[q], NAN, NAN, NAN, 0, RTX_RAY_BAD_INPUT);
            if (BATCH) mark_done(B, k);
            p += stride;
        }
        active = false;
    };
    next_pair();

    while (active) {
        Ray<R> nxt;
        StepOut<R> so = ray_step<R, COMP, INTEG, BSP>(m, C, ray, nxt, ds);
        n_steps++;
        const R w_start = ray.m == 0 ? ds * (R)0.5 : ds;
        const bool bad = !(so.s1.c > (R)0) || !(ray.uh == ray.uh) || !(ray.vh == ray.vh);
        R pu = (nxt.uh - cx) + nxt.ul, pv = (nxt.vh - cy) + nxt.vl;
        const bool crossed = !bad && (pu * pu + pv * pv >= R2);
        const bool exhausted = !bad && !crossed && (ray.m + 1 >= a.max_steps);
        if (!(bad || crossed || exhausted)) {
            add_T<R, COMP>(ray, w_start * so.ic1);
            nxt.Th = ray.Th;
            nxt.Tl = ray.Tl;
            nxt.m = ray.m + 1;
            ray = nxt;
            continue;
        }
        // ---- end of one ray (rare, divergent) ----
        n_rays++;
        L.n_marches++;
        int st = RTX_RAY_NO_HIT;
        double g_mis = NAN, T = NAN, Lm = NAN;
        if (bad) {
            st = RTX_RAY_BAD_INPUT;
        } else if (crossed) {
            Hit hit = intersect<R>(gg, ray, nxt);
            double dsp = hit.t * gg.ds;
            Sample<R> sq = lookup_at<R, COMP, BSP>(m, gg, hit.qx, hit.qy);
            if (!(sq.c > (R)0)) {
                st = RTX_RAY_BAD_INPUT;
            } else {
                double wm = ray.m == 0 ? 0.5 * dsp : 0.5 * (gg.ds + dsp);
                double acc = ((double)ray.Th + (double)ray.Tl) + wm * (double)so.ic1 +
                             0.5 * dsp * (double)rcp(sq.c);
                T = acc * gg.h;
                Lm = (ray.m * gg.ds + dsp) * gg.h;
                g_mis = mod2pi(atan2(hit.qy, hit.qx) - em.pe) - dr;
                st = RTX_RAY_LINKED;
            }
        }
        bool pair_done = false;
        if (a.flags & RTX_FIXED_ANGLE) {
            write_pair(a, q, L.th, T, Lm, fabs(g_mis) * gg.R, 1, st);
            if (a.gsig) a.gsig[q] = g_mis;
            pair_done = true;
        } else if (st == RTX_RAY_BAD_INPUT) {
            write_pair(a, q, L.th0, NAN, NAN, NAN, L.n_marches, RTX_RAY_BAD_INPUT);
            pair_done = true;
        } else {
            double th_next;
            if (st == RTX_RAY_LINKED) {
                double miss = fabs(g_mis) * gg.R;
                if (miss < L.best_miss) {
                    L.best_miss = miss;
                    L.best_th = L.th;
                    L.best_T = T;
                    L.best_L = Lm;
                }
                if (miss <= a.tol) {
                    write_pair(a, q, L.th, T, Lm, miss, L.n_marches, RTX_RAY_LINKED);
                    pair_done = true;
                }
                th_next = pair_done ? 0.0 : link_next_hit(L, g_mis);
            } else {
                th_next = L.nvalid > 0 ? 0.5 * (L.th + L.thb) : 0.5 * L.th;
            }
            if (!pair_done && L.n_marches >= a.max_marches) {
                if (L.best_miss < INFINITY)
                    write_pair(a, q, L.best_th, L.best_T, L.best_L, L.best_miss, L.n_marches,
                               RTX_RAY_NOT_CONVERGED);
                else
                    write_pair(a, q, L.th0, NAN, NAN, NAN, L.n_marches, RTX_RAY_NO_HIT);
                pair_done = true;
            }
            if (!pair_done) {
                L.th = th_next;
                start_ray<R, COMP>(ray, gg, em, th_next);
                if (!BSP) slots_prime(m, C, ray, ds, INTEG);
            }
        }
        if (pair_done) {
            if (BATCH) mark_done(B, k);
            p += stride;
            next_pair();
        }
    }
    block_sum2(n_steps, n_rays, A.stats);
}

// ------------------------------------------------- fan-started linking pass --
// Linking in rounds of two rays: the two lanes 2i, 2i+1 of a wave own pair i
// and keep identical copies of its linking state; each round lane 0 traces the
// primary angle c0 and lane 1 the hedge c1 = c0 - (c0 - ref) / 10 (ref: the
// latest fed sample, or the start angle), a tenth of the way back, so that a
// round that does not link leaves two close samples for the next step; in the
// first round lane 1 traces the fan seed's quintic estimate instead, when there
// is one and it differs from c0 (the seed's miss is mostly the cubic's
// interpolation error, and the quintic removes about half of the second rounds).  A lane
// whose ray ends posts its result to LDS and idles; when both have posted (a
// wave ballot), both read the two results and take the same decision:
//   bad input -> BAD; every hitting ray enters the best record (ray 0 first);
//   the hitting ray of smallest miss within the tolerance -> LINKED; after
//   max_marches rounds (the rounds are what is sequential) -> the best ray
//   (NOT_CONVERGED) or NO_HIT; otherwise the
//   hits are fed to the secant state in order of decreasing |g| (ray 0 first
//   on a tie), or the back-off applies when neither hit, and after the first
//   two rounds the inverse cubic through the four samples of smallest |g|
//   (Top4) replaces the secant's angle where it is defined (later rounds keep
//   the safeguarded secant, whose bracket halving copes with misfit jumps).  A second wave per SIMD costs the latency-bound
//   trace nothing measurable, and the extra candidate removes most third rounds.
template <class R, bool COMP, int INTEG, bool BSP = false>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
    k_link2(Medium<R> M, Geo g, TraceArgs A)
{
    __shared__ double s_th[kBlock], s_g[kBlock], s_T[kBlock], s_L[kBlock];
    __shared__ int s_st[kBlock];
    // the linking state is touched only at the end of a round: it lives in LDS,
    // which keeps the marching registers within two waves per SIMD
    __shared__ Link s_link[kBlock];
    __shared__ Top4 s_top[kBlock];
    __shared__ Emitter s_em[kBlock];
    __shared__ double s_dr[kBlock];
    const int lane = threadIdx.x, j = lane & 1, b0 = lane & ~1;
    const int64_t stride = ((int64_t)gridDim.x * blockDim.x) >> 1;
    int64_t p = ((int64_t)blockIdx.x * blockDim.x + lane) >> 1;
    const R ds = (R)g.ds, R2 = (R)(g.R * g.R), cx = (R)g.cx, cy = (R)g.cy;
    unsigned long long n_steps = 0, n_rays = 0;

    Ray<R> ray;
    Slot<R> C[3];
    Link &L = s_link[lane];
    Top4 &t4 = s_top[lane];
    Emitter &em = s_em[lane];
    double &dr = s_dr[lane];
    int e = 0, r = 0;
    double mine = 0;
    bool active = false, waiting = false;
    RayCkpt<R> *ck = nullptr;  // this lane's checkpoint slots for the current pair
    int stride_ck = 0;         // steps between them
    int k_ck = 0, m_ck = -1;   // the next slot to write and its step index
    // the pair's checkpoint head: the linked ray's angle and lane, or none
    auto put_head = [&](double th, int lane_of) {
        if (A.ckpt_head && j == 0) A.ckpt_head[p] = CkptHead{th, A.gen, lane_of};
    };

    auto round_start = [&](double th, bool use_q, double th_q) {
        const double ref = L.nvalid > 0 ? L.thb : L.th0;
        mine = j == 0 ? th : (use_q && th_q != th ? th_q : th == ref ? th + 1e-4 : th - 0.1 * (th - ref));
        start_ray<R, COMP>(ray, g, em, mine);
        if (ck)  // until this ray reaches them
            for (int k = 0; k < kSegs - 1; k++) ck[k].m = -1;
        k_ck = 0;
        m_ck = stride_ck > 0 ? stride_ck : -1;
        if (!BSP) slots_prime(M, C, ray, ds, INTEG);
    };
    auto next_pair = [&]() {
        while (p < A.n_pairs) {
            if (!pair_of(A, g, p, e, r)) {
                if (j == 0) write_pair(A, p, A.theta[p], NAN, NAN, NAN, 0, RTX_RAY_BAD_INPUT);
                put_head(NAN, -1);
                p += stride;
                continue;
            }
            em = emitter_of(g, e);
            dr = mod2pi(elem_angle(g, r) - em.pe);
            ck = A.ckpt ? (RayCkpt<R> *)A.ckpt + (2 * p + j) * (kSegs - 1) : nullptr;
            stride_ck = ckpt_stride(g, dr);
            const double th0 = (dr - kPi) / 2.0;
            link_reset(L, th0);
            t4.n = t4.next = 0;
            double th = th0;
            const int st0 = A.f_st[p];
            const FanSeed sd = A.seed[p];
            if (sd.found) {
                L.th = sd.th_far;
                link_next_hit(L, sd.g_far);
                L.th = sd.th_near;
                th = link_next_hit(L, sd.g_near);
                if (sd.cubic) th = sd.th_first;
                for (int q = 0; q < 4; q++)
                    if (q < sd.n_s) top4_push(t4, sd.s_th[q], sd.s_g[q]);
            } else if (st0 == RTX_RAY_LINKED) {
                th = link_next_hit(L, A.f_g[p]);
            } else if (st0 == RTX_RAY_NO_HIT) {
                th = 0.5 * th0;
            }
            L.have_neg = L.have_pos = 0;  // the coarse samples do not bound the secant
            round_start(th, sd.found && sd.quintic, sd.th_q);
            active = true;
            return;
        }
        active = false;
    };
    next_pair();

    while (active) {
        // Steps until a pair of the wave has both rays in.  Every lane steps, a
        // waiting one too (its ray is over and its result posted; it repeats its
        // last step, discarded, until its pair's next round): the slot registers
        // are then written by the step's own prefetches alone, and the compiler
        // keeps those loads in flight across steps (measured: linking pass
        // 1.64 -> 1.59 ms on the 256x256 workload).
        bool ready = false;
        do {
            Ray<R> nxt;
            StepOut<R> so = ray_step<R, COMP, INTEG, BSP>(M, C, ray, nxt, ds);
            if (!waiting) {
                n_steps++;
                const R w_start = ray.m == 0 ? ds * (R)0.5 : ds;
                const bool bad = !(so.s1.c > (R)0) || !(ray.uh == ray.uh) || !(ray.vh == ray.vh);
                const R pu = (nxt.uh - cx) + nxt.ul, pv = (nxt.vh - cy) + nxt.vl;
                const bool crossed = !bad && (pu * pu + pv * pv >= R2);
                const bool exhausted = !bad && !crossed && (ray.m + 1 >= A.max_steps);
                if (!(bad || crossed || exhausted)) {
                    add_T<R, COMP>(ray, w_start * so.ic1);
                    nxt.Th = ray.Th;
                    nxt.Tl = ray.Tl;
                    nxt.m = ray.m + 1;
                    if (nxt.m == m_ck && ck) {
                        ck[k_ck] = RayCkpt<R>{nxt.uh,  nxt.ul,  nxt.vh, nxt.vl, nxt.dxh, nxt.dxl,
                                              nxt.dyh, nxt.dyl, nxt.kx, nxt.ky, nxt.m};
                        k_ck++;
                        m_ck = k_ck < kSegs - 1 ? m_ck + stride_ck : -1;
                    }
                    ray = nxt;
                } else {
                    n_rays++;
                    int st = RTX_RAY_NO_HIT;
                    double g_mis = NAN, T = NAN, Lm = NAN;
                    if (bad) {
                        st = RTX_RAY_BAD_INPUT;
                    } else if (crossed) {
                        const Hit hit = intersect<R>(g, ray, nxt);
                        const double dsp = hit.t * g.ds;
                        const Sample<R> sq = lookup_at<R, COMP, BSP>(M, g, hit.qx, hit.qy);
                        if (!(sq.c > (R)0)) {
                            st = RTX_RAY_BAD_INPUT;
                        } else {
                            const double wm = ray.m == 0 ? 0.5 * dsp : 0.5 * (g.ds + dsp);
                            const double acc = ((double)ray.Th + (double)ray.Tl) + wm * (double)so.ic1 +
                                               0.5 * dsp * (double)rcp(sq.c);
                            T = acc * g.h;
                            Lm = (ray.m * g.ds + dsp) * g.h;
                            g_mis = mod2pi(atan2(hit.qy, hit.qx) - em.pe) - dr;
                            st = RTX_RAY_LINKED;
                        }
                    }
                    s_th[lane] = mine;
                    s_g[lane] = g_mis;
                    s_T[lane] = T;
                    s_L[lane] = Lm;
                    s_st[lane] = st;
                    waiting = true;
                }
            }
            compiler_fence();
            const unsigned long long wm = __ballot(waiting);
            ready = waiting && ((wm >> (lane & 62)) & 3ull) == 3ull;
        } while (!__any(ready));
        if (!ready) continue;
        // ---- both rays of the round are in (rare, divergent, FP64) ----
        waiting = false;
        double ca[2], ga[2], Ta[2], La[2];
        int sa[2];
        for (int q = 0; q < 2; q++) {
            ca[q] = s_th[b0 + q];
            ga[q] = s_g[b0 + q];
            Ta[q] = s_T[b0 + q];
            La[q] = s_L[b0 + q];
            sa[q] = s_st[b0 + q];
        }
        L.n_marches += 2;
        bool done = true;
        if (sa[0] == RTX_RAY_BAD_INPUT || sa[1] == RTX_RAY_BAD_INPUT) {
            if (j == 0) write_pair(A, p, L.th0, NAN, NAN, NAN, L.n_marches, RTX_RAY_BAD_INPUT);
            put_head(NAN, -1);
        } else {
            int lk = -1;
            double lmiss = INFINITY;
            for (int q = 0; q < 2; q++) {
                if (sa[q] != RTX_RAY_LINKED) continue;
                const double miss = fabs(ga[q]) * g.R;
                if (miss < L.best_miss) {
                    L.best_miss = miss;
                    L.best_th = ca[q];
                    L.best_T = Ta[q];
                    L.best_L = La[q];
                }
                if (miss <= A.tol && miss < lmiss) {
                    lk = q;
                    lmiss = miss;
                }
            }
            if (lk >= 0) {
                if (j == 0) write_pair(A, p, ca[lk], Ta[lk], La[lk], lmiss, L.n_marches, RTX_RAY_LINKED);
                put_head(ca[lk], lk);
            } else if (L.n_marches >= 2 * A.max_marches) {  // max_marches rounds
                put_head(NAN, -1);  // the best ray may be an earlier round's
                if (j == 0) {
                    if (L.best_miss < INFINITY)
                        write_pair(A, p, L.best_th, L.best_T, L.best_L, L.best_miss, L.n_marches,
                                   RTX_RAY_NOT_CONVERGED);
                    else
                        write_pair(A, p, L.th0, NAN, NAN, NAN, L.n_marches, RTX_RAY_NO_HIT);
                }
            } else {
                const bool h0 = sa[0] == RTX_RAY_LINKED, h1 = sa[1] == RTX_RAY_LINKED;
                if (h0) top4_push(t4, ca[0], ga[0]);
                if (h1) top4_push(t4, ca[1], ga[1]);
                double th;
                if (h0 && h1) {
                    const int f = fabs(ga[0]) >= fabs(ga[1]) ? 0 : 1;
                    L.th = ca[f];
                    link_next_hit(L, ga[f]);
                    L.th = ca[1 - f];
                    th = link_next_hit(L, ga[1 - f]);
                } else if (h0 || h1) {
                    const int q = h0 ? 0 : 1;
                    L.th = ca[q];
                    th = link_next_hit(L, ga[q]);
                } else {
                    th = L.nvalid > 0 ? 0.5 * (ca[0] + L.thb) : 0.5 * ca[0];
                }
                double v;
                if ((h0 || h1) && L.n_marches <= 4 && top4_estimate(t4, L, v)) th = v;
                L.th = th;
                round_start(th, false, 0.0);
                done = false;
            }
        }
        if (done) {
            p += stride;
            next_pair();
        }
    }
    block_sum2(n_steps, n_rays, A.stats);
}

// ---------------------------------------------------------- adjoint kernel --


// Pending hat weights of the current cell's four nodes: a[0] = (ix, iy),
// a[1] = (ix+1, iy), a[2] = (ix, iy+1), a[3] = (ix+1, iy+1).  Consecutive
// samples of a ray in one cell add into registers.  When the ray moves to an
// adjacent cell the accumulator shifts by a column and/or a row: the two nodes
// of the edge it leaves behind are emitted and the shared ones keep their sums
// (two node updates per edge crossing, three per corner crossing).  Node
// indices are 32-bit (grids stay below 2^24 cells).
template <class R>
struct CellAcc {
    int ix, iy;  // current cell; ix < 0: empty
    R a[4];
};

// Up to four node updates produced by one accumulator operation.
template <class R>
struct Emit {
    int n[4];
    R v[4];
    unsigned mask;  // bit k: entry k is valid
};

template <class R>
__device__ __forceinline__ void acc_flush(int nx, CellAcc<R> &A, Emit<R> &E)
{
    if (A.ix >= 0) {
        const int n0 = A.iy * nx + A.ix;
        E.n[0] = n0;
        E.n[1] = n0 + 1;
        E.n[2] = n0 + nx;
        E.n[3] = n0 + nx + 1;
        for (int k = 0; k < 4; k++) E.v[k] = A.a[k];
        E.mask = 0xfu;
    }
    A.ix = -1;
    A.a[0] = A.a[1] = A.a[2] = A.a[3] = (R)0;
}

template <class R>
__device__ __forceinline__ void acc_move(int nx, CellAcc<R> &A, int ix, int iy, Emit<R> &E)
{
    const int dx = ix - A.ix, dy = iy - A.iy;
    if (A.ix < 0 || dx < -1 || dx > 1 || dy < -1 || dy > 1) {
        acc_flush(nx, A, E);  // nothing on an empty accumulator
    } else {
        int n0 = A.iy * nx + A.ix;
        if (dx == 1) {  // leaves column ix_old behind
            E.n[0] = n0;
            E.v[0] = A.a[0];
            E.n[1] = n0 + nx;
            E.v[1] = A.a[2];
            E.mask |= 3u;
            A.a[0] = A.a[1];
            A.a[2] = A.a[3];
            A.a[1] = A.a[3] = (R)0;
        } else if (dx == -1) {  // leaves column ix_old + 1 behind
            E.n[0] = n0 + 1;
            E.v[0] = A.a[1];
            E.n[1] = n0 + nx + 1;
            E.v[1] = A.a[3];
            E.mask |= 3u;
            A.a[1] = A.a[0];
            A.a[3] = A.a[2];
            A.a[0] = A.a[2] = (R)0;
        }
        n0 = A.iy * nx + ix;  // the accumulator now holds cell (ix, iy_old)
        if (dy == 1) {
            E.n[2] = n0;
            E.v[2] = A.a[0];
            E.n[3] = n0 + 1;
            E.v[3] = A.a[1];
            E.mask |= 0xcu;
            A.a[0] = A.a[2];
            A.a[1] = A.a[3];
            A.a[2] = A.a[3] = (R)0;
        } else if (dy == -1) {
            E.n[2] = n0 + nx;
            E.v[2] = A.a[2];
            E.n[3] = n0 + nx + 1;
            E.v[3] = A.a[3];
            E.mask |= 0xcu;
            A.a[2] = A.a[0];
            A.a[3] = A.a[1];
            A.a[0] = A.a[1] = (R)0;
        }
    }
    A.ix = ix;
    A.iy = iy;
}

template <class R>
__device__ __forceinline__ void acc_add(int nx, CellAcc<R> &A, const Sample<R> &s, R a, Emit<R> &E)
{
    E.mask = 0;
    if (s.ix != A.ix || s.iy != A.iy) acc_move(nx, A, s.ix, s.iy, E);
    R omt = (R)1 - s.t, oms = (R)1 - s.s;
    A.a[0] = fma(a * omt, oms, A.a[0]);
    A.a[1] = fma(a * s.t, oms, A.a[1]);
    A.a[2] = fma(a * omt, s.s, A.a[2]);
    A.a[3] = fma(a * s.t, s.s, A.a[3]);
}

// Node updates travel from the marching lanes of a block to its last wave
// through one ring per lane in LDS; that wave alone issues the global float
// atomics.  (Vector memory operations of a wave complete in issue order, so
// atomics issued by a marching wave would hold up its next table loads.)  A
// ring has one writer, its lane, which stores entries and then publishes its
// head, and one reader, a lane of the last wave, which reads up to the head and
// then publishes its tail.  LDS operations of a wave take effect in program
// order, and compiler barriers keep that order in the code, so an entry is
// stored before its head is visible and read before its slot is reused.  Every
// wait is bounded: a bound that is hit sets the error word and the wait gives up.
constexpr int kFlushLanes = 64;
constexpr unsigned kQDone = 0x80000000u;
constexpr unsigned kQSpin = 1u << 26;

template <class R>
struct QEntry {
    unsigned node;  // node index; batches add the instance in the top 8 bits
    R val;
};

template <class R>
struct QRing {
    static constexpr int kLen = 16;  // entries per marching lane (32 / 64 KB per block)
};


template <class R>
__device__ __forceinline__ void q_push(QEntry<R> *ring, unsigned *qhead, unsigned *qtail, int lane, int nm,
                                       unsigned &head, unsigned &tailc, const Emit<R> &E, unsigned inst,
                                       unsigned *err)
{
    if (!E.mask) return;
    const unsigned k = __popc(E.mask);
    constexpr unsigned len = QRing<R>::kLen;
    if (head + k - tailc > len) {
        for (unsigned spins = 0;; spins++) {
            tailc = __hip_atomic_load(qtail + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (head + k - tailc <= len) break;
            if (spins > kQSpin) {
                atomicOr(err, 1u);
                return;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        compiler_fence();
    }
    for (int j = 0; j < 4; j++)
        if (E.mask & (1u << j)) {
            QEntry<R> &q = ring[(head & (len - 1)) * nm + lane];
            q.node = (unsigned)E.n[j] | inst;
            q.val = E.v[j];
            head++;
        }
    compiler_fence();
    __hip_atomic_store(qhead + lane, head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The drain wave merges node updates in a direct-mapped cache in LDS (its own;
// no other wave touches it) before they reach the grid: the rays of a block
// run side by side through one band of the grid, so an update usually finds
// its node in the cache, and the grid sees one float atomic per eviction and
// per cached node at the end instead of one per update (on the 256x256
// workload a 16 x 16 tile's ~140k updates touch 5k-11k nodes).  An update
// whose node holds its slot adds to it with an LDS atomic.  A missing node
// claims the slot: each such lane writes a tag (lane, ring) to the slot's
// claim word and reads it back, and the lane whose tag stayed adds the slot's
// old node to the grid and takes the slot; the others add to the grid
// directly.  LDS operations of the wave take effect in program order, so a
// read-back sees every lane's earlier write and every earlier LDS add.
template <class R>
struct NodeCache {
    static constexpr int kBits = sizeof(R) == 4 ? 13 : 12;  // 96 / 64 KB with the claim words
    static constexpr int kSlots = 1 << kBits;
};
constexpr unsigned kCacheEmpty = 0xffffffffu;  // node values stay below it (2^24 nodes, 255 instances)

__device__ __forceinline__ unsigned cache_slot(unsigned node, int bits)
{
    return (node * 0x9E3779B1u) >> (32 - bits);
}

template <class R, bool BATCH>
__device__ __forceinline__ void grid_add(R *grad, const BatchArgs &B, unsigned node, R v)
{
    R *g = grad;
    if (BATCH) {
        g = ((const Inst<R> *)B.inst)[node >> 24].grad;
        node &= 0xffffffu;
    }
    unsafeAtomicAdd(g + node, v);
}

// The last wave of a block drains the rings of marching lanes lane, lane + 64,
// ... (one entry per ring and pass) through the cache until every ring is
// marked done and empty, then adds the cached nodes to the grid.
template <class R, bool BATCH>
__device__ __forceinline__ void q_drain(const QEntry<R> *ring, const unsigned *qhead, unsigned *qtail, int nm,
                                        R *grad, const BatchArgs &B, unsigned *err, unsigned *c_claim,
                                        unsigned *c_key, R *c_val)
{
    constexpr unsigned len = QRing<R>::kLen;
    constexpr int NJ = kBlock / 64;
    constexpr int kBits = NodeCache<R>::kBits;
    const int lane = threadIdx.x - nm;
    for (int i = lane; i < NodeCache<R>::kSlots; i += 64) c_key[i] = kCacheEmpty;
    unsigned tl[NJ] = {};
    for (unsigned idle = 0;;) {
        bool done = true, moved = false;
        unsigned h[NJ];
        for (int j = 0; j < NJ; j++)
            h[j] = j * 64 < nm ? __hip_atomic_load(qhead + lane + 64 * j, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP)
                               : kQDone;
        compiler_fence();
        QEntry<R> q[NJ];
        bool have[NJ];
        for (int j = 0; j < NJ; j++) {
            have[j] = tl[j] != (h[j] & ~kQDone);
            // (read for every ring of this block, in bounds: (len - 1) nm + pl < len kBlock)
            if (j * 64 < nm) q[j] = ring[(tl[j] & (len - 1)) * nm + lane + 64 * j];
        }
        for (int j = 0; j < NJ; j++)
            if (have[j]) {
                tl[j]++;
                moved = true;
            }
        compiler_fence();
        for (int j = 0; j < NJ; j++) {
            if (j * 64 < nm)
                __hip_atomic_store(qtail + lane + 64 * j, tl[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            done = done && (h[j] & kQDone) && tl[j] == (h[j] & ~kQDone);
        }
        // (plain LDS accesses between compiler barriers, which make the compiler
        // re-read what other lanes may have written; loads are issued for every
        // j, unused ones at slot 0, so that each phase's loads go out together)
        unsigned slot[NJ], key[NJ];
        for (int j = 0; j < NJ; j++) slot[j] = have[j] ? cache_slot(q[j].node, kBits) : 0u;
        for (int j = 0; j < NJ; j++) key[j] = c_key[slot[j]];
        // hits add in LDS (atomically: lanes of one instruction may share a node)
        bool miss[NJ];
        for (int j = 0; j < NJ; j++) {
            miss[j] = have[j] && key[j] != q[j].node;
            if (have[j] && !miss[j]) atomicAdd(c_val + slot[j], q[j].val);
            if (miss[j]) c_claim[slot[j]] = (unsigned)(lane * NJ + j);
        }
        compiler_fence();
        unsigned tag[NJ];
        R old[NJ];
        for (int j = 0; j < NJ; j++) {
            tag[j] = c_claim[slot[j]];
            old[j] = c_val[slot[j]];
        }
        compiler_fence();
        // a miss whose claim stayed evicts the slot's node and takes the slot;
        // the other misses go to the grid
        for (int j = 0; j < NJ; j++) {
            if (!miss[j]) continue;
            if (tag[j] == (unsigned)(lane * NJ + j)) {
                if (key[j] != kCacheEmpty) grid_add<R, BATCH>(grad, B, key[j], old[j]);
                c_key[slot[j]] = q[j].node;
                c_val[slot[j]] = q[j].val;
            } else {
                grid_add<R, BATCH>(grad, B, q[j].node, q[j].val);
            }
        }
        compiler_fence();
        if (__all(done)) break;
        if (!__any(moved)) {
            if (++idle > kQSpin) {
                atomicOr(err, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    for (int i = lane; i < NodeCache<R>::kSlots; i += 64) {
        const unsigned k = c_key[i];
        if (k != kCacheEmpty) grid_add<R, BATCH>(grad, B, k, c_val[i]);
    }
}

// Per-ray constants of an adjoint march: step, ring radius squared and ring
// centre (pixels), and the ray's factor rho h.
template <class R>
struct AdjRay {
    R ds, R2, cx, cy, scale;
};

template <class R>
__device__ __forceinline__ AdjRay<R> adj_ray_of(const Geo &g)
{
    return AdjRay<R>{(R)g.ds, (R)(g.R * g.R), (R)g.cx, (R)g.cy, (R)0};
}

// One step of an adjoint ray (the transpose of the path weights of Sec. 3.5):
// the trapezoid weight of the step's start sample, times the ray's factor, goes
// to the cell accumulator, whose outputs are handed to `sink`; on the step that
// leaves the ring, the shortened last step and the interception point instead.
// Returns false once the ray has ended (left the ring, met a bad sample or used
// max_steps) or reached step stop_m (a first half), with the accumulator flushed.
template <class R, bool COMP, int INTEG, class Sink>
__device__ __forceinline__ bool adj_step(const Medium<R> &m, const Geo &gg, const AdjArgs &a, const AdjRay<R> &kr,
                                         Ray<R> &ray, Slot<R> (&C)[3], CellAcc<R> &acc, Emit<R> &E, Sink &sink,
                                         int stop_m)
{
    Ray<R> nxt;
    StepOut<R> so = ray_step<R, COMP, INTEG>(m, C, ray, nxt, kr.ds);
    const R kap = a.weight == RTX_W_DTDC ? -so.ic1 * so.ic1 : (R)1;
    const bool bad = !(so.s1.c > (R)0) || !(ray.uh == ray.uh) || !(ray.vh == ray.vh);
    R pu = (nxt.uh - kr.cx) + nxt.ul, pv = (nxt.vh - kr.cy) + nxt.vl;
    const bool crossed = !bad && (pu * pu + pv * pv >= kr.R2);
    const bool exhausted = !bad && !crossed && (ray.m + 1 >= a.max_steps);
    if (!(bad || crossed || exhausted)) {
        const R w = ray.m == 0 ? kr.ds * (R)0.5 : kr.ds;
        acc_add(m.nx, acc, so.s1, kr.scale * w * kap, E);
        sink();
        nxt.m = ray.m + 1;
        ray = nxt;
        if (ray.m < stop_m) return true;
        // a first half ends before the sample the second half starts with
        E.mask = 0;
        acc_flush(m.nx, acc, E);
        sink();
        return false;
    }
    if (crossed) {
        Hit hit = intersect<R>(gg, ray, nxt);
        double dsp = hit.t * gg.ds;
        Sample<R> sq = lookup_at<R, COMP>(m, gg, hit.qx, hit.qy);
        if (sq.c > (R)0) {
            R wm = (R)(ray.m == 0 ? 0.5 * dsp : 0.5 * (gg.ds + dsp));
            acc_add(m.nx, acc, so.s1, kr.scale * wm * kap, E);
            sink();
            R icq = rcp(sq.c);
            R kq = a.weight == RTX_W_DTDC ? -icq * icq : (R)1;
            acc_add(m.nx, acc, sq, kr.scale * (R)(0.5 * dsp) * kq, E);
            sink();
        }
    }
    E.mask = 0;
    acc_flush(m.nx, acc, E);
    sink();
    return false;
}

// Marching lanes are threads 0 .. nm-1 (nm = blockDim.x - 64); the last wave
// drains their node updates into the grid.
template <class R, bool COMP, int INTEG, bool BATCH, bool SPLIT = false>
__global__ void __launch_bounds__(kBlock + kFlushLanes) k_adjoint(Medium<R> M, Geo g, AdjArgs A, R *grad,
                                                                   BatchArgs B)
{
    // SPLIT (A.split, all pairs only): the segments of the rays as work items
    constexpr bool kSplit = SPLIT && !BATCH;
    // block b adds into copy b mod n_copies of the gradient (AdjArgs::n_copies)
    if (!BATCH) grad += (size_t)(blockIdx.x % A.n_copies) * M.nx * M.ny;
    __shared__ QEntry<R> q_ring[QRing<R>::kLen * kBlock];
    __shared__ unsigned q_head[kBlock], q_tail[kBlock];
    __shared__ unsigned c_claim[NodeCache<R>::kSlots], c_key[NodeCache<R>::kSlots];
    __shared__ R c_val[NodeCache<R>::kSlots];
    const int nm = (int)blockDim.x - kFlushLanes;
    for (int i = threadIdx.x; i < nm; i += blockDim.x) q_head[i] = q_tail[i] = 0;
    __syncthreads();
    if ((int)threadIdx.x >= nm) {
        q_drain<R, BATCH>(q_ring, q_head, q_tail, nm, grad, B, A.err, c_claim, c_key, c_val);
        block_sum2(0ull, 0ull, A.stats);
        return;
    }
    const int lane = threadIdx.x;
    unsigned qh = 0, qt = 0;
    const int64_t stride = (int64_t)gridDim.x * nm;
    int64_t p = (int64_t)blockIdx.x * nm + lane;
    int64_t n_items = BATCH ? B.off[B.n_inst] : kSplit ? kSegs * A.n_items : A.n_items;
    int64_t q = p;
    int k = 0;
    Medium<R> m = M;
    Geo gg = g;
    AdjArgs a = A;
    AdjRay<R> kr = adj_ray_of<R>(gg);
    unsigned long long n_steps = 0, n_rays = 0;
    Ray<R> ray;
    Slot<R> C[3];
    CellAcc<R> acc;
    acc.ix = acc.iy = -1;
    acc.a[0] = acc.a[1] = acc.a[2] = acc.a[3] = (R)0;
    Emit<R> E;
    E.mask = 0;
    int stop_m = INT_MAX;  // a segment's end
    bool active = false;
    auto push = [&]() { q_push(q_ring, q_head, q_tail, lane, nm, qh, qt, E, BATCH ? (unsigned)k << 24 : 0u, A.err); };

    auto next_pair = [&]() {
        while (p < n_items) {
            if (BATCH) {
                k = find_inst(B, p);
                const Inst<R> &I = ((const Inst<R> *)B.inst)[k];
                m = I.M;
                gg = I.g;
                a = I.J;
                q = p - B.off[k];
                kr = adj_ray_of<R>(gg);
            }
            int e, r;
            // split: items 64 (kSegs w + sg) + t are segment sg of tile item
            // 64 w + t, so a wave's lanes take the same segment of 64
            // neighbouring rays
            const int sg = kSplit ? (int)((p >> 6) % kSegs) : 0;
            const int64_t it = kSplit ? ((p >> 6) / kSegs << 6) | (p & 63) : p;
            bool ok = BATCH ? pair_of(TraceArgs{a.pairs}, gg, q, e, r) : adj_item(a, gg, it, e, r, q);
            ok = ok && (a.status[q] == RTX_RAY_LINKED || a.status[q] == RTX_RAY_NOT_CONVERGED);
            double rho = ok ? a.rho[q] : 0.0;
            RayCkpt<R> ckv;  // the segment's start (sg > 0)
            ckv.m = -1;
            int seg_end = INT_MAX;
            if (kSplit && ok && rho != 0.0) {
                const CkptHead hd = a.ckpt_head[q];
                const RayCkpt<R> *cks = (const RayCkpt<R> *)a.ckpt + (2 * q + max(hd.lane, 0)) * (kSegs - 1);
                // the last checkpoint exists only if the ray wrote all of them
                const bool have = hd.lane >= 0 && hd.gen == a.gen && hd.theta == a.theta[q] &&
                                  cks[kSegs - 2].m > 0;
                if (have) {
                    if (sg > 0) ckv = cks[sg - 1];
                    if (sg < kSegs - 1) seg_end = cks[sg].m;
                } else if (sg > 0) {
                    ok = false;  // no checkpoints: the first segment takes the whole ray
                }
            }
            if (ok && rho != 0.0) {
                stop_m = seg_end;
                if (sg == 0) {
                    start_ray<R, COMP>(ray, gg, emitter_of(gg, e), a.theta[q]);
                } else {
                    ray.uh = ckv.uh;
                    ray.ul = ckv.ul;
                    ray.vh = ckv.vh;
                    ray.vl = ckv.vl;
                    ray.dxh = ckv.dxh;
                    ray.dxl = ckv.dxl;
                    ray.dyh = ckv.dyh;
                    ray.dyl = ckv.dyl;
                    ray.kx = ckv.kx;
                    ray.ky = ckv.ky;
                    ray.Th = ray.Tl = (R)0;
                    ray.m = ckv.m;
                }
                slots_prime(m, C, ray, kr.ds, INTEG);
                kr.scale = (R)(rho * gg.h);
                active = true;
                return;
            }
            if (BATCH) mark_done(B, k);
            p += stride;
        }
        active = false;
    };
    next_pair();

    while (active) {
        n_steps++;
        if (adj_step<R, COMP, INTEG>(m, gg, a, kr, ray, C, acc, E, push, stop_m)) continue;
        n_rays++;
        if (BATCH) mark_done(B, k);
        p += stride;
        next_pair();
    }
    compiler_fence();
    __hip_atomic_store(q_head + lane, qh | kQDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    block_sum2(n_steps, n_rays, A.stats);
}

// Sum of the gradient copies into grad; the copies are left zeroed for the next
// adjoint.
template <class R>
__global__ void __launch_bounds__(kBlock) k_copies_sum(R *__restrict__ cp, int n_copies, int64_t nn,
                                                       R *__restrict__ grad)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= nn) return;
    R sum = (R)0;
    for (int k = 0; k < n_copies; k++) {
        sum += cp[k * nn + i];
        cp[k * nn + i] = (R)0;
    }
    grad[i] += sum;
}

// Start of a batch run: per-instance pair counters and the start timestamp.
__global__ void k_batch_reset(const int64_t *__restrict__ off, int n_inst, unsigned int *remain_fwd,
                              unsigned int *remain_adj, unsigned long long *t0)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_inst) {
        unsigned int n = (unsigned int)(off[k + 1] - off[k]);
        remain_fwd[k] = n;
        remain_adj[k] = n;
    }
    if (k == 0) *t0 = wall_clock64();
}

// One block per emitter e (all ordered pairs in canonical order): samples
// G_j = H_j - D_r of the straight rays at offsets j = 1..n-1 with
// H_j = g_j + D_j; each receiver takes the sign change over consecutive samples
// nearest to its own offset, searched outward (own, own+1, own-1-1, ...).  With
// both outer neighbours of the bracket sampled and G strictly monotone over the
// four samples, the first linking angle is the zero of the cubic interpolating
// theta as a function of G through them (inverse Lagrange interpolation), if it
// falls strictly inside the bracket; else the secant's linear interpolation.
__device__ __forceinline__ double fan_straight(const Geo &g, int e, int j)
{
    int k = (e + j) % g.n_elem;
    return (mod2pi(elem_angle(g, k) - elem_angle(g, e)) - kPi) / 2.0;
}

// Zero of the polynomial interpolating theta as a function of G = H - Dr through
// the 2 HW fan samples around the bracket (found, found + 1): HW = 2 gives the
// cubic first angle, HW = 3 the quintic second angle of the first round.  All
// samples must exist, hit, be strictly monotone in G, and the zero must lie
// strictly inside the bracket.
template <int HW>
__device__ __forceinline__ bool fan_inverse(const Geo &g, int e, const double *H, double Dr, int n, int found,
                                            double &th)
{
    constexpr int NP = 2 * HW;
    const int lo_i = found - (HW - 1);
    if (lo_i < 0 || found + HW > n - 2) return false;
    double gg[NP], tt[NP];
    bool ok = true;
    for (int q = 0; q < NP; q++) {
        gg[q] = H[lo_i + q] - Dr;
        tt[q] = fan_straight(g, e, lo_i + q + 1);  // the sample at index a is the ray at offset a + 1
        ok = ok && gg[q] == gg[q];
    }
    const bool up = gg[1] > gg[0];
    for (int q = 0; q < NP - 1; q++) ok = ok && (up ? gg[q + 1] > gg[q] : gg[q + 1] < gg[q]);
    if (!ok) return false;
    double v = 0.0;
    for (int q = 0; q < NP; q++) {
        double w = 1.0;
        for (int m = 0; m < NP; m++)
            if (m != q) w *= (0.0 - gg[m]) / (gg[q] - gg[m]);
        v += w * tt[q];
    }
    const double lo = fmin(tt[HW - 1], tt[HW]), hi = fmax(tt[HW - 1], tt[HW]);
    if (!(v > lo && v < hi)) return false;
    th = v;
    return true;
}

__global__ void __launch_bounds__(kBlock) k_fan_seed(Geo g, const double *__restrict__ f_g,
                                                     const int8_t *__restrict__ f_st, FanSeed *__restrict__ seed)
{
    extern __shared__ double H[];  // [n-1] hit angle of the ray at offset j (NaN: no hit)
    const int n = g.n_elem, e = blockIdx.x;
    const double pe = elem_angle(g, e);
    for (int j = 1 + threadIdx.x; j < n; j += blockDim.x) {
        int k = (e + j) % n;
        int64_t i = (int64_t)e * (n - 1) + (k < e ? k : k - 1);
        double Dj = mod2pi(elem_angle(g, k) - pe);
        H[j - 1] = f_st[i] == RTX_RAY_LINKED ? f_g[i] + Dj : NAN;
    }
    __syncthreads();
    for (int jr = 1 + threadIdx.x; jr < n; jr += blockDim.x) {
        int r = (e + jr) % n;
        int64_t i = (int64_t)e * (n - 1) + (r < e ? r : r - 1);
        double Dr = mod2pi(elem_angle(g, r) - pe);
        int found = -1;
        for (int d = 0; d < n && found < 0; d++) {
            int cand[2] = {jr - 1 + d, jr - 1 - d - 1};
            for (int c = 0; c < 2; c++) {
                int a = cand[c];
                if (a < 0 || a + 1 > n - 2) continue;
                double ga = H[a] - Dr, gb = H[a + 1] - Dr;
                if (ga == ga && gb == gb && ga * gb <= 0.0) {
                    found = a;
                    break;
                }
            }
        }
        FanSeed sd;
        sd.found = found >= 0;
        sd.th_far = sd.g_far = sd.th_near = sd.g_near = sd.th_first = sd.th_q = 0.0;
        sd.cubic = found >= 0 && fan_inverse<2>(g, e, H, Dr, n, found, sd.th_first);
        sd.quintic = found >= 0 && fan_inverse<3>(g, e, H, Dr, n, found, sd.th_q);
        // the samples that hit, packed in order (unrolled, so that the record
        // stays in registers)
        sd.n_s = 0;
        for (int q = 0; q < 4; q++) sd.s_th[q] = sd.s_g[q] = 0.0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int a = found - 1 + u;
            const bool use = found >= 0 && a >= 0 && a <= n - 2 && H[a] - Dr == H[a] - Dr;
            const double ga = use ? H[a] - Dr : 0.0, ta = use ? fan_straight(g, e, a + 1) : 0.0;
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (use && q == sd.n_s) {
                    sd.s_th[q] = ta;
                    sd.s_g[q] = ga;
                }
            sd.n_s += use;
        }
        if (found >= 0) {
            double ga = H[found] - Dr, gb = H[found + 1] - Dr;
            int nr = fabs(ga) <= fabs(gb) ? found : found + 1;
            int fr = nr == found ? found + 1 : found;
            double gn = nr == found ? ga : gb, gf = nr == found ? gb : ga;
            int kn = (e + nr + 1) % n, kf = (e + fr + 1) % n;
            sd.th_near = (mod2pi(elem_angle(g, kn) - pe) - kPi) / 2.0;
            sd.th_far = (mod2pi(elem_angle(g, kf) - pe) - kPi) / 2.0;
            sd.g_near = gn;
            sd.g_far = gf;
        }
        seed[i] = sd;
    }
}

// ------------------------------------------------------------ path weights --
// Row i of the system matrix, W_ij = h sum_m w_m phi_j(p_m), is emitted in three
// passes: count cell visits (4 entries each), fill the entries of every visit
// into the row's segment of a scratch buffer, then sort + merge each row in LDS.
struct WArgs {
    const int32_t *pairs;
    int64_t n_pairs;
    const double *theta;
    const int8_t *status;
    int max_steps;
    int64_t *rawcnt;        // count pass: entries per row
    const int64_t *rawoff;  // fill pass: row offsets into cols/vals
    int32_t *cols;
    void *vals;
};

template <class R, bool FILL>
struct RowSink {
    int32_t n0;  // node index of the visited cell's lower-left corner, -1 = none
    R a00, a10, a01, a11;
    int64_t at, end;  // fill cursor and end of the row's segment
    int64_t count;
    int32_t *cols;
    R *vals;
    int nx;

    __device__ __forceinline__ void put(int32_t c, R v)
    {
        if (at < end) {
            cols[at] = c;
            vals[at] = v;
        }
        at++;
    }
    __device__ __forceinline__ void emit(int32_t c, R v)
    {
        if (FILL) put(c, v);
        count++;
    }
    // writes the sums of the cell's four corners (the end of a row)
    __device__ __forceinline__ void flush()
    {
        if (n0 >= 0) {
            emit(n0, a00);
            emit(n0 + 1, a10);
            emit(n0 + nx, a01);
            emit(n0 + nx + 1, a11);
        }
        n0 = -1;
        a00 = a10 = a01 = a11 = (R)0;
    }
    // the ray moves on to cell c: the two corners that c shares with the cell
    // when they are edge neighbours carry their sums over, the others are
    // written (a row then holds about two entries per cell instead of four)
    __device__ __forceinline__ void move_to(int32_t c)
    {
        // the four edge moves by selects, not branches: the lanes of a wave
        // move in different directions
        const bool px = c == n0 + 1, mx = c == n0 - 1, py = c == n0 + nx, my = c == n0 - nx;
        if (n0 >= 0 && (px || mx || py || my)) {
            emit(px || py ? n0 : mx ? n0 + 1 : n0 + nx, px || py ? a00 : mx ? a10 : a01);
            emit(px ? n0 + nx : py ? n0 + 1 : n0 + nx + 1, px ? a01 : py ? a10 : a11);
            const R b00 = px ? a10 : py ? a01 : (R)0, b10 = mx ? a00 : py ? a11 : (R)0;
            const R b01 = px ? a11 : my ? a00 : (R)0, b11 = mx ? a01 : my ? a10 : (R)0;
            a00 = b00, a10 = b10, a01 = b01, a11 = b11;
            n0 = c;
            return;
        }
        flush();
        n0 = c;
    }
    __device__ __forceinline__ void add(const Sample<R> &s, R a)
    {
        int32_t c = s.iy * nx + s.ix;
        if (c != n0) move_to(c);
        R omt = (R)1 - s.t, oms = (R)1 - s.s;
        a00 = fma(a * omt, oms, a00);
        a10 = fma(a * s.t, oms, a10);
        a01 = fma(a * omt, s.s, a01);
        a11 = fma(a * s.t, s.s, a11);
    }
};

template <class R, bool COMP, int INTEG, bool FILL>
__global__ void __launch_bounds__(kBlock) k_weights(Medium<R> M, Geo g, WArgs A)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const R ds = (R)g.ds;
    const R R2 = (R)(g.R * g.R);
    const R cx = (R)g.cx, cy = (R)g.cy;
    const R hh = (R)g.h;
    Ray<R> ray;
    Slot<R> C[3];
    RowSink<R, FILL> sink;
    sink.cols = A.cols;
    sink.vals = (R *)A.vals;
    sink.nx = M.nx;
    bool active = false;
    TraceArgs pa;
    pa.pairs = A.pairs;

    auto begin_row = [&]() {
        sink.n0 = -1;
        sink.a00 = sink.a10 = sink.a01 = sink.a11 = (R)0;
        sink.count = 0;
        if (FILL) {
            sink.at = A.rawoff[p];
            sink.end = A.rawoff[p] + A.rawcnt[p];
        }
    };
    auto end_row = [&]() {
        sink.flush();
        if (!FILL) A.rawcnt[p] = sink.count;
    };
    auto next_pair = [&]() {
        while (p < A.n_pairs) {
            int e, r;
            bool ok = pair_of(pa, g, p, e, r);
            ok = ok && (A.status[p] == RTX_RAY_LINKED || A.status[p] == RTX_RAY_NOT_CONVERGED);
            begin_row();
            if (ok) {
                start_ray<R, COMP>(ray, g, emitter_of(g, e), A.theta[p]);
                slots_prime(M, C, ray, ds, INTEG);
                active = true;
                return;
            }
            end_row();
            p += stride;
        }
        active = false;
    };
    next_pair();

    while (active) {
        Ray<R> nxt;
        StepOut<R> so = ray_step<R, COMP, INTEG>(M, C, ray, nxt, ds);
        const bool bad = !(so.s1.c > (R)0) || !(ray.uh == ray.uh) || !(ray.vh == ray.vh);
        R pu = (nxt.uh - cx) + nxt.ul, pv = (nxt.vh - cy) + nxt.vl;
        const bool crossed = !bad && (pu * pu + pv * pv >= R2);
        const bool exhausted = !bad && !crossed && (ray.m + 1 >= A.max_steps);
        if (!(bad || crossed || exhausted)) {
            sink.add(so.s1, hh * (ray.m == 0 ? ds * (R)0.5 : ds));
            nxt.m = ray.m + 1;
            ray = nxt;
            continue;
        }
        if (crossed) {
            Hit hit = intersect<R>(g, ray, nxt);
            double dsp = hit.t * g.ds;
            Sample<R> sq = lookup_at<R, COMP>(M, g, hit.qx, hit.qy);
            if (sq.c > (R)0) {
                sink.add(so.s1, (R)(g.h * (ray.m == 0 ? 0.5 * dsp : 0.5 * (g.ds + dsp))));
                sink.add(sq, (R)(g.h * 0.5 * dsp));
            }
        }
        end_row();
        p += stride;
        next_pair();
    }
}

// One block per row: the row's entries are sorted by node index in LDS
// (bitonic), equal nodes are summed, zero sums dropped, and the merged row is
// written back to the start of its segment; ucnt[row] = merged length.
template <class R>
__global__ void __launch_bounds__(kBlock) k_wmerge(const int64_t *__restrict__ rawoff,
                                                   const int64_t *__restrict__ rawcnt, int32_t *cols, R *vals,
                                                   int64_t *__restrict__ ucnt, int cap)
{
    extern __shared__ __align__(16) unsigned char smem[];
    R *val = (R *)smem;
    int32_t *key = (int32_t *)(smem + (size_t)cap * sizeof(R));
    __shared__ int part[kBlock];
    const int64_t row = blockIdx.x;
    const int n = (int)rawcnt[row];
    const int64_t off = rawoff[row];
    const int tid = threadIdx.x;
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = tid; i < np; i += blockDim.x) {
        key[i] = i < n ? cols[off + i] : 0x7fffffff;
        val[i] = i < n ? vals[off + i] : (R)0;
    }
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            // every thread takes whole compare-exchange pairs (i, i + j): t's
            // bits with a zero inserted at j's position give the lower index i
            for (int t = tid; t < (np >> 1); t += blockDim.x) {
                const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1)), q = i | j;
                const bool up = (i & k) == 0;
                const int32_t a = key[i], b = key[q];
                if ((a > b) == up) {
                    key[i] = b;
                    key[q] = a;
                    const R x = val[i];
                    val[i] = val[q];
                    val[q] = x;
                }
            }
            __syncthreads();
        }
    }
    // each thread owns a contiguous chunk; a head sums its run (which may run
    // into the next chunk) and is kept if the sum is not zero
    const int chunk = (np + blockDim.x - 1) / blockDim.x;
    const int lo = tid * chunk, hi = min(n, lo + chunk);
    int kept = 0;
    for (int i = lo; i < hi; i++) {
        if (i > 0 && key[i] == key[i - 1]) continue;
        R sum = val[i];
        for (int j = i + 1; j < n && key[j] == key[i]; j++) sum += val[j];
        val[i] = sum;
        kept += sum != (R)0;
    }
    part[tid] = kept;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
        int v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int pos = part[tid] - kept;
    for (int i = lo; i < hi; i++) {
        if (i > 0 && key[i] == key[i - 1]) continue;
        if (val[i] != (R)0) {
            cols[off + pos] = key[i];
            vals[off + pos] = val[i];
            pos++;
        }
    }
    if (tid == blockDim.x - 1) ucnt[row] = part[tid];
}

// Copies each merged row to its place in the caller's CSR arrays.
template <class R>
__global__ void __launch_bounds__(kBlock) k_wcompact(const int64_t *__restrict__ rawoff,
                                                     const int64_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ cols, const R *__restrict__ vals,
                                                     int32_t *__restrict__ w_col, R *__restrict__ w_val)
{
    const int64_t row = blockIdx.x;
    const int64_t src = rawoff[row], dst = rowptr[row], n = rowptr[row + 1] - rowptr[row];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        w_col[dst + i] = cols[src + i];
        w_val[dst + i] = vals[src + i];
    }
}

// Per pair: rho_i = sum_k w_k Im(exp(-i w_k T_i) r_ik), one wave per pair, lanes
// over frequencies (coalesced 8-byte complex64 loads), phase reduced in FP64.
__global__ void __launch_bounds__(kBlock) k_rayborn_rho(int64_t n, int n_freq, const double *__restrict__ T,
                                                         const double *__restrict__ omega,
                                                         const float2 *__restrict__ resid, double *__restrict__ rho)
{
    int lane = threadIdx.x & 63;
    int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= n) return;
    double Ti = T[i], acc = 0.0;
    for (int k = lane; k < n_freq; k += 64) {
        double w = omega[k];
        double ph = fmod(w * Ti, kTwoPi);
        double sp, cp;
        sincos(ph, &sp, &cp);
        float2 rr = resid[i * n_freq + k];
        acc += w * ((double)rr.y * cp - (double)rr.x * sp);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) rho[i] = acc;
}

// Free march without a ring (the ray equations of Sec. 3.2 followed for a fixed
// number of steps, as in the radius experiment of Sec. 4.1).  One lane per ray:
// ray i starts at x0[i] (metres from the grid centre) along d0[i] (normalised
// here) and takes n_steps steps; the start and every step's end point are
// written to pts[i] in metres.  From the first point outside the node
// rectangle on (or for a zero or non-finite direction) the points are NaN and
// the ray stops.
template <class R, bool COMP, int INTEG, bool BSP>
__global__ void __launch_bounds__(kBlock)
    k_march(Medium<R> M, Geo g, int64_t n_rays, const double *__restrict__ x0, const double *__restrict__ d0,
            int n_steps, double *__restrict__ pts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_rays) return;
    const double ddx = d0[2 * i], ddy = d0[2 * i + 1];
    const double nrm = sqrt(ddx * ddx + ddy * ddy);
    Ray<R> ray;
    ray_set<R, COMP>(ray, x0[2 * i] / g.h + g.cx, x0[2 * i + 1] / g.h + g.cy, ddx / nrm, ddy / nrm);
    const R ds = (R)g.ds;
    Slot<R> C[3];
    if (!BSP) slots_prime(M, C, ray, ds, INTEG);
    double *o = pts + (size_t)i * (size_t)(n_steps + 1) * 2;
    bool out = false;
    for (int k = 0; k <= n_steps; k++) {
        if (k > 0 && !out) {
            Ray<R> nxt;
            (void)ray_step<R, COMP, INTEG, BSP>(M, C, ray, nxt, ds);
            ray = nxt;
        }
        const double u = (double)ray.uh + (double)ray.ul, v = (double)ray.vh + (double)ray.vl;
        const double dl = (double)ray.dxh + (double)ray.dxl;
        out = out || !(u >= 0.0 && u <= g.nx - 1.0 && v >= 0.0 && v <= g.ny - 1.0 && dl == dl);
        o[2 * k] = out ? (double)NAN : (u - g.cx) * g.h;
        o[2 * k + 1] = out ? (double)NAN : (v - g.cy) * g.h;
    }
}

// ----------------------------------------------------------- paraxial ray --
// The paraxial ray of Sec. 3.5 (the default way to the ray Jacobian): the
// first-order perturbation (q, p) = (dx, dd) of a ray's position and direction
// caused by a perturbation of its launch angle, from the variational equations
// of the ray ODE x' = d, d' = K(x, d) = -(G - (G.d) d) / c:
//   q' = p,   p' = dK = (((H q).d + G.p) d - H q + (G.d) p) / c - K (grad c . q) / c,
// with grad c the gradient of the interpolated c and H = dG/dx the derivative
// of the interpolated G.  The reference ray is advanced by the tracer's own
// stage arithmetic (so it is the traced ray), the perturbation by the same
// Runge-Kutta stages on the tangent-linear system, and the renormalisation of
// d is linearised.  One lane per ray, direct lookups.
template <class R>
struct SampleP {
    Sample<R> b;              // c, G and the cell, as the tracer sees them
    R cx, cy;                 // gradient of the interpolated c
    R hxx, hxy, hyx, hyy;     // dG_x/dx, dG_x/dy, dG_y/dx, dG_y/dy
};

template <class R>
__device__ __forceinline__ SampleP<R> lookup_para(const Medium<R> &M, R uh, R du, R vh, R dv)
{
    SampleP<R> o;
    o.b.ix = min(max((int)(uh + du), 0), M.nx - 2);
    o.b.iy = min(max((int)(vh + dv), 0), M.ny - 2);
    o.b.t = fmin_(fmax_((uh - (R)o.b.ix) + du, (R)0), (R)1);
    o.b.s = fmin_(fmax_((vh - (R)o.b.iy) + dv, (R)0), (R)1);
    R v[12];
    load_cell(M.tab, __umul24((uint32_t)o.b.iy, (uint32_t)(M.nx - 1)) + (uint32_t)o.b.ix, v);
    interp(v, o.b.t, o.b.s, o.b);
    const R t = o.b.t, s = o.b.s;  // f = a + b t + c s + d t s per field
    o.cx = fma(s, v[3], v[1]);
    o.cy = fma(t, v[3], v[2]);
    o.hxx = fma(s, v[7], v[5]);
    o.hxy = fma(t, v[7], v[6]);
    o.hyx = fma(s, v[11], v[9]);
    o.hyy = fma(t, v[11], v[10]);
    return o;
}

template <class R>
__device__ __forceinline__ SampleP<R> lookup_para_bsp(const Medium<R> &M, R uh, R du, R vh, R dv)
{
    SampleP<R> o;
    o.b = lookup_bsp(M, uh, du, vh, dv);
    R q[16], wx[4], dwx[4], wy[4], dwy[4];
    load_stencil(M.tab, __umul24((uint32_t)o.b.iy, (uint32_t)(M.nx - 1)) + (uint32_t)o.b.ix, q);
    bsp_weights(o.b.t, wx, dwx);
    bsp_weights(o.b.s, wy, dwy);
    const R t = o.b.t, s = o.b.s;  // second derivatives of the cubic's weights
    const R ddx[4] = {(R)1 - t, fma((R)3, t, (R)-2), fma((R)-3, t, (R)1), t};
    const R ddy[4] = {(R)1 - s, fma((R)3, s, (R)-2), fma((R)-3, s, (R)1), s};
    R cxx = 0, cxy = 0, cyy = 0;
    for (int b = 0; b < 4; b++) {
        R rxx = 0, rx = 0, r = 0;
        for (int a = 0; a < 4; a++) {
            rxx = fma(q[4 * b + a], ddx[a], rxx);
            rx = fma(q[4 * b + a], dwx[a], rx);
            r = fma(q[4 * b + a], wx[a], r);
        }
        cxx = fma(rxx, wy[b], cxx);
        cxy = fma(rx, dwy[b], cxy);
        cyy = fma(r, ddy[b], cyy);
    }
    o.cx = o.b.gx;
    o.cy = o.b.gy;
    o.hxx = cxx;
    o.hxy = o.hyx = cxy;
    o.hyy = cyy;
    return o;
}

// Records the extended sample of every stage for the tangent-linear pass.
template <class R, bool BSP>
struct ParaSampler {
    const Medium<R> &M;
    R uh, vh;
    SampleP<R> s[4];
    __device__ __forceinline__ Sample<R> get(int k, R du, R dv)
    {
        s[k] = BSP ? lookup_para_bsp(M, uh, du, vh, dv) : lookup_para(M, uh, du, vh, dv);
        return s[k].b;
    }
    __device__ __forceinline__ void done(int) {}
};

// dK at a stage with direction d and curvature k, perturbation (q, p).
template <class R>
__device__ __forceinline__ void dcurv(const SampleP<R> &S, R ic, R dx, R dy, R kx, R ky, R qx, R qy, R px, R py,
                                      R &ox, R &oy)
{
    const R hqx = fma(S.hxy, qy, S.hxx * qx), hqy = fma(S.hyy, qy, S.hyx * qx);
    const R a = fma(hqy, dy, hqx * dx) + fma(S.b.gy, py, S.b.gx * px);  // (H q).d + G.p
    const R gd = fma(S.b.gy, dy, S.b.gx * dx), dcq = ic * fma(S.cy, qy, S.cx * qx);
    ox = fma(-kx, dcq, ic * (fma(a, dx, gd * px) - hqx));
    oy = fma(-ky, dcq, ic * (fma(a, dy, gd * py) - hqy));
}

// Tangent-linear Runge-Kutta step of (q, p) along the step the sampler recorded
// (the stage directions and curvatures are recomputed as the tracer's stages
// computed them).
template <class R, int INTEG, bool BSP>
__device__ __forceinline__ void para_tangent(const ParaSampler<R, BSP> &P, const Ray<R> &y, R ds, R &qx, R &qy,
                                             R &px, R &py)
{
    const R d1x = y.dxh + y.dxl, d1y = y.dyh + y.dyl;
    R ic, k1x, k1y, k2x, k2y, e1x, e1y, e2x, e2y;
    ic = rcp(P.s[0].b.c);
    curvature(P.s[0].b, ic, d1x, d1y, k1x, k1y);
    dcurv(P.s[0], ic, d1x, d1y, k1x, k1y, qx, qy, px, py, e1x, e1y);
    if (INTEG == 4) {
        const R h2 = ds * (R)0.5;
        R k3x, k3y, k4x, k4y, e3x, e3y, e4x, e4y;
        const R d2x = fma(h2, k1x, d1x), d2y = fma(h2, k1y, d1y);
        const R q2x = fma(h2, px, qx), q2y = fma(h2, py, qy), p2x = fma(h2, e1x, px), p2y = fma(h2, e1y, py);
        ic = rcp(P.s[1].b.c);
        curvature(P.s[1].b, ic, d2x, d2y, k2x, k2y);
        dcurv(P.s[1], ic, d2x, d2y, k2x, k2y, q2x, q2y, p2x, p2y, e2x, e2y);
        const R d3x = fma(h2, k2x, d1x), d3y = fma(h2, k2y, d1y);
        const R q3x = fma(h2, p2x, qx), q3y = fma(h2, p2y, qy), p3x = fma(h2, e2x, px), p3y = fma(h2, e2y, py);
        ic = rcp(P.s[2].b.c);
        curvature(P.s[2].b, ic, d3x, d3y, k3x, k3y);
        dcurv(P.s[2], ic, d3x, d3y, k3x, k3y, q3x, q3y, p3x, p3y, e3x, e3y);
        const R d4x = fma(ds, k3x, d1x), d4y = fma(ds, k3y, d1y);
        const R q4x = fma(ds, p3x, qx), q4y = fma(ds, p3y, qy), p4x = fma(ds, e3x, px), p4y = fma(ds, e3y, py);
        ic = rcp(P.s[3].b.c);
        curvature(P.s[3].b, ic, d4x, d4y, k4x, k4y);
        dcurv(P.s[3], ic, d4x, d4y, k4x, k4y, q4x, q4y, p4x, p4y, e4x, e4y);
        const R s6 = ds * (R)(1.0 / 6.0);
        qx = fma(s6, px + (R)2 * (p2x + p3x) + p4x, qx);
        qy = fma(s6, py + (R)2 * (p2y + p3y) + p4y, qy);
        px = fma(s6, e1x + (R)2 * (e2x + e3x) + e4x, px);
        py = fma(s6, e1y + (R)2 * (e2y + e3y) + e4y, py);
    } else {
        const R d2x = fma(ds, k1x, d1x), d2y = fma(ds, k1y, d1y);
        const R q2x = fma(ds, px, qx), q2y = fma(ds, py, qy), p2x = fma(ds, e1x, px), p2y = fma(ds, e1y, py);
        ic = rcp(P.s[3].b.c);
        curvature(P.s[3].b, ic, d2x, d2y, k2x, k2y);
        dcurv(P.s[3], ic, d2x, d2y, k2x, k2y, q2x, q2y, p2x, p2y, e2x, e2y);
        const R s2 = ds * (R)0.5;
        qx = fma(s2, px + p2x, qx);
        qy = fma(s2, py + p2y, qy);
        px = fma(s2, e1x + e2x, px);
        py = fma(s2, e1y + e2y, py);
    }
}

template <class R, bool COMP, int INTEG, bool BSP>
__global__ void __launch_bounds__(kBlock)
    k_paraxial(Medium<R> M, Geo g, const int32_t *__restrict__ pairs, int64_t n, const double *__restrict__ theta,
               int max_steps, double *__restrict__ dgdth, double *__restrict__ jac, double *__restrict__ amp,
               int32_t *__restrict__ kmah, int8_t *__restrict__ status)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int e, r;
    TraceArgs pa;
    pa.pairs = pairs;
    double o_dg = NAN, o_j = NAN, o_a = NAN;
    int o_k = -1, st = RTX_RAY_BAD_INPUT;
    if (pair_of(pa, g, i, e, r)) {
        const Emitter em = emitter_of(g, e);
        Ray<R> ray;
        start_ray<R, COMP>(ray, g, em, theta[i]);
        double sp, cp;
        sincos(em.pe + kPi + theta[i], &sp, &cp);
        R qx = (R)0, qy = (R)0, px = (R)(-sp), py = (R)cp;  // d(direction)/d(theta)
        const R ds = (R)g.ds, R2 = (R)(g.R * g.R), cxr = (R)g.cx, cyr = (R)g.cy;
        const double ce = (double)lookup_at<R, COMP, BSP>(M, g, em.ex, em.ey).c;
        R jprev = (R)0;
        int changes = 0;
        st = RTX_RAY_NO_HIT;
        for (int m = 0; m < max_steps; m++) {
            ParaSampler<R, BSP> P{M, ray.uh, ray.vh};
            StageOut<R> so;
            stages<R, INTEG>(P, ray, ds, so);
            if (!(so.s1.c > (R)0) || !(ray.uh == ray.uh) || !(ray.vh == ray.vh)) {
                st = RTX_RAY_BAD_INPUT;
                break;
            }
            R nqx = qx, nqy = qy, npx = px, npy = py;
            para_tangent<R, INTEG, BSP>(P, ray, ds, nqx, nqy, npx, npy);
            Ray<R> nxt;
            (void)advance<R, COMP>(ray, so, nxt);
            {  // linearised renormalisation: p <- (p - (n.p) n) / |d| of the unnormalised d
                const R ux = (ray.dxh + ray.dxl) + so.idx, uy = (ray.dyh + ray.dyl) + so.idy;
                const R nrm = sqrt(ux * ux + uy * uy), nx = ux / nrm, ny = uy / nrm;
                const R np = fma(ny, npy, nx * npx);
                npx = (npx - np * nx) / nrm;
                npy = (npy - np * ny) / nrm;
            }
            const R pu = (nxt.uh - cxr) + nxt.ul, pv = (nxt.vh - cyr) + nxt.vl;
            if (pu * pu + pv * pv >= R2) {
                const Hit hit = intersect<R>(g, ray, nxt);
                const double ax = (((double)nxt.uh - g.cx) + (double)nxt.ul) - (((double)ray.uh - g.cx) + (double)ray.ul);
                const double ay = (((double)nxt.vh - g.cy) + (double)nxt.vl) - (((double)ray.vh - g.cy) + (double)ray.vl);
                double dqx = (double)qx + hit.t * ((double)nqx - (double)qx);
                double dqy = (double)qy + hit.t * ((double)nqy - (double)qy);
                const double dt = -(hit.qx * dqx + hit.qy * dqy) / (hit.qx * ax + hit.qy * ay);
                dqx += dt * ax;
                dqy += dt * ay;
                const double la = sqrt(ax * ax + ay * ay);
                const double jq = (ax / la) * dqy - (ay / la) * dqx;
                if (jq * (double)jprev < 0) changes++;
                const double cq = (double)lookup_at<R, COMP, BSP>(M, g, hit.qx, hit.qy).c;
                st = cq > 0.0 ? RTX_RAY_LINKED : RTX_RAY_BAD_INPUT;
                if (st == RTX_RAY_LINKED) {
                    o_dg = (hit.qx * dqy - hit.qy * dqx) / (g.R * g.R);
                    o_j = jq * g.h;
                    o_a = sqrt(cq / (ce * fabs(o_j)));
                    o_k = changes;
                }
                break;
            }
            const R jn = (nxt.dxh + nxt.dxl) * nqy - (nxt.dyh + nxt.dyl) * nqx;
            if (jn * jprev < (R)0) changes++;
            if (jn != (R)0) jprev = jn;
            ray = nxt;
            qx = nqx;
            qy = nqy;
            px = npx;
            py = npy;
        }
    }
    if (dgdth) dgdth[i] = o_dg;
    if (jac) jac[i] = o_j;
    if (amp) amp[i] = o_a;
    if (kmah) kmah[i] = o_k;
    status[i] = (int8_t)st;
}

// ------------------------------------------------------------------- SART --
// SART on the system matrix W (Sec. 3.1's default solver of the linearised ToF
// subproblem).  Every step streams W with one wave per row (CSR) or per column
// (CSC), the line's entries read by consecutive lanes, kSartU entries in flight
// per lane, and gathers from a small L2-resident vector:
//   once per call: row sums M_i and the sort input (CSR pass: every entry keyed
//   by its column, carrying its row and weight), a stable radix sort of the
//   entries by column (the transpose; rows stay ascending inside a column, so
//   the result does not depend on the run), column offsets from the sorted
//   keys, column sums V_j (CSC pass);
//   per iteration: r_i = (b_i - W_i x) / M_i (CSR pass), then
//   x_j += lambda / V_j sum_i W_ij r_i (CSC pass).
// No float atomics; all sums in FP64.  Entries whose column lies outside
// [0, n_nodes), and entries in no row, are sorted into the last column with
// row -1 and left out.  (Measured on the 256x256 workload: 8 entries in flight
// per lane, non-temporal loads, or persistent waves that load the next line
// before the current one's gathers wait were no faster, or slower, than this
// plain form.)
constexpr int kSartU = 4;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

// one entry of the transpose in a single load
__device__ __forceinline__ CscEnt<float> load_ent(const CscEnt<float> *p)
{
    const u32x2_t v = *(const u32x2_t *)p;
    return {(int32_t)v.x, __uint_as_float(v.y)};
}
__device__ __forceinline__ CscEnt<double> load_ent(const CscEnt<double> *p)
{
    const u32x4_t v = *(const u32x4_t *)p;
    return {(int32_t)v.x, __hiloint2double((int)v.w, (int)v.z)};
}

// M_i, and every entry's sort key (its column) and payload (row, weight).  Wave
// n_rows takes the entries before the first row and after the last.
template <class R>
__global__ void __launch_bounds__(kBlock)
    k_sart_rows(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col, const R *__restrict__ val,
                int64_t n_rows, int64_t nnz, int64_t n_nodes, double *__restrict__ M, uint32_t *__restrict__ key,
                CscEnt<R> *__restrict__ ent)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i > n_rows) return;
    const uint32_t last = (uint32_t)(n_nodes - 1);
    if (i == n_rows) {
        const int64_t a = min(max(rowptr[0], (int64_t)0), nnz), z = max(min(rowptr[n_rows], nnz), a);
        for (int64_t k = lane; k < a; k += 64) key[k] = last, ent[k] = {-1, (R)0};
        for (int64_t k = z + lane; k < nnz; k += 64) key[k] = last, ent[k] = {-1, (R)0};
        return;
    }
    double m = 0.0;
    const int64_t k1 = min(rowptr[i + 1], nnz);
    for (int64_t k0 = max(rowptr[i], (int64_t)0) + lane; k0 < k1; k0 += kSartU * 64) {
        int32_t j[kSartU];
        R w[kSartU];
#pragma unroll
        for (int u = 0; u < kSartU; u++) {
            const int64_t k = k0 + 64 * u;
            j[u] = k < k1 ? col[k] : -1;
            w[u] = k < k1 ? val[k] : (R)0;
        }
#pragma unroll
        for (int u = 0; u < kSartU; u++) {
            const int64_t k = k0 + 64 * u;
            if (k >= k1) continue;
            const bool ok = (uint64_t)j[u] < (uint64_t)n_nodes;
            key[k] = ok ? (uint32_t)j[u] : last;
            ent[k] = {ok ? (int32_t)i : -1, w[u]};
            if (ok) m += (double)w[u];
        }
    }
    m = wave_sum(m);
    if (lane == 0) M[i] = m;
}

// colptr[j] = the first sorted position whose key is >= j, for j in [0, n]: a
// binary search over the sorted keys (clamped to n - 1) per column.
__global__ void __launch_bounds__(kBlock)
    k_sart_bounds(const uint32_t *__restrict__ key, int64_t nnz, int64_t n, int64_t *__restrict__ colptr)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > n) return;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (min((int64_t)key[mid], n - 1) < j)
            lo = mid + 1;
        else
            hi = mid;
    }
    colptr[j] = lo;
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_sart_colsum(const int64_t *__restrict__ colptr,
                                                        const CscEnt<R> *__restrict__ ent, int64_t n_nodes,
                                                        int64_t n_rows, int64_t nnz, double *__restrict__ V)
{
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (j >= n_nodes) return;
    double v = 0.0;
    const int64_t k1 = min(colptr[j + 1], nnz);
    for (int64_t k = colptr[j] + lane; k < k1; k += 64) {
        const CscEnt<R> e = load_ent(ent + k);
        if ((uint64_t)e.row < (uint64_t)n_rows) v += (double)e.val;
    }
    v = wave_sum(v);
    if (lane == 0) V[j] = v;
}

template <class R>
__global__ void __launch_bounds__(kBlock)
    k_sart_resid(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col, const R *__restrict__ val,
                 int64_t n_rows, int64_t nnz, int64_t n_nodes, const double *__restrict__ b,
                 const double *__restrict__ M, const double *__restrict__ x, double *__restrict__ r)
{
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= n_rows) return;
    const double m = M[i];
    double proj = 0.0;
    const int64_t k1 = min(rowptr[i + 1], nnz);
    if (m != 0.0)
        for (int64_t k0 = max(rowptr[i], (int64_t)0) + lane; k0 < k1; k0 += kSartU * 64) {
            int32_t j[kSartU];
            R w[kSartU];
#pragma unroll
            for (int u = 0; u < kSartU; u++) {
                const int64_t k = k0 + 64 * u;
                j[u] = k < k1 ? col[k] : -1;
                w[u] = k < k1 ? val[k] : (R)0;
            }
            double xv[kSartU];
#pragma unroll
            for (int u = 0; u < kSartU; u++) xv[u] = (uint64_t)j[u] < (uint64_t)n_nodes ? x[j[u]] : 0.0;
#pragma unroll
            for (int u = 0; u < kSartU; u++) proj = fma((double)w[u], xv[u], proj);
        }
    proj = wave_sum(proj);
    if (lane == 0) r[i] = m != 0.0 ? (b[i] - proj) / m : 0.0;
}

template <class R>
__global__ void __launch_bounds__(kBlock)
    k_sart_back(const int64_t *__restrict__ colptr, const CscEnt<R> *__restrict__ ent, int64_t n_nodes,
                int64_t n_rows, int64_t nnz, const double *__restrict__ r, const double *__restrict__ V,
                double lambda, double *__restrict__ x)
{
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (j >= n_nodes) return;
    const double v = V[j];
    if (v == 0.0) return;
    double u = 0.0;
    const int64_t k1 = min(colptr[j + 1], nnz);
    for (int64_t k0 = colptr[j] + lane; k0 < k1; k0 += kSartU * 64) {
        CscEnt<R> e[kSartU];
#pragma unroll
        for (int t = 0; t < kSartU; t++) {
            const int64_t k = k0 + 64 * t;
            e[t] = k < k1 ? load_ent(ent + k) : CscEnt<R>{-1, (R)0};
        }
        double rv[kSartU];
#pragma unroll
        for (int t = 0; t < kSartU; t++) rv[t] = (uint64_t)e[t].row < (uint64_t)n_rows ? r[e[t].row] : 0.0;
#pragma unroll
        for (int t = 0; t < kSartU; t++) u = fma((double)e[t].val, rv[t], u);
    }
    u = wave_sum(u);
    if (lane == 0) x[j] += lambda * u / v;
}

}  // namespace

// ===================================================================== plan ==
struct rtx_plan_s {
    rtx_grid grid;
    rtx_ring ring;
    rtx_opts opts;
    int64_t max_pairs;
    void *tab = nullptr;  // packed medium
    bool have_medium = false;
    void *sart = nullptr;      // SART scratch: M, r [max_pairs]; V [nx*ny]; colptr [nx*ny+1]; counts
    void *sart_csc = nullptr;  // SART transpose of W and the sort's buffers (sart_csc_bytes)
    size_t sart_csc_bytes = 0;
    bool bsp = false;          // cubic B-spline interpolation (RTX_INTERP_BSPLINE)
    double *bsp_q = nullptr;   // [ny][nx] B-spline coefficients (FP64)
    unsigned long long *stats = nullptr;  // [3][kMaxBlocks][2]: trace, fan link pass, adjoint
    unsigned int *err = nullptr;          // device error word of the adjoint's LDS queue
    int stat_blocks[3] = {0, 0, 0};
    double *rho = nullptr;     // [max_pairs] ray-Born reduction
    double *omega = nullptr;   // [n_freq_cap]
    int n_freq_cap = 0;
    int n_cu = 0;
    int block = kBlock;  // threads (rays) per block of the persistent kernels
    // fan-start workspace (allocated on first use): own straight ray of each pair
    double *f_g = nullptr;
    int8_t *f_st = nullptr;
    void *f_seed = nullptr;
    void *adj_cp = nullptr;  // adjoint: zeroed gradient copies (allocated on first use)
    void *w_small = nullptr;  // path weights: per-row counts and offsets (w_small_bytes), kept between calls
    size_t w_small_bytes = 0;
    void *w_raw = nullptr;  // path weights: raw and merged row entries (w_raw_bytes), kept between calls
    size_t w_raw_bytes = 0;
    // fan start: mid-path checkpoints of the linking rays (RayCkpt [max_pairs][2])
    // and per-pair heads, for the adjoint's split; gen counts changes of the
    // medium and of the path options (step, integrator, step limit)
    void *ckpt = nullptr;
    CkptHead *ckpt_head = nullptr;
    unsigned gen = 1;
    // optional per-kernel timing with HIP events on the launch stream
    bool timing = false;
    std::vector<hipEvent_t> ev[RTX_NUM_SLOTS];
    int ev_used[RTX_NUM_SLOTS] = {};
};

struct rtx_batch_s {
    rtx_opts opts;
    int32_t weight;
    int n_inst = 0;
    int block = kBlock;
    int n_cu = 0;
    bool adjoint = false;
    std::vector<rtx_instance> inst;
    std::vector<size_t> tab_off;   // byte offset of each instance's packed table
    void *tabs = nullptr;          // all packed tables
    void *dinst = nullptr;         // Inst<R>[n_inst]
    int64_t *off = nullptr;        // [n_inst + 1]
    unsigned int *remain = nullptr;          // [2][n_inst]
    unsigned long long *times = nullptr;     // [1 + 2 n_inst]: t0, fwd done, adjoint done
    unsigned long long *stats = nullptr;     // [2][kMaxBlocks][2]
    unsigned int *err = nullptr;             // device error word of the adjoint's LDS queue
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t total_pairs = 0;
};

namespace {

constexpr int kMaxBlocks = 8192;
constexpr int kMaxCopies = 8;                // adjoint gradient copies (one per XCD)
constexpr int64_t kCopiesBytes = 64ll << 20;  // device memory they may take

int check_opts(const rtx_grid *g, const rtx_ring *r, const rtx_opts *o)
{
    if (!g || !r || !o) return fail(RTX_E_ARG, "null grid/ring/opts");
    if (g->nx < 4 || g->ny < 4) return fail(RTX_E_ARG, "grid must be at least 4x4 (got %dx%d)", g->nx, g->ny);
    if (!(g->h > 0)) return fail(RTX_E_ARG, "grid spacing h must be > 0");
    if ((int64_t)(g->nx - 1) * (g->ny - 1) >= (1 << 24))
        return fail(RTX_E_ARG, "grid of %dx%d nodes exceeds 2^24 cells", g->nx, g->ny);
    if (r->n_elem < 2) return fail(RTX_E_ARG, "ring needs >= 2 elements");
    if (!(r->radius > 0)) return fail(RTX_E_ARG, "ring radius must be > 0");
    if (o->prec != RTX_F64 && o->prec != RTX_F32C) return fail(RTX_E_ARG, "unknown precision %d", o->prec);
    if (o->integ != RTX_HEUN && o->integ != RTX_RK4) return fail(RTX_E_ARG, "unknown integrator %d", o->integ);
    if (!(o->ds_px > 0 && o->ds_px <= 2)) return fail(RTX_E_ARG, "ds_px must be in (0, 2]");
    if (!(o->tol_px >= 0)) return fail(RTX_E_ARG, "tol_px must be >= 0");
    if (o->max_marches < 1) return fail(RTX_E_ARG, "max_marches must be >= 1");
    if (o->max_steps < 0) return fail(RTX_E_ARG, "max_steps must be >= 0");
    double rpx = r->radius / g->h;
    double half = 0.5 * (std::min(g->nx, g->ny) - 1);
    if (rpx + std::max(1.0, o->ds_px) > half)
        return fail(RTX_E_ARG, "ring (radius %.3f px) does not fit the grid with a margin of max(1, ds) px", rpx);
    return RTX_OK;
}

Geo make_geo(const rtx_plan_s *P)
{
    Geo g;
    g.nx = P->grid.nx;
    g.ny = P->grid.ny;
    g.n_elem = P->ring.n_elem;
    g.cx = 0.5 * (P->grid.nx - 1);
    g.cy = 0.5 * (P->grid.ny - 1);
    g.R = P->ring.radius / P->grid.h;
    g.phi0 = P->ring.phi0;
    g.h = P->grid.h;
    g.ds = P->opts.ds_px;
    return g;
}

int max_steps_of(const rtx_plan_s *P)
{
    if (P->opts.max_steps > 0) return P->opts.max_steps;
    return (int)ceil(8.0 * (P->ring.radius / P->grid.h) / P->opts.ds_px);
}

// Event pair bracketing one launch when the plan's timing is on.
int time_mark(rtx_plan_s *P, int slot, int end, hipStream_t s)
{
    if (!P->timing) return RTX_OK;
    int k = P->ev_used[slot] * 2 + end;
    while ((int)P->ev[slot].size() <= k) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        P->ev[slot].push_back(e);
    }
    HIP_TRY(hipEventRecord(P->ev[slot][k], s));
    if (end) P->ev_used[slot]++;
    return RTX_OK;
}

int pack(rtx_plan_s *P, const double *c, hipStream_t s)
{
    if (!c) {
        if (!P->have_medium) return fail(RTX_E_ARG, "c is NULL and no medium was set");
        return RTX_OK;
    }
    int64_t cells = (int64_t)(P->grid.nx - 1) * (P->grid.ny - 1);
    int blocks = (int)((cells + kBlock - 1) / kBlock);
    P->gen++;  // checkpoints of rays through the previous medium no longer apply
    if (int rc = time_mark(P, RTX_SLOT_PACK, 0, s)) return rc;
    if (P->bsp) {
        const int nx = P->grid.nx, ny = P->grid.ny;
        hipLaunchKernelGGL(k_bsp_lines, dim3((ny + 63) / 64), dim3(64), 0, s, c, P->bsp_q, nx, ny, true);
        hipLaunchKernelGGL(k_bsp_lines, dim3((nx + 63) / 64), dim3(64), 0, s, c, P->bsp_q, nx, ny, false);
        if (P->opts.prec == RTX_F32C)
            hipLaunchKernelGGL(k_pack_bsp<float>, dim3(blocks), dim3(kBlock), 0, s, P->bsp_q, nx, ny, (float *)P->tab);
        else
            hipLaunchKernelGGL(k_pack_bsp<double>, dim3(blocks), dim3(kBlock), 0, s, P->bsp_q, nx, ny,
                               (double *)P->tab);
    } else if (P->opts.prec == RTX_F32C)
        hipLaunchKernelGGL(k_pack<float>, dim3(blocks), dim3(kBlock), 0, s, c, P->grid.nx, P->grid.ny,
                           (float *)P->tab);
    else
        hipLaunchKernelGGL(k_pack<double>, dim3(blocks), dim3(kBlock), 0, s, c, P->grid.nx, P->grid.ny,
                           (double *)P->tab);
    HIP_TRY(hipGetLastError());
    P->have_medium = true;
    return time_mark(P, RTX_SLOT_PACK, 1, s);
}

// Persistent launch: no more blocks than can be resident at once (lanes take
// further pairs with a fixed stride), and no more than the pairs need.
template <class K>
int grid_blocks_for(int n_cu, int block, K kernel, int64_t n)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t want = (n + block - 1) / block;
    int64_t cap = (int64_t)n_cu * per_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>({want, cap, (int64_t)kMaxBlocks}));
}

// The adjoint's blocks carry one extra wave (the queue drain) besides the
// `block` marching lanes.
template <class K>
int adjoint_blocks_for(int n_cu, int block, K kernel, int64_t n)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block + kFlushLanes, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t want = (n + block - 1) / block;
    int64_t cap = (int64_t)n_cu * per_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>({want, cap, (int64_t)kMaxBlocks}));
}

template <class K>
int grid_blocks(const rtx_plan_s *P, K kernel, int64_t n)
{
    return grid_blocks_for(P->n_cu, P->block, kernel, n);
}

template <class R, bool COMP>
int launch_trace(rtx_plan_s *P, const TraceArgs &A, hipStream_t s, int region = 0, int slot = RTX_SLOT_TRACE,
                 double ds_px = 0.0)
{
    Medium<R> M{(const R *)P->tab, P->grid.nx, P->grid.ny};
    Geo g = make_geo(P);
    if (ds_px > 0.0) g.ds = ds_px;
    auto kern = P->bsp ? (P->opts.integ == RTX_RK4 ? k_trace<R, COMP, 4, false, true>
                                                   : k_trace<R, COMP, 2, false, true>)
                       : (P->opts.integ == RTX_RK4 ? k_trace<R, COMP, 4, false> : k_trace<R, COMP, 2, false>);
    int blocks = grid_blocks(P, kern, A.n_pairs);
    P->stat_blocks[region] = blocks;
    BatchArgs B{};
    TraceArgs a = A;
    a.stats = P->stats + (size_t)region * 2 * kMaxBlocks;
    if (int rc = time_mark(P, slot, 0, s)) return rc;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(P->block), 0, s, M, g, a, B);
    HIP_TRY(hipGetLastError());
    return time_mark(P, slot, 1, s);
}

// Fan start: fixed pass at straight angles, seeds, linking pass.
template <class R, bool COMP>
int launch_fan(rtx_plan_s *P, const TraceArgs &A, hipStream_t s)
{
    const int64_t n = A.n_pairs;
    if (!P->f_g) {
        if (hipMalloc((void **)&P->f_g, sizeof(double) * P->max_pairs) != hipSuccess ||
            hipMalloc((void **)&P->f_st, sizeof(int8_t) * P->max_pairs) != hipSuccess ||
            hipMalloc(&P->f_seed, sizeof(FanSeed) * P->max_pairs) != hipSuccess)
            return fail(RTX_E_NOMEM, "fan-start workspace");
    }
    if (!P->ckpt && !P->bsp) {  // (B-spline plans have no adjoint)
        if (hipMalloc(&P->ckpt, sizeof(RayCkpt<R>) * 2 * (kSegs - 1) * P->max_pairs) != hipSuccess ||
            hipMalloc((void **)&P->ckpt_head, sizeof(CkptHead) * P->max_pairs) != hipSuccess)
            return fail(RTX_E_NOMEM, "fan-start checkpoints");
        // generation 0 is never current: no head applies before the pass writes it
        HIP_TRY(hipMemset(P->ckpt_head, 0, sizeof(CkptHead) * P->max_pairs));
    }
    // the fan rays seed the linking only: four tracing steps per fan step, at
    // most a pixel (never below the tracing step), the step limit scaled alike
    const double ds_fan = std::max(P->opts.ds_px, std::min(4.0 * P->opts.ds_px, 1.0));
    TraceArgs A1 = A;
    A1.flags = RTX_FIXED_ANGLE | kStraight;
    A1.tof = nullptr;  // the seed rays' misfits and statuses only
    A1.len = nullptr;
    A1.miss = nullptr;
    A1.n_marches = nullptr;
    A1.status = P->f_st;
    A1.gsig = P->f_g;
    A1.max_steps = (int)ceil(A.max_steps * P->opts.ds_px / ds_fan);
    if (int rc = launch_trace<R, COMP>(P, A1, s, 0, RTX_SLOT_TRACE, ds_fan)) return rc;
    Geo g = make_geo(P);
    if (int rc = time_mark(P, RTX_SLOT_FAN_SEED, 0, s)) return rc;
    hipLaunchKernelGGL(k_fan_seed, dim3(P->ring.n_elem), dim3(kBlock), sizeof(double) * (P->ring.n_elem - 1), s, g,
                       P->f_g, P->f_st, (FanSeed *)P->f_seed);
    HIP_TRY(hipGetLastError());
    if (int rc = time_mark(P, RTX_SLOT_FAN_SEED, 1, s)) return rc;
    TraceArgs A3 = A;
    A3.flags = RTX_FAN_START;
    A3.gsig = nullptr;
    A3.seed = (const FanSeed *)P->f_seed;
    A3.f_g = P->f_g;
    A3.f_st = P->f_st;
    A3.ckpt = P->ckpt;
    A3.ckpt_head = P->ckpt_head;
    A3.gen = P->gen;
    (void)n;
    Medium<R> M{(const R *)P->tab, P->grid.nx, P->grid.ny};
    auto kern = P->bsp ? (P->opts.integ == RTX_RK4 ? k_link2<R, COMP, 4, true> : k_link2<R, COMP, 2, true>)
                       : (P->opts.integ == RTX_RK4 ? k_link2<R, COMP, 4> : k_link2<R, COMP, 2>);
    const int blocks = grid_blocks(P, kern, 2 * A3.n_pairs);
    P->stat_blocks[1] = blocks;
    A3.stats = P->stats + (size_t)1 * 2 * kMaxBlocks;
    if (int rc = time_mark(P, RTX_SLOT_FAN_LINK, 0, s)) return rc;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(P->block), 0, s, M, g, A3);
    HIP_TRY(hipGetLastError());
    return time_mark(P, RTX_SLOT_FAN_LINK, 1, s);
}

template <class R, bool COMP>
int launch_adjoint(rtx_plan_s *P, const AdjArgs &A, R *grad, hipStream_t s)
{
    Medium<R> M{(const R *)P->tab, P->grid.nx, P->grid.ny};
    Geo g = make_geo(P);
    AdjArgs a = A;
    a.err = P->err;
    const int64_t nn = (int64_t)P->grid.nx * P->grid.ny;
    // zeroed copies of the gradient (kept zeroed by k_copies_sum), as many as
    // fit in kCopiesBytes, at most kMaxCopies; one copy means grad itself
    const int n_copies =
        (int)std::max<int64_t>(1, std::min<int64_t>(kMaxCopies, kCopiesBytes / (nn * (int64_t)sizeof(R))));
    if (n_copies > 1 && !P->adj_cp) {
        const size_t bytes = (size_t)n_copies * nn * sizeof(R);
        if (hipMalloc(&P->adj_cp, bytes) != hipSuccess) {
            P->adj_cp = nullptr;
            return fail(RTX_E_NOMEM, "adjoint gradient copies");
        }
        HIP_TRY(hipMemset(P->adj_cp, 0, bytes));
    }
    a.n_copies = n_copies;
    auto kern = a.split ? (P->opts.integ == RTX_RK4 ? k_adjoint<R, COMP, 4, false, true>
                                                    : k_adjoint<R, COMP, 2, false, true>)
                        : (P->opts.integ == RTX_RK4 ? k_adjoint<R, COMP, 4, false> : k_adjoint<R, COMP, 2, false>);
    int blocks = adjoint_blocks_for(P->n_cu, P->block, kern, A.n_items);
    P->stat_blocks[2] = blocks;
    BatchArgs B{};
    if (int rc = time_mark(P, RTX_SLOT_ADJOINT, 0, s)) return rc;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(P->block + kFlushLanes), 0, s, M, g, a,
                       n_copies > 1 ? (R *)P->adj_cp : grad, B);
    HIP_TRY(hipGetLastError());
    if (n_copies > 1) {
        hipLaunchKernelGGL(k_copies_sum<R>, dim3((unsigned)((nn + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           (R *)P->adj_cp, n_copies, nn, grad);
        HIP_TRY(hipGetLastError());
    }
    return time_mark(P, RTX_SLOT_ADJOINT, 1, s);
}

constexpr int kMergeCap = 8192;  // entries per row the LDS merge can sort

// Grows a plan-owned buffer to at least `bytes` (contents are not kept).
static bool grow(void *&buf, size_t &have, size_t bytes)
{
    if (bytes <= have) return true;
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    have = 0;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        buf = nullptr;
        return false;
    }
    have = bytes;
    return true;
}

template <class R, bool COMP>
int emit_weights(rtx_plan_s *P, const TraceArgs &T, int64_t *w_rowptr, int32_t *w_col, R *w_val, int64_t nnz_cap,
                 hipStream_t s)
{
    const int64_t n = T.n_pairs;
    Medium<R> M{(const R *)P->tab, P->grid.nx, P->grid.ny};
    Geo g = make_geo(P);
    // plan-owned scratch: rawcnt, rawoff, ucnt [n] and the device row pointers
    // [n + 1]; then the raw entries (columns, values)
    if (!grow(P->w_small, P->w_small_bytes, sizeof(int64_t) * (4 * (size_t)n + 1)))
        return fail(RTX_E_NOMEM, "weights scratch");
    int64_t *rawcnt = (int64_t *)P->w_small, *rawoff = rawcnt + n, *ucnt = rawoff + n, *rowptr_d = ucnt + n;
    WArgs A;
    A.pairs = T.pairs;
    A.n_pairs = n;
    A.theta = T.theta;
    A.status = T.status;
    A.max_steps = T.max_steps;
    A.rawcnt = rawcnt;
    A.rawoff = rawoff;
    A.cols = nullptr;
    A.vals = nullptr;
    auto kc = P->opts.integ == RTX_RK4 ? k_weights<R, COMP, 4, false> : k_weights<R, COMP, 2, false>;
    auto kf = P->opts.integ == RTX_RK4 ? k_weights<R, COMP, 4, true> : k_weights<R, COMP, 2, true>;
    hipLaunchKernelGGL(kc, dim3(grid_blocks(P, kc, n)), dim3(P->block), 0, s, M, g, A);
    HIP_TRY(hipGetLastError());
    std::vector<int64_t> h(n), off(n);
    HIP_TRY(hipMemcpyAsync(h.data(), rawcnt, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t total = 0, mx = 0;
    for (int64_t i = 0; i < n; i++) {
        off[i] = total;
        total += h[i];
        mx = std::max(mx, h[i]);
    }
    if (mx > kMergeCap)
        return fail(RTX_E_UNSUPPORTED, "a path-weight row has %lld raw entries, above the %d the row merge handles",
                    (long long)mx, kMergeCap);
    const size_t b_cols = ((size_t)std::max<int64_t>(total, 1) * sizeof(int32_t) + 255) & ~(size_t)255;
    if (!grow(P->w_raw, P->w_raw_bytes, b_cols + (size_t)std::max<int64_t>(total, 1) * sizeof(R)))
        return fail(RTX_E_NOMEM, "weights scratch (%lld entries)", (long long)total);
    int32_t *cols = (int32_t *)P->w_raw;
    R *vals = (R *)((char *)P->w_raw + b_cols);
    HIP_TRY(hipMemcpyAsync(rawoff, off.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
    A.cols = cols;
    A.vals = vals;
    hipLaunchKernelGGL(kf, dim3(grid_blocks(P, kf, n)), dim3(P->block), 0, s, M, g, A);
    HIP_TRY(hipGetLastError());
    int cap = 256;
    while (cap < mx) cap <<= 1;
    size_t shmem = (size_t)cap * (sizeof(R) + sizeof(int32_t));
    hipLaunchKernelGGL(k_wmerge<R>, dim3((unsigned)n), dim3(kBlock), shmem, s, rawoff, rawcnt, cols, vals, ucnt,
                       cap);
    HIP_TRY(hipGetLastError());
    std::vector<int64_t> u(n), rp(n + 1);
    HIP_TRY(hipMemcpyAsync(u.data(), ucnt, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    rp[0] = 0;
    for (int64_t i = 0; i < n; i++) rp[i + 1] = rp[i] + u[i];
    HIP_TRY(hipMemcpyAsync(w_rowptr, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    if (w_col) {
        if (!w_val) return fail(RTX_E_ARG, "w_val is required with w_col");
        if (rp[n] > nnz_cap) {
            HIP_TRY(hipStreamSynchronize(s));
            return fail(RTX_E_CAPACITY, "%lld path weights exceed nnz_cap %lld", (long long)rp[n],
                        (long long)nnz_cap);
        }
        HIP_TRY(hipMemcpyAsync(rowptr_d, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_wcompact<R>, dim3((unsigned)n), dim3(kBlock), 0, s, rawoff, rowptr_d, cols, vals,
                           w_col, w_val);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));  // host vectors die here
    return RTX_OK;
}

int check_pairs(const rtx_plan_s *P, const int32_t *pairs, int64_t n)
{
    if (n < 0) return fail(RTX_E_ARG, "n_pairs < 0");
    if (n > P->max_pairs) return fail(RTX_E_ARG, "n_pairs %lld exceeds the plan's max_pairs %lld", (long long)n,
                                      (long long)P->max_pairs);
    if (!pairs && n != 0 && n != (int64_t)P->ring.n_elem * (P->ring.n_elem - 1))
        return fail(RTX_E_ARG, "pairs == NULL requires n_pairs = n_elem (n_elem - 1)");
    return RTX_OK;
}

Geo geo_of(const rtx_grid &gr, const rtx_ring &ri, const rtx_opts &o)
{
    Geo g;
    g.nx = gr.nx;
    g.ny = gr.ny;
    g.n_elem = ri.n_elem;
    g.cx = 0.5 * (gr.nx - 1);
    g.cy = 0.5 * (gr.ny - 1);
    g.R = ri.radius / gr.h;
    g.phi0 = ri.phi0;
    g.h = gr.h;
    g.ds = o.ds_px;
    return g;
}

int max_steps_for(const rtx_grid &gr, const rtx_ring &ri, const rtx_opts &o)
{
    if (o.max_steps > 0) return o.max_steps;
    return (int)ceil(8.0 * (ri.radius / gr.h) / o.ds_px);
}

// Enqueues one batch run on s: reset, pack every medium, trace, adjoint.
template <class R, bool COMP>
int batch_enqueue(rtx_batch_s *Bt, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3((Bt->n_inst + kBlock - 1) / kBlock), dim3(kBlock), 0, s, Bt->off,
                       Bt->n_inst, Bt->remain, Bt->remain + Bt->n_inst, Bt->times);
    HIP_TRY(hipGetLastError());
    for (int k = 0; k < Bt->n_inst; k++) {
        const rtx_instance &I = Bt->inst[k];
        int64_t cells = (int64_t)(I.grid.nx - 1) * (I.grid.ny - 1);
        hipLaunchKernelGGL(k_pack<R>, dim3((unsigned)((cells + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, I.c,
                           I.grid.nx, I.grid.ny, (R *)((char *)Bt->tabs + Bt->tab_off[k]));
        HIP_TRY(hipGetLastError());
    }
    BatchArgs B;
    B.inst = Bt->dinst;
    B.off = Bt->off;
    B.n_inst = Bt->n_inst;
    B.remain = Bt->remain;
    B.t_done = Bt->times + 1;
    Medium<R> M{nullptr, 0, 0};
    Geo g{};
    TraceArgs A{};
    A.stats = Bt->stats;
    auto kt = Bt->opts.integ == RTX_RK4 ? k_trace<R, COMP, 4, true> : k_trace<R, COMP, 2, true>;
    int blocks = grid_blocks_for(Bt->n_cu, Bt->block, kt, Bt->total_pairs);
    hipLaunchKernelGGL(kt, dim3(blocks), dim3(Bt->block), 0, s, M, g, A, B);
    HIP_TRY(hipGetLastError());
    if (Bt->adjoint) {
        AdjArgs J{};
        J.stats = Bt->stats + 2 * kMaxBlocks;
        B.remain = Bt->remain + Bt->n_inst;
        B.t_done = Bt->times + 1 + Bt->n_inst;
        J.err = Bt->err;
        J.n_copies = 1;  // instances add into their own gradients
        auto ka = Bt->opts.integ == RTX_RK4 ? k_adjoint<R, COMP, 4, true> : k_adjoint<R, COMP, 2, true>;
        int ablocks = adjoint_blocks_for(Bt->n_cu, Bt->block, ka, Bt->total_pairs);
        hipLaunchKernelGGL(ka, dim3(ablocks), dim3(Bt->block + kFlushLanes), 0, s, M, g, J, (R *)nullptr, B);
        HIP_TRY(hipGetLastError());
    }
    return RTX_OK;
}

template <class R>
int batch_upload(rtx_batch_s *Bt)
{
    std::vector<Inst<R>> h(Bt->n_inst);
    for (int k = 0; k < Bt->n_inst; k++) {
        const rtx_instance &I = Bt->inst[k];
        Inst<R> &d = h[k];
        memset(&d, 0, sizeof d);
        d.M = Medium<R>{(const R *)((char *)Bt->tabs + Bt->tab_off[k]), I.grid.nx, I.grid.ny};
        d.g = geo_of(I.grid, I.ring, Bt->opts);
        d.A.pairs = I.pairs;
        d.A.n_pairs = I.n_pairs;
        d.A.theta = I.theta;
        d.A.tof = I.tof;
        d.A.len = I.len;
        d.A.miss = I.miss_px;
        d.A.n_marches = I.n_marches;
        d.A.status = I.status;
        d.A.max_marches = Bt->opts.max_marches;
        d.A.max_steps = max_steps_for(I.grid, I.ring, Bt->opts);
        d.A.tol = Bt->opts.tol_px;
        d.A.flags = Bt->opts.flags;
        d.J.pairs = I.pairs;
        d.J.n_pairs = I.n_pairs;
        d.J.theta = I.theta;
        d.J.status = I.status;
        d.J.rho = I.resid;
        d.J.weight = Bt->weight;
        d.J.max_steps = d.A.max_steps;
        d.grad = (R *)I.grad;
    }
    HIP_TRY(hipMemcpy(Bt->dinst, h.data(), sizeof(Inst<R>) * Bt->n_inst, hipMemcpyHostToDevice));
    return RTX_OK;
}

}  // namespace

// ====================================================================== ABI ==
template <class R, bool COMP>
int launch_paraxial(rtx_plan_s *P, const int32_t *pairs, int64_t n, const double *theta, double *dgdth, double *jac,
                    double *amp, int32_t *kmah, int8_t *status, hipStream_t s)
{
    Medium<R> M{(const R *)P->tab, P->grid.nx, P->grid.ny};
    Geo g = make_geo(P);
    auto kern = P->bsp ? (P->opts.integ == RTX_RK4 ? k_paraxial<R, COMP, 4, true> : k_paraxial<R, COMP, 2, true>)
                       : (P->opts.integ == RTX_RK4 ? k_paraxial<R, COMP, 4, false> : k_paraxial<R, COMP, 2, false>);
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s, M, g, pairs, n, theta, max_steps_of(P), dgdth, jac,
                       amp, kmah, status);
    HIP_TRY(hipGetLastError());
    return RTX_OK;
}

template <class R, bool COMP>
int launch_march(rtx_plan_s *P, int64_t n_rays, const double *x0, const double *d0, int n_steps, double *pts,
                 hipStream_t s)
{
    Medium<R> M{(const R *)P->tab, P->grid.nx, P->grid.ny};
    Geo g = make_geo(P);
    auto kern = P->bsp ? (P->opts.integ == RTX_RK4 ? k_march<R, COMP, 4, true> : k_march<R, COMP, 2, true>)
                       : (P->opts.integ == RTX_RK4 ? k_march<R, COMP, 4, false> : k_march<R, COMP, 2, false>);
    const unsigned blocks = (unsigned)((n_rays + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s, M, g, n_rays, x0, d0, n_steps, pts);
    HIP_TRY(hipGetLastError());
    return RTX_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

template <class R>
int launch_sart(rtx_plan_s *P, int64_t n_rows, int64_t nnz, const int64_t *rowptr, const int32_t *col, const R *val,
                const double *b, double *x, int n_iter, double lambda, hipStream_t s)
{
    const int64_t nodes = (int64_t)P->grid.nx * P->grid.ny;
    double *M = (double *)P->sart, *r = M + P->max_pairs, *V = r + P->max_pairs;
    int64_t *colptr = (int64_t *)(V + nodes);
    unsigned end_bit = 1;  // keys are columns, < nodes
    while (end_bit < 32 && ((int64_t)1 << end_bit) < nodes) end_bit++;
    // plan-owned: the transpose, the sort's input entries, keys in and out, and
    // the sort's own scratch
    size_t tmp_bytes = 0;
    if (nnz > 0)
        HIP_TRY(csc_sort<R>(nullptr, tmp_bytes, nullptr, nullptr, nullptr, nullptr, (size_t)nnz, end_bit, s));
    const size_t b_ent = align256(sizeof(CscEnt<R>) * (size_t)nnz), b_key = align256(sizeof(uint32_t) * (size_t)nnz);
    const size_t need = 2 * b_ent + 2 * b_key + align256(tmp_bytes);
    if (need > P->sart_csc_bytes) {
        if (P->sart_csc) (void)hipFree(P->sart_csc);
        P->sart_csc = nullptr;
        P->sart_csc_bytes = 0;
        if (hipMalloc(&P->sart_csc, need) != hipSuccess) {
            P->sart_csc = nullptr;
            return fail(RTX_E_NOMEM, "SART transpose allocation (%lld entries) failed", (long long)nnz);
        }
        P->sart_csc_bytes = need;
    }
    char *base = (char *)P->sart_csc;
    CscEnt<R> *ent = (CscEnt<R> *)base, *ent_in = (CscEnt<R> *)(base + b_ent);
    uint32_t *key_in = (uint32_t *)(base + 2 * b_ent), *key = (uint32_t *)(base + 2 * b_ent + b_key);
    void *tmp = base + 2 * b_ent + 2 * b_key;
    const unsigned rb = (unsigned)((n_rows * 64 + kBlock - 1) / kBlock);
    const unsigned cb = (unsigned)((nodes * 64 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_sart_rows<R>, dim3((unsigned)(((n_rows + 1) * 64 + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, rowptr, col, val, n_rows, nnz, nodes, M, key_in, ent_in);
    if (nnz > 0) HIP_TRY(csc_sort<R>(tmp, tmp_bytes, key_in, key, ent_in, ent, (size_t)nnz, end_bit, s));
    hipLaunchKernelGGL(k_sart_bounds, dim3((unsigned)((nodes + 1 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       (const uint32_t *)key, nnz, nodes, colptr);
    hipLaunchKernelGGL(k_sart_colsum<R>, dim3(cb), dim3(kBlock), 0, s, (const int64_t *)colptr,
                       (const CscEnt<R> *)ent, nodes, n_rows, nnz, V);
    for (int it = 0; it < n_iter; it++) {
        hipLaunchKernelGGL(k_sart_resid<R>, dim3(rb), dim3(kBlock), 0, s, rowptr, col, val, n_rows, nnz, nodes, b,
                           (const double *)M, (const double *)x, r);
        hipLaunchKernelGGL(k_sart_back<R>, dim3(cb), dim3(kBlock), 0, s, (const int64_t *)colptr,
                           (const CscEnt<R> *)ent, nodes, n_rows, nnz, (const double *)r, (const double *)V, lambda,
                           x);
    }
    HIP_TRY(hipGetLastError());
    return RTX_OK;
}

extern "C" {

const char *rtx_last_error(void) { return g_last_error.c_str(); }

int rtx_plan_create(rtx_plan *out, const rtx_grid *grid, const rtx_ring *ring, const rtx_opts *opts,
                    int64_t max_pairs)
{
    g_last_error.clear();
    if (!out) return fail(RTX_E_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_opts(grid, ring, opts);
    if (rc) return rc;
    if (max_pairs < 1) return fail(RTX_E_ARG, "max_pairs must be >= 1");
    rtx_plan_s *P = new rtx_plan_s();
    P->grid = *grid;
    P->ring = *ring;
    P->opts = *opts;
    P->max_pairs = max_pairs;
    size_t esz = opts->prec == RTX_F32C ? sizeof(float) : sizeof(double);
    P->bsp = (opts->flags & RTX_INTERP_BSPLINE) != 0;
    size_t tab_bytes = (size_t)(grid->nx - 1) * (grid->ny - 1) * (P->bsp ? 16 : kCoef) * esz;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete P;
        return fail(RTX_E_HIP, "no HIP device");
    }
    P->n_cu = prop.multiProcessorCount;
    if (hipMalloc(&P->tab, tab_bytes) != hipSuccess ||
        hipMalloc((void **)&P->stats, sizeof(unsigned long long) * 3 * 2 * kMaxBlocks) != hipSuccess ||
        hipMalloc((void **)&P->err, sizeof(unsigned int)) != hipSuccess ||
        hipMalloc((void **)&P->rho, sizeof(double) * max_pairs) != hipSuccess ||
        (P->bsp && hipMalloc((void **)&P->bsp_q, sizeof(double) * grid->nx * grid->ny) != hipSuccess)) {
        rtx_plan_destroy(P);
        return fail(RTX_E_NOMEM, "device allocation of the plan workspace failed");
    }
    if (hipMemset(P->err, 0, sizeof(unsigned int)) != hipSuccess) {
        rtx_plan_destroy(P);
        return fail(RTX_E_HIP, "clearing the plan's error word failed");
    }
    *out = P;
    return RTX_OK;
}

int rtx_plan_destroy(rtx_plan P)
{
    if (!P) return RTX_OK;
    (void)hipDeviceSynchronize();
    if (P->tab) (void)hipFree(P->tab);
    if (P->stats) (void)hipFree(P->stats);
    if (P->err) (void)hipFree(P->err);
    if (P->bsp_q) (void)hipFree(P->bsp_q);
    if (P->sart) (void)hipFree(P->sart);
    if (P->sart_csc) (void)hipFree(P->sart_csc);
    for (void *q : {(void *)P->f_g, (void *)P->f_st, P->f_seed})
        if (q) (void)hipFree(q);
    for (int k = 0; k < RTX_NUM_SLOTS; k++)
        for (hipEvent_t e : P->ev[k]) (void)hipEventDestroy(e);
    if (P->rho) (void)hipFree(P->rho);
    if (P->omega) (void)hipFree(P->omega);
    if (P->adj_cp) (void)hipFree(P->adj_cp);
    if (P->w_small) (void)hipFree(P->w_small);
    if (P->w_raw) (void)hipFree(P->w_raw);
    if (P->ckpt) (void)hipFree(P->ckpt);
    if (P->ckpt_head) (void)hipFree(P->ckpt_head);
    delete P;
    return RTX_OK;
}

int rtx_plan_set_opts(rtx_plan P, const rtx_opts *opts)
{
    g_last_error.clear();
    if (!P || !opts) return fail(RTX_E_ARG, "null plan/opts");
    if (opts->prec != P->opts.prec) return fail(RTX_E_ARG, "precision of a plan cannot change");
    if ((opts->flags ^ P->opts.flags) & RTX_INTERP_BSPLINE)
        return fail(RTX_E_ARG, "the interpolation (RTX_INTERP_BSPLINE) of a plan cannot change");
    int rc = check_opts(&P->grid, &P->ring, opts);
    if (rc) return rc;
    if (opts->ds_px != P->opts.ds_px || opts->integ != P->opts.integ || opts->max_steps != P->opts.max_steps)
        P->gen++;  // the rays' paths change
    P->opts = *opts;
    return RTX_OK;
}

int rtx_set_medium(rtx_plan P, const double *c, void *stream)
{
    g_last_error.clear();
    if (!P || !c) return fail(RTX_E_ARG, "null plan or c");
    return pack(P, c, (hipStream_t)stream);
}

int rtx_trace_rays(rtx_plan P, const double *c, const int32_t *pairs, int64_t n_pairs, double *theta,
                   double *tof, double *len, double *miss_px, int32_t *n_marches, int8_t *status,
                   int64_t *w_rowptr, int32_t *w_col, void *w_val, int64_t nnz_cap, void *stream)
{
    g_last_error.clear();
    if (!P) return fail(RTX_E_ARG, "null plan");
    int rc = check_pairs(P, pairs, n_pairs);
    if (rc) return rc;
    if (n_pairs == 0) {
        rc = pack(P, c, (hipStream_t)stream);
        if (rc || !w_rowptr) return rc;
        static const int64_t zero = 0;
        HIP_TRY(hipMemcpyAsync(w_rowptr, &zero, sizeof zero, hipMemcpyHostToDevice, (hipStream_t)stream));
        HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
        return RTX_OK;
    }
    if (!theta || !status) return fail(RTX_E_ARG, "theta and status are required");
    if (!w_rowptr && (w_col || w_val)) return fail(RTX_E_ARG, "w_col/w_val need w_rowptr");
    if (w_rowptr && P->bsp) return fail(RTX_E_UNSUPPORTED, "path weights are bilinear-only (plan uses RTX_INTERP_BSPLINE)");
    if (w_col && nnz_cap < 0) return fail(RTX_E_ARG, "nnz_cap < 0");
    hipStream_t s = (hipStream_t)stream;
    rc = pack(P, c, s);
    if (rc) return rc;
    if (n_pairs == 0) return RTX_OK;
    TraceArgs A;
    A.pairs = pairs;
    A.n_pairs = n_pairs;
    A.theta = theta;
    A.tof = tof;
    A.len = len;
    A.miss = miss_px;
    A.n_marches = n_marches;
    A.status = status;
    A.max_marches = P->opts.max_marches;
    A.max_steps = max_steps_of(P);
    A.tol = P->opts.tol_px;
    A.flags = P->opts.flags;
    A.stats = P->stats;
    A.gsig = nullptr;
    A.seed = nullptr;
    A.f_g = nullptr;
    A.f_st = nullptr;
    P->stat_blocks[1] = 0;
    const bool fan = (A.flags & RTX_FAN_START) != 0;
    if (fan && (pairs || (A.flags & (RTX_FIXED_ANGLE | RTX_WARM_START))))
        return fail(RTX_E_ARG, "RTX_FAN_START needs all ordered pairs (pairs == NULL) and no warm/fixed start");
    if (P->opts.prec == RTX_F32C) {
        rc = fan ? launch_fan<float, true>(P, A, s) : launch_trace<float, true>(P, A, s);
        if (rc || !w_rowptr) return rc;
        return emit_weights<float, true>(P, A, w_rowptr, w_col, (float *)w_val, nnz_cap, s);
    }
    rc = fan ? launch_fan<double, false>(P, A, s) : launch_trace<double, false>(P, A, s);
    if (rc || !w_rowptr) return rc;
    return emit_weights<double, false>(P, A, w_rowptr, w_col, (double *)w_val, nnz_cap, s);
}

int rtx_sart(rtx_plan P, int64_t n_rows, int64_t nnz, const int64_t *w_rowptr, const int32_t *w_col,
             const void *w_val, const double *b, double *x, int32_t n_iter, double lambda, void *stream)
{
    g_last_error.clear();
    if (!P) return fail(RTX_E_ARG, "null plan");
    if (n_rows < 0 || n_rows > P->max_pairs)
        return fail(RTX_E_ARG, "n_rows %lld outside [0, max_pairs = %lld]", (long long)n_rows,
                    (long long)P->max_pairs);
    if (n_iter < 0) return fail(RTX_E_ARG, "n_iter < 0");
    if (nnz < 0 || nnz >= ((int64_t)1 << 40)) return fail(RTX_E_ARG, "bad nnz %lld", (long long)nnz);
    if (!(lambda > 0.0 && lambda < 2.0)) return fail(RTX_E_ARG, "lambda must lie in (0, 2)");
    if (!x || (n_rows > 0 && (!w_rowptr || !w_col || !w_val || !b)))
        return fail(RTX_E_ARG, "x, and with rows w_rowptr, w_col, w_val and b, are required");
    const int64_t nodes = (int64_t)P->grid.nx * P->grid.ny;
    if (n_rows == 0 || n_iter == 0) return RTX_OK;
    if (!P->sart) {
        const size_t bytes = sizeof(double) * (2 * P->max_pairs + nodes) + sizeof(int64_t) * (nodes + 1);
        if (hipMalloc(&P->sart, bytes) != hipSuccess) {
            P->sart = nullptr;
            return fail(RTX_E_NOMEM, "SART scratch allocation failed");
        }
    }
    hipStream_t s = (hipStream_t)stream;
    if (P->opts.prec == RTX_F32C)
        return launch_sart<float>(P, n_rows, nnz, w_rowptr, w_col, (const float *)w_val, b, x, n_iter, lambda, s);
    return launch_sart<double>(P, n_rows, nnz, w_rowptr, w_col, (const double *)w_val, b, x, n_iter, lambda, s);
}

int rtx_paraxial(rtx_plan P, const double *c, const int32_t *pairs, int64_t n_pairs, const double *theta,
                 double *dgdth, double *jac, double *amp, int32_t *kmah, int8_t *status, void *stream)
{
    g_last_error.clear();
    if (!P) return fail(RTX_E_ARG, "null plan");
    int rc = check_pairs(P, pairs, n_pairs);
    if (rc) return rc;
    if (n_pairs > 0 && (!theta || !status)) return fail(RTX_E_ARG, "theta and status are required");
    hipStream_t s = (hipStream_t)stream;
    rc = pack(P, c, s);
    if (rc || n_pairs == 0) return rc;
    if (P->opts.prec == RTX_F32C)
        return launch_paraxial<float, true>(P, pairs, n_pairs, theta, dgdth, jac, amp, kmah, status, s);
    return launch_paraxial<double, false>(P, pairs, n_pairs, theta, dgdth, jac, amp, kmah, status, s);
}

int rtx_march_free(rtx_plan P, const double *c, int64_t n_rays, const double *x0, const double *d0,
                   int32_t n_steps, double *pts, void *stream)
{
    g_last_error.clear();
    if (!P) return fail(RTX_E_ARG, "null plan");
    if (n_rays < 0 || n_rays > ((int64_t)1 << 31) - kBlock) return fail(RTX_E_ARG, "bad n_rays %lld", (long long)n_rays);
    if (n_steps < 0 || n_steps >= (1 << 30)) return fail(RTX_E_ARG, "bad n_steps %d", n_steps);
    if (n_rays > 0 && (!x0 || !d0 || !pts)) return fail(RTX_E_ARG, "x0, d0 and pts are required");
    hipStream_t s = (hipStream_t)stream;
    int rc = pack(P, c, s);
    if (rc || n_rays == 0) return rc;
    if (P->opts.prec == RTX_F32C) return launch_march<float, true>(P, n_rays, x0, d0, n_steps, pts, s);
    return launch_march<double, false>(P, n_rays, x0, d0, n_steps, pts, s);
}

int rtx_tof_forward(rtx_plan P, const double *c, const int32_t *pairs, int64_t n_pairs, double *theta,
                    double *tof, int8_t *status, void *stream)
{
    return rtx_trace_rays(P, c, pairs, n_pairs, theta, tof, nullptr, nullptr, nullptr, status, nullptr, nullptr,
                          nullptr, 0, stream);
}

int rtx_tof_adjoint(rtx_plan P, const double *c, const int32_t *pairs, int64_t n_pairs, const double *theta,
                    const int8_t *status, const double *tof, const void *resid, int32_t resid_kind,
                    const double *freqs_hz, int32_t n_freq, int32_t weight, void *grad, void *stream)
{
    g_last_error.clear();
    if (!P) return fail(RTX_E_ARG, "null plan");
    int rc = check_pairs(P, pairs, n_pairs);
    if (rc) return rc;
    if (!grad) return fail(RTX_E_ARG, "grad is required");
    if (P->bsp) return fail(RTX_E_UNSUPPORTED, "the adjoint is bilinear-only (plan uses RTX_INTERP_BSPLINE)");
    if (n_pairs == 0) return pack(P, c, (hipStream_t)stream);
    if (!theta || !status || !resid) return fail(RTX_E_ARG, "theta, status and resid are required");
    if (weight != RTX_W_LENGTH && weight != RTX_W_DTDC) return fail(RTX_E_ARG, "unknown weight %d", weight);
    if (resid_kind != RTX_RESID_REAL && resid_kind != RTX_RESID_RAYBORN_C64)
        return fail(RTX_E_ARG, "unknown resid_kind %d", resid_kind);
    hipStream_t s = (hipStream_t)stream;
    const double *rho = (const double *)resid;
    if (resid_kind == RTX_RESID_RAYBORN_C64) {
        if (!tof || !freqs_hz || n_freq < 1) return fail(RTX_E_ARG, "ray-Born residuals need tof and freqs_hz");
        if (n_freq > P->n_freq_cap) {
            if (P->omega) {
                HIP_TRY(hipStreamSynchronize(s));
                (void)hipFree(P->omega);
                P->omega = nullptr;
            }
            if (hipMalloc((void **)&P->omega, sizeof(double) * n_freq) != hipSuccess)
                return fail(RTX_E_NOMEM, "omega buffer");
            P->n_freq_cap = n_freq;
        }
        std::vector<double> om(n_freq);
        for (int k = 0; k < n_freq; k++) om[k] = 2.0 * kPi * freqs_hz[k];
        HIP_TRY(hipMemcpyAsync(P->omega, om.data(), sizeof(double) * n_freq, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // `om` is pageable host memory
        if (n_pairs > 0) {
            int64_t blocks = (n_pairs * 64 + kBlock - 1) / kBlock;
            hipLaunchKernelGGL(k_rayborn_rho, dim3((unsigned)blocks), dim3(kBlock), 0, s, n_pairs, n_freq, tof,
                               P->omega, (const float2 *)resid, P->rho);
            HIP_TRY(hipGetLastError());
        }
        rho = P->rho;
    }
    rc = pack(P, c, s);
    if (rc) return rc;
    if (n_pairs == 0) return RTX_OK;
    AdjArgs A;
    A.pairs = pairs;
    A.n_pairs = n_pairs;
    A.theta = theta;
    A.status = status;
    A.rho = rho;
    A.weight = weight;
    A.max_steps = max_steps_of(P);
    A.stats = P->stats + 2 * 2 * kMaxBlocks;
    A.err = P->err;
    A.tile = 0;
    A.n_items = n_pairs;
    A.split = 0;
    A.ckpt = P->ckpt;
    A.ckpt_head = P->ckpt_head;
    A.gen = P->gen;
    if (!pairs) {  // all ordered pairs: walk 16 x 16 element-cluster tiles
        const int n = P->ring.n_elem;
        A.tile = std::min(16, n);
        const int64_t nc = (n + A.tile - 1) / A.tile;
        A.n_items = nc * nc * A.tile * A.tile;
        // segments from the fan start's checkpoints (the walk's items come in
        // whole waves: nc^2 t^2 is a multiple of 64 when t = 16)
        A.split = P->ckpt != nullptr && A.tile == 16;
    }
    if (P->opts.prec == RTX_F32C) return launch_adjoint<float, true>(P, A, (float *)grad, s);
    return launch_adjoint<double, false>(P, A, (double *)grad, s);
}

int rtx_plan_stats(rtx_plan P, int64_t *trace_steps, int64_t *trace_rays, int64_t *adjoint_steps)
{
    g_last_error.clear();
    if (!P) return fail(RTX_E_ARG, "null plan");
    HIP_TRY(hipDeviceSynchronize());
    std::vector<unsigned long long> h(6 * kMaxBlocks);
    HIP_TRY(hipMemcpy(h.data(), P->stats, sizeof(unsigned long long) * 6 * kMaxBlocks, hipMemcpyDeviceToHost));
    unsigned long long ts = 0, tr = 0, as = 0;
    for (int region = 0; region < 2; region++)
        for (int b = 0; b < P->stat_blocks[region]; b++) {
            ts += h[(size_t)region * 2 * kMaxBlocks + 2 * b];
            tr += h[(size_t)region * 2 * kMaxBlocks + 2 * b + 1];
        }
    for (int b = 0; b < P->stat_blocks[2]; b++) as += h[4 * (size_t)kMaxBlocks + 2 * b];
    if (trace_steps) *trace_steps = (int64_t)ts;
    if (trace_rays) *trace_rays = (int64_t)tr;
    if (adjoint_steps) *adjoint_steps = (int64_t)as;
    unsigned int e = 0;
    HIP_TRY(hipMemcpy(&e, P->err, sizeof e, hipMemcpyDeviceToHost));
    if (e) return fail(RTX_E_HIP, "an adjoint's node-update queue hit its wait bound; its gradient is incomplete");
    return RTX_OK;
}

int rtx_plan_region_stats(rtx_plan P, int32_t region, int64_t *steps, int64_t *rays)
{
    g_last_error.clear();
    if (!P || region < 0 || region > 2) return fail(RTX_E_ARG, "null plan or region outside 0..2");
    HIP_TRY(hipDeviceSynchronize());
    std::vector<unsigned long long> h(2 * kMaxBlocks);
    HIP_TRY(hipMemcpy(h.data(), P->stats + (size_t)region * 2 * kMaxBlocks, sizeof(unsigned long long) * 2 * kMaxBlocks,
                      hipMemcpyDeviceToHost));
    unsigned long long a = 0, b = 0;
    for (int k = 0; k < P->stat_blocks[region]; k++) {
        a += h[2 * k];
        b += h[2 * k + 1];
    }
    if (steps) *steps = (int64_t)a;
    if (rays) *rays = (int64_t)b;
    return RTX_OK;
}

int rtx_plan_timing(rtx_plan P, int32_t enable)
{
    g_last_error.clear();
    if (!P) return fail(RTX_E_ARG, "null plan");
    HIP_TRY(hipDeviceSynchronize());
    P->timing = enable != 0;
    for (int k = 0; k < RTX_NUM_SLOTS; k++) P->ev_used[k] = 0;
    return RTX_OK;
}

int rtx_plan_timings(rtx_plan P, double *total_ms, int32_t *count)
{
    g_last_error.clear();
    if (!P || !total_ms || !count) return fail(RTX_E_ARG, "null argument");
    HIP_TRY(hipDeviceSynchronize());
    for (int k = 0; k < RTX_NUM_SLOTS; k++) {
        double t = 0;
        for (int i = 0; i < P->ev_used[k]; i++) {
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, P->ev[k][2 * i], P->ev[k][2 * i + 1]));
            t += ms;
        }
        total_ms[k] = t;
        count[k] = P->ev_used[k];
    }
    return RTX_OK;
}

int rtx_plan_set_launch(rtx_plan P, int32_t rays_per_block)
{
    g_last_error.clear();
    if (!P) return fail(RTX_E_ARG, "null plan");
    if (rays_per_block != 64 && rays_per_block != 128 && rays_per_block != 256)
        return fail(RTX_E_ARG, "rays_per_block must be 64, 128 or 256 (got %d)", rays_per_block);
    P->block = rays_per_block;
    return RTX_OK;
}

int rtx_batch_create(rtx_batch *out, const rtx_opts *opts, int32_t weight, int32_t rays_per_block,
                     int32_t n_inst, const rtx_instance *inst)
{
    g_last_error.clear();
    if (!out) return fail(RTX_E_ARG, "out is NULL");
    *out = nullptr;
    if (!opts || !inst || n_inst < 1) return fail(RTX_E_ARG, "need opts and at least one instance");
    if (n_inst > 255) return fail(RTX_E_UNSUPPORTED, "a batch holds at most 255 instances (got %d)", n_inst);
    if (opts->flags & RTX_INTERP_BSPLINE) return fail(RTX_E_UNSUPPORTED, "batches are bilinear-only");
    if (weight != RTX_W_LENGTH && weight != RTX_W_DTDC) return fail(RTX_E_ARG, "unknown weight %d", weight);
    if (rays_per_block == 0) rays_per_block = kBlock;
    if (rays_per_block != 64 && rays_per_block != 128 && rays_per_block != 256)
        return fail(RTX_E_ARG, "rays_per_block must be 64, 128 or 256");
    int n_with_resid = 0;
    for (int k = 0; k < n_inst; k++) {
        const rtx_instance &I = inst[k];
        int rc = check_opts(&I.grid, &I.ring, opts);
        if (rc) return fail(rc, "instance %d: %s", k, g_last_error.c_str());
        if (!I.c || !I.theta || !I.status) return fail(RTX_E_ARG, "instance %d: c, theta and status are required", k);
        int64_t all = (int64_t)I.ring.n_elem * (I.ring.n_elem - 1);
        if (I.n_pairs < 1 || (!I.pairs && I.n_pairs != all))
            return fail(RTX_E_ARG, "instance %d: bad n_pairs %lld", k, (long long)I.n_pairs);
        if ((int64_t)I.grid.nx * I.grid.ny > (1 << 24))
            return fail(RTX_E_ARG, "instance %d: a batch instance's grid holds at most 2^24 nodes", k);
        if (I.resid && !I.grad) return fail(RTX_E_ARG, "instance %d: resid needs grad", k);
        n_with_resid += I.resid != nullptr;
    }
    if (n_with_resid != 0 && n_with_resid != n_inst)
        return fail(RTX_E_ARG, "either every instance has an adjoint residual or none has");
    rtx_batch_s *Bt = new rtx_batch_s();
    Bt->opts = *opts;
    Bt->weight = weight;
    Bt->n_inst = n_inst;
    Bt->block = rays_per_block;
    Bt->adjoint = n_with_resid > 0;
    Bt->inst.assign(inst, inst + n_inst);
    size_t esz = opts->prec == RTX_F32C ? sizeof(float) : sizeof(double);
    size_t bytes = 0;
    std::vector<int64_t> off(n_inst + 1, 0);
    for (int k = 0; k < n_inst; k++) {
        Bt->tab_off.push_back(bytes);
        bytes += ((size_t)(inst[k].grid.nx - 1) * (inst[k].grid.ny - 1) * kCoef * esz + 255) / 256 * 256;
        off[k + 1] = off[k] + inst[k].n_pairs;
    }
    Bt->total_pairs = off[n_inst];
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete Bt;
        return fail(RTX_E_HIP, "no HIP device");
    }
    Bt->n_cu = prop.multiProcessorCount;
    size_t inst_bytes = opts->prec == RTX_F32C ? sizeof(Inst<float>) : sizeof(Inst<double>);
    if (hipMalloc(&Bt->tabs, bytes) != hipSuccess || hipMalloc(&Bt->dinst, inst_bytes * n_inst) != hipSuccess ||
        hipMalloc((void **)&Bt->off, sizeof(int64_t) * (n_inst + 1)) != hipSuccess ||
        hipMalloc((void **)&Bt->remain, sizeof(unsigned int) * 2 * n_inst) != hipSuccess ||
        hipMalloc((void **)&Bt->times, sizeof(unsigned long long) * (1 + 2 * n_inst)) != hipSuccess ||
        hipMalloc((void **)&Bt->stats, sizeof(unsigned long long) * 4 * kMaxBlocks) != hipSuccess ||
        hipMalloc((void **)&Bt->err, sizeof(unsigned int)) != hipSuccess) {
        rtx_batch_destroy(Bt);
        return fail(RTX_E_NOMEM, "batch workspace");
    }
    int rc = RTX_OK;
    if (hipMemset(Bt->err, 0, sizeof(unsigned int)) != hipSuccess) rc = fail(RTX_E_HIP, "clearing the error word failed");
    if (!rc && hipMemcpy(Bt->off, off.data(), sizeof(int64_t) * (n_inst + 1), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(RTX_E_HIP, "upload of instance offsets failed");
    if (!rc) rc = opts->prec == RTX_F32C ? batch_upload<float>(Bt) : batch_upload<double>(Bt);
    if (rc) {
        rtx_batch_destroy(Bt);
        return rc;
    }
    *out = Bt;
    return RTX_OK;
}

int rtx_batch_run(rtx_batch Bt, void *stream)
{
    g_last_error.clear();
    if (!Bt) return fail(RTX_E_ARG, "null batch");
    hipStream_t s = (hipStream_t)stream;
    if (!Bt->exec) {  // capture the whole run once into a graph
        if (!Bt->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&Bt->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(Bt->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = Bt->opts.prec == RTX_F32C ? batch_enqueue<float, true>(Bt, Bt->cap_stream)
                                           : batch_enqueue<double, false>(Bt, Bt->cap_stream);
        hipGraph_t gph = nullptr;
        hipError_t e = hipStreamEndCapture(Bt->cap_stream, &gph);
        if (rc) {
            if (gph) (void)hipGraphDestroy(gph);
            return rc;
        }
        if (e != hipSuccess) return fail(RTX_E_HIP, "graph capture: %s", hipGetErrorString(e));
        Bt->graph = gph;
        HIP_TRY(hipGraphInstantiate(&Bt->exec, Bt->graph, nullptr, nullptr, 0));
    }
    HIP_TRY(hipGraphLaunch(Bt->exec, s));
    return RTX_OK;
}

int rtx_batch_times(rtx_batch Bt, double *fwd_ms, double *done_ms)
{
    g_last_error.clear();
    if (!Bt) return fail(RTX_E_ARG, "null batch");
    HIP_TRY(hipDeviceSynchronize());
    std::vector<unsigned long long> t(1 + 2 * Bt->n_inst);
    HIP_TRY(hipMemcpy(t.data(), Bt->times, sizeof(unsigned long long) * t.size(), hipMemcpyDeviceToHost));
    unsigned int e = 0;
    HIP_TRY(hipMemcpy(&e, Bt->err, sizeof e, hipMemcpyDeviceToHost));
    if (e) return fail(RTX_E_HIP, "an adjoint's node-update queue hit its wait bound; its gradients are incomplete");
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    double ms_per_tick = 1.0 / (double)khz;
    for (int k = 0; k < Bt->n_inst; k++) {
        if (fwd_ms) fwd_ms[k] = (double)(long long)(t[1 + k] - t[0]) * ms_per_tick;
        if (done_ms)
            done_ms[k] = (double)(long long)(t[1 + (Bt->adjoint ? Bt->n_inst : 0) + k] - t[0]) * ms_per_tick;
    }
    return RTX_OK;
}

int rtx_batch_destroy(rtx_batch Bt)
{
    if (!Bt) return RTX_OK;
    (void)hipDeviceSynchronize();
    if (Bt->exec) (void)hipGraphExecDestroy(Bt->exec);
    if (Bt->graph) (void)hipGraphDestroy(Bt->graph);
    if (Bt->cap_stream) (void)hipStreamDestroy(Bt->cap_stream);
    for (void *q : {(void *)Bt->tabs, Bt->dinst, (void *)Bt->off, (void *)Bt->remain, (void *)Bt->times,
                    (void *)Bt->stats, (void *)Bt->err})
        if (q) (void)hipFree(q);
    delete Bt;
    return RTX_OK;
}

}  // extern "C"
