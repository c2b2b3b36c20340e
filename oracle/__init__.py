"""FP64 CPU oracle for linked ray tracing (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark import
this package.  The arithmetic lives in ``oracle_rt.c`` (plain C, FP64), which is
built with gcc into ``liboracle_rt.so`` next to it; this module only marshals
numpy arrays.  It shares no code with the HIP path.

Media are described by a dict:
  {"kind": "grid", "c": float64[ny, nx], "h": h}          (bilinear)
  {"kind": "grid_bspline", "c": float64[ny, nx], "h": h}  (cubic B-spline)
  {"kind": "fisheye", "nx": nx, "ny": ny, "h": h, "c0": c0, "R": R}   (analytic)
  {"kind": "linear", "nx": nx, "ny": ny, "h": h, "c0": c0, "ax": ax, "ay": ay}
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_rt.c")
_SRC3 = os.path.join(_HERE, "oracle_rt3.c")
_LIB = os.path.join(_HERE, "liboracle_rt.so")

LINKED, NOT_CONVERGED, NO_HIT, BAD_INPUT = 0, 1, 2, 3
WARM, FIXED, FAN = 1, 2, 4
HEUN, RK4 = 2, 4
LENGTH, DTDC = 0, 1


def build(force=True, src=_SRC, out=_LIB, src3=_SRC3):
    """Compile the oracle (2-D and 3-D sources) with gcc (no fast-math, no FMA
    contraction)."""
    if not force and os.path.exists(out) and os.path.getmtime(out) >= max(os.path.getmtime(src),
                                                                          os.path.getmtime(src3)):
        return out
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                           "-o", tmp, src, src3, "-lm"])
    os.replace(tmp, out)
    return out


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_bp = C.POINTER(C.c_int8)


def lib():
    if _lib is None:
        build(force=False)
        _load(_LIB)
    return _lib


def _load(path):
    global _lib
    L = C.CDLL(path)
    med = [C.c_int, C.c_int, C.c_int, C.c_double, _dp, _dp]
    L.or_gradient.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
    L.or_trace.argtypes = med + [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                 C.c_int, C.c_int, C.c_int, C.c_int, _ip, _dp, _dp, _dp, _dp, _ip, _bp]
    L.or_march_points.argtypes = med + [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int,
                                        C.c_int, C.c_int, C.c_double, _dp, C.c_int, _dp, _dp]
    L.or_march_free.argtypes = med + [C.c_int, C.c_double, _dp, _dp, C.c_int, _dp]
    L.or_fan_cubic.argtypes = [_dp, _dp, C.c_int, C.c_int, _dp]
    L.or_fan_quintic.argtypes = [_dp, _dp, C.c_int, C.c_int, _dp]
    L.or_interp.argtypes = med + [C.c_int, _dp, _dp, _dp, _dp]
    L.or_weights_row.argtypes = [C.c_int, C.c_int, C.c_double, _dp, C.c_int, C.c_double, C.c_double,
                                 C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_double, _ip, _dp,
                                 C.c_long]
    L.or_weights_row.restype = C.c_long
    L.or_adjoint.argtypes = [C.c_int, C.c_int, C.c_double, _dp, C.c_int, C.c_double, C.c_double, C.c_int,
                             C.c_double, C.c_int, C.c_int, _ip, _dp, _bp, _dp, C.c_int, _dp]
    L.or_rayborn_rho.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp]
    L.or_paraxial.argtypes = med + [C.c_int, C.c_double, C.c_double, C.c_int, C.c_double, C.c_int, C.c_int, _ip,
                                     _dp, _dp, _dp, _dp, _ip, _bp]
    med3 = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _dp, _dp]
    L.or3_trace.argtypes = med3 + [C.c_int, _dp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                   C.c_int, _ip, _dp, _dp, _dp, _dp, _ip, _bp]
    L.or3_march_free.argtypes = med3 + [C.c_int, C.c_double, _dp, _dp, C.c_int, _dp]
    L.or3_jac0.argtypes = [C.c_int, _dp, C.c_double, C.c_int, C.c_int, _dp, _dp, _dp]
    L.or3_interp.argtypes = med3 + [C.c_int, _dp, _dp, _dp]
    L.or3_misfit.argtypes = med3 + [C.c_int, _dp, C.c_int, C.c_double, C.c_int, C.c_int, _dp, _dp, _dp]
    L.or_sart.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int64), _ip, _dp, _dp, _dp, C.c_int, C.c_double]
    _lib = L


class use_library:
    """Context manager that swaps in another build of the oracle (used by the
    test that plants mistakes in a copy of the oracle source)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = None
        _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _b(a):
    return a.ctypes.data_as(_bp)


def _medium_args(medium):
    kind = medium["kind"]
    h = float(medium["h"])
    if kind in ("grid", "grid_bspline"):
        c = np.ascontiguousarray(medium["c"], dtype=np.float64)
        ny, nx = c.shape
        return [0 if kind == "grid" else 3, nx, ny, h, _d(c), None], (c,)
    par = np.zeros(4)
    if kind == "fisheye":
        par[:2] = (medium["c0"], medium["R"])
        code = 1
    elif kind == "linear":
        par[:3] = (medium["c0"], medium["ax"], medium["ay"])
        code = 2
    else:
        raise ValueError(kind)
    return [code, int(medium.get("nx", 8)), int(medium.get("ny", 8)), h, None, _d(par)], (par,)


def grid_medium(c, h, interp="bilinear"):
    kind = {"bilinear": "grid", "bspline": "grid_bspline"}[interp]
    return {"kind": kind, "c": np.asarray(c, dtype=np.float64), "h": float(h)}


def gradient(c):
    """Per-index second-order differences of c [ny, nx] -> (gx, gy)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    ny, nx = c.shape
    gx = np.empty_like(c)
    gy = np.empty_like(c)
    if lib().or_gradient(nx, ny, _d(c), _d(gx), _d(gy)):
        raise ValueError("grid too small")
    return gx, gy


def interp(medium, pts):
    """c and per-pixel gradient at pixel points pts [n, 2] (ring-centred)."""
    args, keep = _medium_args(medium)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n = pts.shape[0]
    cv, gx, gy = np.empty(n), np.empty(n), np.empty(n)
    if lib().or_interp(*args, n, _d(pts), _d(cv), _d(gx), _d(gy)):
        raise ValueError("bad medium")
    return cv, gx, gy


def _integ_code(integ):
    return {"heun": HEUN, "rk4": RK4, HEUN: HEUN, RK4: RK4}[integ]


def trace(medium, ring, pairs, theta=None, integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
          max_steps=0, fixed=False, warm=False, fan=False):
    """Linked (or fixed-angle) tracing of pairs [n, 2] = (emitter, receiver).

    ring = (n_elem, radius_m, phi0).  fan=True: fan start (needs all ordered
    pairs in canonical order).  Returns a dict of numpy arrays:
    theta, tof (s), len (m), miss_px, n_marches, status."""
    args, keep = _medium_args(medium)
    n_elem, radius, phi0 = ring
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    n = pairs.shape[0]
    th = np.zeros(n) if theta is None else np.array(theta, dtype=np.float64).copy()
    T, L, miss = np.empty(n), np.empty(n), np.empty(n)
    nm = np.empty(n, dtype=np.int32)
    st = np.empty(n, dtype=np.int8)
    flags = (FIXED if fixed else 0) | (WARM if warm else 0) | (FAN if fan else 0)
    rc = lib().or_trace(*args, int(n_elem), float(radius), float(phi0), _integ_code(integ), float(ds_px),
                        float(tol_px), int(max_marches), int(max_steps), flags, n, _i(pairs), _d(th), _d(T),
                        _d(L), _d(miss), _i(nm), _b(st))
    if rc:
        raise ValueError("bad arguments")
    return {"theta": th, "tof": T, "len": L, "miss_px": miss, "n_marches": nm, "status": st}


def march_points(medium, ring, e, r, theta, integ="rk4", ds_px=0.25, max_steps=0, cap=1 << 16):
    """Samples of one fixed-angle march: (points [M+1, 2] px, ds', misfit g)."""
    args, keep = _medium_args(medium)
    n_elem, radius, phi0 = ring
    pts = np.empty((cap, 2))
    dsp, g = C.c_double(0), C.c_double(0)
    n = lib().or_march_points(*args, int(n_elem), float(radius), float(phi0), _integ_code(integ), float(ds_px),
                              int(max_steps), int(e), int(r), float(theta), _d(pts), cap, C.byref(dsp),
                              C.byref(g))
    if n < 0:
        return None, float("nan"), float("nan")
    return pts[: min(n, cap)].copy(), dsp.value, g.value


def march_free(medium, x0_px, d0, n_steps, integ="rk4", ds_px=0.25):
    """n_steps steps from x0 (pixels) along d0 without a ring: points [n+1, 2]."""
    args, keep = _medium_args(medium)
    x0 = np.ascontiguousarray(x0_px, dtype=np.float64)
    d0 = np.ascontiguousarray(d0, dtype=np.float64)
    pts = np.empty((n_steps + 1, 2))
    if lib().or_march_free(*args, _integ_code(integ), float(ds_px), _d(x0), _d(d0), int(n_steps), _d(pts)):
        raise ValueError("bad medium")
    return pts


def weights_row(c, h, ring, e, r, theta, integ="rk4", ds_px=0.25, max_steps=0):
    """One system-matrix row (cols int32 sorted, vals float64 metres)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    ny, nx = c.shape
    n_elem, radius, phi0 = ring
    cap = 1 << 15
    while True:
        cols = np.empty(cap, dtype=np.int32)
        vals = np.empty(cap)
        nnz = lib().or_weights_row(nx, ny, float(h), _d(c), int(n_elem), float(radius), float(phi0),
                                   _integ_code(integ), float(ds_px), int(max_steps), int(e), int(r),
                                   float(theta), _i(cols), _d(vals), cap)
        if nnz < 0:
            return None, None
        if nnz <= cap:
            return cols[:nnz].copy(), vals[:nnz].copy()
        cap = int(nnz)


def weights_csr(c, h, ring, pairs, theta, **kw):
    """Whole system matrix as (rowptr int64, cols int32, vals float64)."""
    rows = [weights_row(c, h, ring, int(e), int(r), float(t), **kw) for (e, r), t in zip(pairs, theta)]
    counts = [0 if cc is None else len(cc) for cc, _ in rows]
    rowptr = np.zeros(len(rows) + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(counts)
    cols = np.concatenate([cc for cc, _ in rows if cc is not None] or [np.empty(0, np.int32)])
    vals = np.concatenate([v for cc, v in rows if cc is not None] or [np.empty(0)])
    return rowptr, cols, vals


def adjoint(c, h, ring, pairs, theta, rho, weight="length", status=None, integ="rk4", ds_px=0.25,
            max_steps=0):
    """grad [ny, nx] = sum_i rho_i sum_m w_m h kappa_m phi_j(p_m)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    ny, nx = c.shape
    n_elem, radius, phi0 = ring
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    st = None if status is None else np.ascontiguousarray(status, dtype=np.int8)
    grad = np.zeros((ny, nx))
    mode = {"length": LENGTH, "dtdc": DTDC}[weight]
    rc = lib().or_adjoint(nx, ny, float(h), _d(c), int(n_elem), float(radius), float(phi0), _integ_code(integ),
                          float(ds_px), int(max_steps), pairs.shape[0], _i(pairs), _d(theta),
                          None if st is None else _b(st), _d(rho), mode, _d(grad))
    if rc:
        raise ValueError("bad arguments")
    return grad


def fan_cubic(G, TH, a):
    """Cubic refinement of a fan seed with bracket (a, a+1): the angle, or None
    when the secant's linear interpolation stands."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    TH = np.ascontiguousarray(TH, dtype=np.float64)
    out = np.zeros(1)
    ok = lib().or_fan_cubic(_d(G), _d(TH), len(G), int(a), _d(out))
    return float(out[0]) if ok else None


def fan_quintic(G, TH, a):
    """Quintic estimate of a fan seed with bracket (a, a+1) from the samples
    a-2..a+3 (the first round's second ray): the angle, or None."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    TH = np.ascontiguousarray(TH, dtype=np.float64)
    out = np.zeros(1)
    ok = lib().or_fan_quintic(_d(G), _d(TH), len(G), int(a), _d(out))
    return float(out[0]) if ok else None


def rayborn_rho(tof, freqs, resid):
    """rho_i = sum_k w_k Im(exp(-i w_k T_i) r_ik), w_k = 2 pi f_k."""
    tof = np.ascontiguousarray(tof, dtype=np.float64)
    freqs = np.ascontiguousarray(freqs, dtype=np.float64)
    r = np.ascontiguousarray(resid).astype(np.complex128)
    n, nf = r.shape
    ri = np.ascontiguousarray(r.view(np.float64).reshape(n, nf, 2))
    rho = np.empty(n)
    lib().or_rayborn_rho(n, nf, _d(tof), _d(freqs), _d(ri), _d(rho))
    return rho


def sart(rowptr, cols, vals, b, x0, n_iter, lam=1.0):
    """n_iter SART iterations on W x = b (W as CSR) from x0; returns x."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True).ravel()
    if len(rowptr) != len(b) + 1 or len(cols) != rowptr[-1] or len(vals) != rowptr[-1]:
        raise ValueError("inconsistent CSR")
    rc = lib().or_sart(len(b), len(x), rowptr.ctypes.data_as(C.POINTER(C.c_int64)), _i(cols), _d(vals), _d(b),
                       _d(x), int(n_iter), float(lam))
    if rc:
        raise ValueError("column index out of range")
    return x


def paraxial(medium, ring, pairs, theta, integ="rk4", ds_px=0.25, max_steps=0):
    """Paraxial ray quantities at fixed launch angles: dict of dgdth, jac (m/rad),
    amp (1/sqrt(m)), kmah (int32) and status."""
    args, keep = _medium_args(medium)
    n_elem, radius, phi0 = ring
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    n = pairs.shape[0]
    out = {k: np.empty(n) for k in ("dgdth", "jac", "amp")}
    out["kmah"] = np.empty(n, np.int32)
    out["status"] = np.empty(n, np.int8)
    rc = lib().or_paraxial(*args, int(n_elem), float(radius), float(phi0), _integ_code(integ), float(ds_px),
                           int(max_steps), n, _i(pairs), _d(theta), _d(out["dgdth"]), _d(out["jac"]),
                           _d(out["amp"]), _i(out["kmah"]), _b(out["status"]))
    if rc:
        raise ValueError("bad medium")
    return out


# ------------------------------------------------------------------- 3-D ----
# Volumes: {"kind": "grid", "c": float64[nz, ny, nx], "h": h} (trilinear),
# {"kind": "fisheye", "n": (nx, ny, nz), "h": h, "c0": c0, "R": R} or
# {"kind": "linear", "n": (nx, ny, nz), "h": h, "c0": c0, "a": (ax, ay, az)}.
def _medium3_args(medium):
    kind, h = medium["kind"], float(medium["h"])
    if kind == "grid":
        c = np.ascontiguousarray(medium["c"], dtype=np.float64)
        nz, ny, nx = c.shape
        return [0, nx, ny, nz, h, _d(c), None], (c,)
    par = np.zeros(4)
    if kind == "fisheye":
        par[:2] = (medium["c0"], medium["R"])
        code = 1
    elif kind == "linear":
        par[0] = medium["c0"]
        par[1:4] = medium["a"]
        code = 2
    else:
        raise ValueError(kind)
    nx, ny, nz = medium.get("n", (8, 8, 8))
    return [code, int(nx), int(ny), int(nz), h, None, _d(par)], (par,)


def trace3(medium, elem, pairs, u=None, integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30, max_steps=0,
           warm=False, fixed=False):
    """3-D tracing between elements elem [n][3] (metres from the grid centre,
    on one sphere): dict of u [n, 2], tof, len, miss_px, n_marches, status."""
    args, keep = _medium3_args(medium)
    elem = np.ascontiguousarray(elem, dtype=np.float64)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    n = pairs.shape[0]
    uu = np.zeros((n, 2)) if u is None else np.array(u, dtype=np.float64, copy=True).reshape(n, 2)
    out = {k: np.empty(n) for k in ("tof", "len", "miss_px")}
    nm = np.empty(n, np.int32)
    st = np.empty(n, np.int8)
    flags = (WARM if warm else 0) | (FIXED if fixed else 0)
    rc = lib().or3_trace(*args, elem.shape[0], _d(elem), _integ_code(integ), float(ds_px), float(tol_px),
                         int(max_marches), int(max_steps), flags, n, _i(pairs), _d(uu), _d(out["tof"]),
                         _d(out["len"]), _d(out["miss_px"]), _i(nm), _b(st))
    if rc:
        raise ValueError("bad medium")
    out.update(u=uu, n_marches=nm, status=st)
    return out


def march3_free(medium, x0_px, d0, n_steps, integ="rk4", ds_px=0.25):
    """n_steps free steps from pixel point x0 along d0: points [n+1, 3] (pixels)."""
    args, keep = _medium3_args(medium)
    x0 = np.ascontiguousarray(x0_px, dtype=np.float64)
    d0 = np.ascontiguousarray(d0, dtype=np.float64)
    pts = np.empty((n_steps + 1, 3))
    if lib().or3_march_free(*args, _integ_code(integ), float(ds_px), _d(x0), _d(d0), int(n_steps), _d(pts)):
        raise ValueError("bad medium")
    return pts


def jac0_3(elem, h, e, r, u):
    """Homogeneous-medium Jacobian dg/du [2, 2] and the launch direction at u."""
    elem = np.ascontiguousarray(elem, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    J, d = np.empty(4), np.empty(3)
    if lib().or3_jac0(elem.shape[0], _d(elem), float(h), int(e), int(r), _d(u), _d(J), _d(d)):
        raise ValueError("bad element")
    return J.reshape(2, 2), d


def interp3(medium, pts):
    args, keep = _medium3_args(medium)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    cv, G = np.empty(len(pts)), np.empty((len(pts), 3))
    if lib().or3_interp(*args, len(pts), _d(pts), _d(cv), _d(G)):
        raise ValueError("bad medium")
    return cv, G


def misfit3(medium, elem, e, r, u, integ="rk4", ds_px=0.25):
    """One fixed-direction ray: (status, g [2], interception q [3] pixels)."""
    args, keep = _medium3_args(medium)
    elem = np.ascontiguousarray(elem, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    g, q = np.empty(2), np.empty(3)
    st = lib().or3_misfit(*args, elem.shape[0], _d(elem), _integ_code(integ), float(ds_px), int(e), int(r), _d(u),
                          _d(g), _d(q))
    if st < 0:
        raise ValueError("bad arguments")
    return st, g, q
