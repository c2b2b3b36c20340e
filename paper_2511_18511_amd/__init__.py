"""MI355X-native linked ray tracing for ring-array ultrasound tomography.

Two-point (shooting) ray tracing of every emitter/receiver pair through a gridded
sound-speed map, with ray linking on the launch angle, travel time, path length
and the adjoint of the path weights (arXiv 2511.18511, Sec. 3.1-3.4).  All
computation runs in the HIP kernels of ``librtx.so``; this package only moves
torch tensors (device memory) and the current stream across the C ABI.
"""
import ctypes as C

import torch

from . import _binding as B
from ._binding import (  # noqa: F401
    RTX_F32C, RTX_F64, RTX_HEUN, RTX_RK4, RTX_RAY_BAD_INPUT, RTX_RAY_LINKED, RTX_RAY_NO_HIT,
    RTX_RAY_NOT_CONVERGED, RTX_W_DTDC, RTX_W_LENGTH, RtxError,
)

PRECISIONS = {"f64": B.RTX_F64, "f32c": B.RTX_F32C}
INTEGRATORS = {"heun": B.RTX_HEUN, "rk4": B.RTX_RK4}
INTERPOLATIONS = {"bilinear": 0, "bspline": B.RTX_INTERP_BSPLINE}


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_check(t, dtype, shape=None, name="tensor"):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA(HIP) tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """Geometry + options + device workspace (the packed medium).

    Lengths are metres; ``ds_px``/``tol_px`` are in grid pixels.  ``interp``
    is "bilinear" (all calls) or "bspline" (the cubic B-spline of Sec. 3.3:
    tracing only, no adjoint or path weights)."""

    def __init__(self, nx, ny, h, n_elem, radius, phi0=0.0, prec="f32c", integ="rk4", ds_px=0.25, tol_px=1e-3,
                 max_marches=30, max_steps=0, max_pairs=None, interp="bilinear"):
        self.nx, self.ny, self.h = int(nx), int(ny), float(h)
        self.n_elem, self.radius, self.phi0 = int(n_elem), float(radius), float(phi0)
        self._w_hint = {}  # rows -> entries to allocate first in weights()
        self.prec = prec
        self.interp = interp
        self._interp_flag = INTERPOLATIONS[interp]
        self.real = torch.float32 if prec == "f32c" else torch.float64
        self.n_all = self.n_elem * (self.n_elem - 1)
        self.max_pairs = int(max_pairs or self.n_all)
        self._opts = dict(integ=integ, ds_px=ds_px, tol_px=tol_px, max_marches=max_marches, max_steps=max_steps)
        self._grid = B.rtx_grid(self.nx, self.ny, self.h)
        self._ring = B.rtx_ring(self.n_elem, self.radius, self.phi0)
        self._handle = B.rtx_plan_create(self._grid, self._ring, self._make_opts(0), self.max_pairs)

    def _make_opts(self, flags, **over):
        o = dict(self._opts, **over)
        return B.rtx_opts(PRECISIONS[self.prec], INTEGRATORS[o["integ"]], float(o["ds_px"]), float(o["tol_px"]),
                          int(o["max_marches"]), int(o["max_steps"]), int(flags) | self._interp_flag)

    def _apply(self, flags, **over):
        B.rtx_plan_set_opts(self._handle, self._make_opts(flags, **over))

    def close(self):
        if getattr(self, "_handle", None):
            B.rtx_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def set_medium(self, c):
        """Packs c (float64 [ny, nx] on the device) for later calls with c=None."""
        _dev_check(c, torch.float64, (self.ny, self.nx), "c")
        B.rtx_set_medium(self._handle, _ptr(c), _stream())

    def _pairs(self, pairs):
        if pairs is None:
            return None, self.n_all
        _dev_check(pairs, torch.int32, None, "pairs")
        return pairs, pairs.shape[0]

    def trace(self, c=None, pairs=None, theta=None, warm=False, fixed=False, out=None, weights=False, fan=False,
              **over):
        """Linked (or fixed-angle) tracing.  Returns a dict of device tensors:
        theta, tof (s), len (m), miss_px, n_marches, status, and with
        weights=True the system matrix of the traced rays (w_rowptr, w_col,
        w_val; see weights()).  fan=True: cold start seeded from each emitter's
        fan of straight rays (all ordered pairs only)."""
        if c is not None:
            _dev_check(c, torch.float64, (self.ny, self.nx), "c")
        pairs, n = self._pairs(pairs)
        dev = torch.device("cuda", torch.cuda.current_device())
        if out is None:
            out = {
                "theta": torch.zeros(n, dtype=torch.float64, device=dev),
                "tof": torch.empty(n, dtype=torch.float64, device=dev),
                "len": torch.empty(n, dtype=torch.float64, device=dev),
                "miss_px": torch.empty(n, dtype=torch.float64, device=dev),
                "n_marches": torch.empty(n, dtype=torch.int32, device=dev),
                "status": torch.empty(n, dtype=torch.int8, device=dev),
            }
        if theta is not None:
            out["theta"].copy_(theta)
        flags = (B.RTX_WARM_START if warm else 0) | (B.RTX_FIXED_ANGLE if fixed else 0) | \
            (B.RTX_FAN_START if fan else 0)
        self._apply(flags, **over)
        B.rtx_trace_rays(self._handle, _ptr(c), _ptr(pairs), n, _ptr(out["theta"]), _ptr(out.get("tof")),
                         _ptr(out.get("len")), _ptr(out.get("miss_px")), _ptr(out.get("n_marches")),
                         _ptr(out["status"]), None, None, None, 0, _stream())
        if weights:
            out["w_rowptr"], out["w_col"], out["w_val"] = self.weights(out["theta"], pairs=pairs, **over)
        return out

    def march(self, x0, d0, n_steps, c=None, **over):
        """Free march without the ring: rays from x0 (float64 [n, 2] device,
        metres from the grid centre) along d0 (float64 [n, 2], any length),
        n_steps steps each.  Returns float64 [n, n_steps + 1, 2] positions in
        metres (NaN once a ray has left the grid)."""
        if c is not None:
            _dev_check(c, torch.float64, (self.ny, self.nx), "c")
        n = x0.shape[0]
        _dev_check(x0, torch.float64, (n, 2), "x0")
        _dev_check(d0, torch.float64, (n, 2), "d0")
        pts = torch.empty(n, int(n_steps) + 1, 2, dtype=torch.float64, device=x0.device)
        self._apply(0, **over)
        B.rtx_march_free(self._handle, _ptr(c), n, _ptr(x0), _ptr(d0), int(n_steps), _ptr(pts), _stream())
        return pts

    def paraxial(self, theta, pairs=None, c=None, **over):
        """Paraxial ray along the rays at the given launch angles (Sec. 3.5):
        dict of device tensors dgdth, jac (m/rad), amp (1/sqrt(m)), kmah
        (int32) and status."""
        if c is not None:
            _dev_check(c, torch.float64, (self.ny, self.nx), "c")
        pairs, n = self._pairs(pairs)
        _dev_check(theta, torch.float64, (n,), "theta")
        dev = theta.device
        out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("dgdth", "jac", "amp")}
        out["kmah"] = torch.empty(n, dtype=torch.int32, device=dev)
        out["status"] = torch.empty(n, dtype=torch.int8, device=dev)
        self._apply(0, **over)
        B.rtx_paraxial(self._handle, _ptr(c), _ptr(pairs), n, _ptr(theta), _ptr(out["dgdth"]), _ptr(out["jac"]),
                       _ptr(out["amp"]), _ptr(out["kmah"]), _ptr(out["status"]), _stream())
        return out

    def sart(self, w_rowptr, w_col, w_val, b, x=None, n_iter=10, lam=1.0):
        """SART iterations (Sec. 3.1) on W x = b with W as returned by
        weights()/trace(weights=True); x (float64 [ny, nx] device, updated in
        place) starts at zero when None.  Returns x."""
        n = b.shape[0]
        _dev_check(w_rowptr, torch.int64, (n + 1,), "w_rowptr")
        _dev_check(w_col, torch.int32, None, "w_col")
        _dev_check(w_val, self.real, (w_col.shape[0],), "w_val")
        _dev_check(b, torch.float64, (n,), "b")
        if x is None:
            x = torch.zeros(self.ny, self.nx, dtype=torch.float64, device=b.device)
        _dev_check(x, torch.float64, (self.ny, self.nx), "x")
        B.rtx_sart(self._handle, n, w_col.shape[0], _ptr(w_rowptr), _ptr(w_col), _ptr(w_val), _ptr(b), _ptr(x),
                   int(n_iter), float(lam), _stream())
        return x

    def weights(self, theta, pairs=None, **over):
        """System-matrix rows W_ij = h sum_m w_m phi_j(p_m) of the rays traced at
        the given angles, as CSR device tensors (rowptr int64 [n+1], col int32
        ascending per row, val float/double per precision, metres).  Rows of
        rays that do not reach the ring are empty."""
        pairs, n = self._pairs(pairs)
        _dev_check(theta, torch.float64, (n,), "theta")
        dev = theta.device
        th = theta.clone()
        st = torch.empty(n, dtype=torch.int8, device=dev)
        rowptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
        self._apply(B.RTX_FIXED_ANGLE, **over)
        # One call when the entries fit a first guess: the previous call's
        # count plus 10 %, else ~2.5 entries per pixel of a path as long as the
        # ring's diameter, with 50 % slack.  A call that does not fit leaves the
        # exact row pointers in rowptr, and a second call fills exact buffers.
        cap = self._w_hint.get(n) or n * (int(3.75 * 2 * self.radius / self.h) + 8)
        col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(cap, 1), dtype=self.real, device=dev)
        try:
            B.rtx_trace_rays(self._handle, None, _ptr(pairs), n, _ptr(th), None, None, None, None, _ptr(st),
                             _ptr(rowptr), _ptr(col), _ptr(val), cap, _stream())
            nnz = int(rowptr[-1].item())
        except B.RtxError as e:
            if e.code != B.RTX_E_CAPACITY:
                raise
            nnz = int(rowptr[-1].item())
            col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
            val = torch.empty(max(nnz, 1), dtype=self.real, device=dev)
            B.rtx_trace_rays(self._handle, None, _ptr(pairs), n, _ptr(th), None, None, None, None, _ptr(st),
                             _ptr(rowptr), _ptr(col), _ptr(val), nnz, _stream())
        self._w_hint[n] = int(1.1 * nnz) + n
        if col.shape[0] > 1.25 * nnz + 4096:  # give the slack back
            return rowptr, col[:nnz].clone(), val[:nnz].clone()
        return rowptr, col[:nnz], val[:nnz]

    def adjoint(self, theta, status, resid, weight="length", c=None, pairs=None, tof=None, freqs_hz=None,
                grad=None, **over):
        """grad[ny, nx] += sum_i rho_i sum_m w_m h kappa_m phi_j(p_m) along the rays
        at the given angles (kappa = 1 for "length", -1/c^2 for "dtdc").  resid is
        float64 [n] (rho) or complex64 [n, n_freq] with freqs_hz (ray-Born-style
        phase data, needs tof)."""
        pairs, n = self._pairs(pairs)
        _dev_check(theta, torch.float64, (n,), "theta")
        _dev_check(status, torch.int8, (n,), "status")
        if grad is None:
            grad = torch.zeros(self.ny, self.nx, dtype=self.real, device=theta.device)
        _dev_check(grad, self.real, (self.ny, self.nx), "grad")
        if resid.dtype == torch.complex64:
            if tof is None or freqs_hz is None:
                raise ValueError("complex residuals need tof and freqs_hz")
            _dev_check(resid, torch.complex64, (n, len(freqs_hz)), "resid")
            kind, nf = B.RTX_RESID_RAYBORN_C64, len(freqs_hz)
        else:
            _dev_check(resid, torch.float64, (n,), "resid")
            kind, nf = B.RTX_RESID_REAL, 0
        self._apply(0, **over)
        wcode = {"length": B.RTX_W_LENGTH, "dtdc": B.RTX_W_DTDC}[weight]
        B.rtx_tof_adjoint(self._handle, _ptr(c), _ptr(pairs), n, _ptr(theta), _ptr(status), _ptr(tof), _ptr(resid),
                          kind, freqs_hz, nf, wcode, _ptr(grad), _stream())
        return grad

    def stats(self):
        """(trace steps, trace rays, adjoint steps) of the last calls."""
        return B.rtx_plan_stats(self._handle)

    def region_stats(self, region):
        """(steps, rays) of one kernel of the last call: 0 = trace (the fixed
        straight pass under a fan start), 1 = fan linking pass, 2 = adjoint."""
        return B.rtx_plan_region_stats(self._handle, region)

    def timing(self, enable=True):
        """Starts (resets) or stops per-kernel HIP-event timing of this plan."""
        B.rtx_plan_timing(self._handle, enable)

    def timings(self):
        """{slot: (total ms, launches)} since timing(True); slots: pack, trace,
        fan_seed, fan_link, adjoint."""
        t, n = B.rtx_plan_timings(self._handle)
        names = ("pack", "trace", "fan_seed", "fan_link", "adjoint")
        return {k: (t[i], n[i]) for i, k in enumerate(names)}

    def set_launch(self, rays_per_block):
        """Rays (threads) per block of the persistent kernels: 64, 128 or 256."""
        B.rtx_plan_set_launch(self._handle, rays_per_block)
        self.rays_per_block = int(rays_per_block)


class Batch:
    """Independent (medium, ring) problems traced together: one persistent trace
    kernel over all pairs of all instances (+ one adjoint kernel when residuals
    are given), captured once into a HIP graph and replayed by run().

    instances: list of dicts with c (float64 [ny, nx] device), h, n_elem,
    radius, phi0 (optional), and optionally resid (float64 [n_pairs] device).
    Outputs per instance (device tensors, reused across runs): theta, tof, len,
    miss_px, n_marches, status, and grad with resid."""

    def __init__(self, instances, prec="f32c", integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
                 max_steps=0, weight="length", rays_per_block=256, warm=False):
        self.prec = prec
        self.real = torch.float32 if prec == "f32c" else torch.float64
        self.opts = B.rtx_opts(PRECISIONS[prec], INTEGRATORS[integ], float(ds_px), float(tol_px), int(max_marches),
                               int(max_steps), B.RTX_WARM_START if warm else 0)
        self.inst = []
        descs = []
        for spec in instances:
            c = spec["c"]
            _dev_check(c, torch.float64, None, "c")
            ny, nx = c.shape
            n_elem = int(spec["n_elem"])
            n = n_elem * (n_elem - 1)
            dev = c.device
            o = {
                "c": c,
                "theta": torch.zeros(n, dtype=torch.float64, device=dev) if spec.get("theta") is None
                else spec["theta"].clone(),
                "tof": torch.empty(n, dtype=torch.float64, device=dev),
                "len": torch.empty(n, dtype=torch.float64, device=dev),
                "miss_px": torch.empty(n, dtype=torch.float64, device=dev),
                "n_marches": torch.empty(n, dtype=torch.int32, device=dev),
                "status": torch.empty(n, dtype=torch.int8, device=dev),
            }
            if spec.get("resid") is not None:
                _dev_check(spec["resid"], torch.float64, (n,), "resid")
                o["resid"] = spec["resid"]
                o["grad"] = torch.zeros(ny, nx, dtype=self.real, device=dev)
            self.inst.append(o)
            descs.append(B.rtx_instance(
                B.rtx_grid(nx, ny, float(spec["h"])), B.rtx_ring(n_elem, float(spec["radius"]),
                                                                 float(spec.get("phi0", 0.0))),
                c.data_ptr(), None, n, o["theta"].data_ptr(), o["tof"].data_ptr(), o["len"].data_ptr(),
                o["miss_px"].data_ptr(), o["n_marches"].data_ptr(), o["status"].data_ptr(),
                o["resid"].data_ptr() if "resid" in o else None, o["grad"].data_ptr() if "grad" in o else None))
        wcode = {"length": B.RTX_W_LENGTH, "dtdc": B.RTX_W_DTDC}[weight]
        self._handle = B.rtx_batch_create(self.opts, wcode, rays_per_block, descs)
        self.n_pairs = sum(int(o["tof"].numel()) for o in self.inst)

    def run(self):
        """Enqueues one run on the current stream (the adjoint accumulates into
        each instance's grad: zero them first to get one run's gradient)."""
        B.rtx_batch_run(self._handle, _stream())

    def times(self):
        """Per-instance completion of the last run, ms from its start:
        (forward linked, forward + adjoint done)."""
        return B.rtx_batch_times(self._handle, len(self.inst))

    def close(self):
        if getattr(self, "_handle", None):
            B.rtx_batch_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan3:
    """3-D tracing between point transducers on a sphere (hemispherical arrays)
    through a sound-speed volume, with Broyden-like linking (Sec. 3.4).

    elem: float64 [n_elem, 3] host array (metres from the grid centre, all on
    one sphere); lengths in metres, ``ds_px``/``tol_px`` in grid pixels."""

    def __init__(self, nx, ny, nz, h, elem, prec="f32c", integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
                 max_steps=0, max_pairs=None):
        import numpy as np

        self.nx, self.ny, self.nz, self.h = int(nx), int(ny), int(nz), float(h)
        self.elem = np.ascontiguousarray(elem, dtype=np.float64).reshape(-1, 3)
        self.n_elem = self.elem.shape[0]
        self.prec = prec
        self.n_all = self.n_elem * (self.n_elem - 1)
        self.max_pairs = int(max_pairs or self.n_all)
        self._opts = dict(integ=integ, ds_px=ds_px, tol_px=tol_px, max_marches=max_marches, max_steps=max_steps)
        self._grid = B.rtx3_grid(self.nx, self.ny, self.nz, self.h)
        self._handle = B.rtx3_plan_create(self._grid, self.elem, self._make_opts(0), self.max_pairs)

    def _make_opts(self, flags, **over):
        o = dict(self._opts, **over)
        return B.rtx_opts(PRECISIONS[self.prec], INTEGRATORS[o["integ"]], float(o["ds_px"]), float(o["tol_px"]),
                          int(o["max_marches"]), int(o["max_steps"]), int(flags))

    def close(self):
        if getattr(self, "_handle", None):
            B.rtx3_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_medium(self, c):
        _dev_check(c, torch.float64, (self.nz, self.ny, self.nx), "c")
        B.rtx3_set_medium(self._handle, _ptr(c), _stream())

    def trace(self, c=None, pairs=None, u=None, warm=False, fixed=False, **over):
        """Linked (or warm-started, or fixed-direction) tracing: dict of device
        tensors u [n, 2], tof (s), len (m), miss_px, n_marches, status."""
        if c is not None:
            _dev_check(c, torch.float64, (self.nz, self.ny, self.nx), "c")
        if pairs is None:
            n = self.n_all
        else:
            _dev_check(pairs, torch.int32, None, "pairs")
            n = pairs.shape[0]
        dev = torch.device("cuda", torch.cuda.current_device())
        out = {
            "u": torch.zeros(n, 2, dtype=torch.float64, device=dev),
            "tof": torch.empty(n, dtype=torch.float64, device=dev),
            "len": torch.empty(n, dtype=torch.float64, device=dev),
            "miss_px": torch.empty(n, dtype=torch.float64, device=dev),
            "n_marches": torch.empty(n, dtype=torch.int32, device=dev),
            "status": torch.empty(n, dtype=torch.int8, device=dev),
        }
        if u is not None:
            out["u"].copy_(u)
        flags = (B.RTX_WARM_START if warm else 0) | (B.RTX_FIXED_ANGLE if fixed else 0)
        B.rtx3_plan_set_opts(self._handle, self._make_opts(flags, **over))
        B.rtx3_trace_rays(self._handle, _ptr(c), _ptr(pairs), n, _ptr(out["u"]), _ptr(out["tof"]), _ptr(out["len"]),
                          _ptr(out["miss_px"]), _ptr(out["n_marches"]), _ptr(out["status"]), _stream())
        return out

    def march(self, x0, d0, n_steps, c=None, **over):
        """Free march: float64 [n, n_steps + 1, 3] positions in metres."""
        if c is not None:
            _dev_check(c, torch.float64, (self.nz, self.ny, self.nx), "c")
        n = x0.shape[0]
        _dev_check(x0, torch.float64, (n, 3), "x0")
        _dev_check(d0, torch.float64, (n, 3), "d0")
        pts = torch.empty(n, int(n_steps) + 1, 3, dtype=torch.float64, device=x0.device)
        B.rtx3_plan_set_opts(self._handle, self._make_opts(0, **over))
        B.rtx3_march_free(self._handle, _ptr(c), n, _ptr(x0), _ptr(d0), int(n_steps), _ptr(pts), _stream())
        return pts

    def stats(self):
        """(RK steps, rays) of the last trace call."""
        return B.rtx3_plan_stats(self._handle)


def trace_rays(c, h, n_elem, radius, phi0=0.0, pairs=None, theta=None, warm=False, fixed=False, **opts):
    """One-shot linked tracing of a float64 [ny, nx] device medium."""
    ny, nx = c.shape
    plan = Plan(nx, ny, h, n_elem, radius, phi0, **opts)
    try:
        return plan.trace(c, pairs=pairs, theta=theta, warm=warm, fixed=fixed)
    finally:
        torch.cuda.current_stream().synchronize()
        plan.close()


class ToF(torch.autograd.Function):
    """T = ToF(c): linked travel times of all pairs of ``plan`` through c.

    forward: linked tracing, warm-started from ``state["theta"]`` when present
    (the linked angles are stored back into ``state``); backward: the
    frozen-path travel-time gradient dT/dc (adjoint with kappa = -1/c^2)."""

    @staticmethod
    def forward(ctx, c, plan, state=None, pairs=None):
        warm = state is not None and state.get("theta") is not None
        out = plan.trace(c, pairs=pairs, theta=state["theta"] if warm else None, warm=warm)
        if state is not None:
            state["theta"] = out["theta"]
            state["status"] = out["status"]
        ctx.plan, ctx.pairs = plan, pairs
        ctx.save_for_backward(c, out["theta"], out["status"])
        return out["tof"]

    @staticmethod
    def backward(ctx, grad_t):
        c, theta, status = ctx.saved_tensors
        g = ctx.plan.adjoint(theta, status, grad_t.contiguous().to(torch.float64), weight="dtdc", c=c,
                             pairs=ctx.pairs)
        return g.to(c.dtype), None, None, None

