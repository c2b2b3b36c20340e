"""ctypes binding of librtx.so (argument marshalling only; every step of the
computation runs in the HIP kernels of the library).  The names mirror the C
ABI declared in include/rtx.h."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtx.so")

RTX_OK, RTX_E_ARG, RTX_E_HIP, RTX_E_NOMEM, RTX_E_UNSUPPORTED, RTX_E_CAPACITY = 0, -1, -2, -3, -4, -5
RTX_F64, RTX_F32C = 0, 1
RTX_HEUN, RTX_RK4 = 2, 4
RTX_WARM_START, RTX_FIXED_ANGLE, RTX_FAN_START, RTX_INTERP_BSPLINE = 1, 2, 4, 8
RTX_SLOT_PACK, RTX_SLOT_TRACE, RTX_SLOT_FAN_SEED, RTX_SLOT_FAN_LINK, RTX_SLOT_ADJOINT, RTX_NUM_SLOTS = 0, 1, 2, 3, 4, 5
RTX_W_LENGTH, RTX_W_DTDC = 0, 1
RTX_RESID_REAL, RTX_RESID_RAYBORN_C64 = 0, 1
RTX_RAY_LINKED, RTX_RAY_NOT_CONVERGED, RTX_RAY_NO_HIT, RTX_RAY_BAD_INPUT = 0, 1, 2, 3

# every symbol include/rtx.h declares
EXPORTS = ("rtx_plan_create", "rtx_plan_destroy", "rtx_plan_set_opts", "rtx_set_medium", "rtx_trace_rays",
           "rtx_tof_forward", "rtx_march_free", "rtx_paraxial", "rtx_sart", "rtx_tof_adjoint", "rtx_plan_stats", "rtx_plan_region_stats", "rtx_plan_timing",
           "rtx_plan_timings", "rtx_plan_set_launch", "rtx_batch_create",
           "rtx_batch_run", "rtx_batch_times", "rtx_batch_destroy", "rtx_last_error",
           # include/rtx3d.h
           "rtx3_plan_create", "rtx3_plan_destroy", "rtx3_plan_set_opts", "rtx3_set_medium", "rtx3_trace_rays",
           "rtx3_march_free", "rtx3_plan_stats", "rtx3_last_error")


class rtx_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("h", C.c_double)]


class rtx3_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double)]


class rtx_ring(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("radius", C.c_double), ("phi0", C.c_double)]


class rtx_opts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("integ", C.c_int32), ("ds_px", C.c_double), ("tol_px", C.c_double),
                ("max_marches", C.c_int32), ("max_steps", C.c_int32), ("flags", C.c_uint32)]


class rtx_instance(C.Structure):
    _fields_ = [("grid", rtx_grid), ("ring", rtx_ring), ("c", C.c_void_p), ("pairs", C.c_void_p),
                ("n_pairs", C.c_int64), ("theta", C.c_void_p), ("tof", C.c_void_p), ("len", C.c_void_p),
                ("miss_px", C.c_void_p), ("n_marches", C.c_void_p), ("status", C.c_void_p), ("resid", C.c_void_p),
                ("grad", C.c_void_p)]


class RtxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rtx error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Loads librtx.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                          "g.build()'` (hipcc, gfx950); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    L.rtx_plan_create.argtypes = [C.POINTER(vp), C.POINTER(rtx_grid), C.POINTER(rtx_ring), C.POINTER(rtx_opts), i64]
    L.rtx_plan_destroy.argtypes = [vp]
    L.rtx_plan_set_opts.argtypes = [vp, C.POINTER(rtx_opts)]
    L.rtx_set_medium.argtypes = [vp, vp, vp]
    L.rtx_trace_rays.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp]
    L.rtx_tof_forward.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    L.rtx_march_free.argtypes = [vp, vp, i64, vp, vp, C.c_int32, vp, vp]
    L.rtx_paraxial.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
    L.rtx_sart.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, C.c_int32, C.c_double, vp]
    L.rtx_tof_adjoint.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, i32, C.POINTER(C.c_double), i32, i32, vp, vp]
    L.rtx_plan_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.rtx_plan_set_launch.argtypes = [vp, i32]
    L.rtx_plan_region_stats.argtypes = [vp, i32, C.POINTER(i64), C.POINTER(i64)]
    L.rtx_plan_timing.argtypes = [vp, i32]
    L.rtx_plan_timings.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    L.rtx_batch_create.argtypes = [C.POINTER(vp), C.POINTER(rtx_opts), i32, i32, i32, C.POINTER(rtx_instance)]
    L.rtx_batch_run.argtypes = [vp, vp]
    L.rtx_batch_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.rtx_batch_destroy.argtypes = [vp]
    L.rtx3_plan_create.argtypes = [C.POINTER(vp), C.POINTER(rtx3_grid), i32, vp, C.POINTER(rtx_opts), i64]
    L.rtx3_plan_destroy.argtypes = [vp]
    L.rtx3_plan_set_opts.argtypes = [vp, C.POINTER(rtx_opts)]
    L.rtx3_set_medium.argtypes = [vp, vp, vp]
    L.rtx3_trace_rays.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
    L.rtx3_march_free.argtypes = [vp, vp, i64, vp, vp, C.c_int32, vp, vp]
    L.rtx3_plan_stats.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
    for name in EXPORTS:
        getattr(L, name).restype = C.c_char_p if name.endswith("last_error") else C.c_int
    _lib = L
    return L


def check(code):
    if code != RTX_OK:
        raise RtxError(code, load().rtx_last_error().decode())
    return code


def check3(code):
    if code != RTX_OK:
        raise RtxError(code, load().rtx3_last_error().decode())
    return code


def rtx3_plan_create(grid, elem_host, opts, max_pairs):
    """elem_host: float64 [n][3] numpy array (metres)."""
    h = C.c_void_p()
    e = elem_host
    check3(load().rtx3_plan_create(C.byref(h), C.byref(grid), int(e.shape[0]), C.c_void_p(e.ctypes.data),
                                   C.byref(opts), int(max_pairs)))
    return h


def rtx3_plan_destroy(plan):
    return check3(load().rtx3_plan_destroy(plan))


def rtx3_plan_set_opts(plan, opts):
    return check3(load().rtx3_plan_set_opts(plan, C.byref(opts)))


def rtx3_set_medium(plan, c, stream):
    return check3(load().rtx3_set_medium(plan, c, stream))


def rtx3_trace_rays(plan, c, pairs, n_pairs, u, tof, len_, miss_px, n_marches, status, stream):
    return check3(load().rtx3_trace_rays(plan, c, pairs, int(n_pairs), u, tof, len_, miss_px, n_marches, status,
                                         stream))


def rtx3_march_free(plan, c, n_rays, x0, d0, n_steps, pts, stream):
    return check3(load().rtx3_march_free(plan, c, int(n_rays), x0, d0, int(n_steps), pts, stream))


def rtx3_plan_stats(plan):
    a, b = C.c_int64(), C.c_int64()
    check3(load().rtx3_plan_stats(plan, C.byref(a), C.byref(b)))
    return a.value, b.value


def rtx_plan_create(grid, ring, opts, max_pairs):
    h = C.c_void_p()
    check(load().rtx_plan_create(C.byref(h), C.byref(grid), C.byref(ring), C.byref(opts), int(max_pairs)))
    return h


def rtx_plan_destroy(plan):
    return check(load().rtx_plan_destroy(plan))


def rtx_plan_set_opts(plan, opts):
    return check(load().rtx_plan_set_opts(plan, C.byref(opts)))


def rtx_set_medium(plan, c, stream):
    return check(load().rtx_set_medium(plan, c, stream))


def rtx_trace_rays(plan, c, pairs, n_pairs, theta, tof, len_, miss_px, n_marches, status, w_rowptr, w_col, w_val,
                   nnz_cap, stream):
    return check(load().rtx_trace_rays(plan, c, pairs, int(n_pairs), theta, tof, len_, miss_px, n_marches, status,
                                       w_rowptr, w_col, w_val, int(nnz_cap), stream))


def rtx_tof_forward(plan, c, pairs, n_pairs, theta, tof, status, stream):
    return check(load().rtx_tof_forward(plan, c, pairs, int(n_pairs), theta, tof, status, stream))


def rtx_march_free(plan, c, n_rays, x0, d0, n_steps, pts, stream):
    return check(load().rtx_march_free(plan, c, int(n_rays), x0, d0, int(n_steps), pts, stream))


def rtx_paraxial(plan, c, pairs, n_pairs, theta, dgdth, jac, amp, kmah, status, stream):
    return check(load().rtx_paraxial(plan, c, pairs, int(n_pairs), theta, dgdth, jac, amp, kmah, status, stream))


def rtx_sart(plan, n_rows, nnz, w_rowptr, w_col, w_val, b, x, n_iter, lam, stream):
    return check(load().rtx_sart(plan, int(n_rows), int(nnz), w_rowptr, w_col, w_val, b, x, int(n_iter), float(lam),
                                 stream))


def rtx_tof_adjoint(plan, c, pairs, n_pairs, theta, status, tof, resid, resid_kind, freqs_hz, n_freq, weight, grad,
                    stream):
    fr = None
    if freqs_hz is not None:
        fr = (C.c_double * len(freqs_hz))(*[float(f) for f in freqs_hz])
    return check(load().rtx_tof_adjoint(plan, c, pairs, int(n_pairs), theta, status, tof, resid, int(resid_kind), fr,
                                        int(n_freq), int(weight), grad, stream))


def rtx_plan_stats(plan):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    check(load().rtx_plan_stats(plan, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def rtx_plan_set_launch(plan, rays_per_block):
    return check(load().rtx_plan_set_launch(plan, int(rays_per_block)))


def rtx_batch_create(opts, weight, rays_per_block, instances):
    arr = (rtx_instance * len(instances))(*instances)
    h = C.c_void_p()
    check(load().rtx_batch_create(C.byref(h), C.byref(opts), int(weight), int(rays_per_block), len(instances), arr))
    return h


def rtx_batch_run(batch, stream):
    return check(load().rtx_batch_run(batch, stream))


def rtx_batch_times(batch, n_inst):
    f = (C.c_double * n_inst)()
    d = (C.c_double * n_inst)()
    check(load().rtx_batch_times(batch, f, d))
    return list(f), list(d)


def rtx_batch_destroy(batch):
    return check(load().rtx_batch_destroy(batch))


def rtx_plan_region_stats(plan, region):
    a, b = C.c_int64(), C.c_int64()
    check(load().rtx_plan_region_stats(plan, int(region), C.byref(a), C.byref(b)))
    return a.value, b.value


def rtx_plan_timing(plan, enable):
    return check(load().rtx_plan_timing(plan, int(bool(enable))))


def rtx_plan_timings(plan):
    t = (C.c_double * RTX_NUM_SLOTS)()
    n = (C.c_int32 * RTX_NUM_SLOTS)()
    check(load().rtx_plan_timings(plan, t, n))
    return list(t), list(n)
