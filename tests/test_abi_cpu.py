"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/rtx.h and include/rtx3d.h declare, and the Python structs match the C
layout."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("rtx.h", "rtx3d.h")]


@pytest.fixture(scope="module")
def lib():
    from paper_2511_18511_amd import _binding, build

    if not os.path.exists(_binding.LIB_PATH):
        build.build()
    return _binding.load()


def declared_functions():
    src = "\n".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rtx3?_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rtx_trace_rays", "rtx_tof_forward", "rtx_tof_adjoint", "rtx_plan_create", "rtx_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2511_18511_amd import _binding

    names = declared_functions()
    assert sorted(_binding.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rtx3?_\w+)", out))
    assert set(names) <= exported
    for n in names:
        assert hasattr(lib, n)


def test_struct_layouts_match_c():
    from paper_2511_18511_amd import _binding as B

    assert C.sizeof(B.rtx_grid) == 16 and B.rtx_grid.h.offset == 8
    assert C.sizeof(B.rtx_ring) == 24 and B.rtx_ring.radius.offset == 8
    assert C.sizeof(B.rtx_opts) == 40 and B.rtx_opts.flags.offset == 32
    assert C.sizeof(B.rtx_instance) == 128 and B.rtx_instance.c.offset == 40 and B.rtx_instance.grad.offset == 120


def test_no_cpu_fallback_in_product_path():
    """The package never imports the oracle and has no host compute path."""
    pkg = os.path.join(ROOT, "paper_2511_18511_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle_rt" not in text, f


def test_batch_limits_are_checked_on_the_host(lib):
    """rtx_batch_create rejects more than 255 instances (the adjoint tags node
    updates with an 8-bit instance index) before it touches a device."""
    from paper_2511_18511_amd import _binding as B

    opts = B.rtx_opts(B.RTX_F32C, B.RTX_RK4, 0.25, 1e-3, 30, 0, 0)
    inst = (B.rtx_instance * 256)()
    out = C.c_void_p()
    lib.rtx_batch_create.restype = C.c_int
    lib.rtx_last_error.restype = C.c_char_p
    rc = lib.rtx_batch_create(C.byref(out), C.byref(opts), B.RTX_W_LENGTH, 0, 256, inst)
    assert rc == B.RTX_E_UNSUPPORTED, rc
    assert b"255" in lib.rtx_last_error()
    rc = lib.rtx_batch_create(C.byref(out), C.byref(opts), 7, 0, 1, inst)  # unknown weight
    assert rc == B.RTX_E_ARG
    # the cubic B-spline medium is a tracing-only option: batches reject it
    opts_b = B.rtx_opts(B.RTX_F32C, B.RTX_RK4, 0.25, 1e-3, 30, 0, B.RTX_INTERP_BSPLINE)
    rc = lib.rtx_batch_create(C.byref(out), C.byref(opts_b), B.RTX_W_LENGTH, 0, 1, inst)
    assert rc == B.RTX_E_UNSUPPORTED, rc
