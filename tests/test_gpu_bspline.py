"""The cubic B-spline medium (Sec. 3.3) on the HIP path, through the C ABI,
against the oracle's B-spline medium: fixed-angle traces pair by pair, linked
traces by re-tracing the GPU's angles, the paper's Section 4 fish-eye
experiments (acoustic length, Sec. 4.2, over a sweep of ds/dx; radius
deviation of the free-marched ray, Sec. 4.1) with both integrators, and the
calls a B-spline plan refuses (adjoint, path weights, changing the
interpolation)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
HERE = os.path.dirname(__file__)
TOL_T = {"f64": 1e-12, "f32c": 1e-5}


@pytest.fixture(scope="module")
def rtx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2511_18511_amd as rtx

    return rtx


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _bsp(c, h):
    return oracle.grid_medium(c, h, interp="bspline")


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("integ", ["rk4", "heun"])
def test_bspline_fixed_angle_matches_oracle(rtx, prec, integ):
    """1000 random pairs and angles (several tiles and a ragged tail)."""
    n, h = 96, 0.5e-3
    c = synth.gaussian_inclusions(n, n, h, seed=23, r_max=0.7 * 0.45 * n * h)
    ring = (40, 0.45 * n * h * 0.9, 0.1)
    rng = np.random.default_rng(5)
    allp = synth.all_pairs(40)
    pairs = allp[rng.choice(len(allp), 1000, replace=False)]
    theta = rng.uniform(-1.4, 1.4, len(pairs))
    plan = rtx.Plan(n, n, h, *ring, prec=prec, integ=integ, max_pairs=len(pairs), interp="bspline")
    print(f"\nB-spline fixed angle {prec} {integ}", flush=True)
    out = {k: _np(v) for k, v in plan.trace(_dev(c), pairs=_dev(pairs.astype(np.int32)), theta=_dev(theta),
                                            fixed=True).items()}
    plan.close()
    ref = oracle.trace(_bsp(c, h), ring, pairs, theta=theta, fixed=True, integ=integ)
    assert np.array_equal(out["status"], ref["status"])
    hit = ref["status"] == oracle.LINKED
    assert hit.sum() > 900
    assert np.abs(out["tof"][hit] / ref["tof"][hit] - 1).max() < TOL_T[prec]
    assert np.abs(out["len"][hit] / ref["len"][hit] - 1).max() < TOL_T[prec]
    assert np.abs(out["miss_px"][hit] - ref["miss_px"][hit]).max() < (1e-9 if prec == "f64" else 2e-4)
    # the spline and the bilinear field are different media: the times differ
    refb = oracle.trace(oracle.grid_medium(c, h), ring, pairs[:50], theta=theta[:50], fixed=True, integ=integ)
    assert np.abs(refb["tof"] / ref["tof"][:50] - 1).max() > 1e-6


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("fan", [False, True])
def test_bspline_linked_matches_oracle(rtx, prec, fan):
    """All 992 pairs of a 32-element ring: every GPU angle re-traced by the
    oracle, and the same root as the oracle's own linking."""
    n, h = 96, 0.5e-3
    c = synth.gaussian_inclusions(n, n, h, seed=29, r_max=0.7 * 0.45 * n * h)
    ring = (32, 0.45 * n * h * 0.9, 0.0)
    pairs = synth.all_pairs(32)
    tol = 1e-3
    plan = rtx.Plan(n, n, h, *ring, prec=prec, interp="bspline")
    print(f"\nB-spline linked {prec} fan={fan}", flush=True)
    out = {k: _np(v) for k, v in plan.trace(_dev(c), fan=fan).items()}
    plan.close()
    ref = oracle.trace(_bsp(c, h), ring, pairs, fan=fan)
    assert np.array_equal(out["status"], ref["status"])
    ok = out["status"] == oracle.LINKED
    assert ok.mean() > 0.99
    chk = oracle.trace(_bsp(c, h), ring, pairs[ok], theta=out["theta"][ok], fixed=True)
    assert np.abs(out["tof"][ok] / chk["tof"] - 1).max() < TOL_T[prec]
    assert chk["miss_px"].max() <= tol * (1 + 1e-6) + (0 if prec == "f64" else 2e-4)
    R_px = ring[1] / h
    assert np.abs(out["theta"][ok] - ref["theta"][ok]).max() < 4 * tol / R_px / 0.05
    if prec == "f64":
        same = out["n_marches"][ok] == ref["n_marches"][ok]
        assert same.mean() > 0.95
        assert np.abs(out["tof"][ok][same] / ref["tof"][ok][same] - 1).max() < 1e-10


def test_bspline_full_size_sampled(rtx):
    """The 256x256 Gaussian-inclusion workload (65,280 pairs) with the B-spline
    medium in FP32-compensated arithmetic; 300 sampled pairs re-traced by the
    oracle."""
    cfg, c = synth.make_config("c2_gauss_256")
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    pairs = synth.all_pairs(cfg["n_elem"])
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], *ring, prec="f32c", interp="bspline")
    out = {k: _np(v) for k, v in plan.trace(_dev(c)).items()}
    plan.close()
    assert np.all(out["status"] == oracle.LINKED)
    idx = np.sort(np.random.default_rng(9).choice(len(pairs), 300, replace=False))
    chk = oracle.trace(_bsp(c, cfg["h"]), ring, pairs[idx], theta=out["theta"][idx], fixed=True)
    assert np.abs(out["tof"][idx] / chk["tof"] - 1).max() < 1e-5
    assert chk["miss_px"].max() <= cfg["tol_px"] + 2e-4


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("integ", ["rk4", "heun"])
def test_paper_fisheye_acoustic_length_on_gpu(rtx, prec, integ):
    """Section 4.2 on the HIP path: Maxwell's fish-eye (n0 = a = 1) on the
    B-spline grid with a 1-degree spacing, 101 rays from [0, a] spread over
    [-pi/3, pi/3], all intercepted at [0, -a]; with c0 = 1 the travel time is
    the acoustic length, a pi / 2.  Ray by ray against the oracle, and the mean
    relative error RE_al within the oracle's own budget for this setting."""
    with open(os.path.join(HERE, "golden", "fisheye_paper.json")) as f:
        g = json.load(f)
    a, dx, ds = g["a"], g["dx_over_a"] * g["a"], g["ds_over_dx"]
    n = 2 * int(math.ceil(1.1 * a / dx)) + 1
    c = synth.fisheye(n, n, dx, c0=1.0, R=a)
    ring = (4, a, math.pi / 2)
    th = np.linspace(*g["al_theta_range"], g["al_n_rays"])
    pairs = np.tile(np.array([[0, 2]], np.int32), (len(th), 1))
    plan = rtx.Plan(n, n, dx, *ring, prec=prec, integ=integ, ds_px=ds, max_pairs=len(pairs), interp="bspline")
    out = {k: _np(v) for k, v in plan.trace(_dev(c), pairs=_dev(pairs), theta=_dev(th), fixed=True).items()}
    plan.close()
    ref = oracle.trace(_bsp(c, dx), ring, pairs, theta=th, fixed=True, integ=integ, ds_px=ds)
    assert np.all(out["status"] == oracle.LINKED)
    assert np.abs(out["tof"] / ref["tof"] - 1).max() < TOL_T[prec]
    re_al = np.mean((out["tof"] - g["L_true"]) / g["L_true"]) * 100
    re_ref = np.mean((ref["tof"] - g["L_true"]) / g["L_true"]) * 100
    print(f"\nRE_al {prec} {integ}: GPU {re_al:.3e} %, oracle {re_ref:.3e} %", flush=True)
    assert abs(re_al) < {"rk4": 0.003, "heun": 0.005}[integ]
    assert np.max(out["miss_px"]) * dx < 2e-4 * a


def _golden():
    with open(os.path.join(HERE, "golden", "fisheye_paper.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("integ", ["rk4", "heun"])
def test_paper_fisheye_acoustic_length_ds_sweep(rtx, prec, integ):
    """Section 4.2's deviation RE_al over ds/dx = 1/4 .. 2 (the paper plots it
    against ds/dx): GPU equal to the oracle at every step size, and the error
    second order in ds (the trapezoid quadrature dominates the B-spline field's
    error on this grid)."""
    g = _golden()
    a, dx = g["a"], g["dx_over_a"] * g["a"]
    n = 2 * int(math.ceil(1.1 * a / dx)) + 1
    c = synth.fisheye(n, n, dx, c0=1.0, R=a)
    ring = (4, a, math.pi / 2)
    th = np.linspace(*g["al_theta_range"], g["al_n_rays"])
    pairs = np.tile(np.array([[0, 2]], np.int32), (len(th), 1))
    plan = rtx.Plan(n, n, dx, *ring, prec=prec, integ=integ, max_pairs=len(pairs), interp="bspline")
    plan.set_medium(_dev(c))
    res = []
    for ds in (0.25, 0.5, 1.0, 2.0):
        out = plan.trace(None, pairs=_dev(pairs), theta=_dev(th), fixed=True, ds_px=ds)
        T = _np(out["tof"])
        assert np.all(_np(out["status"]) == oracle.LINKED)
        ref = oracle.trace(_bsp(c, dx), ring, pairs, theta=th, fixed=True, integ=integ, ds_px=ds)
        res.append((np.mean((T - g["L_true"]) / g["L_true"]) * 100,
                    np.mean((ref["tof"] - g["L_true"]) / g["L_true"]) * 100))
    plan.close()
    print(f"\nRE_al (%) {prec} {integ} at ds/dx 0.25, 0.5, 1, 2: GPU " + ", ".join("%.3e" % r[0] for r in res)
          + "; oracle " + ", ".join("%.3e" % r[1] for r in res), flush=True)
    for gpu, ref in res:
        assert abs(gpu - ref) < (1e-9 if prec == "f64" else 5e-5)
    if prec == "f64":  # FP32 rounding (~1e-5 %) blurs the ratios at the smallest steps
        for (r1, _), (r2, _) in zip(res, res[1:]):
            assert 3.0 < r2 / r1 < 5.0


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("integ", ["rk4", "heun"])
def test_paper_fisheye_radius_deviation_on_gpu(rtx, prec, integ):
    """Section 4.1 on the HIP path: the ray from [0, a] launched clockwise,
    normal to x_c - x_p, circles x_c = [a, 0] with radius sqrt(2) a; marched
    free over 1.2 turns at ds/dx = 1 and 1/2, point by point against the
    oracle's march, and RE_rd over the first turn within the oracle's budget."""
    g = _golden()
    a, dx = g["a"], g["dx_over_a"] * g["a"]
    n = 2 * int(math.ceil(2.6 * a / dx)) + 1
    c = synth.fisheye(n, n, dx, c0=1.0, R=a)
    plan = rtx.Plan(n, n, dx, 4, a, math.pi / 2, prec=prec, integ=integ, interp="bspline")
    x0 = np.array(g["rd_start"])
    d0 = np.array(g["rd_direction_clockwise"])
    for ds in (1.0, 0.5):
        circ = 2 * math.pi * g["R_true"] / dx
        n_steps = int(1.2 * circ / ds)
        pts = _np(plan.march(_dev(x0[None]), _dev(d0[None]), n_steps, c=_dev(c), ds_px=ds))[0]
        ref = oracle.march_free(_bsp(c, dx), x0 / dx, d0, n_steps, ds_px=ds, integ=integ) * dx
        dev_px = np.abs(pts - ref).max() / dx
        assert dev_px < (1e-9 if prec == "f64" else 2e-3), dev_px
        dist0 = np.linalg.norm(pts - x0, axis=1)
        far = np.nonzero(dist0 > 10 * ds * dx)[0][0]
        M = far + np.nonzero(dist0[far:] < ds * dx)[0][0]
        rad = np.linalg.norm(pts[1:M + 1] - np.array(g["rd_centre"]), axis=1)
        re_rd = np.mean(np.abs(rad - g["R_true"]) / g["R_true"]) * 100
        print(f"\nRE_rd {prec} {integ} ds/dx {ds}: {re_rd:.3e} % (max point deviation from the oracle "
              f"{dev_px:.1e} px)", flush=True)
        # FP32 marching holds the radius to ~5e-7 relative (a few ulps of the
        # FP32 field and curvature), above RK4's truncation error on this ray
        bound = {"rk4": 2e-5 if prec == "f64" else 1e-4, "heun": 0.02}[integ]
        assert re_rd < bound * ds ** (0 if integ == "rk4" else 2)
    plan.close()


def test_bspline_plan_refuses_bilinear_only_calls(rtx):
    from paper_2511_18511_amd import _binding as B

    n, h = 64, 1e-3
    c = synth.gaussian_inclusions(n, n, h, seed=11, r_max=0.015)
    ring = (16, 0.025, 0.0)
    plan = rtx.Plan(n, n, h, *ring, prec="f32c", interp="bspline")
    out = plan.trace(_dev(c))
    assert bool((out["status"] == 0).all())
    with pytest.raises(rtx.RtxError, match="bilinear-only"):
        plan.adjoint(out["theta"], out["status"], _dev(np.ones(len(out["tof"]))))
    with pytest.raises(rtx.RtxError, match="bilinear-only"):
        plan.weights(out["theta"])
    # the interpolation is fixed when the plan is created
    with pytest.raises(rtx.RtxError, match="cannot change"):
        B.rtx_plan_set_opts(plan._handle, B.rtx_opts(B.RTX_F32C, B.RTX_RK4, 0.25, 1e-3, 30, 0, 0))
    plan.close()
