"""The paraxial ray (Sec. 3.5) on the HIP path, through the C ABI: misfit
derivative, ray-tube width, amplitude and caustic count pair by pair against
the oracle at the oracle's linked angles (bilinear and B-spline media, both
integrators, both precisions), the 256x256 workload sampled, and the
fish-eye's perfect focus (Section 4)."""
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
# FP64: same arithmetic up to fused multiply-adds; FP32: the perturbation is
# integrated in plain FP32 over ~10^3 steps
TOL = {"f64": 1e-9, "f32c": 2e-4}


@pytest.fixture(scope="module")
def rtx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2511_18511_amd as rtx

    return rtx


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _check(out, ref, prec):
    assert np.array_equal(out["status"], ref["status"])
    ok = ref["status"] == oracle.LINKED
    for k in ("dgdth", "jac", "amp"):
        rel = np.abs(out[k][ok] - ref[k][ok]) / np.maximum(np.abs(ref[k][ok]), 1e-3 * np.abs(ref[k][ok]).max())
        assert rel.max() < TOL[prec], (k, rel.max())
    assert np.array_equal(out["kmah"][ok], ref["kmah"][ok])
    assert np.all(np.isnan(out["dgdth"][~ok]))


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("integ", ["rk4", "heun"])
@pytest.mark.parametrize("interp", ["bilinear", "bspline"])
def test_paraxial_matches_oracle(rtx, prec, integ, interp):
    """All 552 pairs of a 24-element ring through a 96x96 Gaussian-inclusion
    medium, at the oracle's own linked angles, plus an invalid pair."""
    n, h = 96, 0.5e-3
    c = synth.gaussian_inclusions(n, n, h, seed=91, r_max=0.7 * 0.45 * n * h)
    ring = (24, 0.45 * n * h * 0.9, 0.1)
    pairs = np.concatenate([synth.all_pairs(24), [[5, 5]]]).astype(np.int32)
    med = oracle.grid_medium(c, h, interp=interp)
    th = oracle.trace(med, ring, pairs, integ=integ)["theta"]
    ref = oracle.paraxial(med, ring, pairs, th, integ=integ)
    plan = rtx.Plan(n, n, h, *ring, prec=prec, integ=integ, max_pairs=len(pairs), interp=interp)
    print(f"\nparaxial {interp} {integ} {prec}", flush=True)
    out = {k: v.cpu().numpy() for k, v in plan.paraxial(_dev(th), pairs=_dev(pairs), c=_dev(c)).items()}
    plan.close()
    assert out["status"][-1] == oracle.BAD_INPUT
    _check(out, ref, prec)


def test_paraxial_full_size_sampled(rtx):
    """The 256x256 workload, all 65,280 pairs at their GPU-linked angles in
    FP32-compensated arithmetic; 300 sampled pairs against the oracle at the
    same angles.  Travel-time-level tolerance: the Jacobian of nearly focused
    pairs is small, so errors are taken relative to the workload's typical
    width."""
    cfg, c = synth.make_config("c2_gauss_256")
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    pairs = synth.all_pairs(cfg["n_elem"])
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], *ring, prec="f32c")
    tr = plan.trace(_dev(c), fan=True)
    out = {k: v.cpu().numpy() for k, v in plan.paraxial(tr["theta"]).items()}
    plan.close()
    assert np.all(out["status"] == oracle.LINKED)
    idx = np.sort(np.random.default_rng(92).choice(len(pairs), 300, replace=False))
    th = tr["theta"].cpu().numpy()[idx]
    ref = oracle.paraxial(oracle.grid_medium(c, cfg["h"]), ring, pairs[idx], th)
    assert np.abs(out["dgdth"][idx] - ref["dgdth"]).max() < 2e-4 * np.abs(ref["dgdth"]).max()
    assert np.abs(out["jac"][idx] - ref["jac"]).max() < 2e-4 * np.abs(ref["jac"]).max()
    assert np.array_equal(out["kmah"][idx], ref["kmah"])
    print(f"\ncaustics crossed on the 256x256 workload: {np.bincount(out['kmah'])}", flush=True)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_paraxial_fisheye_focus_on_gpu(rtx, prec):
    """Maxwell's fish-eye on the B-spline grid (Section 4, a = 1, 1-degree
    spacing, ds/dx = 1): rays from [0, a] focus on [0, -a] (dg/dtheta and the
    width vanish to the discretisation error); on a ring of radius 2a every ray
    crosses the focus at [0, -a/2] once."""
    with open(os.path.join(HERE, "golden", "fisheye_paper.json")) as f:
        g = json.load(f)
    a, dx = g["a"], g["dx_over_a"] * g["a"]
    th = np.linspace(*g["al_theta_range"], 21)
    pairs = np.tile(np.array([[0, 2]], np.int32), (len(th), 1))
    for R_ring in (a, 2 * a):
        n = 2 * int(math.ceil(1.1 * R_ring / dx)) + 1
        c = synth.fisheye(n, n, dx, c0=1.0, R=a)
        plan = rtx.Plan(n, n, dx, 4, R_ring, math.pi / 2, prec=prec, ds_px=1.0, max_pairs=len(pairs),
                        interp="bspline")
        out = {k: v.cpu().numpy() for k, v in plan.paraxial(_dev(th), pairs=_dev(pairs), c=_dev(c)).items()}
        plan.close()
        assert np.all(out["status"] == oracle.LINKED)
        if R_ring == a:
            assert np.abs(out["dgdth"]).max() < 0.01
            assert np.abs(out["jac"]).max() < 0.005 * a
        else:
            assert np.all(out["kmah"] == 1)
