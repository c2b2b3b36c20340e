"""The 3-D tracer (hemispherical arrays, Broyden-like linking, Sec. 3.4) on the
HIP path, through the C ABI of include/rtx3d.h, against the 3-D oracle:
fixed-direction rays pair by pair, linked pairs (same status, the GPU's
parameters re-traced by the oracle, the same root), free marches point by
point, homogeneous straight rays, the fish-eye's antipodal focus (Section 4
with dim = 3), the 128^3 hemispherical workload sampled, and argument errors."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
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


def _vol(n, h, seed):
    return synth.gaussian_inclusions3(n, n, n, h, seed=seed, r_max=0.35 * n * h, sigma=(0.001, 0.004))


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("integ", ["rk4", "heun"])
def test3_fixed_direction_matches_oracle(rtx, prec, integ):
    """600 random pairs at random launch parameters (several tiles and a ragged
    tail) through a 40^3 Gaussian-blob volume."""
    n, h = 40, 0.5e-3
    c = _vol(n, h, 61)
    el = synth.hemisphere_elements(24, 0.0085)
    rng = np.random.default_rng(62)
    allp = synth.all_pairs(24)
    pairs = allp[rng.choice(len(allp), 500, replace=False)]
    u = rng.uniform(-0.6, 0.6, (len(pairs), 2))
    plan = rtx.Plan3(n, n, n, h, el, prec=prec, integ=integ, max_pairs=len(pairs))
    print(f"\n3-D fixed {prec} {integ}", flush=True)
    out = {k: _np(v) for k, v in plan.trace(_dev(c), pairs=_dev(pairs), u=_dev(u), fixed=True).items()}
    plan.close()
    ref = oracle.trace3({"kind": "grid", "c": c, "h": h}, el, pairs, u=u, fixed=True, integ=integ)
    assert np.array_equal(out["status"], ref["status"])
    hit = ref["status"] == oracle.LINKED
    assert hit.sum() > 400
    assert np.abs(out["tof"][hit] / ref["tof"][hit] - 1).max() < TOL_T[prec]
    assert np.abs(out["len"][hit] / ref["len"][hit] - 1).max() < TOL_T[prec]
    assert np.abs(out["miss_px"][hit] - ref["miss_px"][hit]).max() < (1e-9 if prec == "f64" else 2e-4)
    assert np.array_equal(out["u"], u)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test3_linked_matches_oracle(rtx, prec):
    """All 552 ordered pairs of a 24-element hemispherical array through a
    48^3 Gaussian-blob volume, linked from the straight ray."""
    n, h = 48, 0.5e-3
    c = _vol(n, h, 63)
    el = synth.hemisphere_elements(24, 0.010)
    pairs = synth.all_pairs(24)
    plan = rtx.Plan3(n, n, n, h, el, prec=prec)
    print(f"\n3-D linked {prec}", flush=True)
    out = {k: _np(v) for k, v in plan.trace(_dev(c)).items()}
    steps, rays = plan.stats()
    plan.close()
    med = {"kind": "grid", "c": c, "h": h}
    ref = oracle.trace3(med, el, pairs)
    assert np.array_equal(out["status"], ref["status"])
    ok = out["status"] == oracle.LINKED
    assert ok.mean() > 0.99
    assert rays == out["n_marches"].sum() and steps > rays
    chk = oracle.trace3(med, el, pairs[ok], u=out["u"][ok], fixed=True)
    assert np.abs(out["tof"][ok] / chk["tof"] - 1).max() < TOL_T[prec]
    assert chk["miss_px"].max() <= 1e-3 * (1 + 1e-6) + (0 if prec == "f64" else 2e-4)
    # the same root: parameters within what the linking tolerance allows
    assert np.abs(out["u"][ok] - ref["u"][ok]).max() < 1e-3
    if prec == "f64":
        same = out["n_marches"] == ref["n_marches"]
        assert same.mean() > 0.95
        assert np.abs(out["tof"][same & ok] / ref["tof"][same & ok] - 1).max() < 1e-10


def test3_homogeneous_and_status_paths(rtx):
    """Straight rays in a homogeneous volume (one ray, T = |r - e| / c0);
    invalid pairs are BAD_INPUT; a ray budget of one gives NOT_CONVERGED or an
    exact straight link; the empty call packs only."""
    n, h = 32, 1e-3
    el = synth.hemisphere_elements(16, 0.0125)
    pairs = np.concatenate([synth.all_pairs(16), [[2, 2], [-1, 3], [5, 16]]]).astype(np.int32)
    plan = rtx.Plan3(n, n, n, h, el, prec="f64", max_pairs=len(pairs))
    out = {k: _np(v) for k, v in plan.trace(_dev(np.full((n, n, n), 1500.0)), pairs=_dev(pairs)).items()}
    d = np.linalg.norm(el[pairs[:-3, 1]] - el[pairs[:-3, 0]], axis=1)
    assert np.all(out["status"][:-3] == oracle.LINKED) and np.all(out["n_marches"][:-3] == 1)
    np.testing.assert_allclose(out["tof"][:-3], d / 1500.0, rtol=1e-12)
    assert np.all(out["status"][-3:] == oracle.BAD_INPUT)
    c = _vol(n, h, 64)
    one = {k: _np(v) for k, v in plan.trace(_dev(c), pairs=_dev(pairs[:-3]), max_marches=1).items()}
    ref = oracle.trace3({"kind": "grid", "c": c, "h": h}, el, pairs[:-3], max_marches=1)
    assert np.array_equal(one["status"], ref["status"])
    e = plan.trace(None, pairs=_dev(np.zeros((0, 2), np.int32)))
    assert e["tof"].numel() == 0
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test3_free_march_matches_oracle(rtx, prec):
    """Free marches through a Gaussian-blob volume, point by point while on
    the grid; the GPU stops (NaN) at its first point outside the node box."""
    n, h = 40, 0.5e-3
    c = _vol(n, h, 65)
    rng = np.random.default_rng(66)
    nr, steps = 70, 300
    x0 = rng.uniform(-0.25, 0.25, (nr, 3)) * n * h
    d0 = rng.standard_normal((nr, 3))
    el = synth.hemisphere_elements(8, 0.008)
    plan = rtx.Plan3(n, n, n, h, el, prec=prec, max_pairs=1)
    pts = _np(plan.march(_dev(x0), _dev(d0), steps, c=_dev(c)))
    plan.close()
    med = {"kind": "grid", "c": c, "h": h}
    half = (n - 1) / 2 * h
    n_left = 0
    for i in range(nr):
        ref = oracle.march3_free(med, x0[i] / h, d0[i], steps) * h
        fin = np.isfinite(pts[i, :, 0])
        k = int(np.argmin(fin)) if not fin.all() else steps + 1
        assert fin[:k].all() and not fin[k:].any()
        assert np.all(np.abs(pts[i, :k]) <= half)
        dev = np.abs(pts[i, :k] - ref[:k]).max() / h
        assert dev < (1e-9 if prec == "f64" else 2e-3), (i, dev)
        n_left += k <= steps
    assert n_left > 10


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test3_fisheye_antipodal_focus_on_gpu(rtx, prec):
    """Section 4 with dim = 3 (a = 1, 1-degree spacing, ds/dx = 1) on the
    trilinear grid: 35 rays from [0, 0, a] into the lens reach the antipode
    [0, 0, -a] with acoustic length a pi / 2; ray by ray against the oracle on
    the same grid."""
    a, dx = 1.0, 2 * math.pi / 360
    n = 2 * int(math.ceil(1.1 * a / dx)) + 1
    c = synth.fisheye3(n, n, n, dx, c0=1.0, R=a)
    el = np.array([[0.0, 0.0, a], [0.0, 0.0, -a]])
    us = []
    for t in np.linspace(-math.pi / 3, math.pi / 3, 7):
        for ph in np.linspace(0, 2 * math.pi, 5, endpoint=False):
            us.append([math.tan(t) * math.cos(ph), math.tan(t) * math.sin(ph)])
    us = np.array(us)
    pairs = np.tile(np.array([[0, 1]], np.int32), (len(us), 1))
    plan = rtx.Plan3(n, n, n, dx, el, prec=prec, ds_px=1.0, max_pairs=len(pairs))
    out = {k: _np(v) for k, v in plan.trace(_dev(c), pairs=_dev(pairs), u=_dev(us), fixed=True).items()}
    plan.close()
    ref = oracle.trace3({"kind": "grid", "c": c, "h": dx}, el, pairs, u=us, fixed=True, ds_px=1.0)
    assert np.all(out["status"] == oracle.LINKED)
    assert np.abs(out["tof"] / ref["tof"] - 1).max() < TOL_T[prec]
    re_al = np.mean((out["tof"] - math.pi / 2) / (math.pi / 2)) * 100
    print(f"\n3-D RE_al {prec}: {re_al:.3e} %", flush=True)
    assert abs(re_al) < 0.05


def test3_hemisphere_workload_sampled(rtx):
    """The 128^3 hemispherical workload (256 elements, 65,280 pairs, 12
    Gaussian blobs) linked on the GPU in FP32-compensated arithmetic; 200
    sampled pairs re-traced by the oracle at the GPU's parameters."""
    cfg, c = synth.make_config3("c6_hemi_128")
    el = synth.hemisphere_elements(cfg["n_elem"], cfg["radius"])
    pairs = synth.all_pairs(cfg["n_elem"])
    plan = rtx.Plan3(cfg["n"], cfg["n"], cfg["n"], cfg["h"], el, prec="f32c")
    out = {k: _np(v) for k, v in plan.trace(_dev(c)).items()}
    plan.close()
    ok = out["status"] == oracle.LINKED
    print(f"\n3-D workload: linked {ok.mean():.4%}, rays per pair {out['n_marches'].mean():.2f} "
          f"(max {out['n_marches'].max()})", flush=True)
    assert ok.mean() > 0.995
    idx = np.sort(np.random.default_rng(67).choice(np.nonzero(ok)[0], 200, replace=False))
    chk = oracle.trace3({"kind": "grid", "c": c, "h": cfg["h"]}, el, pairs[idx], u=out["u"][idx], fixed=True)
    assert np.abs(out["tof"][idx] / chk["tof"] - 1).max() < 1e-5
    assert chk["miss_px"].max() <= cfg["tol_px"] + 2e-4


def test3_argument_errors(rtx):
    el = synth.hemisphere_elements(8, 0.010)
    with pytest.raises(rtx.RtxError):
        rtx.Plan3(16, 16, 16, 1e-3, el)  # the sphere does not fit the grid
    bad = el.copy()
    bad[3] *= 1.01
    with pytest.raises(rtx.RtxError):
        rtx.Plan3(32, 32, 32, 1e-3, bad)  # an element off the sphere
    plan = rtx.Plan3(32, 32, 32, 1e-3, el, max_pairs=10)
    with pytest.raises(rtx.RtxError):
        plan.trace(_dev(np.full((32, 32, 32), 1500.0)))  # 56 pairs > max_pairs
    with pytest.raises(rtx.RtxError):
        plan.trace(None, pairs=_dev(np.zeros((2, 2), np.int32)))  # no medium set
    plan.close()
