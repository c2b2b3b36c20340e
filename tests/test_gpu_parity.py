"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Fixed-angle traces are unique results: T, L, miss and status are compared pair
by pair.  A linked angle is one of many valid results (any angle whose miss is
within the tolerance), so linked runs are checked by (a) re-tracing the GPU's
angle in the oracle (T, L, miss <= tol), (b) the same root as the oracle's own
linking, and (c) pair-by-pair T agreement where both took the same number of
rays (FP64)."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rtx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2511_18511_amd as rtx

    return rtx


DEV = "cuda:0"
TOL_T = {"f64": 1e-12, "f32c": 1e-5}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _gauss(n=96, h=0.5e-3, seed=21):
    return synth.gaussian_inclusions(n, n, h, seed=seed, r_max=0.7 * 0.45 * n * h)


def _fixed_case(rtx, prec, c, h, ring, pairs, theta, integ="rk4", ds=0.25):
    n_elem, radius, phi0 = ring
    ny, nx = c.shape
    plan = rtx.Plan(nx, ny, h, n_elem, radius, phi0, prec=prec, integ=integ, ds_px=ds, max_pairs=len(pairs))
    out = plan.trace(_dev(c), pairs=_dev(pairs.astype(np.int32)), theta=_dev(theta), fixed=True)
    ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs, theta=theta, fixed=True, integ=integ, ds_px=ds)
    plan.close()
    return {k: _np(v) for k, v in out.items()}, ref


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("integ", ["rk4", "heun"])
def test_fixed_angle_matches_oracle(rtx, prec, integ):
    """Several tiles of lanes plus a ragged tail (1000 pairs), random angles."""
    n, h = 96, 0.5e-3
    c = _gauss(n, h)
    ring = (40, 0.45 * n * h * 0.9, 0.1)
    rng = np.random.default_rng(0)
    allp = synth.all_pairs(40)
    pairs = allp[rng.choice(len(allp), 1000, replace=False)]
    theta = rng.uniform(-1.4, 1.4, len(pairs))
    out, ref = _fixed_case(rtx, prec, c, h, ring, pairs, theta, integ)
    assert np.array_equal(out["status"], ref["status"])
    hit = ref["status"] == oracle.LINKED
    assert hit.sum() > 900
    rel = np.abs(out["tof"][hit] / ref["tof"][hit] - 1)
    assert rel.max() < TOL_T[prec], rel.max()
    assert np.abs(out["len"][hit] / ref["len"][hit] - 1).max() < TOL_T[prec]
    assert np.abs(out["miss_px"][hit] - ref["miss_px"][hit]).max() < (1e-9 if prec == "f64" else 2e-4)
    assert np.all(out["n_marches"] == 1)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_linked_fisheye_c1(rtx, prec):
    """The 128x128 fish-eye workload, all 992 pairs (strong focusing: reversed
    misfit orientation, trapped near-grazing rays)."""
    cfg, c = synth.make_config("c1_fisheye_128")
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    pairs = synth.all_pairs(cfg["n_elem"])
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], *ring, prec=prec)
    out = {k: _np(v) for k, v in plan.trace(_dev(c)).items()}
    plan.close()
    ref = oracle.trace(oracle.grid_medium(c, cfg["h"]), ring, pairs)
    _check_linked(out, ref, c, cfg["h"], ring, pairs, prec, cfg["tol_px"])


def _check_linked(out, ref, c, h, ring, pairs, prec, tol, idx=None, same_path=True):
    if idx is None:
        idx = np.arange(len(pairs))
    st = out["status"][idx]
    assert np.array_equal(st, ref["status"]), (np.bincount(st, minlength=4), np.bincount(ref["status"], minlength=4))
    ok = st == oracle.LINKED
    # (a) the oracle re-traces the GPU's angle: same T/L, and it really links
    chk = oracle.trace(oracle.grid_medium(c, h), ring, pairs[idx][ok], theta=out["theta"][idx][ok], fixed=True)
    assert np.abs(out["tof"][idx][ok] / chk["tof"] - 1).max() < TOL_T[prec]
    assert np.abs(out["len"][idx][ok] / chk["len"] - 1).max() < TOL_T[prec]
    assert chk["miss_px"].max() <= tol * (1 + 1e-6) + (0 if prec == "f64" else 2e-4)
    # (b) the same root as the oracle's own linking: angles within the tolerance
    # band (|dg/dtheta| >= 0.05 on these workloads) and T within the band it spans
    R_px = ring[1] / h
    dth = np.abs(out["theta"][idx][ok] - ref["theta"][ok])
    assert dth.max() < 4 * tol / R_px / 0.05
    cmin = c.min()
    assert np.abs(out["tof"][idx][ok] - ref["tof"][ok]).max() < 4 * tol * h / cmin + 1e-5 * ref["tof"][ok].max()
    # (c) FP64 with the same number of rays: same iterates, T to 1e-10
    if prec == "f64" and same_path:
        same = out["n_marches"][idx][ok] == ref["n_marches"][ok]
        assert same.mean() > 0.95
        assert np.abs(out["tof"][idx][ok][same] / ref["tof"][ok][same] - 1).max() < 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_linked_gaussian_sampled_full_size(rtx, prec):
    """256x256 Gaussian-inclusion workload (65,280 pairs) traced in full on the
    GPU in the benchmark's launch configuration; 600 sampled pairs checked
    against the oracle."""
    cfg, c = synth.make_config("c2_gauss_256")
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    pairs = synth.all_pairs(cfg["n_elem"])
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], *ring, prec=prec)
    out = {k: _np(v) for k, v in plan.trace(_dev(c)).items()}
    plan.close()
    assert np.all(out["status"] == oracle.LINKED)
    idx = np.sort(np.random.default_rng(3).choice(len(pairs), 600, replace=False))
    ref = oracle.trace(oracle.grid_medium(c, cfg["h"]), ring, pairs[idx])
    _check_linked(out, ref, c, cfg["h"], ring, pairs, prec, cfg["tol_px"], idx)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_warm_start_and_explicit_pairs(rtx, prec):
    n, h = 96, 0.5e-3
    c = _gauss(n, h, seed=4)
    ring = (24, 0.45 * n * h * 0.9, 0.0)
    pairs = synth.all_pairs(24)[::3].copy()
    ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs)
    plan = rtx.Plan(n, n, h, *ring, prec=prec, max_pairs=len(pairs))
    th0 = ref["theta"] + 1e-3
    out = {k: _np(v) for k, v in plan.trace(_dev(c), pairs=_dev(pairs), theta=_dev(th0), warm=True).items()}
    plan.close()
    refw = oracle.trace(oracle.grid_medium(c, h), ring, pairs, theta=th0, warm=True)
    assert np.all(out["status"] == oracle.LINKED)
    assert np.all(out["n_marches"] <= 3)
    _check_linked(out, refw, c, h, ring, pairs, prec, 1e-3)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("weight", ["length", "dtdc"])
def test_adjoint_matches_oracle(rtx, prec, weight):
    n, h = 96, 0.5e-3
    c = _gauss(n, h, seed=8)
    ring = (32, 0.45 * n * h * 0.9, 0.0)
    pairs = synth.all_pairs(32)
    ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs)
    rho = synth.real_residual(len(pairs), 2002)
    plan = rtx.Plan(n, n, h, *ring, prec=prec)
    g = plan.adjoint(_dev(ref["theta"]), _dev(ref["status"]), _dev(rho), weight=weight, c=_dev(c))
    plan.close()
    gref = oracle.adjoint(c, h, ring, pairs, ref["theta"], rho, weight=weight, status=ref["status"])
    err = np.linalg.norm(_np(g).astype(np.float64) - gref) / np.linalg.norm(gref)
    assert err < (1e-11 if prec == "f64" else 1e-5), err


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_adjoint_accumulates_across_calls(rtx, prec):
    """grad is added into, call after call: the plan's zeroed gradient copies
    (one per group of blocks) are summed into grad and left zeroed, so a second
    call with rho and a third with -2 rho bring grad back to 0 + rho - 2 rho +
    rho = 0 up to rounding, and an explicit pair list (queue path, same copies)
    gives the all-pairs result."""
    n, h = 96, 0.5e-3
    c = _gauss(n, h, seed=9)
    ring = (32, 0.45 * n * h * 0.9, 0.0)
    pairs = synth.all_pairs(32)
    ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs)
    rho = synth.real_residual(len(pairs), 2003)
    plan = rtx.Plan(n, n, h, *ring, prec=prec)
    th, st = _dev(ref["theta"]), _dev(ref["status"])
    g1 = _np(plan.adjoint(th, st, _dev(rho), c=_dev(c))).astype(np.float64)
    g = plan.adjoint(th, st, _dev(rho))
    g = plan.adjoint(th, st, _dev(-2.0 * rho), grad=g)
    g = plan.adjoint(th, st, _dev(rho), grad=g)
    scale = np.abs(g1).max()
    assert np.abs(_np(g).astype(np.float64)).max() < (1e-12 if prec == "f64" else 1e-5) * scale
    gp = _np(plan.adjoint(th, st, _dev(rho), pairs=_dev(pairs))).astype(np.float64)
    plan.close()
    assert np.abs(gp - g1).max() < (1e-12 if prec == "f64" else 1e-5) * scale


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_adjoint_segments_from_fan_checkpoints(rtx, prec):
    """After a fan-started trace the all-pairs adjoint marches each linked ray
    in segments (two), the later ones from the linking pass's checkpoints: two
    segments per ray, the same total steps, the oracle's adjoint at the traced
    angles, and the whole-ray adjoint of a plan without checkpoints;
    re-setting the medium (a new generation) and changing one angle make the
    checkpoints stop applying (whole rays again)."""
    n, h = 96, 0.5e-3
    c = _gauss(n, h, seed=10)
    ring = (32, 0.45 * n * h * 0.9, 0.0)
    pairs = synth.all_pairs(32)
    rho = synth.real_residual(len(pairs), 2005)
    tol = 1e-11 if prec == "f64" else 1e-5
    plan = rtx.Plan(n, n, h, *ring, prec=prec)
    out = plan.trace(_dev(c), fan=True)
    th, st = out["theta"], out["status"]
    used = int(((_np(st) == oracle.LINKED) | (_np(st) == oracle.NOT_CONVERGED)).sum())
    assert used == len(pairs)
    g_split = _np(plan.adjoint(th, st, _dev(rho))).astype(np.float64)
    steps_split, segs = plan.region_stats(2)
    assert segs == 2 * used
    gref = oracle.adjoint(c, h, ring, pairs, _np(th), rho, status=_np(st))
    assert np.linalg.norm(g_split - gref) / np.linalg.norm(gref) < tol
    fresh = rtx.Plan(n, n, h, *ring, prec=prec)
    g_whole = _np(fresh.adjoint(th, st, _dev(rho), c=_dev(c))).astype(np.float64)
    steps_whole, rays = fresh.region_stats(2)
    fresh.close()
    assert rays == used and steps_whole == steps_split
    assert np.linalg.norm(g_split - g_whole) / np.linalg.norm(g_whole) < (1e-14 if prec == "f64" else 1e-6)
    # the same plan after the medium is packed again: whole rays
    g_reset = _np(plan.adjoint(th, st, _dev(rho), c=_dev(c))).astype(np.float64)
    assert plan.region_stats(2)[1] == used
    assert np.linalg.norm(g_reset - g_whole) / np.linalg.norm(g_whole) < (1e-14 if prec == "f64" else 1e-6)
    # a fresh fan trace, then one pair's angle changed: that pair alone is whole
    out = plan.trace(None, fan=True, out=out)
    th2 = out["theta"].clone()
    th2[5] += 1e-9
    plan.adjoint(th2, st, _dev(rho))
    assert plan.region_stats(2)[1] == 2 * used - 1
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_rayborn_adjoint_matches_oracle(rtx, prec):
    n, h = 96, 0.5e-3
    c = _gauss(n, h, seed=12)
    ring = (24, 0.45 * n * h * 0.9, 0.0)
    pairs = synth.all_pairs(24)
    ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs)
    freqs = np.linspace(0.5e6, 1.5e6, 64)
    r = synth.complex_residual(len(pairs), 64, 2004)
    plan = rtx.Plan(n, n, h, *ring, prec=prec)
    g = plan.adjoint(_dev(ref["theta"]), _dev(ref["status"]), _dev(r), weight="length", c=_dev(c),
                     tof=_dev(ref["tof"]), freqs_hz=list(freqs))
    plan.close()
    rho = oracle.rayborn_rho(ref["tof"], freqs, r)
    gref = oracle.adjoint(c, h, ring, pairs, ref["theta"], rho, weight="length", status=ref["status"])
    err = np.linalg.norm(_np(g).astype(np.float64) - gref) / np.linalg.norm(gref)
    assert err < (1e-11 if prec == "f64" else 1e-5), err


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_status_paths_match_oracle(rtx, prec):
    n, h = 64, 1e-3
    c = synth.gaussian_inclusions(n, n, h, seed=11, r_max=0.015)
    ring = (16, 0.025, 0.0)
    pairs = np.array([[0, 5], [3, 3], [2, 16], [-1, 4], [7, 2]], np.int32)
    plan = rtx.Plan(n, n, h, *ring, prec=prec, max_pairs=16)
    for over, kw in (({}, {}), ({"max_marches": 1}, {"max_marches": 1}), ({"tol_px": 0.0, "max_marches": 4},
                     {"tol_px": 0.0, "max_marches": 4}), ({"max_steps": 3}, {"max_steps": 3})):
        out = {k: _np(v) for k, v in plan.trace(_dev(c), pairs=_dev(pairs), **over).items()}
        ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs, **kw)
        assert np.array_equal(out["status"], ref["status"]), (over, out["status"], ref["status"])
        assert np.array_equal(out["n_marches"][ref["status"] != oracle.BAD_INPUT],
                              ref["n_marches"][ref["status"] != oracle.BAD_INPUT])
    for bad in (np.nan, -1.0):
        cb = c.copy()
        cb[30:34, 28:36] = bad
        out = {k: _np(v) for k, v in plan.trace(_dev(cb), pairs=_dev(np.array([[0, 8], [4, 12]], np.int32))).items()}
        ref = oracle.trace(oracle.grid_medium(cb, h), ring, np.array([[0, 8], [4, 12]], np.int32))
        assert np.array_equal(out["status"], ref["status"])
    # empty batch
    e = plan.trace(_dev(c), pairs=_dev(np.zeros((0, 2), np.int32)))
    assert e["tof"].numel() == 0
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("integ", ["rk4", "heun"])
def test_free_march_matches_oracle(rtx, prec, integ):
    """rtx_march_free: 301 rays (two blocks and a ragged tail) from random points
    in random directions of random length, 500 steps; many leave the grid.
    Point by point against the oracle's free march while both are on the grid;
    the GPU ray stops (NaN) at its first point outside the node rectangle, and a
    zero direction gives NaN throughout."""
    n, h = 96, 0.5e-3
    c = _gauss(n, h, seed=41)
    ring = (16, 0.45 * n * h * 0.9, 0.0)
    rng = np.random.default_rng(41)
    nr, steps = 301, 500
    x0 = rng.uniform(-0.3, 0.3, (nr, 2)) * n * h
    ang = rng.uniform(0, 2 * np.pi, nr)
    d0 = np.stack([np.cos(ang), np.sin(ang)], 1) * rng.uniform(0.5, 2.0, (nr, 1))
    d0[7] = 0.0
    plan = rtx.Plan(n, n, h, *ring, prec=prec, integ=integ, max_pairs=1)
    pts = _np(plan.march(_dev(x0), _dev(d0), steps, c=_dev(c)))
    empty = plan.march(_dev(np.zeros((0, 2))), _dev(np.zeros((0, 2))), steps)
    plan.close()
    assert empty.shape == (0, steps + 1, 2)
    assert np.all(np.isnan(pts[7]))
    half = (n - 1) / 2 * h
    med = oracle.grid_medium(c, h)
    tol = (1e-9 if prec == "f64" else 2e-3) * h
    n_left = 0
    for i in range(nr):
        if i == 7:
            continue
        ref = oracle.march_free(med, x0[i] / h, d0[i], steps, integ=integ) * h
        fin = np.isfinite(pts[i, :, 0])
        k = int(np.argmin(fin)) if not fin.all() else steps + 1
        assert fin[:k].all() and not fin[k:].any()
        assert np.all(np.abs(pts[i, :k]) <= half)
        both = fin & np.isfinite(ref[:, 0])
        assert both[:k].sum() >= min(k, 10)
        assert np.abs(pts[i][both] - ref[both]).max() < tol, (i, np.abs(pts[i][both] - ref[both]).max() / h)
        if k <= steps:  # the GPU stopped: the oracle's point there is off the grid too (or already NaN)
            n_left += 1
            assert not np.isfinite(ref[k, 0]) or np.abs(ref[k]).max() > half - 1e-9 * h
    assert n_left > 50


def test_argument_errors(rtx):
    with pytest.raises(rtx.RtxError):
        rtx.Plan(64, 64, 1e-3, 16, 0.040)  # ring does not fit the grid
    with pytest.raises(rtx.RtxError):
        rtx.Plan(64, 64, 1e-3, 16, 0.020, ds_px=3.0)
    plan = rtx.Plan(64, 64, 1e-3, 16, 0.020, max_pairs=10)
    with pytest.raises(rtx.RtxError):
        plan.trace(_dev(np.full((64, 64), 1500.0)))  # 240 pairs > max_pairs
    with pytest.raises(rtx.RtxError):
        plan.trace(None, pairs=_dev(np.zeros((2, 2), np.int32)))  # no medium set
    plan.close()


def test_fisheye_f64_linked_matches_closed_form(rtx):
    """Closed form through the GPU path: gridded fish-eye T within the bilinear
    bias of the analytic travel time."""
    from tests import closed_form as cf

    cfg, c = synth.make_config("c1_fisheye_128")
    ring = (cfg["n_elem"], cfg["radius"], 0.0)
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], *ring, prec="f64")
    out = {k: _np(v) for k, v in plan.trace(_dev(c)).items()}
    plan.close()
    pts, _ = cf.ring_points(*ring)
    T = np.array([cf.fisheye_tof(pts[e], pts[r], 1500.0, 0.040) for e, r in synth.all_pairs(32)])
    assert np.max(np.abs(out["tof"] / T - 1)) < 5e-4
    assert math.isfinite(out["tof"].sum())


def _dense_rows(rowptr, cols, vals, n_nodes):
    rows = []
    for i in range(len(rowptr) - 1):
        r = np.zeros(n_nodes)
        r[cols[rowptr[i]:rowptr[i + 1]]] = vals[rowptr[i]:rowptr[i + 1]]
        rows.append(r)
    return np.array(rows)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_path_weights_match_oracle(rtx, prec):
    """System-matrix rows of the linked rays: node sets (bit-exact, sorted,
    unique) and values against the oracle's rows at the same angles."""
    n, h = 80, 0.5e-3
    c = _gauss(n, h, seed=31)
    ring = (20, 0.45 * n * h * 0.9, 0.0)
    pairs = synth.all_pairs(20)
    plan = rtx.Plan(n, n, h, *ring, prec=prec)
    out = plan.trace(_dev(c), weights=True)
    th = _np(out["theta"])
    rp, col, val = _np(out["w_rowptr"]), _np(out["w_col"]), _np(out["w_val"]).astype(np.float64)
    plan.close()
    orp, ocol, oval = oracle.weights_csr(c, h, ring, pairs, th)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0)
    for i in range(len(pairs)):
        cc = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cc) > 0)
    tol = 1e-12 if prec == "f64" else 2e-5
    G, O = _dense_rows(rp, col, val, n * n), _dense_rows(orp, ocol, oval, n * n)
    scale = O.max(axis=1, keepdims=True)
    assert np.abs(G - O).max(axis=1).max() <= tol * scale.max()
    if prec == "f64":
        assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    else:  # entries may differ only where a weight is at rounding level
        assert np.all(((G != 0) == (O != 0)) | (np.abs(G - O) <= tol * scale))
    # rows sum to the path length
    np.testing.assert_allclose(np.add.reduceat(val, rp[:-1]), _np(out["len"]), rtol=tol * 10)
    # capacity error path
    plan = rtx.Plan(n, n, h, *ring, prec=prec)
    out2 = plan.trace(_dev(c))
    # weights() at the same angles: the first-guess buffers (one call), then a
    # first guess too small (the second call fills exact buffers): same CSR
    for hint in (None, 10):
        if hint:
            plan._w_hint[len(pairs)] = hint
        rp2, col2, val2 = plan.weights(_dev(th))
        assert np.array_equal(_np(rp2), rp) and np.array_equal(_np(col2), col)
        assert np.array_equal(_np(val2).astype(np.float64), val)
    with pytest.raises(rtx.RtxError):
        import ctypes as C
        from paper_2511_18511_amd import _binding as B
        rowptr = torch.zeros(len(pairs) + 1, dtype=torch.int64, device=DEV)
        colb = torch.empty(10, dtype=torch.int32, device=DEV)
        valb = torch.empty(10, dtype=plan.real, device=DEV)
        st = torch.empty(len(pairs), dtype=torch.int8, device=DEV)
        plan._apply(B.RTX_FIXED_ANGLE)
        B.rtx_trace_rays(plan._handle, None, None, len(pairs), C.c_void_p(out2["theta"].data_ptr()), None, None,
                         None, None, C.c_void_p(st.data_ptr()), C.c_void_p(rowptr.data_ptr()),
                         C.c_void_p(colb.data_ptr()), C.c_void_p(valb.data_ptr()), 10, C.c_void_p(0))
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("case", ["fisheye", "gauss"])
def test_fan_start_matches_oracle(rtx, prec, case):
    """Fan start, all pairs: against the oracle's own fan start pair by pair."""
    if case == "fisheye":
        cfg, c = synth.make_config("c1_fisheye_128")
        h, ring = cfg["h"], (cfg["n_elem"], cfg["radius"], 0.0)
        ny, nx = c.shape
    else:
        ny = nx = 96
        h = 0.5e-3
        c = _gauss(nx, h, seed=19)
        ring = (40, 0.45 * nx * h * 0.9, 0.1)
    pairs = synth.all_pairs(ring[0])
    plan = rtx.Plan(nx, ny, h, *ring, prec=prec)
    out = {k: _np(v) for k, v in plan.trace(_dev(c), fan=True).items()}
    s0, r0 = plan.region_stats(0)
    s1, r1 = plan.region_stats(1)
    plan.close()
    assert r0 == len(pairs)  # the coarse fan pass traces every straight ray once
    ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs, fan=True)
    _check_linked(out, ref, c, h, ring, pairs, prec, 1e-3)
    assert r1 == out["n_marches"].sum()  # a pair's rays are the linking pass's


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_fan_start_full_size_sampled(rtx, prec):
    """256x256 Gaussian workload, fan start on the GPU at full size; sampled
    pairs re-traced by the oracle and compared with its straight-start roots."""
    cfg, c = synth.make_config("c2_gauss_256")
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    pairs = synth.all_pairs(cfg["n_elem"])
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], *ring, prec=prec)
    out = {k: _np(v) for k, v in plan.trace(_dev(c), fan=True).items()}
    plan.close()
    assert np.all(out["status"] == oracle.LINKED)
    assert out["n_marches"].max() <= 6
    idx = np.sort(np.random.default_rng(5).choice(len(pairs), 600, replace=False))
    ref = oracle.trace(oracle.grid_medium(c, cfg["h"]), ring, pairs[idx])
    _check_linked(out, ref, c, cfg["h"], ring, pairs, prec, cfg["tol_px"], idx, same_path=False)
