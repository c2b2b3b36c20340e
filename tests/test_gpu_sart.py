"""SART (Sec. 3.1's default solver of the linearised ToF subproblem) on the HIP
path, through the C ABI: iterates against the oracle's SART on the oracle's
system matrix, and at full size (the 256x256 workload's own matrix, 65,280
rows) the oracle's iterates, run-to-run identical bits, and the properties
that hold at any size: exact recovery of a constant slowness in one
iteration, linearity in the data, and a decreasing row-sum weighted
residual."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


@pytest.fixture(scope="module")
def rtx():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2511_18511_amd as rtx

    return rtx


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_sart_matches_oracle(rtx, prec):
    """The oracle's system matrix of a 64x64 Gaussian medium (20-element ring,
    380 rows, several waves' worth of ragged rows) plus an empty row with a
    huge datum; 8 iterations with lambda = 1.2 from a random start.  The matrix
    is rounded to the plan's precision on both sides; both compute in FP64."""
    n, h = 64, 1e-3
    c = synth.gaussian_inclusions(n, n, h, seed=71, r_max=0.015)
    ring = (20, 0.025, 0.0)
    pairs = synth.all_pairs(20)
    ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs)
    rp, col, val = oracle.weights_csr(c, h, ring, pairs, ref["theta"])
    # an empty row (a ray that never reached the ring) at position 7
    rp = np.insert(rp, 7, rp[7])
    rng = np.random.default_rng(72)
    b = rng.standard_normal(len(rp) - 1) * 1e-6
    b[7] = 1e30
    x0 = rng.standard_normal(n * n) * 1e-7
    vr = val.astype(np.float32 if prec == "f32c" else np.float64)
    want = oracle.sart(rp, col, vr.astype(np.float64), b, x0, 8, 1.2)
    plan = rtx.Plan(n, n, h, *ring, prec=prec, max_pairs=len(b))
    x = _dev(x0.reshape(n, n))
    plan.sart(_dev(rp), _dev(col), _dev(vr), _dev(b), x=x, n_iter=8, lam=1.2)
    got = x.cpu().numpy().ravel()
    untouched = np.ones(n * n, bool)
    untouched[col] = False
    assert untouched.any() and np.array_equal(got[untouched], x0[untouched])
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err < 1e-12, err
    # argument errors
    with pytest.raises(rtx.RtxError):
        plan.sart(_dev(rp), _dev(col), _dev(vr), _dev(b), x=x, lam=0.0)
    plan.close()
    small = rtx.Plan(n, n, h, *ring, prec=prec, max_pairs=10)
    with pytest.raises(rtx.RtxError):
        small.sart(_dev(rp), _dev(col), _dev(vr), _dev(b))
    small.close()


def test_sart_full_size_properties(rtx):
    """The 256x256 workload's own FP32 system matrix from the GPU trace."""
    cfg, c = synth.make_config("c2_gauss_256")
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], *ring, prec="f32c")
    out = plan.trace(_dev(c), weights=True)
    rp, col, val = out["w_rowptr"], out["w_col"], out["w_val"]
    n_rows = rp.shape[0] - 1
    rpn, coln, valn = rp.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy().astype(np.float64)
    M = np.add.reduceat(valn, rpn[:-1]) * (np.diff(rpn) > 0)
    V = np.bincount(coln, weights=valn, minlength=cfg["nx"] * cfg["ny"])
    print(f"\nW: {n_rows} rows, {len(coln)} entries", flush=True)
    # (a) a constant slowness s0 is recovered in one iteration wherever a ray
    # passes: b = W s0 = s0 M
    s0 = 1 / 1500.0
    x = plan.sart(rp, col, val, _dev(s0 * M), n_iter=1, lam=1.0).cpu().numpy().ravel()
    hit = V > 0
    assert np.abs(x[hit] / s0 - 1).max() < 1e-12
    assert np.all(x[~hit] == 0)
    # (b) linear in the data, from a zero start
    rng = np.random.default_rng(73)
    b = rng.standard_normal(n_rows) * 1e-6
    x1 = plan.sart(rp, col, val, _dev(b), n_iter=3, lam=1.0).cpu().numpy().ravel()
    x2 = plan.sart(rp, col, val, _dev(2 * b), n_iter=3, lam=1.0).cpu().numpy().ravel()
    assert np.abs(x2 - 2 * x1).max() <= 1e-12 * np.abs(x1).max()
    # (b') the same three iterations by the oracle on the same matrix; and a
    # second call gives the same bits (the transpose keeps rows ascending inside
    # a column, so no sum depends on the run)
    want = oracle.sart(rpn, coln, valn, b, np.zeros(cfg["nx"] * cfg["ny"]), 3, 1.0)
    assert np.abs(x1 - want).max() <= 1e-12 * np.abs(want).max()
    x1b = plan.sart(rp, col, val, _dev(b), n_iter=3, lam=1.0).cpu().numpy().ravel()
    assert np.array_equal(x1, x1b)
    # (c) the row-sum weighted residual of a consistent system decreases
    import scipy.sparse as sp

    W = sp.csr_matrix((valn, coln.astype(np.int64), rpn), shape=(n_rows, cfg["nx"] * cfg["ny"]))
    xt = rng.standard_normal(cfg["nx"] * cfg["ny"]) * 1e-5
    bt = W @ xt
    xg = torch.zeros(cfg["ny"], cfg["nx"], dtype=torch.float64, device=DEV)
    ok = M > 0
    res = []
    for _ in range(4):
        plan.sart(rp, col, val, _dev(bt), x=xg, n_iter=1, lam=1.0)
        r = bt - W @ xg.cpu().numpy().ravel()
        res.append(np.sqrt(np.sum(r[ok] ** 2 / M[ok])))
    print("weighted residual over iterations: " + ", ".join("%.3e" % v for v in res), flush=True)
    assert all(b2 < b1 for b1, b2 in zip(res, res[1:]))
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_sart_leaves_out_stray_entries(rtx, prec):
    """Entries in no row (before the first row pointer and after the last) and
    entries whose column lies outside the grid (-1, n*n, n*n + 7) take no part:
    the result equals the one on the clean matrix, bit for bit (the transpose
    sorts them into the last column, flagged; the grid's last node lies
    outside the ring, so no kept entry shares that column, and the bad columns
    come after row 5's own entries, so those keep their lanes)."""
    n, h = 32, 1e-3
    c = synth.gaussian_inclusions(n, n, h, seed=75, r_max=0.008)
    ring = (12, 0.013, 0.0)
    pairs = synth.all_pairs(12)
    ref = oracle.trace(oracle.grid_medium(c, h), ring, pairs)
    rp, col, val = oracle.weights_csr(c, h, ring, pairs, ref["theta"])
    rng = np.random.default_rng(76)
    b = rng.standard_normal(len(rp) - 1) * 1e-6
    vr = val.astype(np.float32 if prec == "f32c" else np.float64)
    plan = rtx.Plan(n, n, h, *ring, prec=prec, max_pairs=len(b))
    x_clean = _dev(np.zeros((n, n)))
    plan.sart(_dev(rp), _dev(col), _dev(vr), _dev(b), x=x_clean, n_iter=4, lam=1.0)
    assert n * n - 1 not in set(col.tolist())
    # three stray entries at the end of row 5 (bad columns), two before row 0, three after the last row
    bad = np.array([-1, n * n, n * n + 7], np.int32)
    k5 = rp[6]
    col2 = np.concatenate([[3, 4], col[:k5], bad, col[k5:], [1, 2, 3]]).astype(np.int32)
    val2 = np.concatenate([[1.0, 2.0], vr[:k5], [5.0, 6.0, 7.0], vr[k5:], [1.0, 1.0, 1.0]]).astype(vr.dtype)
    rp2 = rp + 2
    rp2[6:] += 3
    x_stray = _dev(np.zeros((n, n)))
    plan.sart(_dev(rp2), _dev(col2), _dev(val2), _dev(b), x=x_stray, n_iter=4, lam=1.0)
    plan.close()
    assert np.abs(x_clean.cpu().numpy()).max() > 0
    assert np.array_equal(x_clean.cpu().numpy(), x_stray.cpu().numpy())
