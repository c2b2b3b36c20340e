"""The ToF autograd Function (forward = linked trace, backward = frozen-path
travel-time gradient) on the GPU: against the oracle's gradient, against
finite differences of the GPU's own linked travel times, and in a short
gradient-descent ToF inversion on the 384x384 smooth-field workload."""
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
def test_tof_gradient_matches_oracle(rtx, prec):
    n, h = 96, 0.5e-3
    c = synth.gaussian_inclusions(n, n, h, seed=41, r_max=0.015)
    c_obs = synth.gaussian_inclusions(n, n, h, seed=42, r_max=0.015)
    ring = (24, 0.45 * n * h * 0.9, 0.0)
    pairs = synth.all_pairs(24)
    plan = rtx.Plan(n, n, h, *ring, prec=prec)
    T_obs = plan.trace(_dev(c_obs))["tof"].clone()
    cd = _dev(c).requires_grad_(True)
    state = {}
    T = rtx.ToF.apply(cd, plan, state)
    loss = 0.5 * ((T - T_obs) ** 2).sum()
    loss.backward()
    g = cd.grad.cpu().numpy()
    th = state["theta"].cpu().numpy()
    rho = (T - T_obs).detach().cpu().numpy()
    gref = oracle.adjoint(c, h, ring, pairs, th, rho, weight="dtdc", status=state["status"].cpu().numpy())
    err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    assert err < (1e-11 if prec == "f64" else 1e-5), err
    plan.close()


def test_c3_gradient_fd_and_descent(rtx):
    """384x384 smooth random field, 512-element ring (261,632 pairs): the
    autograd gradient of the ToF misfit against central differences on 16
    pixels (FP64, tight linking), then 10 gradient-descent iterations from a
    homogeneous start, each re-tracing with a warm start; the loss must fall."""
    cfg, c_true = synth.make_config("c3_smooth_384")
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    ny, nx, h = cfg["ny"], cfg["nx"], cfg["h"]
    plan = rtx.Plan(nx, ny, h, *ring, prec="f64", tol_px=1e-9)
    T_obs = plan.trace(_dev(c_true))["tof"].clone()
    c0 = _dev(np.full((ny, nx), 1500.0) + 0.25 * (c_true - 1500.0))

    def loss_of(c, state=None):
        T = rtx.ToF.apply(c, plan, state)
        return 0.5 * ((T - T_obs) ** 2).sum()

    cg = c0.clone().requires_grad_(True)
    state = {}
    L0 = loss_of(cg, state)
    L0.backward()
    g = cg.grad.detach().cpu().numpy()
    rng = np.random.default_rng(7)
    cand = np.argwhere(np.abs(g) > 0.1 * np.abs(g).max())
    pick = cand[rng.choice(len(cand), 16, replace=False)]
    eps = 0.5
    theta = state["theta"].clone()
    for iy, ix in pick:
        vals = []
        for sgn in (1, -1):
            cp = c0.clone()
            cp[iy, ix] += sgn * eps
            T = plan.trace(cp, theta=theta, warm=True)["tof"]
            vals.append(0.5 * float(((T - T_obs) ** 2).sum()))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - g[iy, ix]) <= 1e-2 * abs(g[iy, ix]), (iy, ix, fd, g[iy, ix])
    # gradient descent with backtracking on a max-norm step, warm-started traces
    plan32 = rtx.Plan(nx, ny, h, *ring, prec="f32c")
    c = c0.clone()
    st = {}
    losses = []
    step = 8.0  # m/s for the largest update
    for it in range(10):
        cg = c.clone().requires_grad_(True)
        L = 0.5 * ((rtx.ToF.apply(cg, plan32, st) - T_obs) ** 2).sum()
        L.backward()
        losses.append(float(L))
        d = cg.grad / cg.grad.abs().max()
        while step > 0.05:
            cn = c - step * d
            Ln = float(0.5 * ((plan32.trace(cn, theta=st["theta"], warm=True)["tof"] - T_obs) ** 2).sum())
            if Ln < losses[-1]:
                c = cn
                break
            step *= 0.5
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.7 * losses[0], losses
    plan.close()
    plan32.close()
