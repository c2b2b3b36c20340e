"""Batched instances (one persistent launch over every pair of every instance,
captured in a HIP graph) against single-plan runs and the oracle, graph
replays, and the 48-instance uneven workload at full size."""
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


def _small_instances(k=5):
    out = []
    for i, (n, ne) in enumerate([(48, 8), (64, 16), (80, 12), (96, 20), (64, 24)][:k]):
        h = 0.5e-3
        c = synth.gaussian_inclusions(n, n, h, seed=500 + i, r_max=0.3 * n * h)
        out.append(dict(c=c, h=h, n_elem=ne, radius=0.42 * n * h, phi0=0.1 * i))
    return out


@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("rpb", [64, 256])
def test_batch_matches_single_plans_and_oracle(rtx, prec, rpb):
    specs = _small_instances()
    rng = np.random.default_rng(9)
    dspecs = []
    for s in specs:
        n = s["n_elem"] * (s["n_elem"] - 1)
        s["rho"] = rng.standard_normal(n) * 1e-4
        dspecs.append(dict(s, c=_dev(s["c"]), resid=_dev(s["rho"])))
    bt = rtx.Batch(dspecs, prec=prec, rays_per_block=rpb)
    bt.run()
    torch.cuda.synchronize()
    first = [{k: v.detach().cpu().numpy().copy() for k, v in o.items() if k != "c"} for o in bt.inst]
    fwd, done = bt.times()
    assert all(np.isfinite(fwd)) and all(f > 0 for f in fwd) and all(d >= f for f, d in zip(fwd, done))
    tol_t = 1e-12 if prec == "f64" else 1e-5
    for s, o in zip(specs, first):
        ring = (s["n_elem"], s["radius"], s["phi0"])
        pairs = synth.all_pairs(s["n_elem"])
        n = s["c"].shape[0]
        # single-plan GPU run of the same instance
        plan = rtx.Plan(n, n, s["h"], *ring, prec=prec)
        single = plan.trace(_dev(s["c"]))
        g1 = plan.adjoint(single["theta"], single["status"], _dev(s["rho"]))
        plan.close()
        assert np.array_equal(o["status"], single["status"].cpu().numpy())
        np.testing.assert_allclose(o["tof"], single["tof"].cpu().numpy(), rtol=tol_t)
        # oracle re-trace of the batch's angles, and its adjoint
        ok = o["status"] == oracle.LINKED
        assert ok.all()
        chk = oracle.trace(oracle.grid_medium(s["c"], s["h"]), ring, pairs, theta=o["theta"], fixed=True)
        assert np.abs(o["tof"] / chk["tof"] - 1).max() < tol_t
        assert chk["miss_px"].max() <= 1e-3 + (0 if prec == "f64" else 2e-4)
        gref = oracle.adjoint(s["c"], s["h"], ring, pairs, o["theta"], s["rho"], status=o["status"])
        err = np.linalg.norm(o["grad"].astype(np.float64) - gref) / np.linalg.norm(gref)
        assert err < (1e-11 if prec == "f64" else 1e-5), err
        np.testing.assert_allclose(o["grad"], g1.cpu().numpy(), rtol=0, atol=1e-5 * np.abs(gref).max())
    # graph replays with eager work in between: every replay equals the first
    for rep in range(3):
        for o in bt.inst:
            o["grad"].zero_()
        torch.ones(1000, device=DEV).sum().item()
        bt.run()
        torch.cuda.synchronize()
        for o, f in zip(bt.inst, first):
            assert np.array_equal(o["status"].cpu().numpy(), f["status"])
            np.testing.assert_array_equal(o["tof"].cpu().numpy(), f["tof"])
            np.testing.assert_allclose(o["grad"].cpu().numpy(), f["grad"], rtol=0,
                                       atol=1e-6 * np.abs(f["grad"]).max())
    bt.close()


def test_batch_rejects_mixed_adjoint(rtx):
    specs = _small_instances(2)
    d = [dict(s, c=_dev(s["c"])) for s in specs]
    d[0]["resid"] = _dev(np.zeros(specs[0]["n_elem"] * (specs[0]["n_elem"] - 1)))
    with pytest.raises(rtx.RtxError):
        rtx.Batch(d)


def test_c5_uneven_instances_full_size(rtx):
    """48 instances (grid side 64..384, 64..512 elements, ~4 M pairs) in one
    graph, FP32-compensated forward + adjoint; 16 sampled pairs per instance
    are re-traced by the oracle; per-instance completion times are reported."""
    insts = synth.c5_instances()
    rng = np.random.default_rng(3005)
    dspecs = []
    for cfg, c in insts:
        n = cfg["n_elem"] * (cfg["n_elem"] - 1)
        dspecs.append(dict(c=_dev(c), h=cfg["h"], n_elem=cfg["n_elem"], radius=cfg["radius"], phi0=0.0,
                           resid=_dev(rng.normal(0, 1e-4, n))))
    bt = rtx.Batch(dspecs, prec="f32c")
    bt.run()
    torch.cuda.synchronize()
    fwd, done = bt.times()
    print(f"\n48 instances, {bt.n_pairs} pairs: completion p50 {np.percentile(done, 50):.2f} ms, "
          f"p99 {np.percentile(done, 99):.2f} ms", flush=True)
    for (cfg, c), o in zip(insts, bt.inst):
        st = o["status"].cpu().numpy()
        assert np.mean(st == oracle.LINKED) > 0.999
        pairs = synth.all_pairs(cfg["n_elem"])
        idx = rng.choice(np.nonzero(st == oracle.LINKED)[0], 16, replace=False)
        ring = (cfg["n_elem"], cfg["radius"], 0.0)
        th = o["theta"].cpu().numpy()[idx]
        chk = oracle.trace(oracle.grid_medium(c, cfg["h"]), ring, pairs[idx], theta=th, fixed=True)
        T = o["tof"].cpu().numpy()[idx]
        assert np.abs(T / chk["tof"] - 1).max() < 1e-5
        assert chk["miss_px"].max() <= 1e-3 + 2e-4
    bt.close()


def test_autotune_picks_a_candidate(rtx, tmp_path):
    from paper_2511_18511_amd import autotune

    n, h = 96, 0.5e-3
    c = _dev(synth.gaussian_inclusions(n, n, h, seed=77, r_max=0.015))
    plan = rtx.Plan(n, n, h, 32, 0.45 * n * h * 0.9, prec="f32c")
    cache = str(tmp_path / "tune.json")
    best = autotune.tune_plan(plan, c, ds_candidates=(0.25, 0.5), rel_tol=1e-5, cache_path=cache)
    assert best["rays_per_block"] in autotune.BLOCKS and best["ds_px"] in (0.25, 0.5)
    assert len(best["candidates"]) == 6
    again = autotune.tune_plan(plan, c, ds_candidates=(0.25, 0.5), rel_tol=1e-5, cache_path=cache)
    assert again["rays_per_block"] == best["rays_per_block"]
    out = plan.trace(c)
    assert bool((out["status"] == 0).all())
    plan.close()
