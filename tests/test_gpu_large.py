"""The 512x512, 1024-element striped-disc workload (1,047,552 pairs) at full
size: FP32-compensated linked trace in the autotuned launch shape, sampled
against the oracle; the 64-frequency ray-Born-style adjoint on a seeded subset
of pairs against the oracle, and on all pairs for finiteness and linearity."""
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


def test_c4_full_size(rtx, tmp_path):
    from paper_2511_18511_amd import autotune

    cfg, c = synth.make_config("c4_stripes_512")
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    pairs = synth.all_pairs(cfg["n_elem"])
    n = len(pairs)
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], *ring, prec="f32c")
    cd = _dev(c)
    best = autotune.tune_plan(plan, cd, reps=1, cache_path=str(tmp_path / "tune.json"))
    cands = ", ".join("%d: %.1f ms" % (r["rays_per_block"], r["ms"]) for r in best["candidates"])
    print(f"\nautotuned rays per block: {best['rays_per_block']} ({cands})", flush=True)
    out = plan.trace(cd)
    st = out["status"].cpu().numpy()
    # the striped disc's row discontinuities make the misfit jump across zero for
    # a few pairs (no root): those must be the oracle's failures too
    assert np.mean(st == oracle.LINKED) > 0.99, np.bincount(st, minlength=4)
    rng = np.random.default_rng(4004)
    bad = np.nonzero(st != oracle.LINKED)[0]
    if len(bad):
        pick = np.sort(rng.choice(bad, min(40, len(bad)), replace=False))
        refb = oracle.trace(oracle.grid_medium(c, cfg["h"]), ring, pairs[pick])
        agree = np.mean(refb["status"] == st[pick])
        print(f"\n{len(bad)} unlinked pairs; oracle status agrees on {agree:.0%} of {len(pick)} sampled", flush=True)
        assert agree >= 0.9
    idx = np.sort(rng.choice(np.nonzero(st == oracle.LINKED)[0], 400, replace=False))
    th = out["theta"].cpu().numpy()
    T = out["tof"].cpu().numpy()
    chk = oracle.trace(oracle.grid_medium(c, cfg["h"]), ring, pairs[idx], theta=th[idx], fixed=True)
    assert np.abs(T[idx] / chk["tof"] - 1).max() < 1e-5
    assert chk["miss_px"].max() <= 1e-3 + 2e-4
    # same roots as the oracle's own linking on a sample
    ref = oracle.trace(oracle.grid_medium(c, cfg["h"]), ring, pairs[idx[:100]])
    ok = ref["status"] == oracle.LINKED
    assert np.abs(T[idx[:100]][ok] - ref["tof"][ok]).max() < 4e-3 * cfg["h"] / 1500 + 1e-5 * ref["tof"].max()

    freqs = list(np.linspace(cfg["f_lo"], cfg["f_hi"], cfg["n_freq"]))
    # subset adjoint against the oracle
    sub = np.sort(rng.choice(n, 4096, replace=False))
    r_sub = synth.complex_residual(len(sub), cfg["n_freq"], cfg["resid_seed"] + 1)
    psub = _dev(pairs[sub].astype(np.int32))
    isub = _dev(sub)
    g = plan.adjoint(out["theta"][isub], out["status"][isub], _dev(r_sub), pairs=psub, tof=out["tof"][isub],
                     freqs_hz=freqs)
    rho = oracle.rayborn_rho(T[sub], np.array(freqs), r_sub)
    gref = oracle.adjoint(c, cfg["h"], ring, pairs[sub], th[sub], rho, status=st[sub])
    err = np.linalg.norm(g.double().cpu().numpy() - gref) / np.linalg.norm(gref)
    assert err < 1e-5, err
    # all pairs: finite, and linear in the residual
    r_all = synth.complex_residual(n, cfg["n_freq"], cfg["resid_seed"])
    rd = _dev(r_all)
    g1 = plan.adjoint(out["theta"], out["status"], rd, tof=out["tof"], freqs_hz=freqs).double()
    g2 = plan.adjoint(out["theta"], out["status"], (2 * rd).contiguous(), tof=out["tof"], freqs_hz=freqs).double()
    assert bool(torch.isfinite(g1).all())
    assert float((g2 - 2 * g1).norm() / g1.norm()) < 1e-5
    plan.close()
