"""Host logic of the autotuner: accuracy-gated choice and the on-disk cache."""
from paper_2511_18511_amd import autotune


def test_pick_respects_accuracy_target():
    res = [
        {"ds_px": 0.25, "rays_per_block": 64, "ms": 5.0, "max_rel_dT": 0.0},
        {"ds_px": 0.25, "rays_per_block": 256, "ms": 4.0, "max_rel_dT": 0.0},
        {"ds_px": 0.5, "rays_per_block": 128, "ms": 2.5, "max_rel_dT": 5e-7},
        {"ds_px": 1.0, "rays_per_block": 128, "ms": 1.0, "max_rel_dT": 3e-5},
    ]
    assert autotune.pick(res, 1e-6) == res[2]
    assert autotune.pick(res, 1e-9) == res[1]  # only the finest step is eligible
    assert autotune.pick(res, 1e-4) == res[3]


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(p) == {}
    autotune.save_cache({"k": {"rays_per_block": 128}}, p)
    assert autotune.load_cache(p) == {"k": {"rays_per_block": 128}}
