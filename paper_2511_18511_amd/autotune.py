"""Autotuner for the launch shape (rays per block) and the march step.

The step is chosen for accuracy first: every candidate step is traced and its
linked travel times are compared with those of the finest candidate; only steps
whose largest relative difference stays within ``rel_tol`` are eligible.  Among
the eligible (step, rays-per-block) combinations the fastest (median of timed
runs, HIP events on the current stream) wins.  Results are cached in a JSON
file keyed by the workload shape, so later plans of the same shape reuse them.
"""
import json
import os

import torch

DEFAULT_CACHE = os.environ.get("RTX_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                              "rtx_autotune.json"))
BLOCKS = (64, 128, 256)


def _key(plan, n_pairs, tag):
    return (f"{tag}|{plan.prec}|{plan._opts['integ']}|{plan.nx}x{plan.ny}|h={plan.h:.6g}|n_elem={plan.n_elem}|"
            f"R={plan.radius:.6g}|pairs={n_pairs}|tol={plan._opts['tol_px']:.3g}")


def load_cache(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=DEFAULT_CACHE):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(results, rel_tol):
    """results: list of dicts {ds_px, rays_per_block, ms, max_rel_dT}.  Returns
    the fastest entry whose step meets the accuracy target (the finest step is
    always eligible)."""
    finest = min(r["ds_px"] for r in results)
    ok = [r for r in results if r["ds_px"] == finest or r["max_rel_dT"] <= rel_tol]
    return min(ok, key=lambda r: r["ms"])


def _time_ms(fn, reps):
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    fn()  # warm-up
    for k in range(reps):
        ev[2 * k].record()
        fn()
        ev[2 * k + 1].record()
    torch.cuda.synchronize()
    t = sorted(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(reps))
    return t[len(t) // 2]


def tune_plan(plan, c, pairs=None, ds_candidates=(0.25,), blocks=BLOCKS, rel_tol=1e-6, reps=3,
              cache_path=DEFAULT_CACHE, use_cache=True):
    """Tunes a Plan on medium c (float64 [ny, nx] device) and applies the winner
    (set_launch + step).  Returns the chosen entry."""
    n = plan.n_all if pairs is None else int(pairs.shape[0])
    key = _key(plan, n, "plan") + f"|ds={sorted(ds_candidates)}|rt={rel_tol:g}"
    cache = load_cache(cache_path) if use_cache else {}
    if key in cache:
        best = cache[key]
    else:
        plan.set_medium(c)
        ref = None
        results = []
        for ds in sorted(ds_candidates):
            out = plan.trace(None, pairs=pairs, ds_px=ds)
            T = out["tof"].clone()
            if ref is None:
                ref = T
                err = 0.0
            else:
                ok = torch.isfinite(T) & torch.isfinite(ref)
                err = float(((T[ok] / ref[ok]) - 1).abs().max().item()) if bool(ok.any()) else float("inf")
            for b in blocks:
                plan.set_launch(b)
                ms = _time_ms(lambda: plan.trace(None, pairs=pairs, out=out, ds_px=ds), reps)
                results.append({"ds_px": ds, "rays_per_block": b, "ms": ms, "max_rel_dT": err})
        best = dict(pick(results, rel_tol))
        best["candidates"] = results
        if use_cache:
            cache[key] = best
            save_cache(cache, cache_path)
    plan.set_launch(best["rays_per_block"])
    plan._opts["ds_px"] = best["ds_px"]
    return best


def tune_batch(make_batch, blocks=BLOCKS, reps=3, cache_path=DEFAULT_CACHE, key=None, use_cache=True):
    """Tunes the rays per block of a Batch: make_batch(rays_per_block) builds one;
    the fastest graph replay wins.  Returns (batch, entry)."""
    cache = load_cache(cache_path) if (use_cache and key) else {}
    if key and key in cache:
        entry = cache[key]
        return make_batch(entry["rays_per_block"]), entry
    results = []
    for b in blocks:
        bt = make_batch(b)
        ms = _time_ms(bt.run, reps)
        results.append({"rays_per_block": b, "ms": ms})
        bt.close()
    entry = dict(min(results, key=lambda r: r["ms"]))
    entry["candidates"] = results
    if use_cache and key:
        cache[key] = entry
        save_cache(cache, cache_path)
    return make_batch(entry["rays_per_block"]), entry
