"""Benchmark: linked ray tracing (travel time + path length) plus the adjoint
A^T r on the 256x256 Gaussian-inclusion ring workload (0.5 mm pixels, 256
elements on a 60 mm ring, 65,280 ordered pairs, RK4 at 0.25 px, 1e-3 px linking
tolerance), FP32-compensated (headline) and plain FP64, on one GPU.

One step = pack the medium (node gradient + cell coefficients) -> linked trace
of every pair (cold start seeded by each emitter's fan of straight rays; the
plain straight-ray start is measured too) -> adjoint of the path weights for a
residual r ~ N(0, (1e-4 s)^2).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

WORKLOAD = "c2_gauss_256"
# algorithmic cost of one RK4 step of one ray: 4 stages x 4
# cell corners x 3 fields of gathered medium values, and the FP32 flops of the
# interpolation, ray equation, RK4 combination, renormalisation and quadrature
GATHER_VALUES_PER_STEP = 4 * 4 * 3
FLOPS_PER_STEP = 170
# ALU ceiling of the FP32 path: the build disables packed FP32 (v_pk_*_f32), so
# one FMA per lane per cycle: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz.
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # 78.6
PEAK_FP32_TFLOPS = 157.3  # published FP32 vector peak (with packed math)
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def run_gpu(prec, c_host, cfg, steps, warmup, resid_host, fan=True):
    import torch

    import paper_2511_18511_amd as rtx

    dev = torch.device("cuda", 0)
    c = torch.from_numpy(c_host).to(dev)
    resid = torch.from_numpy(resid_host).to(dev)
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], cfg["n_elem"], cfg["radius"], cfg["phi0"], prec=prec,
                    integ=cfg["integ"], ds_px=cfg["ds_px"], tol_px=cfg["tol_px"], max_marches=cfg["max_marches"])
    n = plan.n_all
    out = plan.trace(c, fan=fan)  # allocates the output tensors once
    grad = torch.zeros(cfg["ny"], cfg["nx"], dtype=plan.real, device=dev)

    def step():
        plan.set_medium(c)
        plan.trace(None, out=out, fan=fan)
        grad.zero_()
        plan.adjoint(out["theta"], out["status"], resid, weight="length", grad=grad)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.timing(True)  # HIP events around every kernel, on its launch stream
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = plan.timings()
    plan.timing(False)
    trace_steps, trace_rays, adj_steps = plan.stats()
    link_region = 1 if fan else 0  # the dominant kernel: the linking pass
    link_steps, link_rays = plan.region_stats(link_region)
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in tm.items()}
    st = out["status"].cpu().numpy()
    fwd_ms = avg["pack"] + avg["trace"] + avg["fan_seed"] + avg["fan_link"]
    res = {
        "prec": prec,
        "linking_start": "fan" if fan else "straight",
        "wall_s": wall,
        "ms_per_step": 1e3 * wall / steps,
        "rays_per_s": n * steps / wall,
        "kernel_ms": avg,
        "forward_ms": fwd_ms,
        "adjoint_ms": avg["adjoint"],
        "forward_rays_per_s": n / (fwd_ms * 1e-3),
        "dominant_kernel": "linking pass (k_link2, fan-seeded, two lanes per pair)" if fan else "k_trace",
        "dominant_ms": avg["fan_link"] if fan else avg["trace"],
        "dominant_rk_steps": int(link_steps),
        "trace_rk_steps": int(trace_steps),
        "trace_rays": int(trace_rays),
        "adjoint_rk_steps": int(adj_steps),
        "linked_fraction": float(np.mean(st == rtx.RTX_RAY_LINKED)),
        "mean_marches": float(out["n_marches"].double().mean().item()),
        "max_marches": int(out["n_marches"].max().item()),
    }
    plan.close()
    return res, out


def run_sart(c_host, cfg, iters=10):
    """The path weights W of the workload's linked rays (CSR with merged rows,
    wall time of the call that emits them), and SART (Sec. 3.1) on that FP32
    system matrix: the once-per-call setup (sums and the device transpose of
    W) and the time of one
    iteration (residual pass over the rows, back-projection pass over the
    columns), with its HBM rate against the algorithmic bytes of an iteration."""
    import torch

    import paper_2511_18511_amd as rtx

    dev = torch.device("cuda", 0)
    plan = rtx.Plan(cfg["nx"], cfg["ny"], cfg["h"], cfg["n_elem"], cfg["radius"], cfg["phi0"], prec="f32c",
                    integ=cfg["integ"], ds_px=cfg["ds_px"], tol_px=cfg["tol_px"], max_marches=cfg["max_marches"])
    out = plan.trace(torch.from_numpy(c_host).to(dev), weights=True, fan=False)
    rp, col, val = out["w_rowptr"], out["w_col"], out["w_val"]

    def timed_weights():  # the path weights W of all linked rays at their angles (CSR, merged rows)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.weights(out["theta"])
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3

    w_ms = min(timed_weights() for _ in range(3))
    n_rows, nnz, nodes = rp.shape[0] - 1, col.shape[0], cfg["nx"] * cfg["ny"]
    b = torch.from_numpy(np.random.default_rng(5).standard_normal(n_rows) * 1e-6).to(dev)
    x = torch.zeros(cfg["ny"], cfg["nx"], dtype=torch.float64, device=dev)
    plan.sart(rp, col, val, b, x=x, n_iter=3)

    def timed(n_iter):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        plan.sart(rp, col, val, b, x=x, n_iter=n_iter)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    t1 = min(timed(1) for _ in range(3))
    tn = min(timed(1 + iters) for _ in range(3))
    per = (tn - t1) / iters  # one iteration: a CSR residual pass and a CSC back-projection pass
    setup = t1 - per  # row/column sums and the transpose, once per call
    plan.close()
    # per iteration: W's columns/values in both layouts (int32 + FP32 each),
    # rowptr/b/M/r per row, colptr/V/x per node
    bytes_it = 2 * nnz * 8 + n_rows * 32 + nodes * 32
    ms = per * iters
    return {"rows": int(n_rows), "nnz": int(nnz), "weights_ms": w_ms, "iterations": iters, "setup_ms": setup,
            "ms_per_iteration": ms / iters,
            "bytes_per_iteration": int(bytes_it), "achieved_GBs": bytes_it / (ms / iters * 1e-3) / 1e9,
            "vs_hbm_peak_frac": bytes_it / (ms / iters * 1e-3) / 1e9 / PEAK_HBM_GBS}


def run_3d(prec, steps=5, warmup=2):
    """The 3-D workload (128^3 volume at 0.75 mm, 256-element hemispherical
    bowl of radius 40 mm, 65,280 pairs, 12 Gaussian blobs): linked tracing from
    the straight ray with Broyden-like updates (Sec. 3.4), ms per call and
    linked rays/s."""
    import torch

    import paper_2511_18511_amd as rtx

    cfg, c = synth.make_config3("c6_hemi_128")
    el = synth.hemisphere_elements(cfg["n_elem"], cfg["radius"])
    dev = torch.device("cuda", 0)
    cd = torch.from_numpy(c).to(dev)
    plan = rtx.Plan3(cfg["n"], cfg["n"], cfg["n"], cfg["h"], el, prec=prec, integ=cfg["integ"], ds_px=cfg["ds_px"],
                     tol_px=cfg["tol_px"], max_marches=cfg["max_marches"])
    for _ in range(warmup):
        out = plan.trace(cd)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        out = plan.trace(cd)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = out["status"].cpu().numpy()
    rk, rays = plan.stats()
    plan.close()
    return {"prec": prec, "pairs": plan.n_all, "ms_per_call": ms, "rays_per_s": plan.n_all / (ms * 1e-3),
            "linked_fraction": float(np.mean(st == 0)), "mean_marches": float(out["n_marches"].double().mean()),
            "max_marches": int(out["n_marches"].max()), "rk_steps": int(rk), "rays_traced": int(rays)}


def cpu_baseline(c, cfg, resid, max_seconds=30.0):
    """The FP64 oracle on the host cores: linked trace + adjoint of the same
    workload, pairs split over a thread pool (the oracle releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    threads = min(16, os.cpu_count() or 1)
    ring = (cfg["n_elem"], cfg["radius"], cfg["phi0"])
    pairs = synth.all_pairs(cfg["n_elem"])
    med = oracle.grid_medium(c, cfg["h"])
    # probe: time 2 x threads pairs, then size the sample to ~max_seconds/2
    rng = np.random.default_rng(0)
    order = rng.permutation(len(pairs))
    t0 = time.perf_counter()
    oracle.trace(med, ring, pairs[order[:64]])
    per_pair = (time.perf_counter() - t0) / 64
    n_sample = int(min(len(pairs), max(256, 0.5 * max_seconds * threads / max(per_pair, 1e-9))))
    sub = np.sort(order[:n_sample])
    chunks = np.array_split(sub, threads * 4)

    def work(idx):
        o = oracle.trace(med, ring, pairs[idx])
        g = oracle.adjoint(c, cfg["h"], ring, pairs[idx], o["theta"], resid[idx], status=o["status"])
        return g

    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, chunks))
    wall = time.perf_counter() - t0
    full = n_sample == len(pairs)
    return {"value": n_sample / wall, "unit": "linked rays/s", "cores": threads, "kind": "oracle",
            "sample": ("all" if full else f"{n_sample} of {len(pairs)} seeded-uniform") +
            f" pairs of the same workload, linked trace + adjoint, {wall:.1f} s wall"}


def measured_traffic(_unused=None):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    kernel source changed since the counters were taken."""
    import glob
    import hashlib

    src = os.path.join(ROOT, "paper_2511_18511_amd", "csrc", "rtx.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.json"))):
        try:
            d = json.load(open(path))
        except ValueError:
            continue
        if d.get("source_sha256") != sha:
            continue
        for name, v in d.get("kernels", {}).items():
            if name.startswith("k_link2<float, true, 4, false>"):  # the fan-seeded linking pass
                return v["fetch_bytes"] + v["write_bytes"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--fan-only", action="store_true", help="skip the straight-start comparison runs")
    ap.add_argument("--no-sart", action="store_true", help="skip the SART measurement")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 256 MiB device-to-device copy (the reference kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profile)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path needs no cross-GPU exchange "
              "for the forward pass, see DESIGN.md for how it shards", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        import torch

        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cfg, c = synth.make_config(WORKLOAD)
    n_pairs = cfg["n_elem"] * (cfg["n_elem"] - 1)
    resid = synth.real_residual(n_pairs, cfg["resid_seed"], cfg["resid_std"])

    runs = {}
    for prec in ("f32c",) + (() if args.no_f64 else ("f64",)):
        for fan in (True,) if args.fan_only else (True, False):
            r, _ = run_gpu(prec, c, cfg, args.steps, args.warmup, resid, fan=fan)
            runs[(prec, fan)] = r
            print(f"# {prec} {r['linking_start']}: {r['ms_per_step']:.3f} ms/step, forward {r['forward_ms']:.3f} ms "
                  f"(max {r['max_marches']} rays/pair), adjoint {r['adjoint_ms']:.3f} ms", file=sys.stderr, flush=True)
    f32 = runs[("f32c", True)]
    f64 = runs.get(("f64", True))

    # roofline of the dominant kernel (the linking pass), per launch
    t_s = f32["dominant_ms"] * 1e-3
    flops = f32["dominant_rk_steps"] * FLOPS_PER_STEP
    roof = {"bound": "alu", "achieved": flops / t_s / 1e12, "peak": PEAK_FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
            "frac": flops / t_s / 1e12 / PEAK_FP32_NONPACKED_TFLOPS, "traffic": None,
            "frac_vs_published_157": flops / t_s / 1e12 / PEAK_FP32_TFLOPS}
    gbytes = f32["dominant_rk_steps"] * GATHER_VALUES_PER_STEP * 4
    # algorithmic gathered bytes (48 table values per step); the packed table
    # stays in L1/L2, so this rate is not bounded by HBM (the HBM traffic of
    # the launch is roofline["traffic"])
    gather = {"kernel": "k_link2<float> linking pass", "bytes_per_launch": gbytes,
              "achieved_GBs": gbytes / t_s / 1e9, "served_from": "L1/L2 (table cache-resident)"}

    roof["traffic"] = measured_traffic()
    sart = None if args.no_sart else run_sart(c, cfg)
    w3 = None
    if not args.no_3d:
        w3 = {p: run_3d(p) for p in ("f32c",) + (() if args.no_f64 else ("f64",))}
        for p, r in w3.items():
            print(f"# 3-D {p}: {r['ms_per_call']:.3f} ms per linked trace of {r['pairs']} pairs, "
                  f"{r['rays_per_s'] / 1e6:.2f} M rays/s, {r['mean_marches']:.2f} rays/pair (max {r['max_marches']})",
                  file=sys.stderr, flush=True)
    if sart:
        print(f"# path weights W: {sart['weights_ms']:.3f} ms for {sart['rows']} rows, {sart['nnz']} entries; "
              f"SART: setup {sart['setup_ms']:.3f} ms, {sart['ms_per_iteration']:.3f} ms/iteration "
              f"({sart['achieved_GBs']:.0f} GB/s)", file=sys.stderr, flush=True)
    cpu = None if args.no_cpu else cpu_baseline(c, cfg, resid)
    line = {
        "metric": "linked rays/s (ToF+path) and adjoint time; FP32-comp vs FP64 plain, same GPU",
        "value": f32["rays_per_s"],
        "unit": "linked rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256x256 grid at 0.5 mm, 12 seeded Gaussian inclusions on 1500 m/s, 256-element "
                               "ring of radius 60 mm, all 65,280 ordered pairs, RK4 ds=0.25 px, linking tol 1e-3 px, "
                               "cold start (fan-seeded secant), forward T+L then adjoint A^T r",
                   "pairs": n_pairs, "grid": [cfg["ny"], cfg["nx"]], "ring_elements": cfg["n_elem"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "f32c": f32,
        "f64": f64,
        "f32c_over_f64": (f32["rays_per_s"] / f64["rays_per_s"]) if f64 else None,
        "straight_start": {p: runs[(p, False)] for p, fan in runs if not fan},
        "gather": gather,
        "sart": sart,
        "hemisphere_3d": ({"workload": "128^3 volume at 0.75 mm, 12 Gaussian blobs on 1500 m/s, 256-element "
                                       "hemispherical bowl of radius 40 mm, all 65,280 ordered pairs, RK4 ds=0.25 px, "
                                       "Broyden-like linking to 1e-3 px from the straight ray", **w3} if w3 else None),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
