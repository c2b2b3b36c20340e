"""The five ring-array workloads and their seeded inputs.

Each config is a plain dict.  Geometry: ``n_elem`` point transducers evenly
spaced on a ring of ``radius`` metres centred on the grid, element k at angle
``phi0 + 2 pi k / n_elem``.  Every element emits once and all others record,
giving n_elem (n_elem - 1) ordered pairs.
"""
import math

import numpy as np

from . import media, volume

# Seeds: media 1000 + config number, residuals 2000 + config number,
# batched instance i: 3000 + i.
CONFIGS = {
    "c1_fisheye_128": dict(
        nx=128, ny=128, h=1.0e-3, n_elem=32, radius=0.060, phi0=0.0,
        medium="fisheye", medium_args=dict(c0=1500.0, R=0.040),
        integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
    ),
    "c2_gauss_256": dict(
        nx=256, ny=256, h=0.5e-3, n_elem=256, radius=0.060, phi0=0.0,
        medium="gaussian_inclusions", medium_args=dict(seed=1002),
        integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
        resid_seed=2002, resid_std=1e-4,
    ),
    "c3_smooth_384": dict(
        nx=384, ny=384, h=0.5e-3, n_elem=512, radius=0.090, phi0=0.0,
        medium="smooth_random", medium_args=dict(seed=1003),
        integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
        resid_seed=2003, resid_std=1e-4,
    ),
    "c4_stripes_512": dict(
        nx=512, ny=512, h=0.25e-3, n_elem=1024, radius=0.060, phi0=0.0,
        medium="striped_disc", medium_args=dict(),
        integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
        resid_seed=2004, n_freq=64, f_lo=0.5e6, f_hi=1.5e6,
    ),
}


# 3-D workload: a hemispherical bowl of point transducers around a volume of
# Gaussian blobs (the 3-D acquisition geometries of the ToF method, Sec. 3).
CONFIGS3 = {
    "c6_hemi_128": dict(
        n=128, h=0.75e-3, n_elem=256, radius=0.040,
        medium_args=dict(seed=1006, r_max=0.025),
        integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
    ),
}


def make_config3(name):
    """Return (cfg, c) for a named 3-D workload; c is float64 [n, n, n] and the
    elements are volume.hemisphere_elements(n_elem, radius)."""
    cfg = dict(CONFIGS3[name])
    cfg["name"] = name
    n, h = cfg["n"], cfg["h"]
    return cfg, volume.gaussian_inclusions3(n, n, n, h, **cfg["medium_args"])


def build_medium(cfg):
    kind = cfg["medium"]
    nx, ny, h = cfg["nx"], cfg["ny"], cfg["h"]
    args = dict(cfg.get("medium_args", {}))
    if kind == "fisheye":
        return media.fisheye(nx, ny, h, **args)
    if kind == "gaussian_inclusions":
        return media.gaussian_inclusions(nx, ny, h, **args)
    if kind == "smooth_random":
        return media.smooth_random(nx, ny, h, **args)
    if kind == "striped_disc":
        return media.striped_disc(nx, ny, h, **args)
    if kind == "homogeneous":
        return media.homogeneous(nx, ny, **args)
    raise ValueError(f"unknown medium {kind!r}")


def make_config(name):
    """Return (cfg, c) for a named workload; c is float64 [ny, nx]."""
    cfg = dict(CONFIGS[name])
    cfg["name"] = name
    return cfg, build_medium(cfg)


def all_pairs(n_elem):
    """All ordered (emitter, receiver) pairs, e != r, as int32 [n, 2].

    Row i = e (n_elem - 1) + (r if r < e else r - 1)."""
    e = np.repeat(np.arange(n_elem, dtype=np.int32), n_elem - 1)
    k = np.tile(np.arange(n_elem - 1, dtype=np.int32), n_elem)
    r = np.where(k < e, k, k + 1).astype(np.int32)
    return np.stack([e, r], axis=1)


def real_residual(n, seed, std=1e-4):
    """Real per-pair residual r ~ N(0, std^2) (seconds)."""
    return np.random.default_rng(seed).normal(0.0, std, n)


def complex_residual(n, n_freq, seed):
    """Complex residual r ~ CN(0, 1): real and imaginary parts each N(0, 1/2),
    complex64 [n, n_freq]."""
    rng = np.random.default_rng(seed)
    re = rng.normal(0.0, math.sqrt(0.5), (n, n_freq))
    im = rng.normal(0.0, math.sqrt(0.5), (n, n_freq))
    return (re + 1j * im).astype(np.complex64)


def c5_instances(n_inst=48, seed_base=3000, h=0.5e-3):
    """Independent phantoms of uneven size: grid side uniform in
    {64,128,192,256,384}, ring elements uniform in {64,128,256,512}, ring radius
    0.9375 of the grid half-width, Gaussian inclusions centred within 0.75 of the
    ring radius.  Returns a list of (cfg, c)."""
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng(seed_base + i)
        side = int(rng.choice([64, 128, 192, 256, 384]))
        n_elem = int(rng.choice([64, 128, 256, 512]))
        radius = 0.9375 * side * h / 2.0
        cfg = dict(nx=side, ny=side, h=h, n_elem=n_elem, radius=radius, phi0=0.0,
                   medium="gaussian_inclusions",
                   medium_args=dict(seed=seed_base + i, r_max=0.75 * radius),
                   integ="rk4", ds_px=0.25, tol_px=1e-3, max_marches=30,
                   name=f"c5_inst{i:02d}")
        out.append((cfg, build_medium(cfg)))
    return out

