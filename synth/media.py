"""Sound-speed media on a node grid centred on the ring centre.

Grid convention: node (ix, iy) sits at x = (ix - (nx-1)/2) h, y = (iy - (ny-1)/2) h
(metres), and arrays are row-major ``c[iy, ix]`` in m/s, float64.
"""
import numpy as np


def node_coords(nx, ny, h):
    """Return (X, Y) metre coordinates of every node, each shaped [ny, nx]."""
    x = (np.arange(nx, dtype=np.float64) - 0.5 * (nx - 1)) * h
    y = (np.arange(ny, dtype=np.float64) - 0.5 * (ny - 1)) * h
    return np.meshgrid(x, y, indexing="xy")


def homogeneous(nx, ny, c0=1500.0):
    return np.full((ny, nx), float(c0), dtype=np.float64)


def linear_gradient(nx, ny, h, c0=1500.0, gx=0.0, gy=0.0):
    """c = c0 + gx*x + gy*y (gx, gy in 1/s)."""
    X, Y = node_coords(nx, ny, h)
    return c0 + gx * X + gy * Y


def fisheye(nx, ny, h, c0=1500.0, R=0.04):
    """Maxwell fish-eye in sound speed: c = c0 (1 + |x|^2 / R^2), i.e. refractive
    index n = n0 / (1 + (r/R)^2) with n proportional to 1/c (paper, Section 4)."""
    X, Y = node_coords(nx, ny, h)
    return c0 * (1.0 + (X * X + Y * Y) / (R * R))


def gaussian_inclusions(nx, ny, h, seed, n_incl=12, c0=1500.0, amp=60.0,
                        sigma=(0.002, 0.010), r_max=0.045):
    """Background c0 plus ``n_incl`` Gaussian bumps A exp(-d^2 / (2 s^2)).

    A ~ U(-amp, amp), s ~ U(sigma), centres uniform in area inside radius r_max
    (radius r_max * sqrt(u), angle uniform)."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-amp, amp, n_incl)
    s = rng.uniform(sigma[0], sigma[1], n_incl)
    rr = r_max * np.sqrt(rng.uniform(0.0, 1.0, n_incl))
    aa = rng.uniform(0.0, 2.0 * np.pi, n_incl)
    cx, cy = rr * np.cos(aa), rr * np.sin(aa)
    X, Y = node_coords(nx, ny, h)
    c = np.full((ny, nx), float(c0))
    for k in range(n_incl):
        d2 = (X - cx[k]) ** 2 + (Y - cy[k]) ** 2
        c += A[k] * np.exp(-d2 / (2.0 * s[k] ** 2))
    return c


def smooth_random(nx, ny, h, seed, sigma_m=0.004, peak=40.0, c0=1500.0):
    """White noise N(0,1) filtered by a Gaussian of std ``sigma_m`` (reflect
    boundary), scaled so that max |dc| = peak, on background c0."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, nx))
    f = gaussian_filter(w, sigma=sigma_m / h, mode="reflect")
    f *= peak / np.max(np.abs(f))
    return c0 + f


def striped_disc(nx, ny, h, radius=0.008, c_disc=1580.0, c0=1500.0, period=3):
    """One disc of the given radius at the origin; inside it, every ``period``-th
    node row (iy % period == 0) is set to c_disc, every other node is c0."""
    X, Y = node_coords(nx, ny, h)
    inside = X * X + Y * Y <= radius * radius
    rows = (np.arange(ny) % period == 0)[:, None]
    c = np.full((ny, nx), float(c0))
    c[inside & rows] = c_disc
    return c
