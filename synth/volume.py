"""3-D sound-speed volumes and hemispherical arrays.

Grid convention: node (ix, iy, iz) sits at ((ix - (nx-1)/2) h, (iy - (ny-1)/2) h,
(iz - (nz-1)/2) h) (metres); arrays are ``c[iz, iy, ix]`` in m/s, float64.
"""
import math

import numpy as np


def node_coords3(nx, ny, nz, h):
    """(X, Y, Z) metre coordinates of every node, each shaped [nz, ny, nx]."""
    ax = [(np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * h for n in (nx, ny, nz)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X, Y, Z


def gaussian_inclusions3(nx, ny, nz, h, seed, n_incl=12, c0=1500.0, amp=60.0, sigma=(0.002, 0.010),
                         r_max=0.040):
    """Background c0 plus ``n_incl`` Gaussian blobs A exp(-d^2 / (2 s^2)):
    A ~ U(-amp, amp), s ~ U(sigma), centres uniform in volume inside a ball of
    radius r_max."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-amp, amp, n_incl)
    s = rng.uniform(sigma[0], sigma[1], n_incl)
    rr = r_max * np.cbrt(rng.uniform(0.0, 1.0, n_incl))
    v = rng.standard_normal((n_incl, 3))
    cen = v / np.linalg.norm(v, axis=1, keepdims=True) * rr[:, None]
    X, Y, Z = node_coords3(nx, ny, nz, h)
    c = np.full((nz, ny, nx), float(c0))
    for k in range(n_incl):
        d2 = (X - cen[k, 0]) ** 2 + (Y - cen[k, 1]) ** 2 + (Z - cen[k, 2]) ** 2
        c += A[k] * np.exp(-d2 / (2.0 * s[k] ** 2))
    return c


def fisheye3(nx, ny, nz, h, c0=1500.0, R=0.04):
    """Maxwell fish-eye in sound speed, c = c0 (1 + |x|^2 / R^2) (Section 4, dim = 3)."""
    X, Y, Z = node_coords3(nx, ny, nz, h)
    return c0 * (1.0 + (X * X + Y * Y + Z * Z) / (R * R))


def linear_gradient3(nx, ny, nz, h, c0=1500.0, a=(0.0, 0.0, 0.0)):
    X, Y, Z = node_coords3(nx, ny, nz, h)
    return c0 + a[0] * X + a[1] * Y + a[2] * Z


def hemisphere_elements(n, radius, z_max=0.0):
    """n points on the sphere of the given radius with z <= z_max * radius (a
    hemispherical bowl for z_max = 0), spread by a Fibonacci lattice in z.
    Returns float64 [n, 3] metres."""
    golden = math.pi * (3.0 - math.sqrt(5.0))
    k = np.arange(n, dtype=np.float64)
    z = -1.0 + (1.0 + z_max) * (k + 0.5) / n
    r = np.sqrt(1.0 - z * z)
    phi = golden * k
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1) * radius
