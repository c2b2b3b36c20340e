"""Closed-form ray solutions used to pin the oracle (no ray marching here).

All positions are in metres relative to the ring centre.
"""
import math

import numpy as np


def ring_points(n_elem, radius, phi0=0.0):
    a = phi0 + 2.0 * math.pi * np.arange(n_elem) / n_elem
    return radius * np.stack([np.cos(a), np.sin(a)], axis=1), a


def _wrap(a):
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def launch_theta(e, tangent):
    """Angle of a launch direction relative to the inward normal -e/|e|."""
    phi_e = math.atan2(e[1], e[0])
    return _wrap(math.atan2(tangent[1], tangent[0]) - (phi_e + math.pi))


# ------------------------------------------------------------ homogeneous --
def homogeneous(e, r, c0):
    d = float(np.linalg.norm(np.asarray(r) - np.asarray(e)))
    return d / c0, d


# --------------------------------------------------------- linear gradient --
def linear_tof(e, r, c0, G):
    """Travel time in c = c0 + G.x: arccosh(1 + g^2 |r-e|^2 / (2 c1 c2)) / g."""
    G = np.asarray(G, float)
    g = float(np.linalg.norm(G))
    c1 = c0 + G @ np.asarray(e)
    c2 = c0 + G @ np.asarray(r)
    d2 = float(np.sum((np.asarray(r) - np.asarray(e)) ** 2))
    return math.acosh(1.0 + g * g * d2 / (2.0 * c1 * c2)) / g


def linear_path(e, r, c0, G):
    """Rays in a linear medium are circular arcs centred on the line c = 0.
    Returns (arc length L, launch angle theta relative to the inward normal)."""
    G = np.asarray(G, float)
    e = np.asarray(e, float)
    r = np.asarray(r, float)
    g = float(np.linalg.norm(G))
    gh = G / g
    th = np.array([-gh[1], gh[0]])
    xl = -c0 * G / (g * g)  # foot of the line c = 0
    a1, a2 = e - xl, r - xl
    tau = (a1 @ a1 - a2 @ a2) / (2.0 * (a1 - a2) @ th)
    xc = xl + tau * th
    r1, r2 = e - xc, r - xc
    rho = float(np.linalg.norm(r1))
    cross = r1[0] * r2[1] - r1[1] * r2[0]
    alpha = math.atan2(abs(cross), float(r1 @ r2))
    tan = np.array([-r1[1], r1[0]]) if cross > 0 else np.array([r1[1], -r1[0]])
    return rho * alpha, launch_theta(e, tan / rho)


# -------------------------------------------------------------- fish-eye --
def _stereo(u):
    n2 = float(u @ u)
    return np.array([2.0 * u[0], 2.0 * u[1], n2 - 1.0]) / (n2 + 1.0)


def fisheye_tof(e, r, c0, R):
    """c = c0 (1 + |x|^2/R^2): the metric ds/c is (R / 2c0) times the unit-sphere
    metric under stereographic projection of x/R, rays are great circles.  With
    the ring outside |x| = R the ray inside the ring is the major arc."""
    cosang = float(np.clip(_stereo(np.asarray(e) / R) @ _stereo(np.asarray(r) / R), -1.0, 1.0))
    return R * (2.0 * math.pi - math.acos(cosang)) / (2.0 * c0)


def fisheye_path(e, r, R):
    """Ray = arc of the circle through e, r and the conjugate point
    e* = -R^2 e / |e|^2 (a straight chord when the three are collinear).
    Returns (arc length L inside the ring, launch angle theta)."""
    e = np.asarray(e, float)
    r = np.asarray(r, float)
    es = -R * R * e / float(e @ e)
    ax, ay = e
    bx, by = r
    cx, cy = es
    d = 2.0 * (ax * (by - cy) + bx * (cy - ay) + cx * (ay - by))
    if abs(d) < 1e-14 * float(e @ e):
        return float(np.linalg.norm(r - e)), 0.0
    ux = ((ax * ax + ay * ay) * (by - cy) + (bx * bx + by * by) * (cy - ay) + (cx * cx + cy * cy) * (ay - by)) / d
    uy = ((ax * ax + ay * ay) * (cx - bx) + (bx * bx + by * by) * (ax - cx) + (cx * cx + cy * cy) * (bx - ax)) / d
    ctr = np.array([ux, uy])
    rho = float(np.linalg.norm(e - ctr))
    ang = lambda p: math.atan2(p[1] - ctr[1], p[0] - ctr[0])  # noqa: E731
    a_e, a_r, a_s = ang(e), ang(r), ang(es)
    ccw_er = (a_r - a_e) % (2 * math.pi)
    ccw_es = (a_s - a_e) % (2 * math.pi)
    if ccw_es < ccw_er:  # e* lies on the counter-clockwise arc e -> r
        arc = ccw_er
        tan = np.array([-(e - ctr)[1], (e - ctr)[0]]) / rho
    else:
        arc = 2 * math.pi - ccw_er
        tan = np.array([(e - ctr)[1], -(e - ctr)[0]]) / rho
    return rho * arc, launch_theta(e, tan)


# ------------------------------------------- hat-function line integrals --
def hat_line_integrals(p0, p1, nx, ny):
    """Exact integrals of every bilinear hat function along the straight segment
    p0 -> p1 (pixel coordinates relative to the grid centre, node (ix, iy) at
    (ix - (nx-1)/2, iy - (ny-1)/2)), per unit pixel of arc length.  The segment is
    split at every grid line, each hat is quadratic along each piece, and each
    piece is integrated exactly by Simpson's rule.  Returns a dict node -> value."""
    p0 = np.asarray(p0, float)
    p1 = np.asarray(p1, float)
    ox, oy = 0.5 * (nx - 1), 0.5 * (ny - 1)
    u0 = p0 + [ox, oy]
    u1 = p1 + [ox, oy]
    du = u1 - u0
    Ltot = float(np.linalg.norm(du))
    ts = {0.0, 1.0}
    for k in range(2):
        if du[k] != 0:
            lo, hi = sorted((u0[k], u1[k]))
            for gl in range(int(math.ceil(lo)), int(math.floor(hi)) + 1):
                t = (gl - u0[k]) / du[k]
                if 0 < t < 1:
                    ts.add(t)
    ts = sorted(ts)
    out = {}
    for ta, tb in zip(ts[:-1], ts[1:]):
        if tb - ta <= 0:
            continue
        tm = 0.5 * (ta + tb)
        um = u0 + tm * du
        ix, iy = int(math.floor(um[0])), int(math.floor(um[1]))
        seg = (tb - ta) * Ltot
        for jx, jy in ((ix, iy), (ix + 1, iy), (ix, iy + 1), (ix + 1, iy + 1)):
            def phi(t):
                u = u0 + t * du
                return max(0.0, 1 - abs(u[0] - jx)) * max(0.0, 1 - abs(u[1] - jy))
            val = seg / 6.0 * (phi(ta) + 4 * phi(tm) + phi(tb))
            if val:
                key = jy * nx + jx
                out[key] = out.get(key, 0.0) + val
    return out
