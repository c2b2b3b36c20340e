"""Pins of the 3-D oracle (hemispherical arrays, Broyden-like linking) against
what geometry and the paper fix: straight rays and Euclidean lengths in a
homogeneous volume, the homogeneous Jacobian against differences of the traced
misfit, the closed-form travel time of a linear-gradient volume, the
fish-eye's circles and its antipodal focus with acoustic length pi a / 2
(Section 4 with dim = 3), reciprocity, and the status paths."""
import math

import numpy as np
import pytest

import synth


def _grid(c, h):
    return {"kind": "grid", "c": c, "h": h}


def test3_homogeneous_straight_rays(orc):
    """Every pair links on its straight ray: one ray, T = |r - e| / c0 and
    L = |r - e| to rounding."""
    n, h = 40, 1e-3
    el = synth.hemisphere_elements(24, 0.016)
    pairs = synth.all_pairs(24)
    o = orc.trace3(_grid(np.full((n, n, n), 1500.0), h), el, pairs)
    d = np.linalg.norm(el[pairs[:, 1]] - el[pairs[:, 0]], axis=1)
    assert np.all(o["status"] == orc.LINKED) and np.all(o["n_marches"] == 1)
    np.testing.assert_allclose(o["tof"], d / 1500.0, rtol=1e-12)
    np.testing.assert_allclose(o["len"], d, rtol=1e-12)


def test3_homogeneous_jacobian_matches_traced_misfit(orc):
    """The closed-form Jacobian that seeds the Broyden-like iteration equals
    central differences of the misfit of rays traced through a homogeneous
    volume, at the straight ray and away from it."""
    n, h = 40, 1e-3
    med = _grid(np.full((n, n, n), 1500.0), h)
    el = synth.hemisphere_elements(24, 0.016)
    rng = np.random.default_rng(31)
    for e, r in ((0, 5), (3, 17), (20, 2), (11, 12)):
        o = orc.trace3(med, el, np.array([[e, r]], np.int32))
        for u in (o["u"][0], o["u"][0] + rng.uniform(-0.1, 0.1, 2)):
            J, _ = orc.jac0_3(el, h, e, r, u)
            eps = 1e-6
            fd = np.empty((2, 2))
            for j in range(2):
                du = np.zeros(2)
                du[j] = eps
                fd[:, j] = (orc.misfit3(med, el, e, r, u + du)[1] - orc.misfit3(med, el, e, r, u - du)[1]) / (2 * eps)
            np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("a", [(120.0, 0.0, 0.0), (0.0, 90.0, -60.0), (50.0, -70.0, 80.0)])
def test3_linear_gradient_closed_form(orc, a):
    """c = c0 + a.x: rays are circular arcs and T(e, r) =
    arccosh(1 + |a|^2 |r - e|^2 / (2 c(e) c(r))) / |a| in any dimension."""
    h = 0.5e-3
    el = synth.hemisphere_elements(16, 0.012)
    pairs = synth.all_pairs(16)[::3]
    med = {"kind": "linear", "n": (64, 64, 64), "h": h, "c0": 1500.0, "a": a}
    o = orc.trace3(med, el, pairs, tol_px=1e-6)
    assert np.all(o["status"] == orc.LINKED)
    g = np.linalg.norm(a)
    ce = 1500.0 + el[pairs[:, 0]] @ np.array(a)
    cr = 1500.0 + el[pairs[:, 1]] @ np.array(a)
    d2 = np.sum((el[pairs[:, 1]] - el[pairs[:, 0]]) ** 2, axis=1)
    T = np.arccosh(1 + g * g * d2 / (2 * ce * cr)) / g
    assert np.abs(o["tof"] / T - 1).max() < 1e-7


def _fisheye_dirs():
    """Launch parameters of rays from [0, 0, a] spread over +-pi/3 about the
    inward normal, in five azimuths."""
    us = []
    for t in np.linspace(-math.pi / 3, math.pi / 3, 7):
        for ph in np.linspace(0, 2 * math.pi, 5, endpoint=False):
            us.append([math.tan(t) * math.cos(ph), math.tan(t) * math.sin(ph)])
    return np.array(us)


@pytest.mark.parametrize("kind,bound", [("analytic", 0.003), ("grid", 0.05)])
def test3_fisheye_antipodal_focus(orc, kind, bound):
    """Section 4 with dim = 3 (a = 1, 1-degree spacing, ds/dx = 1): every ray
    from [0, 0, a] into the lens is focused on the antipode [0, 0, -a] with
    acoustic length (travel time at c0 = 1) a pi / 2, the dim = 3 analogue of
    the 2-D experiment of Sec. 4.2 (the paper closes its 3-D rays after a full
    turn, twice this length)."""
    a, dx = 1.0, 2 * math.pi / 360
    n = 2 * int(math.ceil(1.1 * a / dx)) + 1
    if kind == "analytic":
        med = {"kind": "fisheye", "n": (n, n, n), "h": dx, "c0": 1.0, "R": a}
    else:
        med = _grid(synth.fisheye3(n, n, n, dx, c0=1.0, R=a), dx)
    el = np.array([[0.0, 0.0, a], [0.0, 0.0, -a]])
    us = _fisheye_dirs()
    pairs = np.tile(np.array([[0, 1]], np.int32), (len(us), 1))
    o = orc.trace3(med, el, pairs, u=us, fixed=True, ds_px=1.0)
    assert np.all(o["status"] == orc.LINKED)
    re_al = np.mean((o["tof"] - math.pi / 2) / (math.pi / 2)) * 100
    assert abs(re_al) < bound
    assert o["miss_px"].max() * dx < (0.01 if kind == "analytic" else 0.03) * a


@pytest.mark.parametrize("integ,bound", [("rk4", 1e-4), ("heun", 0.05)])
def test3_fisheye_circles(orc, integ, bound):
    """Section 4.1 with dim = 3: rays from x_p = [0, 0, a] launched normal to
    x_c - x_p (x_c = [a, a, 0]), 21 azimuths.  In the lens every ray through
    x_p is a circle through the conjugate point [0, 0, -a]; with direction d
    its centre is lambda d_h / |d_h| (d_h the horizontal part of d, lambda =
    a d_z / |d_h|) and its radius sqrt(lambda^2 + a^2) (sqrt(3) a for the two
    rays whose centre is x_c).  Mean radius deviation over the first turn."""
    a, dx = 1.0, 2 * math.pi / 360
    axis = np.array([a, a, -a]) / math.sqrt(3)
    e1 = np.cross(axis, [0.0, 0.0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(axis, e1)
    n = 2 * int(math.ceil(3.5 * a / dx)) + 1
    med = {"kind": "fisheye", "n": (n, n, n), "h": dx, "c0": 1.0, "R": a}
    res = []
    for ph in np.linspace(0, 2 * math.pi, 21, endpoint=False):
        d = math.cos(ph) * e1 + math.sin(ph) * e2
        dh = np.array([d[0], d[1], 0.0])
        lam = a * d[2] / np.linalg.norm(dh)
        cen = lam * dh / np.linalg.norm(dh)
        rho = math.sqrt(lam * lam + a * a)
        steps = int(1.2 * 2 * math.pi * rho / dx)
        pts = orc.march3_free(med, np.array([0.0, 0.0, a]) / dx, d, steps, integ=integ, ds_px=1.0) * dx
        dist0 = np.linalg.norm(pts - [0.0, 0.0, a], axis=1)
        far = np.nonzero(dist0 > 10 * dx)[0][0]
        M = far + np.nonzero(dist0[far:] < dx)[0][0]
        res.append(np.mean(np.abs(np.linalg.norm(pts[1:M + 1] - cen, axis=1) - rho) / rho))
    assert np.mean(res) * 100 < bound


def test3_reciprocity_gaussian_volume(orc):
    """T(e, r) = T(r, e) for linked pairs (backward rays are reversed forward
    rays, Sec. 3.5), the gap shrinking at second order in the step."""
    n, h = 48, 0.5e-3
    c = synth.gaussian_inclusions3(n, n, n, h, seed=33, r_max=0.007)
    el = synth.hemisphere_elements(12, 0.010)
    pairs = synth.all_pairs(12)
    idx = {(int(e), int(r)): i for i, (e, r) in enumerate(pairs)}
    gaps = []
    for ds in (0.25, 0.125):
        o = orc.trace3(_grid(c, h), el, pairs, tol_px=1e-9, ds_px=ds)
        assert np.all(o["status"] == orc.LINKED)
        gaps.append(max(abs(o["tof"][i] / o["tof"][idx[(r, e)]] - 1) for (e, r), i in idx.items()))
    assert gaps[0] < 5e-6 and gaps[0] / gaps[1] > 3.0, gaps


def test3_broyden_links_and_status_paths(orc):
    """A Gaussian-inclusion volume: every pair links within the tolerance and
    the Broyden-like iteration needs few rays; a ray budget of one returns the
    straight ray as NOT_CONVERGED; invalid pairs are BAD_INPUT."""
    n, h = 48, 0.5e-3
    c = synth.gaussian_inclusions3(n, n, n, h, seed=34, r_max=0.008)
    el = synth.hemisphere_elements(20, 0.011)
    pairs = np.concatenate([synth.all_pairs(20), [[3, 3], [-1, 2], [4, 20]]]).astype(np.int32)
    o = orc.trace3(_grid(c, h), el, pairs)
    ok = o["status"][:-3]
    assert np.all(ok == orc.LINKED) and np.all(o["miss_px"][:-3] <= 1e-3)
    assert o["n_marches"][:-3].mean() < 4 and o["n_marches"].max() <= 10
    assert np.all(o["status"][-3:] == orc.BAD_INPUT)
    one = orc.trace3(_grid(c, h), el, pairs[:-3], max_marches=1)
    assert np.all((one["status"] == orc.NOT_CONVERGED) | (one["miss_px"] <= 1e-3))
