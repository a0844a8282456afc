"""Pins of the oracle's tabulated foveation and lens distortion (Sec. 3.1.1
"Domain": an arbitrary monotone p, inverted numerically; Sec. 5.1 "Lens
Distortion": p = p_c o p_l with only p_c undone by the display) against
things other than itself:

* the identity table reproduces the power law's alpha = 1 render bit for bit;
* a two-segment table: foveate / unfoveate / Jacobian by hand;
* the numeric inverse undoes the table's map (round trip) and converges to
  the analytic inverse of a power law sampled ever more finely (within the
  linear-interpolation bound);
* a linear lens s -> k s equals a pinhole with focal lengths scaled by k
  (ids and depths, as the GPU parity rule compares them);
* the time of a pixel comes from its panel point, its ray from the
  undistorted point;
* the display resampling does not see the lens.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen
from parity import compare


def _view(W=64, H=48, fovea=(0.13, -0.07), alpha=1.0, profile_c=None, profile_l=None, **kw):
    return scenegen.View(W, H, np.zeros(6, np.float32), np.zeros(6, np.float32), fovea=fovea, alpha=alpha,
                         profile_c=profile_c, profile_l=profile_l, **kw)


def test_identity_table_is_alpha_one_bitwise():
    sc = scenegen.make_moving_soup(seed=51, n_tris=400, width=48, height=40, alpha=1.0, roll=(1.0, 0.0),
                                   yaw_deg_s=900.0, obj_speed=8.0, side=(0.1, 0.6))
    v = sc.views[0]
    a = oracle.Oracle(sc.meshes[0], v).render()
    v.profile_c = np.array([0.0, 1.0], np.float32)
    b = oracle.Oracle(sc.meshes[0], v).render()
    assert np.array_equal(a['id'], b['id']) and np.array_equal(a['z'], b['z'])


def test_two_segment_table_by_hand():
    """p_c samples (0, 0.75, 1) at s = 0, 1/2, 1: p_c(s) = 1.5 s below 1/2,
    0.75 + 0.5 (s - 1/2) above.  A foveated point at distance 0.6 R lies on
    the display at 0.4 R, one at 0.9 R at 0.8 R (same direction); the
    foveate map's Jacobian there has radial scale p_c' and tangential scale
    p_c(s)/s."""
    v = _view(profile_c=np.array([0.0, 0.75, 1.0], np.float32))
    R = oracle.fovea_radius(v)
    f = np.array(v.fovea)
    for ang in (0.3, 2.0, -1.2):
        e = np.array([math.cos(ang), math.sin(ang)])
        for sf, sp in ((0.6, 0.4), (0.9, 0.8), (0.3, 0.2), (1.0, 1.0)):
            x = oracle.unfoveate(v, f + sf * R * e)
            assert np.abs(x - (f + sp * R * e)).max() < 1e-14
            assert np.abs(oracle.foveate(v, f + sp * R * e) - (f + sf * R * e)).max() < 1e-14
    vp = oracle.view_params(v)
    L = oracle.lib()
    import ctypes
    for sp, slope in ((0.4, 1.5), (0.8, 0.5)):
        xp = f + sp * R * np.array([1.0, 0.0])
        J = np.empty(4)
        L.orc_foveate_jac(vp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          xp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          J.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        g = 1.5 * sp if sp < 0.5 else 0.75 + 0.5 * (sp - 0.5)
        assert np.abs(J - np.array([slope, 0.0, 0.0, g / sp])).max() < 1e-13


def test_numeric_inverse_round_trip_and_convergence():
    rng = np.random.default_rng(5)
    tab = scenegen.foveal_table(41, 4.0)
    v = _view(profile_c=tab)
    for y in rng.uniform(-1, 1, size=(300, 2)):
        assert np.abs(oracle.foveate(v, oracle.unfoveate(v, y)) - y).max() < 1e-12
    # a power law p_c(s) = s^(1/2) sampled at n points: the tabulated inverse
    # (display distance) is within (max sample gap)^2 / 4 of s_F^2 (the
    # linear-interpolation bound, second derivative 2)
    vp = _view(alpha=2.0)
    errs = []
    for n in (9, 17, 33, 64):
        s = np.linspace(0, 1, n)
        tab = np.sqrt(s).astype(np.float32)
        vt = _view(profile_c=tab)
        gap = np.diff(tab.astype(np.float64)).max()
        R = oracle.fovea_radius(vt)
        err = 0.0
        for y in rng.uniform(-1, 1, size=(100, 2)):
            d = np.linalg.norm(oracle.unfoveate(vt, y) - oracle.unfoveate(vp, y)) / R
            err = max(err, d)
        # float32 samples move each by up to 2^-24 (relative)
        assert err <= gap ** 2 / 4 + 1e-6
        errs.append(err)
    assert errs[-1] < errs[0] / 5   # the first gap, 1/sqrt(n-1), dominates: error ~ 1/n


def test_linear_lens_is_a_scaled_pinhole():
    """p_l(s) = k s about a fovea at the principal point: the undistorted
    point is the panel point / k, so the ray is that of a pinhole with
    focal lengths k fx, k fy; the scan time still comes from the panel."""
    k = 1.25
    base = scenegen.make_moving_soup(seed=52, n_tris=500, width=56, height=44, alpha=2.0, roll=(1.0, 0.0),
                                     yaw_deg_s=1200.0, obj_speed=8.0, side=(0.1, 0.6), fovea=(0.0, 0.0))
    v = base.views[0]
    v.profile_l = np.array([0.0, k], np.float32)
    orc = oracle.Oracle(base.meshes[0], v)
    o = orc.render()
    import copy
    v2 = copy.copy(v)
    v2.profile_l = None
    v2.fx, v2.fy = v.fx * k, v.fy * k
    orc2 = oracle.Oracle(base.meshes[0], v2)
    o2 = orc2.render()
    pix = np.arange(v.width * v.height)
    rep = compare(orc, o, o2['id'], o2['z'].astype(np.float32), pix, v.znear)
    assert rep['hits'] > 300 and not rep['bad'], rep['bad'][:5]
    for p in (0, 777, v.width * v.height - 1):
        _, x, t, r = oracle.pixel_setup(v, p)
        _, x2, t2, r2 = oracle.pixel_setup(v2, p)
        assert t == t2 and np.abs(np.asarray(r) - np.asarray(r2)).max() < 1e-14


def test_time_from_panel_ray_from_undistorted_point():
    """Barrel lens, no foveation: pixel (i, j)'s panel point is its own NDC
    point y, its time (i + 1/2)/W; its ray passes through the undistorted
    point u with |u - f| = R p_l^{-1}(|y - f|/R) along y - f, where the lens
    table's inverse is found here by bisection on its piecewise-linear
    interpolant."""
    lens = scenegen.barrel_table(17, 0.25)
    v = _view(W=40, H=30, fovea=(0.0, 0.0), alpha=1.0, profile_l=lens, roll_dir=(1.0, 0.0), fx=1.3, fy=0.9)
    R = oracle.fovea_radius(v)
    s_nodes = np.linspace(0, 1, lens.size)
    lt = lens.astype(np.float64)

    def p_l(s):
        k = min(int(s * (lens.size - 1)), lens.size - 2)
        return lt[k] + (s - s_nodes[k]) * (lt[k + 1] - lt[k]) * (lens.size - 1)

    for p in (0, 13, 40 * 7 + 33, 40 * 30 - 1, 600):
        i, j = p % 40, p // 40
        y, x, t, r = oracle.pixel_setup(v, p)
        assert abs(t - (i + 0.5) / 40) < 1e-15
        d = np.linalg.norm(y)
        lo, hi = 0.0, 2.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if p_l(mid) < d / R else (lo, mid)
        u = np.asarray(y) * (lo * R / d)
        assert np.abs(np.asarray(x) - u).max() < 1e-12
        assert abs(r[0] - u[0] / 1.3) < 1e-12 and abs(r[1] - u[1] / 0.9) < 1e-12
        assert np.linalg.norm(u) > d   # a barrel pre-distortion pulls the panel inwards


def test_display_does_not_see_the_lens():
    v = _view(W=32, H=24, alpha=2.0)
    rng = np.random.default_rng(9)
    img = rng.uniform(size=(24, 32, 4))
    a = oracle.unfoveate_image(v, img, 40, 30)
    v.profile_l = scenegen.barrel_table(9, 0.2)
    b = oracle.unfoveate_image(v, img, 40, 30)
    assert np.array_equal(a, b)
    v.profile_c = scenegen.foveal_table(17, 2.0)
    c = oracle.unfoveate_image(v, img, 40, 30)
    assert not np.array_equal(a, c)
