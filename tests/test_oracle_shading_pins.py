"""Pins of the oracle's rolling highlight and G-buffer against things other
than itself.

* highlight (Sec. 3.2 "Shading", Sec. 5.1 "Rolling Shading")
    - half-angle closed form on a plane facing the eye: a light at angle
      theta from the normal seen along the normal gives (n.h) = cos(theta/2);
    - the n.l > 0 gate (a light behind the surface gives no highlight);
    - the rolling eye: with a translating camera the highlight equals the one
      computed in world space with the eye at the camera centre interpolated
      to the pixel's time and the hit point from the oracle's own depth;
    - its gradient against central differences.
* G-buffer (Sec. 3.2 "Pipeline", Sec. 7 "Screen-space effects")
    - normal: the facing plane's normal; on a moving soup unit length,
      perpendicular to the triangle's edges at the pixel's time, facing the
      eye;
    - barycentrics: the point they blend lies on the pixel's ray at the
      oracle's depth (an independent route: ray-triangle intersection);
    - density: 1 without foveation, the closed form alpha^(-1/2)
      (rho/R)^(1-alpha), and 1/sqrt(|det|) of the central-difference
      Jacobian of the (separately pinned) unfoveate map.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenegen


def _facing_quad(W=17, H=17, alpha=1.0, pose0=None, pose1=None, z=3.0, half=4.0):
    quad = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], np.float32)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    alb = np.tile(np.array([[0.3, 0.6, 0.9]], np.float32), (4, 1))
    mesh = scenegen.Mesh(quad, quad.copy(), tri, alb)
    p0 = np.zeros(6, np.float32) if pose0 is None else np.asarray(pose0, np.float32)
    p1 = p0.copy() if pose1 is None else np.asarray(pose1, np.float32)
    view = scenegen.View(W, H, p0, p1, alpha=alpha, roll_dir=(1, 0))
    return mesh, view


ALB = np.array([0.3, 0.6, 0.9], np.float32).astype(np.float64)   # the albedo as stored (float32)


def _highlight(orc, ids, light):
    """The highlight alone: shading with it minus shading without it."""
    lt = np.asarray(light, np.float64)
    base = lt.copy()
    base[4] = 0.0
    return orc.shade(ids, lt) - orc.shade(ids, base)


# --------------------------------------------------------------------------
# highlight
# --------------------------------------------------------------------------

@pytest.mark.parametrize('theta_deg', [0.0, 30.0, 70.0])
def test_highlight_half_angle_closed_form(theta_deg):
    """Centre pixel of an odd-sized image (ray along +z, eye direction = the
    plane's normal turned to the eye = (0,0,-1)), light at angle theta from
    the normal: h bisects l and v, so n.h = cos(theta/2) and the colour is
    albedo (k_a + (1-k_a) cos theta) + k_s cos(theta/2)^m."""
    mesh, view = _facing_quad()
    orc = oracle.Oracle(mesh, view)
    ids = orc.render()['id']
    c = (view.height // 2) * view.width + view.width // 2
    th = math.radians(theta_deg)
    ks, m = 0.7, 12.0
    light = np.array([0.0, math.sin(th), -math.cos(th), 0.1, ks, m])
    rgb = orc.shade(ids, light)
    expect = ALB * (0.1 + 0.9 * math.cos(th)) + ks * math.cos(th / 2) ** m
    assert np.abs(rgb[c] - expect).max() < 1e-12


def test_highlight_needs_a_lit_side():
    """Light 120 degrees from the normal: n.h = cos 60 > 0 but n.l < 0, so
    no highlight (and no diffuse term): the colour is albedo k_a."""
    mesh, view = _facing_quad()
    orc = oracle.Oracle(mesh, view)
    ids = orc.render()['id']
    th = math.radians(120.0)
    light = np.array([0.0, math.sin(th), -math.cos(th), 0.1, 0.7, 4.0])
    rgb = orc.shade(ids, light)
    hit = ids >= 0
    assert hit.all()
    assert np.abs(rgb[hit] - ALB * 0.1).max() < 1e-15


def test_highlight_follows_the_rolling_eye():
    """Static world plane, camera translating and turning during the frame
    (rotation equal at both ends, so the camera-space interpolation is a
    rigid motion at every instant): per pixel the highlight equals the
    world-space Blinn-Phong term with the eye at the camera centre
    c(t) = -R^T T(t) at the pixel's time and the hit point X = R^T (z r -
    T(t)) from the oracle's depth z."""
    rot = np.array([0.05, -0.3, 0.02])
    pose0 = np.concatenate([rot, [0.9, -0.2, 0.5]])
    pose1 = np.concatenate([rot, [-1.1, 0.4, -0.3]])
    mesh, view = _facing_quad(W=41, H=33, alpha=2.0, pose0=pose0, pose1=pose1, z=4.0, half=9.0)
    view.fovea = (0.1, -0.05)
    orc = oracle.Oracle(mesh, view)
    o = orc.render()
    ks, m = 0.9, 7.0
    lw = np.array([0.3, 0.5, -0.8])
    spec = _highlight(orc, o['id'], np.array([*lw, 0.1, ks, m]))[:, 0]
    # the poses as the view stores them (float32)
    R = Rotation.from_rotvec(view.pose0[:3].astype(np.float64)).as_matrix()
    assert (view.pose0[:3] == view.pose1[:3]).all()
    nw = np.array([0.0, 0.0, 1.0])          # the quad's plane z = const
    l = lw / np.linalg.norm(lw)
    T0, T1 = view.pose0[3:].astype(np.float64), view.pose1[3:].astype(np.float64)
    checked = lit = 0
    for p in range(view.width * view.height):
        if o['id'][p] < 0:
            continue
        _, _, t, r = oracle.pixel_setup(view, p)
        Tt = (1 - t) * T0 + t * T1
        eye = -R.T @ Tt
        X = R.T @ (o['z'][p] * np.asarray(r) - Tt)
        v = (eye - X) / np.linalg.norm(eye - X)
        n = nw if nw @ v > 0 else -nw
        h = (l + v) / np.linalg.norm(l + v)
        expect = ks * max(n @ h, 0.0) ** m if n @ l > 0 else 0.0
        assert abs(spec[p] - expect) < 1e-10, (p, spec[p], expect)
        checked += 1
        lit += expect > 1e-3
    assert checked > 1000 and lit > 100


def test_highlight_gradient_matches_central_differences():
    sc = scenegen.make_grad(seed=5, size=40, f=8)
    mesh, view, target = sc.meshes[0], sc.views[0], sc.extra['target']
    light = oracle.light_block(sc, specular=0.6, shininess=9.0)
    orc_t = oracle.Oracle(target, view)
    tgt = orc_t.shade(orc_t.render()['id'], light)
    orc = oracle.Oracle(mesh, view)
    ids = orc.render()['id']
    # the highlight is present on the pixels that decide the check
    assert np.abs(_highlight(orc, ids, light)).max() > 1e-2
    L, g0, g1, gp0, gp1 = orc.loss_grad(ids, light, tgt)
    assert abs(L - orc.loss(ids, light, tgt)) < 1e-12 * L
    h = 1e-6
    v0 = mesh.v0.astype(np.float64)
    v1 = mesh.v1.astype(np.float64)
    vis = np.unique(mesh.tri[ids[ids >= 0]].ravel())
    rng = np.random.default_rng(4)
    for vi in rng.choice(vis, size=8, replace=False):
        for d in range(3):
            for which, g in ((0, g0), (1, g1)):
                a, b = v0.copy(), v1.copy()
                arr_p, arr_m = (a, b), (a.copy(), b.copy())
                arr_p[which][vi, d] += h
                arr_m[which][vi, d] -= h
                lp = oracle.Oracle(mesh, view, v0=arr_p[0], v1=arr_p[1]).loss(ids, light, tgt)
                lm = oracle.Oracle(mesh, view, v0=arr_m[0], v1=arr_m[1]).loss(ids, light, tgt)
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[vi, d]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), (vi, d, which)
    for which, gp in ((0, gp0), (1, gp1)):
        for k in range(6):
            pp = [view.pose0.astype(np.float64).copy(), view.pose1.astype(np.float64).copy()]
            pm = [view.pose0.astype(np.float64).copy(), view.pose1.astype(np.float64).copy()]
            pp[which][k] += h
            pm[which][k] -= h
            lp = oracle.Oracle(mesh, view, pose0=pp[0], pose1=pp[1]).loss(ids, light, tgt)
            lm = oracle.Oracle(mesh, view, pose0=pm[0], pose1=pm[1]).loss(ids, light, tgt)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gp[k]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(gp).max()), (which, k, fd, gp[k])


# --------------------------------------------------------------------------
# G-buffer
# --------------------------------------------------------------------------

def test_gbuffer_facing_plane():
    """Plane z = 3 facing the camera: normal (0,0,-1) everywhere; the
    barycentrics of pixel p are those of the point 3 r(p) in the hit
    triangle (a 2x2 solve in the plane)."""
    mesh, view = _facing_quad(W=19, H=15, alpha=1.0)
    orc = oracle.Oracle(mesh, view)
    ids = orc.render()['id']
    g = orc.gbuffer(ids)
    assert (ids >= 0).all()
    assert np.abs(g['normal'] - np.array([0.0, 0.0, -1.0])).max() < 1e-15
    V = mesh.v0.astype(np.float64)
    for p in range(0, view.width * view.height, 7):
        _, _, _, r = oracle.pixel_setup(view, p)
        X = 3.0 * np.asarray(r)
        a, b, c = V[mesh.tri[ids[p]]]
        A = np.stack([b[:2] - a[:2], c[:2] - a[:2]], axis=1)
        mu = np.linalg.solve(A, X[:2] - a[:2])
        assert np.abs(g['bary'][p] - mu).max() < 1e-13


def test_gbuffer_moving_soup_invariants():
    sc = scenegen.make_moving_soup(seed=21, n_tris=300, width=48, height=40, alpha=2.0, roll=(1.0, 0.0),
                                   yaw_deg_s=1500.0, obj_speed=10.0, side=(0.1, 0.6))
    mesh, view = sc.meshes[0], sc.views[0]
    orc = oracle.Oracle(mesh, view)
    o = orc.render()
    g = orc.gbuffer(o['id'])
    Ps = np.asarray(mesh.v0, np.float64) @ Rotation.from_rotvec(view.pose0[:3].astype(np.float64)).as_matrix().T \
        + view.pose0[3:].astype(np.float64)
    Pe = np.asarray(mesh.v1, np.float64) @ Rotation.from_rotvec(view.pose1[:3].astype(np.float64)).as_matrix().T \
        + view.pose1[3:].astype(np.float64)
    hit = np.flatnonzero(o['id'] >= 0)
    assert hit.size > 300
    for p in hit:
        f = o['id'][p]
        _, _, t, r = oracle.pixel_setup(view, p)
        r = np.asarray(r)
        P = (1 - t) * Ps[mesh.tri[f]] + t * Pe[mesh.tri[f]]
        n = g['normal'][p]
        assert abs(np.linalg.norm(n) - 1) < 1e-12
        sc_ = np.linalg.norm(P[1] - P[0]) + np.linalg.norm(P[2] - P[0])
        assert abs(n @ (P[1] - P[0])) < 1e-12 * sc_ and abs(n @ (P[2] - P[0])) < 1e-12 * sc_
        assert n @ r <= 0
        mu1, mu2 = g['bary'][p]
        X = P[0] + mu1 * (P[1] - P[0]) + mu2 * (P[2] - P[0])
        assert np.linalg.norm(np.cross(X, r)) < 1e-9 * np.linalg.norm(X)     # on the ray
        assert abs(X[2] - o['z'][p]) < 1e-9 * o['z'][p]                   # at the hit's depth
    miss = o['id'] < 0
    assert (g['normal'][miss] == 0).all() and (g['bary'][miss] == 0).all()


@pytest.mark.parametrize('alpha', [1.0, 1.5, 2.0, 3.0])
def test_gbuffer_density(alpha):
    """Density = alpha^(-1/2) (rho/R)^(1-alpha) (1 without foveation), and
    1/sqrt(|det|) of the central-difference Jacobian of the unfoveate map."""
    W, H = 33, 27
    view = scenegen.View(W, H, np.zeros(6, np.float32), np.zeros(6, np.float32), fovea=(0.13, -0.07),
                         alpha=alpha, roll_dir=(1, 0))
    mesh, _ = _facing_quad()
    orc = oracle.Oracle(mesh, view)
    ids = np.full(W * H, -1, np.int32)
    dens = orc.gbuffer(ids)['density']
    R = oracle.fovea_radius(view)
    f = np.array(view.fovea)
    for p in range(W * H):
        y, _, _, _ = oracle.pixel_setup(view, p)
        y = np.asarray(y)
        rho = np.linalg.norm(y - f)
        assert abs(dens[p] - alpha ** -0.5 * (rho / R) ** (1 - alpha)) < 1e-10 * dens[p]
        if p % 5 == 0:
            e = 1e-6
            J = np.stack([(oracle.unfoveate(view, y + e * np.eye(2)[k]) - oracle.unfoveate(view, y - e * np.eye(2)[k]))
                          / (2 * e) for k in range(2)], axis=1)
            assert abs(dens[p] - 1 / math.sqrt(abs(np.linalg.det(J)))) < 1e-6 * dens[p]
    if alpha == 1.0:
        assert (dens == 1.0).all()
