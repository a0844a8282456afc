"""Pins of the FP64 oracle against things other than itself.

Each test ties a step of the oracle (numbered as in oracle/pr_oracle.c) to a
library routine, a closed form the paper states, or an independent
formulation:

* Rodrigues' formula and its Jacobian        -> scipy.spatial.transform / FD
* foveation (Sec. 3.1.1, power law p(d)=d^a) -> defining properties
* rolling time (Sec. 3.1.2, r(x) = x . d)    -> closed form per pixel column/row
* ray-cast + z-test (Sec. 3.2)               -> textbook half-space rasteriser
  (identity foveation, one instant) and, per column, the same rasteriser on
  the scene frozen at that column's time (rolling column identity)
* foveated sampling                          -> half-space test at the
  unfoveated display point
* depth ("actual z value")                   -> fronto-parallel plane
* gradient                                   -> central differences, and the
  translation identity sum_v dL/dv = R^T dL/dT
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import scenegen
from oracle import classic


def _view_space(v, pose):
    R = Rotation.from_rotvec(np.asarray(pose[:3], np.float64)).as_matrix()
    return np.asarray(v, np.float64) @ R.T + np.asarray(pose[3:], np.float64)


# --------------------------------------------------------------------------
# Rodrigues
# --------------------------------------------------------------------------

def test_rodrigues_matches_scipy():
    rng = np.random.default_rng(0)
    ws = [np.zeros(3), np.array([1e-9, 0, 0]), np.array([0, -0.0232, 0])]
    ws += list(rng.normal(size=(20, 3)))
    for w in ws:
        R = oracle.rodrigues(w)
        Rs = Rotation.from_rotvec(w).as_matrix()
        assert np.abs(R - Rs).max() < 1e-14


def test_rodrigues_jacobian_matches_central_differences():
    rng = np.random.default_rng(1)
    ws = [np.zeros(3), np.array([0, -0.0232, 0]), np.array([1e-7, 2e-7, 0])] + list(rng.normal(size=(10, 3)))
    h = 1e-6
    for w in ws:
        J = oracle.rodrigues_jac(w)
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            fd = (Rotation.from_rotvec(w + e).as_matrix() - Rotation.from_rotvec(w - e).as_matrix()) / (2 * h)
            assert np.abs(J[i] - fd).max() < 1e-8, (w, i)


# --------------------------------------------------------------------------
# foveation
# --------------------------------------------------------------------------

def _fov_view(fovea=(0.13, -0.07), alpha=2.0):
    return scenegen.View(64, 48, np.zeros(6, np.float32), np.zeros(6, np.float32), fovea=fovea, alpha=alpha)


def test_fovea_radius_is_farthest_corner():
    assert abs(oracle.fovea_radius(_fov_view((0.0, 0.0))) - math.sqrt(2.0)) < 1e-15
    v = _fov_view((0.2, -0.1))
    assert abs(oracle.fovea_radius(v) - math.hypot(1.2, 1.1)) < 1e-15


@pytest.mark.parametrize('alpha', [1.0, 1.5, 2.0, 3.0])
def test_unfoveate_is_radial_power_law(alpha):
    """Display distance from the fovea is R (rho/R)^alpha along the same
    direction: p(d) = d^alpha on normalised distances.  alpha = 1 is the
    identity (constant density)."""
    v = _fov_view(alpha=alpha)
    R = oracle.fovea_radius(v)
    xf = np.array(v.fovea)
    rng = np.random.default_rng(2)
    for y in rng.uniform(-1, 1, size=(200, 2)):
        x = oracle.unfoveate(v, y)
        dy, dx = y - xf, x - xf
        rho = np.linalg.norm(dy)
        assert abs(np.linalg.norm(dx) - R * (rho / R) ** alpha) < 1e-13
        assert abs(dx[0] * dy[1] - dx[1] * dy[0]) < 1e-13 and dx @ dy >= 0  # same direction
        assert np.all(np.abs(x) <= 1.0 + 1e-15)                         # stays on the display
        yb = oracle.foveate(v, x)
        assert np.abs(yb - y).max() < 1e-12                             # F(U(y)) = y
    assert np.abs(oracle.unfoveate(v, xf) - xf).max() == 0.0
    if alpha == 1.0:
        y = np.array([0.3, -0.8])
        assert np.abs(oracle.unfoveate(v, y) - y).max() < 1e-15


def test_foveation_magnifies_the_fovea():
    """Reading of Sec. 3.1.1 (the density is higher near the fovea): a pixel
    step next to the fovea covers a smaller display distance than one in the
    periphery, and display distance grows monotonically along a ray."""
    v = _fov_view((0.0, 0.0), 2.0)
    rhos = np.linspace(0, 1.4, 300)
    d = [np.linalg.norm(oracle.unfoveate(v, np.array([r / math.sqrt(2)] * 2))) for r in rhos]
    assert np.all(np.diff(d) > 0)
    step = 1e-3
    near = np.linalg.norm(oracle.unfoveate(v, np.array([step, 0.0])))
    far = np.linalg.norm(oracle.unfoveate(v, np.array([0.9 + step, 0.0]))) - np.linalg.norm(
        oracle.unfoveate(v, np.array([0.9, 0.0])))
    assert near < 0.01 * step and far > step


# --------------------------------------------------------------------------
# pixel grid, rolling time, ray
# --------------------------------------------------------------------------

def test_pixel_grid_and_rolling_time():
    v = scenegen.View(40, 30, np.zeros(6, np.float32), np.zeros(6, np.float32), fx=1.3, fy=0.8,
                      cx=0.05, cy=-0.1, alpha=1.0, roll_dir=(1.0, 0.0))
    for pix in [0, 39, 40 * 29, 40 * 30 - 1, 617]:
        i, j = pix % 40, pix // 40
        y, x, t, r = oracle.pixel_setup(v, pix)
        assert np.allclose(y, [(2 * i + 1) / 40 - 1, 1 - (2 * j + 1) / 30], atol=1e-15)
        assert abs(t - (i + 0.5) / 40) < 1e-15          # time linear in display column
        # the ray projects back onto the display point
        assert abs(1.3 * r[0] / r[2] + 0.05 - x[0]) < 1e-14 and abs(0.8 * r[1] / r[2] - 0.1 - x[1]) < 1e-14
    v.roll_dir = (0.0, 0.9)                                   # scan along y with a 10 % blank
    y, x, t, r = oracle.pixel_setup(v, 40 * 7 + 3)
    assert abs(t - 0.9 * (1 - 7.5 / 30)) < 1e-15
    v.roll_dir = (0.0, 0.0)
    assert oracle.pixel_setup(v, 5)[2] == 0.0
    v.roll_dir = (1.5, 0.0)                                   # clamped to the frame
    assert oracle.pixel_setup(v, 39)[2] == 1.0


# --------------------------------------------------------------------------
# ray-cast vs textbook rasteriser
# --------------------------------------------------------------------------

def _compare_ids(o, ref_id, ref_z, orc, pix, tol_eh=1e-9, tol_z=1e-12):
    """IDs equal except where the oracle winner or the reference winner is
    within tol_eh of an edge, or their depths tie; depth equal where IDs match."""
    bad = []
    mism = np.nonzero(o['id'] != ref_id)[0]
    if len(mism):
        hit, z, eh = orc.eval_many(pix[mism], np.maximum(ref_id[mism], 0))
    for n, q in enumerate(mism):
        if o['id'][q] >= 0 and o['ehat'][q] < tol_eh:
            continue
        if ref_id[q] >= 0 and eh[n] < tol_eh:
            continue
        if o['id'][q] >= 0 and ref_id[q] >= 0 and abs(ref_z[q] - o['z'][q]) <= 1e-9 * o['z'][q]:
            continue
        bad.append(q)
    same = (o['id'] == ref_id) & (ref_id >= 0)
    zerr = np.abs(o['z'][same] - ref_z[same]) / ref_z[same]
    return bad, (zerr.max() if zerr.size else 0.0), len(mism)


@pytest.mark.parametrize('posed,roll', [(False, (0.0, 0.0)), (True, (0.0, 0.0)), (True, (1.0, 0.0))])
def test_static_identity_foveation_equals_classic_raster(posed, roll):
    """Pin P1: no motion and alpha = 1 reduce the method to common
    rasterization (Sec. 3.1.1 constant density, Sec. 3.2 z-buffering)."""
    rng = np.random.default_rng(10)
    v, tri = scenegen.triangle_soup(rng, 600, (-1.2, -1.0, 1.5), (1.2, 1.0, 5.0), (0.05, 0.6))
    v = v.astype(np.float32)
    mesh = scenegen.Mesh(v, v.copy(), tri, np.ones_like(v))
    pose = np.zeros(6, np.float32)
    if posed:
        pose = np.array([0.05, -0.12, 0.03, 0.1, -0.05, 0.3], np.float32)
    W, H = 96, 80
    view = scenegen.View(W, H, pose, pose.copy(), fx=1.2, fy=1.4, cx=0.03, cy=-0.02, alpha=1.0,
                         fovea=(0.1, 0.1), roll_dir=roll)
    orc = oracle.Oracle(mesh, view)
    o = orc.render()
    ref_id, ref_z = classic.raster(_view_space(v, pose), tri, W, H, 1.2, 1.4, 0.03, -0.02, view.znear)
    pix = np.arange(W * H)
    bad, zerr, nm = _compare_ids(o, ref_id.ravel(), ref_z.ravel(), orc, pix)
    assert (o["id"] >= 0).sum() > 0.25 * W * H
    assert not bad, f'{len(bad)} unexplained id mismatches, e.g. pixel {bad[:5]}'
    assert zerr < 1e-12
    assert nm < 0.002 * W * H


@pytest.mark.parametrize('roll', [(1.0, 0.0), (0.0, 1.0)])
def test_rolling_column_identity(roll):
    """Pin P2: with d = (1,0) every pixel of column i is rendered at time
    t_i = (i + 1/2)/W, so column i of the rolling image equals column i of a
    classic render of the scene frozen at t_i (vertices and camera moving
    linearly in camera space).  d = (0,1) gives the same per row."""
    sc = scenegen.make_moving_soup(seed=11, n_tris=200, width=40, height=32, alpha=1.0, roll=roll,
                                   yaw_deg_s=2000.0, obj_speed=30.0, fovea=(0.0, 0.0), side=(0.2, 0.8))
    mesh, view = sc.meshes[0], sc.views[0]
    W, H = view.width, view.height
    orc = oracle.Oracle(mesh, view)
    o = orc.render()
    Ps = _view_space(mesh.v0, view.pose0)
    Pe = _view_space(mesh.v1, view.pose1)
    ref_id = np.full(W * H, -1, np.int32)
    ref_z = np.full(W * H, np.inf)
    n_lines = W if roll[0] else H
    for k in range(n_lines):
        if roll[0]:
            t = (k + 0.5) / W
        else:
            t = 1.0 - (k + 0.5) / H
        ids, zs = classic.raster((1 - t) * Ps + t * Pe, mesh.tri, W, H, view.fx, view.fy, view.cx, view.cy,
                                 view.znear)
        if roll[0]:
            ref_id.reshape(H, W)[:, k] = ids[:, k]
            ref_z.reshape(H, W)[:, k] = zs[:, k]
        else:
            ref_id.reshape(H, W)[k] = ids[k]
            ref_z.reshape(H, W)[k] = zs[k]
    bad, zerr, nm = _compare_ids(o, ref_id, ref_z, orc, np.arange(W * H))
    assert (o['id'] >= 0).sum() > 0.2 * W * H
    assert not bad and zerr < 1e-12
    # the motion is large enough that a non-rolling render differs
    still = oracle.Oracle(mesh, scenegen.View(W, H, view.pose0, view.pose1, fx=view.fx, fy=view.fy,
                                              alpha=1.0, roll_dir=(0.0, 0.0))).render()
    assert (still['id'] != o['id']).sum() > 0.02 * W * H


def test_foveated_pixels_sample_the_unfoveated_point():
    """Pin P3: a foveated pixel shows what a pinhole camera sees at the
    display point U(y) of its centre."""
    rng = np.random.default_rng(12)
    v, tri = scenegen.triangle_soup(rng, 200, (-1.0, -1.0, 2.0), (1.0, 1.0, 5.0), (0.05, 0.5))
    v = v.astype(np.float32)
    mesh = scenegen.Mesh(v, v.copy(), tri, np.ones_like(v))
    pose = np.array([0.02, 0.05, 0.0, 0.0, 0.1, 0.2], np.float32)
    view = scenegen.View(64, 56, pose, pose.copy(), fx=1.1, fy=1.0, fovea=(0.15, -0.1), alpha=2.0,
                         roll_dir=(0.0, 0.0))
    orc = oracle.Oracle(mesh, view)
    o = orc.render()
    pts = np.array([oracle.pixel_setup(view, p)[1] for p in range(64 * 56)])
    ref_id, ref_z = classic.sample(_view_space(v, pose), tri, pts, 1.1, 1.0, 0.0, 0.0, view.znear)
    bad, zerr, nm = _compare_ids(o, ref_id, ref_z, orc, np.arange(64 * 56))
    assert not bad and zerr < 1e-12
    # foveation changes the picture: the plain pinhole image differs
    plain = oracle.Oracle(mesh, scenegen.View(64, 56, pose, pose.copy(), fx=1.1, fy=1.0, alpha=1.0,
                                              roll_dir=(0.0, 0.0))).render()
    assert (plain['id'] != o['id']).sum() > 0.1 * 64 * 56


def test_depth_is_view_space_z_and_near_plane():
    """A fronto-parallel quad at Z = 3 seen through a rotated, translated
    camera has depth 3 at every covered pixel; moved to Z = 0.04 < znear it
    disappears; straddling the eye it is cut at znear."""
    quad = np.array([[-4, -4, 3], [4, -4, 3], [4, 4, 3], [-4, 4, 3]], np.float64)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    w = np.array([0.1, -0.2, 0.05])
    R = Rotation.from_rotvec(w).as_matrix()
    T = np.array([0.3, -0.1, 0.7])
    world = (quad - T) @ R                       # R world + T = quad
    pose = np.concatenate([w, T]).astype(np.float32)
    world = world.astype(np.float32)
    mesh = scenegen.Mesh(world, world.copy(), tri, np.ones((4, 3), np.float32))
    view = scenegen.View(32, 32, pose, pose.copy(), alpha=2.0, roll_dir=(1.0, 0.0))
    o = oracle.Oracle(mesh, view).render()
    Pv = _view_space(world, pose)
    assert np.abs(Pv[:, 2] - 3).max() < 1e-6
    hit = o['id'] >= 0
    assert hit.all()
    # float32 inputs: the plane is at z = 3 up to the input rounding
    assert np.abs(o['z'][hit] - 3.0).max() < 1e-6
    near = scenegen.Mesh(np.array([[-1, -1, .04], [1, -1, .04], [0, 1, .04]], np.float32),
                         np.array([[-1, -1, .04], [1, -1, .04], [0, 1, .04]], np.float32),
                         np.array([[0, 1, 2]], np.int32), np.ones((3, 3), np.float32))
    vz = scenegen.View(16, 16, np.zeros(6, np.float32), np.zeros(6, np.float32), alpha=1.0, roll_dir=(0, 0))
    assert (oracle.Oracle(near, vz).render()['id'] < 0).all()
    # a triangle with one vertex behind the eye: hits only where z >= znear
    cut = scenegen.Mesh(np.array([[-1, -1, 1.0], [1, -1, 1.0], [0, 1, -0.5]], np.float32),
                        np.array([[-1, -1, 1.0], [1, -1, 1.0], [0, 1, -0.5]], np.float32),
                        np.array([[0, 1, 2]], np.int32), np.ones((3, 3), np.float32))
    oc = oracle.Oracle(cut, vz).render()
    assert (oc['id'] >= 0).any() and (oc['z'][oc['id'] >= 0] >= 0.05).all()


# --------------------------------------------------------------------------
# shading and gradient
# --------------------------------------------------------------------------

def test_lambert_closed_form_for_a_facing_plane():
    """Uniform albedo on a plane facing the camera lit along its normal
    (rolling light with a static camera): c = albedo (k_a + (1-k_a) n.l)."""
    quad = np.array([[-4, -4, 3], [4, -4, 3], [4, 4, 3], [-4, 4, 3]], np.float32)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    alb = np.tile(np.array([[0.3, 0.6, 0.9]], np.float32), (4, 1))
    mesh = scenegen.Mesh(quad, quad.copy(), tri, alb)
    view = scenegen.View(16, 16, np.zeros(6, np.float32), np.zeros(6, np.float32), alpha=2.0, roll_dir=(1, 0))
    orc = oracle.Oracle(mesh, view)
    ids = orc.render()['id']
    for ldir, expect in [((0, 0, -1), 1.0), ((0, 0.6, -0.8), 0.8), ((0, 0, 1), 0.0)]:
        light = np.array([*ldir, 0.1])
        rgb = orc.shade(ids, light)
        s = 0.1 + 0.9 * expect
        assert np.abs(rgb - np.array([0.3, 0.6, 0.9]) * s).max() < 1e-6


def _small_grad_case():
    sc = scenegen.make_grad(seed=5, size=40, f=8)
    mesh, view, target = sc.meshes[0], sc.views[0], sc.extra['target']
    light = oracle.light_block(sc)
    orc_t = oracle.Oracle(target, view)
    tgt = orc_t.shade(orc_t.render()['id'], light)
    orc = oracle.Oracle(mesh, view)
    ids = orc.render()['id']
    return sc, mesh, view, light, tgt, orc, ids


def test_gradient_matches_central_differences():
    sc, mesh, view, light, tgt, orc, ids = _small_grad_case()
    L, g0, g1, gp0, gp1 = orc.loss_grad(ids, light, tgt)
    assert abs(L - orc.loss(ids, light, tgt)) < 1e-12 * L
    h = 1e-6
    v0 = mesh.v0.astype(np.float64)
    v1 = mesh.v1.astype(np.float64)
    vis = np.unique(mesh.tri[ids[ids >= 0]].ravel())
    rng = np.random.default_rng(3)
    checks = 0
    for vi in rng.choice(vis, size=12, replace=False):
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
                checks += 1
    for which, gp in ((0, gp0), (1, gp1)):
        for k in range(6):
            p0 = view.pose0.astype(np.float64).copy()
            p1 = view.pose1.astype(np.float64).copy()
            pp = [p0.copy(), p1.copy()]
            pm = [p0.copy(), p1.copy()]
            pp[which][k] += h
            pm[which][k] -= h
            lp = oracle.Oracle(mesh, view, pose0=pp[0], pose1=pp[1]).loss(ids, light, tgt)
            lm = oracle.Oracle(mesh, view, pose0=pm[0], pose1=pm[1]).loss(ids, light, tgt)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gp[k]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(gp).max()), (which, k, fd, gp[k])
            checks += 1
    assert checks == 84


def test_gradient_translation_identity():
    """Pin P7: moving every start vertex by a world offset u equals moving the
    camera translation by R0 u, so sum_v dL/dv0_v = R0^T dL/dT0 (and the same at t1)."""
    sc, mesh, view, light, tgt, orc, ids = _small_grad_case()
    L, g0, g1, gp0, gp1 = orc.loss_grad(ids, light, tgt)
    R0 = Rotation.from_rotvec(view.pose0[:3].astype(np.float64)).as_matrix()
    R1 = Rotation.from_rotvec(view.pose1[:3].astype(np.float64)).as_matrix()
    assert np.abs(g0.sum(0) - R0.T @ gp0[3:]).max() < 1e-9 * np.abs(gp0[3:]).max()
    assert np.abs(g1.sum(0) - R1.T @ gp1[3:]).max() < 1e-9 * np.abs(gp1[3:]).max()
    assert np.abs(gp0).max() > 0 and np.abs(gp1).max() > 0


def test_rolling_shading_column_identity():
    """Shading at a pixel uses the scene and the light at that pixel's time
    (Sec. 3.2 "Shading"): column i of the rolling shaded image equals a
    static Lambert shading of the scene frozen at t_i = (i+1/2)/W, whose
    camera-space light is the start/end light interpolated to t_i, with
    albedo blended by the classic rasteriser's perspective-correct weights."""
    sc = scenegen.make_moving_soup(seed=13, n_tris=500, width=36, height=28, alpha=1.0, roll=(1.0, 0.0),
                                   yaw_deg_s=2000.0, obj_speed=20.0, fovea=(0.0, 0.0), side=(0.2, 0.8),
                                   centre_lo=(-1.5, -1.5, 2.0))
    mesh, view = sc.meshes[0], sc.views[0]
    W, H = view.width, view.height
    light = oracle.light_block(sc)
    orc = oracle.Oracle(mesh, view)
    o = orc.render()
    rgb = orc.shade(o['id'], light).reshape(H, W, 3)
    R0 = Rotation.from_rotvec(view.pose0[:3].astype(np.float64)).as_matrix()
    R1 = Rotation.from_rotvec(view.pose1[:3].astype(np.float64)).as_matrix()
    Ps, Pe = _view_space(mesh.v0, view.pose0), _view_space(mesh.v1, view.pose1)
    alb = mesh.albedo.astype(np.float64)
    checked = 0
    for i in range(W):
        t = (i + 0.5) / W
        P = (1 - t) * Ps + t * Pe
        ids, zs, bc = classic.raster(P, mesh.tri, W, H, view.fx, view.fy, view.cx, view.cy, view.znear,
                                     cols=[i], bary=True)
        lt = (1 - t) * (R0 @ light[:3]) + t * (R1 @ light[:3])
        lt /= np.linalg.norm(lt)
        for j in range(H):
            f = ids[j, i]
            if f < 0 or f != o['id'][j * W + i] or o['ehat'][j * W + i] < 1e-9:
                continue
            a, b, c = P[mesh.tri[f]]
            n = np.cross(b - a, c - a)
            n /= np.linalg.norm(n)
            ray = np.array([(2 * (i + 0.5) / W - 1 - view.cx) / view.fx, (1 - 2 * (j + 0.5) / H - view.cy) / view.fy, 1])
            if n @ ray > 0:
                n = -n
            s = light[3] + (1 - light[3]) * max(0.0, n @ lt)
            expect = (bc[j, i] @ alb[mesh.tri[f]]) * s
            assert np.abs(rgb[j, i] - expect).max() < 1e-12, (i, j)
            checked += 1
    assert checked > 0.2 * W * H


def test_exact_depth_tie_goes_to_lower_index():
    """Coincident triangles tie exactly in depth; the packed (depth, id) order
    resolves the tie to the lower triangle index, and the runner-up is the
    other copy."""
    v = np.array([[-1, -1, 2], [1, -1, 2], [0, 1, 2.5]], np.float32)
    v = np.concatenate([v, v, v + np.float32([0, 0, 1])])
    tri = np.array([[6, 7, 8], [3, 4, 5], [0, 1, 2]], np.int32)
    mesh = scenegen.Mesh(v, v.copy(), tri, np.ones_like(v))
    view = scenegen.View(24, 24, np.zeros(6, np.float32), np.zeros(6, np.float32), alpha=2.0, roll_dir=(1, 0))
    o = oracle.Oracle(mesh, view).render()
    hit = o['id'] >= 0
    assert hit.sum() > 50
    assert (o['id'][hit] == 1).all() and (o['id2'][hit] == 2).all()
    assert (o['z'][hit] == o['z2'][hit]).all()


def test_edge_metric_and_incidence_cosine_closed_forms():
    """ehat is the sine of the angle between the pixel ray and the nearest
    edge plane through the eye; cosinc is |cos| of the ray / normal angle.
    A triangle with one edge in the plane y = 0 (through the eye) and its
    face in the plane z = 3: near that edge ehat = |r_y| / |r| and
    cosinc = 1 / |r| everywhere."""
    v = np.array([[-3, 0, 3], [3, 0, 3], [0, 3, 3]], np.float32)   # edge (0,1) lies in y = 0
    mesh = scenegen.Mesh(v, v.copy(), np.array([[0, 1, 2]], np.int32), np.ones_like(v))
    view = scenegen.View(32, 32, np.zeros(6, np.float32), np.zeros(6, np.float32), alpha=1.0, roll_dir=(0, 0))
    orc = oracle.Oracle(mesh, view)
    o = orc.render()
    rows = [15, 14]                      # the two rows just above y = 0
    checked = 0
    for j in rows:
        for i in range(12, 20):
            p = j * 32 + i
            _, x, t, r = oracle.pixel_setup(view, p)
            hit, z, eh, cs = orc.eval_many(np.array([p]), np.array([0]), with_cos=True)
            assert hit[0] and o['id'][p] == 0
            assert abs(eh[0] - abs(r[1]) / np.linalg.norm(r)) < 1e-12
            assert abs(cs[0] - 1.0 / np.linalg.norm(r)) < 1e-12
            assert abs(o['ehat'][p] - eh[0]) < 1e-15
            checked += 1
    assert checked == 16


# --------------------------------------------------------------------------
# every hit (the bound invariant's checker) and the grid-accelerated render
# --------------------------------------------------------------------------

def _soup(seed=41, n=300, w=48, h=40, **kw):
    base = dict(alpha=2.0, roll=(1.0, 0.0), yaw_deg_s=3000.0, obj_speed=30.0, side=(0.05, 0.6))
    base.update(kw)
    return scenegen.make_moving_soup(seed=seed, n_tris=n, width=w, height=h, **base)


def _near_plane_scene():
    """A soup plus triangles that cross the near plane (some space-time
    vertices behind z = znear, one behind the eye) and cover many pixels,
    and one triangle entirely behind the eye."""
    sc = _soup(seed=43, n=200, w=56, h=44)
    m = sc.meshes[0]
    extra0 = np.array([[-2.0, -1.5, 0.01], [2.5, -1.0, 4.0], [0.0, 2.0, 3.0],
                       [-1.0, 1.0, -0.5], [1.5, 1.5, 2.0], [1.0, -2.0, 0.04],
                       [-1.0, -1.0, -1.0], [1.0, -1.0, -2.0], [0.0, 1.0, -1.5]], np.float32)
    extra1 = extra0 + np.float32([0.02, 0.0, 0.06])
    nv = m.v0.shape[0]
    v0 = np.concatenate([m.v0, extra0])
    v1 = np.concatenate([m.v1, extra1])
    tri = np.concatenate([m.tri, nv + np.arange(9, dtype=np.int32).reshape(3, 3)])
    alb = np.concatenate([m.albedo, np.full((9, 3), 0.5, np.float32)])
    return scenegen.Scene('near', [scenegen.Mesh(v0, v1, tri, alb)], sc.views)


def test_all_hits_equals_pairwise_evaluation():
    """orc_all_hits (the checker of the bound invariant: every covered
    fragment, occluded or not) returns exactly the (pixel, triangle) pairs
    the per-pair evaluation calls hits, over every pair of a small moving
    scene, with the same edge metric; it contains every winner and
    runner-up of the render; with a pixel subset it reports the given pixel
    indices."""
    for sc in (_soup(), _near_plane_scene()):
        v = sc.views[0]
        orc = oracle.Oracle(sc.meshes[0], v)
        npx, nt = v.width * v.height, sc.meshes[0].nt
        hp, ht, he = orc.all_hits()
        pp = np.repeat(np.arange(npx), nt)
        ff = np.tile(np.arange(nt, dtype=np.int32), npx)
        hit, _, eh = orc.eval_many(pp, ff)
        ref = set(zip(pp[hit].tolist(), ff[hit].tolist()))
        got = list(zip(hp.tolist(), ht.tolist()))
        assert len(got) == len(set(got)) == len(ref) and set(got) == ref
        # many pixels see more than one triangle (occluded hits are kept)
        assert np.bincount(hp, minlength=npx).max() >= 3
        ehref = dict(zip(zip(pp[hit].tolist(), ff[hit].tolist()), eh[hit].tolist()))
        assert all(ehref[k] == e for k, e in zip(got, he.tolist()))
        o = orc.render()
        for key in ('id', 'id2'):
            win = np.nonzero(o[key] >= 0)[0]
            assert set(zip(win.tolist(), o[key][win].tolist())) <= ref
        sub = np.random.default_rng(5).permutation(npx)[: npx // 3]
        sp, st, _ = orc.all_hits(sub)
        subset = set(sub.tolist())
        assert set(zip(sp.tolist(), st.tolist())) == {k for k in ref if k[0] in subset}


@pytest.mark.parametrize('grid', [0, 1, 7, 64])
def test_fast_render_equals_brute_force(grid):
    """orc_render_fast gives orc_render's outputs bit for bit (winner and
    runner-up ids, depths, edge metric): moving soups under fast yaw with
    foveation and rolling, triangles crossing the near plane or behind the
    eye, rolling off, ragged sizes, full frames and pixel subsets."""
    scenes = [_soup(), _soup(seed=44, n=400, w=61, h=37, alpha=3.0, roll=(0.0, 0.9), fovea=(-0.2, 0.2)),
              _soup(seed=45, n=250, w=40, h=52, alpha=1.0, roll=(0.0, 0.0)), _near_plane_scene()]
    for sc in scenes:
        v = sc.views[0]
        orc = oracle.Oracle(sc.meshes[0], v)
        a, b = orc.render(), orc.render_fast(grid=grid)
        assert (a['id'] >= 0).sum() > 200
        for k in a:
            assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), (sc.name, grid, k)
        pix = np.random.default_rng(6).permutation(v.width * v.height)[:500]
        a, b = orc.render(pix), orc.render_fast(pix, grid=grid)
        for k in a:
            assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), (sc.name, grid, k)


def test_fast_render_exact_ties():
    """The grid render keeps the brute force's tie order: coincident
    triangles tie exactly in depth and resolve to the lower index, the other
    copy being the runner-up."""
    v = np.array([[-1, -1, 2], [1, -1, 2], [0, 1, 2.5]], np.float32)
    v = np.concatenate([v, v, v + np.float32([0, 0, 1])])
    tri = np.array([[6, 7, 8], [3, 4, 5], [0, 1, 2]], np.int32)
    mesh = scenegen.Mesh(v, v.copy(), tri, np.ones_like(v))
    view = scenegen.View(24, 24, np.zeros(6, np.float32), np.zeros(6, np.float32), alpha=2.0, roll_dir=(1, 0))
    o = oracle.Oracle(mesh, view).render_fast(grid=4)
    hit = o['id'] >= 0
    assert hit.sum() > 50
    assert (o['id'][hit] == 1).all() and (o['id2'][hit] == 2).all()
