"""Seeded synthetic inputs for perceptual rasterization.

This module only draws inputs: meshes (vertex positions at frame start and
end, triangle indices, per-vertex albedo), camera poses at frame start and
end, fovea points, image sizes and light directions.  It holds none of the
method's arithmetic (no projection, foveation, pixel time, intersection or
shading); both the CPU oracle and the GPU library consume what it returns.

Units are metres; a frame interval of 11.1 ms (90 Hz) maps to unit time
[0, 1].  All arrays are float32 / int32.  Poses are world-to-view
transforms given as a rotation vector (3) followed by a translation (3):
a view-space point is ``R(omega) @ v + T``.  View space: x right, y up,
+z forward; NDC x = fx*X/Z + cx, y = fy*Y/Z + cy.

Workloads (sizes follow the paper's scene range of 13k..1.4M triangles,
Tables 1 and 2; the scenes themselves are not available, so these stand in):

* ``tiny``   2,000-triangle soup, static camera, 256x256, fovea at centre,
             alpha 2, rolling off.
* ``hmd``    displaced geodesic sphere (147,920 tris) + 500 tessellated boxes
             (54,000 tris) = 201,920 tris; two eyes at 1512x1680; head yaw
             120 deg/s and translation 0.5 m/s over the frame; fovea in the
             central 20 % of each eye; alpha 2; rolling left to right.
* ``large``  1,000 geodesic spheres of 2,000 tris (2M tris) each with its own
             linear velocity (|v| <= 2 m/s); two eyes at 2160x2160.
* ``batch``  64 views, log-uniform sizes 128..2048 and scenes 1k..500k tris.
* ``grad``   displaced geodesic(71) sphere (100,820 tris), one 512x512 view,
             plus a target mesh with N(0, 0.01^2) vertex noise.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field

import numpy as np

FRAME_S = 0.0111          # frame interval in seconds (90 Hz)
ZNEAR = 0.05              # near plane in metres
AMBIENT = 0.1             # Lambert ambient term k_a
LIGHT_W = (-0.3, 0.8, -0.5)  # world-space direction towards the light (normalised below)


@dataclass
class View:
    width: int
    height: int
    pose0: np.ndarray            # float32 [6]: rotation vector, translation (world -> view at t0)
    pose1: np.ndarray            # float32 [6]: same at t1
    fx: float = 1.0
    fy: float = 1.0
    cx: float = 0.0
    cy: float = 0.0
    znear: float = ZNEAR
    fovea: tuple = (0.0, 0.0)    # fovea point in foveated NDC
    alpha: float = 2.0           # power-law foveation exponent, 1 = off
    roll_dir: tuple = (1.0, 0.0)  # rolling skew direction d, (0, 0) = off
    mesh: int = 0                # index of the mesh this view renders
    profile_c: np.ndarray = None  # float32 samples of a tabulated foveation p_c (None: the power law)
    profile_l: np.ndarray = None  # float32 samples of a tabulated lens distortion p_l (None: no lens)


@dataclass
class Mesh:
    v0: np.ndarray      # float32 [V, 3] world positions at t0
    v1: np.ndarray      # float32 [V, 3] world positions at t1
    tri: np.ndarray     # int32 [T, 3]
    albedo: np.ndarray  # float32 [V, 3]

    @property
    def nv(self) -> int:
        return int(self.v0.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tri.shape[0])


@dataclass
class Scene:
    name: str
    meshes: list
    views: list
    light_dir: np.ndarray = field(default_factory=lambda: _unit(np.array(LIGHT_W, np.float64)).astype(np.float32))
    ambient: float = AMBIENT
    extra: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------
# small helpers (input construction only)
# ----------------------------------------------------------------------------

def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _random_rotation_matrices(rng, n):
    """Uniform random rotations (normalised Gaussian quaternions)."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    m = np.empty((n, 3, 3))
    m[:, 0, 0] = 1 - 2 * (y * y + z * z)
    m[:, 0, 1] = 2 * (x * y - z * w)
    m[:, 0, 2] = 2 * (x * z + y * w)
    m[:, 1, 0] = 2 * (x * y + z * w)
    m[:, 1, 1] = 1 - 2 * (x * x + z * z)
    m[:, 1, 2] = 2 * (y * z - x * w)
    m[:, 2, 0] = 2 * (x * z - y * w)
    m[:, 2, 1] = 2 * (y * z + x * w)
    m[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return m


def _yaw_matrix(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def head_pose(t_s: float, yaw_rate_deg: float, vel: tuple, eye_offset: float):
    """World->view pose (rotvec, T) of an eye on a head that yaws about +y at
    ``yaw_rate_deg`` and translates at ``vel`` (m/s), ``t_s`` seconds into the
    frame.  The eye sits ``eye_offset`` metres along the head's x axis."""
    theta = math.radians(yaw_rate_deg) * t_s
    rh = _yaw_matrix(theta)                       # head -> world rotation
    head = np.array(vel, np.float64) * t_s
    eye = head + rh @ np.array([eye_offset, 0.0, 0.0])
    r_wv = rh.T                                   # world -> view rotation
    t_wv = -(r_wv @ eye)
    omega = np.array([0.0, -theta, 0.0])          # rotation vector of rh.T
    return np.concatenate([omega, t_wv]).astype(np.float32)


@functools.lru_cache(maxsize=64)
def _geodesic_unit(f: int):
    """Icosahedron with every face split f x f, vertices pushed to the unit
    sphere.  Returns (verts [10f^2+2, 3] float64, tris [20 f^2, 3] int32);
    cached per f (callers must not modify the arrays)."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    ico_v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                      [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                      [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], np.float64)
    ico_v /= np.linalg.norm(ico_v, axis=1, keepdims=True)
    ico_f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    # every grid point of every face as integer weights on <= 3 icosahedron
    # vertices; points shared by faces have equal canonical keys
    ii, jj = np.meshgrid(np.arange(f + 1), np.arange(f + 1), indexing='ij')
    sel = (ii + jj) <= f
    gi, gj = ii[sel], jj[sel]                   # i outer, j inner
    npf = gi.size
    grid_id = -np.ones((f + 1, f + 1), np.int64)
    grid_id[gi, gj] = np.arange(npf)
    fa = np.array(ico_f)
    idx = np.stack([np.repeat(fa[:, 0], npf), np.repeat(fa[:, 1], npf), np.repeat(fa[:, 2], npf)], axis=1)
    wts = np.stack([np.tile(f - gi - gj, 20), np.tile(gi, 20), np.tile(gj, 20)], axis=1)
    idx = np.where(wts > 0, idx, 15)
    order = np.argsort(idx, axis=1, kind='stable')
    idx_s = np.take_along_axis(idx, order, 1)
    w_s = np.take_along_axis(wts, order, 1)
    keys = ((idx_s[:, 0] * 256 + w_s[:, 0]) << 24) | ((idx_s[:, 1] * 256 + w_s[:, 1]) << 12) | (idx_s[:, 2] * 256 + w_s[:, 2])
    _, first, inverse = np.unique(keys, return_index=True, return_inverse=True)
    rank = np.empty(first.size, np.int64)
    rank[np.argsort(first, kind='stable')] = np.arange(first.size)
    vid = rank[inverse]                         # vertex id of every (face, point), first-appearance order
    pos = np.zeros((first.size, 3))
    wsum = (wts[:, :, None] * ico_v[np.minimum(idx, 11)]).sum(1) / f
    pos[vid] = wsum
    verts = pos / np.linalg.norm(pos, axis=1, keepdims=True)
    tri_i, tri_j = np.meshgrid(np.arange(f), np.arange(f), indexing='ij')
    ts = (tri_i + tri_j) < f
    ti, tj = tri_i[ts], tri_j[ts]
    t1 = np.stack([grid_id[ti, tj], grid_id[ti + 1, tj], grid_id[ti, tj + 1]], axis=1)
    has2 = (ti + tj + 1) < f
    t2 = np.stack([grid_id[ti + 1, tj], grid_id[np.minimum(ti + 1, f), np.minimum(tj + 1, f)],
                   grid_id[ti, tj + 1]], axis=1)
    both = np.stack([t1, t2], axis=1).reshape(-1, 3)
    keep = np.stack([np.ones_like(has2), has2], axis=1).reshape(-1)
    local = both[keep]
    tris = (local[None, :, :] + (np.arange(20) * npf)[:, None, None]).reshape(-1, 3)
    tris = vid[tris]
    v = np.ascontiguousarray(verts)
    t = np.ascontiguousarray(tris, np.int32)
    assert v.shape[0] == 10 * f * f + 2 and t.shape[0] == 20 * f * f
    v.flags.writeable = False
    t.flags.writeable = False
    return v, t


def _displacement(rng, dirs):
    """Radial displacement 0.05 * sum_o 2^-o sin(k_o . v + phi_o), |k_o| = 3*2^o."""
    out = np.zeros(dirs.shape[0])
    for o in range(1, 5):
        k = _unit(rng.normal(size=3)) * (3.0 * 2 ** o)
        phi = rng.uniform(0, 2 * math.pi)
        out += 2.0 ** (-o) * np.sin(dirs @ k + phi)
    return 0.05 * out


def displaced_sphere(rng, f, radius, centre):
    d, tri = _geodesic_unit(f)
    r = radius + _displacement(rng, d)
    v = d * r[:, None] + np.asarray(centre, np.float64)
    return v, tri.copy()


@functools.lru_cache(maxsize=8)
def _box_template(tess: int):
    """Unit-half-size box [-1,1]^3, every face split tess x tess, faces not
    sharing vertices: (verts [6 (tess+1)^2, 3], tris [12 tess^2, 3])."""
    verts, tris = [], []
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            u_ax, v_ax = [a for a in range(3) if a != axis]
            base = len(verts)
            for i in range(tess + 1):
                for j in range(tess + 1):
                    p = np.zeros(3)
                    p[axis] = sgn
                    p[u_ax] = -1 + 2 * i / tess
                    p[v_ax] = -1 + 2 * j / tess
                    verts.append(p)
            for i in range(tess):
                for j in range(tess):
                    a = base + i * (tess + 1) + j
                    b = a + tess + 1
                    tris.append((a, b, a + 1))
                    tris.append((b, b + 1, a + 1))
    return np.array(verts), np.array(tris, np.int32)


def random_boxes(rng, n, tess=1, lo=(-4, -2.5, 1.5), hi=(4, 2.5, 12), size=(0.05, 0.5)):
    """n boxes at once: per-axis size log-U(size), uniform rotation, centre
    U(lo, hi).  Returns (verts, tris)."""
    tv, tt = _box_template(tess)
    half = np.exp(rng.uniform(math.log(size[0]), math.log(size[1]), size=(n, 3))) / 2.0
    rot = _random_rotation_matrices(rng, n)
    centre = rng.uniform(lo, hi, size=(n, 3))
    v = np.einsum('nij,nkj->nki', rot, tv[None] * half[:, None, :]) + centre[:, None, :]
    t = tt[None] + (np.arange(n) * tv.shape[0])[:, None, None]
    return v.reshape(-1, 3), t.reshape(-1, 3).astype(np.int32)


def _box(rng, size, rot, centre, tess=3):
    """Axis box (per-axis ``size``) with every face split tess x tess quads;
    faces do not share vertices.  Returns (verts, tris)."""
    verts, tris = [], []
    half = np.asarray(size, np.float64) / 2.0
    for axis in range(3):
        for sgn in (-1.0, 1.0):
            u_ax, v_ax = [a for a in range(3) if a != axis]
            base = len(verts)
            for i in range(tess + 1):
                for j in range(tess + 1):
                    p = np.zeros(3)
                    p[axis] = sgn * half[axis]
                    p[u_ax] = (-1 + 2 * i / tess) * half[u_ax]
                    p[v_ax] = (-1 + 2 * j / tess) * half[v_ax]
                    verts.append(p)
            for i in range(tess):
                for j in range(tess):
                    a = base + i * (tess + 1) + j
                    b = a + tess + 1
                    tris.append((a, b, a + 1))
                    tris.append((b, b + 1, a + 1))
    v = np.array(verts) @ rot.T + np.asarray(centre, np.float64)
    return v, np.array(tris, np.int32)


def _concat(parts):
    vs, ts, off = [], [], 0
    for v, t in parts:
        vs.append(v)
        ts.append(t + off)
        off += v.shape[0]
    return np.concatenate(vs), np.concatenate(ts).astype(np.int32)


def _identity_pose():
    return np.zeros(6, np.float32)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def triangle_soup(rng, n, centre_lo=(-1, -1, 2), centre_hi=(1, 1, 6), side=(0.02, 0.2)):
    """n random triangles: side lengths U(side) redrawn until the triangle
    inequality holds, built in-plane about their centroid, uniformly rotated
    and placed at a centroid drawn from the given box.  No shared vertices."""
    sides = np.empty((n, 3))
    for k in range(n):
        while True:
            a, b, c = rng.uniform(side[0], side[1], size=3)
            if a + b > c and a + c > b and b + c > a:
                break
        sides[k] = (a, b, c)
    a, b, c = sides[:, 0], sides[:, 1], sides[:, 2]
    x2 = (b * b + c * c - a * a) / (2 * c)
    y2 = np.sqrt(np.maximum(b * b - x2 * x2, 0.0))
    p = np.zeros((n, 3, 3))
    p[:, 1, 0] = c
    p[:, 2, 0] = x2
    p[:, 2, 1] = y2
    p -= p.mean(axis=1, keepdims=True)
    rot = _random_rotation_matrices(rng, n)
    p = np.einsum('nij,nkj->nki', rot, p)
    centre = rng.uniform(centre_lo, centre_hi, size=(n, 3))
    p += centre[:, None, :]
    v = p.reshape(-1, 3)
    tri = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    return v, tri


def _albedo(rng, nv):
    return rng.uniform(0.2, 1.0, size=(nv, 3)).astype(np.float32)


def make_tiny(seed: int = 1, n_tris: int = 2000, size: int = 256) -> Scene:
    rng = np.random.default_rng(seed)
    v, tri = triangle_soup(rng, n_tris)
    v = v.astype(np.float32)
    mesh = Mesh(v0=v, v1=v.copy(), tri=tri, albedo=_albedo(rng, v.shape[0]))
    f = float(np.float32(1.0 / math.tan(math.radians(30.0))))
    view = View(size, size, _identity_pose(), _identity_pose(), fx=f, fy=f,
                fovea=(0.0, 0.0), alpha=2.0, roll_dir=(0.0, 0.0))
    return Scene('tiny', [mesh], [view])


def _hmd_views(rng, width, height, fx, fy, yaw_deg_s=120.0, vel=(0.5, 0.0, 0.0), ipd=0.064, n_eyes=2):
    views = []
    offs = [-ipd / 2, ipd / 2] if n_eyes == 2 else [0.0]
    for off in offs:
        fov = tuple(float(np.float32(x)) for x in rng.uniform(-0.2, 0.2, size=2))
        views.append(View(width, height,
                          head_pose(0.0, yaw_deg_s, vel, off),
                          head_pose(FRAME_S, yaw_deg_s, vel, off),
                          fx=fx, fy=fy, fovea=fov, alpha=2.0, roll_dir=(1.0, 0.0)))
    return views


def make_hmd(seed: int = 2, width: int = 1512, height: int = 1680, sphere_f: int = 86,
             n_boxes: int = 500) -> Scene:
    rng = np.random.default_rng(seed)
    parts = [displaced_sphere(rng, sphere_f, 1.0, (0.0, 0.0, 3.0))]
    for _ in range(n_boxes):
        size = np.exp(rng.uniform(math.log(0.05), math.log(0.5), size=3))
        rot = _random_rotation_matrices(rng, 1)[0]
        centre = rng.uniform((-4, -2.5, 1.5), (4, 2.5, 12))
        parts.append(_box(rng, size, rot, centre))
    v, tri = _concat(parts)
    v = v.astype(np.float32)
    mesh = Mesh(v0=v, v1=v.copy(), tri=tri, albedo=_albedo(rng, v.shape[0]))
    fy = float(np.float32(1.0 * width / height))
    views = _hmd_views(rng, width, height, 1.0, fy)
    return Scene('hmd', [mesh], views)


def make_large(seed: int = 3, size: int = 2160, n_obj: int = 1000, f: int = 10) -> Scene:
    rng = np.random.default_rng(seed)
    unit_v, unit_t = _geodesic_unit(f)
    vs, ts, vel = [], [], []
    for k in range(n_obj):
        r = math.exp(rng.uniform(math.log(0.05), math.log(0.5)))
        c = rng.uniform((-6, -3, 1.5), (6, 3, 20))
        d = _unit(rng.normal(size=3)) * 2.0 * rng.uniform() ** (1.0 / 3.0)
        vs.append(unit_v * r + c)
        ts.append(unit_t + k * unit_v.shape[0])
        vel.append(np.broadcast_to(d, unit_v.shape))
    v0 = np.concatenate(vs)
    v1 = v0 + np.concatenate(vel) * FRAME_S
    tri = np.concatenate(ts).astype(np.int32)
    mesh = Mesh(v0=v0.astype(np.float32), v1=v1.astype(np.float32), tri=tri,
                albedo=_albedo(rng, v0.shape[0]))
    views = _hmd_views(rng, size, size, 1.0, 1.0)
    return Scene('large', [mesh], views)


def make_batch(seed: int = 4, n_views: int = 64, max_side: int = 2048, max_tris: int = 500_000,
               min_side: int = 128, min_tris: int = 1000) -> Scene:
    meshes, views = [], []
    for k in range(n_views):
        rng = np.random.default_rng(4000 + k)
        side = int(round(math.exp(rng.uniform(math.log(min_side), math.log(max_side)))))
        n_t = int(round(math.exp(rng.uniform(math.log(min_tris), math.log(max_tris)))))
        n_sphere = int(0.75 * n_t)
        f = max(1, int(round(math.sqrt(n_sphere / 20.0))))
        parts = [displaced_sphere(rng, f, 1.0, (0.0, 0.0, 3.0))]
        n_box = max(0, (n_t - 20 * f * f) // 12)
        if n_box:
            parts.append(random_boxes(rng, n_box, tess=1))
        v, tri = _concat(parts)
        v = v.astype(np.float32)
        meshes.append(Mesh(v0=v, v1=v.copy(), tri=tri, albedo=_albedo(rng, v.shape[0])))
        yaw = rng.uniform(-120, 120)
        vel = tuple(_unit(rng.normal(size=3)) * rng.uniform(0, 0.5))
        fov = tuple(float(np.float32(x)) for x in rng.uniform(-0.2, 0.2, size=2))
        views.append(View(side, side, head_pose(0.0, yaw, vel, 0.0), head_pose(FRAME_S, yaw, vel, 0.0),
                          fx=1.0, fy=1.0, fovea=fov, alpha=2.0, roll_dir=(1.0, 0.0), mesh=k))
    return Scene('batch', meshes, views)


def make_grad(seed: int = 5, size: int = 512, f: int = 71, noise: float = 0.01) -> Scene:
    rng = np.random.default_rng(seed)
    v, tri = displaced_sphere(rng, f, 1.0, (0.0, 0.0, 3.0))
    v = v.astype(np.float32)
    mesh = Mesh(v0=v, v1=v.copy(), tri=tri, albedo=_albedo(rng, v.shape[0]))
    noise_v = rng.normal(0.0, noise, size=v.shape)
    vt = (v.astype(np.float64) + noise_v).astype(np.float32)
    target = Mesh(v0=vt, v1=vt.copy(), tri=tri, albedo=mesh.albedo)
    fov = tuple(float(np.float32(x)) for x in rng.uniform(-0.2, 0.2, size=2))
    view = View(size, size, head_pose(0.0, 120.0, (0.5, 0.0, 0.0), 0.0),
                head_pose(FRAME_S, 120.0, (0.5, 0.0, 0.0), 0.0),
                fx=1.0, fy=1.0, fovea=fov, alpha=2.0, roll_dir=(1.0, 0.0))
    return Scene('grad', [mesh], [view], extra={'target': target})


def make_moving_soup(seed: int, n_tris: int, width: int, height: int, alpha: float = 2.0,
                     roll=(1.0, 0.0), yaw_deg_s: float = 120.0, obj_speed: float = 2.0,
                     fovea=None, fx: float = 1.0, fy: float = 1.0, centre_lo=(-1.5, -1.5, 1.0),
                     centre_hi=(1.5, 1.5, 5.0), side=(0.02, 0.3), profile_c=None, profile_l=None) -> Scene:
    """Small test workload: a triangle soup whose triangles each move with
    their own velocity (|v| <= obj_speed m/s) under a yawing, translating
    camera, foveated and rolling.  Small enough for full brute force."""
    rng = np.random.default_rng(seed)
    v, tri = triangle_soup(rng, n_tris, centre_lo, centre_hi, side)
    vel = _unit(rng.normal(size=(n_tris, 3))) * obj_speed * rng.uniform(size=(n_tris, 1)) ** (1 / 3)
    v1 = v + np.repeat(vel, 3, axis=0) * FRAME_S
    mesh = Mesh(v0=v.astype(np.float32), v1=v1.astype(np.float32), tri=tri, albedo=_albedo(rng, v.shape[0]))
    if fovea is None:
        fovea = tuple(float(np.float32(x)) for x in rng.uniform(-0.2, 0.2, size=2))
    view = View(width, height, head_pose(0.0, yaw_deg_s, (0.5, 0, 0), 0.0),
                head_pose(FRAME_S, yaw_deg_s, (0.5, 0, 0), 0.0), fx=fx, fy=fy,
                fovea=fovea, alpha=alpha, roll_dir=roll, profile_c=profile_c, profile_l=profile_l)
    return Scene('moving_soup', [mesh], [view])


def foveal_table(n: int = 33, gain: float = 3.0) -> np.ndarray:
    """n float32 samples on s = k/(n-1) of the monotone profile
    u(s) = s (1 + gain) / (1 + gain s): u(0) = 0, u(1) = 1, slope 1 + gain at
    the fovea and 1 / (1 + gain) at the farthest corner (an input for the
    tabulated foveation, of a shape no power law has)."""
    s = np.linspace(0.0, 1.0, n)
    return (s * (1.0 + gain) / (1.0 + gain * s)).astype(np.float32)


def barrel_table(n: int = 33, k: float = 0.2) -> np.ndarray:
    """n float32 samples of a barrel pre-distortion u(s) = s (1 - k s^2)
    (undistorted -> panel distance, increasing for k < 1/3)."""
    s = np.linspace(0.0, 1.0, n)
    return (s * (1.0 - k * s * s)).astype(np.float32)


WORKLOADS = {
    'tiny': make_tiny,
    'hmd': make_hmd,
    'large': make_large,
    'batch': make_batch,
    'grad': make_grad,
}


def sample_pixels(seed: int, view: View, n: int) -> np.ndarray:
    """n distinct pixel indices (row-major) of a view: half uniform over the
    image, half within 0.1 NDC of the fovea (where magnification is largest)."""
    rng = np.random.default_rng(seed)
    w, h = view.width, view.height
    n_u = n // 2
    uni = rng.choice(w * h, size=min(n_u, w * h), replace=False)
    fx, fy = view.fovea
    x0 = int(max(0, math.floor((fx - 0.1 + 1) * w / 2)))
    x1 = int(min(w, math.ceil((fx + 0.1 + 1) * w / 2)))
    y0 = int(max(0, math.floor((1 - (fy + 0.1)) * h / 2)))
    y1 = int(min(h, math.ceil((1 - (fy - 0.1)) * h / 2)))
    nb = (x1 - x0) * (y1 - y0)
    loc = rng.choice(nb, size=min(n - n_u, nb), replace=False)
    fov = (y0 + loc // (x1 - x0)) * w + (x0 + loc % (x1 - x0))
    return np.unique(np.concatenate([uni, fov])).astype(np.int64)
