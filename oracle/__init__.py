"""FP64 CPU oracle for perceptual rasterization -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never uses it, and the
two share no code: the only common module is the seeded input generator
(``scenegen``), which holds none of the method's arithmetic.

``pr_oracle.c`` is the brute-force definition (every triangle at every pixel,
the paper's "correct, but slow" solution, Sec. 3); this module compiles it
with gcc (OpenMP) and wraps it with ctypes.  ``orc_render_fast`` computes
the same render bit for bit with a conservative display-space grid of its
own (pinned against the brute force); ``classic.py`` holds the independent
textbook half-space rasteriser used to pin the brute force.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, 'pr_oracle.c')
_LIB = os.path.join(_HERE, '_pr_oracle.so')
_lib = None

NPARAM = 26 + 2 * 64
PMAX = 64


def build(force: bool = True) -> str:
    """Compile the C oracle into oracle/_pr_oracle.so (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + '.tmp'
        subprocess.check_call(['gcc', '-O2', '-fopenmp', '-fPIC', '-shared', '-std=c11',
                               '-o', tmp, _SRC, '-lm'])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    """The loaded oracle library.  ``PR_ORACLE_LIB`` may name another build of
    pr_oracle.c (the mutation tests load copies with planted mistakes)."""
    global _lib
    if _lib is None:
        path = os.environ.get('PR_ORACLE_LIB') or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.orc_rodrigues.argtypes = [dp, dp]
        L.orc_rodrigues_jac.argtypes = [dp, dp]
        L.orc_fovea_radius.argtypes = [dp]
        L.orc_fovea_radius.restype = ctypes.c_double
        L.orc_unfoveate.argtypes = [dp, dp, dp]
        L.orc_undistort.argtypes = [dp, dp, dp]
        L.orc_foveate.argtypes = [dp, dp, dp]
        L.orc_pixel_time.argtypes = [dp, dp]
        L.orc_pixel_time.restype = ctypes.c_double
        L.orc_pixel_setup.argtypes = [dp, i64, dp, dp, dp, dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        mesh = [dp, dp, ctypes.c_int, ip, ctypes.c_int]
        L.orc_render.argtypes = [dp] + mesh + [lp, i64, ip, dp, dp, ip, dp]
        L.orc_render_fast.argtypes = [dp] + mesh + [lp, i64, ip, dp, dp, ip, dp, ctypes.c_int]
        L.orc_eval.argtypes = [dp] + mesh + [i64, ctypes.c_int, dp]
        L.orc_eval.restype = ctypes.c_int
        L.orc_eval_many.argtypes = [dp] + mesh + [lp, ip, i64, ip, dp, dp, dp]
        L.orc_all_hits.argtypes = [dp] + mesh + [lp, i64, lp, ip, dp, i64]
        L.orc_all_hits.restype = i64
        L.orc_shade.argtypes = [dp] + mesh + [dp, dp, lp, i64, ip, dp]
        L.orc_loss.argtypes = [dp] + mesh + [dp, dp, ip, dp]
        L.orc_loss.restype = ctypes.c_double
        L.orc_loss_grad.argtypes = [dp] + mesh + [dp, dp, ip, dp, dp, dp, dp, dp]
        L.orc_loss_grad.restype = ctypes.c_double
        L.orc_gbuffer.argtypes = [dp] + mesh + [lp, i64, ip, dp, dp, dp]
        L.orc_foveate_jac.argtypes = [dp, dp, dp]
        L.orc_unfov_coord.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_unfov_lod.argtypes = [dp]
        L.orc_unfov_lod.restype = ctypes.c_double
        L.orc_unfoveate_image.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          lp, i64, dp]
        L.orc_mip_level.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ip, ip]
        L.orc_mip_level.restype = ctypes.c_int
        L.orc_unfov_filter_at.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def view_params(view, pose0=None, pose1=None) -> np.ndarray:
    """Parameter block of a scenegen.View (optionally overriding poses)."""
    p = np.zeros(NPARAM)
    p[0], p[1] = view.width, view.height
    p[2:8] = view.pose0 if pose0 is None else pose0
    p[8:14] = view.pose1 if pose1 is None else pose1
    p[14:19] = (view.fx, view.fy, view.cx, view.cy, view.znear)
    p[19:21] = view.fovea
    p[21] = view.alpha
    p[22:24] = view.roll_dir
    pc, pl = getattr(view, 'profile_c', None), getattr(view, 'profile_l', None)
    if pc is not None:
        pc = np.asarray(pc, np.float32).astype(np.float64)   # the float32 samples, exactly
        assert 2 <= pc.size <= PMAX
        p[24] = pc.size
        p[26:26 + pc.size] = pc
    if pl is not None:
        pl = np.asarray(pl, np.float32).astype(np.float64)
        assert 2 <= pl.size <= PMAX
        p[25] = pl.size
        p[26 + PMAX:26 + PMAX + pl.size] = pl
    return p


class Oracle:
    """Oracle bound to one mesh + view.  Vertex arrays are held in float64
    (exact copies of the float32 inputs unless overridden)."""

    def __init__(self, mesh, view, v0=None, v1=None, pose0=None, pose1=None, threads: int = 0):
        self.L = lib()
        if threads:
            self.L.orc_set_threads(threads)
        self.vp = view_params(view, pose0, pose1)
        self.v0 = _d(mesh.v0 if v0 is None else v0)
        self.v1 = _d(mesh.v1 if v1 is None else v1)
        self.tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
        self.albedo = _d(mesh.albedo)
        self.W, self.H = view.width, view.height

    def _m(self):
        return (_p(self.v0, ctypes.c_double), _p(self.v1, ctypes.c_double), self.v0.shape[0],
                _p(self.tri, ctypes.c_int32), self.tri.shape[0])

    def render(self, pix=None):
        n = self.W * self.H if pix is None else len(pix)
        pp = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
        out = dict(id=np.empty(n, np.int32), z=np.empty(n), ehat=np.empty(n),
                   id2=np.empty(n, np.int32), z2=np.empty(n))
        self.L.orc_render(_p(self.vp, ctypes.c_double), *self._m(),
                          None if pp is None else _p(pp, ctypes.c_int64), n,
                          _p(out['id'], ctypes.c_int32), _p(out['z'], ctypes.c_double),
                          _p(out['ehat'], ctypes.c_double), _p(out['id2'], ctypes.c_int32),
                          _p(out['z2'], ctypes.c_double))
        return out

    def render_fast(self, pix=None, grid: int = 0):
        """The same as render() (bit for bit) through a conservative
        display-space grid of grid x grid cells (0: from the image size)."""
        n = self.W * self.H if pix is None else len(pix)
        if grid <= 0:
            grid = int(min(1024, max(16, (self.W * self.H) ** 0.5 / 4)))
        pp = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
        out = dict(id=np.empty(n, np.int32), z=np.empty(n), ehat=np.empty(n),
                   id2=np.empty(n, np.int32), z2=np.empty(n))
        self.L.orc_render_fast(_p(self.vp, ctypes.c_double), *self._m(),
                               None if pp is None else _p(pp, ctypes.c_int64), n,
                               _p(out['id'], ctypes.c_int32), _p(out['z'], ctypes.c_double),
                               _p(out['ehat'], ctypes.c_double), _p(out['id2'], ctypes.c_int32),
                               _p(out['z2'], ctypes.c_double), grid)
        return out

    def eval_many(self, pix, fid, with_cos: bool = False):
        """Per (pixel, triangle): hit flag, depth, ehat (and |cos| of the
        ray / normal angle with with_cos)."""
        pix = np.ascontiguousarray(pix, dtype=np.int64)
        fid = np.ascontiguousarray(fid, dtype=np.int32)
        n = len(pix)
        hit, z, eh, cs = np.empty(n, np.int32), np.empty(n), np.empty(n), np.empty(n)
        self.L.orc_eval_many(_p(self.vp, ctypes.c_double), *self._m(), _p(pix, ctypes.c_int64),
                             _p(fid, ctypes.c_int32), n, _p(hit, ctypes.c_int32), _p(z, ctypes.c_double),
                             _p(eh, ctypes.c_double), _p(cs, ctypes.c_double))
        if with_cos:
            return hit.astype(bool), z, eh, cs
        return hit.astype(bool), z, eh

    def all_hits(self, pix=None, cap: int = 1 << 24):
        n = self.W * self.H if pix is None else len(pix)
        pp = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
        op, ot, oe = np.empty(cap, np.int64), np.empty(cap, np.int32), np.empty(cap)
        cnt = self.L.orc_all_hits(_p(self.vp, ctypes.c_double), *self._m(),
                                  None if pp is None else _p(pp, ctypes.c_int64), n,
                                  _p(op, ctypes.c_int64), _p(ot, ctypes.c_int32), _p(oe, ctypes.c_double), cap)
        if cnt > cap:
            raise RuntimeError(f'all_hits: {cnt} hits exceed capacity {cap}')
        return op[:cnt], ot[:cnt], oe[:cnt]

    def shade(self, ids, light, pix=None):
        n = self.W * self.H if pix is None else len(pix)
        pp = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        lt = _light6(light)
        out = np.empty((n, 3))
        self.L.orc_shade(_p(self.vp, ctypes.c_double), *self._m(), _p(self.albedo, ctypes.c_double),
                         _p(lt, ctypes.c_double), None if pp is None else _p(pp, ctypes.c_int64), n,
                         _p(ids, ctypes.c_int32), _p(out, ctypes.c_double))
        return out

    def loss(self, ids, light, target):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        lt, tg = _light6(light), _d(target)
        return self.L.orc_loss(_p(self.vp, ctypes.c_double), *self._m(), _p(self.albedo, ctypes.c_double),
                               _p(lt, ctypes.c_double), _p(ids, ctypes.c_int32), _p(tg, ctypes.c_double))

    def loss_grad(self, ids, light, target):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        lt, tg = _light6(light), _d(target)
        nv = self.v0.shape[0]
        g0, g1 = np.zeros((nv, 3)), np.zeros((nv, 3))
        gp0, gp1 = np.zeros(6), np.zeros(6)
        L = self.L.orc_loss_grad(_p(self.vp, ctypes.c_double), *self._m(), _p(self.albedo, ctypes.c_double),
                                 _p(lt, ctypes.c_double), _p(ids, ctypes.c_int32), _p(tg, ctypes.c_double),
                                 _p(g0, ctypes.c_double), _p(g1, ctypes.c_double),
                                 _p(gp0, ctypes.c_double), _p(gp1, ctypes.c_double))
        return L, g0, g1, gp0, gp1


    def gbuffer(self, ids, pix=None):
        """Per pixel: unit normal (turned to the eye) and barycentrics
        (mu_1, mu_2) of its id (zeros for misses), and the pixel density."""
        n = self.W * self.H if pix is None else len(pix)
        pp = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        out = dict(normal=np.empty((n, 3)), bary=np.empty((n, 2)), density=np.empty(n))
        self.L.orc_gbuffer(_p(self.vp, ctypes.c_double), *self._m(),
                           None if pp is None else _p(pp, ctypes.c_int64), n, _p(ids, ctypes.c_int32),
                           _p(out['normal'], ctypes.c_double), _p(out['bary'], ctypes.c_double),
                           _p(out['density'], ctypes.c_double))
        return out


def _light6(light) -> np.ndarray:
    """(l_w[3], k_a[, k_s, m]) -> the oracle's six-entry light (k_s = 0: no
    highlight)."""
    lt = np.asarray(light, np.float64).ravel()
    if lt.size == 4:
        lt = np.concatenate([lt, [0.0, 1.0]])
    assert lt.size == 6, 'light: (dir[3], ambient) or (dir[3], ambient, specular, shininess)'
    return np.ascontiguousarray(lt)


def light_block(scene, specular: float = 0.0, shininess: float = 1.0) -> np.ndarray:
    return np.array([*scene.light_dir, scene.ambient, specular, shininess], np.float64)


def rodrigues(w) -> np.ndarray:
    w = _d(w)
    R = np.empty(9)
    lib().orc_rodrigues(_p(w, ctypes.c_double), _p(R, ctypes.c_double))
    return R.reshape(3, 3)


def rodrigues_jac(w) -> np.ndarray:
    w = _d(w)
    J = np.empty(27)
    lib().orc_rodrigues_jac(_p(w, ctypes.c_double), _p(J, ctypes.c_double))
    return J.reshape(3, 3, 3)


def unfoveate(view, y) -> np.ndarray:
    vp = view_params(view)
    y = _d(y)
    x = np.empty(2)
    lib().orc_unfoveate(_p(vp, ctypes.c_double), _p(y, ctypes.c_double), _p(x, ctypes.c_double))
    return x


def undistort(view, x) -> np.ndarray:
    """Panel point -> undistorted point (the view's lens inverted; identity
    without a lens)."""
    vp = view_params(view)
    x = _d(x)
    u = np.empty(2)
    lib().orc_undistort(_p(vp, ctypes.c_double), _p(x, ctypes.c_double), _p(u, ctypes.c_double))
    return u


def foveate(view, x) -> np.ndarray:
    vp = view_params(view)
    x = _d(x)
    y = np.empty(2)
    lib().orc_foveate(_p(vp, ctypes.c_double), _p(x, ctypes.c_double), _p(y, ctypes.c_double))
    return y


def fovea_radius(view) -> float:
    return lib().orc_fovea_radius(_p(view_params(view), ctypes.c_double))


def pixel_setup(view, pix: int):
    vp = view_params(view)
    y, x, t, r = np.empty(2), np.empty(2), ctypes.c_double(), np.empty(3)
    lib().orc_pixel_setup(_p(vp, ctypes.c_double), pix, _p(y, ctypes.c_double), _p(x, ctypes.c_double),
                          ctypes.byref(t), _p(r, ctypes.c_double))
    return y, x, t.value, r


# --------------------------------------------------------------------------
# display unfoveation (Sec. 3.1.1 "Display")
# --------------------------------------------------------------------------
UNFOV_MIP = 0
UNFOV_FILTER = 1


def _rgba01(img) -> np.ndarray:
    """Foveated image as float64 RGBA in [0, 1] ([H, W, 4]; uint8 / 255)."""
    a = np.asarray(img)
    if a.dtype == np.uint8:
        return np.ascontiguousarray(a, dtype=np.float64) / 255.0
    return np.ascontiguousarray(a, dtype=np.float64)


def unfoveate_image(view, fov, width: int, height: int, mode: int = UNFOV_MIP, sigma: float = 0.5,
                    pix=None) -> np.ndarray:
    """Display image (float64 RGBA, [height*width, 4] or [len(pix), 4]) of
    the foveated image ``fov`` ([view.height, view.width, 4]) of ``view``."""
    vp = view_params(view)
    f = _rgba01(fov)
    assert f.shape == (view.height, view.width, 4)
    n = width * height if pix is None else len(pix)
    pp = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    out = np.empty((n, 4))
    lib().orc_unfoveate_image(_p(vp, ctypes.c_double), _p(f, ctypes.c_double), width, height, mode, sigma,
                              None if pp is None else _p(pp, ctypes.c_int64), n, _p(out, ctypes.c_double))
    return out


def unfov_coord(view, width: int, height: int, a: float, b: float):
    """Continuous foveated pixel coordinates u of display pixel (a, b) and
    the Jacobian du/d(a, b) (2x2), and the level of detail."""
    vp = view_params(view)
    u, J = np.empty(2), np.empty(4)
    lib().orc_unfov_coord(_p(vp, ctypes.c_double), width, height, a, b, _p(u, ctypes.c_double),
                          _p(J, ctypes.c_double))
    return u, J.reshape(2, 2), lib().orc_unfov_lod(_p(J, ctypes.c_double))


def mip_level(fov, k: int):
    """Level k of the oracle's MIP pyramid (float64 [h, w, 4]) and the number
    of levels."""
    f = _rgba01(fov)
    H, W = f.shape[:2]
    w, h = ctypes.c_int(0), ctypes.c_int(0)
    n = lib().orc_mip_level(_p(f, ctypes.c_double), W, H, k, None, ctypes.byref(w), ctypes.byref(h))
    out = np.empty((h.value, w.value, 4))
    lib().orc_mip_level(_p(f, ctypes.c_double), W, H, k, _p(out, ctypes.c_double), ctypes.byref(w),
                        ctypes.byref(h))
    return out, n


def to_rgba8(c) -> np.ndarray:
    """floor(clamp(c, 0, 1) * 255 + 1/2) as uint8."""
    return np.floor(np.clip(c, 0.0, 1.0) * 255.0 + 0.5).astype(np.uint8)


def unfov_filter_at(view, fov, width: int, height: int, a: int, b: int, i0: int, j0: int,
                    sigma: float) -> np.ndarray:
    """The reconstruction filter at display pixel (a, b) with its 5 x 5
    window centred on foveated pixel (i0, j0)."""
    vp = view_params(view)
    f = _rgba01(fov)
    out = np.empty(4)
    lib().orc_unfov_filter_at(_p(vp, ctypes.c_double), _p(f, ctypes.c_double), width, height, a, b, i0, j0, sigma,
                              _p(out, ctypes.c_double))
    return out
