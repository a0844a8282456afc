"""ctypes binding of libpr.so (include/pr.h).  Argument marshalling only:
every step of the hot path runs in the library's HIP kernels.  Importing
this module fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libpr.so')

PR_OK = 0
PR_ERR_INVALID = -1
PR_ERR_UNSUPPORTED = -2
PR_ERR_WORKSPACE = -3
PR_ERR_HIP = -4
PR_MAX_VIEWS = 64
PR_FLAG_COUNT = 1
PR_FLAG_PERSISTENT = 2
PR_STATIC_SCRATCH_BYTES = 256 << 20
PR_BOUND_ZENON = 0
PR_BOUND_ADAPTIVE = 1
PR_BOUND_HULL = 2
PR_BOUND_QUAD = 3
PR_FOV_EXACT, PR_FOV_QUAD, PR_FOV_SIMPLE, PR_FOV_RECURSIVE = 0, 1, 2, 3
PR_UNFOV_MIP = 0
PR_UNFOV_FILTER = 1

c_float_p = ctypes.POINTER(ctypes.c_float)
c_int32_p = ctypes.POINTER(ctypes.c_int32)


class PrMesh(ctypes.Structure):
    _fields_ = [('v0', ctypes.c_void_p), ('v1', ctypes.c_void_p), ('tri', ctypes.c_void_p),
                ('nv', ctypes.c_int32), ('nt', ctypes.c_int32)]


PR_PROFILE_MAX = 64


class PrProfile(ctypes.Structure):
    _fields_ = [('n_c', ctypes.c_int32), ('n_l', ctypes.c_int32), ('p_c', ctypes.c_float * PR_PROFILE_MAX),
                ('p_l', ctypes.c_float * PR_PROFILE_MAX)]


class PrView(ctypes.Structure):
    _fields_ = [('width', ctypes.c_int32), ('height', ctypes.c_int32), ('mesh', ctypes.c_int32),
                ('reserved', ctypes.c_int32), ('pose0', ctypes.c_float * 6), ('pose1', ctypes.c_float * 6),
                ('fx', ctypes.c_float), ('fy', ctypes.c_float), ('cx', ctypes.c_float), ('cy', ctypes.c_float),
                ('znear', ctypes.c_float), ('fovea', ctypes.c_float * 2), ('alpha', ctypes.c_float),
                ('roll_dir', ctypes.c_float * 2), ('profile', ctypes.POINTER(PrProfile))]


class PrLight(ctypes.Structure):
    _fields_ = [('dir_world', ctypes.c_float * 3), ('ambient', ctypes.c_float), ('specular', ctypes.c_float),
                ('shininess', ctypes.c_float)]


class PrTuning(ctypes.Structure):
    _fields_ = [('tile', ctypes.c_int32), ('bin_capacity', ctypes.c_int32), ('flags', ctypes.c_int32),
                ('bound', ctypes.c_int32), ('fov_bound', ctypes.c_int32)]


class PrDisplay(ctypes.Structure):
    _fields_ = [('width', ctypes.c_int32), ('height', ctypes.c_int32), ('mode', ctypes.c_int32),
                ('sigma', ctypes.c_float)]


class PrStatus(ctypes.Structure):
    _fields_ = [('overflow', ctypes.c_int32), ('nonfinite', ctypes.c_int32), ('pairs_required', ctypes.c_int64),
                ('pairs_total', ctypes.c_int64), ('tests', ctypes.c_int64), ('hits', ctypes.c_int64)]


class PrError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f'{fn} failed: {code} ({lib().pr_status_string(code).decode()})')
        self.code = code


# name -> (restype, argtypes); every symbol include/pr.h declares
_MP, _VP, _TP = ctypes.POINTER(PrMesh), ctypes.POINTER(PrView), ctypes.POINTER(PrTuning)
_PP = ctypes.POINTER(ctypes.c_void_p)
_FRAME = [_MP, ctypes.c_int, _VP, ctypes.c_int, _TP, ctypes.c_void_p, ctypes.c_size_t]
SIGNATURES = {
    'pr_workspace_size': (ctypes.c_int, [_MP, ctypes.c_int, _VP, ctypes.c_int, _TP, ctypes.POINTER(ctypes.c_size_t)]),
    'pr_bound': (ctypes.c_int, _FRAME + [ctypes.c_void_p]),
    'pr_bin': (ctypes.c_int, _FRAME + [ctypes.c_void_p]),
    'pr_raycast': (ctypes.c_int, _FRAME + [_PP, _PP, ctypes.c_void_p]),
    'pr_shade': (ctypes.c_int, _FRAME + [_PP, ctypes.POINTER(PrLight), _PP, _PP, _PP, ctypes.c_void_p]),
    'pr_raycast_shade': (ctypes.c_int, _FRAME + [_PP, _PP, ctypes.POINTER(PrLight), _PP, _PP, _PP, ctypes.c_void_p]),
    'pr_gbuffer': (ctypes.c_int, _FRAME + [_PP, _PP, _PP, _PP, ctypes.c_void_p]),
    'pr_backward': (ctypes.c_int, _FRAME + [_PP, ctypes.POINTER(PrLight), _PP, _PP, _PP, _PP, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    'pr_frame_static': (ctypes.c_int, _FRAME[:5] + [_PP, _PP, ctypes.POINTER(PrLight), _PP, _PP, _PP, ctypes.c_void_p]),
    'pr_unfoveate_workspace_size': (ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(PrDisplay),
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    'pr_unfoveate': (ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(PrDisplay), _PP, _PP, ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_void_p]),
    'pr_status_read': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(PrStatus), ctypes.c_void_p]),
    'pr_status_string': (ctypes.c_char_p, [ctypes.c_int]),
    'pr_debug_tile_lists': (ctypes.c_int, _FRAME[:5] + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, c_int32_p,
                                                         c_int32_p, ctypes.c_int64, c_int32_p,
                                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    'pr_batch_create': (ctypes.c_int, [_MP, ctypes.c_int, _VP, ctypes.c_int, _TP, ctypes.POINTER(PrLight), _PP, _PP,
                                       _PP, _PP, _PP, ctypes.POINTER(ctypes.c_void_p)]),
    'pr_batch_launch': (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    'pr_batch_info': (ctypes.c_int, [ctypes.c_void_p, _TP, ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_double)]),
    'pr_batch_status': (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PrStatus), ctypes.c_void_p]),
    'pr_batch_destroy': (ctypes.c_int, [ctypes.c_void_p]),
    'pr_host_time_interval': (ctypes.c_int, [_MP, ctypes.c_int32, _VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    'pr_host_tile_rect': (ctypes.c_int, [_MP, ctypes.c_int32, _VP, ctypes.c_int32, ctypes.c_int32, c_int32_p]),
    'pr_host_tile_test_fov': (ctypes.c_int, [_MP, ctypes.c_int32, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.c_int32]),
    'pr_host_tile_test': (ctypes.c_int, [_MP, ctypes.c_int32, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32]),
}

_lib = None


def lib():
    """The loaded libpr.so.  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f'{LIB_PATH} is not built; run `python -m paper_1806_05385_amd.build` '
                              '(or __graft_entry__.build()) first')
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(fn_name: str, code: int):
    if code != PR_OK:
        raise PrError(fn_name, code)


def make_view(v, mesh_index: int = None) -> PrView:
    """PrView from any object with scenegen.View's attributes."""
    pv = PrView()
    pv.width, pv.height = int(v.width), int(v.height)
    pv.mesh = int(v.mesh if mesh_index is None else mesh_index)
    pv.reserved = 0
    for k in range(6):
        pv.pose0[k] = float(v.pose0[k])
        pv.pose1[k] = float(v.pose1[k])
    pv.fx, pv.fy, pv.cx, pv.cy, pv.znear = float(v.fx), float(v.fy), float(v.cx), float(v.cy), float(v.znear)
    pv.fovea[0], pv.fovea[1] = float(v.fovea[0]), float(v.fovea[1])
    pv.alpha = float(v.alpha)
    pv.roll_dir[0], pv.roll_dir[1] = float(v.roll_dir[0]), float(v.roll_dir[1])
    pc, pl = getattr(v, 'profile_c', None), getattr(v, 'profile_l', None)
    if pc is not None or pl is not None:
        prof = PrProfile()
        for arr, n_name, field in ((pc, 'n_c', 'p_c'), (pl, 'n_l', 'p_l')):
            if arr is None:
                continue
            a = [float(x) for x in arr]
            if len(a) > PR_PROFILE_MAX:
                raise ValueError(f'profile: at most {PR_PROFILE_MAX} samples')
            setattr(prof, n_name, len(a))
            dst = getattr(prof, field)
            for k, x in enumerate(a):
                dst[k] = x
        # the pointer keeps prof alive as long as pv (or an array built from pv) lives
        pv.profile = ctypes.pointer(prof)
    return pv


def make_views(views, mesh_index: int = None):
    """ctypes array of PrView for a list of views; the profiles the entries
    point to stay alive with the array."""
    pvs = [make_view(v, mesh_index) for v in views]
    arr = (PrView * max(1, len(pvs)))(*pvs)
    arr._keep = pvs
    return arr


def make_light(direction, ambient: float, specular: float = 0.0, shininess: float = 1.0) -> PrLight:
    pl = PrLight()
    for k in range(3):
        pl.dir_world[k] = float(direction[k])
    pl.ambient = float(ambient)
    pl.specular = float(specular)
    pl.shininess = float(shininess)
    return pl


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * max(1, len(ptrs)))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr


def host_mesh(v0, v1, tri) -> PrMesh:
    """PrMesh over HOST numpy arrays (for the pr_host_* test hooks)."""
    m = PrMesh()
    m.v0, m.v1, m.tri = v0.ctypes.data, v1.ctypes.data, tri.ctypes.data
    m.nv, m.nt = int(v0.shape[0]), int(tri.shape[0])
    return m
