"""C ABI checks that need no GPU: the library loads, exports every function
include/pr.h declares, and rejects bad arguments before launching anything."""
import ctypes
import os
import re

import numpy as np
import pytest

import scenegen
from paper_1806_05385_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, 'include', 'pr.h')).read()
    src = re.sub(r'/\*.*?\*/', '', src, flags=re.S)
    return sorted(set(re.findall(r'\b(pr_\w+)\s*\(', src)))


def test_every_declared_symbol_is_exported_and_bound():
    L = B.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
        assert n in B.SIGNATURES, f'{n} not bound in binding.SIGNATURES'
    assert set(B.SIGNATURES) == set(names)


def test_status_strings():
    L = B.lib()
    for code in (B.PR_OK, B.PR_ERR_INVALID, B.PR_ERR_UNSUPPORTED, B.PR_ERR_WORKSPACE, B.PR_ERR_HIP, -99):
        assert L.pr_status_string(code)


def _frame(tile=16, cap=1000, **view_kw):
    sc = scenegen.make_tiny(n_tris=10, size=32)
    m = sc.meshes[0]
    mesh = B.host_mesh(m.v0, m.v1, m.tri)   # pointers are not dereferenced on these paths
    meshes = (B.PrMesh * 1)(mesh)
    v = sc.views[0]
    for k, val in view_kw.items():
        setattr(v, k, val)
    views = B.make_views([v])
    tu = B.PrTuning(tile, cap, 0, 0)
    return meshes, views, tu, sc


def test_workspace_size_and_argument_checks():
    L = B.lib()
    meshes, views, tu, sc = _frame()
    size = ctypes.c_size_t(0)
    assert L.pr_workspace_size(meshes, 1, views, 1, ctypes.byref(tu), ctypes.byref(size)) == B.PR_OK
    assert size.value > 10 * 128
    big = ctypes.c_size_t(0)
    tu2 = B.PrTuning(16, 100000, 0, 0)
    assert L.pr_workspace_size(meshes, 1, views, 1, ctypes.byref(tu2), ctypes.byref(big)) == B.PR_OK
    assert big.value >= size.value + (100000 - 1000) * 16 - 1024   # 12-byte pair + 4-byte list entry
    bad = [
        dict(width=0), dict(height=20000), dict(mesh=3), dict(alpha=0.5), dict(znear=0.0), dict(fx=0.0),
        dict(fovea=(1.5, 0.0)), dict(alpha=float('nan')),
    ]
    for kw in bad:
        m, v, t, _ = _frame(**kw)
        assert L.pr_workspace_size(m, 1, v, 1, ctypes.byref(t), ctypes.byref(size)) == B.PR_ERR_INVALID, kw
    m, v, t, _ = _frame(tile=12)
    assert L.pr_workspace_size(m, 1, v, 1, ctypes.byref(t), ctypes.byref(size)) == B.PR_ERR_UNSUPPORTED
    m, v, t, _ = _frame(cap=0)
    assert L.pr_workspace_size(m, 1, v, 1, ctypes.byref(t), ctypes.byref(size)) == B.PR_ERR_INVALID
    assert L.pr_workspace_size(None, 1, views, 1, ctypes.byref(tu), ctypes.byref(size)) == B.PR_ERR_INVALID
    assert L.pr_workspace_size(meshes, 1, views, 0, ctypes.byref(tu), ctypes.byref(size)) == B.PR_ERR_INVALID
    assert L.pr_workspace_size(meshes, 1, views, 65, ctypes.byref(tu), ctypes.byref(size)) == B.PR_ERR_INVALID
    nullmesh = (B.PrMesh * 1)(B.PrMesh(None, None, None, 5, 5))
    assert L.pr_workspace_size(nullmesh, 1, views, 1, ctypes.byref(tu), ctypes.byref(size)) == B.PR_ERR_INVALID


def test_profile_checks():
    """A tabulated p_c / p_l needs 2..64 finite samples from 0, strictly
    increasing, and p_c(s_k) >= s_k."""
    L = B.lib()
    size = ctypes.c_size_t(0)
    good_c, good_l = scenegen.foveal_table(9, 2.0), scenegen.barrel_table(9, 0.2)
    for kw in (dict(profile_c=good_c), dict(profile_l=good_l), dict(profile_c=good_c, profile_l=good_l)):
        m, v, t, _ = _frame(**kw)
        assert L.pr_workspace_size(m, 1, v, 1, ctypes.byref(t), ctypes.byref(size)) == B.PR_OK, kw
    bad = [
        dict(profile_c=np.array([0.0], np.float32)),                      # one sample
        dict(profile_c=np.array([0.1, 0.5, 1.0], np.float32)),             # not from 0
        dict(profile_c=np.array([0.0, 0.6, 0.6, 1.0], np.float32)),        # not strictly increasing
        dict(profile_c=np.array([0.0, 0.2, 1.0], np.float32)),             # p_c(1/2) < 1/2
        dict(profile_c=np.array([0.0, float('nan'), 1.0], np.float32)),
        dict(profile_l=np.array([0.0, -0.5], np.float32)),
        dict(profile_l=np.array([0.0, float('inf')], np.float32)),
    ]
    for kw in bad:
        m, v, t, _ = _frame(**kw)
        assert L.pr_workspace_size(m, 1, v, 1, ctypes.byref(t), ctypes.byref(size)) == B.PR_ERR_INVALID, kw
    m, v, t, _ = _frame(profile_c=good_c)
    for n in (1, 65, -1):   # sample counts out of range (the binding refuses to build them)
        v[0].profile.contents.n_c = n
        assert L.pr_workspace_size(m, 1, v, 1, ctypes.byref(t), ctypes.byref(size)) == B.PR_ERR_INVALID, n


def test_triangle_count_limit():
    """A view's records (176 B each) are addressed with 32-bit byte offsets:
    the largest accepted mesh has 24,403,223 triangles (records < 4 GiB); one
    more is rejected before anything is allocated or launched."""
    L = B.lib()
    _, views, tu, _ = _frame()
    size = ctypes.c_size_t(0)
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced by pr_workspace_size
    for nt, want in ((24_403_223, B.PR_OK), (24_403_224, B.PR_ERR_INVALID), (1 << 28, B.PR_ERR_INVALID)):
        mesh = (B.PrMesh * 1)(B.PrMesh(fake, fake, fake, 100, nt))
        assert L.pr_workspace_size(mesh, 1, views, 1, ctypes.byref(tu), ctypes.byref(size)) == want, nt
    mesh = (B.PrMesh * 1)(B.PrMesh(fake, fake, fake, 100, 24_403_223))
    L.pr_workspace_size(mesh, 1, views, 1, ctypes.byref(tu), ctypes.byref(size))
    assert size.value > 24_403_223 * (96 + 64)   # static view: 96-byte records, 64-byte bounds


def test_calls_reject_bad_workspace_before_launch():
    """Workspace and pointer checks run on the host before any HIP call, so
    they answer the same with or without a GPU."""
    L = B.lib()
    meshes, views, tu, sc = _frame()
    size = ctypes.c_size_t(0)
    L.pr_workspace_size(meshes, 1, views, 1, ctypes.byref(tu), ctypes.byref(size))
    args = (meshes, 1, views, 1, ctypes.byref(tu))
    assert L.pr_bound(*args, None, size.value, None) == B.PR_ERR_WORKSPACE
    assert L.pr_bound(*args, ctypes.c_void_p(256 * 1000 + 8), size.value, None) == B.PR_ERR_WORKSPACE
    assert L.pr_bound(*args, ctypes.c_void_p(256 * 1000), size.value - 1, None) == B.PR_ERR_WORKSPACE
    assert L.pr_bin(*args, None, size.value, None) == B.PR_ERR_WORKSPACE
    assert L.pr_raycast(*args, ctypes.c_void_p(256 * 1000), size.value, None, None, None) == B.PR_ERR_INVALID
    assert L.pr_shade(*args, ctypes.c_void_p(256 * 1000), size.value, None, None, None, None, None,
                      None) == B.PR_ERR_INVALID
    st = B.PrStatus()
    assert L.pr_status_read(None, 1024, ctypes.byref(st), None) == B.PR_ERR_INVALID


def test_light_and_gbuffer_arguments_checked_before_launch():
    """A highlight needs k_s >= 0 and exponent m >= 1 (finite): pr_shade,
    pr_raycast_shade and pr_backward reject other lights on the host;
    pr_gbuffer checks its ids and workspace before any HIP call."""
    L = B.lib()
    meshes, views, tu, sc = _frame()
    size = ctypes.c_size_t(0)
    L.pr_workspace_size(meshes, 1, views, 1, ctypes.byref(tu), ctypes.byref(size))
    args = (meshes, 1, views, 1, ctypes.byref(tu), ctypes.c_void_p(256 * 1000), size.value)
    fake = B.ptr_array([1 << 20])
    for ks, m in ((-0.1, 8.0), (0.5, 0.5), (float('nan'), 8.0), (0.5, float('inf'))):
        bad = B.make_light(sc.light_dir, sc.ambient, ks, m)
        assert L.pr_shade(*args, fake, ctypes.byref(bad), fake, fake, None, None) == B.PR_ERR_INVALID
        assert L.pr_raycast_shade(*args, fake, fake, ctypes.byref(bad), fake, fake, None, None) == B.PR_ERR_INVALID
        assert L.pr_backward(*args, fake, ctypes.byref(bad), fake, fake, fake, fake, ctypes.c_void_p(1 << 20),
                             ctypes.c_void_p(1 << 20), None) == B.PR_ERR_INVALID
    assert L.pr_gbuffer(*args, None, fake, fake, fake, None) == B.PR_ERR_INVALID
    assert L.pr_gbuffer(*args, B.ptr_array([0]), fake, fake, fake, None) == B.PR_ERR_INVALID
    assert L.pr_gbuffer(*args[:5], None, size.value, fake, fake, None, None, None) == B.PR_ERR_WORKSPACE


def huge_candidate_scene(n_tris: int = 520):
    """A 16384 x 16384 view at tile 8 (2048 x 2048 tiles) and n_tris
    triangles that each cover the whole display: every triangle's tile
    rectangle is the whole grid, 4,194,304 candidates each."""
    import numpy as np
    import scenegen
    base = np.array([[-40.0, -40.0, 2.0], [40.0, -40.0, 2.0], [0.0, 40.0, 2.0]], np.float32)
    v = np.concatenate([base + np.float32([0.0, 0.0, 0.001 * k]) for k in range(n_tris)])
    tri = np.arange(3 * n_tris, dtype=np.int32).reshape(n_tris, 3)
    mesh = scenegen.Mesh(v, v.copy(), tri, np.full_like(v, 0.5))
    view = scenegen.View(16384, 16384, np.zeros(6, np.float32), np.zeros(6, np.float32), alpha=1.0,
                         roll_dir=(0.0, 0.0))
    return scenegen.Scene('huge_candidates', [mesh], [view])


def test_candidate_count_beyond_int32():
    """The candidate count of huge_candidate_scene exceeds 2^31 - 1 (the
    binning's slot offsets are 64-bit; the GPU test checks the frame reports
    exactly this count as an overflow): each triangle's tile rectangle,
    from the host build of the bound, is the full 2048 x 2048 grid."""
    sc = huge_candidate_scene()
    mesh, view = sc.meshes[0], sc.views[0]
    L = B.lib()
    hm = B.host_mesh(mesh.v0, mesh.v1, mesh.tri)
    pv = B.make_view(view)
    rect = (ctypes.c_int32 * 4)()
    total = 0
    for f in range(mesh.nt):
        assert L.pr_host_tile_rect(ctypes.byref(hm), f, ctypes.byref(pv), 0, 8, rect) == 1
        assert tuple(rect) == (0, 0, 2047, 2047)
        total += (rect[2] - rect[0] + 1) * (rect[3] - rect[1] + 1)
    assert total == 520 * 2048 * 2048 == 2_181_038_080 > 2 ** 31 - 1


def test_unfoveate_arguments_checked_before_launch():
    """pr_unfoveate's sizes and checks are host-side: bad displays, views or
    workspaces are rejected before any HIP call; the workspace holds the MIP
    views' pyramids (about a third of a float4 per foveated pixel) and nothing
    for the filter form."""
    L = B.lib()
    v = scenegen.View(64, 48, np.zeros(6, np.float32), np.zeros(6, np.float32), fovea=(0.1, 0.0), alpha=2.0)
    views = (B.PrView * 1)(B.make_view(v))
    size = ctypes.c_size_t(0)

    def ws_size(w, h, mode, sigma, vv=views):
        d = (B.PrDisplay * 1)(B.PrDisplay(w, h, mode, sigma))
        return L.pr_unfoveate_workspace_size(vv, 1, d, ctypes.byref(size)), size.value

    rc, mip = ws_size(80, 60, B.PR_UNFOV_MIP, 0.0)
    assert rc == B.PR_OK and mip >= 16 * (32 * 24 + 16 * 12 + 8 * 6 + 4 * 3 + 2 * 2 + 1)
    rc, filt = ws_size(80, 60, B.PR_UNFOV_FILTER, 0.5)
    assert rc == B.PR_OK and filt < mip
    for bad in [(0, 60, B.PR_UNFOV_MIP, 0.5), (80, 16385, B.PR_UNFOV_MIP, 0.5), (80, 60, 7, 0.5),
                (80, 60, B.PR_UNFOV_FILTER, 0.0), (80, 60, B.PR_UNFOV_FILTER, float('nan'))]:
        assert ws_size(*bad)[0] == B.PR_ERR_INVALID, bad
    v.alpha = 0.5
    assert ws_size(80, 60, B.PR_UNFOV_MIP, 0.5, (B.PrView * 1)(B.make_view(v)))[0] == B.PR_ERR_INVALID
    d = (B.PrDisplay * 1)(B.PrDisplay(80, 60, B.PR_UNFOV_MIP, 0.5))
    arr = B.ptr_array([1 << 20])
    assert L.pr_unfoveate(views, 1, d, arr, arr, None, mip, None) == B.PR_ERR_WORKSPACE
    assert L.pr_unfoveate(views, 1, d, arr, arr, ctypes.c_void_p(256 * 1000), mip - 1, None) == B.PR_ERR_WORKSPACE
    assert L.pr_unfoveate(views, 1, d, None, arr, ctypes.c_void_p(256 * 1000), mip, None) == B.PR_ERR_INVALID
    assert L.pr_unfoveate(views, 0, d, arr, arr, ctypes.c_void_p(256 * 1000), mip, None) == B.PR_ERR_INVALID


def test_static_frame_rejects_large_frames_before_launch():
    """pr_frame_static checks its sizes on the host: a frame whose workspace
    exceeds PR_STATIC_SCRATCH_BYTES returns PR_ERR_WORKSPACE before any HIP
    call (so the answer is the same without a GPU)."""
    L = B.lib()
    meshes, views, _, sc = _frame(cap=1 << 24)
    tu = B.PrTuning(16, 1 << 24, B.PR_FLAG_PERSISTENT, 0)
    size = ctypes.c_size_t(0)
    assert L.pr_workspace_size(meshes, 1, views, 1, ctypes.byref(tu), ctypes.byref(size)) == B.PR_OK
    assert size.value > B.PR_STATIC_SCRATCH_BYTES
    fake = B.ptr_array([1 << 20])
    light = B.make_light(sc.light_dir, sc.ambient)
    assert L.pr_frame_static(meshes, 1, views, 1, ctypes.byref(tu), fake, fake, ctypes.byref(light), fake, None,
                             None, None) == B.PR_ERR_WORKSPACE
