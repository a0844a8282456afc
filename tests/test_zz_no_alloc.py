"""pr_frame_static, the allocation-free frame (bound, bin and ray cast with
fused shading on the library's static device scratch array), against the
same frame through pr_bound / pr_bin / pr_raycast_shade with a caller
workspace: bitwise equal ids, depths and RGBA8 on two calls in a row, the
second with a smaller input; a frame larger than the array is rejected
before anything runs."""
import ctypes

import numpy as np
import pytest

import scenegen
from paper_1806_05385_amd import binding as B

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail('no GPU visible')
    return torch


def _frames(sc, tile=16):
    """(static, reference) outputs of one scene, each a list per view of
    dicts of numpy arrays."""
    torch = _torch()
    from paper_1806_05385_amd.render import Renderer
    L = B.lib()
    r = Renderer(sc.meshes, sc.views, tile=tile, light=sc.light_dir, ambient=sc.ambient)
    r.frame(check=True, rgb32=False)          # sizes the capacity (allocating path)
    ref = [{k: o[k].cpu().numpy().copy() for k in ('id', 'depth', 'rgba8')} for o in r.outputs]
    outs = [dict(id=torch.full((v.height, v.width), -7, dtype=torch.int32, device='cuda'),
                 depth=torch.full((v.height, v.width), -1.0, dtype=torch.float32, device='cuda'),
                 rgba8=torch.full((v.height, v.width, 4), 3, dtype=torch.uint8, device='cuda')) for v in sc.views]
    torch.cuda.synchronize()
    rc = L.pr_frame_static(r.c_meshes, len(r.meshes), r.c_views, len(r.views), ctypes.byref(r.tuning),
                           B.ptr_array([o['id'].data_ptr() for o in outs]),
                           B.ptr_array([o['depth'].data_ptr() for o in outs]), ctypes.byref(r.light),
                           B.ptr_array([m.albedo.data_ptr() for m in r.meshes]),
                           B.ptr_array([o['rgba8'].data_ptr() for o in outs]), None,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    B.check('pr_frame_static', rc)
    torch.cuda.synchronize()
    got = [{k: o[k].cpu().numpy() for k in ('id', 'depth', 'rgba8')} for o in outs]
    return got, ref


def test_static_frame_equals_workspace_frame_twice():
    big = scenegen.make_moving_soup(seed=34, n_tris=1500, width=203, height=171, alpha=2.0, roll=(1.0, 0.0),
                                    yaw_deg_s=1500.0, obj_speed=10.0, side=(0.03, 0.5))
    small = scenegen.make_moving_soup(seed=7, n_tris=400, width=96, height=80, alpha=2.0, roll=(1.0, 0.0),
                                      yaw_deg_s=1000.0, obj_speed=10.0, side=(0.05, 0.5))
    for sc in (big, small):
        got, ref = _frames(sc)
        assert (ref[0]['id'] >= 0).sum() > 1000
        for g, f in zip(got, ref):
            for k in ('id', 'depth', 'rgba8'):
                assert np.array_equal(g[k].view(np.uint8), f[k].view(np.uint8)), (sc.name, k)


def test_static_frame_rejects_frames_beyond_the_array():
    """A view whose workspace exceeds PR_STATIC_SCRATCH_BYTES returns
    PR_ERR_WORKSPACE and leaves the outputs untouched."""
    torch = _torch()
    L = B.lib()
    sc = scenegen.make_tiny(n_tris=300, size=64)
    m = sc.meshes[0]
    from paper_1806_05385_amd.render import DeviceMesh
    dm = DeviceMesh.from_numpy(m)
    meshes = (B.PrMesh * 1)(dm.pr())
    views = (B.PrView * 1)(B.make_view(sc.views[0]))
    tu = B.PrTuning(16, 1 << 24, B.PR_FLAG_PERSISTENT, 0)      # 16M candidate slots: 256 MiB of pairs
    size = ctypes.c_size_t(0)
    B.check('pr_workspace_size', L.pr_workspace_size(meshes, 1, views, 1, ctypes.byref(tu), ctypes.byref(size)))
    assert size.value > B.PR_STATIC_SCRATCH_BYTES
    ids = torch.full((64, 64), -7, dtype=torch.int32, device='cuda')
    dep = torch.zeros((64, 64), dtype=torch.float32, device='cuda')
    rc = L.pr_frame_static(meshes, 1, views, 1, ctypes.byref(tu), B.ptr_array([ids.data_ptr()]),
                           B.ptr_array([dep.data_ptr()]), ctypes.byref(B.make_light(sc.light_dir, sc.ambient)),
                           B.ptr_array([dm.albedo.data_ptr()]), None, None,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == B.PR_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((ids == -7).all())
