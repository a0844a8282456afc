"""Torch front end of libpr: device buffers and streams come from PyTorch,
every computation runs in the library's kernels (include/pr.h)."""
from __future__ import annotations

import copy
import ctypes
from dataclasses import dataclass

import torch

from . import binding as B


@dataclass
class DeviceMesh:
    v0: torch.Tensor       # float32 [V, 3] (cuda)
    v1: torch.Tensor       # float32 [V, 3]
    tri: torch.Tensor      # int32 [T, 3]
    albedo: torch.Tensor   # float32 [V, 3]

    @staticmethod
    def from_numpy(mesh, device='cuda') -> 'DeviceMesh':
        def t(a, dt):
            return torch.as_tensor(a, dtype=dt).contiguous().to(device)
        return DeviceMesh(t(mesh.v0, torch.float32), t(mesh.v1, torch.float32), t(mesh.tri, torch.int32),
                          t(mesh.albedo, torch.float32))

    def pr(self) -> B.PrMesh:
        m = B.PrMesh()
        for name in ('v0', 'v1', 'tri'):
            x = getattr(self, name)
            assert x.is_cuda and x.is_contiguous(), name
        m.v0, m.v1, m.tri = self.v0.data_ptr(), self.v1.data_ptr(), self.tri.data_ptr()
        m.nv, m.nt = int(self.v0.shape[0]), int(self.tri.shape[0])
        return m


def _stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


class Renderer:
    """One frame pipeline over a fixed set of meshes and views.

    ``frame()`` enqueues pr_bound, pr_bin and pr_raycast_shade (pr_raycast
    when ``shade=False``) on the current torch stream and returns the output
    tensors.
    The workspace is a torch uint8 tensor sized by pr_workspace_size; on a
    tile-list overflow (checked only when ``check=True``) the capacity is
    raised to what the device reported and the frame is run again."""

    def __init__(self, meshes, views, tile: int = 16, bin_capacity: int = 0, light=None, ambient: float = 0.1,
                 flags: int = B.PR_FLAG_PERSISTENT, device='cuda', bound: int = B.PR_BOUND_ZENON,
                 specular: float = 0.0, shininess: float = 1.0, fov_bound: int = B.PR_FOV_EXACT):
        self.L = B.lib()
        self.bound_mode = int(bound)
        self.fov_bound = int(fov_bound)
        self.device = torch.device(device)
        self.meshes = [m if isinstance(m, DeviceMesh) else DeviceMesh.from_numpy(m, device) for m in meshes]
        self.views = [copy.copy(v) for v in views]
        self.tile = tile
        self.flags = flags
        if not bin_capacity:
            bin_capacity = max(1 << 16, 4 * sum(self.meshes[v.mesh].tri.shape[0] for v in self.views) // len(self.views))
        self.cap = int(bin_capacity)
        self.light = B.make_light(light if light is not None else (0.0, 0.0, -1.0), ambient, specular, shininess)
        self._prepare()
        self.outputs = []
        for v in self.views:
            h, w = v.height, v.width
            self.outputs.append(dict(
                id=torch.empty((h, w), dtype=torch.int32, device=self.device),
                depth=torch.empty((h, w), dtype=torch.float32, device=self.device),
                rgba8=torch.empty((h, w, 4), dtype=torch.uint8, device=self.device),
                rgb32=torch.empty((h, w, 3), dtype=torch.float32, device=self.device)))

    def _prepare(self):
        nm = len(self.meshes)
        self.c_meshes = (B.PrMesh * nm)(*[m.pr() for m in self.meshes])
        self.c_views = B.make_views(self.views)
        self.tuning = B.PrTuning(self.tile, self.cap, self.flags, self.bound_mode, self.fov_bound)
        size = ctypes.c_size_t(0)
        B.check('pr_workspace_size', self.L.pr_workspace_size(self.c_meshes, nm, self.c_views, len(self.views),
                                                              ctypes.byref(self.tuning), ctypes.byref(size)))
        self.ws_bytes = size.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255

    def _args(self):
        return (self.c_meshes, len(self.meshes), self.c_views, len(self.views), ctypes.byref(self.tuning),
                ctypes.c_void_p(self.ws_ptr), self.ws_bytes)

    def bound(self):
        B.check('pr_bound', self.L.pr_bound(*self._args(), ctypes.c_void_p(_stream_handle())))

    def bin(self):
        B.check('pr_bin', self.L.pr_bin(*self._args(), ctypes.c_void_p(_stream_handle())))

    def raycast(self):
        ids = B.ptr_array([o['id'].data_ptr() for o in self.outputs])
        deps = B.ptr_array([o['depth'].data_ptr() for o in self.outputs])
        B.check('pr_raycast', self.L.pr_raycast(*self._args(), ids, deps, ctypes.c_void_p(_stream_handle())))

    def shade(self, rgba8: bool = True, rgb32: bool = True, ids=None):
        idp = B.ptr_array([(ids[i] if ids is not None else o['id']).data_ptr() for i, o in enumerate(self.outputs)])
        alb = B.ptr_array([m.albedo.data_ptr() for m in self.meshes])
        o8 = B.ptr_array([o['rgba8'].data_ptr() for o in self.outputs]) if rgba8 else None
        o32 = B.ptr_array([o['rgb32'].data_ptr() for o in self.outputs]) if rgb32 else None
        B.check('pr_shade', self.L.pr_shade(*self._args(), idp, ctypes.byref(self.light), alb, o8, o32,
                                            ctypes.c_void_p(_stream_handle())))

    def gbuffer(self, ids=None):
        """pr_gbuffer of this frame's ids (or ``ids``): per view a dict of
        normal [H,W,3], bary [H,W,2] and density [H,W] float32 tensors."""
        idp = B.ptr_array([(ids[i] if ids is not None else o['id']).data_ptr() for i, o in enumerate(self.outputs)])
        out = [dict(normal=torch.empty((v.height, v.width, 3), dtype=torch.float32, device=self.device),
                    bary=torch.empty((v.height, v.width, 2), dtype=torch.float32, device=self.device),
                    density=torch.empty((v.height, v.width), dtype=torch.float32, device=self.device))
               for v in self.views]
        B.check('pr_gbuffer', self.L.pr_gbuffer(
            *self._args(), idp, B.ptr_array([g['normal'].data_ptr() for g in out]),
            B.ptr_array([g['bary'].data_ptr() for g in out]), B.ptr_array([g['density'].data_ptr() for g in out]),
            ctypes.c_void_p(_stream_handle())))
        return out

    def raycast_shade(self, rgba8: bool = True, rgb32: bool = True):
        """pr_raycast_shade: the ray cast with the shading of its ids fused in."""
        ids = B.ptr_array([o['id'].data_ptr() for o in self.outputs])
        deps = B.ptr_array([o['depth'].data_ptr() for o in self.outputs])
        alb = B.ptr_array([m.albedo.data_ptr() for m in self.meshes])
        o8 = B.ptr_array([o['rgba8'].data_ptr() for o in self.outputs]) if rgba8 else None
        o32 = B.ptr_array([o['rgb32'].data_ptr() for o in self.outputs]) if rgb32 else None
        B.check('pr_raycast_shade', self.L.pr_raycast_shade(*self._args(), ids, deps, ctypes.byref(self.light), alb,
                                                            o8, o32, ctypes.c_void_p(_stream_handle())))

    def backward(self, dl_drgb, ids=None):
        """pr_backward: dL/drgb per view (float32 [H,W,3] cuda) -> (dv0, dv1)
        per mesh ([V,3] cuda) and (dpose0, dpose1) [n_views, 6] cuda, with
        visibility fixed to ``ids`` (default: this frame's ids)."""
        nv = len(self.views)
        if ids is None:
            ids = [o['id'] for o in self.outputs]
        dl = [d.contiguous() for d in dl_drgb]
        for d, v in zip(dl, self.views):
            assert d.is_cuda and d.dtype == torch.float32 and tuple(d.shape) == (v.height, v.width, 3)
        dv0 = [torch.empty_like(m.v0) for m in self.meshes]
        dv1 = [torch.empty_like(m.v1) for m in self.meshes]
        dp0 = torch.empty((nv, 6), dtype=torch.float32, device=self.device)
        dp1 = torch.empty((nv, 6), dtype=torch.float32, device=self.device)
        B.check('pr_backward', self.L.pr_backward(
            *self._args(), B.ptr_array([i.data_ptr() for i in ids]), ctypes.byref(self.light),
            B.ptr_array([m.albedo.data_ptr() for m in self.meshes]), B.ptr_array([d.data_ptr() for d in dl]),
            B.ptr_array([x.data_ptr() for x in dv0]), B.ptr_array([x.data_ptr() for x in dv1]),
            ctypes.c_void_p(dp0.data_ptr()), ctypes.c_void_p(dp1.data_ptr()), ctypes.c_void_p(_stream_handle())))
        return dv0, dv1, dp0, dp1

    def set_geometry(self, mesh: int, v0=None, v1=None):
        """Point mesh ``mesh`` at new vertex tensors (float32 [V,3] cuda)."""
        m = self.meshes[mesh]
        if v0 is not None:
            m.v0 = v0.detach().contiguous()
        if v1 is not None:
            m.v1 = v1.detach().contiguous()
        self.c_meshes[mesh] = m.pr()

    def set_poses(self, view: int, pose0=None, pose1=None):
        """New world->view poses (6 floats: rotation vector, translation)."""
        pv = self.c_views[view]
        if pose0 is not None:
            self.views[view].pose0 = [float(x) for x in pose0]
            for k in range(6):
                pv.pose0[k] = float(pose0[k])
        if pose1 is not None:
            self.views[view].pose1 = [float(x) for x in pose1]
            for k in range(6):
                pv.pose1[k] = float(pose1[k])

    def status(self) -> B.PrStatus:
        st = B.PrStatus()
        B.check('pr_status_read', self.L.pr_status_read(ctypes.c_void_p(self.ws_ptr), self.ws_bytes,
                                                        ctypes.byref(st), ctypes.c_void_p(_stream_handle())))
        return st

    def frame(self, shade: bool = True, check: bool = True, rgb32: bool = True):
        for _ in range(4):
            self.bound()
            self.bin()
            if shade:
                self.raycast_shade(rgba8=True, rgb32=rgb32)
            else:
                self.raycast()
            if not check:
                break
            st = self.status()
            if not st.overflow:
                break
            self.cap = int(st.pairs_required * 1.25) + 1024
            self._prepare()
        return self.outputs

    def tile_lists(self, view: int):
        """(offsets [tiles+1], triangle [pairs], quadrant mask [pairs]) of one
        view's tile lists, copied to the host."""
        import numpy as np
        ntiles = ctypes.c_int32(0)
        npairs = ctypes.c_int64(0)
        a = self._args()
        B.check('pr_debug_tile_lists', self.L.pr_debug_tile_lists(*a[:5], *a[5:], view, None, None, 0,
                                                                  ctypes.byref(ntiles), ctypes.byref(npairs),
                                                                  ctypes.c_void_p(_stream_handle())))
        off = np.empty(ntiles.value + 1, np.int32)
        lst = np.empty(max(1, npairs.value), np.int32)
        B.check('pr_debug_tile_lists', self.L.pr_debug_tile_lists(
            *a[:5], *a[5:], view, off.ctypes.data_as(B.c_int32_p), lst.ctypes.data_as(B.c_int32_p),
            lst.shape[0], ctypes.byref(ntiles), ctypes.byref(npairs), ctypes.c_void_p(_stream_handle())))
        ent = lst[:npairs.value].view(np.uint32)
        return off, (ent & 0x0FFFFFFF).astype(np.int32), (ent >> 28).astype(np.int32)


class Batch:
    """Batched form (pr_batch_*): all views rendered as one frame, captured
    once into a hipGraph; ``launch()`` replays it on the current stream.
    tile = 0 / bin_capacity = 0 let the library's autotuner choose."""

    def __init__(self, meshes, views, tile: int = 0, bin_capacity: int = 0, light=None, ambient: float = 0.1,
                 rgba8: bool = True, rgb32: bool = False, device='cuda'):
        self.L = B.lib()
        self.device = torch.device(device)
        self.meshes = [m if isinstance(m, DeviceMesh) else DeviceMesh.from_numpy(m, device) for m in meshes]
        self.views = [copy.copy(v) for v in views]
        self.outputs = []
        for v in self.views:
            h, w = v.height, v.width
            o = dict(id=torch.empty((h, w), dtype=torch.int32, device=self.device),
                     depth=torch.empty((h, w), dtype=torch.float32, device=self.device))
            if rgba8:
                o['rgba8'] = torch.empty((h, w, 4), dtype=torch.uint8, device=self.device)
            if rgb32:
                o['rgb32'] = torch.empty((h, w, 3), dtype=torch.float32, device=self.device)
            self.outputs.append(o)
        nm = len(self.meshes)
        self.c_meshes = (B.PrMesh * nm)(*[m.pr() for m in self.meshes])
        self.c_views = B.make_views(self.views)
        self.light = B.make_light(light if light is not None else (0.0, 0.0, -1.0), ambient)
        tu = B.PrTuning(tile, bin_capacity, 0, 0)
        self.ptr = ctypes.c_void_p(0)

        def arr(key):
            if key not in self.outputs[0]:
                return None
            return B.ptr_array([o[key].data_ptr() for o in self.outputs])
        torch.cuda.synchronize()
        B.check('pr_batch_create', self.L.pr_batch_create(
            self.c_meshes, nm, self.c_views, len(self.views), ctypes.byref(tu), ctypes.byref(self.light),
            B.ptr_array([m.albedo.data_ptr() for m in self.meshes]), arr('id'), arr('depth'), arr('rgba8'),
            arr('rgb32'), ctypes.byref(self.ptr)))

    def launch(self):
        B.check('pr_batch_launch', self.L.pr_batch_launch(self.ptr, ctypes.c_void_p(_stream_handle())))
        return self.outputs

    def info(self):
        tu = B.PrTuning()
        size = ctypes.c_size_t(0)
        ms = (ctypes.c_double * 3)()
        B.check('pr_batch_info', self.L.pr_batch_info(self.ptr, ctypes.byref(tu), ctypes.byref(size), ms))
        return dict(tile=tu.tile, bin_capacity=tu.bin_capacity, flags=tu.flags, ws_bytes=size.value,
                    trial_ms={8: ms[0], 16: ms[1], 32: ms[2]})

    def status(self) -> B.PrStatus:
        st = B.PrStatus()
        B.check('pr_batch_status', self.L.pr_batch_status(self.ptr, ctypes.byref(st),
                                                          ctypes.c_void_p(_stream_handle())))
        return st

    def close(self):
        if self.ptr:
            self.L.pr_batch_destroy(self.ptr)
            self.ptr = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Display:
    """Display unfoveation (pr_unfoveate): each view's foveated RGBA8 image
    resampled to its display's regular grid.  ``sizes``: display (width,
    height) per view (default: the view's own size); ``mode``:
    B.PR_UNFOV_MIP or B.PR_UNFOV_FILTER (Gaussian ``sigma`` in display
    pixels)."""

    def __init__(self, views, sizes=None, mode: int = B.PR_UNFOV_MIP, sigma: float = 0.5, device='cuda'):
        self.L = B.lib()
        self.device = torch.device(device)
        self.views = [copy.copy(v) for v in views]
        n = len(self.views)
        sizes = sizes or [(v.width, v.height) for v in self.views]
        self.c_views = B.make_views(self.views, 0)
        self.c_disp = (B.PrDisplay * n)(*[B.PrDisplay(int(w), int(h), int(mode), float(sigma)) for w, h in sizes])
        size = ctypes.c_size_t(0)
        B.check('pr_unfoveate_workspace_size', self.L.pr_unfoveate_workspace_size(self.c_views, n, self.c_disp,
                                                                                  ctypes.byref(size)))
        self.ws_bytes = size.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255
        self.outputs = [torch.empty((h, w, 4), dtype=torch.uint8, device=self.device) for w, h in sizes]

    def run(self, fov_rgba8):
        """fov_rgba8: per view uint8 [H, W, 4] cuda tensors (contiguous)."""
        for f, v in zip(fov_rgba8, self.views):
            assert f.is_cuda and f.dtype == torch.uint8 and f.is_contiguous() and tuple(f.shape) == (v.height,
                                                                                                    v.width, 4)
        B.check('pr_unfoveate', self.L.pr_unfoveate(
            self.c_views, len(self.views), self.c_disp, B.ptr_array([f.data_ptr() for f in fov_rgba8]),
            B.ptr_array([o.data_ptr() for o in self.outputs]), ctypes.c_void_p(self.ws_ptr), self.ws_bytes,
            ctypes.c_void_p(_stream_handle())))
        return self.outputs


def render_scene(scene, tile: int = 16, shade: bool = True, flags: int = B.PR_FLAG_PERSISTENT, device='cuda'):
    """Render a scenegen.Scene; returns (renderer, outputs)."""
    r = Renderer(scene.meshes, scene.views, tile=tile, light=scene.light_dir, ambient=scene.ambient, flags=flags,
                 device=device)
    out = r.frame(shade=shade)
    return r, out


class PerceptualRender(torch.autograd.Function):
    """Differentiable rolling + foveated Lambert render of one mesh seen by
    the renderer's views (all of one size).  Visibility (the triangle id of
    every pixel) is held fixed in the backward pass.

    forward(renderer, v0, v1, pose0, pose1) -> rgb [n_views, H, W, 3]
      v0, v1: float32 [V, 3] cuda (world positions at the frame's start/end)
      pose0, pose1: float32 [n_views, 6] (rotation vector, translation)
    Gradients flow to v0, v1, pose0 and pose1 (same devices as the inputs)."""

    @staticmethod
    def forward(ctx, renderer, v0, v1, pose0, pose1):
        v0c, v1c = v0.detach().contiguous(), v1.detach().contiguous()
        p0 = pose0.detach().cpu().tolist()
        p1 = pose1.detach().cpu().tolist()
        renderer.set_geometry(0, v0c, v1c)
        for i in range(len(renderer.views)):
            renderer.set_poses(i, p0[i], p1[i])
        out = renderer.frame(shade=True)
        ctx.renderer = renderer
        ctx.ids = [o['id'].clone() for o in out]
        # this forward's own geometry and poses: another forward on the same
        # renderer (a second loss term, a target render) may run before the
        # backward and re-point the renderer
        ctx.save_for_backward(v0c, v1c)
        ctx.poses = (p0, p1)
        ctx.pose_devices = (pose0.device, pose1.device)
        return torch.stack([o['rgb32'] for o in out]).clone()

    @staticmethod
    def backward(ctx, grad_rgb):
        r = ctx.renderer
        v0c, v1c = ctx.saved_tensors
        p0, p1 = ctx.poses
        r.set_geometry(0, v0c, v1c)
        for i in range(len(r.views)):
            r.set_poses(i, p0[i], p1[i])
        dl = [grad_rgb[i].contiguous().float() for i in range(grad_rgb.shape[0])]
        dv0, dv1, dp0, dp1 = r.backward(dl, ids=ctx.ids)
        return None, dv0[0], dv1[0], dp0.to(ctx.pose_devices[0]), dp1.to(ctx.pose_devices[1])
