"""Benchmark: one step = one perceptual rasterization frame of the HMD
workload (201,920 triangles, two eyes at 1512x1680, foveated alpha = 2,
rolling, head yaw 120 deg/s + 0.5 m/s over an 11.1 ms frame): pr_bound ->
pr_bin -> pr_raycast -> pr_shade for both eyes on one GPU.  Inputs are
resident in HBM before timing starts.  Prints one JSON line.

The CPU baseline is the FP64 brute-force oracle timed on a bounded sample of
pixels of the same workload and extrapolated to a full frame."""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_TEST_MOVING = 48   # 3 edges x 8 multiply-adds over the ray terms (rx, ry, t rx, t ry, t, t^2 rx, t^2 ry, t^2)
FLOP_PER_TEST_STATIC = 12   # 3 edges x 2 multiply-adds (rx, ry)
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 matrix (MFMA) peak


def kernel_source_sha() -> str:
    """Hash of the kernel sources; a stored counter figure is valid only for
    the sources it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ('pr_kernels.hip', 'pr_kernels.h', 'pr_geom.h'):
        with open(os.path.join(ROOT, 'paper_1806_05385_amd', 'csrc', f), 'rb') as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per ray-cast launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when the summary is
    missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, 'profiles', 'k_raycast_hmd_traffic.txt')
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ':' in line and not line.startswith(' '):
            k, v = line.split(':', 1)
            kv[k.strip()] = v.strip()
    if kv.get('kernel_source_sha') != kernel_source_sha():
        return None
    try:
        return int(kv['bytes_per_launch'])
    except (KeyError, ValueError):
        return None


def grad_leg(args, stream):
    """Backward / forward on the differentiation workload (100,820 triangles,
    512x512, rolling + foveated, moving camera): forward = bound + bin + ray
    cast with fp32 rgb shading, backward = pr_backward.  Median ms of each."""
    import numpy as np
    import torch

    import scenegen
    from paper_1806_05385_amd.render import Renderer
    gsc = scenegen.make_grad()
    gr = Renderer(gsc.meshes, gsc.views, tile=args.tile, light=gsc.light_dir, ambient=gsc.ambient)
    gr.frame(check=True)
    dl = [torch.ones_like(gr.outputs[0]['rgb32'])]
    for _ in range(3):
        gr.frame(check=False)
        gr.backward(dl)
    nrep = max(10, args.steps)
    f0, f1, b1 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    fwd_ms, bwd_ms = [], []
    for _ in range(nrep):
        f0.record(stream)
        gr.bound()
        gr.bin()
        gr.raycast_shade(rgba8=False, rgb32=True)
        f1.record(stream)
        gr.backward(dl)
        b1.record(stream)
        torch.cuda.synchronize()
        fwd_ms.append(f0.elapsed_time(f1))
        bwd_ms.append(f1.elapsed_time(b1))
    return float(np.median(fwd_ms)), float(np.median(bwd_ms))


def frame_distribution(r, stream, n):
    """Per-frame times (ms) of n frames timed one by one with HIP events on
    the frame's stream (bound, bin, ray cast with fused shading)."""
    import numpy as np
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        r.bound()
        r.bin()
        r.raycast_shade(rgba8=True, rgb32=False)
        b.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def sequential_eyes(sc, args, stream, n):
    """The frame with each eye rendered by its own calls, one after the
    other (two single-view renderers): mean ms over n frames."""
    import torch

    import scenegen
    from paper_1806_05385_amd.render import Renderer
    rs = []
    for v in sc.views:
        vv = scenegen.View(**{**v.__dict__, 'mesh': 0})
        rr = Renderer([sc.meshes[v.mesh]], [vv], tile=args.tile, light=sc.light_dir, ambient=sc.ambient)
        rr.frame(check=True, rgb32=False)
        rs.append(rr)
    for _ in range(3):
        for rr in rs:
            rr.frame(check=False, rgb32=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n):
        for rr in rs:
            rr.bound()
            rr.bin()
            rr.raycast_shade(rgba8=True, rgb32=False)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def display_leg(sc, r, stream, n):
    """Display unfoveation of the HMD frame (both eyes, displays of the
    foveated images' size) in both forms: median ms, and HBM GB/s of the
    algorithmic bytes (4 B read per foveated pixel, 4 B written per display
    pixel) against 8 TB/s."""
    import numpy as np
    import torch

    from paper_1806_05385_amd import binding as B
    from paper_1806_05385_amd.render import Display
    fov = [o['rgba8'] for o in r.outputs]
    out = {}
    for name, mode in (('mip', B.PR_UNFOV_MIP), ('filter', B.PR_UNFOV_FILTER)):
        d = Display(sc.views, mode=mode, sigma=0.7)
        for _ in range(3):
            d.run(fov)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        torch.cuda.synchronize()
        for a, b in ev:
            a.record(stream)
            d.run(fov)
            b.record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        px = sum(v.width * v.height for v in sc.views)
        nbytes = 8 * px
        out[name] = {'ms': round(ms, 4), 'algorithmic_bytes': nbytes, 'GBps': round(nbytes / (ms * 1e-3) / 1e9, 1),
                     'frac_of_hbm_peak': round(nbytes / (ms * 1e-3) / 8e12, 4)}
    return out


def _ablation_run(sc, args, stream, n, **kw):
    """One bound setting on scene sc: listed pairs, candidates, ray-triangle
    tests, sample test efficiency (hits / tests, counted in a separate
    frame) and the mean frame time."""
    import torch

    from paper_1806_05385_amd import binding as B
    from paper_1806_05385_amd.render import Renderer
    rr = Renderer(sc.meshes, sc.views, tile=args.tile, light=sc.light_dir, ambient=sc.ambient, **kw)
    rr.frame(check=True, rgb32=False)
    rr.flags = B.PR_FLAG_COUNT | B.PR_FLAG_PERSISTENT
    rr._prepare()
    rr.frame(check=True, rgb32=False)
    st = rr.status()
    rr.flags = B.PR_FLAG_PERSISTENT
    rr._prepare()
    for _ in range(3):
        rr.frame(check=False, rgb32=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n):
        rr.bound()
        rr.bin()
        rr.raycast_shade(rgba8=True, rgb32=False)
    e1.record(stream)
    torch.cuda.synchronize()
    out = {'frame_ms': round(e0.elapsed_time(e1) / n, 4), 'pairs': int(st.pairs_total),
           'candidates': int(st.pairs_required), 'tests': int(st.tests),
           'ste': round(int(st.hits) / max(int(st.tests), 1), 4)}
    del rr
    return out


def bound_ablation(sc, args, stream, n):
    """The HMD frame under each rolling bound of Sec. 4.2 (Zenon, Adaptive,
    Hull, Quad), and under each foveated per-tile test (Sec. 4.1: exact
    display-space test, box only, Simple and Recursive support lines) on
    the same frame and on its static form (no rolling, no motion)."""
    import copy as _copy

    import numpy as np

    from paper_1806_05385_amd import binding as B
    out = {}
    for name, mode in (('zenon', B.PR_BOUND_ZENON), ('adaptive', B.PR_BOUND_ADAPTIVE), ('hull', B.PR_BOUND_HULL),
                       ('quad', B.PR_BOUND_QUAD)):
        out[name] = _ablation_run(sc, args, stream, n, bound=mode)
    static = _copy.copy(sc)
    static.views = []
    for v in sc.views:
        vv = _copy.copy(v)
        vv.roll_dir = (0.0, 0.0)
        vv.pose1 = np.array(vv.pose0, copy=True)
        static.views.append(vv)
    static.meshes = [_copy.copy(m) for m in sc.meshes]
    for m in static.meshes:
        m.v1 = m.v0
    fovs = (('exact', B.PR_FOV_EXACT), ('box', B.PR_FOV_QUAD), ('simple', B.PR_FOV_SIMPLE),
            ('recursive', B.PR_FOV_RECURSIVE))
    out['foveated'] = {name: _ablation_run(sc, args, stream, n, fov_bound=mode) for name, mode in fovs}
    out['foveated_static'] = {name: _ablation_run(static, args, stream, n, fov_bound=mode) for name, mode in fovs}
    return out


def shading_leg(sc, args, stream, n):
    """Richer rolling shading on the HMD frame: the fused ray cast with the
    Blinn-Phong highlight (eye at each pixel's time) against the Lambert-only
    one, and the G-buffer pass (normal, barycentrics, density: 24 B written
    and 4 B of id read per pixel, plus the record gathers) with its HBM rate
    on the algorithmic bytes."""
    import torch

    from paper_1806_05385_amd import binding as B
    from paper_1806_05385_amd.render import Renderer

    def timed(fn):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    out = {}
    for name, ks in (('lambert', 0.0), ('highlight', 0.6)):
        rr = Renderer(sc.meshes, sc.views, tile=args.tile, light=sc.light_dir, ambient=sc.ambient, specular=ks,
                      shininess=24.0, flags=B.PR_FLAG_PERSISTENT)
        rr.frame(check=True, rgb32=False)
        out[name + '_raycast_shade_ms'] = round(timed(lambda: rr.raycast_shade(rgba8=True, rgb32=False)), 4)
        if ks > 0:
            g = rr.gbuffer()
            px = sum(v.width * v.height for v in sc.views)
            ms = timed(lambda: rr.gbuffer())
            nbytes = 28 * px
            out['gbuffer_ms'] = round(ms, 4)
            out['gbuffer_GBps'] = round(nbytes / (ms * 1e-3) / 1e9, 1)
            out['gbuffer_frac_of_hbm_peak'] = round(nbytes / (ms * 1e-3) / 8e12, 4)
            del g
        del rr
    return out


def profile_leg(sc, args, stream, n):
    """The HMD frame with a tabulated foveation (64 samples of the alpha = 2
    power law's p_c(s) = sqrt(s)) and with that table composed with a barrel
    lens pre-distortion (33 samples of s (1 - 0.2 s^2)): frame ms, listed
    pairs and ray-triangle tests, against the analytic power law."""
    import copy as _copy

    import numpy as np
    import scenegen
    import torch

    from paper_1806_05385_amd import binding as B
    from paper_1806_05385_amd.render import Renderer
    out = {}
    table = np.sqrt(np.linspace(0.0, 1.0, 64)).astype(np.float32)
    for name, pc, pl in (('power_law', None, None), ('table', table, None),
                         ('table_lens', table, scenegen.barrel_table(33, 0.2))):
        views = []
        for v in sc.views:
            vv = _copy.copy(v)
            vv.profile_c, vv.profile_l = pc, pl
            views.append(vv)
        rr = Renderer(sc.meshes, views, tile=args.tile, light=sc.light_dir, ambient=sc.ambient)
        rr.frame(check=True, rgb32=False)
        rr.flags = B.PR_FLAG_COUNT | B.PR_FLAG_PERSISTENT
        rr._prepare()
        rr.frame(check=True, rgb32=False)
        st = rr.status()
        rr.flags = B.PR_FLAG_PERSISTENT
        rr._prepare()
        for _ in range(3):
            rr.frame(check=False, rgb32=False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            rr.bound()
            rr.bin()
            rr.raycast_shade(rgba8=True, rgb32=False)
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = {'frame_ms': round(e0.elapsed_time(e1) / n, 4), 'pairs': int(st.pairs_total),
                     'tests': int(st.tests)}
        del rr
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=50)
    ap.add_argument('--warmup', type=int, default=100)
    ap.add_argument('--tile', type=int, default=16)
    ap.add_argument('--no-persistent', dest='persistent', action='store_false',
                    help='one block per tile item instead of the longest-first persistent ray cast')
    ap.add_argument('--cpu-pixels', type=int, default=49152)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--only', choices=['all', 'hmd', 'grad'], default='all',
                    help='hmd: only the headline frame (no backward, batch or CPU legs; for profiling); '
                         'grad: only the backward / forward leg (prints that leg\'s line; for profiling)')
    ap.add_argument('--source-sha', action='store_true', help='print the kernel source hash and exit')
    ap.add_argument('--copy-bytes', type=int, default=0,
                    help='only run a plain device copy of this many bytes 10 times (counter calibration)')
    args = ap.parse_args()
    if args.source_sha:
        print(kernel_source_sha())
        return
    if args.gpus != 1:
        print(json.dumps({'error': 'this build runs on one GPU; --gpus above 1 is not supported'}))
        sys.exit(2)

    import numpy as np
    import torch

    import scenegen
    from paper_1806_05385_amd import binding as B
    from paper_1806_05385_amd.render import Renderer

    torch.cuda.set_device(0)
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device='cuda')
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({'copy_bytes': args.copy_bytes, 'launches': 10}))
        return
    if args.only == 'grad':
        fwd_med, bwd_med = grad_leg(args, torch.cuda.current_stream())
        print(json.dumps({'grad_workload': {'triangles': 100820, 'size': 512, 'fwd_ms': round(fwd_med, 4),
                                            'bwd_ms': round(bwd_med, 4)}, 'bwd_fwd': round(bwd_med / fwd_med, 3)}))
        return
    sc = scenegen.make_hmd()
    mesh = sc.meshes[0]
    r = Renderer(sc.meshes, sc.views, tile=args.tile, light=sc.light_dir, ambient=sc.ambient)
    # every frame shades RGBA8 only, as the timed ones do
    r.frame(check=True, rgb32=False)            # sizes the tile-list capacity
    # one counting frame (not timed): ray-triangle tests and hits
    r.flags = B.PR_FLAG_COUNT | (B.PR_FLAG_PERSISTENT if args.persistent else 0)
    r._prepare()
    r.frame(check=True, rgb32=False)
    st = r.status()
    tests, hits = int(st.tests), int(st.hits)
    r.flags = B.PR_FLAG_PERSISTENT if args.persistent else 0
    r._prepare()
    r.frame(check=True, rgb32=False)

    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        r.frame(check=False, rgb32=False)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for k in range(args.steps):
        r.bound()
        r.bin()
        r.raycast_shade(rgba8=True, rgb32=False)   # ray cast with the shading fused in
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    st = r.status()
    assert not st.overflow
    ms_step = t0.elapsed_time(t1) / args.steps
    # (after the timed frames) the ray cast bracketed by an event pair inside
    # each frame: each pair adds the event's own wait to the span
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for k in range(args.steps):
        r.bound()
        r.bin()
        ev[k][0].record(stream)
        r.raycast_shade(rgba8=True, rgb32=False)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    ray_ms_bracketed = float(np.array([a.elapsed_time(b) for a, b in ev]).mean())
    # its average launch duration (the roofline's): the same launch, on the
    # same lists, issued `steps` times back to back between one event pair
    b0 = torch.cuda.Event(enable_timing=True)
    b1 = torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    for _ in range(args.steps):
        r.raycast_shade(rgba8=True, rgb32=False)
    b1.record(stream)
    torch.cuda.synchronize()
    ray_ms_avg = b0.elapsed_time(b1) / args.steps
    # the frame's distribution, timed frame by frame (not the headline)
    dist = frame_distribution(r, stream, max(200, args.steps))
    px_total = sum(v.width * v.height for v in sc.views)
    fb_bytes = 12 * px_total     # id, depth and RGBA8 written once per pixel

    rolling = any(v.roll_dir[0] or v.roll_dir[1] for v in sc.views)
    flop_test = FLOP_PER_TEST_MOVING if rolling else FLOP_PER_TEST_STATIC
    achieved = tests * flop_test / (ray_ms_avg * 1e-3) / 1e12
    traffic = measured_traffic()

    if args.only == 'hmd':
        args.no_cpu_baseline = True
    fwd_med = bwd_med = float('nan')
    batch_out = large_out = seq_eyes_ms = display_out = ablation_out = shading_out = profile_out = None
    if args.only == 'all':
        seq_eyes_ms = sequential_eyes(sc, args, stream, 50)
        shading_out = shading_leg(sc, args, stream, 50)
        profile_out = profile_leg(sc, args, stream, 20)
        display_out = display_leg(sc, r, stream, 50)
        ablation_out = bound_ablation(sc, args, stream, 20)
        fwd_med, bwd_med = grad_leg(args, stream)

        # batched form: 64 views (log-uniform 128..2048 px, 1k..500k triangles)
        # in one autotuned hipGraph frame vs 64 sequential plain frames
        from paper_1806_05385_amd.render import Batch
        bsc = scenegen.make_batch()
        torch.cuda.synchronize()
        bt = Batch(bsc.meshes, bsc.views, tile=0, light=bsc.light_dir, ambient=bsc.ambient, rgba8=True)
        binfo = bt.info()
        for _ in range(2):
            bt.launch()
        nb = max(5, args.steps // 5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(nb):
            bt.launch()
        e1.record(stream)
        torch.cuda.synchronize()
        batch_ms = e0.elapsed_time(e1) / nb
        assert not bt.status().overflow
        seq = []
        for v in bsc.views:
            vv = scenegen.View(**{**v.__dict__, 'mesh': 0})
            rr = Renderer([bt.meshes[v.mesh]], [vv], tile=binfo['tile'], light=bsc.light_dir, ambient=bsc.ambient)
            rr.frame(check=True)
            seq.append(rr)

        def seq_round():
            for rr in seq:
                rr.bound()
                rr.bin()
                rr.raycast_shade(rgba8=True, rgb32=False)
        seq_round()
        torch.cuda.synchronize()
        h0 = time.perf_counter()
        e0.record(stream)
        for _ in range(nb):
            seq_round()
        e1.record(stream)
        h1 = time.perf_counter()
        torch.cuda.synchronize()
        seq_ms = e0.elapsed_time(e1) / nb
        seq_enqueue_ms = (h1 - h0) * 1e3 / nb
        # the same 64 plain frames captured once into a graph and replayed:
        # their GPU time without the host's launch overhead
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(side):
            seq_round()
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=side):
                seq_round()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(nb):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        seq_graph_ms = e0.elapsed_time(e1) / nb
        n_views = len(bsc.views)
        batch_out = {'views': n_views, 'pixels': int(sum(v.width * v.height for v in bsc.views)),
                     'triangles': int(sum(bsc.meshes[v.mesh].nt for v in bsc.views)), 'tile': binfo['tile'],
                     'trial_ms': binfo['trial_ms'], 'batched_ms': round(batch_ms, 4), 'sequential_ms': round(seq_ms, 4),
                     'batched_views_per_s': round(n_views / (batch_ms * 1e-3), 1),
                     'sequential_views_per_s': round(n_views / (seq_ms * 1e-3), 1),
                     'speedup': round(seq_ms / batch_ms, 3),
                     'sequential_host_enqueue_ms': round(seq_enqueue_ms, 4),
                     'sequential_graph_ms': round(seq_graph_ms, 4),
                     'speedup_vs_sequential_graph': round(seq_graph_ms / batch_ms, 3)}
        bt.close()
        del seq

        # large workload (1,000 moving spheres = 2M triangles, 2 x 2160x2160)
        lsc = scenegen.make_large()
        lr = Renderer(lsc.meshes, lsc.views, tile=args.tile, light=lsc.light_dir, ambient=lsc.ambient)
        lr.frame(check=True)
        for _ in range(2):
            lr.frame(check=False)
        nl = max(5, args.steps // 5)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(nl):
            lr.bound()
            lr.bin()
            lr.raycast_shade(rgba8=True, rgb32=False)
        e1.record(stream)
        torch.cuda.synchronize()
        assert not lr.status().overflow
        large_out = {'triangles': int(lsc.meshes[0].nt), 'views': len(lsc.views), 'width': lsc.views[0].width,
                     'height': lsc.views[0].height, 'frame_ms': round(e0.elapsed_time(e1) / nl, 4)}
        del lr

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        view = sc.views[0]
        pix = scenegen.sample_pixels(1234, view, args.cpu_pixels)
        orc = oracle.Oracle(mesh, view)
        threads = oracle.lib().orc_get_threads()
        c0 = time.perf_counter()
        orc.render(pix)
        c1 = time.perf_counter()
        cpu_ms = (c1 - c0) / len(pix) * px_total * 1e3
        cpu = {'value': round(cpu_ms, 1), 'unit': 'ms/frame', 'cores': threads, 'kind': 'oracle',
               'sample': f'{len(pix)} pixels of eye 0 (half within 0.1 NDC of the fovea) x {mesh.nt} triangles, '
                         f'FP64 brute force, {c1 - c0:.1f} s, extrapolated to {px_total} pixels'}

    out = {
        'metric': 'frame ms + ray-tri tests/s, fov+rolling 2x1512x1680 @200k tris; bwd/fwd',
        'value': round(ms_step, 4),
        'unit': 'ms/frame',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': round(ms_step, 4),
        'higher_is_better': False,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f32',
        'data': 'synthetic (seeded displaced geodesic sphere + 500 boxes)',
        'config': {'workload': 'hmd: 201,920 triangles, 2 eyes x 1512x1680, foveated (alpha 2) + rolling, '
                               'head yaw 120 deg/s + 0.5 m/s, Lambert', 'triangles': int(mesh.nt),
                   'views': len(sc.views), 'width': sc.views[0].width, 'height': sc.views[0].height,
                   'tile': args.tile},
        'frames_per_s': round(1e3 / ms_step, 1),
        'frame_ms_dist': {'frames': int(len(dist)), 'median': round(float(np.median(dist)), 4),
                          'p10': round(float(np.percentile(dist, 10)), 4),
                          'p90': round(float(np.percentile(dist, 90)), 4)},
        'sequential_eyes_ms': round(seq_eyes_ms, 4) if seq_eyes_ms is not None else None,
        'framebuffer': {'bytes': fb_bytes, 'GBps': round(fb_bytes / (ray_ms_avg * 1e-3) / 1e9, 1),
                        'frac_of_hbm_peak': round(fb_bytes / (ray_ms_avg * 1e-3) / 8e12, 4)},
        'display': display_out,
        'bound_ablation': ablation_out,
        'shading': shading_out,
        'profiles': profile_out,
        'raycast_shade_ms': round(ray_ms_avg, 4),
        'raycast_shade_bracketed_ms': round(ray_ms_bracketed, 4),
        'tests_per_frame': tests,
        'tests_per_s': round(tests / (ray_ms_avg * 1e-3), 1),
        'ste': round(hits / max(tests, 1), 4),
        'pairs_per_frame': int(st.pairs_total),
        'bwd_fwd': round(bwd_med / fwd_med, 3) if args.only == 'all' else None,
        'batch': batch_out,
        'large': large_out,
        'grad_workload': {'triangles': 100820, 'size': 512, 'fwd_ms': round(fwd_med, 4),
                          'bwd_ms': round(bwd_med, 4)} if args.only == 'all' else None,
        'wall_s': round(wall, 3),
        'roofline': {'bound': 'mfma', 'achieved': round(achieved, 3), 'peak': PEAK_FP32_TFLOPS,
                     'unit': 'TFLOP/s', 'frac': round(achieved / PEAK_FP32_TFLOPS, 4), 'traffic': traffic,
                     'kernel': ('k_raycast_queue (shading fused)' if args.persistent else 'k_raycast + k_shade'),
                     'flop_per_test': flop_test},
        'cpu_baseline': cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()
