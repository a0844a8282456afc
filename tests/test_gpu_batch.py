"""Batched form: many views of uneven size and triangle count in one
hipGraph-captured frame with a persistent, longest-list-first ray cast."""
import os

import numpy as np
import pytest

import oracle
import scenegen
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail('no GPU visible')
    return torch


def _small_batch(n=6):
    return scenegen.make_batch(seed=4, n_views=n, max_side=320, max_tris=20000, min_side=40, min_tris=200)


def test_batched_equals_plain_bitwise_and_replays():
    """Every view of the batch equals the plain per-view frame bitwise (ids
    and depth bits), on every graph replay, with eager torch work and
    synchronisations between replays."""
    torch = _torch()
    from paper_1806_05385_amd.render import Batch, Renderer
    sc = _small_batch()
    bt = Batch(sc.meshes, sc.views, tile=16, light=sc.light_dir, ambient=sc.ambient, rgba8=True)
    refs = []
    for v in sc.views:
        r = Renderer([sc.meshes[v.mesh]], [scenegen.View(**{**v.__dict__, 'mesh': 0})], tile=16,
                     light=sc.light_dir, ambient=sc.ambient)
        o = r.frame()[0]
        refs.append({k: o[k].cpu().numpy() for k in ('id', 'depth', 'rgba8')})
    for rep in range(3):
        for o in bt.outputs:
            o['id'].fill_(-7)
            o['depth'].fill_(-1.0)
        x = torch.randn(1000, 1000, device='cuda')
        (x @ x).sum().item()                       # eager work between replays
        out = bt.launch()
        torch.cuda.synchronize()
        assert bt.status().overflow == 0
        for v, (o, ref) in enumerate(zip(out, refs)):
            assert np.array_equal(o['id'].cpu().numpy(), ref['id']), (rep, v)
            assert np.array_equal(o['depth'].cpu().numpy().view(np.uint32), ref['depth'].view(np.uint32)), (rep, v)
            assert np.array_equal(o['rgba8'].cpu().numpy(), ref['rgba8']), (rep, v)
    bt.close()


def test_batch_parity_with_oracle():
    _torch()
    from paper_1806_05385_amd.render import Batch
    sc = _small_batch(5)
    bt = Batch(sc.meshes, sc.views, tile=8, light=sc.light_dir, ambient=sc.ambient)
    out = bt.launch()
    for v, view in enumerate(sc.views):
        orc = oracle.Oracle(sc.meshes[view.mesh], view)
        o = orc.render()
        pix = np.arange(view.width * view.height)
        rep = compare(orc, o, out[v]['id'].cpu().numpy().ravel(), out[v]['depth'].cpu().numpy().ravel(), pix,
                      view.znear)
        print(f"\nbatch view {v} {view.width}x{view.height}, {sc.meshes[view.mesh].nt} tris: {rep['hits']} hits, "
              f"{rep['mismatch']} exempt", flush=True)
        assert_parity(rep)
    bt.close()


def test_autotuner_chooses_and_caches(tmp_path, monkeypatch):
    _torch()
    from paper_1806_05385_amd.render import Batch
    cache = tmp_path / 'tune.txt'
    monkeypatch.setenv('PR_TUNE_CACHE', str(cache))
    sc = _small_batch(4)
    bt = Batch(sc.meshes, sc.views, tile=0, light=sc.light_dir, ambient=sc.ambient)
    info = bt.info()
    assert info['tile'] in (8, 16, 32)
    assert all(ms > 0 for ms in info['trial_ms'].values())
    assert info['trial_ms'][info['tile']] == min(info['trial_ms'].values())
    assert info['bin_capacity'] >= bt.status().pairs_required
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f"\t{info['tile']}")
    bt2 = Batch(sc.meshes, sc.views, tile=0, light=sc.light_dir, ambient=sc.ambient)
    info2 = bt2.info()
    assert info2['tile'] == info['tile'] and all(ms == 0 for ms in info2['trial_ms'].values())
    ref = bt.launch()
    out = bt2.launch()
    for a, b in zip(ref, out):
        assert np.array_equal(a['id'].cpu().numpy(), b['id'].cpu().numpy())
    bt.close()
    bt2.close()


def test_full_batch_parity_with_oracle():
    """The benchmark's batch (64 views, sides log-uniform 128..2048, scenes
    log-uniform 1k..500k triangles, each view with its own fovea, poses,
    foveation and rolling), autotuned and replayed from its hipGraph as the
    benchmark runs it: every pixel of every view against the oracle
    (orc_render_fast, re-checked by the brute force on 200 sampled pixels
    per view)."""
    _torch()
    from paper_1806_05385_amd.render import Batch
    sc = scenegen.make_batch()
    assert len(sc.views) == 64
    bt = Batch(sc.meshes, sc.views, tile=0, light=sc.light_dir, ambient=sc.ambient, rgba8=True)
    bt.launch()
    out = bt.launch()
    st = bt.status()
    assert st.overflow == 0
    total = exempt = 0
    for v, view in enumerate(sc.views):
        orc = oracle.Oracle(sc.meshes[view.mesh], view)
        o = orc.render_fast()
        pix = scenegen.sample_pixels(4100 + v, view, 200)
        bf = orc.render(pix)
        assert np.array_equal(bf['id'], o['id'][pix]) and np.array_equal(bf['z'].view(np.uint8),
                                                                           o['z'][pix].view(np.uint8))
        allpix = np.arange(view.width * view.height)
        rep = compare(orc, o, out[v]['id'].cpu().numpy().ravel(), out[v]['depth'].cpu().numpy().ravel(), allpix,
                      view.znear)
        total += len(allpix)
        exempt += rep['mismatch'] + rep['grazing']
        assert_parity(rep)
    print(f"\nbatch: 64 views, {total} pixels, tile {bt.info()['tile']}, {exempt} exempt pixels", flush=True)
    bt.close()
