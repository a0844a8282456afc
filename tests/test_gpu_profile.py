"""GPU parity of the tabulated foveation p_c and the lens distortion p_l
(Sec. 3.1.1 "Domain"; Sec. 5.1 "Lens Distortion") against the FP64 oracle,
whose tabulated maps are pinned in test_oracle_profile_pins.py:

* full-frame ids and depths (tabulated p_c, a barrel lens, both, the power
  law with a lens; tiles 8 / 16 / 32, both ray-cast launch forms), under the
  parity rule of tests/parity.py;
* the bound invariant on the device's own tile lists (every oracle hit is
  listed, with its quadrant);
* shading, G-buffer density, the display resampling (p_c only) and the
  backward with a profile;
* the batched graph copies the profiles it is given.

Where the device's FP32 evaluation meets a sample of a table (the profile's
slope changes there), the two sides may take either segment's slope: the
display's level of detail and the density are compared with either slope
for pixels within 1e-5 (normalised distance) of a sample.
"""
import copy

import numpy as np
import pytest

import oracle
import scenegen
from paper_1806_05385_amd import binding as B
from parity import assert_parity, compare

pytestmark = pytest.mark.gpu

PROFILES = {
    'table': (lambda: scenegen.foveal_table(33, 3.0), lambda: None),
    'lens': (lambda: None, lambda: scenegen.barrel_table(33, 0.22)),
    'table_lens': (lambda: scenegen.foveal_table(17, 2.0), lambda: scenegen.barrel_table(25, 0.2)),
    # scales G(s)/s that are not monotone (the bound's sector-box fallback)
    'kinked': (lambda: np.array([0.0, 0.4, 0.5, 0.8, 1.0], np.float32),
               lambda: np.array([0.0, 0.2, 0.6, 0.7, 1.0], np.float32)),
}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail('no GPU visible')
    return torch


def _soup(prof, seed=41, n_tris=1500, width=203, height=171, alpha=2.0, roll=(1.0, 0.0), fovea=(0.1, -0.15),
          yaw=2000.0, speed=20.0):
    pc, pl = PROFILES[prof]
    return scenegen.make_moving_soup(seed=seed, n_tris=n_tris, width=width, height=height, alpha=alpha, roll=roll,
                                     yaw_deg_s=yaw, obj_speed=speed, fovea=fovea, side=(0.03, 0.5),
                                     profile_c=pc(), profile_l=pl())


def _render(sc, tile=16, **kw):
    _torch()
    from paper_1806_05385_amd.render import Renderer
    r = Renderer(sc.meshes, sc.views, tile=tile, light=sc.light_dir, ambient=sc.ambient, **kw)
    out = r.frame()
    return r, [{k: v.cpu().numpy() for k, v in o.items()} for o in out]


@pytest.mark.parametrize('prof', sorted(PROFILES))
@pytest.mark.parametrize('tile,flags', [(8, 0), (16, 2), (32, 2), (16, 0)])
def test_profile_full_frame(prof, tile, flags):
    sc = _soup(prof)
    r, out = _render(sc, tile, flags=flags)
    v = sc.views[0]
    orc = oracle.Oracle(sc.meshes[0], v)
    o = orc.render()
    pix = np.arange(v.width * v.height)
    rep = compare(orc, o, out[0]['id'].ravel(), out[0]['depth'].ravel(), pix, v.znear)
    print(f"\n{prof} tile {tile} flags {flags}: {rep['hits']} hits, {rep['mismatch']} exempt "
          f"(edge {rep['near_edge']}, tie {rep['depth_tie']}, near {rep['near_plane']}), "
          f"depth max rel {rep['depth_max_rel']:.2e}", flush=True)
    assert rep['hits'] > 5000
    assert_parity(rep)


@pytest.mark.parametrize('prof,alpha,roll', [('table', 2.0, (1.0, 0.0)), ('lens', 1.0, (0.0, 0.9)),
                                             ('lens', 3.0, (1.0, 0.5)), ('table_lens', 2.0, (1.0, 0.0)),
                                             ('kinked', 2.0, (0.0, 0.9))])
def test_profile_bound_invariant_on_device_lists(prof, alpha, roll):
    """Every oracle hit (occluded or not) lies in a tile whose device-built
    list holds the triangle, with the pixel's quadrant in the mask."""
    sc = _soup(prof, seed=42, n_tris=800, width=160, height=144, alpha=alpha, roll=roll, yaw=3000.0, speed=30.0)
    v = sc.views[0]
    hp, ht, _ = oracle.Oracle(sc.meshes[0], v).all_hits()
    for tile in (8, 16, 32):
        r, out = _render(sc, tile)
        off, lst, qm = r.tile_lists(0)
        tiles_x = (v.width + tile - 1) // tile
        tid = (hp // v.width // tile) * tiles_x + (hp % v.width) // tile
        h = tile // 2
        quad = ((hp % v.width) % tile >= h).astype(int) + 2 * ((hp // v.width) % tile >= h).astype(int)
        members = {}
        for t in np.unique(tid):
            for f, m in zip(lst[off[t]:off[t + 1]], qm[off[t]:off[t + 1]]):
                members[(int(t), int(f))] = int(m)
        missing = [(int(p), int(f)) for p, f, t, q in zip(hp, ht, tid, quad)
                   if (members.get((int(t), int(f)), 0) >> (int(q) if tile >= 16 else 0)) & 1 == 0]
        assert len(hp) > 2000 and not missing, (prof, tile, missing[:5])


def _near_sample(s, n, tol=1e-5):
    q = np.asarray(s) * (n - 1)
    return np.abs(q - np.round(q)) < tol * (n - 1)


@pytest.mark.parametrize('prof', sorted(PROFILES))
def test_profile_shading_and_density(prof):
    torch = _torch()
    sc = _soup(prof, seed=43)
    v = sc.views[0]
    from paper_1806_05385_amd.render import Renderer
    r = Renderer(sc.meshes, sc.views, tile=16, light=sc.light_dir, ambient=sc.ambient, specular=0.5,
                 shininess=16.0)
    r.frame()
    orc = oracle.Oracle(sc.meshes[0], v)
    o = orc.render()
    oid = o['id']
    ids = [torch.as_tensor(oid.reshape(v.height, v.width)).cuda()]
    r.shade(ids=ids)
    g32 = r.outputs[0]['rgb32'].cpu().numpy().reshape(-1, 3)
    ref = orc.shade(oid, oracle.light_block(sc, 0.5, 16.0))
    ok = (oid >= 0) & (o['ehat'] > 1e-4)
    assert ok.sum() > 5000
    assert np.abs(g32[ok] - ref[ok]).max() < 5e-4
    g = r.gbuffer(ids=ids)[0]
    d = g['density'].cpu().numpy().ravel().astype(np.float64)
    gb = orc.gbuffer(oid)
    rd = gb['density']
    assert np.abs(g['normal'].cpu().numpy().reshape(-1, 3)[oid >= 0] - gb['normal'][oid >= 0]).max() < 1e-5
    rel = np.abs(d - rd) / rd
    if v.profile_c is None:   # the power law: as test_gpu_shading.py
        assert np.isfinite(d).sum() >= d.size - 1
        return
    # the panel points' normalised distances: a pixel there takes either
    # neighbouring segment's slope
    R = oracle.fovea_radius(v)
    sp = np.array([np.linalg.norm(oracle.unfoveate(v, oracle.pixel_setup(v, p)[0]) - np.array(v.fovea)) / R
                   for p in range(v.width * v.height)])
    tie = _near_sample(sp, len(v.profile_c))
    print(f'\n{prof}: density max rel {rel[~tie].max():.2e}, {tie.sum()} pixels at a sample', flush=True)
    assert rel[~tie].max() < 2e-6
    assert tie.sum() < 0.01 * d.size


def test_profile_display():
    """pr_unfoveate with a tabulated p_c (and a lens, which the display
    ignores) against the oracle's resampling: 1 LSB, except display pixels
    at a table sample (either side's slope) and the filter's window ties."""
    torch = _torch()
    from paper_1806_05385_amd.render import Display
    rng = np.random.default_rng(12)
    for prof in ('table', 'table_lens'):
        pc, pl = PROFILES[prof]
        view = scenegen.View(203, 171, np.zeros(6, np.float32), np.zeros(6, np.float32), fovea=(0.1, -0.15),
                             alpha=2.0, roll_dir=(0.0, 0.0), profile_c=pc(), profile_l=pl())
        fov = rng.integers(0, 256, size=(171, 203, 4), dtype=np.uint8)
        for mode, (Wd, Hd) in ((B.PR_UNFOV_MIP, (190, 160)), (B.PR_UNFOV_FILTER, (220, 180))):
            d = Display([view], sizes=[(Wd, Hd)], mode=mode, sigma=0.8)
            out = d.run([torch.as_tensor(fov).cuda()])
            torch.cuda.synchronize()
            got = out[0].cpu().numpy().reshape(-1, 4).astype(int)
            ref = oracle.to_rgba8(oracle.unfoveate_image(view, fov, Wd, Hd, mode, 0.8)).astype(int)
            bad = np.nonzero(np.abs(got - ref).max(axis=1) > 1)[0]
            R = oracle.fovea_radius(view)
            xs = np.stack([(2 * (bad % Wd) + 1) / Wd - 1, 1 - (2 * (bad // Wd) + 1) / Hd], 1)
            sp = np.linalg.norm(xs - np.array(view.fovea), axis=1) / R
            tie_sample = _near_sample(sp, len(view.profile_c), 1e-4)
            unexplained = []
            for p, ts in zip(bad, tie_sample):
                if ts:
                    continue
                if mode == B.PR_UNFOV_FILTER:
                    a, b = int(p % Wd), int(p // Wd)
                    u, _, _ = oracle.unfov_coord(view, Wd, Hd, float(a), float(b))
                    frac = (u + 0.5) - np.floor(u + 0.5)
                    if (np.minimum(frac, 1 - frac) < 2e-3).any():
                        continue
                unexplained.append(int(p))
            print(f'\n{prof} mode {mode}: {len(bad)} pixels beyond 1 LSB, {int(tie_sample.sum())} at a sample',
                  flush=True)
            assert not unexplained, (prof, mode, unexplained[:5], got[unexplained[:5]], ref[unexplained[:5]])
            assert len(bad) <= 2e-3 * Wd * Hd + 5


def test_profile_backward():
    """pr_backward with a tabulated p_c and a lens against the oracle's
    analytic gradient (same visibility and upstream gradient)."""
    torch = _torch()
    sc = scenegen.make_grad(seed=5, size=96, f=16)
    mesh, view, target = sc.meshes[0], sc.views[0], sc.extra['target']
    view.profile_c = scenegen.foveal_table(17, 2.0)
    view.profile_l = scenegen.barrel_table(17, 0.2)
    light = oracle.light_block(sc)
    orc_t = oracle.Oracle(target, view)
    tgt = orc_t.shade(orc_t.render()['id'], light)
    orc = oracle.Oracle(mesh, view)
    oid = orc.render()['id']
    c_ref = orc.shade(oid, light)
    L, g0, g1, gp0, gp1 = orc.loss_grad(oid, light, tgt)
    from paper_1806_05385_amd.render import Renderer
    r = Renderer(sc.meshes, sc.views, tile=16, light=sc.light_dir, ambient=sc.ambient)
    r.frame()
    ids = torch.as_tensor(oid.reshape(view.height, view.width)).cuda()
    dl = torch.as_tensor(2.0 * (c_ref - tgt).reshape(view.height, view.width, 3), dtype=torch.float32).cuda()
    dv0, dv1, dp0, dp1 = r.backward([dl], ids=[ids])
    for g, ref in ((dv0[0], g0), (dv1[0], g1), (dp0[0], gp0), (dp1[0], gp1)):
        g = g.cpu().numpy().astype(np.float64)
        tol = 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
        assert (np.abs(g - ref) <= tol).all(), np.abs(g - ref).max()


def test_batch_copies_profiles():
    """A batch built from views with profiles renders what the plain frame
    renders (ids bitwise) after the caller's profile objects are gone."""
    torch = _torch()
    from paper_1806_05385_amd.render import Batch, Renderer
    scs = [_soup('table_lens', seed=44, n_tris=600, width=120, height=100),
           _soup('lens', seed=45, n_tris=600, width=96, height=128, fovea=(0.0, 0.0))]
    meshes = [s.meshes[0] for s in scs]
    views = []
    for k, s in enumerate(scs):
        vv = copy.copy(s.views[0])
        vv.mesh = k
        views.append(vv)
    bt = Batch(meshes, views, tile=16, light=scs[0].light_dir, ambient=scs[0].ambient, rgba8=False)
    import gc
    bt.c_views = None   # the caller's view array and its profiles go away
    gc.collect()
    bt.launch()
    torch.cuda.synchronize()
    for k, s in enumerate(scs):
        r, out = _render(s, 16)
        assert np.array_equal(bt.outputs[k]['id'].cpu().numpy(), out[0]['id']), k
