"""GPU backward (pr_backward, PerceptualRender) against the FP64 oracle's
analytic frozen-visibility gradient of L = sum (c - c*)^2, itself pinned by
central differences in test_oracle_pins.py.  Both sides use the oracle's
visibility (its id buffer is handed to the GPU) and the same upstream
gradient dL/dc = 2 (c - c*) with c the oracle's colours: near grazing
incidence the barycentric terms scale like 1/S^2, so the few silhouette
pixels whose FP32 forward colour differs from the FP64 one by ~1e-4 would
otherwise move the pose sums by more than the backward's own error (the
forward colours are checked separately, to 1 LSB in RGBA8).

Tolerance: |g - g_ref| <= 1e-3 max(|g_ref|, 1e-3 max|g_ref|) for every
component (the backward sets up each pixel's ray and the shading chain in
FP64, so no component is exempt)."""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu

REL = 1e-3


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail('no GPU visible')
    return torch


def _close(g, ref, floor_frac=1e-3):
    """|g - ref| <= 1e-3 max(|ref|, 1e-3 max|ref|) componentwise."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    tol = REL * np.maximum(np.abs(ref), floor_frac * np.abs(ref).max())
    bad = np.abs(g - ref) > tol
    return bad, np.abs(g - ref) / np.maximum(np.abs(ref), 1e-30)


def _case(size, f):
    sc = scenegen.make_grad(seed=5, size=size, f=f)
    return _case_scene(sc, sc.extra['target'])


def _case_scene(sc, target):
    torch = _torch()
    from paper_1806_05385_amd.render import Renderer
    mesh, view = sc.meshes[0], sc.views[0]
    light = oracle.light_block(sc)
    orc_t = oracle.Oracle(target, view)
    tgt = orc_t.shade(orc_t.render()['id'], light)
    orc = oracle.Oracle(mesh, view)
    oid = orc.render()['id']
    L, g0, g1, gp0, gp1 = orc.loss_grad(oid, light, tgt)
    r = Renderer(sc.meshes, sc.views, tile=16, light=sc.light_dir, ambient=sc.ambient)
    r.frame()
    ids = torch.as_tensor(oid.reshape(view.height, view.width)).cuda()
    r.shade(ids=[ids])
    rgb = r.outputs[0]['rgb32']
    tg = torch.as_tensor(tgt.reshape(view.height, view.width, 3), dtype=torch.float32).cuda()
    c_ref = orc.shade(oid, light)
    dl = torch.as_tensor(2.0 * (c_ref - tgt).reshape(view.height, view.width, 3), dtype=torch.float32).cuda()
    dv0, dv1, dp0, dp1 = r.backward([dl], ids=[ids])
    return dict(L=L, g0=g0, g1=g1, gp0=gp0, gp1=gp1, dv0=dv0[0].cpu().numpy(), dv1=dv1[0].cpu().numpy(),
                dp0=dp0[0].cpu().numpy(), dp1=dp1[0].cpu().numpy(), gpu_L=float(((rgb - tg) ** 2).sum()),
                r=r, sc=sc, oid=oid, tgt=tgt)


def _soup_case():
    """40,000 disjoint triangles of about one pixel (own vertices each) over
    64x64: a block of 256 pixels sees up to 234 distinct triangles (702
    vertices), more than the backward's 512-entry LDS table holds, so part
    of its vertex gradients take the direct-atomic path."""
    sc = scenegen.make_moving_soup(seed=36, n_tris=40000, width=64, height=64, alpha=2.0, roll=(1.0, 0.0),
                                   yaw_deg_s=300.0, obj_speed=2.0, side=(0.05, 0.12),
                                   centre_lo=(-2.0, -2.0, 2.0), centre_hi=(2.0, 2.0, 3.0))
    m = sc.meshes[0]
    rng = np.random.default_rng(37)
    noise = rng.normal(0.0, 0.003, size=m.v0.shape).astype(np.float32)
    target = scenegen.Mesh(m.v0 + noise, m.v1 + noise, m.tri, m.albedo)
    return _case_scene(sc, target)


@pytest.mark.parametrize('case', ['grad96', 'grad512', 'soup64'])
def test_gradients_match_fp64_reference(case):
    """grad96 (f=16, 96x96): small; grad512 (f=71, 512x512): the
    differentiation workload at full size (100,820 triangles, rolling +
    foveated, moving camera); soup64: see _soup_case."""
    c = {'grad96': lambda: _case(96, 16), 'grad512': lambda: _case(512, 71), 'soup64': _soup_case}[case]()
    if case == 'soup64':
        ids, tri = c['oid'], c['sc'].meshes[0].tri
        most = max(len(np.unique(tri[seg[seg >= 0]])) for seg in np.split(ids, len(ids) // 256))
        assert most > 512, most
    assert abs(c['gpu_L'] - c['L']) <= 1e-4 * c['L']
    for name, g, ref in [('dv0', c['dv0'], c['g0']), ('dv1', c['dv1'], c['g1']),
                         ('dpose0', c['dp0'], c['gp0']), ('dpose1', c['dp1'], c['gp1'])]:
        bad, rel = _close(g, ref)
        nz = np.abs(ref) > 1e-3 * np.abs(ref).max()
        print(f'\n{name}: {bad.sum()} of {bad.size} outside tolerance; '
              f'median rel err of significant components {np.median(rel[nz]):.2e}, max {rel[nz].max():.2e}',
              flush=True)
        assert np.abs(ref).max() > 0
        assert not bad.any(), (name, np.argwhere(bad)[:5], g[bad][:5], ref[bad][:5])


def test_autograd_function_matches_library_backward():
    torch = _torch()
    from paper_1806_05385_amd.render import PerceptualRender, Renderer
    sc = scenegen.make_grad(seed=5, size=96, f=16)
    r = Renderer(sc.meshes, sc.views, tile=16, light=sc.light_dir, ambient=sc.ambient)
    m = r.meshes[0]
    v0 = m.v0.clone().requires_grad_(True)
    v1 = m.v1.clone().requires_grad_(True)
    p0 = torch.tensor(np.array([sc.views[0].pose0]), dtype=torch.float32, requires_grad=True)
    p1 = torch.tensor(np.array([sc.views[0].pose1]), dtype=torch.float32, requires_grad=True)
    rgb = PerceptualRender.apply(r, v0, v1, p0, p1)
    target = torch.rand(rgb.shape, generator=torch.Generator(device='cuda').manual_seed(0), device='cuda')
    loss = ((rgb - target) ** 2).sum()
    loss.backward()
    dv0, dv1, dp0, dp1 = r.backward([2.0 * (rgb[0].detach() - target[0])], ids=[r.outputs[0]['id']])
    # two runs differ only in the order of FP32 atomic additions
    for g, ref in [(v0.grad, dv0[0]), (v1.grad, dv1[0]), (p0.grad, dp0.cpu()), (p1.grad, dp1.cpu())]:
        assert torch.allclose(g, ref, rtol=1e-4, atol=1e-5 * float(ref.abs().max()))
    assert p0.grad.abs().max() > 0 and v0.grad.abs().max() > 0


def test_translation_identity_on_device():
    """sum_v dL/dv0_v = R0^T dL/dT0 holds for the device gradients too."""
    c = _case(96, 16)
    from scipy.spatial.transform import Rotation
    v = c['sc'].views[0]
    R0 = Rotation.from_rotvec(np.asarray(v.pose0[:3], np.float64)).as_matrix()
    lhs = c['dv0'].astype(np.float64).sum(0)
    rhs = R0.T @ c['dp0'][3:].astype(np.float64)
    assert np.abs(lhs - rhs).max() <= 1e-4 * np.abs(rhs).max()


def test_backward_after_a_second_forward():
    """A second forward on the same renderer with other poses and vertices
    (a target render, a second loss term) runs before the backward of the
    first: the gradients are still those of the first forward's own
    geometry and poses, checked against the FP64 reference at the 1e-3
    rule.  The loss is linear, sum(w * rgb), so both sides take the same
    upstream gradient w (the oracle's L2 loss with target c - w/2)."""
    torch = _torch()
    from paper_1806_05385_amd.render import PerceptualRender, Renderer
    sc = scenegen.make_grad(seed=5, size=96, f=16)
    mesh, view = sc.meshes[0], sc.views[0]
    r = Renderer(sc.meshes, sc.views, tile=16, light=sc.light_dir, ambient=sc.ambient)
    m = r.meshes[0]
    v0 = m.v0.clone().requires_grad_(True)
    v1 = m.v1.clone().requires_grad_(True)
    p0 = torch.tensor(np.array([view.pose0]), dtype=torch.float32, requires_grad=True)
    p1 = torch.tensor(np.array([view.pose1]), dtype=torch.float32, requires_grad=True)
    rgb = PerceptualRender.apply(r, v0, v1, p0, p1)
    ids = r.outputs[0]['id'].cpu().numpy().ravel().copy()
    # the second forward: shifted vertices and poses
    q0 = (p0.detach() + torch.tensor([[0.01, -0.02, 0.0, 0.05, 0.0, 0.1]])).requires_grad_(True)
    q1 = (p1.detach() + torch.tensor([[0.0, 0.02, 0.01, -0.05, 0.02, 0.0]])).requires_grad_(True)
    rgb2 = PerceptualRender.apply(r, v0.detach() * 1.01, v1.detach() * 0.99, q0, q1)
    assert not torch.equal(rgb, rgb2)
    w = torch.rand(rgb.shape, generator=torch.Generator(device='cuda').manual_seed(3), device='cuda')
    (rgb * w).sum().backward()
    light = oracle.light_block(sc)
    orc = oracle.Oracle(mesh, view)
    c_ref = orc.shade(ids, light)
    wn = w[0].detach().cpu().numpy().astype(np.float64).reshape(-1, 3)
    _, g0, g1, gp0, gp1 = orc.loss_grad(ids, light, c_ref - 0.5 * wn)
    assert (ids >= 0).sum() > 2000
    for name, g, ref in [('dv0', v0.grad, g0), ('dv1', v1.grad, g1), ('dpose0', p0.grad[0], gp0),
                         ('dpose1', p1.grad[0], gp1)]:
        bad, _ = _close(g.detach().cpu().numpy(), ref)
        assert np.abs(ref).max() > 0
        assert not bad.any(), (name, np.argwhere(bad)[:5])
