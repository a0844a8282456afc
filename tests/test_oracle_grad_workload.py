"""The oracle's analytic frozen-visibility gradient at the differentiation
workload's full size (100,820 triangles, 512x512, foveated alpha = 2,
rolling, head yaw 120 deg/s + 0.5 m/s), against FP64 central differences
of its own loss on 200 sampled parameters: 188 vertex coordinates (start or
end position of vertices of visible triangles) and all 12 pose parameters.

The step h = 1e-3 is coarser than the scale over which this loss is smooth:
with visibility frozen, a pixel near a silhouette sees its triangle almost
edge-on, and the barycentric terms e_k / S have a pole where the ray lies in
the triangle's plane (S = 0), so a 1e-3 move of a vertex or pose can carry
S close to or across that pole.  There the difference quotient is not a
derivative.  So at h = 1e-3 the parameters whose difference quotient has
converged (it changes by at most 1e-4 relative when h is halved) are held to
the 1e-3 rule, and at h = 1e-6 every one of the 200 is (FP64 sums of
262,144 pixels keep the rounding of the quotient near 1e-9 / 2e-6).

Tolerance (the gradient rule): |fd - g| <= 1e-3 max(|g|, 1e-3 max|g|), the
floor taken over the vertex gradients or over the pose gradients."""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.slow


def test_gradient_matches_central_differences_at_full_size():
    sc = scenegen.make_grad()
    mesh, view, target = sc.meshes[0], sc.views[0], sc.extra['target']
    assert mesh.nt == 100_820 and (view.width, view.height) == (512, 512)
    light = oracle.light_block(sc)
    orc_t = oracle.Oracle(target, view)
    tgt = orc_t.shade(orc_t.render_fast()['id'], light)
    orc = oracle.Oracle(mesh, view)
    ids = orc.render_fast()['id']
    _, g0, g1, gp0, gp1 = orc.loss_grad(ids, light, tgt)
    v0, v1 = mesh.v0.astype(np.float64), mesh.v1.astype(np.float64)
    pose = [view.pose0.astype(np.float64), view.pose1.astype(np.float64)]

    def loss_at(which, what, k, d):
        a, b = v0, v1
        p = [pose[0], pose[1]]
        if what == 'v':
            a, b = v0.copy(), v1.copy()
            (a, b)[which][k // 3, k % 3] += d
        else:
            p = [pose[0].copy(), pose[1].copy()]
            p[which][k] += d
        return oracle.Oracle(mesh, view, v0=a, v1=b, pose0=p[0], pose1=p[1]).loss(ids, light, tgt)

    def fd(which, what, k, h):
        return (loss_at(which, what, k, h) - loss_at(which, what, k, -h)) / (2 * h)

    vis = np.unique(mesh.tri[ids[ids >= 0]].ravel())
    sel = np.random.default_rng(8).choice(len(vis) * 6, size=188, replace=False)
    params = [((s % 6) // 3, 'v', 3 * int(vis[s // 6]) + s % 3) for s in sel]
    params += [(w, 'p', k) for w in (0, 1) for k in range(6)]
    g = np.array([(g0, g1)[w].ravel()[k] if what == 'v' else (gp0, gp1)[w][k] for w, what, k in params])
    floor = np.where(np.arange(200) < 188, 1e-3 * max(np.abs(g0).max(), np.abs(g1).max()),
                     1e-3 * np.abs(np.concatenate([gp0, gp1])).max())

    def rel(f):
        return np.abs(f - g) / np.maximum(np.abs(g), floor)

    f_fine = np.array([fd(*p, 1e-6) for p in params])
    assert rel(f_fine).max() <= 1e-3, rel(f_fine).max()
    f_h = np.array([fd(*p, 1e-3) for p in params])
    f_h2 = np.array([fd(*p, 5e-4) for p in params])
    conv = np.abs(f_h - f_h2) / np.maximum(np.abs(f_h), floor) <= 1e-4
    print(f'\nh=1e-6: max rel {rel(f_fine).max():.2e}; h=1e-3: {int(conv.sum())} of 200 converged, '
          f'max rel there {rel(f_h)[conv].max():.2e}; {int((rel(f_h) > 1e-3).sum())} of 200 beyond 1e-3 '
          f'(pole-limited)', flush=True)
    assert conv.sum() >= 40
    assert rel(f_h)[conv].max() <= 1e-3
