"""Parity of GPU ids/depths against the FP64 oracle.

IDs must match exactly except at listed pixels where several answers are
correct within the stated precision:
  * near-edge: the oracle's winner, or the GPU's winner evaluated by the
    oracle, has a normalised edge magnitude below 1e-6 (the ray grazes an
    edge plane to within 1e-6 rad);
  * depth tie: the GPU chose the oracle's runner-up and the two depths agree
    to 1e-5 relative;
  * near plane: the winner's depth is within 1e-5 relative of znear.
Depth must match to 1e-5 relative where the ids agree, except at listed
grazing pixels: when the ray meets the triangle's plane at an angle whose
cosine is c, rounding the ray direction to FP32 alone (relative 2^-24)
moves the depth by about 2^-24 / c, so there the bound is 16 * 2^-24 / c,
with c floored at 1e-3 (the bound never exceeds 9.6e-4 relative).  Grazing
pixels count against the same exemption budget as the id mismatches.
"""
from __future__ import annotations

import numpy as np

EHAT_TOL = 1e-6
DEPTH_TOL = 1e-5
EPS32 = 2.0 ** -24
GRAZE_K = 16.0
GRAZE_COS_FLOOR = 1e-3


def compare(orc, o, gid, gdepth, pix, znear):
    """o: oracle render dict at pixels ``pix``; gid / gdepth: GPU values at
    the same pixels.  Returns a report dict; report['bad'] lists unexplained
    mismatches as (pixel, oracle id, gpu id)."""
    gid = np.asarray(gid, np.int64)
    gdepth = np.asarray(gdepth, np.float64)
    oid = o['id'].astype(np.int64)
    mism = np.nonzero(oid != gid)[0]
    rep = dict(n=len(pix), mismatch=len(mism), near_edge=0, depth_tie=0, near_plane=0, bad=[])
    if len(mism):
        g = gid[mism]
        hit, z, eh = orc.eval_many(pix[mism], np.maximum(g, 0))
        for n, q in enumerate(mism):
            if oid[q] >= 0 and o['ehat'][q] < EHAT_TOL:
                rep['near_edge'] += 1
                continue
            if g[n] >= 0 and eh[n] < EHAT_TOL:
                rep['near_edge'] += 1
                continue
            if oid[q] >= 0 and g[n] >= 0 and g[n] == o['id2'][q] and \
                    abs(o['z2'][q] - o['z'][q]) <= DEPTH_TOL * o['z'][q]:
                rep['depth_tie'] += 1
                continue
            zs = [o['z'][q]] if oid[q] >= 0 else []
            if g[n] >= 0:
                zs.append(z[n])
            if any(abs(zz - znear) <= DEPTH_TOL * znear for zz in zs):
                rep['near_plane'] += 1
                continue
            rep['bad'].append((int(pix[q]), int(oid[q]), int(g[n])))
    same = np.nonzero((oid == gid) & (oid >= 0))[0]
    rel = np.abs(gdepth[same] - o['z'][same]) / o['z'][same]
    rep['grazing'] = 0
    rep['depth_bad'] = []
    over = rel > DEPTH_TOL
    if over.any():
        q = same[over]
        _, _, _, cs = orc.eval_many(pix[q], oid[q], with_cos=True)
        for n, qq in enumerate(q):
            if rel[over][n] <= GRAZE_K * EPS32 / max(cs[n], GRAZE_COS_FLOOR):
                rep['grazing'] += 1
            else:
                rep['depth_bad'].append((int(pix[qq]), int(oid[qq]), float(rel[over][n]), float(cs[n])))
        rel = rel[~over]
    rep['depth_max_rel'] = float(rel.max()) if rel.size else 0.0
    miss = (oid == gid) & (oid < 0)
    rep['miss_depth_inf'] = bool(np.all(np.isinf(gdepth[miss]))) if miss.any() else True
    rep['hits'] = int((oid >= 0).sum())
    return rep


def assert_parity(rep, max_exempt_frac=0.01):
    assert not rep['bad'], f"{len(rep['bad'])} unexplained id mismatches, e.g. {rep['bad'][:5]}; {rep}"
    assert not rep['depth_bad'], f"depth off at {len(rep['depth_bad'])} pixels, e.g. {rep['depth_bad'][:5]}"
    assert rep['depth_max_rel'] <= DEPTH_TOL, rep
    assert rep['miss_depth_inf'], rep
    assert rep['mismatch'] + rep['grazing'] <= max_exempt_frac * rep['n'] + 5, rep
