"""Textbook half-space triangle rasteriser (Pineda-style edge functions in
screen space, perspective-correct depth) -- TEST INFRASTRUCTURE ONLY.

This is the independent "common rasterization" special case the paper
contrasts with (Sec. 3.1.1: constant density; Sec. 3.1.2 with no rolling):
with the identity foveation and a single instant, the brute-force ray-cast
oracle must agree with it.  It shares no code with the oracle: it works on
projected 2D pixel coordinates, evaluates 2D edge functions at pixel centres
and interpolates 1/z with screen-space barycentrics.

Inputs are view-space vertex positions (x right, y up, +z forward), pinhole
intrinsics and the image size.  Every vertex must lie in front of the eye.
"""
from __future__ import annotations

import numpy as np


def raster(P: np.ndarray, tri: np.ndarray, W: int, H: int, fx: float, fy: float,
           cx: float = 0.0, cy: float = 0.0, znear: float = 0.05, cols=None, bary: bool = False):
    """Rasterise view-space triangles.  Returns (id [H,W] int32, z [H,W] float64);
    misses are -1 / +inf.  Exact depth ties keep the lower triangle index.
    ``cols``: optional iterable of pixel columns to restrict the work to.
    ``bary``: also return perspective-correct barycentrics [H,W,3] of the
    visible triangle (screen weights divided by vertex depth, renormalised)."""
    P = np.asarray(P, np.float64)
    tri = np.asarray(tri, np.int64)
    Z = P[:, 2]
    if np.any(Z <= 0):
        raise ValueError('classic raster needs every vertex in front of the eye')
    # screen coordinates: pixel (i, j) has its centre at (i + 1/2, j + 1/2)
    sx = (fx * P[:, 0] / Z + cx + 1.0) * 0.5 * W
    sy = (1.0 - (fy * P[:, 1] / Z + cy)) * 0.5 * H
    zbuf = np.full((H, W), np.inf)
    ibuf = np.full((H, W), -1, np.int32)
    bbuf = np.zeros((H, W, 3))
    colmask = None
    if cols is not None:
        colmask = np.zeros(W, bool)
        colmask[list(cols)] = True
    for f in range(tri.shape[0]):
        a, b, c = tri[f]
        xa, ya, xb, yb, xc, yc = sx[a], sy[a], sx[b], sy[b], sx[c], sy[c]
        area = (xb - xa) * (yc - ya) - (yb - ya) * (xc - xa)
        if area == 0.0:
            continue
        i0 = max(int(np.floor(min(xa, xb, xc) - 0.5)), 0)
        i1 = min(int(np.ceil(max(xa, xb, xc) - 0.5)), W - 1)
        j0 = max(int(np.floor(min(ya, yb, yc) - 0.5)), 0)
        j1 = min(int(np.ceil(max(ya, yb, yc) - 0.5)), H - 1)
        if i0 > i1 or j0 > j1:
            continue
        px = np.arange(i0, i1 + 1) + 0.5
        py = np.arange(j0, j1 + 1) + 0.5
        X, Y = np.meshgrid(px, py)
        # 2D edge functions; barycentric weight of a vertex = opposite edge / area
        wa = (xc - xb) * (Y - yb) - (yc - yb) * (X - xb)
        wb = (xa - xc) * (Y - yc) - (ya - yc) * (X - xc)
        wc = (xb - xa) * (Y - ya) - (yb - ya) * (X - xa)
        inside = ((wa >= 0) & (wb >= 0) & (wc >= 0)) | ((wa <= 0) & (wb <= 0) & (wc <= 0))
        if colmask is not None:
            inside &= colmask[i0:i1 + 1][None, :]
        if not inside.any():
            continue
        la, lb, lc = wa / area, wb / area, wc / area
        invz = la / Z[a] + lb / Z[b] + lc / Z[c]
        with np.errstate(divide='ignore'):
            z = 1.0 / invz
        sub_z = zbuf[j0:j1 + 1, i0:i1 + 1]
        sub_i = ibuf[j0:j1 + 1, i0:i1 + 1]
        upd = inside & (z >= znear) & (z < sub_z)
        sub_z[upd] = z[upd]
        sub_i[upd] = f
        if bary:
            pc = np.stack([la / Z[a], lb / Z[b], lc / Z[c]], axis=-1)
            pc /= pc.sum(axis=-1, keepdims=True)
            bbuf[j0:j1 + 1, i0:i1 + 1][upd] = pc[upd]
    if bary:
        return ibuf, zbuf, bbuf
    return ibuf, zbuf


def sample(P: np.ndarray, tri: np.ndarray, pts: np.ndarray, fx: float, fy: float,
           cx: float = 0.0, cy: float = 0.0, znear: float = 0.05):
    """Half-space test of every triangle at arbitrary display points given in
    NDC (``pts`` [n, 2]); returns (id [n], z [n]).  Same projection, 2D edge
    functions and 1/z interpolation as ``raster``; used for foveated images,
    whose pixels sample the display at the unfoveated points."""
    P = np.asarray(P, np.float64)
    tri = np.asarray(tri, np.int64)
    Z = P[:, 2]
    if np.any(Z <= 0):
        raise ValueError('classic sampler needs every vertex in front of the eye')
    sx = fx * P[:, 0] / Z + cx
    sy = fy * P[:, 1] / Z + cy
    X, Y = pts[:, 0], pts[:, 1]
    zbuf = np.full(len(pts), np.inf)
    ibuf = np.full(len(pts), -1, np.int32)
    for f in range(tri.shape[0]):
        a, b, c = tri[f]
        xa, ya, xb, yb, xc, yc = sx[a], sy[a], sx[b], sy[b], sx[c], sy[c]
        area = (xb - xa) * (yc - ya) - (yb - ya) * (xc - xa)
        if area == 0.0:
            continue
        wa = (xc - xb) * (Y - yb) - (yc - yb) * (X - xb)
        wb = (xa - xc) * (Y - yc) - (ya - yc) * (X - xc)
        wc = (xb - xa) * (Y - ya) - (yb - ya) * (X - xa)
        inside = ((wa >= 0) & (wb >= 0) & (wc >= 0)) | ((wa <= 0) & (wb <= 0) & (wc <= 0))
        if not inside.any():
            continue
        invz = (wa / Z[a] + wb / Z[b] + wc / Z[c]) / area
        with np.errstate(divide='ignore'):
            z = 1.0 / invz
        upd = inside & (z >= znear) & (z < zbuf)
        zbuf[upd] = z[upd]
        ibuf[upd] = f
    return ibuf, zbuf
