"""Pins of the oracle's display unfoveation (Sec. 3.1.1 "Display") against
things other than itself: block means (the MIP pyramid), the identity
foveation (the image comes back unchanged), constants, linear ramps (every
interpolation stage reproduces a linear function of the foveated pixel
coordinates exactly), the foveation map already pinned in
test_oracle_pins.py with central differences of its own coordinates, the
closed-form stretch of the power map along a radius, and two limits of the
reconstruction filter (a narrow Gaussian picks the foveated pixel nearest
in display distance, a wide one averages the 5 x 5 neighbourhood)."""
import math

import numpy as np
import pytest

import oracle
import scenegen


def _view(W, H, fovea=(0.13, -0.07), alpha=2.0):
    return scenegen.View(W, H, np.zeros(6, np.float32), np.zeros(6, np.float32), fovea=fovea, alpha=alpha,
                         roll_dir=(0.0, 0.0))


def _img(W, H, seed=0):
    return np.random.default_rng(seed).integers(0, 256, size=(H, W, 4), dtype=np.uint8)


def test_mip_levels_are_block_means():
    """Level 1 of an even-sized image is the mean of 2x2 blocks; of an odd
    size, of the blocks of the image with its last row and column repeated;
    levels halve (rounding up) down to 1x1, whose value for a power-of-two
    square is the image mean."""
    f = _img(64, 48).astype(np.float64) / 255.0
    l1, n = oracle.mip_level(f, 1)
    assert np.abs(l1 - f.reshape(24, 2, 32, 2, 4).mean(axis=(1, 3))).max() < 1e-15
    assert n == 7     # 64x48, 32x24, 16x12, 8x6, 4x3, 2x2, 1x1
    g = _img(7, 5, 1).astype(np.float64) / 255.0
    gp = np.pad(g, ((0, 1), (0, 1), (0, 0)), mode='edge')
    l1, n = oracle.mip_level(g, 1)
    assert np.abs(l1 - gp.reshape(3, 2, 4, 2, 4).mean(axis=(1, 3))).max() < 1e-15 and n == 4
    sq = _img(32, 32, 2).astype(np.float64) / 255.0
    top, n = oracle.mip_level(sq, 5)
    assert n == 6 and top.shape == (1, 1, 4) and np.abs(top[0, 0] - sq.mean(axis=(0, 1))).max() < 1e-14


def test_identity_foveation_returns_the_image():
    """alpha = 1 and a display of the foveated image's size: every display
    pixel samples its own foveated pixel centre at level of detail 0."""
    W, H = 37, 29
    v = _view(W, H, alpha=1.0)
    f = _img(W, H, 3)
    out = oracle.unfoveate_image(v, f, W, H, oracle.UNFOV_MIP)
    assert np.abs(out - f.reshape(-1, 4) / 255.0).max() < 1e-12
    u, J, lod = oracle.unfov_coord(v, W, H, 11.0, 7.0)
    assert np.abs(u - [11.0, 7.0]).max() < 1e-12 and abs(lod) < 1e-12


@pytest.mark.parametrize('mode', [oracle.UNFOV_MIP, oracle.UNFOV_FILTER])
def test_constant_image_stays_constant(mode):
    v = _view(45, 38, fovea=(-0.15, 0.1), alpha=2.5)
    f = np.empty((38, 45, 4))
    f[:] = [0.2, 0.55, 0.9, 1.0]
    out = oracle.unfoveate_image(v, f, 60, 50, mode, 0.7)
    assert np.abs(out - [0.2, 0.55, 0.9, 1.0]).max() < 1e-12


def test_coordinates_follow_the_foveation_map():
    """u is the foveated pixel position of the display pixel's centre (the
    foveation map pinned in test_oracle_pins.py), and its Jacobian matches
    central differences of u in the display pixel coordinates."""
    W, H, Wd, Hd = 80, 64, 100, 90
    v = _view(W, H, fovea=(0.2, -0.1), alpha=2.0)
    h = 1e-5
    for a, b in [(3.0, 5.0), (50.0, 40.0), (99.0, 0.0), (61.0, 33.0)]:
        u, J, _ = oracle.unfov_coord(v, Wd, Hd, a, b)
        x = np.array([2 * (a + 0.5) / Wd - 1, 1 - 2 * (b + 0.5) / Hd])
        y = oracle.foveate(v, x)
        assert np.abs(u - [(y[0] + 1) / 2 * W - 0.5, (1 - y[1]) / 2 * H - 0.5]).max() < 1e-12
        for c, (da, db) in enumerate([(h, 0.0), (0.0, h)]):
            up, _, _ = oracle.unfov_coord(v, Wd, Hd, a + da, b + db)
            um, _, _ = oracle.unfov_coord(v, Wd, Hd, a - da, b - db)
            assert np.abs((up - um) / (2 * h) - J[:, c]).max() < 1e-6 * np.abs(J).max()


def test_level_of_detail_closed_forms():
    """alpha = 1 with a display twice / half the image's size: lod -1 / +1.
    alpha = 2 on the row through the fovea (display and image of one size):
    the power map y = f + R (rho/R)^(1/2) along the radius stretches a
    display step by (1/2)(rho/R)^(-1/2) radially and (rho/R)^(-1/2) across,
    so lod = log2((rho/R)^(-1/2))."""
    v1 = _view(32, 32, alpha=1.0)
    assert abs(oracle.unfov_coord(v1, 64, 64, 10.0, 10.0)[2] + 1.0) < 1e-12
    assert abs(oracle.unfov_coord(v1, 16, 16, 5.0, 5.0)[2] - 1.0) < 1e-12
    W = 64
    v2 = _view(W, W, fovea=(0.0, 1.0 / W), alpha=2.0)     # fovea on row 31's centre line
    R = oracle.fovea_radius(v2)
    for a in (40.0, 55.0, 63.0):
        x0 = 2 * (a + 0.5) / W - 1
        rho = abs(x0)
        _, _, lod = oracle.unfov_coord(v2, W, W, a, 31.0)
        assert abs(lod - math.log2((rho / R) ** -0.5)) < 1e-12, a


def test_linear_ramp_is_reproduced():
    """A foveated image linear in its pixel coordinates (no clamping) comes
    back as that linear function of u at every display pixel whose samples
    stay inside the image: the block means of a ramp are the ramp at the
    blocks' centres, and bilinear, Catmull-Rom and the level blend all
    reproduce linear functions."""
    W = H = 128
    jj, ii = np.mgrid[0:H, 0:W].astype(np.float64)
    coef = np.array([[0.002, 0.001, 0.1], [-0.001, 0.003, 0.4], [0.0015, -0.002, 0.55], [0.0, 0.0, 1.0]])
    f = np.stack([c[0] * ii + c[1] * jj + c[2] for c in coef], axis=-1)
    assert f.min() > 0 and f.max() <= 1
    v = _view(W, H, fovea=(0.1, -0.05), alpha=2.0)
    Wd, Hd = 192, 176      # larger than the image: the periphery magnifies, the fovea minifies
    out = oracle.unfoveate_image(v, f, Wd, Hd, oracle.UNFOV_MIP)
    checked = mag = mini = 0
    for p in range(Wd * Hd):
        u, _, lod = oracle.unfov_coord(v, Wd, Hd, float(p % Wd), float(p // Wd))
        k = max(0, math.ceil(lod)) + 1
        margin = 2 ** (k + 1) + 2
        if lod > 4 or not (margin <= u[0] <= W - 1 - margin and margin <= u[1] <= H - 1 - margin):
            continue
        ref = coef[:, 0] * u[0] + coef[:, 1] * u[1] + coef[:, 2]
        assert np.abs(out[p] - ref).max() < 1e-12, (p, lod)
        checked += 1
        mag += lod <= 0
        mini += lod >= 1
    assert checked > 1500 and mag > 200 and mini > 200, (checked, mag, mini)


def test_reconstruction_filter_limits():
    """A narrow Gaussian (sigma 1e-3 display pixels) returns the foveated
    pixel of the 5 x 5 neighbourhood whose unfoveated centre is nearest the
    display pixel; a very wide one returns the plain mean of the
    neighbourhood's pixels inside the image."""
    W, H, Wd, Hd = 40, 36, 50, 44
    v = _view(W, H, fovea=(-0.1, 0.12), alpha=2.0)
    f = _img(W, H, 4).astype(np.float64) / 255.0
    narrow = oracle.unfoveate_image(v, f, Wd, Hd, oracle.UNFOV_FILTER, 1e-3)
    wide = oracle.unfoveate_image(v, f, Wd, Hd, oracle.UNFOV_FILTER, 1e6)
    rng = np.random.default_rng(9)
    for p in rng.choice(Wd * Hd, size=300, replace=False):
        a, b = p % Wd, p // Wd
        u, _, _ = oracle.unfov_coord(v, Wd, Hd, float(a), float(b))
        i0, j0 = int(np.floor(u[0] + 0.5)), int(np.floor(u[1] + 0.5))
        best, bd, vals = None, np.inf, []
        for j in range(j0 - 2, j0 + 3):
            for i in range(i0 - 2, i0 + 3):
                if not (0 <= i < W and 0 <= j < H):
                    continue
                x = oracle.unfoveate(v, np.array([2 * (i + 0.5) / W - 1, 1 - 2 * (j + 0.5) / H]))
                d = math.hypot((x[0] + 1) / 2 * Wd - 0.5 - a, (1 - x[1]) / 2 * Hd - 0.5 - b)
                vals.append(f[j, i])
                if d < bd:
                    best, bd = f[j, i], d
        if not vals:
            # the display pixel lies beyond the foveated image (the power map
            # with R the farthest corner's distance covers less than the
            # display square): the edge pixel nearest to u, clamped
            ic, jc = min(max(i0, 0), W - 1), min(max(j0, 0), H - 1)
            assert np.abs(wide[p] - f[jc, ic]).max() < 1e-15 and np.abs(narrow[p] - f[jc, ic]).max() < 1e-15
            continue
        assert np.abs(wide[p] - np.mean(vals, axis=0)).max() < 1e-9
        if bd < 0.05:      # the narrow limit is sharp only when one centre is clearly nearest
            assert np.abs(narrow[p] - best).max() < 1e-9, p


def test_trilinear_blend_between_levels():
    """Columns striped 1,1,0,0 (period 4), identity foveation, a display of
    width 100 for an image of width 256: every display pixel has lod
    log2(2.56) = 1 + 0.356; level 1 is then the stripes 1,0,1,0 (bilinear
    between them: a triangle wave of the level-1 coordinate) and level 2 is
    0.5, and the finer level weighs 1 - 0.356."""
    W, H, Wd, Hd = 256, 8, 100, 8
    v = _view(W, H, fovea=(0.0, 0.0), alpha=1.0)
    col = ((np.arange(W) // 2) % 2 == 0).astype(np.float64)
    f = np.zeros((H, W, 4))
    f[:, :, 0] = col[None, :]
    f[:, :, 3] = 1.0
    out = oracle.unfoveate_image(v, f, Wd, Hd, oracle.UNFOV_MIP, pix=np.arange(Wd) + 3 * Wd)
    lam = math.log2(W / Wd)
    fr = lam - 1.0
    for a in range(Wd):
        u, _, lod = oracle.unfov_coord(v, Wd, Hd, float(a), 3.0)
        assert abs(lod - lam) < 1e-12
        u1 = (u[0] + 0.5) / 2 - 0.5
        if not (0.0 <= u1 <= W / 2 - 1):
            continue
        m = u1 % 2.0                       # level-1 column 2c is 1, column 2c + 1 is 0
        tri = 1.0 - m if m <= 1.0 else m - 1.0
        assert abs(out[a, 0] - ((1 - fr) * tri + fr * 0.5)) < 1e-12, (a, u1)


def test_reconstruction_weights_follow_display_distance():
    """The filter is linear in the image, so a foveated image that is 1 at
    one pixel and 0 elsewhere returns that pixel's normalised weight.  For
    pairs of pixels of a display pixel's 5 x 5 neighbourhood the weights'
    ratio is the Gaussian's, exp(-(d_a^2 - d_b^2) / (2 sigma^2)), with d the
    distance in display pixels between the display pixel and each foveated
    pixel's unfoveated centre (computed here from the pinned foveation
    map)."""
    W, H, Wd, Hd = 40, 36, 50, 44
    sigma = 0.9
    v = _view(W, H, fovea=(-0.1, 0.12), alpha=2.0)
    checked = 0
    for p in (5 * Wd + 7, 20 * Wd + 25, 31 * Wd + 40, 12 * Wd + 33):
        a, b = p % Wd, p // Wd
        u, _, _ = oracle.unfov_coord(v, Wd, Hd, float(a), float(b))
        i0, j0 = int(np.floor(u[0] + 0.5)), int(np.floor(u[1] + 0.5))
        w, d2 = [], []
        for j, i in [(j0, i0), (j0 + 1, i0 - 1), (j0 - 2, i0 + 2), (j0, i0 + 1)]:
            if not (0 <= i < W and 0 <= j < H):
                continue
            f = np.zeros((H, W, 4))
            f[j, i] = 1.0
            w.append(oracle.unfoveate_image(v, f, Wd, Hd, oracle.UNFOV_FILTER, sigma, pix=np.array([p]))[0, 0])
            x = oracle.unfoveate(v, np.array([2 * (i + 0.5) / W - 1, 1 - 2 * (j + 0.5) / H]))
            d2.append(((x[0] + 1) / 2 * Wd - 0.5 - a) ** 2 + ((1 - x[1]) / 2 * Hd - 0.5 - b) ** 2)
        for k in range(1, len(w)):
            assert abs(math.log(w[k] / w[0]) + (d2[k] - d2[0]) / (2 * sigma ** 2)) < 1e-9
            checked += 1
    assert checked >= 8
