// pr_display.hip -- display unfoveation (Sec. 3.1.1 "Display"): the
// foveated image of each view, whose pixel grid lives in the foveated
// domain, resampled to the display's regular grid.  Included by pr_api.hip
// (one translation unit).
//
// A display pixel (a, b) has display NDC x = (2(a+1/2)/Wd - 1,
// 1 - 2(b+1/2)/Hd); its foveated NDC y = foveate(x) = f + (x - f) s,
// s = (|x - f| / R)^(1/alpha - 1) (the inverse of the ray cast's unfoveate
// map); its continuous foveated pixel coordinates are u = ((y0+1)/2 W - 1/2,
// (1-y1)/2 H - 1/2), texel centres at integers.
//
//   MIP form: a pyramid of the foveated image (level k+1 = 2x2 box mean of
//   level k, sizes halved rounding up, the last row / column repeated) is
//   sampled at u with the level of detail lambda = log2 of the longer image
//   of a display pixel step in foveated pixels: lambda <= 0 (the display
//   magnifies) Catmull-Rom interpolation of level 0; 0 < lambda < 1 its
//   linear blend with the bilinear sample of level 1; lambda >= 1
//   trilinear; edges clamped.
//   Filter form: the 5 x 5 foveated pixels around the nearest one to u,
//   each weighted by exp(-d^2 / (2 sigma^2)) with d the distance in display
//   pixels from the display pixel to the pixel's unfoveated centre,
//   normalised.
//
// Kernels (all views of a call in one launch each):
//   k_disp_views  the per-view table (sizes, foveation, pyramid offsets)
//   k_mip_tile    levels 1..5 of one 32 x 32 tile of level 0, through LDS
//   k_mip_top     levels 6.. of one view (its level 5 fits one block's LDS)
//   k_unfov       one lane per display pixel, 32 x 8 pixels per block
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pr.h"

namespace prd {

constexpr int kMaxLevels = 16;   // 16384 pixels halve to 1 in 15 steps
constexpr int kTileLevels = 5;   // levels built per 32 x 32 tile
constexpr int kDispViewsPerWrite = 4;

// One view as the display kernels see it.
struct DispView {
    int32_t W, H, Wd, Hd;        // foveated image, display
    int32_t mode, nlev;          // PR_UNFOV_*, pyramid levels (MIP form)
    int32_t tiles_x, tiles_y;    // 32 x 32 tiles of level 0
    float fov0, fov1, e, invR;   // fovea, 1 / alpha, 1 / R
    float inv2s2, pad;           // filter form: 1 / (2 sigma^2)
    int32_t powmode;             // 0: alpha == 1, 1: alpha == 2, 2: general, 3: tabulated p_c
    int32_t blk0;                // first display block (32 x 8 pixels)
    int32_t tile0;               // first 32 x 32 tile (pyramid build)
    int32_t ntab;                // samples of a tabulated p_c (powmode 3)
    int32_t lw[kMaxLevels], lh[kMaxLevels];
    int64_t loff[kMaxLevels];    // float4 offset of level k >= 1 in the pyramid
    float tab[PR_PROFILE_MAX];   // p_c samples (powmode 3; the lens is undone by the optics)
};

struct DispTable {
    int32_t nv, total_blocks, total_tiles, pad;
    int32_t blk0[PR_MAX_VIEWS + 1];
    int32_t tile0[PR_MAX_VIEWS + 1];
    DispView v[PR_MAX_VIEWS];
};

struct DispPack {
    int32_t first, count, nv, total_blocks, total_tiles, pad[3];
    DispView v[kDispViewsPerWrite];
};
static_assert(sizeof(DispPack) <= 4096, "kernel arguments are limited to 4 KiB");

struct DispIO {
    const uint8_t *fov[PR_MAX_VIEWS];
    uint8_t *out[PR_MAX_VIEWS];
};

__device__ __forceinline__ int find_base(const int32_t *base, int nv, int key) {
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= key) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_disp_views(DispPack p, DispTable *__restrict__ T) {
    const int i = threadIdx.x;
    if (i < p.count) {
        T->v[p.first + i] = p.v[i];
        T->blk0[p.first + i] = p.v[i].blk0;
        T->tile0[p.first + i] = p.v[i].tile0;
    }
    if (i == 0 && p.first + p.count == p.nv) {
        T->nv = p.nv;
        T->total_blocks = p.total_blocks;
        T->total_tiles = p.total_tiles;
        T->blk0[p.nv] = p.total_blocks;
        T->tile0[p.nv] = p.total_tiles;
    }
}

__device__ __forceinline__ float4 unpack8(uint32_t w) {
    const float k = 1.0f / 255.0f;
    return make_float4((float)(w & 0xFFu) * k, (float)((w >> 8) & 0xFFu) * k, (float)((w >> 16) & 0xFFu) * k,
                       (float)(w >> 24) * k);
}
__device__ __forceinline__ float4 f4add(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ __forceinline__ float4 f4mul(float4 a, float s) { return make_float4(a.x * s, a.y * s, a.z * s, a.w * s); }
__device__ __forceinline__ float4 f4fma(float4 a, float s, float4 c) {
    return make_float4(fmaf(a.x, s, c.x), fmaf(a.y, s, c.y), fmaf(a.z, s, c.z), fmaf(a.w, s, c.w));
}

// ---------------------------------------------------------------------------
// pyramid
// ---------------------------------------------------------------------------
// Level 0 texel (i, j) of a view, clamped to the image.
__device__ __forceinline__ float4 lev0(const DispView &d, const uint8_t *__restrict__ img, int i, int j) {
    i = min(max(i, 0), d.W - 1);
    j = min(max(j, 0), d.H - 1);
    return unpack8(reinterpret_cast<const uint32_t *>(img)[(int64_t)j * d.W + i]);
}

// One block (256 threads) per 32 x 32 tile of level 0: level 1 (16 x 16)
// from level 0, then levels 2..5 from the previous level in LDS; every
// level's texels of the tile are stored.  A texel of level k + 1 averages
// level-k texels 2i, 2i + 1 (and rows), the index clamped to level k's last
// one, which lies in the same tile.
__global__ __launch_bounds__(256) void k_mip_tile(const DispTable *__restrict__ T, DispIO io,
                                                  float4 *__restrict__ pyr) {
    __shared__ float4 s[2][16 * 16];
    const int v = find_base(T->tile0, T->nv, blockIdx.x);
    const DispView &d = T->v[v];
    if (d.mode != PR_UNFOV_MIP || d.nlev < 2) return;
    const int t = blockIdx.x - d.tile0;
    const int tx = t % d.tiles_x, ty = t / d.tiles_x;
    const int li = threadIdx.x & 15, lj = threadIdx.x >> 4;
    // level 1: texel (16 tx + li, 16 ty + lj)
    {
        const int i = 16 * tx + li, j = 16 * ty + lj;
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < d.lw[1] && j < d.lh[1]) {
            const int i0 = 2 * i, j0 = 2 * j, i1 = min(2 * i + 1, d.W - 1), j1 = min(2 * j + 1, d.H - 1);
            const uint8_t *img = io.fov[v];
            c = f4mul(f4add(f4add(lev0(d, img, i0, j0), lev0(d, img, i1, j0)),
                            f4add(lev0(d, img, i0, j1), lev0(d, img, i1, j1))), 0.25f);
            pyr[d.loff[1] + (int64_t)j * d.lw[1] + i] = c;
        }
        s[0][threadIdx.x] = c;
    }
    __syncthreads();
    // levels 2..5: level k of the tile has n = 32 >> k texels per side
    int src = 0;
    for (int k = 2; k <= kTileLevels && k < d.nlev; ++k) {
        const int n = 32 >> k, np = 2 * n;
        const int bi = (32 >> k) * tx, bj = (32 >> k) * ty;   // the tile's first level-k texel
        const int pw = d.lw[k - 1], ph = d.lh[k - 1];
        const int pbi = 2 * bi, pbj = 2 * bj;                 // first level-(k-1) texel of the tile
        if ((int)threadIdx.x < n * n) {
            const int ii = threadIdx.x % n, jj = threadIdx.x / n;
            const int i = bi + ii, j = bj + jj;
            if (i < d.lw[k] && j < d.lh[k]) {
                // level-(k-1) texels 2i, 2i+1 clamped to the level's last one,
                // as tile-local indices
                const int a0 = 2 * i - pbi, a1 = min(2 * i + 1, pw - 1) - pbi;
                const int b0 = 2 * j - pbj, b1 = min(2 * j + 1, ph - 1) - pbj;
                const float4 c = f4mul(f4add(f4add(s[src][b0 * np + a0], s[src][b0 * np + a1]),
                                             f4add(s[src][b1 * np + a0], s[src][b1 * np + a1])),
                                       0.25f);
                pyr[d.loff[k] + (int64_t)j * d.lw[k] + i] = c;
                s[src ^ 1][jj * n + ii] = c;
            }
        }
        __syncthreads();
        src ^= 1;
    }
}

// One block per view: levels kTileLevels + 1 .. nlev - 1 from level
// kTileLevels (at most 512 x 512 texels for a 16384 image: read from the
// pyramid, small levels through LDS once they fit).
__global__ __launch_bounds__(1024) void k_mip_top(const DispTable *__restrict__ T, float4 *__restrict__ pyr) {
    const int v = blockIdx.x;
    if (v >= T->nv) return;
    const DispView &d = T->v[v];
    if (d.mode != PR_UNFOV_MIP) return;
    for (int k = kTileLevels + 1; k < d.nlev; ++k) {
        const int w = d.lw[k], h = d.lh[k], pw = d.lw[k - 1], ph = d.lh[k - 1];
        const float4 *p = pyr + d.loff[k - 1];
        for (int e = threadIdx.x; e < w * h; e += blockDim.x) {
            const int i = e % w, j = e / w;
            const int i0 = 2 * i, j0 = 2 * j, i1 = min(2 * i + 1, pw - 1), j1 = min(2 * j + 1, ph - 1);
            pyr[d.loff[k] + e] = f4mul(f4add(f4add(p[(int64_t)j0 * pw + i0], p[(int64_t)j0 * pw + i1]),
                                             f4add(p[(int64_t)j1 * pw + i0], p[(int64_t)j1 * pw + i1])),
                                       0.25f);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// sampling
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 lev(const DispView &d, const float4 *__restrict__ pyr, int k, int i, int j) {
    i = min(max(i, 0), d.lw[k] - 1);
    j = min(max(j, 0), d.lh[k] - 1);
    return pyr[d.loff[k] + (int64_t)j * d.lw[k] + i];
}

__device__ __forceinline__ float4 bilinear(const DispView &d, const uint8_t *__restrict__ img,
                                           const float4 *__restrict__ pyr, int k, float u0, float u1) {
    const float sc = ldexpf(1.0f, -k);
    const float x = fmaf(u0 + 0.5f, sc, -0.5f), y = fmaf(u1 + 0.5f, sc, -0.5f);
    const float fx = floorf(x), fy = floorf(y);
    const float tx = x - fx, ty = y - fy;
    const int i = (int)fx, j = (int)fy;
    float4 c00, c10, c01, c11;
    if (k == 0) {
        c00 = lev0(d, img, i, j); c10 = lev0(d, img, i + 1, j);
        c01 = lev0(d, img, i, j + 1); c11 = lev0(d, img, i + 1, j + 1);
    } else {
        c00 = lev(d, pyr, k, i, j); c10 = lev(d, pyr, k, i + 1, j);
        c01 = lev(d, pyr, k, i, j + 1); c11 = lev(d, pyr, k, i + 1, j + 1);
    }
    const float4 r0 = f4fma(c00, 1.0f - tx, f4mul(c10, tx)), r1 = f4fma(c01, 1.0f - tx, f4mul(c11, tx));
    return f4fma(r0, 1.0f - ty, f4mul(r1, ty));
}

// Catmull-Rom weights of the taps at offsets -1, 0, 1, 2 from floor(u).
__device__ __forceinline__ void catmull_rom(float t, float w[4]) {
    const float t2 = t * t, t3 = t2 * t;
    w[0] = 0.5f * (-t + 2.0f * t2 - t3);
    w[1] = 0.5f * (2.0f - 5.0f * t2 + 3.0f * t3);
    w[2] = 0.5f * (t + 4.0f * t2 - 3.0f * t3);
    w[3] = 0.5f * (-t2 + t3);
}

__device__ __forceinline__ float4 cubic0(const DispView &d, const uint8_t *__restrict__ img, float u0, float u1) {
    const float fx = floorf(u0), fy = floorf(u1);
    float wx[4], wy[4];
    catmull_rom(u0 - fx, wx);
    catmull_rom(u1 - fy, wy);
    const int i = (int)fx - 1, j = (int)fy - 1;
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        float4 r = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int a = 0; a < 4; ++a) r = f4fma(lev0(d, img, i + a, j + b), wx[a], r);
        c = f4fma(r, wy[b], c);
    }
    return c;
}

// (rho / R)^(p) for the power modes (p = e - 1 or alpha - 1 written out).
__device__ __forceinline__ float fov_scale(const DispView &d, float rho, float pw) {
    const float q = rho * d.invR;
    return powf(q, pw);
}

// Numeric inverse of the tabulated p_c (the segment bracketing u, found by
// binary search over the samples, then linear).
__device__ __forceinline__ float tab_inv(const DispView &d, float u) {
    const int n = d.ntab;
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d.tab[mid] <= u) lo = mid; else hi = mid - 1;
    }
    const float a = d.tab[lo], b = d.tab[lo + 1];
    return ((float)lo + (u - a) / (b - a)) / (float)(n - 1);
}

// Foveated position of display NDC x, and the foveation Jacobian.
__device__ __forceinline__ void foveate_j(const DispView &d, float x0, float x1, float &y0, float &y1, float JF[4]) {
    const float d0 = x0 - d.fov0, d1 = x1 - d.fov1;
    const float rho2 = d0 * d0 + d1 * d1;
    if (d.powmode == 3) {
        // tabulated p_c: y - f = (x - f) p_c(s)/s, s = |x - f|/R; Jacobian
        // (p_c/s) I + (p_c' - p_c/s) n n^T, n the unit direction
        const int n = d.ntab;
        const float rho = __builtin_amdgcn_sqrtf(rho2), sp = rho * d.invR;
        const float q = sp * (float)(n - 1);
        const int k = q >= (float)(n - 2) ? n - 2 : (int)q;
        const float a = d.tab[k], b = d.tab[k + 1], slope = (b - a) * (float)(n - 1);
        if (rho2 == 0.0f) {
            y0 = x0; y1 = x1;
            JF[0] = slope; JF[1] = 0.f; JF[2] = 0.f; JF[3] = slope;
            return;
        }
        const float s = fmaf(q - (float)k, b - a, a) / sp;
        y0 = fmaf(d0, s, d.fov0);
        y1 = fmaf(d1, s, d.fov1);
        const float g = (slope - s) / rho2;
        JF[0] = fmaf(g, d0 * d0, s);
        JF[1] = g * d0 * d1;
        JF[2] = JF[1];
        JF[3] = fmaf(g, d1 * d1, s);
        return;
    }
    if (d.powmode == 0) {
        y0 = x0; y1 = x1;
        JF[0] = 1.f; JF[1] = 0.f; JF[2] = 0.f; JF[3] = 1.f;
        return;
    }
    if (rho2 == 0.0f) {
        y0 = x0; y1 = x1;
        JF[0] = INFINITY; JF[1] = 0.f; JF[2] = 0.f; JF[3] = INFINITY;
        return;
    }
    const float rho = __builtin_amdgcn_sqrtf(rho2);
    // alpha = 2: s = (rho/R)^(-1/2)
    const float s = d.powmode == 1 ? __builtin_amdgcn_rsqf(rho * d.invR) : fov_scale(d, rho, d.e - 1.0f);
    y0 = fmaf(d0, s, d.fov0);
    y1 = fmaf(d1, s, d.fov1);
    const float g = (d.e - 1.0f) * s / rho2;
    JF[0] = fmaf(g, d0 * d0, s);
    JF[1] = g * d0 * d1;
    JF[2] = JF[1];
    JF[3] = fmaf(g, d1 * d1, s);
}

// Display NDC of foveated texel (i, j)'s centre (the ray cast's unfoveate).
__device__ __forceinline__ void unfoveate_texel(const DispView &d, int i, int j, float &x0, float &x1) {
    const float y0 = (float)(2 * i + 1) / (float)d.W - 1.0f, y1 = 1.0f - (float)(2 * j + 1) / (float)d.H;
    const float d0 = y0 - d.fov0, d1 = y1 - d.fov1;
    float s = 1.0f;
    if (d.powmode == 3) {
        const float rho = __builtin_amdgcn_sqrtf(d0 * d0 + d1 * d1), sf = rho * d.invR;
        s = rho > 0.0f ? tab_inv(d, sf) / sf : 1.0f;
    } else if (d.powmode != 0) {
        const float rho = __builtin_amdgcn_sqrtf(d0 * d0 + d1 * d1);
        s = d.powmode == 1 ? rho * d.invR : (rho > 0.0f ? fov_scale(d, rho, 1.0f / d.e - 1.0f) : 0.0f);
    }
    x0 = fmaf(d0, s, d.fov0);
    x1 = fmaf(d1, s, d.fov1);
}

__global__ __launch_bounds__(256) void k_unfov(const DispTable *__restrict__ T, DispIO io,
                                               const float4 *__restrict__ pyr) {
    const int v = find_base(T->blk0, T->nv, blockIdx.x);
    const DispView &d = T->v[v];
    const int bx = (d.Wd + 31) >> 5;
    const int b = blockIdx.x - d.blk0;
    const int a = ((b % bx) << 5) + (threadIdx.x & 31), row = ((b / bx) << 3) + (threadIdx.x >> 5);
    if (a >= d.Wd || row >= d.Hd) return;
    const uint8_t *img = io.fov[v];
    const float x0 = (float)(2 * a + 1) / (float)d.Wd - 1.0f, x1 = 1.0f - (float)(2 * row + 1) / (float)d.Hd;
    float y0, y1, JF[4];
    foveate_j(d, x0, x1, y0, y1, JF);
    const float u0 = fmaf(y0 + 1.0f, 0.5f * (float)d.W, -0.5f), u1 = fmaf(1.0f - y1, 0.5f * (float)d.H, -0.5f);
    float4 c;
    if (d.mode == PR_UNFOV_MIP) {
        // du/d(a, b) = diag(W/2, -H/2) JF diag(2/Wd, -2/Hd)
        const float sa = (float)d.W / (float)d.Wd, sb = (float)d.H / (float)d.Hd;
        const float j00 = sa * JF[0], j01 = -(float)d.W / (float)d.Hd * JF[1];
        const float j10 = -(float)d.H / (float)d.Wd * JF[2], j11 = sb * JF[3];
        const float c0 = j00 * j00 + j10 * j10, c1 = j01 * j01 + j11 * j11;
        const float lam = 0.5f * __log2f(fmaxf(c0, c1));
        const int top = d.nlev - 1;
        if (!(lam > 0.0f)) {
            c = cubic0(d, img, u0, u1);
        } else if (lam < 1.0f) {
            const float4 a0 = cubic0(d, img, u0, u1);
            const float4 b1 = bilinear(d, img, pyr, top >= 1 ? 1 : 0, u0, u1);
            c = f4fma(a0, 1.0f - lam, f4mul(b1, lam));
        } else {
            const float k = floorf(lam), fr = lam - k;
            if (k >= (float)top) {
                c = bilinear(d, img, pyr, top, u0, u1);
            } else {
                const int ki = (int)k;
                const float4 a0 = bilinear(d, img, pyr, ki, u0, u1), b1 = bilinear(d, img, pyr, ki + 1, u0, u1);
                c = f4fma(a0, 1.0f - fr, f4mul(b1, fr));
            }
        }
    } else {
        const int i0 = (int)floorf(u0 + 0.5f), j0 = (int)floorf(u1 + 0.5f);
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        float ws = 0.0f;
        const float ka = 0.5f * (float)d.Wd, kb = 0.5f * (float)d.Hd;
        for (int dj = -2; dj <= 2; ++dj)
            for (int di = -2; di <= 2; ++di) {
                const int i = i0 + di, j = j0 + dj;
                if (i < 0 || i >= d.W || j < 0 || j >= d.H) continue;
                float xv0, xv1;
                unfoveate_texel(d, i, j, xv0, xv1);
                const float da = fmaf(xv0 + 1.0f, ka, -0.5f) - (float)a, db = fmaf(1.0f - xv1, kb, -0.5f) - (float)row;
                const float w = __expf(-(da * da + db * db) * d.inv2s2);
                ws += w;
                acc = f4fma(lev0(d, img, i, j), w, acc);
            }
        c = ws > 0.0f ? f4mul(acc, 1.0f / ws) : lev0(d, img, i0, j0);
    }
    uint32_t o = 0;
    const float ch[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) o |= (uint32_t)floorf(fminf(fmaxf(ch[q], 0.0f), 1.0f) * 255.0f + 0.5f) << (8 * q);
    reinterpret_cast<uint32_t *>(io.out[v])[(int64_t)row * d.Wd + a] = o;
}

}  // namespace prd
