// pr_kernels.h -- device data layouts shared by the kernels and the host
// launcher of libpr (gfx950).
#pragma once

#include <stdint.h>

#include "pr.h"
#include "pr_geom.h"

namespace prk {

// Intersection record of one triangle, written by the bound kernel.  For
// edge o (opposite vertex o) the camera-space edge-plane normal
// c_o(t) = P_a(t) x P_b(t) = A_o + t B_o + t^2 C_o; the ray r = (rx, ry, 1)
// at time t passes edge o on the side sign(e_o), e_o = r . c_o(t).  The face
// normal N(t) = (P_1 - P_0) x (P_2 - P_0) = N0 + t N1 + t^2 N2 gives the hit
// depth z = D(t) / (r . N(t)), D(t) = P_0(t) . (P_1(t) x P_2(t)) = d0 + t d1
// + t^2 d2 + t^3 d3.  N is stored although it equals sum_o c_o: near grazing
// incidence r . N is much smaller than the edge terms and their sum would
// lose it to cancellation in FP32.  Every quantity is linear in the ray
// terms (rx, ry, t rx, t ry, t, t^2 rx, t^2 ry, t^2) plus a constant; the
// record stores, for outputs o = e_0, e_1, e_2, S = r . N, the coefficient
// matrix M[k][o] (k: ray term) at 4k + o, then the constants (A_oz, N0z),
// d0..d3 and the triangle index.  Rolling views: 11 float4 (M 32, constants
// 4 at 32, d 4 at 36, id at 40, 3 pad).  Non-rolling views (t = 0): 6 float4
// (M for terms rx, ry and two zero terms: 16, constants 4 at 16, d0 at 20,
// id at 21, 2 pad).
constexpr int kRecRoll = 11;
constexpr int kRecStatic = 6;

// Spread slots of the PR_FLAG_COUNT counters (tests, hits).
constexpr int kCountSlots = 64;

// Per-triangle bound (64 bytes).
// Per-triangle bound (64 bytes).
struct TriBound {
    int32_t rect[4];   // inclusive tile rectangle x0, y0, x1, y1 (x0 > x1: culled)
    int32_t kind;      // prg::kCulled / kWindow / kClipped
    int32_t pad;
    double w[4];       // kWindow: time window w[0..1]; kClipped: display box
    int32_t pad2[2];   // to 4 float4 (coalesced stores)
};

// Display-space box of a tile's pixel centres and its frame-time window;
// for tiles split into quadrants, the box of each quadrant (qvalid bit k:
// quadrant k holds pixels of the image).  Computed in FP64 and rounded
// outwards to FP32 (lower ends down, upper ends up), so each stored box
// contains the exact one.  96 bytes.
struct TileInfo {
    float box[4];
    float tw[2];
    int32_t qvalid;
    int32_t pad;
    float qb[4][4];
};

// Tile-list entry: triangle index in bits 0..27, quadrant mask in 28..31.
constexpr int kListTriBits = 28;
constexpr uint32_t kListTriMask = (1u << kListTriBits) - 1u;

// A view's tabulated profiles in the workspace (pr_profile's samples).
struct ProfDev {
    int32_t nc, nl, pad[2];
    float c[PR_PROFILE_MAX];   // p_c samples (nc >= 2: tabulated foveation)
    float l[PR_PROFILE_MAX];   // p_l samples (nl >= 2: lens)
};

// Per-pixel constants of a view (FP32 setup in the ray cast and shading).
struct PixelConst {
    float invW2, invH2;    // 2/W, 2/H
    float fov0, fov1, invR, alpha;
    float roll0, roll1;
    float cx, cy, invfx, invfy;
    float znear;
    int W, H;
    int mode;              // 0: alpha == 1, 1: alpha == 2, 2: general power, 3: tabulated p_c
    int lens;              // a tabulated lens p_l follows the foveation
    const ProfDev *prof;   // the view's profiles (modes 3 and lens)
};

// One view as the kernels see it (lives in the workspace's view table).
struct ViewDev {
    pr_view view;
    pr_mesh mesh;
    PixelConst pc;
    int32_t tile, tiles_x, tiles_y, ntiles;
    int32_t tile_base;     // global index of the view's first tile
    int32_t tri_block0;    // first 256-triangle block (bound and bin grids)
    int32_t pix_block0;    // first 256-pixel block (shade and backward grids)
    int32_t rec_w;         // float4 per record
    int32_t rolling;
    int32_t bound;         // rolling bound mode (prg::kBound*; pr_tuning.bound)
    int64_t rec_off;       // float4 offset of the view's first record
    int64_t tri_off;       // TriBound index of the view's first triangle
    int32_t vtx_block0;    // first 256-vertex block (backward vertex pass)
    int32_t fov_bound;     // foveated per-tile test (prg::kFov*; pr_tuning.fov_bound)
    int64_t gacc_off;      // float offset of the view's backward accumulators [2][nv][3]
    float light0[3];       // R0 * light direction (written by pr_shade / pr_backward)
    float light1[3];       // R1 * light direction
    float R0f[9], T0f[3], R1f[9], T1f[3];   // FP32 copies of the poses (backward)
    prg::Geom g;           // FP64 camera geometry (written by k_write_views)
};

// Backward partial sums (FP64) of one pixel block, stored per block and
// added per view by k_bwd_pose: [0..2] sum (1-t) dL/dLw,
// [3..5] sum t dL/dLw (light direction before normalisation), [6..8] dL/dT0,
// [9..17] dL/dR0 (vertex part), [18..20] dL/dT1, [21..29] dL/dR1, 2 pad.
constexpr int kPoseAcc = 32;

struct ViewTable {
    int32_t nv, total_tiles, total_tri_blocks, total_pix_blocks;
    int32_t tri_block0[PR_MAX_VIEWS + 1];
    int32_t tile_base[PR_MAX_VIEWS + 1];
    int32_t pix_block0[PR_MAX_VIEWS + 1];
    int32_t vtx_block0[PR_MAX_VIEWS + 1];
    int32_t total_vtx_blocks;
    int32_t pad[2];
    ViewDev v[PR_MAX_VIEWS];
};

// Views written per k_write_views launch (kernel-argument size).
constexpr int kViewsPerWrite = 2;
struct ViewPack {
    int32_t first, count, nv, total_tiles, total_tri_blocks, total_pix_blocks, total_vtx_blocks;
    int32_t reset_status;   // the frame's first launch clears the status block (pr_bound, not pr_backward)
    ViewDev v[kViewsPerWrite];
};
static_assert(sizeof(ViewPack) <= 4096, "kernel arguments are limited to 4 KiB");

// Status block at the start of the workspace.
struct DevStatus {
    int32_t overflow;
    int32_t nonfinite;
    unsigned long long pairs_required;
    unsigned long long pairs_total;
    unsigned long long tests;
    unsigned long long hits;
    uint32_t pad[2];
    unsigned long long cnt[kCountSlots][2];   // ray-cast tests, hits, spread over slots
};

// Schedule of the persistent ray cast.  Every tile belongs to one XCD's
// share (64 x 64-pixel super-tiles spread over the XCDs, so the tiles that
// read a triangle's record mostly run on one XCD and share its L2); each
// share is walked longest list first (counting sort by power-of-two list
// length bucket).
constexpr int kBuckets = 33;
constexpr int kXcds = 8;
constexpr int kSchedCounters = 2 * kXcds * kBuckets + kXcds + 1;   // cleared by k_tiles
struct Sched {
    uint32_t count[kXcds][kBuckets];    // tiles per (XCD share, bucket)
    uint32_t cursor[kXcds][kBuckets];
    uint32_t ntile[kXcds];              // tiles of each share
    uint32_t ticket;                    // k_scan's block order
};
static_assert(sizeof(Sched) == 4 * kSchedCounters, "Sched is kSchedCounters words");

// Output / input pointers of the per-pixel passes, indexed by view.
struct RayOut {
    int32_t *id[PR_MAX_VIEWS];
    float *depth[PR_MAX_VIEWS];
};
struct ShadeIO {
    const int32_t *id[PR_MAX_VIEWS];
    uint8_t *rgba8[PR_MAX_VIEWS];
    float *rgb32[PR_MAX_VIEWS];
    const float *albedo[PR_MAX_VIEWS];   // per view (the albedo of its mesh)
};

struct GbufIO {
    const int32_t *id[PR_MAX_VIEWS];
    float *normal[PR_MAX_VIEWS];    // [H][W][3]
    float *bary[PR_MAX_VIEWS];      // [H][W][2]
    float *density[PR_MAX_VIEWS];   // [H][W]
};

struct BwdIO {
    const int32_t *id[PR_MAX_VIEWS];
    const float *dl[PR_MAX_VIEWS];       // dL/drgb [H][W][3]
    const float *albedo[PR_MAX_VIEWS];   // per view (the albedo of its mesh)
};
struct BwdOut {
    float *dv0[PR_MAX_VIEWS];            // per mesh
    float *dv1[PR_MAX_VIEWS];
};

}  // namespace prk
