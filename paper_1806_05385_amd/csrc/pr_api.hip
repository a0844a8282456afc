// pr_api.hip -- the C ABI declared in include/pr.h: argument checks,
// workspace layout and the launch sequence of each call.  One translation
// unit with the kernels (templates are instantiated here).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "pr.h"
#include "pr_display.hip"
#include "pr_kernels.hip"

using namespace prk;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxDevices = 64;   // devices a process may drive (per-device caches)
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Workspace: [status | view table | tile infos | records | triangle bounds |
// tile counts | tile offsets | scan partials | pairs | lists], 256-aligned.
struct Layout {
    int nv;
    ViewDev vd[PR_MAX_VIEWS];
    int total_tiles, total_tri_blocks, total_pix_blocks, total_vtx_blocks, nparts;
    int64_t cap, total_rec4, total_tris, total_gacc;
    size_t table, tinfo, rec, tb, bcand, bnf, bperm, boff, bpart, tcount, toff, part, pairs, lists, gacc, pacc, sched, order, prof,
        bytes;
    ProfDev prof_host[PR_MAX_VIEWS];   // the views' tabulated profiles (used where prof_used)
    bool prof_used[PR_MAX_VIEWS];
    bool any_prof;                     // some view has one (the bound kernels' general form)
    bool any_fov;                      // a foveated bound other than the exact one (the binning's general form)
};

// A view's tabulated profiles are usable: sample counts in range, samples
// finite, starting at 0 and strictly increasing; p_c(s_k) >= s_k.
bool profile_ok(const pr_profile &P) {
    if (P.n_c != 0 && (P.n_c < 2 || P.n_c > PR_PROFILE_MAX)) return false;
    if (P.n_l != 0 && (P.n_l < 2 || P.n_l > PR_PROFILE_MAX)) return false;
    for (int w = 0; w < 2; ++w) {
        const int n = w ? P.n_l : P.n_c;
        const float *g = w ? P.p_l : P.p_c;
        if (n == 0) continue;
        if (!(g[0] == 0.0f)) return false;
        for (int k = 1; k < n; ++k) {
            if (!isfinite(g[k]) || !(g[k] > g[k - 1])) return false;
            if (!w && (double)g[k] < (double)k / (n - 1)) return false;
        }
    }
    return true;
}

bool finite_all(const float *p, int n) {
    for (int i = 0; i < n; ++i)
        if (!isfinite(p[i])) return false;
    return true;
}

int check_args(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tu) {
    if (!meshes || !views || !tu || nm < 1 || nv < 1 || nv > PR_MAX_VIEWS) return PR_ERR_INVALID;
    for (int m = 0; m < nm; ++m) {
        const pr_mesh &M = meshes[m];
        if (M.nv < 0 || M.nt < 0) return PR_ERR_INVALID;
        if (M.nt > 0 && (!M.v0 || !M.v1 || !M.tri || M.nv < 1)) return PR_ERR_INVALID;
        if ((int64_t)M.nt * 3 > INT32_MAX || (int64_t)M.nv * 3 > INT32_MAX) return PR_ERR_INVALID;
        if ((uint32_t)M.nt > kListTriMask) return PR_ERR_INVALID;   // list entries hold 28-bit indices
        // a view's records are addressed with 32-bit byte offsets
        if ((uint64_t)M.nt * kRecRoll * 16 >= (1ull << 32)) return PR_ERR_INVALID;
    }
    for (int v = 0; v < nv; ++v) {
        const pr_view &V = views[v];
        if (V.width < 1 || V.height < 1 || V.width > 16384 || V.height > 16384) return PR_ERR_INVALID;
        if (V.mesh < 0 || V.mesh >= nm) return PR_ERR_INVALID;
        if (!finite_all(V.pose0, 6) || !finite_all(V.pose1, 6)) return PR_ERR_INVALID;
        float misc[10] = {V.fx, V.fy, V.cx, V.cy, V.znear, V.fovea[0], V.fovea[1], V.alpha, V.roll_dir[0], V.roll_dir[1]};
        if (!finite_all(misc, 10)) return PR_ERR_INVALID;
        if (V.fx == 0.0f || V.fy == 0.0f || !(V.znear > 0.0f)) return PR_ERR_INVALID;
        if (!(V.alpha >= 1.0f) || V.alpha > 16.0f) return PR_ERR_INVALID;
        if (fabsf(V.fovea[0]) > 1.0f || fabsf(V.fovea[1]) > 1.0f) return PR_ERR_INVALID;
        if (V.profile && !profile_ok(*V.profile)) return PR_ERR_INVALID;
    }
    if (tu->tile != 8 && tu->tile != 16 && tu->tile != 32) return PR_ERR_UNSUPPORTED;
    if (tu->bin_capacity < 1) return PR_ERR_INVALID;
    if (tu->bound < PR_BOUND_ZENON || tu->bound > PR_BOUND_QUAD) return PR_ERR_INVALID;
    if (tu->fov_bound < PR_FOV_EXACT || tu->fov_bound > PR_FOV_RECURSIVE) return PR_ERR_INVALID;
    return PR_OK;
}

bool rolling(const pr_view &v) { return v.roll_dir[0] != 0.0f || v.roll_dir[1] != 0.0f; }

PixelConst pixel_const(const pr_view &v) {
    PixelConst pc;
    pc.invW2 = (float)(2.0 / v.width);
    pc.invH2 = (float)(2.0 / v.height);
    pc.fov0 = v.fovea[0];
    pc.fov1 = v.fovea[1];
    double ex = fabs((double)v.fovea[0]) + 1.0, ey = fabs((double)v.fovea[1]) + 1.0;
    pc.invR = (float)(1.0 / sqrt(ex * ex + ey * ey));
    pc.alpha = v.alpha;
    pc.mode = v.alpha == 1.0f ? 0 : (v.alpha == 2.0f ? 1 : 2);
    if (v.profile && v.profile->n_c >= 2) pc.mode = 3;
    pc.lens = v.profile && v.profile->n_l >= 2 ? 1 : 0;
    pc.prof = nullptr;   // the workspace's copy, set when the views are written
    pc.roll0 = v.roll_dir[0];
    pc.roll1 = v.roll_dir[1];
    pc.cx = v.cx;
    pc.cy = v.cy;
    pc.invfx = (float)(1.0 / v.fx);
    pc.invfy = (float)(1.0 / v.fy);
    pc.znear = v.znear;
    pc.W = v.width;
    pc.H = v.height;
    return pc;
}

int layout(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tu, Layout &L) {
    int rc = check_args(meshes, nm, views, nv, tu);
    if (rc) return rc;
    L.nv = nv;
    L.any_prof = false;
    L.any_fov = false;
    int64_t tiles = 0, tri_blocks = 0, pix_blocks = 0, vtx_blocks = 0, rec4 = 0, tris = 0, gacc = 0;
    for (int v = 0; v < nv; ++v) {
        const pr_view &V = views[v];
        const pr_mesh &M = meshes[V.mesh];
        ViewDev &d = L.vd[v];
        memset(&d, 0, sizeof(d));
        d.view = V;
        d.mesh = M;
        d.pc = pixel_const(V);
        d.tile = tu->tile;
        d.tiles_x = (V.width + tu->tile - 1) / tu->tile;
        d.tiles_y = (V.height + tu->tile - 1) / tu->tile;
        d.ntiles = d.tiles_x * d.tiles_y;
        d.tile_base = (int32_t)tiles;
        d.tri_block0 = (int32_t)tri_blocks;
        d.pix_block0 = (int32_t)pix_blocks;
        d.rolling = rolling(V) ? 1 : 0;
        d.bound = tu->bound;
        d.fov_bound = tu->fov_bound;
        L.any_fov = L.any_fov || tu->fov_bound != PR_FOV_EXACT;
        d.rec_w = d.rolling ? kRecRoll : kRecStatic;
        d.rec_off = rec4;
        d.tri_off = tris;
        d.vtx_block0 = (int32_t)vtx_blocks;
        d.gacc_off = gacc;
        L.prof_used[v] = V.profile && (V.profile->n_c >= 2 || V.profile->n_l >= 2);
        L.any_prof = L.any_prof || L.prof_used[v];
        if (L.prof_used[v]) {
            ProfDev &P = L.prof_host[v];
            memset(&P, 0, sizeof(P));
            P.nc = V.profile->n_c >= 2 ? V.profile->n_c : 0;
            P.nl = V.profile->n_l >= 2 ? V.profile->n_l : 0;
            for (int k = 0; k < P.nc; ++k) P.c[k] = V.profile->p_c[k];
            for (int k = 0; k < P.nl; ++k) P.l[k] = V.profile->p_l[k];
        }
        d.view.profile = nullptr;   // a host pointer: never read on the device
        // FP64 camera geometry (host; the same code the host test hooks use)
        prg::make_geom(V, d.g);
        for (int q = 0; q < 9; ++q) { d.R0f[q] = (float)d.g.R0[q]; d.R1f[q] = (float)d.g.R1[q]; }
        for (int q = 0; q < 3; ++q) { d.T0f[q] = (float)d.g.T0[q]; d.T1f[q] = (float)d.g.T1[q]; }
        vtx_blocks += (M.nv + 255) / 256;
        gacc += 6 * (int64_t)M.nv;
        tiles += d.ntiles;
        tri_blocks += (M.nt + 255) / 256;
        pix_blocks += ((int64_t)V.width * V.height + 255) / 256;
        rec4 += (int64_t)M.nt * d.rec_w;
        tris += M.nt;
    }
    if (tiles + 1 > INT32_MAX / 2 || tri_blocks > INT32_MAX / 2 || pix_blocks > INT32_MAX / 2 ||
        vtx_blocks > INT32_MAX / 2)
        return PR_ERR_INVALID;
    L.total_vtx_blocks = (int)vtx_blocks;
    L.total_gacc = gacc;
    L.total_tiles = (int)tiles;
    L.total_tri_blocks = (int)tri_blocks;
    L.total_pix_blocks = (int)pix_blocks;
    L.nparts = (int)((tiles + 1 + kScanBlock - 1) / kScanBlock);
    L.cap = tu->bin_capacity;
    L.total_rec4 = rec4;
    L.total_tris = tris;
    size_t off = up(sizeof(DevStatus));
    L.table = off; off = up(off + sizeof(ViewTable));
    L.tinfo = off; off = up(off + (size_t)tiles * sizeof(TileInfo));
    L.rec = off; off = up(off + (size_t)rec4 * sizeof(float4));
    L.tb = off; off = up(off + (size_t)tris * sizeof(TriBound));
    L.bcand = off; off = up(off + ((size_t)tri_blocks + 1) * 4);
    L.bnf = off; off = up(off + ((size_t)tri_blocks + 1) * 4);
    L.bperm = off; off = up(off + ((size_t)tri_blocks + 1) * 4);
    L.boff = off; off = up(off + ((size_t)tri_blocks + 1) * 8);
    L.bpart = off; off = up(off + ((size_t)tri_blocks / 256 + 1) * 8);
    L.tcount = off; off = up(off + ((size_t)tiles + 1) * 4);
    L.toff = off; off = up(off + ((size_t)tiles + 1) * 4);
    L.part = off; off = up(off + (size_t)L.nparts * 8);   // the tile scan's block flags
    L.pairs = off; off = up(off + (size_t)L.cap * 12);   // Pairs: tile, slot, entry arrays
    L.lists = off; off = up(off + (size_t)L.cap * 4);
    L.gacc = off; off = up(off + (size_t)gacc * 4);
    L.pacc = off; off = up(off + ((size_t)pix_blocks + 1) * kPoseAcc * 8);   // per pixel block (backward)
    L.sched = off; off = up(off + sizeof(Sched));
    L.order = off; off = up(off + (size_t)tiles * 16 * kXcds);   // one tile order per XCD share
    L.prof = off; off = up(off + (size_t)nv * sizeof(ProfDev));
    L.bytes = off;
    return PR_OK;
}

int check_ws(const void *ws, size_t ws_bytes, size_t need) {
    if (!ws || ((uintptr_t)ws & (kAlign - 1))) return PR_ERR_WORKSPACE;
    if (ws_bytes < need) return PR_ERR_WORKSPACE;
    return PR_OK;
}

template <typename T>
T *at(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

int launched() { return hipGetLastError() == hipSuccess ? PR_OK : PR_ERR_HIP; }

// The candidate pair arrays (cap words each) in the workspace.
Pairs pairs_at(const Layout &L, void *ws) {
    int32_t *base = at<int32_t>(ws, L.pairs);
    return Pairs{base, reinterpret_cast<uint32_t *>(base + L.cap), reinterpret_cast<uint32_t *>(base + 2 * (size_t)L.cap)};
}

void fill_u32(void *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, (uint32_t *)p, v, n);
}

#define PR_PREP()                                                         \
    static thread_local Layout L;                                        \
    {                                                                     \
        int rc_ = layout(meshes, nm, views, nv, tuning, L);               \
        if (rc_) return rc_;                                              \
        rc_ = check_ws(ws, ws_bytes, L.bytes);                            \
        if (rc_) return rc_;                                              \
    }                                                                     \
    hipStream_t s = (hipStream_t)stream;                                  \
    DevStatus *st = at<DevStatus>(ws, 0);                                 \
    ViewTable *T = at<ViewTable>(ws, L.table);

// The views' tabulated profiles into the workspace (before the view table,
// whose geometry points at them).
ProfDev *write_profiles(const Layout &L, ViewTable *T, hipStream_t s) {
    ProfDev *prof = reinterpret_cast<ProfDev *>(reinterpret_cast<char *>(T) - L.table + L.prof);
    for (int v = 0; v < L.nv; ++v)
        if (L.prof_used[v]) hipLaunchKernelGGL(k_write_profile, dim3(1), dim3(64), 0, s, L.prof_host[v], prof + v);
    return prof;
}

// Views first .. first + kViewsPerWrite - 1 of the call as one pack of
// kernel arguments; reset_status: the launch that takes it also clears the
// status block (the frame's first pass).
ViewPack make_pack(const Layout &L, ProfDev *prof, int first, bool reset_status) {
    ViewPack p;
    memset(&p, 0, sizeof(p));
    p.first = first;
    p.count = std::min(kViewsPerWrite, L.nv - first);
    p.nv = L.nv;
    p.total_tiles = L.total_tiles;
    p.total_tri_blocks = L.total_tri_blocks;
    p.total_pix_blocks = L.total_pix_blocks;
    p.total_vtx_blocks = L.total_vtx_blocks;
    p.reset_status = reset_status ? 1 : 0;
    for (int i = 0; i < p.count; ++i) {
        ViewDev &d = p.v[i];
        d = L.vd[first + i];
        d.pc.prof = L.prof_used[first + i] ? prof + first + i : nullptr;
        if (d.pc.prof) {
            // the workspace's copy (k_write_profile, earlier on the stream):
            // device addresses, counts from the host copy
            const ProfDev &H = L.prof_host[first + i];
            prg::attach_profile(d.g, d.pc.prof->c, H.nc, d.pc.prof->l, H.nl, H.c, H.l);
        }
    }
    return p;
}

// The workspace's view table from the call's own meshes and views (FP64
// camera geometry computed on the host); reset_status: also clear the
// status block (the frame's first pass).
void write_views(const Layout &L, ViewTable *T, DevStatus *st, bool reset_status, hipStream_t s) {
    ProfDev *prof = write_profiles(L, T, s);
    for (int first = 0; first < L.nv; first += kViewsPerWrite)
        hipLaunchKernelGGL(k_write_views, dim3(1), dim3(64), 0, s, make_pack(L, prof, first, reset_status), T, st);
}

// Blocks of a kernel the whole device keeps resident (persistent grids).
template <typename K>
int resident_blocks(K kernel, int threads) {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu * prop.multiProcessorCount;
}

// The ray cast; with SHADE the resolved pixels are also shaded (fused into
// the persistent ray cast; the one-block-per-item form runs k_shade after).
template <int TILE, bool COUNT, bool SHADE>
void launch_raycast_t(int flags, const Layout &L, void *ws, const RayOut &out, const ShadeIO &sio,
                      const pr_light &light, DevStatus *st, ViewTable *T, hipStream_t s) {
    using C = RayCfg<TILE>;
    if (!(flags & PR_FLAG_PERSISTENT)) {
        hipLaunchKernelGGL((k_raycast<TILE, COUNT>), dim3(ray_items<TILE>(L.total_tiles)), dim3(C::NT), 0, s, T,
                           at<float4>(ws, L.rec),
                           at<uint32_t>(ws, L.toff), at<uint32_t>(ws, L.lists), out, st);
        if (SHADE)
            hipLaunchKernelGGL(k_shade, dim3(L.total_pix_blocks), dim3(256), 0, s, T, at<float4>(ws, L.rec), sio,
                               light);
        return;
    }
    // resident blocks per device (each instantiation its own cache; a race
    // between threads only computes the same value twice)
    static std::atomic<int> resident[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    int res = resident[dev].load(std::memory_order_relaxed);
    if (!res) {
        res = resident_blocks(k_raycast_queue<TILE, COUNT, SHADE>, C::NT);
        resident[dev].store(res, std::memory_order_relaxed);
    }
    // items: at most every tile in one XCD share (the device knows the
    // exact count); the grid a multiple of the XCD count
    const int64_t bound_items = (int64_t)kXcds * share_items(TILE, L.total_tiles);
    int grid = (int)std::min<int64_t>(bound_items, (int64_t)std::max(res, kXcds));
    grid = std::max(kXcds, grid - grid % kXcds);
    hipLaunchKernelGGL((k_raycast_queue<TILE, COUNT, SHADE>), dim3(grid), dim3(C::NT), 0, s, T, at<float4>(ws, L.rec),
                       at<uint32_t>(ws, L.lists), out, st, at<int4>(ws, L.order), at<Sched>(ws, L.sched), sio,
                       light);
}

template <int TILE, bool SHADE>
void launch_raycast(int flags, const Layout &L, void *ws, const RayOut &out, const ShadeIO &sio,
                    const pr_light &light, DevStatus *st, ViewTable *T, hipStream_t s) {
    if (flags & PR_FLAG_COUNT) launch_raycast_t<TILE, true, SHADE>(flags, L, ws, out, sio, light, st, T, s);
    else launch_raycast_t<TILE, false, SHADE>(flags, L, ws, out, sio, light, st, T, s);
}

template <bool SHADE>
void launch_raycast_any(int tile, int flags, const Layout &L, void *ws, const RayOut &out, const ShadeIO &sio,
                        const pr_light &light, DevStatus *st, ViewTable *T, hipStream_t s) {
    if (tile == 8) launch_raycast<8, SHADE>(flags, L, ws, out, sio, light, st, T, s);
    else if (tile == 16) launch_raycast<16, SHADE>(flags, L, ws, out, sio, light, st, T, s);
    else launch_raycast<32, SHADE>(flags, L, ws, out, sio, light, st, T, s);
}

// Checks the shading arguments and fills io (ids from tri_id, may be NULL
// when the ids come from the ray cast); *any: some view has an output.
// A usable light: finite direction and ambient, highlight k_s >= 0 and
// exponent m >= 1 (finite).
bool light_ok(const pr_light *light) {
    return light && isfinite(light->ambient) && isfinite(light->dir_world[0]) && isfinite(light->dir_world[1]) &&
           isfinite(light->dir_world[2]) && isfinite(light->specular) && light->specular >= 0.0f &&
           isfinite(light->shininess) && light->shininess >= 1.0f;
}

int shade_args(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const int32_t *const *tri_id,
               const pr_light *light, const float *const *albedo, uint8_t *const *rgba8, float *const *rgb32,
               ShadeIO &io, bool &any) {
    if (!light || !albedo || !views || nv < 1 || nv > PR_MAX_VIEWS) return PR_ERR_INVALID;
    if (!light_ok(light)) return PR_ERR_INVALID;
    if (tri_id)
        for (int v = 0; v < nv; ++v)
            if (!tri_id[v]) return PR_ERR_INVALID;
    if (meshes)
        for (int v = 0; v < nv; ++v) {
            int m = views[v].mesh;
            if (m >= 0 && m < nm && meshes[m].nt > 0 && !albedo[m]) return PR_ERR_INVALID;
        }
    memset(&io, 0, sizeof(io));
    any = false;
    for (int v = 0; v < nv; ++v) {
        const int m = views[v].mesh;
        io.id[v] = tri_id ? tri_id[v] : nullptr;
        io.rgba8[v] = rgba8 ? rgba8[v] : nullptr;
        io.rgb32[v] = rgb32 ? rgb32[v] : nullptr;
        io.albedo[v] = (m >= 0 && m < nm) ? albedo[m] : nullptr;
        any = any || io.rgba8[v] || io.rgb32[v];
    }
    return PR_OK;
}

}  // namespace

extern "C" {

int pr_workspace_size(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                      size_t *bytes) {
    if (!bytes) return PR_ERR_INVALID;
    static thread_local Layout L;
    int rc = layout(meshes, nm, views, nv, tuning, L);
    if (rc) return rc;
    *bytes = L.bytes;
    return PR_OK;
}

int pr_bound(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
             size_t ws_bytes, void *stream) {
    PR_PREP();
    // up to kViewsPerWrite views travel in k_bound's arguments (its block 0
    // writes the view table), more need the table written first
    const bool pack = L.nv <= kViewsPerWrite && L.total_tri_blocks > 0;
    ViewPack p;
    if (pack) p = make_pack(L, write_profiles(L, T, s), 0, true);
    else {
        write_views(L, T, st, true, s);
        memset(&p, 0, sizeof(p));
    }
    if (L.total_tri_blocks > 0) {
        auto k = L.any_prof ? (pack ? k_bound<true, true> : k_bound<true, false>)
                            : (pack ? k_bound<false, true> : k_bound<false, false>);
        hipLaunchKernelGGL(k, dim3(L.total_tri_blocks), dim3(256), 0, s, p, T, at<float4>(ws, L.rec),
                           at<TriBound>(ws, L.tb), st, at<int32_t>(ws, L.bcand), at<int32_t>(ws, L.bnf));
    }
    return launched();
}

int pr_bin(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
           size_t ws_bytes, void *stream) {
    PR_PREP();
    const int tile_blocks = ((L.total_tiles + 1) * 4 + 255) / 256;
    const int chunk_blocks = (L.total_tri_blocks + 255) / 256;
    // one block more than the tiles and chunks need: the last orders the
    // binning blocks
    hipLaunchKernelGGL(L.any_prof ? k_tiles<true> : k_tiles<false>, dim3(std::max(tile_blocks, chunk_blocks) + 1),
                       dim3(256), 0, s, T, at<TileInfo>(ws, L.tinfo), at<uint32_t>(ws, L.tcount),
                       at<Sched>(ws, L.sched), at<int32_t>(ws, L.bcand), at<int32_t>(ws, L.bnf),
                       at<int64_t>(ws, L.boff),
                       at<int64_t>(ws, L.bpart), st, at<int32_t>(ws, L.bperm),
                       at<unsigned long long>(ws, L.part), L.nparts);
    if (L.total_tri_blocks > 0)
        hipLaunchKernelGGL(L.any_fov ? k_bin<true> : k_bin<false>, dim3(L.total_tri_blocks), dim3(kBinThreads), 0, s,
                           T, at<TriBound>(ws, L.tb),
                           at<TileInfo>(ws, L.tinfo), at<uint32_t>(ws, L.tcount), at<int64_t>(ws, L.boff),
                           at<int64_t>(ws, L.bpart), pairs_at(L, ws), L.cap, at<int32_t>(ws, L.bperm), st);
    int n = L.total_tiles + 1;
    hipLaunchKernelGGL(k_scan, dim3(L.nparts), dim3(256), 0, s, T, at<uint32_t>(ws, L.tcount), n, L.total_tiles,
                       at<unsigned long long>(ws, L.part), at<uint32_t>(ws, L.toff), at<Sched>(ws, L.sched));
    // pairs (grid-stride) and the persistent ray cast's tile order (one
    // block per 256 tiles)
    int sb = (int)std::min<int64_t>(std::max<int64_t>((L.cap + 255) / 256, 1), 2048);
    sb = std::max(sb, (L.total_tiles + 255) / 256);
    hipLaunchKernelGGL(k_scatter, dim3(sb), dim3(256), 0, s, T, pairs_at(L, ws), at<uint32_t>(ws, L.toff),
                       at<int32_t>(ws, L.lists), L.cap, L.total_tiles, st, at<Sched>(ws, L.sched),
                       at<int4>(ws, L.order));
    return launched();
}

int pr_raycast(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
               size_t ws_bytes, int32_t *const *tri_id, float *const *depth, void *stream) {
    if (!tri_id || !depth) return PR_ERR_INVALID;
    for (int v = 0; v < nv && v < PR_MAX_VIEWS; ++v)
        if (!tri_id[v] || !depth[v]) return PR_ERR_INVALID;
    PR_PREP();
    RayOut out;
    memset(&out, 0, sizeof(out));
    for (int v = 0; v < nv; ++v) {
        out.id[v] = tri_id[v];
        out.depth[v] = depth[v];
    }
    ShadeIO io;
    memset(&io, 0, sizeof(io));
    const pr_light none{};
    launch_raycast_any<false>(tuning->tile, tuning->flags, L, ws, out, io, none, st, T, s);
    return launched();
}

int pr_shade(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
             size_t ws_bytes, const int32_t *const *tri_id, const pr_light *light, const float *const *albedo,
             uint8_t *const *rgba8, float *const *rgb32, void *stream) {
    if (!tri_id) return PR_ERR_INVALID;
    ShadeIO io;
    bool any = false;
    int rc = shade_args(meshes, nm, views, nv, tri_id, light, albedo, rgba8, rgb32, io, any);
    if (rc) return rc;
    PR_PREP();
    if (!any) return PR_OK;
    hipLaunchKernelGGL(k_shade, dim3(L.total_pix_blocks), dim3(256), 0, s, T, at<float4>(ws, L.rec), io, *light);
    return launched();
}

int pr_gbuffer(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
               size_t ws_bytes, const int32_t *const *tri_id, float *const *normal, float *const *bary,
               float *const *density, void *stream) {
    if (!tri_id || !views || nv < 1 || nv > PR_MAX_VIEWS) return PR_ERR_INVALID;
    for (int v = 0; v < nv; ++v)
        if (!tri_id[v]) return PR_ERR_INVALID;
    GbufIO io;
    memset(&io, 0, sizeof(io));
    bool any = false;
    for (int v = 0; v < nv; ++v) {
        io.id[v] = tri_id[v];
        io.normal[v] = normal ? normal[v] : nullptr;
        io.bary[v] = bary ? bary[v] : nullptr;
        io.density[v] = density ? density[v] : nullptr;
        any |= io.normal[v] || io.bary[v] || io.density[v];
    }
    PR_PREP();
    (void)st;
    if (!any) return PR_OK;
    hipLaunchKernelGGL(k_gbuffer, dim3(L.total_pix_blocks), dim3(256), 0, s, T, at<float4>(ws, L.rec), io);
    return launched();
}

int pr_raycast_shade(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
                     size_t ws_bytes, int32_t *const *tri_id, float *const *depth, const pr_light *light,
                     const float *const *albedo, uint8_t *const *rgba8, float *const *rgb32, void *stream) {
    if (!tri_id || !depth) return PR_ERR_INVALID;
    for (int v = 0; v < nv && v < PR_MAX_VIEWS; ++v)
        if (!tri_id[v] || !depth[v]) return PR_ERR_INVALID;
    ShadeIO io;
    bool any = false;
    int rc = shade_args(meshes, nm, views, nv, tri_id, light, albedo, rgba8, rgb32, io, any);
    if (rc) return rc;
    PR_PREP();
    RayOut out;
    memset(&out, 0, sizeof(out));
    for (int v = 0; v < nv; ++v) {
        out.id[v] = tri_id[v];
        out.depth[v] = depth[v];
    }
    if (any) launch_raycast_any<true>(tuning->tile, tuning->flags, L, ws, out, io, *light, st, T, s);
    else launch_raycast_any<false>(tuning->tile, tuning->flags, L, ws, out, io, *light, st, T, s);
    return launched();
}

int pr_backward(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
                size_t ws_bytes, const int32_t *const *tri_id, const pr_light *light, const float *const *albedo,
                const float *const *dl_drgb, float *const *dv0, float *const *dv1, float *dpose0, float *dpose1,
                void *stream) {
    if (!tri_id || !light || !albedo || !dl_drgb || !dv0 || !dv1 || !dpose0 || !dpose1) return PR_ERR_INVALID;
    if (!light_ok(light)) return PR_ERR_INVALID;
    if (!views || !meshes || nv < 1 || nv > PR_MAX_VIEWS || nm < 1 || nm > PR_MAX_VIEWS) return PR_ERR_INVALID;
    for (int v = 0; v < nv; ++v) {
        if (!tri_id[v] || !dl_drgb[v]) return PR_ERR_INVALID;
        int m = views[v].mesh;
        if (m < 0 || m >= nm) return PR_ERR_INVALID;
        if (meshes[m].nv > 0 && (!dv0[m] || !dv1[m] || (meshes[m].nt > 0 && !albedo[m]))) return PR_ERR_INVALID;
    }
    PR_PREP();
    BwdIO io;
    BwdOut out;
    memset(&io, 0, sizeof(io));
    memset(&out, 0, sizeof(out));
    for (int v = 0; v < nv; ++v) {
        io.id[v] = tri_id[v];
        io.dl[v] = dl_drgb[v];
        io.albedo[v] = albedo[views[v].mesh];
    }
    bool used[PR_MAX_VIEWS] = {false};
    for (int v = 0; v < nv; ++v) used[views[v].mesh] = true;
    for (int m = 0; m < nm; ++m) {
        out.dv0[m] = dv0[m];
        out.dv1[m] = dv1[m];
        if (used[m] && meshes[m].nv > 0) {
            fill_u32(dv0[m], 0u, 3 * (int64_t)meshes[m].nv, s);
            fill_u32(dv1[m], 0u, 3 * (int64_t)meshes[m].nv, s);
        }
    }
    fill_u32(at<void>(ws, L.gacc), 0u, L.total_gacc, s);
    // the geometry and poses are this call's own (the view table of the
    // frame's pr_bound may hold another frame's by now)
    write_views(L, T, st, false, s);
    hipLaunchKernelGGL(k_view_light, dim3(1), dim3(64), 0, s, T, *light);
    hipLaunchKernelGGL(k_bwd_pixel, dim3(L.total_pix_blocks), dim3(256), 0, s, T, io, *light,
                       at<float>(ws, L.gacc), at<double>(ws, L.pacc));
    if (L.total_vtx_blocks > 0)
        hipLaunchKernelGGL(k_bwd_vertex, dim3(L.total_vtx_blocks), dim3(256), 0, s, T, at<float>(ws, L.gacc), out);
    hipLaunchKernelGGL(k_bwd_pose, dim3(nv), dim3(kPoseThreads), 0, s, T, at<double>(ws, L.pacc), *light, dpose0,
                       dpose1);
    return launched();
}

int pr_status_read(const void *ws, size_t ws_bytes, pr_status *out, void *stream) {
    if (!ws || !out || ws_bytes < sizeof(DevStatus)) return PR_ERR_INVALID;
    DevStatus d;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&d, ws, sizeof(d), hipMemcpyDeviceToHost, s) != hipSuccess) return PR_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PR_ERR_HIP;
    out->overflow = d.overflow;
    out->nonfinite = d.nonfinite;
    out->pairs_required = (int64_t)d.pairs_required;
    out->pairs_total = (int64_t)d.pairs_total;
    unsigned long long tests = d.tests, hits = d.hits;
    for (int i = 0; i < kCountSlots; ++i) {
        tests += d.cnt[i][0];
        hits += d.cnt[i][1];
    }
    out->tests = (int64_t)tests;
    out->hits = (int64_t)hits;
    return PR_OK;
}

const char *pr_status_string(int code) {
    switch (code) {
        case PR_OK: return "ok";
        case PR_ERR_INVALID: return "invalid argument";
        case PR_ERR_UNSUPPORTED: return "unsupported parameter";
        case PR_ERR_WORKSPACE: return "workspace too small or misaligned";
        case PR_ERR_HIP: return "HIP runtime error";
        default: return "unknown status code";
    }
}

int pr_debug_tile_lists(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                        const void *ws_c, size_t ws_bytes, int view, int32_t *offsets, int32_t *lists, int64_t cap,
                        int32_t *ntiles, int64_t *npairs, void *stream) {
    void *ws = const_cast<void *>(ws_c);
    if (!ntiles || !npairs || view < 0 || view >= nv) return PR_ERR_INVALID;
    PR_PREP();
    (void)st;
    (void)T;
    const ViewDev &d = L.vd[view];
    *ntiles = d.ntiles;
    uint32_t ends[2] = {0, 0};
    if (hipMemcpyAsync(&ends[0], at<uint32_t>(ws, L.toff) + d.tile_base, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&ends[1], at<uint32_t>(ws, L.toff) + d.tile_base + d.ntiles, 4, hipMemcpyDeviceToHost, s) !=
            hipSuccess)
        return PR_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PR_ERR_HIP;
    uint32_t total = ends[1] - ends[0];
    *npairs = total;
    if (offsets) {
        if (hipMemcpyAsync(offsets, at<uint32_t>(ws, L.toff) + d.tile_base, ((size_t)d.ntiles + 1) * 4,
                           hipMemcpyDeviceToHost, s) != hipSuccess)
            return PR_ERR_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return PR_ERR_HIP;
        for (int i = 0; i <= d.ntiles; ++i) offsets[i] -= (int32_t)ends[0];
    }
    if (lists) {
        if (cap < (int64_t)total || (int64_t)ends[1] > L.cap) return PR_ERR_INVALID;
        if (total && hipMemcpyAsync(lists, at<int32_t>(ws, L.lists) + ends[0], (size_t)total * 4,
                                    hipMemcpyDeviceToHost, s) != hipSuccess)
            return PR_ERR_HIP;
    }
    return hipStreamSynchronize(s) == hipSuccess ? PR_OK : PR_ERR_HIP;
}

// ---------------------------------------------------------------------------
// host evaluation of the bound (tests)
// ---------------------------------------------------------------------------
int pr_host_time_interval(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t bound, double *t) {
    if (!mesh || !view || !t || f < 0 || f >= mesh->nt || bound < 0 || bound > PR_BOUND_QUAD) return -1;
    if (view->profile && !profile_ok(*view->profile)) return -1;
    prg::Geom g;
    prg::make_geom(*view, g);
    if (view->profile)
        prg::attach_profile(g, view->profile->p_c, view->profile->n_c, view->profile->p_l, view->profile->n_l);
    double Ps[3][3], Pe[3][3];
    int32_t idx[3];
    if (!prg::load_tri(mesh->v0, mesh->v1, mesh->tri, mesh->nv, f, g, Ps, Pe, idx)) return 0;
    return prg::time_window(g, Ps, Pe, t, bound);
}

int pr_host_tile_rect(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t bound, int32_t tile,
                      int32_t *rect) {
    if (!mesh || !view || !rect || f < 0 || f >= mesh->nt || tile < 1 || bound < 0 || bound > PR_BOUND_QUAD)
        return -1;
    if (view->profile && !profile_ok(*view->profile)) return -1;
    prg::Geom g;
    prg::make_geom(*view, g);
    if (view->profile)
        prg::attach_profile(g, view->profile->p_c, view->profile->n_c, view->profile->p_l, view->profile->n_l);
    double Ps[3][3], Pe[3][3], win[2], box[4];
    int32_t idx[3];
    if (!prg::load_tri(mesh->v0, mesh->v1, mesh->tri, mesh->nv, f, g, Ps, Pe, idx)) return 0;
    int kind = prg::time_window(g, Ps, Pe, win, bound);
    if (kind == prg::kCulled) return 0;
    prg::display_box(g, Ps, Pe, win[0], win[1], kind, box);
    int r[4];
    if (!prg::tile_rect(g, box, tile, r)) return 0;
    for (int k = 0; k < 4; ++k) rect[k] = r[k];
    return 1;
}

int pr_host_tile_test_fov(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t bound, int32_t fov,
                          int32_t tile, int32_t tx, int32_t ty) {
    if (fov < PR_FOV_EXACT || fov > PR_FOV_RECURSIVE) return -1;
    if (!mesh || !view || f < 0 || f >= mesh->nt || tile < 1 || bound < 0 || bound > PR_BOUND_QUAD) return -1;
    if (view->profile && !profile_ok(*view->profile)) return -1;
    prg::Geom g;
    prg::make_geom(*view, g);
    if (view->profile)
        prg::attach_profile(g, view->profile->p_c, view->profile->n_c, view->profile->p_l, view->profile->n_l);
    double Ps[3][3], Pe[3][3], win[2], box[4];
    int32_t idx[3];
    if (!prg::load_tri(mesh->v0, mesh->v1, mesh->tri, mesh->nv, f, g, Ps, Pe, idx)) return 0;
    int kind = prg::time_window(g, Ps, Pe, win, bound);
    if (kind == prg::kCulled) return 0;
    prg::display_box(g, Ps, Pe, win[0], win[1], kind, box);
    int r[4];
    if (!prg::tile_rect(g, box, tile, r)) return 0;
    if (tx < r[0] || tx > r[2] || ty < r[1] || ty > r[3]) return 0;
    double w[4];
    if (kind == prg::kWindow) { w[0] = win[0]; w[1] = win[1]; w[2] = w[3] = 0.0; }
    else for (int k = 0; k < 4; ++k) w[k] = box[k];
    return prg::tile_mask(g, Ps, Pe, kind, w, tile, tx, ty, bound, fov);
}

int pr_host_tile_test(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t bound, int32_t tile, int32_t tx,
                      int32_t ty) {
    return pr_host_tile_test_fov(mesh, f, view, bound, PR_FOV_EXACT, tile, tx, ty);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// display unfoveation
// ---------------------------------------------------------------------------
namespace {

struct DispLayout {
    int nv;
    prd::DispView v[PR_MAX_VIEWS];
    int total_blocks, total_tiles, max_levels;
    bool any_mip;
    size_t pyr, bytes;
};

int disp_layout(const pr_view *views, int nv, const pr_display *disp, DispLayout &L) {
    if (!views || !disp || nv < 1 || nv > PR_MAX_VIEWS) return PR_ERR_INVALID;
    L.nv = nv;
    int64_t blocks = 0, tiles = 0, f4 = 0;
    L.max_levels = 1;
    L.any_mip = false;
    for (int i = 0; i < nv; ++i) {
        const pr_view &V = views[i];
        const pr_display &D = disp[i];
        if (V.width < 1 || V.height < 1 || V.width > 16384 || V.height > 16384) return PR_ERR_INVALID;
        if (D.width < 1 || D.height < 1 || D.width > 16384 || D.height > 16384) return PR_ERR_INVALID;
        float misc[4] = {V.fovea[0], V.fovea[1], V.alpha, D.sigma};
        if (!finite_all(misc, 3)) return PR_ERR_INVALID;
        if (!(V.alpha >= 1.0f) || V.alpha > 16.0f) return PR_ERR_INVALID;
        if (fabsf(V.fovea[0]) > 1.0f || fabsf(V.fovea[1]) > 1.0f) return PR_ERR_INVALID;
        if (D.mode != PR_UNFOV_MIP && D.mode != PR_UNFOV_FILTER) return PR_ERR_INVALID;
        if (D.mode == PR_UNFOV_FILTER && !(isfinite(D.sigma) && D.sigma > 0.0f)) return PR_ERR_INVALID;
        prd::DispView &d = L.v[i];
        memset(&d, 0, sizeof(d));
        d.W = V.width; d.H = V.height; d.Wd = D.width; d.Hd = D.height;
        d.mode = D.mode;
        d.fov0 = V.fovea[0]; d.fov1 = V.fovea[1];
        d.e = (float)(1.0 / (double)V.alpha);
        d.invR = (float)(1.0 / prg::fovea_radius(V.fovea[0], V.fovea[1]));
        d.powmode = V.alpha == 1.0f ? 0 : (V.alpha == 2.0f ? 1 : 2);
        if (V.profile && !profile_ok(*V.profile)) return PR_ERR_INVALID;
        if (V.profile && V.profile->n_c >= 2) {   // tabulated p_c (a lens is undone by the optics)
            d.powmode = 3;
            d.ntab = V.profile->n_c;
            for (int k = 0; k < d.ntab; ++k) d.tab[k] = V.profile->p_c[k];
        }
        if (D.mode == PR_UNFOV_FILTER) d.inv2s2 = (float)(1.0 / (2.0 * (double)D.sigma * D.sigma));
        d.blk0 = (int32_t)blocks;
        blocks += (int64_t)((D.width + 31) / 32) * ((D.height + 7) / 8);
        d.tile0 = (int32_t)tiles;
        int w = V.width, h = V.height, n = 0;
        for (;;) {
            d.lw[n] = w;
            d.lh[n] = h;
            ++n;
            if (w == 1 && h == 1) break;
            w = (w + 1) / 2;
            h = (h + 1) / 2;
        }
        d.nlev = n;
        if (D.mode == PR_UNFOV_MIP) {
            L.any_mip = true;
            L.max_levels = std::max(L.max_levels, n);
            d.tiles_x = (V.width + 31) / 32;
            d.tiles_y = (V.height + 31) / 32;
            tiles += (int64_t)d.tiles_x * d.tiles_y;
            for (int k = 1; k < n; ++k) {   // each level on its own 256-byte lines
                d.loff[k] = f4;
                f4 += ((int64_t)d.lw[k] * d.lh[k] + 15) & ~(int64_t)15;
            }
        }
    }
    if (blocks > INT32_MAX / 2 || tiles > INT32_MAX / 2) return PR_ERR_INVALID;
    L.total_blocks = (int)blocks;
    L.total_tiles = (int)tiles;
    L.pyr = up(sizeof(prd::DispTable));
    L.bytes = up(L.pyr + (size_t)f4 * 16);
    return PR_OK;
}

}  // namespace

extern "C" int pr_unfoveate_workspace_size(const pr_view *views, int nv, const pr_display *disp, size_t *bytes) {
    if (!bytes) return PR_ERR_INVALID;
    static thread_local DispLayout L;
    int rc = disp_layout(views, nv, disp, L);
    if (rc) return rc;
    *bytes = L.bytes;
    return PR_OK;
}

extern "C" int pr_unfoveate(const pr_view *views, int nv, const pr_display *disp, const uint8_t *const *fov_rgba8,
                            uint8_t *const *disp_rgba8, void *ws, size_t ws_bytes, void *stream) {
    static thread_local DispLayout L;
    int rc = disp_layout(views, nv, disp, L);
    if (rc) return rc;
    rc = check_ws(ws, ws_bytes, L.bytes);
    if (rc) return rc;
    if (!fov_rgba8 || !disp_rgba8) return PR_ERR_INVALID;
    prd::DispIO io;
    memset(&io, 0, sizeof(io));
    for (int v = 0; v < nv; ++v) {
        if (!fov_rgba8[v] || !disp_rgba8[v]) return PR_ERR_INVALID;
        io.fov[v] = fov_rgba8[v];
        io.out[v] = disp_rgba8[v];
    }
    hipStream_t s = (hipStream_t)stream;
    prd::DispTable *T = at<prd::DispTable>(ws, 0);
    float4 *pyr = at<float4>(ws, L.pyr);
    for (int first = 0; first < nv; first += prd::kDispViewsPerWrite) {
        prd::DispPack p;
        memset(&p, 0, sizeof(p));
        p.first = first;
        p.count = std::min(prd::kDispViewsPerWrite, nv - first);
        p.nv = nv;
        p.total_blocks = L.total_blocks;
        p.total_tiles = L.total_tiles;
        for (int i = 0; i < p.count; ++i) p.v[i] = L.v[first + i];
        hipLaunchKernelGGL(prd::k_disp_views, dim3(1), dim3(64), 0, s, p, T);
    }
    if (L.any_mip && L.total_tiles > 0)
        hipLaunchKernelGGL(prd::k_mip_tile, dim3(L.total_tiles), dim3(256), 0, s, T, io, pyr);
    if (L.max_levels > prd::kTileLevels + 1) hipLaunchKernelGGL(prd::k_mip_top, dim3(nv), dim3(1024), 0, s, T, pyr);
    if (L.total_blocks > 0) hipLaunchKernelGGL(prd::k_unfov, dim3(L.total_blocks), dim3(256), 0, s, T, io, pyr);
    return launched();
}

// ---------------------------------------------------------------------------
// the frame on a static scratch array (callers that cannot allocate)
// ---------------------------------------------------------------------------
// Workspace of pr_frame_static: a file-scope device array, one per device
// the library runs on, held until the process ends.  Host code never passes
// this name to a kernel or a copy (on the host it is only a stand-in for the
// symbol): it takes the array's device address from hipGetSymbolAddress,
// once per device, and uses that.
static __device__ __align__(256) unsigned char scratch[PR_STATIC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (looked up on the device's first
// call, with that device current).
int static_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PR_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PR_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PR_OK;
}

}  // namespace

extern "C" int pr_frame_static(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                               int32_t *const *tri_id, float *const *depth, const pr_light *light,
                               const float *const *albedo, uint8_t *const *rgba8, float *const *rgb32,
                               void *stream) {
    // every argument is checked before anything is enqueued
    size_t need = 0;
    int rc = pr_workspace_size(meshes, nm, views, nv, tuning, &need);
    if (rc) return rc;
    if (need > (size_t)PR_STATIC_SCRATCH_BYTES) return PR_ERR_WORKSPACE;
    if (!tri_id || !depth) return PR_ERR_INVALID;
    for (int v = 0; v < nv; ++v)
        if (!tri_id[v] || !depth[v]) return PR_ERR_INVALID;
    ShadeIO io;
    bool any = false;
    rc = shade_args(meshes, nm, views, nv, tri_id, light, albedo, rgba8, rgb32, io, any);
    if (rc) return rc;
    void *ws = nullptr;
    rc = static_scratch(&ws);
    if (rc) return rc;
    // the frame's passes clear what they accumulate into (status block,
    // counters, cursors), so the array's previous contents do not matter
    rc = pr_bound(meshes, nm, views, nv, tuning, ws, PR_STATIC_SCRATCH_BYTES, stream);
    if (!rc) rc = pr_bin(meshes, nm, views, nv, tuning, ws, PR_STATIC_SCRATCH_BYTES, stream);
    if (!rc)
        rc = pr_raycast_shade(meshes, nm, views, nv, tuning, ws, PR_STATIC_SCRATCH_BYTES, tri_id, depth, light,
                              albedo, rgba8, rgb32, stream);
    return rc;
}

// ---------------------------------------------------------------------------
// batched form: hipGraph of one frame over all views, autotuned
// ---------------------------------------------------------------------------
struct pr_batch {
    std::vector<pr_mesh> meshes;
    std::vector<pr_view> views;
    std::vector<pr_profile> profiles;   // the views' profiles, owned (views point here)
    pr_tuning tuning;
    pr_light light;
    std::vector<const float *> albedo;
    std::vector<int32_t *> ids;
    std::vector<float *> depth;
    std::vector<uint8_t *> rgba8;
    std::vector<float *> rgb32;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double trial_ms[3] = {0, 0, 0};
};

namespace {

int batch_frame(pr_batch *b, hipStream_t s) {
    const int nm = (int)b->meshes.size(), nv = (int)b->views.size();
    const pr_mesh *M = b->meshes.data();
    const pr_view *V = b->views.data();
    int rc = pr_bound(M, nm, V, nv, &b->tuning, b->ws, b->ws_bytes, s);
    if (!rc) rc = pr_bin(M, nm, V, nv, &b->tuning, b->ws, b->ws_bytes, s);
    // ray cast and shading in one pass (plain ray cast when nothing is shaded)
    if (!rc)
        rc = pr_raycast_shade(M, nm, V, nv, &b->tuning, b->ws, b->ws_bytes, b->ids.data(), b->depth.data(), &b->light,
                              b->albedo.data(), b->rgba8.data(), b->rgb32.data(), s);
    return rc;
}

int batch_alloc(pr_batch *b) {
    if (b->ws) {
        (void)hipFree(b->ws);
        b->ws = nullptr;
    }
    size_t bytes = 0;
    int rc = pr_workspace_size(b->meshes.data(), (int)b->meshes.size(), b->views.data(), (int)b->views.size(),
                               &b->tuning, &bytes);
    if (rc) return rc;
    if (hipMalloc(&b->ws, bytes) != hipSuccess) {
        b->ws = nullptr;
        return PR_ERR_HIP;
    }
    b->ws_bytes = bytes;
    return PR_OK;
}

// Runs frames until the tile lists fit; returns the capacity-checked status.
int batch_fit(pr_batch *b) {
    for (int attempt = 0; attempt < 6; ++attempt) {
        int rc = batch_alloc(b);
        if (rc) return rc;
        rc = batch_frame(b, b->cs);
        if (rc) return rc;
        pr_status st;
        rc = pr_status_read(b->ws, b->ws_bytes, &st, b->cs);
        if (rc) return rc;
        if (!st.overflow) return PR_OK;
        int64_t need = st.pairs_required + st.pairs_required / 4 + 1024;
        if (need > INT32_MAX) return PR_ERR_UNSUPPORTED;
        b->tuning.bin_capacity = (int32_t)need;
    }
    return PR_ERR_HIP;
}

double batch_time(pr_batch *b, int reps) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1e30;
    // a trial whose launches or timing fail counts as infinitely slow
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        float ms = 0.f;
        if (hipEventRecord(e0, b->cs) != hipSuccess || batch_frame(b, b->cs) != PR_OK ||
            hipEventRecord(e1, b->cs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            best = 1e30;
            break;
        }
        best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

std::string tune_key(const pr_batch *b) {
    int dev = 0;
    hipDeviceProp_t prop;
    const char *arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    double px = 0, tris = 0;
    for (const pr_view &v : b->views) {
        px += (double)v.width * v.height;
        tris += b->meshes[v.mesh].nt;
    }
    char key[256];
    snprintf(key, sizeof(key), "%s nv=%d px=2^%d tris=2^%d", arch, (int)b->views.size(),
             (int)lround(log2(std::max(px, 1.0))), (int)lround(log2(std::max(tris, 1.0))));
    for (char *c = key; *c; ++c)
        if (*c == '\t' || *c == '\n') *c = ' ';
    return key;
}

bool cache_lookup(const std::string &key, int &tile) {
    const char *path = getenv("PR_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool hit = false;
    while (fgets(line, sizeof(line), f)) {
        char *tab = strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        if (key == line) {
            int t = atoi(tab + 1);
            if (t == 8 || t == 16 || t == 32) {
                tile = t;
                hit = true;
            }
        }
    }
    fclose(f);
    return hit;
}

void cache_store(const std::string &key, int tile) {
    const char *path = getenv("PR_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s\t%d\n", key.c_str(), tile);
    fclose(f);
}

}  // namespace

extern "C" {

int pr_batch_create(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                    const pr_light *light, const float *const *albedo, int32_t *const *tri_id, float *const *depth,
                    uint8_t *const *rgba8, float *const *rgb32, pr_batch **out) {
    if (!out || !tuning || !light || !albedo || !tri_id || !depth) return PR_ERR_INVALID;
    *out = nullptr;
    if (!light_ok(light)) return PR_ERR_INVALID;
    pr_tuning probe = *tuning;
    if (probe.tile == 0) probe.tile = 16;
    if (probe.bin_capacity == 0) probe.bin_capacity = 1;
    size_t bytes = 0;
    int rc = pr_workspace_size(meshes, nm, views, nv, &probe, &bytes);
    if (rc) return rc;
    for (int v = 0; v < nv; ++v)
        if (!tri_id[v] || !depth[v]) return PR_ERR_INVALID;
    pr_batch *b = new pr_batch();
    b->meshes.assign(meshes, meshes + nm);
    b->views.assign(views, views + nv);
    b->profiles.resize(nv);
    for (int v = 0; v < nv; ++v)
        if (views[v].profile) {
            b->profiles[v] = *views[v].profile;
            b->views[v].profile = &b->profiles[v];
        }
    b->light = *light;
    b->albedo.assign(albedo, albedo + nm);
    b->ids.assign(tri_id, tri_id + nv);
    b->depth.assign(depth, depth + nv);
    b->rgba8.assign(nv, nullptr);
    b->rgb32.assign(nv, nullptr);
    for (int v = 0; v < nv; ++v) {
        if (rgba8) b->rgba8[v] = rgba8[v];
        if (rgb32) b->rgb32[v] = rgb32[v];
    }
    b->tuning = *tuning;
    b->tuning.flags |= PR_FLAG_PERSISTENT;
    if (b->tuning.bin_capacity == 0) {
        int64_t tris = 0;
        for (const pr_view &v : b->views) tris += meshes[v.mesh].nt;
        b->tuning.bin_capacity = (int32_t)std::min<int64_t>(2 * tris + 65536, INT32_MAX / 2);
    }
    if (hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return PR_ERR_HIP;
    }
    rc = PR_OK;
    if (tuning->tile == 0) {
        std::string key = tune_key(b);
        int cached = 0;
        if (cache_lookup(key, cached)) {
            b->tuning.tile = cached;
        } else {
            const int cand[3] = {8, 16, 32};
            double best = 1e30;
            int best_tile = 16;
            int32_t cap = b->tuning.bin_capacity;
            for (int i = 0; i < 3 && !rc; ++i) {
                b->tuning.tile = cand[i];
                b->tuning.bin_capacity = cap;
                rc = batch_fit(b);
                if (rc) break;
                double ms = batch_time(b, 3);
                b->trial_ms[i] = ms;
                if (ms < best) {
                    best = ms;
                    best_tile = cand[i];
                }
            }
            b->tuning.tile = best_tile;
            b->tuning.bin_capacity = cap;
            if (!rc) cache_store(key, best_tile);
        }
    }
    if (!rc) rc = batch_fit(b);
    if (!rc && hipStreamSynchronize(b->cs) != hipSuccess) rc = PR_ERR_HIP;
    if (!rc) {
        if (hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = PR_ERR_HIP;
        if (!rc) {
            int frc = batch_frame(b, b->cs);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->cs, &g);
            b->graph = g;
            if (frc) rc = frc;
            else if (e != hipSuccess || !g) rc = PR_ERR_HIP;
        }
        if (!rc && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) rc = PR_ERR_HIP;
    }
    if (rc) {
        pr_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PR_OK;
}

int pr_batch_launch(pr_batch *b, void *stream) {
    if (!b || !b->exec) return PR_ERR_INVALID;
    return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? PR_OK : PR_ERR_HIP;
}

int pr_batch_info(const pr_batch *b, pr_tuning *chosen, size_t *ws_bytes, double *trial_ms) {
    if (!b) return PR_ERR_INVALID;
    if (chosen) *chosen = b->tuning;
    if (ws_bytes) *ws_bytes = b->ws_bytes;
    if (trial_ms)
        for (int i = 0; i < 3; ++i) trial_ms[i] = b->trial_ms[i];
    return PR_OK;
}

int pr_batch_status(const pr_batch *b, pr_status *out, void *stream) {
    if (!b || !b->ws) return PR_ERR_INVALID;
    return pr_status_read(b->ws, b->ws_bytes, out, stream);
}

int pr_batch_destroy(pr_batch *b) {
    if (!b) return PR_OK;
    // teardown: errors of these calls leave nothing further to release
    if (b->cs) (void)hipStreamSynchronize(b->cs);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ws) (void)hipFree(b->ws);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    delete b;
    return PR_OK;
}

}  // extern "C"
