// pr_api.hip -- the C ABI declared in include/pr.h: argument checks,
// workspace layout and the launch sequence of each call.  One translation
// unit with the kernels (templates are instantiated here).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "pr.h"
#include "pr_kernels.hip"

using namespace prk;

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct ViewLayout {
    int tiles_x, tiles_y, ntiles, nparts, recw;
    int64_t cap;
    size_t rec, tb, vb, tcount, toff, part, pairs, lists;
};

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
    }
    if (tu->tile != 8 && tu->tile != 16 && tu->tile != 32) return PR_ERR_UNSUPPORTED;
    if (tu->bin_capacity < 1) return PR_ERR_INVALID;
    return PR_OK;
}

bool rolling(const pr_view &v) { return v.roll_dir[0] != 0.0f || v.roll_dir[1] != 0.0f; }

// Workspace: [status | view 0 | view 1 | ...], every buffer 256-aligned.
int layout(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tu, ViewLayout *L,
           size_t *total) {
    int rc = check_args(meshes, nm, views, nv, tu);
    if (rc) return rc;
    size_t off = up(sizeof(DevStatus));
    for (int v = 0; v < nv; ++v) {
        const pr_view &V = views[v];
        const pr_mesh &M = meshes[V.mesh];
        ViewLayout &l = L[v];
        l.tiles_x = (V.width + tu->tile - 1) / tu->tile;
        l.tiles_y = (V.height + tu->tile - 1) / tu->tile;
        l.ntiles = l.tiles_x * l.tiles_y;
        l.nparts = (l.ntiles + 1 + kScanBlock - 1) / kScanBlock;
        l.recw = rolling(V) ? kRecRoll : kRecStatic;
        l.cap = tu->bin_capacity;
        size_t nt = (size_t)M.nt;
        l.rec = off; off = up(off + nt * l.recw * sizeof(float4));
        l.tb = off; off = up(off + nt * sizeof(TriBound));
        l.vb = off; off = up(off + sizeof(ViewBlock));
        l.tcount = off; off = up(off + ((size_t)l.ntiles + 1) * 4);
        l.toff = off; off = up(off + ((size_t)l.ntiles + 1) * 4);
        l.part = off; off = up(off + (size_t)l.nparts * 4);
        l.pairs = off; off = up(off + (size_t)l.cap * sizeof(Pair));
        l.lists = off; off = up(off + (size_t)l.cap * 4);
    }
    *total = off;
    return PR_OK;
}

int check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (!ws || ((uintptr_t)ws & (kAlign - 1))) return PR_ERR_WORKSPACE;
    if (ws_bytes < need) return PR_ERR_WORKSPACE;
    return PR_OK;
}

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

template <typename T>
T *at(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

int launched() { return hipGetLastError() == hipSuccess ? PR_OK : PR_ERR_HIP; }

void fill_u32(void *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, (uint32_t *)p, v, n);
}

#define PR_PREP()                                                         \
    ViewLayout L[PR_MAX_VIEWS];                                           \
    size_t need = 0;                                                      \
    {                                                                     \
        int rc_ = layout(meshes, nm, views, nv, tuning, L, &need);        \
        if (rc_) return rc_;                                              \
        rc_ = check_ws(ws, ws_bytes, need);                               \
        if (rc_) return rc_;                                              \
    }                                                                     \
    hipStream_t s = (hipStream_t)stream;                                  \
    DevStatus *st = at<DevStatus>(ws, 0);

template <bool ROLL, int TILE>
void launch_raycast(int flags, const PixelConst &pc, const ViewLayout &l, void *ws, int32_t *id, float *depth, int v,
                    DevStatus *st, hipStream_t s) {
    using C = RayCfg<ROLL, TILE>;
    if (flags & PR_FLAG_COUNT)
        hipLaunchKernelGGL((k_raycast<ROLL, TILE, true>), dim3(l.ntiles), dim3(C::NT), 0, s, pc, l.tiles_x,
                           at<float4>(ws, l.rec), at<uint32_t>(ws, l.toff), at<int32_t>(ws, l.lists), id, depth, v, st);
    else
        hipLaunchKernelGGL((k_raycast<ROLL, TILE, false>), dim3(l.ntiles), dim3(C::NT), 0, s, pc, l.tiles_x,
                           at<float4>(ws, l.rec), at<uint32_t>(ws, l.toff), at<int32_t>(ws, l.lists), id, depth, v, st);
}

template <bool ROLL>
void dispatch_raycast(int tile, int flags, const PixelConst &pc, const ViewLayout &l, void *ws, int32_t *id,
                      float *depth, int v, DevStatus *st, hipStream_t s) {
    if (tile == 8) launch_raycast<ROLL, 8>(flags, pc, l, ws, id, depth, v, st, s);
    else if (tile == 16) launch_raycast<ROLL, 16>(flags, pc, l, ws, id, depth, v, st, s);
    else launch_raycast<ROLL, 32>(flags, pc, l, ws, id, depth, v, st, s);
}

}  // namespace

extern "C" {

int pr_workspace_size(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                      size_t *bytes) {
    if (!bytes) return PR_ERR_INVALID;
    ViewLayout L[PR_MAX_VIEWS];
    return layout(meshes, nm, views, nv, tuning, L, bytes);
}

int pr_bound(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
             size_t ws_bytes, void *stream) {
    PR_PREP();
    fill_u32(st, 0u, (int64_t)(sizeof(DevStatus) / 4), s);
    for (int v = 0; v < nv; ++v) {
        const pr_view &V = views[v];
        const pr_mesh &M = meshes[V.mesh];
        if (M.nt == 0) continue;
        dim3 grid((M.nt + 255) / 256);
        if (rolling(V))
            hipLaunchKernelGGL(k_bound<true>, grid, dim3(256), 0, s, V, M, tuning->tile, at<float4>(ws, L[v].rec),
                               at<TriBound>(ws, L[v].tb), st);
        else
            hipLaunchKernelGGL(k_bound<false>, grid, dim3(256), 0, s, V, M, tuning->tile, at<float4>(ws, L[v].rec),
                               at<TriBound>(ws, L[v].tb), st);
    }
    return launched();
}

int pr_bin(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
           size_t ws_bytes, void *stream) {
    PR_PREP();
    for (int v = 0; v < nv; ++v) {
        const pr_view &V = views[v];
        const pr_mesh &M = meshes[V.mesh];
        const ViewLayout &l = L[v];
        fill_u32(at<void>(ws, l.tcount), 0u, (int64_t)l.ntiles + 1, s);
        fill_u32(&st->num_pairs[v], 0u, 1, s);
        if (M.nt > 0)
            hipLaunchKernelGGL(k_bin, dim3((M.nt + 255) / 256), dim3(256), 0, s, V, M, tuning->tile, l.tiles_x,
                               at<TriBound>(ws, l.tb), at<uint32_t>(ws, l.tcount), at<Pair>(ws, l.pairs), l.cap,
                               &st->num_pairs[v]);
        int n = l.ntiles + 1;
        hipLaunchKernelGGL(k_scan_reduce, dim3(l.nparts), dim3(256), 0, s, at<uint32_t>(ws, l.tcount), n,
                           at<uint32_t>(ws, l.part));
        hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(1024), 0, s, at<uint32_t>(ws, l.part), l.nparts);
        hipLaunchKernelGGL(k_scan_apply, dim3(l.nparts), dim3(256), 0, s, at<uint32_t>(ws, l.tcount), n,
                           at<uint32_t>(ws, l.part), at<uint32_t>(ws, l.toff));
        int sb = (int)std::min<int64_t>(std::max<int64_t>((l.cap + 255) / 256, 1), 2048);
        hipLaunchKernelGGL(k_scatter, dim3(sb), dim3(256), 0, s, at<Pair>(ws, l.pairs), at<uint32_t>(ws, l.toff),
                           at<int32_t>(ws, l.lists), l.cap, v, st);
    }
    return launched();
}

int pr_raycast(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
               size_t ws_bytes, int32_t *const *tri_id, float *const *depth, void *stream) {
    if (!tri_id || !depth) return PR_ERR_INVALID;
    for (int v = 0; v < nv && v < PR_MAX_VIEWS; ++v)
        if (!tri_id[v] || !depth[v]) return PR_ERR_INVALID;
    PR_PREP();
    for (int v = 0; v < nv; ++v) {
        PixelConst pc = pixel_const(views[v]);
        if (rolling(views[v]))
            dispatch_raycast<true>(tuning->tile, tuning->flags, pc, L[v], ws, tri_id[v], depth[v], v, st, s);
        else
            dispatch_raycast<false>(tuning->tile, tuning->flags, pc, L[v], ws, tri_id[v], depth[v], v, st, s);
    }
    return launched();
}

int pr_shade(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
             size_t ws_bytes, const int32_t *const *tri_id, const pr_light *light, const float *const *albedo,
             uint8_t *const *rgba8, float *const *rgb32, void *stream) {
    if (!tri_id || !light || !albedo) return PR_ERR_INVALID;
    if (!isfinite(light->ambient) || !isfinite(light->dir_world[0]) || !isfinite(light->dir_world[1]) ||
        !isfinite(light->dir_world[2]))
        return PR_ERR_INVALID;
    for (int v = 0; v < nv && v < PR_MAX_VIEWS; ++v)
        if (!tri_id[v]) return PR_ERR_INVALID;
    for (int m = 0; m < nm; ++m)
        if (meshes && meshes[m].nt > 0 && !albedo[m]) return PR_ERR_INVALID;
    PR_PREP();
    for (int v = 0; v < nv; ++v) {
        const pr_view &V = views[v];
        const pr_mesh &M = meshes[V.mesh];
        PixelConst pc = pixel_const(V);
        int64_t np = (int64_t)V.width * V.height;
        uint8_t *o8 = rgba8 ? rgba8[v] : nullptr;
        float *o32 = rgb32 ? rgb32[v] : nullptr;
        if (!o8 && !o32) continue;
        dim3 grid((unsigned)((np + 255) / 256));
        hipLaunchKernelGGL(k_view_light, dim3(1), dim3(1), 0, s, V, *light, at<ViewBlock>(ws, L[v].vb));
        if (rolling(V))
            hipLaunchKernelGGL(k_shade<true>, grid, dim3(256), 0, s, pc, at<float4>(ws, L[v].rec), tri_id[v], M.tri,
                               albedo[V.mesh], at<ViewBlock>(ws, L[v].vb), light->ambient, M.nt, o8, o32);
        else
            hipLaunchKernelGGL(k_shade<false>, grid, dim3(256), 0, s, pc, at<float4>(ws, L[v].rec), tri_id[v], M.tri,
                               albedo[V.mesh], at<ViewBlock>(ws, L[v].vb), light->ambient, M.nt, o8, o32);
    }
    return launched();
}

int pr_backward(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning, void *ws,
                size_t ws_bytes, const int32_t *const *tri_id, const pr_light *light, const float *const *albedo,
                const float *const *dl_drgb, float *const *dv0, float *const *dv1, float *dpose0, float *dpose1,
                void *stream) {
    (void)meshes; (void)nm; (void)views; (void)nv; (void)tuning; (void)ws; (void)ws_bytes; (void)tri_id;
    (void)light; (void)albedo; (void)dl_drgb; (void)dv0; (void)dv1; (void)dpose0; (void)dpose1; (void)stream;
    return PR_ERR_UNSUPPORTED;
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
    out->tests = (int64_t)d.tests;
    out->hits = (int64_t)d.hits;
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
    const ViewLayout &l = L[view];
    *ntiles = l.ntiles;
    uint32_t total = 0;
    if (hipMemcpyAsync(&total, at<uint32_t>(ws, l.toff) + l.ntiles, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        return PR_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PR_ERR_HIP;
    *npairs = total;
    if (offsets &&
        hipMemcpyAsync(offsets, at<void>(ws, l.toff), ((size_t)l.ntiles + 1) * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
        return PR_ERR_HIP;
    if (lists) {
        if (cap < (int64_t)total || (int64_t)total > l.cap) return PR_ERR_INVALID;
        if (total && hipMemcpyAsync(lists, at<void>(ws, l.lists), (size_t)total * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
            return PR_ERR_HIP;
    }
    return hipStreamSynchronize(s) == hipSuccess ? PR_OK : PR_ERR_HIP;
}

// ---------------------------------------------------------------------------
// host evaluation of the bound (tests)
// ---------------------------------------------------------------------------
int pr_host_time_interval(const pr_mesh *mesh, int32_t f, const pr_view *view, double *t) {
    if (!mesh || !view || !t || f < 0 || f >= mesh->nt) return -1;
    prg::Geom g;
    prg::make_geom(*view, g);
    double Ps[3][3], Pe[3][3];
    int32_t idx[3];
    if (!prg::load_tri(mesh->v0, mesh->v1, mesh->tri, mesh->nv, f, g, Ps, Pe, idx)) return 0;
    return prg::time_window(g, Ps, Pe, t);
}

int pr_host_tile_rect(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t tile, int32_t *rect) {
    if (!mesh || !view || !rect || f < 0 || f >= mesh->nt || tile < 1) return -1;
    prg::Geom g;
    prg::make_geom(*view, g);
    double Ps[3][3], Pe[3][3], win[2], box[4];
    int32_t idx[3];
    if (!prg::load_tri(mesh->v0, mesh->v1, mesh->tri, mesh->nv, f, g, Ps, Pe, idx)) return 0;
    int kind = prg::time_window(g, Ps, Pe, win);
    if (kind == prg::kCulled) return 0;
    prg::display_box(g, Ps, Pe, win[0], win[1], kind, box);
    int r[4];
    if (!prg::tile_rect(g, box, tile, r)) return 0;
    for (int k = 0; k < 4; ++k) rect[k] = r[k];
    return 1;
}

int pr_host_tile_test(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t tile, int32_t tx, int32_t ty) {
    if (!mesh || !view || f < 0 || f >= mesh->nt || tile < 1) return -1;
    prg::Geom g;
    prg::make_geom(*view, g);
    double Ps[3][3], Pe[3][3], win[2], box[4];
    int32_t idx[3];
    if (!prg::load_tri(mesh->v0, mesh->v1, mesh->tri, mesh->nv, f, g, Ps, Pe, idx)) return 0;
    int kind = prg::time_window(g, Ps, Pe, win);
    if (kind == prg::kCulled) return 0;
    prg::display_box(g, Ps, Pe, win[0], win[1], kind, box);
    int r[4];
    if (!prg::tile_rect(g, box, tile, r)) return 0;
    if (tx < r[0] || tx > r[2] || ty < r[1] || ty > r[3]) return 0;
    double w[4];
    if (kind == prg::kWindow) { w[0] = win[0]; w[1] = win[1]; w[2] = w[3] = 0.0; }
    else for (int k = 0; k < 4; ++k) w[k] = box[k];
    return prg::tile_test(g, Ps, Pe, kind, w, w, tile, tx, ty) ? 1 : 0;
}

}  // extern "C"
