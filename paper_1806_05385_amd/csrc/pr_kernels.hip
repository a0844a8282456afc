// pr_kernels.hip -- gfx950 kernels of the perceptual rasterization hot path.
//
// Every pass covers all views of a call in one launch: views are laid end to
// end in a global triangle / tile / pixel index space and a block finds its
// view in the workspace's view table.
//
//   k_bound    one lane per triangle, FP64: camera-space vertices, near plane,
//              rolling time window, foveated tile rectangle, FP32
//              intersection record (Sec. 3.2 "Bounding", Sec. 4)
//   k_tiles    four lanes per tile: display box of its pixel centres (and of
//              each quadrant's) and its frame-time window
//   k_bin      one block per 256 triangles: every (triangle, tile) candidate
//              of the block's rectangles tested conservatively; the round's
//              survivors counted per tile in LDS take their list places with
//              one global atomic per tile
//   k_scan     exclusive scan of per-tile counts (single pass, look-back)
//   k_scatter  pairs -> per-tile triangle lists
//   k_raycast  one wave per 8x8 cell: every pixel's ray (foveated position,
//   (_queue)   rolling time) tested against the cell's triangles of the tile
//              list on the matrix cores, four triangles x 64 pixels per
//              group; nearest packed (depth bits << 32 | id) kept in
//              registers (Sec. 3.2 "Intersection"); the persistent form
//              walks the tiles longest list first and may shade each cell
//   k_shade    rolling shading of resolved ids (Sec. 3.2 "Shading"): Lambert
//              and a Blinn-Phong highlight with the eye at the pixel's time
//   k_gbuffer  normals, barycentrics and pixel density of resolved ids
//   k_bwd_*    frozen-visibility gradient of the shaded image
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pr_geom.h"
#include "pr_kernels.h"

namespace prk {

// ---------------------------------------------------------------------------
// wave / block helpers (wave64)
// ---------------------------------------------------------------------------
__device__ inline unsigned lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ inline int wave_incl_scan(int v) {
    int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int n = __shfl_up(v, o, 64);
        if (lane >= o) v += n;
    }
    return v;
}

// Exclusive block scan for blockDim.x a multiple of 64 (<= 1024).
__device__ inline int block_excl_scan(int v, int *lds, int &total) {
    int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    if (threadIdx.x < 64) {
        int w = threadIdx.x < nw ? lds[threadIdx.x] : 0;
        int wi = wave_incl_scan(w);
        if (threadIdx.x < nw) lds[32 + threadIdx.x] = wi - w;
        if (threadIdx.x == nw - 1) lds[64] = wi;
    }
    __syncthreads();
    int out = inc - v + lds[32 + wid];
    total = lds[64];
    __syncthreads();
    return out;
}

// The same in 64 bits (candidate slot offsets: a frame's candidates may
// exceed 2^31 before the capacity check rejects it).
__device__ inline long long wave_incl_scan64(long long v) {
    int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        long long n = __shfl_up(v, o, 64);
        if (lane >= o) v += n;
    }
    return v;
}

__device__ inline long long block_excl_scan64(long long v, long long *lds, long long &total) {
    int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    long long inc = wave_incl_scan64(v);
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    if (threadIdx.x < 64) {
        long long w = threadIdx.x < nw ? lds[threadIdx.x] : 0;
        long long wi = wave_incl_scan64(w);
        if (threadIdx.x < nw) lds[32 + threadIdx.x] = wi - w;
        if (threadIdx.x == nw - 1) lds[64] = wi;
    }
    __syncthreads();
    long long out = inc - v + lds[32 + wid];
    total = lds[64];
    __syncthreads();
    return out;
}

// ---------------------------------------------------------------------------
// small fills (used instead of hipMemsetAsync so the frame can be captured)
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// view table
// ---------------------------------------------------------------------------
// Index of the last view whose base <= key (bases ascending, nv entries).
__device__ __forceinline__ int find_view(const int32_t *base, int nv, int key) {
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= key) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The views arrive complete (geometry included, computed on the host): the
// block copies them word by word into the view table.
// Thread i of n threads: its share of writing pack p into the view table
// (and of clearing the status block when p asks for it).
__device__ __forceinline__ void write_pack(const ViewPack &p, ViewTable *__restrict__ T, DevStatus *__restrict__ st,
                                           int i, int n) {
    if (p.first == 0 && p.reset_status) {   // the frame's first launch resets the status block
        uint32_t *w = reinterpret_cast<uint32_t *>(st);
        for (int k = i; k < (int)(sizeof(DevStatus) / 4); k += n) w[k] = 0u;
    }
    static_assert(sizeof(ViewDev) % 4 == 0, "ViewDev is whole words");
    constexpr int kWords = (int)(sizeof(ViewDev) / 4);
    for (int k = i; k < p.count * kWords; k += n) {
        const int v = k / kWords, wd = k - v * kWords;
        reinterpret_cast<uint32_t *>(&T->v[p.first + v])[wd] = reinterpret_cast<const uint32_t *>(&p.v[v])[wd];
    }
    if (i < p.count) {
        const ViewDev &v = p.v[i];
        T->vtx_block0[p.first + i] = v.vtx_block0;
        T->tri_block0[p.first + i] = v.tri_block0;
        T->tile_base[p.first + i] = v.tile_base;
        T->pix_block0[p.first + i] = v.pix_block0;
    }
    if (i == 0 && p.first + p.count == p.nv) {
        T->nv = p.nv;
        T->total_tiles = p.total_tiles;
        T->total_tri_blocks = p.total_tri_blocks;
        T->total_pix_blocks = p.total_pix_blocks;
        T->total_vtx_blocks = p.total_vtx_blocks;
        T->vtx_block0[p.nv] = p.total_vtx_blocks;
        T->tri_block0[p.nv] = p.total_tri_blocks;
        T->tile_base[p.nv] = p.total_tiles;
        T->pix_block0[p.nv] = p.total_pix_blocks;
    }
}

__global__ void k_write_views(ViewPack p, ViewTable *__restrict__ T, DevStatus *__restrict__ st) {
    write_pack(p, T, st, threadIdx.x, blockDim.x);
}

// One view's tabulated profiles into the workspace (before k_write_views).
__global__ void k_write_profile(ProfDev p, ProfDev *__restrict__ dst) {
    const int i = threadIdx.x;
    if (i == 0) { dst->nc = p.nc; dst->nl = p.nl; dst->pad[0] = dst->pad[1] = 0; }
    if (i < PR_PROFILE_MAX) { dst->c[i] = p.c[i]; dst->l[i] = p.l[i]; }
}

// Camera-space light direction at each view's start and end.
__global__ void k_view_light(ViewTable *__restrict__ T, pr_light light) {
    int v = threadIdx.x;
    if (v >= T->nv) return;
    const prg::Geom &g = T->v[v].g;
    double l[3] = {light.dir_world[0], light.dir_world[1], light.dir_world[2]};
    for (int r = 0; r < 3; ++r) {
        T->v[v].light0[r] = (float)(g.R0[3 * r] * l[0] + g.R0[3 * r + 1] * l[1] + g.R0[3 * r + 2] * l[2]);
        T->v[v].light1[r] = (float)(g.R1[3 * r] * l[0] + g.R1[3 * r + 1] * l[1] + g.R1[3 * r + 2] * l[2]);
    }
}

// ---------------------------------------------------------------------------
// bound
// ---------------------------------------------------------------------------
__device__ inline void dcross(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double ddot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Per-triangle bound and record of one triangle (k_bound).  Returns the
// number of (triangle, tile) candidates of its tile rectangle.
// Coalesced stores of per-lane rows: lane j holds rows [r0, r0 + n) (n <= 4)
// of item j of the wave, item j's rows at base + j * stride + r0.  The rows
// pass through the wave's 320-float4 LDS buffer so that each store
// instruction writes 64-byte runs (four rows of one item) instead of one
// row per lane; items whose bit of `valid` is clear are not written.
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row q of item j sits in the buffer at 5 j + q: the sixteen-byte writes of
// eight consecutive lanes (80 bytes apart) hit eight different 16-byte bank
// groups.
template <int N>
__device__ __forceinline__ void wave_rows(float4 *__restrict__ base, int stride, int r0, const float4 *v,
                                          unsigned long long valid, float4 *s_buf) {
    const int lane = __lane_id();
#pragma unroll
    for (int q = 0; q < N; ++q) s_buf[5 * lane + q] = v[q];
    wave_fence();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 64 * i + lane, j = k >> 2, q = k & 3;
        if (q < N && ((valid >> j) & 1ull)) base[(int64_t)j * stride + r0 + q] = s_buf[5 * j + q];
    }
    wave_fence();
}

// Triangle f of the view (every lane of the wave calls it; lanes with valid
// false compute on an in-range triangle and store nothing); f0: the wave's
// first triangle (wave-uniform; lane j's triangle is f0 + j).  nonfinite:
// the (valid) triangle has an index out of range or a non-finite vertex.
template <bool PROF>
__device__ __forceinline__ int bound_tri(const ViewDev &vd, int f, bool valid, int f0, float4 *__restrict__ rec,
                                         TriBound *__restrict__ tb, bool &nonfinite, float4 *s_buf) {
    const prg::Geom &g = vd.g;
    double Ps[3][3], Pe[3][3];
    int32_t idx[3];
    bool ok = prg::load_tri(vd.mesh.v0, vd.mesh.v1, vd.mesh.tri, vd.mesh.nv, f, g, Ps, Pe, idx);
    TriBound b;
    b.rect[0] = 1; b.rect[1] = 1; b.rect[2] = 0; b.rect[3] = 0;
    b.kind = prg::kCulled;
    b.pad = 0;
    b.pad2[0] = b.pad2[1] = 0;
    for (int k = 0; k < 4; ++k) b.w[k] = 0.0;
    nonfinite = valid && !ok;
    if (ok) {
        double win[2];
        int kind = prg::time_window<PROF>(g, Ps, Pe, win, vd.bound);
        if (kind != prg::kCulled) {
            double box[4];
            prg::display_box(g, Ps, Pe, win[0], win[1], kind, box);
            int rect[4];
            if (prg::tile_rect<PROF>(g, box, vd.tile, rect)) {
                for (int k = 0; k < 4; ++k) b.rect[k] = rect[k];
                b.kind = kind;
                if (kind == prg::kWindow) { b.w[0] = win[0]; b.w[1] = win[1]; }
                else for (int k = 0; k < 4; ++k) b.w[k] = box[k];
            }
        }
    }
    const unsigned long long vmask = __ballot(valid);
    {
        float4 w[4];
        static_assert(sizeof(TriBound) == sizeof(w), "TriBound is 4 float4");
        __builtin_memcpy(w, &b, sizeof(w));
        wave_rows<4>(reinterpret_cast<float4 *>(tb + vd.tri_off + f0), 4, 0, w, vmask, s_buf);
    }

    // Intersection record.  Edge k joins vertices a = k+1, b = k+2.  Its
    // plane normal is computed from the lower-indexed mesh vertex as
    // P_lo x (P_hi - P_lo) and negated when a > b, so the two triangles
    // sharing an edge hold exactly negated coefficients (watertight).
    double A[3][3], B[3][3], C[3][3];
    for (int k = 0; k < 3; ++k) {
        int a = (k + 1) % 3, bb = (k + 2) % 3;
        bool flip = idx[a] > idx[bb];
        int lo = flip ? bb : a, hi = flip ? a : bb;
        double s = flip ? -1.0 : 1.0;
        double P0[3], dP[3], E0[3], dE[3];
        for (int r = 0; r < 3; ++r) {
            P0[r] = Ps[lo][r];
            dP[r] = Pe[lo][r] - Ps[lo][r];
            E0[r] = Ps[hi][r] - Ps[lo][r];
            dE[r] = (Pe[hi][r] - Pe[lo][r]) - E0[r];
        }
        double t1[3], t2[3];
        dcross(P0, E0, A[k]);
        dcross(P0, dE, t1);
        dcross(dP, E0, t2);
        dcross(dP, dE, C[k]);
        for (int r = 0; r < 3; ++r) {
            A[k][r] *= s;
            B[k][r] = s * (t1[r] + t2[r]);
            C[k][r] *= s;
        }
    }
    double dq[3];
    for (int r = 0; r < 3; ++r) dq[r] = Pe[0][r] - Ps[0][r];
    // D(t) = P0(t) . c_0(t), P0(t) = Ps0 + t dq
    double d0 = ddot(Ps[0], A[0]);
    double d1 = ddot(Ps[0], B[0]) + ddot(dq, A[0]);
    double d2 = ddot(Ps[0], C[0]) + ddot(dq, B[0]);
    double d3 = ddot(dq, C[0]);
    // N(t) = E1(t) x E2(t), E_i(t) = (P_i - P_0)(t) linear in t
    double E1[3], E2[3], dE1[3], dE2[3], N0[3], N1[3], N2[3], u1[3], u2[3];
    for (int r = 0; r < 3; ++r) {
        E1[r] = Ps[1][r] - Ps[0][r];
        E2[r] = Ps[2][r] - Ps[0][r];
        dE1[r] = (Pe[1][r] - Pe[0][r]) - E1[r];
        dE2[r] = (Pe[2][r] - Pe[0][r]) - E2[r];
    }
    dcross(E1, E2, N0);
    dcross(E1, dE2, u1);
    dcross(dE1, E2, u2);
    dcross(dE1, dE2, N2);
    for (int r = 0; r < 3; ++r) N1[r] = u1[r] + u2[r];
    if (!ok) {
        d0 = d1 = d2 = d3 = 0.0;
        for (int r = 0; r < 3; ++r) N0[r] = N1[r] = N2[r] = 0.0;
    }
    // Record (layout in RecLayout): M[k][o] = coefficient of ray term k in
    // output o (e_0, e_1, e_2: the edge functions r . c_o(t); S = r . N(t)),
    // the terms being (rx, ry, t rx, t ry, t, t^2 rx, t^2 ry, t^2) and the
    // constant (term 1) stored apart.
    double M[8][4], K4[4];
    for (int o = 0; o < 4; ++o) {
        const double *a0 = o < 3 ? A[o] : N0, *b0 = o < 3 ? B[o] : N1, *c0 = o < 3 ? C[o] : N2;
        M[0][o] = a0[0]; M[1][o] = a0[1];
        M[2][o] = b0[0]; M[3][o] = b0[1]; M[4][o] = b0[2];
        M[5][o] = c0[0]; M[6][o] = c0[1]; M[7][o] = c0[2];
        K4[o] = a0[2];
    }
    if (vd.rolling) {
        float out[44];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int o = 0; o < 4; ++o) out[4 * k + o] = (float)M[k][o];
#pragma unroll
        for (int o = 0; o < 4; ++o) out[32 + o] = (float)K4[o];
        out[36] = (float)d0; out[37] = (float)d1; out[38] = (float)d2; out[39] = (float)d3;
        out[40] = __int_as_float(f);
        out[41] = out[42] = out[43] = 0.0f;
        float4 w[kRecRoll];
#pragma unroll
        for (int q = 0; q < kRecRoll; ++q) w[q] = make_float4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
        float4 *dst = rec + vd.rec_off + (int64_t)f0 * kRecRoll;
        wave_rows<4>(dst, kRecRoll, 0, w, vmask, s_buf);
        wave_rows<4>(dst, kRecRoll, 4, w + 4, vmask, s_buf);
        wave_rows<3>(dst, kRecRoll, 8, w + 8, vmask, s_buf);
    } else {
        float out[24];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            out[o] = (float)M[0][o];
            out[4 + o] = (float)M[1][o];
            out[8 + o] = 0.0f;
            out[12 + o] = 0.0f;
            out[16 + o] = (float)K4[o];
        }
        out[20] = (float)d0;
        out[21] = __int_as_float(f);
        out[22] = out[23] = 0.0f;
        float4 w[kRecStatic];
#pragma unroll
        for (int q = 0; q < kRecStatic; ++q) w[q] = make_float4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
        float4 *dst = rec + vd.rec_off + (int64_t)f0 * kRecStatic;
        wave_rows<4>(dst, kRecStatic, 0, w, vmask, s_buf);
        wave_rows<2>(dst, kRecStatic, 4, w + 4, vmask, s_buf);
    }
    return (!valid || b.kind == prg::kCulled) ? 0 : (b.rect[2] - b.rect[0] + 1) * (b.rect[3] - b.rect[1] + 1);
}

// One lane per triangle; the block's candidate total (the binning block of
// the same 256 triangles) goes to bcand[block], its count of triangles with
// bad data to bnf[block] (k_tiles adds them to the status block).
// PROF: some view of the call has a tabulated profile or a lens (false: the
// power-law code alone, with its own register allocation).  PACK: the
// call's views come in the kernel arguments (all of them: at most
// kViewsPerWrite), and block 0 also writes them into the view table and
// clears the status block for the kernels after (none of this kernel's
// blocks reads either); otherwise the view table was written before.
static_assert(kViewsPerWrite == 2, "k_bound takes a packed view by constant index 0 or 1");
template <bool PROF, bool PACK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_bound(
    ViewPack P, ViewTable *__restrict__ T, float4 *__restrict__ rec, TriBound *__restrict__ tb,
    DevStatus *__restrict__ st, int32_t *__restrict__ bcand, int32_t *__restrict__ bnf) {
    __shared__ int s_tmp[72];
    __shared__ float4 s_rows[4][320];   // per-wave store staging (rows padded to 5 per item)
    __shared__ int s_nf;
    if (PACK && blockIdx.x == 0) write_pack(P, T, st, threadIdx.x, 256);
    if (threadIdx.x == 0) s_nf = 0;
    __syncthreads();
    int v;
    if (PACK) v = P.count > 1 && (int)blockIdx.x >= P.v[1].tri_block0 ? 1 : 0;
    else v = find_view(T->tri_block0, T->nv, blockIdx.x);
    auto run = [&](const ViewDev &vd, bool &nonfinite) {
        const int f = (blockIdx.x - vd.tri_block0) * 256 + threadIdx.x;
        // every lane takes part in the wave's coalesced stores; lanes past
        // the mesh work on triangle 0 (a block exists only for nt >= 1)
        const bool valid = f < vd.mesh.nt;
        const int fw0 = (blockIdx.x - vd.tri_block0) * 256 + (int)(threadIdx.x & ~63u);
        return bound_tri<PROF>(vd, valid ? f : 0, valid, fw0, rec, tb, nonfinite, s_rows[threadIdx.x >> 6]);
    };
    bool nonfinite = false;
    // (the packed views by constant index: a dynamic one into the kernel
    // arguments costs the bound spilled registers)
    const int cnt = !PACK ? run(T->v[v], nonfinite) : (v == 0 ? run(P.v[0], nonfinite) : run(P.v[1], nonfinite));
    if (nonfinite) atomicAdd(&s_nf, 1);
    int total;
    block_excl_scan(cnt, s_tmp, total);   // (its barriers also order the count above)
    if (threadIdx.x == 0) {
        bcand[blockIdx.x] = total;
        bnf[blockIdx.x] = s_nf;
    }
}

// ---------------------------------------------------------------------------
// per-tile display boxes
// ---------------------------------------------------------------------------
// Binning blocks with at least this many candidates are dispatched first.
constexpr int kHeavyCand = 512;
constexpr int kPermItems = 8;

// Four lanes per tile, lane q computing quadrant q's box; a split tile's box
// is the union of its quadrants' boxes (every pixel centre of the tile lies
// in its quadrant's box), an unsplit tile's box is computed by lane 0.  The
// kernel also clears the binning counters and scans the binning blocks'
// candidate totals in chunks of 256; its last block (one more than the
// tiles and chunks need) writes the binning blocks' dispatch order.
template <bool PROF>   // as k_bound's
__global__ __launch_bounds__(256) void k_tiles(const ViewTable *__restrict__ T, TileInfo *__restrict__ ti,
                                               uint32_t *__restrict__ tcount, Sched *__restrict__ S, const int32_t *__restrict__ bcand,
                                               const int32_t *__restrict__ bnf,
                                               int64_t *__restrict__ boff, int64_t *__restrict__ part,
                                               DevStatus *__restrict__ st, int32_t *__restrict__ bperm,
                                               unsigned long long *__restrict__ scan_flags, int nscan) {
    __shared__ int s_tmp[72];
    __shared__ long long s_tmp64[72];
    const int gid = blockIdx.x * 256 + threadIdx.x;
    const int gt = gid >> 2, q = gid & 3;
    const bool valid = gt < T->total_tiles;
    // clear the counters the binning pass accumulates into, and the tile
    // scan's block flags
    if (q == 0 && gt <= T->total_tiles) tcount[gt] = 0u;
    for (int e = gid; e < kSchedCounters; e += (int)gridDim.x * 256) reinterpret_cast<uint32_t *>(S)[e] = 0u;
    for (int e = gid; e < nscan; e += (int)gridDim.x * 256) scan_flags[e] = 0ull;
    if (blockIdx.x < (T->total_tri_blocks + 255) / 256) {
        // the binning blocks' candidate slots: local exclusive scan of 256
        // block totals here; k_bin adds the totals of the chunks before.
        // A block's total fits 32 bits (256 rectangles of at most 2^22
        // tiles), a chunk's does not.
        const int nb = T->total_tri_blocks;
        const int b = blockIdx.x * 256 + threadIdx.x;
        const long long c = b < nb ? bcand[b] : 0;
        long long tot;
        const long long ex = block_excl_scan64(c, s_tmp64, tot);
        if (b < nb) boff[b] = ex;
        long long nf;   // the chunk's triangles with bad data
        block_excl_scan64(b < nb ? bnf[b] : 0, s_tmp64, nf);
        if (threadIdx.x == 0) {
            part[blockIdx.x] = tot;
            atomicAdd(&st->pairs_required, (unsigned long long)tot);
            if (nf) atomicAdd(&st->nonfinite, (int)nf);
        }
    }
    if (blockIdx.x == gridDim.x - 1) {
        // (the grid's extra last block, which has no tiles and runs beside
        // the others) Dispatch order of the binning blocks: the few with
        // many candidates (large triangles near the eye) first, the others
        // in index order; started last, the heavy ones would set the
        // binning's end.  A stable partition: heavy block i goes to place
        // (heavy blocks before it), light block i to nheavy + (light blocks
        // before it).  One pass when the blocks fit one round of the scan
        // (its total is then nheavy), else a counting pass first.
        const int nb = T->total_tri_blocks;
        int nheavy = 0;
        for (int b0 = 0; nb > 256 * kPermItems && b0 < nb; b0 += 256 * kPermItems) {
            const int i0 = b0 + (int)threadIdx.x * kPermItems;
            int cnt = 0;
#pragma unroll
            for (int k = 0; k < kPermItems; ++k) cnt += i0 + k < nb && bcand[i0 + k] >= kHeavyCand;
            int tot;
            block_excl_scan(cnt, s_tmp, tot);
            nheavy += tot;
        }
        int hbase = 0;
        for (int b0 = 0; b0 < nb; b0 += 256 * kPermItems) {
            const int i0 = b0 + (int)threadIdx.x * kPermItems;
            bool fl[kPermItems];
            int cnt = 0;
#pragma unroll
            for (int k = 0; k < kPermItems; ++k) {
                fl[k] = i0 + k < nb && bcand[i0 + k] >= kHeavyCand;
                cnt += fl[k];
            }
            int tot;
            int hp = block_excl_scan(cnt, s_tmp, tot) + hbase;
            if (nb <= 256 * kPermItems) nheavy = tot;
#pragma unroll
            for (int k = 0; k < kPermItems; ++k) {
                const int i = i0 + k;
                if (i < nb) bperm[fl[k] ? hp : nheavy + (i - hp)] = i;
                hp += fl[k];
            }
            hbase += tot;
        }
    }
    const int v = find_view(T->tile_base, T->nv, valid ? gt : 0);
    const ViewDev &vd = T->v[v];
    const prg::Geom &g = vd.g;
    const int lt = (valid ? gt : 0) - vd.tile_base;
    const int tx = lt % vd.tiles_x, ty = lt / vd.tiles_x;
    const bool split = prg::split_quads(vd.tile);
    const bool prof = PROF && (vd.pc.mode == 3 || vd.pc.lens);
    double qb[4] = {1e300, -1e300, 1e300, -1e300}, qp[4] = {1e300, -1e300, 1e300, -1e300};
    bool qok = false;
    if (valid && split)
        qok = prof ? prg::quad_display<true>(g, vd.tile, tx, ty, q, qb, qp)
                   : prg::quad_display<false>(g, vd.tile, tx, ty, q, qb);
    // the quadrants' ray (undistorted) boxes, and through a lens their panel
    // boxes (which set the times)
    double box[4] = {qb[0], qb[1], qb[2], qb[3]};
    if (!qok) { box[0] = box[2] = 1e300; box[1] = box[3] = -1e300; }
#pragma unroll
    for (int o = 1; o < 4; o <<= 1) {   // union over the tile's four lanes
        box[0] = prg::dmin(box[0], __shfl_xor(box[0], o, 64));
        box[1] = prg::dmax(box[1], __shfl_xor(box[1], o, 64));
        box[2] = prg::dmin(box[2], __shfl_xor(box[2], o, 64));
        box[3] = prg::dmax(box[3], __shfl_xor(box[3], o, 64));
    }
    double pbox[4] = {box[0], box[1], box[2], box[3]};
    if (PROF && vd.pc.lens) {
        for (int k = 0; k < 4; ++k) pbox[k] = qok ? qp[k] : ((k & 1) ? -1e300 : 1e300);
#pragma unroll
        for (int o = 1; o < 4; o <<= 1) {
            pbox[0] = prg::dmin(pbox[0], __shfl_xor(pbox[0], o, 64));
            pbox[1] = prg::dmax(pbox[1], __shfl_xor(pbox[1], o, 64));
            pbox[2] = prg::dmin(pbox[2], __shfl_xor(pbox[2], o, 64));
            pbox[3] = prg::dmax(pbox[3], __shfl_xor(pbox[3], o, 64));
        }
    }
    const unsigned long long okb = __ballot(qok);
    if (!valid) return;
    TileInfo &t = ti[gt];
    if (split) {
        t.qb[q][0] = qok ? prg::f32_down(qb[0]) : 0.0f;
        t.qb[q][1] = qok ? prg::f32_up(qb[1]) : 0.0f;
        t.qb[q][2] = qok ? prg::f32_down(qb[2]) : 0.0f;
        t.qb[q][3] = qok ? prg::f32_up(qb[3]) : 0.0f;
    }
    if (q != 0) return;
    double tw[2];
    if (split) {
        prg::tile_time(g, pbox, tw);
        t.qvalid = (int32_t)((okb >> (__lane_id() & ~3)) & 0xFull);
    } else {
        if (prof) prg::tile_display<true>(g, vd.tile, tx, ty, box, tw);
        else prg::tile_display<false>(g, vd.tile, tx, ty, box, tw);
        t.qvalid = 0;
        for (int k = 0; k < 4; ++k)
            for (int r = 0; r < 4; ++r) t.qb[k][r] = 0.0f;
    }
    t.box[0] = prg::f32_down(box[0]);
    t.box[1] = prg::f32_up(box[1]);
    t.box[2] = prg::f32_down(box[2]);
    t.box[3] = prg::f32_up(box[3]);
    t.tw[0] = prg::f32_down(tw[0]);
    t.tw[1] = prg::f32_up(tw[1]);
    t.pad = 0;
}

// ---------------------------------------------------------------------------
// bin
// ---------------------------------------------------------------------------
// Candidate pairs, one slot per candidate, as three arrays of cap words
// (separate word stores: no register copies into store tuples).
struct Pairs {
    int32_t *tile;     // global tile, -1: rejected candidate
    uint32_t *slot;    // slot in the tile's list
    uint32_t *entry;   // list entry (triangle index | quadrant mask)
};

// Each round gives every thread up to kBinPer consecutive candidates
// (mostly of one or two triangles, found with one binary search over the
// block's candidate prefix).  A thread keeps its candidates' quadrant masks
// in a register (4 bits each); the round's survivors are counted per tile in
// LDS and reserve their places in the tiles' lists with one global atomic
// per tile.  A survivor's list entry carries its quadrant mask above the
// triangle index.
constexpr int kBinPer = 4;
// LDS table of a round's survivors per tile: 2^kBinHashBits entries,
// kBinProbe linear probes.
constexpr int kBinHashBits = 10;
constexpr int kBinHash = 1 << kBinHashBits;
constexpr int kBinProbe = 8;

// A thread's walk over its consecutive candidates: triangle q of the block,
// candidate `local` of its tile rectangle, the rectangle column lx and the
// global tile gt.  Only the start divides; each step moves one tile right
// or to the next row or triangle.
struct BinCursor {
    int q, local, lx, gt;
};

__device__ __forceinline__ int bin_count(const int *s_pref, int q) { return s_pref[q + 1] - s_pref[q]; }

__device__ __forceinline__ BinCursor bin_start(const ViewDev &vd, const int (*s_rect)[5], const int *s_pref, int q,
                                               int local) {
    while (local >= bin_count(s_pref, q)) { ++q; local = 0; }
    const int rw = s_rect[q][2] - s_rect[q][0] + 1;
    const int lx = local % rw, ly = local / rw;
    return BinCursor{q, local, lx, vd.tile_base + (s_rect[q][1] + ly) * vd.tiles_x + s_rect[q][0] + lx};
}

// Next candidate (the caller knows one follows).
__device__ __forceinline__ void bin_step(BinCursor &c, const ViewDev &vd, const int (*s_rect)[5], const int *s_pref) {
    ++c.local;
    if (c.local >= bin_count(s_pref, c.q)) {
        do { ++c.q; } while (bin_count(s_pref, c.q) == 0);
        c.local = 0;
        c.lx = 0;
        c.gt = vd.tile_base + s_rect[c.q][1] * vd.tiles_x + s_rect[c.q][0];
        return;
    }
    const int rw = s_rect[c.q][2] - s_rect[c.q][0] + 1;
    ++c.lx;
    ++c.gt;
    if (c.lx == rw) {
        c.lx = 0;
        c.gt += vd.tiles_x - rw;
    }
}

// One block per kBinTris triangles.  Each triangle's test record is built
// once (FP64, rounded outwards to FP32) into LDS; each round gives every
// thread `per` consecutive candidates, per = ceil(candidates / kBinThreads)
// up to kBinPer, tested in FP32 against the tile's FP32 boxes.
constexpr int kBinTris = 256;
// threads of a binning block: the triangles' records are built by the
// first kBinTris, the candidates are shared by all
constexpr int kBinThreads = 512;

// FOV: some view of the call uses a foveated per-tile test other than the
// exact one (its general form; false keeps that code out).
template <bool FOV>
__global__ __launch_bounds__(kBinThreads) void k_bin(const ViewTable *__restrict__ T, const TriBound *__restrict__ tb,
                                             const TileInfo *__restrict__ ti, uint32_t *__restrict__ tcount,
                                             const int64_t *__restrict__ boff, const int64_t *__restrict__ bpart,
                                             Pairs pairs, int64_t cap, const int32_t *__restrict__ bperm,
                                             const DevStatus *__restrict__ st) {
    // A frame whose candidates exceed the capacity (k_tiles summed them) is
    // not binned at all: its pairs would not fit, the overflow is reported
    // and the ray cast writes misses.
    if ((int64_t)st->pairs_required > cap) return;
    // odd row strides (33 and 5 words) keep lanes reading different
    // triangles on different LDS banks
    __shared__ uint32_t s_sat[kBinTris][33];
    __shared__ int s_rect[kBinTris][5];
    __shared__ int s_pref[kBinTris + 1];
    __shared__ int s_tmp[72];
    __shared__ long long s_tmp64[72];
    // survivors per tile of the current round (open addressing on the tile)
    __shared__ int32_t s_hkey[kBinHash];
    __shared__ uint32_t s_hcnt[kBinHash], s_hbase[kBinHash];
    const int j = threadIdx.x;
    for (int e = j; e < kBinHash; e += kBinThreads) {
        s_hkey[e] = -1;
        s_hcnt[e] = 0u;
    }
    {
        const int bb = bperm[blockIdx.x];   // this block's 256 triangles (heavy blocks first)
        const int v = find_view(T->tri_block0, T->nv, bb);
        const ViewDev &vd = T->v[v];
        const prg::Geom &g = vd.g;
        const int f0 = (bb - vd.tri_block0) * kBinTris;
        {
            // one lane per triangle: its tile rectangle and its test record
            // (FP64, once per triangle)
            const int f = f0 + j;
            int cnt = 0;
            if (j < kBinTris && f < vd.mesh.nt) {
                const TriBound b = tb[vd.tri_off + f];
                if (b.kind != prg::kCulled && b.rect[0] <= b.rect[2] && b.rect[1] <= b.rect[3]) {
                    cnt = (b.rect[2] - b.rect[0] + 1) * (b.rect[3] - b.rect[1] + 1);
                    double Ps[3][3], Pe[3][3];
                    int32_t idx[3];
                    prg::load_tri(vd.mesh.v0, vd.mesh.v1, vd.mesh.tri, vd.mesh.nv, f, g, Ps, Pe, idx);
                    prg::SatRec R;
                    if (FOV && (vd.fov_bound == prg::kFovSimple || vd.fov_bound == prg::kFovRecursive))
                        prg::sat_build_fov(g, Ps, Pe, b.kind, b.w, R, vd.fov_bound);
                    else
                        prg::sat_build(g, Ps, Pe, b.kind, b.w, R, vd.bound);
                    uint32_t rw[32];   // the record's words (memcpy: no type punning)
                    static_assert(sizeof(R) == sizeof(rw), "SatRec is 32 words");
                    __builtin_memcpy(rw, &R, sizeof(rw));
#pragma unroll
                    for (int i = 0; i < 32; ++i) s_sat[j][i] = rw[i];
                    for (int k = 0; k < 4; ++k) s_rect[j][k] = b.rect[k];
                }
            }
            int total;
            const int ex = block_excl_scan(cnt, s_tmp, total);
            if (j < kBinTris) s_pref[j] = ex;
            if (j == kBinTris - 1) s_pref[kBinTris] = total;
        }
        // the block's first candidate slot: its offset in its chunk of 256
        // blocks plus the totals of the chunks before
        long long cpre = 0;
        for (int i = j; i < (bb >> 8); i += kBinThreads) cpre += bpart[i];
        long long ctot;
        block_excl_scan64(cpre, s_tmp64, ctot);
        const int64_t s_off = boff[bb] + ctot;
        const int total = s_pref[kBinTris];
        const int per = min(kBinPer, max(1, (total + kBinThreads - 1) / kBinThreads));
        const bool split = prg::split_quads(vd.tile);
        for (int c0 = 0; c0 < total; c0 += kBinThreads * per) {
            const int my0 = c0 + j * per;
            const int myn = max(0, min(per, total - my0));
            int q0 = 0, l0 = 0;
            uint32_t masks = 0;
            if (myn > 0) {
                int lo = 0, hi = kBinTris - 1;   // last triangle whose candidates start at or before my0
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_pref[mid] <= my0) lo = mid; else hi = mid - 1;
                }
                q0 = lo;
                l0 = my0 - s_pref[q0];
                // the next candidate's tile info is loaded while the current
                // one is tested; the triangle's test record is read from LDS
                // when the triangle changes
                BinCursor cur = bin_start(vd, s_rect, s_pref, q0, l0);
                float4 nt[6];
#pragma unroll
                for (int i = 0; i < 6; ++i) nt[i] = reinterpret_cast<const float4 *>(&ti[cur.gt])[i];
                uint32_t rw[32];   // words of the current triangle's test record
                int rq = -1;
                for (int k = 0; k < myn; ++k) {
                    float4 tt[6];
#pragma unroll
                    for (int i = 0; i < 6; ++i) tt[i] = nt[i];
                    const int cq = cur.q, cgt = cur.gt;
                    if (k + 1 < myn) {
                        bin_step(cur, vd, s_rect, s_pref);
#pragma unroll
                        for (int i = 0; i < 6; ++i) nt[i] = reinterpret_cast<const float4 *>(&ti[cur.gt])[i];
                    }
                    if (cq != rq) {
#pragma unroll
                        for (int i = 0; i < 32; ++i) rw[i] = s_sat[cq][i];
                        rq = cq;
                    }
                    prg::SatRec R;
                    __builtin_memcpy(&R, rw, sizeof(R));
                    // TileInfo words: box 0..3, tw 4..5, qvalid 6, pad 7, qb 8..23
                    const float tbx[4] = {tt[0].x, tt[0].y, tt[0].z, tt[0].w}, tw[2] = {tt[1].x, tt[1].y};
                    int mask;
                    if (FOV && vd.fov_bound == prg::kFovQuad) {
                        // the time window alone
                        mask = (R.win[1] < tw[0] || R.win[0] > tw[1]) ? 0 : (split ? __float_as_int(tt[1].z) : 0xF);
                    } else if (FOV && vd.fov_bound != prg::kFovExact) {
                        // foveated space: the tile's own pixel-centre boxes
                        const int lt = cgt - vd.tile_base;
                        float fb[4], fqb[4][4];
                        int fq;
                        prg::tile_foveated(g, vd.tile, lt % vd.tiles_x, lt / vd.tiles_x, fb, fqb, fq);
                        mask = prg::sat_mask(R, fb, tw, split ? fqb : nullptr, fq);
                    } else if (split) {
                        const float qb[4][4] = {{tt[2].x, tt[2].y, tt[2].z, tt[2].w}, {tt[3].x, tt[3].y, tt[3].z, tt[3].w},
                                                {tt[4].x, tt[4].y, tt[4].z, tt[4].w}, {tt[5].x, tt[5].y, tt[5].z, tt[5].w}};
                        mask = prg::sat_mask(R, tbx, tw, qb, __float_as_int(tt[1].z));
                    } else {
                        mask = prg::sat_mask(R, tbx, tw, nullptr, 0);
                    }
                    masks |= (uint32_t)mask << (4 * k);
                }
            }
            // Every candidate owns a pair slot (boff: the block's first).  A
            // survivor's place in its tile's list: the round's survivors are
            // counted per tile in LDS (LDS atomics give each its rank), one
            // global atomic per tile and round reserves the tile's places
            // (a survivor that finds no table entry takes its place with its
            // own global atomic).
            int ptile[kBinPer], hslot[kBinPer];
            uint32_t pslot[kBinPer], pent[kBinPer];
            {
                BinCursor cur{0, 0, 0, 0};
                if (myn > 0) cur = bin_start(vd, s_rect, s_pref, q0, l0);
#pragma unroll
                for (int k = 0; k < kBinPer; ++k) {
                    ptile[k] = -1;
                    hslot[k] = -1;
                    pslot[k] = 0u;
                    pent[k] = 0u;
                    if (k < myn) {
                        if (k > 0) bin_step(cur, vd, s_rect, s_pref);
                        const uint32_t m = (masks >> (4 * k)) & 0xFu;
                        if (m) {
                            const int gt = cur.gt;
                            ptile[k] = gt;
                            int h = (int)(((uint32_t)gt * 2654435761u) >> (32 - kBinHashBits));
                            for (int probe = 0; probe < kBinProbe; ++probe) {
                                const int old = atomicCAS(&s_hkey[h], -1, gt);
                                if (old == -1 || old == gt) {
                                    hslot[k] = h;
                                    break;
                                }
                                h = (h + 1) & (kBinHash - 1);
                            }
                            pslot[k] = hslot[k] >= 0 ? atomicAdd(&s_hcnt[hslot[k]], 1u) : atomicAdd(&tcount[gt], 1u);
                        }
                        pent[k] = (uint32_t)(f0 + cur.q) | (m << kListTriBits);
                    }
                }
            }
            __syncthreads();
            {
                // one global atomic per used entry (issued together), then
                // the entry is cleared for the next round
                constexpr int kPerThread = kBinHash / kBinThreads;
                uint32_t eb[kPerThread];
#pragma unroll
                for (int i = 0; i < kPerThread; ++i) {
                    const int e = j + kBinThreads * i;
                    const int key = s_hkey[e];
                    eb[i] = 0u;
                    if (key >= 0) eb[i] = atomicAdd(&tcount[key], s_hcnt[e]);
                }
#pragma unroll
                for (int i = 0; i < kPerThread; ++i) {
                    const int e = j + kBinThreads * i;
                    if (s_hkey[e] >= 0) {
                        s_hbase[e] = eb[i];
                        s_hkey[e] = -1;
                        s_hcnt[e] = 0u;
                    }
                }
            }
            __syncthreads();
            if (myn > 0) {
#pragma unroll
                for (int k = 0; k < kBinPer; ++k)
                    if (hslot[k] >= 0) pslot[k] += s_hbase[hslot[k]];
                // slots past the capacity are dropped (the overflow is
                // reported); one set of addresses with immediate offsets
                const int64_t base = s_off + my0;
                const int nw = (int)min<int64_t>((int64_t)myn, cap - base);
                int32_t *pt = pairs.tile + base;
                uint32_t *ps = pairs.slot + base, *pe = pairs.entry + base;
#pragma unroll
                for (int k = 0; k < kBinPer; ++k)
                    if (k < nw) {
                        pt[k] = ptile[k];
                        ps[k] = pslot[k];
                        pe[k] = pent[k];
                    }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// exclusive scan of n uint32 counts (n < 2^31; totals fit in 32 bits)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 1;
constexpr int kScanBlock = 256 * kScanItems;


// Exclusive scan of the per-tile counts: the block's offset is the sum of
// the partial sums of the blocks before it (one per 256 tiles: many short
// blocks finish sooner than few long ones).  The block also adds its
// tiles' (XCD share, list-length bucket) pairs to the persistent ray
// cast's histogram (S->count, cleared by k_tiles).
__device__ __forceinline__ int len_bucket(uint32_t len) { return len == 0u ? 0 : 32 - __clz(len); }

// The XCD share of global tile gt: its view's 32 x 32-pixel super-tile
// (32 / tile is a power of two) on a diagonal pattern over the XCDs.
__device__ __forceinline__ int tile_xcd(const ViewTable *__restrict__ T, int gt) {
    const int v = find_view(T->tile_base, T->nv, gt);
    const ViewDev &vd = T->v[v];
    const int lt = gt - vd.tile_base, tx = lt % vd.tiles_x, ty = lt / vd.tiles_x;
    const int per = vd.tile >= 32 ? 1 : 32 / vd.tile;
    return (tx / per + 3 * (ty / per) + 5 * v) & (kXcds - 1);
}

// Single-pass exclusive scan of the tile counts (decoupled look-back):
// blocks take their place in the scan in the order they start (a ticket),
// publish their sum, and wave 0 finds the exclusive prefix from the flags
// of the blocks before: 64 at a time, each a 64-bit word (value << 32 |
// state), state 1 = the block's own sum, 2 = the inclusive prefix through
// it; the nearest inclusive flag ends the walk.  A block before has taken
// its ticket earlier and publishes its sum before it looks back itself, so
// every wait ends; a wait beyond kScanSpin polls (never expected) makes the
// block sum the counts before it directly instead.  The kernel also builds
// the tile-order histogram (XCD share x length bucket) of the ray cast.
constexpr int kScanSpin = 1 << 16;

__global__ __launch_bounds__(256) void k_scan(const ViewTable *__restrict__ T, const uint32_t *__restrict__ in,
                                              int n, int ntiles, unsigned long long *__restrict__ flags,
                                              uint32_t *__restrict__ out, Sched *__restrict__ S) {
    __shared__ int s_tmp[72];
    __shared__ uint32_t h[kXcds * kBuckets];
    __shared__ int s_bid, s_fallback;
    __shared__ uint32_t s_pre;
    if (threadIdx.x == 0) {
        s_bid = (int)atomicAdd(&S->ticket, 1u);
        s_fallback = 0;
    }
    for (int e = threadIdx.x; e < kXcds * kBuckets; e += 256) h[e] = 0u;
    __syncthreads();
    const int bid = s_bid;
    const int base = bid * kScanBlock + threadIdx.x * kScanItems;
    int v[kScanItems];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? (int)in[base + k] : 0;
        sum += v[k];
    }
    int total;
    int ex = block_excl_scan(sum, s_tmp, total);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        constexpr unsigned long long kAgg = 1ull, kIncl = 2ull;
        if (lane == 0 && bid > 0)
            __hip_atomic_store(&flags[bid], ((unsigned long long)(uint32_t)total << 32) | kAgg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        uint32_t pre = 0;
        bool late = false;
        for (int end = bid; end > 0 && !late;) {
            const int i = end - 1 - lane;
            unsigned long long w = 0ull;
            if (i >= 0) {
                int spin = 0;
                do {
                    w = __hip_atomic_load(&flags[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } while ((w & 3ull) == 0ull && ++spin < kScanSpin);
            }
            late = __ballot(i >= 0 && (w & 3ull) == 0ull) != 0ull;
            const unsigned long long incl = __ballot(i < 0 || (w & 3ull) == kIncl);
            const int first = incl ? __ffsll((long long)incl) - 1 : 64;
            uint32_t val = (lane <= first && i >= 0) ? (uint32_t)(w >> 32) : 0u;
            for (int o = 32; o > 0; o >>= 1) val += __shfl_xor(val, o, 64);
            pre += val;
            end = first < 64 ? 0 : end - 64;
        }
        if (lane == 0) {
            s_pre = pre;
            s_fallback = late ? 1 : 0;
            if (!late)
                __hip_atomic_store(&flags[bid], ((unsigned long long)(pre + (uint32_t)total) << 32) | kIncl,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    uint32_t pre = s_pre;
    if (s_fallback) {
        // the prefix from the counts themselves (correct whatever the flags)
        uint32_t acc = 0;
        for (int i = threadIdx.x; i < bid * kScanBlock && i < n; i += 256) acc += in[i];
        int tot2;
        block_excl_scan((int)acc, s_tmp, tot2);
        pre = (uint32_t)tot2;
        if (threadIdx.x == 0)
            __hip_atomic_store(&flags[bid], ((unsigned long long)(pre + (uint32_t)total) << 32) | 2ull,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    ex += (int)pre;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = (uint32_t)ex;
        if (base + k < ntiles) atomicAdd(&h[tile_xcd(T, base + k) * kBuckets + len_bucket((uint32_t)v[k])], 1u);
        ex += v[k];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kXcds * kBuckets; e += 256)
        if (h[e]) atomicAdd(&S->count[e / kBuckets][e % kBuckets], h[e]);
}

// ---------------------------------------------------------------------------
// scatter pairs into tile lists (slot order within a list is arbitrary)
// ---------------------------------------------------------------------------
// A tile as the ray cast takes it: tile coordinates in its view (tx | ty <<
// 16), view, list begin and end (x < 0: none).
__device__ __forceinline__ int4 tile_rec(const ViewTable *__restrict__ T, const uint32_t *__restrict__ toff,
                                         int gt, bool ovf) {
    const int v = find_view(T->tile_base, T->nv, gt);
    const int lt = gt - T->v[v].tile_base, tx = lt % T->v[v].tiles_x, ty = lt / T->v[v].tiles_x;
    const int xy = tx | (ty << 16);   // tile coordinates in the view (below 2^16)
    return ovf ? make_int4(xy, v, 0, 0) : make_int4(xy, v, (int)toff[gt], (int)toff[gt + 1]);
}

// Items of the persistent ray cast for n tiles of a share: 8x8 tiles run
// four per item, 16x16 one, 32x32 one quadrant per item.
__host__ __device__ __forceinline__ int share_items(int tile, int n) {
    return tile == 8 ? (n + 3) / 4 : (tile == 16 ? n : 4 * n);
}

// Pairs -> lists.  Blocks below ceil(ntiles / 256) also write the tile
// orders of the persistent ray cast: XCD share x's tiles at order[x ntiles
// ...], longest lists first by power-of-two length bucket (counting sort on
// the histogram k_scan built; S->cursor cleared by k_tiles).
__global__ __launch_bounds__(256) void k_scatter(const ViewTable *__restrict__ T, Pairs pairs,
                                                 const uint32_t *__restrict__ toff, int32_t *__restrict__ lists,
                                                 int64_t cap, int ntiles, DevStatus *__restrict__ st,
                                                 Sched *__restrict__ S, int4 *__restrict__ order) {
    const int64_t n = (int64_t)st->pairs_required;
    const bool ovf = n > cap;   // overflow: the ray cast writes misses
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pairs_total = toff[ntiles];
        if (ovf) st->overflow = 1;
        for (int x = 0; x < kXcds; ++x) {
            uint32_t nt = 0;
            for (int b = 0; b < kBuckets; ++b) nt += S->count[x][b];
            S->ntile[x] = nt;
        }
    }
    if (blockIdx.x < (ntiles + 255) / 256) {
        __shared__ uint32_t h[kXcds * kBuckets], base[kXcds * kBuckets], first[kXcds * kBuckets];
        if (threadIdx.x < kXcds) {
            uint32_t sum = 0;
            for (int b = kBuckets - 1; b >= 0; --b) {   // longest lists first
                first[threadIdx.x * kBuckets + b] = sum;
                sum += S->count[threadIdx.x][b];
            }
        }
        for (int e = threadIdx.x; e < kXcds * kBuckets; e += 256) h[e] = 0u;
        __syncthreads();
        const int i = blockIdx.x * 256 + threadIdx.x;
        int key = 0;
        uint32_t rank = 0;
        if (i < ntiles) {
            key = tile_xcd(T, i) * kBuckets + len_bucket(toff[i + 1] - toff[i]);
            rank = atomicAdd(&h[key], 1u);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kXcds * kBuckets; e += 256)
            if (h[e]) base[e] = first[e] + atomicAdd(&S->cursor[e / kBuckets][e % kBuckets], h[e]);
        __syncthreads();
        if (i < ntiles) order[(int64_t)(key / kBuckets) * ntiles + base[key] + rank] = tile_rec(T, toff, i, ovf);
    }
    if (ovf) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t tile = pairs.tile[i];
        if (tile >= 0) lists[toff[tile] + pairs.slot[i]] = (int32_t)pairs.entry[i];
    }
}

// ---------------------------------------------------------------------------
// ray cast
// ---------------------------------------------------------------------------
// Numeric inverse of a tabulated profile (samples tab[k] = G(k/(n-1)),
// increasing): binary search for the segment bracketing u, then linear.
__device__ __forceinline__ float prof_inv_f(const float *__restrict__ tab, int n, float u) {
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid] <= u) lo = mid; else hi = mid - 1;
    }
    const float a = tab[lo], b = tab[lo + 1];
    return ((float)lo + (u - a) / (b - a)) / (float)(n - 1);
}

// Per-pixel setup: foveated sample -> panel (display) point (unfoveate) ->
// time; panel point -> undistorted point (a lens) -> ray direction (rx, ry, 1).
__device__ __forceinline__ void pixel_setup(const PixelConst &pc, int px, int py, float &t, float &rx, float &ry) {
    float y0 = (float)(2 * px + 1) * (0.5f * pc.invW2) - 1.0f;
    float y1 = 1.0f - (float)(2 * py + 1) * (0.5f * pc.invH2);
    float d0 = y0 - pc.fov0, d1 = y1 - pc.fov1;
    float s = 1.0f, rho = 0.0f;
    if (pc.mode != 0 || pc.lens) rho = __builtin_amdgcn_sqrtf(d0 * d0 + d1 * d1);   // hardware square root (1 ulp)
    if (pc.mode == 1 || pc.mode == 2) {
        s = pc.mode == 1 ? rho * pc.invR : (rho > 0.0f ? powf(rho * pc.invR, pc.alpha - 1.0f) : 0.0f);
    } else if (pc.mode == 3) {
        const float sf = rho * pc.invR;
        s = rho > 0.0f ? prof_inv_f(pc.prof->c, pc.prof->nc, sf) / sf : 1.0f;
    }
    float x0 = pc.fov0 + d0 * s, x1 = pc.fov1 + d1 * s;
    float u = 0.5f * (pc.roll0 * (x0 + 1.0f) + pc.roll1 * (x1 + 1.0f));
    t = fminf(fmaxf(u, 0.0f), 1.0f);
    if (pc.lens) {
        // the undistorted point: the panel offset (d s) scaled by
        // p_l^{-1}(s_p) / s_p, s_p the panel point's normalised distance
        const float sp = rho * s * pc.invR;
        const float k = sp > 0.0f ? prof_inv_f(pc.prof->l, pc.prof->nl, sp) / sp : 1.0f;
        x0 = pc.fov0 + d0 * (s * k);
        x1 = pc.fov1 + d1 * (s * k);
    }
    rx = (x0 - pc.cx) * pc.invfx;
    ry = (x1 - pc.cy) * pc.invfy;
}

// Ray terms of one pixel: w = (rx, ry, t rx, t ry, t, t^2 rx, t^2 ry, t^2).
// Shading of one resolved pixel (k_shade, and the ray cast's fused form).
// Edge-plane normals c_k(t), face normal N(t) of triangle id at time t.
__device__ __forceinline__ void record_at(const ViewDev &vd, const float4 *__restrict__ rec, int id, float t,
                                          float ck[3][3], float N[3]) {
    // c_o(t) = (M0 + t M2 + t^2 M5, M1 + t M3 + t^2 M6, K + t M4 + t^2 M7)
    if (vd.rolling) {
        const float *R = reinterpret_cast<const float *>(rec + vd.rec_off + (int64_t)id * kRecRoll);
        for (int o = 0; o < 4; ++o) {
            float *dst = o < 3 ? ck[o] : N;
            dst[0] = fmaf(t, fmaf(t, R[20 + o], R[8 + o]), R[o]);
            dst[1] = fmaf(t, fmaf(t, R[24 + o], R[12 + o]), R[4 + o]);
            dst[2] = fmaf(t, fmaf(t, R[28 + o], R[16 + o]), R[32 + o]);
        }
    } else {
        const float *R = reinterpret_cast<const float *>(rec + vd.rec_off + (int64_t)id * kRecStatic);
        for (int o = 0; o < 4; ++o) {
            float *dst = o < 3 ? ck[o] : N;
            dst[0] = R[o];
            dst[1] = R[4 + o];
            dst[2] = R[16 + o];
        }
    }
}

// Rolling Blinn-Phong highlight k_s (n.h)^m (white) of a pixel with ray
// (rx, ry, 1): the eye is the camera's origin at the pixel's time, so the
// direction towards it is -r; h = normalize(l + v).  Zero where n.l <= 0,
// n.h <= 0 or l = -v.  n and l unit, ndl = n.l.
__device__ __forceinline__ float specular_at(const pr_light &light, const float n[3], const float l[3], float ndl,
                                             float rx, float ry) {
    if (!(light.specular > 0.0f) || !(ndl > 0.0f)) return 0.0f;
    const float ir = rsqrtf(fmaf(rx, rx, fmaf(ry, ry, 1.0f)));
    const float H[3] = {fmaf(-rx, ir, l[0]), fmaf(-ry, ir, l[1]), l[2] - ir};
    const float hh = H[0] * H[0] + H[1] * H[1] + H[2] * H[2];
    if (!(hh > 0.0f)) return 0.0f;
    const float ndh = (n[0] * H[0] + n[1] * H[1] + n[2] * H[2]) * rsqrtf(hh);
    if (!(ndh > 0.0f)) return 0.0f;
    // (n.h)^m = 2^(m log2(n.h)), n.h in (0, 1]
    return light.specular * __builtin_amdgcn_exp2f(light.shininess * __builtin_amdgcn_logf(ndh));
}

// Rolling colour of triangle id (0 <= id < nt) at a pixel whose time and
// ray pixel_setup gave as (t, rx, ry): Lambert plus the rolling highlight.
// The light direction in the camera frame at the view's start and end.
__device__ __forceinline__ void view_light(const ViewDev &vd, const pr_light &light, float l0[3], float l1[3]) {
    for (int r = 0; r < 3; ++r) {
        l0[r] = vd.R0f[3 * r] * light.dir_world[0] + vd.R0f[3 * r + 1] * light.dir_world[1] +
                vd.R0f[3 * r + 2] * light.dir_world[2];
        l1[r] = vd.R1f[3 * r] * light.dir_world[0] + vd.R1f[3 * r + 1] * light.dir_world[1] +
                vd.R1f[3 * r + 2] * light.dir_world[2];
    }
}

// l0, l1: view_light's directions (computed once per view by the caller).
__device__ __forceinline__ void shade_pixel_at(const ViewDev &vd, const float4 *__restrict__ rec,
                                               const float *__restrict__ alb, const pr_light &light,
                                               const float l0[3], const float l1[3], float t, float rx, float ry,
                                               int id, float c[3]) {
    const float ambient = light.ambient;
    // gathers first (vertex indices, then all nine albedo values), so their
    // latencies overlap each other and the arithmetic below
    int32_t vi[3];
    for (int k = 0; k < 3; ++k) vi[k] = vd.mesh.tri[3 * (int64_t)id + k];
    float a[3][3];
    for (int k = 0; k < 3; ++k)
        for (int ch = 0; ch < 3; ++ch) a[k][ch] = alb[3 * (int64_t)vi[k] + ch];
    float ck[3][3], N[3];
    record_at(vd, rec, id, t, ck, N);
    float e[3];
    for (int k = 0; k < 3; ++k) e[k] = fmaf(ry, ck[k][1], fmaf(rx, ck[k][0], ck[k][2]));
    float S = e[0] + e[1] + e[2];
    float inn = rsqrtf(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
    float sg = (N[0] * rx + N[1] * ry + N[2]) > 0.0f ? -inn : inn;
    // light direction in camera space at the pixel's time
    float L[3];
    for (int r = 0; r < 3; ++r) L[r] = fmaf(t, l1[r] - l0[r], l0[r]);
    float inl = rsqrtf(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    float ndl = sg * inl * (N[0] * L[0] + N[1] * L[1] + N[2] * L[2]);
    // (1 - ambient is uniform: kept in a scalar register, not a vector one)
    const float amb1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(1.0f - ambient)));
    float s = ambient + amb1 * fmaxf(ndl, 0.0f);
    const float nu[3] = {sg * N[0], sg * N[1], sg * N[2]}, lu[3] = {inl * L[0], inl * L[1], inl * L[2]};
    const float sp = specular_at(light, nu, lu, ndl, rx, ry);
    const float invS = __builtin_amdgcn_rcpf(S);   // (1 ulp)
    c[0] = c[1] = c[2] = 0.0f;
    for (int k = 0; k < 3; ++k) {
        float mu = e[k] * invS;
        for (int ch = 0; ch < 3; ++ch) c[ch] = fmaf(mu, a[k][ch], c[ch]);
    }
    for (int ch = 0; ch < 3; ++ch) c[ch] = fmaf(c[ch], s, sp);
}

// Rolling Lambert colour of triangle id (0 <= id < nt) at pixel (px, py).
__device__ __forceinline__ void shade_pixel(const ViewDev &vd, const float4 *__restrict__ rec,
                                            const float *__restrict__ alb, const pr_light &light, int px, int py,
                                            int id, float c[3]) {
    float t, rx, ry, l0[3], l1[3];
    pixel_setup(vd.pc, px, py, t, rx, ry);
    view_light(vd, light, l0, l1);
    shade_pixel_at(vd, rec, alb, light, l0, l1, t, rx, ry, id, c);
}

// The shaded outputs of pixel p of view v (id < 0: a miss, colour 0).
__device__ __forceinline__ void store_shade(const ShadeIO &io, int v, int64_t p, const float c[3], int id) {
    if (io.rgb32[v]) {
        float *o = io.rgb32[v];
        o[3 * p] = c[0];
        o[3 * p + 1] = c[1];
        o[3 * p + 2] = c[2];
    }
    if (io.rgba8[v]) {
        // one 32-bit store of the four bytes (R in the lowest address)
        uint32_t o = id >= 0 ? 0xFF000000u : 0u;
        for (int ch = 0; ch < 3; ++ch)
            o |= (uint32_t)floorf(fminf(fmaxf(c[ch], 0.0f), 1.0f) * 255.0f + 0.5f) << (8 * ch);
        reinterpret_cast<uint32_t *>(io.rgba8[v])[p] = o;
    }
}

__device__ __forceinline__ void ray_terms(const PixelConst &pc, int px, int py, float w[8]) {
    float t, rx, ry;
    pixel_setup(pc, px, py, t, rx, ry);
    const float t2 = t * t;
    w[0] = rx; w[1] = ry;
    w[2] = t * rx; w[3] = t * ry; w[4] = t;
    w[5] = t2 * rx; w[6] = t2 * ry; w[7] = t2;
}

// The ray cast works on 8x8 cells: one wave per cell, four waves (cells) per
// block.  8x8 tiles: a block takes four consecutive tiles; 16x16 tiles: a
// block takes one tile, wave w its quadrant w; 32x32 tiles: a block takes
// one quadrant of a tile, wave w one 8x8 cell of it.  A wave walks its
// tile's list, keeps the triangles whose quadrant mask covers its cell
// (ballot + mbcnt into a per-wave LDS buffer) and tests them four at a time
// against its 64 pixels with MFMA.
//
// The edge functions of a group of four triangles at 16 pixels are one
// v_mfma_f32_16x16x4f32 product per four ray terms: rows (A operand) are
// (triangle g, output o) with o = e_0, e_1, e_2 and the depth denominator
// S = r . N(t); columns (B operand) are pixels; K runs over the ray terms
// w = (rx, ry, t rx, t ry, t, t^2 rx, t^2 ry, t^2) (two products; one for
// non-rolling views, whose terms are (rx, ry, 0, 0)), and the accumulator
// starts at the constant terms.  Lane l then holds e_0, e_1, e_2, S of
// triangle l / 16 at pixel l % 16 of the 16-pixel block.  Every operation
// on a shared edge's coefficients is odd in them (products and sums of
// exactly negated values round to exactly negated results), so the two
// triangles of an edge evaluate exactly negated edge functions
// (watertight).
typedef float v4f __attribute__((ext_vector_type(4)));

template <int TILE>
struct RayCfg {
    static constexpr int NT = 256;                    // four cells per block
};

// Work items (blocks) of a frame for a tile size.
template <int TILE>
__host__ __device__ inline int ray_items(int ntiles) {
    return TILE == 8 ? (ntiles + 3) / 4 : (TILE == 16 ? ntiles : 4 * ntiles);
}

// Per-wave buffer of selected list entries: up to 3 carried + 64 new.
constexpr int kSelCap = 68;

// Record layout (floats).  Rolling: M[k][o] at 4k + o (k: the eight ray
// terms, o: e_0, e_1, e_2, S), constants at 32..35, d0..d3 at 36..39, id at
// 40.  Non-rolling: M[k][o] at 4k + o for k < 4 (terms rx, ry, 0, 0),
// constants at 16..19, d0 at 20, id at 21.
template <bool ROLL>
struct RecLayout {
    static constexpr int W = ROLL ? 4 * kRecRoll : 4 * kRecStatic;
    static constexpr int C = ROLL ? 32 : 16;
    static constexpr int D = ROLL ? 36 : 20;
    static constexpr int ID = ROLL ? 40 : 21;
};

// One 8x8 cell of one view.  (cx0, cy0): its first pixel; q: the quadrant
// bit its list entries must carry (-1: no filter).
// SHADE: the cell's pixels are shaded right after they are resolved
// (pixel colours as k_shade gives them for the same ids).
struct ShadeArgs {
    const ShadeIO *io;
    const pr_light *light;
    const float *l01;   // the view's light directions at its start (0..2) and end (3..5)
    const float4 *rec;
    int v;
};

// Cross-row register swaps of gfx950 (rows of 16 lanes): permlane32 swaps
// the upper half of a with the lower half of b, permlane16 the odd rows of
// a with the even rows of b.
__device__ __forceinline__ void swap_rows32(uint32_t &a, uint32_t &b) {
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void swap_rows16(uint32_t &a, uint32_t &b) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}
// Row broadcast: out[r] holds, in every row, row r of x.
__device__ __forceinline__ void rows_broadcast(float x, float out[4]) {
    uint32_t a = __float_as_uint(x), b = a;
    swap_rows32(a, b);            // a = rows (0, 1, 0, 1), b = rows (2, 3, 2, 3)
    uint32_t a2 = a, b2 = b;
    swap_rows16(a, a2);           // a = row 0 everywhere, a2 = row 1
    swap_rows16(b, b2);           // b = row 2, b2 = row 3
    out[0] = __uint_as_float(a);
    out[1] = __uint_as_float(a2);
    out[2] = __uint_as_float(b);
    out[3] = __uint_as_float(b2);
}

// The lane index, computed where it is used (an opaque mbcnt pair the
// compiler cannot move out of loops).
__device__ __forceinline__ int lane_fresh() {
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

template <bool ROLL, bool COUNT, bool SHADE>
__device__ __forceinline__ void raycast_cell(const ViewDev &vd, int cx0, int cy0, int q, const float *__restrict__ vrec,
                                             int beg, int end, const uint32_t *__restrict__ lists, uint32_t ent0,
                                             int32_t *__restrict__ out_id, float *__restrict__ out_depth,
                                             unsigned long long *__restrict__ cnt, int32_t *s_sel,
                                             const ShadeArgs &sa) {
    using RL = RecLayout<ROLL>;
    const PixelConst &pc = vd.pc;
    const int lane = __lane_id();
    const int kq = lane >> 4, jl = lane & 15;
    // the pixel's coordinates from a lane index read per cell: they are not
    // hoisted out of the caller's loop over items (where they would hold
    // registers through every cell, or be spilled)
    const int pl = lane_fresh();
    // B operands: ray terms kq and kq + 4 of pixel 16 b + jl of the cell.
    // Lane l sets up pixel l; the others fetch its (t, rx, ry).
    float bt0[4], bt1[4], tb[4];
    float t, rx, ry;   // lane l's own pixel l (shaded by lane l at the end)
    {
        pixel_setup(pc, cx0 + (pl & 7), cy0 + (pl >> 3), t, rx, ry);
        // pixel 16 b + jl's values are row b's: broadcast each row to all
        float tr[4], rxr[4], ryr[4];
        rows_broadcast(t, tr);
        rows_broadcast(rx, rxr);
        rows_broadcast(ry, ryr);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float tj = tr[b], rxj = rxr[b], ryj = ryr[b];
            if (ROLL) {
                // terms (rx, ry, t rx, t ry) and (t, t^2 rx, t^2 ry, t^2),
                // from the lane's selections of rx / ry (the same products)
                const float r0 = (kq & 1) ? ryj : rxj, r1 = kq == 1 ? rxj : ryj;
                const float t2 = tj * tj;
                bt0[b] = kq < 2 ? r0 : tj * r0;
                bt1[b] = kq == 0 ? tj : (kq == 3 ? t2 : t2 * r1);
            } else {
                bt0[b] = kq == 0 ? rxj : kq == 1 ? ryj : 0.0f;
                bt1[b] = 0.0f;
            }
            tb[b] = tj;
        }
    }
    // packed (depth bits, id) keys; kFar (depth +inf) is above every finite
    // positive depth's key, so a key below it is a finite hit
    constexpr unsigned long long kFar = 0x7f80000000000000ull;
    // (the initial keys from a scalar register written per cell: a constant
    // held in vector registers through the caller's item loop would be
    // spilled)
    uint32_t far_hi;
    asm volatile("s_mov_b32 %0, 0x7f800000" : "=s"(far_hi));
    const unsigned long long far_key = (unsigned long long)far_hi << 32;
    unsigned long long best[4] = {far_key, far_key, far_key, far_key};
    const float znear = pc.znear;
    unsigned hits = 0;
    unsigned long long tests = 0;
    int nvc = 0;   // valid pixels of the cell (PR_FLAG_COUNT)
    if (COUNT) {
        const int px = cx0 + (pl & 7), py = cy0 + (pl >> 3);
        nvc = __popcll(__ballot(px < pc.W && py < pc.H));
    }
    // A operand of lane l: triangle (l >> 2) & 3 of the group, output l & 3,
    // term kq (+ 4)
    // (aoff4: that term's byte offset in the record)
    const int ga = (lane >> 2) & 3;
    const uint32_t aoff4 = 4u * (uint32_t)(4 * kq + (lane & 3));
    int nbuf = 0;
    uint32_t ent_next = ent0;   // lists[beg + lane], loaded by the caller
    for (int c = beg; c < end; c += 64) {
        const uint32_t ent = ent_next;
        const bool inl = c + lane < end;
        if (c + 64 + lane < end) ent_next = lists[c + 64 + lane];
        const bool sel = inl && (q < 0 || ((ent >> (kListTriBits + q)) & 1u));
        const unsigned long long m = __ballot(sel);
        const int pos = nbuf + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        // the record's float4 offset (below 2^28: a view's records are
        // smaller than 4 GiB)
        if (sel) s_sel[pos] = (int32_t)((ent & kListTriMask) * (uint32_t)(RL::W / 4));
        nbuf += __popcll(m);
        const bool last = c + 64 >= end;
        const int ngr = last ? (nbuf + 3) >> 2 : nbuf >> 2;
        // Two register sets alternate (software pipeline without copies):
        // the next group's loads are issued before the current group's
        // products.  Lanes past the selection load the first selected
        // triangle's record (always in bounds).  Record offsets are 32-bit
        // byte offsets from the view's record base.
        struct Group {
            float a0, a1, d0, d1, d2, d3;
            v4f c;
            uint32_t id;
            bool valid;
        };
        const char *vbase = reinterpret_cast<const char *>(vrec);
        auto load_group = [&](Group &G, int g) {
            const int ia = 4 * g + ga, ic = 4 * g + kq;
            // (32-bit offsets from the uniform base: one VGPR per address)
            const uint32_t oa = ((uint32_t)s_sel[ia < nbuf ? ia : 0] << 4) + aoff4;
            const uint32_t oc = (uint32_t)s_sel[ic < nbuf ? ic : 0] << 4;
            G.a0 = *reinterpret_cast<const float *>(vbase + oa);
            G.a1 = ROLL ? *reinterpret_cast<const float *>(vbase + oa + 64) : 0.0f;
            G.valid = ic < nbuf;
            const float4 c4 = *reinterpret_cast<const float4 *>(vbase + oc + 4 * RL::C);
            G.c = v4f{c4.x, c4.y, c4.z, c4.w};
            if (ROLL) {
                const float4 d4 = *reinterpret_cast<const float4 *>(vbase + oc + 4 * RL::D);
                G.d0 = d4.x; G.d1 = d4.y; G.d2 = d4.z; G.d3 = d4.w;
            } else {
                G.d0 = *reinterpret_cast<const float *>(vbase + oc + 4 * RL::D);
                G.d1 = G.d2 = G.d3 = 0.0f;
            }
            G.id = *reinterpret_cast<const uint32_t *>(vbase + oc + 4 * RL::ID);
        };
        auto run_group = [&](const Group &G, int g) {
            if (COUNT) tests += (unsigned long long)min(4, nbuf - 4 * g) * (unsigned)nvc;
            // all products first, so the matrix pipe runs ahead of the tests
            v4f acc[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(G.a0, bt0[b], G.c, 0, 0, 0);
            if (ROLL) {
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(G.a1, bt1[b], acc[b], 0, 0, 0);
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float lo = fminf(fminf(acc[b][0], acc[b][1]), acc[b][2]);
                const float hi = fmaxf(fmaxf(acc[b][0], acc[b][1]), acc[b][2]);
                // rows past the selection repeat the first selected triangle
                // (same keys), so only the counts need `valid`
                if ((!COUNT | G.valid) & ((lo >= 0.0f) | (hi <= 0.0f))) {   // skipped when no lane passes
                    const float t = tb[b];
                    const float D = ROLL ? fmaf(t, fmaf(t, fmaf(t, G.d3, G.d2), G.d1), G.d0) : G.d0;
                    const float z = D * __builtin_amdgcn_rcpf(acc[b][3]);
                    const bool hit = z >= znear;   // (and key < kFar: finite)
                    const unsigned long long key = ((unsigned long long)__float_as_uint(z) << 32) | G.id;
                    best[b] = (hit & (key < best[b])) ? key : best[b];
                    if (COUNT) hits += hit & (key < kFar) & G.valid;
                }
            }
        };
        Group GA, GB;
        if (ngr > 0) load_group(GA, 0);
        int g = 0;
        for (; g + 1 < ngr; g += 2) {
            load_group(GB, g + 1);
            run_group(GA, g);
            load_group(GA, g + 2);   // unconditional: keeps the wait for GB partial
            run_group(GB, g + 1);
        }
        if (g < ngr) run_group(GA, g);
        // carry the entries of an incomplete group to the next chunk
        const int used = ngr << 2;
        if (!last) {
            const int left = nbuf - used;
            int32_t keep = 0;
            if (lane < left) keep = s_sel[used + lane];
            if (lane < left) s_sel[lane] = keep;
            nbuf = left;
        }
    }
    // Lanes l, l ^ 16, l ^ 32, l ^ 48 (the four rows) hold pixel 16 b + jl
    // for different triangles of each group: best[b] in row kq is entry
    // (b, kq) of a 4 x 4 table per jl.  Transposing it across the registers
    // and the rows (permlane32 swaps of blocks (0, 2) and (1, 3), then
    // permlane16 swaps of (0, 1) and (2, 3)) leaves in row r the four
    // candidates of block r, i.e. of the lane's own pixel 16 r + jl = l.
    uint32_t klo[4], khi[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        klo[b] = (uint32_t)best[b];
        khi[b] = (uint32_t)(best[b] >> 32);
    }
    swap_rows32(klo[0], klo[2]); swap_rows32(khi[0], khi[2]);
    swap_rows32(klo[1], klo[3]); swap_rows32(khi[1], khi[3]);
    swap_rows16(klo[0], klo[1]); swap_rows16(khi[0], khi[1]);
    swap_rows16(klo[2], klo[3]); swap_rows16(khi[2], khi[3]);
    unsigned long long mine = ((unsigned long long)khi[0] << 32) | klo[0];
#pragma unroll
    for (int b = 1; b < 4; ++b) {
        const unsigned long long o = ((unsigned long long)khi[b] << 32) | klo[b];
        mine = o < mine ? o : mine;
    }
    const int pl2 = lane_fresh();
    const int px = cx0 + (pl2 & 7), py = cy0 + (pl2 >> 3);
    if (px < pc.W && py < pc.H) {
        const int64_t p = (int64_t)py * pc.W + px;
        const bool miss = mine == kFar;
        const int32_t id = miss ? -1 : (int32_t)(uint32_t)(mine & 0xffffffffu);
        out_id[p] = id;
        out_depth[p] = miss ? __int_as_float(0x7f800000) : __uint_as_float((uint32_t)(mine >> 32));
        if (SHADE) {
            float c[3] = {0.0f, 0.0f, 0.0f};
            if (id >= 0)
                shade_pixel_at(vd, sa.rec, sa.io->albedo[sa.v], *sa.light, sa.l01, sa.l01 + 3, t, rx, ry, id, c);
            store_shade(*sa.io, sa.v, p, c, id);
        }
    }
    if (COUNT) {
        unsigned long long h = hits;
        for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o, 64);
        if (lane == 0) {
            atomicAdd(&cnt[0], tests);
            atomicAdd(&cnt[1], h);
        }
    }
}

// The wave's tile index of a block item: 8x8 tiles: four tiles per item;
// 16x16: one; 32x32: one quadrant of a tile per item.
template <int TILE>
__device__ __forceinline__ int item_tile(int item, int wv) {
    return TILE == 8 ? 4 * item + wv : (TILE == 16 ? item : item >> 2);
}

// The lane's entry of the first 64 of a tile record's list.
__device__ __forceinline__ uint32_t first_entries(const uint32_t *__restrict__ lists, int4 tr) {
    const int i = tr.z + (int)__lane_id();
    return tr.x >= 0 && i < tr.w ? lists[i] : 0u;
}

// Block item -> the wave's 8x8 cell of tile record tr (ent0: the lane's
// first list entry; quad: the item's quadrant of a 32x32 tile).
template <int TILE, bool COUNT, bool SHADE>
__device__ __forceinline__ void raycast_item(const ViewTable *__restrict__ T, const float4 *__restrict__ rec,
                                             const uint32_t *__restrict__ lists, const RayOut &out,
                                             DevStatus *__restrict__ st, int wv, int quad, int4 tr, uint32_t ent0,
                                             int32_t *s_sel_block, const ShadeIO *sio, const pr_light *light,
                                             const float *l01) {
    if (tr.x < 0) return;
    const int v = tr.y;
    const ViewDev &vd = T->v[v];
    const int tx = tr.x & 0xFFFF, ty = tr.x >> 16;
    int cx0 = tx * TILE, cy0 = ty * TILE, q = -1;
    if (TILE == 16) {
        q = wv;
        cx0 += (q & 1) * 8;
        cy0 += (q >> 1) * 8;
    } else if (TILE == 32) {
        q = quad;
        cx0 += (q & 1) * 16 + (wv & 1) * 8;
        cy0 += (q >> 1) * 16 + (wv >> 1) * 8;
    }
    if (cx0 >= vd.pc.W || cy0 >= vd.pc.H) return;   // cell outside the image
    const float *vrec = reinterpret_cast<const float *>(rec + vd.rec_off);
    unsigned long long *cnt = &st->cnt[blockIdx.x & (kCountSlots - 1)][0];
    int32_t *s_sel = s_sel_block + wv * kSelCap;
    const ShadeArgs sa{sio, light, l01 ? l01 + 6 * v : nullptr, rec, v};
    if (vd.rolling)
        raycast_cell<true, COUNT, SHADE>(vd, cx0, cy0, q, vrec, tr.z, tr.w, lists, ent0, out.id[v], out.depth[v], cnt,
                                         s_sel, sa);
    else
        raycast_cell<false, COUNT, SHADE>(vd, cx0, cy0, q, vrec, tr.z, tr.w, lists, ent0, out.id[v], out.depth[v], cnt,
                                          s_sel, sa);
}

// Block b -> item: consecutive blocks go to the eight XCDs in turn, so XCD
// x is given the x-th contiguous eighth of the items (neighbouring tiles
// share triangle records in that XCD's L2).
__device__ __forceinline__ int xcd_item(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <int TILE, bool COUNT>
__global__ __launch_bounds__((RayCfg<TILE>::NT)) void k_raycast(const ViewTable *__restrict__ T,
                                                               const float4 *__restrict__ rec,
                                                               const uint32_t *__restrict__ toff,
                                                               const uint32_t *__restrict__ lists, RayOut out,
                                                               DevStatus *__restrict__ st) {
    __shared__ int32_t s_sel[4 * kSelCap];
    const int item = xcd_item(blockIdx.x, gridDim.x);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k = item_tile<TILE>(item, wv);
    const int4 tr = k < T->total_tiles ? tile_rec(T, toff, k, st->overflow != 0) : make_int4(-1, 0, 0, 0);
    raycast_item<TILE, COUNT, false>(T, rec, lists, out, st, wv, item & 3, tr, first_entries(lists, tr), s_sel, nullptr,
                                     nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// persistent ray cast over a longest-list-first tile queue
// ---------------------------------------------------------------------------
// A grid sized to the device's resident blocks walks the longest-first tile
// order (written by k_scatter) in rounds, so the longest lists start first.
template <int TILE, bool COUNT, bool SHADE>
__global__ __launch_bounds__((RayCfg<TILE>::NT)) __attribute__((amdgpu_waves_per_eu(7))) void k_raycast_queue(
    const ViewTable *__restrict__ T, const float4 *__restrict__ rec, const uint32_t *__restrict__ lists, RayOut out,
    DevStatus *__restrict__ st, const int4 *__restrict__ order, const Sched *__restrict__ S, ShadeIO sio,
    pr_light light) {
    __shared__ int32_t s_sel[4 * kSelCap];
    // Blocks are dispatched to the XCDs in turn and the grid is a multiple
    // of their count, so block b runs on XCD x = b % 8 and walks that XCD's
    // share of the items, longest list first.  Its k = b / 8 of the K = grid
    // / 8 blocks of the share takes one item per round, in serpentine order
    // (round r: position r K + k for even r, r K + K - 1 - k for odd), which
    // evens out the blocks' summed list lengths.  (Shared queues drawing
    // each cell with a device-scope atomic ran several times slower.)
    // While an item is cast, the tile record two rounds ahead and the first
    // list entries of the next round are loaded.
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntiles = T->total_tiles;
    const int x = (int)blockIdx.x & (kXcds - 1), k = (int)blockIdx.x >> 3, K = (int)gridDim.x >> 3;
    const int share = (int)S->ntile[x];
    const int nitems = share_items(TILE, share);
    const int rounds = (nitems + K - 1) / K;
    const int4 *ord = order + (int64_t)x * ntiles;
    // the views' light directions (the fused shading's), once per block
    __shared__ float s_l01[PR_MAX_VIEWS][6];
    if (SHADE) {
        for (int v = threadIdx.x; v < T->nv; v += RayCfg<TILE>::NT)
            view_light(T->v[v], light, &s_l01[v][0], &s_l01[v][3]);
        __syncthreads();
    }
    auto fetch = [&](int r, int &quad) {
        const int j = r * K + ((r & 1) ? K - 1 - k : k);
        const int pos = TILE == 8 ? 4 * j + wv : (TILE == 16 ? j : j >> 2);
        quad = j & 3;
        return j < nitems && pos < share ? ord[pos] : make_int4(-1, 0, 0, 0);
    };
    int qcur, qn1, qn2;
    int4 cur = fetch(0, qcur), nx1 = fetch(1, qn1);
    uint32_t ecur = first_entries(lists, cur);
    for (int r = 0; r < rounds; ++r) {
        const int4 nx2 = fetch(r + 2, qn2);
        const uint32_t enx = first_entries(lists, nx1);
        // Waves of equal priority issue oldest first, so the blocks
        // dispatched last fall behind and end up running alone; a wave in
        // the first quarter of its rounds runs at priority 3, in the last at
        // 0, so lagging waves are issued first and the grid drains evenly.
        const int quarter = 4 * r / rounds;
        if (quarter == 0) __builtin_amdgcn_s_setprio(3);
        else if (quarter == 1) __builtin_amdgcn_s_setprio(2);
        else if (quarter == 2) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        raycast_item<TILE, COUNT, SHADE>(T, rec, lists, out, st, wv, qcur, cur, ecur, s_sel, &sio, &light, &s_l01[0][0]);
        cur = nx1;
        qcur = qn1;
        nx1 = nx2;
        qn1 = qn2;
        ecur = enx;
    }
}

// ---------------------------------------------------------------------------
// shade
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_shade(const ViewTable *__restrict__ T, const float4 *__restrict__ rec,
                                               ShadeIO io, pr_light light) {
    const int v = find_view(T->pix_block0, T->nv, blockIdx.x);
    const ViewDev &vd = T->v[v];
    const PixelConst &pc = vd.pc;
    int64_t p = (int64_t)(blockIdx.x - vd.pix_block0) * 256 + threadIdx.x;
    if (p >= (int64_t)pc.W * pc.H) return;
    int id = io.id[v][p];
    if (id >= vd.mesh.nt) id = -1;   // ids outside the mesh shade as misses
    float c[3] = {0.0f, 0.0f, 0.0f};
    if (id >= 0) shade_pixel(vd, rec, io.albedo[v], light, (int)(p % pc.W), (int)(p / pc.W), id, c);
    store_shade(io, v, p, c, id);
}

// ---------------------------------------------------------------------------
// G-buffer
// ---------------------------------------------------------------------------
// Pixel density of the foveation at pixel (px, py): the linear scale of the
// foveate map at the pixel's display point (square root of its Jacobian
// determinant; a lens is undone optically and does not enter).  With
// display distance d = R (rho/R)^alpha of foveated distance rho, the map's
// radial and tangential scales are (1/alpha)(rho/R)^(1-alpha) and
// (rho/R)^(1-alpha), so the density is alpha^(-1/2) (rho/R)^(1-alpha): 1
// without foveation, +inf at the fovea.  A tabulated p_c: the square root
// of p_c'(s_p) times p_c(s_p) / s_p (the first segment's slope at the
// fovea).
__device__ __forceinline__ float pixel_density(const PixelConst &pc, int px, int py) {
    if (pc.mode == 0) return 1.0f;
    const float y0 = (float)(2 * px + 1) * (0.5f * pc.invW2) - 1.0f;
    const float y1 = 1.0f - (float)(2 * py + 1) * (0.5f * pc.invH2);
    const float d0 = y0 - pc.fov0, d1 = y1 - pc.fov1;
    const float rho = sqrtf(d0 * d0 + d1 * d1);
    if (pc.mode == 3) {
        // tabulated p_c at the panel distance s_p = p_c^{-1}(s_f): radial
        // scale p_c'(s_p) (the slope of its segment), tangential s_f / s_p
        const float *c = pc.prof->c;
        const int n = pc.prof->nc;
        const float sf = rho * pc.invR;
        const float sp = sf > 0.0f ? prof_inv_f(c, n, sf) : 0.0f;
        const float q = sp * (float)(n - 1);
        const int k = q >= (float)(n - 2) ? n - 2 : (int)q;
        const float slope = (c[k + 1] - c[k]) * (float)(n - 1);
        return sf > 0.0f ? sqrtf(slope * (sf / sp)) : slope;
    }
    if (!(rho > 0.0f)) return INFINITY;
    return rsqrtf(pc.alpha) * powf(rho * pc.invR, 1.0f - pc.alpha);
}

// One thread per pixel: for a resolved id the camera-space unit face normal
// at the pixel's time turned towards the eye and the perspective-correct
// barycentrics (mu_1, mu_2) (zeros for misses); the density for every pixel.
__global__ __launch_bounds__(256) void k_gbuffer(const ViewTable *__restrict__ T, const float4 *__restrict__ rec,
                                                 GbufIO io) {
    const int v = find_view(T->pix_block0, T->nv, blockIdx.x);
    const ViewDev &vd = T->v[v];
    const PixelConst &pc = vd.pc;
    const int64_t p = (int64_t)(blockIdx.x - vd.pix_block0) * 256 + threadIdx.x;
    if (p >= (int64_t)pc.W * pc.H) return;
    const int px = (int)(p % pc.W), py = (int)(p / pc.W);
    int id = io.id[v][p];
    if (id >= vd.mesh.nt) id = -1;
    float n[3] = {0.0f, 0.0f, 0.0f}, mu1 = 0.0f, mu2 = 0.0f;
    if (id >= 0) {
        float t, rx, ry;
        pixel_setup(pc, px, py, t, rx, ry);
        float ck[3][3], N[3];
        record_at(vd, rec, id, t, ck, N);
        float e[3];
        for (int k = 0; k < 3; ++k) e[k] = fmaf(ry, ck[k][1], fmaf(rx, ck[k][0], ck[k][2]));
        const float invS = 1.0f / (e[0] + e[1] + e[2]);
        mu1 = e[1] * invS;
        mu2 = e[2] * invS;
        const float inn = rsqrtf(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        const float sg = (N[0] * rx + N[1] * ry + N[2]) > 0.0f ? -inn : inn;
        for (int q = 0; q < 3; ++q) n[q] = sg * N[q];
    }
    if (io.normal[v]) {
        float *o = io.normal[v] + 3 * p;
        o[0] = n[0]; o[1] = n[1]; o[2] = n[2];
    }
    if (io.bary[v]) {
        float *o = io.bary[v] + 2 * p;
        o[0] = mu1; o[1] = mu2;
    }
    if (io.density[v]) io.density[v][p] = pixel_density(pc, px, py);
}

// ---------------------------------------------------------------------------
// backward: gradient of a loss of the shaded image with visibility fixed
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cross3f(const float a[3], const float b[3], float o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ float dot3f(const float a[3], const float b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

__device__ __forceinline__ float wave_sum(float x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ void cross3d(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// FP64 pixel setup (the backward is per pixel, not per test, so it can
// afford it): foveated sample -> panel point -> time; panel point ->
// undistorted point -> ray.
__device__ __forceinline__ void pixel_setup_d(const prg::Geom &g, int px, int py, double &t, double r[3]) {
    double y0 = (2.0 * px + 1.0) / g.W - 1.0, y1 = 1.0 - (2.0 * py + 1.0) / g.H;
    double x0, x1, u0, u1;
    prg::unfoveate_pt(g, y0, y1, x0, x1);
    double u = 0.5 * (g.roll[0] * (x0 + 1.0) + g.roll[1] * (x1 + 1.0));
    t = prg::clamp01(u);
    prg::undistort_pt(g, x0, x1, u0, u1);
    r[0] = (u0 - g.cx) / g.fx;
    r[1] = (u1 - g.cy) / g.fy;
    r[2] = 1.0;
}

// Per pixel: the shading chain c = (sum_k mu_k a_k) (k_a + (1-k_a) max(0,
// n.l)) taken back through the barycentrics mu_k = e_k / S (e_1 = r.(P2 x
// P0), e_2 = r.(P0 x P1), mu_0 = 1 - mu_1 - mu_2), the face normal n, the
// rolling light l(t) and the camera-space interpolation P_k(t) =
// (1-t) Ps_k + t Pe_k.  Writes dL/dPs, dL/dPe per vertex (FP32 atomics) and
// the view's pose and light partial sums (FP64).  The geometry is FP64: near
// grazing incidence (ray almost in the triangle's plane) the barycentric
// terms scale like 1/S^2 and FP32 rounding of the ray alone would move
// them by 2^-24 / cos(incidence).
// Vertex gradients of a block's pixels are summed per vertex in an LDS
// table (open addressing on the vertex index, kBwdProbe probes) and added to
// the global accumulators once per vertex and block; a pixel whose vertex
// finds no entry adds directly.
constexpr int kBwdHashBits = 9;
constexpr int kBwdHash = 1 << kBwdHashBits;
constexpr int kBwdProbe = 8;

__global__ __launch_bounds__(256) void k_bwd_pixel(const ViewTable *__restrict__ T, BwdIO io, pr_light light,
                                                   float *__restrict__ gacc, double *__restrict__ pblk) {
    const double ka = light.ambient, ks = light.specular, shin = light.shininess;
    __shared__ int32_t s_vkey[kBwdHash];
    __shared__ float s_vg[kBwdHash][7];   // start xyz, end xyz (odd stride)
    __shared__ double s_pp[4][30];
    for (int e = threadIdx.x; e < kBwdHash; e += 256) {
        s_vkey[e] = -1;
        for (int c = 0; c < 6; ++c) s_vg[e][c] = 0.0f;
    }
    __syncthreads();
    const int v = find_view(T->pix_block0, T->nv, blockIdx.x);
    const ViewDev &vd = T->v[v];
    const prg::Geom &g = vd.g;
    const PixelConst &pc = vd.pc;
    int64_t p = (int64_t)(blockIdx.x - vd.pix_block0) * 256 + threadIdx.x;
    double part[30];
    for (int q = 0; q < 30; ++q) part[q] = 0.0;
    int id = p < (int64_t)pc.W * pc.H ? io.id[v][p] : -1;
    if (id >= vd.mesh.nt) id = -1;
    if (id >= 0) {
        int px = (int)(p % pc.W), py = (int)(p / pc.W);
        double t, r[3];
        pixel_setup_d(g, px, py, t, r);
        // base vertex P0 and edges E1 = P1 - P0, E2 = P2 - P0 at time t, the
        // edges from exact world-space differences
        int vi[3];
        for (int k = 0; k < 3; ++k) vi[k] = vd.mesh.tri[3 * (int64_t)id + k];
        double a0[3], b0[3], ds[2][3], de[2][3];
        for (int q = 0; q < 3; ++q) {
            a0[q] = vd.mesh.v0[3 * (int64_t)vi[0] + q];
            b0[q] = vd.mesh.v1[3 * (int64_t)vi[0] + q];
        }
        for (int k = 1; k < 3; ++k)
            for (int q = 0; q < 3; ++q) {
                ds[k - 1][q] = (double)vd.mesh.v0[3 * (int64_t)vi[k] + q] - a0[q];
                de[k - 1][q] = (double)vd.mesh.v1[3 * (int64_t)vi[k] + q] - b0[q];
            }
        double P0[3], E1[3], E2[3];
        for (int q = 0; q < 3; ++q) {
            const double *R0 = g.R0 + 3 * q, *R1 = g.R1 + 3 * q;
            double ps = R0[0] * a0[0] + R0[1] * a0[1] + R0[2] * a0[2] + g.T0[q];
            double pe = R1[0] * b0[0] + R1[1] * b0[1] + R1[2] * b0[2] + g.T1[q];
            P0[q] = (1.0 - t) * ps + t * pe;
            double s1 = R0[0] * ds[0][0] + R0[1] * ds[0][1] + R0[2] * ds[0][2];
            double e1 = R1[0] * de[0][0] + R1[1] * de[0][1] + R1[2] * de[0][2];
            double s2 = R0[0] * ds[1][0] + R0[1] * ds[1][1] + R0[2] * ds[1][2];
            double e2 = R1[0] * de[1][0] + R1[1] * de[1][1] + R1[2] * de[1][2];
            E1[q] = (1.0 - t) * s1 + t * e1;
            E2[q] = (1.0 - t) * s2 + t * e2;
        }
        // forward: N = E1 x E2, S = r.N, e1 = r.(E2 x P0), e2 = r.(P0 x E1)
        double N[3], x1[3], x2[3];
        cross3d(E1, E2, N);
        cross3d(E2, P0, x1);
        cross3d(P0, E1, x2);
        auto dot = [](const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
        const double S = dot(r, N);
        const double mu1 = dot(r, x1) / S, mu2 = dot(r, x2) / S;
        const double nn = sqrt(dot(N, N));
        double m[3] = {N[0] / nn, N[1] / nn, N[2] / nn};
        const double sg = dot(m, r) > 0.0 ? -1.0 : 1.0;
        double n[3] = {sg * m[0], sg * m[1], sg * m[2]};
        double Lw[3];
        for (int q = 0; q < 3; ++q) Lw[q] = (1.0 - t) * vd.light0[q] + t * vd.light1[q];
        const double ln = sqrt(dot(Lw, Lw));
        double l[3] = {Lw[0] / ln, Lw[1] / ln, Lw[2] / ln};
        const double ndl = dot(n, l);
        const double s = ka + (1.0 - ka) * (ndl > 0.0 ? ndl : 0.0);
        const float *alb = io.albedo[v];
        double al0[3], d1a[3], d2a[3], a[3];
        for (int ch = 0; ch < 3; ++ch) {
            al0[ch] = alb[3 * (int64_t)vi[0] + ch];
            d1a[ch] = alb[3 * (int64_t)vi[1] + ch] - al0[ch];
            d2a[ch] = alb[3 * (int64_t)vi[2] + ch] - al0[ch];
            a[ch] = al0[ch] + mu1 * d1a[ch] + mu2 * d2a[ch];   // a = sum_k mu_k a_k
        }
        // backward
        const float *gcp = io.dl[v] + 3 * p;
        double gc[3] = {gcp[0], gcp[1], gcp[2]};
        const double gs = dot(gc, a);
        double ga[3] = {gc[0] * s, gc[1] * s, gc[2] * s};
        const double gmu1 = dot(ga, d1a), gmu2 = dot(ga, d2a);
        const double gndl = ndl > 0.0 ? gs * (1.0 - ka) : 0.0;
        double gm[3], gl[3];
        for (int q = 0; q < 3; ++q) { gm[q] = sg * gndl * l[q]; gl[q] = gndl * n[q]; }
        // rolling highlight sigma = k_s (n.h)^m added to every channel:
        // h = H / |H|, H = l + v, v = -r / |r| (the eye at the pixel's time)
        if (ks > 0.0 && ndl > 0.0) {
            const double ir = 1.0 / sqrt(dot(r, r));
            double H[3] = {l[0] - r[0] * ir, l[1] - r[1] * ir, l[2] - r[2] * ir};
            const double hn = sqrt(dot(H, H));
            if (hn > 0.0) {
                double h[3] = {H[0] / hn, H[1] / hn, H[2] / hn};
                const double ndh = dot(n, h);
                if (ndh > 0.0) {
                    const double gsig = (gc[0] + gc[1] + gc[2]) * ks * shin * pow(ndh, shin - 1.0);
                    double gh[3];
                    for (int q = 0; q < 3; ++q) { gm[q] += sg * gsig * h[q]; gh[q] = gsig * n[q]; }
                    const double hg = dot(h, gh);
                    for (int q = 0; q < 3; ++q) gl[q] += (gh[q] - h[q] * hg) / hn;
                }
            }
        }
        const double mg = dot(m, gm), lg = dot(l, gl);
        const double ge1 = gmu1 / S, ge2 = gmu2 / S;
        const double gS = -(gmu1 * mu1 + gmu2 * mu2) / S;
        double gN[3];
        for (int q = 0; q < 3; ++q) {
            gN[q] = (gm[q] - m[q] * mg) / nn + gS * r[q];
            const double gLw = (gl[q] - l[q] * lg) / ln;
            part[q] = (1.0 - t) * gLw;
            part[3 + q] = t * gLw;
        }
        double P0xr[3], rxP0[3], rxE2[3], E1xr[3], E2xgN[3], gNxE1[3];
        cross3d(P0, r, P0xr);
        cross3d(r, P0, rxP0);
        cross3d(r, E2, rxE2);
        cross3d(E1, r, E1xr);
        cross3d(E2, gN, E2xgN);
        cross3d(gN, E1, gNxE1);
        double gP[3][3], gd[3];   // gd = sum_k gP_k (the translation part)
        for (int q = 0; q < 3; ++q) {
            const double gE1 = ge2 * rxP0[q] + E2xgN[q];
            const double gE2 = ge1 * P0xr[q] + gNxE1[q];
            gd[q] = ge1 * rxE2[q] + ge2 * E1xr[q];
            gP[1][q] = gE1;
            gP[2][q] = gE2;
            gP[0][q] = gd[q] - gE1 - gE2;
        }
        float *gs_ = gacc + vd.gacc_off;
        float *ge_ = gs_ + 3 * (int64_t)vd.mesh.nv;
        for (int k = 0; k < 3; ++k) {
            int h = (int)(((uint32_t)vi[k] * 2654435761u) >> (32 - kBwdHashBits)), slot = -1;
            for (int probe = 0; probe < kBwdProbe; ++probe) {
                const int old = atomicCAS(&s_vkey[h], -1, vi[k]);
                if (old == -1 || old == vi[k]) {
                    slot = h;
                    break;
                }
                h = (h + 1) & (kBwdHash - 1);
            }
            for (int q = 0; q < 3; ++q) {
                const float a = (float)((1.0 - t) * gP[k][q]), b = (float)(t * gP[k][q]);
                if (slot >= 0) {
                    atomicAdd(&s_vg[slot][q], a);
                    atomicAdd(&s_vg[slot][3 + q], b);
                } else {
                    atomicAdd(&gs_[3 * (int64_t)vi[k] + q], a);
                    atomicAdd(&ge_[3 * (int64_t)vi[k] + q], b);
                }
            }
        }
        // Pose partials of this pixel: dL/dT = sum_k w gP_k = w gd and
        // dL/dR = sum_k w gP_k v_k^T = w (gd v_0^T + gE1 (v_1 - v_0)^T +
        // gE2 (v_2 - v_0)^T), w = 1-t (start) or t (end).
        for (int e2 = 0; e2 < 2; ++e2) {
            const double w = e2 ? t : 1.0 - t;
            const double *v0p = e2 ? b0 : a0;
            const double(*dd)[3] = e2 ? de : ds;
            for (int rr = 0; rr < 3; ++rr) {
                part[6 + 12 * e2 + rr] = w * gd[rr];
                for (int c = 0; c < 3; ++c)
                    part[6 + 12 * e2 + 3 + 3 * rr + c] =
                        w * (gd[rr] * v0p[c] + gP[1][rr] * dd[0][c] + gP[2][rr] * dd[1][c]);
            }
        }
    }
    // pose and light partials: FP64 wave sums, then the block's sums stored
    // (k_bwd_pose adds the blocks of each view)
    for (int q = 0; q < 30; ++q) {
        double x = part[q];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if (__lane_id() == 0) s_pp[threadIdx.x >> 6][q] = x;
    }
    __syncthreads();
    if (threadIdx.x < kPoseAcc) {
        const int q = threadIdx.x;
        pblk[(int64_t)blockIdx.x * kPoseAcc + q] =
            q < 30 ? ((s_pp[0][q] + s_pp[1][q]) + s_pp[2][q]) + s_pp[3][q] : 0.0;
    }
    // the block's vertex sums
    float *gs_ = gacc + vd.gacc_off;
    float *ge_ = gs_ + 3 * (int64_t)vd.mesh.nv;
    for (int e = threadIdx.x; e < kBwdHash; e += 256) {
        const int key = s_vkey[e];
        if (key < 0) continue;
        for (int q = 0; q < 3; ++q) {
            atomicAdd(&gs_[3 * (int64_t)key + q], s_vg[e][q]);
            atomicAdd(&ge_[3 * (int64_t)key + q], s_vg[e][3 + q]);
        }
    }
}

// Per vertex of each view: world-space gradients dv = R^T dP (accumulated
// over the views sharing a mesh).
__global__ __launch_bounds__(256) void k_bwd_vertex(const ViewTable *__restrict__ T, const float *__restrict__ gacc,
                                                    BwdOut out) {
    const int v = find_view(T->vtx_block0, T->nv, blockIdx.x);
    const ViewDev &vd = T->v[v];
    const int i = (blockIdx.x - vd.vtx_block0) * 256 + threadIdx.x;
    if (i >= vd.mesh.nv) return;
    const float *gs = gacc + vd.gacc_off + 3 * (int64_t)i;
    const float *ge = gs + 3 * (int64_t)vd.mesh.nv;
    float *o0 = out.dv0[vd.view.mesh] + 3 * (int64_t)i;
    float *o1 = out.dv1[vd.view.mesh] + 3 * (int64_t)i;
    for (int c = 0; c < 3; ++c) {
        float d0 = vd.R0f[c] * gs[0] + vd.R0f[3 + c] * gs[1] + vd.R0f[6 + c] * gs[2];
        float d1 = vd.R1f[c] * ge[0] + vd.R1f[3 + c] * ge[1] + vd.R1f[6 + c] * ge[2];
        atomicAdd(&o0[c], d0);
        atomicAdd(&o1[c], d1);
    }
}

// Per view: dL/dR = vertex part + light part (sum (1-t) dL/dLw) l^T, then the
// rotation-vector gradient through Rodrigues' Jacobian.
// One block per view: the view's pixel blocks' partial sums are added (in a
// fixed order: deterministic), then turned into the pose gradients.
constexpr int kPoseThreads = 1024;

__global__ __launch_bounds__(kPoseThreads) void k_bwd_pose(const ViewTable *__restrict__ T,
                                                           const double *__restrict__ pblk, pr_light light,
                                                           float *__restrict__ dpose0, float *__restrict__ dpose1) {
    constexpr int kRows = kPoseThreads / kPoseAcc;   // blocks read at once
    __shared__ double s_w[kPoseThreads];
    __shared__ double a[kPoseAcc];
    const int v = blockIdx.x;
    if (v >= T->nv) return;
    const ViewDev &vd = T->v[v];
    const int b0 = T->pix_block0[v], b1 = T->pix_block0[v + 1];
    // thread t adds value t % 32 of blocks b0 + t / 32, + kRows, ... with
    // four independent partial sums (coalesced: the view's partials are read
    // as one array)
    const int q = threadIdx.x & (kPoseAcc - 1);
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    int b = b0 + (int)(threadIdx.x / kPoseAcc);
    for (; b + 3 * kRows < b1; b += 4 * kRows)
        for (int k = 0; k < 4; ++k) x[k] += pblk[(int64_t)(b + k * kRows) * kPoseAcc + q];
    for (; b < b1; b += kRows) x[0] += pblk[(int64_t)b * kPoseAcc + q];
    s_w[threadIdx.x] = (x[0] + x[1]) + (x[2] + x[3]);
    __syncthreads();
    if (threadIdx.x < kPoseAcc) {
        double y = 0.0;
        for (int k = 0; k < kRows; ++k) y += s_w[k * kPoseAcc + q];
        a[q] = y;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double lw[3] = {light.dir_world[0], light.dir_world[1], light.dir_world[2]};
    for (int e = 0; e < 2; ++e) {
        double gR[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) gR[3 * r + c] = a[6 + 12 * e + 3 + 3 * r + c] + a[3 * e + r] * lw[c];
        double J[27];
        prg::rodrigues_jac(e ? vd.view.pose1 : vd.view.pose0, J);
        float *o = (e ? dpose1 : dpose0) + 6 * v;
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
            for (int q = 0; q < 9; ++q) s += gR[q] * J[9 * i + q];
            o[i] = (float)s;
            o[3 + i] = (float)a[6 + 12 * e + i];
        }
    }
}

}  // namespace prk
