/*
 * pr.h -- C ABI of the perceptual rasterization library (libpr.so, gfx950).
 *
 * Perceptual rasterization (Friston, Ritschel & Steed, "Perceptual
 * Rasterization for Head-mounted Display Image Synthesis") renders, in one
 * pass, an image that is both foveated (its pixel grid is magnified about a
 * fovea point, Sec. 3.1.1) and rolling (each pixel is rendered at the time
 * its display column is lit, Sec. 3.1.2; jointly Sec. 3.1.3).  Every triangle
 * moves linearly in camera space between the frame's start and end
 * (Sec. 3.1.2, third display property).  A conservative per-triangle pixel
 * bound (Sec. 4) selects the pixels whose rays are intersected with the
 * triangle at the pixel's own time (Sec. 3.2, "Intersection"); the nearest
 * hit wins.  Shading interpolates the light to the pixel's time (Sec. 3.2,
 * "Shading").
 *
 * The calls of one frame are, in order:
 *   pr_bound    per-triangle camera-space transform, clipping/culling,
 *               rolling time interval and foveated screen bound (Sec. 3.2
 *               "Bounding", Sec. 4.1-4.3)
 *   pr_bin      per-(triangle, tile) conservative test and tile lists
 *               (replaces the fixed-function rasterisation of the bound)
 *   pr_raycast  per-pixel ray at the pixel's foveated position and time,
 *               ray-triangle test, nearest-depth resolve (Sec. 3.2)
 *   pr_shade    rolling shading of the resolved ids (Sec. 3.2)
 *   pr_gbuffer  normals, barycentrics and pixel density of the resolved ids
 * and, for differentiable rendering,
 *   pr_backward gradient of an image loss w.r.t. vertex positions and the
 *               start/end camera poses with visibility held fixed.
 *
 * CONVENTIONS
 *   World->view pose: rotation vector omega (3), translation T (3);
 *   P = R(omega) v + T (Rodrigues).  View space: x right, y up, +z forward.
 *   NDC of a view-space point: (fx X/Z + cx, fy Y/Z + cy).
 *   Pixel (i, j) (row 0 at the top) samples the foveated NDC point
 *   y = (2(i+1/2)/W - 1, 1 - 2(j+1/2)/H); its display point is
 *   x = f + (y - f) (|y - f|/R)^(alpha-1) with f the fovea and R the distance
 *   from f to the farthest image corner (power-law density, alpha = 1 is the
 *   identity); its time is t = clamp(d . (x+1)/2, 0, 1) with d = roll_dir
 *   ((0,0) = rolling off); its ray is ((x0-cx)/fx, (x1-cy)/fy, 1).
 *   The triangle at time t has camera-space vertices
 *   (1-t)(R0 v0 + T0) + t(R1 v1 + T1).  A pixel is covered when the ray
 *   meets the triangle (inclusive edges, both faces) at depth z >= znear;
 *   depth is camera-space z.  Among covered triangles the smallest
 *   (depth, triangle index) pair wins.
 *
 * MEMORY AND OWNERSHIP
 *   All array pointers inside pr_mesh and all output pointers are DEVICE
 *   pointers on the current HIP device; the pr_mesh / pr_view / pr_light /
 *   pr_tuning structs themselves live in host memory and are only read
 *   during the call.  The caller owns every buffer, including one workspace
 *   of pr_workspace_size() bytes (256-byte aligned) that carries state from
 *   pr_bound to the later calls of the same frame.  The library allocates no
 *   device memory in these calls.  Outputs are fully overwritten (misses:
 *   id -1, depth +inf, rgba 0); gradient outputs are overwritten, not
 *   accumulated.
 *
 * ORDERING
 *   Every call only enqueues work on `stream` (a hipStream_t; NULL = the
 *   default stream) and returns; nothing synchronises except
 *   pr_status_read.  Calls are thread-safe; concurrent frames need their
 *   own workspaces.
 *
 * ERRORS
 *   Every call returns PR_OK (0) or a negative code.  Arguments are checked
 *   before anything is enqueued; on an error nothing is launched.  Conditions
 *   found on the device (tile-list capacity overflow, non-finite vertices)
 *   are recorded in a status block inside the workspace and read with
 *   pr_status_read.  After an overflow, pr_raycast writes misses for every
 *   view; rerun with bin_capacity >= pr_status.pairs_required.
 *
 * All views of a call are processed together: each pass is one launch over
 * the views laid end to end.  pr_bound writes the workspace's view table;
 * the later calls of the frame must pass the same meshes, views and
 * tuning.
 */
#ifndef PR_H
#define PR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PR_OK 0
#define PR_ERR_INVALID (-1)     /* null pointer, bad size or parameter */
#define PR_ERR_UNSUPPORTED (-2) /* valid but not implemented (e.g. tile size) */
#define PR_ERR_WORKSPACE (-3)   /* workspace too small or misaligned */
#define PR_ERR_HIP (-4)         /* a HIP runtime call failed */

#define PR_MAX_VIEWS 64         /* views per call */

/* A triangle mesh.  v0 / v1: float32 [nv][3] world positions at the frame's
 * start / end (v1 may equal v0); tri: int32 [nt][3] vertex indices in
 * [0, nv).  0 <= nt <= 24,403,223 (records of a view stay under 4 GiB). */
typedef struct pr_mesh {
    const float *v0;
    const float *v1;
    const int32_t *tri;
    int32_t nv;
    int32_t nt;
} pr_mesh;

/* Tabulated foveation and lens distortion (Sec. 3.1.1 "Domain": the
 * density function p may be any monotone function and change every frame;
 * Sec. 5.1 "Lens Distortion": p = p_c o p_l, with only p_c undone when the
 * image is displayed).  Each profile is a radial function of normalised
 * distance s = d / R about the view's fovea (R: distance from the fovea to
 * the farthest image corner) given by n samples G(k / (n-1)), linear between
 * samples and continued past the last one with the last segment's slope;
 * G(0) = 0 and the samples strictly increase (finite).
 *   p_c (n_c samples, 2..PR_PROFILE_MAX; 0 = the power law of alpha): the
 *     foveation, panel (display) distance -> foveated distance; a pixel at
 *     foveated distance rho has its panel point at distance R
 *     p_c^{-1}(rho / R) (the numeric inverse: the segment bracketing rho / R,
 *     then linear).  Requires p_c(s_k) >= s_k at every sample (the foveation
 *     never moves a pixel's panel point outwards, as the power law does
 *     not), else PR_ERR_INVALID.
 *   p_l (n_l samples, 2..PR_PROFILE_MAX; 0 = no lens): the lens
 *     pre-distortion, undistorted distance -> panel distance, about the same
 *     centre; the pixel's ray passes through the point at undistorted
 *     distance R p_l^{-1}(panel distance / R).
 * A pixel's time comes from its panel point (the panel scans), its ray from
 * the undistorted point.  With a lens the rolling bound's time window is
 * the scan-time range of the triangle's panel image over the frame (the
 * catch-up window assumes a straight scan in the projected image). */
#define PR_PROFILE_MAX 64
typedef struct pr_profile {
    int32_t n_c, n_l;
    float p_c[PR_PROFILE_MAX];
    float p_l[PR_PROFILE_MAX];
} pr_profile;

/* One view (eye, frame or batch entry).  width, height in pixels
 * (1..16384); mesh indexes the pr_mesh array; pose0 / pose1 world->view at
 * the frame's start / end; fx, fy non-zero; znear > 0; fovea in NDC;
 * alpha >= 1 (1 = no foveation); roll_dir = d ((0,0) = rolling off);
 * profile: NULL (the power law of alpha, no lens) or a host pointer to the
 * view's tabulated foveation / lens (read during the call only). */
typedef struct pr_view {
    int32_t width, height, mesh, reserved;
    float pose0[6];
    float pose1[6];
    float fx, fy, cx, cy, znear;
    float fovea[2];
    float alpha;
    float roll_dir[2];
    const pr_profile *profile;
} pr_view;

/* Directional light: dir_world points towards the light (need not be unit);
 * ambient = k_a in c = albedo (k_a + (1 - k_a) max(0, n.l)).
 * specular = k_s >= 0 and shininess = m >= 1 add a white Blinn-Phong
 * highlight k_s max(0, n.h)^m to every channel where n.l > 0, with the
 * half vector h = normalize(l + v) of the light and the direction v = -ray
 * towards the eye; k_s = 0 is pure Lambert.  Like the light, the eye rolls:
 * v is taken in the camera frame at the pixel's own time (Sec. 3.2
 * "Shading", Sec. 5.1 "Rolling Shading"). */
typedef struct pr_light {
    float dir_world[3];
    float ambient;
    float specular;
    float shininess;
} pr_light;

/* tile: square tile side in pixels, one of 8, 16, 32.
 * bound: the rolling bound (Sec. 4.2), PR_BOUND_ZENON (default, 0): the
 *   exact frame-time window in which the rolling scan catches up with the
 *   moving triangle, hull of the triangle at its ends; PR_BOUND_ADAPTIVE:
 *   the window spanned by the scan times of the six projected start / end
 *   vertices, hull at its ends; PR_BOUND_HULL: the whole frame, hull of the
 *   six projected vertices; PR_BOUND_QUAD: the whole frame, their bounding
 *   box.  All are conservative (no covered pixel is dropped) and give the
 *   same images; they differ in the pairs and tests a frame spends.  Views
 *   without rolling use one instant whatever the bound.
 * bin_capacity: (triangle, tile) candidate pairs a frame can hold (all
 *   views; each candidate of a triangle's tile rectangle takes one slot,
 *   and the tile lists hold the candidates that survive the tile test).
 * fov_bound: how the binning tests a triangle against a tile of a foveated
 *   view (an ablation of Sec. 4.1's foveated bounds; all conservative, same
 *   images): PR_FOV_EXACT (default, 0) in display space, the tile's pixel
 *   centres unfoveated to an exact box; PR_FOV_QUAD no spatial test, every
 *   tile of the triangle's foveated bounding box; PR_FOV_SIMPLE /
 *   PR_FOV_RECURSIVE in foveated space against lines supporting the
 *   foveated triangle, normal to its display-space edges (Simple) or to
 *   the chords between its edges' foveated end points (Recursive), their
 *   offsets bounded from exact image boxes of pieces of the edges.
 * flags: PR_FLAG_COUNT makes pr_raycast count ray-triangle tests and hits
 * (sample test efficiency) into the status block: a test is one triangle at
 * one pixel the ray cast evaluates; PR_FLAG_PERSISTENT makes it order the
 * tiles longest list first and run one resident grid that walks that order
 * in rounds, a fixed set of items per block. */
typedef struct pr_tuning {
    int32_t tile;
    int32_t bin_capacity;
    int32_t flags;
    int32_t bound;
    int32_t fov_bound;
} pr_tuning;

#define PR_FLAG_COUNT 1
#define PR_FLAG_PERSISTENT 2

#define PR_BOUND_ZENON 0
#define PR_BOUND_ADAPTIVE 1
#define PR_BOUND_HULL 2
#define PR_BOUND_QUAD 3

#define PR_FOV_EXACT 0
#define PR_FOV_QUAD 1
#define PR_FOV_SIMPLE 2
#define PR_FOV_RECURSIVE 3

/* Device-side conditions of the last frame (all views). */
typedef struct pr_status {
    int32_t overflow;          /* 1 if the frame's candidates exceeded bin_capacity */
    int32_t nonfinite;         /* triangles with a bad index or non-finite vertex (culled) */
    int64_t pairs_required;    /* candidate slots the frame needed (all views) */
    int64_t pairs_total;       /* (triangle, tile) pairs in the tile lists */
    int64_t tests;             /* ray-triangle tests (PR_FLAG_COUNT) */
    int64_t hits;              /* tests that passed (PR_FLAG_COUNT) */
} pr_status;

/* Bytes of workspace a frame with these meshes, views and tuning needs.
 * Writes *bytes; returns PR_OK or PR_ERR_INVALID. */
int pr_workspace_size(const pr_mesh *meshes, int nm, const pr_view *views, int nv,
                      const pr_tuning *tuning, size_t *bytes);

/* Per-triangle bound (Sec. 3.2 "Bounding", Sec. 4): camera-space vertices
 * at start and end, near-plane clipping of the space-time triangle
 * (Sec. 4.2.2), the interval of frame time in which the rolling scan can
 * meet the triangle (Sec. 4.2.3-4.2.4, the scan catching up with each moving
 * vertex solved exactly), the display-space box of the triangle over that
 * interval and its conservative foveated image (Sec. 4.1, 4.3) as a tile
 * rectangle.  Also writes each triangle's intersection record.  Resets the
 * status block.  Reads the meshes; writes only the workspace. */
int pr_bound(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
             void *ws, size_t ws_bytes, void *stream);

/* Tile binning: every (triangle, tile) pair of the triangle's rectangle is
 * tested conservatively against the tile's display region over the tile's
 * own time window, and for tiles of 16 and 32 pixels against each quadrant
 * of the tile; surviving pairs are compacted (wave ballot + prefix) and
 * gathered into per-tile triangle lists that carry the quadrant mask of
 * each triangle (the ray cast skips the quadrants a triangle cannot
 * cover).  Needs pr_bound first. */
int pr_bin(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
           void *ws, size_t ws_bytes, void *stream);

/* Ray cast (Sec. 3.2 "Intersection"): per pixel, the ray at the pixel's
 * foveated position and time against every triangle of its tile list;
 * nearest (depth, id) wins.  tri_id[v]: int32 [H][W], depth[v]: float32
 * [H][W] for view v (device).  Needs pr_bin first. */
int pr_raycast(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
               void *ws, size_t ws_bytes, int32_t *const *tri_id, float *const *depth, void *stream);

/* Rolling shading (Sec. 3.2 "Shading"): light direction
 * normalize((1-t) R0 l + t R1 l) at the pixel's time t, face normal turned
 * towards the eye, per-vertex albedo (float32 [nv][3] per mesh) blended with
 * the perspective-correct barycentrics of the hit, Lambert plus the rolling
 * Blinn-Phong highlight of pr_light (eye direction at the pixel's time).  rgba8[v] (uint8
 * [H][W][4]) and rgb32[v] (float32 [H][W][3]) may each be NULL (or hold NULL
 * entries).  Needs pr_bound of the same frame. */
int pr_shade(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
             void *ws, size_t ws_bytes, const int32_t *const *tri_id, const pr_light *light,
             const float *const *albedo, uint8_t *const *rgba8, float *const *rgb32, void *stream);

/* pr_raycast followed by pr_shade of the ids it resolves, in one pass: the
 * persistent ray cast (PR_FLAG_PERSISTENT) shades each 8x8 cell right after
 * resolving it, which overlaps the shading's gathers with the ray cast's
 * arithmetic; otherwise the two kernels run in turn.  Arguments and outputs
 * as for the two calls (tri_id and depth required; rgba8 / rgb32 may be
 * NULL or hold NULL entries, and with no shaded output this is pr_raycast).
 * The outputs are bitwise those of pr_raycast then pr_shade.  Needs pr_bin
 * first. */
int pr_raycast_shade(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                     void *ws, size_t ws_bytes, int32_t *const *tri_id, float *const *depth,
                     const pr_light *light, const float *const *albedo, uint8_t *const *rgba8,
                     float *const *rgb32, void *stream);

/* G-buffer of the resolved ids (the deferred-shading buffer of Sec. 3.2
 * "Pipeline", for screen-space effects, Sec. 7 "Screen-space effects").
 * Per pixel of view v:
 *   normal[v]  float32 [H][W][3]: the triangle's unit face normal in the
 *              camera frame at the pixel's time, turned towards the eye
 *              (0 for misses);
 *   bary[v]    float32 [H][W][2]: the perspective-correct barycentrics
 *              (mu_1, mu_2) of the hit (mu_0 = 1 - mu_1 - mu_2; 0 for
 *              misses), which interpolate any per-vertex attribute such as
 *              texture coordinates;
 *   density[v] float32 [H][W]: the foveation's pixel density at the pixel,
 *              the factor by which a short distance in the display grows in
 *              the foveated image: the square root of the Jacobian
 *              determinant of the foveate map at the pixel's display point,
 *              alpha^(-1/2) (rho/R)^(1-alpha) with rho the pixel's foveated
 *              distance to the fovea (1 for alpha = 1, +inf at the fovea
 *              itself); written for every pixel.
 * Screen-space effects that measure distances in display pixels (an SSAO
 * radius) multiply them by density.  tri_id as pr_raycast wrote it; any
 * output array may be NULL or hold NULL entries.  Needs pr_bound of the
 * same frame. */
int pr_gbuffer(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
               void *ws, size_t ws_bytes, const int32_t *const *tri_id, float *const *normal,
               float *const *bary, float *const *density, void *stream);

/* Gradient of a loss L(rgb32) with visibility fixed to tri_id: given
 * dL/drgb[v] (float32 [H][W][3]), writes dL/dv0 and dL/dv1 (float32 [nv][3]
 * per mesh, summed over the views that use the mesh) and dL/dpose0,
 * dL/dpose1 (float32 [nv_views][6]: rotation vector then translation).
 * The shading is differentiated at this call's own vertices and poses
 * (meshes, views): the call rewrites the workspace's view table from them
 * and needs no earlier pass, so a forward frame run after the one that
 * produced tri_id does not change the result.  The status block is left
 * as it is. */
int pr_backward(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                void *ws, size_t ws_bytes, const int32_t *const *tri_id, const pr_light *light,
                const float *const *albedo, const float *const *dl_drgb, float *const *dv0,
                float *const *dv1, float *dpose0, float *dpose1, void *stream);

/* DISPLAY UNFOVEATION (Sec. 3.1.1 "Display").  The foveated image of each
 * view (the ray cast's RGBA8 output: its pixel grid lives in the foveated
 * domain) is resampled to the display's regular pixel grid.  Display pixel
 * (a, b) of a width x height display has display NDC x = (2(a+1/2)/width -
 * 1, 1 - 2(b+1/2)/height); it samples the foveated image at the foveated
 * position of x (the inverse of the view's unfoveate map, same fovea,
 * alpha and normalising radius), in continuous foveated pixel coordinates
 * u = ((y0+1)/2 W - 1/2, (1-y1)/2 H - 1/2), edges clamped.
 *   PR_UNFOV_MIP: a MIP pyramid of the foveated image (2x2 box means,
 *     sizes halved rounding up, the last row / column repeated) sampled
 *     with level of detail log2 of the longer image of a display pixel step
 *     in foveated pixels: Catmull-Rom interpolation of the finest level
 *     where the display magnifies (lod <= 0), blended linearly into the
 *     bilinear sample of level 1 for 0 < lod < 1, trilinear above.
 *   PR_UNFOV_FILTER: the 5 x 5 foveated pixels around the nearest one, each
 *     weighted by exp(-d^2 / (2 sigma^2)), d its distance in display pixels
 *     from the display pixel after unfoveating its centre, normalised
 *     (the paper's reconstruction filter r, Gaussian).
 * Display pixels whose foveated position lies beyond the foveated image
 * (the power map leaves parts of the display uncovered when the fovea is
 * not at the centre) take the image's edge.  Arithmetic in FP32; output
 * RGBA8 = floor(clamp(c, 0, 1) 255 + 1/2) per channel (alpha filtered too).
 */
#define PR_UNFOV_MIP 0
#define PR_UNFOV_FILTER 1

/* The display of one view: its size (1..16384 pixels each way), the form,
 * and for PR_UNFOV_FILTER the Gaussian's sigma in display pixels (> 0). */
typedef struct pr_display {
    int32_t width, height;
    int32_t mode;
    float sigma;
} pr_display;

/* Bytes of workspace pr_unfoveate needs (the pyramids of the MIP views:
 * about 16/3 bytes per foveated pixel).  Returns PR_OK or PR_ERR_INVALID. */
int pr_unfoveate_workspace_size(const pr_view *views, int nv, const pr_display *disp, size_t *bytes);

/* Display unfoveation of nv views (one launch per pass over all views).
 * views: the views whose foveated images are given (width, height, fovea,
 * alpha are used); disp[v]: view v's display; fov_rgba8[v]: uint8
 * [H][W][4] device (read only); disp_rgba8[v]: uint8 [height][width][4]
 * device (fully overwritten); ws: device workspace of at least
 * pr_unfoveate_workspace_size bytes, 256-byte aligned (contents need no
 * initialisation).  Stream-ordered, allocates nothing.  Returns PR_OK,
 * PR_ERR_INVALID, PR_ERR_WORKSPACE or PR_ERR_HIP; arguments are checked
 * before anything is enqueued. */
int pr_unfoveate(const pr_view *views, int nv, const pr_display *disp, const uint8_t *const *fov_rgba8,
                 uint8_t *const *disp_rgba8, void *ws, size_t ws_bytes, void *stream);

/* BATCHED FORM.  A batch renders many views (eyes, frames, scenes) of
 * uneven size and triangle count as one frame: every pass is one launch over
 * all views, the ray cast (with the shading fused in) is one resident grid
 * walking the (view, tile) items longest list first, and the whole frame
 * (bound, bin, ray cast and shade) is captured once into a hipGraph that
 * pr_batch_launch replays.
 *
 * pr_batch_create: meshes / views / light / albedo / outputs as for the
 * per-call functions (device pointers; outputs tri_id and depth required,
 * rgba8 and rgb32 may be NULL or hold NULL entries); they are bound into the
 * graph, so their contents may change between launches but not their
 * addresses, sizes or the views' parameters.  tuning->tile = 0 picks the
 * tile size (8, 16, 32) by timed trial frames; tuning->bin_capacity = 0
 * sizes the tile lists from a counting frame.  If the environment variable
 * PR_TUNE_CACHE names a file, choices are read from and appended to it,
 * keyed by device, view count and size classes.  The batch owns its
 * workspace (allocated here), a private capture stream and the graph until
 * pr_batch_destroy.  Synchronises the device while tuning.  Returns PR_OK
 * and *out, or a negative code (nothing allocated). */
typedef struct pr_batch pr_batch;
int pr_batch_create(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                    const pr_light *light, const float *const *albedo, int32_t *const *tri_id, float *const *depth,
                    uint8_t *const *rgba8, float *const *rgb32, pr_batch **out);
/* Enqueues one frame of the batch on `stream`. */
int pr_batch_launch(pr_batch *batch, void *stream);
/* The tuning chosen, workspace bytes and the trial frame times (ms) for
 * tiles 8, 16, 32 (0 where not tried).  Any pointer may be NULL. */
int pr_batch_info(const pr_batch *batch, pr_tuning *chosen, size_t *ws_bytes, double *trial_ms);
/* pr_status_read on the batch's workspace (synchronises `stream`). */
int pr_batch_status(const pr_batch *batch, pr_status *out, void *stream);
/* Frees everything the batch owns.  NULL is allowed. */
int pr_batch_destroy(pr_batch *batch);

/* ALLOCATION-FREE FRAME, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  pr_frame_static runs pr_bound, pr_bin and pr_raycast_shade
 * with the same arguments (minus the workspace) and writes the same outputs
 * bitwise, using as workspace a static device array of
 * PR_STATIC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends; it calls no hipMalloc, hipFree or other
 * allocating routine.  A frame whose pr_workspace_size exceeds
 * PR_STATIC_SCRATCH_BYTES is rejected with PR_ERR_WORKSPACE before anything
 * is enqueued.  The array keeps the last call's contents (the frame's
 * passes clear what they need); every call on one device shares it, so
 * calls that overlap on one device (other streams, other threads) race and
 * must be serialised by the caller.  Device-side conditions (tile-list
 * overflow: misses written) stay in the array and are not returned; size
 * bin_capacity with the allocating path first. */
#define PR_STATIC_SCRATCH_BYTES (256u << 20)
int pr_frame_static(const pr_mesh *meshes, int nm, const pr_view *views, int nv, const pr_tuning *tuning,
                    int32_t *const *tri_id, float *const *depth, const pr_light *light, const float *const *albedo,
                    uint8_t *const *rgba8, float *const *rgb32, void *stream);

/* Waits for `stream`, copies the workspace's status block into *out.
 * Returns PR_OK, PR_ERR_INVALID or PR_ERR_HIP. */
int pr_status_read(const void *ws, size_t ws_bytes, pr_status *out, void *stream);

/* Static text for a return code. */
const char *pr_status_string(int code);

/* Copies one view's tile lists to host memory for inspection:
 * offsets: int32 [tiles+1] (host), lists: int32 [cap] (host; may be NULL to
 * query).  Each list entry holds the triangle index in bits 0..27 and, in
 * bits 28..31, the mask of the tile's quadrants (bit qx + 2 qy: the
 * tile/2 x tile/2 pixels at column offset qx tile/2, row offset qy tile/2)
 * the triangle may cover; 8x8 tiles are not split (mask 0xF).
 * *ntiles receives the tile count, *npairs the list length.
 * Synchronises `stream`.  Used by tests of the bound's conservativeness. */
int pr_debug_tile_lists(const pr_mesh *meshes, int nm, const pr_view *views, int nv,
                        const pr_tuning *tuning, const void *ws, size_t ws_bytes, int view,
                        int32_t *offsets, int32_t *lists, int64_t cap, int32_t *ntiles,
                        int64_t *npairs, void *stream);

/* Host evaluation of the bound pieces, for CPU tests of their
 * conservativeness without a GPU (the same code the kernels run).  `mesh`
 * holds HOST pointers here; bound is a PR_BOUND_* mode (-1 for another
 * value).
 * pr_host_time_interval: the frame-time window of triangle f in `view`;
 *   returns 0 (culled: never visible), 1 (window t[0..1]) or 2 (the near
 *   plane cuts the triangle; the window is the whole frame).
 * pr_host_tile_rect: the triangle's inclusive tile rectangle
 *   rect = {x0, y0, x1, y1}; returns 0 if culled, 1 otherwise.
 * pr_host_tile_test: the quadrant mask binning gives the pair (triangle f,
 *   tile (tx, ty)) (as in pr_debug_tile_lists); 0 if the pair is rejected
 *   (or the triangle is culled).
 * pr_host_tile_test_fov: the same under foveated bound fov (a PR_FOV_*
 *   mode; -1 for another value). */
int pr_host_time_interval(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t bound, double *t);
int pr_host_tile_rect(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t bound, int32_t tile,
                      int32_t *rect);
int pr_host_tile_test(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t bound, int32_t tile,
                      int32_t tx, int32_t ty);
int pr_host_tile_test_fov(const pr_mesh *mesh, int32_t f, const pr_view *view, int32_t bound, int32_t fov,
                          int32_t tile, int32_t tx, int32_t ty);

#ifdef __cplusplus
}
#endif

#endif /* PR_H */
