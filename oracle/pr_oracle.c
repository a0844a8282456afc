/*
 * FP64 CPU oracle for perceptual rasterization (Friston, Ritschel & Steed,
 * "Perceptual Rasterization for Head-mounted Display Image Synthesis").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition that
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product path never
 * does, and it shares no code with the GPU library.
 *
 * What it computes is the "correct, but slow" solution the paper names in
 * Sec. 3 (every primitive tested against every pixel, then a z-test), with
 * the ray-primitive models of Sec. 3.1:
 *   - foveation (Sec. 3.1.1): the pixel grid lives in the foveated domain; a
 *     pixel's display position is the unfoveated point of its centre;
 *   - rolling (Sec. 3.1.2): the pixel's time is r(x) = x . d of its unit
 *     display position;
 *   - joint (Sec. 3.1.3): time taken from the unfoveated display position;
 *   - intersection (Sec. 3.2, "Intersection"): the triangle is linearly
 *     interpolated to the pixel's time in camera space and intersected with
 *     the pixel's ray; the nearest hit wins;
 *   - shading (Sec. 3.2, "Shading"): light direction and eye interpolated
 *     to the pixel's time, Lambert with one directional light plus a
 *     Blinn-Phong highlight (Sec. 5.1 "Rolling Shading");
 *   - the G-buffer of the resolved pixels (normals, barycentrics) and the
 *     foveation's pixel density (Sec. 7 "Screen-space effects").
 * Plus the analytic gradient of an L2 image loss with visibility held fixed
 * (an AI-systems form of the method; pinned by central differences).
 *
 * Everything is double precision; float32 inputs convert exactly.
 *
 * View parameter block (ORC_NPARAM doubles), see ORC_* indices below:
 *   width, height, pose0[6], pose1[6], fx, fy, cx, cy, znear,
 *   fovea[2], alpha, roll_dir[2], n_c, n_l, p_c samples [64], p_l samples [64]
 * n_c = 0: the power-law foveation of alpha; n_c >= 2: the tabulated
 * foveation p_c (alpha unused); n_l >= 2: a tabulated lens distortion p_l
 * composed before it (Sec. 5.1 "Lens Distortion"), 0: none.
 * A pose is a world->view rotation vector omega (3) then translation T (3):
 *   P = R(omega) v + T.
 * View space: x right, y up, +z forward.  NDC: x = fx X/Z + cx,
 * y = fy Y/Z + cy.  Pixel (i, j), row 0 at the top, samples the foveated NDC
 * point y = (2(i+1/2)/W - 1, 1 - 2(j+1/2)/H).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PMAX 64   /* samples of a tabulated profile */
enum {
    ORC_W = 0, ORC_H = 1, ORC_POSE0 = 2, ORC_POSE1 = 8, ORC_FX = 14, ORC_FY = 15,
    ORC_CX = 16, ORC_CY = 17, ORC_ZNEAR = 18, ORC_FOV = 19, ORC_ALPHA = 21,
    ORC_ROLL = 22, ORC_NC = 24, ORC_NL = 25, ORC_PC = 26, ORC_PL = 26 + ORC_PMAX,
    ORC_NPARAM = 26 + 2 * ORC_PMAX
};

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                       */
/* ------------------------------------------------------------------------- */
static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static void matvec(const double R[9], const double v[3], double o[3]) {
    for (int r = 0; r < 3; ++r) o[r] = R[3 * r] * v[0] + R[3 * r + 1] * v[1] + R[3 * r + 2] * v[2];
}
static void matTvec(const double R[9], const double v[3], double o[3]) {
    for (int c = 0; c < 3; ++c) o[c] = R[c] * v[0] + R[3 + c] * v[1] + R[6 + c] * v[2];
}

/* Rotation matrix of a rotation vector (Rodrigues' formula):
 * R = I + sin(th)/th [w]x + (1 - cos(th))/th^2 [w]x^2, th = |w|. */
void orc_rodrigues(const double w[3], double R[9]) {
    double th = norm3(w);
    double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += K[3 * r + k] * K[3 * k + c];
            K2[3 * r + c] = s;
        }
    double a, b;
    if (th < 1e-8) {            /* series: sin(th)/th ~ 1 - th^2/6, (1-cos)/th^2 ~ 1/2 - th^2/24 */
        a = 1.0 - th * th / 6.0;
        b = 0.5 - th * th / 24.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / (th * th);
    }
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + a * K[i] + b * K2[i];
}

/* dR/dw_i for the rotation vector w (Gallego & Yezzi 2015, "A compact
 * formula for the derivative of a 3-D rotation in exponential coordinates"):
 *   dR/dw_i = ( w_i [w]x + [ w x ((I - R) e_i) ]x ) R / |w|^2,
 * with the first-order expansion [e_i]x + ([e_i]x[w]x + [w]x[e_i]x)/2 near 0. */
static void skew(const double v[3], double S[9]) {
    S[0] = 0; S[1] = -v[2]; S[2] = v[1];
    S[3] = v[2]; S[4] = 0; S[5] = -v[0];
    S[6] = -v[1]; S[7] = v[0]; S[8] = 0;
}
static void matmul3(const double A[9], const double B[9], double C[9]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[3 * r + k] * B[3 * k + c];
            C[3 * r + c] = s;
        }
}
void orc_rodrigues_jac(const double w[3], double dR[27]) {
    double th = norm3(w);
    double R[9];
    orc_rodrigues(w, R);
    for (int i = 0; i < 3; ++i) {
        double e[3] = {0, 0, 0};
        e[i] = 1.0;
        double Ei[9];
        skew(e, Ei);
        double *out = dR + 9 * i;
        if (th < 1e-6) {
            double W[9], A[9], B[9];
            skew(w, W);
            matmul3(Ei, W, A);
            matmul3(W, Ei, B);
            for (int k = 0; k < 9; ++k) out[k] = Ei[k] + 0.5 * (A[k] + B[k]);
        } else {
            double ImR_e[3], u[3], W[9], U[9], M[9];
            for (int r = 0; r < 3; ++r) ImR_e[r] = e[r] - R[3 * r + i];
            cross3(w, ImR_e, u);
            skew(w, W);
            skew(u, U);
            for (int k = 0; k < 9; ++k) M[k] = (w[i] * W[k] + U[k]) / (th * th);
            matmul3(M, R, out);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* ray-primitive models (Sec. 3.1)                                             */
/* ------------------------------------------------------------------------- */

/* Normalising radius of the foveation domain: distance from the fovea to the
 * farthest corner of [-1,1]^2 (sqrt 2 for a central fovea). */
double orc_fovea_radius(const double *vp) {
    double best = 0;
    for (int c = 0; c < 4; ++c) {
        double dx = (c & 1 ? 1.0 : -1.0) - vp[ORC_FOV];
        double dy = (c & 2 ? 1.0 : -1.0) - vp[ORC_FOV + 1];
        double d = sqrt(dx * dx + dy * dy);
        if (d > best) best = d;
    }
    return best;
}

/* Tabulated radial profile (Sec. 3.1.1 "Domain": p is arbitrary, only
 * monotone, and may change every frame): a function g of normalised distance
 * given by its samples tab[k] = g(k / (n-1)), tab[0] = 0, strictly
 * increasing; linear between samples and continued past the last sample
 * with the last segment's slope. */
static double tab_eval(const double *tab, int n, double s) {
    double h = 1.0 / (n - 1);
    int k = (int)floor(s / h);
    if (k < 0) k = 0;
    if (k > n - 2) k = n - 2;
    return tab[k] + (s - k * h) / h * (tab[k + 1] - tab[k]);
}

/* Slope of the segment that tab_eval uses at s. */
static double tab_slope(const double *tab, int n, double s) {
    double h = 1.0 / (n - 1);
    int k = (int)floor(s / h);
    if (k < 0) k = 0;
    if (k > n - 2) k = n - 2;
    return (tab[k + 1] - tab[k]) / h;
}

/* The numeric inverse of a tabulated profile: the segment whose end values
 * bracket u (a scan from the fovea outwards), then the linear inverse on it
 * (the inverse of a piecewise-linear increasing function is the
 * piecewise-linear function through the swapped samples). */
static double tab_inv(const double *tab, int n, double u) {
    int k = 0;
    while (k < n - 2 && tab[k + 1] <= u) ++k;
    double h = 1.0 / (n - 1);
    return (k + (u - tab[k]) / (tab[k + 1] - tab[k])) * h;
}

/* Scale of a radial map about the fovea taking distance rho to g(rho / R) R
 * (g = the profile, inverted when inv), as the factor on (point - fovea). */
static double tab_scale(const double *vp, int which, int inv, double rho) {
    const double *tab = vp + (which ? ORC_PL : ORC_PC);
    int n = (int)vp[which ? ORC_NL : ORC_NC];
    double s = rho / orc_fovea_radius(vp);
    return (inv ? tab_inv(tab, n, s) : tab_eval(tab, n, s)) / s;
}

/* Unfoveate (foveated NDC y -> display NDC x): radial about the fovea; with
 * the power law display distance = R (rho/R)^alpha (alpha = 1 is the
 * identity: constant density, common rasterization); with a tabulated p_c
 * display distance = R p_c^{-1}(rho/R).  The display point is the panel's:
 * a lens distortion (orc_undistort) applies after it. */
void orc_unfoveate(const double *vp, const double y[2], double x[2]) {
    double fx = vp[ORC_FOV], fy = vp[ORC_FOV + 1];
    double dx = y[0] - fx, dy = y[1] - fy;
    double rho = sqrt(dx * dx + dy * dy);
    if (rho == 0.0) { x[0] = fx; x[1] = fy; return; }
    double s = vp[ORC_NC] > 0 ? tab_scale(vp, 0, 1, rho) : pow(rho / orc_fovea_radius(vp), vp[ORC_ALPHA] - 1.0);
    x[0] = fx + dx * s;
    x[1] = fy + dy * s;
}

/* Foveate (display NDC x -> foveated NDC y), the inverse of orc_unfoveate:
 * foveated distance = R (d/R)^(1/alpha), or R p_c(d/R). */
void orc_foveate(const double *vp, const double x[2], double y[2]) {
    double fx = vp[ORC_FOV], fy = vp[ORC_FOV + 1];
    double dx = x[0] - fx, dy = x[1] - fy;
    double rho = sqrt(dx * dx + dy * dy);
    if (rho == 0.0) { y[0] = fx; y[1] = fy; return; }
    double s = vp[ORC_NC] > 0 ? tab_scale(vp, 0, 0, rho) : pow(rho / orc_fovea_radius(vp), 1.0 / vp[ORC_ALPHA] - 1.0);
    y[0] = fx + dx * s;
    y[1] = fy + dy * s;
}

/* Lens distortion (Sec. 5.1 "Lens Distortion": p = p_c o p_l, p_l undone by
 * the optics): p_l takes the undistorted distance of a view direction to
 * its panel distance, about the same centre as p_c (the paper composes the
 * two distance functions).  Panel point x -> undistorted point u, whose
 * pinhole ray the pixel casts; the identity without a lens. */
void orc_undistort(const double *vp, const double x[2], double u[2]) {
    double fx = vp[ORC_FOV], fy = vp[ORC_FOV + 1];
    double dx = x[0] - fx, dy = x[1] - fy;
    double rho = sqrt(dx * dx + dy * dy);
    if (vp[ORC_NL] <= 0 || rho == 0.0) { u[0] = x[0]; u[1] = x[1]; return; }
    double s = tab_scale(vp, 1, 1, rho);
    u[0] = fx + dx * s;
    u[1] = fy + dy * s;
}

/* Rolling function: unit display position (x+1)/2 dotted with the skew
 * direction d, clamped to the frame [0, 1].  d = (0,0) gives t = 0. */
double orc_pixel_time(const double *vp, const double x[2]) {
    double t = vp[ORC_ROLL] * (x[0] + 1.0) * 0.5 + vp[ORC_ROLL + 1] * (x[1] + 1.0) * 0.5;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    return t;
}

/* Per-pixel setup: foveated sample y, its panel point (unfoveated) whose
 * scan time is t, and the undistorted point x of that panel point (x is the
 * panel point without a lens), whose pinhole ray is r. */
void orc_pixel_setup(const double *vp, int64_t pix, double y[2], double x[2], double *t, double r[3]) {
    int W = (int)vp[ORC_W], H = (int)vp[ORC_H];
    int64_t i = pix % W, j = pix / W;
    y[0] = 2.0 * (i + 0.5) / W - 1.0;
    y[1] = 1.0 - 2.0 * (j + 0.5) / H;
    double xp[2];
    orc_unfoveate(vp, y, xp);
    *t = orc_pixel_time(vp, xp);
    orc_undistort(vp, xp, x);
    r[0] = (x[0] - vp[ORC_CX]) / vp[ORC_FX];
    r[1] = (x[1] - vp[ORC_CY]) / vp[ORC_FY];
    r[2] = 1.0;
}

/* ------------------------------------------------------------------------- */
/* camera-space vertices (vertex program, Sec. 3.2 "Bounding")                */
/* ------------------------------------------------------------------------- */
typedef struct {
    double R0[9], T0[3], R1[9], T1[3];
    double *Ps, *Pe;   /* [nv][3] view space at t0 / t1 */
} orc_cam;

static void cam_init(orc_cam *c, const double *vp, const double *v0, const double *v1, int nv) {
    orc_rodrigues(vp + ORC_POSE0, c->R0);
    orc_rodrigues(vp + ORC_POSE1, c->R1);
    for (int k = 0; k < 3; ++k) { c->T0[k] = vp[ORC_POSE0 + 3 + k]; c->T1[k] = vp[ORC_POSE1 + 3 + k]; }
    c->Ps = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
    c->Pe = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
    for (int v = 0; v < nv; ++v) {
        matvec(c->R0, v0 + 3 * (size_t)v, c->Ps + 3 * (size_t)v);
        matvec(c->R1, v1 + 3 * (size_t)v, c->Pe + 3 * (size_t)v);
        for (int k = 0; k < 3; ++k) { c->Ps[3 * v + k] += c->T0[k]; c->Pe[3 * v + k] += c->T1[k]; }
    }
}
static void cam_free(orc_cam *c) { free(c->Ps); free(c->Pe); }

/* Triangle interpolated to time t (linear vertex motion in camera space). */
static void tri_at(const orc_cam *c, const int32_t *tri, int64_t f, double t, double P[3][3]) {
    for (int k = 0; k < 3; ++k) {
        int64_t v = tri[3 * f + k];
        for (int d = 0; d < 3; ++d) P[k][d] = (1.0 - t) * c->Ps[3 * v + d] + t * c->Pe[3 * v + d];
    }
}

/* Ray-triangle test for a ray from the eye (origin) along r.
 * e_k = r . (P_a x P_b), (a,b) = (k+1, k+2) mod 3; S = sum e_k;
 * D = P_0 . (P_1 x P_2).  Hit iff S != 0, the e_k share a sign (zero allowed,
 * two-sided), and the hit depth z = D/S is at least znear.
 * Returns 1 on hit; fills z and the normalised edge magnitude
 * ehat = min_k |e_k| / (|r| |P_a x P_b|) (sine of the ray / edge-plane angle). */
static int ray_tri(const double P[3][3], const double r[3], double znear, double *z, double *ehat, double e[3]) {
    double c[3][3];
    for (int k = 0; k < 3; ++k) {
        cross3(P[(k + 1) % 3], P[(k + 2) % 3], c[k]);
        e[k] = dot3(r, c[k]);
    }
    double S = e[0] + e[1] + e[2];
    double D = dot3(P[0], c[0]);
    int pos = e[0] >= 0 && e[1] >= 0 && e[2] >= 0;
    int neg = e[0] <= 0 && e[1] <= 0 && e[2] <= 0;
    double rn = norm3(r);
    double em = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double cn = norm3(c[k]);
        double v = cn > 0 ? fabs(e[k]) / (rn * cn) : 0.0;
        if (v < em) em = v;
    }
    *ehat = em;
    if (S == 0.0 || !(pos || neg)) { *z = INFINITY; return 0; }
    *z = D / S;
    return *z >= znear;
}

/* ------------------------------------------------------------------------- */
/* public entry points                                                        */
/* ------------------------------------------------------------------------- */

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Brute force render of the given pixels (pix == NULL: all W*H pixels).
 * Per pixel: winner id (-1 = miss), its depth (+inf = miss) and ehat, and the
 * runner-up (second in (depth, id) order) id and depth.  Exact depth ties go
 * to the lower triangle index. */
void orc_render(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
                const int64_t *pix, int64_t npix, int32_t *out_id, double *out_z, double *out_ehat,
                int32_t *out_id2, double *out_z2) {
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
    if (!pix) npix = (int64_t)vp[ORC_W] * (int64_t)vp[ORC_H];
    double znear = vp[ORC_ZNEAR];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t p = pix ? pix[q] : q;
        double y[2], x[2], t, r[3];
        orc_pixel_setup(vp, p, y, x, &t, r);
        double bz = INFINITY, bz2 = INFINITY, beh = 0;
        int32_t bid = -1, bid2 = -1;
        for (int f = 0; f < nt; ++f) {
            double P[3][3], z, eh, e[3];
            tri_at(&cam, tri, f, t, P);
            if (!ray_tri(P, r, znear, &z, &eh, e)) continue;
            if (z < bz) {            /* f > bid always, so equal z keeps the lower id */
                bz2 = bz; bid2 = bid;
                bz = z; bid = f; beh = eh;
            } else if (z < bz2) {
                bz2 = z; bid2 = f;
            }
        }
        if (out_id) out_id[q] = bid;
        if (out_z) out_z[q] = bz;
        if (out_ehat) out_ehat[q] = bid >= 0 ? beh : INFINITY;
        if (out_id2) out_id2[q] = bid2;
        if (out_z2) out_z2[q] = bz2;
    }
    cam_free(&cam);
}

/* Evaluate one (pixel, triangle) pair: returns hit flag; out[0] = z (D/S, or
 * +inf if no line hit), out[1] = ehat, out[2] = pixel time. */
int orc_eval(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
             int64_t pix, int f, double *out) {
    (void)nt;
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
    double y[2], x[2], t, r[3], P[3][3], z, eh, e[3];
    orc_pixel_setup(vp, pix, y, x, &t, r);
    tri_at(&cam, tri, f, t, P);
    int hit = ray_tri(P, r, vp[ORC_ZNEAR], &z, &eh, e);
    out[0] = z;
    out[1] = eh;
    out[2] = t;
    cam_free(&cam);
    return hit;
}

/* Batched orc_eval over (pix[q], tri_ids[q]) pairs.  cosinc (may be NULL):
 * |cos| of the angle between the ray and the triangle's normal, which sets
 * how strongly the hit depth reacts to a perturbation of the ray. */
void orc_eval_many(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
                   const int64_t *pix, const int32_t *fid, int64_t n, int32_t *hit, double *z, double *ehat,
                   double *cosinc) {
    (void)nt;
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        double y[2], x[2], t, r[3], P[3][3], zz, eh, e[3];
        orc_pixel_setup(vp, pix[q], y, x, &t, r);
        tri_at(&cam, tri, fid[q], t, P);
        hit[q] = ray_tri(P, r, vp[ORC_ZNEAR], &zz, &eh, e);
        z[q] = zz;
        ehat[q] = eh;
        if (cosinc) {
            double e1[3], e2[3], N[3];
            for (int d = 0; d < 3; ++d) { e1[d] = P[1][d] - P[0][d]; e2[d] = P[2][d] - P[0][d]; }
            cross3(e1, e2, N);
            double nn = norm3(N) * norm3(r);
            cosinc[q] = nn > 0 ? fabs(dot3(N, r)) / nn : 0.0;
        }
    }
    cam_free(&cam);
}

/* Every (pixel, triangle) hit, occluded or not, over the given pixels.
 * Writes up to cap pairs; returns the total count (may exceed cap). */
int64_t orc_all_hits(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
                     const int64_t *pix, int64_t npix, int64_t *out_pix, int32_t *out_tri, double *out_ehat,
                     int64_t cap) {
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
    if (!pix) npix = (int64_t)vp[ORC_W] * (int64_t)vp[ORC_H];
    int64_t count = 0;
    for (int64_t q = 0; q < npix; ++q) {
        int64_t p = pix ? pix[q] : q;
        double y[2], x[2], t, r[3];
        orc_pixel_setup(vp, p, y, x, &t, r);
        for (int f = 0; f < nt; ++f) {
            double P[3][3], z, eh, e[3];
            tri_at(&cam, tri, f, t, P);
            if (!ray_tri(P, r, vp[ORC_ZNEAR], &z, &eh, e)) continue;
            if (count < cap) { out_pix[count] = p; out_tri[count] = f; out_ehat[count] = eh; }
            ++count;
        }
    }
    cam_free(&cam);
    return count;
}

/* ------------------------------------------------------------------------- */
/* the same render with a conservative display-space grid (oracle_fast)       */
/* ------------------------------------------------------------------------- */

/* Keeps the two smallest (z, f) pairs in lexicographic order: exactly the
 * winner and runner-up of orc_render whatever order triangles arrive in. */
static void keep_two(double z, int32_t f, double eh, double *bz, int32_t *bid, double *beh, double *bz2,
                     int32_t *bid2) {
    if (z < *bz || (z == *bz && f < *bid)) {
        *bz2 = *bz; *bid2 = *bid;
        *bz = z; *bid = f; *beh = eh;
    } else if (z < *bz2 || (z == *bz2 && f < *bid2)) {
        *bz2 = z; *bid2 = f;
    }
}

/* Grid cell of a display coordinate: [-1, 1] split into g equal cells,
 * clamped (monotone, so a clamped box still contains every clamped point
 * of it). */
static int grid_cell(double x, int g) {
    double u = (x + 1.0) * 0.5 * g;
    if (!(u > 0.0)) return 0;
    if (u >= g) return g - 1;
    return (int)u;
}

/* orc_render with the same outputs, bit for bit, computed faster: a
 * triangle can only be hit at a pixel whose display point lies in the
 * projection of the triangle at the pixel's time, which lies in the convex
 * hull of the six projected start and end vertices when all six are in
 * front of the near plane (every point of the triangle at any time in
 * [0, 1] is a convex combination of them, and projection keeps convex
 * hulls in front of the eye); so each such triangle is listed in the cells
 * of a g x g grid over the display square that its six points' box
 * (padded) touches.  A triangle with every space-time vertex behind the
 * near plane can never be hit (its points all have z < znear); one with
 * some in front and some behind is tested at every pixel.  Per pixel the
 * same ray_tri test as orc_render runs on the triangles of its display
 * point's cell, and the pixel keeps the same winner and runner-up. */
void orc_render_fast(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
                     const int64_t *pix, int64_t npix, int32_t *out_id, double *out_z, double *out_ehat,
                     int32_t *out_id2, double *out_z2, int g) {
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
    if (!pix) npix = (int64_t)vp[ORC_W] * (int64_t)vp[ORC_H];
    if (g < 1) g = 1;
    const double znear = vp[ORC_ZNEAR];
    int *rect = (int *)malloc(sizeof(int) * 4 * (size_t)(nt > 0 ? nt : 1));
    unsigned char *kind = (unsigned char *)malloc((size_t)(nt > 0 ? nt : 1));   /* 0 never, 1 grid, 2 everywhere */
    int64_t *cnt = (int64_t *)calloc((size_t)g * g + 1, sizeof(int64_t));
    int64_t nglob = 0;
    for (int f = 0; f < nt; ++f) {
        double pts[6][3];
        int n_in = 0;
        for (int k = 0; k < 3; ++k) {
            int64_t v = tri[3 * (int64_t)f + k];
            for (int d = 0; d < 3; ++d) {
                pts[k][d] = cam.Ps[3 * v + d];
                pts[3 + k][d] = cam.Pe[3 * v + d];
            }
        }
        for (int i = 0; i < 6; ++i) n_in += pts[i][2] >= znear;
        if (n_in == 0) { kind[f] = 0; continue; }
        if (n_in < 6) { kind[f] = 2; ++nglob; continue; }
        double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
        for (int i = 0; i < 6; ++i) {
            double q[2] = {vp[ORC_FX] * pts[i][0] / pts[i][2] + vp[ORC_CX], vp[ORC_FY] * pts[i][1] / pts[i][2] + vp[ORC_CY]};
            for (int a = 0; a < 2; ++a) {
                if (q[a] < lo[a]) lo[a] = q[a];
                if (q[a] > hi[a]) hi[a] = q[a];
            }
        }
        for (int a = 0; a < 2; ++a) {   /* far above the rounding of the projections */
            lo[a] -= 1e-9 * (1.0 + fabs(lo[a]));
            hi[a] += 1e-9 * (1.0 + fabs(hi[a]));
        }
        kind[f] = 1;
        int *r = rect + 4 * (size_t)f;
        r[0] = grid_cell(lo[0], g); r[1] = grid_cell(hi[0], g);
        r[2] = grid_cell(lo[1], g); r[3] = grid_cell(hi[1], g);
        for (int cy = r[2]; cy <= r[3]; ++cy)
            for (int cx = r[0]; cx <= r[1]; ++cx) ++cnt[(size_t)cy * g + cx + 1];
    }
    for (size_t c = 0; c < (size_t)g * g; ++c) cnt[c + 1] += cnt[c];
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt[(size_t)g * g] > 0 ? cnt[(size_t)g * g] : 1));
    int32_t *glob = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nglob > 0 ? nglob : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)g * g);
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)g * g);
    nglob = 0;
    for (int f = 0; f < nt; ++f) {
        if (kind[f] == 2) glob[nglob++] = f;
        if (kind[f] != 1) continue;
        const int *r = rect + 4 * (size_t)f;
        for (int cy = r[2]; cy <= r[3]; ++cy)
            for (int cx = r[0]; cx <= r[1]; ++cx) list[fill[(size_t)cy * g + cx]++] = f;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t p = pix ? pix[q] : q;
        double y[2], x[2], t, r[3];
        orc_pixel_setup(vp, p, y, x, &t, r);
        double bz = INFINITY, bz2 = INFINITY, beh = 0;
        int32_t bid = -1, bid2 = -1;
        size_t c = (size_t)grid_cell(x[1], g) * g + grid_cell(x[0], g);
        for (int pass = 0; pass < 2; ++pass) {
            const int32_t *L = pass ? glob : list + cnt[c];
            int64_t n = pass ? nglob : cnt[c + 1] - cnt[c];
            for (int64_t i = 0; i < n; ++i) {
                double P[3][3], z, eh, e[3];
                tri_at(&cam, tri, L[i], t, P);
                if (!ray_tri(P, r, znear, &z, &eh, e)) continue;
                keep_two(z, L[i], eh, &bz, &bid, &beh, &bz2, &bid2);
            }
        }
        if (out_id) out_id[q] = bid;
        if (out_z) out_z[q] = bz;
        if (out_ehat) out_ehat[q] = bid >= 0 ? beh : INFINITY;
        if (out_id2) out_id2[q] = bid2;
        if (out_z2) out_z2[q] = bz2;
    }
    free(rect); free(kind); free(cnt); free(list); free(glob); free(fill);
    cam_free(&cam);
}

/* ------------------------------------------------------------------------- */
/* rolling Lambert shading and its gradient (frozen visibility)              */
/* ------------------------------------------------------------------------- */

/* Rolling highlight (Sec. 3.2 "Shading": the eye position rolls like the
 * light; Sec. 5.1 "Rolling Shading"): in the camera frame at the pixel's
 * time the eye is the origin, so the direction from the surface towards it
 * is v = -r/|r|.  Blinn-Phong, white: h = normalize(l + v),
 * sigma = k_s (n.h)^m where n.l > 0 and n.h > 0, else 0 (also when l = -v). */
static double highlight(const double n[3], const double l[3], const double r[3], double ks, double m) {
    if (ks == 0.0 || dot3(n, l) <= 0.0) return 0.0;
    double rn = norm3(r);
    double H[3] = {l[0] - r[0] / rn, l[1] - r[1] / rn, l[2] - r[2] / rn};
    double hn = norm3(H);
    if (hn == 0.0) return 0.0;
    double ndh = dot3(n, H) / hn;
    return ndh > 0.0 ? ks * pow(ndh, m) : 0.0;
}

/* Shade one pixel whose visible triangle is f.  light = (l_w[3], k_a, k_s, m).
 * n = face normal flipped to face the eye; l(t) = normalize((1-t) R0 l_w +
 * t R1 l_w); albedo = barycentric (mu_k = e_k/S) blend of per-vertex albedo;
 * c = albedo * (k_a + (1-k_a) max(0, n.l)) + highlight(n, l, r). */
static void shade_px(const orc_cam *cam, const double *vp, const int32_t *tri, const double *albedo,
                     const double *light, int64_t p, int f, double c[3]) {
    double y[2], x[2], t, r[3], P[3][3];
    orc_pixel_setup(vp, p, y, x, &t, r);
    tri_at(cam, tri, f, t, P);
    double e[3], ck[3][3];
    for (int k = 0; k < 3; ++k) {
        cross3(P[(k + 1) % 3], P[(k + 2) % 3], ck[k]);
        e[k] = dot3(r, ck[k]);
    }
    double S = e[0] + e[1] + e[2];
    double N[3], e1[3], e2[3];
    for (int d = 0; d < 3; ++d) { e1[d] = P[1][d] - P[0][d]; e2[d] = P[2][d] - P[0][d]; }
    cross3(e1, e2, N);
    double nn = norm3(N);
    double n[3] = {N[0] / nn, N[1] / nn, N[2] / nn};
    if (dot3(n, r) > 0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
    double l0[3], l1[3], L[3];
    matvec(cam->R0, light, l0);
    matvec(cam->R1, light, l1);
    for (int d = 0; d < 3; ++d) L[d] = (1.0 - t) * l0[d] + t * l1[d];
    double ln = norm3(L);
    double ndl = dot3(n, L) / ln;
    double s = light[3] + (1.0 - light[3]) * (ndl > 0 ? ndl : 0.0);
    double l[3] = {L[0] / ln, L[1] / ln, L[2] / ln};
    double sigma = highlight(n, l, r, light[4], light[5]);
    for (int ch = 0; ch < 3; ++ch) {
        double a = 0;
        for (int k = 0; k < 3; ++k) a += e[k] / S * albedo[3 * (size_t)tri[3 * f + k] + ch];
        c[ch] = a * s + sigma;
    }
}

/* Shade pixels given their (frozen) triangle ids; misses give 0. */
void orc_shade(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
               const double *albedo, const double *light, const int64_t *pix, int64_t npix,
               const int32_t *ids, double *out_rgb) {
    (void)nt;
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
    if (!pix) npix = (int64_t)vp[ORC_W] * (int64_t)vp[ORC_H];
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t p = pix ? pix[q] : q;
        double c[3] = {0, 0, 0};
        if (ids[q] >= 0) shade_px(&cam, vp, tri, albedo, light, p, ids[q], c);
        for (int ch = 0; ch < 3; ++ch) out_rgb[3 * q + ch] = c[ch];
    }
    cam_free(&cam);
}

/* L = sum over pixels and channels of (c - target)^2 with the full-image id
 * buffer frozen (background contributes (0 - target)^2). */
double orc_loss(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
                const double *albedo, const double *light, const int32_t *ids, const double *target) {
    (void)nt;
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
    int64_t npix = (int64_t)vp[ORC_W] * (int64_t)vp[ORC_H];
    double L = 0;
#pragma omp parallel for schedule(static) reduction(+ : L)
    for (int64_t p = 0; p < npix; ++p) {
        double c[3] = {0, 0, 0};
        if (ids[p] >= 0) shade_px(&cam, vp, tri, albedo, light, p, ids[p], c);
        for (int ch = 0; ch < 3; ++ch) {
            double d = c[ch] - target[3 * p + ch];
            L += d * d;
        }
    }
    cam_free(&cam);
    return L;
}

/* Analytic gradient of orc_loss by the chain rule through shading,
 * barycentrics, the face normal, the rolling light, camera-space
 * interpolation, the vertex transform and Rodrigues' formula.
 * Outputs: gv0, gv1 [nv][3] (world vertex positions at t0 / t1),
 * gpose0, gpose1 [6] (rotation vector then translation).  Returns L. */
double orc_loss_grad(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
                     const double *albedo, const double *light, const int32_t *ids, const double *target,
                     double *gv0, double *gv1, double *gpose0, double *gpose1) {
    (void)nt;
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
    int64_t npix = (int64_t)vp[ORC_W] * (int64_t)vp[ORC_H];
    int nth = orc_get_threads();
    /* per-thread accumulators: gradient w.r.t. camera-space start/end vertex
     * positions, the rotation matrices (light term) and the loss */
    double *gPs = (double *)calloc((size_t)nth * 3 * nv, sizeof(double));
    double *gPe = (double *)calloc((size_t)nth * 3 * nv, sizeof(double));
    double *gRl = (double *)calloc((size_t)nth * 18, sizeof(double));
    double *Lt = (double *)calloc((size_t)nth, sizeof(double));
    double lw0[3], lw1[3];
    matvec(cam.R0, light, lw0);
    matvec(cam.R1, light, lw1);
    const double ka = light[3];
#pragma omp parallel num_threads(nth)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mPs = gPs + (size_t)tid * 3 * nv, *mPe = gPe + (size_t)tid * 3 * nv, *mR = gRl + 18 * tid;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < npix; ++p) {
            int f = ids[p];
            double c[3] = {0, 0, 0};
            if (f < 0) {
                for (int ch = 0; ch < 3; ++ch) { double d = -target[3 * p + ch]; Lt[tid] += d * d; }
                continue;
            }
            double y[2], x[2], t, r[3], P[3][3];
            orc_pixel_setup(vp, p, y, x, &t, r);
            tri_at(&cam, tri, f, t, P);
            double ck[3][3], e[3];
            for (int k = 0; k < 3; ++k) {
                cross3(P[(k + 1) % 3], P[(k + 2) % 3], ck[k]);
                e[k] = dot3(r, ck[k]);
            }
            double S = e[0] + e[1] + e[2];
            double mu[3] = {e[0] / S, e[1] / S, e[2] / S};
            double N[3] = {ck[0][0] + ck[1][0] + ck[2][0], ck[0][1] + ck[1][1] + ck[2][1],
                           ck[0][2] + ck[1][2] + ck[2][2]};
            double nn = norm3(N);
            double m[3] = {N[0] / nn, N[1] / nn, N[2] / nn};
            double sg = dot3(m, r) > 0 ? -1.0 : 1.0;
            double n[3] = {sg * m[0], sg * m[1], sg * m[2]};
            double Lw[3];
            for (int d = 0; d < 3; ++d) Lw[d] = (1.0 - t) * lw0[d] + t * lw1[d];
            double lnorm = norm3(Lw);
            double l[3] = {Lw[0] / lnorm, Lw[1] / lnorm, Lw[2] / lnorm};
            double ndl = dot3(n, l);
            double s = ka + (1.0 - ka) * (ndl > 0 ? ndl : 0.0);
            double sigma = highlight(n, l, r, light[4], light[5]);
            double a[3];
            const int32_t *tv = tri + 3 * (size_t)f;
            for (int ch = 0; ch < 3; ++ch) {
                a[ch] = 0;
                for (int k = 0; k < 3; ++k) a[ch] += mu[k] * albedo[3 * (size_t)tv[k] + ch];
                c[ch] = a[ch] * s + sigma;
            }
            double gc[3];
            for (int ch = 0; ch < 3; ++ch) {
                double d = c[ch] - target[3 * p + ch];
                Lt[tid] += d * d;
                gc[ch] = 2.0 * d;
            }
            /* c = a s */
            double gs = dot3(gc, a);
            double ga[3] = {gc[0] * s, gc[1] * s, gc[2] * s};
            /* a = sum_k mu_k albedo_k */
            double gmu[3];
            for (int k = 0; k < 3; ++k) gmu[k] = dot3(ga, albedo + 3 * (size_t)tv[k]);
            /* s = ka + (1-ka) max(0, n.l) */
            double gndl = ndl > 0 ? gs * (1.0 - ka) : 0.0;
            double gn[3] = {gndl * l[0], gndl * l[1], gndl * l[2]};
            double gl[3] = {gndl * n[0], gndl * n[1], gndl * n[2]};
            /* sigma = k_s (n.h)^m (each channel), h = H/|H|, H = l - r/|r|:
             * dsigma/dn = k_s m (n.h)^(m-1) h, dsigma/dh = k_s m (n.h)^(m-1) n */
            if (sigma > 0.0) {
                double rn = norm3(r);
                double H[3] = {l[0] - r[0] / rn, l[1] - r[1] / rn, l[2] - r[2] / rn};
                double hn = norm3(H);
                double h[3] = {H[0] / hn, H[1] / hn, H[2] / hn};
                double gsig = (gc[0] + gc[1] + gc[2]) * light[4] * light[5] * pow(dot3(n, h), light[5] - 1.0);
                double gh[3] = {gsig * n[0], gsig * n[1], gsig * n[2]};
                double hg = dot3(h, gh);
                for (int d = 0; d < 3; ++d) {
                    gn[d] += gsig * h[d];
                    gl[d] += (gh[d] - h[d] * hg) / hn;
                }
            }
            /* n = sg N/|N| */
            double gm[3] = {sg * gn[0], sg * gn[1], sg * gn[2]};
            double mg = dot3(m, gm);
            double gN[3];
            for (int d = 0; d < 3; ++d) gN[d] = (gm[d] - m[d] * mg) / nn;
            /* l = Lw/|Lw|, Lw = (1-t) R0 lw + t R1 lw */
            double lg = dot3(l, gl);
            double gLw[3];
            for (int d = 0; d < 3; ++d) gLw[d] = (gl[d] - l[d] * lg) / lnorm;
            for (int rr = 0; rr < 3; ++rr)
                for (int cc = 0; cc < 3; ++cc) {
                    mR[3 * rr + cc] += (1.0 - t) * gLw[rr] * light[cc];
                    mR[9 + 3 * rr + cc] += t * gLw[rr] * light[cc];
                }
            /* mu_k = e_k / S */
            double sm = gmu[0] * mu[0] + gmu[1] * mu[1] + gmu[2] * mu[2];
            double ge[3];
            for (int k = 0; k < 3; ++k) ge[k] = (gmu[k] - sm) / S;
            /* e_k = r . c_k, N = sum_k c_k, c_k = P_a x P_b */
            double gP[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int k = 0; k < 3; ++k) {
                double g[3];
                for (int d = 0; d < 3; ++d) g[d] = ge[k] * r[d] + gN[d];
                int ia = (k + 1) % 3, ib = (k + 2) % 3;
                double ta[3], tb[3];
                cross3(P[ib], g, ta);   /* d/dP_a of g.(P_a x P_b) = P_b x g */
                cross3(g, P[ia], tb);   /* d/dP_b of g.(P_a x P_b) = g x P_a */
                for (int d = 0; d < 3; ++d) { gP[ia][d] += ta[d]; gP[ib][d] += tb[d]; }
            }
            /* P_k = (1-t) Ps_k + t Pe_k */
            for (int k = 0; k < 3; ++k)
                for (int d = 0; d < 3; ++d) {
                    mPs[3 * (size_t)tv[k] + d] += (1.0 - t) * gP[k][d];
                    mPe[3 * (size_t)tv[k] + d] += t * gP[k][d];
                }
        }
    }
    /* reduce thread partials in thread order */
    double L = 0;
    for (int th = 0; th < nth; ++th) L += Lt[th];
    for (int th = 1; th < nth; ++th) {
        for (size_t i = 0; i < 3 * (size_t)nv; ++i) { gPs[i] += gPs[(size_t)th * 3 * nv + i]; gPe[i] += gPe[(size_t)th * 3 * nv + i]; }
        for (int i = 0; i < 18; ++i) gRl[i] += gRl[18 * th + i];
    }
    /* Ps_v = R0 v0_v + T0 -> gv0 = R0^T gPs, gT0 = sum gPs, gR0 = sum gPs v0^T (+ light term) */
    double gR0[9], gR1[9], gT0[3] = {0, 0, 0}, gT1[3] = {0, 0, 0};
    for (int i = 0; i < 9; ++i) { gR0[i] = gRl[i]; gR1[i] = gRl[9 + i]; }
    for (int v = 0; v < nv; ++v) {
        const double *gs_ = gPs + 3 * (size_t)v, *ge_ = gPe + 3 * (size_t)v;
        matTvec(cam.R0, gs_, gv0 + 3 * (size_t)v);
        matTvec(cam.R1, ge_, gv1 + 3 * (size_t)v);
        for (int rr = 0; rr < 3; ++rr) {
            gT0[rr] += gs_[rr];
            gT1[rr] += ge_[rr];
            for (int cc = 0; cc < 3; ++cc) {
                gR0[3 * rr + cc] += gs_[rr] * v0[3 * (size_t)v + cc];
                gR1[3 * rr + cc] += ge_[rr] * v1[3 * (size_t)v + cc];
            }
        }
    }
    double J0[27], J1[27];
    orc_rodrigues_jac(vp + ORC_POSE0, J0);
    orc_rodrigues_jac(vp + ORC_POSE1, J1);
    for (int i = 0; i < 3; ++i) {
        double s0 = 0, s1 = 0;
        for (int k = 0; k < 9; ++k) { s0 += gR0[k] * J0[9 * i + k]; s1 += gR1[k] * J1[9 * i + k]; }
        gpose0[i] = s0;
        gpose1[i] = s1;
        gpose0[3 + i] = gT0[i];
        gpose1[3 + i] = gT1[i];
    }
    free(gPs); free(gPe); free(gRl); free(Lt);
    cam_free(&cam);
    return L;
}

/* ------------------------------------------------------------------------- */
/* G-buffer (Sec. 3.2 "Pipeline": the deferred shading buffer; Sec. 7         */
/* "Screen-space effects": image distances scaled by the pixel density)       */
/* ------------------------------------------------------------------------- */
void orc_foveate_jac(const double *vp, const double x[2], double JF[4]);

/* Per pixel: the visible triangle's unit face normal at the pixel's time in
 * the camera frame, turned towards the eye; the barycentrics mu_1, mu_2 of
 * the ray's hit (mu_k = e_k / S); the pixel density, the square root of the
 * Jacobian determinant of the foveate map at the pixel's display (panel)
 * point (how much a short display-space length grows in the foveated image;
 * a lens is undone optically, not by the display, so it does not enter).  Misses
 * give zero normal and barycentrics; the density is written for every pixel. */
void orc_gbuffer(const double *vp, const double *v0, const double *v1, int nv, const int32_t *tri, int nt,
                 const int64_t *pix, int64_t npix, const int32_t *ids, double *out_normal, double *out_bary,
                 double *out_density) {
    (void)nt;
    orc_cam cam;
    cam_init(&cam, vp, v0, v1, nv);
    if (!pix) npix = (int64_t)vp[ORC_W] * (int64_t)vp[ORC_H];
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t p = pix ? pix[q] : q;
        double y[2], x[2], t, r[3];
        orc_pixel_setup(vp, p, y, x, &t, r);
        double xp[2], JF[4];   /* the foveation's Jacobian at the panel point */
        orc_unfoveate(vp, y, xp);
        orc_foveate_jac(vp, xp, JF);
        out_density[q] = sqrt(fabs(JF[0] * JF[3] - JF[1] * JF[2]));
        double n[3] = {0, 0, 0}, mu[3] = {0, 0, 0};
        int f = ids[q];
        if (f >= 0) {
            double P[3][3], e[3], ck[3];
            tri_at(&cam, tri, f, t, P);
            for (int k = 0; k < 3; ++k) {
                cross3(P[(k + 1) % 3], P[(k + 2) % 3], ck);
                e[k] = dot3(r, ck);
            }
            double S = e[0] + e[1] + e[2];
            for (int k = 0; k < 3; ++k) mu[k] = e[k] / S;
            double e1[3], e2[3], N[3];
            for (int d = 0; d < 3; ++d) { e1[d] = P[1][d] - P[0][d]; e2[d] = P[2][d] - P[0][d]; }
            cross3(e1, e2, N);
            double nn = norm3(N);
            for (int d = 0; d < 3; ++d) n[d] = N[d] / nn;
            if (dot3(n, r) > 0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
        }
        for (int d = 0; d < 3; ++d) out_normal[3 * q + d] = n[d];
        out_bary[2 * q] = mu[1];
        out_bary[2 * q + 1] = mu[2];
    }
    cam_free(&cam);
}

/* ------------------------------------------------------------------------- */
/* display unfoveation (Sec. 3.1.1 "Display")                                 */
/* ------------------------------------------------------------------------- */
/* The foveated image I_f (W x H, its pixel grid in the foveated domain) is
 * resampled to the display's regular grid (Wd x Hd): display pixel (a, b)
 * has display NDC x = (2(a+1/2)/Wd - 1, 1 - 2(b+1/2)/Hd), foveated NDC
 * y = foveate(x), and continuous foveated pixel coordinates
 * u = ((y0+1)/2 W - 1/2, (1-y1)/2 H - 1/2) (texel centres at integers).
 *
 * Fast form: a MIP pyramid of I_f (level k+1 = 2x2 box mean of level k,
 * sizes halved rounding up, the last row / column repeated where a level
 * is odd) sampled at u with level of detail lambda = log2 of the longer
 * image of a display pixel step in foveated pixels: lambda <= 0 (the
 * display magnifies, the periphery) a separable cubic interpolation
 * (Catmull-Rom) of level 0; 0 < lambda < 1 its linear blend with the
 * bilinear sample of level 1; lambda >= 1 trilinear (bilinear at levels
 * floor(lambda) and floor(lambda)+1, linear between them), the top level
 * held past the pyramid.  Level k is addressed at u_k = (u + 1/2)/2^k - 1/2,
 * edges clamped.
 *
 * Reconstruction-filter form: the 5 x 5 foveated pixels around the nearest
 * one to u, each weighted by a Gaussian of its distance to the display
 * pixel measured in display pixels after unfoveating its centre,
 * exp(-d^2 / (2 sigma^2)), normalised by the sum of the weights; pixels
 * outside the image are skipped.
 *
 * Images: RGBA in [0,1], row-major [rows][cols][4] doubles. */

/* u of display pixel (a, b) and the 2x2 Jacobian du/d(a, b) (J[0] = du0/da,
 * J[1] = du0/db, J[2] = du1/da, J[3] = du1/db).  The foveation is the radial
 * power map y = f + (x - f) s, s = (|x - f|/R)^(1/alpha - 1); its Jacobian
 * is s I + (1/alpha - 1) s (x - f)(x - f)^T / |x - f|^2.  At the fovea
 * itself (alpha > 1) the map's derivative is unbounded: lambda = +inf. */
/* Jacobian dy/dx of the foveate map at display NDC x (row-major 2x2). */
void orc_foveate_jac(const double *vp, const double x[2], double JF[4]) {
    double d[2] = {x[0] - vp[ORC_FOV], x[1] - vp[ORC_FOV + 1]};
    double rho2 = d[0] * d[0] + d[1] * d[1];
    if (vp[ORC_NC] > 0) {
        /* y - f = (x - f) g(s)/s, s = |x - f|/R: J = (g/s) I + (g' - g/s) n n^T
         * with n the unit direction; at the fovea g/s -> g'(0) */
        const double *tab = vp + ORC_PC;
        int n = (int)vp[ORC_NC];
        double rho = sqrt(rho2), s = rho / orc_fovea_radius(vp);
        double gp = tab_slope(tab, n, s), gs = rho2 == 0.0 ? gp : tab_eval(tab, n, s) / s;
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c)
                JF[2 * r + c] = (r == c ? gs : 0.0) + (rho2 == 0.0 ? 0.0 : (gp - gs) * d[r] * d[c] / rho2);
        return;
    }
    double e = 1.0 / vp[ORC_ALPHA];
    if (rho2 == 0.0) {
        double v = e == 1.0 ? 1.0 : INFINITY;
        JF[0] = v; JF[1] = 0.0; JF[2] = 0.0; JF[3] = v;
    } else {
        double s = pow(sqrt(rho2) / orc_fovea_radius(vp), e - 1.0);
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) JF[2 * r + c] = (r == c ? s : 0.0) + (e - 1.0) * s * d[r] * d[c] / rho2;
    }
}

void orc_unfov_coord(const double *vp, int Wd, int Hd, double a, double b, double u[2], double J[4]) {
    int W = (int)vp[ORC_W], H = (int)vp[ORC_H];
    double x[2] = {2.0 * (a + 0.5) / Wd - 1.0, 1.0 - 2.0 * (b + 0.5) / Hd};
    double y[2];
    orc_foveate(vp, x, y);
    u[0] = (y[0] + 1.0) * 0.5 * W - 0.5;
    u[1] = (1.0 - y[1]) * 0.5 * H - 0.5;
    double JF[4];
    orc_foveate_jac(vp, x, JF);
    /* u = diag(W/2, -H/2) y + const, x = diag(2/Wd, -2/Hd) (a, b) + const */
    double su[2] = {0.5 * W, -0.5 * H}, sx[2] = {2.0 / Wd, -2.0 / Hd};
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) J[2 * r + c] = su[r] * JF[2 * r + c] * sx[c];
}

typedef struct {
    int n;               /* levels */
    int w[32], h[32];
    double *lev[32];     /* [h][w][4] */
} orc_mip;

static void mip_build(orc_mip *m, const double *img, int W, int H) {
    m->n = 0;
    int w = W, h = H;
    const double *src = img;
    for (;;) {
        double *dst = (double *)malloc(sizeof(double) * 4 * (size_t)w * h);
        if (m->n == 0) {
            memcpy(dst, img, sizeof(double) * 4 * (size_t)w * h);
        } else {
            int pw = m->w[m->n - 1], ph = m->h[m->n - 1];
            for (int j = 0; j < h; ++j)
                for (int i = 0; i < w; ++i)
                    for (int c = 0; c < 4; ++c) {
                        double s = 0.0;
                        for (int dj = 0; dj < 2; ++dj)
                            for (int di = 0; di < 2; ++di) {
                                int ii = 2 * i + di, jj = 2 * j + dj;
                                if (ii > pw - 1) ii = pw - 1;
                                if (jj > ph - 1) jj = ph - 1;
                                s += src[4 * ((size_t)jj * pw + ii) + c];
                            }
                        dst[4 * ((size_t)j * w + i) + c] = 0.25 * s;
                    }
        }
        m->w[m->n] = w; m->h[m->n] = h; m->lev[m->n] = dst;
        src = dst;
        ++m->n;
        if ((w == 1 && h == 1) || m->n == 32) break;
        w = (w + 1) / 2;
        h = (h + 1) / 2;
    }
}

static void mip_free(orc_mip *m) {
    for (int k = 0; k < m->n; ++k) free(m->lev[k]);
}

static double texel(const orc_mip *m, int k, int i, int j, int c) {
    int w = m->w[k], h = m->h[k];
    if (i < 0) i = 0;
    if (i > w - 1) i = w - 1;
    if (j < 0) j = 0;
    if (j > h - 1) j = h - 1;
    return m->lev[k][4 * ((size_t)j * w + i) + c];
}

static void bilinear(const orc_mip *m, int k, const double u[2], double out[4]) {
    double sc = ldexp(1.0, -k);
    double uk0 = (u[0] + 0.5) * sc - 0.5, uk1 = (u[1] + 0.5) * sc - 0.5;
    double fi = floor(uk0), fj = floor(uk1);
    double ti = uk0 - fi, tj = uk1 - fj;
    int i = (int)fi, j = (int)fj;
    for (int c = 0; c < 4; ++c)
        out[c] = (1 - tj) * ((1 - ti) * texel(m, k, i, j, c) + ti * texel(m, k, i + 1, j, c)) +
                 tj * ((1 - ti) * texel(m, k, i, j + 1, c) + ti * texel(m, k, i + 1, j + 1, c));
}

/* Catmull-Rom weights of the taps at offsets -1, 0, 1, 2 from floor(u). */
static void catmull_rom_w(double t, double w[4]) {
    w[0] = 0.5 * (-t + 2 * t * t - t * t * t);
    w[1] = 0.5 * (2 - 5 * t * t + 3 * t * t * t);
    w[2] = 0.5 * (t + 4 * t * t - 3 * t * t * t);
    w[3] = 0.5 * (-t * t + t * t * t);
}

static void cubic0(const orc_mip *m, const double u[2], double out[4]) {
    double fi = floor(u[0]), fj = floor(u[1]);
    double wi[4], wj[4];
    catmull_rom_w(u[0] - fi, wi);
    catmull_rom_w(u[1] - fj, wj);
    for (int c = 0; c < 4; ++c) {
        double s = 0.0;
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) s += wj[b] * wi[a] * texel(m, 0, (int)fi - 1 + a, (int)fj - 1 + b, c);
        out[c] = s;
    }
}

/* The MIP form's value at continuous foveated coordinates u with level of
 * detail lam. */
static void mip_sample(const orc_mip *m, const double u[2], double lam, double out[4]) {
    double a[4], b[4];
    int top = m->n - 1;
    if (!(lam > 0.0)) {
        cubic0(m, u, out);
    } else if (lam < 1.0) {
        cubic0(m, u, a);
        bilinear(m, top >= 1 ? 1 : 0, u, b);
        for (int c = 0; c < 4; ++c) out[c] = (1.0 - lam) * a[c] + lam * b[c];
    } else {
        double k = floor(lam), fr = lam - k;
        if (k >= top) {
            bilinear(m, top, u, out);
        } else {
            bilinear(m, (int)k, u, a);
            bilinear(m, (int)k + 1, u, b);
            for (int c = 0; c < 4; ++c) out[c] = (1.0 - fr) * a[c] + fr * b[c];
        }
    }
}

/* Level of detail from the Jacobian: log2 of the longer column. */
double orc_unfov_lod(const double J[4]) {
    double c0 = sqrt(J[0] * J[0] + J[2] * J[2]), c1 = sqrt(J[1] * J[1] + J[3] * J[3]);
    double l = c0 > c1 ? c0 : c1;
    return log2(l);
}

/* The reconstruction filter at display pixel (a, b) with its 5 x 5 window
 * centred on foveated pixel (i0, j0) (the nearest one to u in the
 * definition; tests evaluate the neighbouring windows where the nearest is
 * a floating-point tie).  fov: [H][W][4]; out: 4 doubles. */
void orc_unfov_filter_at(const double *vp, const double *fov, int Wd, int Hd, int a, int b, int i0, int j0,
                         double sigma, double out[4]) {
    int W = (int)vp[ORC_W], H = (int)vp[ORC_H];
    double acc[4] = {0, 0, 0, 0}, ws = 0.0;
    for (int dj = -2; dj <= 2; ++dj)
        for (int di = -2; di <= 2; ++di) {
            int i = i0 + di, j = j0 + dj;
            if (i < 0 || i >= W || j < 0 || j >= H) continue;
            double yv[2] = {2.0 * (i + 0.5) / W - 1.0, 1.0 - 2.0 * (j + 0.5) / H}, xv[2];
            orc_unfoveate(vp, yv, xv);
            double da = (xv[0] + 1.0) * 0.5 * Wd - 0.5 - a, db = (1.0 - xv[1]) * 0.5 * Hd - 0.5 - b;
            double w = exp(-(da * da + db * db) / (2.0 * sigma * sigma));
            ws += w;
            for (int ch = 0; ch < 4; ++ch) acc[ch] += w * fov[4 * ((size_t)j * W + i) + ch];
        }
    int ic = i0 < 0 ? 0 : (i0 > W - 1 ? W - 1 : i0), jc = j0 < 0 ? 0 : (j0 > H - 1 ? H - 1 : j0);
    for (int ch = 0; ch < 4; ++ch) out[ch] = ws > 0.0 ? acc[ch] / ws : fov[4 * ((size_t)jc * W + ic) + ch];
}

/* Display image of the MIP form (mode 0) or the reconstruction filter
 * (mode 1, Gaussian sigma in display pixels).  fov: [H][W][4], out:
 * [Hd][Wd][4].  pix (nullable) selects display pixels (row-major indices);
 * out then holds npix entries. */
void orc_unfoveate_image(const double *vp, const double *fov, int Wd, int Hd, int mode, double sigma,
                         const int64_t *pix, int64_t npix, double *out) {
    orc_mip m;
    mip_build(&m, fov, (int)vp[ORC_W], (int)vp[ORC_H]);
    if (!pix) npix = (int64_t)Wd * Hd;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < npix; ++q) {
        int64_t p = pix ? pix[q] : q;
        double a = (double)(p % Wd), b = (double)(p / Wd);
        double u[2], J[4], c[4];
        orc_unfov_coord(vp, Wd, Hd, a, b, u, J);
        if (mode == 0) {
            mip_sample(&m, u, orc_unfov_lod(J), c);
        } else {
            int i0 = (int)floor(u[0] + 0.5), j0 = (int)floor(u[1] + 0.5);
            orc_unfov_filter_at(vp, fov, Wd, Hd, (int)a, (int)b, i0, j0, sigma, c);
        }
        for (int ch = 0; ch < 4; ++ch) out[4 * q + ch] = c[ch];
    }
    mip_free(&m);
}

/* The MIP pyramid itself (tests): level k into out (w_k x h_k x 4), returns
 * the number of levels; *w, *h receive level k's size. */
int orc_mip_level(const double *fov, int W, int H, int k, double *out, int *w, int *h) {
    orc_mip m;
    mip_build(&m, fov, W, H);
    int n = m.n;
    if (k >= 0 && k < n) {
        *w = m.w[k];
        *h = m.h[k];
        if (out) memcpy(out, m.lev[k], sizeof(double) * 4 * (size_t)m.w[k] * m.h[k]);
    }
    mip_free(&m);
    return n;
}
