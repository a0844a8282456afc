// pr_geom.h -- bound geometry shared by the gfx950 kernels and the host
// test hooks (compiled for both).  Everything here is double precision: it
// runs once per triangle (bound) or once per (triangle, tile) pair (bin),
// where the cost is small next to the per-pixel ray cast, and it must be
// conservative: a pair may only be dropped when the triangle provably covers
// no pixel centre of the tile at that pixel's own time.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pr.h"

#define PRG __host__ __device__ inline

namespace prg {

// Absolute slack (NDC units / frame-time units) added to every bound; far
// above the double rounding of the computations it protects.
constexpr double kSlackNdc = 1e-9;
constexpr double kSlackTime = 1e-6;

struct Geom {
    double R0[9], T0[3], R1[9], T1[3];
    double fx, fy, cx, cy, znear;
    double fov[2], alpha, rad;   // fovea, exponent, normalising radius
    double inv_alpha, inv_rad;   // 1 / alpha, 1 / rad
    double roll[2];
    int W, H;
    bool rolling;
    // tabulated foveation p_c (nc >= 2; otherwise the power law of alpha)
    // and lens distortion p_l (nl >= 2; otherwise none): float samples on
    // normalised distance (pr_profile), attached by attach_profile
    const float *tc, *tl;
    int nc, nl;
    // trend of each table's scale G(s)/s (+1 non-decreasing, -1
    // non-increasing, 0 neither), which decides where the image of a box
    // takes its extremes
    int tc_trend, tl_trend;
};

// fmin / fmax (one instruction each on the device; the bound's values are
// never NaN, and which zero a tie of -0 and +0 returns does not matter)
PRG double dmin(double a, double b) { return fmin(a, b); }
PRG double dmax(double a, double b) { return fmax(a, b); }
PRG double clamp01(double t) { return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t); }

// Rotation matrix of a rotation vector (Rodrigues' formula).
PRG void rodrigues(const float *wf, double R[9]) {
    double w[3] = {wf[0], wf[1], wf[2]};
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double a, b;
    if (th < 1e-8) {
        a = 1.0 - th * th / 6.0;
        b = 0.5 - th * th / 24.0;
    } else {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / (th * th);
    }
    // R = I + a K + b K^2, K = [w]x ; K^2 = w w^T - th^2 I
    double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double k2 = w[r] * w[c] - (r == c ? th * th : 0.0);
            R[3 * r + c] = (r == c ? 1.0 : 0.0) + a * K[3 * r + c] + b * k2;
        }
}

// dR/dw_i of Rodrigues' formula, dR[9 i + 3 r + c] (Gallego & Yezzi,
// "A compact formula for the derivative of a 3-D rotation in exponential
// coordinates", 2015):  dR/dw_i = (w_i [w]x + [w x ((I - R) e_i)]x) R / |w|^2,
// and [e_i]x + ([e_i]x [w]x + [w]x [e_i]x) / 2 for |w| < 1e-6.
PRG void rodrigues_jac(const float *wf, double dR[27]) {
    double w[3] = {wf[0], wf[1], wf[2]};
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double R[9];
    rodrigues(wf, R);
    auto skew = [](const double v[3], double S[9]) {
        S[0] = 0; S[1] = -v[2]; S[2] = v[1];
        S[3] = v[2]; S[4] = 0; S[5] = -v[0];
        S[6] = -v[1]; S[7] = v[0]; S[8] = 0;
    };
    double W[9];
    skew(w, W);
    for (int i = 0; i < 3; ++i) {
        double e[3] = {0, 0, 0};
        e[i] = 1.0;
        double Ei[9];
        skew(e, Ei);
        double *o = dR + 9 * i;
        if (th2 < 1e-12) {
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k) s += Ei[3 * r + k] * W[3 * k + c] + W[3 * r + k] * Ei[3 * k + c];
                    o[3 * r + c] = Ei[3 * r + c] + 0.5 * s;
                }
        } else {
            double u[3] = {e[0] - R[i], e[1] - R[3 + i], e[2] - R[6 + i]};   // (I - R) e_i
            double x[3] = {w[1] * u[2] - w[2] * u[1], w[2] * u[0] - w[0] * u[2], w[0] * u[1] - w[1] * u[0]};
            double X[9], M[9];
            skew(x, X);
            for (int k = 0; k < 9; ++k) M[k] = (w[i] * W[k] + X[k]) / th2;
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k) s += M[3 * r + k] * R[3 * k + c];
                    o[3 * r + c] = s;
                }
        }
    }
}

// Distance from the fovea to the farthest image corner.
PRG double fovea_radius(double f0, double f1) {
    double ex = fabs(f0) + 1.0, ey = fabs(f1) + 1.0;
    return sqrt(ex * ex + ey * ey);
}

PRG void make_geom(const pr_view &v, Geom &g) {
    rodrigues(v.pose0, g.R0);
    rodrigues(v.pose1, g.R1);
    for (int k = 0; k < 3; ++k) {
        g.T0[k] = v.pose0[3 + k];
        g.T1[k] = v.pose1[3 + k];
    }
    g.fx = v.fx; g.fy = v.fy; g.cx = v.cx; g.cy = v.cy; g.znear = v.znear;
    g.fov[0] = v.fovea[0]; g.fov[1] = v.fovea[1];
    g.alpha = v.alpha;
    g.rad = fovea_radius(g.fov[0], g.fov[1]);
    g.inv_alpha = 1.0 / g.alpha;
    g.inv_rad = 1.0 / g.rad;
    g.roll[0] = v.roll_dir[0]; g.roll[1] = v.roll_dir[1];
    g.rolling = (v.roll_dir[0] != 0.0f) || (v.roll_dir[1] != 0.0f);
    g.W = v.width; g.H = v.height;
    g.tc = g.tl = nullptr;
    g.nc = g.nl = 0;
    g.tc_trend = g.tl_trend = 0;
}

// The view's tabulated profiles (samples in memory the caller's side can
// read: host memory for the host hooks, the workspace on the device).
// Trend of the scale G(s)/s of the piecewise-linear profile through the
// samples t[k] = G(k/(n-1)) (G(0) = 0, increasing): on segment k the
// profile is the line a_k + m_k s, so its scale a_k / s + m_k falls where
// the intercept a_k = (k+1) t[k] - k t[k+1] is positive and rises where it
// is negative; the scale is continuous, so it is monotone when all
// intercepts share a sign.  -1: non-increasing (a concave profile), +1:
// non-decreasing (a convex one), 0: neither.
PRG int scale_trend(const float *t, int n) {
    bool down = true, up = true;
    for (int k = 0; k + 1 < n; ++k) {
        const double a = (k + 1.0) * (double)t[k] - (double)k * (double)t[k + 1];
        if (a > 0.0) up = false;
        if (a < 0.0) down = false;
    }
    return down ? -1 : (up ? 1 : 0);
}

// ht / hl: host-readable copies of the samples (the table pointers may be
// device addresses), from which the scale trends are taken.
PRG void attach_profile(Geom &g, const float *tc, int nc, const float *tl, int nl, const float *hc = nullptr,
                        const float *hl = nullptr) {
    g.tc = nc >= 2 ? tc : nullptr;
    g.nc = nc >= 2 ? nc : 0;
    g.tl = nl >= 2 ? tl : nullptr;
    g.nl = nl >= 2 ? nl : 0;
    g.tc_trend = g.nc ? scale_trend(hc ? hc : tc, nc) : 0;
    g.tl_trend = g.nl ? scale_trend(hl ? hl : tl, nl) : 0;
}

// Tabulated radial profile (Sec. 3.1.1 "Domain": p arbitrary and monotone):
// samples tab[k] = G(k / (n-1)) of an increasing function of normalised
// distance, G(0) = 0, linear between samples and continued past the last
// sample with the last segment's slope.  Segment of s:
PRG int prof_seg(int n, double s) {
    const double q = s * (n - 1);
    return q >= (double)(n - 2) ? n - 2 : (q > 0.0 ? (int)q : 0);
}
PRG double prof_eval(const float *tab, int n, double s) {
    const int k = prof_seg(n, s);
    const double a = tab[k], b = tab[k + 1];
    return a + (s * (n - 1) - k) * (b - a);
}
PRG double prof_slope(const float *tab, int n, double s) {
    const int k = prof_seg(n, s);
    return ((double)tab[k + 1] - (double)tab[k]) * (n - 1);
}
// The numeric inverse: the segment whose samples bracket u (binary search
// over the samples), then its linear inverse (exact: the inverse of the
// piecewise-linear profile is piecewise linear through the swapped samples).
PRG double prof_inv(const float *tab, int n, double u) {
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((double)tab[mid] <= u) lo = mid; else hi = mid - 1;
    }
    const double a = tab[lo], b = tab[lo + 1];
    return (lo + (u - a) / (b - a)) / (n - 1);
}

// Radial power map about the fovea: |m(x) - f| = R (|x - f| / R)^e.
// e = alpha: foveated -> display (unfoveate); e = 1/alpha: display ->
// foveated (foveate).
PRG void radial_map(const Geom &g, double e, double x0, double x1, double &o0, double &o1) {
    double d0 = x0 - g.fov[0], d1 = x1 - g.fov[1];
    double rho = sqrt(d0 * d0 + d1 * d1);
    if (rho == 0.0 || e == 1.0) { o0 = x0; o1 = x1; return; }
    // (rho/R)^(e-1); the square-law density (e = 2 or 1/2) avoids pow
    double s = e == 2.0 ? rho * g.inv_rad : (e == 0.5 ? sqrt(g.rad / rho) : pow(rho * g.inv_rad, e - 1.0));
    o0 = g.fov[0] + d0 * s;
    o1 = g.fov[1] + d1 * s;
}

// Exact bounding box of the image of the rectangle [a0,a1] x [b0,b1] under
// a radial map about the fovea, x -> f + (x - f) sigma(|x - f|), whose
// distance map rho sigma(rho) is increasing and whose scale sigma is
// monotone (grows: non-decreasing).  Component k of the map is increasing
// in coordinate k (its derivative sigma + d_k^2 sigma' / rho is at least
// the distance map's slope); in the other coordinate it depends only on
// the distance to the fovea through sigma.  So each extreme sits on the
// matching rectangle side at the point nearest to or farthest from the
// fovea's coordinate.
template <class Map>
PRG void radial_bbox_map(const Geom &g, bool grows, double a0, double a1, double b0, double b1, double out[4],
                         Map &&map) {
    auto nearest = [](double c, double lo, double hi) { return c < lo ? lo : (c > hi ? hi : c); };
    auto farthest = [](double c, double lo, double hi) { return (c - lo) > (hi - c) ? lo : hi; };
    double o0, o1, y;
    // max of component 0: at x = a1
    y = ((a1 - g.fov[0] >= 0) == grows) ? farthest(g.fov[1], b0, b1) : nearest(g.fov[1], b0, b1);
    map(a1, y, o0, o1);
    out[1] = o0;
    // min of component 0: at x = a0
    y = ((a0 - g.fov[0] <= 0) == grows) ? farthest(g.fov[1], b0, b1) : nearest(g.fov[1], b0, b1);
    map(a0, y, o0, o1);
    out[0] = o0;
    // max of component 1: at y = b1
    double x = ((b1 - g.fov[1] >= 0) == grows) ? farthest(g.fov[0], a0, a1) : nearest(g.fov[0], a0, a1);
    map(x, b1, o0, o1);
    out[3] = o1;
    x = ((b0 - g.fov[1] <= 0) == grows) ? farthest(g.fov[0], a0, a1) : nearest(g.fov[0], a0, a1);
    map(x, b0, o0, o1);
    out[2] = o1;
}

// The power law: sigma = (rho/R)^(e-1) grows for e > 1, shrinks for e < 1.
PRG void radial_bbox(const Geom &g, double e, double a0, double a1, double b0, double b1, double out[4]) {
    radial_bbox_map(g, e > 1.0, a0, a1, b0, b1, out,
                    [&](double x0, double x1, double &o0, double &o1) { radial_map(g, e, x0, x1, o0, o1); });
}

// The tabulated radial map: distance rho -> R G(rho / R), G the profile tab
// (its inverse when inv).
PRG void table_map(const Geom &g, const float *tab, int n, bool inv, double x0, double x1, double &o0,
                   double &o1) {
    const double d0 = x0 - g.fov[0], d1 = x1 - g.fov[1];
    const double rho = sqrt(d0 * d0 + d1 * d1);
    if (rho == 0.0) { o0 = x0; o1 = x1; return; }
    const double s = rho * g.inv_rad, sc = (inv ? prof_inv(tab, n, s) : prof_eval(tab, n, s)) / s;
    o0 = g.fov[0] + d0 * sc;
    o1 = g.fov[1] + d1 * sc;
}

// The maps below take a template flag PROF: false compiles only the power
// law without a lens (what a view without a pr_profile uses), so kernels can
// keep that path free of the tabulated paths' registers; true handles both.

// Foveated point -> panel (display) point: display distance R p_c^{-1}(rho/R)
// with a tabulated p_c, else the power law.
template <bool PROF = true>
PRG void unfoveate_pt(const Geom &g, double y0, double y1, double &x0, double &x1) {
    if (!PROF || g.nc < 2) {
        radial_map(g, g.alpha, y0, y1, x0, x1);
        return;
    }
    table_map(g, g.tc, g.nc, true, y0, y1, x0, x1);
}

// Panel point -> undistorted point (Sec. 5.1 "Lens Distortion": p = p_c o p_l
// about the same centre; the undistorted distance is R p_l^{-1}(d/R)); the
// identity without a lens.
template <bool PROF = true>
PRG void undistort_pt(const Geom &g, double x0, double x1, double &u0, double &u1) {
    if (!PROF || g.nl < 2) { u0 = x0; u1 = x1; return; }
    table_map(g, g.tl, g.nl, true, x0, x1, u0, u1);
}

// Box of the image of box b = [b0,b1] x [b2,b3] under the radial map about
// the fovea taking normalised distance s to G(s) (the profile tab, or its
// inverse when inv; G increasing): the image lies in the annular sector of
// radii R G(s_min), R G(s_max) (s_min, s_max the box's nearest and farthest
// points) over the angles the box spans as seen from the fovea, and this is
// the box of that sector (its corners, and its outer arc where it crosses
// an axis direction).  Conservative for any increasing G; a box holding the
// fovea gives the disc of the outer radius.
PRG void sector_box(const Geom &g, const float *tab, int n, bool inv, const double b[4], double out[4]) {
    const double f0 = g.fov[0], f1 = g.fov[1], R = g.rad;
    const double nx = (f0 < b[0] ? b[0] : (f0 > b[1] ? b[1] : f0)) - f0;
    const double ny = (f1 < b[2] ? b[2] : (f1 > b[3] ? b[3] : f1)) - f1;
    const double fx = dmax(fabs(b[0] - f0), fabs(b[1] - f0)), fy = dmax(fabs(b[2] - f1), fabs(b[3] - f1));
    const double s0 = sqrt(nx * nx + ny * ny) * g.inv_rad, s1 = sqrt(fx * fx + fy * fy) * g.inv_rad;
    const double r0 = R * (inv ? prof_inv(tab, n, s0) : prof_eval(tab, n, s0)) * (1.0 - 1e-12);
    const double r1 = R * (inv ? prof_inv(tab, n, s1) : prof_eval(tab, n, s1)) * (1.0 + 1e-12);
    if (s0 == 0.0) {
        out[0] = f0 - r1; out[1] = f0 + r1; out[2] = f1 - r1; out[3] = f1 + r1;
        return;
    }
    // the angles of the corners about the direction of the nearest point
    // (the box does not hold the fovea, so it spans less than a half turn)
    const double c = atan2(ny, nx);
    double lo = 0.0, hi = 0.0;
    for (int k = 0; k < 4; ++k) {
        double a = atan2(b[2 + (k >> 1)] - f1, b[k & 1] - f0) - c;
        if (a > M_PI) a -= 2.0 * M_PI;
        if (a < -M_PI) a += 2.0 * M_PI;
        lo = dmin(lo, a);
        hi = dmax(hi, a);
    }
    lo = c + lo - 1e-12;
    hi = c + hi + 1e-12;
    double o[4] = {1e300, -1e300, 1e300, -1e300};
    auto add = [&](double r, double a) {
        const double x = f0 + r * cos(a), y = f1 + r * sin(a);
        o[0] = dmin(o[0], x); o[1] = dmax(o[1], x);
        o[2] = dmin(o[2], y); o[3] = dmax(o[3], y);
    };
    add(r0, lo); add(r0, hi); add(r1, lo); add(r1, hi);
    for (int k = 0; k < 4; ++k) {   // axis directions inside the span: the outer arc's extreme
        double d = k * 0.5 * M_PI - lo;
        d -= 2.0 * M_PI * floor(d / (2.0 * M_PI));
        if (d <= hi - lo) add(r1, k * 0.5 * M_PI);
    }
    for (int k = 0; k < 4; ++k) out[k] = o[k];
}

// Box of the image of box b under a tabulated radial map (G = tab, or its
// inverse when inv; trend: the trend of tab's scale): exact when the map's
// scale is monotone (the inverse's scale runs the other way), else the
// sector box.
PRG void table_box(const Geom &g, const float *tab, int n, int trend, bool inv, const double b[4], double out[4]) {
    const int t = inv ? -trend : trend;
    if (t == 0) {
        sector_box(g, tab, n, inv, b, out);
        return;
    }
    radial_bbox_map(g, t > 0, b[0], b[1], b[2], b[3], out,
                    [&](double x0, double x1, double &o0, double &o1) { table_map(g, tab, n, inv, x0, x1, o0, o1); });
}

// Panel box of the foveated box b (the pixels' display points).
template <bool PROF = true>
PRG void box_unfoveate(const Geom &g, const double b[4], double out[4]) {
    if (!PROF || g.nc < 2) radial_bbox(g, g.alpha, b[0], b[1], b[2], b[3], out);
    else table_box(g, g.tc, g.nc, g.tc_trend, true, b, out);
}
// Foveated box of the panel box b.
template <bool PROF = true>
PRG void box_foveate(const Geom &g, const double b[4], double out[4]) {
    if (!PROF || g.nc < 2) radial_bbox(g, g.inv_alpha, b[0], b[1], b[2], b[3], out);
    else table_box(g, g.tc, g.nc, g.tc_trend, false, b, out);
}
// Panel box of the undistorted box b (the lens applied); b itself without one.
template <bool PROF = true>
PRG void box_distort(const Geom &g, const double b[4], double out[4]) {
    if (!PROF || g.nl < 2) for (int k = 0; k < 4; ++k) out[k] = b[k];
    else table_box(g, g.tl, g.nl, g.tl_trend, false, b, out);
}
// Undistorted box of the panel box b (the lens inverted).
template <bool PROF = true>
PRG void box_undistort(const Geom &g, const double b[4], double out[4]) {
    if (!PROF || g.nl < 2) for (int k = 0; k < 4; ++k) out[k] = b[k];
    else table_box(g, g.tl, g.nl, g.tl_trend, true, b, out);
}

// Camera-space start / end vertices of triangle f.  Returns false if an
// index is out of range or a vertex is not finite.
PRG bool load_tri(const float *v0, const float *v1, const int32_t *tri, int32_t nv, int32_t f, const Geom &g,
                  double Ps[3][3], double Pe[3][3], int32_t idx[3]) {
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
        int32_t i = tri[3 * (int64_t)f + k];
        if (i < 0 || i >= nv) { i = 0; ok = false; }
        idx[k] = i;
        double a[3] = {v0[3 * (int64_t)i], v0[3 * (int64_t)i + 1], v0[3 * (int64_t)i + 2]};
        double b[3] = {v1[3 * (int64_t)i], v1[3 * (int64_t)i + 1], v1[3 * (int64_t)i + 2]};
        for (int r = 0; r < 3; ++r) {
            Ps[k][r] = g.R0[3 * r] * a[0] + g.R0[3 * r + 1] * a[1] + g.R0[3 * r + 2] * a[2] + g.T0[r];
            Pe[k][r] = g.R1[3 * r] * b[0] + g.R1[3 * r + 1] * b[1] + g.R1[3 * r + 2] * b[2] + g.T1[r];
            ok = ok && isfinite(Ps[k][r]) && isfinite(Pe[k][r]);
        }
    }
    return ok;
}

// Unclamped unit scan time of the projection of camera-space point P,
// multiplied by P.z: N(P) = d . ((fx X + (cx+1) Z)/2, (fy Y + (cy+1) Z)/2).
PRG double scan_numer(const Geom &g, const double P[3]) {
    return 0.5 * (g.roll[0] * (g.fx * P[0] + (g.cx + 1.0) * P[2]) + g.roll[1] * (g.fy * P[1] + (g.cy + 1.0) * P[2]));
}

// Real roots of a t^2 + b t + c in the open interval (0, 1).
PRG int quad_roots01(double a, double b, double c, double r[2]) {
    int n = 0;
    double scale = fabs(a) + fabs(b) + fabs(c);
    if (scale == 0.0) return 0;
    if (fabs(a) <= 1e-14 * scale) {
        if (b != 0.0) {
            double t = -c / b;
            if (t > 0.0 && t < 1.0) r[n++] = t;
        }
        return n;
    }
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) {
        // a (near-)double root: keep the vertex of the parabola as a breakpoint
        if (disc > -1e-12 * b * b) {
            double t = -b / (2.0 * a);
            if (t > 0.0 && t < 1.0) r[n++] = t;
        }
        return n;
    }
    double q = -0.5 * (b + (b >= 0 ? sqrt(disc) : -sqrt(disc)));
    double t1 = q / a;
    double t2 = q != 0.0 ? c / q : t1;
    const bool k1 = t1 > 0.0 && t1 < 1.0, k2 = t2 > 0.0 && t2 < 1.0 && t2 != t1;
    if (k1) r[0] = t1;
    if (k2) {
        if (k1) r[1] = t2;
        else r[0] = t2;
    }
    return (int)k1 + (int)k2;
}

// Compare-exchange and an 8-input sorting network (Batcher's odd-even
// merge sort, 19 comparators): fixed indices keep the array in registers.
PRG void cswap(double &a, double &b) {
    const double lo = dmin(a, b), hi = dmax(a, b);
    a = lo;
    b = hi;
}
PRG void sort8(double v[8]) {
    cswap(v[0], v[1]); cswap(v[2], v[3]); cswap(v[4], v[5]); cswap(v[6], v[7]);
    cswap(v[0], v[2]); cswap(v[1], v[3]); cswap(v[4], v[6]); cswap(v[5], v[7]);
    cswap(v[1], v[2]); cswap(v[5], v[6]);
    cswap(v[0], v[4]); cswap(v[1], v[5]); cswap(v[2], v[6]); cswap(v[3], v[7]);
    cswap(v[2], v[4]); cswap(v[3], v[5]);
    cswap(v[1], v[2]); cswap(v[3], v[4]); cswap(v[5], v[6]);
}

enum { kCulled = 0, kWindow = 1, kClipped = 2 };

// Rolling bound modes (Sec. 4.2): the frame-time window and the display
// region the per-tile test uses.
//  kBoundZenon    the exact window in which the scan catches up with the
//                 moving triangle (Sec. 4.2.4, made exact), hull at its ends
//  kBoundAdaptive the window spanned by the scan times of the six projected
//                 start / end vertices (Sec. 4.2.3), hull at its ends
//  kBoundHull     the whole frame, hull of the six projected vertices
//                 (Sec. 4.2.2)
//  kBoundQuad     the whole frame, bounding box of the six (Sec. 4.2.1)
// Every mode is conservative; the hull is the separating-axis test on the
// edges of the two end triangles (any axis separates validly).
enum { kBoundZenon = 0, kBoundAdaptive = 1, kBoundHull = 2, kBoundQuad = 3 };

// Foveated per-tile tests (an ablation of Sec. 4.1's bounds): kFovExact
// tests in display space against the tile's unfoveated box (the default);
// kFovQuad keeps every tile of the triangle's foveated box (no spatial
// test); kFovSimple / kFovRecursive test in foveated space against support
// lines of the foveated triangle whose normals are those of the display-
// space edges (Simple) or of the chords between the edges' foveated end
// points (Recursive).
enum { kFovExact = 0, kFovQuad = 1, kFovSimple = 2, kFovRecursive = 3 };

// The time window of a triangle seen through a lens (kWindow or kCulled).
PRG int lens_window(const Geom &g, const double Ps[3][3], const double Pe[3][3], double win[2]) {
    // Through a lens the scan is no straight line of the projected
    // (undistorted) image, so the catch-up analysis does not apply.  A
    // pixel at time t in the window [w0, w1] sees the triangle inside
    // the hull of its projected vertices at w0 and w1 (linear motion in
    // front of the eye), whose box's panel image bounds the pixel's
    // panel point, whose scan time bounds t: so t also lies in that
    // panel box's scan-time range (clamped to the frame, as pixel times
    // are).  Starting from the whole frame, the window is narrowed
    // three times that way.
    double w0 = 0.0, w1 = 1.0;
    for (int it = 0; it < 3; ++it) {
        double ub[4] = {1e300, -1e300, 1e300, -1e300};
        for (int k = 0; k < 6; ++k) {
            const double t = k < 3 ? w0 : w1;
            const double *A = Ps[k % 3], *B = Pe[k % 3];
            double P[3];
            for (int r = 0; r < 3; ++r) P[r] = (1.0 - t) * A[r] + t * B[r];
            const double x = g.fx * P[0] / P[2] + g.cx, y = g.fy * P[1] / P[2] + g.cy;
            ub[0] = dmin(ub[0], x); ub[1] = dmax(ub[1], x);
            ub[2] = dmin(ub[2], y); ub[3] = dmax(ub[3], y);
        }
        for (int k = 0; k < 4; ++k) ub[k] += ((k & 1) ? 1.0 : -1.0) * kSlackNdc * (1.0 + fabs(ub[k]));
        double pb[4];
        box_distort(g, ub, pb);
        double lo = 1e300, hi = -1e300;
        for (int c = 0; c < 4; ++c) {
            const double u = 0.5 * (g.roll[0] * (pb[c & 1] + 1.0) + g.roll[1] * (pb[2 + (c >> 1)] + 1.0));
            lo = dmin(lo, u);
            hi = dmax(hi, u);
        }
        w0 = dmax(w0, clamp01(lo - kSlackTime));
        w1 = dmin(w1, clamp01(hi + kSlackTime));
        if (w0 > w1) return kCulled;
    }
    win[0] = w0;
    win[1] = w1;
    return kWindow;
}

// Frame-time window in which the triangle can affect a pixel.
//  kCulled : never (every space-time vertex behind the near plane, or the
//            rolling scan never meets the triangle).
//  kWindow : every vertex stays at Z >= znear through the frame; win is the
//            exact set of times at which the scan line (the iso-time line of
//            the display) crosses the projected triangle, padded.
//  kClipped: the near plane cuts the space-time triangle; win is the whole
//            frame (or [0,0] without rolling).
// Without rolling every pixel is at t = 0, so win = [0, 0].
//
// Catch-up test (the scan "catching up" with a moving vertex): vertex k
// projects to display time u_k(t) = N_k(t) / Z_k(t) with N_k, Z_k linear in
// t, so u_k(t) - t has the sign of the quadratic h_k(t) = N_k(t) - t Z_k(t).
// The scan at time t meets the triangle only if min_k h_k(t) <= 0 <=
// max_k h_k(t) (the projected triangle's scan-time range contains t); at
// t = 0 pixels with u <= 0 count, at t = 1 pixels with u >= 1.  Between the
// roots of the h_k no sign changes, so testing each root and each gap's
// midpoint gives the window exactly.
template <bool PROF = true>
PRG int time_window(const Geom &g, const double Ps[3][3], const double Pe[3][3], double win[2],
                    int mode = kBoundZenon) {
    int n_in = 0, n_pts = g.rolling ? 6 : 3;
    for (int k = 0; k < 3; ++k) {
        n_in += Ps[k][2] >= g.znear;
        if (g.rolling) n_in += Pe[k][2] >= g.znear;
    }
    if (n_in == 0) return kCulled;
    if (n_in < n_pts) {
        win[0] = 0.0;
        win[1] = g.rolling ? 1.0 : 0.0;
        return kClipped;
    }
    if (!g.rolling) {
        win[0] = win[1] = 0.0;
        return kWindow;
    }
    if (mode == kBoundHull || mode == kBoundQuad) {
        win[0] = 0.0;
        win[1] = 1.0;
        return kWindow;
    }
    if (PROF && g.nl >= 2) return lens_window(g, Ps, Pe, win);
    if (mode == kBoundAdaptive) {
        // every covered display point lies in the hull of the six projected
        // vertices, and its (unclamped) scan time is linear in the point:
        // its frame time lies between the vertices' extreme scan times
        double lo = 1e300, hi = -1e300;
        for (int k = 0; k < 3; ++k) {
            const double a = scan_numer(g, Ps[k]) / Ps[k][2], b = scan_numer(g, Pe[k]) / Pe[k][2];
            lo = dmin(lo, dmin(a, b));
            hi = dmax(hi, dmax(a, b));
        }
        win[0] = clamp01(lo - kSlackTime);
        win[1] = clamp01(hi + kSlackTime);
        return kWindow;
    }
    double hc[3][3];  // h_k = hc[k][0] + hc[k][1] t + hc[k][2] t^2
    // breakpoints: 0, 1 and each quadratic's roots in (0, 1), sorted; an
    // unused slot holds 2 (past the frame), sorts last and is skipped
    double bp[8] = {0.0, 1.0, 2.0, 2.0, 2.0, 2.0, 2.0, 2.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double n0 = scan_numer(g, Ps[k]);
        double n1 = scan_numer(g, Pe[k]) - n0;
        double z0 = Ps[k][2], z1 = Pe[k][2] - Ps[k][2];
        hc[k][0] = n0;
        hc[k][1] = n1 - z0;
        hc[k][2] = -z1;
        double r[2] = {2.0, 2.0};
        quad_roots01(hc[k][2], hc[k][1], hc[k][0], r);
        bp[2 + 2 * k] = r[0];
        bp[3 + 2 * k] = r[1];
    }
    sort8(bp);
    double lo = 2.0, hi = -1.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        // the breakpoint itself
        double t = bp[i];
        if (t > 1.0) continue;
        double hmin = 1e300, hmax = -1e300;
        for (int k = 0; k < 3; ++k) {
            double h = hc[k][0] + t * (hc[k][1] + t * hc[k][2]);
            hmin = dmin(hmin, h);
            hmax = dmax(hmax, h);
        }
        bool rel;
        if (t == 0.0) rel = hmin <= 0.0;
        else if (t == 1.0) rel = hmax >= 0.0;
        else rel = hmin <= 0.0 && hmax >= 0.0;
        if (rel) { lo = dmin(lo, t); hi = dmax(hi, t); }
        // the gap to the next breakpoint
        if (i + 1 < 8 && bp[i + 1] <= 1.0 && bp[i + 1] > t) {
            double m = 0.5 * (t + bp[i + 1]);
            hmin = 1e300; hmax = -1e300;
            for (int k = 0; k < 3; ++k) {
                double h = hc[k][0] + m * (hc[k][1] + m * hc[k][2]);
                hmin = dmin(hmin, h);
                hmax = dmax(hmax, h);
            }
            if (hmin <= 0.0 && hmax >= 0.0) { lo = dmin(lo, t); hi = dmax(hi, bp[i + 1]); }
        }
    }
    if (lo > hi) return kCulled;
    win[0] = clamp01(lo - kSlackTime);
    win[1] = clamp01(hi + kSlackTime);
    return kWindow;
}

// Display-space (NDC) box of the triangle over [w0, w1].  kWindow: the box
// of the six projected vertices at the window ends (linear motion keeps the
// triangle inside the hull of its end positions, and projection of the
// segments in front of the eye keeps that hull's image inside the hull of
// the projected ends).  kClipped: the box of the projected part of the
// space-time hull in front of the near plane: the end points at Z >= znear
// and every end-point segment's crossing of Z = znear.
PRG void display_box(const Geom &g, const double Ps[3][3], const double Pe[3][3], double w0, double w1,
                     int kind, double box[4]) {
    double pts[6][3];
    int n = (w1 > w0) ? 6 : 3;
    for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 3; ++r) {
            pts[k][r] = (1.0 - w0) * Ps[k][r] + w0 * Pe[k][r];
            pts[3 + k][r] = (1.0 - w1) * Ps[k][r] + w1 * Pe[k][r];
        }
    box[0] = box[2] = 1e300;
    box[1] = box[3] = -1e300;
    auto add = [&](const double *P) {
        const double iz = 1.0 / P[2];
        double x = g.fx * P[0] * iz + g.cx, y = g.fy * P[1] * iz + g.cy;
        box[0] = dmin(box[0], x); box[1] = dmax(box[1], x);
        box[2] = dmin(box[2], y); box[3] = dmax(box[3], y);
    };
    // fixed trip counts (guarded by n) keep pts in registers
    if (kind == kWindow) {
#pragma unroll
        for (int i = 0; i < 6; ++i)
            if (i < n) add(pts[i]);
    } else {
#pragma unroll
        for (int i = 0; i < 6; ++i)
            if (i < n && pts[i][2] >= g.znear) add(pts[i]);
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j) {
                if (j >= n) continue;
                bool ii = pts[i][2] >= g.znear, jj = pts[j][2] >= g.znear;
                if (ii == jj) continue;
                double s = (g.znear - pts[i][2]) / (pts[j][2] - pts[i][2]);
                double q[3];
                for (int r = 0; r < 3; ++r) q[r] = pts[i][r] + s * (pts[j][r] - pts[i][r]);
                q[2] = g.znear;
                add(q);
            }
    }
    for (int k = 0; k < 4; ++k) {
        double m = kSlackNdc * (1.0 + fabs(box[k]));
        box[k] += (k & 1) ? m : -m;
    }
}

// Range of pixel indices whose centre coordinate lies in [lo, hi] for an
// axis with n pixels; returns false if none.  flip: row axis (NDC y up).
PRG bool pixel_range(double lo, double hi, int n, bool flip, int &i0, int &i1) {
    double a, b;
    if (!flip) { a = (lo + 1.0) * 0.5 * n - 0.5; b = (hi + 1.0) * 0.5 * n - 0.5; }
    else { a = (1.0 - hi) * 0.5 * n - 0.5; b = (1.0 - lo) * 0.5 * n - 0.5; }
    a = dmax(a, 0.0);
    b = dmin(b, (double)(n - 1));
    if (!(a <= b)) return false;
    i0 = (int)ceil(a - 1e-7);
    i1 = (int)floor(b + 1e-7);
    if (i0 < 0) i0 = 0;
    if (i1 > n - 1) i1 = n - 1;
    return i0 <= i1;
}

// Tile rectangle (inclusive tile coordinates) of a display box (of projected
// points; through a lens first mapped to the panel).  The box is clipped to
// the display square (every pixel's display point lies in it: the power law
// and a tabulated p_c with p_c(s) >= s never move a pixel outwards), mapped
// to the foveated domain (the exact box rule of the power law, the sector
// box of a table), and converted to the pixel centres it contains.  Returns
// false if it covers no pixel centre.
template <bool PROF = true>
PRG bool tile_rect(const Geom &g, const double box[4], int tile, int rect[4]) {
    double pb[4];
    box_distort<PROF>(g, box, pb);   // through a lens: the box's panel image
    double a0 = dmax(pb[0], -1.0), a1 = dmin(pb[1], 1.0);
    double b0 = dmax(pb[2], -1.0), b1 = dmin(pb[3], 1.0);
    if (!(a0 <= a1 && b0 <= b1)) return false;
    double fb[4];
    const double cb[4] = {a0, a1, b0, b1};
    box_foveate<PROF>(g, cb, fb);
    for (int k = 0; k < 4; ++k) {
        double m = kSlackNdc * (1.0 + fabs(fb[k]));
        fb[k] += (k & 1) ? m : -m;
    }
    int i0, i1, j0, j1;
    if (!pixel_range(fb[0], fb[1], g.W, false, i0, i1)) return false;
    if (!pixel_range(fb[2], fb[3], g.H, true, j0, j1)) return false;
    if ((tile & (tile - 1)) == 0) {   // power of two (every supported size): shifts
        const int sh = __builtin_ctz((unsigned)tile);
        rect[0] = i0 >> sh; rect[1] = j0 >> sh; rect[2] = i1 >> sh; rect[3] = j1 >> sh;
    } else {
        rect[0] = i0 / tile; rect[1] = j0 / tile; rect[2] = i1 / tile; rect[3] = j1 / tile;
    }
    return true;
}

// Display-space box of the pixel centres of columns [i0, i1] x rows [j0, j1]
// (clipped to the image; false if that leaves no pixel): box holds their
// rays' (undistorted) points, pbox (if given) their panel points, which set
// their times.  Without a lens the two are the same.
template <bool PROF = true>
PRG bool region_display(const Geom &g, int i0, int i1, int j0, int j1, double box[4], double *pbox = nullptr) {
    if (i1 > g.W - 1) i1 = g.W - 1;
    if (j1 > g.H - 1) j1 = g.H - 1;
    if (i0 > i1 || j0 > j1) return false;
    double a0 = 2.0 * (i0 + 0.5) / g.W - 1.0, a1 = 2.0 * (i1 + 0.5) / g.W - 1.0;
    double b0 = 1.0 - 2.0 * (j1 + 0.5) / g.H, b1 = 1.0 - 2.0 * (j0 + 0.5) / g.H;
    const double fb[4] = {a0, a1, b0, b1};
    double pb[4];
    box_unfoveate<PROF>(g, fb, pb);
    for (int k = 0; k < 4; ++k) {
        double m = kSlackNdc * (1.0 + fabs(pb[k]));
        pb[k] += (k & 1) ? m : -m;
    }
    if (pbox)
        for (int k = 0; k < 4; ++k) pbox[k] = pb[k];
    if (!PROF || g.nl < 2) {
        for (int k = 0; k < 4; ++k) box[k] = pb[k];
        return true;
    }
    box_undistort<PROF>(g, pb, box);
    for (int k = 0; k < 4; ++k) {
        double m = kSlackNdc * (1.0 + fabs(box[k]));
        box[k] += (k & 1) ? m : -m;
    }
    return true;
}

// Frame-time window of the panel points in a box.
PRG void tile_time(const Geom &g, const double box[4], double tw[2]) {
    if (!g.rolling) { tw[0] = tw[1] = 0.0; return; }
    double umin = 1e300, umax = -1e300;
    for (int c = 0; c < 4; ++c) {
        double x = box[c & 1], y = box[2 + (c >> 1)];
        double u = 0.5 * (g.roll[0] * (x + 1.0) + g.roll[1] * (y + 1.0));
        umin = dmin(umin, u);
        umax = dmax(umax, u);
    }
    tw[0] = clamp01(umin - kSlackTime);
    tw[1] = clamp01(umax + kSlackTime);
}

// Display box of a tile's pixel centres and its frame-time window.
template <bool PROF = true>
PRG void tile_display(const Geom &g, int tile, int tx, int ty, double box[4], double tw[2]) {
    double pb[4];
    region_display<PROF>(g, tx * tile, tx * tile + tile - 1, ty * tile, ty * tile + tile - 1, box, pb);
    tile_time(g, pb, tw);
}

// Quadrant k = qx + 2 qy of a tile: the (tile/2)^2 pixels at column offset
// qx * tile/2 and row offset qy * tile/2.  Display box of its pixel centres
// (and of their panel points in pbox, if given); false if the quadrant lies
// outside the image.
template <bool PROF = true>
PRG bool quad_display(const Geom &g, int tile, int tx, int ty, int k, double box[4], double *pbox = nullptr) {
    const int h = tile / 2;
    const int i0 = tx * tile + (k & 1) * h, j0 = ty * tile + (k >> 1) * h;
    return region_display<PROF>(g, i0, i0 + h - 1, j0, j0 + h - 1, box, pbox);
}

// FP32 bounds of x rounded outwards (the stored tile boxes and test
// records): x's nearest float moved out by 2^-22 of its magnitude and by
// 1e-30.  The conversion is off by at most 2^-24 of the magnitude and the
// move's own rounding by as much again, so the bound is on the right side of
// x with a margin (the 1e-30 covers floats near zero).  Magnitudes beyond
// 3e38 are taken as 3e38 (the callers clamp their bounds to 1e30 or hold
// values far smaller).
PRG float f32_down(double x) {
    const float f = (float)dmin(dmax(x, -3e38), 3e38);
    return fmaf(-fabsf(f), 2.384185791015625e-7f, f) - 1e-30f;
}
PRG float f32_up(double x) {
    const float f = (float)dmin(dmax(x, -3e38), 3e38);
    return fmaf(fabsf(f), 2.384185791015625e-7f, f) + 1e-30f;
}
// The triangle's image over its whole time window as the per-tile test
// sees it, built once per triangle: the projected window-end vertices'
// x and y extents and six edge axes of the two end triangles, each
// interval computed in FP64 for the FP32-rounded axis and rounded outwards
// to FP32 (any axis direction gives a valid separating-axis test).
// kClipped triangles: their display box as extents, no edge axes.  128 B.
struct SatRec {
    float ext[4];      // x lo, x hi, y lo, y hi
    float win[2];      // time window (kClipped: [0, 1])
    int32_t kind;
    int32_t pad;
    float ax[6][4];    // axis n0, n1 and the interval lo, hi
};

PRG float f32_clamp(float x) { return fminf(fmaxf(x, -1e30f), 1e30f); }

PRG void sat_build(const Geom &g, const double Ps[3][3], const double Pe[3][3], int kind, const double w[4],
                   SatRec &R, int mode = kBoundZenon) {
    R.kind = kind;
    R.pad = 0;
    if (kind == kWindow && mode == kBoundQuad) {
        // the box alone: the display box of the window ends, no edge axes
        double box[4];
        display_box(g, Ps, Pe, w[0], w[1], kind, box);
        R.ext[0] = f32_clamp(f32_down(box[0])); R.ext[1] = f32_clamp(f32_up(box[1]));
        R.ext[2] = f32_clamp(f32_down(box[2])); R.ext[3] = f32_clamp(f32_up(box[3]));
        R.win[0] = f32_down(w[0]);
        R.win[1] = f32_up(w[1]);
        for (int a = 0; a < 6; ++a) { R.ax[a][0] = R.ax[a][1] = 0.0f; R.ax[a][2] = -1.0f; R.ax[a][3] = 1.0f; }
        return;
    }
    if (kind != kWindow) {
        R.ext[0] = f32_down(w[0]); R.ext[1] = f32_up(w[1]);
        R.ext[2] = f32_down(w[2]); R.ext[3] = f32_up(w[3]);
        R.win[0] = 0.0f; R.win[1] = 1.0f;
        for (int a = 0; a < 6; ++a) { R.ax[a][0] = R.ax[a][1] = 0.0f; R.ax[a][2] = -1.0f; R.ax[a][3] = 1.0f; }
        return;
    }
    const double w0 = w[0], w1 = w[1];
    R.win[0] = f32_down(w0);
    R.win[1] = f32_up(w1);
    double q[6][2];
    for (int k = 0; k < 3; ++k)
        for (int e = 0; e < 2; ++e) {
            const double t = e ? w1 : w0;
            double P[3];
            for (int r = 0; r < 3; ++r) P[r] = (1.0 - t) * Ps[k][r] + t * Pe[k][r];
            const double iz = 1.0 / P[2];
            q[3 * e + k][0] = g.fx * P[0] * iz + g.cx;
            q[3 * e + k][1] = g.fy * P[1] * iz + g.cy;
        }
    double big = 1.0;
    for (int i = 0; i < 6; ++i) big = dmax(big, dmax(fabs(q[i][0]), fabs(q[i][1])));
    double ext[4] = {1e300, -1e300, 1e300, -1e300};
    for (int i = 0; i < 6; ++i) {
        ext[0] = dmin(ext[0], q[i][0]); ext[1] = dmax(ext[1], q[i][0]);
        ext[2] = dmin(ext[2], q[i][1]); ext[3] = dmax(ext[3], q[i][1]);
    }
    const double mxy = 1e-12 * big;
    R.ext[0] = f32_clamp(f32_down(ext[0] - mxy)); R.ext[1] = f32_clamp(f32_up(ext[1] + mxy));
    R.ext[2] = f32_clamp(f32_down(ext[2] - mxy)); R.ext[3] = f32_clamp(f32_up(ext[3] + mxy));
    for (int a = 0; a < 6; ++a) {
        const int e = a / 3, k = a % 3;
        const double *p = q[3 * e + k], *r = q[3 * e + (k + 1) % 3];
        const float n0 = (float)(-(r[1] - p[1])), n1 = (float)(r[0] - p[0]);
        double lo = 1e300, hi = -1e300;
        for (int i = 0; i < 6; ++i) {
            const double sp = (double)n0 * q[i][0] + (double)n1 * q[i][1];
            lo = dmin(lo, sp);
            hi = dmax(hi, sp);
        }
        const double m = 1e-12 * (fabs((double)n0) + fabs((double)n1)) * big;
        R.ax[a][0] = n0;
        R.ax[a][1] = n1;
        R.ax[a][2] = f32_clamp(f32_down(lo - m));
        R.ax[a][3] = f32_clamp(f32_up(hi + m));
    }
}

// Panel point -> foveated point (the inverse of unfoveate_pt), and
// undistorted point -> panel point (the lens applied; the identity without
// one).
template <bool PROF = true>
PRG void foveate_pt(const Geom &g, double x0, double x1, double &y0, double &y1) {
    if (!PROF || g.nc < 2) radial_map(g, g.inv_alpha, x0, x1, y0, y1);
    else table_map(g, g.tc, g.nc, false, x0, x1, y0, y1);
}
template <bool PROF = true>
PRG void distort_pt(const Geom &g, double u0, double u1, double &x0, double &x1) {
    if (!PROF || g.nl < 2) { x0 = u0; x1 = u1; return; }
    table_map(g, g.tl, g.nl, false, u0, u1, x0, x1);
}

// Pieces per hull edge of the foveated record's boundary sampling.
constexpr int kFovPieces = 8;

// The per-tile test record in foveated space (kFovSimple, kFovRecursive).
// The space-time triangle's display points over its window lie in the hull
// H of its six projected window-end vertices; the foveated image of H is
// bounded by the image of H's boundary.  Each hull edge is cut into
// kFovPieces pieces whose boxes (padded by 1e-12 of the coordinates' scale,
// which covers the hull's rounding) are carried to foveated space as exact
// image boxes (lens, then foveation): every corner of those boxes together
// bounds the image, so the box of the corners and, for any direction, the
// range of the corners' projections are conservative.  The directions: the
// normals of the six window-end edges (Simple) or of the chords between
// their foveated end points (Recursive).  A triangle the near plane cuts
// keeps the foveated box of its display box alone.
template <bool PROF = true>
PRG void sat_build_fov(const Geom &g, const double Ps[3][3], const double Pe[3][3], int kind, const double w[4],
                       SatRec &R, int fov) {
    R.kind = kind;
    R.pad = 0;
    for (int a = 0; a < 6; ++a) { R.ax[a][0] = R.ax[a][1] = 0.0f; R.ax[a][2] = -1.0f; R.ax[a][3] = 1.0f; }
    if (kind != kWindow) {
        double pb[4], fb[4];
        box_distort<PROF>(g, w, pb);
        box_foveate<PROF>(g, pb, fb);
        R.ext[0] = f32_clamp(f32_down(fb[0])); R.ext[1] = f32_clamp(f32_up(fb[1]));
        R.ext[2] = f32_clamp(f32_down(fb[2])); R.ext[3] = f32_clamp(f32_up(fb[3]));
        R.win[0] = 0.0f; R.win[1] = 1.0f;
        return;
    }
    const double w0 = w[0], w1 = w[1];
    R.win[0] = f32_down(w0);
    R.win[1] = f32_up(w1);
    double q[6][2];
    for (int k = 0; k < 3; ++k)
        for (int e = 0; e < 2; ++e) {
            const double t = e ? w1 : w0;
            double P[3];
            for (int r = 0; r < 3; ++r) P[r] = (1.0 - t) * Ps[k][r] + t * Pe[k][r];
            const double iz = 1.0 / P[2];
            q[3 * e + k][0] = g.fx * P[0] * iz + g.cx;
            q[3 * e + k][1] = g.fy * P[1] * iz + g.cy;
        }
    // the six axes
    double n[6][2];
    for (int a = 0; a < 6; ++a) {
        const int e = a / 3, k = a % 3;
        const double *p = q[3 * e + k], *r = q[3 * e + (k + 1) % 3];
        if (fov == kFovRecursive) {
            double u0, u1, v0, v1, fp0, fp1, fr0, fr1;
            distort_pt<PROF>(g, p[0], p[1], u0, u1);
            foveate_pt<PROF>(g, u0, u1, fp0, fp1);
            distort_pt<PROF>(g, r[0], r[1], v0, v1);
            foveate_pt<PROF>(g, v0, v1, fr0, fr1);
            n[a][0] = -(fr1 - fp1);
            n[a][1] = fr0 - fp0;
        } else {
            n[a][0] = -(r[1] - p[1]);
            n[a][1] = r[0] - p[0];
        }
        const double l = fabs(n[a][0]) + fabs(n[a][1]);
        if (!(l > 0.0)) { n[a][0] = 1.0; n[a][1] = 0.0; }   // a degenerate edge: any direction bounds
        else { n[a][0] /= l; n[a][1] /= l; }
        n[a][0] = (double)(float)n[a][0];   // the stored (FP32) direction
        n[a][1] = (double)(float)n[a][1];
    }
    // the hull of the six points (monotone chain over the points sorted by
    // x, then y; collinear points dropped): h[0..m)
    int o[6] = {0, 1, 2, 3, 4, 5};
    for (int i = 1; i < 6; ++i)
        for (int j = i; j > 0 && (q[o[j]][0] < q[o[j - 1]][0] ||
                                  (q[o[j]][0] == q[o[j - 1]][0] && q[o[j]][1] < q[o[j - 1]][1])); --j) {
            const int tmp = o[j]; o[j] = o[j - 1]; o[j - 1] = tmp;
        }
    auto cross = [&](int a, int b, int c) {
        return (q[b][0] - q[a][0]) * (q[c][1] - q[a][1]) - (q[b][1] - q[a][1]) * (q[c][0] - q[a][0]);
    };
    int h[12], m = 0;
    for (int i = 0; i < 6; ++i) {   // lower hull
        while (m >= 2 && cross(h[m - 2], h[m - 1], o[i]) <= 0.0) --m;
        h[m++] = o[i];
    }
    for (int i = 4, m0 = m + 1; i >= 0; --i) {   // upper hull
        while (m >= m0 && cross(h[m - 2], h[m - 1], o[i]) <= 0.0) --m;
        h[m++] = o[i];
    }
    if (m > 1) --m;   // the last point repeats the first
    double scale = 1.0;
    for (int i = 0; i < 6; ++i) scale = dmax(scale, dmax(fabs(q[i][0]), fabs(q[i][1])));
    const double pad = 1e-12 * scale;
    double ext[4] = {1e300, -1e300, 1e300, -1e300}, lo[6], hi[6];
    for (int a = 0; a < 6; ++a) { lo[a] = 1e300; hi[a] = -1e300; }
    for (int i = 0; i < m; ++i) {
        const double *P0 = q[h[i]], *P1 = q[h[(i + 1) % m]];
        for (int c = 0; c < kFovPieces; ++c) {
            const double s0 = (double)c / kFovPieces, s1 = (double)(c + 1) / kFovPieces;
            const double x0 = P0[0] + s0 * (P1[0] - P0[0]), x1 = P0[0] + s1 * (P1[0] - P0[0]);
            const double y0 = P0[1] + s0 * (P1[1] - P0[1]), y1 = P0[1] + s1 * (P1[1] - P0[1]);
            const double b[4] = {dmin(x0, x1) - pad, dmax(x0, x1) + pad, dmin(y0, y1) - pad, dmax(y0, y1) + pad};
            double pb[4], fb[4];
            box_distort<PROF>(g, b, pb);
            box_foveate<PROF>(g, pb, fb);
            ext[0] = dmin(ext[0], fb[0]); ext[1] = dmax(ext[1], fb[1]);
            ext[2] = dmin(ext[2], fb[2]); ext[3] = dmax(ext[3], fb[3]);
            for (int a = 0; a < 6; ++a) {
                const double cx0 = n[a][0] * fb[0], cx1 = n[a][0] * fb[1];
                const double cy0 = n[a][1] * fb[2], cy1 = n[a][1] * fb[3];
                lo[a] = dmin(lo[a], dmin(cx0, cx1) + dmin(cy0, cy1));
                hi[a] = dmax(hi[a], dmax(cx0, cx1) + dmax(cy0, cy1));
            }
        }
    }
    double big = 1.0;
    for (int k = 0; k < 4; ++k) big = dmax(big, fabs(ext[k]));
    const double mxy = 1e-12 * big;
    R.ext[0] = f32_clamp(f32_down(ext[0] - mxy)); R.ext[1] = f32_clamp(f32_up(ext[1] + mxy));
    R.ext[2] = f32_clamp(f32_down(ext[2] - mxy)); R.ext[3] = f32_clamp(f32_up(ext[3] + mxy));
    for (int a = 0; a < 6; ++a) {
        const double m = 1e-12 * (fabs(n[a][0]) + fabs(n[a][1])) * big;
        R.ax[a][0] = (float)n[a][0];
        R.ax[a][1] = (float)n[a][1];
        R.ax[a][2] = f32_clamp(f32_down(lo[a] - m));
        R.ax[a][3] = f32_clamp(f32_up(hi[a] + m));
    }
}

// Pixel-centre box in foveated NDC of pixels [i0, i1] x [j0, j1] (clipped to
// the image; false if empty), widened by kSlackNdc.
PRG bool region_foveated(const Geom &g, int i0, int i1, int j0, int j1, double box[4]) {
    if (i1 > g.W - 1) i1 = g.W - 1;
    if (j1 > g.H - 1) j1 = g.H - 1;
    if (i0 > i1 || j0 > j1) return false;
    box[0] = 2.0 * (i0 + 0.5) / g.W - 1.0;
    box[1] = 2.0 * (i1 + 0.5) / g.W - 1.0;
    box[2] = 1.0 - 2.0 * (j1 + 0.5) / g.H;
    box[3] = 1.0 - 2.0 * (j0 + 0.5) / g.H;
    for (int k = 0; k < 4; ++k) box[k] += ((k & 1) ? 1.0 : -1.0) * kSlackNdc * (1.0 + fabs(box[k]));
    return true;
}

// A tile's foveated box and its quadrants' (outward-rounded FP32; qvalid:
// the quadrants inside the image), for the foveated-space tests.
PRG void tile_foveated(const Geom &g, int tile, int tx, int ty, float tb[4], float qb[4][4], int &qvalid) {
    double b[4];
    region_foveated(g, tx * tile, tx * tile + tile - 1, ty * tile, ty * tile + tile - 1, b);
    tb[0] = f32_down(b[0]); tb[1] = f32_up(b[1]); tb[2] = f32_down(b[2]); tb[3] = f32_up(b[3]);
    qvalid = 0;
    const int h = tile / 2;
    for (int k = 0; k < 4; ++k) {
        const int i0 = tx * tile + (k & 1) * h, j0 = ty * tile + (k >> 1) * h;
        double c[4];
        const bool ok = region_foveated(g, i0, i0 + h - 1, j0, j0 + h - 1, c);
        qvalid |= ok ? 1 << k : 0;
        qb[k][0] = ok ? f32_down(c[0]) : 0.0f; qb[k][1] = ok ? f32_up(c[1]) : 0.0f;
        qb[k][2] = ok ? f32_down(c[2]) : 0.0f; qb[k][3] = ok ? f32_up(c[3]) : 0.0f;
    }
}

PRG bool fbox_meets(const float a[4], const float b[4]) {
    return !(a[1] < b[0] || a[0] > b[1] || a[3] < b[2] || a[2] > b[3]);
}

// Per-tile test in FP32 against a tile's display box tb and time window tw
// (outward-rounded FP32).  Returns the 4-bit mask of the quadrants (boxes
// qb[k] with bit k of qvalid) the triangle may cover; 0 rejects the pair;
// qb == nullptr: no split (0xF when kept).  The box's projection on an axis
// is rounded at most twice in FP32 (2^-23 relative); the test widens it by
// 1e-6 of its magnitude.
PRG int sat_mask(const SatRec &R, const float tb[4], const float tw[2], const float (*qb)[4], int qvalid) {
    if (R.win[1] < tw[0] || R.win[0] > tw[1]) return 0;
    if (!fbox_meets(R.ext, tb)) return 0;
    const float B = fmaxf(1.0f, fmaxf(fmaxf(fabsf(tb[0]), fabsf(tb[1])), fmaxf(fabsf(tb[2]), fabsf(tb[3]))));
    for (int a = 0; a < 6; ++a) {
        const float n0 = R.ax[a][0], n1 = R.ax[a][1];
        const float bmin = fmaf(n0, n0 >= 0.0f ? tb[0] : tb[1], n1 * (n1 >= 0.0f ? tb[2] : tb[3]));
        const float bmax = fmaf(n0, n0 >= 0.0f ? tb[1] : tb[0], n1 * (n1 >= 0.0f ? tb[3] : tb[2]));
        const float m = 1e-6f * (fabsf(n0) + fabsf(n1)) * B;
        if (R.ax[a][3] < bmin - m || R.ax[a][2] > bmax + m) return 0;
    }
    if (!qb) return 0xF;
    int mask = 0;
    for (int k = 0; k < 4; ++k)
        if (((qvalid >> k) & 1) && fbox_meets(R.ext, qb[k])) mask |= 1 << k;
    return mask;
}

// Tiles of 16 pixels and more are split into quadrants.
PRG bool split_quads(int tile) { return tile >= 16; }

// The same from the tile's coordinates (host tests), with the tile boxes
// and window built and rounded as the device builds them: a split tile's
// box is the union of its quadrants' boxes.
PRG int tile_mask(const Geom &g, const double Ps[3][3], const double Pe[3][3], int kind, const double w[4],
                  int tile, int tx, int ty, int mode = kBoundZenon, int fov = kFovExact) {
    double tb[4], tw[2], qb[4][4];
    int qvalid = 0;
    if (!split_quads(tile)) {
        tile_display(g, tile, tx, ty, tb, tw);
    } else {
        double pb[4] = {1e300, -1e300, 1e300, -1e300};
        tb[0] = tb[2] = 1e300;
        tb[1] = tb[3] = -1e300;
        for (int k = 0; k < 4; ++k) {
            double qp[4];
            if (quad_display(g, tile, tx, ty, k, qb[k], qp)) {
                qvalid |= 1 << k;
                tb[0] = dmin(tb[0], qb[k][0]); tb[1] = dmax(tb[1], qb[k][1]);
                tb[2] = dmin(tb[2], qb[k][2]); tb[3] = dmax(tb[3], qb[k][3]);
                pb[0] = dmin(pb[0], qp[0]); pb[1] = dmax(pb[1], qp[1]);
                pb[2] = dmin(pb[2], qp[2]); pb[3] = dmax(pb[3], qp[3]);
            }
        }
        tile_time(g, pb, tw);
    }
    float ftb[4] = {f32_down(tb[0]), f32_up(tb[1]), f32_down(tb[2]), f32_up(tb[3])};
    float ftw[2] = {f32_down(tw[0]), f32_up(tw[1])};
    float fqb[4][4];
    for (int k = 0; k < 4; ++k) {
        const bool ok = (qvalid >> k) & 1;
        fqb[k][0] = ok ? f32_down(qb[k][0]) : 0.0f; fqb[k][1] = ok ? f32_up(qb[k][1]) : 0.0f;
        fqb[k][2] = ok ? f32_down(qb[k][2]) : 0.0f; fqb[k][3] = ok ? f32_up(qb[k][3]) : 0.0f;
    }
    SatRec R;
    sat_build(g, Ps, Pe, kind, w, R, mode);
    if (fov == kFovQuad) {   // the time window alone
        if (R.win[1] < ftw[0] || R.win[0] > ftw[1]) return 0;
        return split_quads(tile) ? qvalid : 0xF;
    }
    if (fov == kFovSimple || fov == kFovRecursive) {
        SatRec F;
        sat_build_fov(g, Ps, Pe, kind, w, F, fov);
        F.win[0] = R.win[0];
        F.win[1] = R.win[1];
        int fq;
        tile_foveated(g, tile, tx, ty, ftb, fqb, fq);
        return sat_mask(F, ftb, ftw, split_quads(tile) ? fqb : nullptr, fq);
    }
    return sat_mask(R, ftb, ftw, split_quads(tile) ? fqb : nullptr, qvalid);
}

}  // namespace prg
