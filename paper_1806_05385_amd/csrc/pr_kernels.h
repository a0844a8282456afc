// pr_kernels.h -- device data layouts shared by the kernels and the host
// launcher of libpr (gfx950).
#pragma once

#include <stdint.h>

#include "pr.h"

namespace prk {

// Intersection record of one triangle, written by the bound kernel.
// Rolling views (float4 x 11): for edge k (opposite vertex k) the camera-
// space edge-plane normal c_k(t) = P_a(t) x P_b(t) = A_k + t B_k + t^2 C_k,
// laid out A0 B0 C0 A1 B1 C1 A2 B2 C2 (27 floats); the triple product
// D(t) = P_0(t) . (P_1(t) x P_2(t)) = d0 + t d1 + t^2 d2 + t^3 d3; the face
// normal N(t) = (P_1 - P_0) x (P_2 - P_0) = N0 + t N1 + t^2 N2; the
// triangle index (int bits); 3 pad.  The ray r = (rx, ry, 1) at time t
// passes edge k on the side sign(e_k), e_k = r . c_k(t); the hit depth is
// z = D(t) / (r . N(t)).  N is stored separately although it equals
// sum_k c_k: near grazing incidence r . N is much smaller than the edge
// terms and their sum would lose it to cancellation in FP32.
// Non-rolling views (float4 x 4, t = 0): A0 A1 A2 d0 N0 id pad pad.
constexpr int kRecRoll = 11;
constexpr int kRecStatic = 4;

// Per-triangle bound (64 bytes).
struct TriBound {
    int32_t rect[4];   // inclusive tile rectangle x0, y0, x1, y1 (x0 > x1: culled)
    int32_t kind;      // prg::kCulled / kWindow / kClipped
    int32_t pad;
    double w[4];       // kWindow: time window w[0..1]; kClipped: display box
};

// Per-view constants the later passes read (written by the bound kernel).
struct ViewBlock {
    float light0[3];   // R0 * light direction (camera space at t0)
    float light1[3];   // R1 * light direction
    float pad[2];
};

// Status block at the start of the workspace.
struct DevStatus {
    int32_t overflow;
    int32_t nonfinite;
    unsigned long long pairs_required;
    unsigned long long pairs_total;
    unsigned long long tests;
    unsigned long long hits;
    uint32_t num_pairs[PR_MAX_VIEWS];   // per-view emission cursor
    int32_t view_overflow[PR_MAX_VIEWS];
};

}  // namespace prk
