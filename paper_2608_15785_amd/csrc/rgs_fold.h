// Coefficient folding and per-half-tile culling of one staged list entry
// (Sec. IV-B: Eqs. expand, c0, coeff, dot, dual_pixel), shared by the
// dual-pixel rasterizer and the backward pass of the training variant, so that
// both evaluate every folded exponent with the same instructions.
//
// Coordinates are relative to the centre of the 16x16 tile: pixel (lx, ly)
// sits at (lx - 7.5, ly - 7.5), and the two half-tiles of the two waves of a
// dual-pixel workgroup are the rows [-7.5, -0.5] and [0.5, 7.5].
#pragma once

#include "rgs_internal.h"

namespace rgs {

constexpr float LOG2E_F = 1.4426950408889634f;
constexpr float LOG2_255F = 7.994353436858858f;     // ln 255 * log2 e

// Margin added to the alpha-ellipse half-extents before culling a Gaussian for
// a wave: float32 rounding of the folded exponent near the 1/255 threshold
// must never hide a pair that the exact test would keep.
constexpr float BOX_MARGIN_REL = 1.0e-3f;
constexpr float BOX_MARGIN_ABS = 0.05f;
// The same safety margin on the quadratic form q = A dx^2 + 2 B dx dy + C dy^2
// (P = ln o - q / 2): a band is kept when min q <= tau (1 + 1e-3) + 0.02.
constexpr float Q_MARGIN_REL = 1.0e-3f;
constexpr float Q_MARGIN_ABS = 0.02f;

// Smallest q over the rectangle [-7.5, 7.5] x [y0, y1] (tile-centre
// coordinates) for a Gaussian at (u, v) with a positive-definite conic: 0 when
// the mean is inside, else the least of the four edge minima (on an edge q is
// a parabola in the free coordinate, minimised at a clamped closed form).
__device__ inline float conic_rect_min(float u, float v, float A, float B, float C, float iA, float iC,
                                       float y0, float y1) {
    if (u >= -7.5f && u <= 7.5f && v >= y0 && v <= y1) return 0.0f;
    float best = 3.0e38f;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dx = (e ? 7.5f : -7.5f) - u;                 // vertical edge x = -7.5 or 7.5
        const float dy = fminf(y1, fmaxf(y0, fmaf(-B * dx, iC, v))) - v;
        best = fminf(best, fmaf(A * dx, dx, fmaf(2.0f * B * dx, dy, C * dy * dy)));
        const float ey = (e ? y1 : y0) - v;                       // horizontal edge y = y0 or y1
        const float ex = fminf(7.5f, fmaxf(-7.5f, fmaf(-B * ey, iA, u))) - u;
        best = fminf(best, fmaf(A * ex, ex, fmaf(2.0f * B * ex, ey, C * ey * ey)));
    }
    return best;
}

// One record folded for the tile whose centre is (ox, oy): u, v is its mean in
// tile-centre coordinates, ca = (C1, C2, C3, C4) and cbv = (C5, C6, r, g), so
// that P = C1 x^2 + C2 xy + C3 y^2 + C4 x + C5 y + C6 = ln o + p (the record
// holds ln o in its opacity field).  With LOG2 the coefficients are scaled by
// log2 e, and P log2 e comes out instead (alpha = exp2 of it).
template <bool LOG2>
__device__ inline void fold_record(const Record& rec, float ox, float oy, float& u, float& v, float4& ca,
                                   float4& cbv) {
    u = (rec.u_hi - ox) + rec.u_lo;
    v = (rec.v_hi - oy) + rec.v_lo;
    const float A = rec.A, B = rec.B, C = rec.C;
    const float C0 = fmaf(A * u, u, fmaf(2.0f * B * u, v, C * v * v));
    ca = make_float4(-0.5f * A, -B, -0.5f * C, fmaf(A, u, B * v));
    cbv = make_float4(fmaf(C, v, B * u), fmaf(-0.5f, C0, rec.opa), rec.r, rec.g);
    if (LOG2) {
        ca = make_float4(ca.x * LOG2E_F, ca.y * LOG2E_F, ca.z * LOG2E_F, ca.w * LOG2E_F);
        cbv.x *= LOG2E_F;
        cbv.y *= LOG2E_F;
    }
}

// Whether the record (mean u, v in tile-centre coordinates) can reach a pixel
// of each half-tile with P >= -ln 255.  First the box |x - u| <= hx,
// |y - v| <= hy of its alpha >= 1/255 ellipse (half-extents stored by the front
// end as FP16, rounded up, then widened); then the ellipse itself: the
// half-tile must hold a point with q <= tau = 2 (ln 255 + ln o), up to the
// margin.  Comparisons are phrased so that a NaN keeps the Gaussian.  A culled
// pair would have failed the skip test, so culling changes no result.
__device__ inline void cull_half_tiles(const Record& rec, float u, float v, bool& hit0, bool& hit1) {
    const float A = rec.A, B = rec.B, C = rec.C;
    const float hx = fmaf(half_lo(rec.extra), 1.0f + BOX_MARGIN_REL, BOX_MARGIN_ABS);
    const float hy = fmaf(half_hi(rec.extra), 1.0f + BOX_MARGIN_REL, BOX_MARGIN_ABS);
    const bool x_out = u - hx > 7.5f || u + hx < -7.5f;
    hit0 = !(x_out || v - hy > -0.5f || v + hy < -7.5f);
    hit1 = !(x_out || v - hy > 7.5f || v + hy < 0.5f);
    const float qlim = fmaf(2.0f * (LN255F + rec.opa), 1.0f + Q_MARGIN_REL, Q_MARGIN_ABS);
    // the reciprocals only place the nearest point of an edge, where q is
    // then evaluated exactly; an error of an ulp moves q by ~C (1e-6 px)^2
    const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
    if (hit0) hit0 = !(conic_rect_min(u, v, A, B, C, iA, iC, -7.5f, -0.5f) > qlim);
    if (hit1) hit1 = !(conic_rect_min(u, v, A, B, C, iA, iC, 0.5f, 7.5f) > qlim);
}

// The folded exponents of a dual pixel: P0 at (x, y) by Eq. dot (x2 = x^2,
// xy = x y, y2 = y^2 precomputed), and P1 at (x, y + 1) by Eq. dual_pixel's
// step, P0 + C2 x + C3 (2y + 1) + C5 (y21 = 2y + 1).
__device__ inline void folded_exponents(const float4& a, float c5, float c6, float x, float y, float x2, float xy,
                                        float y2, float y21, float& P0, float& P1) {
    P0 = fmaf(a.x, x2, fmaf(a.y, xy, fmaf(a.z, y2, fmaf(a.w, x, fmaf(c5, y, c6)))));
    P1 = P0 + fmaf(a.y, x, fmaf(a.z, y21, c5));
}

}  // namespace rgs
