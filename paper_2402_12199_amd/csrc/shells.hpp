// Lower bound on the closest bead-centre distance of a body pair from convex
// shells around each body's bead centres: the bead-centre box, a capsule
// along the body's longest axis and the solid cylinder around that axis with
// the capsule's radius and the box's extent (all in the context's templates;
// the last two only for types whose cylinder is narrower than their box).
//
// Arithmetic in FP32 (the bound decides a route, with a safety margin far
// above the rounding).  The separation of two convex sets along any unit axis
// bounds their
// distance from below (separating-axis theorem): for the boxes, the 15
// candidate axes (each box's face normals and the cross products of their
// edge directions, normalised; near-parallel edge pairs give no axis).  For
// the capsules, the distance of their segments minus both radii.  For the
// cylinders, the projected gap along a few directions found by a support-
// point iteration.  The bound is the largest of these.  A pair whose bound
// reaches rc has no bead pair within rc; a pair whose bound reaches the
// network's training minimum lies inside the network's domain.
#pragma once

#include "rb_common.hpp"

namespace rb {

// Routes of a pair by its bound G: the bead sum (G < gap_min), the network
// (gap_min <= G < gap_max) or neither (G >= gap_max).
constexpr int kRouteBead = 0, kRouteNet = 1, kRouteSkip = 2;

// Distance between the segments c1 + s e1 (|s| <= H1) and c2 + t e2
// (|t| <= H2), e1 and e2 unit: the unconstrained optimum of the squared
// distance (a convex quadratic in s, t), s clamped, t optimal for it, and
// s re-optimised when t had to be clamped.  diff: closest point on the
// second segment minus closest point on the first.
__device__ inline float segment_distance(const float c1[3], const float e1[3], float H1, const float c2[3],
                                         const float e2[3], float H2, float diff[3]) {
    float w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = c1[a] - c2[a];
    const float b = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const float dd = e1[0] * w[0] + e1[1] * w[1] + e1[2] * w[2];
    const float e = e2[0] * w[0] + e2[1] * w[1] + e2[2] * w[2];
    const float den = 1.f - b * b;
    // (nearly) parallel: s = 0, and the result is lowered by the most the
    // distance can fall over the segment, H1 sin(angle), so that it stays a
    // lower bound; otherwise a parameter error of the FP32 solve raises the
    // distance only to second order
    const bool par = !(den > 1e-4f);
    float s = par ? 0.f : fminf(fmaxf((b * e - dd) / den, -H1), H1);
    float t = b * s + e;
    if (t < -H2 || t > H2) {
        t = fminf(fmaxf(t, -H2), H2);
        s = fminf(fmaxf(b * t - dd, -H1), H1);
    }
    float r2 = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        diff[a] = -(w[a] + s * e1[a] - t * e2[a]);
        r2 += diff[a] * diff[a];
    }
    return sqrtf(r2) - (par ? H1 * sqrtf(fmaxf(den, 0.f)) : 0.f);
}

// Support point of the solid cylinder (centre c, unit axis a, half-height H,
// radius R) in the unit direction n: the point of the cylinder farthest along
// n (on the rim of the cap facing n; at the cap's centre when n is along the
// axis).
__device__ inline void cyl_support(const float c[3], const float a[3], float H, float R, const float n[3],
                                   float s[3]) {
    const float na = n[0] * a[0] + n[1] * a[1] + n[2] * a[2];
    float p[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = n[k] - na * a[k];
    const float pn2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    const float rs = pn2 > 1e-12f ? R * rsqrtf(pn2) : 0.f;
    const float hs = na >= 0.f ? H : -H;
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = c[k] + hs * a[k] + rs * p[k];
}

// Gap between the projections of cylinders A and B onto the unit direction n
// (a lower bound on their distance for every n), and the difference of the
// two support points (B's nearest to A along n minus A's farthest toward B),
// whose direction is the next trial direction: for the direction between the
// cylinders' closest points the gap equals their distance.
__device__ inline float cyl_gap_along(const float ca[3], const float aa[3], float Ha, float Ra, const float cb[3],
                                      const float ab[3], float Hb, float Rb, const float n[3], float diff[3]) {
    float sa[3], sb[3];
    const float m[3] = {-n[0], -n[1], -n[2]};
    cyl_support(ca, aa, Ha, Ra, n, sa);
    cyl_support(cb, ab, Hb, Rb, m, sb);
#pragma unroll
    for (int k = 0; k < 3; ++k) diff[k] = sb[k] - sa[k];
    return n[0] * diff[0] + n[1] * diff[1] + n[2] * diff[2];
}

// Route of body j (type tj) at d with rotation R (row major, body j's axes
// are the columns) in the frame of body i (type ti), from the bound G (FP32;
// G is lowered by 2e-4 before each comparison, above its rounding -- at most
// ~1e-6 sigma of position over the smallest cross-product axis norm used,
// 0.01 -- so that both decisions stay on the safe side).  The bounds are
// formed from the cheapest up and the pair leaves as soon as one reaches
// gap_max.
//
// gap_exit (>= gap_max): the bound at which the formation stops early;
// keep (may be null) is set to whether the final bound stays below it.  The
// route does not depend on gap_exit (the bound only grows).
__device__ inline int shell_route(const Templates &T, int ti, int tj, const double dd[3], const double Rd[9],
                                  float gap_min, float gap_max, float gap_exit = -1.f, bool *keep = nullptr) {
    if (!(gap_exit >= gap_max)) gap_exit = gap_max;
    if (keep) *keep = false;
    constexpr float kSafe = 2e-4f;
    const float a[3] = {T.hx[ti], T.hy[ti], T.hz[ti]};
    const float b[3] = {T.hx[tj], T.hy[tj], T.hz[tj]};
    const float d[3] = {(float)dd[0], (float)dd[1], (float)dd[2]};
    float R[9], AR[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        R[k] = (float)Rd[k];
        AR[k] = fabsf(R[k]);
    }
    float G = -1e30f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        G = fmaxf(G, fabsf(d[i]) - (a[i] + b[0] * AR[3 * i] + b[1] * AR[3 * i + 1] + b[2] * AR[3 * i + 2]));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float tp = d[0] * R[j] + d[1] * R[3 + j] + d[2] * R[6 + j];
        G = fmaxf(G, fabsf(tp) - (a[0] * AR[j] + a[1] * AR[3 + j] + a[2] * AR[6 + j] + b[j]));
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const float L2 = 1.f - R[3 * i + j] * R[3 * i + j];
            if (L2 > 1e-4f) {
                const float ra = a[i1] * AR[3 * i2 + j] + a[i2] * AR[3 * i1 + j];
                const float rb = b[j1] * AR[3 * i + j2] + b[j2] * AR[3 * i + j1];
                G = fmaxf(G, (fabsf(d[i2] * R[3 * i1 + j] - d[i1] * R[3 * i2 + j]) - (ra + rb)) * rsqrtf(L2));
            }
        }
    }
    if (G - kSafe >= gap_exit) return kRouteSkip;
    if (!T.round[ti] || !T.round[tj]) {
        if (keep) *keep = true;
        return G - kSafe >= gap_max ? kRouteSkip : (G - kSafe < gap_min ? kRouteBead : kRouteNet);
    }
    const int ki = T.cax[ti], kj = T.cax[tj];
    const float c1[3] = {0.f, 0.f, 0.f};
    const float e1[3] = {ki == 0 ? 1.f : 0.f, ki == 1 ? 1.f : 0.f, ki == 2 ? 1.f : 0.f};
    const float e2[3] = {R[kj], R[3 + kj], R[6 + kj]};
    float cp[3];
    G = fmaxf(G, segment_distance(c1, e1, T.cH[ti], d, e2, T.cH[tj], cp) - T.cR[ti] - T.cR[tj]);
    if (G - kSafe >= gap_exit) return kRouteSkip;
    // Cylinders around the same axes (radius that of the capsule, half-height
    // the box's extent along the axis), which hold every bead centre: trial
    // directions from the capsules' closest points and from the centres,
    // each refined by moving to the direction between the current support
    // points, the largest projected gap kept.
    const float Ha = ki == 0 ? a[0] : (ki == 1 ? a[1] : a[2]);
    const float Hb = kj == 0 ? b[0] : (kj == 1 ? b[1] : b[2]);
    const float Ra = T.cR[ti], Rb = T.cR[tj];
    const float dn2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const float cpn2 = cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2];
    for (int start = 0; start < 2; ++start) {
        const bool use_cp = start == 0 && cpn2 > 1e-12f;
        if (!use_cp && !(dn2 > 0.f)) break;
        const float inv = rsqrtf(use_cp ? cpn2 : dn2);
        float n[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) n[k] = (use_cp ? cp[k] : d[k]) * inv;
        for (int it = 0; it < 6; ++it) {
            float diff[3];
            G = fmaxf(G, cyl_gap_along(c1, e1, Ha, Ra, d, e2, Hb, Rb, n, diff));
            if (G - kSafe >= gap_exit) return kRouteSkip;
            const float dd2 = diff[0] * diff[0] + diff[1] * diff[1] + diff[2] * diff[2];
            if (!(dd2 > 1e-20f)) break;
            const float r = rsqrtf(dd2);
#pragma unroll
            for (int k = 0; k < 3; ++k) n[k] = diff[k] * r;
        }
    }
    if (keep) *keep = true;
    return G - kSafe >= gap_max ? kRouteSkip : (G - kSafe < gap_min ? kRouteBead : kRouteNet);
}

}  // namespace rb
