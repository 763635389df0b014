// Lower bound on the closest bead-centre distance of a body pair from convex
// shells around each body's bead centres: the bead-centre box, a capsule
// along the body's longest axis and the solid cylinder around that axis with
// the capsule's radius and the box's extent (all in the context's templates).
//
// The separation of two convex sets along any unit axis bounds their
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

// Distance between the segments c1 + s e1 (|s| <= H1) and c2 + t e2
// (|t| <= H2), e1 and e2 unit: the unconstrained optimum of the squared
// distance (a convex quadratic in s, t), s clamped, t optimal for it, and
// s re-optimised when t had to be clamped.
__device__ inline double segment_distance(const double c1[3], const double e1[3], double H1, const double c2[3],
                                          const double e2[3], double H2, double diff[3]) {
    double w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = c1[a] - c2[a];
    const double b = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const double dd = e1[0] * w[0] + e1[1] * w[1] + e1[2] * w[2];
    const double e = e2[0] * w[0] + e2[1] * w[1] + e2[2] * w[2];
    const double den = 1.0 - b * b;
    double s = den > 1e-12 ? fmin(fmax((b * e - dd) / den, -H1), H1) : 0.0;
    double t = b * s + e;
    if (t < -H2 || t > H2) {
        t = fmin(fmax(t, -H2), H2);
        s = fmin(fmax(b * t - dd, -H1), H1);
    }
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        diff[a] = -(w[a] + s * e1[a] - t * e2[a]);   // closest point on 2 minus closest point on 1
        r2 += diff[a] * diff[a];
    }
    return sqrt(r2);
}

// Support point of the solid cylinder (centre c, unit axis a, half-height H,
// radius R) in the unit direction n: the point of the cylinder farthest along
// n (on the rim of the cap facing n; at the cap's centre when n is along the
// axis).
__device__ inline void cyl_support(const double c[3], const double a[3], double H, double R, const double n[3],
                                   double s[3]) {
    const double na = n[0] * a[0] + n[1] * a[1] + n[2] * a[2];
    double p[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = n[k] - na * a[k];
    const double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    const double rs = pn > 1e-12 ? R / pn : 0.0;
    const double hs = na >= 0.0 ? H : -H;
#pragma unroll
    for (int k = 0; k < 3; ++k) s[k] = c[k] + hs * a[k] + rs * p[k];
}

// Gap between the projections of cylinders A and B onto the unit direction n
// (a lower bound on their distance for every n), and the difference of the
// two support points (B's nearest to A along n minus A's farthest toward B),
// whose direction is the next trial direction: for the direction between the
// cylinders' closest points the gap equals their distance.
__device__ inline double cyl_gap_along(const double ca[3], const double aa[3], double Ha, double Ra,
                                       const double cb[3], const double ab[3], double Hb, double Rb, const double n[3],
                                       double diff[3]) {
    double sa[3], sb[3], m[3] = {-n[0], -n[1], -n[2]};
    cyl_support(ca, aa, Ha, Ra, n, sa);
    cyl_support(cb, ab, Hb, Rb, m, sb);
#pragma unroll
    for (int k = 0; k < 3; ++k) diff[k] = sb[k] - sa[k];
    return n[0] * diff[0] + n[1] * diff[1] + n[2] * diff[2];
}

// Bound for body j (type tj) at d with rotation R (row major, body j's axes
// are the columns) in the frame of body i (type ti).
__device__ inline double shell_gap(const Templates &T, int ti, int tj, const double d[3], const double R[9]) {
    const double a[3] = {T.hx[ti], T.hy[ti], T.hz[ti]};
    const double b[3] = {T.hx[tj], T.hy[tj], T.hz[tj]};
    double AR[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) AR[k] = fabs(R[k]);
    double G = -1e300;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        G = fmax(G, fabs(d[i]) - (a[i] + b[0] * AR[3 * i] + b[1] * AR[3 * i + 1] + b[2] * AR[3 * i + 2]));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double tp = d[0] * R[j] + d[1] * R[3 + j] + d[2] * R[6 + j];
        G = fmax(G, fabs(tp) - (a[0] * AR[j] + a[1] * AR[3 + j] + a[2] * AR[6 + j] + b[j]));
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const double L2 = 1.0 - R[3 * i + j] * R[3 * i + j];
            if (L2 > 1e-12) {
                const double ra = a[i1] * AR[3 * i2 + j] + a[i2] * AR[3 * i1 + j];
                const double rb = b[j1] * AR[3 * i + j2] + b[j2] * AR[3 * i + j1];
                G = fmax(G, (fabs(d[i2] * R[3 * i1 + j] - d[i1] * R[3 * i2 + j]) - (ra + rb)) / sqrt(L2));
            }
        }
    }
    const int ki = T.cax[ti], kj = T.cax[tj];
    const double c1[3] = {0.0, 0.0, 0.0};
    const double e1[3] = {ki == 0 ? 1.0 : 0.0, ki == 1 ? 1.0 : 0.0, ki == 2 ? 1.0 : 0.0};
    const double e2[3] = {R[kj], R[3 + kj], R[6 + kj]};
    double cp[3];
    const double sd = segment_distance(c1, e1, T.cH[ti], d, e2, T.cH[tj], cp);
    G = fmax(G, sd - (double)T.cR[ti] - (double)T.cR[tj]);
    // Cylinders around the same axes (radius that of the capsule, half-height
    // the box's extent along the axis), which hold every bead centre: trial
    // directions from the capsules' closest points and from the centres,
    // each refined by moving to the direction between the current support
    // points, the largest projected gap kept.
    const double Ha = ki == 0 ? a[0] : (ki == 1 ? a[1] : a[2]);
    const double Hb = kj == 0 ? b[0] : (kj == 1 ? b[1] : b[2]);
    const double Ra = T.cR[ti], Rb = T.cR[tj];
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double cpn = sqrt(cp[0] * cp[0] + cp[1] * cp[1] + cp[2] * cp[2]);
#pragma unroll
    for (int start = 0; start < 2; ++start) {
        double n[3];
        const bool use_cp = start == 0 && cpn > 1e-9;
        const double inv = use_cp ? 1.0 / cpn : (dn > 0.0 ? 1.0 / dn : 0.0);
#pragma unroll
        for (int k = 0; k < 3; ++k) n[k] = (use_cp ? cp[k] : d[k]) * inv;
        if (!use_cp && dn == 0.0) break;
        for (int it = 0; it < 6; ++it) {
            double diff[3];
            G = fmax(G, cyl_gap_along(c1, e1, Ha, Ra, d, e2, Hb, Rb, n, diff));
            const double dd = sqrt(diff[0] * diff[0] + diff[1] * diff[1] + diff[2] * diff[2]);
            if (!(dd > 1e-12)) break;
#pragma unroll
            for (int k = 0; k < 3; ++k) n[k] = diff[k] / dd;
        }
    }
    return G;
}

}  // namespace rb
