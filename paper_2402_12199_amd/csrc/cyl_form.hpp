// Four-number descriptor of a pair of identical cylinders (paper section 2:
// thanks to the cylindrical symmetry a cylinder pair depends on four numbers;
// supplementary section 2: body 1's axis is the frame's z axis, oriented so
// that p_z >= 0, the x axis chosen so that p_y = 0, and body 2's axis in
// spherical angles (theta, phi)).
//
// The network takes the four numbers through smooth functions that are also
// unchanged when body 2 is turned end over end (a -> -a) and under the
// mirror y -> -y of that frame:
//   s = (p_r^2, p_z^2, a_z^2, (p_r a_x)^2, p_r a_x a_z p_z, 0, 0),
// which in the pair descriptor u = (d, q) are polynomials: with
// A = q e_z q^* = (2(xz + wy), 2(yz - wx), w^2 - x^2 - y^2 + z^2) (body 2's
// axis, homogeneous in q) and t = d_x A_x + d_y A_y,
//   s = (d_x^2 + d_y^2, d_z^2, A_z^2, t^2, t A_z d_z, 0, 0),
// smooth where the frame choice is not (p_r = 0, p_z = 0).  The Jacobian is
// written out from these polynomials.  Templated on the arithmetic type: the
// network kernels take FP32 (their inputs are FP32), the descriptor kernel
// FP64.
#pragma once

#include "rb_common.hpp"

namespace rb {

template <typename Real>
__device__ inline void cyl_features(const Real u[7], Real s[7]) {
    const Real dx = u[0], dy = u[1], dz = u[2], w = u[3], x = u[4], y = u[5], z = u[6];
    const Real Ax = 2 * (x * z + w * y), Ay = 2 * (y * z - w * x), Az = w * w - x * x - y * y + z * z;
    const Real t = dx * Ax + dy * Ay;
    s[0] = dx * dx + dy * dy;
    s[1] = dz * dz;
    s[2] = Az * Az;
    s[3] = t * t;
    s[4] = t * Az * dz;
    s[5] = 0;
    s[6] = 0;
}

// J[r][m] = d s_r / d u_m (rows 5, 6 are zero).
template <typename Real>
__device__ inline void cyl_jacobian(const Real u[7], Real J[7][7]) {
    const Real dx = u[0], dy = u[1], dz = u[2], w = u[3], x = u[4], y = u[5], z = u[6];
    const Real Ax = 2 * (x * z + w * y), Ay = 2 * (y * z - w * x), Az = w * w - x * x - y * y + z * z;
    const Real t = dx * Ax + dy * Ay;
    // d A / d (w, x, y, z)
    const Real dAx[4] = {2 * y, 2 * z, 2 * w, 2 * x};
    const Real dAy[4] = {-2 * x, -2 * w, 2 * z, 2 * y};
    const Real dAz[4] = {2 * w, -2 * x, -2 * y, 2 * z};
    Real dt[7];
    dt[0] = Ax;
    dt[1] = Ay;
    dt[2] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) dt[3 + k] = dx * dAx[k] + dy * dAy[k];
#pragma unroll
    for (int r = 0; r < 7; ++r)
#pragma unroll
        for (int m = 0; m < 7; ++m) J[r][m] = 0;
    J[0][0] = 2 * dx;
    J[0][1] = 2 * dy;
    J[1][2] = 2 * dz;
#pragma unroll
    for (int k = 0; k < 4; ++k) J[2][3 + k] = 2 * Az * dAz[k];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        J[3][m] = 2 * t * dt[m];
        J[4][m] = Az * dz * dt[m];
    }
    J[4][2] += t * Az;
#pragma unroll
    for (int k = 0; k < 4; ++k) J[4][3 + k] += t * dz * dAz[k];
}

}  // namespace rb
