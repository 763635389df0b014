// Symmetry-reduced descriptor of a pair of identical cubes (paper,
// supplementary section 1) and its Jacobian with respect to the pair
// descriptor u = (d, q).
//
// Body 1's axes are relabelled and their signs chosen (a signed permutation
// g, reflections included) so that body 2's centre p = g d has
// p_x >= p_y >= p_z >= 0; with M = g R(q) g^T, w is body 2's face normal
// with the largest x component, alpha_1 = acos(w_x), alpha_2 =
// atan2(w_z, w_y), and alpha_3 is the angle, modulo pi/2, of Q v in the y-z
// plane, Q the smallest rotation taking w to (1, 0, 0) and v a second face
// normal (Q v = v - (w + e_x) v_x / (1 + w_x) for v perpendicular to w).
// Ties in the sort and in the choice of w go to the lower index.  The
// network takes s = (p_x, p_y, p_z, w_y, w_z, cos 4 alpha_3, sin 4 alpha_3),
// smooth functions of the six numbers (w_y = sin a1 cos a2, w_z =
// sin a1 sin a2) without the polar singularity of (alpha_1, alpha_2) at
// w = (1, 0, 0) and without the cut of alpha_3 between 0 and pi/2.
//
// One thread per pair, FP64.  p is a signed permutation of d, so its rows of
// the Jacobian are those of g; the angles depend on d only through the
// discrete choice of g, and carry forward-mode derivatives with respect to
// the four quaternion components (value and 4 partials per quantity), so
// their Jacobian rows follow the branch the pair takes without a separate
// derivation.
#include "rb_common.hpp"
#include "cyl_form.hpp"

namespace rb {

constexpr int kND = 4;   // derivative slots: the quaternion components

struct Dual {
    double v;
    double d[kND];
};

__device__ inline Dual dconst(double v) {
    Dual r;
    r.v = v;
#pragma unroll
    for (int k = 0; k < kND; ++k) r.d[k] = 0.0;
    return r;
}
__device__ inline Dual dvar(double v, int k) {
    Dual r = dconst(v);
    r.d[k] = 1.0;
    return r;
}
__device__ inline Dual operator+(const Dual &a, const Dual &b) {
    Dual r;
    r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < kND; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
__device__ inline Dual operator-(const Dual &a, const Dual &b) {
    Dual r;
    r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < kND; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
__device__ inline Dual operator*(const Dual &a, const Dual &b) {
    Dual r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < kND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
__device__ inline Dual operator*(double s, const Dual &a) {
    Dual r;
    r.v = s * a.v;
#pragma unroll
    for (int k = 0; k < kND; ++k) r.d[k] = s * a.d[k];
    return r;
}
__device__ inline Dual operator/(const Dual &a, const Dual &b) {
    Dual r;
    r.v = a.v / b.v;
    const double ib = 1.0 / b.v;
#pragma unroll
    for (int k = 0; k < kND; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}
__device__ inline Dual datan2(const Dual &y, const Dual &x) {
    Dual r;
    r.v = atan2(y.v, x.v);
    const double den = 1.0 / fmax(x.v * x.v + y.v * y.v, 1e-300);
#pragma unroll
    for (int k = 0; k < kND; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) * den;
    return r;
}

// One of three duals by index, component by component (a select between the
// objects themselves would take their addresses and move them to scratch).
__device__ inline Dual dsel(int k, const Dual &a, const Dual &b, const Dual &c) {
    Dual r;
    r.v = k == 0 ? a.v : (k == 1 ? b.v : c.v);
#pragma unroll
    for (int m = 0; m < kND; ++m) r.d[m] = k == 0 ? a.d[m] : (k == 1 ? b.d[m] : c.d[m]);
    return r;
}

__device__ void cube_sym(const double u[7], double s[7], double J[7][7]) {
    Dual q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = dvar(u[3 + k], k);
    // R(q), body 2's axes in body 1's frame (columns), as the homogeneous
    // quadratic form v -> q v q^* (equal to the rotation for unit q; off the
    // unit sphere it scales by |q|^2, which fixes the Jacobian's radial
    // column the same way as the quaternion product does)
    const Dual &w = q[0], &x = q[1], &y = q[2], &z = q[3];
    const Dual one = dconst(1.0);
    const Dual ww = w * w, xx = x * x, yy = y * y, zz = z * z;
    Dual R[3][3];
    R[0][0] = ww + xx - yy - zz;
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = ww - xx + yy - zz;
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = ww - xx - yy + zz;
    // signed permutation g (no lane-dependent array indexing: selects only):
    // row r of g picks axis i_r, the axes ordered by decreasing |d|, ties to
    // the lower index, with the sign of that component
    const double a0 = fabs(u[0]), a1 = fabs(u[1]), a2 = fabs(u[2]);
    const int i0 = (a0 >= a1 && a0 >= a2) ? 0 : (a1 >= a2 ? 1 : 2);
    const int j = i0 == 0 ? 1 : 0, l = i0 == 2 ? 1 : 2;        // the other two, j < l
    const double aj = j == 0 ? a0 : a1, al = l == 1 ? a1 : a2;
    const int i1 = aj >= al ? j : l, i2 = aj >= al ? l : j;
    const int ax[3] = {i0, i1, i2};
    double g[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double ur = ax[r] == 0 ? u[0] : (ax[r] == 1 ? u[1] : u[2]);
        const double sr = ur >= 0.0 ? 1.0 : -1.0;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) g[r][cc] = ax[r] == cc ? sr : 0.0;
    }
    // p = g d, M = g R g^T
    double p[3];
    Dual GR[3][3], M[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        p[r] = g[r][0] * u[0] + g[r][1] * u[1] + g[r][2] * u[2];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) GR[r][cc] = g[r][0] * R[0][cc] + g[r][1] * R[1][cc] + g[r][2] * R[2][cc];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) M[r][cc] = g[cc][0] * GR[r][0] + g[cc][1] * GR[r][1] + g[cc][2] * GR[r][2];
    // face normal with the largest x component (column k of M, sign sk) and
    // the next column as the second normal
    int k = 0;
    if (fabs(M[0][1].v) > fabs(M[0][k].v)) k = 1;
    if (fabs(M[0][2].v) > fabs(M[0][k].v)) k = 2;
    const double sk = (k == 0 ? M[0][0].v : (k == 1 ? M[0][1].v : M[0][2].v)) < 0.0 ? -1.0 : 1.0;
    const int k1 = k == 2 ? 0 : k + 1;
    Dual wv[3], vv[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        wv[r] = sk * dsel(k, M[r][0], M[r][1], M[r][2]);
        vv[r] = dsel(k1, M[r][0], M[r][1], M[r][2]);
    }
    const Dual c = vv[0] / (one + wv[0]);
    const Dual beta = datan2(vv[2] - wv[2] * c, vv[1] - wv[1] * c);
    const double c4 = cos(4.0 * beta.v), s4 = sin(4.0 * beta.v);
    s[0] = p[0];
    s[1] = p[1];
    s[2] = p[2];
    s[3] = wv[1].v;
    s[4] = wv[2].v;
    s[5] = c4;
    s[6] = s4;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int m = 0; m < 7; ++m) J[r][m] = m < 3 ? g[r][m] : 0.0;
#pragma unroll
    for (int r = 3; r < 7; ++r)
#pragma unroll
        for (int m = 0; m < 3; ++m) J[r][m] = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        J[3][3 + m] = wv[1].d[m];
        J[4][3 + m] = wv[2].d[m];
        J[5][3 + m] = -4.0 * s4 * beta.d[m];
        J[6][3 + m] = 4.0 * c4 * beta.d[m];
    }
}

// k-th listed pair (pid = idx[k], or k): s to the 7 rows of sym, J to jac
// (49 rows, r * 7 + m), both with row stride max_count.
__global__ __launch_bounds__(256) void k_cube_sym(const float *__restrict__ desc, int64_t stride, const int32_t *__restrict__ idx,
                           const int32_t *__restrict__ count_dev, int64_t n_pairs, int64_t max_count,
                           float *__restrict__ sym, float *__restrict__ jac) {
    int64_t count = n_pairs;
    if (count_dev) {
        const int64_t c = *count_dev;
        count = c < max_count ? c : max_count;
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pid = idx ? idx[k] : k;
        double u[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) u[m] = desc[m * stride + pid];
        double s[7], J[7][7];
        cube_sym(u, s, J);
#pragma unroll
        for (int r = 0; r < 7; ++r) sym[r * max_count + k] = (float)s[r];
#pragma unroll
        for (int r = 0; r < 7; ++r)
#pragma unroll
            for (int m = 0; m < 7; ++m) jac[(r * 7 + m) * max_count + k] = (float)J[r][m];
    }
}

// Cylinder pairs: k-th listed pair's four-number form and its Jacobian,
// same layout as k_cube_sym.
__global__ __launch_bounds__(256) void k_cyl_sym(const float *__restrict__ desc, int64_t stride,
                                                 const int32_t *__restrict__ idx, const int32_t *__restrict__ count_dev,
                                                 int64_t n_pairs, int64_t max_count, float *__restrict__ sym,
                                                 float *__restrict__ jac) {
    int64_t count = n_pairs;
    if (count_dev) {
        const int64_t c = *count_dev;
        count = c < max_count ? c : max_count;
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pid = idx ? idx[k] : k;
        double u[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) u[m] = desc[m * stride + pid];
        double s[7], J[7][7];
        cyl_features(u, s);
        cyl_jacobian(u, J);
#pragma unroll
        for (int r = 0; r < 7; ++r) sym[r * max_count + k] = (float)s[r];
#pragma unroll
        for (int r = 0; r < 7; ++r)
#pragma unroll
            for (int m = 0; m < 7; ++m) jac[(r * 7 + m) * max_count + k] = (float)J[r][m];
    }
}

}  // namespace rb

using namespace rb;

extern "C" int rb_cyl_sym_descriptors(int64_t n_pairs, const float *desc, int64_t stride, const int32_t *idx,
                                      const int32_t *count_dev, int64_t max_count, float *sym, float *jac,
                                      void *stream) {
    RB_REQUIRE(n_pairs >= 0 && max_count >= 0 && stride >= 0, "rb_cyl_sym_descriptors: negative size");
    if ((count_dev ? max_count : n_pairs) == 0) return RB_OK;
    RB_REQUIRE(desc && sym && jac, "rb_cyl_sym_descriptors: null argument");
    RB_REQUIRE(count_dev || n_pairs <= max_count, "rb_cyl_sym_descriptors: n_pairs > max_count");
    const int64_t work = count_dev ? max_count : n_pairs;
    k_cyl_sym<<<grid_for(work, 256, 4096), 256, 0, (hipStream_t)stream>>>(desc, stride, idx, count_dev, n_pairs,
                                                                         max_count, sym, jac);
    RB_LAUNCH_CHECK("rb_cyl_sym_descriptors");
    return RB_OK;
}

extern "C" int rb_cube_sym_descriptors(int64_t n_pairs, const float *desc, int64_t stride, const int32_t *idx,
                                       const int32_t *count_dev, int64_t max_count, float *sym, float *jac,
                                       void *stream) {
    RB_REQUIRE(n_pairs >= 0 && max_count >= 0 && stride >= 0, "rb_cube_sym_descriptors: negative size");
    if ((count_dev ? max_count : n_pairs) == 0) return RB_OK;
    RB_REQUIRE(desc && sym && jac, "rb_cube_sym_descriptors: null argument");
    RB_REQUIRE(count_dev || n_pairs <= max_count, "rb_cube_sym_descriptors: n_pairs > max_count");
    const int64_t work = count_dev ? max_count : n_pairs;
    k_cube_sym<<<grid_for(work, 256, 4096), 256, 0, (hipStream_t)stream>>>(desc, stride, idx, count_dev, n_pairs,
                                                                          max_count, sym, jac);
    RB_LAUNCH_CHECK("rb_cube_sym_descriptors");
    return RB_OK;
}
