// Per-pair bead double sum shared by the bead kernels and the network
// forces kernel's fallback phase (paper section 2, first equation): a
// wave's LDS staging arrays, the culling and staging of both bodies' beads
// in body i's frame, the branch-free bead-pair sums, the pair geometry from
// the FP64 state, and the per-body outputs of one pair (md_pair).  The work
// mapping is described at the top of bead.hip.
#pragma once

#include "rb_common.hpp"

namespace rb {

constexpr float kCullMargin = 1.0e-3f;

// A wave's LDS: three arrays of `stride` float4 (stride >= the largest
// template), carved from the block's dynamic LDS, so that the occupancy
// follows the templates in use rather than the largest one allowed.
struct WaveLds {
    float4 *j;     // body j's surviving beads (FP32), body i frame
    float4 *jlo;   // their FP32 rounding residuals
    float4 *i;     // body i's surviving beads, body i frame
};

__device__ inline WaveLds wave_lds(float4 *base, int w, int stride) {
    float4 *p = base + (size_t)w * 3 * stride;
    return WaveLds{p, p + stride, p + 2 * stride};
}

// Copies every template into the block's LDS after the waves' arrays (the
// staging loops then read beads from LDS instead of global memory).
__device__ inline const float4 *stage_templates(const Templates &T, float4 *base, int nwaves, int stride) {
    float4 *tb = base + (size_t)nwaves * 3 * stride;
    for (int k = threadIdx.x; k < T.total; k += blockDim.x) tb[k] = T.beads[k];
    __syncthreads();
    return tb;
}

// Separating-axis test (15 axes) between box A, centred at the origin with
// the axes of body i's frame and half extents a, and box B, centred at t with
// axes the columns of R and half extents b.  Returns false when an axis
// separates them.  FP32 with a small widening of the absolute rotation terms;
// the caller grows A by rc plus a margin well above the rounding.
__device__ inline bool boxes_overlap(const float a[3], const float b[3], const float t[3], const float R[9]) {
    float AR[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) AR[k] = fabsf(R[k]) + 1.0e-6f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (fabsf(t[i]) > a[i] + b[0] * AR[3 * i] + b[1] * AR[3 * i + 1] + b[2] * AR[3 * i + 2]) return false;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float tp = t[0] * R[j] + t[1] * R[3 + j] + t[2] * R[6 + j];
        if (fabsf(tp) > a[0] * AR[j] + a[1] * AR[3 + j] + a[2] * AR[6 + j] + b[j]) return false;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const float ra = a[i1] * AR[3 * i2 + j] + a[i2] * AR[3 * i1 + j];
            const float rb = b[j1] * AR[3 * i + j2] + b[j2] * AR[3 * i + j1];
            if (fabsf(t[i2] * R[3 * i1 + j] - t[i1] * R[3 * i2 + j]) > ra + rb) return false;
        }
    }
    return true;
}

// Whether body j (type tj, at d with rotation R in body i's frame) can have
// a bead within rc of a bead of body i (type ti).
__device__ inline bool may_interact(const Templates &T, int ti, int tj, const double d[3], const double R[9],
                                    float rc) {
    const float a[3] = {T.hx[ti] + rc, T.hy[ti] + rc, T.hz[ti] + rc};
    const float b[3] = {T.hx[tj], T.hy[tj], T.hz[tj]};
    const float t[3] = {(float)d[0], (float)d[1], (float)d[2]};
    float Rf[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rf[k] = (float)R[k];
    return boxes_overlap(a, b, t, Rf);
}

__device__ inline float box_dist2(float x, float y, float z, float hx, float hy, float hz) {
    const float ax = fmaxf(fabsf(x) - hx, 0.f), ay = fmaxf(fabsf(y) - hy, 0.f), az = fmaxf(fabsf(z) - hz, 0.f);
    return fmaf(ax, ax, fmaf(ay, ay, az * az));
}

// Appends `v` (and `vlo`) for the lanes with keep set, in lane order, at
// dst[count ...]; returns the new count (wave uniform).
__device__ inline int wave_compact(bool keep, float4 v, float4 vlo, float4 *dst, float4 *dstlo, int count,
                                   int lane) {
    const unsigned long long m = __ballot(keep);
    if (keep) {
        const int pos = count + __popcll(m & ((1ull << lane) - 1ull));
        dst[pos] = v;
        if (dstlo) dstlo[pos] = vlo;
    }
    return count + __popcll(m);
}

// Stages the beads of body j (type tj, at d with rotation R relative to body
// i) that can reach body i's box; r_l = d + R b_l is formed in FP64.
__device__ inline int stage_j(const Templates &T, const float4 *tb, int ti, int tj, const double d[3],
                              const double R[9], float cut2, WaveLds &L, int lane) {
    const int nj = T.n[tj];
    const float4 *bj = tb + T.off[tj];
    const float hx = T.hx[ti], hy = T.hy[ti], hz = T.hz[ti];
    int count = 0;
    for (int l0 = 0; l0 < nj; l0 += kWave) {
        const int l = l0 + lane;
        bool keep = false;
        float4 hi = make_float4(0.f, 0.f, 0.f, 0.f), lo = hi;
        if (l < nj) {
            const float4 b = bj[l];
            const double bx = b.x, by = b.y, bz = b.z;
            const double x = d[0] + R[0] * bx + R[1] * by + R[2] * bz;
            const double y = d[1] + R[3] * bx + R[4] * by + R[5] * bz;
            const double z = d[2] + R[6] * bx + R[7] * by + R[8] * bz;
            hi = make_float4((float)x, (float)y, (float)z, 0.f);
            lo = make_float4((float)(x - hi.x), (float)(y - hi.y), (float)(z - hi.z), 0.f);
            keep = box_dist2(hi.x, hi.y, hi.z, hx, hy, hz) < cut2;
        }
        count = wave_compact(keep, hi, lo, L.j, L.jlo, count, lane);
    }
    return count;
}

// Stages the beads of body i that can reach body j's box: a bead b of i sits
// at R^T (b - d) in body j's frame (FP32 is ample for the test: the margin
// is far above its rounding).
__device__ inline int stage_i(const Templates &T, const float4 *tb, int ti, int tj, const double d[3],
                              const double R[9], float cut2, WaveLds &L, int lane) {
    const int ni = T.n[ti];
    const float4 *bi = tb + T.off[ti];
    const float hx = T.hx[tj], hy = T.hy[tj], hz = T.hz[tj];
    const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
    float Rf[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) Rf[a] = (float)R[a];
    int count = 0;
    for (int k0 = 0; k0 < ni; k0 += kWave) {
        const int k = k0 + lane;
        bool keep = false;
        float4 b = make_float4(0.f, 0.f, 0.f, 0.f);
        if (k < ni) {
            b = bi[k];
            const float ux = b.x - dx, uy = b.y - dy, uz = b.z - dz;
            const float px = Rf[0] * ux + Rf[3] * uy + Rf[6] * uz;
            const float py = Rf[1] * ux + Rf[4] * uy + Rf[7] * uz;
            const float pz = Rf[2] * ux + Rf[5] * uy + Rf[8] * uz;
            keep = box_dist2(px, py, pz, hx, hy, hz) < cut2;
        }
        count = wave_compact(keep, b, b, L.i, nullptr, count, lane);
    }
    return count;
}

// Both stagings in one pass (independent work in flight together): body
// j's beads as stage_j keeps them, body i's as stage_i does.  Outputs the
// counts of both.
__device__ inline void stage_pair(const Templates &T, const float4 *tb, int ti, int tj, const double d[3],
                                  const double R[9], float cut2, WaveLds &L, int lane, int &ni_out, int &nj_out) {
    const int nj = T.n[tj], ni = T.n[ti];
    const float4 *bj = tb + T.off[tj];
    const float4 *bi = tb + T.off[ti];
    const float hxi = T.hx[ti], hyi = T.hy[ti], hzi = T.hz[ti];
    const float hxj = T.hx[tj], hyj = T.hy[tj], hzj = T.hz[tj];
    const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
    float Rf[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) Rf[a] = (float)R[a];
    int cj = 0, ci = 0;
    const int nm = nj > ni ? nj : ni;
    for (int l0 = 0; l0 < nm; l0 += kWave) {
        const int l = l0 + lane;
        bool kj = false, ki = false;
        float4 hi = make_float4(0.f, 0.f, 0.f, 0.f), lo = hi, b = hi;
        if (l < nj) {
            const float4 c = bj[l];
            const double bx = c.x, by = c.y, bz = c.z;
            const double x = d[0] + R[0] * bx + R[1] * by + R[2] * bz;
            const double y = d[1] + R[3] * bx + R[4] * by + R[5] * bz;
            const double z = d[2] + R[6] * bx + R[7] * by + R[8] * bz;
            hi = make_float4((float)x, (float)y, (float)z, 0.f);
            lo = make_float4((float)(x - hi.x), (float)(y - hi.y), (float)(z - hi.z), 0.f);
            kj = box_dist2(hi.x, hi.y, hi.z, hxi, hyi, hzi) < cut2;
        }
        if (l < ni) {
            b = bi[l];
            const float ux = b.x - dx, uy = b.y - dy, uz = b.z - dz;
            const float px = Rf[0] * ux + Rf[3] * uy + Rf[6] * uz;
            const float py = Rf[1] * ux + Rf[4] * uy + Rf[7] * uz;
            const float pz = Rf[2] * ux + Rf[5] * uy + Rf[8] * uz;
            ki = box_dist2(px, py, pz, hxj, hyj, hzj) < cut2;
        }
        cj = wave_compact(kj, hi, lo, L.j, L.jlo, cj, lane);
        ci = wave_compact(ki, b, b, L.i, nullptr, ci, lane);
    }
    ni_out = ci;
    nj_out = cj;
}

// Sums over the wave of eight per-lane values with ten lane exchanges
// instead of 8 x 6: three halving exchanges leave value v summed over eight
// lanes in lanes 8v .. 8v + 7, three more finish it there; every lane
// receives the eight sums.  Fixed order: the result does not depend on
// timing.
__device__ inline void wave_sum8(const float v[8], int lane, float out[8]) {
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0, b3 = (lane & 8) != 0;
    float a[4], c[2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float send = b5 ? v[r] : v[4 + r], keep = b5 ? v[4 + r] : v[r];
        a[r] = keep + __shfl_xor(send, 32, kWave);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const float send = b4 ? a[r] : a[2 + r], keep = b4 ? a[2 + r] : a[r];
        c[r] = keep + __shfl_xor(send, 16, kWave);
    }
    float e;
    {
        const float send = b3 ? c[0] : c[1], keep = b3 ? c[1] : c[0];
        e = keep + __shfl_xor(send, 8, kWave);
    }
    e += __shfl_xor(e, 4, kWave);
    e += __shfl_xor(e, 2, kWave);
    e += __shfl_xor(e, 1, kWave);
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(e), 8 * k));
}

// Energy and -(du/dr)/r of one bead pair at squared distance r2 < rc2.
// Lennard-Jones: from 1/r^2.  Half-power half-cosine, with the attractive
// branch read as -A (1 + cos(c (r - b))) (continuous with zero slope at b
// and at rc = b + pi / c): (b - r)^p - 2A up to b, the cosine well beyond.
template <int POT>
__device__ inline void bead_pot(const LJ &lj, float r2, float &ee, float &fr) {
    if constexpr (POT == kPotLJ) {
        const float ir2 = __builtin_amdgcn_rcpf(r2);
        const float s2 = lj.sig2 * ir2;
        const float s6 = s2 * s2 * s2;
        const float s12 = s6 * s6;
        ee = fmaf(lj.c4e, s12 - s6, -lj.ushift);
        fr = lj.c24e * fmaf(2.f, s12, -s6) * ir2;
    } else {
        const float r = sqrtf(r2);
        const float ir = 1.f / r;
        const float t = fmaxf(lj.b - r, 0.f);
        const float tp1 = powf(t, lj.p - 1.f);
        float sx, cx;
        sincosf(lj.c * (r - lj.b), &sx, &cx);
        const bool core = r <= lj.b;
        ee = core ? fmaf(t, tp1, -2.f * lj.A) : -lj.A * (1.f + cx);
        fr = (core ? lj.p * tp1 : -lj.A * lj.c * sx) * ir;
    }
}

// The ni x nj surviving tests.  Returns, reduced over the wave (valid in
// every lane): r[0] = E, r[1..3] = F_i, r[4..6] = tau_i (body i frame, about
// its centre), r[7] = min squared distance over the tests performed (only
// when TRACK_MIN).
// Lane mapping: body i's beads in blocks of P lanes, the 64 / P lane groups
// of a block splitting body j's beads.  Two choices of blocks, the cheaper
// in iterations per lane taken (a wave-uniform decision): one P for all, the
// smallest power of two not below n_i (at most 64; the last block may have
// idle lanes), or P the largest power of two not above the beads left, so
// that every lane holds a bead (one extra iteration charged per extra
// block).  72 x 72 beads take 72 + 9 iterations instead of 2 x 72, 41 x 41
// take 21 + 6 + 1 instead of 41, 11 x 11 keep one block of 16 (3).
template <bool TRACK_MIN, int POT>
__device__ inline void pair_sum(const LJ &lj, int ni, int nj, const WaveLds &L, int lane, float r[8]) {
    float e = 0.f, r2min = 3.0e38f;
    float F[3] = {0.f, 0.f, 0.f}, t[3] = {0.f, 0.f, 0.f};
    int lgfix = 0;
    while ((1 << lgfix) < ni && lgfix < 6) ++lgfix;
    const int cost_fix = ((ni + (1 << lgfix) - 1) >> lgfix) * ((nj << lgfix) + kWave - 1) / kWave;
    int cost_pow = -1;
    for (int left = ni; left > 0;) {
        const int lg = left >= kWave ? 6 : 31 - __builtin_clz(left);
        cost_pow += 1 + ((nj << lg) + kWave - 1) / kWave;
        left -= 1 << lg;
    }
    const bool greedy = cost_pow < cost_fix;
    for (int kb = 0; kb < ni;) {
        const int left = ni - kb;
        const int lg = greedy ? (left >= kWave ? 6 : 31 - __builtin_clz(left)) : lgfix;
        const int P = 1 << lg, G = kWave >> lg, g = lane >> lg, kk = lane & (P - 1);
        const bool kv = kb + kk < ni;
        const float4 b = kv ? L.i[kb + kk] : make_float4(1.0e4f, 1.0e4f, 1.0e4f, 0.f);
        float fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll 2
        for (int l = g; l < nj; l += G) {
            const float4 p = L.j[l];
            const float4 lo = L.jlo[l];
            const float dx = (b.x - p.x) - lo.x, dy = (b.y - p.y) - lo.y, dz = (b.z - p.z) - lo.z;
            const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            if (TRACK_MIN) r2min = fminf(r2min, r2);
            const bool in = r2 < lj.rc2;
            float ee, fr;
            bead_pot<POT>(lj, r2, ee, fr);
            e += in ? ee : 0.f;
            const float frm = in ? fr : 0.f;
            fx = fmaf(frm, dx, fx);
            fy = fmaf(frm, dy, fy);
            fz = fmaf(frm, dz, fz);
        }
        F[0] += fx; F[1] += fy; F[2] += fz;
        t[0] += b.y * fz - b.z * fy;
        t[1] += b.z * fx - b.x * fz;
        t[2] += b.x * fy - b.y * fx;
        kb += P;
    }
    const float v8[8] = {e, F[0], F[1], F[2], t[0], t[1], t[2], 0.f};
    wave_sum8(v8, lane, r);
    r[7] = TRACK_MIN ? wave_min(r2min) : 0.f;
}

struct Box {
    double L[3], inv[3];
};

// Geometry of pair (i, j) from the FP64 state: dl = minimum-image x_j - x_i
// (lab), d = R_i^T dl and R = R_i^T R_j (from q_i^* q_j).  Shared by the
// screen and the force kernel so that both take the same decisions.
__device__ inline void pair_frame(int32_t n, const double *__restrict__ x, const double *__restrict__ q,
                                  const Box &box, int i, int j, double dl[3], double d[3], double qr[4],
                                  double qa[4], double Ri[9]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) dl[a] = min_image(x[a * n + j] - x[a * n + i], box.L[a], box.inv[a]);
    const double aw = q[i], ax = q[n + i], ay = q[2 * n + i], az = q[3 * n + i];
    const double bw = q[j], bx = q[n + j], by = q[2 * n + j], bz = q[3 * n + j];
    qa[0] = aw;
    qa[1] = ax;
    qa[2] = ay;
    qa[3] = az;
    quat_to_rot<double>(aw, ax, ay, az, Ri);
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = Ri[a] * dl[0] + Ri[3 + a] * dl[1] + Ri[6 + a] * dl[2];
    qr[0] = aw * bw + ax * bx + ay * by + az * bz;
    qr[1] = aw * bx - ax * bw - ay * bz + az * by;
    qr[2] = aw * by + ax * bz - ay * bw - az * bx;
    qr[3] = aw * bz - ax * by + ay * bx - az * bw;
}

__device__ inline void pair_geometry(int32_t n, const double *__restrict__ x, const double *__restrict__ q,
                                     const Box &box, int i, int j, double dl[3], double d[3], double R[9]) {
    double qr[4], qa[4], Ri[9];
    pair_frame(n, x, q, box, i, j, dl, d, qr, qa, Ri);
    quat_to_rot<double>(qr[0], qr[1], qr[2], qr[3], R);
}

// One body pair, whole wave: staging, culling, the bead sum and the
// lab-frame outputs, one component per lane: lanes 0..11 add F and tau of
// both bodies to the accumulator, lanes 12..21 the energy and the 9 virial
// components to the wave's sums.
template <int POT>
__device__ inline void md_pair(const Templates &T, const LJ &lj, const float4 *tb, WaveLds &L, int lane, float cut2,
                               int32_t n, int i, int j, int ti, int tj, const double dl[3], const double d[3],
                               const double R[9], const double Ri[9], int64_t *__restrict__ acc, long long *wacc,
                               long long &ntests, bool &bad, bool &ovf) {
    int ni, nj;
    stage_pair(T, tb, ti, tj, d, R, cut2, L, lane, ni, nj);
    if (ni == 0 || nj == 0) return;   // no bead pair within rc: zero contribution
    wave_lds_sync();
    float r[8];
    pair_sum<false, POT>(lj, ni, nj, L, lane, r);
    ntests += (long long)ni * nj;
    wave_lds_sync();
    if (lane < 22) {
        // per-lane choices by selects, not by indexing (a lane-dependent
        // index into a register array would put the array in scratch memory)
        auto sel3 = [](int k, double x0, double x1, double x2) { return k == 0 ? x0 : (k == 1 ? x1 : x2); };
        const double F[3] = {r[1], r[2], r[3]}, tI[3] = {r[4], r[5], r[6]};
        const double tJ[3] = {d[1] * F[2] - d[2] * F[1] - tI[0], d[2] * F[0] - d[0] * F[2] - tI[1],
                              d[0] * F[1] - d[1] * F[0] - tI[2]};
        if (lane < 12) {
            const int which = lane / 3, a = lane % 3;   // 0: F on i, 1: F on j, 2: tau_i, 3: tau_j
            const double R0 = sel3(a, Ri[0], Ri[3], Ri[6]), R1 = sel3(a, Ri[1], Ri[4], Ri[7]),
                         R2 = sel3(a, Ri[2], Ri[5], Ri[8]);
            const double V0 = which < 2 ? F[0] : (which == 2 ? tI[0] : tJ[0]);
            const double V1 = which < 2 ? F[1] : (which == 2 ? tI[1] : tJ[1]);
            const double V2 = which < 2 ? F[2] : (which == 2 ? tI[2] : tJ[2]);
            double v = R0 * V0 + R1 * V1 + R2 * V2;
            if (which == 1) v = -v;
            const int body = (which == 0 || which == 2) ? i : j;
            acc_add(acc + (int64_t)((which < 2 ? 0 : 3) + a) * n + body, v, ovf);
        } else {
            const int e = lane - 12;
            double v = r[0];
            if (e > 0) {
                const int a = (e - 1) / 3, b = (e - 1) % 3;
                const double Flb = sel3(b, Ri[0], Ri[3], Ri[6]) * F[0] + sel3(b, Ri[1], Ri[4], Ri[7]) * F[1] +
                                   sel3(b, Ri[2], Ri[5], Ri[8]) * F[2];
                v = -sel3(a, dl[0], dl[1], dl[2]) * Flb;
            }
            ovf |= !fix_ok(v);
            wacc[e] += to_fixed(v);
        }
    }
    if (lane == 0 && (!isfinite(r[0]) || !isfinite(r[1]) || !isfinite(r[2]) || !isfinite(r[3]))) bad = true;
}

}  // namespace rb
