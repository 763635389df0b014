// Bead double sum between composite rigid bodies (paper section 2, first
// equation: the body-body energy is the sum of the bead potential over all
// N_i x N_j bead pairs), with the workloads' bead potential, Lennard-Jones
// 12-6 shifted in energy at rc.
//
// Work mapping (gfx950, wave64): one wavefront per body pair, evaluated in
// body i's frame, where body i's beads are its template.
//  0. A separating-axis test between body j's bead box and body i's bead box
//     grown by rc skips pairs that cannot have a bead pair within rc (most
//     pairs of a list built with a skin) before any bead is touched.
//  1. Body j's beads are rotated into body i's frame in FP64 and kept when
//     they lie within rc of body i's bead box (the box that holds every bead
//     centre of i); survivors go to LDS, compacted with a ballot, as an FP32
//     value plus its FP32 rounding residual.
//  2. Body i's beads are kept when they lie within rc of body j's bead box;
//     survivors go to LDS.  A bead outside these boxes has no partner within
//     rc, so the culling drops no interacting bead pair.
//  3. The surviving ni x nj distance tests are spread over the 64 lanes:
//     lanes form groups of P >= ni (a power of two) that each hold one of
//     body i's beads, and the 64/P groups stride through body j's beads, so
//     every LDS read is a broadcast to a group.  The tests are branch free:
//     every lane evaluates the LJ term and keeps it when r < rc.
//  4. Per-bead forces stay in registers; E, F_i and tau_i are reduced across
//     the wave with lane shuffles, and body j's force and torque follow from
//     pair identities (central bead forces): F_j = -F_i and
//     tau_j = d x F_i - tau_i.
#include "rb_common.hpp"
#include "shells.hpp"

namespace rb {

constexpr int kBeadWaves = 4;        // waves per block (per-pair form)
constexpr int kMdWaves = 8;          // waves per block (per-body form: one work queue per block)
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

// The ni x nj surviving tests.  Returns, reduced over the wave (valid in
// every lane): r[0] = E, r[1..3] = F_i, r[4..6] = tau_i (body i frame, about
// its centre), r[7] = min squared distance over the tests performed (only
// when TRACK_MIN).
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

template <bool TRACK_MIN, int POT>
__device__ inline void pair_sum(const LJ &lj, int ni, int nj, const WaveLds &L, int lane, float r[8]) {
    int P = 1;
    while (P < ni && P < kWave) P <<= 1;
    const int G = kWave / P, g = lane / P, kk = lane % P;
    float e = 0.f, r2min = 3.0e38f;
    float F[3] = {0.f, 0.f, 0.f}, t[3] = {0.f, 0.f, 0.f};
    for (int kb = 0; kb < ni; kb += P) {
        const int k = kb + kk;
        const bool kv = k < ni;
        const float4 b = kv ? L.i[k] : make_float4(1.0e4f, 1.0e4f, 1.0e4f, 0.f);
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
    }
    const float v8[8] = {e, F[0], F[1], F[2], t[0], t[1], t[2], 0.f};
    wave_sum8(v8, lane, r);
    r[7] = TRACK_MIN ? wave_min(r2min) : 0.f;
}

// Per-pair form: descriptors in, per-pair outputs in body i's frame out.
// r_min is exact when some bead pair is closer than rc; otherwise the value
// reported is at least rc (culled bead pairs are all farther than rc).
template <int POT>
__global__ __launch_bounds__(256) void k_bead_desc(Templates T, LJ lj, int ti, int tj, int64_t P,
                                                   const float *__restrict__ desc, float *__restrict__ out,
                                                   int32_t *__restrict__ flags, int stride) {
    extern __shared__ float4 bead_lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    WaveLds L = wave_lds(bead_lds, w, stride);
    const float4 *tb = stage_templates(T, bead_lds, kBeadWaves, stride);
    const float rcm = sqrtf(lj.rc2) + kCullMargin, cut2 = rcm * rcm;
    long long ntests = 0;
    const int64_t step = (int64_t)gridDim.x * kBeadWaves;
    for (int64_t p = (int64_t)blockIdx.x * kBeadWaves + w; p < P; p += step) {
        double d[3] = {desc[p], desc[P + p], desc[2 * P + p]};
        double qw = desc[3 * P + p], qx = desc[4 * P + p], qy = desc[5 * P + p], qz = desc[6 * P + p];
        const double inv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        double R[9];
        quat_to_rot<double>(qw * inv, qx * inv, qy * inv, qz * inv, R);
        const int nj = may_interact(T, ti, tj, d, R, rcm) ? stage_j(T, tb, ti, tj, d, R, cut2, L, lane) : 0;
        const int ni = nj ? stage_i(T, tb, ti, tj, d, R, cut2, L, lane) : 0;
        wave_lds_sync();
        float r[8];
        pair_sum<true, POT>(lj, ni, nj, L, lane, r);
        ntests += (long long)ni * nj;
        wave_lds_sync();
        if (lane == 0) {
            const float Fx = r[1], Fy = r[2], Fz = r[3];
            const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
            out[p] = r[0];
            out[1 * P + p] = -Fx; out[2 * P + p] = -Fy; out[3 * P + p] = -Fz;
            out[4 * P + p] = r[4]; out[5 * P + p] = r[5]; out[6 * P + p] = r[6];
            out[7 * P + p] = (dy * Fz - dz * Fy) - r[4];
            out[8 * P + p] = (dz * Fx - dx * Fz) - r[5];
            out[9 * P + p] = (dx * Fy - dy * Fx) - r[6];
            out[10 * P + p] = ni * nj ? fminf(sqrtf(r[7]), sqrtf(lj.rc2)) : sqrtf(lj.rc2);
        }
    }
    long long part[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, ntests};
    __shared__ long long tred[kBeadWaves];
    if (lane == 0) tred[w] = part[10];
    __syncthreads();
    if (flags && threadIdx.x == 0) {
        long long t = 0;
        for (int k = 0; k < kBeadWaves; ++k) t += tred[k];
        if (t) atomicAdd(reinterpret_cast<unsigned long long *>(flags + RB_FLAG_NTESTS), (unsigned long long)t);
    }
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

// Screen: one thread per listed pair; keeps the pairs whose shells' bound on
// the closest bead distance is below rc (the others have exactly zero bead
// energy, force and torque) and appends them to idx_out with one atomic per wave.  tmp[0]
// (append counter) and tmp[1] (finishing ticket) are zero on entry and left
// zero; the last workgroup publishes the count.  The screened-out pairs are
// counted as evaluated (their contribution is known to be zero).
__global__ __launch_bounds__(256) void k_bead_screen(Templates T, float rcm, int32_t n, const double *__restrict__ x,
                                                     const double *__restrict__ q, const int32_t *__restrict__ type,
                                                     Box box, const int32_t *__restrict__ pi,
                                                     const int32_t *__restrict__ pj, const int32_t *__restrict__ idx,
                                                     const int32_t *__restrict__ count_dev, int32_t max_count,
                                                     int32_t *__restrict__ idx_out, int32_t *__restrict__ count_out,
                                                     int32_t *__restrict__ tmp, int32_t *__restrict__ flags) {
    __shared__ bool last;
    int count = *count_dev;
    if (count > max_count) count = max_count;
    // the grid is sized for the capacity: only the blocks that own pairs take
    // part (and take a finishing ticket)
    const int nb = min((int)gridDim.x, (count + (int)blockDim.x - 1) / (int)blockDim.x);
    if (count == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *count_out = 0;
        return;
    }
    if ((int)blockIdx.x >= nb) return;
    const int lane = threadIdx.x & (kWave - 1);
    for (int base = blockIdx.x * blockDim.x; base < count; base += gridDim.x * blockDim.x) {
        const int p = base + threadIdx.x;
        bool keep = false;
        int pid = 0;
        if (p < count) {
            pid = idx ? idx[p] : p;
            const int i = pi[pid], j = pj[pid];
            double dl[3], d[3], R[9];
            pair_geometry(n, x, q, box, i, j, dl, d, R);
            keep = shell_route(T, type[i], type[j], d, R, 0.f, rcm) != kRouteSkip;
        }
        const unsigned long long m = __ballot(keep);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            int at = 0;
            if (lane == leader) at = atomicAdd(tmp, __popcll(m));
            at = __shfl(at, leader, kWave);
            if (keep) idx_out[at + __popcll(m & ((1ull << lane) - 1ull))] = pid;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(tmp + 1, 1) == nb - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        const int kept = __hip_atomic_load(tmp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *count_out = kept;
        if (flags) atomicAdd(flags + RB_FLAG_NEVAL, count - kept);
        tmp[0] = 0;
        tmp[1] = 0;
    }
}

// Per-body form for dynamics.  A block takes the pairs b, b + G, b + 2G, ...
// (G blocks) in rounds of 64, one lane of the first wave per pair: indices,
// FP64 geometry and the separating-axis test run for the round at once (one
// round of memory latency); the pairs that can interact go, with their
// geometry, to an LDS queue from which the block's waves take them one at a
// time, each evaluated by a whole wave.  Two queues alternate, so that the
// first wave screens the next round while the block drains the current one
// (and the first round while the other waves copy the templates).  The
// pair's outputs are rotated to the lab frame and added to the fixed-point
// accumulator.
//
// Two-level form (SCREENED): the list of body pairs (built with a skin on
// the centre distance) is screened once more with the separating-axis test
// widened by a margin m; a listed pair outside that screened list has no
// bead pair within rc for as long as no body has moved by more than m / 2
// (a bead moves by at most |dx| + 2 rho sin(theta / 2) for a body
// displacement dx and rotation theta, rho the body's largest bead radius),
// which the integrator watches, raising the rescreen flag.  A launch with
// the flag set runs the form above over the whole list and rebuilds the
// screened list (pairs that pass the plain test first, those that pass only
// the widened one from the end of the array) and the reference state; a
// launch with the flag clear runs the same rounds over the screened list
// only, whose pairs that passed the plain test are dealt out evenly over
// the blocks.  This pays where the list spans several rounds per block
// (large systems); with one round per block the two forms cost the same.
constexpr int kRound = 64;

struct PairQueue {
    int i[kRound], j[kRound], ti[kRound], tj[kRound];
    double dl[3][kRound], d[3][kRound], qr[4][kRound], qa[4][kRound];
    int n, head;
};

struct ScreenArgs {
    int32_t *list;          // screened pair indices (capacity max_count)
    double *x_ref, *q_ref;  // state at the last screening (3 x n, 4 x n)
    int32_t *tmp;           // [0], [1]: append counters, [2]: ticket (zero between launches), [3]: pairs of the list that passed the plain test
    float rcm_wide;         // rc + cull margin + screening margin
};

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

// Wave-aggregated append of the lanes with `keep` at list[base + rank]
// (forward) or list[end - 1 - (base + rank)] (backward), base from counter.
__device__ inline void list_append(bool keep, int value, int32_t *counter, int32_t *list, int end, bool backward,
                                   int lane) {
    const unsigned long long m = __ballot(keep);
    if (!m) return;
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader, kWave);
    if (keep) {
        const int at = base + __popcll(m & ((1ull << lane) - 1ull));
        list[backward ? end - 1 - at : at] = value;
    }
}

// at least four waves per SIMD (two 8-wave blocks per CU, which the LDS
// allows for templates of up to ~150 beads)
template <int POT, bool SCREENED>
__global__ __launch_bounds__(kMdWaves * kWave) __attribute__((amdgpu_waves_per_eu(4))) void k_bead_md(Templates T, LJ lj, int32_t n, const double *__restrict__ x,
                                                 const double *__restrict__ q, const int32_t *__restrict__ type,
                                                 Box box, const int32_t *__restrict__ pi,
                                                 const int32_t *__restrict__ pj, const int32_t *__restrict__ idx,
                                                 const int32_t *__restrict__ count_dev, int32_t max_count,
                                                 int64_t *__restrict__ acc, int32_t *__restrict__ flags,
                                                 int stride, ScreenArgs S) {
    extern __shared__ float4 bead_lds[];
    __shared__ long long wacc[kMdWaves][10];   // per-wave energy/virial sums (fixed point)
    __shared__ PairQueue Qs[2];                // this round's queue and the next round's
    static_assert(kMdWaves > 1, "wave 0 screens while the others copy the templates");
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    WaveLds L = wave_lds(bead_lds, w, stride);
    if (lane < 10) wacc[w][lane] = 0;
    // the templates are copied by waves 1.. while wave 0 screens the first
    // round; one barrier publishes both
    float4 *tbw = bead_lds + (size_t)kMdWaves * 3 * stride;
    if (w != 0)
        for (int k = threadIdx.x - kWave; k < T.total; k += blockDim.x - kWave) tbw[k] = T.beads[k];
    const float4 *tb = tbw;
    const float rcm = sqrtf(lj.rc2) + kCullMargin, cut2 = rcm * rcm;
    int count = *count_dev;
    if (count > max_count) count = max_count;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(flags + RB_FLAG_NEVAL, count);
    long long ntests = 0;
    bool bad = false, ovf = false;
    const int G = gridDim.x;
    const bool full = !SCREENED || flags[RB_FLAG_RESCREEN] != 0;
    // pairs of this launch: the whole list, or the screened pairs (those that
    // passed the plain test at the screening first, spread evenly over the
    // blocks by the interleaved assignment)
    int npass = count, core = 0;
    if (SCREENED && !full) {
        npass = flags[RB_FLAG_NSCREEN];
        if (npass > count) npass = count;
        core = min(S.tmp[3], npass);
    }
    if (SCREENED && full) {
        for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += G * blockDim.x) {
#pragma unroll
            for (int a = 0; a < 3; ++a) S.x_ref[a * n + b] = x[a * n + b];
#pragma unroll
            for (int a = 0; a < 4; ++a) S.q_ref[a * n + b] = q[a * n + b];
        }
    }
    // Screening of the round starting at p0 into Q (wave 0 only): one lane
    // per pair, the pairs that can interact go to the queue with their
    // geometry.
    auto screen = [&](int p0, PairQueue &Q) {
        const int p = p0 + lane * G;
        bool hit = false, wide = false;
        int pid = 0, i = 0, j = 0, ti = 0, tj = 0;
        double dl[3], d[3], qr[4], qa[4];
        if (p < npass) {
            if (SCREENED && !full)
                pid = p < core ? S.list[p] : S.list[max_count - 1 - (p - core)];
            else
                pid = idx ? idx[p] : p;
            i = pi[pid];
            j = pj[pid];
            ti = type[i];
            tj = type[j];
            double R[9], Ri[9];
            pair_frame(n, x, q, box, i, j, dl, d, qr, qa, Ri);
            quat_to_rot<double>(qr[0], qr[1], qr[2], qr[3], R);
            // the shells' bound on the closest bead distance (box, and for
            // cylinder-like types capsule and cylinder) decides which pairs
            // can have a bead pair within rc
            hit = shell_route(T, ti, tj, d, R, 0.f, rcm) != kRouteSkip;
            if (SCREENED && full) wide = hit || shell_route(T, ti, tj, d, R, 0.f, S.rcm_wide) != kRouteSkip;
        }
        if (SCREENED && full) {
            list_append(hit, pid, S.tmp, S.list, max_count, false, lane);
            list_append(wide && !hit, pid, S.tmp + 1, S.list, max_count, true, lane);
        }
        const unsigned long long m = __ballot(hit);
        if (hit) {
            const int at = __popcll(m & ((1ull << lane) - 1ull));
            Q.i[at] = i;
            Q.j[at] = j;
            Q.ti[at] = ti;
            Q.tj[at] = tj;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Q.dl[a][at] = dl[a];
                Q.d[a][at] = d[a];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                Q.qr[a][at] = qr[a];
                Q.qa[a][at] = qa[a];
            }
        }
        if (lane == 0) {
            Q.n = __popcll(m);
            Q.head = 0;
        }
    };
    // Rounds: wave 0 screens round r + 1 into the other queue while the
    // block drains round r (wave 0 joins when done); the barrier at the end
    // of a round orders the drained queue's reuse after every read of it.
    int p0 = blockIdx.x;
    if (w == 0 && p0 < npass) screen(p0, Qs[0]);
    __syncthreads();
    for (int r = 0; p0 < npass; p0 += G * kRound, ++r) {
        PairQueue &Q = Qs[r & 1];
        const int pn = p0 + G * kRound;
        if (w == 0 && pn < npass) screen(pn, Qs[(r + 1) & 1]);
        {
            const int nq = Q.n;
            for (;;) {
                int k = 0;
                if (lane == 0) k = atomicAdd(&Q.head, 1);
                k = __builtin_amdgcn_readfirstlane(k);
                if (k >= nq) break;
                double dl[3], d[3], R[9], Ri[9];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    dl[a] = Q.dl[a][k];
                    d[a] = Q.d[a][k];
                }
                quat_to_rot<double>(Q.qr[0][k], Q.qr[1][k], Q.qr[2][k], Q.qr[3][k], R);
                quat_to_rot<double>(Q.qa[0][k], Q.qa[1][k], Q.qa[2][k], Q.qa[3][k], Ri);
                md_pair<POT>(T, lj, tb, L, lane, cut2, n, Q.i[k], Q.j[k], Q.ti[k], Q.tj[k], dl, d, R, Ri, acc, wacc[w],
                             ntests, bad, ovf);
            }
        }
        __syncthreads();
    }
    long long part[11];
#pragma unroll
    for (int a = 0; a < 10; ++a) part[a] = wacc[w][a];
    part[10] = ntests;
    block_flush_globals<kMdWaves>(part, acc + 6 * (int64_t)n, flags);
    if (lane == 0 && bad) atomicOr(flags + RB_FLAG_NONFINITE, 1);
    report_fixovf(ovf, flags);
    if (SCREENED && full) {
        // the last block to finish publishes the screened list
        __shared__ bool last;
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            last = atomicAdd(S.tmp + 2, 1) == G - 1;
        }
        __syncthreads();
        if (last && threadIdx.x == 0) {
            __threadfence();
            const int c = __hip_atomic_load(S.tmp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int m = __hip_atomic_load(S.tmp + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            flags[RB_FLAG_NSCREEN] = c + m;
            S.tmp[3] = c;
            S.tmp[0] = 0;
            S.tmp[1] = 0;
            S.tmp[2] = 0;
            flags[RB_FLAG_RESCREEN] = 0;
            flags[RB_FLAG_NRESCREENS] += 1;
        }
    }
}

// Dynamic LDS of a block (kBeadWaves waves, three arrays each) and the
// number of such blocks a CU holds, cached per size.
static size_t bead_lds_bytes(const rb_ctx *ctx, int waves, int &stride) {
    stride = (ctx->max_beads + 3) & ~3;
    return sizeof(float4) * (3 * (size_t)stride * waves + (size_t)ctx->total_beads);
}

template <typename K>
static int blocks_per_cu(K kernel, int threads, size_t lds, int *cache_lds, int *cache_nb) {
    if (*cache_lds == (int)lds && *cache_nb > 0) return *cache_nb;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess || nb < 1) nb = 1;
    *cache_lds = (int)lds;
    *cache_nb = nb;
    return nb;
}

// Largest dynamic + static LDS a block may use on the current device.
static size_t device_max_lds() {
    static size_t cached = 0;
    if (cached > 0) return cached;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        v = 65536;
    cached = (size_t)v;
    return cached;
}

}  // namespace rb

using namespace rb;

extern "C" int rb_bead_pair_eval(const rb_ctx *ctx, int64_t n_pairs, const float *desc, int32_t type_i,
                                 int32_t type_j, float *out, int32_t *flags, void *stream) {
    RB_REQUIRE(ctx && (n_pairs == 0 || (desc && out)), "rb_bead_pair_eval: null argument");
    RB_REQUIRE(n_pairs >= 0, "rb_bead_pair_eval: n_pairs < 0");
    RB_REQUIRE(type_i >= 0 && type_i < ctx->n_types && type_j >= 0 && type_j < ctx->n_types,
               "rb_bead_pair_eval: bad type");
    if (n_pairs == 0) return RB_OK;
    int stride;
    const size_t lds = bead_lds_bytes(ctx, kBeadWaves, stride);
    RB_REQUIRE(lds <= 65536, "rb_bead_pair_eval: templates need %zu bytes of LDS (max 65536)", lds);
    static int c_lds = -1, c_nb = 0;
    const int nb = blocks_per_cu(k_bead_desc<kPotLJ>, 256, lds, &c_lds, &c_nb);
    const int grid = grid_for(n_pairs, kBeadWaves, nb * device_cu_count());
    if (ctx->dev.lj.kind == kPotHPHC)
        k_bead_desc<kPotHPHC><<<grid, 256, lds, (hipStream_t)stream>>>(ctx->dev.t, ctx->dev.lj, type_i, type_j,
                                                                      n_pairs, desc, out, flags, stride);
    else
        k_bead_desc<kPotLJ><<<grid, 256, lds, (hipStream_t)stream>>>(ctx->dev.t, ctx->dev.lj, type_i, type_j,
                                                                    n_pairs, desc, out, flags, stride);
    RB_LAUNCH_CHECK("rb_bead_pair_eval");
    return RB_OK;
}

// Launch of the per-body form: a persistent grid of 8-wave blocks, as many
// as a CU holds (LDS sized for the templates in use); each block flushes its
// global sums once.
template <bool SCREENED>
static int launch_bead_md(const rb_ctx *ctx, int32_t n, const double *x, const double *q, const int32_t *type,
                          const double *box, const int32_t *pair_i, const int32_t *pair_j, const int32_t *idx,
                          const int32_t *count_dev, int32_t max_count, int64_t *acc, int32_t *flags,
                          const ScreenArgs &S, void *stream, const char *who) {
    Box b;
    for (int a = 0; a < 3; ++a) {
        RB_REQUIRE(box[a] > 0, "%s: box must be > 0", who);
        b.L[a] = box[a];
        b.inv[a] = 1.0 / box[a];
    }
    int stride;
    const size_t lds = bead_lds_bytes(ctx, kMdWaves, stride);
    RB_REQUIRE(lds + 2 * sizeof(PairQueue) + 1024 <= device_max_lds(),
               "%s: templates need %zu bytes of LDS per block (device max %zu)", who, lds, device_max_lds());
    const bool hphc = ctx->dev.lj.kind == kPotHPHC;
    auto kern = hphc ? k_bead_md<kPotHPHC, SCREENED> : k_bead_md<kPotLJ, SCREENED>;
    static int c_lds[2] = {-1, -1}, c_nb[2] = {0, 0};
    const int nb = blocks_per_cu(kern, kMdWaves * kWave, lds, &c_lds[hphc], &c_nb[hphc]);
    const int grid = grid_for(max_count, kMdWaves, nb * device_cu_count());
    kern<<<grid, kMdWaves * kWave, lds, (hipStream_t)stream>>>(ctx->dev.t, ctx->dev.lj, n, x, q, type, b, pair_i,
                                                              pair_j, idx, count_dev, max_count, acc, flags, stride,
                                                              S);
    return RB_OK;
}

extern "C" int rb_bead_pair_forces(const rb_ctx *ctx, int32_t n, const double *x, const double *q,
                                   const int32_t *type, const double *box, const int32_t *pair_i,
                                   const int32_t *pair_j, const int32_t *idx, const int32_t *count_dev,
                                   int32_t max_count, int64_t *acc, int32_t *flags, void *stream) {
    RB_REQUIRE(ctx && x && q && type && box && pair_i && pair_j && count_dev && acc && flags,
               "rb_bead_pair_forces: null argument");
    RB_REQUIRE(n >= 0 && max_count >= 0, "rb_bead_pair_forces: negative size");
    if (max_count == 0 || n == 0) return RB_OK;
    const int rc = launch_bead_md<false>(ctx, n, x, q, type, box, pair_i, pair_j, idx, count_dev, max_count, acc,
                                         flags, ScreenArgs{}, stream, "rb_bead_pair_forces");
    if (rc != RB_OK) return rc;
    RB_LAUNCH_CHECK("rb_bead_pair_forces");
    return RB_OK;
}

extern "C" int rb_bead_pair_forces_screened(const rb_ctx *ctx, int32_t n, const double *x, const double *q,
                                            const int32_t *type, const double *box, const int32_t *pair_i,
                                            const int32_t *pair_j, const int32_t *count_dev, int32_t max_count,
                                            double margin, int32_t *screen_list, double *x_sref, double *q_sref,
                                            int32_t *tmp, int64_t *acc, int32_t *flags, void *stream) {
    RB_REQUIRE(ctx && x && q && type && box && pair_i && pair_j && count_dev && screen_list && x_sref && q_sref &&
                   tmp && acc && flags,
               "rb_bead_pair_forces_screened: null argument");
    RB_REQUIRE(n >= 0 && max_count >= 0, "rb_bead_pair_forces_screened: negative size");
    RB_REQUIRE(margin >= 0 && margin < 1e6, "rb_bead_pair_forces_screened: margin must be in [0, 1e6)");
    if (max_count == 0 || n == 0) return RB_OK;
    ScreenArgs S;
    S.list = screen_list;
    S.x_ref = x_sref;
    S.q_ref = q_sref;
    S.tmp = tmp;
    S.rcm_wide = (float)(sqrt((double)ctx->dev.lj.rc2) + kCullMargin + margin);
    const int rc = launch_bead_md<true>(ctx, n, x, q, type, box, pair_i, pair_j, nullptr, count_dev, max_count, acc,
                                        flags, S, stream, "rb_bead_pair_forces_screened");
    if (rc != RB_OK) return rc;
    RB_LAUNCH_CHECK("rb_bead_pair_forces_screened");
    return RB_OK;
}

extern "C" int rb_bead_screen(const rb_ctx *ctx, int32_t n, const double *x, const double *q, const int32_t *type,
                              const double *box, const int32_t *pair_i, const int32_t *pair_j, const int32_t *idx,
                              const int32_t *count_dev, int32_t max_count, int32_t *idx_out, int32_t *count_out,
                              int32_t *tmp, int32_t *flags, void *stream) {
    RB_REQUIRE(ctx && x && q && type && box && pair_i && pair_j && count_dev && idx_out && count_out && tmp,
               "rb_bead_screen: null argument");
    RB_REQUIRE(n > 0 && max_count > 0, "rb_bead_screen: sizes must be > 0");
    Box b;
    for (int a = 0; a < 3; ++a) {
        RB_REQUIRE(box[a] > 0, "rb_bead_screen: box must be > 0");
        b.L[a] = box[a];
        b.inv[a] = 1.0 / box[a];
    }
    const float rcm = sqrtf(ctx->dev.lj.rc2) + kCullMargin;
    k_bead_screen<<<grid_for(max_count, 256, 4 * device_cu_count()), 256, 0, (hipStream_t)stream>>>(
        ctx->dev.t, rcm, n, x, q, type, b, pair_i, pair_j, idx, count_dev, max_count, idx_out, count_out, tmp, flags);
    RB_LAUNCH_CHECK("rb_bead_screen");
    return RB_OK;
}
