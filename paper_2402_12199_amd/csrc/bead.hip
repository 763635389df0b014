// Bead double sum between composite rigid bodies (paper section 2, first
// equation: the body-body energy is the sum of the bead potential over all
// N_i x N_j bead pairs), with the workloads' bead potential, Lennard-Jones
// 12-6 shifted in energy at rc.
//
// Work mapping (gfx950, wave64): one wavefront per body pair.  The pair is
// evaluated in body i's frame, where body i's beads are just its template.
// Each lane keeps S = ceil(N_i / 64) of body i's beads in registers; body
// j's beads are rotated into body i's frame (FP64, then rounded to FP32) and
// staged in LDS, and every lane streams them with broadcast LDS reads, so
// each LDS read feeds S distance tests.  Per-bead forces stay in registers;
// F_i and tau_i are reduced across the wave with lane shuffles, and body j's
// force and torque follow from pair identities (central bead forces):
// F_j = -F_i and tau_j = d x F_i - tau_i.
#include "rb_common.hpp"

namespace rb {

constexpr int kBeadWaves = 4;      // waves per block
constexpr float kFar = 1.0e4f;     // coordinate of padding beads: never inside rc

// Body j's beads, rotated and shifted into body i's frame, into this wave's
// LDS slice: r_l = d + R b_l, computed in FP64 and split into an FP32 value
// (sj) and its FP32 rounding residual (sjlo).
__device__ inline void stage_j(const Templates &T, int tj, const double d[3], const double R[9],
                               float4 *sj, float4 *sjlo, int lane) {
    const int nj = T.n[tj];
    const float4 *bj = T.beads + T.off[tj];
    for (int l = lane; l < nj; l += kWave) {
        const float4 b = bj[l];
        const double bx = b.x, by = b.y, bz = b.z;
        const double x = d[0] + R[0] * bx + R[1] * by + R[2] * bz;
        const double y = d[1] + R[3] * bx + R[4] * by + R[5] * bz;
        const double z = d[2] + R[6] * bx + R[7] * by + R[8] * bz;
        const float fx = (float)x, fy = (float)y, fz = (float)z;
        sj[l] = make_float4(fx, fy, fz, 0.f);
        sjlo[l] = make_float4((float)(x - fx), (float)(y - fy), (float)(z - fz), 0.f);
    }
}

template <int S>
__device__ inline void load_i(const Templates &T, int ti, int lane, float (&bx)[S], float (&by)[S],
                              float (&bz)[S]) {
    const int ni = T.n[ti];
    const float4 *b = T.beads + T.off[ti];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int k = lane + kWave * s;
        if (k < ni) {
            const float4 v = b[k];
            bx[s] = v.x; by[s] = v.y; bz[s] = v.z;
        } else {
            bx[s] = kFar; by[s] = kFar; bz[s] = kFar;
        }
    }
}

// All N_i x N_j distance tests of one pair.  The screening distance uses
// the FP32 positions; a bead pair that passes (r^2 < rc^2 + a margin far
// above the FP32 rounding of r^2) is recomputed with the residuals of body
// j's positions, so the cutoff test and the LJ terms see the positions to
// about 1e-13 sigma.  Returns, reduced over the wave (valid in every lane):
// r[0] = E, r[1..3] = F_i, r[4..6] = tau_i (about body i's centre, body i
// frame), r[7] = min squared bead distance (only when TRACK_MIN).
template <int S, bool TRACK_MIN>
__device__ inline void pair_sum(const LJ &lj, int nj, const float (&bx)[S], const float (&by)[S],
                                const float (&bz)[S], const float4 *sj, const float4 *sjlo, float r[8]) {
    float fx[S], fy[S], fz[S];
#pragma unroll
    for (int s = 0; s < S; ++s) fx[s] = fy[s] = fz[s] = 0.f;
    float e = 0.f, r2min = 3.0e38f;
    const float screen = lj.rc2 + 1.0e-3f;
    for (int l = 0; l < nj; ++l) {
        const float4 p = sj[l];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            float dx = bx[s] - p.x, dy = by[s] - p.y, dz = bz[s] - p.z;
            float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            if (TRACK_MIN) r2min = fminf(r2min, r2);
            if (r2 < screen) {
                const float4 lo = sjlo[l];
                dx -= lo.x; dy -= lo.y; dz -= lo.z;
                r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                if (r2 < lj.rc2) {
                    const float ir2 = __builtin_amdgcn_rcpf(r2);
                    const float s2 = lj.sig2 * ir2;
                    const float s6 = s2 * s2 * s2;
                    const float s12 = s6 * s6;
                    e += fmaf(lj.c4e, s12 - s6, -lj.ushift);
                    const float fr = lj.c24e * fmaf(2.f, s12, -s6) * ir2;
                    fx[s] = fmaf(fr, dx, fx[s]);
                    fy[s] = fmaf(fr, dy, fy[s]);
                    fz[s] = fmaf(fr, dz, fz[s]);
                }
            }
        }
    }
    float F[3] = {0.f, 0.f, 0.f}, t[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < S; ++s) {
        F[0] += fx[s]; F[1] += fy[s]; F[2] += fz[s];
        t[0] += by[s] * fz[s] - bz[s] * fy[s];
        t[1] += bz[s] * fx[s] - bx[s] * fz[s];
        t[2] += bx[s] * fy[s] - by[s] * fx[s];
    }
    r[0] = wave_sum(e);
    r[1] = wave_sum(F[0]); r[2] = wave_sum(F[1]); r[3] = wave_sum(F[2]);
    r[4] = wave_sum(t[0]); r[5] = wave_sum(t[1]); r[6] = wave_sum(t[2]);
    r[7] = TRACK_MIN ? wave_min(r2min) : 0.f;
}

// Per-pair form: descriptors in, per-pair outputs in body i's frame out.
template <int S>
__global__ __launch_bounds__(256) void k_bead_desc(Templates T, LJ lj, int ti, int tj, int64_t P,
                                                   const float *__restrict__ desc,
                                                   float *__restrict__ out) {
    __shared__ float4 lds[kBeadWaves][kMaxBeads];
    __shared__ float4 ldslo[kBeadWaves][kMaxBeads];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float4 *sj = lds[w];
    float4 *sjlo = ldslo[w];
    float bx[S], by[S], bz[S];
    load_i<S>(T, ti, lane, bx, by, bz);
    const int nj = T.n[tj];
    const int64_t step = (int64_t)gridDim.x * kBeadWaves;
    for (int64_t p = (int64_t)blockIdx.x * kBeadWaves + w; p < P; p += step) {
        double d[3] = {desc[p], desc[P + p], desc[2 * P + p]};
        double qw = desc[3 * P + p], qx = desc[4 * P + p], qy = desc[5 * P + p], qz = desc[6 * P + p];
        const double inv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        double R[9];
        quat_to_rot<double>(qw * inv, qx * inv, qy * inv, qz * inv, R);
        stage_j(T, tj, d, R, sj, sjlo, lane);
        wave_lds_sync();
        float r[8];
        pair_sum<S, true>(lj, nj, bx, by, bz, sj, sjlo, r);
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
            out[10 * P + p] = sqrtf(r[7]);
        }
    }
}

struct Box {
    double L[3], inv[3];
};

// Per-body form for dynamics.  Geometry from FP64 state; the pair's outputs
// are rotated to the lab frame and added to the fixed-point accumulator.
template <int S>
__global__ __launch_bounds__(256) void k_bead_md(Templates T, LJ lj, int32_t n,
                                                 const double *__restrict__ x,
                                                 const double *__restrict__ q,
                                                 const int32_t *__restrict__ type, Box box,
                                                 const int32_t *__restrict__ pi,
                                                 const int32_t *__restrict__ pj,
                                                 const int32_t *__restrict__ idx,
                                                 const int32_t *__restrict__ count_dev,
                                                 int32_t max_count, int64_t *__restrict__ acc,
                                                 int32_t *__restrict__ flags) {
    __shared__ float4 lds[kBeadWaves][kMaxBeads];
    __shared__ float4 ldslo[kBeadWaves][kMaxBeads];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float4 *sj = lds[w];
    float4 *sjlo = ldslo[w];
    int count = *count_dev;
    if (count > max_count) count = max_count;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(flags + RB_FLAG_NEVAL, count);
    long long eacc[10];
#pragma unroll
    for (int a = 0; a < 10; ++a) eacc[a] = 0;
    bool bad = false;
    const int step = gridDim.x * kBeadWaves;
    for (int p = blockIdx.x * kBeadWaves + w; p < count; p += step) {
        const int pid = idx ? idx[p] : p;
        const int i = pi[pid], j = pj[pid];
        const int ti = type[i], tj = type[j];
        double dl[3], Ri[9], Rj[9], d[3], R[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            dl[a] = min_image(x[a * n + j] - x[a * n + i], box.L[a], box.inv[a]);
        quat_to_rot<double>(q[i], q[n + i], q[2 * n + i], q[3 * n + i], Ri);
        quat_to_rot<double>(q[j], q[n + j], q[2 * n + j], q[3 * n + j], Rj);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            d[a] = Ri[a] * dl[0] + Ri[3 + a] * dl[1] + Ri[6 + a] * dl[2];
#pragma unroll
            for (int b = 0; b < 3; ++b)
                R[3 * a + b] = Ri[a] * Rj[b] + Ri[3 + a] * Rj[3 + b] + Ri[6 + a] * Rj[6 + b];
        }
        float bx[S], by[S], bz[S];
        load_i<S>(T, ti, lane, bx, by, bz);
        stage_j(T, tj, d, R, sj, sjlo, lane);
        wave_lds_sync();
        float r[8];
        pair_sum<S, false>(lj, T.n[tj], bx, by, bz, sj, sjlo, r);
        wave_lds_sync();
        if (lane == 0) {
            const double F[3] = {r[1], r[2], r[3]}, ti_[3] = {r[4], r[5], r[6]};
            const double tj_[3] = {d[1] * F[2] - d[2] * F[1] - ti_[0], d[2] * F[0] - d[0] * F[2] - ti_[1],
                                   d[0] * F[1] - d[1] * F[0] - ti_[2]};
            double Fl[3], til[3], tjl[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Fl[a] = Ri[3 * a] * F[0] + Ri[3 * a + 1] * F[1] + Ri[3 * a + 2] * F[2];
                til[a] = Ri[3 * a] * ti_[0] + Ri[3 * a + 1] * ti_[1] + Ri[3 * a + 2] * ti_[2];
                tjl[a] = Ri[3 * a] * tj_[0] + Ri[3 * a + 1] * tj_[1] + Ri[3 * a + 2] * tj_[2];
            }
            if (!isfinite(r[0]) || !isfinite(r[1]) || !isfinite(r[2]) || !isfinite(r[3])) bad = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                acc_add(acc + (int64_t)a * n + i, Fl[a]);
                acc_add(acc + (int64_t)a * n + j, -Fl[a]);
                acc_add(acc + (int64_t)(3 + a) * n + i, til[a]);
                acc_add(acc + (int64_t)(3 + a) * n + j, tjl[a]);
            }
            eacc[0] += to_fixed(r[0]);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) eacc[1 + 3 * a + b] += to_fixed(-dl[a] * Fl[b]);
        }
    }
    if (lane == 0) {
        int64_t *g = acc + 6 * (int64_t)n;
#pragma unroll
        for (int a = 0; a < 10; ++a)
            if (eacc[a]) atomicAdd(reinterpret_cast<unsigned long long *>(g + a), (unsigned long long)eacc[a]);
        if (bad) atomicOr(flags + RB_FLAG_NONFINITE, 1);
    }
}

static int slots_for(int nbeads) { return (nbeads + kWave - 1) / kWave; }

}  // namespace rb

using namespace rb;

extern "C" int rb_bead_pair_eval(const rb_ctx *ctx, int64_t n_pairs, const float *desc, int32_t type_i,
                                 int32_t type_j, float *out, void *stream) {
    RB_REQUIRE(ctx && (n_pairs == 0 || (desc && out)), "rb_bead_pair_eval: null argument");
    RB_REQUIRE(n_pairs >= 0, "rb_bead_pair_eval: n_pairs < 0");
    RB_REQUIRE(type_i >= 0 && type_i < ctx->n_types && type_j >= 0 && type_j < ctx->n_types,
               "rb_bead_pair_eval: bad type");
    if (n_pairs == 0) return RB_OK;
    const int S = slots_for(ctx->n_beads[type_i]);
    const int grid = grid_for(n_pairs, kBeadWaves, 65536);
    hipStream_t st = (hipStream_t)stream;
    switch (S) {
        case 1: k_bead_desc<1><<<grid, 256, 0, st>>>(ctx->dev.t, ctx->dev.lj, type_i, type_j, n_pairs, desc, out); break;
        case 2: k_bead_desc<2><<<grid, 256, 0, st>>>(ctx->dev.t, ctx->dev.lj, type_i, type_j, n_pairs, desc, out); break;
        case 3: k_bead_desc<3><<<grid, 256, 0, st>>>(ctx->dev.t, ctx->dev.lj, type_i, type_j, n_pairs, desc, out); break;
        default: k_bead_desc<4><<<grid, 256, 0, st>>>(ctx->dev.t, ctx->dev.lj, type_i, type_j, n_pairs, desc, out); break;
    }
    RB_LAUNCH_CHECK("rb_bead_pair_eval");
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
    int maxb = 0;
    for (int t = 0; t < ctx->n_types; ++t) maxb = ctx->n_beads[t] > maxb ? ctx->n_beads[t] : maxb;
    Box b;
    for (int a = 0; a < 3; ++a) {
        RB_REQUIRE(box[a] > 0, "rb_bead_pair_forces: box must be > 0");
        b.L[a] = box[a];
        b.inv[a] = 1.0 / box[a];
    }
    const int S = slots_for(maxb);
    const int grid = grid_for(max_count, kBeadWaves, 8192);
    hipStream_t st = (hipStream_t)stream;
#define RB_MD_LAUNCH(SS)                                                                               \
    k_bead_md<SS><<<grid, 256, 0, st>>>(ctx->dev.t, ctx->dev.lj, n, x, q, type, b, pair_i, pair_j, idx, \
                                        count_dev, max_count, acc, flags)
    switch (S) {
        case 1: RB_MD_LAUNCH(1); break;
        case 2: RB_MD_LAUNCH(2); break;
        case 3: RB_MD_LAUNCH(3); break;
        default: RB_MD_LAUNCH(4); break;
    }
#undef RB_MD_LAUNCH
    RB_LAUNCH_CHECK("rb_bead_pair_forces");
    return RB_OK;
}
