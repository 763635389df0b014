// Per-tile forward / reverse passes of the energy network, shared by the
// inference kernels and the training kernel.
#pragma once

#include "nn_common.hpp"

namespace rb {

// Optional output of the per-pair activations and reverse-pass deltas of a
// tile (training): H rows h0 (7, normalised input), h1..h4 (128 each);
// D rows delta1..delta4 (128 each, dX/dz_l) and delta5 (1, dX/de'); both
// feature-major with row stride B, column = this lane's batch row.
constexpr int kHRows = kIn + 4 * kH;
constexpr int kDRows = 4 * kH + 1;
struct Emit {
    float *H = nullptr;
    float *D = nullptr;
    float *R = nullptr;     // residual e' - y' per batch row
    int64_t B = 0;
    int64_t b = 0;
    bool live = false;
    float y = 0.f;          // normalised label of this row
    float k2 = 0.f;         // 2 / B: the loss gradient is k2 (e' - y')
    __device__ float &h(int row) const { return H[row * B + b]; }
    __device__ float &d(int row) const { return D[row * B + b]; }
};

// ------------------------------------------------------------------ BF16
// Forward (and optionally reverse) pass of one 16-pair tile.  Returns E for
// this lane's pair; gu receives dX/du when GRAD (X = seed * E).  Each 16-row
// output tile is finished (bias, MFMA chain, SiLU, BF16 packing) before the
// next one starts, which keeps the live register set small.
template <bool GRAD, bool EMIT = false>
__device__ inline float tile_bf16(const LdsBF16 &L, const Norm &nm, const float u[kIn], float seed,
                                  float gu[kIn], const Emit &em = Emit{}) {
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
    float un[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) un[k] = (u[k] - nm.shift[k]) * nm.scale[k];
    if (EMIT && em.live && g == 0)
#pragma unroll
        for (int k = 0; k < kIn; ++k) em.h(k) = un[k];
    bf16x8 act[4];
    f16x8 sp[4][4];
    {
        float hv[8][4], dv[8][4];
        float x0, x1;
        l1_inputs(un, g, x0, x1);
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            const f32x4 z = layer1_rows(L.w1, L.b[0], x0, x1, n, g, mt);
#pragma unroll
            for (int r = 0; r < 4; ++r) silu(z[r], hv[mt][r], dv[mt][r]);
        }
        if (EMIT && em.live)
#pragma unroll
            for (int mt = 0; mt < 8; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) em.h(kIn + 16 * mt + 4 * g + r) = hv[mt][r];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            act[kb] = pack8(hv[2 * kb], hv[2 * kb + 1]);
            if (GRAD) sp[0][kb] = pack8h(dv[2 * kb], dv[2 * kb + 1]);
        }
    }
    float e = 0.f;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        bf16x8 nact[4];
        float hlo[4], dlo[4];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            __asm__ volatile("" ::: "memory");
            f32x4 c = *reinterpret_cast<const f32x4 *>(&L.b[l + 1][16 * mt + 4 * g]);
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&L.w[l][16 * mt + n][wcol(16 * mt + n, 32 * kb + 8 * g)]);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, act[kb], c, 0, 0, 0);
            }
            float h[4], d[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) silu(c[r], h[r], d[r]);
            if (EMIT && em.live)
#pragma unroll
                for (int r = 0; r < 4; ++r) em.h(kIn + kH * (l + 1) + 16 * mt + 4 * g + r) = h[r];
            if (l == 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) e = fmaf(L.w5[16 * mt + 4 * g + r], h[r], e);
            }
            if ((mt & 1) == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) { hlo[r] = h[r]; dlo[r] = d[r]; }
            } else {
                if (l < 2) nact[mt >> 1] = pack8(hlo, h);
                if (GRAD) sp[l + 1][mt >> 1] = pack8h(dlo, d);
            }
        }
        if (l < 2) {
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) act[kb] = nact[kb];
        }
    }
    e = group_sum(e) + L.b5;
    const float E = fmaf(e, nm.oscale, nm.oshift);
    if (!GRAD) return E;
    if (EMIT) {
        seed = em.live ? em.k2 * (E - em.y) : 0.f;
        if (em.live && g == 0) em.R[em.b] = E - em.y;
    }

    // reverse pass: delta_4 = seed * oscale * w5 (.) h4'
    const float s0 = seed * nm.oscale;
    bf16x8 dpk[4], dlk[4];   // delta as BF16 head + BF16 remainder
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        float a0[4], a1[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a0[r] = s0 * L.w5[32 * kb + 4 * g + r] * (float)sp[3][kb][r];
            a1[r] = s0 * L.w5[32 * kb + 16 + 4 * g + r] * (float)sp[3][kb][4 + r];
            if (EMIT && em.live) {
                em.d(3 * kH + 32 * kb + 4 * g + r) = a0[r];
                em.d(3 * kH + 32 * kb + 16 + 4 * g + r) = a1[r];
            }
        }
        split8(a0, a1, dpk[kb], dlk[kb]);
    }
    if (EMIT && em.live && g == 0) em.d(4 * kH) = s0;
    float gk[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) gk[k] = 0.f;
#pragma unroll
    for (int l = 2; l >= 0; --l) {
        bf16x8 ndpk[4], ndlk[4];
        float dlo[4];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            __asm__ volatile("" ::: "memory");
            f32x4 c = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x8 a = wt_frag(L, l, kb, mt, lane);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, dpk[kb], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, dlk[kb], c, 0, 0, 0);
            }
            float d[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) d[r] = c[r] * (float)sp[l][mt >> 1][4 * (mt & 1) + r];
            if (EMIT && em.live)
#pragma unroll
                for (int r = 0; r < 4; ++r) em.d(kH * l + 16 * mt + 4 * g + r) = d[r];
            if (l > 0) {
                if ((mt & 1) == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) dlo[r] = d[r];
                } else {
                    split8(dlo, d, ndpk[mt >> 1], ndlk[mt >> 1]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int f = 16 * mt + 4 * g + r;
#pragma unroll
                    for (int k = 0; k < kIn; ++k) gk[k] = fmaf(L.w1[f][k], d[r], gk[k]);
                }
            }
        }
        if (l > 0) {
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                dpk[kb] = ndpk[kb];
                dlk[kb] = ndlk[kb];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kIn; ++k) gu[k] = group_sum(gk[k]) * nm.scale[k];
    return E;
}

// ------------------------------------------------------------ BF16, wide
// One 16-pair tile evaluated by a group of four waves.  Wave v of the group
// owns the hidden features 32 v .. 32 v + 31 of every layer (output tiles
// 2 v and 2 v + 1, i.e. the MFMA operand block kb = v of the next layer) and
// the waves exchange their activation and delta blocks through LDS after
// each layer; the energy and dX/du are summed over the four waves in a fixed
// order.  Each wave does a quarter of the SiLU and MFMA work of a tile, so a
// tile's latency is about a quarter of the single-wave form's, which is what
// small batches (one tile per wave) are bound by.  Same arithmetic per
// feature as tile_bf16 except the order of the final sums.
constexpr int kWideGroup = 4;
struct WideX {
    bf16x8 a[kWideGroup][kWave];     // activation blocks
    bf16x8 dh[kWideGroup][kWave];    // delta blocks, BF16 head
    bf16x8 dl[kWideGroup][kWave];    // delta blocks, BF16 remainder
    float red[kWideGroup][8][16];    // per-row partial sums (energy, dX/du)
};

// Barrier of the four-wave tiles: their waves exchange data through LDS only,
// so the barrier waits for the wave's LDS operations and not for its global
// memory operations (which a full __syncthreads also waits for, e.g. loads
// a caller has in flight across the tile); the compiler fences keep LDS
// accesses on their side of it.
__device__ inline void wide_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Work a caller interleaves with a tile (e.g. fetching the next tile's
// inputs): hook(1) runs after layer 1's exchange, hook(2) after the energy,
// before the reverse pass.
struct NoHook {
    __device__ void operator()(int) const {}
};

// Synchronisation of a tile's four waves: the whole block (BlockSync), or the
// group alone (GroupSync): each wave of the group writes the number of
// barriers it has reached into its own LDS word (after its own LDS
// operations are done) and waits until all four words have reached it; the
// waits of one group then do not hold the block's other groups.  The wait is
// bounded: past kGroupSyncSpins polls it records a timeout (an internal
// error the caller reports) and goes on, so a kernel always ends.
struct BlockSync {
    __device__ void operator()() const { wide_sync(); }
};

constexpr int kGroupSyncSpins = 1 << 16;

typedef __attribute__((address_space(3))) int lds_int;
typedef __attribute__((address_space(3))) unsigned lds_uint;
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) volatile i32x4 lds_vi32x4;

struct GroupSync {
    lds_int *word;      // the group's four LDS words (16-byte aligned), zero at the first barrier
    int v;              // this wave's index in the group
    int *gen;           // barriers this wave has passed (a register of the caller)
    lds_int *timeout;   // LDS word set on a timeout
    __device__ void operator()() const {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): this wave's LDS writes are done
        const int target = ++*gen;
        if ((threadIdx.x & (kWave - 1)) == 0) *(volatile lds_int *)(word + v) = target;
        for (int spin = 0;; ++spin) {
            const i32x4 w = *(lds_vi32x4 *)word;
            if (w[0] >= target && w[1] >= target && w[2] >= target && w[3] >= target) break;
            if (spin >= kGroupSyncSpins) {
                *timeout = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
};

template <bool GRAD, bool EMIT = false, class Hook = NoHook, class Sync = BlockSync>
__device__ inline float tile_bf16_wide(const LdsBF16 &L, WideX &X, const Norm &nm, const float u[kIn], float seed,
                                       float gu[kIn], int v, const Emit &em = Emit{}, const Hook &hook = Hook{},
                                       const Sync &sync = Sync{}) {
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
    float un[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) un[k] = (u[k] - nm.shift[k]) * nm.scale[k];
    if (EMIT && em.live && g == 0 && v == 0)
#pragma unroll
        for (int k = 0; k < kIn; ++k) em.h(k) = un[k];
    bf16x8 act[4];
    f16x8 spo[4];
    {
        float h[2][4], d[2][4];
        float x0, x1;
        l1_inputs(un, g, x0, x1);
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
            const f32x4 z = layer1_rows(L.w1, L.b[0], x0, x1, n, g, 2 * v + mm);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                silu(z[r], h[mm][r], d[mm][r]);
                if (EMIT && em.live) em.h(kIn + 32 * v + 16 * mm + 4 * g + r) = h[mm][r];
            }
        }
        X.a[v][lane] = pack8(h[0], h[1]);
        if (GRAD) spo[0] = pack8h(d[0], d[1]);
    }
    sync();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) act[kb] = X.a[kb][lane];
    sync();
    hook(1);
    float e = 0.f;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        float h[2][4], d[2][4];
        // the wave's two output blocks as two interleaved MFMA chains (each
        // accumulates over kb in order, as a single chain would)
        f32x4 c2[2];
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) c2[mm] = *reinterpret_cast<const f32x4 *>(&L.b[l + 1][16 * (2 * v + mm) + 4 * g]);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) {
                const bf16x8 a =
                    *reinterpret_cast<const bf16x8 *>(&L.w[l][16 * (2 * v + mm) + n][wcol(16 * (2 * v + mm) + n, 32 * kb + 8 * g)]);
                c2[mm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, act[kb], c2[mm], 0, 0, 0);
            }
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
            const int mt = 2 * v + mm;
            const f32x4 c = c2[mm];
#pragma unroll
            for (int r = 0; r < 4; ++r) silu(c[r], h[mm][r], d[mm][r]);
            if (EMIT && em.live)
#pragma unroll
                for (int r = 0; r < 4; ++r) em.h(kIn + kH * (l + 1) + 16 * mt + 4 * g + r) = h[mm][r];
            if (l == 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) e = fmaf(L.w5[16 * mt + 4 * g + r], h[mm][r], e);
            }
        }
        if (GRAD) spo[l + 1] = pack8h(d[0], d[1]);
        if (l < 2) {
            X.a[v][lane] = pack8(h[0], h[1]);
            sync();
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) act[kb] = X.a[kb][lane];
            sync();
        }
    }
    e = group_sum(e);
    if (g == 0) X.red[v][0][n] = e;
    sync();
    e = ((X.red[0][0][n] + X.red[1][0][n]) + X.red[2][0][n]) + X.red[3][0][n] + L.b5;
    sync();
    hook(2);
    const float E = fmaf(e, nm.oscale, nm.oshift);
    if (!GRAD) return E;
    if (EMIT) {
        seed = em.live ? em.k2 * (E - em.y) : 0.f;
        if (em.live && g == 0 && v == 0) em.R[em.b] = E - em.y;
    }

    // reverse pass: this wave's block of delta_4 = seed * oscale * w5 (.) h4'
    const float s0 = seed * nm.oscale;
    if (EMIT && em.live && g == 0 && v == 0) em.d(4 * kH) = s0;
    bf16x8 dpk[4], dlk[4];
    {
        float a0[4], a1[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a0[r] = s0 * L.w5[32 * v + 4 * g + r] * (float)spo[3][r];
            a1[r] = s0 * L.w5[32 * v + 16 + 4 * g + r] * (float)spo[3][4 + r];
            if (EMIT && em.live) {
                em.d(3 * kH + 32 * v + 4 * g + r) = a0[r];
                em.d(3 * kH + 32 * v + 16 + 4 * g + r) = a1[r];
            }
        }
        bf16x8 hi, lo;
        split8(a0, a1, hi, lo);
        X.dh[v][lane] = hi;
        X.dl[v][lane] = lo;
    }
    sync();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        dpk[kb] = X.dh[kb][lane];
        dlk[kb] = X.dl[kb][lane];
    }
    sync();
    float gk[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) gk[k] = 0.f;
#pragma unroll
    for (int l = 2; l >= 0; --l) {
        float d[2][4];
        // two interleaved chains, one per output block of the wave (each in
        // the order of a single chain: kb ascending, head then remainder)
        f32x4 c2[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            bf16x8 a2[2];
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) a2[mm] = wt_frag(L, l, kb, 2 * v + mm, lane);
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) c2[mm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[mm], dpk[kb], c2[mm], 0, 0, 0);
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) c2[mm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[mm], dlk[kb], c2[mm], 0, 0, 0);
        }
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
            const int mt = 2 * v + mm;
            const f32x4 c = c2[mm];
#pragma unroll
            for (int r = 0; r < 4; ++r) d[mm][r] = c[r] * (float)spo[l][4 * mm + r];
            if (EMIT && em.live)
#pragma unroll
                for (int r = 0; r < 4; ++r) em.d(kH * l + 16 * mt + 4 * g + r) = d[mm][r];
            if (l == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int f = 16 * mt + 4 * g + r;
#pragma unroll
                    for (int k = 0; k < kIn; ++k) gk[k] = fmaf(L.w1[f][k], d[mm][r], gk[k]);
                }
            }
        }
        if (l > 0) {
            bf16x8 hi, lo;
            split8(d[0], d[1], hi, lo);
            X.dh[v][lane] = hi;
            X.dl[v][lane] = lo;
            sync();
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                dpk[kb] = X.dh[kb][lane];
                dlk[kb] = X.dl[kb][lane];
            }
            sync();
        }
    }
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        const float s = group_sum(gk[k]);
        if (g == 0) X.red[v][1 + k][n] = s;
    }
    sync();
#pragma unroll
    for (int k = 0; k < kIn; ++k)
        gu[k] = (((X.red[0][1 + k][n] + X.red[1][1 + k][n]) + X.red[2][1 + k][n]) + X.red[3][1 + k][n]) * nm.scale[k];
    sync();
    return E;
}

// ------------------------------------------------------------------ FP32
// Small LDS image for the FP32 path: W1, biases, w5, and per wave the SiLU
// derivatives of the forward pass (4 layers x 32 values x 64 lanes).
constexpr int kF32Waves = 4;
struct alignas(16) LdsFP32 {
    float w1[kH][8];
    float b[4][kH];
    float w5[kH];
    float b5;
    float sp[kF32Waves][4][32][kWave];
};

template <bool GRAD, bool EMIT = false>
__device__ inline float tile_fp32(const LdsFP32 &Lc, LdsFP32 &L, const float *__restrict__ p, const Norm &nm,
                                  const float u[kIn], float seed, float gu[kIn], const Emit &em = Emit{}) {
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
    const int w = threadIdx.x >> 6;
    float un[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) un[k] = (u[k] - nm.shift[k]) * nm.scale[k];
    if (EMIT && em.live && g == 0)
#pragma unroll
        for (int k = 0; k < kIn; ++k) em.h(k) = un[k];
    float hv[8][4], dv[8][4];
    layer1(Lc.w1, Lc.b[0], un, g, hv, dv);
    if (EMIT && em.live)
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) em.h(kIn + 16 * mt + 4 * g + r) = hv[mt][r];
    if (GRAD) {
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) L.sp[w][0][4 * mt + r][lane] = dv[mt][r];
    }
    for (int l = 0; l < 3; ++l) {
        const float *W = p + w_off(l + 2);
        f32x4 acc[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) acc[mt] = *reinterpret_cast<const f32x4 *>(&Lc.b[l + 1][16 * mt + 4 * g]);
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            __asm__ volatile("" ::: "memory");
            const float *row = W + (16 * mt + n) * kH + 4 * g;
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2) {
                const float4 a = *reinterpret_cast<const float4 *>(row + 16 * m2);
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, hv[m2][0], acc[mt], 0, 0, 0);
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, hv[m2][1], acc[mt], 0, 0, 0);
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, hv[m2][2], acc[mt], 0, 0, 0);
                acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, hv[m2][3], acc[mt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                silu(acc[mt][r], hv[mt][r], dv[mt][r]);
                if (GRAD) L.sp[w][l + 1][4 * mt + r][lane] = dv[mt][r];
                if (EMIT && em.live) em.h(kIn + kH * (l + 1) + 16 * mt + 4 * g + r) = hv[mt][r];
            }
    }
    float e = 0.f;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) e = fmaf(Lc.w5[16 * mt + 4 * g + r], hv[mt][r], e);
    e = group_sum(e) + Lc.b5;
    const float E = fmaf(e, nm.oscale, nm.oshift);
    if (!GRAD) return E;
    if (EMIT) {
        seed = em.live ? em.k2 * (E - em.y) : 0.f;
        if (em.live && g == 0) em.R[em.b] = E - em.y;
    }
    const float s0 = seed * nm.oscale;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dv[mt][r] = s0 * Lc.w5[16 * mt + 4 * g + r] * L.sp[w][3][4 * mt + r][lane];
            if (EMIT && em.live) em.d(3 * kH + 16 * mt + 4 * g + r) = dv[mt][r];
        }
    if (EMIT && em.live && g == 0) em.d(4 * kH) = s0;
    for (int l = 2; l >= 0; --l) {
        const float *W = p + w_off(l + 2);
        f32x4 acc[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            __asm__ volatile("" ::: "memory");
            const float *colp = W + 16 * mt + n;   // column (input feature) 16 mt + n
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(colp[(16 * m2 + 4 * g + r) * kH], dv[m2][r],
                                                                  acc[mt], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dv[mt][r] = acc[mt][r] * L.sp[w][l][4 * mt + r][lane];
                if (EMIT && em.live) em.d(kH * l + 16 * mt + 4 * g + r) = dv[mt][r];
            }
    }
    float gk[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) gk[k] = 0.f;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = 16 * mt + 4 * g + r;
#pragma unroll
            for (int k = 0; k < kIn; ++k) gk[k] = fmaf(Lc.w1[f][k], dv[mt][r], gk[k]);
        }
#pragma unroll
    for (int k = 0; k < kIn; ++k) gu[k] = group_sum(gk[k]) * nm.scale[k];
    return E;
}

// Stages W1, biases and w5 (the FP32 path reads W2..W4 from global memory).
__device__ inline void stage_small(LdsFP32 &L, const float *__restrict__ p) {
    for (int idx = threadIdx.x; idx < kH * 8; idx += blockDim.x) {
        const int o = idx >> 3, k = idx & 7;
        L.w1[o][k] = k < kIn ? p[OFF_W1 + o * kIn + k] : 0.f;
    }
    for (int idx = threadIdx.x; idx < 4 * kH; idx += blockDim.x)
        L.b[idx / kH][idx % kH] = p[b_off(idx / kH + 1) + idx % kH];
    for (int idx = threadIdx.x; idx < kH; idx += blockDim.x) L.w5[idx] = p[OFF_W5 + idx];
    if (threadIdx.x == 0) L.b5 = p[OFF_B5];
}

// Waves per block: the BF16 forward fits two waves per SIMD (<= 256
// registers); the BF16 reverse pass holds the SiLU derivatives of four layers
// in registers and runs one wave per SIMD; the FP32 path keeps them in LDS.
template <bool BF16, int MODE>
struct NNCfg {
    static constexpr int waves = BF16 ? (MODE == 0 ? kNnWaves : 4) : kF32Waves;
};
__host__ __device__ constexpr int nn_threads(bool bf16, int mode) {
    return (bf16 ? (mode == 0 ? kNnWaves : 4) : kF32Waves) * kWave;
}
template <bool BF16>
struct NNLds {
    typedef LdsBF16 T;
};
template <>
struct NNLds<false> {
    typedef LdsFP32 T;
};

// ------------------------------------------- force matching: exact gradient
// The parameter gradient of v . dE/du (v = dloss/dg held fixed, g = dE/du)
// is the parameter gradient of the directional derivative D_v E: carried
// forward as tangents (z'_l = W_l h'_{l-1}, h'_l = s'(z_l) z'_l, h'_0 the
// direction in normalised input units), then differentiated in reverse
// through both chains: with output adjoints delta_5 (primal, the energy loss)
// and alpha (tangent),
//   zt_bar_l = s'(z_l) (.) ht_bar_l,
//   z_bar_l  = s'(z_l) (.) h_bar_l + s''(z_l) z'_l (.) ht_bar_l,
//   h_bar_{l-1} = W_l^T z_bar_l, ht_bar_{l-1} = W_l^T zt_bar_l,
// and dW_l = z_bar_l h_{l-1}^T + zt_bar_l h'_{l-1}^T, db_l = z_bar_l (the
// tangent chain has no bias).  Each sample therefore becomes two rows of the
// weight-gradient GEMMs: the primal row (h_{l-1}, z_bar_l; its energy-loss
// deltas included) and the tangent row (h'_{l-1}, zt_bar_l), which adds to
// the weights but not to the biases.
struct EmitFM {
    float *H = nullptr, *D = nullptr, *R = nullptr;
    int64_t Btot = 0;   // row stride: primal rows 0 .. B1, tangent rows B1 .. 2 B1
    int64_t B1 = 0;
    int64_t b = 0;      // this sample
    bool live = false;
    float y = 0.f;      // normalised label
    float k2 = 0.f;     // 2 / B1: energy-loss seed k2 (e' - y')
    float alpha = 0.f;  // output adjoint of the tangent chain
    __device__ float &hp(int row) const { return H[row * Btot + b]; }
    __device__ float &ht(int row) const { return H[row * Btot + B1 + b]; }
    __device__ float &dp(int row) const { return D[row * Btot + b]; }
    __device__ float &dt(int row) const { return D[row * Btot + B1 + b]; }
};

// Exchange blocks of the tangent chain (four-wave form).
struct WideT {
    bf16x8 a[kWideGroup][kWave];
    bf16x8 dh[kWideGroup][kWave];
    bf16x8 dl[kWideGroup][kWave];
};

// BF16, four waves per 16-row tile (as tile_bf16_wide); u the pair
// descriptor, vt the tangent direction in normalised input units.  The
// output layer is the identity in training (normalised energies).
__device__ inline void tile_bf16_wide_fm(const LdsBF16 &L, WideX &X, WideT &XT, const Norm &nm, const float u[kIn],
                                         const float vt[kIn], int v, const EmitFM &em) {
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
    float un[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) un[k] = (u[k] - nm.shift[k]) * nm.scale[k];
    if (em.live && g == 0 && v == 0)
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            em.hp(k) = un[k];
            em.ht(k) = vt[k];
        }
    bf16x8 act[4], tact[4];
    f16x8 spo[4], cpo[4];   // s'(z_l) and s''(z_l) z'_l of this wave's features
    {
        float h[2][4], d[2][4], th[2][4], c[2][4];
        float x0, x1, t0, t1;
        l1_inputs(un, g, x0, x1);
        l1_inputs(vt, g, t0, t1);
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
            const int mt = 2 * v + mm;
            const f32x4 z = layer1_rows(L.w1, L.b[0], x0, x1, n, g, mt);
            const f32x4 zt = layer1_rows_nobias(L.w1, t0, t1, n, g, mt);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float dd;
                silu2(z[r], h[mm][r], d[mm][r], dd);
                th[mm][r] = d[mm][r] * zt[r];
                c[mm][r] = dd * zt[r];
                if (em.live) {
                    em.hp(kIn + 32 * v + 16 * mm + 4 * g + r) = h[mm][r];
                    em.ht(kIn + 32 * v + 16 * mm + 4 * g + r) = th[mm][r];
                }
            }
        }
        X.a[v][lane] = pack8(h[0], h[1]);
        XT.a[v][lane] = pack8(th[0], th[1]);
        spo[0] = pack8h(d[0], d[1]);
        cpo[0] = pack8h(c[0], c[1]);
    }
    wide_sync();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        act[kb] = X.a[kb][lane];
        tact[kb] = XT.a[kb][lane];
    }
    wide_sync();
    float e = 0.f;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        float h[2][4], d[2][4], th[2][4], c[2][4];
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
            const int mt = 2 * v + mm;
            f32x4 cz = *reinterpret_cast<const f32x4 *>(&L.b[l + 1][16 * mt + 4 * g]);
            f32x4 ct = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&L.w[l][16 * mt + n][wcol(16 * mt + n, 32 * kb + 8 * g)]);
                cz = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, act[kb], cz, 0, 0, 0);
                ct = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, tact[kb], ct, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float dd;
                silu2(cz[r], h[mm][r], d[mm][r], dd);
                th[mm][r] = d[mm][r] * ct[r];
                c[mm][r] = dd * ct[r];
                if (em.live) {
                    em.hp(kIn + kH * (l + 1) + 16 * mt + 4 * g + r) = h[mm][r];
                    em.ht(kIn + kH * (l + 1) + 16 * mt + 4 * g + r) = th[mm][r];
                }
            }
            if (l == 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) e = fmaf(L.w5[16 * mt + 4 * g + r], h[mm][r], e);
            }
        }
        spo[l + 1] = pack8h(d[0], d[1]);
        cpo[l + 1] = pack8h(c[0], c[1]);
        if (l < 2) {
            X.a[v][lane] = pack8(h[0], h[1]);
            XT.a[v][lane] = pack8(th[0], th[1]);
            wide_sync();
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                act[kb] = X.a[kb][lane];
                tact[kb] = XT.a[kb][lane];
            }
            wide_sync();
        }
    }
    e = group_sum(e);
    if (g == 0) X.red[v][0][n] = e;
    wide_sync();
    const float E = ((X.red[0][0][n] + X.red[1][0][n]) + X.red[2][0][n]) + X.red[3][0][n] + L.b5;
    wide_sync();
    const float seed = em.live ? em.k2 * (E - em.y) : 0.f;
    const float alpha = em.live ? em.alpha : 0.f;
    if (em.live && g == 0 && v == 0) {
        em.R[em.b] = E - em.y;
        em.dp(4 * kH) = seed;
        em.dt(4 * kH) = alpha;
    }
    bf16x8 dpk[4], dlk[4], tpk[4], tlk[4];
    {
        float zb[2][4], ztb[2][4];
#pragma unroll
        for (int mm = 0; mm < 2; ++mm)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int f = 32 * v + 16 * mm + 4 * g + r;
                const float w5 = L.w5[f], dd = (float)spo[3][4 * mm + r], cc = (float)cpo[3][4 * mm + r];
                ztb[mm][r] = dd * (alpha * w5);
                zb[mm][r] = fmaf(dd, seed * w5, cc * (alpha * w5));
                if (em.live) {
                    em.dp(3 * kH + f) = zb[mm][r];
                    em.dt(3 * kH + f) = ztb[mm][r];
                }
            }
        bf16x8 hi, lo;
        split8(zb[0], zb[1], hi, lo);
        X.dh[v][lane] = hi;
        X.dl[v][lane] = lo;
        split8(ztb[0], ztb[1], hi, lo);
        XT.dh[v][lane] = hi;
        XT.dl[v][lane] = lo;
    }
    wide_sync();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        dpk[kb] = X.dh[kb][lane];
        dlk[kb] = X.dl[kb][lane];
        tpk[kb] = XT.dh[kb][lane];
        tlk[kb] = XT.dl[kb][lane];
    }
    wide_sync();
#pragma unroll
    for (int l = 2; l >= 0; --l) {
        float zb[2][4], ztb[2][4];
#pragma unroll
        for (int mm = 0; mm < 2; ++mm) {
            const int mt = 2 * v + mm;
            f32x4 c = f32x4{0.f, 0.f, 0.f, 0.f}, ct = c;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x8 a = wt_frag(L, l, kb, mt, lane);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, dpk[kb], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, dlk[kb], c, 0, 0, 0);
                ct = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, tpk[kb], ct, 0, 0, 0);
                ct = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, tlk[kb], ct, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float dd = (float)spo[l][4 * mm + r], cc = (float)cpo[l][4 * mm + r];
                ztb[mm][r] = dd * ct[r];
                zb[mm][r] = fmaf(dd, c[r], cc * ct[r]);
                if (em.live) {
                    em.dp(kH * l + 16 * mt + 4 * g + r) = zb[mm][r];
                    em.dt(kH * l + 16 * mt + 4 * g + r) = ztb[mm][r];
                }
            }
        }
        if (l > 0) {
            bf16x8 hi, lo;
            split8(zb[0], zb[1], hi, lo);
            X.dh[v][lane] = hi;
            X.dl[v][lane] = lo;
            split8(ztb[0], ztb[1], hi, lo);
            XT.dh[v][lane] = hi;
            XT.dl[v][lane] = lo;
            wide_sync();
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                dpk[kb] = X.dh[kb][lane];
                dlk[kb] = X.dl[kb][lane];
                tpk[kb] = XT.dh[kb][lane];
                tlk[kb] = XT.dl[kb][lane];
            }
            wide_sync();
        }
    }
}

// FP32, one wave per 16-row tile (as tile_fp32): weights from global memory,
// s'(z_l) and s''(z_l) z'_l of every layer kept in LDS for the reverse pass.
constexpr int kF32FmWaves = 2;
struct alignas(16) LdsFP32FM {
    float w1[kH][8];
    float b[4][kH];
    float w5[kH];
    float b5;
    float sp[kF32FmWaves][4][32][kWave];
    float cp[kF32FmWaves][4][32][kWave];
};

__device__ inline void tile_fp32_fm(LdsFP32FM &L, const float *__restrict__ p, const Norm &nm, const float u[kIn],
                                    const float vt[kIn], const EmitFM &em) {
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
    const int w = threadIdx.x >> 6;
    float un[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) un[k] = (u[k] - nm.shift[k]) * nm.scale[k];
    if (em.live && g == 0)
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            em.hp(k) = un[k];
            em.ht(k) = vt[k];
        }
    float hv[8][4], tv[8][4];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = 16 * mt + 4 * g + r;
            float z = L.b[0][f], zt = 0.f;
#pragma unroll
            for (int k = 0; k < kIn; ++k) {
                z = fmaf(L.w1[f][k], un[k], z);
                zt = fmaf(L.w1[f][k], vt[k], zt);
            }
            float d, dd;
            silu2(z, hv[mt][r], d, dd);
            tv[mt][r] = d * zt;
            L.sp[w][0][4 * mt + r][lane] = d;
            L.cp[w][0][4 * mt + r][lane] = dd * zt;
            if (em.live) {
                em.hp(kIn + f) = hv[mt][r];
                em.ht(kIn + f) = tv[mt][r];
            }
        }
    for (int l = 0; l < 3; ++l) {
        const float *W = p + w_off(l + 2);
        f32x4 acc[8], tac[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            acc[mt] = *reinterpret_cast<const f32x4 *>(&L.b[l + 1][16 * mt + 4 * g]);
            tac[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            __asm__ volatile("" ::: "memory");
            const float *row = W + (16 * mt + n) * kH + 4 * g;
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2) {
                const float4 a = *reinterpret_cast<const float4 *>(row + 16 * m2);
                const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], hv[m2][r], acc[mt], 0, 0, 0);
                    tac[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], tv[m2][r], tac[mt], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float d, dd;
                silu2(acc[mt][r], hv[mt][r], d, dd);
                tv[mt][r] = d * tac[mt][r];
                L.sp[w][l + 1][4 * mt + r][lane] = d;
                L.cp[w][l + 1][4 * mt + r][lane] = dd * tac[mt][r];
                if (em.live) {
                    em.hp(kIn + kH * (l + 1) + 16 * mt + 4 * g + r) = hv[mt][r];
                    em.ht(kIn + kH * (l + 1) + 16 * mt + 4 * g + r) = tv[mt][r];
                }
            }
    }
    float e = 0.f;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) e = fmaf(L.w5[16 * mt + 4 * g + r], hv[mt][r], e);
    const float E = group_sum(e) + L.b5;
    const float seed = em.live ? em.k2 * (E - em.y) : 0.f;
    const float alpha = em.live ? em.alpha : 0.f;
    if (em.live && g == 0) {
        em.R[em.b] = E - em.y;
        em.dp(4 * kH) = seed;
        em.dt(4 * kH) = alpha;
    }
    // hv, tv now hold the primal and tangent deltas of the current layer
#pragma unroll
    for (int mt = 0; mt < 8; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = 16 * mt + 4 * g + r;
            const float w5 = L.w5[f], d = L.sp[w][3][4 * mt + r][lane], c = L.cp[w][3][4 * mt + r][lane];
            tv[mt][r] = d * (alpha * w5);
            hv[mt][r] = fmaf(d, seed * w5, c * (alpha * w5));
            if (em.live) {
                em.dp(3 * kH + f) = hv[mt][r];
                em.dt(3 * kH + f) = tv[mt][r];
            }
        }
    for (int l = 2; l >= 0; --l) {
        const float *W = p + w_off(l + 2);
        f32x4 acc[8], tac[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
            tac[mt] = acc[mt];
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            __asm__ volatile("" ::: "memory");
            const float *colp = W + 16 * mt + n;
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float a = colp[(16 * m2 + 4 * g + r) * kH];
                    acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, hv[m2][r], acc[mt], 0, 0, 0);
                    tac[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, tv[m2][r], tac[mt], 0, 0, 0);
                }
        }
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float d = L.sp[w][l][4 * mt + r][lane], c = L.cp[w][l][4 * mt + r][lane];
                tv[mt][r] = d * tac[mt][r];
                hv[mt][r] = fmaf(d, acc[mt][r], c * tac[mt][r]);
                if (em.live) {
                    em.dp(kH * l + 16 * mt + 4 * g + r) = hv[mt][r];
                    em.dt(kH * l + 16 * mt + 4 * g + r) = tv[mt][r];
                }
            }
    }
}

// Stages W1, biases and w5 for tile_fp32_fm.
__device__ inline void stage_small_fm(LdsFP32FM &L, const float *__restrict__ p) {
    for (int idx = threadIdx.x; idx < kH * 8; idx += blockDim.x) {
        const int o = idx >> 3, k = idx & 7;
        L.w1[o][k] = k < kIn ? p[OFF_W1 + o * kIn + k] : 0.f;
    }
    for (int idx = threadIdx.x; idx < 4 * kH; idx += blockDim.x)
        L.b[idx / kH][idx % kH] = p[b_off(idx / kH + 1) + idx % kH];
    for (int idx = threadIdx.x; idx < kH; idx += blockDim.x) L.w5[idx] = p[OFF_W5 + idx];
    if (threadIdx.x == 0) L.b5 = p[OFF_B5];
}

}  // namespace rb
