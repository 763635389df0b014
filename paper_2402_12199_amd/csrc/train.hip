// Training step of the energy network: loss mean((e' - y')^2) over a batch
// in normalised units, hand-written reverse pass, weight gradients, Adam
// (Kingma and Ba, ICLR 2015) on the FP32 master parameters.
//
//   k_train_fb     per 16-row tile: forward with the activations h_l and
//                  reverse pass with the deltas dX/dz_l written to the
//                  workspace (feature-major), residuals for the loss
//   k_train_wgrad  per 256-row chunk of the batch: partial weight gradients
//                  dW_l = sum_b delta_l h_{l-1}^T and db_l = sum_b delta_l.
//                  BF16 mode: one block per layer, each an MFMA GEMM over the
//                  chunk with BF16 hi/lo operands staged once in LDS for all
//                  eight waves (the 128 x 7 input layer and the 1 x 128
//                  output layer padded to 16-row tiles), the loss beside the
//                  output layer.  FP32 mode: FP32 MFMA from global memory for
//                  the 128x128 layers, plain sums for the rest
//   k_adam         sums the chunk partials in a fixed order (deterministic)
//                  and applies the Adam update
#include "nn_tile.hpp"

namespace rb {

constexpr int kChunk = 256;
constexpr int kPart = NPARAMS + 1;   // per chunk: gradient, then the loss sum

struct TrainArgs {
    const float *params;
    Norm nm;          // input normalisation; output mapped to identity
    float oshift, oscale;
    int32_t B;        // rows of the weight-gradient GEMMs: B1, or 2 B1 with force matching
    int32_t B1;       // samples; rows 0 .. B1 are their primal rows (the only ones in the
                      // bias gradients and the loss), rows B1 .. 2 B1 their tangent rows
    float k2;         // 2 / B1
    const float *desc;
    int64_t nd;
    const float *labels;
    const int32_t *idx;
    const float *vt;      // force matching: tangent direction per sample (7 x B1, normalised units)
    const float *alpha;   // and the tangent chain's output adjoint (B1)
    float *H, *D, *R, *part;
};

// Sample b of a step: descriptor through idx and normalised label; samples
// past B1 are padding.
__device__ inline void load_row(const TrainArgs &a, int b, Emit &em, float u[kIn]) {
    em.H = a.H;
    em.D = a.D;
    em.R = a.R;
    em.B = a.B;
    em.b = b;
    em.live = b < a.B1;
    em.k2 = a.k2;
    const int64_t pid = em.live ? a.idx[b] : 0;
#pragma unroll
    for (int k = 0; k < kIn; ++k) u[k] = em.live ? a.desc[k * a.nd + pid] : (k == 3 ? 1.f : 0.f);
    em.y = em.live ? (a.labels[pid] - a.oshift) / a.oscale : 0.f;
}

// The same for the force-matching step: both rows of sample b and its
// tangent direction.
__device__ inline void load_row_fm(const TrainArgs &a, int b, EmitFM &em, float u[kIn], float vt[kIn]) {
    em.H = a.H;
    em.D = a.D;
    em.R = a.R;
    em.Btot = a.B;
    em.B1 = a.B1;
    em.b = b;
    em.live = b < a.B1;
    em.k2 = a.k2;
    const int64_t pid = em.live ? a.idx[b] : 0;
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        u[k] = em.live ? a.desc[k * a.nd + pid] : (k == 3 ? 1.f : 0.f);
        vt[k] = em.live ? a.vt[(int64_t)k * a.B1 + b] : 0.f;
    }
    em.y = em.live ? (a.labels[pid] - a.oshift) / a.oscale : 0.f;
    em.alpha = em.live ? a.alpha[b] : 0.f;
}

template <bool BF16>
__global__ __launch_bounds__(nn_threads(BF16, 1)) void k_train_fb(TrainArgs a) {
    constexpr int kWaves = nn_threads(BF16, 1) / kWave;
    __shared__ typename NNLds<BF16>::T L;
    if constexpr (BF16)
        stage_bf16<nn_threads(true, 1)>(L, a.params);
    else
        stage_small(L, a.params);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), n = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntiles = (a.B1 + kTile - 1) / kTile;
    for (int t = blockIdx.x * kWaves + w; t < ntiles; t += gridDim.x * kWaves) {
        __asm__ volatile("" ::: "memory");
        const int b = t * kTile + n;
        Emit em;
        float u[kIn];
        load_row(a, b, em, u);
        float gu[kIn];
        if constexpr (BF16)
            (void)tile_bf16<true, true>(L, a.nm, u, 0.f, gu, em);
        else
            (void)tile_fp32<true, true>(L, L, a.params, a.nm, u, 0.f, gu, em);
    }
}

// BF16 forward + reverse with four waves per 16-row tile (tile_bf16_wide),
// two tiles in flight per block, the block walking the tiles in lockstep.
constexpr int kTrainGroups = 2;
constexpr int kTrainWideThreads = kTrainGroups * kWideGroup * kWave;

__global__ __launch_bounds__(kTrainWideThreads) void k_train_fb_wide(TrainArgs a) {
    __shared__ LdsBF16 L;
    __shared__ WideX X[kTrainGroups];
    stage_bf16<kTrainWideThreads>(L, a.params);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), n = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = wave / kWideGroup, v = wave % kWideGroup;
    const int ntiles = (a.B1 + kTile - 1) / kTile;
    for (int base = blockIdx.x * kTrainGroups; base < ntiles; base += gridDim.x * kTrainGroups) {
        const int b = (base + grp) * kTile + n;
        Emit em;
        float u[kIn];
        load_row(a, b, em, u);
        float gu[kIn];
        (void)tile_bf16_wide<true, true>(L, X[grp], a.nm, u, 0.f, gu, v, em);
    }
}

// Force matching, BF16: one four-wave group per block (the tangent chain's
// exchange blocks take the LDS a second group would use), tiles of 16
// samples, each emitting its primal and tangent rows.
__global__ __launch_bounds__(kWideGroup * kWave) void k_train_fb_fm_wide(TrainArgs a) {
    __shared__ LdsBF16 L;
    __shared__ WideX X;
    __shared__ WideT XT;
    stage_bf16<kWideGroup * kWave>(L, a.params);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), n = lane & 15;
    const int v = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntiles = (a.B1 + kTile - 1) / kTile;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        EmitFM em;
        float u[kIn], vt[kIn];
        load_row_fm(a, t * kTile + n, em, u, vt);
        tile_bf16_wide_fm(L, X, XT, a.nm, u, vt, v, em);
    }
}

// Force matching, FP32: one wave per tile of 16 samples.
__global__ __launch_bounds__(kF32FmWaves * kWave) void k_train_fb_fm_fp32(TrainArgs a) {
    __shared__ LdsFP32FM L;
    stage_small_fm(L, a.params);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), n = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntiles = (a.B1 + kTile - 1) / kTile;
    for (int t = blockIdx.x * kF32FmWaves + w; t < ntiles; t += gridDim.x * kF32FmWaves) {
        __asm__ volatile("" ::: "memory");
        EmitFM em;
        float u[kIn], vt[kIn];
        load_row_fm(a, t * kTile + n, em, u, vt);
        tile_fp32_fm(L, a.params, a.nm, u, vt, em);
    }
}

// FP32 mode, edge block of a chunk: dW1 (128 x 7), db1, dW5, db5 and the loss sum, one
// dot product over the chunk per output (lanes stride over the rows), with
// the chunk's 7 input rows and the output delta staged in LDS.
__device__ void wgrad_edge(const TrainArgs &a, int r0, int nr, float *part, float (*E)[kChunk]) {
    const int64_t B = a.B;
    for (int i = threadIdx.x; i < 8 * nr; i += blockDim.x) {
        const int row = i / nr, col = i - row * nr;
        E[row][col] = (row < kIn ? a.H + (int64_t)row * B : a.D + (int64_t)(4 * kH) * B)[r0 + col];
    }
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    constexpr int kPer = kChunk / kWave;
    for (int f = w; f < kH; f += nw) {
        // dW1[f][:], db1[f]
        const float *d1 = a.D + (int64_t)f * B + r0;
        float dv[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) dv[q] = lane + kWave * q < nr ? d1[lane + kWave * q] : 0.f;
        float s[kIn + 1];
#pragma unroll
        for (int k = 0; k <= kIn; ++k) s[k] = 0.f;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int b = lane + kWave * q;
            if (b < nr) {
#pragma unroll
                for (int k = 0; k < kIn; ++k) s[k] = fmaf(dv[q], E[k][b], s[k]);
            }
            if (r0 + b < a.B1) s[kIn] += dv[q];    // primal rows only: the tangent chain has no bias
        }
#pragma unroll
        for (int k = 0; k <= kIn; ++k) s[k] = wave_sum(s[k]);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < kIn; ++k) part[OFF_W1 + f * kIn + k] = s[k];
            part[OFF_B1 + f] = s[kIn];
        }
        // dW5[f] = sum_b delta_5 h_4[f]
        const float *h4 = a.H + (int64_t)(kIn + 3 * kH + f) * B + r0;
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int b = lane + kWave * q;
            if (b < nr) t = fmaf(E[kIn][b], h4[b], t);
        }
        t = wave_sum(t);
        if (lane == 0) part[OFF_W5 + f] = t;
    }
    if (w == 0) {
        float s5 = 0.f, l = 0.f;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int b = lane + kWave * q;
            if (b < nr && r0 + b < a.B1) {
                s5 += E[kIn][b];
                const float r = a.R[r0 + b];
                l = fmaf(r, r, l);
            }
        }
        s5 = wave_sum(s5);
        l = wave_sum(l);
        if (lane == 0) {
            part[OFF_B5] = s5;
            part[NPARAMS] = l;
        }
    }
}

// BF16 mode: dW (ma x nb, row stride ldw) = sum over the chunk's rows b of
// A[:, b] B[:, b]^T for feature-major A (ma <= 128 rows) and B (nb <= 128
// rows), and optionally db = sum_b A[:, b].  Per 32-row step every thread
// loads eight consecutive batch entries of one feature row of A and of B:
// exactly the MFMA operand fragment of one lane of one 16-row tile, so it is
// split into BF16 hi/lo once and stored in LDS in fragment order (rows past
// ma or nb as zeros; double-buffered, one barrier per step; the next step's
// global loads are in flight during the MFMAs).  Wave w computes the 4 x 2
// output tiles rows 64 (w / 4) .., columns 32 (w % 4) .., skipping tiles
// outside ma x nb.
__device__ __attribute__((always_inline)) inline void wgrad_gemm_bf16(const float *Ar, int ma, const float *Br, int nb,
                                                                    int64_t B, int r0, int r1,
                                                                    float *dW, int ldw, float *db, int bias_end,
                                                                    bf16x8 *S) {
    const int t = threadIdx.x, f = t >> 2, p = t & 3;
    const bool va = f < ma, vb = f < nb;
    const float *arow = Ar + (int64_t)(va ? f : 0) * B + 8 * p;
    const float *brow = Br + (int64_t)(vb ? f : 0) * B + 8 * p;
    // fragment slot of this thread's data: tile f / 16, lane 16 p + f % 16
    const int slot = (f >> 4) * kWave + 16 * p + (f & 15);
    constexpr int kOp = 8 * kWave;   // one operand half (hi or lo) of 8 tiles
    constexpr int kBuf = 4 * kOp;    // A hi, A lo, B hi, B lo
    const int lane = t & (kWave - 1), w = t >> 6, g = lane >> 4, n = lane & 15;
    const int mt0 = 4 * (w >> 2), nt0 = 2 * (w & 3);
    const int mtn = min(4, (ma + 15) / 16 - mt0), ntn = min(2, (nb + 15) / 16 - nt0);   // tiles of this wave
    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const float4 z4 = {0.f, 0.f, 0.f, 0.f};
    float4 a0 = z4, a1 = z4, b0 = z4, b1 = z4;
    if (va) {
        a0 = *reinterpret_cast<const float4 *>(arow + r0);
        a1 = *reinterpret_cast<const float4 *>(arow + r0 + 4);
    }
    if (vb) {
        b0 = *reinterpret_cast<const float4 *>(brow + r0);
        b1 = *reinterpret_cast<const float4 *>(brow + r0 + 4);
    }
    float dsum = 0.f;
    for (int k0 = r0, buf = 0; k0 < r1; k0 += 32, buf ^= 1) {
        bf16x8 *Sb = S + buf * kBuf;
        {
            const float av0[4] = {a0.x, a0.y, a0.z, a0.w}, av1[4] = {a1.x, a1.y, a1.z, a1.w};
            const float bv0[4] = {b0.x, b0.y, b0.z, b0.w}, bv1[4] = {b1.x, b1.y, b1.z, b1.w};
            if (k0 < bias_end) {   // 32-row steps lie wholly before or after it (multiples of 32)
#pragma unroll
                for (int r = 0; r < 4; ++r) dsum += av0[r];
#pragma unroll
                for (int r = 0; r < 4; ++r) dsum += av1[r];
            }
            bf16x8 hi, lo;
            split8(av0, av1, hi, lo);
            Sb[slot] = hi;
            Sb[kOp + slot] = lo;
            split8(bv0, bv1, hi, lo);
            Sb[2 * kOp + slot] = hi;
            Sb[3 * kOp + slot] = lo;
        }
        __syncthreads();
        if (k0 + 32 < r1) {
            if (va) {
                a0 = *reinterpret_cast<const float4 *>(arow + k0 + 32);
                a1 = *reinterpret_cast<const float4 *>(arow + k0 + 36);
            }
            if (vb) {
                b0 = *reinterpret_cast<const float4 *>(brow + k0 + 32);
                b1 = *reinterpret_cast<const float4 *>(brow + k0 + 36);
            }
        }
        if (mtn > 0 && ntn > 0) {
            bf16x8 Bh[2], Bl[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                Bh[j] = Sb[2 * kOp + (nt0 + j) * kWave + lane];
                Bl[j] = Sb[3 * kOp + (nt0 + j) * kWave + lane];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i >= mtn) break;
                const bf16x8 Ah = Sb[(mt0 + i) * kWave + lane], Al = Sb[kOp + (mt0 + i) * kWave + lane];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    if (j >= ntn) break;
                    // three BF16 passes: hi*hi + hi*lo + lo*hi (lo*lo is below FP32 rounding)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, Bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh[j], acc[i][j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * (mt0 + i) + 4 * g + r, col = 16 * (nt0 + j) + n;
                if (i < mtn && j < ntn && row < ma && col < nb) dW[row * ldw + col] = acc[i][j][r];
            }
    if (db) {
        // the four threads of row f are adjacent lanes
        dsum += __shfl_xor(dsum, 1, kWave);
        dsum += __shfl_xor(dsum, 2, kWave);
        if (p == 0 && va) db[f] = dsum;
    }
}

// BF16 mode, block y of a chunk: 0..2 the 128x128 layers 2..4 (dW_l, db_l);
// 3 the input layer (dW1 = delta_1 u^T, db1); 4 the output layer
// (dW5 = delta_5 h_4^T, db5) and the chunk's loss
__device__ void wgrad_block_bf16(const TrainArgs &a, int y, int r0, int r1, float *part, bf16x8 *S) {
    const int64_t B = a.B;
    if (y < 3) {
        const int layer = y + 2;
        wgrad_gemm_bf16(a.D + (int64_t)kH * (layer - 1) * B, kH, a.H + (int64_t)(kIn + kH * (layer - 2)) * B, kH, B,
                        r0, r1, part + w_off(layer), kH, part + b_off(layer), a.B1, S);
    } else if (y == 3) {
        wgrad_gemm_bf16(a.D, kH, a.H, kIn, B, r0, r1, part + OFF_W1, kIn, part + OFF_B1, a.B1, S);
    } else {
        if (threadIdx.x < kWave) {
            const int lane = threadIdx.x;
            float rv[kChunk / kWave], l = 0.f;
#pragma unroll
            for (int q = 0; q < kChunk / kWave; ++q) {
                const int b = r0 + lane + kWave * q;
                rv[q] = b < r1 && b < a.B1 ? a.R[b] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < kChunk / kWave; ++q) l = fmaf(rv[q], rv[q], l);
            l = wave_sum(l);
            if (lane == 0) part[NPARAMS] = l;
        }
        wgrad_gemm_bf16(a.D + (int64_t)(4 * kH) * B, 1, a.H + (int64_t)(kIn + 3 * kH) * B, kH, B, r0, r1,
                        part + OFF_W5, kH, part + OFF_B5, a.B1, S);
    }
}

// FP32 mode, one 128x128 layer over one chunk: FP32 MFMA straight from
// global memory, wave w owns the 16-row tile w of dW_l and of db_l.
__device__ void wgrad_layer_fp32(const TrainArgs &a, int layer, int r0, int r1, float *part) {
    const int64_t B = a.B;
    const float *Dl = a.D + (int64_t)kH * (layer - 1) * B;
    const float *Hl = a.H + (int64_t)(kIn + kH * (layer - 2)) * B;
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
    const int mt = threadIdx.x >> 6;
    f32x4 acc[8];
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    float dsum = 0.f;
    for (int k0 = r0; k0 < r1; k0 += 4) {
        const float A = Dl[(int64_t)(16 * mt + n) * B + k0 + g];
        if (k0 + g < a.B1) dsum += A;
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A, Hl[(int64_t)(16 * nt + n) * B + k0 + g], acc[nt], 0, 0,
                                                          0);
    }
    float *dW = part + w_off(layer);
#pragma unroll
    for (int nt = 0; nt < 8; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) dW[(16 * mt + 4 * g + r) * kH + 16 * nt + n] = acc[nt][r];
    dsum = group_sum(dsum);
    if (g == 0) part[b_off(layer) + 16 * mt + n] = dsum;
}

// grid (chunks, 5) in BF16 mode (blocks as in wgrad_block_bf16), (chunks, 4)
// in FP32 mode: blockIdx.y 0..2 = layers 2..4, 3 = edge block
template <bool BF16>
__global__ __launch_bounds__(512) void k_train_wgrad(TrainArgs a) {
    __shared__ __align__(16) bf16x8 S[2 * 4 * 8 * kWave];   // 64 KiB
    const int c = blockIdx.x;
    const int r0 = c * kChunk;
    const int r1 = min(a.B, r0 + kChunk);
    float *part = a.part + (int64_t)c * kPart;
    if constexpr (BF16) {
        wgrad_block_bf16(a, blockIdx.y, r0, r1, part, S);
    } else if (blockIdx.y == 3) {
        static_assert(sizeof(S) >= sizeof(float) * 8 * kChunk, "edge staging fits the operand buffer");
        wgrad_edge(a, r0, r1 - r0, part, reinterpret_cast<float (*)[kChunk]>(S));
    } else {
        wgrad_layer_fp32(a, blockIdx.y + 2, r0, r1, part);
    }
}

// Sum of n partials base[c * stride], c = 0 .. n - 1, added in order c = 0,
// 1, ...; the loads are issued 32 (then 4) at a time so that at most a few
// memory round trips are paid.
__device__ inline float ordered_sum(const float *__restrict__ base, int n, int64_t stride) {
    float s = 0.f;
    int c = 0;
    for (; c + 32 <= n; c += 32) {
        float v[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) v[k] = base[(int64_t)(c + k) * stride];
#pragma unroll
        for (int k = 0; k < 32; ++k) s += v[k];
    }
    for (; c + 4 <= n; c += 4) {
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = base[(int64_t)(c + k) * stride];
#pragma unroll
        for (int k = 0; k < 4; ++k) s += v[k];
    }
    for (; c < n; ++c) s += base[(int64_t)c * stride];
    return s;
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ part, int nchunks, float lr, float b1, float b2, float eps, float c1,
                       float c2, float invB, float *__restrict__ loss, float *__restrict__ grad_out,
                       const float *__restrict__ fmpart, int nfm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    // the losses are summed by one thread of the last block (the one with
    // the fewest parameters)
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1) {
        loss[0] = ordered_sum(part + NPARAMS, nchunks, kPart) * invB;
        if (fmpart) loss[1] = ordered_sum(fmpart, nfm, 1);
    }
    if (i >= NPARAMS) return;
    // chunk partials summed in chunk order
    const float g = ordered_sum(part + i, nchunks, kPart);
    if (grad_out) grad_out[i] = g;
    const float mi = fmaf(b1, m[i], (1.f - b1) * g);
    const float vi = fmaf(b2, v[i], (1.f - b2) * g * g);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ------------------------------------------------ force/torque matching
// The loss adds lam_f mean |F_j - F_j*|^2 + lam_t mean |tau_j - tau_j*|^2,
// where F_j = -g_d and tau_j = -(w g_v - g_w v + v x g_v) / 2 come from the
// network's input gradient g = dE/du (pair descriptors u = (d, q), q =
// (w, v)).  Its parameter gradient is sum_b v_b . dg_b/dtheta with
// v_b = dL/dg_b (linear in the errors), i.e. the parameter gradient of the
// directional derivative of E along v_b, which the tangent rows of the
// training kernels carry exactly (tile_bf16_wide_fm, tile_fp32_fm): the
// direction in normalised input units is (v_b / |v_b|) (.) in_scale and the
// tangent chain's output adjoint out_scale |v_b| (E = out_scale e' + ...).

constexpr int kFmThreads = 256;

__global__ void k_fm_gather(int32_t B1, const float *__restrict__ desc, int64_t nd, const int32_t *__restrict__ idx,
                            float *__restrict__ descb) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B1) return;
    const int64_t pid = idx[b];
#pragma unroll
    for (int k = 0; k < kIn; ++k) descb[(int64_t)k * B1 + b] = desc[k * nd + pid];
}

// Per sample: the force and torque errors, the loss term, v = dL/dg, the
// tangent direction and its output adjoint; per-block loss partials.
__global__ __launch_bounds__(kFmThreads) void k_fm_rows(int32_t B1, const float *__restrict__ descb,
                                                        const float *__restrict__ gb,
                                                        const float *__restrict__ ft_labels, int64_t nd,
                                                        const int32_t *__restrict__ idx, float lam_f, float lam_t,
                                                        Norm nm, float *__restrict__ vt, float *__restrict__ alpha,
                                                        float *__restrict__ fmpart) {
    __shared__ float red[kFmThreads / kWave];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    float lsum = 0.f;
    if (b < B1) {
        float u[kIn], g[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            u[k] = descb[(int64_t)k * B1 + b];
            g[k] = gb[(int64_t)k * B1 + b];
        }
        const float w = u[3], vx = u[4], vy = u[5], vz = u[6];
        const float gw = g[3], gx = g[4], gy = g[5], gz = g[6];
        const float F[3] = {-g[0], -g[1], -g[2]};
        const float T[3] = {-0.5f * (w * gx - gw * vx + (vy * gz - vz * gy)),
                            -0.5f * (w * gy - gw * vy + (vz * gx - vx * gz)),
                            -0.5f * (w * gz - gw * vz + (vx * gy - vy * gx))};
        const int64_t pid = idx[b];
        float dF[3], dT[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dF[a] = F[a] - ft_labels[a * nd + pid];
            dT[a] = T[a] - ft_labels[(3 + a) * nd + pid];
            lsum += lam_f * dF[a] * dF[a] + lam_t * dT[a] * dT[a];
        }
        lsum /= (float)B1;
        const float cf = 2.f * lam_f / (float)B1, ct = 2.f * lam_t / (float)B1;
        const float wF[3] = {cf * dF[0], cf * dF[1], cf * dF[2]}, wT[3] = {ct * dT[0], ct * dT[1], ct * dT[2]};
        // v = dL/dg: F_j = -g_d; tau_j as above (w_T x v_q from the cross product)
        float v[kIn];
        v[0] = -wF[0];
        v[1] = -wF[1];
        v[2] = -wF[2];
        v[3] = 0.5f * (wT[0] * vx + wT[1] * vy + wT[2] * vz);
        v[4] = -0.5f * (w * wT[0] + (wT[1] * vz - wT[2] * vy));
        v[5] = -0.5f * (w * wT[1] + (wT[2] * vx - wT[0] * vz));
        v[6] = -0.5f * (w * wT[2] + (wT[0] * vy - wT[1] * vx));
        float nv2 = 0.f;
#pragma unroll
        for (int k = 0; k < kIn; ++k) nv2 += v[k] * v[k];
        const float nv = sqrtf(nv2), inv = nv > 0.f ? 1.f / nv : 0.f;
#pragma unroll
        for (int k = 0; k < kIn; ++k) vt[(int64_t)k * B1 + b] = v[k] * inv * nm.scale[k];
        alpha[b] = nm.oscale * nv;
    }
    lsum = wave_sum(lsum);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < kFmThreads / kWave; ++k) t += red[k];
        fmpart[blockIdx.x] = t;
    }
}

struct TrainLayout {
    size_t H, D, R, part, total;
};

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

static TrainLayout train_layout(int32_t B) {
    TrainLayout t;
    const int nchunks = (B + kChunk - 1) / kChunk;
    size_t o = 0;
    t.H = o; o += al(sizeof(float) * (size_t)kHRows * B);
    t.D = o; o += al(sizeof(float) * (size_t)kDRows * B);
    t.R = o; o += al(sizeof(float) * (size_t)B);
    t.part = o; o += al(sizeof(float) * (size_t)kPart * nchunks);
    t.total = o;
    return t;
}


// Forward/reverse, weight gradients and Adam over the rows of `a` (a.B1
// samples; with a.vt set, each sample's primal and tangent rows, and fmpart
// (nfm partials) adds the matching loss to loss[1]).
static void train_launch(TrainArgs &a, int precision, float *params, float *adam_m, float *adam_v, int32_t t,
                         float lr, float beta1, float beta2, float eps, float *loss, float *grad_out,
                         const float *fmpart, int nfm, hipStream_t st) {
    const int ntiles = (a.B1 + kTile - 1) / kTile;
    const int cus = device_cu_count();
    if (a.vt) {
        if (precision == RB_PREC_BF16)
            k_train_fb_fm_wide<<<grid_for(ntiles, 1, cus), kWideGroup * kWave, 0, st>>>(a);
        else
            k_train_fb_fm_fp32<<<grid_for(ntiles, kF32FmWaves, cus), kF32FmWaves * kWave, 0, st>>>(a);
    } else if (precision == RB_PREC_BF16) {
        k_train_fb_wide<<<grid_for(ntiles, kTrainGroups, cus), kTrainWideThreads, 0, st>>>(a);
    } else {
        constexpr int wv = nn_threads(false, 1) / kWave;
        k_train_fb<false><<<grid_for(ntiles, wv, cus), wv * kWave, 0, st>>>(a);
    }
    const int nchunks = (a.B + kChunk - 1) / kChunk;
    if (precision == RB_PREC_BF16)
        k_train_wgrad<true><<<dim3(nchunks, 5), 512, 0, st>>>(a);
    else
        k_train_wgrad<false><<<dim3(nchunks, 4), 512, 0, st>>>(a);
    const double c1 = 1.0 / (1.0 - pow((double)beta1, (double)t));
    const double c2 = 1.0 / (1.0 - pow((double)beta2, (double)t));
    k_adam<<<(NPARAMS + 255) / 256, 256, 0, st>>>(params, adam_m, adam_v, a.part, nchunks, lr, beta1, beta2, eps,
                                                   (float)c1, (float)c2, 1.f / (float)a.B1, loss, grad_out, fmpart,
                                                   nfm);
}

static TrainArgs train_args(float *params, const float *norm, const float *desc, int64_t n_data,
                            const float *labels, const int32_t *idx, int32_t rows, int32_t batch, char *w,
                            const TrainLayout &Lw) {
    TrainArgs a;
    a.params = params;
    a.nm = norm_from_host(norm);
    a.oshift = a.nm.oshift;
    a.oscale = a.nm.oscale;
    a.nm.oshift = 0.f;
    a.nm.oscale = 1.f;
    a.B = rows;
    a.B1 = batch;
    a.k2 = 2.f / (float)batch;
    a.desc = desc;
    a.nd = n_data;
    a.labels = labels;
    a.idx = idx;
    a.vt = nullptr;
    a.alpha = nullptr;
    a.H = reinterpret_cast<float *>(w + Lw.H);
    a.D = reinterpret_cast<float *>(w + Lw.D);
    a.R = reinterpret_cast<float *>(w + Lw.R);
    a.part = reinterpret_cast<float *>(w + Lw.part);
    return a;
}

// Workspace of the matching step: the training rows (2 per sample), then the
// gathered descriptors, their input gradients, the tangent directions, their
// output adjoints and the loss partials.
struct FmLayout {
    TrainLayout tr;
    size_t descb, gb, vt, alpha, fmpart, total;
};

static FmLayout fm_layout(int32_t batch) {
    FmLayout f;
    f.tr = train_layout(2 * batch);
    size_t o = f.tr.total;
    f.descb = o; o += al(sizeof(float) * (size_t)kIn * batch);
    f.gb = o; o += al(sizeof(float) * (size_t)kIn * batch);
    f.vt = o; o += al(sizeof(float) * (size_t)kIn * batch);
    f.alpha = o; o += al(sizeof(float) * (size_t)batch);
    f.fmpart = o; o += al(sizeof(float) * (size_t)((batch + kFmThreads - 1) / kFmThreads));
    f.total = o;
    return f;
}

}  // namespace rb

using namespace rb;

extern "C" size_t rb_nn_train_workspace_bytes(int32_t batch) {
    if (batch <= 0 || batch % 32 != 0 || batch > (1 << 20)) return 0;
    return train_layout(batch).total;
}

extern "C" size_t rb_nn_train_fm_workspace_bytes(int32_t batch) {
    if (batch <= 0 || batch % 32 != 0 || batch > (1 << 18)) return 0;
    return fm_layout(batch).total;
}

extern "C" int rb_nn_train_step(float *params, float *adam_m, float *adam_v, int32_t t, const float *norm,
                                int precision, int32_t batch, const float *desc, int64_t n_data,
                                const float *labels, const int32_t *idx, float lr, float beta1, float beta2,
                                float eps, float *loss, float *grad_out, void *ws, size_t ws_bytes, void *stream) {
    RB_REQUIRE(params && adam_m && adam_v && norm && desc && labels && idx && loss && ws,
               "rb_nn_train_step: null argument");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_train_step: bad precision");
    RB_REQUIRE(batch > 0 && batch % 32 == 0 && batch <= (1 << 20),
               "rb_nn_train_step: batch must be a positive multiple of 32, at most 2^20");
    RB_REQUIRE(n_data > 0 && t >= 1, "rb_nn_train_step: n_data > 0 and t >= 1 required");
    const TrainLayout Lw = train_layout(batch);
    RB_REQUIRE(ws_bytes >= Lw.total, "rb_nn_train_step: workspace too small (%zu < %zu)", ws_bytes, Lw.total);
    TrainArgs a = train_args(params, norm, desc, n_data, labels, idx, batch, batch, static_cast<char *>(ws), Lw);
    train_launch(a, precision, params, adam_m, adam_v, t, lr, beta1, beta2, eps, loss, grad_out, nullptr, 0,
                 (hipStream_t)stream);
    RB_LAUNCH_CHECK("rb_nn_train_step");
    return RB_OK;
}

extern "C" int rb_nn_train_step_fm(float *params, float *adam_m, float *adam_v, int32_t t, const float *norm,
                                   int precision, int32_t batch, const float *desc, int64_t n_data,
                                   const float *labels, const float *ft_labels, const int32_t *idx, float lam_f,
                                   float lam_t, float lr, float beta1, float beta2, float eps, float *loss,
                                   float *grad_out, void *ws, size_t ws_bytes, void *stream) {
    RB_REQUIRE(params && adam_m && adam_v && norm && desc && labels && ft_labels && idx && loss && ws,
               "rb_nn_train_step_fm: null argument");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_train_step_fm: bad precision");
    RB_REQUIRE(batch > 0 && batch % 32 == 0 && batch <= (1 << 18),
               "rb_nn_train_step_fm: batch must be a positive multiple of 32, at most 2^18");
    RB_REQUIRE(n_data > 0 && t >= 1, "rb_nn_train_step_fm: n_data > 0 and t >= 1 required");
    RB_REQUIRE(lam_f >= 0.f && lam_t >= 0.f, "rb_nn_train_step_fm: lam >= 0 required");
    const FmLayout F = fm_layout(batch);
    RB_REQUIRE(ws_bytes >= F.total, "rb_nn_train_step_fm: workspace too small (%zu < %zu)", ws_bytes, F.total);
    char *w = static_cast<char *>(ws);
    hipStream_t st = (hipStream_t)stream;
    float *descb = reinterpret_cast<float *>(w + F.descb), *gb = reinterpret_cast<float *>(w + F.gb);
    float *vt = reinterpret_cast<float *>(w + F.vt), *alpha = reinterpret_cast<float *>(w + F.alpha);
    float *fmpart = reinterpret_cast<float *>(w + F.fmpart);
    const int nblk = (batch + kFmThreads - 1) / kFmThreads;
    k_fm_gather<<<nblk, kFmThreads, 0, st>>>(batch, desc, n_data, idx, descb);
    const int rc = rb_nn_pair_grad(params, norm, precision, batch, descb, nullptr, nullptr, gb, nullptr, stream);
    if (rc != RB_OK) return rc;
    k_fm_rows<<<nblk, kFmThreads, 0, st>>>(batch, descb, gb, ft_labels, n_data, idx, lam_f, lam_t,
                                           norm_from_host(norm), vt, alpha, fmpart);
    TrainArgs a = train_args(params, norm, desc, n_data, labels, idx, 2 * batch, batch, w, F.tr);
    a.vt = vt;
    a.alpha = alpha;
    train_launch(a, precision, params, adam_m, adam_v, t, lr, beta1, beta2, eps, loss, grad_out, fmpart, nblk, st);
    RB_LAUNCH_CHECK("rb_nn_train_step_fm");
    return RB_OK;
}
