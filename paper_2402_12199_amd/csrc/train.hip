// Training step of the energy network: loss mean((e' - y')^2) over a batch
// in normalised units, hand-written reverse pass, weight gradients, Adam
// (Kingma and Ba, ICLR 2015) on the FP32 master parameters.
//
//   k_train_fb     per 16-row tile: forward with the activations h_l and
//                  reverse pass with the deltas dX/dz_l written to the
//                  workspace (feature-major), residuals for the loss
//   k_train_wgrad  per 512-row chunk of the batch: partial weight gradients.
//                  dW_l = sum_b delta_l h_{l-1}^T for the three 128x128
//                  layers as MFMA GEMMs over the batch (BF16 operands in the
//                  BF16 mode, FP32 otherwise), the FP32 layers (W1, W5) and
//                  the biases as plain sums, and the chunk's loss
//   k_adam         sums the chunk partials in a fixed order (deterministic)
//                  and applies the Adam update
#include "nn_tile.hpp"

namespace rb {

constexpr int kChunk = 256;
constexpr int kSmallBlocks = 8;   // blocks per chunk for the FP32 layers, biases and loss
constexpr int kPart = NPARAMS + 1;   // per chunk: gradient, then the loss sum

struct TrainArgs {
    const float *params;
    Norm nm;          // input normalisation; output mapped to identity
    float oshift, oscale;
    int32_t B;
    const float *desc;
    int64_t nd;
    const float *labels;
    const int32_t *idx;
    float *H, *D, *R, *part;
};

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
    const int ntiles = (a.B + kTile - 1) / kTile;
    for (int t = blockIdx.x * kWaves + w; t < ntiles; t += gridDim.x * kWaves) {
        __asm__ volatile("" ::: "memory");
        const int b = t * kTile + n;
        Emit em;
        em.H = a.H;
        em.D = a.D;
        em.R = a.R;
        em.B = a.B;
        em.b = b;
        em.live = b < a.B;
        em.k2 = 2.f / (float)a.B;
        const int64_t pid = em.live ? a.idx[b] : 0;
        float u[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) u[k] = em.live ? a.desc[k * a.nd + pid] : (k == 3 ? 1.f : 0.f);
        em.y = em.live ? (a.labels[pid] - a.oshift) / a.oscale : 0.f;
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
    const int ntiles = (a.B + kTile - 1) / kTile;
    for (int base = blockIdx.x * kTrainGroups; base < ntiles; base += gridDim.x * kTrainGroups) {
        const int b = (base + grp) * kTile + n;
        Emit em;
        em.H = a.H;
        em.D = a.D;
        em.R = a.R;
        em.B = a.B;
        em.b = b;
        em.live = b < a.B;
        em.k2 = 2.f / (float)a.B;
        const int64_t pid = em.live ? a.idx[b] : 0;
        float u[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) u[k] = em.live ? a.desc[k * a.nd + pid] : (k == 3 ? 1.f : 0.f);
        em.y = em.live ? (a.labels[pid] - a.oshift) / a.oscale : 0.f;
        float gu[kIn];
        (void)tile_bf16_wide<true, true>(L, X[grp], a.nm, u, 0.f, gu, v, em);
    }
}

template <bool BF16>
__global__ __launch_bounds__(512) void k_train_wgrad(TrainArgs a) {
    const int c = blockIdx.x;
    const int r0 = c * kChunk;
    const int r1 = min(a.B, r0 + kChunk);
    const int64_t B = a.B;
    float *part = a.part + (int64_t)c * kPart;
    if (blockIdx.y < 3) {
        const int layer = blockIdx.y + 2;
        const float *Dl = a.D + (int64_t)kH * (layer - 1) * B;
        const float *Hl = a.H + (int64_t)(kIn + kH * (layer - 2)) * B;
        const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
        const int mt = threadIdx.x >> 6;   // 8 waves: one 16-row tile of dW each
        f32x4 acc[8];
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (BF16) {
            for (int k0 = r0; k0 < r1; k0 += 32) {
                const float *ap = Dl + (int64_t)(16 * mt + n) * B + k0 + 8 * g;
                const float4 a0 = *reinterpret_cast<const float4 *>(ap);
                const float4 a1 = *reinterpret_cast<const float4 *>(ap + 4);
                const float av0[4] = {a0.x, a0.y, a0.z, a0.w}, av1[4] = {a1.x, a1.y, a1.z, a1.w};
                bf16x8 Ahi, Alo;
                split8(av0, av1, Ahi, Alo);
#pragma unroll
                for (int nt = 0; nt < 8; ++nt) {
                    const float *bp = Hl + (int64_t)(16 * nt + n) * B + k0 + 8 * g;
                    const float4 b0 = *reinterpret_cast<const float4 *>(bp);
                    const float4 b1 = *reinterpret_cast<const float4 *>(bp + 4);
                    const float bv0[4] = {b0.x, b0.y, b0.z, b0.w}, bv1[4] = {b1.x, b1.y, b1.z, b1.w};
                    bf16x8 Bhi, Blo;
                    split8(bv0, bv1, Bhi, Blo);
                    // three BF16 passes: hi*hi + hi*lo + lo*hi (the lo*lo term is below FP32 rounding)
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi, Bhi, acc[nt], 0, 0, 0);
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi, Blo, acc[nt], 0, 0, 0);
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Alo, Bhi, acc[nt], 0, 0, 0);
                }
            }
        } else {
            for (int k0 = r0; k0 < r1; k0 += 4) {
                const float A = Dl[(int64_t)(16 * mt + n) * B + k0 + g];
#pragma unroll
                for (int nt = 0; nt < 8; ++nt)
                    acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A, Hl[(int64_t)(16 * nt + n) * B + k0 + g], acc[nt],
                                                                  0, 0, 0);
            }
        }
        float *dW = part + w_off(layer);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) dW[(16 * mt + 4 * g + r) * kH + 16 * nt + n] = acc[nt][r];
    } else {
        // FP32 layers, biases and the loss: one dot product over the chunk
        // per wave (lanes stride over the rows, coalesced), spread over
        // kSmallBlocks blocks
        const int lane = threadIdx.x & (kWave - 1);
        const int wpb = blockDim.x / kWave;
        const int nw = kSmallBlocks * wpb;
        const int nsmall = kH * kIn + 4 * kH + kH + 2;
        for (int j = (blockIdx.y - 3) * wpb + (threadIdx.x >> 6); j < nsmall; j += nw) {
            const float *x = nullptr, *y = nullptr;
            int dst;
            if (j < kH * kIn) {                       // dW1[f][k]
                const int f = j / kIn, k = j % kIn;
                x = a.D + (int64_t)f * B;
                y = a.H + (int64_t)k * B;
                dst = OFF_W1 + j;
            } else if (j < kH * kIn + 4 * kH) {       // db_l
                const int jj = j - kH * kIn, l = jj / kH + 1, f = jj % kH;
                x = a.D + (int64_t)(kH * (l - 1) + f) * B;
                dst = b_off(l) + f;
            } else if (j < kH * kIn + 5 * kH) {       // dW5[f]
                const int f = j - kH * kIn - 4 * kH;
                x = a.D + (int64_t)(4 * kH) * B;
                y = a.H + (int64_t)(kIn + 3 * kH + f) * B;
                dst = OFF_W5 + f;
            } else if (j == kH * kIn + 5 * kH) {      // db5
                x = a.D + (int64_t)(4 * kH) * B;
                dst = OFF_B5;
            } else {                                  // loss: sum of squared residuals
                x = a.R;
                y = a.R;
                dst = NPARAMS;
            }
            float s = 0.f;
            if (y)
                for (int b = r0 + lane; b < r1; b += kWave) s = fmaf(x[b], y[b], s);
            else
                for (int b = r0 + lane; b < r1; b += kWave) s += x[b];
            s = wave_sum(s);
            if (lane == 0) part[dst] = s;
        }
    }
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ part, int nchunks, float lr, float b1, float b2, float eps, float c1,
                       float c2, float invB, float *__restrict__ loss, float *__restrict__ grad_out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        float s = 0.f;
        for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * kPart + NPARAMS];
        loss[0] = s * invB;
    }
    if (i >= NPARAMS) return;
    float g = 0.f;
    for (int c = 0; c < nchunks; ++c) g += part[(int64_t)c * kPart + i];
    if (grad_out) grad_out[i] = g;
    const float mi = fmaf(b1, m[i], (1.f - b1) * g);
    const float vi = fmaf(b2, v[i], (1.f - b2) * g * g);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
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

static int device_cus_train() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

}  // namespace rb

using namespace rb;

extern "C" size_t rb_nn_train_workspace_bytes(int32_t batch) {
    if (batch <= 0 || batch % 32 != 0 || batch > (1 << 20)) return 0;
    return train_layout(batch).total;
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
    char *w = static_cast<char *>(ws);
    TrainArgs a;
    a.params = params;
    a.nm = norm_from_host(norm);
    a.oshift = a.nm.oshift;
    a.oscale = a.nm.oscale;
    a.nm.oshift = 0.f;
    a.nm.oscale = 1.f;
    a.B = batch;
    a.desc = desc;
    a.nd = n_data;
    a.labels = labels;
    a.idx = idx;
    a.H = reinterpret_cast<float *>(w + Lw.H);
    a.D = reinterpret_cast<float *>(w + Lw.D);
    a.R = reinterpret_cast<float *>(w + Lw.R);
    a.part = reinterpret_cast<float *>(w + Lw.part);
    hipStream_t st = (hipStream_t)stream;
    const int ntiles = (batch + kTile - 1) / kTile;
    const int cus = device_cus_train();
    if (precision == RB_PREC_BF16) {
        k_train_fb_wide<<<grid_for(ntiles, kTrainGroups, cus), kTrainWideThreads, 0, st>>>(a);
    } else {
        constexpr int wv = nn_threads(false, 1) / kWave;
        k_train_fb<false><<<grid_for(ntiles, wv, cus), wv * kWave, 0, st>>>(a);
    }
    const int nchunks = (batch + kChunk - 1) / kChunk;
    dim3 g2(nchunks, 3 + kSmallBlocks);
    if (precision == RB_PREC_BF16)
        k_train_wgrad<true><<<g2, 512, 0, st>>>(a);
    else
        k_train_wgrad<false><<<g2, 512, 0, st>>>(a);
    const double c1 = 1.0 / (1.0 - pow((double)beta1, (double)t));
    const double c2 = 1.0 / (1.0 - pow((double)beta2, (double)t));
    k_adam<<<(NPARAMS + 255) / 256, 256, 0, st>>>(params, adam_m, adam_v, a.part, nchunks, lr, beta1, beta2, eps,
                                                   (float)c1, (float)c2, 1.f / (float)batch, loss, grad_out);
    RB_LAUNCH_CHECK("rb_nn_train_step");
    return RB_OK;
}
