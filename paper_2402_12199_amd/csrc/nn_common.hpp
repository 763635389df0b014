// Shared pieces of the energy-network kernels (inference, gradient, training).
//
// Network (paper section 2, g_NN_U, sized by the workload): u (7) ->
// 128 -> 128 -> 128 -> 128 (SiLU) -> 1.  Parameter blob, layer by layer:
// W_l (out x in, row major) then b_l.
//
// Register layout.  A wave processes a tile of 16 pairs.  The three
// 128x128 layers run as 16x16 MFMA tiles with the pairs as the N
// dimension: z^T (128 x 16) = W (128 x 128) h^T (128 x 16).  An MFMA result
// fragment gives lane l the pair n = l % 16 and, for each of the eight
// 16-row tiles mt, the four features 16 mt + 4 (l / 16) + r (r = 0..3).
// The next layer consumes those values directly as its B operand: for the
// K-block kb of 32 input features, lane group g = l / 16 supplies slots
// k = 8 g + i, which hold the features 32 kb + perm32(8 g + i) with
// perm32(s) = 16 ((s % 8) / 4) + 4 (s / 8) + (s % 4).  Reordering K is free
// for a dot product, so the weights are staged with their input columns
// permuted the same way and no activation ever moves between lanes.
#pragma once

#include "rb_common.hpp"

namespace rb {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kH = 128;
constexpr int kIn = 7;
constexpr int kNnWaves = 8;
constexpr int kNnThreads = kNnWaves * kWave;
constexpr int kTile = 16;

constexpr int OFF_W1 = 0, OFF_B1 = 896, OFF_W2 = 1024, OFF_B2 = 17408, OFF_W3 = 17536, OFF_B3 = 33920,
              OFF_W4 = 34048, OFF_B4 = 50432, OFF_W5 = 50560, OFF_B5 = 50688, NPARAMS = 50689;
static_assert(NPARAMS == RB_MLP_NPARAMS, "parameter count");

__host__ __device__ constexpr int w_off(int layer) {  // layer 2..4
    return layer == 2 ? OFF_W2 : (layer == 3 ? OFF_W3 : OFF_W4);
}
__host__ __device__ constexpr int b_off(int layer) {  // layer 1..4
    return layer == 1 ? OFF_B1 : (layer == 2 ? OFF_B2 : (layer == 3 ? OFF_B3 : OFF_B4));
}

__host__ __device__ inline int perm32(int s) { return 16 * ((s & 7) >> 2) + 4 * (s >> 3) + (s & 3); }
__host__ __device__ inline int perm32_inv(int f) { return 8 * ((f & 15) >> 2) + 4 * (f >> 4) + (f & 3); }

struct Norm {
    float shift[kIn], scale[kIn], oshift, oscale;
};

inline Norm norm_from_host(const float *h) {
    Norm n;
    for (int k = 0; k < kIn; ++k) {
        n.shift[k] = h ? h[k] : 0.f;
        n.scale[k] = h ? h[kIn + k] : 1.f;
    }
    n.oshift = h ? h[14] : 0.f;
    n.oscale = h ? h[15] : 1.f;
    return n;
}

// SiLU and its derivative: s = 1/(1+exp(-z)), h = z s, h' = s + h (1 - s).
__device__ inline void silu(float z, float &h, float &dh) {
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * z);
    const float s = __builtin_amdgcn_rcpf(1.f + e);
    h = z * s;
    dh = fmaf(h, 1.f - s, s);
}

// SiLU with its first and second derivatives: h'' = s (1 - s) (2 + z (1 - 2 s)).
__device__ inline void silu2(float z, float &h, float &dh, float &d2h) {
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * z);
    const float s = __builtin_amdgcn_rcpf(1.f + e);
    h = z * s;
    dh = fmaf(h, 1.f - s, s);
    d2h = s * (1.f - s) * fmaf(z, 1.f - 2.f * s, 2.f);
}

__device__ inline bf16x8 pack8(const float a[4], const float b[4]) {
    bf16x8 v;
    v[0] = (__bf16)a[0]; v[1] = (__bf16)a[1]; v[2] = (__bf16)a[2]; v[3] = (__bf16)a[3];
    v[4] = (__bf16)b[0]; v[5] = (__bf16)b[1]; v[6] = (__bf16)b[2]; v[7] = (__bf16)b[3];
    return v;
}

// LDS image of the weights used by the BF16 kernels, 16-byte aligned so that
// 16-byte weight fragments and bias vectors load as single ds_read_b128.
// Rows of the BF16 weight image are 256 bytes (16 chunks of 8 BF16) with no
// padding; chunk c of row r is stored at chunk c ^ wswz(r).  Over any 16
// consecutive rows wswz is a permutation of 0..15, so the forward pass's
// 16-byte fragment reads (16 lanes, 16 consecutive rows, one chunk) hit 16
// different bank groups; the reverse pass's transposing reads (per 32 lanes:
// 8 rows 4 g + j / 4 of one 32-row block, 4 chunks) spread over all 16 bank
// groups twice, the least for reads that all take the same half of a chunk
// (a plain 68-dword stride gives four-way conflicts there).
__device__ inline int wswz(int r) { return ((r >> 2) & 3) | ((r & 3) << 2); }
__device__ inline int wcol(int r, int c) { return (((c >> 3) ^ wswz(r)) << 3) | (c & 7); }

struct alignas(16) LdsBF16 {
    __bf16 w[3][kH][kH];     // W2..W4, columns permuted per 32-block, 16-byte chunks swizzled (wcol)
    float w1[kH][8];          // W1 (7 columns, padded)
    float b[4][kH];           // b1..b4
    float w5[kH];
    float b5;
};

// Reverse-pass operand of W^T (the A fragment of v_mfma_f32_16x16x32_bf16 for
// lane (n, g), n = lane % 16, g = lane / 16): slot i holds W[32 kb +
// 16 (i / 4) + 4 g + (i % 4)][input feature 16 mt + n] of layer l's LDS image.
// Read with two transposing LDS loads (ds_read_b64_tr_b16, gfx950): within
// each 16-lane group, lane n receives as its value k element n % 4 of the
// 8 bytes that lane 4 k + n / 4 of the group addresses.  Lane j therefore
// addresses row 32 kb + 4 g + j / 4 (+ 16 for slots 4..7) at the column of
// input features 16 mt + 4 (j % 4) .. + 3, which the staging's column
// permutation keeps consecutive (columns 32 (mt / 2) + 8 (j % 4) +
// 4 (mt % 2) .. + 3).  The values are those of eight 2-byte column reads.
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

__device__ inline bf16x8 wt_frag(const LdsBF16 &L, int l, int kb, int mt, int lane) {
    const int j = lane & 15, g = lane >> 4;
    const int row = 32 * kb + 4 * g + (j >> 2);
    const int col = 32 * (mt >> 1) + 8 * (j & 3) + 4 * (mt & 1);
    const s16x4 a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(const_cast<__bf16 *>(&L.w[l][row][wcol(row, col)])));
    const s16x4 b =
        __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(const_cast<__bf16 *>(&L.w[l][row + 16][wcol(row + 16, col)])));
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    const s16x8 v = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
    return __builtin_bit_cast(bf16x8, v);
}

// NT = threads of the block.  The loops have compile-time trip counts so
// that a batch of global loads is in flight before the first LDS store (a
// block that evaluates a single tile spends most of its time here).
template <int NT>
__device__ inline void stage_bf16(LdsBF16 &L, const float *__restrict__ p) {
    // One 16-byte LDS store per work item: columns 32 cb + 8 g .. + 7 of row
    // o hold the input features 32 cb + perm32(8 g + i), i.e. two runs of four
    // consecutive features (32 cb + 4 g and 32 cb + 16 + 4 g).
    constexpr int kItems = 3 * kH * 16;
    static_assert(kItems % NT == 0, "block size must divide the weight items");
    constexpr int kIter = kItems / NT;
    constexpr int kBatch = kIter % 8 == 0 ? 8 : (kIter % 6 == 0 ? 6 : (kIter % 4 == 0 ? 4 : 1));
#pragma unroll
    for (int b0 = 0; b0 < kIter; b0 += kBatch) {
        float4 va[kBatch], vb[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int idx = threadIdx.x + (b0 + k) * NT;
            const int l = idx / (kH * 16), o = (idx / 16) % kH, u = idx % 16, cb = u >> 2, g = u & 3;
            const float *row = p + w_off(l + 2) + o * kH + 32 * cb + 4 * g;
            va[k] = *reinterpret_cast<const float4 *>(row);
            vb[k] = *reinterpret_cast<const float4 *>(row + 16);
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int idx = threadIdx.x + (b0 + k) * NT;
            const int l = idx / (kH * 16), o = (idx / 16) % kH, u = idx % 16, cb = u >> 2, g = u & 3;
            const float av[4] = {va[k].x, va[k].y, va[k].z, va[k].w};
            const float bv[4] = {vb[k].x, vb[k].y, vb[k].z, vb[k].w};
            *reinterpret_cast<bf16x8 *>(&L.w[l][o][wcol(o, 32 * cb + 8 * g)]) = pack8(av, bv);
        }
    }
#pragma unroll
    for (int it = 0; it < (kH * 8 + NT - 1) / NT; ++it) {
        const int idx = threadIdx.x + it * NT;
        if (idx < kH * 8) {
            const int o = idx >> 3, k = idx & 7;
            L.w1[o][k] = k < kIn ? p[OFF_W1 + o * kIn + k] : 0.f;
        }
    }
#pragma unroll
    for (int it = 0; it < (4 * kH + NT - 1) / NT; ++it) {
        const int idx = threadIdx.x + it * NT;
        if (idx < 4 * kH) L.b[idx / kH][idx % kH] = p[b_off(idx / kH + 1) + idx % kH];
    }
    for (int idx = threadIdx.x; idx < kH; idx += NT) L.w5[idx] = p[OFF_W5 + idx];
    if (threadIdx.x == 0) L.b5 = p[OFF_B5];
}

// Layer 1 in FP32 on the VALU for this lane's 32 features (16 mt + 4 g + r)
// (FP32 path).
__device__ inline void layer1(const float (*w1)[8], const float *b1, const float un[kIn], int g, float hv[8][4],
                              float dv[8][4]) {
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        __asm__ volatile("" ::: "memory");   // one tile's weights in flight at a time
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = 16 * mt + 4 * g + r;
            const float4 wa = *reinterpret_cast<const float4 *>(&w1[f][0]);
            const float4 wb = *reinterpret_cast<const float4 *>(&w1[f][4]);
            float z = b1[f];
            z = fmaf(wa.x, un[0], z); z = fmaf(wa.y, un[1], z); z = fmaf(wa.z, un[2], z);
            z = fmaf(wa.w, un[3], z); z = fmaf(wb.x, un[4], z); z = fmaf(wb.y, un[5], z);
            z = fmaf(wb.z, un[6], z);
            silu(z, hv[mt][r], dv[mt][r]);
        }
    }
}


// Layer 1 on the FP32 matrix cores (v_mfma_f32_16x16x4_f32, the 7 inputs
// padded to 8 in two k-steps): pre-activations of rows 16 mt + 4 g + r
// (r = 0..3) for the tile's pair n.  A = W1 rows 16 mt .. + 15 (lane: row n,
// column 4 s + g), B = the normalised inputs (lane: input 4 s + g of pair
// n; l1_inputs picks them), C starts from the bias.  The padding column of
// W1 in LDS is zero.
__device__ inline void l1_inputs(const float un[kIn], int g, float &x0, float &x1) {
    x0 = g == 0 ? un[0] : (g == 1 ? un[1] : (g == 2 ? un[2] : un[3]));
    x1 = g == 0 ? un[4] : (g == 1 ? un[5] : (g == 2 ? un[6] : 0.f));
}

__device__ inline f32x4 layer1_rows(const float (*w1)[8], const float *b1, float x0, float x1, int n, int g, int mt) {
    f32x4 c = *reinterpret_cast<const f32x4 *>(&b1[16 * mt + 4 * g]);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(w1[16 * mt + n][g], x0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(w1[16 * mt + n][4 + g], x1, c, 0, 0, 0);
    return c;
}

// The same product without the bias (tangents of layer 1's inputs).
__device__ inline f32x4 layer1_rows_nobias(const float (*w1)[8], float x0, float x1, int n, int g, int mt) {
    f32x4 c = f32x4{0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(w1[16 * mt + n][g], x0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(w1[16 * mt + n][4 + g], x1, c, 0, 0, 0);
    return c;
}

// FP16 packing of the SiLU derivatives kept for the reverse pass (values in
// [-0.1, 1.1]; FP16 keeps 11 significant bits against BF16's 8).
__device__ inline f16x8 pack8h(const float a[4], const float b[4]) {
    f16x8 v;
    v[0] = (_Float16)a[0]; v[1] = (_Float16)a[1]; v[2] = (_Float16)a[2]; v[3] = (_Float16)a[3];
    v[4] = (_Float16)b[0]; v[5] = (_Float16)b[1]; v[6] = (_Float16)b[2]; v[7] = (_Float16)b[3];
    return v;
}

// Split of FP32 values into a BF16 head and the BF16 rounding of the
// remainder: x ~ hi + lo to about 16 significant bits, so an MFMA product
// with a BF16 operand can be carried as two BF16 MFMAs.
__device__ inline void split8(const float a[4], const float b[4], bf16x8 &hi, bf16x8 &lo) {
    hi = pack8(a, b);
    float ra[4], rb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        ra[r] = a[r] - (float)hi[r];
        rb[r] = b[r] - (float)hi[4 + r];
    }
    lo = pack8(ra, rb);
}

// Sum over the four lane groups that share a pair.
__device__ inline float group_sum(float v) {
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    return v;
}

// Forces and torques of a pair from g = dE/du (supplementary section 6
// defines f = -dE/dx and tau = -dE/dtheta; with the quaternion descriptor
// the rotation derivative has the closed form below), body i's frame:
// F_j = -g_d, tau_j = -(w g_v - g_w v + v x g_v)/2, tau_i = -tau_j - d x F_j.
__device__ inline void pair_ft_from_grad(const float u[kIn], const float gu[kIn], float ft[9]) {
    const float w = u[3], vx = u[4], vy = u[5], vz = u[6];
    const float gw = gu[3], gx = gu[4], gy = gu[5], gz = gu[6];
    const float Fx = -gu[0], Fy = -gu[1], Fz = -gu[2];
    const float tjx = -0.5f * (w * gx - gw * vx + (vy * gz - vz * gy));
    const float tjy = -0.5f * (w * gy - gw * vy + (vz * gx - vx * gz));
    const float tjz = -0.5f * (w * gz - gw * vz + (vx * gy - vy * gx));
    const float dx = u[0], dy = u[1], dz = u[2];
    ft[0] = Fx; ft[1] = Fy; ft[2] = Fz;
    ft[3] = -tjx - (dy * Fz - dz * Fy);
    ft[4] = -tjy - (dz * Fx - dx * Fz);
    ft[5] = -tjz - (dx * Fy - dy * Fx);
    ft[6] = tjx; ft[7] = tjy; ft[8] = tjz;
}

}  // namespace rb
