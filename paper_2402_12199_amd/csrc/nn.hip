// Energy network: forward pass, hand-written reverse pass (input gradient),
// and per-pair or per-body forces and torques from that gradient.
//
// BF16 path: layer 1 (7 -> 128) in FP32 on v_mfma_f32_16x16x4_f32, layer 5
// (128 -> 1) in FP32 on the VALU; the three 128 x 128 layers on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation, weights staged once per
// block in a 16-byte aligned LDS image, activations rounded to BF16 as MFMA
// operands.  SiLU derivatives of the forward pass are kept in registers
// (FP16) for the reverse pass.  The reverse pass multiplies by
// W^T: the forward reads a 16-byte row fragment of the LDS weights, the
// reverse gathers eight 2-byte elements down a column of the same array.
//
// FP32 path: the same tiling on v_mfma_f32_16x16x4_f32, weights read from
// global memory (they stay in the caches), activations and derivatives in
// FP32.
#include "bead_pair.hpp"
#include "cyl_form.hpp"
#include "nn_tile.hpp"

namespace rb {

enum NNMode { kEval = 0, kGrad = 1, kForces = 2 };

struct NNArgs {
    const float *params;
    Norm nm;
    int64_t P;              // rows (eval/grad) or max_count (forces)
    const float *desc;
    int64_t stride;         // row stride of desc
    const float *gE;
    float *energy;
    float *dEdu;
    float *ft;
    // dynamics form
    const int32_t *idx;
    const int32_t *count_dev;
    const double *q;
    int32_t n;
    const int32_t *pi;
    const int32_t *pj;
    float sw_lo, sw_hi;
    int64_t *acc;
    int32_t *flags;
    // symmetry-reduced inputs (cube pairs): the network sees sym (7 x P, row
    // k of the launch), and dE/du = J^T dE/ds with jac (49 x P, r * 7 + m);
    // desc then holds the pairs' (d, q) for the forces.  Null: plain (d, q).
    const float *sym;
    const float *jac;
    // cylinder pairs: the network sees the four-number form of desc's
    // (d, q), computed here together with its Jacobian (no sym/jac arrays)
    int cyl;
    // forces mode with the bead-sum fallback in the same launch: after its
    // network tiles each wave takes pairs idx_bead[0 .. *bead_count) one at a
    // time and adds their bead double sums (null idx_bead: no fallback)
    const int32_t *idx_bead;
    const int32_t *bead_count;
    const double *x;
    const int32_t *type;
    Box box;
    Templates T;
    LJ lj;
    int bead_stride;    // float4 per wave staging array
};

// Whether the network's input differs from the pair's (d, q).
__device__ inline bool reduced_input(const NNArgs &a) { return a.sym || a.cyl; }

// |d| from the network input u of a pair: the cube form's first three
// numbers are a signed permutation of d, the cylinder form starts with
// (d_x^2 + d_y^2, d_z^2).
__device__ inline float centre_distance(const NNArgs &a, const float u[kIn]) {
    return a.cyl ? sqrtf(u[0] + u[1]) : sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

// The network's input of launch row `row` (pair pid).
__device__ inline void net_input(const NNArgs &a, int64_t row, int64_t pid, bool live, float u[kIn]) {
    if (a.cyl && live) {
        float ud[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) ud[k] = a.desc[k * a.stride + pid];
        cyl_features(ud, u);
        return;
    }
#pragma unroll
    for (int k = 0; k < kIn; ++k)
        u[k] = !live ? (k == 3 ? 1.f : 0.f) : (a.sym ? a.sym[k * a.P + row] : a.desc[k * a.stride + pid]);
}

// dE/ds -> dE/du through the descriptor's Jacobian (symmetry-reduced and
// cylinder forms).
__device__ inline void sym_chain(const NNArgs &a, int64_t row, int64_t pid, float gu[kIn]) {
    if (!a.jac && !a.cyl) return;
    float gs[kIn];
#pragma unroll
    for (int r = 0; r < kIn; ++r) gs[r] = gu[r];
    if (a.cyl) {
        float ud[kIn], J[kIn][kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) ud[k] = a.desc[k * a.stride + pid];
        cyl_jacobian(ud, J);
#pragma unroll
        for (int m = 0; m < kIn; ++m) {
            float v = 0.f;
#pragma unroll
            for (int r = 0; r < kIn; ++r) v = fmaf(J[r][m], gs[r], v);
            gu[m] = v;
        }
        return;
    }
#pragma unroll
    for (int m = 0; m < kIn; ++m) {
        float v = 0.f;
#pragma unroll
        for (int r = 0; r < kIn; ++r) v = fmaf(a.jac[(r * kIn + m) * a.P + row], gs[r], v);
        gu[m] = v;
    }
}

// ------------------------------------------------------------------ kernels
__device__ inline float smooth_switch(float r, float lo, float hi, float &dsdr) {
    dsdr = 0.f;
    if (!(hi > lo) || r <= lo) return 1.f;
    if (r >= hi) return 0.f;
    const float w = 1.f / (hi - lo), t = (r - lo) * w;
    dsdr = -6.f * t * (1.f - t) * w;
    return 1.f - t * t * (3.f - 2.f * t);
}

// Forces of one pair for dynamics: switched energy, body-i-frame force and
// torques, rotation to the lab frame, fixed-point accumulation on both
// bodies; the energy and virial of the 16 rows of the wave's tile are summed
// over the row lanes and added to the wave's LDS sums by lane 0.
// Per-pair inputs of the forces epilogue, loaded before the tile is
// evaluated so that their latency overlaps the network.
struct EpiIn {
    int i = 0, j = 0;
    double q[4] = {1.0, 0.0, 0.0, 0.0};
};

__device__ inline EpiIn load_epi(const NNArgs &a, int64_t pid, bool live) {
    EpiIn e;
    if (live) {
        e.i = a.pi[pid];
        e.j = a.pj[pid];
#pragma unroll
        for (int c = 0; c < 4; ++c) e.q[c] = a.q[c * a.n + e.i];
    }
    return e;
}

__device__ inline void forces_epilogue(const NNArgs &a, const EpiIn &in, float gu[kIn], float E, int64_t pid,
                                       bool mine, int lane, long long *wsum, bool &bad, bool &ovf) {
    long long ev[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) ev[k] = 0;
    if (mine) {
        // the descriptor and the switch are reloaded and recomputed here
        // rather than kept in registers across the tile
        float u[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) u[k] = a.desc[k * a.stride + pid];
        const float r = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        float dsdr;
        const float S = smooth_switch(r, a.sw_lo, a.sw_hi, dsdr);
        // switched energy: E_s = S E, dE_s/dd = S g_d + E S'(r) d / r
        if (dsdr != 0.f) {
            const float c = E * dsdr / r;
            gu[0] = fmaf(c, u[0], gu[0]);
            gu[1] = fmaf(c, u[1], gu[1]);
            gu[2] = fmaf(c, u[2], gu[2]);
        }
        const float Es = S * E;
        float ft[9];
        pair_ft_from_grad(u, gu, ft);
        const int i = in.i, j = in.j;
        double R[9];
        quat_to_rot<double>(in.q[0], in.q[1], in.q[2], in.q[3], R);
        double Fj[3], ti[3], tj[3], dl[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Fj[c] = R[3 * c] * ft[0] + R[3 * c + 1] * ft[1] + R[3 * c + 2] * ft[2];
            ti[c] = R[3 * c] * ft[3] + R[3 * c + 1] * ft[4] + R[3 * c + 2] * ft[5];
            tj[c] = R[3 * c] * ft[6] + R[3 * c + 1] * ft[7] + R[3 * c + 2] * ft[8];
            dl[c] = R[3 * c] * u[0] + R[3 * c + 1] * u[1] + R[3 * c + 2] * u[2];
        }
        if (!isfinite(Es) || !isfinite(ft[0]) || !isfinite(ft[3]) || !isfinite(ft[6])) bad = true;
        const int64_t nn = a.n;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc_add(a.acc + c * nn + i, -Fj[c], ovf);
            acc_add(a.acc + c * nn + j, Fj[c], ovf);
            acc_add(a.acc + (3 + c) * nn + i, ti[c], ovf);
            acc_add(a.acc + (3 + c) * nn + j, tj[c], ovf);
        }
        ovf |= !fix_ok(Es);
        ev[0] = to_fixed(Es);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                ovf |= !fix_ok(dl[c] * Fj[b]);
                ev[1 + 3 * c + b] = to_fixed(dl[c] * Fj[b]);
            }
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        long long v = ev[k];
        v += __shfl_xor(v, 1, kWave);
        v += __shfl_xor(v, 2, kWave);
        v += __shfl_xor(v, 4, kWave);
        v += __shfl_xor(v, 8, kWave);
        if (lane == 0) wsum[k] += v;
    }
}

template <int MODE, bool BF16>
__global__ __launch_bounds__(nn_threads(BF16, MODE)) void k_nn(NNArgs a) {
    constexpr int kWaves = NNCfg<BF16, MODE>::waves;
    __shared__ typename NNLds<BF16>::T L;
    if (MODE == kForces) {
        // the grid is sized for the capacity; blocks without a tile leave
        // before staging the weights
        const int64_t c = *a.count_dev;
        if ((int64_t)blockIdx.x * kWaves * kTile >= (c < a.P ? c : a.P)) return;
    }
    if constexpr (BF16)
        stage_bf16<nn_threads(true, MODE)>(L, a.params);
    else
        stage_small(L, a.params);
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t count = a.P;
    if (MODE == kForces) {
        const int64_t c = *a.count_dev;
        count = c < a.P ? c : a.P;
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.flags + RB_FLAG_NEVAL, (int)count);
    }
    // per-wave energy/virial sums live in LDS, not registers, so that they
    // add nothing to the register pressure of the tile evaluation
    __shared__ long long wacc[kWaves][10];
    if (MODE == kForces && lane < 10) wacc[w][lane] = 0;
    bool bad = false, ovf = false;
    const int64_t ntiles = (count + kTile - 1) / kTile;
    for (int64_t t = (int64_t)blockIdx.x * kWaves + w; t < ntiles; t += (int64_t)gridDim.x * kWaves) {
        // Keeps the compiler from hoisting the (tile-invariant) LDS weight
        // reads out of the loop, which would pin ~600 registers.
        __asm__ volatile("" ::: "memory");
        const int64_t row = t * kTile + n;
        const bool live = row < count;
        int64_t pid = row;
        if (MODE == kForces && live && a.idx) pid = a.idx[row];
        float u[kIn];
        net_input(a, row, pid, live, u);
        float seed = 1.f;
        if (MODE == kGrad && a.gE) seed = live ? a.gE[pid] : 0.f;
        if (MODE == kForces) {
            float dsdr;
            seed = smooth_switch(centre_distance(a, u), a.sw_lo, a.sw_hi, dsdr);
        }
        EpiIn ein;
        if (MODE == kForces) ein = load_epi(a, pid, live && g == 0);
        float gu[kIn];
        float E;
        if constexpr (BF16)
            E = tile_bf16<MODE != kEval>(L, a.nm, u, seed, gu);
        else
            E = tile_fp32<MODE != kEval>(L, L, a.params, a.nm, u, seed, gu);
        if (MODE != kEval && live && g == 0) sym_chain(a, row, pid, gu);
        if (MODE == kForces) {
            // every lane takes part in the shuffles below; the results of
            // the lanes of groups 1..3 and of dead rows are discarded
            forces_epilogue(a, ein, gu, E, pid, live && g == 0, lane, wacc[w], bad, ovf);
            continue;
        }
        if (!live || g != 0) continue;
        if (MODE == kEval) {
            a.energy[pid] = E;
        } else if (MODE == kGrad) {
            if (a.energy) a.energy[pid] = E;
            if (a.dEdu)
#pragma unroll
                for (int k = 0; k < kIn; ++k) a.dEdu[k * a.P + pid] = gu[k];
            if (a.ft) {
                float ft[9], ud[kIn];
                if (reduced_input(a))
#pragma unroll
                    for (int k = 0; k < kIn; ++k) ud[k] = a.desc[k * a.stride + pid];
                else
#pragma unroll
                    for (int k = 0; k < kIn; ++k) ud[k] = u[k];
                pair_ft_from_grad(ud, gu, ft);
#pragma unroll
                for (int k = 0; k < 9; ++k) a.ft[k * a.P + pid] = ft[k];
            }
        }
    }
    if (MODE == kForces) {
        long long part[11];
#pragma unroll
        for (int k = 0; k < 10; ++k) part[k] = wacc[w][k];
        part[10] = 0;
        block_flush_globals<kWaves>(part, a.acc + 6 * (int64_t)a.n, nullptr);
        if (__any(bad) && lane == 0) atomicOr(a.flags + RB_FLAG_NONFINITE, 1);
        report_fixovf(ovf, a.flags);
    }
}

// Four waves per tile (tile_bf16_wide), two tiles in flight per block; the
// block walks the tiles in lockstep (a group past the end evaluates a dead
// tile) so that every wave meets the same barriers.
constexpr int kWideGroups = 3;
constexpr int kWideThreads = kWideGroups * kWideGroup * kWave;
// Fallback phase: LDS words of the chunks in use, a 6-bit chunk tag above
// a 26-bit first pair index (the fused launch is taken only for lists below
// kFbMaxPairs, so that the counter, which runs past the count by at most two
// chunks per block, stays below 2^26).
constexpr int kFbSlots = 4;
constexpr int kFbBaseBits = 26;
constexpr unsigned kFbBaseMask = (1u << kFbBaseBits) - 1u;
constexpr int64_t kFbMaxPairs = (1 << kFbBaseBits) - (1 << 16);

// Inputs of one lane's row of a tile: the network input, the backward seed
// (the switch for dynamics, dL/dE for gradients) and, for the lanes that
// run the forces epilogue, that epilogue's per-pair inputs.
struct TileIn {
    int64_t row, pid;
    bool live;
    float u[kIn];
    float seed;
    EpiIn ein;
};

template <int MODE>
__device__ inline TileIn tile_in(const NNArgs &a, int64_t row, int64_t count, bool epi) {
    TileIn t;
    t.row = row;
    t.live = row < count;
    t.pid = row;
    if (MODE == kForces && t.live && a.idx) t.pid = a.idx[row];
    net_input(a, row, t.pid, t.live, t.u);
    t.seed = 1.f;
    if (MODE == kGrad && a.gE) t.seed = t.live ? a.gE[t.pid] : 0.f;
    if (MODE == kForces) {
        float dsdr;
        t.seed = smooth_switch(centre_distance(a, t.u), a.sw_lo, a.sw_hi, dsdr);
        t.ein = load_epi(a, t.pid, t.live && epi);
    }
    return t;
}

// Per-pair outputs of the gradient mode: energy, dE/du and the pair's
// body-frame force and torques.
__device__ inline void store_grad(const NNArgs &a, const TileIn &t, const float gu[kIn], float E) {
    const int64_t pid = t.pid;
    if (a.energy) a.energy[pid] = E;
    if (a.dEdu)
#pragma unroll
        for (int k = 0; k < kIn; ++k) a.dEdu[k * a.P + pid] = gu[k];
    if (a.ft) {
        float ft[9], ud[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) ud[k] = reduced_input(a) ? a.desc[k * a.stride + pid] : t.u[k];
        pair_ft_from_grad(ud, gu, ft);
#pragma unroll
        for (int k = 0; k < 9; ++k) a.ft[k * a.P + pid] = ft[k];
    }
}

// Per-pair inputs of a group's forces epilogue, held in LDS across the tile
// (16 pairs): the pair's bodies, body i's orientation and the pair's (d, q).
struct EpiLds {
    double q[4][kTile];
    float d[kIn][kTile];
    int i[kTile], j[kTile];
};

// u: the network input, which is the pair's (d, q) unless the network sees
// the symmetry-reduced form (then (d, q) is read here).
__device__ inline void put_epi(const NNArgs &a, EpiLds &e, const EpiIn &in, const float u[kIn], int64_t pid,
                               bool live, int n) {
    e.i[n] = in.i;
    e.j[n] = in.j;
#pragma unroll
    for (int c = 0; c < 4; ++c) e.q[c][n] = in.q[c];
#pragma unroll
    for (int k = 0; k < kIn; ++k) e.d[k][n] = reduced_input(a) && live ? a.desc[k * a.stride + pid] : u[k];
}

// Forces epilogue of the four-wave form: the group's 16 pairs are shared
// out over its waves by quantity, so each lane converts and adds three
// values.  Lanes g = 0 of wave v add, to the lab-frame accumulators, the
// force on j (v = 0), the force on i (v = 1), the torque on i (v = 2) or the
// torque on j (v = 3); in wave 0 lane group g adds the energy (g = 0) or
// row g - 1 of the pair virial d (x) F_j, summed over the 16 pairs into the
// wave's LDS sums.  Same values as forces_epilogue (fixed-point sums are
// exact and order-free).
__device__ inline void forces_epilogue_wide(const NNArgs &a, const EpiLds &e, const float gu_in[kIn], float E,
                                            bool live, int v, int g, int n, long long *wsum, bool &bad, bool &ovf) {
    long long ev[3] = {0, 0, 0};
    if (live && (g == 0 || v == 0)) {
        float u[kIn], gu[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) {
            u[k] = e.d[k][n];
            gu[k] = gu_in[k];
        }
        const float r = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        float dsdr;
        const float S = smooth_switch(r, a.sw_lo, a.sw_hi, dsdr);
        if (dsdr != 0.f) {
            const float c = E * dsdr / r;
            gu[0] = fmaf(c, u[0], gu[0]);
            gu[1] = fmaf(c, u[1], gu[1]);
            gu[2] = fmaf(c, u[2], gu[2]);
        }
        const float Es = S * E;
        float ft[9];
        pair_ft_from_grad(u, gu, ft);
        // this wave's body-frame vector (v is uniform over the wave)
        const float f0 = v < 2 ? ft[0] : (v == 2 ? ft[3] : ft[6]);
        const float f1 = v < 2 ? ft[1] : (v == 2 ? ft[4] : ft[7]);
        const float f2 = v < 2 ? ft[2] : (v == 2 ? ft[5] : ft[8]);
        double R[9];
        quat_to_rot<double>(e.q[0][n], e.q[1][n], e.q[2][n], e.q[3][n], R);
        double V[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) V[c] = R[3 * c] * f0 + R[3 * c + 1] * f1 + R[3 * c + 2] * f2;
        if (g == 0) {
            const int64_t nn = a.n;
            const int64_t body = (v == 1 || v == 2) ? e.i[n] : e.j[n];
            const int64_t row0 = v < 2 ? 0 : 3;
            const double sgn = v == 1 ? -1.0 : 1.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) acc_add(a.acc + (row0 + c) * nn + body, sgn * V[c], ovf);
            if (!isfinite(f0) || (v == 0 && !isfinite(Es))) bad = true;
            if (v == 0) {
                ovf |= !fix_ok(Es);
                ev[0] = to_fixed(Es);
            }
        } else {
            // virial row c = g - 1: (R d)_c * F_j
            const int c = g - 1;
            const double r0 = c == 0 ? R[0] : (c == 1 ? R[3] : R[6]);
            const double r1 = c == 0 ? R[1] : (c == 1 ? R[4] : R[7]);
            const double r2 = c == 0 ? R[2] : (c == 1 ? R[5] : R[8]);
            const double dl = r0 * u[0] + r1 * u[1] + r2 * u[2];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                ovf |= !fix_ok(dl * V[b]);
                ev[b] = to_fixed(dl * V[b]);
            }
        }
    }
    if (v != 0) return;
    // each lane adds its terms into the wave's LDS sums (integer adds: the
    // totals do not depend on their order)
#pragma unroll
    for (int b = 0; b < 3; ++b)
        if ((g > 0 || b == 0) && ev[b] != 0)
            atomicAdd(reinterpret_cast<unsigned long long *>(&wsum[g == 0 ? 0 : 1 + 3 * (g - 1) + b]),
                      (unsigned long long)ev[b]);
}

// Inputs of the next tile fetched while the current one is computed (forces
// mode, (d, q) and cylinder inputs): one wave of each group runs a
// three-level chain -- the routed pair index at the tile's start; after
// layer 1 the pair's (d, q) and its two bodies, straight from global memory
// into the group's second epilogue buffer in LDS (global_load_lds: lane l's
// dword lands at the uniform LDS base + 4 l); after the forward pass body
// i's FP64 orientation the same way, 32 lanes a component (lane l: half
// l % 2 of pair l / 2).  The wave waits for all of it before the next
// tile's first barrier.
using lds_ptr = __attribute__((address_space(3))) void *;
using gbl_ptr = const __attribute__((address_space(1))) void *;

__device__ inline void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0f70); }   // vmcnt(0)

struct NextTile {
    const NNArgs *a;
    EpiLds *e;
    int64_t row0, count;   // first row of the next tile, rows in the launch
    bool active;           // this wave fetches and there is a next tile
    int lane;
    int32_t pid;           // level 1: routed pair index (lanes 0..15)

    __device__ bool live_row(int r) const { return row0 + r < count; }

    __device__ void start() {
        pid = 0;
        if (active && lane < kTile && live_row(lane)) pid = a->idx ? a->idx[row0 + lane] : (int32_t)(row0 + lane);
    }

    // Every wave waits at each stage (only the fetching wave has loads in
    // flight), so that no wave reaches code past a stage with a fetch the
    // compiler cannot prove complete.
    __device__ void operator()(int stage) const {
        wait_vmem();
        if (!active) return;
        if (stage == 1) {
            if (lane < kTile && live_row(lane)) {
#pragma unroll
                for (int k = 0; k < kIn; ++k)
                    __builtin_amdgcn_global_load_lds((gbl_ptr)(a->desc + k * a->stride + pid), (lds_ptr)&e->d[k][0], 4,
                                                     0, 0);
                __builtin_amdgcn_global_load_lds((gbl_ptr)(a->pi + pid), (lds_ptr)&e->i[0], 4, 0, 0);
                __builtin_amdgcn_global_load_lds((gbl_ptr)(a->pj + pid), (lds_ptr)&e->j[0], 4, 0, 0);
            }
        } else if (stage == 2) {
            const int r = lane >> 1;
            if (lane < 2 * kTile && live_row(r)) {
                const int bi = e->i[r];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    __builtin_amdgcn_global_load_lds(
                        (gbl_ptr)(reinterpret_cast<const uint32_t *>(a->q + (int64_t)c * a->n + bi) + (lane & 1)),
                        (lds_ptr)&e->q[c][0], 4, 0, 0);
            }
        }
    }
};

// A tile's network input read back from the epilogue buffer the previous
// tile filled.
__device__ inline TileIn tile_from_lds(const NNArgs &a, const EpiLds &e, int64_t row, int64_t count, int n) {
    TileIn t;
    t.row = row;
    t.live = row < count;
    t.pid = 0;
    float ud[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) ud[k] = t.live ? e.d[k][n] : (k == 3 ? 1.f : 0.f);
    if (a.cyl)
        cyl_features(ud, t.u);
    else
#pragma unroll
        for (int k = 0; k < kIn; ++k) t.u[k] = ud[k];
    float dsdr;
    t.seed = smooth_switch(centre_distance(a, t.u), a.sw_lo, a.sw_hi, dsdr);
    return t;
}

// dE/ds -> dE/du of the cylinder form from the pair's (d, q) held in LDS.
__device__ inline void cyl_chain_lds(const EpiLds &e, int n, float gu[kIn]) {
    float ud[kIn], J[kIn][kIn], gs[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) {
        ud[k] = e.d[k][n];
        gs[k] = gu[k];
    }
    cyl_jacobian(ud, J);
#pragma unroll
    for (int m = 0; m < kIn; ++m) {
        float v = 0.f;
#pragma unroll
        for (int r = 0; r < kIn; ++r) v = fmaf(J[r][m], gs[r], v);
        gu[m] = v;
    }
}

// PRE (forces with (d, q) or cylinder inputs): the next tile's inputs are
// fetched during the current one into the group's other epilogue buffer.
// FB (PRE only; 1: Lennard-Jones, 2: half-power half-cosine beads): the
// launch also adds the bead double sums of the fallback pairs.  Every block
// of the grid takes part: after the block's network tiles (if any) the
// weight image's LDS holds the bead templates and the waves' staging arrays,
// and the block's waves take the fallback pairs one at a time from chunks
// the block claims from a counter in flags (RB_FLAG_FB_WORK; FB_WORK + 1 is
// the finishing ticket; both zero between launches), so that blocks with
// fewer network tiles take more pairs and no wave waits for another's pair.
// One global claim per chunk keeps the counter's atomics few (one per wave
// serialised the grid on that address).
template <int MODE, bool PRE = false, int FB = 0>
__global__ __launch_bounds__(kWideThreads) void k_nn_wide(NNArgs a) {
    static_assert(!PRE || MODE == kForces, "prefetching is a forces-mode form");
    static_assert(FB == 0 || PRE, "the bead fallback runs in the prefetching forces form");
    __shared__ LdsBF16 L;
    __shared__ WideX X[kWideGroups];
    __shared__ long long wacc[kWideGroups * kWideGroup][10];
    __shared__ EpiLds EL[MODE == kForces ? kWideGroups : 1][PRE ? 2 : 1];
    // PRE: the tile groups synchronise on their own (GroupSync) after the
    // first tile's block-wide barrier
    __shared__ __attribute__((aligned(16))) int gword[kWideGroups][kWideGroup];
    __shared__ int gtimeout;
    int64_t count = a.P;
    int nbead = 0;
    if (MODE == kForces) {
        const int64_t c = *a.count_dev;
        count = c < a.P ? c : a.P;
        if (FB) {
            nbead = *a.bead_count;
            if (nbead > a.P) nbead = (int)a.P;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.flags + RB_FLAG_NEVAL, (int)count + nbead);
    }
    const int64_t ntiles = (count + kTile - 1) / kTile;
    // the grid is sized for the capacity; without a fallback, blocks without
    // a tile leave before staging the weights
    const bool net = (int64_t)blockIdx.x * kWideGroups < ntiles;
    if (!FB && !net) return;
    const int lane = threadIdx.x & (kWave - 1), g = lane >> 4, n = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int grp = wave / kWideGroup, v = wave % kWideGroup;
    if (MODE == kForces && lane < 10) wacc[wave][lane] = 0;
    if (PRE && threadIdx.x == 0) gtimeout = 0;
    bool bad = false, ovf = false;
    if (net) {
        // the first tile's inputs are requested before the weights are
        // staged, so that their latency overlaps the staging
        int64_t base = (int64_t)blockIdx.x * kWideGroups;
        TileIn t = tile_in<MODE>(a, (base + grp) * kTile + n, count, g == 0 && v == 0);
        stage_bf16<kWideThreads>(L, a.params);
        if (PRE && v == 0 && g == 0) put_epi(a, EL[grp][0], t.ein, t.u, t.pid, t.live, n);
        if (PRE && threadIdx.x < kWideGroups * kWideGroup)
            gword[threadIdx.x / kWideGroup][threadIdx.x % kWideGroup] = 0;
        int gen = 0;
        const GroupSync gsync{(lds_int *)&gword[grp][0], v, &gen, (lds_int *)&gtimeout};
        for (int it = 0;; ++it) {
            EpiLds &ecur = EL[MODE == kForces ? grp : 0][PRE ? (it & 1) : 0];
            if (MODE == kForces && !PRE && v == 0 && g == 0) put_epi(a, ecur, t.ein, t.u, t.pid, t.live, n);
            if (!PRE || it == 0)
                __syncthreads();
            else
                gsync();
            if (PRE && it > 0) t = tile_from_lds(a, ecur, (base + grp) * kTile + n, count, n);
            const int64_t nbase = base + (int64_t)gridDim.x * kWideGroups;
            NextTile nx;
            nx.a = &a;
            nx.e = &EL[MODE == kForces ? grp : 0][PRE ? ((it + 1) & 1) : 0];
            nx.row0 = (nbase + grp) * kTile;
            nx.count = count;
            nx.active = PRE && v == 1 && nbase < ntiles;
            nx.lane = lane;
            nx.start();
            float gu[kIn];
            float E;
            if constexpr (PRE)
                E = tile_bf16_wide<true, false, NextTile, GroupSync>(L, X[grp], a.nm, t.u, t.seed, gu, v, Emit{}, nx,
                                                                     gsync);
            else
                E = tile_bf16_wide<true, false, NextTile>(L, X[grp], a.nm, t.u, t.seed, gu, v, Emit{}, nx);
            // the group's results are the same in its four waves
            if (MODE == kForces) {
                if (PRE && a.cyl) {
                    // dE/du = J^T dE/ds in every lane from the pair's (d, q) in
                    // LDS (the same arithmetic in each, so the group's lanes agree)
                    if (t.live) cyl_chain_lds(ecur, n, gu);
                } else if (a.jac || a.cyl) {
                    // dE/du = J^T dE/ds once per pair, shared through LDS
                    if (v == 0 && g == 0 && t.live) {
                        sym_chain(a, t.row, t.pid, gu);
#pragma unroll
                        for (int k = 0; k < kIn; ++k) X[grp].red[0][1 + k][n] = gu[k];
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < kIn; ++k) gu[k] = X[grp].red[0][1 + k][n];
                }
                forces_epilogue_wide(a, ecur, gu, E, t.live, v, g, n, wacc[wave], bad, ovf);
            } else if (v == 0 && t.live && g == 0) {
                sym_chain(a, t.row, t.pid, gu);
                store_grad(a, t, gu, E);
            }
            // the fetching wave's loads into LDS have landed before the next
            // tile's first barrier
            if (nx.active) wait_vmem();
            base = nbase;
            if (base >= ntiles) break;
            if (!PRE) {
                t = tile_in<MODE>(a, (base + grp) * kTile + n, count, g == 0 && v == 0);
                // the previous tile's epilogue has read its inputs from LDS
                __syncthreads();
            }
        }
    }
    long long ntests = 0;
    if constexpr (FB != 0) {
        constexpr int POT = FB == 1 ? kPotLJ : kPotHPHC;
        constexpr int kWaves = kWideThreads / kWave;
        __syncthreads();   // every group of the block is done with the weight image
        float4 *bl = reinterpret_cast<float4 *>(&L);
        float4 *tb = bl + (size_t)kWaves * 3 * a.bead_stride;
        for (int k = threadIdx.x; k < a.T.total; k += blockDim.x) tb[k] = a.T.beads[k];
        __syncthreads();
        WaveLds WL = wave_lds(bl, wave, a.bead_stride);
        const float rcm = sqrtf(a.lj.rc2) + kCullMargin, cut2 = rcm * rcm;
        // The block takes the pairs from the global counter in chunks of
        // kWaves (one atomic per chunk); each wave takes its next slot from
        // an LDS counter, without waiting for the block's other waves.  The
        // wave whose slot opens a chunk fetches the chunk's first pair index
        // and publishes it in one of kFbSlots LDS words, tagged with the
        // chunk's number; the chunk's other waves wait for that word (a
        // bounded wait: past kGroupSyncSpins polls it records a timeout and
        // the wave stops).  The fetching wave waits on nothing, so the waits
        // end.  A word is reused four chunks later, long after its readers
        // have read it (they wait only for one atomic).
        __shared__ int fb_next;
        __shared__ unsigned fb_word[kFbSlots];
        int32_t *work = a.flags + RB_FLAG_FB_WORK;
        if (threadIdx.x == 0) fb_next = 0;
        if (threadIdx.x < kFbSlots) fb_word[threadIdx.x] = 0u;
        __syncthreads();
        for (;;) {
            int m = 0;
            if (lane == 0) m = atomicAdd(&fb_next, 1);
            m = __builtin_amdgcn_readfirstlane(m);
            const int c = m / kWaves, o = m - c * kWaves;
            const unsigned tag = (unsigned)((c + 1) & 63) << kFbBaseBits;
            volatile lds_uint *slot = (volatile lds_uint *)&fb_word[c % kFbSlots];
            int base;
            if (o == 0) {
                int b0 = 0;
                if (lane == 0) {
                    b0 = atomicAdd(work, kWaves);
                    *slot = tag | (unsigned)b0;
                }
                base = __builtin_amdgcn_readfirstlane(b0);
            } else {
                unsigned w = 0;
                for (int spin = 0;; ++spin) {
                    w = __builtin_amdgcn_readfirstlane(*slot);
                    if ((w & ~kFbBaseMask) == tag) break;
                    if (spin >= kGroupSyncSpins) {
                        if (lane == 0) gtimeout = 1;
                        w = tag | (unsigned)nbead;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                base = (int)(w & kFbBaseMask);
            }
            const int k = base + o;
            if (k >= nbead) break;
            const int pid = a.idx_bead[k];
            const int i = a.pi[pid], j = a.pj[pid];
            const bool one = a.T.n_types == 1;   // one template: no type loads
            const int ti = one ? 0 : a.type[i], tj = one ? 0 : a.type[j];
            double dl[3], d[3], qr[4], qa[4], Ri[9], R[9];
            pair_frame(a.n, a.x, a.q, a.box, i, j, dl, d, qr, qa, Ri);
            quat_to_rot<double>(qr[0], qr[1], qr[2], qr[3], R);
            md_pair<POT>(a.T, a.lj, tb, WL, lane, cut2, a.n, i, j, ti, tj, dl, d, R, Ri, a.acc, wacc[wave], ntests,
                         bad, ovf);
        }
        __syncthreads();
        // every claim of every block has returned before its ticket; the last
        // block clears the counter and the ticket for the next launch
        if (threadIdx.x == 0 && atomicAdd(work + 1, 1) == (int)gridDim.x - 1) {
            work[0] = 0;
            work[1] = 0;
        }
    }
    if (MODE == kForces) {
        long long part[11];
#pragma unroll
        for (int k = 0; k < 10; ++k) part[k] = wacc[wave][k];
        part[10] = ntests;
        block_flush_globals<kWideGroups * kWideGroup>(part, a.acc + 6 * (int64_t)a.n, FB ? a.flags : nullptr);
        if (__any(bad) && lane == 0) atomicOr(a.flags + RB_FLAG_NONFINITE, 1);
        report_fixovf(ovf, a.flags);
        if (PRE && threadIdx.x == 0 && gtimeout) atomicOr(a.flags + RB_FLAG_WAIT_TIMEOUT, 1);
    }
}

// BF16 gradients and forces take the four-waves-per-tile form at every
// size (on 2^20 rows it is 5 % faster than the one-wave-per-tile form, which
// the FP32 path and the BF16 forward pass keep).

template <int MODE>
static int launch(const NNArgs &a, int precision, int64_t rows, hipStream_t st) {
    const int64_t tiles = (rows + kTile - 1) / kTile;
    const int cus = device_cu_count();
    if (precision == RB_PREC_BF16) {
        if constexpr (MODE == kEval) {
            constexpr int w = NNCfg<true, kEval>::waves;
            k_nn<kEval, true><<<grid_for(tiles, w, cus), w * kWave, 0, st>>>(a);
        } else if (MODE == kForces && !a.sym) {
            k_nn_wide<kForces, true><<<grid_for(tiles, kWideGroups, cus), kWideThreads, 0, st>>>(a);
        } else {
            k_nn_wide<MODE><<<grid_for(tiles, kWideGroups, cus), kWideThreads, 0, st>>>(a);
        }
    } else {
        constexpr int w = NNCfg<false, MODE>::waves;
        k_nn<MODE, false><<<grid_for(tiles, w, cus), w * kWave, 0, st>>>(a);
    }
    return hip_check(hipGetLastError(), "network kernel launch");
}

}  // namespace rb

using namespace rb;

extern "C" int rb_nn_pair_eval(const float *params, const float *norm, int precision, int64_t n_pairs,
                               const float *desc, float *energy, void *stream) {
    RB_REQUIRE(params && norm, "rb_nn_pair_eval: null params/norm");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_pair_eval: bad precision");
    RB_REQUIRE(n_pairs >= 0, "rb_nn_pair_eval: n_pairs < 0");
    if (n_pairs == 0) return RB_OK;
    RB_REQUIRE(desc && energy, "rb_nn_pair_eval: null desc/energy");
    NNArgs a = {};
    a.params = params;
    a.nm = norm_from_host(norm);
    a.P = n_pairs;
    a.desc = desc;
    a.stride = n_pairs;
    a.energy = energy;
    return launch<kEval>(a, precision, n_pairs, (hipStream_t)stream);
}

extern "C" int rb_nn_pair_grad(const float *params, const float *norm, int precision, int64_t n_pairs,
                               const float *desc, const float *gE, float *energy, float *dE_ddesc, float *pair_ft,
                               void *stream) {
    RB_REQUIRE(params && norm, "rb_nn_pair_grad: null params/norm");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_pair_grad: bad precision");
    RB_REQUIRE(n_pairs >= 0, "rb_nn_pair_grad: n_pairs < 0");
    if (n_pairs == 0) return RB_OK;
    RB_REQUIRE(desc, "rb_nn_pair_grad: null desc");
    NNArgs a = {};
    a.params = params;
    a.nm = norm_from_host(norm);
    a.P = n_pairs;
    a.desc = desc;
    a.stride = n_pairs;
    a.gE = gE;
    a.energy = energy;
    a.dEdu = dE_ddesc;
    a.ft = pair_ft;
    return launch<kGrad>(a, precision, n_pairs, (hipStream_t)stream);
}

extern "C" int rb_nn_pair_forces(const float *params, const float *norm, int precision, int32_t n, const double *q,
                                 const int32_t *pair_i, const int32_t *pair_j, const float *desc, int32_t desc_stride,
                                 const int32_t *idx, const int32_t *count_dev, int32_t max_count, float sw_lo,
                                 float sw_hi, int64_t *acc, int32_t *flags, void *stream) {
    RB_REQUIRE(params && norm && q && pair_i && pair_j && desc && count_dev && acc && flags,
               "rb_nn_pair_forces: null argument");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_pair_forces: bad precision");
    RB_REQUIRE(n > 0 && max_count >= 0 && desc_stride >= max_count, "rb_nn_pair_forces: bad sizes");
    if (max_count == 0) return RB_OK;
    NNArgs a = {};
    a.params = params;
    a.nm = norm_from_host(norm);
    a.P = max_count;
    a.desc = desc;
    a.stride = desc_stride;
    a.idx = idx;
    a.count_dev = count_dev;
    a.q = q;
    a.n = n;
    a.pi = pair_i;
    a.pj = pair_j;
    a.sw_lo = sw_lo;
    a.sw_hi = sw_hi;
    a.acc = acc;
    a.flags = flags;
    return launch<kForces>(a, precision, max_count, (hipStream_t)stream);
}

extern "C" int rb_nn_pair_forces_routed(const rb_ctx *ctx, const float *params, const float *norm, int precision,
                                        int form, int32_t n, const double *x, const double *q, const int32_t *type,
                                        const double *box, const int32_t *pair_i, const int32_t *pair_j,
                                        const float *desc, int32_t desc_stride, const int32_t *idx_nn,
                                        const int32_t *nn_count_dev, const int32_t *idx_bead,
                                        const int32_t *bead_count_dev, int32_t max_count, float sw_lo, float sw_hi,
                                        int64_t *acc, int32_t *flags, void *stream) {
    RB_REQUIRE(ctx && params && norm && x && q && type && box && pair_i && pair_j && desc && nn_count_dev &&
                   idx_bead && bead_count_dev && acc && flags,
               "rb_nn_pair_forces_routed: null argument");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_pair_forces_routed: bad precision");
    RB_REQUIRE(form == 0 || form == 1, "rb_nn_pair_forces_routed: form must be 0 ((d, q)) or 1 (cylinder)");
    RB_REQUIRE(n > 0 && max_count >= 0 && desc_stride >= max_count, "rb_nn_pair_forces_routed: bad sizes");
    RB_REQUIRE(box[0] > 0 && box[1] > 0 && box[2] > 0, "rb_nn_pair_forces_routed: box must be > 0");
    if (max_count == 0) return RB_OK;
    hipStream_t st = (hipStream_t)stream;
    NNArgs a = {};
    a.params = params;
    a.nm = norm_from_host(norm);
    a.P = max_count;
    a.desc = desc;
    a.stride = desc_stride;
    a.idx = idx_nn;
    a.count_dev = nn_count_dev;
    a.q = q;
    a.n = n;
    a.pi = pair_i;
    a.pj = pair_j;
    a.sw_lo = sw_lo;
    a.sw_hi = sw_hi;
    a.acc = acc;
    a.flags = flags;
    a.cyl = form;
    const int stride = (ctx->max_beads + 3) & ~3;
    const size_t need = sizeof(float4) * (3 * (size_t)stride * (kWideThreads / kWave) + (size_t)ctx->total_beads);
    if (precision != RB_PREC_BF16 || need > sizeof(LdsBF16) || max_count >= kFbMaxPairs) {
        const int rc = launch<kForces>(a, precision, max_count, st);
        if (rc != RB_OK) return rc;
        return rb_bead_pair_forces(ctx, n, x, q, type, box, pair_i, pair_j, idx_bead, bead_count_dev, max_count, acc,
                                   flags, stream);
    }
    a.idx_bead = idx_bead;
    a.bead_count = bead_count_dev;
    a.x = x;
    a.type = type;
    for (int k = 0; k < 3; ++k) {
        a.box.L[k] = box[k];
        a.box.inv[k] = 1.0 / box[k];
    }
    a.T = ctx->dev.t;
    a.lj = ctx->dev.lj;
    a.bead_stride = stride;
    const int64_t tiles = ((int64_t)max_count + kTile - 1) / kTile;
    const int grid = grid_for(tiles, kWideGroups, device_cu_count());
    if (ctx->dev.lj.kind == kPotHPHC)
        k_nn_wide<kForces, true, 2><<<grid, kWideThreads, 0, st>>>(a);
    else
        k_nn_wide<kForces, true, 1><<<grid, kWideThreads, 0, st>>>(a);
    return hip_check(hipGetLastError(), "rb_nn_pair_forces_routed launch");
}

extern "C" int rb_nn_pair_grad_sym(const float *params, const float *norm, int precision, int64_t n_pairs,
                                   const float *desc, const float *sym, const float *jac, const float *gE,
                                   float *energy, float *dE_ddesc, float *pair_ft, void *stream) {
    RB_REQUIRE(params && norm, "rb_nn_pair_grad_sym: null params/norm");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_pair_grad_sym: bad precision");
    RB_REQUIRE(n_pairs >= 0, "rb_nn_pair_grad_sym: n_pairs < 0");
    if (n_pairs == 0) return RB_OK;
    RB_REQUIRE(desc && sym && jac, "rb_nn_pair_grad_sym: null desc/sym/jac");
    NNArgs a = {};
    a.params = params;
    a.nm = norm_from_host(norm);
    a.P = n_pairs;
    a.desc = desc;
    a.stride = n_pairs;
    a.gE = gE;
    a.energy = energy;
    a.dEdu = dE_ddesc;
    a.ft = pair_ft;
    a.sym = sym;
    a.jac = jac;
    return launch<kGrad>(a, precision, n_pairs, (hipStream_t)stream);
}

extern "C" int rb_nn_pair_forces_sym(const float *params, const float *norm, int precision, int32_t n,
                                     const double *q, const int32_t *pair_i, const int32_t *pair_j,
                                     const float *desc, int32_t desc_stride, const float *sym, const float *jac,
                                     const int32_t *idx, const int32_t *count_dev, int32_t max_count, float sw_lo,
                                     float sw_hi, int64_t *acc, int32_t *flags, void *stream) {
    RB_REQUIRE(params && norm && q && pair_i && pair_j && desc && sym && jac && count_dev && acc && flags,
               "rb_nn_pair_forces_sym: null argument");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_pair_forces_sym: bad precision");
    RB_REQUIRE(n > 0 && max_count >= 0 && desc_stride >= max_count, "rb_nn_pair_forces_sym: bad sizes");
    if (max_count == 0) return RB_OK;
    NNArgs a = {};
    a.params = params;
    a.nm = norm_from_host(norm);
    a.P = max_count;
    a.desc = desc;
    a.stride = desc_stride;
    a.idx = idx;
    a.count_dev = count_dev;
    a.q = q;
    a.n = n;
    a.pi = pair_i;
    a.pj = pair_j;
    a.sw_lo = sw_lo;
    a.sw_hi = sw_hi;
    a.acc = acc;
    a.flags = flags;
    a.sym = sym;
    a.jac = jac;
    return launch<kForces>(a, precision, max_count, (hipStream_t)stream);
}

extern "C" int rb_nn_pair_forces_cyl(const float *params, const float *norm, int precision, int32_t n,
                                     const double *q, const int32_t *pair_i, const int32_t *pair_j,
                                     const float *desc, int32_t desc_stride, const int32_t *idx,
                                     const int32_t *count_dev, int32_t max_count, float sw_lo, float sw_hi,
                                     int64_t *acc, int32_t *flags, void *stream) {
    RB_REQUIRE(params && norm && q && pair_i && pair_j && desc && count_dev && acc && flags,
               "rb_nn_pair_forces_cyl: null argument");
    RB_REQUIRE(precision == RB_PREC_BF16 || precision == RB_PREC_FP32, "rb_nn_pair_forces_cyl: bad precision");
    RB_REQUIRE(n > 0 && max_count >= 0 && desc_stride >= max_count, "rb_nn_pair_forces_cyl: bad sizes");
    if (max_count == 0) return RB_OK;
    NNArgs a = {};
    a.params = params;
    a.nm = norm_from_host(norm);
    a.P = max_count;
    a.desc = desc;
    a.stride = desc_stride;
    a.idx = idx;
    a.count_dev = count_dev;
    a.q = q;
    a.n = n;
    a.pi = pair_i;
    a.pj = pair_j;
    a.sw_lo = sw_lo;
    a.sw_hi = sw_hi;
    a.acc = acc;
    a.flags = flags;
    a.cyl = 1;
    return launch<kForces>(a, precision, max_count, (hipStream_t)stream);
}
