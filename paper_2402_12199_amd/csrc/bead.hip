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
#include "bead_pair.hpp"
#include "shells.hpp"

namespace rb {

constexpr int kBeadWaves = 4;        // waves per block (per-pair form)
constexpr int kMdWaves = 8;          // waves per block (per-body form: one work queue per block)

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
            // one template: uniform shell sizes, no type loads
            const bool one = T.n_types == 1;
            ti = one ? 0 : type[i];
            tj = one ? 0 : type[j];
            double R[9], Ri[9];
            pair_frame(n, x, q, box, i, j, dl, d, qr, qa, Ri);
            quat_to_rot<double>(qr[0], qr[1], qr[2], qr[3], R);
            // the shells' bound on the closest bead distance (box, and for
            // cylinder-like types capsule and cylinder) decides which pairs
            // can have a bead pair within rc
            auto route = [&](float gap_max) {
                return one ? shell_route(T, 0, 0, d, R, 0.f, gap_max) : shell_route(T, ti, tj, d, R, 0.f, gap_max);
            };
            hit = route(rcm) != kRouteSkip;
            if (SCREENED && full) wide = hit || route(S.rcm_wide) != kRouteSkip;
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
