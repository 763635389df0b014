// Pair descriptors and routing.
//
// Paper section 2: the configuration of a pair is fixed by the position and
// the orientation of body j in the frame of body i.  Here that is
// d = R_i^T minimg(x_j - x_i) and q = q_i^* q_j (R(q) = R_i^T R_j), computed
// in FP64 from the state and stored in FP32 (7 x max_pairs, SoA).  Pairs
// outside the network's training domain go to the bead sum: |d| < d_min,
// and, with shells given, pairs whose lower bound on the closest bead
// distance is below gap_min.  Pairs with d_min <= |d| < d_max and a bound of
// at least gap_min (and below gap_max) go to the network; pairs beyond
// d_max (zero switched network energy) or with a bound of gap_max or more
// (no bead pair within gap_max) go to neither.
#include "rb_common.hpp"
#include "shells.hpp"

namespace rb {

constexpr int kDescThreads = 1024;
constexpr int kDescWaves = kDescThreads / kWave;

// The working word of the appends (64 bits at flags + RB_FLAG_ROUTE_WORK):
// the network list's count in bits 0..26, the bead list's in bits 27..53 and
// the finishing ticket (blocks done) in bits 54..63.  One atomic per block
// then reserves both ranges and takes the ticket, and its return value holds
// every other block's contribution.
constexpr int kRouteCountBits = 27;
constexpr unsigned long long kRouteCountMask = (1ull << kRouteCountBits) - 1ull;
constexpr int kRouteTicketShift = 2 * kRouteCountBits;
constexpr int kRouteMaxBlocks = (1 << (64 - kRouteTicketShift)) - 1;

// Appends the block's lanes with take0 / take1 to two lists with one atomic
// per block (many waves adding to one counter serialise on it): ballots give
// each wave's count and each lane's rank in its wave, the wave counts are
// scanned in LDS, thread 0 reserves the block's ranges (and takes the ticket
// in the block's final round).  With CAND the lanes with take2 go to a third
// list through their own counter (work2), whose atomic has returned before
// the barrier that precedes the ticket, so that the last block finds every
// block's reservation in it.  Every thread of the block calls it.  Returns
// true in every thread of the last block to finish, with the lists' final
// lengths in n0, n1.
template <bool CAND>
__device__ inline bool block_append(bool take0, bool take1, bool take2, int value, int32_t *list0, int32_t *list1,
                                    int32_t *list2, unsigned long long *work, int32_t *work2, bool final_round,
                                    int nactive, int &n0, int &n1) {
    __shared__ int wcount[3][kDescWaves];
    __shared__ int base[3], total[2];
    __shared__ bool last;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    const unsigned long long m0 = __ballot(take0), m1 = __ballot(take1), m2 = CAND ? __ballot(take2) : 0ull;
    if (lane == 0) {
        wcount[0][w] = __popcll(m0);
        wcount[1][w] = __popcll(m1);
        if (CAND) wcount[2][w] = __popcll(m2);
    }
    __syncthreads();
    if (CAND) {
        if (threadIdx.x == 0) {
            int t2 = 0;
            for (int k = 0; k < kDescWaves; ++k) t2 += wcount[2][k];
            base[2] = t2 ? atomicAdd(work2, t2) : 0;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int t0 = 0, t1 = 0;
        for (int k = 0; k < kDescWaves; ++k) {
            t0 += wcount[0][k];
            t1 += wcount[1][k];
        }
        const unsigned long long add = (unsigned long long)t0 | ((unsigned long long)t1 << kRouteCountBits) |
                                       (final_round ? 1ull << kRouteTicketShift : 0ull);
        const unsigned long long old = add ? atomicAdd(work, add) : 0ull;
        base[0] = (int)(old & kRouteCountMask);
        base[1] = (int)((old >> kRouteCountBits) & kRouteCountMask);
        total[0] = base[0] + t0;
        total[1] = base[1] + t1;
        last = final_round && (int)(old >> kRouteTicketShift) == nactive - 1;
    }
    __syncthreads();
    int off0 = base[0], off1 = base[1], off2 = CAND ? base[2] : 0;
    for (int k = 0; k < w; ++k) {
        off0 += wcount[0][k];
        off1 += wcount[1][k];
        if (CAND) off2 += wcount[2][k];
    }
    const unsigned long long below = (1ull << lane) - 1ull;
    if (take0) list0[off0 + __popcll(m0 & below)] = value;
    if (take1) list1[off1 + __popcll(m1 & below)] = value;
    if (CAND && take2) list2[off2 + __popcll(m2 & below)] = value;
    n0 = total[0];
    n1 = total[1];
    const bool is_last = last;
    __syncthreads();   // the shared words are reused by the next round
    return is_last;
}

// Screened routing (rb_pair_descriptors_screened): the candidates kept by a
// screening launch, and the reference state, as in the bead path's two-level
// list.
struct RouteScreen {
    int32_t *list;           // candidate pair indices (capacity max_pairs)
    double *x_ref, *q_ref;   // state at the screening (3 x n, 4 x n)
    float margin;
};

// SCREENED: a launch with flags[RESCREEN] set routes every listed pair and
// rebuilds the candidate list (the pairs that can still be routed while no
// bead has moved margin / 2: centres closer than d_max + margin, and closer
// than d_min + margin or with the shells' bound below gap_max + margin); a
// launch with the flag clear routes the candidates only.  A candidate is
// routed exactly as by a launch over the whole list.  ONE: the context has a
// single template, so the shells' sizes are the same for every pair (uniform
// values, no type loads).
template <bool SCREENED, bool ONE>
__global__ __launch_bounds__(kDescThreads) void k_descriptors(int32_t n, const double *__restrict__ x,
                                                     const double *__restrict__ q, double L0, double L1, double L2,
                                                     const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                                                     int32_t maxp, float dmin2, float dmax2, float *__restrict__ desc,
                                                     int32_t *__restrict__ idx_nn, int32_t *__restrict__ idx_bead,
                                                     int32_t *__restrict__ flags, Templates T,
                                                     const int32_t *__restrict__ type, float gap_min,
                                                     float gap_max, RouteScreen S) {
    // Each block takes a span of the list: the count spread evenly over the
    // grid (one block per CU) in whole waves, at most the block's threads, so
    // that every CU has work and none more than its share; lists longer than
    // the grid's threads take several rounds.  Appends go through the
    // working word; the last block to finish publishes the counts and clears
    // it for the next call.
    const bool full = !SCREENED || flags[RB_FLAG_RESCREEN] != 0;
    int count = full ? flags[RB_FLAG_NPAIRS] : flags[RB_FLAG_NSCREEN];
    if (count > maxp) count = maxp;
    unsigned long long *work = reinterpret_cast<unsigned long long *>(flags + RB_FLAG_ROUTE_WORK);
    int32_t *work2 = flags + RB_FLAG_ROUTE_WORK + 2;
    if (SCREENED && full) {
        // the reference state of this screening
        for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n; b += gridDim.x * blockDim.x) {
#pragma unroll
            for (int a = 0; a < 3; ++a) S.x_ref[a * n + b] = x[a * n + b];
#pragma unroll
            for (int a = 0; a < 4; ++a) S.q_ref[a * n + b] = q[a * n + b];
        }
    }
    int span = (count + (int)gridDim.x - 1) / (int)gridDim.x;
    span = min((int)blockDim.x, max(kWave, (span + kWave - 1) / kWave * kWave));
    // only the blocks with pairs take part (and take the completion ticket);
    // with no pairs block 0 publishes zeros
    const int nactive = min((int)gridDim.x, (count + span - 1) / span);
    if ((int)blockIdx.x >= nactive) {
        if (nactive == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
            flags[RB_FLAG_NNN] = 0;
            flags[RB_FLAG_NBEAD] = 0;
            if (SCREENED && full) {
                flags[RB_FLAG_NSCREEN] = 0;
                flags[RB_FLAG_RESCREEN] = 0;
                flags[RB_FLAG_NRESCREENS] += 1;
            }
        }
        return;
    }
    const double Ls[3] = {L0, L1, L2};
    const float dcand2 = SCREENED ? (sqrtf(dmax2) + S.margin) * (sqrtf(dmax2) + S.margin) : 0.f;
    const float dnear2 = SCREENED ? (sqrtf(dmin2) + S.margin) * (sqrtf(dmin2) + S.margin) : 0.f;
    const float gap_exit = SCREENED && full ? gap_max + S.margin : gap_max;
    const int stride = gridDim.x * span;
    for (int base = blockIdx.x * span; base < count; base += stride) {
        const int item = base + threadIdx.x;
        const bool live = (int)threadIdx.x < span && item < count;
        bool to_nn = false, to_bead = false, cand = false;
        int p = item;
        if (live) {
            if (SCREENED && !full) p = S.list[item];
            const int i = pi[p], j = pj[p];
            double dl[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) dl[a] = min_image(x[a * n + j] - x[a * n + i], Ls[a], 1.0 / Ls[a]);
            const double w = q[i], vx = q[n + i], vy = q[2 * n + i], vz = q[3 * n + i];
            double R[9];
            quat_to_rot<double>(w, vx, vy, vz, R);
            double d[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) d[a] = R[a] * dl[0] + R[3 + a] * dl[1] + R[6 + a] * dl[2];
            // q_i^* q_j
            const double bw = q[j], bx = q[n + j], by = q[2 * n + j], bz = q[3 * n + j];
            const double rw = w * bw + vx * bx + vy * by + vz * bz;
            const double rx = w * bx - vx * bw - vy * bz + vz * by;
            const double ry = w * by + vx * bz - vy * bw - vz * bx;
            const double rz = w * bz - vx * by + vy * bx - vz * bw;
            desc[p] = (float)d[0];
            desc[maxp + p] = (float)d[1];
            desc[2 * maxp + p] = (float)d[2];
            desc[3 * maxp + p] = (float)rw;
            desc[4 * maxp + p] = (float)rx;
            desc[5 * maxp + p] = (float)ry;
            desc[6 * maxp + p] = (float)rz;
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const bool in_range = r2 < (double)dmax2;
            bool near = r2 < (double)dmin2, far = false, keep = true;
            if (type && in_range && !near) {
                double Rr[9];
                quat_to_rot<double>(rw, rx, ry, rz, Rr);
                const int route = ONE ? shell_route(T, 0, 0, d, Rr, gap_min, gap_max, gap_exit, &keep)
                                      : shell_route(T, type[i], type[j], d, Rr, gap_min, gap_max, gap_exit, &keep);
                near = route == kRouteBead;
                far = route == kRouteSkip;
            }
            to_nn = in_range && !near && !far;
            to_bead = in_range && near;
            if (!type) to_bead = near;    // no shells: every pair below d_min, as before
            if (SCREENED && full)
                cand = r2 < (double)dcand2 && (!in_range || r2 < (double)dnear2 || keep);
        }
        int nn = 0, nb = 0;
        const bool final_round = base + stride >= count;
        if (block_append<SCREENED>(live && to_nn, live && to_bead, SCREENED && full && live && cand, p, idx_nn,
                                   idx_bead, S.list, work, work2, final_round, nactive, nn, nb) &&
            threadIdx.x == 0) {
            // every block's atomic is in the value this one returned: the
            // counts are final and the word can be cleared.  No fence: the
            // counts reach their consumers through the kernel boundary.
            flags[RB_FLAG_NNN] = nn;
            flags[RB_FLAG_NBEAD] = nb;
            *work = 0ull;
            if (SCREENED && full) {
                // every block's candidate atomic returned before its ticket
                flags[RB_FLAG_NSCREEN] = __hip_atomic_load(work2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                *work2 = 0;
                flags[RB_FLAG_RESCREEN] = 0;
                flags[RB_FLAG_NRESCREENS] += 1;
            }
        }
    }
}

}  // namespace rb

using namespace rb;

static int route_launch(const char *who, int32_t n, const double *x, const double *q, const double *box,
                        const int32_t *pair_i, const int32_t *pair_j, int32_t max_pairs, float d_min, float d_max,
                        float *desc, int32_t *idx_nn, int32_t *idx_bead, int32_t *flags, const rb_ctx *ctx,
                        const int32_t *type, float gap_min, float gap_max, const RouteScreen *S, void *stream) {
    RB_REQUIRE(x && q && box && pair_i && pair_j && desc && idx_nn && idx_bead && flags, "%s: null argument", who);
    RB_REQUIRE(!ctx == !type, "%s: ctx and type go together", who);
    RB_REQUIRE(n > 0 && max_pairs > 0, "%s: sizes must be > 0", who);
    RB_REQUIRE(max_pairs <= (int32_t)kRouteCountMask, "%s: max_pairs must be below 2^27", who);
    RB_REQUIRE(((uintptr_t)flags & 7) == 0, "%s: flags must be 8-byte aligned", who);
    RB_REQUIRE(box[0] > 0 && box[1] > 0 && box[2] > 0, "%s: box must be > 0", who);
    hipStream_t st = (hipStream_t)stream;
    const float dm2 = d_min > 0 ? d_min * d_min : 0.f;
    const float dx2 = d_max > 0 ? d_max * d_max : 3.0e38f;
    Templates T = {};
    if (ctx) T = ctx->dev.t;
    const float gmax = gap_max > 0.f ? gap_max : 3.0e38f;
    const int grid = grid_for(max_pairs, kWave, std::min(device_cu_count(), kRouteMaxBlocks));
    const bool one = ctx && ctx->n_types == 1;
    const RouteScreen S0 = S ? *S : RouteScreen{};
    auto go = [&](auto kernel) {
        kernel<<<grid, kDescThreads, 0, st>>>(n, x, q, box[0], box[1], box[2], pair_i, pair_j, max_pairs, dm2, dx2,
                                              desc, idx_nn, idx_bead, flags, T, type, gap_min, gmax, S0);
    };
    if (S)
        one ? go(k_descriptors<true, true>) : go(k_descriptors<true, false>);
    else
        one ? go(k_descriptors<false, true>) : go(k_descriptors<false, false>);
    RB_LAUNCH_CHECK(who);
    return RB_OK;
}

extern "C" int rb_pair_descriptors(int32_t n, const double *x, const double *q, const double *box,
                                   const int32_t *pair_i, const int32_t *pair_j, int32_t max_pairs, float d_min,
                                   float d_max, float *desc, int32_t *idx_nn, int32_t *idx_bead, int32_t *flags,
                                   const rb_ctx *ctx, const int32_t *type, float gap_min, float gap_max,
                                   void *stream) {
    return route_launch("rb_pair_descriptors", n, x, q, box, pair_i, pair_j, max_pairs, d_min, d_max, desc, idx_nn,
                        idx_bead, flags, ctx, type, gap_min, gap_max, nullptr, stream);
}

extern "C" int rb_pair_descriptors_screened(int32_t n, const double *x, const double *q, const double *box,
                                            const int32_t *pair_i, const int32_t *pair_j, int32_t max_pairs,
                                            float d_min, float d_max, float *desc, int32_t *idx_nn,
                                            int32_t *idx_bead, int32_t *flags, const rb_ctx *ctx,
                                            const int32_t *type, float gap_min, float gap_max, float margin,
                                            int32_t *cand_list, double *x_sref, double *q_sref, void *stream) {
    RB_REQUIRE(ctx && type && cand_list && x_sref && q_sref, "rb_pair_descriptors_screened: null argument");
    RB_REQUIRE(margin >= 0.f && margin < 1e6f, "rb_pair_descriptors_screened: margin must be in [0, 1e6)");
    RB_REQUIRE(gap_max > 0.f, "rb_pair_descriptors_screened: gap_max must be > 0");
    const RouteScreen S{cand_list, x_sref, q_sref, margin};
    return route_launch("rb_pair_descriptors_screened", n, x, q, box, pair_i, pair_j, max_pairs, d_min, d_max, desc,
                        idx_nn, idx_bead, flags, ctx, type, gap_min, gap_max, &S, stream);
}
