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

__global__ void k_route_reset(int32_t *flags) {
    flags[RB_FLAG_NNN] = 0;
    flags[RB_FLAG_NBEAD] = 0;
}

// Appends this lane's pair to one of two lists with one atomic per wave and
// list (ballot + popcount of the lanes below).
__device__ inline void wave_append(bool take, int value, int32_t *list, int32_t *counter) {
    const unsigned long long m = __ballot(take);
    if (m == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    int base = 0;
    const int leader = __ffsll((long long)m) - 1;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader, kWave);
    if (take) {
        const unsigned long long below = m & ((1ull << lane) - 1ull);
        list[base + __popcll(below)] = value;
    }
}

__global__ __launch_bounds__(256) void k_descriptors(int32_t n, const double *__restrict__ x,
                                                     const double *__restrict__ q, double L0, double L1, double L2,
                                                     const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                                                     int32_t maxp, float dmin2, float dmax2, float *__restrict__ desc,
                                                     int32_t *__restrict__ idx_nn, int32_t *__restrict__ idx_bead,
                                                     int32_t *__restrict__ flags, Templates T,
                                                     const int32_t *__restrict__ type, double gap_min,
                                                     double gap_max) {
    // the first round's pair indices are requested together with the count
    // (any slot below the capacity may be read; only live ones are used)
    const int p0 = blockIdx.x * blockDim.x + threadIdx.x;
    int i0 = 0, j0 = 0;
    if (p0 < maxp) {
        i0 = pi[p0];
        j0 = pj[p0];
    }
    int count = flags[RB_FLAG_NPAIRS];
    if (count > maxp) count = maxp;
    const double Ls[3] = {L0, L1, L2};
    for (int base = blockIdx.x * blockDim.x; base < count; base += gridDim.x * blockDim.x) {
        const int p = base + threadIdx.x;
        const bool live = p < count;
        bool to_nn = false, to_bead = false;
        if (live) {
            const int i = p == p0 ? i0 : pi[p], j = p == p0 ? j0 : pj[p];
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
            bool near = r2 < (double)dmin2, far = false;
            if (type && in_range && !near) {
                double Rr[9];
                quat_to_rot<double>(rw, rx, ry, rz, Rr);
                const double G = shell_gap(T, type[i], type[j], d, Rr);
                near = G < gap_min;
                far = G >= gap_max;
            }
            to_nn = in_range && !near && !far;
            to_bead = in_range && near;
            if (!type) to_bead = near;    // no shells: every pair below d_min, as before
        }
        wave_append(live && to_nn, p, idx_nn, flags + RB_FLAG_NNN);
        wave_append(live && to_bead, p, idx_bead, flags + RB_FLAG_NBEAD);
    }
}

}  // namespace rb

using namespace rb;

extern "C" int rb_pair_descriptors(int32_t n, const double *x, const double *q, const double *box,
                                   const int32_t *pair_i, const int32_t *pair_j, int32_t max_pairs, float d_min,
                                   float d_max, float *desc, int32_t *idx_nn, int32_t *idx_bead, int32_t *flags,
                                   const rb_ctx *ctx, const int32_t *type, float gap_min, float gap_max,
                                   void *stream) {
    RB_REQUIRE(x && q && box && pair_i && pair_j && desc && idx_nn && idx_bead && flags,
               "rb_pair_descriptors: null argument");
    RB_REQUIRE(!ctx == !type, "rb_pair_descriptors: ctx and type go together");
    RB_REQUIRE(n > 0 && max_pairs > 0, "rb_pair_descriptors: sizes must be > 0");
    RB_REQUIRE(box[0] > 0 && box[1] > 0 && box[2] > 0, "rb_pair_descriptors: box must be > 0");
    hipStream_t st = (hipStream_t)stream;
    k_route_reset<<<1, 1, 0, st>>>(flags);
    const float dm2 = d_min > 0 ? d_min * d_min : 0.f;
    const float dx2 = d_max > 0 ? d_max * d_max : 3.0e38f;
    Templates T = {};
    if (ctx) T = ctx->dev.t;
    const double gmax = gap_max > 0.f ? (double)gap_max : 1e300;
    k_descriptors<<<grid_for(max_pairs, 256, 4096), 256, 0, st>>>(n, x, q, box[0], box[1], box[2], pair_i, pair_j,
                                                                  max_pairs, dm2, dx2, desc, idx_nn, idx_bead, flags,
                                                                  T, type, (double)gap_min, gmax);
    RB_LAUNCH_CHECK("rb_pair_descriptors");
    return RB_OK;
}
