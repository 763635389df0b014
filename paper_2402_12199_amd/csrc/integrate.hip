// Rigid-body velocity Verlet in FP64 with the NO_SQUISH free-rotation
// splitting (Miller, Eleftheriou, Pattnaik, Ndirango, Newns, Martyna,
// J. Chem. Phys. 116, 8649 (2002)).  The paper itself only fixes the time
// step (section 3, dt = 0.005 tau).
//
// The rotational state is kept as the body-frame angular momentum L.  The
// NO_SQUISH sub-step about body axis k over a time h is the exact flow of
// the k-th kinetic term L_k^2 / (2 I_k): the body turns by the angle
// h L_k / I_k about its own axis k, i.e. q <- q (cos z, sin z e_k) with
// z = h L_k / (2 I_k), and L turns by -2z about the same axis, which keeps
// the lab-frame angular momentum fixed.  A kick adds the body-frame torque:
// L <- L + (dt/2) R(q)^T tau.
//
// Constant temperature (the paper's ensemble, section 3: Nose-Hoover): one
// thermostat variable xi with mass Q acts on every momentum, translational
// and angular, through the flow dP/dt = -xi P, dL/dt = -xi L,
// dxi/dt = (2K - g kT) / Q, deta/dt = xi (g degrees of freedom, K the total
// kinetic energy).  Split as U_T(dt/2) U_T(dt/2) after each velocity-Verlet
// step (the end-of-step half and the next step's opening half), each half
// U_T(h): xi += (h/2) G(K); P, L *= exp(-xi h); eta += xi h;
// xi += (h/2) G(K') with G(K) = (2K - g kT) / Q and K' = exp(-2 xi h) K.
// Only the total kinetic energy enters, so the last block of the phase-2
// reduction does the whole update and leaves the momentum scale factor, which
// the next phase 1 applies before its half kick.  The conserved quantity is
// K + U + Q xi^2 / 2 + g kT eta.

// Multiply-add fusion only inside one source expression (also for the
// helpers of the common header, hence before it): the fused step kernel
// repeats the arithmetic of the two phase kernels and must round the same
// way, which fusion across statements, chosen per kernel, would break.
#pragma clang fp contract(on)
#include "rb_common.hpp"

#include <mutex>

namespace rb {

constexpr int kIntThreads = 256;

struct Sub {
    int k;
    double h;
};

// sin and cos of a sub-step's half angle.  The angles of a step are tiny
// (|z| ~ 1e-4 at the workloads' temperatures); below 2^-7 the Taylor series
// to z^7 (sin) and z^8 (cos) is exact to FP64 rounding (the next terms are
// below 2^-60 relative), which skips the library's range reduction.
__device__ inline void half_angle_sincos(double z, double &s, double &c) {
    if (fabs(z) < 0x1p-7) {
        const double z2 = z * z;
        s = z * (1.0 - z2 * (1.0 / 6.0 - z2 * (1.0 / 120.0 - z2 * (1.0 / 5040.0))));
        c = 1.0 - z2 * (0.5 - z2 * (1.0 / 24.0 - z2 * (1.0 / 720.0 - z2 * (1.0 / 40320.0))));
    } else {
        sincos(z, &s, &c);
    }
}

__device__ inline void free_sub(int k, double h, double I, double q[4], double L[3]) {
    const double z = h * L[k] / (2.0 * I);
    double s, c;
    half_angle_sincos(z, s, c);
    // q <- q * (c, s e_k), written out per axis
    const double w = q[0], x = q[1], y = q[2], zz = q[3];
    if (k == 0) {
        q[0] = c * w - s * x; q[1] = c * x + s * w; q[2] = c * y + s * zz; q[3] = c * zz - s * y;
    } else if (k == 1) {
        q[0] = c * w - s * y; q[1] = c * x - s * zz; q[2] = c * y + s * w; q[3] = c * zz + s * x;
    } else {
        q[0] = c * w - s * zz; q[1] = c * x + s * y; q[2] = c * y - s * x; q[3] = c * zz + s * w;
    }
    // L turns by -2z about axis k: (L_a, L_b) with (k, a, b) cyclic
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    const double c2 = c * c - s * s, s2 = 2.0 * s * c;
    const double La = L[a], Lb = L[b];
    L[a] = c2 * La + s2 * Lb;
    L[b] = -s2 * La + c2 * Lb;
}

// Half kick with the body's force f and lab-frame torque tq (turned into
// the body frame of the angular momentum L).
__device__ inline void kick_with(double dt, double q[4], double P[3], double L[3], const float f[3],
                                 const float tq[3]) {
    double R[9];
    quat_to_rot<double>(q[0], q[1], q[2], q[3], R);
    const double t[3] = {tq[0], tq[1], tq[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        P[a] += 0.5 * dt * (double)f[a];
        L[a] += 0.5 * dt * (R[a] * t[0] + R[3 + a] * t[1] + R[6 + a] * t[2]);
    }
}

__device__ inline void kick(double dt, double q[4], double P[3], double L[3], const float *force,
                            const float *torque, int n, int i) {
    const float f[3] = {force[i], force[n + i], force[2 * n + i]};
    const float tq[3] = {torque[i], torque[n + i], torque[2 * n + i]};
    kick_with(dt, q, P, L, f, tq);
}

// Displacement watch of the lists built from an earlier state.  Pair list:
// raise the rebuild flag when a centre has moved by more than half the skin
// since the build (x_ref).  Screened list of the two-level bead sum: raise
// the rescreen flag when some bead of a body may have moved by more than
// half the screening margin since the screening (x_sref, q_sref): a bead at
// radius rho moves by at most |dx| + 2 rho |vec(q_ref^* q)| = |dx| +
// 2 rho sin(theta / 2) under a displacement dx and a rotation by theta.
struct Watch {
    const double *x_ref;
    double half_skin2;
    const double *x_sref, *q_sref;
    double half_margin;
    double rho[kMaxTypes];   // largest bead radius per type, rounded up
};

// The body's reference positions and orientation of the watch (zeros for
// the lists the watch does not follow).
struct WatchRef {
    double x[3], xs[3], qs[4];
};

__device__ inline WatchRef watch_ref(const Watch &wt, int32_t n, int i) {
    WatchRef r = {};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (wt.x_ref) r.x[a] = wt.x_ref[a * n + i];
        if (wt.x_sref) r.xs[a] = wt.x_sref[a * n + i];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
        if (wt.x_sref) r.qs[a] = wt.q_sref[a * n + i];
    return r;
}

__device__ inline void watch_with(const Watch &wt, const WatchRef &r, int t, const double xn[3], const double qn[4],
                                  bool &rebuild, bool &rescreen) {
    if (wt.x_ref) {
        double d2 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double dd = xn[a] - r.x[a];
            d2 += dd * dd;
        }
        rebuild = d2 > wt.half_skin2;
    }
    if (wt.x_sref) {
        double d2 = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double dd = xn[a] - r.xs[a];
            d2 += dd * dd;
        }
        const double sw = r.qs[0], sx = r.qs[1], sy = r.qs[2], sz = r.qs[3];
        // vector part of q_ref^* q = sw v - w s - s x v
        const double vx = sw * qn[1] - qn[0] * sx - (sy * qn[3] - sz * qn[2]);
        const double vy = sw * qn[2] - qn[0] * sy - (sz * qn[1] - sx * qn[3]);
        const double vz = sw * qn[3] - qn[0] * sz - (sx * qn[2] - sy * qn[1]);
        rescreen = sqrt(d2) + 2.0 * wt.rho[t] * sqrt(vx * vx + vy * vy + vz * vz) > wt.half_margin;
    }
}

__device__ inline void watch(const Watch &wt, int32_t n, int i, int t, const double xn[3], const double qn[4],
                             bool &rebuild, bool &rescreen) {
    watch_with(wt, watch_ref(wt, n, i), t, xn, qn, rebuild, rescreen);
}

__device__ inline void raise_flags(bool rebuild, bool rescreen, int32_t *flags) {
    const bool lead = (threadIdx.x & (kWave - 1)) == 0;
    if (__any(rebuild) && lead) atomicOr(flags + RB_FLAG_REBUILD, 1);
    if (__any(rescreen) && lead) atomicOr(flags + RB_FLAG_RESCREEN, 1);
}

// Renormalises q in place; returns true when |q|^2 had drifted from 1 by
// more than 1e-10 (or was not finite) before the renormalisation.
__device__ inline bool renormalise(double qi[4]) {
    const double n2 = qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3];
    const double inv = 1.0 / sqrt(n2);
#pragma unroll
    for (int a = 0; a < 4; ++a) qi[a] *= inv;
    return !(fabs(n2 - 1.0) <= 1.0e-10);
}

// Adds the number of drifted quaternions of the wave to flags[QDRIFT].
__device__ inline void count_drift(bool drift, int32_t *flags) {
    const unsigned long long m = __ballot(drift);
    if (m && (threadIdx.x & (kWave - 1)) == 0 && flags) atomicAdd(flags + RB_FLAG_QDRIFT, (int)__popcll(m));
}

// Grid-wide sums of (a, b) into out[0..1]: wave and block sums, one partial
// pair per block, and the last block to finish adds the partials in a fixed
// tree order (lane k takes blocks k, k + 64, ...), so the result depends only
// on the grid size.
__device__ inline bool grid_sum2(double a, double b, double *__restrict__ partial, unsigned *__restrict__ ticket,
                                 double *__restrict__ out) {
    __shared__ double red[2][kIntThreads / kWave];
    __shared__ bool last;
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = a;
        red[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0, sb = 0;
        for (int k = 0; k < kIntThreads / kWave; ++k) {
            sa += red[0][k];
            sb += red[1][k];
        }
        partial[2 * blockIdx.x] = sa;
        partial[2 * blockIdx.x + 1] = sb;
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last && w == 0) {
        __threadfence();
        double sa = 0, sb = 0;
        for (int k = lane; k < (int)gridDim.x; k += kWave) {
            sa += __hip_atomic_load(partial + 2 * k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sb += __hip_atomic_load(partial + 2 * k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        sa = wave_sum(sa);
        sb = wave_sum(sb);
        if (lane == 0) {
            out[0] = sa;
            out[1] = sb;
            *ticket = 0u;
            return true;
        }
    }
    return false;
}

// Nose-Hoover state (caller-owned device doubles): xi, eta, the momentum
// scale for the next phase 1, Q, g kT.
constexpr int kNhXi = 0, kNhEta = 1, kNhScale = 2, kNhQ = 3, kNhGkT = 4;

__device__ inline void nh_update(double *nh, double K, double dt) {
    double xi = nh[kNhXi], eta = nh[kNhEta], scale = 1.0;
    const double Q = nh[kNhQ], gkT = nh[kNhGkT], h = 0.5 * dt;
    for (int half = 0; half < 2; ++half) {
        xi += 0.5 * h * (2.0 * K - gkT) / Q;
        const double s = exp(-xi * h);
        eta += xi * h;
        K *= s * s;
        scale *= s;
        xi += 0.5 * h * (2.0 * K - gkT) / Q;
    }
    nh[kNhXi] = xi;
    nh[kNhEta] = eta;
    nh[kNhScale] = scale;
}

__global__ __launch_bounds__(kIntThreads) void k_phase1(int32_t n, double dt, double *__restrict__ x,
                                                        double *__restrict__ P, double *__restrict__ q,
                                                        double *__restrict__ L, const int32_t *__restrict__ type,
                                                        const double *__restrict__ mass,
                                                        const double *__restrict__ inertia,
                                                        const float *__restrict__ force,
                                                        const float *__restrict__ torque, Watch wt,
                                                        int32_t *__restrict__ flags, const double *__restrict__ nh) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool rebuild = false, rescreen = false, drift = false;
    if (i < n) {
        const int t = type[i];
        double qi[4] = {q[i], q[n + i], q[2 * n + i], q[3 * n + i]};
        double Pi[3] = {P[i], P[n + i], P[2 * n + i]};
        double Li[3] = {L[i], L[n + i], L[2 * n + i]};
        if (nh) {
            const double s = nh[kNhScale];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                Pi[a] *= s;
                Li[a] *= s;
            }
        }
        kick(dt, qi, Pi, Li, force, torque, n, i);
        const double im = 1.0 / mass[t];
        double xn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xn[a] = x[a * n + i] + dt * Pi[a] * im;
            x[a * n + i] = xn[a];
        }
        const double I[3] = {inertia[3 * t], inertia[3 * t + 1], inertia[3 * t + 2]};
        free_sub(2, 0.5 * dt, I[2], qi, Li);
        free_sub(1, 0.5 * dt, I[1], qi, Li);
        free_sub(0, dt, I[0], qi, Li);
        free_sub(1, 0.5 * dt, I[1], qi, Li);
        free_sub(2, 0.5 * dt, I[2], qi, Li);
        drift = renormalise(qi);
#pragma unroll
        for (int a = 0; a < 4; ++a) q[a * n + i] = qi[a];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P[a * n + i] = Pi[a];
            L[a * n + i] = Li[a];
        }
        watch(wt, n, i, t, xn, qi, rebuild, rescreen);
    }
    raise_flags(rebuild, rescreen, flags);
    count_drift(drift, flags);
}

// Second half kick; per-block FP64 kinetic partial sums, summed in block
// order by the last block to finish, so the result is deterministic.
__global__ __launch_bounds__(kIntThreads) void k_phase2(int32_t n, double dt, double *__restrict__ P,
                                                        const double *__restrict__ q, double *__restrict__ L,
                                                        const int32_t *__restrict__ type,
                                                        const double *__restrict__ mass,
                                                        const double *__restrict__ inertia,
                                                        const float *__restrict__ force,
                                                        const float *__restrict__ torque,
                                                        double *__restrict__ partial, unsigned *__restrict__ ticket,
                                                        double *__restrict__ kinetic, double *__restrict__ nh) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double kt = 0, kr = 0;
    if (i < n) {
        const int t = type[i];
        double qi[4] = {q[i], q[n + i], q[2 * n + i], q[3 * n + i]};
        double Pi[3] = {P[i], P[n + i], P[2 * n + i]};
        double Li[3] = {L[i], L[n + i], L[2 * n + i]};
        kick(dt, qi, Pi, Li, force, torque, n, i);
        const double m = mass[t];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P[a * n + i] = Pi[a];
            L[a * n + i] = Li[a];
            kt += Pi[a] * Pi[a] / (2.0 * m);
            kr += Li[a] * Li[a] / (2.0 * inertia[3 * t + a]);
        }
    }
    if (grid_sum2(kt, kr, partial, ticket, kinetic) && nh) nh_update(nh, kinetic[0] + kinetic[1], dt);
}

// Fused step boundary: the forces of step k come from the fixed-point
// accumulator (converted to FP32 exactly as rb_accum_finalize does, stored,
// and the accumulator cleared); then the second half kick of step k, the
// kinetic energy at the full step, and the first half kick, drift and free
// rotation of step k + 1.  Same arithmetic, in the same order, as
// rb_accum_finalize + phase 2 + phase 1.
__global__ __launch_bounds__(kIntThreads) void k_fused(int32_t n, double dt, double *__restrict__ x,
                                                       double *__restrict__ P, double *__restrict__ q,
                                                       double *__restrict__ L, const int32_t *__restrict__ type,
                                                       const double *__restrict__ mass,
                                                       const double *__restrict__ inertia, int64_t *__restrict__ acc,
                                                       float *__restrict__ force, float *__restrict__ torque,
                                                       double *__restrict__ ev, Watch wt, int32_t *__restrict__ flags,
                                                       double *__restrict__ partial, unsigned *__restrict__ ticket,
                                                       double *__restrict__ kinetic, int one_type) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double s = 1.0 / RB_ACC_SCALE;
    double kt = 0, kr = 0;
    bool rebuild = false, rescreen = false, drift = false, ovf = false;
    if (i < n) {
        // every load of the body first (accumulator, state, the watch's
        // references; with one template no type load), then the arithmetic
        long long fw[3], tw[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            fw[a] = acc[a * (int64_t)n + i];
            tw[a] = acc[(3 + a) * (int64_t)n + i];
        }
        const int t = one_type ? 0 : type[i];
        double qi[4] = {q[i], q[n + i], q[2 * n + i], q[3 * n + i]};
        double Pi[3] = {P[i], P[n + i], P[2 * n + i]};
        double Li[3] = {L[i], L[n + i], L[2 * n + i]};
        const double x0[3] = {x[i], x[n + i], x[2 * n + i]};
        const WatchRef ref = watch_ref(wt, n, i);
        float f[3], tq[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ovf |= !fix_word_ok(fw[a]) || !fix_word_ok(tw[a]);
            f[a] = (float)((double)fw[a] * s);
            tq[a] = (float)((double)tw[a] * s);
            force[a * n + i] = f[a];
            torque[a * n + i] = tq[a];
            acc[a * (int64_t)n + i] = 0;
            acc[(3 + a) * (int64_t)n + i] = 0;
        }
        kick_with(dt, qi, Pi, Li, f, tq);
        const double m = mass[t];
        const double I[3] = {inertia[3 * t], inertia[3 * t + 1], inertia[3 * t + 2]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            kt += Pi[a] * Pi[a] / (2.0 * m);
            kr += Li[a] * Li[a] / (2.0 * I[a]);
        }
        // next step: half kick, drift, free rotation
        kick_with(dt, qi, Pi, Li, f, tq);
        const double im = 1.0 / m;
        double xn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xn[a] = x0[a] + dt * Pi[a] * im;
            x[a * n + i] = xn[a];
        }
        free_sub(2, 0.5 * dt, I[2], qi, Li);
        free_sub(1, 0.5 * dt, I[1], qi, Li);
        free_sub(0, dt, I[0], qi, Li);
        free_sub(1, 0.5 * dt, I[1], qi, Li);
        free_sub(2, 0.5 * dt, I[2], qi, Li);
        drift = renormalise(qi);
#pragma unroll
        for (int a = 0; a < 4; ++a) q[a * n + i] = qi[a];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P[a * n + i] = Pi[a];
            L[a * n + i] = Li[a];
        }
        watch_with(wt, ref, t, xn, qi, rebuild, rescreen);
    }
    raise_flags(rebuild, rescreen, flags);
    count_drift(drift, flags);
    if (blockIdx.x == gridDim.x - 1) finalize_globals(acc + 6 * (int64_t)n, ev, ovf);
    report_fixovf(ovf, flags);
    if (kinetic) grid_sum2(kt, kr, partial, ticket, kinetic);
}

static size_t nblocks(int32_t n) { return (size_t)((n + kIntThreads - 1) / kIntThreads); }

// Allocation-free form of the fused step: the per-block kinetic partial sums
// and the completion ticket live in this file-scope array (one copy per
// device, held until the process ends) instead of a caller workspace.
constexpr int32_t kNoAllocMaxBodies = 1 << 22;
constexpr size_t kNoAllocPartialBytes =
    ((sizeof(double) * 2 * (((size_t)kNoAllocMaxBodies + kIntThreads - 1) / kIntThreads + 1) + 255) & ~(size_t)255);
constexpr size_t kNoAllocScratchBytes = kNoAllocPartialBytes + 256;   // partial sums, then the ticket
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Clears the completion ticket (a kernel, so that the call can be captured
// in a graph).
__global__ void k_clear_ticket(unsigned *ticket) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ticket = 0u;
}

}  // namespace rb

using namespace rb;

extern "C" size_t rb_rigid_workspace_bytes(int32_t n) {
    if (n <= 0) return 256;
    return ((sizeof(double) * 2 * (nblocks(n) + 1) + 255) & ~(size_t)255) + 256;
}

static Watch make_watch(const rb_ctx *ctx, const double *x_ref, double half_skin, const double *x_sref,
                        const double *q_sref, double half_margin) {
    Watch wt;
    wt.x_ref = x_ref;
    wt.half_skin2 = half_skin * half_skin;
    wt.x_sref = x_sref;
    wt.q_sref = q_sref;
    wt.half_margin = half_margin;
    for (int t = 0; t < kMaxTypes; ++t) wt.rho[t] = t < ctx->n_types ? (double)ctx->rmax[t] * (1.0 + 1e-6) : 0.0;
    return wt;
}

extern "C" int rb_rigid_step(const rb_ctx *ctx, int phase, int32_t n, double dt, double *x, double *P,
                             double *q, double *L, const int32_t *type, const float *force,
                             const float *torque, const double *x_ref, double half_skin, const double *x_sref,
                             const double *q_sref, double half_margin, double *kinetic, double *nh,
                             int32_t *flags, void *ws, size_t ws_bytes, void *stream) {
    RB_REQUIRE(ctx && P && q && L && type && force && torque, "rb_rigid_step: null argument");
    RB_REQUIRE(phase == 1 || phase == 2, "rb_rigid_step: phase must be 1 or 2");
    RB_REQUIRE(n > 0, "rb_rigid_step: n must be > 0");
    hipStream_t st = (hipStream_t)stream;
    const int grid = (int)nblocks(n);
    if (phase == 1) {
        RB_REQUIRE(x, "rb_rigid_step: x is null");
        RB_REQUIRE((!x_ref && !x_sref) || flags, "rb_rigid_step: the displacement tests need flags");
        RB_REQUIRE(!x_sref || q_sref, "rb_rigid_step: x_sref needs q_sref");
        k_phase1<<<grid, kIntThreads, 0, st>>>(n, dt, x, P, q, L, type, ctx->dev.mass, ctx->dev.inertia, force,
                                               torque, make_watch(ctx, x_ref, half_skin, x_sref, q_sref, half_margin),
                                               flags, nh);
    } else {
        RB_REQUIRE(kinetic && ws, "rb_rigid_step: phase 2 needs kinetic and ws");
        RB_REQUIRE(ws_bytes >= rb_rigid_workspace_bytes(n), "rb_rigid_step: workspace too small");
        char *w = static_cast<char *>(ws);
        double *partial = reinterpret_cast<double *>(w);
        unsigned *ticket = reinterpret_cast<unsigned *>(w + rb_rigid_workspace_bytes(n) - 256);
        k_phase2<<<grid, kIntThreads, 0, st>>>(n, dt, P, q, L, type, ctx->dev.mass, ctx->dev.inertia, force, torque,
                                               partial, ticket, kinetic, nh);
    }
    RB_LAUNCH_CHECK("rb_rigid_step");
    return RB_OK;
}

extern "C" int rb_rigid_step_fused(const rb_ctx *ctx, int32_t n, double dt, double *x, double *P, double *q,
                                   double *L, const int32_t *type, int64_t *acc, float *force, float *torque,
                                   double *energy_virial, const double *x_ref, double half_skin,
                                   const double *x_sref, const double *q_sref, double half_margin, double *kinetic,
                                   int32_t *flags, void *ws, size_t ws_bytes, void *stream) {
    RB_REQUIRE(ctx && x && P && q && L && type && acc && force && torque && flags && ws,
               "rb_rigid_step_fused: null argument");
    RB_REQUIRE(n > 0, "rb_rigid_step_fused: n must be > 0");
    RB_REQUIRE(ws_bytes >= rb_rigid_workspace_bytes(n), "rb_rigid_step_fused: workspace too small");
    RB_REQUIRE(!x_sref || q_sref, "rb_rigid_step_fused: x_sref needs q_sref");
    char *w = static_cast<char *>(ws);
    double *partial = reinterpret_cast<double *>(w);
    unsigned *ticket = reinterpret_cast<unsigned *>(w + rb_rigid_workspace_bytes(n) - 256);
    // one block more than the bodies need: it adds up the global sums
    k_fused<<<(int)nblocks(n) + 1, kIntThreads, 0, (hipStream_t)stream>>>(
        n, dt, x, P, q, L, type, ctx->dev.mass, ctx->dev.inertia, acc, force, torque, energy_virial,
        make_watch(ctx, x_ref, half_skin, x_sref, q_sref, half_margin), flags, partial, ticket, kinetic,
        ctx->n_types == 1);
    RB_LAUNCH_CHECK("rb_rigid_step_fused");
    return RB_OK;
}

// Device address of `scratch` on each device, taken once per device with that
// device current (each device holds its own copy of the array).
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(unsigned char **out) {
    int dev = -1;
    const int rc = rb::hip_check(hipGetDevice(&dev), "rb_rigid_step_fused_noalloc: hipGetDevice");
    if (rc != RB_OK) return rc;
    if (dev < 0 || dev >= kMaxDevices) {
        rb::set_error("rb_rigid_step_fused_noalloc: device %d beyond the %d devices supported", dev, kMaxDevices);
        return RB_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const int rs = rb::hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                                     "rb_rigid_step_fused_noalloc: hipGetSymbolAddress");
        if (rs != RB_OK) return rs;
        if (!p) {
            rb::set_error("rb_rigid_step_fused_noalloc: hipGetSymbolAddress returned a null address");
            return RB_ERR_HIP;
        }
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return RB_OK;
}
}  // namespace

extern "C" size_t rb_rigid_step_fused_noalloc_max_bodies(void) { return (size_t)kNoAllocMaxBodies; }

extern "C" int rb_rigid_step_fused_noalloc(const rb_ctx *ctx, int32_t n, double dt, double *x, double *P, double *q,
                                           double *L, const int32_t *type, int64_t *acc, float *force,
                                           float *torque, double *energy_virial, const double *x_ref,
                                           double half_skin, const double *x_sref, const double *q_sref,
                                           double half_margin, double *kinetic, int32_t *flags, void *stream) {
    RB_REQUIRE(ctx && x && P && q && L && type && acc && force && torque && flags,
               "rb_rigid_step_fused_noalloc: null argument");
    RB_REQUIRE(n > 0, "rb_rigid_step_fused_noalloc: n must be > 0");
    RB_REQUIRE(n <= kNoAllocMaxBodies, "rb_rigid_step_fused_noalloc: n exceeds the scratch limit of 4194304 bodies");
    RB_REQUIRE(!x_sref || q_sref, "rb_rigid_step_fused_noalloc: x_sref needs q_sref");
    unsigned char *base = nullptr;
    const int rc = scratch_address(&base);
    if (rc != RB_OK) return rc;
    double *partial = reinterpret_cast<double *>(base);
    unsigned *ticket = reinterpret_cast<unsigned *>(base + kNoAllocPartialBytes);
    hipStream_t st = (hipStream_t)stream;
    k_clear_ticket<<<1, 64, 0, st>>>(ticket);
    k_fused<<<(int)nblocks(n) + 1, kIntThreads, 0, st>>>(
        n, dt, x, P, q, L, type, ctx->dev.mass, ctx->dev.inertia, acc, force, torque, energy_virial,
        make_watch(ctx, x_ref, half_skin, x_sref, q_sref, half_margin), flags, partial, ticket, kinetic,
        ctx->n_types == 1);
    RB_LAUNCH_CHECK("rb_rigid_step_fused_noalloc");
    return RB_OK;
}
