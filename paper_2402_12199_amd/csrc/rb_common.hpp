// Shared device helpers of the rigidnn HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rigidnn.h"

namespace rb {

constexpr int kWave = 64;
constexpr int kMaxTypes = 8;
constexpr int kMaxBeads = 256;

// Error string for rb_last_error (thread local), set by the entry points.
void set_error(const char *fmt, ...);
int hip_check(hipError_t e, const char *what);

#define RB_REQUIRE(cond, ...)                  \
    do {                                       \
        if (!(cond)) {                         \
            ::rb::set_error(__VA_ARGS__);      \
            return RB_ERR_INVALID_ARG;         \
        }                                      \
    } while (0)

#define RB_LAUNCH_CHECK(what)                                       \
    do {                                                            \
        int _rc = ::rb::hip_check(hipGetLastError(), what);         \
        if (_rc != RB_OK) return _rc;                               \
    } while (0)

struct Templates {
    const float4 *beads;       // all types concatenated, w unused
    int total;                 // beads of all types
    int n[kMaxTypes];
    int off[kMaxTypes];
    float hx[kMaxTypes], hy[kMaxTypes], hz[kMaxTypes];   // half extents of the bead-centre box
    // capsule around the bead centres along body axis cax: radius cR, the
    // segment from -cH to +cH on that axis
    int cax[kMaxTypes];
    float cR[kMaxTypes], cH[kMaxTypes];
    // whether the capsule and cylinder bounds are worth forming for a type:
    // the cylinder's cross-section pi cR^2 is smaller than the box's across
    // the axis (true for cylinders, false for cubes)
    int round[kMaxTypes];
    int n_types;
};

// Bead-bead potential: kind 0 = Lennard-Jones 12-6 shifted in energy at rc
// (the workloads'), kind 1 = half-power half-cosine (paper section 3).
// rc2 is the squared cutoff either way.
constexpr int kPotLJ = 0;
constexpr int kPotHPHC = 1;
struct LJ {
    int kind;
    float rc2, sig2, c4e, c24e, ushift;  // 4 eps, 24 eps, u(rc)
    float A, b, c, p;                     // half-power half-cosine
};

struct CtxDevice {
    Templates t;
    LJ lj;
    const double *mass;      // [type]
    const double *inertia;   // [type][3]
};

// ------------------------------------------------------------- fixed point
// A word holds value * 2^32 in an int64, so totals must stay below 2^31 in
// magnitude.  A single term of 2^28 or more (or a non-finite one) is reported
// through `ovf` (and then flags[RB_FLAG_FIXOVF]): with fewer than eight such
// terms per word no total can wrap unnoticed, and finalize reports totals of
// 2^30 or more.
constexpr double kFixTermLimit = 268435456.0;                 // 2^28
constexpr long long kFixWordLimit = 4611686018427387904LL;    // 2^62 = 2^30 * 2^32

__device__ inline long long to_fixed(double v) { return __double2ll_rn(v * RB_ACC_SCALE); }

// false for |v| >= 2^28 and for NaN
__device__ inline bool fix_ok(double v) { return fabs(v) < kFixTermLimit; }

__device__ inline bool fix_word_ok(long long w) { return w < kFixWordLimit && w > -kFixWordLimit; }

__device__ inline void acc_add(int64_t *a, double v, bool &ovf) {
    ovf |= !fix_ok(v);
    atomicAdd(reinterpret_cast<unsigned long long *>(a),
              static_cast<unsigned long long>(to_fixed(v)));
}

// One atomic per wave that saw an accumulator overflow (every lane calls it).
__device__ inline void report_fixovf(bool ovf, int32_t *flags) {
    if (__any(ovf) && (threadIdx.x & 63) == 0 && flags) atomicOr(flags + RB_FLAG_FIXOVF, 1);
}

// Block-level sum of per-wave global partials (E, virial, tests: 11 int64)
// followed by one atomic per quantity into this block's slot of the
// accumulator, so few atomics hit the same address.  Every thread of the
// block must call it; `part` is meaningful in each wave's lane 0.
template <int NWAVES>
__device__ inline void block_flush_globals(const long long part[11], int64_t *acc_globals, int32_t *flags) {
    __shared__ long long red[NWAVES][11];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int a = 0; a < 11; ++a) red[w][a] = part[a];
    __syncthreads();
    if (threadIdx.x < 11) {
        long long s = 0;
#pragma unroll
        for (int k = 0; k < NWAVES; ++k) s += red[k][threadIdx.x];
        if (s) {
            if (threadIdx.x < 10)
                atomicAdd(reinterpret_cast<unsigned long long *>(acc_globals + threadIdx.x * RB_ACC_SLOTS +
                                                                 blockIdx.x % RB_ACC_SLOTS),
                          (unsigned long long)s);
            else if (flags)
                atomicAdd(reinterpret_cast<unsigned long long *>(flags + RB_FLAG_NTESTS), (unsigned long long)s);
        }
    }
}

// ------------------------------------------------------------- quaternions
// Unit quaternion (w, x, y, z) -> rotation matrix, body to lab, row major.
template <typename T>
__device__ inline void quat_to_rot(T w, T x, T y, T z, T R[9]) {
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

__device__ inline double min_image(double d, double L, double invL) { return d - L * rint(d * invL); }

// --------------------------------------------------------------- reductions
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sums and clears the RB_ACC_SLOTS slots of each of the 10 global fixed-point
// sums (energy, virial), one lane per slot and one wave per sum; every wave of
// the calling block takes part, with all of a wave's loads issued before its
// sums.  Integer sums: the order does not matter.
__device__ inline void finalize_globals(int64_t *acc_globals, double *ev, bool &ovf) {
    static_assert(RB_ACC_SLOTS == kWave, "one lane per slot");
    constexpr int kSums = 10, kPerWave = 3;   // blocks of at least four waves: one round
    const int lane = threadIdx.x & (kWave - 1);
    const int w = (int)(threadIdx.x / kWave), nw = (int)(blockDim.x / kWave);
    for (int g0 = w; g0 < kSums; g0 += kPerWave * nw) {
        long long v[kPerWave];
#pragma unroll
        for (int r = 0; r < kPerWave; ++r) {
            const int g = g0 + r * nw;
            v[r] = g < kSums ? acc_globals[g * RB_ACC_SLOTS + lane] : 0;
        }
#pragma unroll
        for (int r = 0; r < kPerWave; ++r) {
            const int g = g0 + r * nw;
            if (g < kSums) {
                acc_globals[g * RB_ACC_SLOTS + lane] = 0;
                const long long s = wave_sum(v[r]);
                ovf |= !fix_word_ok(v[r]) || !fix_word_ok(s);
                if (lane == 0 && ev) ev[g] = (double)s * (1.0 / RB_ACC_SCALE);
            }
        }
    }
}

template <typename T>
__device__ inline T wave_min(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Orders LDS writes of this wave before later LDS reads of other lanes of the
// same wave.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Compute units of the current device (cached per process; 256 if the
// query fails), for sizing persistent and spread-out grids.
inline int device_cu_count() {
    static int cached = 0;
    if (cached > 0) return cached;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    cached = cus;
    return cus;
}

inline int grid_for(int64_t work, int per_block, int cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

}  // namespace rb

struct rb_ctx {
    rb::CtxDevice dev;
    int n_types;
    int n_beads[rb::kMaxTypes];
    float rmax[rb::kMaxTypes];
    int max_beads;           // largest template
    int total_beads;         // all templates
    void *alloc_beads;
    void *alloc_mass;
};
