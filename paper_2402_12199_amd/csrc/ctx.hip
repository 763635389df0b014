// Context, error reporting and the fixed-point force accumulator.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "rb_common.hpp"

namespace rb {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return RB_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return RB_ERR_HIP;
}

// Fill kernel (graph safe, unlike a memset node).
__global__ void k_zero_i64(int64_t *a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

// Converts the accumulator and clears it for the next evaluation (each word
// is read and cleared by the same thread).  The first nb blocks take the
// bodies, one extra block the global sums.
__global__ void k_finalize(int32_t n, int nb, int64_t *__restrict__ acc, float *__restrict__ force,
                           float *__restrict__ torque, double *__restrict__ ev, int32_t *__restrict__ flags) {
    const double s = 1.0 / RB_ACC_SCALE;
    bool ovf = false;
    if ((int)blockIdx.x == nb) {
        finalize_globals(acc + 6 * (int64_t)n, ev, ovf);
        report_fixovf(ovf, flags);
        return;
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nb * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const long long f = acc[a * (int64_t)n + i], t = acc[(3 + a) * (int64_t)n + i];
            ovf |= !fix_word_ok(f) || !fix_word_ok(t);
            force[a * n + i] = (float)((double)f * s);
            torque[a * n + i] = (float)((double)t * s);
            acc[a * (int64_t)n + i] = 0;
            acc[(3 + a) * (int64_t)n + i] = 0;
        }
    }
    report_fixovf(ovf, flags);
}

}  // namespace rb

using namespace rb;

extern "C" const char *rb_last_error(void) { return g_err; }

extern "C" int rb_flags_check(const int32_t *f) {
    RB_REQUIRE(f, "rb_flags_check: null flags");
    if (f[RB_FLAG_OVERFLOW] > 0) {
        set_error("pair list overflow: %d pairs found", f[RB_FLAG_OVERFLOW]);
        return RB_ERR_CAPACITY;
    }
    if (f[RB_FLAG_NONFINITE]) {
        set_error("non-finite pair force or energy");
        return RB_ERR_NONFINITE;
    }
    if (f[RB_FLAG_FIXOVF]) {
        set_error("fixed-point accumulator overflow (a term of 2^28 or a total of 2^30 in magnitude)");
        return RB_ERR_NONFINITE;
    }
    if (f[RB_FLAG_WAIT_TIMEOUT]) {
        set_error("an internal wait between the waves of a kernel timed out");
        return RB_ERR_NONFINITE;
    }
    if (f[RB_FLAG_QDRIFT]) {
        set_error("quaternion norm drift beyond 1e-10 in %d body updates", f[RB_FLAG_QDRIFT]);
        return RB_ERR_NONFINITE;
    }
    return RB_OK;
}

extern "C" int rb_ctx_create(rb_ctx **out, int32_t n_types, const int32_t *n_beads,
                             const float *beads, const double *mass, const double *inertia,
                             float eps, float sigma, float rc) {
    RB_REQUIRE(out && n_beads && beads && mass && inertia, "rb_ctx_create: null argument");
    RB_REQUIRE(n_types >= 1 && n_types <= kMaxTypes, "rb_ctx_create: 1..%d types", kMaxTypes);
    RB_REQUIRE(eps > 0 && sigma > 0 && rc > 0, "rb_ctx_create: eps, sigma, rc must be > 0");
    int total = 0;
    for (int t = 0; t < n_types; ++t) {
        RB_REQUIRE(n_beads[t] >= 1 && n_beads[t] <= kMaxBeads,
                   "rb_ctx_create: type %d has %d beads (1..%d)", t, n_beads[t], kMaxBeads);
        total += n_beads[t];
    }
    rb_ctx *c = new rb_ctx();
    memset(c, 0, sizeof *c);
    c->n_types = n_types;
    float4 *hb = new float4[total];
    int o = 0;
    for (int t = 0; t < n_types; ++t) {
        c->n_beads[t] = n_beads[t];
        if (n_beads[t] > c->max_beads) c->max_beads = n_beads[t];
        c->dev.t.n[t] = n_beads[t];
        c->dev.t.off[t] = o;
        double r2max = 0;
        float h[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < n_beads[t]; ++k, ++o) {
            hb[o] = make_float4(beads[3 * o], beads[3 * o + 1], beads[3 * o + 2], 0.f);
            double r2 = (double)beads[3 * o] * beads[3 * o] + (double)beads[3 * o + 1] * beads[3 * o + 1] +
                        (double)beads[3 * o + 2] * beads[3 * o + 2];
            if (r2 > r2max) r2max = r2;
            for (int a = 0; a < 3; ++a) h[a] = fmaxf(h[a], fabsf(beads[3 * o + a]));
        }
        c->rmax[t] = (float)sqrt(r2max);
        c->dev.t.hx[t] = h[0];
        c->dev.t.hy[t] = h[1];
        c->dev.t.hz[t] = h[2];
        // capsule along the axis of the largest half extent: radius = largest
        // distance of a bead from the axis, half-length = smallest that keeps
        // every bead inside (rounded outward in FP32)
        const int k = h[2] >= h[1] && h[2] >= h[0] ? 2 : (h[1] >= h[0] ? 1 : 0);
        const float *bt = beads + 3 * (o - n_beads[t]);
        double R2 = 0.0;
        for (int m = 0; m < n_beads[t]; ++m) {
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a)
                if (a != k) r2 += (double)bt[3 * m + a] * bt[3 * m + a];
            if (r2 > R2) R2 = r2;
        }
        double H = 0.0;
        for (int m = 0; m < n_beads[t]; ++m) {
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a)
                if (a != k) r2 += (double)bt[3 * m + a] * bt[3 * m + a];
            const double hm = fabs((double)bt[3 * m + k]) - sqrt(fmax(R2 - r2, 0.0));
            if (hm > H) H = hm;
        }
        c->dev.t.cax[t] = k;
        c->dev.t.cR[t] = nextafterf((float)sqrt(R2), 1e30f);
        c->dev.t.cH[t] = H > 0.0 ? nextafterf((float)H, 1e30f) : 0.f;
        c->dev.t.round[t] = 3.14159265358979 * R2 < 4.0 * (double)h[(k + 1) % 3] * (double)h[(k + 2) % 3];
    }
    c->dev.t.n_types = n_types;
    int rc_ = RB_OK;
    rc_ = hip_check(hipMalloc(&c->alloc_beads, sizeof(float4) * total), "rb_ctx_create hipMalloc");
    if (rc_ == RB_OK)
        rc_ = hip_check(hipMemcpy(c->alloc_beads, hb, sizeof(float4) * total, hipMemcpyHostToDevice),
                        "rb_ctx_create copy");
    delete[] hb;
    size_t mbytes = sizeof(double) * 4 * n_types;
    if (rc_ == RB_OK) rc_ = hip_check(hipMalloc(&c->alloc_mass, mbytes), "rb_ctx_create hipMalloc");
    if (rc_ == RB_OK) {
        double *hm = new double[4 * n_types];
        for (int t = 0; t < n_types; ++t) {
            hm[t] = mass[t];
            for (int a = 0; a < 3; ++a) hm[n_types + 3 * t + a] = inertia[3 * t + a];
        }
        rc_ = hip_check(hipMemcpy(c->alloc_mass, hm, mbytes, hipMemcpyHostToDevice), "rb_ctx_create copy");
        delete[] hm;
    }
    if (rc_ != RB_OK) {
        rb_ctx_destroy(c);
        return rc_;
    }
    c->dev.t.beads = static_cast<const float4 *>(c->alloc_beads);
    c->dev.t.total = total;
    c->total_beads = total;
    c->dev.mass = static_cast<const double *>(c->alloc_mass);
    c->dev.inertia = static_cast<const double *>(c->alloc_mass) + n_types;
    double s2 = (double)sigma * sigma, sr2 = s2 / ((double)rc * rc);
    double sr6 = sr2 * sr2 * sr2;
    c->dev.lj.kind = kPotLJ;
    c->dev.lj.rc2 = rc * rc;
    c->dev.lj.sig2 = (float)s2;
    c->dev.lj.c4e = 4.f * eps;
    c->dev.lj.c24e = 24.f * eps;
    c->dev.lj.ushift = (float)(4.0 * eps * (sr6 * sr6 - sr6));
    *out = c;
    return RB_OK;
}

extern "C" int rb_ctx_set_hphc(rb_ctx *c, double A, double b, double cc, double p) {
    RB_REQUIRE(c, "rb_ctx_set_hphc: null context");
    RB_REQUIRE(A >= 0 && b > 0 && cc > 0 && p >= 1, "rb_ctx_set_hphc: need A >= 0, b > 0, c > 0, p >= 1");
    const double rc = b + 3.14159265358979323846 / cc;
    c->dev.lj.kind = kPotHPHC;
    c->dev.lj.rc2 = (float)(rc * rc);
    c->dev.lj.A = (float)A;
    c->dev.lj.b = (float)b;
    c->dev.lj.c = (float)cc;
    c->dev.lj.p = (float)p;
    return RB_OK;
}

extern "C" int rb_ctx_destroy(rb_ctx *c) {
    if (!c) return RB_OK;
    if (c->alloc_beads) (void)hipFree(c->alloc_beads);
    if (c->alloc_mass) (void)hipFree(c->alloc_mass);
    delete c;
    return RB_OK;
}

extern "C" int rb_accum_zero(int32_t n, int64_t *acc, void *stream) {
    RB_REQUIRE(n >= 0 && acc, "rb_accum_zero: bad arguments");
    int64_t len = RB_ACC_LEN(n);
    k_zero_i64<<<grid_for(len, 256, 4096), 256, 0, (hipStream_t)stream>>>(acc, len);
    RB_LAUNCH_CHECK("rb_accum_zero");
    return RB_OK;
}

extern "C" int rb_accum_finalize(int32_t n, int64_t *acc, float *force, float *torque,
                                 double *energy_virial, int32_t *flags, void *stream) {
    RB_REQUIRE(n >= 0 && acc && force && torque, "rb_accum_finalize: bad arguments");
    const int nb = grid_for(n > 0 ? n : 1, 256, 4096);
    k_finalize<<<nb + 1, 256, 0, (hipStream_t)stream>>>(n, nb, acc, force, torque, energy_virial, flags);
    RB_LAUNCH_CHECK("rb_accum_finalize");
    return RB_OK;
}
