// Cell-list pair builder: half list (i < j) of body pairs whose minimum-image
// centre distance is below r_list.
//
// Up to 65536 bodies: the one-launch pipeline below (k_pl_small).  Beyond:
// the multi-kernel pipeline (each kernel returns at
// once when the list is only rebuilt on request and the rebuild flag is
// clear, so the whole sequence can sit in a captured graph):
//   bin bodies into cells of edge >= r_list (count per cell)
//   exclusive scan of cell counts -> cell starts
//   scatter body ids into cell order, then sort each cell's ids, which makes
//   the cell contents independent of atomic arrival order (with at least 3
//   cells on every axis the binning atomic gives each body's rank in its
//   cell and the scatter moves its cell-relative position along)
//   with at least 3 cells on every axis (half stencil): per position t in
//   cell order, count the pairs with the later bodies of its own cell and
//   the bodies of the 13 forward neighbour cells (FP32 distances from
//   cell-relative positions, the exact FP64 test near r_list); exclusive
//   scan of the counts; write them as (min, max) at t's offset
//   otherwise (full stencil): per body i, count neighbours j > i in the 27
//   surrounding cells, scan, write its pairs at its offset (sorted by i)
// The resulting list is fully deterministic.  Either way the set of pairs is
// exact; the forces built from it do not depend on its order (fixed-point
// accumulation).
#include <algorithm>
#include <cfloat>

#include "rb_common.hpp"

namespace rb {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

struct CellGrid {
    int nc[3];
    int ncell;
    double L[3], inv[3], cinv[3];  // cinv: cells per unit length
    double rl2;
    // half-stencil search (every axis with at least 3 cells): cell edges in
    // FP64 and FP32, and the band around r_list^2 inside which the FP32
    // squared distance is not trusted to decide (the exact FP64 test is
    // taken there)
    double edge[3];
    float edge_f[3];
    float lo2, hi2;
};

__device__ inline bool skip(const int32_t *flags, int mode) {
    return mode == RB_BUILD_IF_FLAGGED && flags[RB_FLAG_REBUILD] == 0;
}

__device__ inline int cell_coord(double x, double L, double cinv, int nc) {
    double w = x - L * floor(x / L);  // wrap into [0, L)
    int c = (int)(w * cinv);
    return c >= nc ? nc - 1 : (c < 0 ? 0 : c);
}

__global__ void k_fill(int32_t *a, int m, int v, const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) a[i] = v;
}

__global__ void k_bin(int32_t n, const double *__restrict__ x, CellGrid g, int32_t *__restrict__ cell_of,
                      int32_t *__restrict__ cnt, double *__restrict__ x_ref, const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double v = x[a * n + i];
        if (x_ref) x_ref[a * n + i] = v;
        c[a] = cell_coord(v, g.L[a], g.cinv[a], g.nc[a]);
    }
    int id = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
    cell_of[i] = id;
    atomicAdd(cnt + id, 1);
}

// Block-local exclusive scan of kScanTile ints; block totals to tmp.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const int32_t *__restrict__ in,
                                                             int32_t *__restrict__ out, int m,
                                                             int32_t *__restrict__ tmp,
                                                             const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    __shared__ int32_t wsum[kScanThreads / kWave];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < m) ? in[base + k] : 0;
        s += v[k];
    }
    // inclusive scan of thread sums within the wave
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    int incl = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    int run = woff + incl - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) tmp[blockIdx.x] = woff + incl;
}

// Scan of the (at most kScanTile) tile totals, in place, by one block; the
// grand total goes to out[m], and optionally to the pair-count flags.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(int32_t *__restrict__ tmp, int ntiles,
                                                           int32_t *__restrict__ out, int m,
                                                           int32_t *flags, int mode, int cap) {
    if (skip(flags, mode)) return;
    __shared__ int32_t wsum[kScanThreads / kWave];
    const int base = threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < ntiles) ? tmp[base + k] : 0;
        s += v[k];
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    int incl = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    int run = woff + incl - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < ntiles) tmp[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) {
        const int total = woff + incl;
        out[m] = total;
        if (cap >= 0) {
            flags[RB_FLAG_NPAIRS] = total < cap ? total : cap;
            flags[RB_FLAG_OVERFLOW] = total > cap ? total : 0;
        }
    }
}

__global__ void k_scan_add(int32_t *__restrict__ out, int m, const int32_t *__restrict__ tmp,
                           const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] += tmp[i / kScanTile];
}

__global__ void k_scatter(int32_t n, const int32_t *__restrict__ cell_of, const int32_t *__restrict__ start,
                          int32_t *__restrict__ fill, int32_t *__restrict__ sorted, const int32_t *flags,
                          int mode) {
    if (skip(flags, mode)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_of[i];
    int slot = atomicAdd(fill + c, 1);
    sorted[start[c] + slot] = i;
}

// Insertion sort of each cell's ids (cells hold a handful of bodies), then
// the positions in the same cell order (xs, 3 x n FP64), so that the
// neighbour scans read each cell's bodies as one contiguous run.
__device__ inline void sort_cell_and_gather(int b, int e, int32_t n, const double *__restrict__ x,
                                            int32_t *__restrict__ sorted, double *__restrict__ xs) {
    for (int k = b + 1; k < e; ++k) {
        int v = sorted[k], m = k - 1;
        while (m >= b && sorted[m] > v) {
            sorted[m + 1] = sorted[m];
            --m;
        }
        sorted[m + 1] = v;
    }
    for (int k = b; k < e; ++k) {
        const int j = sorted[k];
#pragma unroll
        for (int a = 0; a < 3; ++a) xs[a * n + k] = x[a * n + j];
    }
}

__global__ void k_sort_cells(int ncell, int32_t n, const double *__restrict__ x, const int32_t *__restrict__ start,
                             int32_t *__restrict__ sorted, double *__restrict__ xs, const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    sort_cell_and_gather(start[c], start[c + 1], n, x, sorted, xs);
}

// Half-stencil pipeline, first steps.  Binning takes each body's rank in its
// cell from the cell counter's atomic, so that the scatter needs none: it
// writes the body id and the body's position relative to its cell's origin
// (FP32, a 16-byte record) at the body's place in cell order, reading the
// positions in body order.  The per-cell sort then orders each cell's
// (id, record) pairs by id (the cell contents no longer depend on the
// atomics' order) and completes the records the search reads (the body id
// in the fourth word) and the cell index cs of each position.  The offset of a neighbour cell's origin is a
// whole number of edges, the same for all of that cell's bodies.
__global__ void k_bin_rank(int32_t n, const double *__restrict__ x, CellGrid g, int32_t *__restrict__ cell_of,
                           int32_t *__restrict__ cnt, int32_t *__restrict__ rank, double *__restrict__ x_ref,
                           const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = x[a * n + i];
        if (x_ref) x_ref[a * n + i] = v;
        c[a] = cell_coord(v, g.L[a], g.cinv[a], g.nc[a]);
    }
    const int id = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
    cell_of[i] = id;
    rank[i] = atomicAdd(cnt + id, 1);
}

__global__ void k_scatter_rel(int32_t n, const double *__restrict__ x, CellGrid g,
                              const int32_t *__restrict__ cell_of, const int32_t *__restrict__ start,
                              const int32_t *__restrict__ rank, int32_t *__restrict__ sorted,
                              float4 *__restrict__ rec, const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell_of[i];
    const int pos = start[c] + rank[i];
    const int cc[3] = {c / (g.nc[2] * g.nc[1]), (c / g.nc[2]) % g.nc[1], c % g.nc[2]};
    float r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double v = x[a * n + i];
        const double w = v - g.L[a] * floor(v / g.L[a]);
        r[a] = (float)(w - cc[a] * g.edge[a]);
    }
    sorted[pos] = i;
    rec[pos] = make_float4(r[0], r[1], r[2], 0.f);
}

__global__ void k_sort_cells_rec(int ncell, const int32_t *__restrict__ start, int32_t *__restrict__ sorted,
                                 float4 *__restrict__ rec, int32_t *__restrict__ cs, const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int b = start[c], e = start[c + 1];
    for (int k = b + 1; k < e; ++k) {
        const int v = sorted[k];
        const float4 vr = rec[k];
        int m = k - 1;
        while (m >= b && sorted[m] > v) {
            sorted[m + 1] = sorted[m];
            rec[m + 1] = rec[m];
            --m;
        }
        sorted[m + 1] = v;
        rec[m + 1] = vr;
    }
    for (int k = b; k < e; ++k) {
        rec[k].w = __int_as_float(sorted[k]);
        cs[k] = c;
    }
}

// Half-stencil search: thread t takes the t-th body in cell order and pairs
// it with the later bodies of its own cell and all bodies of the 13 cells
// that follow it in the (x, y, z) lexicographic order of the offsets, so
// that each pair is examined once; it is written as (min, max).  The
// candidates' positions are requested in batches, so that a lane has many
// loads in flight (the search is bound by load latency).  The squared distance
// is formed in FP32 from the cell-relative positions; inside the band
// [lo2, hi2) around r_list^2 the FP64 minimum-image test of the full
// pipeline decides, so the set of pairs is exactly that test's.  Counts and
// offsets are indexed by the cell-order position.
// The writing pass stages each wave's pairs in LDS (the wave's pairs form
// one contiguous range of the list) and stores them with coalesced writes;
// pairs beyond kHalfBuf per wave go straight to memory.
constexpr int kHalfThreads = 256;
constexpr int kHalfBuf = 512;
constexpr int kHalfBatch = 4;

template <bool EMIT>
__global__ __launch_bounds__(kHalfThreads) void k_neigh_half(
    int32_t n, const float4 *__restrict__ rec, const double *__restrict__ x, CellGrid g,
    const int32_t *__restrict__ cs, const int32_t *__restrict__ start, int32_t *__restrict__ ncount,
    const int32_t *__restrict__ noff, int32_t *__restrict__ pi, int32_t *__restrict__ pj, int32_t cap,
    const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    __shared__ int2 buf[EMIT ? kHalfThreads / kWave : 1][EMIT ? kHalfBuf : 1];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    const bool live = t < n;
    const int tc = live ? t : n - 1;
    const int c = cs[tc];
    const float4 own = rec[tc];
    const int i = __float_as_int(own.w);
    const int cz = c % g.nc[2], cy = (c / g.nc[2]) % g.nc[1], cx = c / (g.nc[2] * g.nc[1]);
    const float xi = own.x, yi = own.y, zi = own.z;
    int cnt = 0;
    int wbase = 0, wtotal = 0;
    const int t0 = t - lane;   // the wave's first position
    if (EMIT && t0 < n) {
        const int t1 = t0 + kWave < n ? t0 + kWave : n;
        wbase = noff[t0];
        wtotal = noff[t1] - wbase;
    }
    int out = EMIT ? noff[tc] : 0;
    // The 14 cells' ranges (the own cell from position t + 1 on, then the 13
    // forward cells, offsets k = 14 .. 26 with k = 9 (dx + 1) + 3 (dy + 1) +
    // (dz + 1)), requested together; then per cell its first kHalfBatch
    // candidates in one batch of loads (unused slots read a valid position
    // and are not tested), the rest of a fuller cell one by one.
    int mb[14], me[14];
    mb[0] = t + 1;
    me[0] = start[c + 1];
#pragma unroll
    for (int q = 1; q < 14; ++q) {
        const int kk = 13 + q;
        int nx = cx + kk / 9 - 1, ny = cy + (kk / 3) % 3 - 1, nz = cz + kk % 3 - 1;
        nx += nx < 0 ? g.nc[0] : (nx >= g.nc[0] ? -g.nc[0] : 0);
        ny += ny < 0 ? g.nc[1] : (ny >= g.nc[1] ? -g.nc[1] : 0);
        nz += nz < 0 ? g.nc[2] : (nz >= g.nc[2] ? -g.nc[2] : 0);
        const int cn = (nx * g.nc[1] + ny) * g.nc[2] + nz;
        mb[q] = start[cn];
        me[q] = start[cn + 1];
    }
    if (!live)
#pragma unroll
        for (int q = 0; q < 14; ++q) me[q] = mb[q];
    auto test = [&](const float4 p, float ox, float oy, float oz) {
        const float ddx = (p.x + ox) - xi, ddy = (p.y + oy) - yi, ddz = (p.z + oz) - zi;
        const float r2 = fmaf(ddx, ddx, fmaf(ddy, ddy, ddz * ddz));
        const int j = __float_as_int(p.w);
        bool in = r2 < g.lo2;
        if (!in && r2 < g.hi2) {
            const double ex = min_image(x[j] - x[i], g.L[0], g.inv[0]);
            const double ey = min_image(x[n + j] - x[n + i], g.L[1], g.inv[1]);
            const double ez = min_image(x[2 * n + j] - x[2 * n + i], g.L[2], g.inv[2]);
            in = ex * ex + ey * ey + ez * ez < g.rl2;
        }
        if (in) {
            if (EMIT) {
                const int a = i < j ? i : j, b = i < j ? j : i;
                const int local = out - wbase;
                if (local < kHalfBuf)
                    buf[w][local] = make_int2(a, b);
                else if (out < cap) {
                    pi[out] = a;
                    pj[out] = b;
                }
                ++out;
            } else {
                ++cnt;
            }
        }
    };
#pragma unroll
    for (int q = 0; q < 14; ++q) {
        const int kk = q == 0 ? 13 : 13 + q;
        const float ox = (float)(kk / 9 - 1) * g.edge_f[0], oy = (float)((kk / 3) % 3 - 1) * g.edge_f[1],
                    oz = (float)(kk % 3 - 1) * g.edge_f[2];
        float4 pv[kHalfBatch];
#pragma unroll
        for (int v = 0; v < kHalfBatch; ++v) pv[v] = rec[mb[q] + v < n ? mb[q] + v : n - 1];
#pragma unroll
        for (int v = 0; v < kHalfBatch; ++v)
            if (mb[q] + v < me[q]) test(pv[v], ox, oy, oz);
        for (int m = mb[q] + kHalfBatch; m < me[q]; ++m) test(rec[m], ox, oy, oz);
    }
    if (EMIT) {
        // the lanes' LDS writes are done before the wave reads them back
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int nb = wtotal < kHalfBuf ? wtotal : kHalfBuf;
        for (int k = lane; k < nb; k += kWave) {
            const int o = wbase + k;
            if (o < cap) {
                const int2 v = buf[w][k];
                pi[o] = v.x;
                pj[o] = v.y;
            }
        }
    } else if (live) {
        ncount[t] = cnt;
    }
}

// Thread t takes the t-th body in cell order, so that neighbouring threads
// scan the same neighbour cells; counts and offsets stay indexed by body.
template <bool EMIT>
__global__ void k_neigh(int32_t n, const double *__restrict__ xs, CellGrid g, const int32_t *__restrict__ cell_of,
                        const int32_t *__restrict__ start, const int32_t *__restrict__ sorted,
                        int32_t *__restrict__ ncount, const int32_t *__restrict__ noff,
                        int32_t *__restrict__ pi, int32_t *__restrict__ pj, int32_t cap,
                        const int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = sorted[t];
    const double xi = xs[t], yi = xs[n + t], zi = xs[2 * n + t];
    const int id = cell_of[i];
    const int cz = id % g.nc[2], cy = (id / g.nc[2]) % g.nc[1], cx = id / (g.nc[2] * g.nc[1]);
    int lo[3], hi[3];
    const int cc[3] = {cx, cy, cz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = g.nc[a] >= 3 ? -1 : 0;
        hi[a] = g.nc[a] >= 3 ? 1 : g.nc[a] - 1;
    }
    (void)cc;
    int cnt = 0;
    int out = EMIT ? noff[i] : 0;
    for (int ox = lo[0]; ox <= hi[0]; ++ox) {
        int nx = cx + ox;
        nx += nx < 0 ? g.nc[0] : (nx >= g.nc[0] ? -g.nc[0] : 0);
        for (int oy = lo[1]; oy <= hi[1]; ++oy) {
            int ny = cy + oy;
            ny += ny < 0 ? g.nc[1] : (ny >= g.nc[1] ? -g.nc[1] : 0);
            for (int oz = lo[2]; oz <= hi[2]; ++oz) {
                int nz = cz + oz;
                nz += nz < 0 ? g.nc[2] : (nz >= g.nc[2] ? -g.nc[2] : 0);
                const int c = (nx * g.nc[1] + ny) * g.nc[2] + nz;
                for (int m = start[c], e = start[c + 1]; m < e; ++m) {
                    const int j = sorted[m];
                    if (j <= i) continue;
                    const double dx = min_image(xs[m] - xi, g.L[0], g.inv[0]);
                    const double dy = min_image(xs[n + m] - yi, g.L[1], g.inv[1]);
                    const double dz = min_image(xs[2 * n + m] - zi, g.L[2], g.inv[2]);
                    if (dx * dx + dy * dy + dz * dz < g.rl2) {
                        if (EMIT) {
                            if (out < cap) {
                                pi[out] = i;
                                pj[out] = j;
                            }
                            ++out;
                        } else {
                            ++cnt;
                        }
                    }
                }
            }
        }
    }
    if (!EMIT) ncount[i] = cnt;
}

__global__ void k_finish(int32_t *flags, int mode) {
    if (skip(flags, mode)) return;
    flags[RB_FLAG_REBUILD] = 0;
    flags[RB_FLAG_NREBUILDS] += 1;
    flags[RB_FLAG_RESCREEN] = 1;   // a screened list drawn from the old list is stale
}

// ----------------------------------------------------- one-launch pipeline
// For up to kSmallBodies bodies a rebuild is one launch, which returns at
// once when no rebuild is flagged (k_pl_small):
//   the cell phase (workgroup 0, barriers between steps): bin, scan the
//     cell counts, scatter, sort each cell
//   the pair phase (every workgroup, once the cell phase is done): half a
//     wave per body, one lane per neighbour cell; the lanes count their
//     pairs, the body reserves room for all of them with one atomic, and the
//     lanes write them; the last workgroup to finish publishes the count and
//     clears the rebuild flag.
// The pairs of one body are contiguous and in cell order; the order of the
// bodies' runs in the list follows the reservations and is not fixed.
constexpr int kSmallThreads = 1024;
constexpr int kSmallBodies = 65536;
constexpr int kSmallCells = 262144;
constexpr int kSmallLdsCells = 16000;   // LDS counts: 64 000 bytes, with the scan's words below 64 KiB
constexpr int kCellBatch = 4;           // bodies per thread and pass in the cell phase
constexpr int kSmallCell = 8;           // cells up to this size are sorted in registers

// Exclusive scan of in[0..m) into out[0..m) by one block; returns the total
// (all threads).
__device__ int block_scan(const int32_t *in, int32_t *out, int m) {
    __shared__ int32_t wsum[kSmallThreads / kWave];
    __shared__ int32_t carry_s;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < m; base += kSmallThreads) {
        const int i = base + threadIdx.x;
        const int v = i < m ? in[i] : 0;
        int incl = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int t = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += t;
        }
        if (lane == kWave - 1) wsum[w] = incl;
        __syncthreads();
        int woff = 0, total = 0;
        for (int k = 0; k < kSmallThreads / kWave; ++k) {
            if (k < w) woff += wsum[k];
            total += wsum[k];
        }
        const int carry = carry_s;
        if (i < m) out[i] = carry + woff + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + total;
        __syncthreads();
    }
    return carry_s;
}


// The cell phase of a rebuild, by one workgroup.
__device__ void pl_cells(int32_t n, const double *__restrict__ x, const CellGrid &g, int32_t *__restrict__ cell_of,
                         int32_t *__restrict__ cnt, int32_t *__restrict__ start, int32_t *__restrict__ fill,
                         int32_t *__restrict__ sorted, double *__restrict__ xs, double *__restrict__ x_ref,
                         int32_t *__restrict__ counter, int32_t *__restrict__ rank, int lds_counts) {
    const int t = threadIdx.x, T = kSmallThreads;
    if (t < 2) counter[t] = 0;   // pair count and finishing ticket of the pair phase
    if (lds_counts) {
        // cell counts in LDS (grids of at most kSmallLdsCells cells): the
        // count's atomic gives each body its rank in the cell, so the scatter
        // needs no atomics
        extern __shared__ int lcnt[];
        for (int c = t; c < g.ncell; c += T) lcnt[c] = 0;
        __syncthreads();
        // kCellBatch bodies per thread and pass, their loads issued together
        for (int i0 = t; i0 < n; i0 += kCellBatch * T) {
            double v[kCellBatch][3];
#pragma unroll
            for (int u = 0; u < kCellBatch; ++u) {
                const int i = i0 + u * T;
#pragma unroll
                for (int a = 0; a < 3; ++a) v[u][a] = i < n ? x[a * n + i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kCellBatch; ++u) {
                const int i = i0 + u * T;
                if (i >= n) break;
                int c[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (x_ref) x_ref[a * n + i] = v[u][a];
                    c[a] = cell_coord(v[u][a], g.L[a], g.cinv[a], g.nc[a]);
                }
                const int id = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
                cell_of[i] = id;
                rank[i] = atomicAdd(lcnt + id, 1);
            }
        }
        __syncthreads();
        const int total_cells = block_scan(lcnt, start, g.ncell);   // the counts straight from LDS
        if (t == 0) start[g.ncell] = total_cells;
        __syncthreads();
        for (int i0 = t; i0 < n; i0 += kCellBatch * T) {
            int c[kCellBatch], r[kCellBatch], b[kCellBatch];
#pragma unroll
            for (int u = 0; u < kCellBatch; ++u) {
                const int i = i0 + u * T;
                c[u] = i < n ? cell_of[i] : 0;
                r[u] = i < n ? rank[i] : 0;
            }
#pragma unroll
            for (int u = 0; u < kCellBatch; ++u) b[u] = start[c[u]];
#pragma unroll
            for (int u = 0; u < kCellBatch; ++u)
                if (i0 + u * T < n) sorted[b[u] + r[u]] = i0 + u * T;
        }
    } else {
        for (int c = t; c < g.ncell; c += T) {
            cnt[c] = 0;
            fill[c] = 0;
        }
        __syncthreads();
        for (int i = t; i < n; i += T) {
            int c[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double v = x[a * n + i];
                if (x_ref) x_ref[a * n + i] = v;
                c[a] = cell_coord(v, g.L[a], g.cinv[a], g.nc[a]);
            }
            const int id = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
            cell_of[i] = id;
            atomicAdd(cnt + id, 1);
        }
        __syncthreads();
        const int total_cells = block_scan(cnt, start, g.ncell);
        if (t == 0) start[g.ncell] = total_cells;
        __syncthreads();
        for (int i = t; i < n; i += T) {
            const int c = cell_of[i];
            sorted[start[c] + atomicAdd(fill + c, 1)] = i;
        }
    }
    __syncthreads();
    // cells of up to kSmallCell bodies sorted in registers (a cell's loads
    // in flight together); larger cells by the insertion sort in memory
    for (int c = t; c < g.ncell; c += T) {
        const int b = start[c], m = start[c + 1] - b;
        if (m > kSmallCell) {
            sort_cell_and_gather(b, b + m, n, x, sorted, xs);
            continue;
        }
        int v[kSmallCell];
#pragma unroll
        for (int k = 0; k < kSmallCell; ++k) v[k] = k < m ? sorted[b + k] : INT32_MAX;
        // odd-even transposition sort: kSmallCell rounds sort kSmallCell
        // values (the padding goes to the end)
#pragma unroll
        for (int rd = 0; rd < kSmallCell; ++rd)
#pragma unroll
            for (int k = rd & 1; k + 1 < kSmallCell; k += 2) {
                const int lo = min(v[k], v[k + 1]), hi = max(v[k], v[k + 1]);
                v[k] = lo;
                v[k + 1] = hi;
            }
        double p[kSmallCell][3];
#pragma unroll
        for (int k = 0; k < kSmallCell; ++k)
#pragma unroll
            for (int a = 0; a < 3; ++a) p[k][a] = k < m ? x[a * n + v[k]] : 0.0;
#pragma unroll
        for (int k = 0; k < kSmallCell; ++k)
            if (k < m) {
                sorted[b + k] = v[k];
#pragma unroll
                for (int a = 0; a < 3; ++a) xs[a * n + b + k] = p[k][a];
            }
    }
}

// Pairs (i, j > i) of body i with the bodies of one neighbour cell c; writes
// them from out on when EMIT (up to cap), returns their number.
template <bool EMIT>
__device__ inline int cell_pairs(int i, int c, double xi, double yi, double zi, int32_t n,
                                 const double *__restrict__ xs, const CellGrid &g, const int32_t *__restrict__ start,
                                 const int32_t *__restrict__ sorted, int out, int32_t *__restrict__ pi,
                                 int32_t *__restrict__ pj, int32_t cap) {
    int cnt = 0;
    for (int m = start[c], e = start[c + 1]; m < e; ++m) {
        const int j = sorted[m];
        if (j <= i) continue;
        const double dx = min_image(xs[m] - xi, g.L[0], g.inv[0]);
        const double dy = min_image(xs[n + m] - yi, g.L[1], g.inv[1]);
        const double dz = min_image(xs[2 * n + m] - zi, g.L[2], g.inv[2]);
        if (dx * dx + dy * dy + dz * dz < g.rl2) {
            if (EMIT && out + cnt < cap) {
                pi[out + cnt] = i;
                pj[out + cnt] = j;
            }
            ++cnt;
        }
    }
    return cnt;
}

// The pair phase, by every workgroup of the grid once the cell phase is
// visible to it.
__device__ void pl_pairs(int32_t n, const double *__restrict__ xs, const CellGrid &g,
                         const int32_t *__restrict__ cell_of, const int32_t *__restrict__ start,
                         const int32_t *__restrict__ sorted, int32_t *__restrict__ pi, int32_t *__restrict__ pj,
                         int32_t cap, int32_t *__restrict__ counter, int32_t *__restrict__ flags) {
    __shared__ bool last;
    __shared__ int btot[kSmallThreads / 32], bbase;
    const int lane = threadIdx.x & (kWave - 1), k = lane & 31, hw = threadIdx.x >> 5;
    // neighbour cells per axis: all three offsets, or every cell when the
    // axis has fewer than three
    int lo[3], m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = g.nc[a] >= 3 ? -1 : 0;
        m[a] = g.nc[a] >= 3 ? 3 : g.nc[a];
    }
    // a persistent grid (so that a launch with no rebuild flagged costs few
    // workgroups): each round, half-wave h of the block takes the body at
    // cell-order position base + h (neighbouring half-waves scan the same
    // cells)
    constexpr int kBodies = kSmallThreads / 32;
    for (int base = blockIdx.x * kBodies; base < n; base += gridDim.x * kBodies) {
        const int t = base + hw;
        const bool active = t < n && k < m[0] * m[1] * m[2];
        double xi = 0, yi = 0, zi = 0;
        int i = 0, c = 0, cnt = 0;
        if (active) {
            i = sorted[t];
            xi = xs[t];
            yi = xs[n + t];
            zi = xs[2 * n + t];
            const int id = cell_of[i];
            const int cz = id % g.nc[2], cy = (id / g.nc[2]) % g.nc[1], cx = id / (g.nc[2] * g.nc[1]);
            int nx = cx + lo[0] + k / (m[1] * m[2]);
            int ny = cy + lo[1] + (k / m[2]) % m[1];
            int nz = cz + lo[2] + k % m[2];
            nx += nx < 0 ? g.nc[0] : (nx >= g.nc[0] ? -g.nc[0] : 0);
            ny += ny < 0 ? g.nc[1] : (ny >= g.nc[1] ? -g.nc[1] : 0);
            nz += nz < 0 ? g.nc[2] : (nz >= g.nc[2] ? -g.nc[2] : 0);
            c = (nx * g.nc[1] + ny) * g.nc[2] + nz;
            cnt = cell_pairs<false>(i, c, xi, yi, zi, n, xs, g, start, sorted, 0, pi, pj, cap);
        }
        // offsets of the lanes within the body's run (half-wave scan), then
        // of the bodies within the block's run (one reservation per block
        // and round: many reservations on one counter serialise)
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            const int v = __shfl_up(incl, o, 32);
            if (k >= o) incl += v;
        }
        const int total = __shfl(incl, 31, 32);
        if (k == 0) btot[hw] = total;
        __syncthreads();
        if (threadIdx.x == 0) {
            int sum = 0;
            for (int h = 0; h < kBodies; ++h) {
                const int v = btot[h];
                btot[h] = sum;
                sum += v;
            }
            bbase = sum > 0 ? atomicAdd(counter, sum) : 0;
        }
        __syncthreads();
        const int off = bbase + btot[hw];
        if (active && cnt > 0)
            (void)cell_pairs<true>(i, c, xi, yi, zi, n, xs, g, start, sorted, off + incl - cnt, pi, pj, cap);
        __syncthreads();   // btot and bbase are reused by the next round
    }
    // No fence: every reservation of the block has returned before its
    // ticket, and the last block reads the counter with an agent-scope load;
    // the pairs reach their consumers through the kernel boundary.
    if (threadIdx.x == 0) last = atomicAdd(counter + 1, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (last && threadIdx.x == 0) {
        const int tot = __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        flags[RB_FLAG_NPAIRS] = tot < cap ? tot : cap;
        flags[RB_FLAG_OVERFLOW] = tot > cap ? tot : 0;
        flags[RB_FLAG_REBUILD] = 0;
        flags[RB_FLAG_NREBUILDS] += 1;
        flags[RB_FLAG_RESCREEN] = 1;   // a screened list drawn from the old list is stale
    }
}

// A rebuild in one launch (and a launch that returns at once when none is
// flagged): workgroup 0 runs the cell phase and then sets flags[REBUILD] to
// kCellsDone (after a fence, so its writes are visible to every CU); the
// other workgroups wait for that value, fence, and join the pair phase,
// whose last workgroup clears the flag.  Only workgroup 0 is waited for, and
// it is dispatched first, so the wait ends; it is bounded all the same (past
// kCellsWaitSpins polls of ~3 us the workgroup records a timeout and goes
// on, leaving the list invalid).  A workgroup that starts after workgroup 0
// finished its phase sees kCellsDone, not 0, and takes part.
constexpr int kCellsDone = 2;
constexpr int kCellsWaitSpins = 1 << 16;

__global__ __launch_bounds__(kSmallThreads) void k_pl_small(int32_t n, const double *__restrict__ x, CellGrid g,
                                                            int32_t *__restrict__ cell_of, int32_t *__restrict__ cnt,
                                                            int32_t *__restrict__ start, int32_t *__restrict__ fill,
                                                            int32_t *__restrict__ sorted, double *__restrict__ xs,
                                                            double *__restrict__ x_ref, int32_t *__restrict__ counter,
                                                            int32_t *__restrict__ rank, int lds_counts,
                                                            int32_t *__restrict__ pi, int32_t *__restrict__ pj,
                                                            int32_t cap, int32_t *__restrict__ flags, int mode) {
    if (skip(flags, mode)) return;
    if (blockIdx.x == 0) {
        pl_cells(n, x, g, cell_of, cnt, start, fill, sorted, xs, x_ref, counter, rank, lds_counts);
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            __hip_atomic_store(flags + RB_FLAG_REBUILD, kCellsDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else {
        if (threadIdx.x == 0) {
            for (int spin = 0;; ++spin) {
                if (__hip_atomic_load(flags + RB_FLAG_REBUILD, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                    kCellsDone)
                    break;
                if (spin >= kCellsWaitSpins) {
                    atomicOr(flags + RB_FLAG_WAIT_TIMEOUT, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(127);
            }
            __threadfence();
        }
        __syncthreads();
    }
    pl_pairs(n, xs, g, cell_of, start, sorted, pi, pj, cap, counter, flags);
}

struct PLLayout {
    size_t cell_of, cnt, start, fill, sorted, ncount, noff, tmp, counter, xs, cs, rec, total;
};

static bool make_grid(int32_t n, const double *box, double r_list, CellGrid &g) {
    if (!(r_list > 0)) return false;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(box[a] >= 2.0 * r_list)) return false;
        int nc = (int)floor(box[a] / r_list);
        if (nc > 1024) nc = 1024;
        g.nc[a] = nc;
        g.L[a] = box[a];
        g.inv[a] = 1.0 / box[a];
        g.cinv[a] = nc / box[a];
        g.edge[a] = box[a] / nc;
        g.edge_f[a] = (float)g.edge[a];
        ncell *= nc;
    }
    if (ncell > (int64_t)kScanTile * kScanTile) return false;
    g.ncell = (int)ncell;
    g.rl2 = r_list * r_list;
    // FP32 distances from cell-relative positions (|component| < 2 edges)
    // are off by a few ulps of 2 edges per component; the band is far wider
    const double emax = std::max(g.edge[0], std::max(g.edge[1], g.edge[2]));
    const double band = 256.0 * FLT_EPSILON * (2.0 * emax) * (2.0 * emax);
    g.lo2 = (float)(g.rl2 - band);
    g.hi2 = (float)(g.rl2 + band);
    (void)n;
    return true;
}

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

static PLLayout layout(int32_t n, int ncell) {
    PLLayout L;
    size_t o = 0;
    L.cell_of = o; o += al(sizeof(int32_t) * n);
    L.cnt = o; o += al(sizeof(int32_t) * ncell);
    L.start = o; o += al(sizeof(int32_t) * (ncell + 1));
    L.fill = o; o += al(sizeof(int32_t) * ncell);
    L.sorted = o; o += al(sizeof(int32_t) * n);
    L.ncount = o; o += al(sizeof(int32_t) * n);
    L.noff = o; o += al(sizeof(int32_t) * (n + 1));
    L.tmp = o; o += al(sizeof(int32_t) * kScanTile);
    L.counter = o; o += al(sizeof(int32_t) * 2);
    L.xs = o; o += al(sizeof(double) * 3 * (size_t)n);   // FP64 copy (full-stencil search)
    L.cs = o; o += al(sizeof(int32_t) * n);
    L.rec = o; o += al(sizeof(float4) * (size_t)n);
    L.total = o;
    return L;
}

// Exclusive scan of in[0..m) into out[0..m], total into out[m].
static void scan(const int32_t *in, int32_t *out, int m, int32_t *tmp, int32_t *flags, int mode, int cap,
                 hipStream_t st) {
    const int ntiles = (m + kScanTile - 1) / kScanTile;
    k_scan_tiles<<<ntiles > 0 ? ntiles : 1, kScanThreads, 0, st>>>(in, out, m, tmp, flags, mode);
    k_scan_top<<<1, kScanThreads, 0, st>>>(tmp, ntiles, out, m, flags, mode, cap);
    k_scan_add<<<(m + 255) / 256 > 0 ? (m + 255) / 256 : 1, 256, 0, st>>>(out, m, tmp, flags, mode);
}

}  // namespace rb

using namespace rb;

extern "C" size_t rb_pairlist_workspace_bytes(int32_t n, const double *box, double r_list) {
    CellGrid g;
    if (n < 0 || !box || !make_grid(n, box, r_list, g)) return 0;
    return layout(n, g.ncell).total;
}

extern "C" int rb_pairlist_build(int32_t n, const double *x, const double *box, double r_list,
                                 int32_t *pair_i, int32_t *pair_j, int32_t max_pairs, double *x_ref,
                                 int32_t *flags, int mode, void *ws, size_t ws_bytes, void *stream) {
    RB_REQUIRE(x && box && pair_i && pair_j && flags && ws, "rb_pairlist_build: null argument");
    RB_REQUIRE(n > 0 && n <= (1 << 22), "rb_pairlist_build: n must be in 1..2^22");
    RB_REQUIRE(max_pairs > 0, "rb_pairlist_build: max_pairs must be > 0");
    RB_REQUIRE(mode == RB_BUILD_ALWAYS || mode == RB_BUILD_IF_FLAGGED, "rb_pairlist_build: bad mode");
    CellGrid g;
    RB_REQUIRE(make_grid(n, box, r_list, g),
               "rb_pairlist_build: need box >= 2 r_list on every axis and at most 2048^2 cells");
    PLLayout L = layout(n, g.ncell);
    RB_REQUIRE(ws_bytes >= L.total, "rb_pairlist_build: workspace too small (%zu < %zu)", ws_bytes, L.total);
    char *w = static_cast<char *>(ws);
    int32_t *cell_of = (int32_t *)(w + L.cell_of), *cnt = (int32_t *)(w + L.cnt),
            *start = (int32_t *)(w + L.start), *fill = (int32_t *)(w + L.fill),
            *sorted = (int32_t *)(w + L.sorted), *ncount = (int32_t *)(w + L.ncount),
            *noff = (int32_t *)(w + L.noff), *tmp = (int32_t *)(w + L.tmp);
    double *xs = (double *)(w + L.xs);
    hipStream_t st = (hipStream_t)stream;
    if (n <= kSmallBodies && g.ncell <= kSmallCells) {
        int32_t *counter = (int32_t *)(w + L.counter);
        const int lds_counts = g.ncell <= kSmallLdsCells;
        k_pl_small<<<grid_for(n, kSmallThreads / 32, device_cu_count()), kSmallThreads,
                     lds_counts ? sizeof(int) * g.ncell : 0, st>>>(n, x, g, cell_of, cnt, start, fill, sorted, xs,
                                                                   x_ref, counter, ncount, lds_counts, pair_i, pair_j,
                                                                   max_pairs, flags, mode);
        RB_LAUNCH_CHECK("rb_pairlist_build");
        return RB_OK;
    }
    const int gb = (n + 255) / 256, gc = (g.ncell + 255) / 256;
    if (g.nc[0] >= 3 && g.nc[1] >= 3 && g.nc[2] >= 3) {
        int32_t *cs = (int32_t *)(w + L.cs);
        float4 *rec = (float4 *)(w + L.rec);
        int32_t *rank = ncount;   // free until the count pass
        k_fill<<<gc, 256, 0, st>>>(cnt, g.ncell, 0, flags, mode);
        k_bin_rank<<<gb, 256, 0, st>>>(n, x, g, cell_of, cnt, rank, x_ref, flags, mode);
        scan(cnt, start, g.ncell, tmp, flags, mode, -1, st);
        k_scatter_rel<<<gb, 256, 0, st>>>(n, x, g, cell_of, start, rank, sorted, rec, flags, mode);
        k_sort_cells_rec<<<gc, 256, 0, st>>>(g.ncell, start, sorted, rec, cs, flags, mode);
        const int gh = (n + kHalfThreads - 1) / kHalfThreads;
        k_neigh_half<false><<<gh, kHalfThreads, 0, st>>>(n, rec, x, g, cs, start, ncount, nullptr, nullptr, nullptr,
                                                         0, flags, mode);
        scan(ncount, noff, n, tmp, flags, mode, max_pairs, st);
        k_neigh_half<true><<<gh, kHalfThreads, 0, st>>>(n, rec, x, g, cs, start, nullptr, noff, pair_i, pair_j,
                                                        max_pairs, flags, mode);
        k_finish<<<1, 1, 0, st>>>(flags, mode);
        RB_LAUNCH_CHECK("rb_pairlist_build");
        return RB_OK;
    }
    k_fill<<<gc, 256, 0, st>>>(cnt, g.ncell, 0, flags, mode);
    k_fill<<<gc, 256, 0, st>>>(fill, g.ncell, 0, flags, mode);
    k_bin<<<gb, 256, 0, st>>>(n, x, g, cell_of, cnt, x_ref, flags, mode);
    scan(cnt, start, g.ncell, tmp, flags, mode, -1, st);
    k_scatter<<<gb, 256, 0, st>>>(n, cell_of, start, fill, sorted, flags, mode);
    k_sort_cells<<<gc, 256, 0, st>>>(g.ncell, n, x, start, sorted, xs, flags, mode);
    k_neigh<false><<<gb, 256, 0, st>>>(n, xs, g, cell_of, start, sorted, ncount, nullptr, nullptr, nullptr, 0,
                                       flags, mode);
    scan(ncount, noff, n, tmp, flags, mode, max_pairs, st);
    k_neigh<true><<<gb, 256, 0, st>>>(n, xs, g, cell_of, start, sorted, nullptr, noff, pair_i, pair_j, max_pairs,
                                      flags, mode);
    k_finish<<<1, 1, 0, st>>>(flags, mode);
    RB_LAUNCH_CHECK("rb_pairlist_build");
    return RB_OK;
}
