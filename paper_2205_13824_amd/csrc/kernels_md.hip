// Particle bookkeeping kernels of librbsog for gfx950: wrap and quantise,
// the cell list (histogram, exclusive scan, scatter, per-cell id sort,
// gather into cell order) and the velocity-Verlet kick/drift.
//
// Arrays are structure-of-arrays: component d of particle i is at [d*n + i].
// These passes are HBM-bound streams; each thread owns one particle (or one
// cell) and global accesses are coalesced except the cell scatter/gather.
#include "rbsog_internal.h"

namespace rbsog {

namespace {

constexpr int kBlock = 256;
constexpr double kTwo32 = 4294967296.0;

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Optional kick dt/2 and drift (velocity Verlet), then wrap x into [0, L)
// (x_w = frac(x/L) L), fixed-point coordinate u = min(2^32-1,
// floor(frac(x/L) 2^32)), cell c_d = (u n_d) >> 32 and the cell histogram.
// The extra last block stages the k batch of this evaluation.
__global__ void k_kdq(Geom g, KickArgs kick, StageArgs stage, double *__restrict__ x, uint32_t *__restrict__ u,
                      int32_t *__restrict__ cell_of, int32_t *__restrict__ count) {
    if (blockIdx.x == gridDim.x - 1) {
        stage_batch(g, stage);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n) return;
    const int64_t n = g.n;
    if (kick.on) {
        bool bad = false;
        for (int d = 0; d < 3; ++d) {
            const double f = kick.Fn[d * n + i] + kick.Ff[d * n + i];
            bad |= !isfinite(f);
            const double vd = kick.v[d * n + i] + kick.hdm * f;
            kick.v[d * n + i] = vd;
            x[d * n + i] += kick.dt * vd;
        }
        if (bad) atomicOr(kick.flag, 1);
    }
    int64_t c[3];
    for (int d = 0; d < 3; ++d) {
        double t = x[d * n + i] / g.L[d];
        double f = t - floor(t);
        double v = floor(f * kTwo32);
        v = v > kTwo32 - 1.0 ? kTwo32 - 1.0 : v;
        uint32_t ud = (uint32_t)v;
        u[d * n + i] = ud;
        x[d * n + i] = f * g.L[d];
        c[d] = (int64_t)(((uint64_t)ud * (uint64_t)g.nc[d]) >> 32);
    }
    int32_t cell = (int32_t)(c[0] + (int64_t)g.nc[0] * (c[1] + (int64_t)g.nc[1] * c[2]));
    cell_of[i] = cell;
    atomicAdd(&count[cell], 1);
}

// ---- exclusive scan of int32 counts: 1024 elements per block --------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
    __shared__ int32_t wsum[kBlock / 64];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        int32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int32_t base = 0, tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

__global__ void k_scan_blocks(const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ bsum) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    int32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int32_t *bsum, int64_t nb) {
    // one block: exclusive scan of the block totals in place
    int64_t per = (nb + kBlock - 1) / kBlock;
    int64_t lo = threadIdx.x * per, hi = lo + per < nb ? lo + per : nb;
    int32_t s = 0;
    for (int64_t k = lo; k < hi; ++k) s += bsum[k];
    int32_t tot;
    int32_t off = block_exclusive_scan(s, &tot);
    for (int64_t k = lo; k < hi; ++k) {
        int32_t v = bsum[k];
        bsum[k] = off;
        off += v;
    }
}

__global__ void k_scan_apply(const int32_t *__restrict__ in, int64_t n, const int32_t *__restrict__ bsum,
                             int32_t *__restrict__ out, int32_t *__restrict__ fill) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t vals[kScanItems];
    int32_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = base + k < n ? in[base + k] : 0;
        s += vals[k];
    }
    int32_t tot;
    int32_t off = block_exclusive_scan(s, &tot) + bsum[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) {
            out[base + k] = off;
            fill[base + k] = off;
        }
        off += vals[k];
        if (base + k == n - 1) out[n] = off;
    }
}

__global__ void k_cell_scatter(int64_t n, const int32_t *__restrict__ cell_of, int32_t *__restrict__ fill,
                               int32_t *__restrict__ order) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t t = atomicAdd(&fill[cell_of[i]], 1);
    order[t] = (int32_t)i;
}

// Per cell: insertion sort of its ids (the order becomes (cell, id),
// independent of the scatter's atomic order) and reset of its histogram
// count for the next evaluation.
__global__ void k_cell_sort(int64_t ncell, const int32_t *__restrict__ start, int32_t *__restrict__ order,
                            int32_t *__restrict__ count) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int32_t lo = start[c], hi = start[c + 1];
    for (int32_t a = lo + 1; a < hi; ++a) {
        const int32_t v = order[a];
        int32_t b = a - 1;
        while (b >= lo && order[b] > v) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = v;
    }
    count[c] = 0;
}

// Gather into cell order: one thread per sorted slot.
__global__ void k_gather(Geom g, const int32_t *__restrict__ order, const uint32_t *__restrict__ u,
                         const double *__restrict__ x, const double *__restrict__ q, uint32_t *__restrict__ su,
                         double *__restrict__ sx, double *__restrict__ sq, float *__restrict__ sqf, int f64) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.n) return;
    const int64_t n = g.n;
    const int64_t id = order[t];
    for (int d = 0; d < 3; ++d) su[d * n + t] = u[d * n + id];
    const double qi = q[id];
    sqf[t] = (float)qi;
    if (f64) {
        for (int d = 0; d < 3; ++d) sx[d * n + t] = x[d * n + id];
        sq[t] = qi;
    }
}

}  // namespace

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, p, n, v);
}

void launch_kdq(const Geom &g, const KickArgs &kick, const StageArgs &stage, double *x, uint32_t *u,
                int32_t *cell_of, int32_t *cell_count, hipStream_t s) {
    hipLaunchKernelGGL(k_kdq, dim3(grid_for(g.n, kBlock) + 1), dim3(kBlock), 0, s, g, kick, stage, x, u, cell_of,
                       cell_count);
}

int64_t scan_blocksums_size(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_scan(const int32_t *in, int32_t *out_excl, int32_t *fill_copy, int64_t n, int32_t *blocksums,
                 hipStream_t s) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, blocksums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, blocksums, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, blocksums, out_excl,
                       fill_copy);
}

void launch_cell_scatter(const Geom &g, const int32_t *cell_of, int32_t *fill, int32_t *order, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_scatter, dim3(grid_for(g.n, kBlock)), dim3(kBlock), 0, s, g.n, cell_of, fill, order);
}

void launch_sort_gather(const Geom &g, int64_t ncell, const int32_t *start, int32_t *order, int32_t *cell_count,
                        const uint32_t *u, const double *x, const double *q, uint32_t *su, double *sx, double *sq,
                        float *sqf, bool f64, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_sort, dim3(grid_for(ncell, kBlock)), dim3(kBlock), 0, s, ncell, start, order, cell_count);
    hipLaunchKernelGGL(k_gather, dim3(grid_for(g.n, kBlock)), dim3(kBlock), 0, s, g, order, u, x, q, su, sx, sq, sqf,
                       (int)f64);
}

}  // namespace rbsog
