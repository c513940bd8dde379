// Particle bookkeeping kernels of librbsog for gfx950: the velocity-Verlet
// kick/drift, wrap and quantise with the displacement check of the Verlet
// list, the cell list of a list build (histogram, exclusive scan, scatter,
// per-cell id sort and gather of the state into cell order), the kinetic
// energy sum and the mean-square displacement.
//
// Arrays are structure-of-arrays over all systems of the batch: component d
// of slot t is at [d*N + t].  The state is in the cell order of the latest
// list build, so these passes stream it coalesced and a re-sort moves
// particles only as far as they drifted.  The list-build kernels read the
// rebuild flag first and return at once when it is clear.
#include "rbsog_internal.h"
#include "rbsog_math.h"

namespace rbsog {

namespace {

constexpr int kBlock = 256;
inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// The cell scan works on tiles of kScanTile cells.
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Three standard normals for particle `id` at thermostat step `step`
// (Box-Muller on lanes 0 and 1 of Philox stream 2, counter (id, step)).
__device__ __forceinline__ void thermo_normals(uint64_t seed, int64_t step, int32_t id, double xi[3]) {
    const uint64_t idx = ((uint64_t)step << 32) | (uint32_t)id;
    rmath::normals3(seed, 2, idx, xi);
}

// Lanes holding the same cell in a run of consecutive lanes (the state is in
// cell order, so runs are the rule) share one atomic: the run's first lane
// adds the run length and the others take their offset in the run.  Returns
// the old counter value plus the lane's offset (all lanes must be active).
__device__ __forceinline__ int32_t run_atomic_add(int32_t *ctr, int64_t cell, bool valid) {
    const int lane = threadIdx.x & 63;
    const int64_t key = valid ? cell : -1;
    const int64_t prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || key != prev;
    const uint64_t H = __ballot(head);
    const uint64_t after = lane == 63 ? 0ull : (H >> (lane + 1)) << (lane + 1);
    const int nxt = after ? __builtin_ctzll(after) : 64;
    const int first = 63 - __clzll((long long)(H & ((2ull << lane) - 1ull)));
    int32_t base = 0;
    if (head && valid) base = atomicAdd(&ctr[cell], nxt - lane);
    base = __shfl(base, first, 64);
    return base + (lane - first);
}

// Optional kick dt/2 and drift (velocity Verlet), then wrap x into [0, L)
// (x_w = frac(x/L) L) and fixed-point coordinate u = min(2^32-1,
// floor(frac(x/L) 2^32)).  A particle farther than skin r_c / 2 from its
// position at the latest list build sets the rebuild flag: the list holds
// every pair within r_c (1 + skin) at the build, so it holds every pair
// within r_c while no particle has moved farther.
__global__ __launch_bounds__(kBlock) void k_kdq(EvalArgs a) {
    const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = t0 < a.N;
    const int64_t t = valid ? t0 : a.N - 1;
    const int64_t N = a.N;
    double *__restrict__ x = a.cur.x;
    double *__restrict__ v = a.cur.v;
    // every load first: the system's constants and the particle's state
    const SysDev &sd = a.sys[a.sys_of[t]];
    double L[3], xs[3];
    float hf[3];
    uint32_t uref[3];
    for (int d = 0; d < 3; ++d) {
        L[d] = sd.g.L[d];
        hf[d] = sd.g.hf[d];
        xs[d] = x[d * N + t];
        uref[d] = a.u[d * N + t];
    }
    const float dthr2 = sd.g.dthr2_f;
    const double xs0[3] = {xs[0], xs[1], xs[2]};
    if (a.kick) {
        double f[3], vs[3];
        for (int d = 0; d < 3; ++d) {
            f[d] = a.Fn[d * N + t] + a.Ff[d * N + t];
            vs[d] = v[d * N + t];
        }
        if (a.nh) {
            // Nose-Hoover: xi's first half step with the kinetic energy of the
            // step's start, then v scaled by exp(-xi dt/2) (the far kernel
            // scales again after the closing kick and moves xi on)
            const int32_t s = a.sys_of[t];
            const double xh = a.nh_xi[s] + 0.5 * a.dt * (2.0 * a.kin[s] - sd.nh_nf * a.nh_T) / sd.nh_Q;
            const double sc = exp(-0.5 * a.dt * xh);
            for (int d = 0; d < 3; ++d) vs[d] *= sc;
        }
        bool bad = false;
        if (a.thermo) {
            // BAOAB: half kick, half drift, Ornstein-Uhlenbeck, half drift
            double xi[3];
            thermo_normals(a.tseed, *a.tstep, a.cur.id[t], xi);
            for (int d = 0; d < 3; ++d) {
                bad |= !isfinite(f[d]);
                vs[d] += a.hdm * f[d];
                xs[d] += 0.5 * a.dt * vs[d];
                vs[d] = a.c1 * vs[d] + a.c2 * xi[d];
                xs[d] += 0.5 * a.dt * vs[d];
                if (valid) v[d * N + t] = vs[d];
            }
        } else {
            for (int d = 0; d < 3; ++d) {
                bad |= !isfinite(f[d]);
                vs[d] += a.hdm * f[d];
                xs[d] += a.dt * vs[d];
                if (valid) v[d * N + t] = vs[d];
            }
        }
        if (bad && valid) atomicOr(a.flag, 1);
        // the step's drift, unwrapped, for the mean-square displacement
        if (valid && a.cur.dsp)
            for (int d = 0; d < 3; ++d) a.cur.dsp[d * N + t] += xs[d] - xs0[d];
    }
    uint32_t uq[3];
    const float d2 = wrap_store(a, t, valid, xs, L, hf, uref, uq);
    if (a.always_build) {
        // every evaluation builds: the cell and the histogram here (no bin pass)
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.rebuild = 1;
        int64_t c[3];
        for (int d = 0; d < 3; ++d) c[d] = (int64_t)(((uint64_t)uq[d] * (uint64_t)sd.g.nc[d]) >> 32);
        const int64_t cell = sd.c0 + c[0] + (int64_t)sd.g.nc[0] * (c[1] + (int64_t)sd.g.nc[1] * c[2]);
        if (valid) a.cell_of[t] = (int32_t)cell;
        run_atomic_add(a.cell_count, cell, valid);
    } else {
        // one atomic per wave that found a particle past the threshold
        const bool far_ = valid && !(d2 <= dthr2);
        if (__ballot(far_) != 0ull && (threadIdx.x & 63) == 0) atomicOr(a.rebuild, 1);
    }
}

// ---- exclusive scan of int32 counts: 1024 elements per block --------------

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

// Exclusive scan of the counts of n cells by one block (few cells): each
// thread sums a contiguous run, the block scans the run totals, each thread
// writes its run's starts (cell_start, and the scatter's fill counters), and
// out[n] = the total.
__device__ void scan_counts_block(const int32_t *in, int64_t n, int32_t *out, int32_t *fill) {
    const int64_t per = (n + kBlock - 1) / kBlock;
    const int64_t b = (int64_t)threadIdx.x * per;
    const int64_t e = b + per < n ? b + per : n;
    int32_t sum = 0;
    for (int64_t c = b; c < e; ++c) sum += in[c];
    int32_t tot;
    int32_t off = block_exclusive_scan(sum, &tot);
    for (int64_t c = b; c < e; ++c) {
        const int32_t v = in[c];
        out[c] = off;
        fill[c] = off;
        off += v;
    }
    if (threadIdx.x == 0) out[n] = tot;
}

// Cell c_d = (u n_d) >> 32 of each particle and the cell histogram.  SCAN
// (few cells): the last block to finish also scans the counts (the scan
// kernels are not launched).
template <bool SCAN>
__global__ __launch_bounds__(kBlock) void k_bin(EvalArgs a) {
    // the critical path's waves ahead of the structure factor's beside them
    __builtin_amdgcn_s_setprio(2);
    if (!*a.rebuild) return;
    const int64_t N = a.N;
    // grid-stride over blocks of kBlock slots (the grid is capped: on the
    // steps that do not build, few blocks return at once)
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < N; base += (int64_t)gridDim.x * kBlock) {
        const int64_t t0 = base + threadIdx.x;
        const bool valid = t0 < N;
        const int64_t t = valid ? t0 : N - 1;
        const SysDev &sd = a.sys[a.sys_of[t]];
        int64_t c[3];
        int32_t nc[3];
        for (int d = 0; d < 3; ++d) {
            nc[d] = sd.g.nc[d];
            c[d] = (int64_t)(((uint64_t)a.u_tmp[d * N + t] * (uint64_t)nc[d]) >> 32);
        }
        const int64_t cell = sd.c0 + c[0] + (int64_t)nc[0] * (c[1] + (int64_t)nc[1] * c[2]);
        if (valid) a.cell_of[t] = (int32_t)cell;
        run_atomic_add(a.cell_count, cell, valid);
    }
    if constexpr (SCAN) {
        // one device-scope fence per block (it writes the XCD's L2 back),
        // after the block's barrier
        __shared__ int32_t last;
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            last = atomicAdd(a.bin_done, 1u) == gridDim.x - 1 ? 1 : 0;
        }
        __syncthreads();
        if (!last) return;
        // every block's counts are in: scan them, then re-arm the counter
        __threadfence();
        scan_counts_block(a.cell_count, a.C, a.cell_start, a.cell_fill);
        if (threadIdx.x == 0) *a.bin_done = 0u;
    }
}

__global__ void k_scan_blocks(const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ bsum,
                              const int32_t *__restrict__ cond) {
    // the critical path's waves ahead of the structure factor's beside them
    __builtin_amdgcn_s_setprio(2);
    if (!*cond) return;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    int32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of the tile: counts in registers, the block's scan, plus
// `before` (the count of the cells before the tile).
__device__ __forceinline__ void scan_tile(const int32_t *__restrict__ in, int64_t n, int32_t before,
                                          int32_t *__restrict__ out, int32_t *__restrict__ fill) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t vals[kScanItems];
    int32_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = base + k < n ? in[base + k] : 0;
        s += vals[k];
    }
    int32_t tot;
    int32_t off = block_exclusive_scan(s, &tot) + before;
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) {
            out[base + k] = off;
            fill[base + k] = off;
        }
        off += vals[k];
        if (base + k == n - 1) out[n] = off;
    }
}

// Each block adds the totals of the tiles before it (read in parallel from
// L2 and reduced in a fixed order) to its own exclusive scan.
__global__ void k_scan_apply(const int32_t *__restrict__ in, int64_t n, const int32_t *__restrict__ bsum,
                             int32_t *__restrict__ out, int32_t *__restrict__ fill, const int32_t *__restrict__ cond) {
    // the critical path's waves ahead of the structure factor's beside them
    __builtin_amdgcn_s_setprio(2);
    if (!*cond) return;
    int32_t pre = 0;
#pragma unroll 4
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kBlock) pre += bsum[b];
    int32_t before;
    block_exclusive_scan(pre, &before);
    scan_tile(in, n, before, out, fill);
}

// Each particle to a slot of its cell (atomic order), with its id beside it
// for the per-cell sort.
__global__ __launch_bounds__(kBlock) void k_cell_scatter(int64_t N, const int32_t *__restrict__ cell_of,
                                                         const int32_t *__restrict__ id, int32_t *__restrict__ fill,
                                                         int32_t *__restrict__ src, int32_t *__restrict__ skey,
                                                         const int32_t *__restrict__ cond) {
    // the critical path's waves ahead of the structure factor's beside them
    __builtin_amdgcn_s_setprio(2);
    if (!*cond) return;
    // grid-stride as in k_bin (the order of the atomics within a cell is
    // undone by the per-cell id sort)
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < N; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = base + threadIdx.x;
        const bool valid = t < N;
        const int32_t cell = valid ? cell_of[t] : 0;
        const int32_t key = valid ? id[t] : 0;
        const int32_t dst = run_atomic_add(fill, cell, valid);
        if (valid) {
            src[dst] = (int32_t)t;
            skey[dst] = key;
        }
    }
}

// Per cell: order of its slots by particle id (the order becomes (cell, id),
// independent of the scatter's atomic order), and reset of its histogram
// count for the next evaluation; then the block gathers the state of its
// cells' slots into `nxt` in the new order, one thread per slot (writes are
// coalesced, reads stay close: particles move little between builds).  The
// positions become the new list reference `u`.  Cells of up to kRankMax
// particles load their keys at once and rank them in registers; larger cells
// take an insertion sort in memory.
constexpr int kRankMax = 16;

constexpr int kSortCells = 64;  // cells per block of the sort and gather

__global__ __launch_bounds__(kBlock) void k_sort_gather(EvalArgs a) {
    // the critical path's waves ahead of the structure factor's beside them
    __builtin_amdgcn_s_setprio(2);
    if (!*a.rebuild) return;
    int32_t *out = a.sorted;
    // grid-stride over groups of kSortCells cells (the grid is capped)
    for (int64_t c0 = (int64_t)blockIdx.x * kSortCells; c0 < a.C; c0 += (int64_t)gridDim.x * kSortCells) {
        const int64_t c = c0 + threadIdx.x;
        if (threadIdx.x < kSortCells && c < a.C) {
            const int32_t lo = a.cell_start[c], hi = a.cell_start[c + 1];
            const int32_t cnt = hi - lo;
            const int32_t *src = a.src;
            const int32_t *idc = a.cur.id;
            if (cnt <= kRankMax) {
                int32_t sv[kRankMax], key[kRankMax];
#pragma unroll
                for (int i = 0; i < kRankMax; ++i) {
                    sv[i] = i < cnt ? src[lo + i] : 0;
                    key[i] = i < cnt ? a.skey[lo + i] : INT32_MAX;
                }
#pragma unroll
                for (int i = 0; i < kRankMax; ++i) {
                    int32_t rank = 0;
#pragma unroll
                    for (int j = 0; j < kRankMax; ++j) rank += key[j] < key[i] ? 1 : 0;
                    if (i < cnt) out[lo + rank] = sv[i];
                }
            } else {
                for (int32_t i = lo; i < hi; ++i) out[i] = src[i];
                for (int32_t i = lo + 1; i < hi; ++i) {
                    const int32_t v = out[i];
                    const int32_t kv = idc[v];
                    int32_t j = i - 1;
                    while (j >= lo && idc[out[j]] > kv) {
                        out[j + 1] = out[j];
                        --j;
                    }
                    out[j + 1] = v;
                }
            }
            a.cell_count[c] = 0;
        }
        // the block's permutation entries are visible to the whole block here
        __syncthreads();
        const int64_t c1 = c0 + kSortCells < a.C ? c0 + kSortCells : a.C;
        const int64_t k0 = a.cell_start[c0], k1 = a.cell_start[c1];
        const int64_t N = a.N;
        // two slots per thread and pass, all loads issued before the stores
        constexpr int U = 2;
        for (int64_t kb = k0 + threadIdx.x; kb < k1; kb += U * kBlock) {
            int64_t tt[U];
#pragma unroll
            for (int j = 0; j < U; ++j) tt[j] = kb + j * kBlock < k1 ? out[kb + j * kBlock] : -1;
            double xv[U][3], vv[U][3], qv[U];
            uint32_t uv[U][3];
            float qfv[U];
            int32_t idv[U], cv[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t t = tt[j] < 0 ? 0 : tt[j];
                for (int d = 0; d < 3; ++d) {
                    xv[j][d] = a.cur.x[d * N + t];
                    vv[j][d] = a.cur.v[d * N + t];
                    uv[j][d] = a.u_tmp[d * N + t];
                }
                qv[j] = a.cur.q[t];
                qfv[j] = a.cur.qf[t];
                idv[j] = a.cur.id[t];
                cv[j] = a.cell_of[t];
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t k = kb + j * kBlock;
                if (tt[j] < 0) continue;
                for (int d = 0; d < 3; ++d) {
                    a.nxt.x[d * N + k] = xv[j][d];
                    a.nxt.v[d * N + k] = vv[j][d];
                    a.u[d * N + k] = uv[j][d];
                }
                a.nxt.q[k] = qv[j];
                a.nxt.qf[k] = qfv[j];
                a.nxt.id[k] = idv[j];
                a.cell_sorted[k] = cv[j];
            }
            if (a.cur.dsp) {
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    if (tt[j] < 0) continue;
                    for (int d = 0; d < 3; ++d) a.nxt.dsp[d * N + kb + j * kBlock] = a.cur.dsp[d * N + tt[j]];
                }
            }
        }
        // the next group's permutation entries are written after every
        // thread has read this group's
        __syncthreads();
    }
}

// Slot of every caller index (the inverse of the id permutation of the
// current order), then the near and far forces of the requested indices.
__global__ __launch_bounds__(kBlock) void k_invert_ids(int64_t N, const int32_t *__restrict__ id,
                                                       int32_t *__restrict__ slot_of) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < N) slot_of[id[t]] = (int32_t)t;
}

__global__ __launch_bounds__(kBlock) void k_gather_forces(int64_t N, int64_t m, const int64_t *__restrict__ ids,
                                                          const int32_t *__restrict__ slot_of,
                                                          const double *__restrict__ Fn, const double *__restrict__ Ff,
                                                          double *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    const int64_t t = slot_of[ids[k]];
    for (int d = 0; d < 3; ++d) {
        out[6 * k + d] = Fn[d * N + t];
        out[6 * k + 3 + d] = Ff[d * N + t];
    }
}

}  // namespace

void launch_subset_forces(const EvalArgs &a, int64_t m, const int64_t *ids, int32_t *slot_of, double *out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_invert_ids, dim3(grid_for(a.N, kBlock)), dim3(kBlock), 0, s, a.N, a.cur.id, slot_of);
    if (m > 0)
        hipLaunchKernelGGL(k_gather_forces, dim3(grid_for(m, kBlock)), dim3(kBlock), 0, s, a.N, m, ids, slot_of,
                           a.Fn, a.Ff, out);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, p, n, v);
}

void launch_kdq(const EvalArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_kdq, dim3(grid_for(a.N, kBlock)), dim3(kBlock), 0, s, a);
}

int64_t scan_blocksums_size(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

// Grids of the list-build kernels that stride: a step without a build
// dispatches this many blocks at most, each returning at once.
constexpr int64_t kBuildGrid = 2048;
inline unsigned capped(int64_t blocks) { return (unsigned)(blocks < kBuildGrid ? (blocks < 1 ? 1 : blocks) : kBuildGrid); }

// Cell counts scanned by the last block of the bin pass up to this many
// cells (one block reads them twice); above, by the two scan kernels.
constexpr int64_t kScanInBin = 65536;

void launch_bin_scan(const EvalArgs &a, hipStream_t s) {
    const dim3 grid(capped(grid_for(a.N, kBlock)));
    if (a.C <= kScanInBin) {
        hipLaunchKernelGGL(k_bin<true>, grid, dim3(kBlock), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_bin<false>, grid, dim3(kBlock), 0, s, a);
        launch_scan(a, s);
    }
}

void launch_scan(const EvalArgs &a, hipStream_t s) {
    const int64_t n = a.C;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(kBlock), 0, s, a.cell_count, n, a.blocksums,
                       (const int32_t *)a.rebuild);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, s, a.cell_count, n, a.blocksums,
                       a.cell_start, a.cell_fill, (const int32_t *)a.rebuild);
}

void launch_cell_scatter(const EvalArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_scatter, dim3(capped(grid_for(a.N, kBlock))), dim3(kBlock), 0, s, a.N, a.cell_of, a.cur.id,
                       a.cell_fill, a.src, a.skey, (const int32_t *)a.rebuild);
}

void launch_sort_gather(const EvalArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_sort_gather, dim3(capped(grid_for(a.C, kSortCells))), dim3(kBlock), 0, s, a);
}

}  // namespace rbsog
