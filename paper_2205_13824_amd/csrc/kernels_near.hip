// Near part of the sum-of-Gaussians split for gfx950 (Sec. 3.1, eq.
// "forcesplit", with the factor of -grad U_N):
//   F_N,i = sum_{j: r_ij < r_c} q_i q_j (1/r^3 - 2 sum_l omega_l/s_l^2 e^{-r^2/s_l^2}) r_ij
//   U_N   = 1/2 sum_i sum_j q_i q_j (1/r - sum_l omega_l e^{-r^2/s_l^2})
// One thread per particle in cell order walks the 27 (or fewer) neighbouring
// cells; consecutive threads share cells, so the candidate loads hit in cache.
// Pair inclusion follows the fixed-point rule of rbsog.h; a fast test in the
// working precision decides every pair farther than a small band from r_c,
// and the exact FP64 rule decides the rest, so the list is bit-exact.
#include "rbsog_internal.h"

namespace rbsog {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// The pair rule itself: FP64 products and sums without contraction.
__device__ __forceinline__ bool exact_in(const Geom &g, uint32_t dux, uint32_t duy, uint32_t duz) {
#pragma clang fp contract(off)
    double dx = (double)(int32_t)dux * g.h[0];
    double dy = (double)(int32_t)duy * g.h[1];
    double dz = (double)(int32_t)duz * g.h[2];
    double r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    return r2 < g.rc2;
}

__device__ __forceinline__ bool decide64(const Geom &g, double r2, uint32_t dux, uint32_t duy, uint32_t duz) {
    if (r2 >= g.band_hi) return false;
    if (r2 <= g.band_lo) return true;
    return exact_in(g, dux, duy, duz);
}

__device__ __forceinline__ bool decide32(const Geom &g, float r2, uint32_t dux, uint32_t duy, uint32_t duz) {
    if (r2 >= g.band_hi_f) return false;
    if (r2 <= g.band_lo_f) return true;
    return exact_in(g, dux, duy, duz);
}

// Minimum-image FP64 displacement x_j - x_i from wrapped coordinates.
__device__ __forceinline__ double mi64(double d, double L, double invL) { return d - L * rint(d * invL); }

__device__ __forceinline__ int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

__device__ double block_sum(double v) {
    __shared__ double ws[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) ws[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) s += ws[w];
    return s;
}

template <bool F64>
__global__ __launch_bounds__(kBlock) void k_near(Geom g, SogDev c, const int32_t *__restrict__ start,
                                                 const int32_t *__restrict__ order, const uint32_t *__restrict__ su,
                                                 const double *__restrict__ sx, const double *__restrict__ sq,
                                                 const float *__restrict__ sqf, double *__restrict__ Fn,
                                                 double *__restrict__ epart) {
    const int64_t n = g.n;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double e = 0.0;
    if (t < n) {
        const uint32_t ux = su[t], uy = su[n + t], uz = su[2 * n + t];
        const int cx = (int)(((uint64_t)ux * (uint32_t)g.nc[0]) >> 32);
        const int cy = (int)(((uint64_t)uy * (uint32_t)g.nc[1]) >> 32);
        const int cz = (int)(((uint64_t)uz * (uint32_t)g.nc[2]) >> 32);
        double Fx = 0.0, Fy = 0.0, Fz = 0.0;
        float fx = 0.f, fy = 0.f, fz = 0.f;
        double xi = 0, yi = 0, zi = 0, qi = 0;
        float qif = 0.f;
        if constexpr (F64) {
            xi = sx[t]; yi = sx[n + t]; zi = sx[2 * n + t]; qi = sq[t];
        } else {
            qif = sqf[t];
        }
        for (int oz = -g.reach[2]; oz <= g.reach[2]; ++oz) {
            const int jz = wrapc(cz + oz, g.nc[2]);
            for (int oy = -g.reach[1]; oy <= g.reach[1]; ++oy) {
                const int jy = wrapc(cy + oy, g.nc[1]);
                for (int ox = -g.reach[0]; ox <= g.reach[0]; ++ox) {
                    const int jx = wrapc(cx + ox, g.nc[0]);
                    const int32_t cj = jx + g.nc[0] * (jy + g.nc[1] * jz);
                    const int32_t lo = start[cj], hi = start[cj + 1];
                    for (int32_t j = lo; j < hi; ++j) {
                        if (j == t) continue;
                        const uint32_t dux = su[j] - ux, duy = su[n + j] - uy, duz = su[2 * n + j] - uz;
                        if constexpr (F64) {
                            const double dx = mi64(sx[j] - xi, g.L[0], g.invL[0]);
                            const double dy = mi64(sx[n + j] - yi, g.L[1], g.invL[1]);
                            const double dz = mi64(sx[2 * n + j] - zi, g.L[2], g.invL[2]);
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            if (!decide64(g, r2, dux, duy, duz)) continue;
                            const double qq = qi * sq[j];
                            const double rinv = 1.0 / sqrt(r2);
                            double gs = 0.0, ph = 0.0;
                            for (int l = 0; l < g.ngauss; ++l) {
                                const double ex = exp(-r2 * c.a64[l]);
                                gs += c.c64[l] * ex;
                                ph += c.w64[l] * ex;
                            }
                            const double coef = qq * (rinv * rinv * rinv - gs);
                            // r_i - r_j = -(dx, dy, dz)
                            Fx -= coef * dx;
                            Fy -= coef * dy;
                            Fz -= coef * dz;
                            e += 0.5 * qq * (rinv - ph);
                        } else {
                            const float dx = (float)(int32_t)dux * g.hf[0];
                            const float dy = (float)(int32_t)duy * g.hf[1];
                            const float dz = (float)(int32_t)duz * g.hf[2];
                            const float r2 = dx * dx + dy * dy + dz * dz;
                            if (!decide32(g, r2, dux, duy, duz)) continue;
                            const float qq = qif * sqf[j];
                            const float rinv = __builtin_amdgcn_rsqf(r2);
                            float gs = 0.f, ph = 0.f;
                            for (int l = 0; l < g.ngauss; ++l) {
                                const float ex = __builtin_amdgcn_exp2f(-r2 * c.a32[l]);
                                gs += c.c32[l] * ex;
                                ph += c.w32[l] * ex;
                            }
                            const float coef = qq * (rinv * rinv * rinv - gs);
                            fx -= coef * dx;
                            fy -= coef * dy;
                            fz -= coef * dz;
                            e += 0.5 * (double)(qq * (rinv - ph));
                        }
                    }
                }
            }
        }
        const int64_t id = order[t];
        if constexpr (F64) {
            Fn[id] = Fx; Fn[n + id] = Fy; Fn[2 * n + id] = Fz;
        } else {
            Fn[id] = fx; Fn[n + id] = fy; Fn[2 * n + id] = fz;
        }
    }
    const double s = block_sum(e);
    if (threadIdx.x == 0) epart[blockIdx.x] = s;
}

// Debug export of the neighbour list with exactly the decision of k_near.
template <bool F64, bool FILL>
__global__ void k_neighbors(Geom g, const int32_t *__restrict__ start, const int32_t *__restrict__ order,
                            const uint32_t *__restrict__ su, const double *__restrict__ sx,
                            int64_t *__restrict__ counts, const int64_t *__restrict__ row_ptr,
                            int32_t *__restrict__ cols) {
    const int64_t n = g.n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t ux = su[t], uy = su[n + t], uz = su[2 * n + t];
    const int cx = (int)(((uint64_t)ux * (uint32_t)g.nc[0]) >> 32);
    const int cy = (int)(((uint64_t)uy * (uint32_t)g.nc[1]) >> 32);
    const int cz = (int)(((uint64_t)uz * (uint32_t)g.nc[2]) >> 32);
    const int64_t id = order[t];
    int64_t cnt = 0;
    int64_t base = FILL ? row_ptr[id] : 0;
    for (int oz = -g.reach[2]; oz <= g.reach[2]; ++oz)
        for (int oy = -g.reach[1]; oy <= g.reach[1]; ++oy)
            for (int ox = -g.reach[0]; ox <= g.reach[0]; ++ox) {
                const int32_t cj = wrapc(cx + ox, g.nc[0]) +
                                   g.nc[0] * (wrapc(cy + oy, g.nc[1]) + g.nc[1] * wrapc(cz + oz, g.nc[2]));
                for (int32_t j = start[cj]; j < start[cj + 1]; ++j) {
                    if (j == t) continue;
                    const uint32_t dux = su[j] - ux, duy = su[n + j] - uy, duz = su[2 * n + j] - uz;
                    bool in;
                    if constexpr (F64) {
                        const double dx = mi64(sx[j] - sx[t], g.L[0], g.invL[0]);
                        const double dy = mi64(sx[n + j] - sx[n + t], g.L[1], g.invL[1]);
                        const double dz = mi64(sx[2 * n + j] - sx[2 * n + t], g.L[2], g.invL[2]);
                        in = decide64(g, dx * dx + dy * dy + dz * dz, dux, duy, duz);
                    } else {
                        const float dx = (float)(int32_t)dux * g.hf[0];
                        const float dy = (float)(int32_t)duy * g.hf[1];
                        const float dz = (float)(int32_t)duz * g.hf[2];
                        in = decide32(g, dx * dx + dy * dy + dz * dz, dux, duy, duz);
                    }
                    if (!in) continue;
                    if (FILL) cols[base + cnt] = order[j];
                    ++cnt;
                }
            }
    if (!FILL) {
        counts[id] = cnt;
    } else {
        // ascending column order
        for (int64_t a = base + 1; a < base + cnt; ++a) {
            int32_t v = cols[a];
            int64_t b = a - 1;
            while (b >= base && cols[b] > v) {
                cols[b + 1] = cols[b];
                --b;
            }
            cols[b + 1] = v;
        }
    }
}

}  // namespace

int64_t near_blocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

void launch_near(const Geom &g, const SogDev &c, bool f64, const int32_t *start, const int32_t *order,
                 const uint32_t *su, const double *sx, const double *sq, const float *sqf, double *Fn,
                 double *epart, hipStream_t s) {
    dim3 grid(grid_for(g.n, kBlock)), block(kBlock);
    if (f64)
        hipLaunchKernelGGL(k_near<true>, grid, block, 0, s, g, c, start, order, su, sx, sq, sqf, Fn, epart);
    else
        hipLaunchKernelGGL(k_near<false>, grid, block, 0, s, g, c, start, order, su, sx, sq, sqf, Fn, epart);
}

void launch_neighbor_count(const Geom &g, bool f64, const int32_t *start, const int32_t *order,
                           const uint32_t *su, const double *sx, int64_t *counts, hipStream_t s) {
    dim3 grid(grid_for(g.n, kBlock)), block(kBlock);
    if (f64)
        hipLaunchKernelGGL((k_neighbors<true, false>), grid, block, 0, s, g, start, order, su, sx, counts,
                           (const int64_t *)nullptr, (int32_t *)nullptr);
    else
        hipLaunchKernelGGL((k_neighbors<false, false>), grid, block, 0, s, g, start, order, su, sx, counts,
                           (const int64_t *)nullptr, (int32_t *)nullptr);
}

void launch_neighbor_fill(const Geom &g, bool f64, const int32_t *start, const int32_t *order,
                          const uint32_t *su, const double *sx, const int64_t *row_ptr, int32_t *cols,
                          hipStream_t s) {
    dim3 grid(grid_for(g.n, kBlock)), block(kBlock);
    if (f64)
        hipLaunchKernelGGL((k_neighbors<true, true>), grid, block, 0, s, g, start, order, su, sx,
                           (int64_t *)nullptr, row_ptr, cols);
    else
        hipLaunchKernelGGL((k_neighbors<false, true>), grid, block, 0, s, g, start, order, su, sx,
                           (int64_t *)nullptr, row_ptr, cols);
}

}  // namespace rbsog
