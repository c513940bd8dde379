// Near part of the sum-of-Gaussians split for gfx950 (Sec. 3.1, eq.
// "forcesplit", with the factor of -grad U_N):
//   F_N,i = sum_{j: r_ij < r_c} q_i q_j (1/r^3 - 2 sum_l omega_l/s_l^2 e^{-r^2/s_l^2}) r_ij
//   U_N   = 1/2 sum_i sum_j q_i q_j (1/r - sum_l omega_l e^{-r^2/s_l^2})
//
// One wave per home cell.  The candidates of a cell are the particles of its
// 27 (or fewer) neighbouring cells; the three cells of a row are contiguous
// in cell order, so they are up to 18 contiguous ranges of the sorted arrays.
// The wave stages them in LDS with coalesced loads, then tests every (home i,
// candidate j) pair with i uniform across the wave and j on the lanes.  About
// one candidate in six lies inside r_c: accepted pairs are compacted with a
// ballot into an LDS queue and evaluated 64 at a time, so the pair arithmetic
// runs on full waves; forces accumulate into per-home LDS slots.  Blocks take
// contiguous chunks of cells, and chunks are assigned so that each XCD (blocks
// are dealt to the 8 XCDs round robin) works on one contiguous slab of the
// box and keeps it in its own L2.
//
// Gaussians with r_c^2/s_l^2 <= kTailTau are summed as one polynomial in r^2
// (their Taylor series, truncated below rounding), the narrow ones with an
// exponential each.  Pair inclusion follows the fixed-point rule of rbsog.h:
// an FP32 test decides every pair outside a narrow band around r_c, the exact
// FP64 rule decides the rest, so the list is bit-exact in both precisions.
#include <type_traits>

#include "rbsog_internal.h"

namespace rbsog {

namespace {

constexpr int kBlock = 256;
constexpr int kRanges = 18; // 9 rows of cells x up to 2 contiguous pieces

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

__device__ __forceinline__ float fixed_r2(const Geom &g, uint32_t dux, uint32_t duy, uint32_t duz) {
    const float dx = (float)(int32_t)dux * g.hf[0];
    const float dy = (float)(int32_t)duy * g.hf[1];
    const float dz = (float)(int32_t)duz * g.hf[2];
    return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ bool decide(const Geom &g, uint32_t dux, uint32_t duy, uint32_t duz) {
    const float r2 = fixed_r2(g, dux, duy, duz);
    if (r2 >= g.band_hi_f) return false;
    if (r2 <= g.band_lo_f) return true;
    return exact_in(g, dux, duy, duz);
}

__device__ __forceinline__ int wrapc(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// Range r (0..17) of the candidate cells of cell (cx, cy, cz) in cell order.
__device__ __forceinline__ bool row_range(const Geom &g, const int32_t *__restrict__ start, int r, int cx, int cy,
                                          int cz, int32_t &lo, int32_t &hi) {
    const int row = r >> 1, part = r & 1;
    const int oy = row % 3 - 1, oz = row / 3 - 1;
    if ((oy != 0 && !g.reach[1]) || (oz != 0 && !g.reach[2])) return false;
    const int jy = wrapc(cy + oy, g.nc[1]), jz = wrapc(cz + oz, g.nc[2]);
    const int base = g.nc[0] * (jy + g.nc[1] * jz);
    int xa, xb;
    if (!g.reach[0]) {
        if (part) return false;
        xa = xb = 0;
    } else {
        const int x0 = cx - 1, x1 = cx + 1;
        if (x0 < 0) {
            if (part == 0) { xa = xb = g.nc[0] - 1; } else { xa = 0; xb = x1; }
        } else if (x1 >= g.nc[0]) {
            if (part == 0) { xa = x0; xb = g.nc[0] - 1; } else { xa = xb = 0; }
        } else {
            if (part) return false;
            xa = x0; xb = x1;
        }
    }
    lo = start[base + xa];
    hi = start[base + xb + 1];
    return true;
}

__device__ __forceinline__ double mi64(double d, double L, double invL) { return d - L * rint(d * invL); }

__device__ double block_sum(double v) {
    __shared__ double ws[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) ws[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBlock / 64; ++w) s += ws[w];
    return s;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Broadcast the double held by lane `src` (uniform) to the whole wave.
__device__ __forceinline__ double bcast64(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}

constexpr int kNW = 4;        // waves per block
constexpr int kQueue = 128;   // pair queue entries per wave (>= 2 x 64)
constexpr int kExpMax = 12;   // explicit Gaussians held in registers

template <bool F64>
struct NearLds {
    using R = typename std::conditional<F64, double, float>::type;
    static constexpr int HC = F64 ? 64 : 128;   // home particles staged per batch
    static constexpr int CAP = 128;             // candidates staged per pass
    static constexpr int XH = F64 ? HC : 1;
    static constexpr int XC = F64 ? CAP : 1;
    uint4 hu[HC];          // home u_x, u_y, u_z, global sorted index
    R hq[HC];
    double hx[3][XH];
    R hf[3][HC];           // force accumulators of the home batch
    uint4 cu[CAP];         // candidate u_x, u_y, u_z, global sorted index
    R cq[CAP];
    double cx[3][XC];
    typename std::conditional<F64, double4, float4>::type qd[kQueue];  // queued pairs: x_j - x_i, q_i q_j
    uint32_t qs[kQueue];   // home slot of the queued pair
};

// Split coefficients held in registers (uniform): explicit Gaussians l < nexp
// and the tail polynomials.
template <bool F64>
struct NearCoef {
    using R = typename std::conditional<F64, double, float>::type;
    static constexpr int NT = (F64 ? kTailDeg64 : kTailDeg32) + 1;
    R a[kExpMax], cw[kExpMax], w[kExpMax];
    R pt[NT], ft[NT];
    int nexp, ntail;
};

template <bool F64>
__device__ __forceinline__ void load_coef(const Geom &g, const SogDev &c, NearCoef<F64> &k) {
    k.nexp = g.nexp < kExpMax ? g.nexp : kExpMax;
    k.ntail = F64 ? g.ntail64 : g.ntail32;
#pragma unroll
    for (int l = 0; l < kExpMax; ++l) {
        const bool on = l < k.nexp;
        if constexpr (F64) {
            k.a[l] = on ? c.a64[l] : 0.0; k.cw[l] = on ? c.c64[l] : 0.0; k.w[l] = on ? c.w64[l] : 0.0;
        } else {
            k.a[l] = on ? c.a32[l] : 0.f; k.cw[l] = on ? c.c32[l] : 0.f; k.w[l] = on ? c.w32[l] : 0.f;
        }
    }
#pragma unroll
    for (int t = 0; t < NearCoef<F64>::NT; ++t) {
        const bool on = t < k.ntail;
        if constexpr (F64) {
            k.pt[t] = on ? c.pt64[t] : 0.0; k.ft[t] = on ? c.ft64[t] : 0.0;
        } else {
            k.pt[t] = on ? c.pt32[t] : 0.f; k.ft[t] = on ? c.ft32[t] : 0.f;
        }
    }
}

// Evaluate the first `count` queued pairs, one per lane, and add their forces
// to the home accumulators.  Entries of one home are mostly contiguous in the
// queue (homes are tested one after another), so the forces are summed by a
// segmented scan across the wave and the last lane of each segment adds the
// total.
template <bool F64>
__device__ __forceinline__ void eval_batch(const Geom &g, const SogDev &c, const NearCoef<F64> &k, NearLds<F64> &L,
                                           int lane, int count, double &e) {
    using R = typename NearLds<F64>::R;
    const bool act = lane < count;
    R fx = 0, fy = 0, fz = 0;
    int slot = -1;
    if (act) {
        const auto qe = L.qd[lane];
        const R dx = qe.x, dy = qe.y, dz = qe.z, qq = qe.w;
        slot = (int)L.qs[lane];
        const R r2 = dx * dx + dy * dy + dz * dz;
        R rinv, gs = 0, ph = 0;
        if constexpr (F64) rinv = rsqrt(r2);
        else rinv = __builtin_amdgcn_rsqf(r2);
#pragma unroll
        for (int t = NearCoef<F64>::NT - 1; t >= 0; --t) {
            if constexpr (F64) { gs = fma(gs, r2, k.ft[t]); ph = fma(ph, r2, k.pt[t]); }
            else { gs = fmaf(gs, r2, k.ft[t]); ph = fmaf(ph, r2, k.pt[t]); }
        }
#pragma unroll
        for (int l = 0; l < kExpMax; ++l) {
            if (l < k.nexp) {
                R ex;
                if constexpr (F64) ex = exp(-r2 * k.a[l]);
                else ex = __builtin_amdgcn_exp2f(-r2 * k.a[l]);
                gs += k.cw[l] * ex;
                ph += k.w[l] * ex;
            }
        }
        for (int l = kExpMax; l < g.nexp; ++l) {
            if constexpr (F64) {
                const double ex = exp(-r2 * c.a64[l]);
                gs += c.c64[l] * ex; ph += c.w64[l] * ex;
            } else {
                const float ex = __builtin_amdgcn_exp2f(-r2 * c.a32[l]);
                gs += c.c32[l] * ex; ph += c.w32[l] * ex;
            }
        }
        const R coef = qq * (rinv * rinv * rinv - gs);
        // force on the home along r_i - r_j = -(dx, dy, dz)
        fx = -coef * dx;
        fy = -coef * dy;
        fz = -coef * dz;
        e += 0.5 * (double)(qq * (rinv - ph));
    }
    const int prev = __shfl_up(slot, 1, 64);
    const bool head = lane == 0 || slot != prev;
    const uint64_t H = __ballot(head);
    const uint64_t upto = H & ((2ull << lane) - 1ull);
    const int sstart = 63 - __clzll((long long)upto);
    for (int off = 1; off < 64; off <<= 1) {
        const R ux = __shfl_up(fx, off, 64), uy = __shfl_up(fy, off, 64), uz = __shfl_up(fz, off, 64);
        if (lane - off >= sstart) { fx += ux; fy += uy; fz += uz; }
    }
    const bool tail = act && (lane == count - 1 || (lane < 63 && ((H >> (lane + 1)) & 1ull)));
    // a home's entries are contiguous within one candidate pass, but a batch
    // can span two passes, so segment totals are still added atomically
    // (almost always one lane per home)
    if (tail) {
        atomicAdd(&L.hf[0][slot], fx);
        atomicAdd(&L.hf[1][slot], fy);
        atomicAdd(&L.hf[2][slot], fz);
    }
}

template <bool F64>
__global__ __launch_bounds__(64 * kNW) void k_near(Geom g, SogDev c, int64_t ncell, int64_t cells_per_block,
                                                   int32_t nblk, const int32_t *__restrict__ start,
                                                   const int32_t *__restrict__ order, const uint32_t *__restrict__ su,
                                                   const double *__restrict__ sx, const double *__restrict__ sq,
                                                   const float *__restrict__ sqf, double *__restrict__ Fn,
                                                   double *__restrict__ epart) {
    using Lds = NearLds<F64>;
    using R = typename Lds::R;
    __shared__ Lds lds[kNW];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    Lds &L = lds[wave];
    const int64_t n = g.n;
    NearCoef<F64> K;
    load_coef<F64>(g, c, K);
    // blocks are dealt to the 8 XCDs round robin: block b (on XCD b % 8) takes
    // chunk (b % 8) * (nblk / 8) + b / 8, so each XCD sweeps one slab of cells;
    // within the chunk each wave owns a contiguous run of cells
    const int32_t b = blockIdx.x;
    const int32_t chunk = (b % 8) * (nblk / 8) + b / 8;
    const int64_t c0 = (int64_t)chunk * cells_per_block;
    const int64_t c1 = c0 + cells_per_block < ncell ? c0 + cells_per_block : ncell;
    const int64_t per = (cells_per_block + kNW - 1) / kNW;
    const int64_t ra = c0 + wave * per < c1 ? c0 + wave * per : c1;
    const int64_t rb = ra + per < c1 ? ra + per : c1;
    double e = 0.0;
    int qn = 0;
    int32_t t = ra < rb ? start[ra] : 0;
    const int32_t t_hi = ra < rb ? start[rb] : 0;
    int64_t cur = ra;  // cell containing home t
    while (t < t_hi) {
        const int32_t t_end = t + Lds::HC < t_hi ? t + Lds::HC : t_hi;
        const int H = t_end - t;
        {
            // all loads of the batch first, then the LDS stores (one round trip)
            constexpr int S = Lds::HC / 64;
            uint32_t vx[S], vy[S], vz[S];
            R vq[S];
            double wx[S], wy[S], wz[S];
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2) {
                const int k = s2 * 64 + lane;
                if (k < H) {
                    const int64_t tt = t + k;
                    vx[s2] = su[tt]; vy[s2] = su[n + tt]; vz[s2] = su[2 * n + tt];
                    if constexpr (F64) {
                        vq[s2] = sq[tt];
                        wx[s2] = sx[tt]; wy[s2] = sx[n + tt]; wz[s2] = sx[2 * n + tt];
                    } else {
                        vq[s2] = sqf[tt];
                    }
                }
            }
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2) {
                const int k = s2 * 64 + lane;
                if (k < H) {
                    L.hu[k] = make_uint4(vx[s2], vy[s2], vz[s2], (uint32_t)(t + k));
                    L.hq[k] = vq[s2];
                    if constexpr (F64) { L.hx[0][k] = wx[s2]; L.hx[1][k] = wy[s2]; L.hx[2][k] = wz[s2]; }
                    L.hf[0][k] = 0; L.hf[1][k] = 0; L.hf[2][k] = 0;
                }
            }
        }
        while (start[cur + 1] <= t) ++cur;
        for (int64_t cell = cur; cell < rb && start[cell] < t_end; ++cell) {
            const int32_t hs = start[cell] > t ? start[cell] : t;
            const int32_t he = start[cell + 1] < t_end ? start[cell + 1] : t_end;
            if (hs >= he) continue;
            const int i0 = hs - t, i1 = he - t;
            const uint32_t cu32 = (uint32_t)cell;
            const int cx = (int)(cu32 % (uint32_t)g.nc[0]);
            const int cy = (int)((cu32 / (uint32_t)g.nc[0]) % (uint32_t)g.nc[1]);
            const int cz = (int)(cu32 / ((uint32_t)g.nc[0] * (uint32_t)g.nc[1]));
            // lane r < 18 holds candidate range r: first sorted index, and its
            // offsets in the flattened candidate list
            int32_t lo = 0, len = 0;
            if (lane < kRanges) {
                int32_t ra_, rb_;
                if (row_range(g, start, lane, cx, cy, cz, ra_, rb_)) { lo = ra_; len = rb_ - ra_; }
            }
            int32_t incl = len;
            for (int o = 1; o < 32; o <<= 1) {
                const int32_t v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            const int32_t excl = incl - len;
            const int32_t C = __shfl(incl, kRanges - 1, 64);
            for (int32_t cb = 0; cb < C; cb += Lds::CAP) {
                const int Cc = C - cb < Lds::CAP ? C - cb : Lds::CAP;
                // stage: each lane finds the range of its slots by counting range
                // ends (broadcast with readlane), then every load of the pass is
                // in flight at once, then the LDS stores
                wave_sync();
                {
                    constexpr int S = Lds::CAP / 64;
                    int rr[S];
#pragma unroll
                    for (int s2 = 0; s2 < S; ++s2) rr[s2] = 0;
                    for (int r = 0; r < kRanges - 1; ++r) {
                        const int32_t end = __builtin_amdgcn_readlane(incl, r);
#pragma unroll
                        for (int s2 = 0; s2 < S; ++s2) rr[s2] += (cb + s2 * 64 + lane >= end) ? 1 : 0;
                    }
                    uint32_t vj[S], vx[S], vy[S], vz[S];
                    R vq[S];
                    double wx[S], wy[S], wz[S];
                    // the permutes read other lanes' registers: run them with the
                    // whole wave active, before any predication
                    uint32_t jj[S];
#pragma unroll
                    for (int s2 = 0; s2 < S; ++s2)
                        jj[s2] = (uint32_t)(__shfl(lo, rr[s2], 64) + (cb + s2 * 64 + lane - __shfl(excl, rr[s2], 64)));
#pragma unroll
                    for (int s2 = 0; s2 < S; ++s2) {
                        const int k = s2 * 64 + lane;
                        if (k < Cc) {
                            const uint32_t j = jj[s2];
                            vj[s2] = j;
                            vx[s2] = su[j]; vy[s2] = su[n + j]; vz[s2] = su[2 * n + j];
                            if constexpr (F64) {
                                vq[s2] = sq[j];
                                wx[s2] = sx[j]; wy[s2] = sx[n + j]; wz[s2] = sx[2 * n + j];
                            } else {
                                vq[s2] = sqf[j];
                            }
                        }
                    }
#pragma unroll
                    for (int s2 = 0; s2 < S; ++s2) {
                        const int k = s2 * 64 + lane;
                        if (k < Cc) {
                            L.cu[k] = make_uint4(vx[s2], vy[s2], vz[s2], vj[s2]);
                            L.cq[k] = vq[s2];
                            if constexpr (F64) { L.cx[0][k] = wx[s2]; L.cx[1][k] = wy[s2]; L.cx[2][k] = wz[s2]; }
                        }
                    }
                }
                wave_sync();
                // homes of this cell in groups of 64: lane l holds home g0 + l in
                // registers and home i is broadcast with readlane, so the test
                // loop touches LDS only to append accepted pairs
                for (int g0 = i0; g0 < i1; g0 += 64) {
                    const int gn = i1 - g0 < 64 ? i1 - g0 : 64;
                    const int gi = g0 + lane;
                    const bool hv = gi < i1;
                    const uint4 hme = hv ? L.hu[gi] : make_uint4(0u, 0u, 0u, 0xffffffffu);
                    const R hqv = hv ? L.hq[gi] : R(0);
                    double hxv = 0, hyv = 0, hzv = 0;
                    if constexpr (F64) {
                        if (hv) { hxv = L.hx[0][gi]; hyv = L.hx[1][gi]; hzv = L.hx[2][gi]; }
                    }
                    // candidates of this pass in registers, S slots per lane
                    constexpr int S = Lds::CAP / 64;
                    uint4 cj[S];
                    R qj[S];
                    double xj[S], yj[S], zj[S];
#pragma unroll
                    for (int s2 = 0; s2 < S; ++s2) {
                        const int k = s2 * 64 + lane;
                        const bool kv = k < Cc;
                        cj[s2] = kv ? L.cu[k] : make_uint4(0u, 0u, 0u, 0xfffffffeu);
                        qj[s2] = kv ? L.cq[k] : R(0);
                        xj[s2] = yj[s2] = zj[s2] = 0;
                        if constexpr (F64) {
                            if (kv) { xj[s2] = L.cx[0][k]; yj[s2] = L.cx[1][k]; zj[s2] = L.cx[2][k]; }
                        }
                    }
                    for (int ii = 0; ii < gn; ++ii) {
                        const uint32_t hx_ = (uint32_t)__builtin_amdgcn_readlane((int)hme.x, ii);
                        const uint32_t hy_ = (uint32_t)__builtin_amdgcn_readlane((int)hme.y, ii);
                        const uint32_t hz_ = (uint32_t)__builtin_amdgcn_readlane((int)hme.z, ii);
                        const uint32_t hw_ = (uint32_t)__builtin_amdgcn_readlane((int)hme.w, ii);
#pragma unroll
                        for (int s2 = 0; s2 < S; ++s2) {
                            if (s2 * 64 >= Cc) break;
                            const uint32_t dux = cj[s2].x - hx_, duy = cj[s2].y - hy_, duz = cj[s2].z - hz_;
                            const float fx = (float)(int32_t)dux * g.hf[0];
                            const float fy = (float)(int32_t)duy * g.hf[1];
                            const float fz = (float)(int32_t)duz * g.hf[2];
                            const float r2 = fx * fx + fy * fy + fz * fz;
                            bool acc = cj[s2].w != hw_ && r2 < g.band_hi_f;
                            if (acc && r2 > g.band_lo_f) acc = exact_in(g, dux, duy, duz);
                            const uint64_t m = __ballot(acc);
                            if (acc) {
                                const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi(
                                                         (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                                if constexpr (F64) {
                                    L.qd[pos] = make_double4(mi64(xj[s2] - bcast64(hxv, ii), g.L[0], g.invL[0]),
                                                             mi64(yj[s2] - bcast64(hyv, ii), g.L[1], g.invL[1]),
                                                             mi64(zj[s2] - bcast64(hzv, ii), g.L[2], g.invL[2]),
                                                             bcast64(hqv, ii) * qj[s2]);
                                } else {
                                    const float hq_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hqv), ii));
                                    L.qd[pos] = make_float4(fx, fy, fz, hq_ * qj[s2]);
                                }
                                L.qs[pos] = (uint32_t)(g0 + ii);
                            }
                            qn = __builtin_amdgcn_readfirstlane(qn + (int)__popcll(m));
                            if (qn >= 64) {
                                wave_sync();
                                eval_batch<F64>(g, c, K, L, lane, 64, e);
                                const bool mv = lane + 64 < qn;
                                const auto rest = L.qd[mv ? lane + 64 : lane];
                                const uint32_t rs = L.qs[mv ? lane + 64 : lane];
                                wave_sync();
                                if (mv) {
                                    L.qd[lane] = rest;
                                    L.qs[lane] = rs;
                                }
                                qn -= 64;
                                wave_sync();
                            }
                        }
                    }
                }
                wave_sync();
            }
        }
        // the queue refers to this batch's home slots: drain it, then write
        wave_sync();
        if (qn > 0) eval_batch<F64>(g, c, K, L, lane, qn, e);
        qn = 0;
        wave_sync();
        for (int k = lane; k < H; k += 64) {
            const int64_t id = order[t + k];
            Fn[id] = (double)L.hf[0][k]; Fn[n + id] = (double)L.hf[1][k]; Fn[2 * n + id] = (double)L.hf[2][k];
        }
        wave_sync();
        t = t_end;
    }
    const double s = block_sum(e);
    if (threadIdx.x == 0) epart[blockIdx.x] = s;
}

// Debug export of the neighbour list with exactly the decision of k_near.
template <bool FILL>
__global__ void k_neighbors(Geom g, const int32_t *__restrict__ start, const int32_t *__restrict__ order,
                            const uint32_t *__restrict__ su, int64_t *__restrict__ counts,
                            const int64_t *__restrict__ row_ptr, int32_t *__restrict__ cols) {
    const int64_t n = g.n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t ux = su[t], uy = su[n + t], uz = su[2 * n + t];
    const int cx = (int)(((uint64_t)ux * (uint32_t)g.nc[0]) >> 32);
    const int cy = (int)(((uint64_t)uy * (uint32_t)g.nc[1]) >> 32);
    const int cz = (int)(((uint64_t)uz * (uint32_t)g.nc[2]) >> 32);
    const int64_t id = order[t];
    int64_t cnt = 0;
    const int64_t base = FILL ? row_ptr[id] : 0;
    for (int r = 0; r < kRanges; ++r) {
        int32_t lo, hi;
        if (!row_range(g, start, r, cx, cy, cz, lo, hi)) continue;
        for (int32_t j = lo; j < hi; ++j) {
            if (j == t) continue;
            if (!decide(g, su[j] - ux, su[n + j] - uy, su[2 * n + j] - uz)) continue;
            if (FILL) cols[base + cnt] = order[j];
            ++cnt;
        }
    }
    if (!FILL) {
        counts[id] = cnt;
    } else {
        for (int64_t a = base + 1; a < base + cnt; ++a) {
            const int32_t v = cols[a];
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

NearPlan near_plan(int64_t ncell) {
    // a multiple of 8 blocks (one contiguous slab per XCD); each wave owns a
    // run of about 8 cells, capped at 2048 blocks
    NearPlan p;
    int64_t nb = (ncell + 8 * kNW * 8 - 1) / (8 * kNW * 8);
    if (nb > 256) nb = 256;
    if (nb < 1) nb = 1;
    p.nblk = (int32_t)(8 * nb);
    p.cells_per_block = (ncell + p.nblk - 1) / p.nblk;
    return p;
}

void launch_near(const Geom &g, const SogDev &c, bool f64, const NearPlan &np, int64_t ncell, const int32_t *start,
                 const int32_t *order, const uint32_t *su, const double *sx, const double *sq, const float *sqf,
                 double *Fn, double *epart, hipStream_t s) {
    dim3 grid((unsigned)np.nblk), block(64 * kNW);
    if (f64)
        hipLaunchKernelGGL(k_near<true>, grid, block, 0, s, g, c, ncell, np.cells_per_block, np.nblk, start, order,
                           su, sx, sq, sqf, Fn, epart);
    else
        hipLaunchKernelGGL(k_near<false>, grid, block, 0, s, g, c, ncell, np.cells_per_block, np.nblk, start, order,
                           su, sx, sq, sqf, Fn, epart);
}

void launch_neighbor_count(const Geom &g, const int32_t *start, const int32_t *order, const uint32_t *su,
                           int64_t *counts, hipStream_t s) {
    hipLaunchKernelGGL(k_neighbors<false>, dim3(grid_for(g.n, kBlock)), dim3(kBlock), 0, s, g, start, order, su,
                       counts, (const int64_t *)nullptr, (int32_t *)nullptr);
}

void launch_neighbor_fill(const Geom &g, const int32_t *start, const int32_t *order, const uint32_t *su,
                          const int64_t *row_ptr, int32_t *cols, hipStream_t s) {
    hipLaunchKernelGGL(k_neighbors<true>, dim3(grid_for(g.n, kBlock)), dim3(kBlock), 0, s, g, start, order, su,
                       (int64_t *)nullptr, row_ptr, cols);
}

}  // namespace rbsog
