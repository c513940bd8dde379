// Fourier part of the random batch sum-of-Gaussians method for gfx950
// (Sec. 3.1 eq. "fourtrans"; Sec. 3.3 eq. "approximateForce"):
//   rho(k_e) = sum_j q_j e^{i k_e.r_j}
//   F*_i     = -q_i sum_e w_e k_e (Im rho_e cos th_ie - Re rho_e sin th_ie),  th_ie = k_e.r_i
//   U*       = 1/2 sum_e w_e |rho_e|^2
// Phases are taken in revolutions of the fractional coordinate, th/(2 pi) =
// m.s with s = x/L: FP64 forms evaluate kTurnTab t = m.(kTurnTab s) in FP64
// and sin/cos of 2 pi t through a table of 1024 turns in LDS and short
// polynomials of the rest;
// FP32 forms take m.u mod 2^32 exactly on the 32-bit fixed-point coordinate
// and the hardware sin/cos of the revolution.
//
// Work split: the structure factor puts one wave vector on each lane and
// streams particles uniformly through the wave (no cross-lane reduction in
// the inner loop); the force puts one particle on each lane and streams the
// P wave-vector records uniformly.  Both walk lists of work items, each item
// within one system of the batch.  Partial sums of rho are reduced in a
// fixed order, so the result is identical from run to run.
#include "rbsog_internal.h"
#include "rbsog_math.h"

#include <type_traits>

namespace rbsog {

namespace {


using rmath::sincos2pi;

typedef const SysDev __attribute__((address_space(4))) CSys;
// k records are read-only within the kernels that stream them: reading them
// through the constant address space makes the uniform reads scalar loads
typedef const KRec64 __attribute__((address_space(4))) CRec64;
typedef const KRec32 __attribute__((address_space(4))) CRec32;
// whole records (one scalar load each)
__device__ __forceinline__ KRec64 ld(CRec64 *p) {
    KRec64 r;
    r.mx = p->mx; r.my = p->my; r.mz = p->mz;
    r.phi = p->phi;
    r.ax = p->ax; r.ay = p->ay; r.az = p->az;
    r.pad = p->pad;
    return r;
}
// the far sum's part of a record: -m and a (one 24-byte load)
struct KFar32 {
    uint32_t nmx, nmy, nmz;
    float ax, ay, az;
};
__device__ __forceinline__ KFar32 ld(CRec32 *p) {
    typedef const unsigned long long __attribute__((address_space(4))) CU64;
    const unsigned long long w0 = ((CU64 *)p)[0], w1 = ((CU64 *)p)[1], w2 = ((CU64 *)p)[2];
    KFar32 r;
    r.nmx = (uint32_t)w0; r.nmy = (uint32_t)(w0 >> 32);
    r.nmz = (uint32_t)w1; r.ax = __uint_as_float((uint32_t)(w1 >> 32));
    r.ay = __uint_as_float((uint32_t)w2); r.az = __uint_as_float((uint32_t)(w2 >> 32));
    return r;
}

// Uniform values loaded from memory: keep them scalar.
__device__ __forceinline__ int32_t rfl(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t rfl64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Structure factor partial sums over the work items (grid-stride).  Item
// (s, kg, chunk, [j0, j1)): wave w handles k tile (w % kt) of group kg (one
// wave vector per lane) for particle stream (w / kt); kt * streams <= 16
// waves per block.  The block stages kStage particles at a time in LDS (one
// coalesced load per thread: fixed-point coordinates and FP32 charge in
// FP32C, fractional coordinates and charge in FP64); stream st then reads
// every streams-th staged particle from st on, each read an LDS broadcast to
// the wave.  The streams' sums are added in a fixed order.
constexpr int kStage = 1024;
struct Stage64 {
    double sx, sy, sz, q;
};

// FP32C staging of particles [jb, jb + cnt) of the block's chunk for the
// structure factor (blocks of 1024 threads, 16 waves): each wave splits its
// 64 particles by the sign of the charge and pairs consecutive ones of a
// sign (lane order) whose charges are equal; a pair (u1, u2) is written as
// two records, h = u1 + ((u2 - u1) >> 1) with 2q and d = u1 - h (so u1 = h +
// d and u2 = h - d up to one unit of 2^-32 of the box: the pair's phases
// are m.h +- m.d mod 2^32), the particles left single after all pairs as
// (u, q).  Returns the block's number of pairs; the records fill
// st32[0, cnt).  Ends with a barrier.
__device__ __forceinline__ int stage_pairs(const uint32_t *__restrict__ u, const float *__restrict__ qf, int64_t n,
                                           int64_t jb, int cnt, uint4 *st32, int2 *wcnt) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool have = (int)threadIdx.x < cnt;
    uint32_t ux = 0, uy = 0, uz = 0, qb = 0;
    if (have) {
        const int64_t j = jb + threadIdx.x;
        ux = u[j];
        uy = u[n + j];
        uz = u[2 * n + j];
        qb = __float_as_uint(qf[j]);
    }
    const bool pos = __uint_as_float(qb) > 0.f;
    const uint64_t all = __builtin_amdgcn_ballot_w64(have), plus = __builtin_amdgcn_ballot_w64(have && pos);
    const uint64_t mine = pos ? plus : (all & ~plus);
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint64_t below = mine & lt, above = mine & ~(lt | (1ull << lane));
    const int rank = __builtin_popcountll(below), ncls = __builtin_popcountll(mine);
    const int nl = above ? __builtin_ctzll(above) : lane;        // next lane of the class
    const int pl = below ? 63 - __builtin_clzll(below) : lane;   // previous lane of the class
    const uint32_t nx = __shfl(ux, nl, 64), ny = __shfl(uy, nl, 64), nz = __shfl(uz, nl, 64);
    const uint32_t nq = __shfl(qb, nl, 64), pq = __shfl(qb, pl, 64);
    const bool lead = have && (rank & 1) == 0 && rank + 1 < ncls && nq == qb;
    const bool follow = have && (rank & 1) == 1 && pq == qb;
    const bool single = have && !lead && !follow;
    const uint64_t lm = __builtin_amdgcn_ballot_w64(lead), sm = __builtin_amdgcn_ballot_w64(single);
    if (lane == 0) wcnt[wave] = make_int2(__builtin_popcountll(lm), __builtin_popcountll(sm));
    __syncthreads();
    int pofs = 0, sofs = 0, np = 0;
    for (int w = 0; w < 16; ++w) {
        const int2 c = wcnt[w];
        np += c.x;
        if (w < wave) {
            pofs += c.x;
            sofs += c.y;
        }
    }
    if (lead) {
        const int o = 2 * (pofs + __builtin_popcountll(lm & lt));
        const uint32_t hx = ux + (uint32_t)((int32_t)(nx - ux) >> 1), hy = uy + (uint32_t)((int32_t)(ny - uy) >> 1),
                       hz = uz + (uint32_t)((int32_t)(nz - uz) >> 1);
        st32[o] = make_uint4(hx, hy, hz, __float_as_uint(2.f * __uint_as_float(qb)));
        st32[o + 1] = make_uint4(ux - hx, uy - hy, uz - hz, 0u);
    }
    if (single) st32[2 * np + sofs + __builtin_popcountll(sm & lt)] = make_uint4(ux, uy, uz, qb);
    __syncthreads();
    return np;
}

template <bool F64>
__global__ __launch_bounds__(1024, F64 ? 1 : 8) void k_rho(EvalArgs a, const RhoItem *__restrict__ items, int32_t nitems) {
    __shared__ double2 red[1024];
    __shared__ uint4 st32[F64 ? 1 : kStage];
    __shared__ int2 wcnt[F64 ? 1 : 16];
    __shared__ Stage64 st64[F64 ? kStage : 1];
    // FP64: cos and sin of the kTurnTab turns (sincos2pi_tab); the staging
    // loop's first barrier orders the fill before any use
    __shared__ double2 turn[F64 ? rmath::kTurnTab : 1];
    if constexpr (F64) {
        for (int j = threadIdx.x; j < rmath::kTurnTab; j += blockDim.x) {
            const double f = (double)j / rmath::kTurnTab;
            double sn, cs;
            sincos2pi(f - rint(f), &sn, &cs);
            turn[j] = make_double2(cs, sn);
        }
    }
    const int64_t n = a.N;
    // the state as the kick/drift kernel left it, in its copy: the re-sort of
    // the state into cell order may run meanwhile
    const double *__restrict__ x = a.rs_x;
    const double *__restrict__ q = a.rs_q;
    const float *__restrict__ qf = a.rs_qf;
    const uint32_t *__restrict__ u = a.rs_u;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    for (int32_t itx = blockIdx.x; itx < nitems; itx += gridDim.x) {
        const RhoItem item = items[itx];
        const int32_t sys = rfl(item.sys), kg = rfl(item.kg), chunk = rfl(item.chunk);
        CSys *sp = (CSys *)(a.sys + sys);
        const int32_t P = sp->P, kt = sp->kt, streams = sp->streams;
        const int kti = wave % kt, st = wave / kt;
        const int32_t k = (kg * kt + kti) * 64 + lane;
        const bool active = k < P && st < streams;
        // the batch's wave vectors, read from the sequence at the cursor
        const int32_t *__restrict__ mk = sp->kseq + 3 * (rfl64(a.kcur[sys]) + (k < P ? k : 0));
        const int64_t j0 = rfl64(item.j0), j1 = rfl64(item.j1);
        double re = 0.0, im = 0.0;
        if constexpr (F64) {
            const double mx = mk[0], my = mk[1], mz = mk[2];
            // fractional coordinates in table units (kTurnTab per box length)
            const double ix = sp->g.invL[0] * rmath::kTurnTab, iy = sp->g.invL[1] * rmath::kTurnTab,
                         iz = sp->g.invL[2] * rmath::kTurnTab;
            for (int64_t jb = j0; jb < j1; jb += kStage) {
                const int cnt = (int)(j1 - jb < kStage ? j1 - jb : kStage);
                if ((int)threadIdx.x < cnt) {
                    const int64_t j = jb + threadIdx.x;
                    st64[threadIdx.x] = Stage64{x[j] * ix, x[n + j] * iy, x[2 * n + j] * iz, q[j]};
                }
                __syncthreads();
                if (st < streams) {
                    // four staged particles read at once, then used
                    int h = st;
                    for (; h + 4 * streams <= cnt; h += 4 * streams) {
                        Stage64 p[4];
#pragma unroll
                        for (int g = 0; g < 4; ++g) p[g] = st64[h + g * streams];
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const double t = mx * p[g].sx + my * p[g].sy + mz * p[g].sz;
                            double sn, cs;
                            rmath::sincos2pi_tab(t, turn, &sn, &cs);
                            re = fma(p[g].q, cs, re);
                            im = fma(p[g].q, sn, im);
                        }
                    }
                    for (; h < cnt; h += streams) {
                        const Stage64 p = st64[h];
                        const double t = mx * p.sx + my * p.sy + mz * p.sz;
                        double sn, cs;
                        rmath::sincos2pi_tab(t, turn, &sn, &cs);
                        re = fma(p.q, cs, re);
                        im = fma(p.q, sn, im);
                    }
                }
                __syncthreads();
            }
        } else {
            const uint32_t mx = (uint32_t)mk[0], my = (uint32_t)mk[1], mz = (uint32_t)mk[2];
            for (int64_t jb = j0; jb < j1; jb += kStage) {
                const int cnt = (int)(j1 - jb < kStage ? j1 - jb : kStage);
                const int np = stage_pairs(u, qf, n, jb, cnt, st32, wcnt);
                const int ns = cnt - 2 * np;
                if (st < streams) {
                    // pairs of equal charge q with phases t_m +- t_d: the
                    // pair adds 2 q cos(t_d) e^{i t_m} (cos a + cos b = 2
                    // cos((a+b)/2) cos((a-b)/2), sin a + sin b = 2
                    // sin((a+b)/2) cos((a-b)/2)): three transcendentals
                    // and three multiply-adds where the two particles take
                    // four of each.  FP32 sums over runs of 16 pairs (32
                    // singles), then FP64.
                    auto pairs = [&](auto one) {
                        constexpr bool ONE = decltype(one)::value;
                        const int sd = ONE ? 1 : streams;
                        int h = st;
                        for (; h + 16 * sd <= np; h += 16 * sd) {
                            float rf = 0.f, fi = 0.f;
                            for (int g0 = 0; g0 < 16; g0 += 4) {
                                uint4 pa[4], pb[4];
#pragma unroll
                                for (int g = 0; g < 4; ++g) {
                                    pa[g] = st32[2 * (h + (g0 + g) * sd)];
                                    pb[g] = st32[2 * (h + (g0 + g) * sd) + 1];
                                }
#pragma unroll
                                for (int g = 0; g < 4; ++g) {
                                    const float fm = rmath::phase_rev(rmath::dot3_mod32_v(mx, my, mz, pa[g].x, pa[g].y, pa[g].z));
                                    const float fd = rmath::phase_rev(rmath::dot3_mod32_v(mx, my, mz, pb[g].x, pb[g].y, pb[g].z));
                                    const float w = __uint_as_float(pa[g].w) * __builtin_amdgcn_cosf(fd);
                                    rf = fmaf(w, __builtin_amdgcn_cosf(fm), rf);
                                    fi = fmaf(w, __builtin_amdgcn_sinf(fm), fi);
                                }
                            }
                            re += rf;
                            im += fi;
                        }
                        float rf = 0.f, fi = 0.f;
                        for (; h < np; h += sd) {
                            const uint4 pa = st32[2 * h], pb = st32[2 * h + 1];
                            const float fm = rmath::phase_rev(rmath::dot3_mod32_v(mx, my, mz, pa.x, pa.y, pa.z));
                            const float fd = rmath::phase_rev(rmath::dot3_mod32_v(mx, my, mz, pb.x, pb.y, pb.z));
                            const float w = __uint_as_float(pa.w) * __builtin_amdgcn_cosf(fd);
                            rf = fmaf(w, __builtin_amdgcn_cosf(fm), rf);
                            fi = fmaf(w, __builtin_amdgcn_sinf(fm), fi);
                        }
                        re += rf;
                        im += fi;
                    };
                    if (streams == 1) pairs(std::true_type{});
                    else pairs(std::false_type{});
                    // the particles left single (at most two per wave of
                    // the stage, more where charges differ)
                    const uint4 *sg = st32 + 2 * np;
                    float rf = 0.f, fi = 0.f;
                    for (int h = st; h < ns; h += streams) {
                        const uint4 p = sg[h];
                        const float f = rmath::phase_rev(rmath::dot3_mod32_v(mx, my, mz, p.x, p.y, p.z));
                        const float pq = __uint_as_float(p.w);
                        rf = fmaf(pq, __builtin_amdgcn_cosf(f), rf);
                        fi = fmaf(pq, __builtin_amdgcn_sinf(f), fi);
                    }
                    re += rf;
                    im += fi;
                }
                __syncthreads();
            }
        }
        red[threadIdx.x] = make_double2(re, im);
        __syncthreads();
        if (st == 0 && active) {
            double sr = 0.0, si = 0.0;
            for (int s2 = 0; s2 < streams; ++s2) {
                const double2 v = red[(s2 * kt + kti) * 64 + lane];
                sr += v.x;
                si += v.y;
            }
            // layout [k][chunk]: the reduction reads each k's partials contiguously
            const int64_t o = sp->pofs + (int64_t)k * sp->nch + chunk;
            a.partial[2 * o] = sr;
            a.partial[2 * o + 1] = si;
        }
        __syncthreads();
        if (sp->zmode != 0 && kg == 0) {
            // dipole moment of the chunk, sum_j q_j x_j over the wrapped
            // positions, for the zero-frequency mode term (fixed order)
            double mx = 0.0, my = 0.0, mz = 0.0;
            for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
                const double qj = q[j];
                mx = fma(qj, x[j], mx);
                my = fma(qj, x[n + j], my);
                mz = fma(qj, x[2 * n + j], mz);
            }
            red[threadIdx.x] = make_double2(mx, my);
            __syncthreads();
            for (int w = 512; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) {
                    red[threadIdx.x].x += red[threadIdx.x + w].x;
                    red[threadIdx.x].y += red[threadIdx.x + w].y;
                }
                __syncthreads();
            }
            const double2 mxy = red[0];
            __syncthreads();
            red[threadIdx.x] = make_double2(mz, 0.0);
            __syncthreads();
            for (int w = 512; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) red[threadIdx.x].x += red[threadIdx.x + w].x;
                __syncthreads();
            }
            if (threadIdx.x == 0) {
                const int64_t c = 3 * (sp->choff + chunk);
                a.dip_part[c] = mxy.x;
                a.dip_part[c + 1] = mxy.y;
                a.dip_part[c + 2] = red[0].x;
            }
            __syncthreads();
        }
    }
}

// Sum over the wave in a fixed order (the same on every run).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Record r of system sys (its k-th wave vector) from its rho: rho and the
// per-k energy stored, and the amplitude-phase records of both forms
// written.  The cursor still points at the batch.
__device__ __forceinline__ void write_record(const EvalArgs &a, const SysDev &sd, int32_t sys, int64_t r, int32_t k,
                                             double re, double im) {
    a.rho[r] = re;
    a.rho[a.K + r] = im;
    // the batch's k-th vector of the sequence and its weight (the
    // cursor moves once every record of the system is reduced)
    const int64_t e = a.kcur[sys] + k;
    const int32_t m[3] = {sd.kseq[3 * e], sd.kseq[3 * e + 1], sd.kseq[3 * e + 2]};
    const double w = sd.kw ? sd.kw[e] : sd.w_rb;
    a.ek[r] = 0.5 * w * (re * re + im * im);
    // amplitude-phase record: phi = arg(rho) / (2 pi), a = w |rho| k
    const double phi = atan2(im, re) * (1.0 / rmath::kTwoPi);
    const double mag = hypot(re, im);
    const double c = w * mag * rmath::kTwoPi;
    KRec64 h;
    h.mx = m[0];
    h.my = m[1];
    h.mz = m[2];
    h.phi = phi * rmath::kTurnTab;
    h.ax = c * h.mx * sd.g.invL[0];
    h.ay = c * h.my * sd.g.invL[1];
    h.az = c * h.mz * sd.g.invL[2];
    h.pad = 0.0;
    a.kb64[r] = h;
    // FP32 form: phi in 2^-32 turns, plus 2^9 units: the FP32 phases of
    // the structure factor and of the far force are each truncated
    // to 2^-23 turns (half a unit of it low on average), which this
    // offset takes back
    KRec32 f;
    f.nmx = -m[0];
    f.nmy = -m[1];
    f.nmz = -m[2];
    f.phi = (uint32_t)(int64_t)rint(phi * 4294967296.0) + 512u;
    f.ax = (float)h.ax;
    f.ay = (float)h.ay;
    f.az = (float)h.az;
    f.pad = 0.f;
    a.kb32[r] = f;
}

// The structure factor's reduction.  Per k record r: rho = sum over the
// system's chunks of the partials (fixed order), the per-k energy
// 1/2 w |rho|^2, and rho written into the records; then k_rho_finish sums
// each system's far energy.  U_N and U follow in k_kinetic, after the near
// part.  Nothing here waits for the near part.  (A last-block finish inside
// the reduction would need a device-scope fence in every block, a writeback
// of the XCD's L2 each: 0.3 ms for the 6,400 blocks of a 256-system batch.)
// k_rho_reduce: one wave per record, four records per block (systems of few
// chunks, many of them in a batch).
__global__ __launch_bounds__(256) void k_rho_reduce(EvalArgs a) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + wave;
    int32_t sys = -1;
    if (r < a.K) {
        sys = a.ksys[r];
        const SysDev &sd = a.sys[sys];
        const int32_t k = (int32_t)(r - sd.k0);
        const double2 *pk = reinterpret_cast<const double2 *>(a.partial) + sd.pofs + (int64_t)k * sd.nch;
        const int32_t nch = sd.nch;
        // four independent loads in flight per lane, summed in a fixed order
        double2 v0 = make_double2(0.0, 0.0), v1 = v0, v2 = v0, v3 = v0;
        int32_t c = lane;
        for (; c + 192 < nch; c += 256) {
            const double2 a0 = pk[c], a1 = pk[c + 64], a2 = pk[c + 128], a3 = pk[c + 192];
            v0.x += a0.x; v0.y += a0.y; v1.x += a1.x; v1.y += a1.y;
            v2.x += a2.x; v2.y += a2.y; v3.x += a3.x; v3.y += a3.y;
        }
        for (; c < nch; c += 64) {
            const double2 a0 = pk[c];
            v0.x += a0.x; v0.y += a0.y;
        }
        double re = (v0.x + v1.x) + (v2.x + v3.x), im = (v0.y + v1.y) + (v2.y + v3.y);
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) write_record(a, sd, sys, r, k, re, im);
    }
}

// k_rho_reduce_block: one block per record (systems of many chunks): each
// thread a fixed strided subset of the chunks with eight loads in flight,
// then a fixed butterfly across each wave and the four waves in order.
__global__ __launch_bounds__(256) void k_rho_reduce_block(EvalArgs a) {
    __shared__ double2 red[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r = blockIdx.x;
    const int32_t sys = a.ksys[r];
    const SysDev &sd = a.sys[sys];
    const int32_t k = (int32_t)(r - sd.k0);
    const double2 *pk = reinterpret_cast<const double2 *>(a.partial) + sd.pofs + (int64_t)k * sd.nch;
    const int32_t nch = sd.nch;
    double2 v[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) v[h] = make_double2(0.0, 0.0);
    int32_t c = threadIdx.x;
    for (; c + 7 * 256 < nch; c += 8 * 256) {
        double2 w[8];
#pragma unroll
        for (int h = 0; h < 8; ++h) w[h] = pk[c + h * 256];
#pragma unroll
        for (int h = 0; h < 8; ++h) {
            v[h].x += w[h].x;
            v[h].y += w[h].y;
        }
    }
    for (; c < nch; c += 256) {
        const double2 w = pk[c];
        v[0].x += w.x;
        v[0].y += w.y;
    }
    double re = ((v[0].x + v[1].x) + (v[2].x + v[3].x)) + ((v[4].x + v[5].x) + (v[6].x + v[7].x));
    double im = ((v[0].y + v[1].y) + (v[2].y + v[3].y)) + ((v[4].y + v[5].y) + (v[6].y + v[7].y));
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) red[wave] = make_double2(re, im);
    __syncthreads();
    if (threadIdx.x == 0) {
        re = (red[0].x + red[1].x) + (red[2].x + red[3].x);
        im = (red[0].y + red[1].y) + (red[2].y + red[3].y);
        write_record(a, sd, sys, r, k, re, im);
    }
}

// Per system, one block, after the reduction: the far energy U* = sum_e
// ek_e (strided sums, then a fixed tree) with the zero-frequency mode term
// and its dipole (the chunks' dipole partials, the same way), U_self, and
// the sequence cursor moved on by P.  A kernel of its own: the records'
// writes are visible to it without fences.
__global__ __launch_bounds__(256) void k_rho_finish(EvalArgs a) {
    __shared__ double si[4][256];
    const int32_t s = blockIdx.x;
    const SysDev &sd = a.sys[s];
    double us = 0.0;
    for (int64_t e = threadIdx.x; e < sd.P; e += 256) us += a.ek[sd.k0 + e];
    double m[3] = {0.0, 0.0, 0.0};
    if (sd.zmode != 0)
        for (int32_t ch = threadIdx.x; ch < sd.nch; ch += 256)
            for (int d = 0; d < 3; ++d) m[d] += a.dip_part[3 * (sd.choff + ch) + d];
    si[0][threadIdx.x] = us;
    si[1][threadIdx.x] = m[0];
    si[2][threadIdx.x] = m[1];
    si[3][threadIdx.x] = m[2];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int j = 0; j < 4; ++j) si[j][threadIdx.x] += si[j][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double u0 = 0.0;
        if (sd.zmode != 0) {
            const double M[3] = {si[1][0], si[2][0], si[3][0]};
            for (int d = 0; d < 3; ++d) a.dipole[3 * s + d] = M[d];
            u0 = sd.zmode == 1 ? sd.zu * (M[0] * M[0] + M[1] * M[1] + M[2] * M[2]) : sd.zu * M[2] * M[2];
        }
        // U* holds the far part with the zero-frequency mode term
        a.E[4 * s + 1] = si[0][0] + u0;
        a.E[4 * s + 2] = sd.uself;
        a.kcur[s] += sd.P;
        if (s == 0 && a.kick && a.thermo) *a.tstep += 1;
    }
}

// cos and sin of the kTurnTab turns in LDS for sincos2pi_tab (FP64 forms);
// all threads of the block reach the barrier.
__device__ __forceinline__ void fill_turns(double2 *turn) {
    for (int j = threadIdx.x; j < rmath::kTurnTab; j += blockDim.x) {
        const double f = (double)j / rmath::kTurnTab;
        double sn, cs;
        sincos2pi(f - rint(f), &sn, &cs);
        turn[j] = make_double2(cs, sn);
    }
    __syncthreads();
}

// Records whose phases a wave stages at once in the FP32C far sum.
constexpr int kFarStage = 256;
// s_waitcnt lgkmcnt(0) with the other counters left alone (gfx9 encoding)
constexpr int kWaitLgkm0 = 0xC07F;

// Far force on particle i (the factor -q_i included) from its system's P
// amplitude-phase records, streamed as uniform loads: one sine per record,
// F_i = -q_i sum_e a_e sin(2 pi (phi_e - m_e.s_i)).  Positions and charges
// from (u, qf) in FP32C (the phase phi - m.u mod 2^32), (x, q) in FP64.
template <bool F64>
__device__ __forceinline__ void far_sum(CSys *sp, CRec64 *kb64, CRec32 *kb32, int32_t P, int64_t n, int64_t i,
                                        const uint32_t *__restrict__ u, const float *__restrict__ qf,
                                        const double *__restrict__ x, const double *__restrict__ q,
                                        const double2 *turn, uint64_t *phs, double &Fx, double &Fy, double &Fz) {
    Fx = 0.0; Fy = 0.0; Fz = 0.0;
    // records are consumed in groups so that their uniform loads overlap
    if constexpr (F64) {
        // fractional coordinates in table units, as the records' phase
        constexpr double tu = rmath::kTurnTab;
        const double sx = x[i] * (sp->g.invL[0] * tu), sy = x[n + i] * (sp->g.invL[1] * tu),
                     sz = x[2 * n + i] * (sp->g.invL[2] * tu);
        constexpr int G = 4;
        int32_t e = 0;
        for (; e + G <= P; e += G) {
            KRec64 r[G];
#pragma unroll
            for (int h = 0; h < G; ++h) r[h] = ld(kb64 + e + h);
#pragma unroll
            for (int h = 0; h < G; ++h) {
                const double t = fma(-r[h].mx, sx, fma(-r[h].my, sy, fma(-r[h].mz, sz, r[h].phi)));
                double v, cv;
                rmath::sincos2pi_tab(t, turn, &v, &cv);
                Fx = fma(r[h].ax, v, Fx);
                Fy = fma(r[h].ay, v, Fy);
                Fz = fma(r[h].az, v, Fz);
            }
        }
        for (; e < P; ++e) {
            const KRec64 r = ld(kb64 + e);
            const double t = fma(-r.mx, sx, fma(-r.my, sy, fma(-r.mz, sz, r.phi)));
            double v, cv;
            rmath::sincos2pi_tab(t, turn, &v, &cv);
            Fx = fma(r.ax, v, Fx);
            Fy = fma(r.ay, v, Fy);
            Fz = fma(r.az, v, Fz);
        }
        const double qi = q[i];
        Fx *= -qi; Fy *= -qi; Fz *= -qi;
    } else {
        const uint32_t ux = u[i], uy = u[n + i], uz = u[2 * n + i];
        // per stage of up to 256 records: each lane copies four records'
        // phases into the wave's LDS slots, from where they are read back
        // broadcast as the addends of the phase chains (phi + (-m).u = phi -
        // m.u mod 2^32, the records holding -m: the subtraction costs no
        // vector instruction).  The next stage's phases are loaded while the
        // current one is summed.  FP32 partial sums over runs of 64 records,
        // accumulated in FP64.
        const KRec32 *kg = (const KRec32 *)kb32;
        const int lane = threadIdx.x & 63;
        constexpr int G = 4;
        auto rec = [&](const KFar32 &r, uint64_t c, float &fx, float &fy, float &fz) {
            const uint32_t t = rmath::dot3_add_mod32_s(r.nmx, r.nmy, r.nmz, ux, uy, uz, c);
            const float v = __builtin_amdgcn_sinf(rmath::phase_rev(t));
            fx = fmaf(r.ax, v, fx);
            fy = fmaf(r.ay, v, fy);
            fz = fmaf(r.az, v, fz);
        };
        uint32_t nxt[kFarStage / 64];
        auto fetch = [&](int32_t e0) {
#pragma unroll
            for (int h = 0; h < kFarStage / 64; ++h) {
                const int32_t e = e0 + 64 * h + lane;
                nxt[h] = kg[e < P ? e : 0].phi;
            }
        };
        fetch(0);
        for (int32_t e0 = 0; e0 < P; e0 += kFarStage) {
            wave_sync();  // the previous stage's broadcast reads are done
#pragma unroll
            for (int h = 0; h < kFarStage / 64; ++h) phs[64 * h + lane] = (uint64_t)nxt[h];
            wave_sync();
            if (e0 + kFarStage < P) fetch(e0 + kFarStage);
            const int32_t e1 = P - e0 < kFarStage ? P : e0 + kFarStage;
            for (int32_t e = e0; e < e1; e += 64) {
                const int cnt = e1 - e < 64 ? e1 - e : 64;
                const uint64_t *ph = phs + (e - e0);
                float fx = 0.f, fy = 0.f, fz = 0.f;
                if (cnt == 64) {
                    // scalar loads and LDS reads share one wait counter, and
                    // a wait on it covers every scalar load in flight: the
                    // group's phases are read and waited for before the next
                    // group's records are requested, which then arrive while
                    // the group is summed
                    KFar32 r[G];
#pragma unroll
                    for (int h = 0; h < G; ++h) r[h] = ld(kb32 + e + h);
#pragma unroll
                    for (int h4 = 0; h4 < 64; h4 += G) {
                        const ulonglong2 w0 = *(const ulonglong2 *)(ph + h4), w1 = *(const ulonglong2 *)(ph + h4 + 2);
                        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
                        __builtin_amdgcn_sched_barrier(0);
                        KFar32 rn[G];
                        if (h4 + G < 64) {
#pragma unroll
                            for (int h = 0; h < G; ++h) rn[h] = ld(kb32 + e + h4 + G + h);
                        }
                        rec(r[0], w0.x, fx, fy, fz);
                        rec(r[1], w0.y, fx, fy, fz);
                        rec(r[2], w1.x, fx, fy, fz);
                        rec(r[3], w1.y, fx, fy, fz);
                        if (h4 + G < 64) {
#pragma unroll
                            for (int h = 0; h < G; ++h) r[h] = rn[h];
                        }
                    }
                } else {
                    for (int h = 0; h < cnt; ++h) rec(ld(kb32 + e + h), ph[h], fx, fy, fz);
                }
                Fx += fx; Fy += fy; Fz += fz;
            }
        }
        const double qi = -(double)qf[i];
        Fx *= qi; Fy *= qi; Fz *= qi;
    }
}

// The end of an evaluation for slot i (current order) given its far force:
// the zero-frequency mode term, the far force stored, the closing half kick
// (and the second Nose-Hoover scaling) when stepping, and the kinetic energy
// of each wave's particles summed across the wave in a fixed order into
// partial [item * 4 + wave] (k_kinetic adds them up).  FUSE: the next step
// starts here, as the kick/drift kernel would start it: its opening half kick
// with the same force, its drift, wrap and quantisation, and its
// displacement check.  Lanes past the item (valid false) hold slot i = t0 and
// store nothing.
template <bool FUSE>
__device__ __forceinline__ void far_finish(const EvalArgs &a, CSys *sp, int32_t sys, int64_t i, bool valid,
                                           double Fx, double Fy, double Fz, int32_t itx) {
    const int64_t n = a.N;
    // the velocity and the near force are loaded before the far force is
    // stored (the stores could alias them for the compiler), so that their
    // loads overlap the ones before
    double vv[3] = {a.cur.v[i], a.cur.v[n + i], a.cur.v[2 * n + i]};
    const double fn[3] = {a.Fn[i], a.Fn[n + i], a.Fn[2 * n + i]};
    double xs[3], L[3];
    float hf[3];
    uint32_t uref[3];
    if constexpr (FUSE) {
        for (int d = 0; d < 3; ++d) {
            xs[d] = a.cur.x[d * n + i];
            uref[d] = a.u[d * n + i];
            L[d] = sp->g.L[d];
            hf[d] = sp->g.hf[d];
        }
    }
    if (sp->zmode != 0) {
        const double qi = a.cur.q[i], c = sp->zf * qi;
        const double *M = a.dipole + 3 * sys;
        if (sp->zmode == 1) {
            Fx += c * M[0];
            Fy += c * M[1];
        }
        Fz += c * M[2];
    }
    if (valid) {
        a.Ff[i] = Fx;
        a.Ff[n + i] = Fy;
        a.Ff[2 * n + i] = Fz;
    }
    const double f[3] = {fn[0] + Fx, fn[1] + Fy, fn[2] + Fz};
    if (a.kick) {
        // closing half kick of the velocity-Verlet step
        bool bad = false;
        for (int d = 0; d < 3; ++d) {
            bad |= !isfinite(f[d]);
            vv[d] += a.hdm * f[d];
        }
        if (!FUSE && a.nh) {
            // Nose-Hoover: the second scaling with the step's half-step xi
            // (xi and the kinetic energy still hold the step's start)
            const double xh = a.nh_xi[sys] + 0.5 * a.dt * (2.0 * a.kin[sys] - sp->nh_nf * a.nh_T) / sp->nh_Q;
            const double sc = exp(-0.5 * a.dt * xh);
            for (int d = 0; d < 3; ++d) vv[d] *= sc;
        }
        if (!FUSE && valid)
            for (int d = 0; d < 3; ++d) a.cur.v[d * n + i] = vv[d];
        if (bad && valid) atomicOr(a.flag, 1);
    }
    double ke = valid ? 0.5 * a.mass * ((vv[0] * vv[0] + vv[1] * vv[1]) + vv[2] * vv[2]) : 0.0;
    // the wave's kinetic energy (a fixed butterfly), one partial per wave
    for (int o = 32; o > 0; o >>= 1) ke += __shfl_xor(ke, o, 64);
    if ((threadIdx.x & 63) == 0) a.kpart[(int64_t)itx * 4 + (threadIdx.x >> 6)] = ke;
    if constexpr (FUSE) {
        // the next step: half kick and drift, the drift kept for the
        // mean-square displacement, then wrap and quantise
        const double xs0[3] = {xs[0], xs[1], xs[2]};
        for (int d = 0; d < 3; ++d) {
            vv[d] += a.hdm * f[d];
            xs[d] += a.dt * vv[d];
            if (valid) a.cur.v[d * n + i] = vv[d];
        }
        if (valid && a.cur.dsp)
            for (int d = 0; d < 3; ++d) a.cur.dsp[d * n + i] += xs[d] - xs0[d];
        uint32_t uq[3];
        const float d2 = wrap_store(a, i, valid, xs, L, hf, uref, uq);
        // one atomic per wave that found a particle past the threshold
        const bool far_ = valid && !(d2 <= sp->g.dthr2_f);
        if (__ballot(far_) != 0ull && (threadIdx.x & 63) == 0) atomicOr(a.rebuild, 1);
    }
}

// Far force and the end of the evaluation, one particle per lane; items are
// runs of up to 256 slots of one system (grid-stride).  The near-list
// rebuild flag is cleared here (every kernel of the evaluation that reads it
// has run), unless the kernel opens the next step (FUSE), whose displacement
// check sets it: the list pass has cleared it then.
template <bool F64, bool FUSE>
__global__ __launch_bounds__(256) void k_far(EvalArgs a, const FarItem *__restrict__ items, int32_t nitems) {
    __shared__ double2 turn[F64 ? rmath::kTurnTab : 1];
    __shared__ uint64_t phs[F64 ? 1 : 4 * kFarStage];  // FP32C: record phases, per wave
    if constexpr (F64) fill_turns(turn);
    if (!FUSE && blockIdx.x == 0 && threadIdx.x == 0 && a.rebuild) *a.rebuild = 0;
    for (int32_t itx = blockIdx.x; itx < nitems; itx += gridDim.x) {
        const FarItem item = items[itx];
        const int32_t sys = rfl(item.sys);
        CSys *sp = (CSys *)(a.sys + sys);
        const int64_t t0 = rfl64(item.t0), t1 = rfl64(item.t1);
        const int64_t i0 = t0 + threadIdx.x;
        const bool valid = i0 < t1;
        const int64_t i = valid ? i0 : t0;
        double Fx, Fy, Fz;
        far_sum<F64>(sp, (CRec64 *)(a.kb64 + sp->k0), (CRec32 *)(a.kb32 + sp->k0), sp->P, a.N, i, a.u_tmp,
                     a.cur.qf, a.cur.x, a.cur.q, turn, phs + (F64 ? 0 : (threadIdx.x >> 6) * kFarStage), Fx, Fy, Fz);
        far_finish<FUSE>(a, sp, sys, i, valid, Fx, Fy, Fz, itx);
    }
}

// Build-every-step mode: the far force computed beside the re-sort and the
// near part, on the structure factor's stream, from the copy of the state
// that the kick/drift kernel wrote (its order: the slots before the re-sort),
// into Ff_side.
template <bool F64>
__global__ __launch_bounds__(256) void k_far_side(EvalArgs a, const FarItem *__restrict__ items, int32_t nitems) {
    __shared__ double2 turn[F64 ? rmath::kTurnTab : 1];
    __shared__ uint64_t phs[F64 ? 1 : 4 * kFarStage];  // FP32C: record phases, per wave
    if constexpr (F64) fill_turns(turn);
    const int64_t n = a.N;
    for (int32_t itx = blockIdx.x; itx < nitems; itx += gridDim.x) {
        const FarItem item = items[itx];
        CSys *sp = (CSys *)(a.sys + rfl(item.sys));
        const int64_t t0 = rfl64(item.t0), t1 = rfl64(item.t1);
        const int64_t i0 = t0 + threadIdx.x;
        const bool valid = i0 < t1;
        const int64_t i = valid ? i0 : t0;
        double Fx, Fy, Fz;
        far_sum<F64>(sp, (CRec64 *)(a.kb64 + sp->k0), (CRec32 *)(a.kb32 + sp->k0), sp->P, n, i, a.rs_u, a.rs_qf,
                     a.rs_x, a.rs_q, turn, phs + (F64 ? 0 : (threadIdx.x >> 6) * kFarStage), Fx, Fy, Fz);
        if (valid) {
            a.Ff_side[i] = Fx;
            a.Ff_side[n + i] = Fy;
            a.Ff_side[2 * n + i] = Fz;
        }
    }
}

// Build-every-step mode, after the near part: slot i of the new order takes
// the far force of its particle's slot before the re-sort (`sorted`, which
// the re-sort writes at every evaluation of this mode), then the end of the
// evaluation as in k_far.  Clears the rebuild flag.
__global__ __launch_bounds__(256) void k_far_finish(EvalArgs a, const FarItem *__restrict__ items, int32_t nitems) {
    const int64_t n = a.N;
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.rebuild) *a.rebuild = 0;
    for (int32_t itx = blockIdx.x; itx < nitems; itx += gridDim.x) {
        const FarItem item = items[itx];
        const int32_t sys = rfl(item.sys);
        CSys *sp = (CSys *)(a.sys + sys);
        const int64_t t0 = rfl64(item.t0), t1 = rfl64(item.t1);
        const int64_t i0 = t0 + threadIdx.x;
        const bool valid = i0 < t1;
        const int64_t i = valid ? i0 : t0;
        const int64_t o = a.sorted[i];
        const double Fx = a.Ff_side[o], Fy = a.Ff_side[n + o], Fz = a.Ff_side[2 * n + o];
        far_finish<false>(a, sp, sys, i, valid, Fx, Fy, Fz, itx);
    }
}

// Per system, gridDim.x blocks: each sums a contiguous share of the far
// items' wave partials of the kinetic energy and of the near items' energy
// partials of the mode in use (eight loads in flight per thread, a fixed
// tree across the block); with one block it finishes alone, else the last
// block of the system (per-system counter, re-armed) adds the blocks' sums in
// block order.  The finish: U_N and the total U = U_N + U* - U_self, the
// kinetic energy after the evaluation, and for a Nose-Hoover step xi's
// second half step with it.
__global__ __launch_bounds__(256) void k_kinetic(EvalArgs a) {
    __shared__ double kw[256], ew[256];
    const int32_t s = blockIdx.y, g = blockIdx.x, G = gridDim.x;
    const SysDev &sp = a.sys[s];
    // the block's share [lo, hi) of the partials [b0, b1)
    auto share = [&](int64_t b0, int64_t b1, int64_t &lo, int64_t &hi) {
        const int64_t per = (b1 - b0 + G - 1) / G;
        lo = b0 + (int64_t)g * per;
        hi = lo + per < b1 ? lo + per : b1;
        if (lo > hi) lo = hi;
    };
    auto sum8 = [&](const double *p, int64_t lo, int64_t hi) {
        double u8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int64_t i = lo + threadIdx.x;
        for (; i + 7 * 256 < hi; i += 8 * 256) {
#pragma unroll
            for (int h = 0; h < 8; ++h) u8[h] += p[i + h * 256];
        }
        for (; i < hi; i += 256) u8[0] += p[i];
        return ((u8[0] + u8[1]) + (u8[2] + u8[3])) + ((u8[4] + u8[5]) + (u8[6] + u8[7]));
    };
    int64_t lo, hi;
    share((int64_t)sp.ft0 * 4, (int64_t)sp.ft1 * 4, lo, hi);
    kw[threadIdx.x] = sum8(a.kpart, lo, hi);
    const double *ep = a.always_build ? a.epart_cells : a.epart;
    share(a.always_build ? sp.jt0 : sp.it0, a.always_build ? sp.jt1 : sp.it1, lo, hi);
    ew[threadIdx.x] = sum8(ep, lo, hi);
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            kw[threadIdx.x] += kw[threadIdx.x + o];
            ew[threadIdx.x] += ew[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double K = kw[0], un = ew[0];
    if (G > 1) {
        double *part = a.kin_part + (int64_t)s * 2 * G;
        part[2 * g] = K;
        part[2 * g + 1] = un;
        __threadfence();
        if (atomicAdd(&a.sys_done[s], 1u) != (uint32_t)G - 1u) return;
        __threadfence();
        K = 0.0;
        un = 0.0;
        for (int32_t b = 0; b < G; ++b) {
            K += part[2 * b];
            un += part[2 * b + 1];
        }
        a.sys_done[s] = 0u;
    }
    const double tot = un + a.E[4 * s + 1] - a.E[4 * s + 2];
    a.E[4 * s] = un;
    a.E[4 * s + 3] = tot;
    if (!isfinite(tot)) atomicOr(a.flag, 2);
    if (a.kick && a.nh) {
        const double nf = sp.nh_nf, Q = sp.nh_Q;
        const double xh = a.nh_xi[s] + 0.5 * a.dt * (2.0 * a.kin[s] - nf * a.nh_T) / Q;
        a.nh_xi[s] = xh + 0.5 * a.dt * (2.0 * K - nf * a.nh_T) / Q;
    }
    a.kin[s] = K;
}


// One block per system: sum of |dsp|^2 over its slots (strided, then a fixed
// tree), divided by n.
__global__ __launch_bounds__(256) void k_msd(EvalArgs a, double *__restrict__ msd) {
    __shared__ double w[256];
    const int32_t s = blockIdx.x;
    const SysDev &sp = a.sys[s];
    const int64_t n = a.N, p0 = sp.p0, p1 = sp.p0 + sp.g.n;
    double acc = 0.0;
    for (int64_t i = p0 + threadIdx.x; i < p1; i += 256) {
        const double dx = a.cur.dsp[i], dy = a.cur.dsp[n + i], dz = a.cur.dsp[2 * n + i];
        acc += (dx * dx + dy * dy) + dz * dz;
    }
    w[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) w[threadIdx.x] += w[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) msd[s] = w[0] / (double)sp.g.n;
}

}  // namespace

void launch_msd(const EvalArgs &a, double *msd, hipStream_t s) {
    hipLaunchKernelGGL(k_msd, dim3((unsigned)a.nsys), dim3(256), 0, s, a, msd);
}

void launch_rho(const EvalArgs &a, bool f64, const RhoItem *items, int32_t nitems, hipStream_t s) {
    dim3 grid((unsigned)nitems), block(1024);
    if (f64) hipLaunchKernelGGL(k_rho<true>, grid, block, 0, s, a, items, nitems);
    else hipLaunchKernelGGL(k_rho<false>, grid, block, 0, s, a, items, nitems);
}

void launch_rho_reduce(const EvalArgs &a, hipStream_t s) {
    if (a.K <= 0) return;
    if (a.red_waves == 4) hipLaunchKernelGGL(k_rho_reduce_block, dim3((unsigned)a.K), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_rho_reduce, dim3((unsigned)((a.K + 3) / 4)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_rho_finish, dim3((unsigned)a.nsys), dim3(256), 0, s, a);
}

void launch_far(const EvalArgs &a, bool f64, const FarItem *items, int32_t nitems, int32_t block_size,
                hipStream_t s) {
    dim3 grid((unsigned)nitems), block((unsigned)block_size);
    if (a.fuse) {
        if (f64) hipLaunchKernelGGL((k_far<true, true>), grid, block, 0, s, a, items, nitems);
        else hipLaunchKernelGGL((k_far<false, true>), grid, block, 0, s, a, items, nitems);
    } else {
        if (f64) hipLaunchKernelGGL((k_far<true, false>), grid, block, 0, s, a, items, nitems);
        else hipLaunchKernelGGL((k_far<false, false>), grid, block, 0, s, a, items, nitems);
    }
}

void launch_far_side(const EvalArgs &a, bool f64, const FarItem *items, int32_t nitems, int32_t block_size,
                     hipStream_t s) {
    dim3 grid((unsigned)nitems), block((unsigned)block_size);
    if (f64) hipLaunchKernelGGL(k_far_side<true>, grid, block, 0, s, a, items, nitems);
    else hipLaunchKernelGGL(k_far_side<false>, grid, block, 0, s, a, items, nitems);
}

void launch_far_finish(const EvalArgs &a, const FarItem *items, int32_t nitems, int32_t block_size, hipStream_t s) {
    hipLaunchKernelGGL(k_far_finish, dim3((unsigned)nitems), dim3((unsigned)block_size), 0, s, a, items, nitems);
}

void launch_kinetic(const EvalArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_kinetic, dim3((unsigned)a.kin_blocks, (unsigned)a.nsys), dim3(256), 0, s, a);
}

}  // namespace rbsog
