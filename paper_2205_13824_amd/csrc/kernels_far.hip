// Fourier part of the random batch sum-of-Gaussians method for gfx950
// (Sec. 3.1 eq. "fourtrans"; Sec. 3.3 eq. "approximateForce"):
//   rho(k_e) = sum_j q_j e^{i k_e.r_j}
//   F*_i     = -q_i sum_e w_e k_e (Im rho_e cos th_ie - Re rho_e sin th_ie),  th_ie = k_e.r_i
//   U*       = 1/2 sum_e w_e |rho_e|^2
// Phases are taken in revolutions of the fractional coordinate, th/(2 pi) =
// m.s with s = x/L: FP64 forms evaluate f = m.s - rint(m.s) and a polynomial
// sin/cos of 2 pi f; FP32 forms take m.u mod 2^32 exactly on the 32-bit
// fixed-point coordinate and the hardware sin/cos of the revolution.
//
// Work split: the structure factor puts one wave vector on each lane and
// streams particles uniformly through the wave (no cross-lane reduction in
// the inner loop); the force puts one particle on each lane and streams the
// P wave-vector records uniformly.  Partial sums of rho are reduced in a
// fixed order, so the result is identical from run to run.
#include "rbsog_internal.h"

namespace rbsog {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// sin(2 pi f), cos(2 pi f) for |f| <= 1/2 in FP64: quadrant q = rint(4f),
// r = f - q/4 in [-1/8, 1/8], Taylor series of sin/cos(2 pi r) through
// degree 15/16 (truncation below 5e-17), then rotation by q quarter turns.
__device__ __forceinline__ void sincos2pi(double f, double *s, double *c) {
    constexpr double T = kTwoPi;
    constexpr double T2 = T * T;
    constexpr double S0 = T;
    constexpr double S1 = -S0 * T2 / 6.0;
    constexpr double S2 = -S1 * T2 / 20.0;
    constexpr double S3 = -S2 * T2 / 42.0;
    constexpr double S4 = -S3 * T2 / 72.0;
    constexpr double S5 = -S4 * T2 / 110.0;
    constexpr double S6 = -S5 * T2 / 156.0;
    constexpr double S7 = -S6 * T2 / 210.0;
    constexpr double C1 = -T2 / 2.0;
    constexpr double C2 = -C1 * T2 / 12.0;
    constexpr double C3 = -C2 * T2 / 30.0;
    constexpr double C4 = -C3 * T2 / 56.0;
    constexpr double C5 = -C4 * T2 / 90.0;
    constexpr double C6 = -C5 * T2 / 132.0;
    constexpr double C7 = -C6 * T2 / 182.0;
    constexpr double C8 = -C7 * T2 / 240.0;
    const double qd = rint(4.0 * f);
    const double r = fma(-0.25, qd, f);
    const double z = r * r;
    double ps = fma(z, S7, S6);
    ps = fma(z, ps, S5);
    ps = fma(z, ps, S4);
    ps = fma(z, ps, S3);
    ps = fma(z, ps, S2);
    ps = fma(z, ps, S1);
    ps = fma(z, ps, S0);
    const double sr = r * ps;
    double pc = fma(z, C8, C7);
    pc = fma(z, pc, C6);
    pc = fma(z, pc, C5);
    pc = fma(z, pc, C4);
    pc = fma(z, pc, C3);
    pc = fma(z, pc, C2);
    pc = fma(z, pc, C1);
    const double cr = fma(z, pc, 1.0);
    const int q = ((int)qd) & 3;
    const double a = (q & 1) ? cr : sr;
    const double b = (q & 1) ? sr : cr;
    *s = (q & 2) ? -a : a;
    *c = ((q + 1) & 2) ? -b : b;
}

// Structure factor partial sums.  Block (bx, by): particles
// [bx*chunk, (bx+1)*chunk), wave vectors [by*kt*64, (by+1)*kt*64).
// Wave w handles k tile (w % kt) for particle stream (w / kt).
template <bool F64>
__global__ __launch_bounds__(1024) void k_rho(Geom g, int32_t P, int kt, int streams, int64_t chunk,
                                              const double *__restrict__ x, const uint32_t *__restrict__ u,
                                              const double *__restrict__ q, const float *__restrict__ qf,
                                              const KRec64 *__restrict__ kb64, const KRec32 *__restrict__ kb32,
                                              double *__restrict__ partial) {
    __shared__ double2 red[1024];
    const int64_t n = g.n;
    // the wave index is uniform: readfirstlane lets the particle loads below
    // be scalar loads shared by the whole wave
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int kti = wave % kt, st = wave / kt;
    const int32_t k = ((int32_t)blockIdx.y * kt + kti) * 64 + lane;
    const bool active = k < P;
    const int32_t kk = active ? k : 0;
    const int64_t j0 = (int64_t)blockIdx.x * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    const int64_t per = (chunk + streams - 1) / streams;
    const int64_t a = j0 + st * per;
    const int64_t b = a + per < j1 ? a + per : j1;
    double re = 0.0, im = 0.0;
    // particles are consumed in groups of G so that the uniform loads of a
    // group are issued together and their latency is paid once per group
    constexpr int G = 8;
    if constexpr (F64) {
        const double mx = kb64[kk].mx, my = kb64[kk].my, mz = kb64[kk].mz;
        const double ix = g.invL[0], iy = g.invL[1], iz = g.invL[2];
        int64_t j = a;
        for (; j + G <= b; j += G) {
            double px[G], py[G], pz[G], pq[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                px[k] = x[j + k]; py[k] = x[n + j + k]; pz[k] = x[2 * n + j + k]; pq[k] = q[j + k];
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const double t = mx * (px[k] * ix) + my * (py[k] * iy) + mz * (pz[k] * iz);
                double sn, cs;
                sincos2pi(t - rint(t), &sn, &cs);
                re = fma(pq[k], cs, re);
                im = fma(pq[k], sn, im);
            }
        }
        for (; j < b; ++j) {
            const double t = mx * (x[j] * ix) + my * (x[n + j] * iy) + mz * (x[2 * n + j] * iz);
            double sn, cs;
            sincos2pi(t - rint(t), &sn, &cs);
            re = fma(q[j], cs, re);
            im = fma(q[j], sn, im);
        }
    } else {
        const uint32_t mx = (uint32_t)kb32[kk].mx, my = (uint32_t)kb32[kk].my, mz = (uint32_t)kb32[kk].mz;
        int64_t j = a;
        // FP32 partial sums over 32 particles, then accumulated in FP64
        for (; j + 4 * G <= b; j += 4 * G) {
            float rf = 0.f, fi = 0.f;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                uint32_t px[G], py[G], pz[G];
                float pq[G];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const int64_t jj = j + h * G + k;
                    px[k] = u[jj]; py[k] = u[n + jj]; pz[k] = u[2 * n + jj]; pq[k] = qf[jj];
                }
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const uint32_t t = mx * px[k] + my * py[k] + mz * pz[k];
                    const float f = (float)(int32_t)t * 0x1.0p-32f;
                    rf = fmaf(pq[k], __builtin_amdgcn_cosf(f), rf);
                    fi = fmaf(pq[k], __builtin_amdgcn_sinf(f), fi);
                }
            }
            re += rf;
            im += fi;
        }
        float rf = 0.f, fi = 0.f;
        for (; j < b; ++j) {
            const uint32_t t = mx * u[j] + my * u[n + j] + mz * u[2 * n + j];
            const float f = (float)(int32_t)t * 0x1.0p-32f;
            rf = fmaf(qf[j], __builtin_amdgcn_cosf(f), rf);
            fi = fmaf(qf[j], __builtin_amdgcn_sinf(f), fi);
        }
        re += rf;
        im += fi;
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
        partial[2 * ((int64_t)blockIdx.x * P + k)] = sr;
        partial[2 * ((int64_t)blockIdx.x * P + k) + 1] = si;
    }
}

// rho_e = sum over particle blocks of the partials (fixed order), the
// per-k energy 1/2 w_e |rho_e|^2, and rho written into the k records.  The
// last block to finish (counter) sums the energies in a fixed order:
// U_N from the near kernel's block partials, U*, U_self, U; and re-arms the
// counter for the next launch.
__global__ __launch_bounds__(256) void k_rho_reduce(int32_t P, int64_t nblk, const double *__restrict__ partial,
                                                    const double *__restrict__ wk, KRec64 *__restrict__ kb64,
                                                    KRec32 *__restrict__ kb32, double *__restrict__ rho,
                                                    double *__restrict__ ek, int64_t nnear,
                                                    const double *__restrict__ epart, double uself,
                                                    double *__restrict__ E, int32_t *__restrict__ flag,
                                                    uint32_t *__restrict__ counter) {
    __shared__ double sr[256], si[256];
    __shared__ bool last;
    const int32_t k = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t c = threadIdx.x; c < nblk; c += 256) {
        a += partial[2 * (c * P + k)];
        b += partial[2 * (c * P + k) + 1];
    }
    sr[threadIdx.x] = a;
    si[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            si[threadIdx.x] += si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double re = sr[0], im = si[0];
        rho[k] = re;
        rho[P + k] = im;
        kb64[k].re = re;
        kb64[k].im = im;
        kb32[k].re = (float)re;
        kb32[k].im = (float)im;
        ek[k] = 0.5 * wk[k] * (re * re + im * im);
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double un = 0.0, us = 0.0;
    for (int64_t i = threadIdx.x; i < nnear; i += 256) un += epart[i];
    for (int64_t i = threadIdx.x; i < P; i += 256) us += ek[i];
    sr[threadIdx.x] = un;
    si[threadIdx.x] = us;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            sr[threadIdx.x] += sr[threadIdx.x + o];
            si[threadIdx.x] += si[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double tot = sr[0] + si[0] - uself;
        E[0] = sr[0];
        E[1] = si[0];
        E[2] = uself;
        E[3] = tot;
        if (!isfinite(tot)) atomicOr(flag, 2);
        *counter = 0u;
    }
}

// Far force, one particle per lane, the P records streamed uniformly.
template <bool F64>
__global__ __launch_bounds__(256) void k_far(Geom g, int32_t P, const double *__restrict__ x,
                                             const uint32_t *__restrict__ u, const double *__restrict__ q,
                                             const float *__restrict__ qf, const KRec64 *__restrict__ kb64,
                                             const KRec32 *__restrict__ kb32, double *__restrict__ Ff, KickArgs kick) {
    const int64_t n = g.n;
    const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = i0 < n;
    const int64_t i = valid ? i0 : 0;
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    // records are consumed in groups so that their uniform loads overlap
    if constexpr (F64) {
        const double sx = x[i] * g.invL[0], sy = x[n + i] * g.invL[1], sz = x[2 * n + i] * g.invL[2];
        constexpr int G = 2;
        int32_t e = 0;
        for (; e + G <= P; e += G) {
            KRec64 r[G];
#pragma unroll
            for (int k = 0; k < G; ++k) r[k] = kb64[e + k];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const double t = r[k].mx * sx + r[k].my * sy + r[k].mz * sz;
                double sn, cs;
                sincos2pi(t - rint(t), &sn, &cs);
                const double v = cs * r[k].im - sn * r[k].re;
                Fx = fma(r[k].ckx, v, Fx);
                Fy = fma(r[k].cky, v, Fy);
                Fz = fma(r[k].ckz, v, Fz);
            }
        }
        for (; e < P; ++e) {
            const KRec64 r = kb64[e];
            const double t = r.mx * sx + r.my * sy + r.mz * sz;
            double sn, cs;
            sincos2pi(t - rint(t), &sn, &cs);
            const double v = cs * r.im - sn * r.re;
            Fx = fma(r.ckx, v, Fx);
            Fy = fma(r.cky, v, Fy);
            Fz = fma(r.ckz, v, Fz);
        }
        const double qi = q[i];
        Fx *= -qi; Fy *= -qi; Fz *= -qi;
    } else {
        const uint32_t ux = u[i], uy = u[n + i], uz = u[2 * n + i];
        constexpr int G = 4;
        int32_t e = 0;
        // FP32 partial sums over 64 records, then accumulated in FP64
        for (; e + 16 * G <= P; e += 16 * G) {
            float fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll
            for (int h = 0; h < 16; ++h) {
                KRec32 r[G];
#pragma unroll
                for (int k = 0; k < G; ++k) r[k] = kb32[e + h * G + k];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const uint32_t t = (uint32_t)r[k].mx * ux + (uint32_t)r[k].my * uy + (uint32_t)r[k].mz * uz;
                    const float f = (float)(int32_t)t * 0x1.0p-32f;
                    const float v = __builtin_amdgcn_cosf(f) * r[k].im - __builtin_amdgcn_sinf(f) * r[k].re;
                    fx = fmaf(r[k].ckx, v, fx);
                    fy = fmaf(r[k].cky, v, fy);
                    fz = fmaf(r[k].ckz, v, fz);
                }
            }
            Fx += fx; Fy += fy; Fz += fz;
        }
        float fx = 0.f, fy = 0.f, fz = 0.f;
        for (; e < P; ++e) {
            const KRec32 r = kb32[e];
            const uint32_t t = (uint32_t)r.mx * ux + (uint32_t)r.my * uy + (uint32_t)r.mz * uz;
            const float f = (float)(int32_t)t * 0x1.0p-32f;
            const float v = __builtin_amdgcn_cosf(f) * r.im - __builtin_amdgcn_sinf(f) * r.re;
            fx = fmaf(r.ckx, v, fx);
            fy = fmaf(r.cky, v, fy);
            fz = fmaf(r.ckz, v, fz);
        }
        const double qi = -(double)qf[i];
        Fx = qi * (Fx + fx); Fy = qi * (Fy + fy); Fz = qi * (Fz + fz);
    }
    if (valid) {
        Ff[i] = Fx;
        Ff[n + i] = Fy;
        Ff[2 * n + i] = Fz;
        if (kick.on) {
            // closing half kick of the velocity-Verlet step
            const double f[3] = {kick.Fn[i] + Fx, kick.Fn[n + i] + Fy, kick.Fn[2 * n + i] + Fz};
            bool bad = false;
            for (int d = 0; d < 3; ++d) {
                bad |= !isfinite(f[d]);
                kick.v[d * n + i] += kick.hdm * f[d];
            }
            if (bad) atomicOr(kick.flag, 1);
        }
    }
}

}  // namespace

FarPlan far_plan(int64_t n, int32_t P) {
    FarPlan p;
    const int64_t ktiles = (P + 63) / 64;
    p.kt = (int)(ktiles < 16 ? ktiles : 16);
    p.kblk = (ktiles + p.kt - 1) / p.kt;
    p.streams = 16 / p.kt;
    if (p.streams < 1) p.streams = 1;
    // aim for ~2 blocks of 16 waves per CU over 256 CUs
    const int64_t want_blocks = 512 / (p.kblk > 0 ? p.kblk : 1);
    int64_t chunk = (n + want_blocks - 1) / (want_blocks > 0 ? want_blocks : 1);
    const int64_t min_chunk = 64 * p.streams;
    if (chunk < min_chunk) chunk = min_chunk;
    p.chunk = chunk;
    p.nblk = (n + chunk - 1) / chunk;
    return p;
}

void launch_rho(const Geom &g, const FarPlan &fp, int32_t P, bool f64, const double *x, const uint32_t *u,
                const double *q, const float *qf, const KRec64 *kb64, const KRec32 *kb32, double *partial,
                hipStream_t s) {
    dim3 grid((unsigned)fp.nblk, (unsigned)fp.kblk), block(64 * fp.kt * fp.streams);
    if (f64)
        hipLaunchKernelGGL(k_rho<true>, grid, block, 0, s, g, P, fp.kt, fp.streams, fp.chunk, x, u, q, qf, kb64,
                           kb32, partial);
    else
        hipLaunchKernelGGL(k_rho<false>, grid, block, 0, s, g, P, fp.kt, fp.streams, fp.chunk, x, u, q, qf, kb64,
                           kb32, partial);
}

void launch_rho_reduce(int32_t P, int64_t nblk, const double *partial, const double *wk, KRec64 *kb64,
                       KRec32 *kb32, double *rho, double *ek, int64_t nnear, const double *epart, double uself,
                       double *E, int32_t *flag, uint32_t *counter, hipStream_t s) {
    hipLaunchKernelGGL(k_rho_reduce, dim3((unsigned)P), dim3(256), 0, s, P, nblk, partial, wk, kb64, kb32, rho, ek,
                       nnear, epart, uself, E, flag, counter);
}

void launch_far(const Geom &g, int32_t P, bool f64, const double *x, const uint32_t *u, const double *q,
                const float *qf, const KRec64 *kb64, const KRec32 *kb32, double *Ff, const KickArgs &kick,
                hipStream_t s) {
    dim3 grid(grid_for(g.n, 256)), block(256);
    if (f64)
        hipLaunchKernelGGL(k_far<true>, grid, block, 0, s, g, P, x, u, q, qf, kb64, kb32, Ff, kick);
    else
        hipLaunchKernelGGL(k_far<false>, grid, block, 0, s, g, P, x, u, q, qf, kb64, kb32, Ff, kick);
}

}  // namespace rbsog
