// Arithmetic shared by the host side and the kernels of librbsog, written
// once: the Philox4x32-10 generator and the Box-Muller normals drawn from it,
// the Metropolis-Hastings target and proposal weights of the wave-vector
// sampler (Sec. 3.3), and the FP64 sin/cos of a revolution used by the
// structure-factor and far-force kernels.  Every function compiles for the
// host and the device from the same text, so the host chain and the device
// chains take the same steps; their results then agree wherever the host's
// and the device's libm (log, cos, sin, exp, erf, erfc) round alike.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rbsog {
namespace rmath {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// 4x32 multiply-xor round function with the published multipliers and the
// Weyl key increments.  c is the counter block, (k0, k1) the key.
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * c[0];
        const uint64_t b = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t y0 = (uint32_t)(b >> 32) ^ c[1] ^ k0;
        const uint32_t y1 = (uint32_t)b;
        const uint32_t y2 = (uint32_t)(a >> 32) ^ c[3] ^ k1;
        const uint32_t y3 = (uint32_t)a;
        c[0] = y0; c[1] = y1; c[2] = y2; c[3] = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Two 53-bit uniforms in [0, 1) from counter (index_lo, index_hi, stream,
// lane) and key (seed_lo, seed_hi): the top 53 bits of output words (1, 0)
// and (3, 2).
__host__ __device__ inline void uniform2(uint64_t seed, uint32_t stream, uint64_t index, uint32_t lane, double &a,
                                         double &b) {
    uint32_t c[4] = {(uint32_t)index, (uint32_t)(index >> 32), stream, lane};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    a = (double)(((((uint64_t)c[1]) << 32) | c[0]) >> 11) * 0x1.0p-53;
    b = (double)(((((uint64_t)c[3]) << 32) | c[2]) >> 11) * 0x1.0p-53;
}

// Three standard normals by Box-Muller from lanes 0 and 1 of counter
// (index, stream): (u1, u2), (u3, u4) -> (r1 cos 2 pi u2, r1 sin 2 pi u2,
// r2 cos 2 pi u4), r = sqrt(-2 ln(1 - u)).
__host__ __device__ inline void normals3(uint64_t seed, uint32_t stream, uint64_t index, double z[3]) {
    double u1, u2, u3, u4;
    uniform2(seed, stream, index, 0, u1, u2);
    uniform2(seed, stream, index, 1, u3, u4);
    const double r1 = sqrt(-2.0 * log(1.0 - u1));
    const double r2 = sqrt(-2.0 * log(1.0 - u3));
    z[0] = r1 * cos(kTwoPi * u2);
    z[1] = r1 * sin(kTwoPi * u2);
    z[2] = r2 * cos(kTwoPi * u4);
}

// Unnormalised target of the sampler, p(m) ~ F~(2 pi m / L) =
// pi^{3/2} sum_l omega_l s_l^3 exp(-pi^2 s_l^2 |m/L|^2) without the pi^{3/2}
// (Sec. 3.3, eq. "distribution"; G = M + 1 Gaussians).
__host__ __device__ inline double target_weight(const double *omega, const double *s, int G, const double L[3],
                                                const int32_t m[3]) {
    const double t = (double)m[0] * m[0] / (L[0] * L[0]) + (double)m[1] * m[1] / (L[1] * L[1]) +
                     (double)m[2] * m[2] / (L[2] * L[2]);
    double acc = 0.0;
    for (int l = 0; l < G; ++l) {
        const double sl = s[l];
        acc += omega[l] * sl * sl * sl * exp(-kPi * kPi * sl * sl * t);
    }
    return acc;
}

// Proposal pmf of one component (Sec. 3.3, the erf form with the argument
// (m +- 1/2) pi s_0 / L_d): (1/2)[erf((m+1/2) a) - erf((m-1/2) a)], written
// with erfc for m != 0 so that the tails keep their digits; a = pi s_0 / L_d.
__host__ __device__ inline double proposal_1d(int32_t m, double a) {
    if (m == 0) return erf(0.5 * a);
    const double am = fabs((double)m);
    return 0.5 * (erfc((am - 0.5) * a) - erfc((am + 0.5) * a));
}

// One Metropolis-Hastings proposal of the independence chain (Sec. 3.3):
// attempt t draws three normals (lanes 0, 1) and the acceptance uniform
// (lane 2) of counter (t, stream); m*_d = round(z_d sd_d), round half away
// from zero, sd_d = L_d / (sqrt(2) pi s_0).  Returns whether m* is nonzero.
__host__ __device__ inline bool mh_propose(uint64_t seed, uint32_t stream, uint64_t attempt, const double sd[3],
                                           int32_t cand[3], double &ua) {
    double z[3], ub;
    normals3(seed, stream, attempt, z);
    uniform2(seed, stream, attempt, 2, ua, ub);
    for (int d = 0; d < 3; ++d) cand[d] = (int32_t)round(z[d] * sd[d]);
    return (cand[0] | cand[1] | cand[2]) != 0;
}

// Metropolis-Hastings acceptance of candidate (pc, qc) from state (p, q):
// accepted iff ua < (pc q) / (p qc).
__host__ __device__ inline bool mh_accept(double ua, double pc, double qc, double p, double q) {
    return ua < (pc * q) / (p * qc);
}

// The revolution of a 32-bit fixed-point phase t (the fraction t / 2^32 of a
// turn) as an FP32 value for the hardware sin/cos, which take revolutions:
// 1.0's exponent with the top 23 bits of t as the mantissa, 1 + t / 2^32 in
// [1, 2) up to the 9 low bits of t (one funnel shift).  sin and cos of a whole
// turn plus the fraction are those of the fraction.  The truncation offsets
// every phase by half a unit of 2^-23 turns on average and by at most 2^-23
// turns: the common part cancels between the structure factor and the far
// force, which multiply e^{i theta_j} by e^{-i theta_i}.
__device__ __forceinline__ float phase_rev(uint32_t t) {
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, t, 9u));
}

// Fixed-point phase m.u mod 2^32 of three products as a chain of
// v_mad_u64_u32 (a full-rate instruction on gfx950): the first product takes
// the inline constant 0 as its addend and each later one adds the previous
// 64-bit result, whose low half is the running sum mod 2^32 (the high half
// never reaches the low one).  Three instructions where separate products
// and a sum take four.  `s` forms take the first factor from a scalar
// register (wave-uniform wave vectors), `v` forms from a vector register.
// The carry output of the instruction is not used.
__device__ __forceinline__ uint32_t dot3_mod32_v(uint32_t ax, uint32_t ay, uint32_t az, uint32_t bx, uint32_t by,
                                                 uint32_t bz) {
    uint64_t p, q, r, c0, c1, c2;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(p), "=s"(c0) : "v"(az), "v"(bz));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(q), "=s"(c1) : "v"(ay), "v"(by), "v"(p));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(c2) : "v"(ax), "v"(bx), "v"(q));
    return (uint32_t)r;
}
__device__ __forceinline__ uint32_t dot3_mod32_s(uint32_t ax, uint32_t ay, uint32_t az, uint32_t bx, uint32_t by,
                                                 uint32_t bz) {
    uint64_t p, q, r, c0, c1, c2;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(p), "=s"(c0) : "s"(az), "v"(bz));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(q), "=s"(c1) : "s"(ay), "v"(by), "v"(p));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(c2) : "s"(ax), "v"(bx), "v"(q));
    return (uint32_t)r;
}
// c + a.b mod 2^32 for c the low half of the 64-bit addend `c` (its high half
// is not read into the low half of any product): the same chain with c in
// place of the constant 0, so a phase offset costs no instruction.  The
// first factor from scalar registers, the addend from vector registers (one
// scalar operand per instruction).
__device__ __forceinline__ uint32_t dot3_add_mod32_s(uint32_t ax, uint32_t ay, uint32_t az, uint32_t bx, uint32_t by,
                                                     uint32_t bz, uint64_t c) {
    uint64_t p, q, r, c0, c1, c2;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(p), "=s"(c0) : "s"(az), "v"(bz), "v"(c));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(q), "=s"(c1) : "s"(ay), "v"(by), "v"(p));
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(c2) : "s"(ax), "v"(bx), "v"(q));
    return (uint32_t)r;
}

// e^y in FP64 for finite y <= 0 (the narrow Gaussians of the near part),
// by Cody and Waite's reduction: n = rint(y / ln 2), r = y - n ln 2 with
// ln 2 in two parts (|r| <= ln 2 / 2), the Taylor series of e^r through
// degree 11 (truncation below 1e-23 relative), scaled by 2^n.  No overflow
// case (y <= 0); large negative y scale to 0.
__device__ __forceinline__ double exp_nonpos(double y) {
    constexpr double kLog2e = 1.4426950408889634;
    constexpr double kLn2Hi = 0.6931471805599453;       // ln 2 rounded to FP64
    constexpr double kLn2Lo = 2.3190468138462996e-17;   // ln 2 - kLn2Hi
    const double nd = rint(y * kLog2e);
    double r = fma(nd, -kLn2Hi, y);
    r = fma(nd, -kLn2Lo, r);
    double p = 1.0 / 39916800.0;  // 1/11!
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    // 2^n with n clamped (below -1100 the result is 0 either way)
    const int n = (int)fmax(nd, -1100.0);
    return ldexp(p, n);
}

// sin(2 pi t), cos(2 pi t) in FP64, from u = kTurnTab t (t in turns, u of
// moderate size), through a table of the kTurnTab turns 2 pi j / kTurnTab
// (tab[j] = (cos, sin), filled with sincos2pi below): j = rint(u), r = u - j
// (exact, |r| <= 1/2), x = 2 pi r / kTurnTab (|x| <= pi / kTurnTab), the
// Taylor series of sin x through degree 5 and of cos x through degree 4
// (truncation below x^7/5040 < 6e-22 and x^6/720 < 1.2e-18 at |x| <= pi/1024,
// well under an FP64 ulp of sin x and cos x), then the angle sum with entry
// j mod kTurnTab.  Callers scale their positions by kTurnTab (a power of 2,
// so u is exactly kTurnTab times the phase they would form in turns).
constexpr int kTurnTab = 1024;
__device__ __forceinline__ void sincos2pi_tab(double u, const double2 *tab, double *s, double *c) {
    constexpr double T = kTwoPi / kTurnTab;
    constexpr double T2 = T * T;
    constexpr double S1 = -T * T2 / 6.0;
    constexpr double S2 = -S1 * T2 / 20.0;
    constexpr double C1 = -T2 / 2.0;
    constexpr double C2 = -C1 * T2 / 12.0;
    const double jd = rint(u);
    const double r = u - jd;
    const double2 e = tab[(int)jd & (kTurnTab - 1)];
    const double z = r * r;
    const double sr = r * fma(z, fma(z, S2, S1), T);
    const double cr = fma(z, fma(z, C2, C1), 1.0);
    *s = fma(e.y, cr, e.x * sr);
    *c = fma(e.x, cr, -(e.y * sr));
}

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

}  // namespace rmath
}  // namespace rbsog
