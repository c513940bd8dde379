// On-device wave-vector sampler for gfx950: lambda independent
// Metropolis-Hastings independence chains per system (Sec. 3.3; the parallel
// sampling of Sec. 3.4, where lambda processes sample in parallel and each
// serves one step of a lambda-step cycle).  Chain c draws its random numbers
// from Philox4x32-10 stream 3 + c with the system's key, exactly as the host
// chain (stream 0) does: proposal m*_d = round(N(0, (L_d/(pi s_0))^2/2)), zero
// redrawn, acceptance min(1, p(m*) q(m) / (p(m) q(m*))), the first nonzero
// proposal starting the chain and 100 transitions discarded.  One launch
// advances every chain by P states: chain c's states form batch c of the
// next lambda evaluations.
#include "rbsog_internal.h"

namespace rbsog {

namespace {

constexpr double kPiS = 3.14159265358979323846;

__device__ __forceinline__ void philox_u2(uint64_t seed, uint32_t stream, uint64_t index, uint32_t lane, double &a,
                                          double &b) {
    uint32_t c0 = (uint32_t)index, c1 = (uint32_t)(index >> 32), c2 = stream, c3 = lane;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t y1 = (uint32_t)p1;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        const uint32_t y3 = (uint32_t)p0;
        c0 = y0; c1 = y1; c2 = y2; c3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    a = (double)((((uint64_t)c1 << 32) | c0) >> 11) * 0x1.0p-53;
    b = (double)((((uint64_t)c3 << 32) | c2) >> 11) * 0x1.0p-53;
}

// p(m) ~ F~(2 pi m / L) up to constants: sum_l omega_l s_l^3 e^{-pi^2 s_l^2 |m/L|^2}
__device__ double target_weight(const SampDev &d, const int32_t m[3]) {
    const double t = (double)m[0] * m[0] / (d.L[0] * d.L[0]) + (double)m[1] * m[1] / (d.L[1] * d.L[1]) +
                     (double)m[2] * m[2] / (d.L[2] * d.L[2]);
    double acc = 0.0;
    for (int l = 0; l < d.G; ++l) {
        const double s = d.s[l];
        acc += d.omega[l] * s * s * s * exp(-kPiS * kPiS * s * s * t);
    }
    return acc;
}

// proposal pmf of one component: (1/2)[erf((m+1/2) a) - erf((m-1/2) a)], a = pi s_0 / L
__device__ double proposal_1d(int32_t m, double a) {
    if (m == 0) return erf(0.5 * a);
    const double am = fabs((double)m);
    return 0.5 * (erfc((am - 0.5) * a) - erfc((am + 0.5) * a));
}

// One block per (system, chain).  The proposals of an independence sampler do
// not depend on the chain's state: the block first evaluates a window of
// kWin consecutive attempts in parallel (one per thread: Philox draws,
// Box-Muller, candidate, p and q), then one thread runs the accept/reject
// recursion over the window in attempt order, which needs one comparison per
// attempt.  The result is the serial chain's, attempt for attempt.
constexpr int kWin = 256;

struct Attempt {
    int32_t m[3];
    int32_t nonzero;
    double p, q, ua;
};

__global__ __launch_bounds__(kWin) void k_refill(const SampDev *__restrict__ samp, int32_t lambda,
                                                 ChainState *__restrict__ chains, int64_t *__restrict__ kcur,
                                                 int32_t *__restrict__ flag) {
    __shared__ Attempt win[kWin];
    __shared__ ChainState ch;
    __shared__ int32_t made_s, stop_s;
    const int64_t gid = blockIdx.x;
    const int32_t s = (int32_t)(gid / lambda), cidx = (int32_t)(gid % lambda);
    const SampDev &d = samp[s];
    const uint32_t stream = 3u + (uint32_t)cidx;
    int32_t *out = d.out + 3 * (int64_t)cidx * d.P;
    if (threadIdx.x == 0) {
        ch = chains[gid];
        made_s = 0;
        stop_s = 0;
    }
    __syncthreads();
    // a chain whose proposals are almost always m* = 0 (a box far smaller than
    // s_0) would not finish: stop after a bounded number of attempts and flag it
    const uint64_t limit = ch.attempt + 1000ull * (uint64_t)(d.P + 101);
    while (true) {
        const uint64_t base = ch.attempt;
        {
            Attempt at;
            double u1, u2, u3, u4, ua, ub;
            const uint64_t t = base + threadIdx.x;
            philox_u2(d.seed, stream, t, 0, u1, u2);
            philox_u2(d.seed, stream, t, 1, u3, u4);
            philox_u2(d.seed, stream, t, 2, ua, ub);
            const double r1 = sqrt(-2.0 * log(1.0 - u1));
            const double r2 = sqrt(-2.0 * log(1.0 - u3));
            const double z[3] = {r1 * cos(2.0 * kPiS * u2), r1 * sin(2.0 * kPiS * u2), r2 * cos(2.0 * kPiS * u4)};
            for (int k = 0; k < 3; ++k) at.m[k] = (int32_t)round(z[k] * d.sd[k]);
            at.nonzero = (at.m[0] | at.m[1] | at.m[2]) != 0;
            at.p = at.nonzero ? target_weight(d, at.m) : 0.0;
            at.q = at.nonzero ? proposal_1d(at.m[0], d.a[0]) * proposal_1d(at.m[1], d.a[1]) *
                                    proposal_1d(at.m[2], d.a[2])
                              : 0.0;
            at.ua = ua;
            win[threadIdx.x] = at;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t made = made_s;
            int i = 0;
            for (; i < kWin && made < d.P; ++i) {
                const Attempt &at = win[i];
                if (!at.nonzero) continue;
                if (!ch.started) {
                    for (int k = 0; k < 3; ++k) ch.m[k] = at.m[k];
                    ch.p = at.p;
                    ch.qprop = at.q;
                    ch.started = 1;
                    continue;
                }
                if (at.ua < (at.p * ch.qprop) / (ch.p * at.q)) {
                    for (int k = 0; k < 3; ++k) ch.m[k] = at.m[k];
                    ch.p = at.p;
                    ch.qprop = at.q;
                }
                if (ch.burn_left > 0) {
                    --ch.burn_left;
                    continue;
                }
                out[3 * made] = ch.m[0];
                out[3 * made + 1] = ch.m[1];
                out[3 * made + 2] = ch.m[2];
                ++made;
            }
            ch.attempt = base + i;
            made_s = made;
            if (made >= d.P) stop_s = 1;
            else if (ch.attempt >= limit) {
                atomicOr(flag, 4);
                stop_s = 1;
            }
        }
        __syncthreads();
        if (stop_s) break;
    }
    if (threadIdx.x == 0) {
        chains[gid] = ch;
        if (cidx == 0) kcur[s] = 0;
    }
}

}  // namespace

void launch_refill(const SampDev *samp, int32_t nsys, int32_t lambda, ChainState *chains, int64_t *kcur,
                   int32_t *flag, hipStream_t s) {
    const int64_t nb = (int64_t)nsys * lambda;
    hipLaunchKernelGGL(k_refill, dim3((unsigned)nb), dim3(kWin), 0, s, samp, lambda, chains, kcur, flag);
}

}  // namespace rbsog
