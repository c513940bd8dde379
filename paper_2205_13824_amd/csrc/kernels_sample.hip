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
#include "rbsog_math.h"

namespace rbsog {

namespace {

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
            double ua;
            const uint64_t t = base + threadIdx.x;
            at.nonzero = rmath::mh_propose(d.seed, stream, t, d.sd, at.m, ua) ? 1 : 0;
            at.p = at.nonzero ? rmath::target_weight(d.omega, d.s, d.G, d.L, at.m) : 0.0;
            at.q = at.nonzero ? rmath::proposal_1d(at.m[0], d.a[0]) * rmath::proposal_1d(at.m[1], d.a[1]) *
                                    rmath::proposal_1d(at.m[2], d.a[2])
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
                if (rmath::mh_accept(at.ua, at.p, at.q, ch.p, ch.qprop)) {
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
