// Stateless structure factor of one set of point charges for gfx950
// (Sec. 3.1: rho(k) = sum_j q_j e^{i k.r_j}, k = 2 pi (m_x/L_x, m_y/L_y,
// m_z/L_z); Sec. 3.4: the one reduction of the random-batch method, which a
// spatially sharded run computes per device and then sums across devices).
// Device inputs and outputs, no context: rbsog_structure_factor takes its
// partial sums in memory it allocates per call (stream ordered), and
// rbsog_structure_factor_noalloc takes them in the file-scope array `scratch`
// below, for callers that cannot allocate (graph capture, serving loops).
// Both run the same kernels with the same chunk plan, so their results are
// bitwise identical.
//
// Work split: a block owns a chunk of particles and a tile of 256 wave
// vectors (one per thread).  It stages 256 particles at a time in LDS
// (wrapped and quantised once: 32-bit fixed-point fractional coordinates and
// an FP32 charge in FP32C, FP64 fractional coordinates and charge in FP64);
// every thread then reads the same staged particle (an LDS broadcast) and
// accumulates its wave vector's sum.  Each (chunk, k) partial is written once
// and a second kernel adds the chunks of every k in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "rbsog_internal.h"
#include "rbsog_math.h"

namespace rbsog {

rbsog_status fail_noctx(rbsog_status st, const char *fmt, ...);

namespace {

constexpr int kSfBlock = 256;         // threads per block = wave vectors per k tile = particles per LDS batch
constexpr int64_t kSfMaxChunks = 4096;
// Partial sums held by the no-allocation entry point: 2^20 complex FP64
// values (16 MiB per device, held until the process ends).  A call needs
// n_chunks x n_k of them; n_chunks shrinks to fit, so n_k <= 2^20.
constexpr int64_t kScratchComplex = int64_t(1) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double2 scratch[kScratchComplex];

// Chunks of particles: about one per 1024 particles (at least 256
// particles each), no more than the partial buffer holds for n_k vectors.
int64_t sf_chunks(int64_t n, int64_t nk) {
    int64_t want = (n + 1023) / 1024;
    want = want < 1 ? 1 : (want > kSfMaxChunks ? kSfMaxChunks : want);
    int64_t fit = kScratchComplex / nk;
    if (fit < 1) fit = 1;
    return want < fit ? want : fit;
}

struct SfStage64 {
    double sx, sy, sz, q;
};

// Partial structure factor of chunk c = blockIdx.x (particles [c chunk,
// (c+1) chunk)) for wave vector k = blockIdx.y * 256 + threadIdx.x.
template <bool F64>
__global__ __launch_bounds__(kSfBlock) void k_sf_partial(int64_t n, const double *__restrict__ x,
                                                         const double *__restrict__ q, double Lx, double Ly,
                                                         double Lz, int64_t nk, const int32_t *__restrict__ m,
                                                         int64_t chunk, int64_t nchunk, double2 *__restrict__ partial) {
    constexpr double kTwo32 = 4294967296.0;
    __shared__ uint4 st32[F64 ? 1 : kSfBlock];
    __shared__ SfStage64 st64[F64 ? kSfBlock : 1];
    const int64_t c = blockIdx.x;
    const int64_t k = (int64_t)blockIdx.y * kSfBlock + threadIdx.x;
    const bool kv = k < nk;
    const int32_t mx = kv ? m[3 * k] : 0, my = kv ? m[3 * k + 1] : 0, mz = kv ? m[3 * k + 2] : 0;
    const int64_t j0 = c * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    const double L[3] = {Lx, Ly, Lz};
    double re = 0.0, im = 0.0;
    for (int64_t jb = j0; jb < j1; jb += kSfBlock) {
        const int cnt = (int)(j1 - jb < kSfBlock ? j1 - jb : kSfBlock);
        if ((int)threadIdx.x < cnt) {
            const int64_t j = jb + threadIdx.x;
            double s[3];
            for (int d = 0; d < 3; ++d) {
                const double r = x[3 * j + d] / L[d];
                s[d] = r - floor(r);
            }
            if constexpr (F64) {
                st64[threadIdx.x] = SfStage64{s[0], s[1], s[2], q[j]};
            } else {
                // fixed-point rule of the library: u = min(2^32 - 1, floor(frac(x/L) 2^32))
                uint32_t u[3];
                for (int d = 0; d < 3; ++d) {
                    double w = floor(s[d] * kTwo32);
                    // non-finite positions give 0 instead of an undefined conversion
                    w = w >= 0.0 ? (w > kTwo32 - 1.0 ? kTwo32 - 1.0 : w) : 0.0;
                    u[d] = (uint32_t)w;
                }
                st32[threadIdx.x] = make_uint4(u[0], u[1], u[2], __float_as_uint((float)q[j]));
            }
        }
        __syncthreads();
        if constexpr (F64) {
            const double dmx = mx, dmy = my, dmz = mz;
            for (int h = 0; h < cnt; ++h) {
                const SfStage64 p = st64[h];
                const double t = dmx * p.sx + dmy * p.sy + dmz * p.sz;
                double sn, cs;
                rmath::sincos2pi(t - rint(t), &sn, &cs);
                re = fma(p.q, cs, re);
                im = fma(p.q, sn, im);
            }
        } else {
            // FP32 sums over runs of 32 particles, added up in FP64; the phase
            // m.u mod 2^32 is exact, sin/cos take it in revolutions
            const uint32_t ux = (uint32_t)mx, uy = (uint32_t)my, uz = (uint32_t)mz;
            for (int h0 = 0; h0 < cnt; h0 += 32) {
                const int h1 = h0 + 32 < cnt ? h0 + 32 : cnt;
                float rf = 0.f, fi = 0.f;
                for (int h = h0; h < h1; ++h) {
                    const uint4 p = st32[h];
                    const uint32_t t = rmath::dot3_mod32_v(ux, uy, uz, p.x, p.y, p.z);
                    const float f = rmath::phase_rev(t);
                    const float qf = __uint_as_float(p.w);
                    rf = fmaf(qf, __builtin_amdgcn_cosf(f), rf);
                    fi = fmaf(qf, __builtin_amdgcn_sinf(f), fi);
                }
                re += rf;
                im += fi;
            }
        }
        __syncthreads();
    }
    if (kv) partial[k * nchunk + c] = make_double2(re, im);
}

// rho_k = sum over the chunks of the partials of k, one wave per k: four
// strided accumulators per lane, then a fixed butterfly across the wave.
__global__ __launch_bounds__(256) void k_sf_reduce(int64_t nk, int64_t nchunk, const double2 *__restrict__ partial,
                                                   double *__restrict__ rho_re, double *__restrict__ rho_im) {
    const int lane = threadIdx.x & 63;
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= nk) return;
    const double2 *pk = partial + k * nchunk;
    double2 v0 = make_double2(0.0, 0.0), v1 = v0, v2 = v0, v3 = v0;
    int64_t c = lane;
    for (; c + 192 < nchunk; c += 256) {
        const double2 a0 = pk[c], a1 = pk[c + 64], a2 = pk[c + 128], a3 = pk[c + 192];
        v0.x += a0.x; v0.y += a0.y; v1.x += a1.x; v1.y += a1.y;
        v2.x += a2.x; v2.y += a2.y; v3.x += a3.x; v3.y += a3.y;
    }
    for (; c < nchunk; c += 64) {
        const double2 a0 = pk[c];
        v0.x += a0.x; v0.y += a0.y;
    }
    double re = (v0.x + v1.x) + (v2.x + v3.x), im = (v0.y + v1.y) + (v2.y + v3.y);
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
    }
    if (lane == 0) {
        rho_re[k] = re;
        rho_im[k] = im;
    }
}

rbsog_status sf_check(int64_t n, const double *x, const double *q, const double *box, int64_t nk, const int32_t *m,
                      int32_t precision, const double *rho_re, const double *rho_im, const char *who) {
    if (n < 1 || n > (int64_t)INT32_MAX) return fail_noctx(RBSOG_E_ARG, "%s: n must be in [1, 2^31-1]", who);
    if (nk < 1) return fail_noctx(RBSOG_E_ARG, "%s: n_k must be >= 1", who);
    if (!x || !q || !box || !m || !rho_re || !rho_im) return fail_noctx(RBSOG_E_ARG, "%s: null pointer", who);
    for (int d = 0; d < 3; ++d)
        if (!(box[d] > 0.0) || !std::isfinite(box[d]))
            return fail_noctx(RBSOG_E_ARG, "%s: box sides must be finite and > 0", who);
    if (precision != RBSOG_FP64 && precision != RBSOG_FP32C)
        return fail_noctx(RBSOG_E_ARG, "%s: unknown precision %d", who, precision);
    return RBSOG_OK;
}

rbsog_status sf_launch(int64_t n, const double *x, const double *q, const double *box, int64_t nk, const int32_t *m,
                       int32_t precision, double *rho_re, double *rho_im, hipStream_t s, double2 *partial,
                       int64_t nchunk, const char *who) {
    const int64_t chunk = (n + nchunk - 1) / nchunk;
    const int64_t ktiles = (nk + kSfBlock - 1) / kSfBlock;
    if (ktiles > 65535) return fail_noctx(RBSOG_E_ARG, "%s: n_k above %lld", who, (long long)(65535ll * kSfBlock));
    const dim3 grid((unsigned)nchunk, (unsigned)ktiles), block(kSfBlock);
    if (precision == RBSOG_FP64)
        hipLaunchKernelGGL(k_sf_partial<true>, grid, block, 0, s, n, x, q, box[0], box[1], box[2], nk, m, chunk,
                           nchunk, partial);
    else
        hipLaunchKernelGGL(k_sf_partial<false>, grid, block, 0, s, n, x, q, box[0], box[1], box[2], nk, m, chunk,
                           nchunk, partial);
    hipLaunchKernelGGL(k_sf_reduce, dim3((unsigned)((nk + 3) / 4)), dim3(256), 0, s, nk, nchunk,
                       (const double2 *)partial, rho_re, rho_im);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_noctx(RBSOG_E_DEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
    return RBSOG_OK;
}

// Device address of `scratch` on each device, taken once per device with the
// device current (the array's name is a host-side stand-in in host code).
std::mutex g_scratch_mu;
double2 *g_scratch_ptr[kMaxDevices] = {};

rbsog_status scratch_of_current_device(double2 **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_noctx(RBSOG_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail_noctx(RBSOG_E_DEVICE, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail_noctx(RBSOG_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = (double2 *)p;
    }
    *out = g_scratch_ptr[dev];
    return RBSOG_OK;
}

}  // namespace
}  // namespace rbsog

using namespace rbsog;

extern "C" {

rbsog_status rbsog_structure_factor(int64_t n, const double *x, const double *q, const double *box, int64_t n_k,
                                    const int32_t *m, int32_t precision, double *rho_re, double *rho_im,
                                    void *stream) {
    const char *who = "rbsog_structure_factor";
    rbsog_status st = sf_check(n, x, q, box, n_k, m, precision, rho_re, rho_im, who);
    if (st != RBSOG_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nchunk = sf_chunks(n, n_k);
    void *part = nullptr;
    hipError_t e = hipMallocAsync(&part, (size_t)(nchunk * n_k) * sizeof(double2), s);
    if (e != hipSuccess)
        return fail_noctx(RBSOG_E_OOM, "%s: %lld partial sums: %s", who, (long long)(nchunk * n_k),
                          hipGetErrorString(e));
    st = sf_launch(n, x, q, box, n_k, m, precision, rho_re, rho_im, s, (double2 *)part, nchunk, who);
    e = hipFreeAsync(part, s);
    if (st == RBSOG_OK && e != hipSuccess) return fail_noctx(RBSOG_E_DEVICE, "%s: free: %s", who, hipGetErrorString(e));
    return st;
}

rbsog_status rbsog_structure_factor_noalloc(int64_t n, const double *x, const double *q, const double *box,
                                            int64_t n_k, const int32_t *m, int32_t precision, double *rho_re,
                                            double *rho_im, void *stream) {
    const char *who = "rbsog_structure_factor_noalloc";
    rbsog_status st = sf_check(n, x, q, box, n_k, m, precision, rho_re, rho_im, who);
    if (st != RBSOG_OK) return st;
    if (n_k > kScratchComplex)
        return fail_noctx(RBSOG_E_ARG, "%s: n_k = %lld exceeds the %lld wave vectors its scratch holds", who,
                          (long long)n_k, (long long)kScratchComplex);
    double2 *sp = nullptr;
    st = scratch_of_current_device(&sp);
    if (st != RBSOG_OK) return st;
    const int64_t nchunk = sf_chunks(n, n_k);
    return sf_launch(n, x, q, box, n_k, m, precision, rho_re, rho_im, (hipStream_t)stream, sp, nchunk, who);
}

}  // extern "C"
