// Internal declarations shared by the host side (capi.hip) and the kernels
// (kernels_*.hip) of librbsog.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "rbsog.h"

namespace rbsog {

constexpr int kMaxGauss = 160;  // M + 1 <= kMaxGauss

// Per-k record read uniformly by every lane of the far-force kernel
// (FP64 form): integer m as doubles, w k (the weighted wave vector), rho.
struct KRec64 {
    double mx, my, mz;
    double ckx, cky, ckz;
    double re, im;
};
// FP32 form: m as int32, w k and rho rounded to float.
struct KRec32 {
    int32_t mx, my, mz;
    float ckx, cky, ckz;
    float re, im;
};

// Geometry and split constants passed by value to the kernels.
struct Geom {
    int64_t n;
    double L[3], invL[3], h[3];  // h = L * 2^-32
    float hf[3];
    double rc2;                  // rc * rc
    double band_lo, band_hi;     // FP64 r^2 thresholds outside which the fast test decides
    float band_lo_f, band_hi_f;  // same for the FP32 fast test
    int32_t nc[3];
    int32_t reach[3];            // 1 if the stencil spans -1..1 in that dimension, 0 otherwise
};

// The near kernel evaluates the narrow Gaussians (r_c^2 / s_l^2 > tau) with an
// exponential each and replaces the wide ones (s_l grows with l, so they are
// l >= nexp) by the Taylor polynomial of their sum in x = r^2.  Truncation per
// Gaussian: tau^(deg+1)/(deg+1)! of its weight, 5e-18 (FP64) and 1.2e-8 (FP32).
constexpr double kTailTau64 = 0.05;
constexpr double kTailTau32 = 0.25;
constexpr int kTailDeg64 = 8;
constexpr int kTailDeg32 = 6;
constexpr int kMaxExp = 24;  // narrow Gaussians per split (more is rejected)

// Split coefficients, passed by value in the near kernel's arguments so that
// every lane reads them through the scalar unit.
template <typename R, int NT>
struct SplitCoef {
    R a[kMaxExp];   // 1/s_l^2 (FP32: log2(e)/s_l^2, for exp2)
    R cw[kMaxExp];  // 2 omega_l / s_l^2
    R w[kMaxExp];   // omega_l
    R pt[NT];       // sum_{l>=nexp} omega_l e^{-x/s_l^2} = sum_k pt[k] x^k
    R ft[NT];       // sum_{l>=nexp} 2 omega_l/s_l^2 e^{-x/s_l^2} = sum_k ft[k] x^k
    int32_t nexp;
};
using SplitCoef64 = SplitCoef<double, kTailDeg64 + 1>;
using SplitCoef32 = SplitCoef<float, kTailDeg32 + 1>;

// Arguments of the k-batch staging (Algorithm 1: the next P frequencies of the
// pre-sampled sequence, in order) and of the velocity-Verlet half kicks.
struct StageArgs {
    int32_t P;
    const int32_t *kseq;  // sequence, 3 int32 per vector
    const double *kw;     // per-vector weights, or null for the random-batch weight
    double w_rb;          // S pi^{3/2} / (P V)
    int64_t *cursor;      // device cursor (vectors consumed)
    KRec64 *kb64;
    KRec32 *kb32;
    double *wk;
};
struct KickArgs {
    int32_t on;      // 0: no kick
    double hdm;      // dt / (2 m)
    double dt;       // drift step (kick-drift kernel only)
    double *v;
    const double *Fn, *Ff;
    int32_t *flag;   // bit 0: non-finite force
};

// Stage the current batch: per-k records for both precisions and the weights,
// then advance the cursor.  Called by one whole block.
__device__ inline void stage_batch(const Geom &g, const StageArgs &a) {
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    const int64_t base = *a.cursor;
    for (int32_t k = threadIdx.x; k < a.P; k += blockDim.x) {
        const int64_t e = base + k;
        const int32_t mx = a.kseq[3 * e], my = a.kseq[3 * e + 1], mz = a.kseq[3 * e + 2];
        const double w = a.kw ? a.kw[e] : a.w_rb;
        const double kx = kTwoPi * g.invL[0] * mx, ky = kTwoPi * g.invL[1] * my, kz = kTwoPi * g.invL[2] * mz;
        KRec64 r;
        r.mx = mx; r.my = my; r.mz = mz;
        r.ckx = w * kx; r.cky = w * ky; r.ckz = w * kz;
        r.re = 0.0; r.im = 0.0;
        a.kb64[k] = r;
        KRec32 h;
        h.mx = mx; h.my = my; h.mz = mz;
        h.ckx = (float)r.ckx; h.cky = (float)r.cky; h.ckz = (float)r.ckz;
        h.re = 0.f; h.im = 0.f;
        a.kb32[k] = h;
        a.wk[k] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) *a.cursor = base + a.P;
}

// ---- kernel launchers (kernels_md.hip) --------------------------------------
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
// kick dt/2 + drift (if kick.on), wrap, quantise, cell histogram; the last
// block stages the k batch
void launch_kdq(const Geom &g, const KickArgs &kick, const StageArgs &stage, double *x, uint32_t *u,
                int32_t *cell_of, int32_t *cell_count, hipStream_t s);
void launch_scan(const int32_t *in, int32_t *out_excl, int32_t *fill_copy, int64_t n, int32_t *blocksums,
                 hipStream_t s);
int64_t scan_blocksums_size(int64_t n);
void launch_cell_scatter(const Geom &g, const int32_t *cell_of, int32_t *fill, int32_t *order, hipStream_t s);
// per cell: id sort of its segment and reset of its histogram count; then gather into cell order
void launch_sort_gather(const Geom &g, int64_t ncell, const int32_t *start, int32_t *order, int32_t *cell_count,
                        const uint32_t *u, const double *x, const double *q, uint32_t *su, double *sx, double *sq,
                        float *sqf, bool f64, hipStream_t s);

// ---- near part (kernels_near.hip) ------------------------------------------
struct NearPlan {
    int32_t nblk;             // blocks (a multiple of 8)
    int64_t cells_per_block;  // contiguous cells per block
};
NearPlan near_plan(int64_t ncell);
void launch_near(const Geom &g, const SplitCoef64 &c64, const SplitCoef32 &c32, bool f64, const NearPlan &np, int64_t ncell, const int32_t *start,
                 const int32_t *order, const uint32_t *su, const double *sx, const double *sq, const float *sqf,
                 double *Fn, double *epart, hipStream_t s);
void launch_neighbor_count(const Geom &g, const int32_t *start, const int32_t *order, const uint32_t *su,
                           int64_t *counts, hipStream_t s);
void launch_neighbor_fill(const Geom &g, const int32_t *start, const int32_t *order, const uint32_t *su,
                          const int64_t *row_ptr, int32_t *cols, hipStream_t s);

// ---- far part (kernels_far.hip) --------------------------------------------
struct FarPlan {
    int kt;        // k tiles of 64 lanes per block
    int streams;   // particle streams (waves per k tile) per block
    int64_t chunk; // particles per block
    int64_t nblk;  // blocks along the particle axis
    int64_t kblk;  // blocks along the k axis
};
FarPlan far_plan(int64_t n, int32_t P);
void launch_rho(const Geom &g, const FarPlan &fp, int32_t P, bool f64, const double *x, const uint32_t *u,
                const double *q, const float *qf, const KRec64 *kb64, const KRec32 *kb32, double *partial,
                hipStream_t s);
// rho_e, its records and per-k energies; the last block to finish also sums
// the energies (U_N from the near partials, U*, U_self, U) and re-arms counter
void launch_rho_reduce(int32_t P, int64_t nblk, const double *partial, const double *wk, KRec64 *kb64,
                       KRec32 *kb32, double *rho, double *ek, int64_t nnear, const double *epart, double uself,
                       double *E, int32_t *flag, uint32_t *counter, hipStream_t s);
// far force; with kick.on the closing half kick v += dt/(2m) (F_N + F*) follows
void launch_far(const Geom &g, int32_t P, bool f64, const double *x, const uint32_t *u, const double *q,
                const float *qf, const KRec64 *kb64, const KRec32 *kb32, double *Ff, const KickArgs &kick,
                hipStream_t s);

}  // namespace rbsog
