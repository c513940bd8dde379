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
    int32_t ngauss;              // M + 1
};

// Device-resident coefficients of the split.
struct SogDev {
    const double *w64;    // omega_l
    const double *a64;    // 1 / s_l^2
    const double *c64;    // 2 omega_l / s_l^2
    const float *w32;     // omega_l
    const float *a32;     // log2(e) / s_l^2
    const float *c32;     // 2 omega_l / s_l^2
};

// ---- kernel launchers (kernels_md.hip) --------------------------------------
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void launch_quantise(const Geom &g, double *x, uint32_t *u, int32_t *cell_of, int32_t *cell_count,
                     hipStream_t s);
void launch_scan(const int32_t *in, int32_t *out_excl, int32_t *fill_copy, int64_t n, int32_t *blocksums,
                 hipStream_t s);
int64_t scan_blocksums_size(int64_t n);
void launch_cell_scatter(const Geom &g, const int32_t *cell_of, int32_t *fill, int32_t *order, hipStream_t s);
void launch_cell_sort(int64_t ncell, const int32_t *start, int32_t *order, hipStream_t s);
void launch_gather(const Geom &g, const int32_t *order, const uint32_t *u, const double *x, const double *q,
                   uint32_t *su, double *sx, double *sq, float *sqf, bool f64, hipStream_t s);
void launch_kick(int64_t n, double half_dt_over_m, double *v, const double *Fn, const double *Ff, int32_t *flag,
                 hipStream_t s);
void launch_drift(int64_t n, double dt, double *x, const double *v, hipStream_t s);

// ---- near part (kernels_near.hip) ------------------------------------------
int64_t near_blocks(int64_t n);
void launch_near(const Geom &g, const SogDev &c, bool f64, const int32_t *start, const int32_t *order,
                 const uint32_t *su, const double *sx, const double *sq, const float *sqf, double *Fn,
                 double *epart, hipStream_t s);
void launch_neighbor_count(const Geom &g, bool f64, const int32_t *start, const int32_t *order,
                           const uint32_t *su, const double *sx, int64_t *counts, hipStream_t s);
void launch_neighbor_fill(const Geom &g, bool f64, const int32_t *start, const int32_t *order,
                          const uint32_t *su, const double *sx, const int64_t *row_ptr, int32_t *cols,
                          hipStream_t s);

// ---- far part (kernels_far.hip) --------------------------------------------
struct FarPlan {
    int kt;        // k tiles of 64 lanes per block
    int streams;   // particle streams (waves per k tile) per block
    int64_t chunk; // particles per block
    int64_t nblk;  // blocks along the particle axis
    int64_t kblk;  // blocks along the k axis
};
FarPlan far_plan(int64_t n, int32_t P);
void launch_stage_k(const Geom &g, int32_t P, const int32_t *kseq, const double *kw, double w_rb,
                    int64_t *cursor, KRec64 *kb64, KRec32 *kb32, double *wk, hipStream_t s);
void launch_rho(const Geom &g, const FarPlan &fp, int32_t P, bool f64, const double *x, const uint32_t *u,
                const double *q, const float *qf, const KRec64 *kb64, const KRec32 *kb32, double *partial,
                hipStream_t s);
void launch_rho_reduce(int32_t P, int64_t nblk, const double *partial, const double *wk, KRec64 *kb64,
                       KRec32 *kb32, double *rho, double *ek, hipStream_t s);
void launch_far(const Geom &g, int32_t P, bool f64, const double *x, const uint32_t *u, const double *q,
                const float *qf, const KRec64 *kb64, const KRec32 *kb32, double *Ff, hipStream_t s);
void launch_finalize(int64_t nnear, const double *epart, int32_t P, const double *ek, double uself, double *E,
                     int32_t *flag, hipStream_t s);

}  // namespace rbsog
