// Near part of the sum-of-Gaussians split for gfx950 (Sec. 3.1, eq.
// "forcesplit", with the factor of -grad U_N):
//   F_N,i = sum_{j: r_ij < r_c} q_i q_j (1/r^3 - 2 sum_l omega_l/s_l^2 e^{-r^2/s_l^2}) r_ij
//   U_N   = 1/2 sum_i sum_j q_i q_j (1/r - sum_l omega_l e^{-r^2/s_l^2})
//
// A Verlet list with a skin: a build lists, for every particle, the particles
// within r_c (1 + skin) of it, and the list serves every evaluation until a
// particle has moved farther than skin r_c / 2 from its position at the build
// (checked at every step by the kick/drift kernel).  Every listed pair is
// still put to the exact pair rule at its current positions, so the pairs
// evaluated are exactly those within r_c.
//
// Build: work items are 64 consecutive particles (homes) of one system in
// cell order, one wave per item.  The candidates of a home cell are the
// particles of its 27 (or fewer) neighbouring cells (cells are at least
// r_c (1 + skin) wide); the three cells of a row are contiguous in cell order,
// so they are up to 18 contiguous ranges of the sorted arrays.  The wave holds
// candidates on its lanes and tests every (home, candidate) pair with the
// home broadcast; accepted pairs are compacted with a ballot into an LDS ring
// and written out 64 at a time.  The list of item b is the entries
// [b icap, b icap + count) of the pair array.
//
// Evaluation: one block of four waves per item; the waves take turns over the
// item's pairs, 64 per pass, sum each home's forces with a segmented scan
// across the wave and keep them in per-wave LDS slots, added in a fixed order
// at the end, so results are the same on every run.  Blocks are dealt to the
// 8 XCDs so that each XCD sweeps one contiguous slab of items and keeps its
// candidates in its own L2.
//
// Gaussians with r_c^2/s_l^2 <= kTailTau are summed as one polynomial in r^2
// (their Taylor series, truncated below rounding), the narrow ones with an
// exponential each.  Pair inclusion follows the fixed-point rule of rbsog.h:
// an FP32 test decides every pair outside a narrow band around r_c, the exact
// FP64 rule decides the rest, so the pairs are bit-exact in both precisions.
#include <algorithm>
#include <type_traits>

#include "rbsog_internal.h"
#include "rbsog_math.h"

namespace rbsog {

namespace {

constexpr int kBlock = 256;
constexpr int kRanges = 18; // 9 rows of cells x up to 2 contiguous pieces
constexpr float kFarR2 = 3.0e38f;  // r^2 of a pair that no test admits
// narrow Gaussians evaluated with constants held in registers, no test of
// their count (Table 1 row 2 at any cutoff has 3 above the tail's threshold;
// further ones take a counted loop)
template <bool F64>
constexpr int kExpRegs = 3;

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

// Range r (0..17) of the candidate cells of the home cells x = cx .. cx+w-1
// (w = 1 or 2, one row) in cell order: x runs over cx-1 .. cx+w (w = 2 needs
// at least 6 cells along x, so that the pieces never overlap).
__device__ __forceinline__ bool row_range_w(const Geom &g, const int32_t *__restrict__ start, int r, int cx, int cy,
                                            int cz, int w, int32_t &lo, int32_t &hi) {
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
        const int x0 = cx - 1, x1 = cx + w;
        if (x0 < 0) {
            if (part == 0) { xa = xb = g.nc[0] - 1; } else { xa = 0; xb = x1; }
        } else if (x1 >= g.nc[0]) {
            if (part == 0) { xa = x0; xb = g.nc[0] - 1; } else { xa = 0; xb = x1 - g.nc[0]; }
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

// Sum over the wave in a fixed order (the same on every run).
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Mask of the active lanes for which p holds (the lane mask the compare
// already produced, without going through a vector register).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Values the wave holds in common (loaded or broadcast): keep them scalar.
__device__ __forceinline__ int32_t rfl(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Broadcast the double held by lane `src` (uniform) to the whole wave.
__device__ __forceinline__ double bcast64(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}

// Per-system constants are read through the constant address space, so that
// uniform reads become scalar loads.
typedef const SysDev __attribute__((address_space(4))) CSys;
typedef const int32_t __attribute__((address_space(4))) CI32;
typedef const SplitCoef64 __attribute__((address_space(4))) CCoef64;
typedef const SplitCoef32 __attribute__((address_space(4))) CCoef32;
// DPP lane moves (row = 16 lanes): row_shr:n, and row_bcast:15 / row_bcast:31.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (uint32_t)lo);
}
template <int CTRL, int ROWS, typename R>
__device__ __forceinline__ R dpp(R v) {
    if constexpr (sizeof(R) == 8) return dpp_d<CTRL, ROWS>(v);
    else return dpp_f<CTRL, ROWS>(v);
}

// Segmented inclusive sum across the wave: lane l ends with the sum of lanes
// [max(sstart, .), l] of its segment (segments are runs of lanes; sstart is
// the first lane of l's segment).  In-row shifts 1, 2, 4, 8, then the row
// totals: lane 15 into rows 1 and 3, lane 31 into rows 2 and 3.  A moved
// value from outside the segment is multiplied by 0 rather than skipped, so
// that no step changes the lane mask (the moves read 0 where they have no
// source lane).
// Inclusive sum over lanes 0..31 by DPP moves (lanes 32..63 hold sums of
// their own half): in-row shifts 1, 2, 4, 8 (a move reads 0 where it has no
// source lane), then row 1 adds lane 15 (the broadcast leaves rows 0 and 2
// with the move's old value 0).
__device__ __forceinline__ int32_t incl_scan32(int32_t v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    return v;
}

template <typename R>
__device__ __forceinline__ void seg_scan3(R &x, R &y, R &z, int lane, int sstart) {
    if constexpr (sizeof(R) == 4) {
        // FP32: each step is one multiply-add that reads the moved value
        // through DPP (x += m * x[lane - N]), three per step.  A DPP source
        // needs two wait states after the VALU write of it: the leading nop
        // covers the writes before the block, and inside it each accumulator
        // is written two instructions before it is read again.  Lanes of rows
        // that a broadcast step masks out keep their value.
        // the 0/1 factors by clamping integer-valued differences to [0, 1]
        // (no compare and select, whose mask write a select would wait for)
        const float fs = (float)sstart;
        const float d = (float)lane - fs;  // = len
        const float m1 = __builtin_amdgcn_fmed3f(d, 0.0f, 1.0f);          // len >= 1
        const float m2 = __builtin_amdgcn_fmed3f(d - 1.0f, 0.0f, 1.0f);   // len >= 2
        const float m4 = __builtin_amdgcn_fmed3f(d - 3.0f, 0.0f, 1.0f);   // len >= 4
        const float m8 = __builtin_amdgcn_fmed3f(d - 7.0f, 0.0f, 1.0f);   // len >= 8
        // rows 1 and 3 only: lane 16 r - 1 lies in the segment
        const float m15 = __builtin_amdgcn_fmed3f((float)(lane & ~15) - fs, 0.0f, 1.0f);
        const float m31 = __builtin_amdgcn_fmed3f(32.0f - fs, 0.0f, 1.0f);  // rows 2 and 3 only
#define RBSOG_FMAC3(M, CTRL, RM)                                                             \
    "v_fmac_f32_dpp %0, %0, " M " " CTRL " row_mask:" RM " bank_mask:0xf bound_ctrl:1\n\t" \
    "v_fmac_f32_dpp %1, %1, " M " " CTRL " row_mask:" RM " bank_mask:0xf bound_ctrl:1\n\t" \
    "v_fmac_f32_dpp %2, %2, " M " " CTRL " row_mask:" RM " bank_mask:0xf bound_ctrl:1\n\t"
        asm volatile("s_nop 1\n\t"
                     RBSOG_FMAC3("%3", "row_shr:1", "0xf")
                     RBSOG_FMAC3("%4", "row_shr:2", "0xf")
                     RBSOG_FMAC3("%5", "row_shr:4", "0xf")
                     RBSOG_FMAC3("%6", "row_shr:8", "0xf")
                     RBSOG_FMAC3("%7", "row_bcast:15", "0xa")
                     RBSOG_FMAC3("%8", "row_bcast:31", "0xc")
                     : "+v"(x), "+v"(y), "+v"(z)
                     : "v"(m1), "v"(m2), "v"(m4), "v"(m8), "v"(m15), "v"(m31));
#undef RBSOG_FMAC3
    } else {
        const int len = lane - sstart;  // lanes of the segment before this one
#define RBSOG_SHR(N)                                                                     \
    {                                                                                    \
        const R tx = dpp<0x110 + N, 0xf>(x), ty = dpp<0x110 + N, 0xf>(y), tz = dpp<0x110 + N, 0xf>(z); \
        const R m = len >= N ? (R)1 : (R)0;                                              \
        x = fma(tx, m, x); y = fma(ty, m, y); z = fma(tz, m, z);                         \
    }
        RBSOG_SHR(1)
        RBSOG_SHR(2)
        RBSOG_SHR(4)
        RBSOG_SHR(8)
#undef RBSOG_SHR
        {
            // row_bcast:15 to rows 1 and 3 (row mask 0xa)
            const R tx = dpp<0x142, 0xa>(x), ty = dpp<0x142, 0xa>(y), tz = dpp<0x142, 0xa>(z);
            const int row = lane >> 4;
            const R m = (row == 1 || row == 3) && row * 16 - 1 >= sstart ? (R)1 : (R)0;
            x = fma(tx, m, x); y = fma(ty, m, y); z = fma(tz, m, z);
        }
        {
            // row_bcast:31 to rows 2 and 3 (row mask 0xc)
            const R tx = dpp<0x143, 0xc>(x), ty = dpp<0x143, 0xc>(y), tz = dpp<0x143, 0xc>(z);
            const R m = lane >= 32 && 31 >= sstart ? (R)1 : (R)0;
            x = fma(tx, m, x); y = fma(ty, m, y); z = fma(tz, m, z);
        }
    }
}

template <bool F64>
struct CoefOf { using type = CCoef32; };

// Field-wise copy of a system's geometry out of the constant address space.
__device__ __forceinline__ Geom load_geom(CSys *sp) {
    Geom g;
    g.n = sp->g.n;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = sp->g.L[d];
        g.invL[d] = sp->g.invL[d];
        g.h[d] = sp->g.h[d];
        g.hf[d] = sp->g.hf[d];
        g.nc[d] = sp->g.nc[d];
        g.reach[d] = sp->g.reach[d];
    }
    g.rc2 = sp->g.rc2;
    g.band_lo = sp->g.band_lo;
    g.band_hi = sp->g.band_hi;
    g.band_lo_f = sp->g.band_lo_f;
    g.band_hi_f = sp->g.band_hi_f;
    g.rl2_f = sp->g.rl2_f;
    g.dthr2_f = sp->g.dthr2_f;
    return g;
}
template <>
struct CoefOf<true> { using type = CCoef64; };

constexpr int kNW = 4;        // waves per block
constexpr int kU = 2;         // homes tested together in the build
// pair ring entries per wave in the build (a power of two above the
// 63 + kU * S * 64 entries that can be pending)
constexpr int ring_size(int S) { return S <= 3 ? 512 : 1024; }
constexpr uint32_t kNoCand = 0xfffffffeu;  // candidate slot past the end of the list

// Homes per wave: an item's four waves each own a quarter of its homes (and
// the quarter's segment of the item's list), in the build and in the list
// pass alike, so a home's pairs are added by one wave in one order.
constexpr int kQuarter = kListHomes / kNW;
static_assert(kNW == kListWaves, "one wave per quarter of an item");

template <bool F64>
struct EvalLds {
    using R = typename std::conditional<F64, double, float>::type;
    static constexpr int XH = F64 ? kQuarter : 1;
    uint4 hu[kQuarter];    // home u_x, u_y, u_z, slot
    R hq[kQuarter];
    double hx[3][XH];
    R hf[3][kQuarter];     // force accumulators
};

// One listed pair per lane (`have`): the pair rule at the current positions
// (the fixed-point r^2 in FP32 decides below the lower band edge, the exact
// FP64 rule above it), then the exact displacement (fixed point for FP32C,
// wrapped FP64 coordinates for FP64), the pair force and energy.  One home's
// entries are contiguous within a build pass, so forces are summed by a
// segmented scan across the wave and the last lane of each segment adds the
// total to the wave's accumulator of that home.
// Debug record of the pairs a near kernel accepts (the debug launches
// only): the caller indices of home and candidate, appended at an atomic
// counter (entries past the capacity are counted, not written).
struct PairRec {
    const int32_t *id;  // caller index of each slot of the order the kernel reads
    uint2 *out;
    int32_t *cnt;
    int32_t cap;
};

// Homes of one item in LDS, as the evaluation reads them; `hf` is the
// accumulator set the pairs add to.
template <bool F64>
struct HomeView {
    using R = typename std::conditional<F64, double, float>::type;
    const uint4 *hu;       // u_x, u_y, u_z, slot
    const R *hq;
    const double *hx[3];   // FP64 positions (FP64 form only)
    R *hf[3];
    bool we;               // sum the pair energies (else forces only)
    const PairRec *rec;    // debug launches: where accepted pairs are recorded
};

// The candidate's data a pair needs: fixed-point coordinates, charge, and
// the FP64 position in the FP64 form.
template <bool F64>
struct PairData {
    uint32_t u[3];
    typename std::conditional<F64, double, float>::type q;
    double x[3];
};

// The candidate's data from its gather records, given the list entry (the
// byte offset 16 j of candidate slot j's record): one 16-byte load (and one
// 32-byte record in the FP64 form).
template <bool F64>
__device__ __forceinline__ PairData<F64> load_packed(const uint4 *__restrict__ pk, const PosQ64 *__restrict__ pkx,
                                                     uint32_t off) {
    PairData<F64> d;
    // slots below 2^28: 32-bit byte offsets from the arrays' (scalar) bases
    const uint4 r = *(const uint4 *)((const char *)pk + off);
    d.u[0] = r.x; d.u[1] = r.y; d.u[2] = r.z;
    if constexpr (F64) {
        const PosQ64 w = *(const PosQ64 *)((const char *)pkx + (off << 1));
        d.x[0] = w.x; d.x[1] = w.y; d.x[2] = w.z;
        d.q = w.q;
    } else {
        d.q = __uint_as_float(r.w);
    }
    return d;
}

template <bool F64>
__device__ __forceinline__ PairData<F64> load_pair(const uint32_t *__restrict__ su, const double *__restrict__ sx,
                                                   const double *__restrict__ sq, const float *__restrict__ sqf,
                                                   int64_t n, uint2 qe, bool have) {
    PairData<F64> d;
    // slots are below 2^28 (a context's limit): 32-bit byte offsets from the
    // arrays' (scalar) bases
    const uint32_t j = have ? (qe.y & kListSlotMask) : 0u;
    const uint32_t o4 = j * 4u, o8 = j * 8u;
    auto at4 = [&](const void *base) { return *(const uint32_t *)((const char *)base + o4); };
    auto at8 = [&](const void *base) { return *(const double *)((const char *)base + o8); };
    d.u[0] = at4(su); d.u[1] = at4(su + n); d.u[2] = at4(su + 2 * n);
    if constexpr (F64) {
        d.q = at8(sq);
        d.x[0] = at8(sx); d.x[1] = at8(sx + n); d.x[2] = at8(sx + 2 * n);
    } else {
        d.q = __uint_as_float(at4(sqf));
    }
    return d;
}

// The home of a pair as the evaluation needs it: fixed-point coordinates,
// its slot, charge, and the FP64 position in the FP64 form.
template <bool F64>
struct HomeData {
    using R = typename std::conditional<F64, double, float>::type;
    uint32_t u[3];
    uint32_t slot;
    R q;
    double x[3];
};

// One pair (home h, candidate pd at slot cslot) when `have`: the pair rule at
// the current positions (the fixed-point r^2 in FP32 decides below the lower
// band edge, the exact FP64 rule inside the band), then the exact
// displacement (fixed point for FP32C, wrapped FP64 coordinates for FP64),
// the pair force on the home (fx, fy, fz) and, with energies, half the pair
// energy (de).  Returns whether the pair was accepted; a rejected pair leaves
// the outputs 0.  SELF: the candidate may be the home itself (the fused cell
// kernel's test does not leave it out), rejected here by its slot.  DBG:
// record every accepted pair (debug launches).
template <bool F64, bool SELF = false, bool DBG = false>
__device__ __forceinline__ void pair_force(const Geom &g, typename CoefOf<F64>::type *co, const HomeData<F64> &h,
                                           bool we, const PairRec *rec, const float4 *__restrict__ tbl, float rin2,
                                           CSys *csp, uint32_t cslot, bool have, const PairData<F64> &pd,
                                           typename HomeData<F64>::R &fx, typename HomeData<F64>::R &fy,
                                           typename HomeData<F64>::R &fz, double &de) {
    using R = typename HomeData<F64>::R;
    constexpr int NT = (F64 ? kTailDeg64 : kTailDeg32) + 1;
    // every lane computes (no branch on `have` or on the pair rule: a lane
    // mask change costs more than the arithmetic); a select zeroes what a
    // rejected or empty lane produced, whatever its value
    const uint32_t dux = pd.u[0] - h.u[0], duy = pd.u[1] - h.u[1], duz = pd.u[2] - h.u[2];
    const float ex_ = (float)(int32_t)dux * g.hf[0];
    const float ey_ = (float)(int32_t)duy * g.hf[1];
    const float ez_ = (float)(int32_t)duz * g.hf[2];
    const float r2f = ex_ * ex_ + ey_ * ey_ + ez_ * ez_;
    bool in = r2f <= g.band_lo_f;
    // the exact rule only inside the narrow band (rare: a branch)
    if (have && !in && r2f < g.band_hi_f) in = exact_in(g, dux, duy, duz);
    in = in && have;
    if constexpr (SELF) in = in && cslot != h.slot;
    if constexpr (DBG) {
        if (in) {
            const int32_t k = atomicAdd(rec->cnt, 1);
            if (k < rec->cap) rec->out[k] = make_uint2((uint32_t)rec->id[h.slot], (uint32_t)rec->id[cslot]);
        }
    }
    R dx, dy, dz, qq;
    if constexpr (F64) {
        dx = mi64(pd.x[0] - h.x[0], g.L[0], g.invL[0]);
        dy = mi64(pd.x[1] - h.x[1], g.L[1], g.invL[1]);
        dz = mi64(pd.x[2] - h.x[2], g.L[2], g.invL[2]);
    } else {
        dx = ex_; dy = ey_; dz = ez_;
    }
    qq = h.q * pd.q;
    const R r2 = F64 ? dx * dx + dy * dy + dz * dz : r2f;
    R gk, hk;  // force coefficient g and pair potential h of the split
    if (!F64 && tbl) {
        if (r2 >= rin2) {
            // shell: table point from the FP32 bits of r^2, linear in r^2
            const uint32_t bits = __float_as_uint(r2f);
            const float4 tv = tbl[(bits >> (23 - kTabBman)) & (kTabSize - 1)];
            const float fr = (float)(bits & ((1u << (23 - kTabBman)) - 1u)) * (1.0f / (1 << (23 - kTabBman)));
            gk = fmaf(fr, tv.y, tv.x);
            hk = fmaf(fr, tv.w, tv.z);
        } else {
            // core: Taylor terms of the Gaussians, 1/r and 1/r^3 computed
            const float ri = __builtin_amdgcn_rsqf(r2f);
            float pa = csp->ta[kTabQ - 1], pb = csp->tb[kTabQ - 1];
#pragma unroll
            for (int t = kTabQ - 2; t >= 0; --t) pa = fmaf(pa, r2f, csp->ta[t]);
            if (we) {
#pragma unroll
                for (int t = kTabQ - 2; t >= 0; --t) pb = fmaf(pb, r2f, csp->tb[t]);
            }
            gk = ri * ri * ri - 2.0f * pa;
            hk = ri - pb;
        }
    } else {
        // Horner from the leading coefficient
        R rinv, gs = co->ft[NT - 1], ph = 0;
        if constexpr (F64) rinv = rsqrt(r2);
        else rinv = __builtin_amdgcn_rsqf(r2);
#pragma unroll
        for (int t = NT - 2; t >= 0; --t) {
            if constexpr (F64) gs = fma(gs, r2, co->ft[t]);
            else gs = fmaf(gs, r2, co->ft[t]);
        }
        if (we) {
            ph = co->pt[NT - 1];
#pragma unroll
            for (int t = NT - 2; t >= 0; --t) {
                if constexpr (F64) ph = fma(ph, r2, co->pt[t]);
                else ph = fmaf(ph, r2, co->pt[t]);
            }
        }
        // the first kExpRegs terms at fixed indices, with no test of
        // the count: the constants past it are zero (a term of weight
        // 0 adds exactly 0)
        constexpr int NE = kExpRegs<F64>;
        R exv[NE];
#pragma unroll
        for (int l = 0; l < NE; ++l) {
            if constexpr (F64) exv[l] = rmath::exp_nonpos(-r2 * co->a[l]);
            else exv[l] = __builtin_amdgcn_exp2f(-r2 * co->a[l]);
            gs += co->cw[l] * exv[l];
        }
        // the potential's terms only when energies are summed: a
        // uniform branch, kept a branch by the empty asm statement
        // (which the compiler does not speculate)
        if (we) {
            asm volatile("");
#pragma unroll
            for (int l = 0; l < NE; ++l) ph += co->w[l] * exv[l];
        }
        for (int l = NE; l < co->nexp; ++l) {
            R ex;
            if constexpr (F64) ex = rmath::exp_nonpos(-r2 * co->a[l]);
            else ex = __builtin_amdgcn_exp2f(-r2 * co->a[l]);
            gs += co->cw[l] * ex;
            if (we) ph += co->w[l] * ex;
        }
        gk = rinv * rinv * rinv - gs;
        hk = rinv - ph;
    }
    // force on the home along r_i - r_j = -(dx, dy, dz); zero unless accepted
    const R coef = in ? qq * gk : (R)0;
    fx = -coef * dx;
    fy = -coef * dy;
    fz = -coef * dz;
    de = 0.0;
    if (we) {
        asm volatile("");
        de = in ? 0.5 * (double)(qq * hk) : 0.0;
    }
}

// One ring entry per lane (`have`), home `slot` of the wave's LDS homes: the
// pair force, then the wave's segmented sum.  One home's entries are
// contiguous within a pass, so forces are summed by a segmented scan across
// the wave and the last lane of each segment adds the total to the wave's
// accumulator of that home.
template <bool F64, bool SELF = false, bool DBG = false>
__device__ __forceinline__ void eval_loaded(const Geom &g, typename CoefOf<F64>::type *co, const HomeView<F64> &L,
                                            const float4 *__restrict__ tbl, float rin2, CSys *csp,
                                             int lane, uint2 qe, bool have, const PairData<F64> &pd,
                                            double &e) {
    using R = typename HomeView<F64>::R;
    R fx, fy, fz;
    double de;
    const int slot = have ? (int)qe.x : -1;
    // an empty lane reads home 0 (its pair is not accepted)
    const int hs = have ? slot : 0;
    HomeData<F64> h;
    const uint4 hu = L.hu[hs];
    h.u[0] = hu.x; h.u[1] = hu.y; h.u[2] = hu.z; h.slot = hu.w;
    h.q = L.hq[hs];
    if constexpr (F64) {
        h.x[0] = L.hx[0][hs]; h.x[1] = L.hx[1][hs]; h.x[2] = L.hx[2][hs];
    }
    pair_force<F64, SELF, DBG>(g, co, h, L.we, L.rec, tbl, rin2, csp, qe.y, have, pd, fx, fy, fz, de);
    if (L.we) {
        asm volatile("");
        e += de;
    }
    const int prev = __shfl_up(slot, 1, 64);
    const bool seg = lane == 0 || slot != prev;
    const uint64_t H = ballot(seg);
    const uint64_t upto = H & ((2ull << lane) - 1ull);
    const int sstart = 63 - __clzll((long long)upto);
    seg_scan3<R>(fx, fy, fz, lane, sstart);
    // a pass can hold two runs of one home (two candidate passes of the
    // build), so segment totals are added atomically; the adds of one wave
    // into its own slots happen in a fixed order
    // the lanes holding pairs are a prefix: its last lane, and every lane
    // before a segment start, ends a segment
    const uint64_t HM = ballot(have);
    const uint64_t TM = ((H >> 1) | (HM ^ (HM >> 1))) & HM;
    const bool tail = (TM >> lane) & 1ull;
    if (tail) {
        atomicAdd(&L.hf[0][slot], fx);
        atomicAdd(&L.hf[1][slot], fy);
        atomicAdd(&L.hf[2][slot], fz);
    }
}

template <bool F64, bool SELF = false, bool DBG = false>
__device__ __forceinline__ void eval_pair(const Geom &g, typename CoefOf<F64>::type *co, const HomeView<F64> &L,
                                          const uint32_t *__restrict__ su, const double *__restrict__ sx,
                                          const double *__restrict__ sq, const float *__restrict__ sqf, int64_t n,
                                          const float4 *__restrict__ tbl, float rin2, CSys *csp,
                                           int lane, uint2 qe, bool have, double &e) {
    const PairData<F64> pd = load_pair<F64>(su, sx, sq, sqf, n, qe, have);
    eval_loaded<F64, SELF, DBG>(g, co, L, tbl, rin2, csp, lane, qe, have, pd, e);
}

template <int Q>
struct BuildLds {
    uint4 hu[kQuarter];        // home u_x, u_y, u_z, slot
    uint2 q[Q + 64];           // ring of accepted pairs: (home index in the quarter, candidate slot),
                               // then one spare entry per lane for the stores of rejected pairs
    int32_t rlo[32], rex[32];  // non-empty candidate ranges of the cell: first slot, offset in the list
    int32_t flag[64];          // range starts inside the current 64-slot window
};

// The state gathered into `nxt` goes back to `cur`; the new reference
// positions are the current ones (grid-stride from i0).
__device__ __forceinline__ void copy_back(const EvalArgs &a, int64_t i0, int64_t stride) {
    const int64_t n = a.N;
    for (int64_t i = i0; i < n; i += stride) {
        for (int d = 0; d < 3; ++d) {
            a.cur.x[d * n + i] = a.nxt.x[d * n + i];
            a.cur.v[d * n + i] = a.nxt.v[d * n + i];
            a.u_tmp[d * n + i] = a.u[d * n + i];
        }
        if (a.cur.dsp)
            for (int d = 0; d < 3; ++d) a.cur.dsp[d * n + i] = a.nxt.dsp[d * n + i];
        a.cur.q[i] = a.nxt.q[i];
        a.cur.qf[i] = a.nxt.qf[i];
        a.cur.id[i] = a.nxt.id[i];
        a.pk[i] = make_uint4(a.u[i], a.u[n + i], a.u[2 * n + i], __float_as_uint(a.nxt.qf[i]));
        if (a.pkx) a.pkx[i] = PosQ64{a.nxt.x[i], a.nxt.x[n + i], a.nxt.x[2 * n + i], a.nxt.q[i]};
    }
}

// Ring entries [head, head + count), one per lane.
template <bool F64, int Q, bool DBG>
__device__ __forceinline__ void eval_ring(const uint2 *ring, const HomeView<F64> &hv, const Geom &g,
                                          typename CoefOf<F64>::type *co, const uint32_t *__restrict__ su,
                                          const double *__restrict__ sx, const double *__restrict__ sq,
                                          const float *__restrict__ sqf, int64_t n, const float4 *__restrict__ tbl,
                                          float rin2, CSys *csp,  int lane, int head, int count,
                                          double &e) {
    const bool have = lane < count;
    const uint2 qe = have ? ring[(head + lane) & (Q - 1)] : make_uint2(0u, 0u);
    eval_pair<F64, true, DBG>(g, co, hv, su, sx, sq, sqf, n, tbl, rin2, csp, lane, qe, have, e);
}

// Ring entries [head, head + count) appended to the lists of their homes in
// the item's block of the list: the k-th pair of home h is entry
// k * kListHomes + h (column blocks: the list pass reads one row of entries,
// one per home, at a time) or h * rows + k (home-major blocks, for long
// lists).  The entries of one home keep their ring order.
// hcnt: lane h < kQuarter holds the pair count of the wave's home h; entries
// at or beyond `rows` are counted, not stored (the caller flags the
// overflow).  The homes present are taken one at a time (a uniform loop over
// the distinct homes of the 64 entries).
template <int Q>
__device__ __forceinline__ void drain_cols(const uint2 *ring, int head, int count, int lane,
                                           uint32_t *__restrict__ out, int32_t rows, bool hm, int colbase,
                                           int32_t &hcnt) {
    const bool have = lane < count;
    const uint2 qe = have ? ring[(head + lane) & (Q - 1)] : make_uint2(0xffffffffu, 0u);
    int32_t pos = 0;
    uint64_t rem = ballot(have);
    while (rem) {
        const int l0 = (int)__builtin_ctzll(rem);
        const int h = __builtin_amdgcn_readlane((int)qe.x, l0);
        const bool mine = qe.x == (uint32_t)h;
        const uint64_t m = ballot(mine);
        const int32_t c0 = __builtin_amdgcn_readlane(hcnt, h);
        const int32_t r = (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        pos = mine ? c0 + r : pos;
        hcnt = lane == h ? c0 + (int32_t)__popcll(m) : hcnt;
        rem &= ~m;
    }
    if (have && out && pos < rows) {
        // the entry: the byte offset of the candidate's gather record
        const int hcol = colbase + (int)qe.x;
        out[hm ? (int64_t)hcol * rows + pos : (int64_t)pos * kListHomes + hcol] = qe.y << 4;
    }
}

// The build lists, for each home, the candidates within r_l = r_c (1 + skin)
// by the FP32 test, in the column layout of drain_cols; it evaluates no
// forces (the list pass that follows it in the same evaluation does, as on
// every step), so a build step and a list step sum a home's pairs alike.
// out == nullptr (the counting build of the set-up) only counts.
// S: candidate slots per lane and pass (64 S candidates tested per pass)
template <int S>
__global__ __launch_bounds__(64 * kNW) void k_list_build(EvalArgs a, const ListItem *__restrict__ items,
                                                         int32_t nitems, int32_t nblk, int32_t gblk) {
    // the critical path's waves ahead of the structure factor's beside them
    __builtin_amdgcn_s_setprio(2);
    if (!*a.rebuild) return;
    const int64_t n = a.N;  // stride of the structure-of-arrays
    if ((int32_t)blockIdx.x >= gblk) {
        copy_back(a, (int64_t)(blockIdx.x - gblk) * blockDim.x + threadIdx.x, (int64_t)(gridDim.x - gblk) * blockDim.x);
        return;
    }
    constexpr int Q = ring_size(S);
    using Lds = BuildLds<Q>;
    __shared__ Lds lds[kNW];
    __shared__ int32_t wmax[kNW];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    Lds &L = lds[wave];
    const int32_t *__restrict__ start = a.cell_start;
    // the same array for reads at uniform indices (scalar loads)
    CI32 *cstart = (CI32 *)a.cell_start;
    // the build runs on the new reference positions `u` (the current
    // positions in the new order)
    const uint32_t *__restrict__ su = a.u;
    if (blockIdx.x == 0 && threadIdx.x == 0) ++*a.nbuild;
    // one item per virtual block b: blocks are dealt to the 8 XCDs round
    // robin, and b (on XCD b % 8) takes item (b % 8) * (nblk / 8) + b / 8.
    // The gblk blocks launched (a multiple of 8, so that a block stays with
    // its XCD's items) take the nblk virtual ones grid-stride: on the steps
    // that do not build, few blocks return at once.
    for (int32_t b = blockIdx.x; b < nblk; b += gblk) {
    const int32_t it = (b % 8) * (nblk / 8) + b / 8;
    if (it >= nitems) continue;
    {
    const __attribute__((address_space(4))) ListItem *ip = (const __attribute__((address_space(4))) ListItem *)(items + it);
    ListItem item;
    item.sys = ip->sys;
    item.t0 = ip->t0;
    item.t1 = ip->t1;
    const int32_t sys = rfl(item.sys);
    CSys *sp = (CSys *)(a.sys + sys);
    const Geom g = load_geom(sp);
    const int64_t c0s = sp->c0;
    // this wave's quarter of the item's homes: columns [wave kQuarter, ...)
    // of the item's block of the list
    const int32_t t = (int32_t)std::min<int64_t>(item.t0 + wave * kQuarter, item.t1);
    const int32_t t_end = (int32_t)std::min<int64_t>(item.t0 + (wave + 1) * kQuarter, item.t1);
    const int32_t rows = (int32_t)(a.icap / kListHomes);
    uint32_t *out = a.pairs ? a.pairs + (int64_t)it * a.icap : nullptr;
    const int colbase = wave * kQuarter;
    const bool hm = a.list_hm != 0;
    int32_t hcnt = 0;  // lane h < kQuarter: pairs of home h so far
    const bool rel = g.nc[0] >= 4 && g.nc[1] >= 4 && g.nc[2] >= 4;
    if (lane < t_end - t) {
        const int64_t tt = t + lane;
        L.hu[lane] = make_uint4(su[tt], su[n + tt], su[2 * n + tt], (uint32_t)tt);
    }
    wave_sync();
    int qn = 0, qh = 0;  // ring tail (pairs accepted) and head (pairs written)
    for (int64_t cell = t < t_end ? ((CI32 *)a.cell_sorted)[t] : 0; t < t_end; ++cell) {
        const int32_t cs = cstart[cell];
        if (cs >= t_end) break;
        const int32_t ce = cstart[cell + 1];
        const int32_t hs = cs > t ? cs : t;
        const int32_t he = ce < t_end ? ce : t_end;
        if (hs >= he) continue;
        const int i0 = hs - t, i1 = he - t;
        const uint32_t cu32 = (uint32_t)(cell - c0s);
        const int cx = (int)(cu32 % (uint32_t)g.nc[0]);
        const int cy = (int)((cu32 / (uint32_t)g.nc[0]) % (uint32_t)g.nc[1]);
        const int cz = (int)(cu32 / ((uint32_t)g.nc[0] * (uint32_t)g.nc[1]));
        // lane r < 18 holds candidate range r: first sorted index, and its
        // offsets in the flattened candidate list
        int32_t lo = 0, len = 0;
        if (lane < kRanges) {
            int32_t ra_, rb_;
            if (row_range(g, start + c0s, lane, cx, cy, cz, ra_, rb_)) { lo = ra_; len = rb_ - ra_; }
        }
        int32_t incl = len;
        for (int o = 1; o < 32; o <<= 1) {
            const int32_t v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const int32_t excl = incl - len;
        const int32_t C = __builtin_amdgcn_readlane(incl, kRanges - 1);
        // the non-empty ranges, compacted: lane k < nne holds the k-th one's
        // first slot and its offset in the flattened list (offsets strictly
        // increase, the first is 0)
        const bool ne = lane < kRanges && len > 0;
        const uint64_t NE = ballot(ne);
        const int nne = (int)__popcll(NE);
        if (ne) {
            const int k = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(NE >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)NE, 0));
            L.rlo[k] = lo;
            L.rex[k] = excl;
        }
        wave_sync();
        const int32_t clo = lane < nne ? L.rlo[lane < 32 ? lane : 0] : 0;
        const int32_t cex = lane < nne ? L.rex[lane < 32 ? lane : 0] : 0x7fffffff;
        // origin of the cell-relative float coordinates used by the test:
        // the first home of the cell
        const uint4 o4 = L.hu[i0];
        const uint32_t ox = (uint32_t)rfl((int)o4.x), oy = (uint32_t)rfl((int)o4.y), oz = (uint32_t)rfl((int)o4.z);
        for (int32_t cb = 0; cb < C; cb += 64 * S) {
            // candidates of this pass in registers.  For each 64-slot window,
            // the starts of ranges inside it are flagged in LDS; a slot's
            // range is the number of range starts at or before it (those
            // before the window, plus the flagged ones up to its lane) - 1.
            uint32_t cj[S];
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2) {
                const int32_t base = cb + s2 * 64;
                L.flag[lane] = 0;
                wave_sync();
                if (lane < nne && cex >= base && cex < base + 64) L.flag[cex - base] = 1;
                wave_sync();
                const uint64_t B = ballot(L.flag[lane] != 0);
                const int before = (int)__popcll(ballot(lane < nne && cex < base));
                const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
                int k = before + (int)__popcll(B & upto) - 1;
                k = k < 0 ? 0 : k;
                // the permutes read other lanes' registers: the whole wave is active
                cj[s2] = (uint32_t)(__shfl(clo, k, 64) + (base + lane - __shfl(cex, k, 64)));
                wave_sync();
            }
            uint32_t cux[S], cuy[S], cuz[S];
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2) {
                if (cb + s2 * 64 + lane < C) {
                    cux[s2] = su[cj[s2]]; cuy[s2] = su[n + cj[s2]]; cuz[s2] = su[2 * n + cj[s2]];
                } else {
                    cux[s2] = ox; cuy[s2] = oy; cuz[s2] = oz;
                    cj[s2] = kNoCand;
                }
            }
            // relative coordinates: with at least 4 cells per side every
            // candidate lies within 2 cell widths (< L/2) of the origin, so
            // the wrapped difference to the origin is its true offset and
            // differences of relative coordinates are minimum images;
            // smaller grids take the difference of the fixed-point values
            // per pair instead.  Empty slots sit far away.
            float cfx[S], cfy[S], cfz[S];
#pragma unroll
            for (int s2 = 0; s2 < S; ++s2) {
                const bool ok = cj[s2] != kNoCand;
                cfx[s2] = ok ? (float)(int32_t)(cux[s2] - ox) * g.hf[0] : 1e18f;
                cfy[s2] = ok ? (float)(int32_t)(cuy[s2] - oy) * g.hf[1] : 1e18f;
                cfz[s2] = ok ? (float)(int32_t)(cuz[s2] - oz) * g.hf[2] : 1e18f;
            }
            // homes of this cell in groups of 64: lane l holds home g0 + l in
            // registers, homes are broadcast with readlane.  kU homes x S
            // slots are tested independently, then their accepted pairs are
            // appended to the ring, home after home (so one home's pairs of
            // a pass are contiguous).  The home itself is left out.
            // the rel / fixed-point choice is made once, outside the loops
            auto test_homes = [&](auto relc) {
            constexpr bool REL = decltype(relc)::value;
            for (int g0 = i0; g0 < i1; g0 += 64) {
                const int gn = i1 - g0 < 64 ? i1 - g0 : 64;
                const int gi = g0 + lane;
                const uint4 hme = gi < i1 ? L.hu[gi] : make_uint4(ox, oy, oz, 0u);
                const float hfx = (float)(int32_t)(hme.x - ox) * g.hf[0];
                const float hfy = (float)(int32_t)(hme.y - oy) * g.hf[1];
                const float hfz = (float)(int32_t)(hme.z - oz) * g.hf[2];
                for (int ii = 0; ii < gn; ii += kU) {
                    // acceptance as a lane predicate and as the wave's mask,
                    // both from one compare (the home itself and empty slots
                    // are pushed past r_l by their r^2; a home past the
                    // group's end compares against a negative limit)
                    bool acc[kU][S];
                    uint64_t mm[kU][S];
#pragma unroll
                    for (int uu = 0; uu < kU; ++uu) {
                        const bool hok = ii + uu < gn;
                        const int h = hok ? ii + uu : ii;
                        const float lim = hok ? g.rl2_f : -1.0f;
                        const uint32_t self = (uint32_t)(t + g0 + h);
                        if constexpr (REL) {
                            const float hx_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hfx), h));
                            const float hy_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hfy), h));
                            const float hz_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hfz), h));
#pragma unroll
                            for (int s2 = 0; s2 < S; ++s2) {
                                const float dx = cfx[s2] - hx_, dy = cfy[s2] - hy_, dz = cfz[s2] - hz_;
                                const float r2 = dx * dx + dy * dy + dz * dz;
                                const float r2x = cj[s2] == self ? kFarR2 : r2;
                                acc[uu][s2] = r2x < lim;
                                mm[uu][s2] = ballot(r2x < lim);
                            }
                        } else {
                            const uint32_t hux = (uint32_t)__builtin_amdgcn_readlane((int)hme.x, h);
                            const uint32_t huy = (uint32_t)__builtin_amdgcn_readlane((int)hme.y, h);
                            const uint32_t huz = (uint32_t)__builtin_amdgcn_readlane((int)hme.z, h);
#pragma unroll
                            for (int s2 = 0; s2 < S; ++s2) {
                                const float r2 = fixed_r2(g, cux[s2] - hux, cuy[s2] - huy, cuz[s2] - huz);
                                const float r2x = cj[s2] == self || cj[s2] == kNoCand ? kFarR2 : r2;
                                acc[uu][s2] = r2x < lim;
                                mm[uu][s2] = ballot(r2x < lim);
                            }
                        }
                    }
#pragma unroll
                    for (int uu = 0; uu < kU; ++uu) {
#pragma unroll
                        for (int s2 = 0; s2 < S; ++s2) {
                            const uint64_t m = mm[uu][s2];
                            // every lane stores (no branch on the lane mask): a
                            // rejected pair goes to the lane's spare entry
                            const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)qn));
                            L.q[acc[uu][s2] ? (pos & (Q - 1)) : (uint32_t)(Q + lane)] =
                                make_uint2((uint32_t)(g0 + ii + uu), cj[s2]);
                            qn += (int)__popcll(m);
                        }
                    }
                    // at most 63 + kU * S * 64 entries are pending: the ring holds them
                    static_assert(63 + kU * S * 64 < Q, "ring too small");
                    while (qn - qh >= 64) {
                        wave_sync();
                        drain_cols<Q>(L.q, qh, 64, lane, out, rows, hm, colbase, hcnt);
                        qh += 64;
                    }
                }
            }
            };
            if (rel) test_homes(std::true_type{});
            else test_homes(std::false_type{});
        }
    }
    wave_sync();
    if (qn > qh) drain_cols<Q>(L.q, qh, qn - qh, lane, out, rows, hm, colbase, hcnt);
    // the counts (capped at the rows stored), the largest of the block to the
    // context's maximum (one atomic per block) and an overflow flag
    const int nh = t_end - t;
    if (lane < nh) a.pcnt[(int64_t)it * kListHomes + colbase + lane] = hcnt < rows || !out ? hcnt : rows;
    int32_t mx = lane < nh ? hcnt : 0;
    for (int o = 8; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) wmax[wave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t bm = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
        atomicMax(a.pmax, bm);
        if (out && bm > rows) atomicOr(a.flag, 8);
    }
    // the next item reuses the LDS of the waves and wmax
    __syncthreads();
    }
    }
}

// List pass: one block per item; runs at every evaluation with the near
// list, a build's included.  Column blocks: one lane per home (lane h holds
// home h of the item in registers), wave w evaluating rows w, w + 4, ... of
// the item's columns (row k holds the k-th listed pair of every home); each
// lane sums its home's pairs in registers, and the four waves' sums are added
// in a fixed order.  Home-major blocks: see below.
template <bool F64, bool HM, bool DBG = false>
__global__ __launch_bounds__(64 * kNW) void k_near_list(EvalArgs a, const ListItem *__restrict__ items,
                                                        int32_t nitems, int32_t nblk) {
    // the critical path's waves ahead of the structure factor's beside them
    __builtin_amdgcn_s_setprio(2);
    using R = typename std::conditional<F64, double, float>::type;
    __shared__ R pf[kNW][3][kListHomes];
    __shared__ double es_w[kNW];
    __shared__ PairRec rec;
    if constexpr (DBG) {
        if (threadIdx.x == 0) {
            rec = PairRec{a.cur.id, a.dbg_pairs, a.dbg_cnt, a.dbg_cap};
            if (blockIdx.x == 0) atomicOr(a.dbg_kind, 2);
        }
        __syncthreads();
    }
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t n = a.N;
    const uint32_t *__restrict__ su = a.u_tmp;
    const double *__restrict__ sx = a.cur.x;
    const double *__restrict__ sq = a.cur.q;
    const float *__restrict__ sqf = a.cur.qf;
    // one item per block, dealt to the XCDs as in the build
    const int32_t b = blockIdx.x;
    const int32_t it = (b % 8) * (nblk / 8) + b / 8;
    // the far kernel that follows opens the next step and sets the flag: the
    // list build, its last reader in this evaluation, has run
    if (a.fuse && b == 0 && threadIdx.x == 0) *a.rebuild = 0;
    if (it >= nitems) return;
    const __attribute__((address_space(4))) ListItem *ip = (const __attribute__((address_space(4))) ListItem *)(items + it);
    ListItem item;
    item.sys = ip->sys;
    item.t0 = ip->t0;
    item.t1 = ip->t1;
    const int32_t sys = rfl(item.sys);
    CSys *sp = (CSys *)(a.sys + sys);
    const Geom g = load_geom(sp);
    typename CoefOf<F64>::type *co;
    if constexpr (F64) co = &sp->co64;
    else co = &sp->co32;
    const float4 *tbl = F64 ? nullptr : sp->tbl;
    const float rin2 = sp->rin2;
    CSys *csp = sp;  // the core-shell Taylor constants are read where used
    const bool we = a.energy != 0;
    const int64_t t0 = item.t0;
    const int H = (int)(item.t1 - t0);
    const int32_t rlast = (int32_t)(a.icap / kListHomes) - 1;
    double e = 0.0;
    if constexpr (HM) {
        // home-major blocks (long lists): wave w takes homes w, w + kNW, ...
        // of the item one at a time, its lanes on 64 consecutive entries of
        // the home's list (neighbouring candidates: the gathers stay local);
        // the next chunk's entries and data are loaded while one is
        // evaluated; each home's sums close with a fixed-order wave sum
        for (int hh = w; hh < H; hh += kNW) {
            const int64_t th = t0 + hh;
            HomeData<F64> hd;
            hd.u[0] = su[th]; hd.u[1] = su[n + th]; hd.u[2] = su[2 * n + th];
            hd.slot = (uint32_t)th;
            if constexpr (F64) {
                hd.q = sq[th];
                hd.x[0] = sx[th]; hd.x[1] = sx[n + th]; hd.x[2] = sx[2 * n + th];
            } else {
                hd.q = sqf[th];
            }
            const int32_t cnt = ((CI32 *)a.pcnt)[(int64_t)it * kListHomes + hh];
            // the home's block of the list (a uniform base; 32-bit offsets)
            const char *__restrict__ rowp =
                (const char *)(a.pairs + (int64_t)it * a.icap + (int64_t)hh * (rlast + 1));
            auto entry = [&](int32_t r) -> uint32_t {
                const uint32_t v = *(const uint32_t *)(rowp + (uint32_t)(min(r, rlast) * 4));
                return r < cnt ? v : 0u;
            };
            R fx = 0, fy = 0, fz = 0;
            // the entries two chunks ahead and the candidates' data of the
            // next chunk are loaded while one chunk is evaluated
            uint32_t e1 = entry(lane), e2 = entry(64 + lane);
            PairData<F64> pd = load_packed<F64>(a.pk, a.pkx, e1);
            for (int32_t c = 0; c < cnt; c += 64) {
                const bool have = c + lane < cnt;
                const uint32_t cj = e1 >> 4;  // the slot (pair records of debug launches)
                const PairData<F64> cur = pd;
                e1 = e2;
                e2 = entry(c + 128 + lane);
                pd = load_packed<F64>(a.pk, a.pkx, e1);
                R px, py, pz;
                double de;
                pair_force<F64, false, DBG>(g, co, hd, we, DBG ? &rec : nullptr, tbl, rin2, csp, cj, have, cur, px,
                                            py, pz, de);
                fx += px; fy += py; fz += pz;
                if (we) {
                    asm volatile("");
                    e += de;
                }
            }
            fx = wave_sum(fx);
            fy = wave_sum(fy);
            fz = wave_sum(fz);
            if (lane == 0) {
                a.Fn[th] = (double)fx;
                a.Fn[n + th] = (double)fy;
                a.Fn[2 * n + th] = (double)fz;
            }
        }
        const double es = wave_sum(e);
        if (lane == 0) es_w[w] = es;
        __syncthreads();
    } else {
    const bool home = lane < H;
    const int64_t tt = t0 + (home ? lane : 0);
    HomeData<F64> hd;
    hd.u[0] = su[tt]; hd.u[1] = su[n + tt]; hd.u[2] = su[2 * n + tt];
    hd.slot = (uint32_t)tt;
    if constexpr (F64) {
        hd.q = sq[tt];
        hd.x[0] = sx[tt]; hd.x[1] = sx[n + tt]; hd.x[2] = sx[2 * n + tt];
    } else {
        hd.q = sqf[tt];
    }
    const int32_t cnt = home ? a.pcnt[(int64_t)it * kListHomes + lane] : 0;
    int32_t mc = cnt;
    for (int o = 32; o > 0; o >>= 1) mc = max(mc, __shfl_xor(mc, o, 64));
    const int32_t maxcnt = rfl(mc);
    // this lane's column; rows past the stored ones are read as the last
    // stored row and not used (loads without a branch)
    const char *__restrict__ blk = (const char *)(a.pairs + (int64_t)it * a.icap);
    auto entry = [&](int32_t r) -> uint32_t {
        const uint32_t v = *(const uint32_t *)(blk + (uint32_t)((min(r, rlast) * kListHomes + lane) * 4));
        return r < cnt ? v : 0u;
    };
    R fx = 0, fy = 0, fz = 0;
    // rows w, w + kNW, ...: the entries two rows ahead and the candidate's
    // data of the next row are loaded while this one is evaluated
    int32_t k = w;
    uint32_t e1 = entry(k), e2 = entry(k + kNW);
    PairData<F64> pd = load_packed<F64>(a.pk, a.pkx, e1);
    for (; k < maxcnt; k += kNW) {
        const bool have = k < cnt;
        const uint32_t cj = e1 >> 4;  // the slot (pair records of debug launches)
        const PairData<F64> cur = pd;
        e1 = e2;
        e2 = entry(k + 2 * kNW);
        pd = load_packed<F64>(a.pk, a.pkx, e1);
        R px, py, pz;
        double de;
        pair_force<F64, false, DBG>(g, co, hd, we, DBG ? &rec : nullptr, tbl, rin2, csp, cj, have, cur, px, py, pz,
                                    de);
        fx += px; fy += py; fz += pz;
        if (we) {
            asm volatile("");
            e += de;
        }
    }
    pf[w][0][lane] = fx;
    pf[w][1][lane] = fy;
    pf[w][2][lane] = fz;
    const double es = wave_sum(e);
    if (lane == 0) es_w[w] = es;
    __syncthreads();
    if (w == 0 && home) {
        for (int d = 0; d < 3; ++d)
            a.Fn[d * n + tt] = (((double)pf[0][d][lane] + (double)pf[1][d][lane]) + (double)pf[2][d][lane]) +
                               (double)pf[3][d][lane];
    }
    }
    if (threadIdx.x == 0) a.epart[it] = ((es_w[0] + es_w[1]) + es_w[2]) + es_w[3];
}

template <bool F64>
struct NearLds {
    using R = typename std::conditional<F64, double, float>::type;
    static constexpr int HC = 64;                // home particles staged per batch
    static constexpr int XH = F64 ? HC : 1;
    uint4 hu[HC];          // home u_x, u_y, u_z, slot
    R hq[HC];
    double hx[3][XH];
    R hf[3][HC];           // force accumulators of the home batch
    uint2 q[512 + 64];     // ring of queued pairs: (home index in the batch, candidate slot),
                           // then one spare entry per lane for the stores of rejected pairs
    int32_t rlo[32], rex[32];  // non-empty candidate ranges of the cell: first slot, offset in the list
    uint32_t flag4[64];        // byte flags: range starts in a pass's (up to 4) 64-slot windows
};

// Steps that build at every evaluation (skin 0) need no list: this kernel
// finds the pairs and evaluates them in one pass, one wave per run of cells
// (cells r_c wide), the pair ring evaluated 64 entries at a time.  Where a
// row has at least 6 cells, two neighbouring home cells share one candidate
// set (their 4 x 3 x 3 stencil), which halves the candidate set-up per home.
// S: candidate slots per lane and pass.  Blocks past nblk copy the gathered
// state back into `cur`.
template <bool F64, int S, bool DBG = false>
__global__ __launch_bounds__(64 * kNW) void k_near_cells(EvalArgs a, const NearItem *__restrict__ items,
                                                         int32_t nitems, int32_t nblk) {
    // the critical path's waves ahead of the structure factor's beside them
    __builtin_amdgcn_s_setprio(2);
    if (!*a.rebuild) return;
    __shared__ PairRec rec;
    if constexpr (DBG) {
        if (threadIdx.x == 0) {
            rec = PairRec{a.nxt.id, a.dbg_pairs, a.dbg_cnt, a.dbg_cap};
            if (blockIdx.x == 0) atomicOr(a.dbg_kind, 4);
        }
        __syncthreads();
    }
    if ((int32_t)blockIdx.x >= nblk) {
        copy_back(a, (int64_t)(blockIdx.x - nblk) * blockDim.x + threadIdx.x, (int64_t)(gridDim.x - nblk) * blockDim.x);
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ++*a.nbuild;
    using Lds = NearLds<F64>;
    using R = typename Lds::R;
    constexpr int Q = 512;
    __shared__ Lds lds[kNW];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    Lds &L = lds[wave];
    const int64_t n = a.N;  // stride of the structure-of-arrays
    const int32_t *__restrict__ start = a.cell_start;
    // the same array for reads at uniform indices (scalar loads)
    CI32 *cstart = (CI32 *)a.cell_start;
    const uint32_t *__restrict__ su = a.u;
    const double *__restrict__ sx = a.nxt.x;
    const double *__restrict__ sq = a.nxt.q;
    const float *__restrict__ sqf = a.nxt.qf;
    double *__restrict__ Fn = a.Fn;
    HomeView<F64> hv;
    hv.hu = L.hu;
    hv.hq = L.hq;
    hv.we = a.energy != 0;
    hv.rec = DBG ? &rec : nullptr;
    for (int d = 0; d < 3; ++d) {
        hv.hx[d] = L.hx[d];
        hv.hf[d] = L.hf[d];
    }
    // blocks are dealt to the 8 XCDs round robin: block b (on XCD b % 8) takes
    // chunk (b % 8) * (nblk / 8) + b / 8 of the item list, so each XCD sweeps
    // one slab of cells
    const int32_t b = blockIdx.x;
    const int32_t chunk = (b % 8) * (nblk / 8) + b / 8;
    for (int32_t it = chunk * kNW + wave; it < nitems; it += nblk * kNW) {
    const __attribute__((address_space(4))) NearItem *ip = (const __attribute__((address_space(4))) NearItem *)(items + it);
    NearItem item;
    item.sys = ip->sys;
    item.c_begin = ip->c_begin;
    item.c_end = ip->c_end;
    const int32_t sys = rfl(item.sys);
    CSys *sp = (CSys *)(a.sys + sys);
    const Geom g = load_geom(sp);
    typename CoefOf<F64>::type *co;
    if constexpr (F64) co = &sp->co64;
    else co = &sp->co32;
    const int64_t c0s = sp->c0;
    const float4 *tbl = F64 ? nullptr : sp->tbl;
    const float rin2 = sp->rin2;
    CSys *csp = sp;  // the core-shell Taylor constants are read where used
    const int64_t ra = item.c_begin, rb = item.c_end;
    double e = 0.0;
    int qn = 0, qh = 0;  // ring tail (pairs queued) and head (pairs evaluated)
    int32_t t = ra < rb ? cstart[ra] : 0;
    const int32_t t_hi = ra < rb ? cstart[rb] : 0;
    int64_t cur = ra;  // cell containing home t
    const bool rel = g.nc[0] >= 4 && g.nc[1] >= 4 && g.nc[2] >= 4;
    while (t < t_hi) {
        // stage a batch of up to HC consecutive homes (all loads first)
        const int32_t t_end = t + Lds::HC < t_hi ? t + Lds::HC : t_hi;
        const int H = t_end - t;
        {
            constexpr int SH = Lds::HC / 64;
            uint32_t vx[SH], vy[SH], vz[SH];
            R vq[SH];
            double wx[SH], wy[SH], wz[SH];
#pragma unroll
            for (int s2 = 0; s2 < SH; ++s2) {
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
            for (int s2 = 0; s2 < SH; ++s2) {
                const int k = s2 * 64 + lane;
                if (k < H) {
                    L.hu[k] = make_uint4(vx[s2], vy[s2], vz[s2], (uint32_t)(t + k));
                    L.hq[k] = vq[s2];
                    if constexpr (F64) { L.hx[0][k] = wx[s2]; L.hx[1][k] = wy[s2]; L.hx[2][k] = wz[s2]; }
                    L.hf[0][k] = 0; L.hf[1][k] = 0; L.hf[2][k] = 0;
                }
            }
        }
        wave_sync();
        while (cstart[cur + 1] <= t) ++cur;
        const bool pairs = g.nc[0] >= 6;
        int w = 1;
        for (int64_t cell = cur; cell < rb; cell += w) {
            const uint32_t cu32 = (uint32_t)(cell - c0s);
            const int cx = (int)(cu32 % (uint32_t)g.nc[0]);
            const int cy = (int)((cu32 / (uint32_t)g.nc[0]) % (uint32_t)g.nc[1]);
            const int cz = (int)(cu32 / ((uint32_t)g.nc[0] * (uint32_t)g.nc[1]));
            // home cells cx (and cx + 1 in the same row and item)
            w = pairs && cx + 1 < g.nc[0] && cell + 1 < rb ? 2 : 1;
            const int32_t cs = cstart[cell];
            if (cs >= t_end) break;
            const int32_t ce = cstart[cell + w];
            const int32_t hs = cs > t ? cs : t;
            const int32_t he = ce < t_end ? ce : t_end;
            if (hs >= he) continue;
            const int i0 = hs - t, i1 = he - t;
            // lane r < 18 holds candidate range r: first sorted index, and its
            // offsets in the flattened candidate list
            int32_t lo = 0, len = 0;
            if (lane < kRanges) {
                int32_t ra_, rb_;
                if (row_range_w(g, start + c0s, lane, cx, cy, cz, w, ra_, rb_)) { lo = ra_; len = rb_ - ra_; }
            }
            const int32_t incl = incl_scan32(len);
            const int32_t excl = incl - len;
            const int32_t C = __builtin_amdgcn_readlane(incl, kRanges - 1);
            // the non-empty ranges, compacted: lane k < nne holds the k-th one's
            // first slot and its offset in the flattened list (offsets strictly
            // increase, the first is 0)
            const bool ne = lane < kRanges && len > 0;
            const uint64_t NE = ballot(ne);
            const int nne = (int)__popcll(NE);
            if (ne) {
                const int k = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(NE >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)NE, 0));
                L.rlo[k] = lo;
                L.rex[k] = excl;
            }
            wave_sync();
            const int32_t cex = lane < nne ? L.rex[lane < 32 ? lane : 0] : 0x7fffffff;
            // slot of the range's first candidate minus its offset in the list
            const int32_t cdl = lane < nne ? L.rlo[lane < 32 ? lane : 0] - cex : 0;
            // origin of the cell-relative float coordinates used by the test:
            // the first home of the cell
            const uint4 o4 = L.hu[i0];
            const uint32_t ox = (uint32_t)rfl((int)o4.x), oy = (uint32_t)rfl((int)o4.y),
                           oz = (uint32_t)rfl((int)o4.z);
            for (int32_t cb = 0; cb < C; cb += 64 * S) {
                // candidates of this pass in registers.  The starts of ranges
                // inside the pass's S windows of 64 slots are flagged in LDS
                // (one byte per slot); a slot's range is the number of range
                // starts at or before it (those before the pass, those of the
                // earlier windows, and the flagged ones up to its lane) - 1.
                static_assert(S <= 4, "byte flags for at most four windows");
                uint32_t cj[S];
                uint8_t *flag = (uint8_t *)L.flag4;
                L.flag4[lane] = 0u;
                wave_sync();
                if (lane < nne && cex >= cb && cex < cb + 64 * S) flag[cex - cb] = 1;
                wave_sync();
                int before = (int)__popcll(ballot(lane < nne && cex < cb));
                const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2) {
                    const uint64_t B = ballot(flag[s2 * 64 + lane] != 0);
                    int k = before + (int)__popcll(B & upto) - 1;
                    k = k < 0 ? 0 : k;
                    before += (int)__popcll(B);
                    // the permute reads other lanes' registers: the whole wave is active
                    cj[s2] = (uint32_t)(__shfl(cdl, k, 64) + (cb + s2 * 64 + lane));
                }
                wave_sync();
                uint32_t cux[S], cuy[S], cuz[S];
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2) {
                    if (cb + s2 * 64 + lane < C) {
                        cux[s2] = su[cj[s2]]; cuy[s2] = su[n + cj[s2]]; cuz[s2] = su[2 * n + cj[s2]];
                    } else {
                        cux[s2] = ox; cuy[s2] = oy; cuz[s2] = oz;
                        cj[s2] = kNoCand;
                    }
                }
                // relative coordinates: with at least 4 cells per side every
                // candidate lies within 2 cell widths (< L/2) of the origin, so
                // the wrapped difference to the origin is its true offset and
                // differences of relative coordinates are minimum images;
                // smaller grids take the difference of the fixed-point values
                // per pair instead.  Empty slots sit far away.
                float cfx[S], cfy[S], cfz[S];
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2) {
                    const bool ok = cj[s2] != kNoCand;
                    cfx[s2] = ok ? (float)(int32_t)(cux[s2] - ox) * g.hf[0] : 1e18f;
                    cfy[s2] = ok ? (float)(int32_t)(cuy[s2] - oy) * g.hf[1] : 1e18f;
                    cfz[s2] = ok ? (float)(int32_t)(cuz[s2] - oz) * g.hf[2] : 1e18f;
                }
                // homes of this cell in groups of 64: lane l holds home g0 + l in
                // registers, homes are broadcast with readlane.  The test admits
                // every pair below the upper band edge (the pair rule, and the
                // exclusion of the home itself, are applied when the pair is
                // evaluated).  kU homes x S slots are tested independently, then
                // their accepted pairs are appended to the ring, home after home.
                // the rel / fixed-point choice is made once, outside the loops
                auto test_homes = [&](auto relc) {
                constexpr bool REL = decltype(relc)::value;
                for (int g0 = i0; g0 < i1; g0 += 64) {
                    const int gn = i1 - g0 < 64 ? i1 - g0 : 64;
                    const int gi = g0 + lane;
                    const uint4 hme = gi < i1 ? L.hu[gi] : make_uint4(ox, oy, oz, 0u);
                    const float hfx = (float)(int32_t)(hme.x - ox) * g.hf[0];
                    const float hfy = (float)(int32_t)(hme.y - oy) * g.hf[1];
                    const float hfz = (float)(int32_t)(hme.z - oz) * g.hf[2];
                    for (int ii = 0; ii < gn; ii += kU) {
                        // acceptance of each (home, slot) as a lane predicate
                        // and as the wave's mask: both come from one compare
                        // (the empty slots are pushed past the band by their
                        // r^2; a home past the group's end compares against a
                        // negative limit; the home itself is admitted)
                        bool acc[kU][S];
                        uint64_t mm[kU][S];
#pragma unroll
                        for (int uu = 0; uu < kU; ++uu) {
                            const bool hok = ii + uu < gn;
                            const int h = hok ? ii + uu : ii;
                            const float lim = hok ? g.band_hi_f : -1.0f;
                            if constexpr (REL) {
                                const float hx_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hfx), h));
                                const float hy_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hfy), h));
                                const float hz_ = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hfz), h));
#pragma unroll
                                for (int s2 = 0; s2 < S; ++s2) {
                                    const float dx = cfx[s2] - hx_, dy = cfy[s2] - hy_, dz = cfz[s2] - hz_;
                                    const float r2 = dx * dx + dy * dy + dz * dz;
                                    acc[uu][s2] = r2 < lim;
                                    mm[uu][s2] = ballot(r2 < lim);
                                }
                            } else {
                                const uint32_t hux = (uint32_t)__builtin_amdgcn_readlane((int)hme.x, h);
                                const uint32_t huy = (uint32_t)__builtin_amdgcn_readlane((int)hme.y, h);
                                const uint32_t huz = (uint32_t)__builtin_amdgcn_readlane((int)hme.z, h);
#pragma unroll
                                for (int s2 = 0; s2 < S; ++s2) {
                                    const float r2 = fixed_r2(g, cux[s2] - hux, cuy[s2] - huy, cuz[s2] - huz);
                                    const float r2x = cj[s2] == kNoCand ? kFarR2 : r2;
                                    acc[uu][s2] = r2x < lim;
                                    mm[uu][s2] = ballot(r2x < lim);
                                }
                            }
                        }
#pragma unroll
                        for (int uu = 0; uu < kU; ++uu) {
#pragma unroll
                            for (int s2 = 0; s2 < S; ++s2) {
                                const uint64_t m = mm[uu][s2];
                                // every lane stores (no branch on the lane mask): a
                                // rejected pair goes to the lane's spare entry
                                const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
                                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, (uint32_t)qn));
                                L.q[acc[uu][s2] ? (pos & (Q - 1)) : (uint32_t)(Q + lane)] =
                                    make_uint2((uint32_t)(g0 + ii + uu), cj[s2]);
                                qn += (int)__popcll(m);
                            }
                        }
                        // at most 63 + kU * S * 64 entries are pending: the ring holds them
                        static_assert(63 + kU * S * 64 < Q, "ring too small");
                        while (qn - qh >= 64) {
                            wave_sync();
                            eval_ring<F64, Q, DBG>(L.q, hv, g, co, su, sx, sq, sqf, n, tbl, rin2, csp, lane, qh, 64, e);
                            qh += 64;
                        }
                    }
                }
                };
                if (rel) test_homes(std::true_type{});
                else test_homes(std::false_type{});
            }
        }
        // the queue refers to this batch's home slots: drain it, then write
        wave_sync();
        if (qn > qh) eval_ring<F64, Q, DBG>(L.q, hv, g, co, su, sx, sq, sqf, n, tbl, rin2, csp, lane, qh, qn - qh, e);
        qn = 0;
        qh = 0;
        wave_sync();
        for (int k = lane; k < H; k += 64) {
            const int64_t tt = t + k;
            Fn[tt] = (double)L.hf[0][k]; Fn[n + tt] = (double)L.hf[1][k]; Fn[2 * n + tt] = (double)L.hf[2][k];
        }
        wave_sync();
        t = t_end;
    }
    const double es = wave_sum(e);
    if (lane == 0) a.epart_cells[it] = es;
    }
}

// Debug export of the neighbour list of one system with exactly the pair rule
// of the near kernel, at the current positions.  Candidates come from the
// cells of the latest list build, which hold every particle within r_c of the
// home while the list is valid.  Rows and columns are local ids (id - first
// id of the system).
template <bool FILL>
__global__ void k_neighbors(EvalArgs a, int32_t sys, int64_t nloc, int64_t p0, const int32_t *__restrict__ idc,
                            int64_t *__restrict__ counts, const int64_t *__restrict__ row_ptr,
                            int32_t *__restrict__ cols) {
    const int64_t N = a.N;
    const int64_t tl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tl >= nloc) return;
    const SysDev &sd = a.sys[sys];
    const Geom &g = sd.g;
    const int32_t *start = a.cell_start + sd.c0;
    const uint32_t *su = a.u_tmp;
    const int64_t t = p0 + tl;
    const uint32_t ux = su[t], uy = su[N + t], uz = su[2 * N + t];
    const uint32_t cu32 = (uint32_t)(a.cell_sorted[t] - sd.c0);
    const int cx = (int)(cu32 % (uint32_t)g.nc[0]);
    const int cy = (int)((cu32 / (uint32_t)g.nc[0]) % (uint32_t)g.nc[1]);
    const int cz = (int)(cu32 / ((uint32_t)g.nc[0] * (uint32_t)g.nc[1]));
    const int64_t id = idc[t] - p0;
    int64_t cnt = 0;
    const int64_t base = FILL ? row_ptr[id] : 0;
    for (int r = 0; r < kRanges; ++r) {
        int32_t lo, hi;
        if (!row_range(g, start, r, cx, cy, cz, lo, hi)) continue;
        for (int32_t j = lo; j < hi; ++j) {
            if (j == t) continue;
            if (!decide(g, su[j] - ux, su[N + j] - uy, su[2 * N + j] - uz)) continue;
            if (FILL) cols[base + cnt] = (int32_t)(idc[j] - p0);
            ++cnt;
        }
    }
    if (!FILL) {
        counts[id] = cnt;
    } else {
        for (int64_t x = base + 1; x < base + cnt; ++x) {
            const int32_t v = cols[x];
            int64_t y = x - 1;
            while (y >= base && cols[y] > v) {
                cols[y + 1] = cols[y];
                --y;
            }
            cols[y + 1] = v;
        }
    }
}

void list_build_launch(const EvalArgs &a, int32_t slots, dim3 grid, dim3 block, const ListItem *items,
                       int32_t nitems, int32_t nblk, int32_t gblk, hipStream_t s) {
    if (slots <= 2) hipLaunchKernelGGL((k_list_build<2>), grid, block, 0, s, a, items, nitems, nblk, gblk);
    else if (slots == 3) hipLaunchKernelGGL((k_list_build<3>), grid, block, 0, s, a, items, nitems, nblk, gblk);
    else hipLaunchKernelGGL((k_list_build<4>), grid, block, 0, s, a, items, nitems, nblk, gblk);
}

template <bool DBG>
void near_cells_launch(const EvalArgs &a, bool f64, int32_t slots, dim3 grid, dim3 block, const NearItem *items,
                       int32_t nitems, int32_t nblk, hipStream_t s) {
    if (f64) {
        if (slots <= 2) hipLaunchKernelGGL((k_near_cells<true, 2, DBG>), grid, block, 0, s, a, items, nitems, nblk);
        else hipLaunchKernelGGL((k_near_cells<true, 3, DBG>), grid, block, 0, s, a, items, nitems, nblk);
    } else {
        if (slots <= 2) hipLaunchKernelGGL((k_near_cells<false, 2, DBG>), grid, block, 0, s, a, items, nitems, nblk);
        else hipLaunchKernelGGL((k_near_cells<false, 3, DBG>), grid, block, 0, s, a, items, nitems, nblk);
    }
}

}  // namespace

void launch_list_build(const EvalArgs &a, bool f64, const ListItem *items, int32_t nitems, int32_t slots,
                       hipStream_t s, bool copy_back) {
    // one item per virtual block (a wave per quarter); a multiple of 8 so
    // that the XCD mapping is a permutation of the blocks; at most kBuildBlocks
    // launched (grid-stride), then the blocks of the copy back
    constexpr int32_t kBuildBlocks = 4096;
    int32_t nblk = (nitems + 7) / 8 * 8;
    if (nblk < 8) nblk = 8;
    const int32_t gblk = std::min(nblk, kBuildBlocks);
    const int64_t ncopy = copy_back ? std::min<int64_t>(1024, std::max<int64_t>(1, grid_for(a.N, 64 * kNW))) : 0;
    const dim3 grid((unsigned)(gblk + ncopy)), block(64 * kNW);
    (void)f64;  // the build's test is the same in both precisions
    list_build_launch(a, slots, grid, block, items, nitems, nblk, gblk, s);
}

void launch_near_cells(const EvalArgs &a, bool f64, const NearItem *items, int32_t nitems, int32_t slots,
                       hipStream_t s) {
    // one item per wave; a multiple of 8 blocks so that the XCD mapping is a
    // permutation of the blocks; then the blocks of the copy back
    int32_t nblk = (nitems + kNW - 1) / kNW;
    nblk = (nblk + 7) / 8 * 8;
    if (nblk < 8) nblk = 8;
    const int64_t ncopy = std::min<int64_t>(1024, std::max<int64_t>(1, grid_for(a.N, 64 * kNW)));
    const dim3 grid((unsigned)(nblk + ncopy)), block(64 * kNW);
    if (a.dbg_pairs) near_cells_launch<true>(a, f64, slots, grid, block, items, nitems, nblk, s);
    else near_cells_launch<false>(a, f64, slots, grid, block, items, nitems, nblk, s);
}

void launch_near(const EvalArgs &a, bool f64, const ListItem *items, int32_t nitems, hipStream_t s) {
    // one item per block
    int32_t nblk = (nitems + 7) / 8 * 8;
    if (nblk < 8) nblk = 8;
    dim3 grid((unsigned)nblk), block(64 * kNW);
    // one instantiation per layout: each keeps its own register budget
    auto go = [&](auto f64c, auto hmc, auto dbgc) {
        hipLaunchKernelGGL((k_near_list<decltype(f64c)::value, decltype(hmc)::value, decltype(dbgc)::value>), grid,
                           block, 0, s, a, items, nitems, nblk);
    };
    auto by_hm = [&](auto f64c, auto dbgc) {
        if (a.list_hm) go(f64c, std::true_type{}, dbgc);
        else go(f64c, std::false_type{}, dbgc);
    };
    auto by_f64 = [&](auto dbgc) {
        if (f64) by_hm(std::true_type{}, dbgc);
        else by_hm(std::false_type{}, dbgc);
    };
    if (a.dbg_pairs) by_f64(std::true_type{});
    else by_f64(std::false_type{});
}

void launch_neighbor_count(const EvalArgs &a, int32_t sys, int64_t n, int64_t p0, const int32_t *id_cur,
                           int64_t *counts, hipStream_t s) {
    hipLaunchKernelGGL(k_neighbors<false>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, a, sys, n, p0, id_cur,
                       counts, (const int64_t *)nullptr, (int32_t *)nullptr);
}

void launch_neighbor_fill(const EvalArgs &a, int32_t sys, int64_t n, int64_t p0, const int32_t *id_cur,
                          const int64_t *row_ptr, int32_t *cols, hipStream_t s) {
    hipLaunchKernelGGL(k_neighbors<true>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, a, sys, n, p0, id_cur,
                       (int64_t *)nullptr, row_ptr, cols);
}

}  // namespace rbsog
