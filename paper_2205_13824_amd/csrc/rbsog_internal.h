// Internal declarations shared by the host side (capi.hip) and the kernels
// (kernels_*.hip) of librbsog.  Not part of the public ABI.
//
// A context holds a batch of S >= 1 independent periodic systems.  Device
// arrays concatenate the systems: the particles of system s occupy slots
// [p0_s, p0_s + n_s), its cells [c0_s, c0_s + ncell_s) and its wave-vector
// records [k0_s, k0_s + P_s).  Particle state is kept in cell order: each
// force evaluation re-sorts it by (cell, id), id being the particle's index in
// the caller's arrays, so slots of one system stay in that system's range.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rbsog.h"

namespace rbsog {

constexpr int kMaxGauss = 160;  // M + 1 <= kMaxGauss

// Per-k record read uniformly by every lane of the far-force kernel, in
// amplitude-phase form: with rho_e = |rho_e| e^{2 pi i phi_e},
//   Im(e^{-i k.r} rho) = |rho| sin(2 pi (phi - m.s)),  s = r/L (fractional),
// so the far force is F_i = -q_i sum_e a_e sin(2 pi (phi_e - m_e.s_i)) with
// a_e = w_e |rho_e| k_e: one sine per (particle, wave vector).  The
// structure-factor reduction writes the records of the batch (the structure
// factor itself reads m from the sequence at the cursor).
// FP64 form: m as doubles, phi in 1/kTurnTab revolutions (the unit of the
// FP64 phases, rbsog_math.h), a.
struct KRec64 {
    double mx, my, mz;
    double phi;
    double ax, ay, az;
    double pad;
};
// FP32 form: -m as int32 (the far force forms phi + (-m).u), a rounded to
// float, then phi as a 32-bit fixed-point fraction of a turn (mod 2^32):
// the far kernel loads the first 24 bytes as scalars and the phases as
// vectors.
struct KRec32 {
    int32_t nmx, nmy, nmz;
    float ax, ay, az;
    uint32_t phi;
    float pad;
};

// Geometry of one system.
struct Geom {
    int64_t n;
    double L[3], invL[3], h[3];  // h = L * 2^-32
    float hf[3];
    double rc2;                  // rc * rc
    double band_lo, band_hi;     // FP64 r^2 thresholds outside which the fast test decides
    float band_lo_f, band_hi_f;  // same for the FP32 fast test
    int32_t nc[3];               // cells per side: floor(L / (r_c (1 + skin))), or 1 below 3
    int32_t reach[3];            // 1 if the stencil spans -1..1 in that dimension, 0 otherwise
    float rl2_f;                 // FP32 r^2 below which a pair enters the Verlet list (r_c (1 + skin))^2, widened
    float dthr2_f;               // FP32 squared displacement beyond which the list is rebuilt (skin r_c / 2)^2, narrowed
};

// The near kernel evaluates the narrow Gaussians (r_c^2 / s_l^2 > tau) with an
// exponential each and replaces the wide ones (s_l grows with l, so they are
// l >= nexp) by the Taylor polynomial of their sum in x = r^2.  Truncation per
// Gaussian: tau^(deg+1)/(deg+1)! of its weight, 2.4e-18 (FP64) and 1.2e-8
// (FP32).
constexpr double kTailTau64 = 0.25;
constexpr double kTailTau32 = 0.25;
constexpr int kTailDeg64 = 12;
constexpr int kTailDeg32 = 6;
constexpr int kMaxExp = 24;  // narrow Gaussians per split (more is rejected)

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

// Core-shell near kernel (Sec. 3.4), an option of the FP32C form: pairs with
// r < r_in take Q Taylor terms of the Gaussians with 1/r and 1/r^3 computed;
// r_in <= r < r_c take a table indexed by the FP32 bits of r^2 (the low
// kTabBexp exponent bits and the high kTabBman mantissa bits) with linear
// interpolation.  Entry: (g, g_next - g, h, h_next - h) at the table point,
// g = 1/r^3 - 2 sum_l omega_l/s_l^2 e^{-r^2/s_l^2}, h = 1/r - sum_l omega_l e^{-r^2/s_l^2}.
constexpr int kTabQ = 4;
constexpr int kTabBexp = 3;
constexpr int kTabBman = 9;
constexpr int kTabSize = 1 << (kTabBexp + kTabBman);
constexpr double kTabRin = 0.2;  // r_in / r_c

// Per-system constants, one entry per system in a device array.
struct SysDev {
    Geom g;
    SplitCoef64 co64;
    SplitCoef32 co32;
    int64_t p0;           // first particle slot
    int64_t c0;           // first cell
    int32_t P;            // wave vectors per evaluation
    int32_t k0;           // first k record
    const int32_t *kseq;  // the system's wave-vector sequence, 3 int32 per vector
    const double *kw;     // per-vector weights, or null for the random-batch weight
    double w_rb;          // S pi^{3/2} / (P V)
    double uself;         // U_self
    int32_t it0, it1;     // near list items [it0, it1)
    int32_t jt0, jt1;     // near cell-run items [jt0, jt1) (build-every-evaluation mode)
    int64_t pofs;         // first rho partial (complex entries) of the system
    int32_t nch;          // rho particle chunks of the system
    int32_t kt, streams;  // rho block shape: k tiles of 64 lanes x particle streams
    // core-shell near kernel (FP32C option): table, r_in^2, Taylor coefficients
    const float4 *tbl;    // null: direct evaluation
    float rin2;
    float ta[kTabQ];      // sum_l omega_l/s_l^2 (-1)^(i-1)/(i-1)! s_l^(-2(i-1)), i = 1..Q
    float tb[kTabQ];      // sum_l omega_l (-1)^(i-1)/(i-1)! s_l^(-2(i-1))
    // zero-frequency mode (Sec. 3.2): 0 tinfoil, 1 spherical, 2 slab along z;
    // U^0 = zu * |M|^2 (or M_z^2), F_i = zf * q_i M (or M_z e_z)
    int32_t zmode;
    double zu, zf;
    int64_t choff;        // first structure-factor chunk of the system over the batch
    int32_t ft0, ft1;     // far items [ft0, ft1)
    // Nose-Hoover thermostat: degrees of freedom 3n - 3 and thermostat mass N_f T tau^2
    double nh_nf, nh_Q;
};

// Near item of the build-every-evaluation mode: a run of cells of one system.
struct NearItem {
    int32_t sys;
    int32_t pad;
    int64_t c_begin, c_end;
};
// Near list item: up to kListHomes consecutive particle slots [t0, t1) of one
// system (in the cell order of the latest list build).  Its block of the pair
// list is icap entries (rows = icap / kListHomes): the k-th pair of home h
// (slot t0 + h), k < pcnt[item kListHomes + h], is entry k kListHomes + h
// (column blocks) or h rows + k (home-major blocks, for long lists); an
// entry is 16 j for candidate slot j (the byte offset of its gather
// record).  The build writes the lists of its four quarters of homes, one
// wave each.
constexpr int kListHomes = 64;
constexpr int kListWaves = 4;
struct ListItem {
    int32_t sys;
    int32_t pad;
    int64_t t0, t1;
};
// Structure-factor work item: particle slots [j0, j1) of one system against
// the k tiles of group kg; its partials go to chunk `chunk` of the system.
struct RhoItem {
    int32_t sys, kg, chunk, pad;
    int64_t j0, j1;
};
// Far-force work item: particle slots [t0, t1) of one system (<= 256).
struct FarItem {
    int32_t sys, pad;
    int64_t t0, t1;
};

// State arrays.  `cur` holds the state; a list build gathers it into `nxt`
// in the new cell order and copies it back.
struct StateBufs {
    double *x, *v, *q;
    float *qf;
    int32_t *id;
    double *dsp;  // displacement since the mean-square-displacement origin (sum of the drifts)
};
// Slots of a context stay below 2^kListSlotBits (its particle limit): the
// near kernels gather by 32-bit byte offsets (list entries are 16 j) and
// keep a build's ring entries within kListSlotMask.
constexpr int kListSlotBits = 28;
constexpr uint32_t kListSlotMask = (1u << kListSlotBits) - 1u;
constexpr int64_t kMaxParticles = (int64_t)1 << kListSlotBits;

// FP64 position and charge of a slot in one 32-byte record.
struct alignas(32) PosQ64 {
    double x, y, z, q;
};

struct EvalArgs {
    int64_t N;             // particles over all systems
    int64_t C;             // cells over all systems
    int32_t nsys;
    int32_t K;             // k records over all systems
    const SysDev *sys;
    const int32_t *sys_of;  // system of each slot (static)
    const int32_t *ksys;    // system of each k record (static)
    StateBufs cur, nxt;
    uint32_t *u_tmp;       // fixed-point coordinates of the current positions
    uint32_t *u;           // fixed-point coordinates at the latest list build (its reference)
    // copy of the positions and charges taken by the kick/drift kernel for
    // the structure factor, which runs beside the re-sort of the state:
    // fixed-point coordinates and FP32 charges (FP32C), FP64 positions and
    // charges (FP64, or the zero-frequency mode's dipole); null when unused
    uint32_t *rs_u;
    float *rs_qf;
    double *rs_x, *rs_q;
    // what the list pass gathers of a listed candidate, one record per slot
    // in the current order (written by the kick/drift kernel, and in the new
    // order by a build's copy back): fixed-point coordinates with the FP32
    // charge's bits; the FP64 position and charge (FP64 form; else null)
    uint4 *pk;
    PosQ64 *pkx;
    int32_t *cell_of, *cell_count, *cell_start, *cell_fill, *src, *sorted, *blocksums;
    int32_t *skey;         // particle id of each scattered slot (the per-cell sort's key)
    int32_t *cell_sorted;  // cell of each slot at the latest list build
    double *Fn, *Ff;       // forces in slot order
    double *Ff_side;       // build-every-step mode: far forces in the order before the re-sort
    // Verlet list: rebuild flag (set by the displacement check, cleared by the
    // far kernel, or by the list pass when the far kernel opens the next
    // step), pairs (one u32 each: 16 times the candidate's slot, laid out as
    // the near list items state), counts,
    // capacity per item, largest count of the latest build, builds made
    int32_t *rebuild;
    int32_t list_hm;       // nonzero: home-major blocks of the near list (long lists)
    int32_t always_build;  // nonzero: every evaluation builds (no displacement check, no list kept)
    uint32_t *pairs;
    int32_t *pcnt;
    int64_t icap;
    int32_t *pmax;
    int64_t *nbuild;
    int64_t *kcur;         // per-system sequence cursor
    KRec64 *kb64;
    KRec32 *kb32;
    double *rho, *ek, *partial, *epart, *E;
    double *epart_cells;   // near energies per cell-run item (build-every-evaluation mode)
    int32_t energy;        // 1: the near kernels sum the pair energies (else forces only)
    double *dip_part;      // dipole partials per structure-factor chunk (3 per chunk)
    int32_t red_waves;     // waves per k record of the structure factor's reduction (1 or 4)
    double *dipole;        // dipole moment M per system (3 per system)
    int32_t *flag;         // bit 0: non-finite force, bit 1: non-finite energy, bit 3: list overflow
    // debug launches only (null otherwise): the near kernels record every pair
    // they accept as (caller index of the home, of the candidate) at
    // dbg_pairs[atomicAdd(dbg_cnt, 1)] below dbg_cap, and set bit 0 (list
    // build), 1 (list pass) or 2 (fused cell kernel) of *dbg_kind
    uint2 *dbg_pairs;
    int32_t *dbg_cnt;
    int32_t dbg_cap;
    int32_t *dbg_kind;
    uint32_t *sys_done;    // per-system counters of the energy sums' blocks (re-armed to 0)
    uint32_t *bin_done;    // blocks of the bin pass done (its last block scans the counts; re-armed to 0)
    // velocity-Verlet
    int32_t kick;          // nonzero: kick + drift before, kick after
    double hdm, dt;
    double mass;
    // kinetic energy per far item and wave (4 slots per item), and per
    // system after the evaluation; the energy sums' blocks per system
    // (kin_blocks, at most kKinBlocks) and their sums (2 per block)
    double *kpart, *kin;
    double *kin_part;
    int32_t kin_blocks;
    // Nose-Hoover thermostat (nh != 0): xi per system, target temperature
    int32_t nh;
    double nh_T;
    double *nh_xi;
    // Langevin thermostat (BAOAB): half drift, v <- c1 v + c2 xi, half drift
    int32_t thermo;
    double c1, c2;
    uint64_t tseed;
    int64_t *tstep;        // thermostatted steps taken (noise counter)
    // nonzero (plain velocity Verlet on a kept near list): the far kernel
    // also opens the next step (its half kick with the same force, its drift
    // and quantisation, its displacement check), the near list pass clears
    // the rebuild flag in its place, and the next step starts with its
    // structure factor
    int32_t fuse;
};

// Orders a wave's LDS accesses before the barrier against those after it,
// for data exchanged between the lanes of one wave (no block barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wrap of drifted positions into [0, L) (x_w = frac(x/L) L) and their
// fixed-point coordinates u = min(2^32-1, floor(frac(x/L) 2^32)), stored for
// slot t with the copies the structure factor and the near part read (a
// non-finite position, reported by the flag, falls at u = 0).  Returns the
// squared minimum-image displacement from the build's coordinates `uref` in
// FP32 (the wrapped fixed-point difference times hf).  Shared by the
// kick/drift kernel and the far kernel's fused step.
__device__ __forceinline__ float wrap_store(const EvalArgs &a, int64_t t, bool valid, const double xs[3],
                                            const double L[3], const float hf[3], const uint32_t uref[3],
                                            uint32_t uq[3]) {
    constexpr double two32 = 4294967296.0;
    const int64_t N = a.N;
    float d2 = 0.f;
    double xw[3];
    for (int d = 0; d < 3; ++d) {
        const double r = xs[d] / L[d];
        const double f = r - floor(r);
        double w = floor(f * two32);
        w = w >= 0.0 ? (w > two32 - 1.0 ? two32 - 1.0 : w) : 0.0;
        const uint32_t ud = (uint32_t)w;
        uq[d] = ud;
        xw[d] = f * L[d];
        if (valid) {
            a.u_tmp[d * N + t] = ud;
            a.cur.x[d * N + t] = xw[d];
            if (a.rs_u) a.rs_u[d * N + t] = ud;
            if (a.rs_x) a.rs_x[d * N + t] = xw[d];
        }
        const float dd = (float)(int32_t)(ud - uref[d]) * hf[d];
        d2 += dd * dd;
    }
    if (valid) {
        const float qf = a.cur.qf[t];
        const double q = a.cur.q[t];
        if (a.rs_qf) a.rs_qf[t] = qf;
        if (a.rs_q) a.rs_q[t] = q;
        a.pk[t] = make_uint4(uq[0], uq[1], uq[2], __float_as_uint(qf));
        if (a.pkx) a.pkx[t] = PosQ64{xw[0], xw[1], xw[2], q};
    }
    return d2;
}

// ---- on-device sampler (kernels_sample.hip) ---------------------------------
// State of one Metropolis-Hastings chain.
struct ChainState {
    int32_t m[3];
    int32_t started;
    int64_t burn_left;
    uint64_t attempt;
    double p, qprop;
};
// Per-system constants of the chains.
struct SampDev {
    const double *omega, *s;  // split coefficients, G = M + 1 of each
    int32_t G, P;
    double L[3], sd[3], a[3];  // box, proposal standard deviation L/(sqrt(2) pi s_0), pi s_0 / L
    uint64_t seed;
    int32_t *out;             // lambda batches of P vectors (3 int32 each)
};
constexpr int32_t kMaxChains = 4096;
constexpr int32_t kKinBlocks = 64;
// advances every chain of every system by P states and resets the cursors;
// sets bit 4 of *flag if a chain exceeds its attempt limit
void launch_refill(const SampDev *samp, int32_t nsys, int32_t lambda, ChainState *chains, int64_t *kcur,
                   int32_t *flag, hipStream_t s);

// ---- kernel launchers (kernels_md.hip) --------------------------------------
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
// kick dt/2 + drift (if a.kick), wrap, quantise, displacement check against
// the list reference (sets *a.rebuild)
void launch_kdq(const EvalArgs &a, hipStream_t s);
// The list build: each of these returns at once unless *a.rebuild is set.
// Cell of each particle and the histogram, then the exclusive scan of the
// counts (by the bin pass's last block when the cells are few, else by the
// scan kernels); the scan alone (the kick/drift kernel made the histogram);
// scatter into cells; per cell: id sort of its segment, reset of its count,
// gather of the state into `nxt` in the new order
void launch_bin_scan(const EvalArgs &a, hipStream_t s);
void launch_scan(const EvalArgs &a, hipStream_t s);
int64_t scan_blocksums_size(int64_t n);
void launch_cell_scatter(const EvalArgs &a, hipStream_t s);
void launch_sort_gather(const EvalArgs &a, hipStream_t s);
// near and far forces (6 doubles each) of the caller indices ids[0..m) from
// the current order (slot_of: N int32 of scratch for the inverse permutation)
void launch_subset_forces(const EvalArgs &a, int64_t m, const int64_t *ids, int32_t *slot_of, double *out,
                          hipStream_t s);

// ---- near part (kernels_near.hip) ------------------------------------------
// Verlet list of every item (a.pairs null: not written) with this
// evaluation's near forces and energies, and the copy of the gathered state
// back into `cur`; returns at once unless *a.rebuild is set.  slots (2..4):
// candidates per lane and test pass
// copy_back false: the list only (the state stays where it is)
void launch_list_build(const EvalArgs &a, bool f64, const ListItem *items, int32_t nitems, int32_t slots,
                       hipStream_t s, bool copy_back = true);
// build-every-evaluation mode (a.always_build): near forces and energies in
// one pass over cell runs (no list), and the copy back; returns at once
// unless *a.rebuild is set
// slots (2 or 3): candidates per lane and test pass
void launch_near_cells(const EvalArgs &a, bool f64, const NearItem *items, int32_t nitems, int32_t slots,
                       hipStream_t s);
// near forces and energies from the list; returns at once if *a.rebuild is
// set (the build has evaluated them)
void launch_near(const EvalArgs &a, bool f64, const ListItem *items, int32_t nitems, hipStream_t s);
// neighbour list of one system (debug export): counts per local id, then fill
void launch_neighbor_count(const EvalArgs &a, int32_t sys, int64_t n, int64_t p0, const int32_t *id_cur,
                           int64_t *counts, hipStream_t s);
void launch_neighbor_fill(const EvalArgs &a, int32_t sys, int64_t n, int64_t p0, const int32_t *id_cur,
                          const int64_t *row_ptr, int32_t *cols, hipStream_t s);

// ---- far part (kernels_far.hip) --------------------------------------------
void launch_rho(const EvalArgs &a, bool f64, const RhoItem *items, int32_t nitems, hipStream_t s);
// rho_e per record from the partials (fixed order), its records and per-k
// energies; then per system the far energy (with the zero-mode term) and
// the sequence cursor moved on
void launch_rho_reduce(const EvalArgs &a, hipStream_t s);
// far force; with a.kick the closing half kick v += dt/(2m) (F_N + F*) follows
// (items of at most block_size particles, block_size in {64, 128, 256})
void launch_far(const EvalArgs &a, bool f64, const FarItem *items, int32_t nitems, int32_t block_size,
                hipStream_t s);
void launch_far_side(const EvalArgs &a, bool f64, const FarItem *items, int32_t nitems, int32_t block_size,
                     hipStream_t s);
void launch_far_finish(const EvalArgs &a, const FarItem *items, int32_t nitems, int32_t block_size, hipStream_t s);
// per system: U_N and the total U after the near part and U*, the kinetic
// energy from the far kernel's partials, and the second Nose-Hoover half
// step of xi when stepping with that thermostat
void launch_kinetic(const EvalArgs &a, hipStream_t s);
// mean-square displacement of every system since its origin: msd[s] =
// (1/n_s) sum |dsp|^2, fixed order
void launch_msd(const EvalArgs &a, double *msd, hipStream_t s);

}  // namespace rbsog
