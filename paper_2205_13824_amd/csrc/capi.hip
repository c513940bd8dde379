// Host side of librbsog: the C ABI of include/rbsog.h.  Validates inputs,
// builds the split coefficients and the normaliser S of every system, runs
// the wave-vector samplers, builds the work lists of the batch, owns the
// device memory and enqueues the kernels of one force evaluation / one
// velocity-Verlet step of all systems on a single HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rbsog_internal.h"
#include "rbsog_math.h"

using namespace rbsog;

namespace {

// message of the latest failure without a context (a fixed buffer: setting
// it allocates nothing, so the entry points that must not allocate use it too)
thread_local char g_init_error[512] = "";

void set_init_error(const char *msg) {
    std::snprintf(g_init_error, sizeof g_init_error, "%s", msg);
}

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwo32 = 4294967296.0;

// ---------------------------------------------------------------------------
// Metropolis-Hastings independence chain over nonzero m (Sec. 3.3).
struct MHChain {
    bool started = false;
    int64_t burn_left = 100;
    uint64_t attempt = 0;
    int32_t m[3] = {0, 0, 0};
    double p = 0.0, qprop = 0.0;
};

// ---------------------------------------------------------------------------
struct ProfEntry {
    const char *name;
    double ms = 0.0;
    int64_t launches = 0;
};

constexpr int64_t kAdaptSteps = 32;  // steps between checks of the near-list build rate
constexpr int64_t kProbeSteps = 4;   // steps of a renewed try of the caller's skin
constexpr int kGraphSteps = 8;       // steps in the longer step graph
// Step graphs: one step without the near energies, one step with them (the
// last step of a run), kGraphSteps steps without them; and fused steps,
// whose far kernel opens the next step: kGraphSteps or one of them after an
// unfused step (HEAD) or after a fused one (MID), and the unfused step that
// ends their run, without and with the near energies (TAIL)
enum {
    GV_STEP, GV_STEP_E, GV_MULTI, GV_F_HEAD8, GV_F_HEAD1, GV_F_MID8, GV_F_MID1, GV_F_TAIL, GV_F_TAIL_E, GV_COUNT
};
struct GraphShape {
    int len;      // steps
    bool opened;  // the first step was opened by the step before
    bool fused;   // every step opens the next
    bool energy;  // the (single) step sums the near energies
};
constexpr GraphShape kShapes[GV_COUNT] = {
    {1, false, false, false},           {1, false, false, true},          {kGraphSteps, false, false, false},
    {kGraphSteps, false, true, false},  {1, false, true, false},          {kGraphSteps, true, true, false},
    {1, true, true, false},             {1, true, false, false},          {1, true, false, true},
};

enum Kid {
    K_KDQ, K_BIN, K_SCAN, K_SCATTER, K_SORTG, K_LIST, K_NEAR, K_NEARC, K_RHO, K_RHORED, K_FAR, K_SAMPLE, K_FARFIN,
    K_FARSIDE, K_COUNT
};
const char *kKernelNames[K_COUNT] = {"kick_drift_quantise", "bin", "scan_cell_counts", "cell_scatter", "sort_gather",
                                     "list_build", "near", "near_cells", "rho", "rho_reduce", "far",
                                     "sample_refill", "far_finish", "far_side"};


// Launch shapes of the work lists (the tunable part of the plan).
struct Tune {
    int32_t rho_chunk = 0;    // particles per structure-factor chunk
    int32_t far_block = 0;    // particles per far item (= block size)
    int32_t rho_kt = 0;       // k tiles of 64 per structure-factor block (the other waves split the chunk); 0: 16
    int32_t build_slots = 0;  // candidate slots per lane and test pass of the list build (2..4); 0: from occupancy
    int32_t cell_slots = 0;   // the same for the fused cell kernel (2, 3); 0: from occupancy
};

// One system of the batch: host-side parameters, sampler and sequence.
struct SysHost {
    int64_t n = 0, p0 = 0;
    double box[3] = {0, 0, 0};
    double rc = 0;
    int32_t P = 0;
    uint64_t seed = 0;
    int M = 0;
    std::vector<double> omega, s;
    double S = 0, V = 0, uself = 0, w_rb = 0;
    Geom g{};
    int64_t ncell = 0, ncell_max = 0, c0 = 0;
    int32_t k0 = 0;
    SplitCoef64 co64{};
    SplitCoef32 co32{};
    // core-shell near kernel (FP32C option)
    const float4 *tbl = nullptr;
    float rin2 = 0.f;
    float ta[kTabQ] = {0, 0, 0, 0}, tb[kTabQ] = {0, 0, 0, 0};
    // zero-frequency mode
    int32_t zmode = 0;
    double zu = 0.0, zf = 0.0;
    // work lists
    int32_t it0 = 0, it1 = 0, jt0 = 0, jt1 = 0, ft0 = 0, ft1 = 0, nch = 0, kt = 1, streams = 1;
    double nh_nf = 0.0, nh_Q = 0.0;  // Nose-Hoover: degrees of freedom, thermostat mass
    int64_t pofs = 0, choff = 0;
    // sequence
    MHChain chain;
    std::vector<int32_t> kseq;
    std::vector<double> kw;
    bool custom_w = false;
    int64_t cursor = 0;
    int64_t kcap = 0;
    int32_t *dkseq = nullptr;
    double *dkw = nullptr;
    // on-device chains: split coefficients in device memory
    double *domega = nullptr, *ds = nullptr;
};

}  // namespace

namespace rbsog {
// Records the message of a failure that has no context (rbsog_last_error(NULL)
// returns it) and returns the status; formats into a fixed buffer.
rbsog_status fail_noctx(rbsog_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_init_error(buf);
    return st;
}
}  // namespace rbsog

struct rbsog_ctx {
    int32_t nsys = 0;
    std::vector<SysHost> sys;
    int64_t N = 0, C = 0;
    int32_t K = 0;
    int prec = RBSOG_FP64;
    int device = 0;
    double mass = 1.0;
    std::vector<double> q_host;  // charges in the caller's order
    // state
    bool forces_valid = false;
    int64_t evals = 0;
    bool poisoned = false;
    std::string err;
    // stream
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // second stream (default priority) on which the structure factor runs
    // beside the near part, and the events of the fork and the join
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // device memory
    std::vector<void *> allocs;
    SysDev *dsys = nullptr;
    int32_t *sys_of = nullptr, *ksys = nullptr;
    StateBufs buf[2] = {};
    uint32_t *u_tmp = nullptr, *u = nullptr;
    uint4 *pk = nullptr;       // the list pass's gather records (EvalArgs::pk, pkx)
    PosQ64 *pkx = nullptr;
    uint32_t *rs_u = nullptr;  // the structure factor's copy of the state
    float *rs_qf = nullptr;
    double *rs_x = nullptr, *rs_q = nullptr;
    int32_t *cell_of = nullptr, *cell_count = nullptr, *cell_start = nullptr, *cell_fill = nullptr, *src = nullptr,
            *sorted = nullptr, *blocksums = nullptr, *cell_sorted = nullptr, *skey = nullptr;
    // Verlet list: skin (fraction of r_c), pairs, per-item counts and
    // capacity, rebuild flag, largest count of the latest build, builds made
    double skin = 0.1;      // the caller's
    double skin_cur = 0.1;  // in use: the caller's, or 0 while builds come every step
    // adaptive skin: steps and builds since the last check, checks left in
    // the build-every-step mode, and the length of the next such period
    int64_t adapt_steps = 0, adapt_nb0 = 0;
    int64_t adapt_window = kAdaptSteps;  // steps to the next check
    int32_t hold = 0, hold_len = 4;
    uint32_t *pairs = nullptr;
    int32_t *pcnt = nullptr, *rebuild = nullptr, *pmax = nullptr;
    int64_t icap = 0;
    bool list_hm = false;  // home-major blocks (lists longer than kHomeMajorMin at sizing)
    int64_t *nbuild = nullptr;
    int32_t build_slots = 2;  // candidates per lane and test pass of the build
    int32_t cell_slots = 2;   // the same for the fused cell kernel
    double *Fn = nullptr, *Ff = nullptr;
    double *Ff_side = nullptr;  // build-every-step mode: far forces before the re-sort
    int64_t *kcur = nullptr;
    KRec64 *kb64 = nullptr;
    KRec32 *kb32 = nullptr;
    double *rho = nullptr, *ek = nullptr, *partial = nullptr, *epart = nullptr, *E = nullptr;
    double *dip_part = nullptr, *dipole = nullptr;
    // kinetic energy per far item and wave, and per system
    double *kpart = nullptr, *kin = nullptr;
    double *msd = nullptr;  // mean-square displacement per system (rbsog_get_msd)
    // debug record of the pairs the near kernels accept (rbsog_debug_record_pairs)
    uint2 *dbg_pairs = nullptr;
    int32_t *dbg_cnt = nullptr, *dbg_kind = nullptr;
    int32_t dbg_cap = 0;
    // rbsog_get_forces_subset: inverse id permutation, requested ids and the
    // gathered forces (allocated at the first call, grown as needed)
    int32_t *slot_of = nullptr;
    int64_t *sub_ids = nullptr;
    double *sub_out = nullptr;
    int64_t sub_cap = 0;
    // Nose-Hoover thermostat: on, target temperature, tau, xi per system
    bool nh_on = false;
    double nh_T = 0.0, nh_tau = 0.0;
    double *nh_xi = nullptr;
    // Langevin thermostat
    double gamma = 0.0, temp = 0.0;
    uint64_t tseed = 0;
    int64_t *tstep = nullptr;
    // on-device sampler: lambda chains per system (0 = host chain)
    int32_t lambda = 0;
    SampDev *dsamp = nullptr;
    ChainState *chains = nullptr;
    int32_t *flag = nullptr;
    uint32_t *sys_done = nullptr;
    uint32_t *bin_done = nullptr;
    double *kin_part = nullptr;
    ListItem *list_items = nullptr;
    NearItem *near_items = nullptr;  // cell runs of the build-every-evaluation mode
    int32_t n_near = 0;
    double *epart_cells = nullptr;
    RhoItem *rho_items = nullptr;
    FarItem *far_items = nullptr;
    int32_t n_list = 0, n_rho = 0, n_far = 0;
    // work-list shapes: the current ones, whether they were tuned, and
    // whether tuning runs at the first step
    Tune tune;
    bool tuned = false, autotune = false;
    std::string tune_key;
    // graphs of velocity-Verlet steps, per near mode (0: list kept, 1: every
    // step builds, so that the adaptive skin's switches reuse them) and per
    // variant (GV_*)
    bool use_graphs = true;
    // the structure factor on a second stream beside the re-sort and the near
    // part: when its (particle, k) work is small enough that the two do not
    // each fill the device (sum of n P <= kSideMaxWork); larger systems run
    // the kernels one after the other (both are bound by vector issue there,
    // and the overlap only shares the same units)
    bool use_side = true;
    hipGraph_t graph[2][GV_COUNT] = {};
    hipGraphExec_t graph_exec[2][GV_COUNT] = {};
    double graph_dt_m[2][GV_COUNT] = {};
    bool msd_on = false;  // displacements tracked since rbsog_set_msd_origin
    // profiling
    // per-kernel timing: 0 off, 1 every kernel alone on the one stream, 2 as
    // in the steps (the second stream kept, events on each kernel's stream)
    int prof_on = 0;
    ProfEntry prof[K_COUNT];
    std::vector<hipEvent_t> ev_pool;
    struct Pending {
        int kid;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
};

namespace {

rbsog_status fail(rbsog_ctx *c, rbsog_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (st == RBSOG_E_DEVICE || st == RBSOG_E_OOM) c->poisoned = true;
    } else {
        set_init_error(buf);
    }
    return st;
}

#define HIPCHK(ctx, call)                                                                              \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail((ctx), RBSOG_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <class T>
rbsog_status dalloc(rbsog_ctx *c, T **p, int64_t count) {
    void *ptr = nullptr;
    size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess) return fail(c, RBSOG_E_OOM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    c->allocs.push_back(ptr);
    *p = (T *)ptr;
    return RBSOG_OK;
}

#define TRY(expr)                              \
    do {                                       \
        rbsog_status s_ = (expr);              \
        if (s_ != RBSOG_OK) return s_;         \
    } while (0)

// ---- split coefficients and S ------------------------------------------------
void sog_coefficients(const rbsog_sog &p, std::vector<double> &omega, std::vector<double> &s) {
    omega.assign(p.M + 1, 0.0);
    s.assign(p.M + 1, 0.0);
    const double lb = std::log(p.b);
    double bl = 1.0;
    for (int l = 0; l <= p.M; ++l) {
        omega[l] = std::sqrt(2.0 / kPi) * lb / (p.sigma * bl);
        s[l] = std::sqrt(2.0) * bl * p.sigma;
        bl *= p.b;
    }
    omega[0] *= p.w0;
}

// S = sum_l omega_l s_l^3 (prod_d H_l^d - 1) (Sec. 3.3, eq. "S"), with
// H - 1 = 2 sum_{m >= 1} exp(-pi^2 s^2 m^2 / L^2) and the product minus one
// expanded so that wide Gaussians (H -> 1) lose nothing to cancellation.
double normaliser_S(const std::vector<double> &omega, const std::vector<double> &s, const double box[3]) {
    double S = 0.0;
    for (size_t l = 0; l < s.size(); ++l) {
        double h[3];
        for (int d = 0; d < 3; ++d) {
            const double a = kPi * kPi * s[l] * s[l] / (box[d] * box[d]);
            double acc = 0.0;
            for (int64_t m = 1;; ++m) {
                const double t = std::exp(-a * (double)m * (double)m);
                acc += t;
                if (t < 1e-18 * acc || t == 0.0) break;
            }
            h[d] = 2.0 * acc;
        }
        const double pm1 = h[0] + h[1] + h[2] + h[0] * h[1] + h[0] * h[2] + h[1] * h[2] + h[0] * h[1] * h[2];
        S += omega[l] * s[l] * s[l] * s[l] * pm1;
    }
    return S;
}

// ---- sampler -------------------------------------------------------------------
// The host chain: Metropolis-Hastings independence sampler over nonzero m
// (Sec. 3.3) on Philox stream 0 of the system's key; the proposal, target and
// acceptance are the shared ones of rbsog_math.h (the device chains use them too).
void mh_extend(SysHost *c, int64_t count, std::vector<int32_t> &out) {
    MHChain &ch = c->chain;
    const double s0 = c->s[0];
    const int G = (int)c->s.size();
    double sd[3], a[3];
    for (int d = 0; d < 3; ++d) {
        sd[d] = c->box[d] / (std::sqrt(2.0) * kPi * s0);
        a[d] = kPi * s0 / c->box[d];
    }
    int64_t made = 0;
    while (made < count) {
        int32_t cand[3];
        double ua;
        const bool nonzero = rmath::mh_propose(c->seed, 0, ch.attempt, sd, cand, ua);
        ++ch.attempt;
        if (!nonzero) continue;
        const double pc = rmath::target_weight(c->omega.data(), c->s.data(), G, c->box, cand);
        const double qc =
            rmath::proposal_1d(cand[0], a[0]) * rmath::proposal_1d(cand[1], a[1]) * rmath::proposal_1d(cand[2], a[2]);
        if (!ch.started) {
            std::copy(cand, cand + 3, ch.m);
            ch.p = pc;
            ch.qprop = qc;
            ch.started = true;
            continue;
        }
        if (rmath::mh_accept(ua, pc, qc, ch.p, ch.qprop)) {
            std::copy(cand, cand + 3, ch.m);
            ch.p = pc;
            ch.qprop = qc;
        }
        if (ch.burn_left > 0) {
            --ch.burn_left;
            continue;
        }
        out.push_back(ch.m[0]);
        out.push_back(ch.m[1]);
        out.push_back(ch.m[2]);
        ++made;
    }
}

// ---- profiling ---------------------------------------------------------------
hipEvent_t get_event(rbsog_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

rbsog_status prof_collect(rbsog_ctx *c) {
    if (c->pending.empty()) return RBSOG_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof[p.kid].ms += ms;
            c->prof[p.kid].launches += 1;
        }
        c->ev_pool.push_back(p.a);
        c->ev_pool.push_back(p.b);
    }
    c->pending.clear();
    return RBSOG_OK;
}

template <class F>
rbsog_status timed_on(rbsog_ctx *c, int kid, hipStream_t s, F &&launch) {
    if (!c->prof_on) {
        launch();
        return RBSOG_OK;
    }
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return fail(c, RBSOG_E_DEVICE, "hipEventCreate failed");
    HIPCHK(c, hipEventRecord(a, s));
    launch();
    HIPCHK(c, hipEventRecord(b, s));
    c->pending.push_back({kid, a, b});
    if (c->pending.size() > 8192) return prof_collect(c);
    return RBSOG_OK;
}

template <class F>
rbsog_status timed(rbsog_ctx *c, int kid, F &&launch) {
    return timed_on(c, kid, c->stream, launch);
}

// ---- device orchestration --------------------------------------------------------
SysDev sysdev_of(const SysHost &h) {
    SysDev d{};
    d.g = h.g;
    d.co64 = h.co64;
    d.co32 = h.co32;
    d.p0 = h.p0;
    d.c0 = h.c0;
    d.P = h.P;
    d.k0 = h.k0;
    d.kseq = h.dkseq;
    d.kw = h.custom_w ? h.dkw : nullptr;
    d.w_rb = h.w_rb;
    d.uself = h.uself;
    d.it0 = h.it0;
    d.it1 = h.it1;
    d.jt0 = h.jt0;
    d.jt1 = h.jt1;
    d.ft0 = h.ft0;
    d.ft1 = h.ft1;
    d.nh_nf = h.nh_nf;
    d.nh_Q = h.nh_Q;
    d.pofs = h.pofs;
    d.nch = h.nch;
    d.kt = h.kt;
    d.streams = h.streams;
    d.tbl = h.tbl;
    d.rin2 = h.rin2;
    d.zmode = h.zmode;
    d.zu = h.zu;
    d.zf = h.zf;
    d.choff = h.choff;
    for (int i = 0; i < kTabQ; ++i) {
        d.ta[i] = h.ta[i];
        d.tb[i] = h.tb[i];
    }
    return d;
}

rbsog_status upload_sysdev(rbsog_ctx *c, int32_t s) {
    const SysDev d = sysdev_of(c->sys[s]);
    HIPCHK(c, hipMemcpy(c->dsys + s, &d, sizeof d, hipMemcpyHostToDevice));
    return RBSOG_OK;
}

rbsog_status upload_cursor(rbsog_ctx *c, int32_t s) {
    HIPCHK(c, hipMemcpy(c->kcur + s, &c->sys[s].cursor, sizeof(int64_t), hipMemcpyHostToDevice));
    return RBSOG_OK;
}

// Whether the latest evaluation's wave vectors are the batch just below
// every system's cursor: only evaluations move a cursor on, by P, and a new
// sequence (or a refill of the device chains, which an evaluation follows
// at once) sets it to 0.
bool batch_below_cursors(const rbsog_ctx *c) {
    if (c->evals == 0) return false;
    for (const SysHost &h : c->sys)
        if (h.cursor < h.P) return false;
    return true;
}

// Every device cursor back by one batch, at the latest evaluation's wave
// vectors (the structure factor reads the batch at the cursor): the tuner's
// trials of the structure factor and its reduction (which moves the cursor
// on) evaluate that batch again.  Needs batch_below_cursors(c).
rbsog_status rewind_cursors(rbsog_ctx *c) {
    std::vector<int64_t> cur((size_t)c->nsys);
    for (int32_t s = 0; s < c->nsys; ++s) cur[s] = c->sys[s].cursor - c->sys[s].P;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->kcur, cur.data(), cur.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    return RBSOG_OK;
}

rbsog_status ensure_kcap(rbsog_ctx *c, int32_t s, int64_t nvec) {
    SysHost &h = c->sys[s];
    if (nvec <= h.kcap) return RBSOG_OK;
    int64_t cap = std::max<int64_t>(nvec, 2 * h.kcap);
    int32_t *nk = nullptr;
    double *nw = nullptr;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (hipMalloc((void **)&nk, (size_t)cap * 3 * sizeof(int32_t)) != hipSuccess)
        return fail(c, RBSOG_E_OOM, "sequence buffer of %lld vectors", (long long)cap);
    if (hipMalloc((void **)&nw, (size_t)cap * sizeof(double)) != hipSuccess) {
        (void)hipFree(nk);
        return fail(c, RBSOG_E_OOM, "weight buffer of %lld vectors", (long long)cap);
    }
    if (h.dkseq) {
        HIPCHK(c, hipMemcpy(nk, h.dkseq, (size_t)h.kcap * 3 * sizeof(int32_t), hipMemcpyDeviceToDevice));
        HIPCHK(c, hipMemcpy(nw, h.dkw, (size_t)h.kcap * sizeof(double), hipMemcpyDeviceToDevice));
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void *)h.dkseq), c->allocs.end());
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void *)h.dkw), c->allocs.end());
        (void)hipFree(h.dkseq);
        (void)hipFree(h.dkw);
    }
    h.dkseq = nk;
    h.dkw = nw;
    c->allocs.push_back(nk);
    c->allocs.push_back(nw);
    h.kcap = cap;
    return upload_sysdev(c, s);
}

rbsog_status upload_k(rbsog_ctx *c, int32_t s, int64_t from) {
    SysHost &h = c->sys[s];
    const int64_t nvec = (int64_t)h.kseq.size() / 3;
    TRY(ensure_kcap(c, s, nvec));
    if (nvec > from) {
        HIPCHK(c, hipMemcpy(h.dkseq + 3 * from, h.kseq.data() + 3 * from, (size_t)(nvec - from) * 3 * sizeof(int32_t),
                            hipMemcpyHostToDevice));
        if (h.custom_w)
            HIPCHK(c, hipMemcpy(h.dkw + from, h.kw.data() + from, (size_t)(nvec - from) * sizeof(double),
                                hipMemcpyHostToDevice));
    }
    return RBSOG_OK;
}

EvalArgs make_args(rbsog_ctx *c, bool stepping, double dt) {
    EvalArgs a{};
    a.N = c->N;
    a.C = c->C;
    a.nsys = c->nsys;
    a.K = c->K;
    a.sys = c->dsys;
    a.sys_of = c->sys_of;
    a.ksys = c->ksys;
    a.cur = c->buf[0];
    a.nxt = c->buf[1];
    if (!c->msd_on) a.cur.dsp = a.nxt.dsp = nullptr;  // the kernels skip the displacement
    a.u_tmp = c->u_tmp;
    a.u = c->u;
    a.rs_u = c->rs_u;
    a.rs_qf = c->rs_qf;
    a.pk = c->pk;
    a.pkx = c->pkx;
    a.rs_x = c->rs_x;
    a.rs_q = c->rs_q;
    a.cell_of = c->cell_of;
    a.cell_count = c->cell_count;
    a.cell_start = c->cell_start;
    a.cell_fill = c->cell_fill;
    a.src = c->src;
    a.skey = c->skey;
    a.sorted = c->sorted;
    a.blocksums = c->blocksums;
    a.cell_sorted = c->cell_sorted;
    a.rebuild = c->rebuild;
    a.pairs = c->skin_cur > 0.0 ? c->pairs : nullptr;
    a.always_build = c->skin_cur > 0.0 ? 0 : 1;
    a.pcnt = c->pcnt;
    a.icap = c->icap;
    a.list_hm = c->list_hm ? 1 : 0;
    a.pmax = c->pmax;
    a.nbuild = c->nbuild;
    a.Fn = c->Fn;
    a.Ff = c->Ff;
    a.Ff_side = c->Ff_side;
    a.kcur = c->kcur;
    a.kb64 = c->kb64;
    a.kb32 = c->kb32;
    a.rho = c->rho;
    a.ek = c->ek;
    a.partial = c->partial;
    a.epart = c->epart;
    a.epart_cells = c->epart_cells;
    a.E = c->E;
    a.dip_part = c->dip_part;
    a.dipole = c->dipole;
    a.flag = c->flag;
    a.sys_done = c->sys_done;
    a.bin_done = c->bin_done;
    a.kick = stepping ? 1 : 0;
    a.energy = 1;
    a.hdm = 0.5 * dt / c->mass;
    a.dt = dt;
    a.mass = c->mass;
    a.kpart = c->kpart;
    a.kin = c->kin;
    a.nh = c->nh_on ? 1 : 0;
    a.nh_T = c->nh_T;
    a.nh_xi = c->nh_xi;
    a.thermo = c->gamma > 0.0 ? 1 : 0;
    a.c1 = std::exp(-c->gamma * dt);
    a.c2 = std::sqrt((1.0 - a.c1 * a.c1) * c->temp / c->mass);
    a.tseed = c->tseed;
    a.tstep = c->tstep;
    a.dbg_pairs = c->dbg_pairs;
    a.dbg_cnt = c->dbg_cnt;
    a.dbg_cap = c->dbg_cap;
    a.dbg_kind = c->dbg_kind;
    a.fuse = 0;
    // four waves per record once a system has more chunks than one wave
    // takes in a round of eight loads per lane
    int32_t nch = 0;
    int64_t parts = 0;
    for (const SysHost &h : c->sys) {
        nch = std::max(nch, h.nch);
        parts = std::max<int64_t>({parts, 4 * (int64_t)(h.ft1 - h.ft0), (int64_t)(h.it1 - h.it0),
                                   (int64_t)(h.jt1 - h.jt0)});
    }
    a.red_waves = nch > 512 ? 4 : 1;
    // the energy sums: a block per 32768 partials of the largest system
    a.kin_part = c->kin_part;
    a.kin_blocks = (int32_t)std::min<int64_t>(kKinBlocks, std::max<int64_t>(1, (parts + 32767) / 32768));
    return a;
}

// Enqueue one force evaluation (with the velocity-Verlet kick-drift before
// and the closing kick after it when stepping).  The list-build kernels run
// every time and return at once unless the displacement check (or the host)
// asked for a build.  Pure launches: no host state changes, so it can be
// captured into a graph.
// `kinetic`: sum the kinetic energy and U_N, U of the evaluation; `energy`:
// the near kernels sum the pair energies.  Steps without the Nose-Hoover
// thermostat leave both to the last step of their run (nothing reads the
// values in between).
// Fused steps (plain velocity Verlet on a kept list, fusable(c)): `fuse`
// has the far kernel open the next step, whose enqueue then passes `head`
// false: it starts with the structure factor.  Every value is computed as in
// the unfused steps, in the same order.
rbsog_status enqueue_eval(rbsog_ctx *c, bool stepping, double dt, bool kinetic, bool energy, bool head = true,
                          bool fuse = false) {
    hipStream_t s = c->stream;
    const bool f64 = c->prec == RBSOG_FP64;
    EvalArgs a = make_args(c, stepping, dt);
    a.energy = energy ? 1 : 0;
    a.fuse = fuse ? 1 : 0;
    if (c->dbg_pairs) {
        // the record holds this evaluation's pairs only
        launch_fill_i32(c->dbg_cnt, 1, 0, s);
        launch_fill_i32(c->dbg_kind, 1, 0, s);
    }
    if (head) TRY(timed(c, K_KDQ, [&] { launch_kdq(a, s); }));
    // the structure factor and its reduction need the copy of the positions
    // taken by the kick/drift (or the previous far) kernel only: they run on the
    // side stream beside the re-sort and the near part (one stream while
    // profiling kernels alone, and for systems with a lot of far work)
    const bool fork = c->prof_on != 1 && c->use_side;
    // building at every step, the far force joins them there (the near part
    // is long enough to hide it); it is then read back in the new order
    const bool far_side = a.always_build != 0;
    const int32_t fb = c->tune.far_block;
    if (fork) {
        HIPCHK(c, hipEventRecord(c->ev_fork, s));
        HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
        TRY(timed_on(c, K_RHO, c->side, [&] { launch_rho(a, f64, c->rho_items, c->n_rho, c->side); }));
        TRY(timed_on(c, K_RHORED, c->side, [&] { launch_rho_reduce(a, c->side); }));
        if (far_side)
            TRY(timed_on(c, K_FARSIDE, c->side, [&] { launch_far_side(a, f64, c->far_items, c->n_far, fb, c->side); }));
        HIPCHK(c, hipEventRecord(c->ev_join, c->side));
    }
    if (!a.always_build) TRY(timed(c, K_BIN, [&] { launch_bin_scan(a, s); }));
    else TRY(timed(c, K_SCAN, [&] { launch_scan(a, s); }));
    TRY(timed(c, K_SCATTER, [&] { launch_cell_scatter(a, s); }));
    TRY(timed(c, K_SORTG, [&] { launch_sort_gather(a, s); }));
    if (a.always_build) {
        TRY(timed(c, K_NEARC, [&] { launch_near_cells(a, f64, c->near_items, c->n_near, c->cell_slots, s); }));
    } else {
        TRY(timed(c, K_LIST, [&] { launch_list_build(a, f64, c->list_items, c->n_list, c->build_slots, s); }));
        TRY(timed(c, K_NEAR, [&] { launch_near(a, f64, c->list_items, c->n_list, s); }));
    }
    if (fork) {
        HIPCHK(c, hipStreamWaitEvent(s, c->ev_join, 0));
    } else {
        TRY(timed(c, K_RHO, [&] { launch_rho(a, f64, c->rho_items, c->n_rho, s); }));
        TRY(timed(c, K_RHORED, [&] { launch_rho_reduce(a, s); }));
        if (far_side) TRY(timed(c, K_FARSIDE, [&] { launch_far_side(a, f64, c->far_items, c->n_far, fb, s); }));
    }
    if (far_side) TRY(timed(c, K_FARFIN, [&] { launch_far_finish(a, c->far_items, c->n_far, fb, s); }));
    else TRY(timed(c, K_FAR, [&] { launch_far(a, f64, c->far_items, c->n_far, fb, s); }));
    if (kinetic) launch_kinetic(a, s);
    HIPCHK(c, hipGetLastError());
    return RBSOG_OK;
}

// On-device sampler: the ring of lambda batches is refilled (every chain
// advanced by P states, the cursors reset to 0) before the evaluation that
// would run past its end.  The host mirrors the cursors, so the schedule is
// known here and the refill stays outside the captured step graphs.
rbsog_status refill_if_due(rbsog_ctx *c) {
    if (!c->lambda) return RBSOG_OK;
    const SysHost &h0 = c->sys[0];
    if (h0.cursor + h0.P <= (int64_t)c->lambda * h0.P) return RBSOG_OK;
    TRY(timed(c, K_SAMPLE, [&] { launch_refill(c->dsamp, c->nsys, c->lambda, c->chains, c->kcur, c->flag, c->stream); }));
    HIPCHK(c, hipGetLastError());
    for (auto &h : c->sys) h.cursor = 0;
    return RBSOG_OK;
}

void account_eval(rbsog_ctx *c) {
    for (auto &h : c->sys) h.cursor += h.P;
    c->evals += 1;
    c->forces_valid = true;
}

void drop_graph(rbsog_ctx *c, int m, int v) {
    if (c->graph_exec[m][v]) (void)hipGraphExecDestroy(c->graph_exec[m][v]);
    if (c->graph[m][v]) (void)hipGraphDestroy(c->graph[m][v]);
    c->graph_exec[m][v] = nullptr;
    c->graph[m][v] = nullptr;
}

void drop_graphs(rbsog_ctx *c) {
    for (int m = 0; m < 2; ++m)
        for (int v = 0; v < GV_COUNT; ++v) drop_graph(c, m, v);
}

int graph_mode(const rbsog_ctx *c) { return c->skin_cur > 0.0 ? 0 : 1; }

// Steps whose far kernel may open the next step: plain velocity Verlet (no
// thermostat) on a kept near list, without kernel timing or pair records.
bool fusable(const rbsog_ctx *c) {
    return c->skin_cur > 0.0 && !c->nh_on && !(c->gamma > 0.0) && !c->prof_on && !c->dbg_pairs && c->n_list > 0 &&
           c->n_far > 0;
}

// A step graph captures the kernel arguments; it is rebuilt when dt or a
// buffer changes.  Sequence buffers, the cell grid and the cell-run items are
// reached through device tables, so re-sampling and the adaptive skin's
// switches (one graph per near mode) do not invalidate it.
rbsog_status ensure_step_graph(rbsog_ctx *c, double dt, int v) {
    const int m = graph_mode(c);
    if (c->graph_exec[m][v] && c->graph_dt_m[m][v] == dt) return RBSOG_OK;
    drop_graph(c, m, v);
    const GraphShape &g0 = kShapes[v];
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    rbsog_status st = RBSOG_OK;
    for (int i = 0; i < g0.len && st == RBSOG_OK; ++i) {
        const bool head = i == 0 ? !g0.opened : !g0.fused;
        st = enqueue_eval(c, true, dt, c->nh_on, g0.energy, head, g0.fused);
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st != RBSOG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(c, RBSOG_E_DEVICE, "stream capture: %s", hipGetErrorString(e));
    c->graph[m][v] = g;
    e = hipGraphInstantiate(&c->graph_exec[m][v], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graphs(c);
        return fail(c, RBSOG_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    c->graph_dt_m[m][v] = dt;
    return RBSOG_OK;
}

rbsog_status request_build(rbsog_ctx *c);
rbsog_status upload_cell_items(rbsog_ctx *c);
int32_t build_slots_for(const rbsog_ctx *c);
int32_t cell_slots_for(const rbsog_ctx *c);
void set_slots(rbsog_ctx *c);
void set_geometry(SysHost &h, double skin);

// Installs the cell grid and list thresholds of a skin on every system (the
// next evaluation builds).
rbsog_status apply_skin(rbsog_ctx *c, double skin) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (SysHost &h : c->sys) set_geometry(h, skin);
    for (int32_t s = 0; s < c->nsys; ++s) TRY(upload_sysdev(c, s));
    c->skin_cur = skin;
    set_slots(c);
    TRY(upload_cell_items(c));
    // each mode keeps its own step graph (the grid and items are read from
    // device tables; the build's slots per pass are fixed per mode)
    return request_build(c);
}

// Adaptive skin, checked every kAdaptSteps steps: when lists last less than
// two steps (particles far faster than the skin allows for, as when
// oppositely charged ions without a repulsive core fall onto each other),
// keeping a list costs more than it saves, so the steps build every time at
// skin 0 (cells r_c wide, no list written); after a hold of a few checks the
// caller's skin is tried again for kProbeSteps steps (failing when half of
// them build), and the hold doubles (up to 32 checks) each time that try
// fails.  The pairs evaluated are the same in either mode.
rbsog_status adapt_skin(rbsog_ctx *c) {
    c->adapt_steps = 0;
    if (!(c->skin > 0.0)) return RBSOG_OK;
    int64_t nb = 0;
    HIPCHK(c, hipMemcpyAsync(&nb, c->nbuild, sizeof nb, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int64_t builds = nb - c->adapt_nb0;
    c->adapt_nb0 = nb;
    const bool busy = 2 * builds >= c->adapt_window;
    c->adapt_window = kAdaptSteps;
    if (c->skin_cur > 0.0) {
        if (busy) {
            c->hold = c->hold_len;
            c->hold_len = std::min(2 * c->hold_len, 32);
            TRY(apply_skin(c, 0.0));
        } else {
            c->hold_len = 4;
        }
    } else if (--c->hold <= 0) {
        // a short try: lists that still fail cost few steps of builds
        TRY(apply_skin(c, c->skin));
        c->adapt_window = kProbeSteps;
    }
    return RBSOG_OK;
}

// Asks for a list build at the next evaluation (positions set from the host,
// a larger list, or a new cell grid).
// The near list of the latest build again, from the context's reference
// positions, cells and launch shapes (after a state load): the build kernel
// alone, without its copy back of the state.  The build counter, the rebuild
// flag and the largest count keep their values.
rbsog_status relist(rbsog_ctx *c) {
    int64_t nb = 0;
    int32_t rb = 0, pm = 0;
    const int32_t one = 1;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&nb, c->nbuild, sizeof nb, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&rb, c->rebuild, sizeof rb, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&pm, c->pmax, sizeof pm, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(c->rebuild, &one, sizeof one, hipMemcpyHostToDevice));
    EvalArgs a = make_args(c, false, 0.0);
    launch_list_build(a, c->prec == RBSOG_FP64, c->list_items, c->n_list, c->build_slots, c->stream, false);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->nbuild, &nb, sizeof nb, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->rebuild, &rb, sizeof rb, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->pmax, &pm, sizeof pm, hipMemcpyHostToDevice));
    return RBSOG_OK;
}

rbsog_status request_build(rbsog_ctx *c) {
    const int32_t one = 1;
    HIPCHK(c, hipMemcpyAsync(c->rebuild, &one, sizeof one, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBSOG_OK;
}

// (particle, k) pairs of one evaluation up to which the structure factor runs
// beside the near part on the second stream
constexpr double kSideMaxWork = 4e9;

// Lists longer than this (pairs of one home at the sizing build) are kept in
// home-major blocks, evaluated one home per wave; shorter ones in columns, one
// home per lane.
constexpr int64_t kHomeMajorMin = 128;

// Capacity of the pair list: every item holds icap / kListHomes rows of
// kListHomes entries, one list per home.  Sized from the largest count of
// one home at a build with room to spare; a build whose largest count passes
// 3/4 of the rows makes the next call grow it (and build again), and one that
// overflows fails the call.
rbsog_status size_list(rbsog_ctx *c, int64_t largest) {
    const int64_t want = kListHomes * ((2 * std::max<int64_t>(largest, 8) + 3) / 4 * 4);
    if (c->pairs && want <= c->icap) return RBSOG_OK;
    // long lists (beyond kHomeMajorMin pairs of one home) in home-major blocks
    c->list_hm = largest > kHomeMajorMin;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    uint32_t *np = nullptr;
    if (hipMalloc((void **)&np, (size_t)c->n_list * (size_t)want * sizeof(uint32_t)) != hipSuccess)
        return fail(c, RBSOG_E_OOM, "pair list of %lld x %lld entries", (long long)c->n_list, (long long)want);
    if (c->pairs) {
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void *)c->pairs), c->allocs.end());
        (void)hipFree(c->pairs);
    }
    c->pairs = np;
    c->allocs.push_back(np);
    c->icap = want;
    // no item of the new buffer holds pairs until the next build
    HIPCHK(c, hipMemset(c->pcnt, 0, (size_t)kListHomes * c->n_list * sizeof(int32_t)));
    drop_graphs(c);
    return request_build(c);
}

// After a call's evaluations: overflow fails it (the forces after it were
// incomplete); a list close to full is grown for the next call.
rbsog_status check_list(rbsog_ctx *c, int32_t flag) {
    if (flag & 8) {
        c->poisoned = true;
        return fail(c, RBSOG_E_STATE, "a home's near list exceeded its capacity of %lld pairs",
                    (long long)(c->icap / kListHomes));
    }
    int32_t pm = 0;
    HIPCHK(c, hipMemcpy(&pm, c->pmax, sizeof pm, hipMemcpyDeviceToHost));
    if (4 * (int64_t)pm > 3 * (c->icap / kListHomes)) TRY(size_list(c, pm));
    return RBSOG_OK;
}

// Non-finite forces or energies (bits 1 and 2) and a device chain past its
// proposal limit (bit 4) are reported once: the bits are cleared so that a
// context given new finite state (positions, a loaded state) runs on.
rbsog_status check_flag(rbsog_ctx *c, int32_t flag) {
    if (!(flag & 7)) return RBSOG_OK;
    const int32_t keep = flag & ~7;
    HIPCHK(c, hipMemcpyAsync(c->flag, &keep, sizeof keep, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flag & 4) return fail(c, RBSOG_E_STATE, "a device chain exceeded its proposal limit (flag %d)", flag);
    return fail(c, RBSOG_E_NONFINITE, "non-finite force or energy (flag %d)", flag);
}

rbsog_status check_ctx(rbsog_ctx *c) {
    if (!c) return fail(nullptr, RBSOG_E_ARG, "null context");
    if (c->poisoned) return fail(c, RBSOG_E_STATE, "context is poisoned after a device error: %s", c->err.c_str());
    HIPCHK(c, hipSetDevice(c->device));
    return RBSOG_OK;
}

rbsog_status check_sys(rbsog_ctx *c, int32_t s) {
    if (s < 0 || s >= c->nsys) return fail(c, RBSOG_E_ARG, "system %d out of range [0, %d)", s, c->nsys);
    return RBSOG_OK;
}

// ids of the current cell order (slot -> caller index)
rbsog_status current_ids(rbsog_ctx *c, std::vector<int32_t> &id) {
    id.resize((size_t)c->N);
    HIPCHK(c, hipMemcpyAsync(id.data(), c->buf[0].id, (size_t)c->N * sizeof(int32_t), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBSOG_OK;
}

// host n x 3 in caller order -> device SoA in the current cell order
rbsog_status upload_by_id(rbsog_ctx *c, const double *host, double *dev, const char *what) {
    std::vector<int32_t> id;
    TRY(current_ids(c, id));
    std::vector<double> soa((size_t)c->N * 3);
    for (int64_t t = 0; t < c->N; ++t)
        for (int d = 0; d < 3; ++d) {
            const double v = host[3 * (int64_t)id[t] + d];
            if (!std::isfinite(v)) return fail(c, RBSOG_E_NONFINITE, "%s of particle %d is not finite", what, id[t]);
            soa[(size_t)d * c->N + t] = v;
        }
    HIPCHK(c, hipMemcpy(dev, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice));
    return RBSOG_OK;
}

// device SoA in the current cell order -> host n x 3 in caller order
rbsog_status download_by_id(rbsog_ctx *c, const double *dev, double *host) {
    std::vector<int32_t> id;
    TRY(current_ids(c, id));
    std::vector<double> soa((size_t)c->N * 3);
    HIPCHK(c, hipMemcpyAsync(soa.data(), dev, soa.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t t = 0; t < c->N; ++t)
        for (int d = 0; d < 3; ++d) host[3 * (int64_t)id[t] + d] = soa[(size_t)d * c->N + t];
    return RBSOG_OK;
}

// Split coefficients of the near kernel for one system.
void build_split(SysHost &h, int nexp64, int nexp32) {
    // explicit Gaussians and the tail polynomials:
    // sum_{l >= nexp} omega_l e^{-x a_l} = sum_k (-1)^k/k! (sum_l omega_l a_l^k) x^k
    // and the force weights 2 omega_l a_l e^{-x a_l} likewise (a_l = 1/s_l^2)
    const int G = h.M + 1;
    auto tail = [&](int l0, int k) {
        double sp = 0.0, sf = 0.0, fact = 1.0;
        for (int i = 2; i <= k; ++i) fact *= i;
        for (int l = l0; l < G; ++l) {
            const double a = 1.0 / (h.s[l] * h.s[l]);
            sp += h.omega[l] * std::pow(a, k);
            sf += 2.0 * h.omega[l] * std::pow(a, k + 1);
        }
        const double sgn = (k & 1) ? -1.0 : 1.0;
        return std::make_pair(sgn * sp / fact, sgn * sf / fact);
    };
    // value-initialised: the constants past nexp are zero (the kernels run
    // the first few terms without testing the count)
    h.co64 = SplitCoef64{};
    h.co32 = SplitCoef32{};
    h.co64.nexp = nexp64;
    h.co32.nexp = nexp32;
    for (int l = 0; l < nexp64; ++l) {
        const double is2 = 1.0 / (h.s[l] * h.s[l]);
        h.co64.a[l] = is2;
        h.co64.cw[l] = 2.0 * h.omega[l] * is2;
        h.co64.w[l] = h.omega[l];
    }
    for (int l = 0; l < nexp32; ++l) {
        const double is2 = 1.0 / (h.s[l] * h.s[l]);
        h.co32.a[l] = (float)(is2 / std::log(2.0));
        h.co32.cw[l] = (float)(2.0 * h.omega[l] * is2);
        h.co32.w[l] = (float)h.omega[l];
    }
    for (int k = 0; k <= kTailDeg64; ++k) {
        const auto pf = tail(nexp64, k);
        h.co64.pt[k] = pf.first;
        h.co64.ft[k] = pf.second;
    }
    for (int k = 0; k <= kTailDeg32; ++k) {
        const auto pf = tail(nexp32, k);
        h.co32.pt[k] = (float)pf.first;
        h.co32.ft[k] = (float)pf.second;
    }
}

// Cell grid and near-list thresholds of one system for a skin.  skin > 0:
// the list holds the pairs within r_l = r_c (1 + skin) at the build and stays
// valid while no particle has moved farther than skin r_c / 2 (cells at least
// r_l wide hold every pair of the list).  The FP32 list test is widened and
// the FP32 displacement test narrowed by far more than their rounding (2e-5
// relative), so the list holds every pair the exact rule can accept before
// the check asks for a build.  skin = 0: every evaluation builds (the
// displacement threshold is negative) and no list is kept.
void set_geometry(SysHost &h, double skin) {
    Geom &g = h.g;
    for (int d = 0; d < 3; ++d) {
        const int64_t k = (int64_t)std::floor(h.box[d] / (h.rc * (1.0 + skin)));
        g.nc[d] = (int32_t)(k >= 3 ? k : 1);
        g.reach[d] = g.nc[d] >= 3 ? 1 : 0;
    }
    const double rl = h.rc * (1.0 + skin);
    g.rl2_f = (float)(rl * rl * (1.0 + 1e-4) + 1e-30);
    const double dmax = 0.5 * skin * h.rc;
    g.dthr2_f = skin > 0.0 ? (float)(dmax * dmax * (1.0 - 1e-4)) : -1.0f;
    h.ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
}

// Validates one system and fills its host record (everything but offsets
// and work lists).
rbsog_status setup_system(SysHost &h, int64_t n, const double *pos, const double *q, const double *box,
                          const rbsog_sog *sog, double rc, int32_t P, uint64_t seed, double neutral_tol, double skin,
                          int32_t idx) {
    if (n < 2) return fail(nullptr, RBSOG_E_ARG, "system %d: n must be >= 2", idx);
    if (P < 1) return fail(nullptr, RBSOG_E_ARG, "system %d: P must be >= 1", idx);
    for (int d = 0; d < 3; ++d)
        if (!(box[d] > 0.0) || !std::isfinite(box[d]))
            return fail(nullptr, RBSOG_E_ARG, "system %d: box sides must be > 0", idx);
    if (!(sog->b > 1.0) || !std::isfinite(sog->b) || !(sog->sigma > 0.0) || !std::isfinite(sog->sigma) ||
        !(sog->w0 > 0.0) || !std::isfinite(sog->w0) || sog->M < 0 || sog->M + 1 > kMaxGauss)
        return fail(nullptr, RBSOG_E_SOG, "system %d: split parameters need b > 1, sigma > 0, w0 > 0, 0 <= M < %d",
                    idx, kMaxGauss);
    const double lmin = std::min(box[0], std::min(box[1], box[2]));
    if (!(rc > 0.0) || !(rc <= 0.5 * lmin))
        return fail(nullptr, RBSOG_E_CUTOFF, "system %d: need 0 < rc <= min(L)/2", idx);
    double qs = 0.0, qa = 0.0, q2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(q[i]))
            return fail(nullptr, RBSOG_E_NONFINITE, "system %d: charge %lld is not finite", idx, (long long)i);
        qs += q[i];
        qa += std::fabs(q[i]);
        q2 += q[i] * q[i];
    }
    if (std::fabs(qs) > neutral_tol * qa)
        return fail(nullptr, RBSOG_E_NOT_NEUTRAL, "system %d: sum q = %.17g exceeds %.3g * sum|q|", idx, qs,
                    neutral_tol);
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(pos[i]))
            return fail(nullptr, RBSOG_E_NONFINITE, "system %d: position entry %lld is not finite", idx, (long long)i);
    h.n = n;
    std::copy(box, box + 3, h.box);
    h.rc = rc;
    h.P = P;
    h.seed = seed;
    h.M = sog->M;
    sog_coefficients(*sog, h.omega, h.s);
    h.V = box[0] * box[1] * box[2];
    h.S = normaliser_S(h.omega, h.s, box);
    h.w_rb = h.S * std::pow(kPi, 1.5) / ((double)P * h.V);
    double f0 = 0.0;
    for (double w : h.omega) f0 += w;
    h.uself = 0.5 * f0 * q2;
    Geom &g = h.g;
    g.n = n;
    double hmax = 0.0;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = box[d];
        g.invL[d] = 1.0 / box[d];
        g.h[d] = box[d] / kTwo32;
        g.hf[d] = (float)g.h[d];
        hmax = std::max(hmax, g.h[d]);
    }
    g.rc2 = rc * rc;
    const double d64 = 32.0 * hmax / rc + 1e-12;
    // the FP32 test runs on cell-relative float coordinates (cells up to 3 r_c
    // wide): its r^2 is within 2e-5 relative of the exact value
    const double d32 = d64 + 3e-5;
    g.band_lo = g.rc2 * (1.0 - d64);
    g.band_hi = g.rc2 * (1.0 + d64);
    g.band_lo_f = (float)(g.rc2 * (1.0 - d32));
    g.band_hi_f = (float)(g.rc2 * (1.0 + d32));
    // cells are allocated for the finest grid (skin 0); the grid in use is a
    // prefix of that range
    h.ncell_max = 1;
    for (int d = 0; d < 3; ++d) {
        const int64_t k = (int64_t)std::floor(box[d] / rc);
        h.ncell_max *= k >= 3 ? k : 1;
    }
    set_geometry(h, skin);
    // Gaussians wide enough that exp(-x/s_l^2) is a short Taylor series over
    // x = r^2 <= rc^2 form the tail; s_l grows with l, so they are l >= nexp.
    auto first_wide = [&](double tau) {
        for (int l = 0; l <= h.M; ++l)
            if (rc * rc / (h.s[l] * h.s[l]) <= tau) return l;
        return h.M + 1;
    };
    const int nexp64 = first_wide(kTailTau64), nexp32 = first_wide(kTailTau32);
    if (nexp64 > kMaxExp)
        return fail(nullptr, RBSOG_E_SOG, "system %d: more than %d Gaussians narrower than r_c / sqrt(%g)", idx,
                    kMaxExp, kTailTau64);
    build_split(h, nexp64, nexp32);
    return RBSOG_OK;
}

// ---- core-shell near kernel (Sec. 3.4) -------------------------------------
// Exact split kernels at x = r^2: force coefficient g and pair potential h.
void split_kernels(const SysHost &h, double x, double &g, double &hv) {
    g = std::pow(x, -1.5);
    hv = 1.0 / std::sqrt(x);
    for (size_t l = 0; l < h.s.size(); ++l) {
        const double a = 1.0 / (h.s[l] * h.s[l]);
        const double e = std::exp(-x * a);
        g -= 2.0 * h.omega[l] * a * e;
        hv -= h.omega[l] * e;
    }
}

// Table of the shell and Taylor coefficients of the core for one system.  The
// table's 2^kTabBexp binades start at the one holding r_in^2 (as an FP32
// value); index i stands for the point whose FP32 bits are (e << 23) |
// ((i mod 2^kTabBman) << (23 - kTabBman)) with e the binade whose low
// kTabBexp exponent bits are i >> kTabBman.
rbsog_status build_coreshell(SysHost &h, std::vector<float4> &table, int32_t idx) {
    const float rin = (float)(kTabRin * h.rc);
    const float rin2 = rin * rin, rc2 = (float)(h.rc * h.rc);
    uint32_t b0, bt;
    std::memcpy(&b0, &rin2, 4);
    std::memcpy(&bt, &rc2, 4);
    const int e0 = (int)((b0 >> 23) & 0xff), etop = (int)((bt >> 23) & 0xff);
    const int nb = 1 << kTabBexp, sh = 23 - kTabBman;
    if (etop - e0 > nb - 2) return fail(nullptr, RBSOG_E_ARG, "system %d: r_c / r_in spans too many binades", idx);
    table.resize(kTabSize);
    for (int i = 0; i < kTabSize; ++i) {
        const int blk = i >> kTabBman, mant = i & ((1 << kTabBman) - 1);
        const int e = e0 + (((blk - e0) % nb) + nb) % nb;
        const uint32_t bits = ((uint32_t)e << 23) | ((uint32_t)mant << sh);
        const uint32_t nbits = bits + (1u << sh);
        float x, xn;
        std::memcpy(&x, &bits, 4);
        std::memcpy(&xn, &nbits, 4);
        double g, hv, gn, hn;
        split_kernels(h, x, g, hv);
        split_kernels(h, xn, gn, hn);
        table[i] = make_float4((float)g, (float)(gn - g), (float)hv, (float)(hn - hv));
    }
    h.rin2 = rin2;
    for (int i = 0; i < kTabQ; ++i) {
        double a_i = 0.0, b_i = 0.0, fact = 1.0;
        for (int k = 2; k < i + 1; ++k) fact *= k;
        for (size_t l = 0; l < h.s.size(); ++l) {
            const double a = 1.0 / (h.s[l] * h.s[l]);
            const double c = ((i & 1) ? -1.0 : 1.0) / fact * std::pow(a, i);
            a_i += h.omega[l] * a * c;
            b_i += h.omega[l] * c;
        }
        h.ta[i] = (float)a_i;
        h.tb[i] = (float)b_i;
    }
    return RBSOG_OK;
}

// ---- shape cache: tuned shapes by (architecture, precision, batch size,
// log2 N, P per system, log2 cells), kept for the process and optionally in
// the text file named by RBSOG_TUNE_CACHE (one "key cpi chunk block" line per
// entry, later lines win).
std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune_cache;
bool g_tune_loaded = false;

int ilog2(int64_t v) {
    int l = 0;
    while (v > 1) {
        v >>= 1;
        ++l;
    }
    return l;
}

std::string tune_key(const std::string &arch, const rbsog_ctx *c) {
    int64_t psum = 0;
    for (const SysHost &h : c->sys) psum += h.P;
    char buf[160];
    snprintf(buf, sizeof buf, "%s|prec%d|sys%d|n%d|P%lld|c%d", arch.c_str(), c->prec, ilog2(c->nsys), ilog2(c->N),
             (long long)(psum / c->nsys), ilog2(c->C));
    return buf;
}

void tune_cache_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("RBSOG_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512], key[256];
    while (std::fgets(line, sizeof line, f)) {
        Tune t;
        // key rho_chunk far_block [rho_kt build_slots cell_slots]
        if (std::sscanf(line, "%255s %d %d %d %d %d", key, &t.rho_chunk, &t.far_block, &t.rho_kt, &t.build_slots,
                        &t.cell_slots) >= 3)
            g_tune_cache[key] = t;
    }
    std::fclose(f);
}

bool tune_cache_lookup(const std::string &key, Tune &t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load_locked();
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    t = it->second;
    return true;
}

void tune_cache_store(const std::string &key, const Tune &t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load_locked();
    g_tune_cache[key] = t;
    const char *path = std::getenv("RBSOG_TUNE_CACHE");
    if (!path || !*path) return;
    if (FILE *f = std::fopen(path, "a")) {
        std::fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), t.rho_chunk, t.far_block, t.rho_kt, t.build_slots,
                     t.cell_slots);
        std::fclose(f);
    }
}

// Work lists of the batch.  Near: runs of kListHomes slots of one system;
// rho: particle chunks of about t.rho_chunk slots x k-tile groups; far: runs
// of t.far_block slots.
void build_work(rbsog_ctx *c, const Tune &t, std::vector<ListItem> &near, std::vector<RhoItem> &rho,
                std::vector<FarItem> &far) {
    const int64_t chunk = t.rho_chunk, fb = t.far_block;
    int64_t pofs = 0, choff = 0;
    for (int32_t s = 0; s < c->nsys; ++s) {
        SysHost &h = c->sys[s];
        h.it0 = (int32_t)near.size();
        for (int64_t i = 0; i < h.n; i += kListHomes)
            near.push_back(ListItem{s, 0, h.p0 + i, h.p0 + std::min<int64_t>(h.n, i + kListHomes)});
        h.it1 = (int32_t)near.size();
        const int32_t ktiles = (h.P + 63) / 64;
        h.kt = std::min(ktiles, t.rho_kt > 0 ? std::min(t.rho_kt, 16) : 16);
        h.streams = std::max(1, 16 / h.kt);
        const int32_t kgroups = (ktiles + h.kt - 1) / h.kt;
        h.nch = (int32_t)std::max<int64_t>(1, (h.n + chunk - 1) / chunk);
        const int64_t per = (h.n + h.nch - 1) / h.nch;
        for (int32_t kg = 0; kg < kgroups; ++kg)
            for (int32_t ch = 0; ch < h.nch; ++ch) {
                const int64_t j0 = h.p0 + std::min(h.n, ch * per), j1 = h.p0 + std::min(h.n, (ch + 1) * per);
                rho.push_back(RhoItem{s, kg, ch, 0, j0, j1});
            }
        h.pofs = pofs;
        pofs += (int64_t)h.nch * h.P;
        h.choff = choff;
        choff += h.nch;
        h.ft0 = (int32_t)far.size();
        for (int64_t i = 0; i < h.n; i += fb)
            far.push_back(FarItem{s, 0, h.p0 + i, h.p0 + std::min(h.n, i + fb)});
        h.ft1 = (int32_t)far.size();
    }
}

// Default shapes: 512 structure-factor chunks and 256-particle far blocks
// over the batch.
Tune default_tune(const rbsog_ctx *c) {
    Tune t;
    t.rho_chunk = (int32_t)std::max<int64_t>(256, (c->N + 511) / 512);
    t.far_block = 256;
    return t;
}

// Capacities of the work lists and partial buffers: the largest any shape
// below may need (256-particle chunks, 64-particle far items).
void work_caps(const rbsog_ctx *c, int64_t &near_cap, int64_t &rho_cap, int64_t &far_cap, int64_t &part_cap,
               int64_t &chunk_cap) {
    near_cap = rho_cap = far_cap = part_cap = chunk_cap = 0;
    for (const SysHost &h : c->sys) {
        near_cap += (h.n + kListHomes - 1) / kListHomes;
        // the most items any k-tile grouping makes: one k tile per group
        const int64_t ktiles = (h.P + 63) / 64;
        const int64_t nch = std::max<int64_t>(1, (h.n + 255) / 256);
        rho_cap += ktiles * nch;
        part_cap += nch * h.P;
        chunk_cap += nch;
        far_cap += (h.n + 63) / 64;
    }
}

bool valid_tune(const Tune &t) {
    return t.rho_chunk >= 256 && (t.far_block == 64 || t.far_block == 128 || t.far_block == 256) &&
           t.rho_kt >= 0 && t.rho_kt <= 16 && (t.build_slots == 0 || (t.build_slots >= 2 && t.build_slots <= 4)) &&
           (t.cell_slots == 0 || t.cell_slots == 2 || t.cell_slots == 3);
}

// Installs a set of shapes: builds and uploads the work lists and the
// per-system table; captured graphs are dropped (their launch sizes change).
rbsog_status apply_tune(rbsog_ctx *c, const Tune &t) {
    std::vector<ListItem> near;
    std::vector<RhoItem> rho;
    std::vector<FarItem> far;
    build_work(c, t, near, rho, far);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->list_items, near.data(), near.size() * sizeof(ListItem), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->rho_items, rho.data(), rho.size() * sizeof(RhoItem), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->far_items, far.data(), far.size() * sizeof(FarItem), hipMemcpyHostToDevice));
    c->n_list = (int32_t)near.size();
    c->n_rho = (int32_t)rho.size();
    c->n_far = (int32_t)far.size();
    // wave slots of the kinetic-energy partials that a smaller far block leaves unused stay 0
    HIPCHK(c, hipMemset(c->kpart, 0, (size_t)4 * c->n_far * sizeof(double)));
    for (int32_t s = 0; s < c->nsys; ++s) TRY(upload_sysdev(c, s));
    c->tune = t;
    set_slots(c);
    drop_graphs(c);
    return RBSOG_OK;
}

// Near items of the build-every-evaluation mode: runs of about C / 8192
// cells (1..64) of the grid in use, one per wave; per-system ranges in the
// system table.
rbsog_status upload_cell_items(rbsog_ctx *c) {
    int64_t ctot = 0;
    for (const SysHost &h : c->sys) ctot += h.ncell;
    const int64_t cpi = std::max<int64_t>(1, std::min<int64_t>(64, (ctot + 8191) / 8192));
    std::vector<NearItem> items;
    for (int32_t s = 0; s < c->nsys; ++s) {
        SysHost &h = c->sys[s];
        h.jt0 = (int32_t)items.size();
        for (int64_t cb = 0; cb < h.ncell; cb += cpi)
            items.push_back(NearItem{s, 0, h.c0 + cb, h.c0 + std::min(h.ncell, cb + cpi)});
        h.jt1 = (int32_t)items.size();
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->near_items, items.data(), items.size() * sizeof(NearItem), hipMemcpyHostToDevice));
    c->n_near = (int32_t)items.size();
    for (int32_t s = 0; s < c->nsys; ++s) TRY(upload_sysdev(c, s));
    return RBSOG_OK;
}

// Times each phase's candidate shapes on the latest evaluation's data and
// keeps the fastest, one phase after the other: the structure factor's chunk
// size and its k tiles per block (k_rho with k_rho_reduce on the latest
// batch again, the cursors rewound by one batch before each trial; skipped
// when a new sequence has replaced that batch), the far block (k_far, or k_far_side
// with k_far_finish when every step builds), the candidate slots per pass of
// the near kernel in use (k_list_build with the near list, k_near_cells when
// every step builds; each trial rebuilds at the current positions).  No
// cursor moves and no state changes beyond recomputing the same forces with
// the chosen shapes at the end (the build counter is restored).
rbsog_status autotune_now(rbsog_ctx *c, int32_t reps) {
    if (c->evals == 0 || !c->forces_valid)
        return fail(c, RBSOG_E_STATE, "autotuning needs the forces of the current positions first");
    if (reps < 1) reps = 1;
    const bool f64 = c->prec == RBSOG_FP64;
    hipStream_t st = c->stream;
    int64_t nbuild0 = 0;
    HIPCHK(c, hipStreamSynchronize(st));
    HIPCHK(c, hipMemcpy(&nbuild0, c->nbuild, sizeof nbuild0, hipMemcpyDeviceToHost));
    hipEvent_t e0 = get_event(c), e1 = get_event(c);
    if (!e0 || !e1) return fail(c, RBSOG_E_DEVICE, "hipEventCreate failed");
    const bool every = !(c->skin_cur > 0.0);
    // a full build at the current positions (the state is in cell order
    // already, so the re-sort is the identity), its near kernel with `slots`
    auto build = [&]() {
        EvalArgs a = make_args(c, false, 0.0);
        launch_bin_scan(a, st);
        launch_cell_scatter(a, st);
        launch_sort_gather(a, st);
        return a;
    };
    enum { PH_CHUNK, PH_KT, PH_FAR, PH_SLOTS, PH_N };
    // one timed launch of the phase's kernel(s) (summed over reps), after the
    // set-up the trial needs
    auto time_of = [&](int phase, double &ms) -> rbsog_status {
        double tot = 0.0;
        for (int r = 0; r <= reps; ++r) {
            EvalArgs a = make_args(c, false, 0.0);
            a.rebuild = nullptr;  // the far kernels leave the near-list flag alone
            if (phase == PH_SLOTS) {
                TRY(request_build(c));
                a = build();
            }
            if (phase == PH_CHUNK || phase == PH_KT) TRY(rewind_cursors(c));
            HIPCHK(c, hipEventRecord(e0, st));
            if (phase == PH_CHUNK || phase == PH_KT) {
                // the partial sums and their reduction: the chunk count sets both
                launch_rho(a, f64, c->rho_items, c->n_rho, st);
                launch_rho_reduce(a, st);
            } else if (phase == PH_FAR) {
                if (every) {
                    launch_far_side(a, f64, c->far_items, c->n_far, c->tune.far_block, st);
                    launch_far_finish(a, c->far_items, c->n_far, c->tune.far_block, st);
                } else {
                    launch_far(a, f64, c->far_items, c->n_far, c->tune.far_block, st);
                }
            } else if (every) {
                launch_near_cells(a, f64, c->near_items, c->n_near, c->cell_slots, st);
            } else {
                launch_list_build(a, f64, c->list_items, c->n_list, c->build_slots, st);
            }
            HIPCHK(c, hipEventRecord(e1, st));
            HIPCHK(c, hipEventSynchronize(e1));
            HIPCHK(c, hipGetLastError());
            float f = 0.f;
            HIPCHK(c, hipEventElapsedTime(&f, e0, e1));
            if (r > 0) tot += f;  // the first launch warms caches and code
        }
        ms = tot / reps;
        return RBSOG_OK;
    };
    Tune best = c->tune;
    const Tune dflt = default_tune(c);
    int64_t nmax = 0;
    int32_t ktmax = 1;
    for (const SysHost &h : c->sys) {
        nmax = std::max(nmax, h.n);
        ktmax = std::max<int32_t>(ktmax, std::min<int32_t>(16, (h.P + 63) / 64));
    }
    const std::vector<int32_t> cand[PH_N] = {
        {256, 512, 1024, 2048, 4096, 8192, 16384, 32768, dflt.rho_chunk},
        {1, 2, 4, 8, 16},
        {64, 128, 256},
        every ? std::vector<int32_t>{2, 3} : std::vector<int32_t>{2, 3, 4}};
    auto field = [](Tune &t, int phase) -> int32_t & {
        return phase == PH_CHUNK ? t.rho_chunk
               : phase == PH_KT  ? t.rho_kt
               : phase == PH_FAR ? t.far_block
                                 : t.build_slots;
    };
    // the structure factor's trials evaluate the latest batch again: with a
    // new sequence since, its shapes stay as they are
    const bool sf_trials = batch_below_cursors(c);
    for (int phase = 0; phase < PH_N; ++phase) {
        if (!sf_trials && (phase == PH_CHUNK || phase == PH_KT)) continue;
        double best_ms = 1e30;
        int32_t best_v = 0;
        for (int32_t v : cand[phase]) {
            if (phase == PH_CHUNK && v > std::max<int64_t>(256, nmax)) continue;
            if (phase == PH_KT && v > ktmax) continue;
            Tune t = best;
            if (phase == PH_SLOTS) (every ? t.cell_slots : t.build_slots) = v;
            else field(t, phase) = v;
            TRY(apply_tune(c, t));
            double ms = 0.0;
            TRY(time_of(phase, ms));
            if (ms < best_ms) {
                best_ms = ms;
                best_v = v;
            }
        }
        if (best_v == 0) continue;
        if (phase == PH_SLOTS) (every ? best.cell_slots : best.build_slots) = best_v;
        else field(best, phase) = best_v;
    }
    c->ev_pool.push_back(e0);
    c->ev_pool.push_back(e1);
    TRY(apply_tune(c, best));
    // the trials left forces of other shapes: the structure factors (and U*),
    // the near part and the far force again with the chosen ones (same data,
    // same wave vectors, same pairs); then the sequence cursors, the build
    // counter and the build flag as they were
    {
        if (sf_trials) {
            TRY(rewind_cursors(c));
            EvalArgs ar = make_args(c, false, 0.0);
            launch_rho(ar, f64, c->rho_items, c->n_rho, st);
            launch_rho_reduce(ar, st);
            HIPCHK(c, hipGetLastError());
            HIPCHK(c, hipStreamSynchronize(st));
            for (int32_t s = 0; s < c->nsys; ++s) TRY(upload_cursor(c, s));
        }
        TRY(request_build(c));
        EvalArgs a = build();
        if (every) {
            launch_near_cells(a, f64, c->near_items, c->n_near, c->cell_slots, st);
        } else {
            launch_list_build(a, f64, c->list_items, c->n_list, c->build_slots, st);
            launch_near(a, f64, c->list_items, c->n_list, st);
        }
        // the far force of the current order (the re-sorts above left the
        // side copy of the positions out of step with the permutation)
        a.rebuild = nullptr;
        launch_far(a, f64, c->far_items, c->n_far, c->tune.far_block, st);
        HIPCHK(c, hipGetLastError());
        const int32_t zero = 0;
        HIPCHK(c, hipMemcpyAsync(c->rebuild, &zero, sizeof zero, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(c->nbuild, &nbuild0, sizeof nbuild0, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
    }
    c->tuned = true;
    tune_cache_store(c->tune_key, best);
    return RBSOG_OK;
}

// On-device sampler: lambda fresh chains per system (not started, 100
// transitions to discard) and the per-system constants; the cursors start at
// the end of the ring so that the first evaluation refills it.
rbsog_status setup_device_chains(rbsog_ctx *c, int32_t lambda) {
    c->lambda = lambda;
    TRY(dalloc(c, &c->dsamp, c->nsys));
    TRY(dalloc(c, &c->chains, (int64_t)c->nsys * lambda));
    std::vector<SampDev> sd((size_t)c->nsys);
    for (int32_t s = 0; s < c->nsys; ++s) {
        SysHost &h = c->sys[s];
        const int32_t G = (int32_t)h.omega.size();
        TRY(dalloc(c, &h.domega, G));
        TRY(dalloc(c, &h.ds, G));
        HIPCHK(c, hipMemcpy(h.domega, h.omega.data(), G * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(h.ds, h.s.data(), G * sizeof(double), hipMemcpyHostToDevice));
        SampDev &d = sd[s];
        d.omega = h.domega;
        d.s = h.ds;
        d.G = G;
        d.P = h.P;
        for (int k = 0; k < 3; ++k) {
            d.L[k] = h.box[k];
            d.sd[k] = h.box[k] / (std::sqrt(2.0) * kPi * h.s[0]);
            d.a[k] = kPi * h.s[0] / h.box[k];
        }
        d.seed = h.seed;
        d.out = h.dkseq;
        h.cursor = (int64_t)lambda * h.P;
    }
    HIPCHK(c, hipMemcpy(c->dsamp, sd.data(), sd.size() * sizeof(SampDev), hipMemcpyHostToDevice));
    ChainState fresh{};
    fresh.burn_left = 100;
    std::vector<ChainState> ch((size_t)c->nsys * lambda, fresh);
    HIPCHK(c, hipMemcpy(c->chains, ch.data(), ch.size() * sizeof(ChainState), hipMemcpyHostToDevice));
    return RBSOG_OK;
}

// Candidate slots per lane and test pass (2, 3 or 4: passes of 128, 192 or
// 256 candidates) with the fewest slots tested per home cell, the candidate
// count of a cell taken as normal with mean `cand` and its square root as
// spread.
int32_t slots_for_mean(double cand, int32_t smax) {
    const double sd = std::sqrt(std::max(cand, 1.0));
    int32_t best = 2;
    double best_cost = 1e300;
    for (int32_t S = 2; S <= smax; ++S) {
        const double pass = 64.0 * S;
        double cost = 0.0, wsum = 0.0;
        for (int k = -40; k <= 40; ++k) {
            const double x = 0.1 * k, w = std::exp(-0.5 * x * x);
            const double cnt = std::max(1.0, cand + x * sd);
            cost += w * pass * std::ceil(cnt / pass);
            wsum += w;
        }
        cost /= wsum;
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = S;
        }
    }
    return best;
}

// Mean stencil occupancy of the densest system on the grid in use: 27 cells,
// or 36 for the fused cell kernel's pairs of home cells (rows of >= 6 cells).
double stencil_mean(const rbsog_ctx *c, bool pairs) {
    double cand = 0.0;
    for (const SysHost &h : c->sys) {
        double cells = (h.g.reach[0] ? 3.0 : 1.0) * (h.g.reach[1] ? 3.0 : 1.0) * (h.g.reach[2] ? 3.0 : 1.0);
        if (pairs && h.g.nc[0] >= 6) cells *= 4.0 / 3.0;
        cand = std::max(cand, cells * (double)h.n / (double)h.ncell);
    }
    return cand;
}

int32_t build_slots_for(const rbsog_ctx *c) { return slots_for_mean(stencil_mean(c, false), 4); }
int32_t cell_slots_for(const rbsog_ctx *c) { return slots_for_mean(stencil_mean(c, true), 3); }

// Slots per pass of the near kernels: the tuned ones, else from the mean
// stencil occupancy of the grid in use.
void set_slots(rbsog_ctx *c) {
    c->build_slots = c->tune.build_slots > 0 ? c->tune.build_slots : build_slots_for(c);
    c->cell_slots = c->tune.cell_slots > 0 ? c->tune.cell_slots : cell_slots_for(c);
}

// A list build that only counts, at the initial positions: its largest item
// count sizes the pair list.  It also puts the state in cell order; the
// first evaluation builds the list itself.
rbsog_status first_build(rbsog_ctx *c) {
    TRY(upload_cell_items(c));
    const int32_t one = 1, zero = 0;
    const int64_t zero64 = 0;
    HIPCHK(c, hipMemcpy(c->rebuild, &one, sizeof one, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->pmax, &zero, sizeof zero, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->nbuild, &zero64, sizeof zero64, hipMemcpyHostToDevice));
    if (!(c->skin_cur > 0.0)) return RBSOG_OK;  // no list is kept at skin 0
    EvalArgs a = make_args(c, false, 0.0);
    a.K = 0;
    a.pairs = nullptr;
    a.icap = 0;
    hipStream_t s = c->stream;
    launch_kdq(a, s);
    launch_bin_scan(a, s);
    launch_cell_scatter(a, s);
    launch_sort_gather(a, s);
    launch_list_build(a, c->prec == RBSOG_FP64, c->list_items, c->n_list, c->build_slots, s);
    HIPCHK(c, hipGetLastError());
    int32_t pm = 0;
    HIPCHK(c, hipMemcpyAsync(&pm, c->pmax, sizeof pm, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipMemcpy(c->nbuild, &zero64, sizeof zero64, hipMemcpyHostToDevice));
    return size_list(c, pm);
}

rbsog_status init_batch(rbsog_ctx **out, int32_t nsys, const int64_t *offsets, const double *pos, const double *q,
                        const double *boxes, const rbsog_sog *sog, const double *rc, const int32_t *P,
                        const uint64_t *seeds, const rbsog_opts *opts) {
    if (!out) return fail(nullptr, RBSOG_E_ARG, "out is null");
    *out = nullptr;
    if (nsys < 1) return fail(nullptr, RBSOG_E_ARG, "need at least one system");
    if (!offsets || !pos || !q || !boxes || !sog || !rc || !P || !seeds)
        return fail(nullptr, RBSOG_E_ARG, "null input pointer");
    if (offsets[0] != 0) return fail(nullptr, RBSOG_E_ARG, "offsets[0] must be 0");
    for (int32_t s = 0; s < nsys; ++s)
        if (offsets[s + 1] < offsets[s] + 2) return fail(nullptr, RBSOG_E_ARG, "system %d has fewer than 2 particles", s);
    if (offsets[nsys] > kMaxParticles) return fail(nullptr, RBSOG_E_ARG, "more than 2^28 particles");
    rbsog_opts o;
    rbsog_default_opts(&o);
    if (opts) o = *opts;
    if (o.precision != RBSOG_FP64 && o.precision != RBSOG_FP32C)
        return fail(nullptr, RBSOG_E_ARG, "unknown precision %d", o.precision);
    if (o.near_table && o.precision != RBSOG_FP32C)
        return fail(nullptr, RBSOG_E_ARG, "the core-shell near table is an option of the FP32C form");
    if (o.zero_mode < 0 || o.zero_mode > 2) return fail(nullptr, RBSOG_E_ARG, "zero_mode must be 0, 1 or 2");
    if (o.device_chains < 0 || o.device_chains > kMaxChains)
        return fail(nullptr, RBSOG_E_ARG, "device_chains must be in [0, %d]", kMaxChains);
    if (!(o.mass > 0.0) || !std::isfinite(o.mass)) return fail(nullptr, RBSOG_E_ARG, "mass must be > 0");
    if (!(o.neutral_tol >= 0.0)) return fail(nullptr, RBSOG_E_ARG, "neutral_tol must be >= 0");
    if (!(o.skin >= 0.0 && o.skin <= 1.0)) return fail(nullptr, RBSOG_E_ARG, "skin must be in [0, 1]");

    rbsog_ctx *c = new rbsog_ctx();
    c->nsys = nsys;
    c->sys.resize(nsys);
    c->prec = o.precision;
    c->device = o.device;
    c->mass = o.mass;
    c->use_graphs = o.graphs != 0;
    c->skin = o.skin;
    c->skin_cur = o.skin;
    {
        double work = 0.0;
        for (int32_t s = 0; s < nsys; ++s) work += (double)(offsets[s + 1] - offsets[s]) * (double)P[s];
        c->use_side = work <= kSideMaxWork;
    }
    for (int k = 0; k < K_COUNT; ++k) c->prof[k].name = kKernelNames[k];
    for (int32_t s = 0; s < nsys; ++s) {
        SysHost &h = c->sys[s];
        const int64_t p0 = offsets[s], n = offsets[s + 1] - offsets[s];
        rbsog_status st = setup_system(h, n, pos + 3 * p0, q + p0, boxes + 3 * s, sog + s, rc[s], P[s], seeds[s],
                                       o.neutral_tol, o.skin, s);
        if (st != RBSOG_OK) {
            delete c;
            return st;
        }
        h.p0 = p0;
        h.c0 = c->C;
        h.k0 = c->K;
        // zero-frequency mode (Sec. 3.2): spherical (2 pi/3V)|M|^2, slab (2 pi/V) M_z^2
        h.zmode = o.zero_mode;
        if (o.zero_mode == 1) {
            h.zu = 2.0 * kPi / (3.0 * h.V);
            h.zf = -4.0 * kPi / (3.0 * h.V);
        } else if (o.zero_mode == 2) {
            h.zu = 2.0 * kPi / h.V;
            h.zf = -4.0 * kPi / h.V;
        }
        c->C += h.ncell_max;
        if (c->C >= (int64_t)INT32_MAX || (int64_t)c->K + P[s] >= (int64_t)INT32_MAX) {
            delete c;
            return fail(nullptr, RBSOG_E_ARG, "too many cells or wave vectors");
        }
        c->K += P[s];
    }
    c->N = offsets[nsys];
    c->q_host.assign(q, q + c->N);
    set_slots(c);
    std::vector<std::vector<float4>> tables;
    if (o.near_table) {
        tables.resize(nsys);
        for (int32_t s = 0; s < nsys; ++s) {
            rbsog_status st = build_coreshell(c->sys[s], tables[s], s);
            if (st != RBSOG_OK) {
                delete c;
                return st;
            }
        }
    }
    c->autotune = o.autotune != 0;
    int64_t near_cap, rho_cap, far_cap, part_cap, chunk_cap;
    work_caps(c, near_cap, rho_cap, far_cap, part_cap, chunk_cap);

    auto bail = [&](rbsog_status st) {
        set_init_error(c->err.c_str());
        rbsog_destroy(c);
        return st;
    };
    if (hipSetDevice(o.device) != hipSuccess) {
        fail(c, RBSOG_E_DEVICE, "hipSetDevice(%d) failed", o.device);
        return bail(RBSOG_E_DEVICE);
    }
    if (o.stream) {
        c->stream = (hipStream_t)o.stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            fail(c, RBSOG_E_DEVICE, "hipStreamCreate failed");
            return bail(RBSOG_E_DEVICE);
        }
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        fail(c, RBSOG_E_DEVICE, "side stream or events");
        return bail(RBSOG_E_DEVICE);
    }
    const int64_t N = c->N, C = c->C, K = c->K;
    rbsog_status st = RBSOG_OK;
#define ALLOC(ptr, cnt)                                   \
    if ((st = dalloc(c, &c->ptr, (cnt))) != RBSOG_OK) return bail(st);
    for (int p = 0; p < 2; ++p) {
        ALLOC(buf[p].x, 3 * N);
        ALLOC(buf[p].v, 3 * N);
        ALLOC(buf[p].q, N);
        ALLOC(buf[p].qf, N);
        ALLOC(buf[p].id, N);
        ALLOC(buf[p].dsp, 3 * N);
    }
    ALLOC(dsys, nsys);
    ALLOC(sys_of, N);
    ALLOC(ksys, K);
    ALLOC(u_tmp, 3 * N);
    ALLOC(u, 3 * N);
    ALLOC(pk, N);
    if (c->prec == RBSOG_FP64) ALLOC(pkx, N);
    if (c->prec != RBSOG_FP64) {
        ALLOC(rs_u, 3 * N);
        ALLOC(rs_qf, N);
    }
    if (c->prec == RBSOG_FP64 || c->sys[0].zmode != 0) {
        ALLOC(rs_x, 3 * N);
        ALLOC(rs_q, N);
    }
    ALLOC(cell_of, N);
    ALLOC(src, N);
    ALLOC(skey, N);
    ALLOC(sorted, N);
    ALLOC(cell_count, C);
    ALLOC(cell_start, C + 1);
    ALLOC(cell_fill, C);
    ALLOC(blocksums, scan_blocksums_size(C));
    ALLOC(Fn, 3 * N);
    ALLOC(Ff, 3 * N);
    ALLOC(Ff_side, 3 * N);
    ALLOC(kcur, nsys);
    ALLOC(kb64, K);
    ALLOC(kb32, K);
    ALLOC(rho, 2 * K);
    ALLOC(ek, K);
    ALLOC(partial, 2 * part_cap);
    ALLOC(epart, near_cap);
    ALLOC(E, 4 * (int64_t)nsys);
    ALLOC(dip_part, 3 * chunk_cap);
    ALLOC(tstep, 1);
    ALLOC(dipole, 3 * (int64_t)nsys);
    ALLOC(flag, 1);
    ALLOC(sys_done, nsys);
    ALLOC(bin_done, 1);
    ALLOC(kin_part, (int64_t)nsys * 2 * kKinBlocks);
    float4 *dtab = nullptr;
    if (o.near_table) {
        if ((st = dalloc(c, &dtab, (int64_t)nsys * kTabSize)) != RBSOG_OK) return bail(st);
        for (int32_t s = 0; s < nsys; ++s) {
            if (hipMemcpy(dtab + (int64_t)s * kTabSize, tables[s].data(), kTabSize * sizeof(float4),
                          hipMemcpyHostToDevice) != hipSuccess) {
                fail(c, RBSOG_E_DEVICE, "table upload failed");
                return bail(RBSOG_E_DEVICE);
            }
            c->sys[s].tbl = dtab + (int64_t)s * kTabSize;
        }
    }
    ALLOC(kpart, 4 * far_cap);
    ALLOC(kin, nsys);
    ALLOC(msd, nsys);
    ALLOC(nh_xi, nsys);
    ALLOC(list_items, near_cap);
    ALLOC(near_items, C);
    ALLOC(epart_cells, C);
    ALLOC(pcnt, kListHomes * near_cap);
    ALLOC(cell_sorted, N);
    ALLOC(rebuild, 1);
    ALLOC(pmax, 1);
    ALLOC(nbuild, 1);
    ALLOC(rho_items, rho_cap);
    ALLOC(far_items, far_cap);
#undef ALLOC
    {
        // initial state in the caller's order (slot t holds particle t)
        std::vector<double> soa((size_t)3 * N), zero((size_t)3 * N, 0.0);
        for (int64_t i = 0; i < N; ++i)
            for (int d = 0; d < 3; ++d) soa[(size_t)d * N + i] = pos[3 * i + d];
        std::vector<float> qff(N);
        std::vector<int32_t> ids(N), sof(N), ks(K);
        for (int64_t i = 0; i < N; ++i) {
            qff[i] = (float)q[i];
            ids[i] = (int32_t)i;
        }
        for (int32_t s = 0; s < nsys; ++s) {
            const SysHost &h = c->sys[s];
            for (int64_t i = 0; i < h.n; ++i) sof[h.p0 + i] = s;
            for (int32_t k = 0; k < h.P; ++k) ks[h.k0 + k] = s;
        }
        std::vector<SysDev> sd(nsys);
        for (int32_t s = 0; s < nsys; ++s) sd[s] = sysdev_of(c->sys[s]);
        std::vector<int64_t> zc(nsys, 0);
        std::vector<uint32_t> zu(nsys, 0u);
        const int32_t zf = 0;
        const StateBufs &b = c->buf[0];
        bool ok = hipMemcpy(b.x, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(b.v, zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(b.q, q, N * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(b.qf, qff.data(), N * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(b.id, ids.data(), N * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(b.dsp, zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->Fn, zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->Ff, zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->sys_of, sof.data(), N * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->ksys, ks.data(), K * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->dsys, sd.data(), nsys * sizeof(SysDev), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->kcur, zc.data(), nsys * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->tstep, zc.data(), sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->sys_done, zu.data(), nsys * sizeof(uint32_t), hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemset(c->bin_done, 0, sizeof(uint32_t)) == hipSuccess &&
                  hipMemcpy(c->kin, std::vector<double>(nsys, 0.0).data(), nsys * sizeof(double),
                            hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->nh_xi, std::vector<double>(nsys, 0.0).data(), nsys * sizeof(double),
                            hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemcpy(c->flag, &zf, sizeof zf, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMemset(c->cell_count, 0, (size_t)C * sizeof(int32_t)) == hipSuccess;
        if (!ok) {
            fail(c, RBSOG_E_DEVICE, "initial upload failed");
            return bail(RBSOG_E_DEVICE);
        }
    }
    for (int32_t s = 0; s < nsys; ++s)
        if ((st = ensure_kcap(c, s, std::max<int64_t>(4, o.device_chains) * c->sys[s].P)) != RBSOG_OK) return bail(st);
    if (o.device_chains > 0 && (st = setup_device_chains(c, o.device_chains)) != RBSOG_OK) return bail(st);
    {
        // shapes: a tuned entry of the cache for this kind of batch, else defaults
        hipDeviceProp_t prop;
        std::string arch = hipGetDeviceProperties(&prop, o.device) == hipSuccess ? std::string(prop.gcnArchName) : "?";
        arch = arch.substr(0, arch.find(':'));
        c->tune_key = tune_key(arch, c);
        Tune t = default_tune(c);
        if (tune_cache_lookup(c->tune_key, t) && valid_tune(t)) c->tuned = true;
        else t = default_tune(c);
        if ((st = apply_tune(c, t)) != RBSOG_OK) return bail(st);
    }
    if ((st = first_build(c)) != RBSOG_OK) return bail(st);
    *out = c;
    return RBSOG_OK;
}

}  // namespace

// =============================================================================
extern "C" {

void rbsog_default_opts(rbsog_opts *o) {
    if (!o) return;
    o->precision = RBSOG_FP64;
    o->device = 0;
    o->stream = nullptr;
    o->neutral_tol = 1e-10;
    o->mass = 1.0;
    o->graphs = 1;
    o->autotune = 0;
    o->near_table = 0;
    o->zero_mode = 0;
    o->device_chains = 0;
    o->skin = 0.1;
}

rbsog_status rbsog_sog_table1(int32_t row, double rc, rbsog_sog *out) {
    // Table 1 (Sec. 4.1), quoted at r_c = 10 Angstrom.
    static const double tb[5][3] = {{2.0, 5.027010924194599, 0.994446492762232252},
                                    {1.62976708826776469, 3.633717409009413, 1.00780697934380681},
                                    {1.48783512395703226, 2.662784519725113, 0.991911705759818},
                                    {1.32070036405934420, 2.277149356440992, 1.00188914114811980},
                                    {1.21812525709410644, 1.774456369233284, 1.00090146156033341}};
    static const int32_t tm[5] = {6, 16, 30, 64, 102};
    if (!out || row < 1 || row > 5 || !(rc > 0.0) || !std::isfinite(rc))
        return fail(nullptr, RBSOG_E_ARG, "rbsog_sog_table1: row must be 1..5 and rc > 0");
    out->b = tb[row - 1][0];
    out->sigma = tb[row - 1][1] * rc / 10.0;
    out->w0 = tb[row - 1][2];
    out->M = tm[row - 1];
    return RBSOG_OK;
}

rbsog_status rbsog_init(rbsog_ctx **out, int64_t n, const double *pos, const double *q, const double *box,
                        const rbsog_sog *sog, double rc, int32_t P, uint64_t seed, const rbsog_opts *opts) {
    if (!out) return fail(nullptr, RBSOG_E_ARG, "out is null");
    *out = nullptr;
    if (n < 2 || n > kMaxParticles) return fail(nullptr, RBSOG_E_ARG, "n must be in [2, 2^28]");
    const int64_t offsets[2] = {0, n};
    return init_batch(out, 1, offsets, pos, q, box, sog, &rc, &P, &seed, opts);
}

rbsog_status rbsog_init_batch(rbsog_ctx **out, int32_t n_sys, const int64_t *offsets, const double *pos,
                              const double *q, const double *boxes, const rbsog_sog *sog, const double *rc,
                              const int32_t *P, const uint64_t *seeds, const rbsog_opts *opts) {
    return init_batch(out, n_sys, offsets, pos, q, boxes, sog, rc, P, seeds, opts);
}

rbsog_status rbsog_sample_k(rbsog_ctx *c, int64_t n_batches, int32_t *m_out) {
    TRY(check_ctx(c));
    if (c->lambda) return fail(c, RBSOG_E_STATE, "wave vectors are drawn by the device chains (device_chains > 0)");
    if (n_batches < 1) return fail(c, RBSOG_E_ARG, "n_batches must be >= 1");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int64_t written = 0;
    for (int32_t s = 0; s < c->nsys; ++s) {
        SysHost &h = c->sys[s];
        if (h.custom_w) {
            // a caller-given weighted list is replaced by the sampled sequence
            h.kseq.clear();
            h.kw.clear();
            h.custom_w = false;
            h.cursor = 0;
            TRY(upload_cursor(c, s));
            TRY(upload_sysdev(c, s));
        }
        const int64_t start = (int64_t)h.kseq.size() / 3;
        std::vector<int32_t> fresh;
        fresh.reserve((size_t)(n_batches * h.P * 3));
        mh_extend(&h, n_batches * h.P, fresh);
        h.kseq.insert(h.kseq.end(), fresh.begin(), fresh.end());
        TRY(upload_k(c, s, start));
        if (m_out) std::copy(fresh.begin(), fresh.end(), m_out + written);
        written += (int64_t)fresh.size();
    }
    return RBSOG_OK;
}

rbsog_status rbsog_set_k(rbsog_ctx *c, int32_t sys, int64_t n_k, const int32_t *m, const double *w) {
    TRY(check_ctx(c));
    TRY(check_sys(c, sys));
    if (c->lambda) return fail(c, RBSOG_E_STATE, "wave vectors are drawn by the device chains (device_chains > 0)");
    if (n_k < 1 || !m) return fail(c, RBSOG_E_ARG, "need n_k >= 1 vectors");
    for (int64_t e = 0; e < n_k; ++e) {
        if (m[3 * e] == 0 && m[3 * e + 1] == 0 && m[3 * e + 2] == 0)
            return fail(c, RBSOG_E_ARG, "wave vector %lld is zero", (long long)e);
        if (w && !std::isfinite(w[e])) return fail(c, RBSOG_E_NONFINITE, "weight %lld is not finite", (long long)e);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    SysHost &h = c->sys[sys];
    h.kseq.assign(m, m + 3 * n_k);
    h.custom_w = w != nullptr;
    if (w) h.kw.assign(w, w + n_k);
    else h.kw.clear();
    h.cursor = 0;
    TRY(upload_cursor(c, sys));
    TRY(upload_k(c, sys, 0));
    return upload_sysdev(c, sys);
}

static rbsog_status check_kseq(rbsog_ctx *c, int64_t evals) {
    if (c->lambda) return RBSOG_OK;  // the device chains never run out
    for (int32_t s = 0; s < c->nsys; ++s) {
        const SysHost &h = c->sys[s];
        const int64_t nvec = (int64_t)h.kseq.size() / 3;
        if (h.cursor + evals * h.P > nvec)
            return fail(c, RBSOG_E_KSEQ, "system %d: %lld evaluations need %lld vectors, %lld remain", s,
                        (long long)evals, (long long)(evals * h.P), (long long)(nvec - h.cursor));
    }
    return RBSOG_OK;
}

rbsog_status rbsog_forces(rbsog_ctx *c, double *F_out, double *E_out) {
    TRY(check_ctx(c));
    TRY(check_kseq(c, 1));
    TRY(refill_if_due(c));
    TRY(enqueue_eval(c, false, 0.0, true, true));
    account_eval(c);
    {
        int32_t flag = 0;
        HIPCHK(c, hipMemcpyAsync(&flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        TRY(check_list(c, flag));
        TRY(check_flag(c, flag));
    }
    if (F_out) {
        std::vector<double> b((size_t)3 * c->N);
        TRY(download_by_id(c, c->Fn, F_out));
        TRY(download_by_id(c, c->Ff, b.data()));
        for (size_t i = 0; i < b.size(); ++i) F_out[i] += b[i];
        // without a kick no kernel looks at the sum of the two forces
        for (size_t i = 0; i < b.size(); ++i)
            if (!std::isfinite(F_out[i]))
                return fail(c, RBSOG_E_NONFINITE, "force entry %lld is not finite", (long long)i);
    }
    if (E_out) {
        HIPCHK(c, hipMemcpyAsync(E_out, c->E, 4 * (size_t)c->nsys * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < 4 * (int64_t)c->nsys; ++i)
            if (!std::isfinite(E_out[i])) return fail(c, RBSOG_E_NONFINITE, "energy entry %lld is not finite", (long long)i);
    }
    return RBSOG_OK;
}

rbsog_status rbsog_step(rbsog_ctx *c, int64_t n_steps, double dt) {
    TRY(check_ctx(c));
    if (n_steps < 0 || !std::isfinite(dt)) return fail(c, RBSOG_E_ARG, "need n_steps >= 0 and finite dt");
    TRY(check_kseq(c, n_steps + (c->forces_valid ? 0 : 1)));
    if (!c->forces_valid) {
        TRY(refill_if_due(c));
        TRY(enqueue_eval(c, false, 0.0, true, true));
        account_eval(c);
    }
    if (c->autotune && !c->tuned && !c->prof_on) TRY(autotune_now(c, 5));
    const bool graphs = c->use_graphs && !c->prof_on && !c->dbg_pairs && n_steps > 1;
    for (int64_t k = 0; k < n_steps;) {
        // up to the next check of the build rate
        const int64_t chunk = std::min<int64_t>(n_steps - k, c->adapt_window - c->adapt_steps);
        // fused steps within the chunk: each opens the next, the chunk's last
        // step is unfused (the state between calls and at a check is a
        // step's end)
        const bool fuse = graphs && fusable(c);
        bool opened = false;
        for (int64_t i = 0; i < chunk;) {
            TRY(refill_if_due(c));
            // only the run's last step sums the near energies
            const bool last = k + i + 1 == n_steps;
            if (graphs) {
                // kGraphSteps steps at once when they fit in the chunk, stop
                // short of the last step and need no refill of the chains
                const int64_t room = c->lambda ? (int64_t)c->lambda - c->sys[0].cursor / c->sys[0].P : INT64_MAX;
                int v;
                if (fuse) {
                    const int64_t rem = chunk - i;
                    if (rem == 1) v = opened ? (last ? GV_F_TAIL_E : GV_F_TAIL) : (last ? GV_STEP_E : GV_STEP);
                    else if (rem > kGraphSteps && room >= kGraphSteps) v = opened ? GV_F_MID8 : GV_F_HEAD8;
                    else v = opened ? GV_F_MID1 : GV_F_HEAD1;
                    opened = rem > 1;
                } else {
                    const bool multi =
                        i + kGraphSteps <= chunk && k + i + kGraphSteps < n_steps && room >= kGraphSteps;
                    v = multi ? GV_MULTI : (last ? GV_STEP_E : GV_STEP);
                }
                TRY(ensure_step_graph(c, dt, v));
                HIPCHK(c, hipGraphLaunch(c->graph_exec[graph_mode(c)][v], c->stream));
                const int len = kShapes[v].len;
                for (int j = 0; j < len; ++j) account_eval(c);
                i += len;
            } else {
                TRY(enqueue_eval(c, true, dt, c->nh_on, last));
                account_eval(c);
                ++i;
            }
        }
        if (!c->nh_on && k + chunk == n_steps) {
            // the energies of the run's last evaluation (before a switch of
            // the near mode changes where its partial sums are read)
            launch_kinetic(make_args(c, false, 0.0), c->stream);
            HIPCHK(c, hipGetLastError());
        }
        k += chunk;
        c->adapt_steps += chunk;
        if (c->adapt_steps >= c->adapt_window) TRY(adapt_skin(c));
    }
    int32_t flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if ((flag & 3) && (flag & 8)) {
        // particles that went non-finite pile into cell 0 and overflow the
        // list: the cause is reported, the list is beyond repair
        c->poisoned = true;
        return fail(c, RBSOG_E_NONFINITE, "non-finite force or energy, and the near list overflowed (flag %d)", flag);
    }
    TRY(check_list(c, flag));
    return check_flag(c, flag);
}

// Kinetic energy of every system from velocities given in the caller's order
// (n x 3), summed in particle order, uploaded as the systems' current values.
static rbsog_status upload_kinetic(rbsog_ctx *c, const double *v) {
    std::vector<double> K((size_t)c->nsys, 0.0);
    for (int32_t s = 0; s < c->nsys; ++s) {
        const SysHost &h = c->sys[s];
        double acc = 0.0;
        for (int64_t i = h.p0; i < h.p0 + h.n; ++i)
            acc += (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1]) + v[3 * i + 2] * v[3 * i + 2];
        K[s] = 0.5 * c->mass * acc;
    }
    HIPCHK(c, hipMemcpy(c->kin, K.data(), K.size() * sizeof(double), hipMemcpyHostToDevice));
    return RBSOG_OK;
}

rbsog_status rbsog_set_velocities(rbsog_ctx *c, const double *v, double T, uint64_t seed) {
    TRY(check_ctx(c));
    if (v) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        TRY(upload_by_id(c, v, c->buf[0].v, "velocity"));
        return upload_kinetic(c, v);
    }
    if (!(T >= 0.0) || !std::isfinite(T)) return fail(c, RBSOG_E_ARG, "temperature must be >= 0");
    const double sd = std::sqrt(T / c->mass);
    std::vector<double> vv((size_t)3 * c->N);
    for (const SysHost &h : c->sys) {
        double mean[3] = {0, 0, 0};
        for (int64_t i = h.p0; i < h.p0 + h.n; ++i) {
            double z[3];
            rmath::normals3(seed, 1, (uint64_t)i, z);
            for (int d = 0; d < 3; ++d) {
                vv[3 * i + d] = sd * z[d];
                mean[d] += sd * z[d];
            }
        }
        for (int d = 0; d < 3; ++d) {
            mean[d] /= (double)h.n;
            for (int64_t i = h.p0; i < h.p0 + h.n; ++i) vv[3 * i + d] -= mean[d];
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    TRY(upload_by_id(c, vv.data(), c->buf[0].v, "velocity"));
    return upload_kinetic(c, vv.data());
}

rbsog_status rbsog_set_thermostat(rbsog_ctx *c, double gamma, double T, uint64_t seed) {
    TRY(check_ctx(c));
    if (!(gamma >= 0.0) || !std::isfinite(gamma) || !(T >= 0.0) || !std::isfinite(T))
        return fail(c, RBSOG_E_ARG, "need gamma >= 0 and T >= 0");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->gamma = gamma;
    c->temp = T;
    c->tseed = seed;
    if (gamma > 0.0) c->nh_on = false;  // one thermostat at a time
    const int64_t z = 0;
    HIPCHK(c, hipMemcpy(c->tstep, &z, sizeof z, hipMemcpyHostToDevice));
    drop_graphs(c);  // the graphs hold the step's constants
    return RBSOG_OK;
}

rbsog_status rbsog_set_nose_hoover(rbsog_ctx *c, double T, double tau) {
    TRY(check_ctx(c));
    if (!(tau >= 0.0) || !std::isfinite(tau) || !std::isfinite(T) || (tau > 0.0 && !(T > 0.0)))
        return fail(c, RBSOG_E_ARG, "need tau >= 0, and T > 0 when tau > 0");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->nh_on = tau > 0.0;
    c->nh_T = T;
    c->nh_tau = tau;
    for (int32_t s = 0; s < c->nsys; ++s) {
        SysHost &h = c->sys[s];
        h.nh_nf = 3.0 * (double)h.n - 3.0;
        h.nh_Q = c->nh_on ? h.nh_nf * T * tau * tau : 0.0;
        TRY(upload_sysdev(c, s));
    }
    const std::vector<double> zero((size_t)c->nsys, 0.0);
    HIPCHK(c, hipMemcpy(c->nh_xi, zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice));
    if (c->nh_on) {
        c->gamma = 0.0;  // one thermostat at a time
        std::vector<double> v((size_t)3 * c->N);
        TRY(download_by_id(c, c->buf[0].v, v.data()));
        TRY(upload_kinetic(c, v.data()));
    }
    drop_graphs(c);  // the graphs hold the step's constants
    return RBSOG_OK;
}

rbsog_status rbsog_get_kinetic(rbsog_ctx *c, double *K, double *xi) {
    TRY(check_ctx(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (K) HIPCHK(c, hipMemcpy(K, c->kin, (size_t)c->nsys * sizeof(double), hipMemcpyDeviceToHost));
    if (xi) HIPCHK(c, hipMemcpy(xi, c->nh_xi, (size_t)c->nsys * sizeof(double), hipMemcpyDeviceToHost));
    return RBSOG_OK;
}

rbsog_status rbsog_set_msd_origin(rbsog_ctx *c) {
    TRY(check_ctx(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemset(c->buf[0].dsp, 0, (size_t)3 * c->N * sizeof(double)));
    if (!c->msd_on) {
        c->msd_on = true;
        drop_graphs(c);  // the captured steps skip the displacement
    }
    return RBSOG_OK;
}

rbsog_status rbsog_get_msd(rbsog_ctx *c, double *msd) {
    TRY(check_ctx(c));
    if (!msd) return fail(c, RBSOG_E_ARG, "msd is null");
    if (!c->msd_on) return fail(c, RBSOG_E_STATE, "no mean-square-displacement origin: call rbsog_set_msd_origin");
    const EvalArgs a = make_args(c, false, 0.0);
    launch_msd(a, c->msd, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(msd, c->msd, (size_t)c->nsys * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBSOG_OK;
}

rbsog_status rbsog_set_positions(rbsog_ctx *c, const double *pos) {
    TRY(check_ctx(c));
    if (!pos) return fail(c, RBSOG_E_ARG, "pos is null");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    TRY(upload_by_id(c, pos, c->buf[0].x, "position"));
    HIPCHK(c, hipMemset(c->buf[0].dsp, 0, (size_t)3 * c->N * sizeof(double)));  // a new origin
    c->forces_valid = false;
    return request_build(c);
}

rbsog_status rbsog_get_state(rbsog_ctx *c, double *pos, double *vel) {
    TRY(check_ctx(c));
    if (pos) {
        TRY(download_by_id(c, c->buf[0].x, pos));
        // the stored coordinates are wrapped at each evaluation; wrap here too
        for (const SysHost &h : c->sys)
            for (int64_t i = h.p0; i < h.p0 + h.n; ++i)
                for (int d = 0; d < 3; ++d) {
                    const double t = pos[3 * i + d] / h.box[d];
                    pos[3 * i + d] = (t - std::floor(t)) * h.box[d];
                }
    }
    if (vel) TRY(download_by_id(c, c->buf[0].v, vel));
    return RBSOG_OK;
}

rbsog_status rbsog_get_forces(rbsog_ctx *c, double *F_near, double *F_far) {
    TRY(check_ctx(c));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    if (F_near) TRY(download_by_id(c, c->Fn, F_near));
    if (F_far) TRY(download_by_id(c, c->Ff, F_far));
    return RBSOG_OK;
}

rbsog_status rbsog_get_forces_subset(rbsog_ctx *c, int64_t m, const int64_t *ids, double *F_near, double *F_far) {
    TRY(check_ctx(c));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    if (m < 0 || (m > 0 && !ids)) return fail(c, RBSOG_E_ARG, "need m >= 0 caller indices");
    for (int64_t k = 0; k < m; ++k)
        if (ids[k] < 0 || ids[k] >= c->N)
            return fail(c, RBSOG_E_ARG, "index %lld of entry %lld out of range", (long long)ids[k], (long long)k);
    if (m == 0) return RBSOG_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->slot_of) TRY(dalloc(c, &c->slot_of, c->N));
    if (m > c->sub_cap) {
        for (void *p : {(void *)c->sub_ids, (void *)c->sub_out}) {
            if (!p) continue;
            c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), p), c->allocs.end());
            (void)hipFree(p);
        }
        c->sub_ids = nullptr;
        c->sub_out = nullptr;
        c->sub_cap = 0;
        TRY(dalloc(c, &c->sub_ids, m));
        TRY(dalloc(c, &c->sub_out, 6 * m));
        c->sub_cap = m;
    }
    HIPCHK(c, hipMemcpyAsync(c->sub_ids, ids, (size_t)m * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    launch_subset_forces(make_args(c, false, 0.0), m, c->sub_ids, c->slot_of, c->sub_out, c->stream);
    HIPCHK(c, hipGetLastError());
    std::vector<double> out((size_t)(6 * m));
    HIPCHK(c, hipMemcpyAsync(out.data(), c->sub_out, out.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t k = 0; k < m; ++k)
        for (int d = 0; d < 3; ++d) {
            if (F_near) F_near[3 * k + d] = out[6 * k + d];
            if (F_far) F_far[3 * k + d] = out[6 * k + 3 + d];
        }
    return RBSOG_OK;
}

rbsog_status rbsog_get_energy(rbsog_ctx *c, double *E) {
    TRY(check_ctx(c));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    if (!E) return fail(c, RBSOG_E_ARG, "E is null");
    HIPCHK(c, hipMemcpyAsync(E, c->E, 4 * (size_t)c->nsys * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBSOG_OK;
}

rbsog_status rbsog_get_rho(rbsog_ctx *c, int32_t sys, double *re, double *im) {
    TRY(check_ctx(c));
    TRY(check_sys(c, sys));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    const SysHost &h = c->sys[sys];
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (re) HIPCHK(c, hipMemcpy(re, c->rho + h.k0, (size_t)h.P * sizeof(double), hipMemcpyDeviceToHost));
    if (im) HIPCHK(c, hipMemcpy(im, c->rho + c->K + h.k0, (size_t)h.P * sizeof(double), hipMemcpyDeviceToHost));
    return RBSOG_OK;
}

rbsog_status rbsog_get_kbatch(rbsog_ctx *c, int32_t sys, int32_t *m_out) {
    TRY(check_ctx(c));
    TRY(check_sys(c, sys));
    if (!m_out) return fail(c, RBSOG_E_ARG, "m_out is null");
    if (!c->forces_valid) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    const SysHost &h = c->sys[sys];
    std::vector<KRec32> r((size_t)h.P);
    HIPCHK(c, hipMemcpyAsync(r.data(), c->kb32 + h.k0, r.size() * sizeof(KRec32), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int32_t e = 0; e < h.P; ++e) {
        m_out[3 * e] = -r[e].nmx;
        m_out[3 * e + 1] = -r[e].nmy;
        m_out[3 * e + 2] = -r[e].nmz;
    }
    return RBSOG_OK;
}

rbsog_status rbsog_info(rbsog_ctx *c, int32_t sys, rbsog_info_t *info) {
    TRY(check_ctx(c));
    TRY(check_sys(c, sys));
    if (!info) return fail(c, RBSOG_E_ARG, "info is null");
    const SysHost &h = c->sys[sys];
    *info = rbsog_info_t{};
    info->S = h.S;
    info->volume = h.V;
    for (int d = 0; d < 3; ++d) info->ncell[d] = h.g.nc[d];
    info->k_remaining = c->lambda ? (int64_t)c->lambda * h.P - h.cursor : (int64_t)h.kseq.size() / 3 - h.cursor;
    info->evaluations = c->evals;
    info->n = h.n;
    info->n_sys = c->nsys;
    info->list_capacity = c->icap;
    info->skin = c->skin_cur;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&info->list_builds, c->nbuild, sizeof(int64_t), hipMemcpyDeviceToHost));
    info->rho_chunk = c->tune.rho_chunk;
    info->far_block = c->tune.far_block;
    for (const SysHost &h : c->sys) info->rho_ktile = std::max(info->rho_ktile, h.kt);
    info->build_slots = c->build_slots;
    info->cell_slots = c->cell_slots;
    info->list_home_major = c->list_hm ? 1 : 0;
    info->tuned = c->tuned ? 1 : 0;
    return RBSOG_OK;
}

rbsog_status rbsog_autotune(rbsog_ctx *c, int32_t reps) {
    TRY(check_ctx(c));
    if (c->prof_on) return fail(c, RBSOG_E_STATE, "autotuning is not available while profiling");
    return autotune_now(c, reps);
}

rbsog_status rbsog_debug_cells(rbsog_ctx *c, int32_t sys, int32_t *cell_start, int32_t *order) {
    TRY(check_ctx(c));
    TRY(check_sys(c, sys));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    const SysHost &h = c->sys[sys];
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (cell_start) {
        HIPCHK(c, hipMemcpy(cell_start, c->cell_start + h.c0, (size_t)(h.ncell + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToHost));
        for (int64_t k = 0; k <= h.ncell; ++k) cell_start[k] -= (int32_t)h.p0;
    }
    if (order) {
        HIPCHK(c, hipMemcpy(order, c->buf[0].id + h.p0, (size_t)h.n * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < h.n; ++k) order[k] -= (int32_t)h.p0;
    }
    return RBSOG_OK;
}

rbsog_status rbsog_debug_neighbors(rbsog_ctx *c, int32_t sys, int64_t *row_ptr, int32_t *cols, int64_t cap) {
    TRY(check_ctx(c));
    TRY(check_sys(c, sys));
    // the candidates come from the cells of the latest build, which cover
    // the neighbours only while the positions are those of an evaluation
    if (c->evals == 0 || !c->forces_valid)
        return fail(c, RBSOG_E_STATE, "needs the forces of the current positions first");
    if (!row_ptr) return fail(c, RBSOG_E_ARG, "row_ptr is null");
    const SysHost &h = c->sys[sys];
    const int64_t n = h.n;
    // the latest evaluation's arrays: its cell order is the current one
    EvalArgs a = make_args(c, false, 0.0);
    const int32_t *idc = c->buf[0].id;
    int64_t *dcount = nullptr;
    HIPCHK(c, hipMalloc((void **)&dcount, (size_t)(n + 1) * sizeof(int64_t)));
    launch_neighbor_count(a, sys, n, h.p0, idc, dcount, c->stream);
    std::vector<int64_t> cnt(n);
    hipError_t e = hipMemcpyAsync(cnt.data(), dcount, (size_t)n * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipFree(dcount);
        return fail(c, RBSOG_E_DEVICE, "neighbour count: %s", hipGetErrorString(e));
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    const int64_t total = row_ptr[n];
    if (!cols || cap < total) {
        (void)hipFree(dcount);
        return fail(c, RBSOG_E_ARG, "cols needs %lld entries", (long long)total);
    }
    int32_t *dcols = nullptr;
    e = hipMemcpy(dcount, row_ptr, (size_t)(n + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&dcols, (size_t)std::max<int64_t>(total, 1) * sizeof(int32_t));
    if (e == hipSuccess) {
        launch_neighbor_fill(a, sys, n, h.p0, idc, dcount, dcols, c->stream);
        e = hipMemcpyAsync(cols, dcols, (size_t)total * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(dcols);
    (void)hipFree(dcount);
    if (e != hipSuccess) return fail(c, RBSOG_E_DEVICE, "neighbour fill: %s", hipGetErrorString(e));
    return RBSOG_OK;
}

rbsog_status rbsog_debug_record_pairs(rbsog_ctx *c, int64_t cap) {
    TRY(check_ctx(c));
    if (cap < 0 || cap > (int64_t)INT32_MAX) return fail(c, RBSOG_E_ARG, "cap must be in [0, 2^31-1]");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (void *p : {(void *)c->dbg_pairs, (void *)c->dbg_cnt, (void *)c->dbg_kind}) {
        if (!p) continue;
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), p), c->allocs.end());
        (void)hipFree(p);
    }
    c->dbg_pairs = nullptr;
    c->dbg_cnt = c->dbg_kind = nullptr;
    c->dbg_cap = 0;
    drop_graphs(c);  // the captured steps hold the kernels' debug arguments
    if (cap == 0) return RBSOG_OK;
    TRY(dalloc(c, &c->dbg_pairs, cap));
    TRY(dalloc(c, &c->dbg_cnt, 1));
    TRY(dalloc(c, &c->dbg_kind, 1));
    HIPCHK(c, hipMemset(c->dbg_cnt, 0, sizeof(int32_t)));
    HIPCHK(c, hipMemset(c->dbg_kind, 0, sizeof(int32_t)));
    c->dbg_cap = (int32_t)cap;
    return RBSOG_OK;
}

// CSR over the local ids of system sys from (row, col) caller-index pairs:
// rows ascending, columns ascending within a row.  E_ARG (row_ptr filled) if
// cols holds fewer than the entries.
static rbsog_status csr_of_pairs(rbsog_ctx *c, const SysHost &h, const std::vector<uint2> &pairs, int64_t *row_ptr,
                                 int32_t *cols, int64_t cap) {
    std::vector<std::pair<int32_t, int32_t>> loc;
    loc.reserve(pairs.size());
    for (const uint2 &p : pairs) {
        const int64_t i = (int64_t)p.x - h.p0, j = (int64_t)p.y - h.p0;
        if (i >= 0 && i < h.n && j >= 0 && j < h.n) loc.emplace_back((int32_t)i, (int32_t)j);
    }
    std::sort(loc.begin(), loc.end());
    for (int64_t i = 0; i <= h.n; ++i) row_ptr[i] = 0;
    for (const auto &e : loc) row_ptr[e.first + 1] += 1;
    for (int64_t i = 0; i < h.n; ++i) row_ptr[i + 1] += row_ptr[i];
    if (!cols || cap < (int64_t)loc.size())
        return fail(c, RBSOG_E_ARG, "cols needs %lld entries", (long long)loc.size());
    for (size_t k = 0; k < loc.size(); ++k) cols[k] = loc[k].second;
    return RBSOG_OK;
}

rbsog_status rbsog_debug_pairs(rbsog_ctx *c, int32_t sys, int32_t *kinds, int64_t *row_ptr, int32_t *cols,
                               int64_t cap) {
    TRY(check_ctx(c));
    TRY(check_sys(c, sys));
    if (!c->dbg_pairs) return fail(c, RBSOG_E_STATE, "pair recording is off (rbsog_debug_record_pairs)");
    if (!row_ptr) return fail(c, RBSOG_E_ARG, "row_ptr is null");
    int32_t cnt = 0, kind = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&cnt, c->dbg_cnt, sizeof cnt, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(&kind, c->dbg_kind, sizeof kind, hipMemcpyDeviceToHost));
    if (kinds) *kinds = kind;
    if (cnt > c->dbg_cap)
        return fail(c, RBSOG_E_STATE, "the record holds %d pairs, the evaluation accepted %d", c->dbg_cap, cnt);
    std::vector<uint2> pairs((size_t)cnt);
    if (cnt > 0) HIPCHK(c, hipMemcpy(pairs.data(), c->dbg_pairs, (size_t)cnt * sizeof(uint2), hipMemcpyDeviceToHost));
    return csr_of_pairs(c, c->sys[sys], pairs, row_ptr, cols, cap);
}

rbsog_status rbsog_debug_list(rbsog_ctx *c, int32_t sys, int64_t *row_ptr, int32_t *cols, int64_t cap) {
    TRY(check_ctx(c));
    TRY(check_sys(c, sys));
    if (!(c->skin_cur > 0.0) || !c->pairs) return fail(c, RBSOG_E_STATE, "no near list is kept (skin 0)");
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    if (!row_ptr) return fail(c, RBSOG_E_ARG, "row_ptr is null");
    const SysHost &h = c->sys[sys];
    const int64_t nit = h.it1 - h.it0;
    std::vector<int32_t> pc((size_t)(nit * kListHomes));
    std::vector<uint32_t> ent((size_t)(nit * c->icap));
    std::vector<int32_t> id;
    TRY(current_ids(c, id));
    HIPCHK(c, hipMemcpy(pc.data(), c->pcnt + (int64_t)h.it0 * kListHomes, pc.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(ent.data(), c->pairs + (int64_t)h.it0 * c->icap, ent.size() * sizeof(uint32_t),
                        hipMemcpyDeviceToHost));
    std::vector<uint2> pairs;
    for (int64_t it = 0; it < nit; ++it) {
        const int64_t t0 = h.p0 + it * kListHomes;
        for (int hh = 0; hh < kListHomes; ++hh) {
            for (int32_t k = 0; k < pc[(size_t)(it * kListHomes + hh)]; ++k) {
                const int64_t at = c->list_hm ? (int64_t)hh * (c->icap / kListHomes) + k : (int64_t)k * kListHomes + hh;
                const uint32_t e = ent[(size_t)(it * c->icap + at)];
                pairs.push_back(make_uint2((uint32_t)id[(size_t)(t0 + hh)], (uint32_t)id[e >> 4]));
            }
        }
    }
    return csr_of_pairs(c, h, pairs, row_ptr, cols, cap);
}

rbsog_status rbsog_profile(rbsog_ctx *c, int32_t enable) {
    TRY(check_ctx(c));
    if (enable < 0 || enable > 2) return fail(c, RBSOG_E_ARG, "enable must be 0, 1 or 2");
    TRY(prof_collect(c));
    c->prof_on = enable;
    if (enable)
        for (int k = 0; k < K_COUNT; ++k) {
            c->prof[k].ms = 0.0;
            c->prof[k].launches = 0;
        }
    return RBSOG_OK;
}

rbsog_status rbsog_profile_read(rbsog_ctx *c, int32_t idx, const char **name, double *ms, int64_t *launches) {
    TRY(check_ctx(c));
    TRY(prof_collect(c));
    if (idx < 0 || idx >= K_COUNT) return RBSOG_E_ARG;
    if (name) *name = c->prof[idx].name;
    if (ms) *ms = c->prof[idx].ms;
    if (launches) *launches = c->prof[idx].launches;
    return RBSOG_OK;
}

}  // extern "C"

// ---- checkpoint ------------------------------------------------------------
// A saved state: a fixed header that names the context's shape, then every
// host and device quantity a later step reads, in a fixed order.  One writer
// serves both the size query (no buffer) and the copy.
namespace {

constexpr char kStateMagic[8] = {'R', 'B', 'S', 'O', 'G', 'S', 'T', '2'};

struct StateWriter {
    uint8_t *buf;  // null: count only
    int64_t cap, pos = 0;
    bool overflow = false;
    void raw(const void *p, int64_t n) {
        if (buf) {
            if (pos + n > cap) overflow = true;
            else std::memcpy(buf + pos, p, (size_t)n);
        }
        pos += n;
    }
    template <class T>
    void val(const T &v) { raw(&v, sizeof v); }
};

struct StateReader {
    const uint8_t *buf;
    int64_t len, pos = 0;
    bool bad = false;
    void raw(void *p, int64_t n) {
        if (pos + n > len) {
            bad = true;
            return;
        }
        std::memcpy(p, buf + pos, (size_t)n);
        pos += n;
    }
    template <class T>
    T val() {
        T v{};
        raw(&v, sizeof v);
        return v;
    }
};

// Device arrays of the state: (pointer, bytes).  The near list is saved by
// segment (its used entries only) elsewhere.
std::vector<std::pair<void *, int64_t>> device_state(rbsog_ctx *c) {
    const int64_t N = c->N;
    std::vector<std::pair<void *, int64_t>> v = {
        {c->buf[0].x, 3 * N * 8}, {c->buf[0].v, 3 * N * 8},  {c->buf[0].q, N * 8},
        {c->buf[0].qf, N * 4},    {c->buf[0].id, N * 4},     {c->buf[0].dsp, 3 * N * 8},
        {c->u_tmp, 3 * N * 4},    {c->u, 3 * N * 4},         {c->cell_sorted, N * 4},
        {c->cell_start, (c->C + 1) * 4}, {c->Fn, 3 * N * 8}, {c->Ff, 3 * N * 8},
        {c->rebuild, 4},          {c->nbuild, 8},            {c->kcur, (int64_t)c->nsys * 8},
        {c->kin, (int64_t)c->nsys * 8}, {c->nh_xi, (int64_t)c->nsys * 8}, {c->tstep, 8},
        {c->E, 4 * (int64_t)c->nsys * 8}, {c->rho, 2 * (int64_t)c->K * 8},
        {c->kb64, (int64_t)c->K * (int64_t)sizeof(KRec64)}, {c->kb32, (int64_t)c->K * (int64_t)sizeof(KRec32)},
        {c->dipole, 3 * (int64_t)c->nsys * 8}, {c->flag, 4}};
    if (c->lambda) {
        v.push_back({c->chains, (int64_t)c->nsys * c->lambda * (int64_t)sizeof(ChainState)});
        for (const SysHost &h : c->sys) v.push_back({h.dkseq, (int64_t)c->lambda * h.P * 3 * 4});
    }
    return v;
}

rbsog_status write_state(rbsog_ctx *c, StateWriter &w) {
    w.raw(kStateMagic, 8);
    w.val<int32_t>(c->nsys);
    w.val<int64_t>(c->N);
    w.val<int64_t>(c->C);
    w.val<int32_t>(c->K);
    w.val<int32_t>(c->prec);
    w.val<int32_t>(c->lambda);
    for (const SysHost &h : c->sys) {
        w.val(h.n);
        w.val(h.P);
        w.raw(h.box, sizeof h.box);
        w.val(h.rc);
        w.val(h.seed);
    }
    // host state
    w.val(c->evals);
    w.val<int32_t>(c->forces_valid);
    w.val(c->skin_cur);
    w.val(c->adapt_steps);
    w.val(c->adapt_nb0);
    w.val(c->adapt_window);
    w.val(c->hold);
    w.val(c->hold_len);
    w.val(c->gamma);
    w.val(c->temp);
    w.val(c->tseed);
    w.val<int32_t>(c->nh_on);
    w.val(c->nh_T);
    w.val(c->nh_tau);
    w.val<int32_t>(c->msd_on);
    w.val(c->tune);
    w.val<int32_t>(c->tuned);
    w.val(c->icap);
    for (const SysHost &h : c->sys) {
        w.val(h.chain);
        w.val(h.cursor);
        w.val<int32_t>(h.custom_w);
        w.val<int64_t>((int64_t)h.kseq.size());
        w.raw(h.kseq.data(), (int64_t)h.kseq.size() * 4);
        w.val<int64_t>((int64_t)h.kw.size());
        w.raw(h.kw.data(), (int64_t)h.kw.size() * 8);
        w.val(h.nh_nf);
        w.val(h.nh_Q);
    }
    // device state
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (const auto &a : device_state(c)) {
        if (w.buf && w.pos + a.second <= w.cap) {
            HIPCHK(c, hipMemcpy(w.buf + w.pos, a.first, (size_t)a.second, hipMemcpyDeviceToHost));
        } else if (w.buf) {
            w.overflow = true;
        }
        w.pos += a.second;
    }
    // the near list is not stored: it is a function of the saved reference
    // positions, cells and launch shapes, and loading lists it again
    const bool list = c->skin_cur > 0.0 && c->pairs;
    w.val<int32_t>(list ? 1 : 0);
    w.val<int32_t>(c->list_hm ? 1 : 0);
    return RBSOG_OK;
}

}  // namespace

extern "C" {

rbsog_status rbsog_save_state(rbsog_ctx *c, void *buf, int64_t cap, int64_t *size) {
    TRY(check_ctx(c));
    StateWriter probe{nullptr, 0};
    TRY(write_state(c, probe));
    if (size) *size = probe.pos;
    if (!buf) return RBSOG_OK;
    if (cap < probe.pos) return fail(c, RBSOG_E_ARG, "the state needs %lld bytes", (long long)probe.pos);
    StateWriter w{(uint8_t *)buf, cap};
    TRY(write_state(c, w));
    if (w.overflow) return fail(c, RBSOG_E_ARG, "the state needs %lld bytes", (long long)w.pos);
    return RBSOG_OK;
}

rbsog_status rbsog_load_state(rbsog_ctx *c, const void *buf, int64_t len) {
    TRY(check_ctx(c));
    if (!buf || len < 8) return fail(c, RBSOG_E_ARG, "no state");
    StateReader r{(const uint8_t *)buf, len};
    char magic[8];
    r.raw(magic, 8);
    if (std::memcmp(magic, kStateMagic, 8) != 0) return fail(c, RBSOG_E_ARG, "not a saved state of this library");
    const int32_t nsys = r.val<int32_t>();
    const int64_t N = r.val<int64_t>(), C = r.val<int64_t>();
    const int32_t K = r.val<int32_t>(), prec = r.val<int32_t>(), lambda = r.val<int32_t>();
    if (nsys != c->nsys || N != c->N || C != c->C || K != c->K || prec != c->prec || lambda != c->lambda)
        return fail(c, RBSOG_E_ARG, "the state belongs to a context of another shape (systems, particles, "
                                    "cells, wave vectors, precision or device chains differ)");
    for (const SysHost &h : c->sys) {
        const int64_t n = r.val<int64_t>();
        const int32_t P = r.val<int32_t>();
        double box[3];
        r.raw(box, sizeof box);
        const double rc = r.val<double>();
        const uint64_t seed = r.val<uint64_t>();
        if (n != h.n || P != h.P || std::memcmp(box, h.box, sizeof box) != 0 || rc != h.rc || seed != h.seed)
            return fail(c, RBSOG_E_ARG, "the state belongs to other systems (n, P, box, r_c or seed differ)");
    }
    if (r.bad) return fail(c, RBSOG_E_ARG, "truncated state");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // host state (applied once the whole buffer has been read)
    const int64_t evals = r.val<int64_t>();
    const int32_t forces_valid = r.val<int32_t>();
    const double skin_cur = r.val<double>();
    const int64_t adapt_steps = r.val<int64_t>(), adapt_nb0 = r.val<int64_t>(), adapt_window = r.val<int64_t>();
    const int32_t hold = r.val<int32_t>(), hold_len = r.val<int32_t>();
    const double gamma = r.val<double>(), temp = r.val<double>();
    const uint64_t tseed = r.val<uint64_t>();
    const int32_t nh_on = r.val<int32_t>();
    const double nh_T = r.val<double>(), nh_tau = r.val<double>();
    const int32_t msd_on = r.val<int32_t>();
    const Tune tune = r.val<Tune>();
    const int32_t tuned = r.val<int32_t>();
    const int64_t icap = r.val<int64_t>();
    struct SysState {
        MHChain chain;
        int64_t cursor;
        int32_t custom_w;
        std::vector<int32_t> kseq;
        std::vector<double> kw;
        double nh_nf, nh_Q;
    };
    std::vector<SysState> ss((size_t)c->nsys);
    for (SysState &x : ss) {
        x.chain = r.val<MHChain>();
        x.cursor = r.val<int64_t>();
        x.custom_w = r.val<int32_t>();
        const int64_t nk = r.val<int64_t>();
        if (r.bad || nk < 0 || nk > (len - r.pos) / 4) return fail(c, RBSOG_E_ARG, "truncated state");
        x.kseq.resize((size_t)nk);
        r.raw(x.kseq.data(), nk * 4);
        const int64_t nw = r.val<int64_t>();
        if (r.bad || nw < 0 || nw > (len - r.pos) / 8) return fail(c, RBSOG_E_ARG, "truncated state");
        x.kw.resize((size_t)nw);
        r.raw(x.kw.data(), nw * 8);
        x.nh_nf = r.val<double>();
        x.nh_Q = r.val<double>();
    }
    if (r.bad || !valid_tune(tune) || !(skin_cur >= 0.0)) return fail(c, RBSOG_E_ARG, "corrupt state");
    {
        // the device arrays (fixed sizes for this shape) must all be there
        // before anything of the context changes
        int64_t dev = 0;
        for (const auto &a : device_state(c)) dev += a.second;
        if (r.pos + dev + 4 > len) return fail(c, RBSOG_E_ARG, "truncated state");
    }
    // the saved grid, shapes and list capacity first (they size what follows)
    for (SysHost &h : c->sys) set_geometry(h, skin_cur);
    c->skin_cur = skin_cur;
    TRY(apply_tune(c, tune));
    c->tuned = tuned != 0;
    TRY(upload_cell_items(c));
    if (skin_cur > 0.0 && icap != c->icap) {
        // a list of the saved capacity
        uint32_t *np = nullptr;
        if (hipMalloc((void **)&np, (size_t)c->n_list * (size_t)icap * sizeof(uint32_t)) != hipSuccess)
            return fail(c, RBSOG_E_OOM, "pair list of %lld x %lld entries", (long long)c->n_list, (long long)icap);
        if (c->pairs) {
            c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void *)c->pairs), c->allocs.end());
            (void)hipFree(c->pairs);
        }
        c->pairs = np;
        c->allocs.push_back(np);
        c->icap = icap;
    }
    // sequences of the host chains: device copies of the right capacity
    for (int32_t s = 0; s < c->nsys; ++s) {
        SysHost &h = c->sys[s];
        h.chain = ss[s].chain;
        h.cursor = ss[s].cursor;
        h.custom_w = ss[s].custom_w != 0;
        h.kseq = std::move(ss[s].kseq);
        h.kw = std::move(ss[s].kw);
        h.nh_nf = ss[s].nh_nf;
        h.nh_Q = ss[s].nh_Q;
        if (!c->lambda) TRY(upload_k(c, s, 0));
        TRY(upload_sysdev(c, s));
    }
    for (const auto &a : device_state(c)) {
        if (r.pos + a.second > len) return fail(c, RBSOG_E_ARG, "truncated state");
        HIPCHK(c, hipMemcpy(a.first, r.buf + r.pos, (size_t)a.second, hipMemcpyHostToDevice));
        r.pos += a.second;
    }
    const int32_t list = r.val<int32_t>();
    const int32_t list_hm = r.val<int32_t>();
    if (r.bad) return fail(c, RBSOG_E_ARG, "truncated state");
    if (list) {
        if (!(skin_cur > 0.0) || !c->pairs) return fail(c, RBSOG_E_ARG, "corrupt state");
        // the list of the saved build, listed again from the saved reference
        // positions and cells by the build kernel (no re-sort, no copy back)
        c->list_hm = list_hm != 0;
        TRY(relist(c));
    }
    c->evals = evals;
    c->forces_valid = forces_valid != 0;
    c->adapt_steps = adapt_steps;
    c->adapt_nb0 = adapt_nb0;
    c->adapt_window = adapt_window;
    c->hold = hold;
    c->hold_len = hold_len;
    c->gamma = gamma;
    c->temp = temp;
    c->tseed = tseed;
    c->nh_on = nh_on != 0;
    c->nh_T = nh_T;
    c->nh_tau = nh_tau;
    c->msd_on = msd_on != 0;
    drop_graphs(c);  // the captured steps hold the old constants
    return RBSOG_OK;
}

rbsog_status rbsog_sync(rbsog_ctx *c) {
    TRY(check_ctx(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBSOG_OK;
}

const char *rbsog_last_error(const rbsog_ctx *c) { return c ? c->err.c_str() : g_init_error; }

const char *rbsog_status_string(rbsog_status s) {
    switch (s) {
    case RBSOG_OK: return "ok";
    case RBSOG_E_ARG: return "invalid argument";
    case RBSOG_E_NOT_NEUTRAL: return "system not neutral";
    case RBSOG_E_CUTOFF: return "cutoff out of range";
    case RBSOG_E_SOG: return "invalid split parameters";
    case RBSOG_E_DEVICE: return "device error";
    case RBSOG_E_OOM: return "out of device memory";
    case RBSOG_E_NONFINITE: return "non-finite value";
    case RBSOG_E_KSEQ: return "wave-vector sequence exhausted";
    case RBSOG_E_STATE: return "invalid state";
    }
    return "unknown status";
}

void rbsog_destroy(rbsog_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto &p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    drop_graphs(c);
    for (void *p : c->allocs) (void)hipFree(p);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
