// Host side of librbsog: the C ABI of include/rbsog.h.  Validates inputs,
// builds the split coefficients and the normaliser S, runs the wave-vector
// sampler, owns the device memory and enqueues the kernels of one force
// evaluation / one velocity-Verlet step on a single HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rbsog_internal.h"

using namespace rbsog;

namespace {

thread_local std::string g_init_error;

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwo32 = 4294967296.0;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): counter-based generator used by the
// k sampler and the Maxwellian velocity draw.
struct Philox {
    static void block(uint32_t c[4], uint32_t k0, uint32_t k1) {
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
    // Two 53-bit uniforms in [0, 1) from counter (idx_lo, idx_hi, stream, lane).
    static void uniform2(uint64_t seed, uint32_t stream, uint64_t idx, uint32_t lane, double &a, double &b) {
        uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), stream, lane};
        block(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint64_t w0 = ((uint64_t)c[1] << 32) | c[0];
        const uint64_t w1 = ((uint64_t)c[3] << 32) | c[2];
        a = (double)(w0 >> 11) * 0x1.0p-53;
        b = (double)(w1 >> 11) * 0x1.0p-53;
    }
};

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

enum Kid { K_KDQ, K_SCAN, K_SCATTER, K_SORTG, K_NEAR, K_RHO, K_RHORED, K_FAR, K_COUNT };
const char *kKernelNames[K_COUNT] = {"kick_drift_quantise", "scan_cell_counts", "cell_scatter", "sort_gather",
                                     "near",                "rho",              "rho_reduce",   "far"};

}  // namespace

struct rbsog_ctx {
    // system
    int64_t n = 0;
    double box[3] = {0, 0, 0};
    double rc = 0;
    int32_t P = 0;
    uint64_t seed = 0;
    int prec = RBSOG_FP64;
    int device = 0;
    double mass = 1.0;
    // split
    int M = 0;
    std::vector<double> omega, s;
    double S = 0, V = 0, uself = 0, w_rb = 0;
    Geom geom{};
    int64_t ncell = 0;
    FarPlan fplan{};
    NearPlan nplan{};
    // sequence
    MHChain chain;
    std::vector<int32_t> kseq;
    std::vector<double> kw;
    bool custom_w = false;
    int64_t cursor = 0;
    int64_t kcap = 0;
    // state
    bool forces_valid = false;
    int64_t evals = 0;
    bool poisoned = false;
    std::string err;
    // stream
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // device memory
    std::vector<void *> allocs;
    double *x = nullptr, *v = nullptr, *q = nullptr, *Fn = nullptr, *Ff = nullptr;
    float *qf = nullptr, *sqf = nullptr;
    uint32_t *u = nullptr, *su = nullptr;
    double *sx = nullptr, *sq = nullptr;
    int32_t *cell_of = nullptr, *cell_count = nullptr, *cell_start = nullptr, *cell_fill = nullptr,
            *order = nullptr, *blocksums = nullptr;
    int32_t *dkseq = nullptr;
    double *dkw = nullptr;
    int64_t *dcursor = nullptr;
    KRec64 *kb64 = nullptr;
    KRec32 *kb32 = nullptr;
    double *wk = nullptr, *rho = nullptr, *ek = nullptr, *partial = nullptr, *epart = nullptr, *E = nullptr;
    int32_t *flag = nullptr;
    uint32_t *counter = nullptr;
    SplitCoef64 co64{};
    SplitCoef32 co32{};
    // graph of one velocity-Verlet step
    bool use_graphs = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    double graph_dt = 0.0;
    const void *graph_key[3] = {nullptr, nullptr, nullptr};
    // profiling
    bool prof_on = false;
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
        g_init_error = buf;
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
double target_weight(const rbsog_ctx *c, const int32_t m[3]) {
    const double t = (double)m[0] * m[0] / (c->box[0] * c->box[0]) + (double)m[1] * m[1] / (c->box[1] * c->box[1]) +
                     (double)m[2] * m[2] / (c->box[2] * c->box[2]);
    double acc = 0.0;
    for (int l = 0; l <= c->M; ++l)
        acc += c->omega[l] * c->s[l] * c->s[l] * c->s[l] * std::exp(-kPi * kPi * c->s[l] * c->s[l] * t);
    return acc;
}

double proposal_1d(int32_t m, double a) {
    if (m == 0) return std::erf(0.5 * a);
    const double am = std::fabs((double)m);
    return 0.5 * (std::erfc((am - 0.5) * a) - std::erfc((am + 0.5) * a));
}

void mh_extend(rbsog_ctx *c, int64_t count, std::vector<int32_t> &out) {
    MHChain &ch = c->chain;
    const double s0 = c->s[0];
    double sd[3], a[3];
    for (int d = 0; d < 3; ++d) {
        sd[d] = c->box[d] / (std::sqrt(2.0) * kPi * s0);
        a[d] = kPi * s0 / c->box[d];
    }
    int64_t made = 0;
    while (made < count) {
        double u1, u2, u3, u4, ua, ub;
        Philox::uniform2(c->seed, 0, ch.attempt, 0, u1, u2);
        Philox::uniform2(c->seed, 0, ch.attempt, 1, u3, u4);
        Philox::uniform2(c->seed, 0, ch.attempt, 2, ua, ub);
        ++ch.attempt;
        const double r1 = std::sqrt(-2.0 * std::log(1.0 - u1));
        const double r2 = std::sqrt(-2.0 * std::log(1.0 - u3));
        const double z[3] = {r1 * std::cos(2.0 * kPi * u2), r1 * std::sin(2.0 * kPi * u2), r2 * std::cos(2.0 * kPi * u4)};
        int32_t cand[3];
        for (int d = 0; d < 3; ++d) cand[d] = (int32_t)std::round(z[d] * sd[d]);
        if (cand[0] == 0 && cand[1] == 0 && cand[2] == 0) continue;
        const double pc = target_weight(c, cand);
        const double qc = proposal_1d(cand[0], a[0]) * proposal_1d(cand[1], a[1]) * proposal_1d(cand[2], a[2]);
        if (!ch.started) {
            std::copy(cand, cand + 3, ch.m);
            ch.p = pc;
            ch.qprop = qc;
            ch.started = true;
            continue;
        }
        if (ua < (pc * ch.qprop) / (ch.p * qc)) {
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
rbsog_status timed(rbsog_ctx *c, int kid, F &&launch) {
    if (!c->prof_on) {
        launch();
        return RBSOG_OK;
    }
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return fail(c, RBSOG_E_DEVICE, "hipEventCreate failed");
    HIPCHK(c, hipEventRecord(a, c->stream));
    launch();
    HIPCHK(c, hipEventRecord(b, c->stream));
    c->pending.push_back({kid, a, b});
    if (c->pending.size() > 8192) return prof_collect(c);
    return RBSOG_OK;
}

// ---- device orchestration --------------------------------------------------------
rbsog_status ensure_kcap(rbsog_ctx *c, int64_t nvec) {
    if (nvec <= c->kcap) return RBSOG_OK;
    int64_t cap = std::max<int64_t>(nvec, 2 * c->kcap);
    int32_t *nk = nullptr;
    double *nw = nullptr;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (hipMalloc((void **)&nk, (size_t)cap * 3 * sizeof(int32_t)) != hipSuccess)
        return fail(c, RBSOG_E_OOM, "sequence buffer of %lld vectors", (long long)cap);
    if (hipMalloc((void **)&nw, (size_t)cap * sizeof(double)) != hipSuccess) {
        (void)hipFree(nk);
        return fail(c, RBSOG_E_OOM, "weight buffer of %lld vectors", (long long)cap);
    }
    if (c->dkseq) {
        HIPCHK(c, hipMemcpy(nk, c->dkseq, (size_t)c->kcap * 3 * sizeof(int32_t), hipMemcpyDeviceToDevice));
        HIPCHK(c, hipMemcpy(nw, c->dkw, (size_t)c->kcap * sizeof(double), hipMemcpyDeviceToDevice));
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void *)c->dkseq), c->allocs.end());
        c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), (void *)c->dkw), c->allocs.end());
        (void)hipFree(c->dkseq);
        (void)hipFree(c->dkw);
    }
    c->dkseq = nk;
    c->dkw = nw;
    c->allocs.push_back(nk);
    c->allocs.push_back(nw);
    c->kcap = cap;
    return RBSOG_OK;
}

rbsog_status upload_k(rbsog_ctx *c, int64_t from) {
    const int64_t nvec = (int64_t)c->kseq.size() / 3;
    TRY(ensure_kcap(c, nvec));
    if (nvec > from) {
        HIPCHK(c, hipMemcpy(c->dkseq + 3 * from, c->kseq.data() + 3 * from, (size_t)(nvec - from) * 3 * sizeof(int32_t),
                            hipMemcpyHostToDevice));
        if (c->custom_w)
            HIPCHK(c, hipMemcpy(c->dkw + from, c->kw.data() + from, (size_t)(nvec - from) * sizeof(double),
                                hipMemcpyHostToDevice));
    }
    return RBSOG_OK;
}

// Enqueue one force evaluation (with the velocity-Verlet kick-drift before
// and the closing kick after it when dt != 0).  Pure launches: no host state
// changes, so it can be captured into a graph.
rbsog_status enqueue_eval(rbsog_ctx *c, bool stepping, double dt) {
    hipStream_t s = c->stream;
    const Geom &g = c->geom;
    const bool f64 = c->prec == RBSOG_FP64;
    KickArgs kick{stepping ? 1 : 0, 0.5 * dt / c->mass, dt, c->v, c->Fn, c->Ff, c->flag};
    StageArgs stage{c->P, c->dkseq, c->custom_w ? c->dkw : nullptr, c->w_rb, c->dcursor, c->kb64, c->kb32, c->wk};
    TRY(timed(c, K_KDQ, [&] { launch_kdq(g, kick, stage, c->x, c->u, c->cell_of, c->cell_count, s); }));
    TRY(timed(c, K_SCAN, [&] { launch_scan(c->cell_count, c->cell_start, c->cell_fill, c->ncell, c->blocksums, s); }));
    TRY(timed(c, K_SCATTER, [&] { launch_cell_scatter(g, c->cell_of, c->cell_fill, c->order, s); }));
    TRY(timed(c, K_SORTG, [&] {
        launch_sort_gather(g, c->ncell, c->cell_start, c->order, c->cell_count, c->u, c->x, c->q, c->su, c->sx, c->sq,
                           c->sqf, f64, s);
    }));
    TRY(timed(c, K_NEAR, [&] {
        launch_near(g, c->co64, c->co32, f64, c->nplan, c->ncell, c->cell_start, c->order, c->su, c->sx, c->sq, c->sqf, c->Fn,
                    c->epart, s);
    }));
    TRY(timed(c, K_RHO, [&] {
        launch_rho(g, c->fplan, c->P, f64, c->x, c->u, c->q, c->qf, c->kb64, c->kb32, c->partial, s);
    }));
    TRY(timed(c, K_RHORED, [&] {
        launch_rho_reduce(c->P, c->fplan.nblk, c->partial, c->wk, c->kb64, c->kb32, c->rho, c->ek, c->nplan.nblk,
                          c->epart, c->uself, c->E, c->flag, c->counter, s);
    }));
    TRY(timed(c, K_FAR, [&] { launch_far(g, c->P, f64, c->x, c->u, c->q, c->qf, c->kb64, c->kb32, c->Ff, kick, s); }));
    HIPCHK(c, hipGetLastError());
    return RBSOG_OK;
}

void account_eval(rbsog_ctx *c) {
    c->cursor += c->P;
    c->evals += 1;
    c->forces_valid = true;
}

void drop_graph(rbsog_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
}

// The graph of one step captures the kernel arguments: it is rebuilt when dt
// or a buffer it reads (the sequence and its weights) changes.
rbsog_status ensure_step_graph(rbsog_ctx *c, double dt) {
    const void *key[3] = {c->dkseq, c->custom_w ? (const void *)c->dkw : nullptr, (const void *)c->x};
    if (c->graph_exec && c->graph_dt == dt && std::equal(key, key + 3, c->graph_key)) return RBSOG_OK;
    drop_graph(c);
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    rbsog_status st = enqueue_eval(c, true, dt);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st != RBSOG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(c, RBSOG_E_DEVICE, "stream capture: %s", hipGetErrorString(e));
    c->graph = g;
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(c);
        return fail(c, RBSOG_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    c->graph_dt = dt;
    std::copy(key, key + 3, c->graph_key);
    return RBSOG_OK;
}

bool usable(rbsog_ctx *c) { return c && !c->poisoned; }

rbsog_status check_ctx(rbsog_ctx *c) {
    if (!c) return fail(nullptr, RBSOG_E_ARG, "null context");
    if (c->poisoned) return fail(c, RBSOG_E_STATE, "context is poisoned after a device error: %s", c->err.c_str());
    HIPCHK(c, hipSetDevice(c->device));
    return RBSOG_OK;
}

rbsog_status upload_positions(rbsog_ctx *c, const double *pos) {
    std::vector<double> soa((size_t)c->n * 3);
    for (int64_t i = 0; i < c->n; ++i)
        for (int d = 0; d < 3; ++d) {
            const double v = pos[3 * i + d];
            if (!std::isfinite(v)) return fail(c, RBSOG_E_NONFINITE, "position %lld is not finite", (long long)i);
            soa[(size_t)d * c->n + i] = v;
        }
    HIPCHK(c, hipMemcpy(c->x, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice));
    c->forces_valid = false;
    return RBSOG_OK;
}

rbsog_status soa_to_host(rbsog_ctx *c, const double *dev, double *host) {
    std::vector<double> soa((size_t)c->n * 3);
    HIPCHK(c, hipMemcpyAsync(soa.data(), dev, soa.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < c->n; ++i)
        for (int d = 0; d < 3; ++d) host[3 * i + d] = soa[(size_t)d * c->n + i];
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
    if (!pos || !q || !box || !sog) return fail(nullptr, RBSOG_E_ARG, "null input pointer");
    if (n < 2 || n > (int64_t)INT32_MAX) return fail(nullptr, RBSOG_E_ARG, "n must be in [2, 2^31-1]");
    if (P < 1) return fail(nullptr, RBSOG_E_ARG, "P must be >= 1");
    rbsog_opts o;
    rbsog_default_opts(&o);
    if (opts) o = *opts;
    if (o.precision != RBSOG_FP64 && o.precision != RBSOG_FP32C)
        return fail(nullptr, RBSOG_E_ARG, "unknown precision %d", o.precision);
    if (!(o.mass > 0.0) || !std::isfinite(o.mass)) return fail(nullptr, RBSOG_E_ARG, "mass must be > 0");
    if (!(o.neutral_tol >= 0.0)) return fail(nullptr, RBSOG_E_ARG, "neutral_tol must be >= 0");
    for (int d = 0; d < 3; ++d)
        if (!(box[d] > 0.0) || !std::isfinite(box[d])) return fail(nullptr, RBSOG_E_ARG, "box sides must be > 0");
    if (!(sog->b > 1.0) || !std::isfinite(sog->b) || !(sog->sigma > 0.0) || !std::isfinite(sog->sigma) ||
        !(sog->w0 > 0.0) || !std::isfinite(sog->w0) || sog->M < 0 || sog->M + 1 > kMaxGauss)
        return fail(nullptr, RBSOG_E_SOG, "split parameters need b > 1, sigma > 0, w0 > 0, 0 <= M < %d", kMaxGauss);
    const double lmin = std::min(box[0], std::min(box[1], box[2]));
    if (!(rc > 0.0) || !(rc <= 0.5 * lmin)) return fail(nullptr, RBSOG_E_CUTOFF, "need 0 < rc <= min(L)/2");
    double qs = 0.0, qa = 0.0, q2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(q[i])) return fail(nullptr, RBSOG_E_NONFINITE, "charge %lld is not finite", (long long)i);
        qs += q[i];
        qa += std::fabs(q[i]);
        q2 += q[i] * q[i];
    }
    if (std::fabs(qs) > o.neutral_tol * qa)
        return fail(nullptr, RBSOG_E_NOT_NEUTRAL, "sum q = %.17g exceeds %.3g * sum|q|", qs, o.neutral_tol);
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(pos[i])) return fail(nullptr, RBSOG_E_NONFINITE, "position entry %lld is not finite",
                                                (long long)i);

    rbsog_ctx *c = new rbsog_ctx();
    c->n = n;
    std::copy(box, box + 3, c->box);
    c->rc = rc;
    c->P = P;
    c->seed = seed;
    c->prec = o.precision;
    c->device = o.device;
    c->mass = o.mass;
    c->use_graphs = o.graphs != 0;
    c->M = sog->M;
    sog_coefficients(*sog, c->omega, c->s);
    c->V = box[0] * box[1] * box[2];
    c->S = normaliser_S(c->omega, c->s, box);
    c->w_rb = c->S * std::pow(kPi, 1.5) / ((double)P * c->V);
    double f0 = 0.0;
    for (double w : c->omega) f0 += w;
    c->uself = 0.5 * f0 * q2;
    for (int k = 0; k < K_COUNT; ++k) c->prof[k].name = kKernelNames[k];

    Geom &g = c->geom;
    g.n = n;
    double hmax = 0.0;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = box[d];
        g.invL[d] = 1.0 / box[d];
        g.h[d] = box[d] / kTwo32;
        g.hf[d] = (float)g.h[d];
        hmax = std::max(hmax, g.h[d]);
        const int64_t k = (int64_t)std::floor(box[d] / rc);
        g.nc[d] = (int32_t)(k >= 3 ? k : 1);
        g.reach[d] = g.nc[d] >= 3 ? 1 : 0;
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
    // Gaussians wide enough that exp(-x/s_l^2) is a short Taylor series over
    // x = r^2 <= rc^2 form the tail; s_l grows with l, so they are l >= nexp.
    auto first_wide = [&](double tau) {
        for (int l = 0; l <= c->M; ++l)
            if (rc * rc / (c->s[l] * c->s[l]) <= tau) return l;
        return c->M + 1;
    };
    const int nexp64 = first_wide(kTailTau64), nexp32 = first_wide(kTailTau32);
    if (nexp64 > kMaxExp) {
        delete c;
        return fail(nullptr, RBSOG_E_SOG, "more than 24 Gaussians narrower than r_c / sqrt(0.05)");
    }
    c->ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
    if (c->ncell >= (int64_t)INT32_MAX) {
        delete c;
        return fail(nullptr, RBSOG_E_ARG, "too many cells");
    }
    c->fplan = far_plan(n, P);
    c->nplan = near_plan(c->ncell);

    auto bail = [&](rbsog_status st) {
        g_init_error = c->err;
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
    rbsog_status st = RBSOG_OK;
#define ALLOC(ptr, cnt)                                   \
    if ((st = dalloc(c, &c->ptr, (cnt))) != RBSOG_OK) return bail(st);
    ALLOC(x, 3 * n);
    ALLOC(v, 3 * n);
    ALLOC(q, n);
    ALLOC(qf, n);
    ALLOC(Fn, 3 * n);
    ALLOC(Ff, 3 * n);
    ALLOC(u, 3 * n);
    ALLOC(su, 3 * n);
    ALLOC(sqf, n);
    if (c->prec == RBSOG_FP64) {
        ALLOC(sx, 3 * n);
        ALLOC(sq, n);
    }
    ALLOC(cell_of, n);
    ALLOC(order, n);
    ALLOC(cell_count, c->ncell);
    ALLOC(cell_start, c->ncell + 1);
    ALLOC(cell_fill, c->ncell);
    ALLOC(blocksums, scan_blocksums_size(c->ncell));
    ALLOC(dcursor, 1);
    ALLOC(kb64, P);
    ALLOC(kb32, P);
    ALLOC(wk, P);
    ALLOC(rho, 2 * (int64_t)P);
    ALLOC(ek, P);
    ALLOC(partial, 2 * c->fplan.nblk * (int64_t)P);
    ALLOC(epart, c->nplan.nblk);
    ALLOC(E, 4);
    ALLOC(flag, 1);
    ALLOC(counter, 1);
#undef ALLOC
    {
        // explicit Gaussians and the tail polynomials:
        // sum_{l >= nexp} omega_l e^{-x a_l} = sum_k (-1)^k/k! (sum_l omega_l a_l^k) x^k
        // and the force weights 2 omega_l a_l e^{-x a_l} likewise (a_l = 1/s_l^2)
        const int G = c->M + 1;
        auto tail = [&](int l0, int k) {
            double sp = 0.0, sf = 0.0, fact = 1.0;
            for (int i = 2; i <= k; ++i) fact *= i;
            for (int l = l0; l < G; ++l) {
                const double a = 1.0 / (c->s[l] * c->s[l]);
                sp += c->omega[l] * std::pow(a, k);
                sf += 2.0 * c->omega[l] * std::pow(a, k + 1);
            }
            const double sgn = (k & 1) ? -1.0 : 1.0;
            return std::make_pair(sgn * sp / fact, sgn * sf / fact);
        };
        SplitCoef64 &h64 = c->co64;
        SplitCoef32 &h32 = c->co32;
        h64.nexp = nexp64;
        h32.nexp = nexp32;
        for (int l = 0; l < nexp64; ++l) {
            const double is2 = 1.0 / (c->s[l] * c->s[l]);
            h64.a[l] = is2;
            h64.cw[l] = 2.0 * c->omega[l] * is2;
            h64.w[l] = c->omega[l];
        }
        for (int l = 0; l < nexp32; ++l) {
            const double is2 = 1.0 / (c->s[l] * c->s[l]);
            h32.a[l] = (float)(is2 / std::log(2.0));
            h32.cw[l] = (float)(2.0 * c->omega[l] * is2);
            h32.w[l] = (float)c->omega[l];
        }
        for (int k = 0; k <= kTailDeg64; ++k) {
            const auto pf = tail(nexp64, k);
            h64.pt[k] = pf.first;
            h64.ft[k] = pf.second;
        }
        for (int k = 0; k <= kTailDeg32; ++k) {
            const auto pf = tail(nexp32, k);
            h32.pt[k] = (float)pf.first;
            h32.ft[k] = (float)pf.second;
        }
    }
    {
        std::vector<double> qd(q, q + n);
        std::vector<float> qff(n);
        for (int64_t i = 0; i < n; ++i) qff[i] = (float)q[i];
        std::vector<double> zero((size_t)3 * n, 0.0);
        const int64_t zc = 0;
        const int32_t zf = 0;
        if (hipMemcpy(c->q, qd.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->qf, qff.data(), n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->v, zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->Fn, zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->Ff, zero.data(), zero.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->dcursor, &zc, sizeof zc, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->flag, &zf, sizeof zf, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(c->counter, 0, sizeof(uint32_t)) != hipSuccess ||
            hipMemset(c->cell_count, 0, (size_t)c->ncell * sizeof(int32_t)) != hipSuccess) {
            fail(c, RBSOG_E_DEVICE, "initial upload failed");
            return bail(RBSOG_E_DEVICE);
        }
    }
    if ((st = upload_positions(c, pos)) != RBSOG_OK) return bail(st);
    if ((st = ensure_kcap(c, 4 * (int64_t)P)) != RBSOG_OK) return bail(st);
    *out = c;
    return RBSOG_OK;
}

rbsog_status rbsog_sample_k(rbsog_ctx *c, int64_t n_batches, int32_t *m_out) {
    TRY(check_ctx(c));
    if (n_batches < 1) return fail(c, RBSOG_E_ARG, "n_batches must be >= 1");
    const int64_t from = (int64_t)c->kseq.size() / 3;
    if (c->custom_w) {
        // a caller-given weighted list is replaced by the sampled sequence
        c->kseq.clear();
        c->kw.clear();
        c->custom_w = false;
        c->cursor = 0;
        const int64_t zc = 0;
        HIPCHK(c, hipMemcpy(c->dcursor, &zc, sizeof zc, hipMemcpyHostToDevice));
    }
    const int64_t start = (int64_t)c->kseq.size() / 3;
    std::vector<int32_t> fresh;
    fresh.reserve((size_t)(n_batches * c->P * 3));
    mh_extend(c, n_batches * c->P, fresh);
    c->kseq.insert(c->kseq.end(), fresh.begin(), fresh.end());
    TRY(upload_k(c, start));
    if (m_out) std::copy(fresh.begin(), fresh.end(), m_out);
    (void)from;
    return RBSOG_OK;
}

rbsog_status rbsog_set_k(rbsog_ctx *c, int64_t n_k, const int32_t *m, const double *w) {
    TRY(check_ctx(c));
    if (n_k < 1 || !m) return fail(c, RBSOG_E_ARG, "need n_k >= 1 vectors");
    for (int64_t e = 0; e < n_k; ++e) {
        if (m[3 * e] == 0 && m[3 * e + 1] == 0 && m[3 * e + 2] == 0)
            return fail(c, RBSOG_E_ARG, "wave vector %lld is zero", (long long)e);
        if (w && !std::isfinite(w[e])) return fail(c, RBSOG_E_NONFINITE, "weight %lld is not finite", (long long)e);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->kseq.assign(m, m + 3 * n_k);
    c->custom_w = w != nullptr;
    if (w) c->kw.assign(w, w + n_k);
    else c->kw.clear();
    c->cursor = 0;
    const int64_t zc = 0;
    HIPCHK(c, hipMemcpy(c->dcursor, &zc, sizeof zc, hipMemcpyHostToDevice));
    return upload_k(c, 0);
}

rbsog_status rbsog_forces(rbsog_ctx *c, double *F_out, double *E_out) {
    TRY(check_ctx(c));
    const int64_t nvec = (int64_t)c->kseq.size() / 3;
    if (c->cursor + c->P > nvec)
        return fail(c, RBSOG_E_KSEQ, "sequence has %lld unused vectors, P = %d", (long long)(nvec - c->cursor), c->P);
    TRY(enqueue_eval(c, false, 0.0));
    account_eval(c);
    if (F_out) {
        std::vector<double> a((size_t)3 * c->n), b((size_t)3 * c->n);
        TRY(soa_to_host(c, c->Fn, a.data()));
        TRY(soa_to_host(c, c->Ff, b.data()));
        for (size_t i = 0; i < a.size(); ++i) F_out[i] = a[i] + b[i];
    }
    if (E_out) {
        HIPCHK(c, hipMemcpyAsync(E_out, c->E, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return RBSOG_OK;
}

rbsog_status rbsog_step(rbsog_ctx *c, int64_t n_steps, double dt) {
    TRY(check_ctx(c));
    if (n_steps < 0 || !std::isfinite(dt)) return fail(c, RBSOG_E_ARG, "need n_steps >= 0 and finite dt");
    const int64_t need = (n_steps + (c->forces_valid ? 0 : 1)) * (int64_t)c->P;
    const int64_t nvec = (int64_t)c->kseq.size() / 3;
    if (c->cursor + need > nvec)
        return fail(c, RBSOG_E_KSEQ, "%lld steps need %lld vectors, %lld remain", (long long)n_steps, (long long)need,
                    (long long)(nvec - c->cursor));
    if (!c->forces_valid) {
        TRY(enqueue_eval(c, false, 0.0));
        account_eval(c);
    }
    const bool graphs = c->use_graphs && !c->prof_on && n_steps > 1;
    if (graphs) TRY(ensure_step_graph(c, dt));
    for (int64_t k = 0; k < n_steps; ++k) {
        if (graphs) HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
        else TRY(enqueue_eval(c, true, dt));
        account_eval(c);
    }
    int32_t flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flag) return fail(c, RBSOG_E_NONFINITE, "non-finite force or energy (flag %d)", flag);
    return RBSOG_OK;
}

rbsog_status rbsog_set_velocities(rbsog_ctx *c, const double *v, double T, uint64_t seed) {
    TRY(check_ctx(c));
    std::vector<double> soa((size_t)3 * c->n);
    if (v) {
        for (int64_t i = 0; i < c->n; ++i)
            for (int d = 0; d < 3; ++d) {
                if (!std::isfinite(v[3 * i + d])) return fail(c, RBSOG_E_NONFINITE, "velocity %lld", (long long)i);
                soa[(size_t)d * c->n + i] = v[3 * i + d];
            }
    } else {
        if (!(T >= 0.0) || !std::isfinite(T)) return fail(c, RBSOG_E_ARG, "temperature must be >= 0");
        const double sd = std::sqrt(T / c->mass);
        double mean[3] = {0, 0, 0};
        for (int64_t i = 0; i < c->n; ++i) {
            double u1, u2, u3, u4;
            Philox::uniform2(seed, 1, (uint64_t)i, 0, u1, u2);
            Philox::uniform2(seed, 1, (uint64_t)i, 1, u3, u4);
            const double r1 = std::sqrt(-2.0 * std::log(1.0 - u1)), r2 = std::sqrt(-2.0 * std::log(1.0 - u3));
            const double z[3] = {r1 * std::cos(2 * kPi * u2), r1 * std::sin(2 * kPi * u2), r2 * std::cos(2 * kPi * u4)};
            for (int d = 0; d < 3; ++d) {
                soa[(size_t)d * c->n + i] = sd * z[d];
                mean[d] += sd * z[d];
            }
        }
        for (int d = 0; d < 3; ++d) {
            mean[d] /= (double)c->n;
            for (int64_t i = 0; i < c->n; ++i) soa[(size_t)d * c->n + i] -= mean[d];
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->v, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice));
    return RBSOG_OK;
}

rbsog_status rbsog_set_positions(rbsog_ctx *c, const double *pos) {
    TRY(check_ctx(c));
    if (!pos) return fail(c, RBSOG_E_ARG, "pos is null");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return upload_positions(c, pos);
}

rbsog_status rbsog_get_state(rbsog_ctx *c, double *pos, double *vel) {
    TRY(check_ctx(c));
    if (pos) {
        TRY(soa_to_host(c, c->x, pos));
        // the stored coordinates are wrapped at each evaluation; wrap here too
        for (int64_t i = 0; i < c->n; ++i)
            for (int d = 0; d < 3; ++d) {
                const double t = pos[3 * i + d] / c->box[d];
                pos[3 * i + d] = (t - std::floor(t)) * c->box[d];
            }
    }
    if (vel) TRY(soa_to_host(c, c->v, vel));
    return RBSOG_OK;
}

rbsog_status rbsog_get_forces(rbsog_ctx *c, double *F_near, double *F_far) {
    TRY(check_ctx(c));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    if (F_near) TRY(soa_to_host(c, c->Fn, F_near));
    if (F_far) TRY(soa_to_host(c, c->Ff, F_far));
    return RBSOG_OK;
}

rbsog_status rbsog_get_energy(rbsog_ctx *c, double *E4) {
    TRY(check_ctx(c));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    if (!E4) return fail(c, RBSOG_E_ARG, "E4 is null");
    HIPCHK(c, hipMemcpyAsync(E4, c->E, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBSOG_OK;
}

rbsog_status rbsog_get_rho(rbsog_ctx *c, double *re, double *im) {
    TRY(check_ctx(c));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    std::vector<double> r(2 * (size_t)c->P);
    HIPCHK(c, hipMemcpyAsync(r.data(), c->rho, r.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (re) std::copy(r.begin(), r.begin() + c->P, re);
    if (im) std::copy(r.begin() + c->P, r.end(), im);
    return RBSOG_OK;
}

rbsog_status rbsog_info(rbsog_ctx *c, rbsog_info_t *info) {
    TRY(check_ctx(c));
    if (!info) return fail(c, RBSOG_E_ARG, "info is null");
    info->S = c->S;
    info->volume = c->V;
    for (int d = 0; d < 3; ++d) info->ncell[d] = c->geom.nc[d];
    info->k_remaining = (int64_t)c->kseq.size() / 3 - c->cursor;
    info->evaluations = c->evals;
    return RBSOG_OK;
}

rbsog_status rbsog_debug_cells(rbsog_ctx *c, int32_t *cell_start, int32_t *order) {
    TRY(check_ctx(c));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    if (cell_start)
        HIPCHK(c, hipMemcpyAsync(cell_start, c->cell_start, (size_t)(c->ncell + 1) * sizeof(int32_t),
                                 hipMemcpyDeviceToHost, c->stream));
    if (order)
        HIPCHK(c, hipMemcpyAsync(order, c->order, (size_t)c->n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBSOG_OK;
}

rbsog_status rbsog_debug_neighbors(rbsog_ctx *c, int64_t *row_ptr, int32_t *cols, int64_t cap) {
    TRY(check_ctx(c));
    if (c->evals == 0) return fail(c, RBSOG_E_STATE, "no force evaluation yet");
    if (!row_ptr) return fail(c, RBSOG_E_ARG, "row_ptr is null");
    int64_t *dcount = nullptr;
    HIPCHK(c, hipMalloc((void **)&dcount, (size_t)(c->n + 1) * sizeof(int64_t)));
    launch_neighbor_count(c->geom, c->cell_start, c->order, c->su, dcount, c->stream);
    std::vector<int64_t> cnt(c->n);
    hipError_t e = hipMemcpyAsync(cnt.data(), dcount, (size_t)c->n * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        (void)hipFree(dcount);
        return fail(c, RBSOG_E_DEVICE, "neighbour count: %s", hipGetErrorString(e));
    }
    row_ptr[0] = 0;
    for (int64_t i = 0; i < c->n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    const int64_t total = row_ptr[c->n];
    if (!cols || cap < total) {
        (void)hipFree(dcount);
        return fail(c, RBSOG_E_ARG, "cols needs %lld entries", (long long)total);
    }
    int32_t *dcols = nullptr;
    e = hipMemcpy(dcount, row_ptr, (size_t)(c->n + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&dcols, (size_t)std::max<int64_t>(total, 1) * sizeof(int32_t));
    if (e == hipSuccess) {
        launch_neighbor_fill(c->geom, c->cell_start, c->order, c->su, dcount, dcols, c->stream);
        e = hipMemcpyAsync(cols, dcols, (size_t)total * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    (void)hipFree(dcols);
    (void)hipFree(dcount);
    if (e != hipSuccess) return fail(c, RBSOG_E_DEVICE, "neighbour fill: %s", hipGetErrorString(e));
    return RBSOG_OK;
}

rbsog_status rbsog_profile(rbsog_ctx *c, int32_t enable) {
    TRY(check_ctx(c));
    TRY(prof_collect(c));
    c->prof_on = enable != 0;
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

rbsog_status rbsog_sync(rbsog_ctx *c) {
    TRY(check_ctx(c));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RBSOG_OK;
}

const char *rbsog_last_error(const rbsog_ctx *c) { return c ? c->err.c_str() : g_init_error.c_str(); }

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
    drop_graph(c);
    for (void *p : c->allocs) (void)hipFree(p);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"
