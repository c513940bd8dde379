/*
 * rbsog.h - C ABI of librbsog, an MI355X (gfx950) implementation of the
 * per-step electrostatic force evaluation of the random batch
 * sum-of-Gaussians (RBSOG) method (Liang, Xu, Zhou, arXiv 2205.13824).
 *
 * Problem (Sec. 2, eqs. "solutionperiodic", "energy"): N point charges q_i at
 * r_i in a periodic cuboid L_x x L_y x L_z, sum q_i = 0, unit dielectric,
 * tinfoil boundary.  The kernel 1/r is split (Sec. 2, eqs. "SOGDEcomp",
 * "SOGField") into a near part N(r) = 1/r - F(r) for r < r_c and a far part
 * F(r) = sum_{l=0}^{M} omega_l exp(-r^2/s_l^2), omega_l = sqrt(2/pi) ln b /
 * (sigma b^l) (omega_0 scaled by w0), s_l = sqrt(2) b^l sigma.
 *
 * Per force evaluation the library computes
 *   near force   F_N,i = sum_{j: r_ij < r_c} q_i q_j (1/r^3 - 2 sum_l omega_l/s_l^2
 *                 e^{-r^2/s_l^2}) r_ij                  (Sec. 3.1, eq. "forcesplit";
 *                 the printed 1/(2r^3) form is half of -grad U_N)
 *   far force    F*_i = -q_i sum_{e=1}^{P} w_e k_e Im(e^{-i k_e.r_i} rho(k_e)),
 *                 rho(k) = sum_j q_j e^{i k.r_j}, k = 2 pi (m_x/L_x, m_y/L_y, m_z/L_z),
 *                 w_e = S pi^{3/2} / (P V)              (Sec. 3.3, eq. "approximateForce",
 *                 with the leading minus sign of -grad U*)
 *   energies     U_N = sum_{pairs, r<r_c} q_i q_j N(r); U* = 1/2 sum_e w_e |rho(k_e)|^2;
 *                 U_self = 1/2 F(0) sum q_i^2; U = U_N + U* - U_self      (Sec. 3.1)
 * The wave vectors m_e are a pre-sampled sequence (Algorithm 1, step 2), drawn
 * by Metropolis-Hastings from P_k = F~(k)/(pi^{3/2} S) (Sec. 3.3) and consumed
 * P at a time, in order, one batch per force evaluation.
 *
 * A context holds one system (rbsog_init) or a batch of independent systems
 * (rbsog_init_batch, e.g. an ensemble of replicas): every call acts on all of
 * them at once, each system with its own box, charges, cutoff, split, P and
 * sampler; "n" below is the total particle count and particle arrays
 * concatenate the systems in the order of the offsets.
 *
 * Conventions.
 *   - All host arrays are caller-owned, read or written only during the call.
 *     Positions/velocities/forces are row-major n x 3 (x, y, z per particle),
 *     returned in the caller's particle order.
 *   - Every call returns an rbsog_status; nothing throws or aborts across the
 *     ABI.  After RBSOG_E_ARG, E_NOT_NEUTRAL, E_CUTOFF, E_SOG or E_KSEQ the
 *     context is unchanged and usable; after E_DEVICE or E_OOM it must only be
 *     destroyed.  rbsog_last_error() explains the latest failure.
 *   - One context must not be used from two threads at once.  Work is
 *     launched on one HIP stream (the caller's, or one the context owns).
 *   - Fixed-point coordinates: u_d = min(2^32-1, floor(frac(x_d/L_d) 2^32)).
 *     Cells: n_d = floor(L_d/(r_c (1 + skin))) if >= 3, else 1;
 *     c_d = (u_d n_d) >> 32; cell = c_x + n_x (c_y + n_y c_z); particles
 *     ordered by (cell, id) at each near-list build.
 *     A pair is a neighbour iff (dx*dx + dy*dy) + dz*dz < r_c*r_c in FP64
 *     without contraction, dx = (double)(int32)(u_j,x - u_i,x) * (L_x 2^-32).
 *   - Near list: a build lists the pairs within r_c (1 + skin) (cell
 *     stencil, FP32 test widened beyond its rounding); every evaluation
 *     applies the pair rule above to the listed pairs at the current
 *     positions.  An evaluation builds first if some particle has moved
 *     farther than skin r_c / 2 (minimum image of the fixed-point
 *     difference) since the latest build, or after rbsog_set_positions, so
 *     the pairs evaluated are exactly the neighbours.  The list holds up to
 *     twice the largest per-item count seen (grown between calls when a
 *     build passes 3/4 of it); a build that overflows fails the call with
 *     E_STATE and poisons the context.
 */
#ifndef RBSOG_H
#define RBSOG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbsog_ctx rbsog_ctx;

typedef enum {
    RBSOG_OK = 0,
    RBSOG_E_ARG = -1,          /* null pointer, size or value out of range */
    RBSOG_E_NOT_NEUTRAL = -2,  /* |sum q| > neutral_tol * sum |q| */
    RBSOG_E_CUTOFF = -3,       /* r_c <= 0 or r_c > min(L)/2 */
    RBSOG_E_SOG = -4,          /* b <= 1, sigma <= 0, w0 <= 0 or M < 0 */
    RBSOG_E_DEVICE = -5,       /* a HIP call failed; the context is poisoned */
    RBSOG_E_OOM = -6,          /* device allocation failed */
    RBSOG_E_NONFINITE = -7,    /* non-finite input, or non-finite force/energy produced */
    RBSOG_E_KSEQ = -8,         /* the wave-vector sequence has fewer than P unused entries */
    RBSOG_E_STATE = -9         /* call not valid in the context's current state */
} rbsog_status;

typedef enum {
    RBSOG_FP64 = 0,   /* every step in FP64 */
    RBSOG_FP32C = 1   /* FP32 phases and pair arithmetic on fixed-point coordinates,
                         FP64 accumulation of rho(k) partial sums and energies */
} rbsog_precision;

/* Sum-of-Gaussians parameters with Table 1 semantics (Sec. 4.1): sigma for the
 * cutoff in use, w0 the factor applied to the nominal omega_0. */
typedef struct {
    double b;
    double sigma;
    double w0;
    int32_t M;
} rbsog_sog;

typedef struct {
    int32_t precision;    /* rbsog_precision; default RBSOG_FP64 */
    int32_t device;       /* HIP device ordinal; default 0 */
    void *stream;         /* hipStream_t to launch on; NULL = the context creates one */
    double neutral_tol;   /* default 1e-10 */
    double mass;          /* mass of every particle; default 1 */
    int32_t graphs;       /* nonzero: rbsog_step replays captured HIP graphs of one or eight steps;
                             plain velocity-Verlet steps on a kept near list then fuse each step's
                             closing kick with the next one's kick and drift (the same arithmetic in
                             the same order; each call still ends on a whole step); default 1 */
    int32_t autotune;     /* nonzero: the first rbsog_step tunes the launch shapes (rbsog_autotune
                             with 5 repetitions) unless a cached tuning applies; default 0 */
    int32_t near_table;   /* FP32C only, nonzero: core-shell near kernel (Sec. 3.4): pairs with
                             r < r_in = 0.2 r_c take 4 Taylor terms of the Gaussians (the
                             coefficients with the series' alternating sign), pairs with
                             r_in <= r < r_c a 4096-point table indexed by the low 3 exponent
                             bits and high 9 mantissa bits of r^2 in FP32, linearly
                             interpolated; relative error of a pair force below 2e-6.
                             E_ARG with FP64, or if r_c^2/r_in^2 spans more than 6 binades.
                             Default 0 (direct evaluation). */
    int32_t zero_mode;    /* zero-frequency mode term (Sec. 3.2, eqs. "sperical", "planar"),
                             M = sum_i q_i r_i over the wrapped positions:
                             0 tinfoil (none; default), 1 spherical U^0 = (2 pi/3V)|M|^2,
                             2 slab along z U^0 = (2 pi/V) M_z^2; its force -grad U^0 is
                             added to the far force and U^0 to U* and U. */
    int32_t device_chains;/* lambda >= 1: the wave vectors are drawn on the device by lambda
                             independent Metropolis-Hastings chains per system (the parallel
                             sampling of Sec. 3.4): chain c serves evaluations c, c + lambda,
                             c + 2 lambda, ... with P consecutive chain states each; it uses
                             Philox stream 3 + c keyed by the system's seed and otherwise the
                             host chain's algorithm (Sec. 3.3, 100 transitions discarded).
                             Every lambda evaluations one kernel advances all chains by P
                             states.  rbsog_sample_k and rbsog_set_k then return E_STATE.
                             0 (default): the host chain fills the sequence. At most 4096. */
    double skin;          /* near-list skin as a fraction of r_c, in [0, 1]; default 0.1.
                             0 builds the list at every evaluation whose positions moved. */
} rbsog_opts;

/* Fills *o with the defaults above. */
void rbsog_default_opts(rbsog_opts *o);

/* Table 1 row `row` (1..5) scaled to cutoff rc: b and w0 as printed, sigma
 * multiplied by rc / 10 (the table is quoted at r_c = 10 Angstrom; the split
 * is scale covariant).  E_ARG for a row outside 1..5 or rc <= 0. */
rbsog_status rbsog_sog_table1(int32_t row, double rc, rbsog_sog *out);

/* Creates a context for one periodic system (Sec. 2 problem statement;
 * Algorithm 1, step 1): a batch of one.
 *   n     number of particles, 2 <= n <= 2^28 (a near-list entry holds a
 *         particle slot in 28 bits)
 *   pos   host, n x 3, any finite values (wrapped into the box)
 *   q     host, n charges, finite, neutral within opts->neutral_tol
 *   box   host, 3 side lengths > 0
 *   sog   split parameters (b > 1, sigma > 0, w0 > 0, M >= 0)
 *   rc    cutoff, 0 < rc <= min(box)/2
 *   P     wave vectors per force evaluation, >= 1
 *   seed  key of the Metropolis-Hastings sampler's Philox4x32-10 stream
 *   opts  NULL for defaults
 * Computes S (Sec. 3.3, eq. "S"), uploads the system and allocates all device
 * memory; velocities start at zero.  *out is NULL on failure. */
rbsog_status rbsog_init(rbsog_ctx **out, int64_t n, const double *pos, const double *q,
                        const double *box, const rbsog_sog *sog, double rc, int32_t P,
                        uint64_t seed, const rbsog_opts *opts);

/* Creates a context for n_sys independent systems evaluated together (one
 * launch per kernel for the whole batch).  System s owns particles
 * [offsets[s], offsets[s+1]) of pos (n x 3) and q, box boxes[3s..3s+2], split
 * sog[s], cutoff rc[s], P[s] wave vectors per evaluation and sampler key
 * seeds[s]; each is validated as by rbsog_init (errors name the system).
 *   offsets  host n_sys+1 int64, offsets[0] = 0, at least 2 particles each,
 *            at most 2^28 in all
 * Precision, device, stream, mass and graphs of opts apply to all systems. */
rbsog_status rbsog_init_batch(rbsog_ctx **out, int32_t n_sys, const int64_t *offsets,
                              const double *pos, const double *q, const double *boxes,
                              const rbsog_sog *sog, const double *rc, const int32_t *P,
                              const uint64_t *seeds, const rbsog_opts *opts);

/* Extends the wave-vector sequence by n_batches * P states of the
 * Metropolis-Hastings independence chain of Sec. 3.3 (Algorithm 1, step 2):
 * proposal m*_d = round(N(0, (L_d/(pi s_0))^2 / 2)), m* = 0 redrawn, accepted
 * with probability min(1, p(m*) q(m)/(p(m) q(m*))), p ~ F~(2 pi m/L), q the
 * proposal pmf (1/2)[erf((m+1/2) pi s_0/L_d) - erf((m-1/2) pi s_0/L_d)].  The
 * chain starts at its first nonzero proposal and discards 100 transitions.
 * Attempt t uses Philox4x32-10 with counter (t_lo, t_hi, 0, lane) and key
 * (seed_lo, seed_hi): lanes 0 and 1 give two Box-Muller pairs from 53-bit
 * uniforms, lane 2 the acceptance uniform.
 * Every system extends its own chain (key seeds[s]).
 *   m_out  NULL, or host sum_s n_batches * P_s * 3 int32 receiving the new
 *          states, system after system.
 * E_ARG if n_batches < 1. */
rbsog_status rbsog_sample_k(rbsog_ctx *ctx, int64_t n_batches, int32_t *m_out);

/* Replaces the sequence of system sys with n_k caller-given nonzero vectors
 * (host, n_k x 3) and rewinds it.  w: NULL for the random-batch weight S pi^{3/2}/(P V), or
 * host n_k per-vector weights (w = F~(k)/V with every k of the lattice and
 * P = n_k turns the far part into the full Fourier sum of eq. "forcesplit").
 * E_ARG if sys is out of range, n_k < 1 or a vector is zero. */
rbsog_status rbsog_set_k(rbsog_ctx *ctx, int32_t sys, int64_t n_k, const int32_t *m,
                         const double *w);

/* One force evaluation at the current positions with the next P vectors of
 * the sequence (Algorithm 1, step 4): wrap and quantise, near-list check
 * (and build: cell list, re-sort, list), near part, structure factors, far
 * force, energies.
 *   F_out  NULL, or host n x 3 total force F_N + F*
 *   E_out  NULL, or host 4 * n_sys doubles: U_N, U*, U_self, U of each system
 * E_KSEQ if a system has fewer than P vectors left (nothing is computed);
 * E_NONFINITE if a returned force or energy is not finite (coincident ions,
 * positions run off to infinity).  The report is made once: the context
 * stays usable, and new finite positions or a loaded state run on. */
rbsog_status rbsog_forces(rbsog_ctx *ctx, double *F_out, double *E_out);

/* n_steps velocity-Verlet steps of size dt (kick dt/2, drift, wrap, forces
 * with the next batch, kick dt/2; Algorithm 1 with NVE integration, or the
 * Langevin BAOAB step of rbsog_set_thermostat).  If the
 * forces of the current positions are not known yet, one evaluation is made
 * first.  E_KSEQ (before any work) if the sequence cannot serve every
 * evaluation; E_NONFINITE if a force or energy of any step was not finite
 * (the steps are still made: positions that went non-finite stay so, and
 * fall in cell 0 of their system; when they overflow its near list the
 * context is left unusable and can only be destroyed); E_STATE if a device
 * chain exceeded its proposal limit. */
rbsog_status rbsog_step(rbsog_ctx *ctx, int64_t n_steps, double dt);

/* Sets velocities: v host n x 3, or NULL to draw v ~ N(0, T/m) per component
 * (Philox4x32-10 keyed by seed, counter (i, 0, 1, lane) for particle i,
 * Box-Muller) and remove each system's centre-of-mass velocity.  E_ARG if v
 * is NULL and T < 0. */
rbsog_status rbsog_set_velocities(rbsog_ctx *ctx, const double *v, double T, uint64_t seed);

/* Langevin thermostat for rbsog_step (Algorithm 1 leaves the thermostat open;
 * Theorem 3 is stated for Langevin dynamics).  gamma > 0: each step is BAOAB:
 * kick dt/2, drift dt/2, v <- c1 v + c2 xi with c1 = exp(-gamma dt),
 * c2 = sqrt((1 - c1^2) T/m), drift dt/2, forces, kick dt/2; xi are standard
 * normals, for particle i (caller index) at thermostatted step s (counted from
 * this call, from 0) drawn with Philox4x32-10, key (seed_lo, seed_hi), counter
 * (i, s, 2, lane), lanes 0 and 1 giving two 53-bit uniforms each (u1, u2),
 * (u3, u4), xi = (r1 cos 2pi u2, r1 sin 2pi u2, r2 cos 2pi u4), r = sqrt(-2 ln(1-u)).
 * gamma = 0 restores NVE velocity Verlet.  E_ARG for gamma < 0 or T < 0. */
rbsog_status rbsog_set_thermostat(rbsog_ctx *ctx, double gamma, double T, uint64_t seed);

/* Nose-Hoover thermostat (the thermostat of Sec. 5's water runs) for the
 * steps of rbsog_step: one variable xi per system with thermostat mass
 * Q = N_f T tau^2, N_f = 3 n_s - 3.  Each step: xi += dt/2 (2K - N_f T)/Q with
 * the kinetic energy K of the step's start, v *= exp(-xi dt/2), the
 * velocity-Verlet kick, drift, force and kick, v *= exp(-xi dt/2), then
 * xi += dt/2 (2K' - N_f T)/Q with the new K'.  tau = 0 turns it off; tau > 0
 * turns a Langevin thermostat off, and rbsog_set_thermostat with gamma > 0
 * turns this one off.  xi starts at 0.  E_ARG for tau < 0, or T <= 0 with
 * tau > 0. */
rbsog_status rbsog_set_nose_hoover(rbsog_ctx *ctx, double T, double tau);

/* Kinetic energy K = m/2 sum |v|^2 of every system after the latest
 * evaluation (or as set by rbsog_set_velocities), and the Nose-Hoover xi of
 * every system (0 without that thermostat): host n_sys doubles each, either
 * may be NULL.  Each system's K is summed on the device in a fixed order. */
rbsog_status rbsog_get_kinetic(rbsog_ctx *ctx, double *K, double *xi);

/* Mean-square displacement (the water runs' MSD of Sec. 5 and its Appendix
 * formula, over all particles of a system): every step adds its drift,
 * unwrapped, to a per-particle displacement d; rbsog_get_msd returns
 * (1/n_s) sum |d|^2 of every system (host n_sys doubles; summed on the device
 * in a fixed order).  Tracking starts with the first rbsog_set_msd_origin,
 * which sets d = 0 (as does rbsog_set_positions); until then steps do not
 * carry d and rbsog_get_msd returns RBSOG_E_STATE. */
rbsog_status rbsog_set_msd_origin(rbsog_ctx *ctx);
rbsog_status rbsog_get_msd(rbsog_ctx *ctx, double *msd);

/* Replaces the positions (host n x 3, finite); forces become unknown. */
rbsog_status rbsog_set_positions(rbsog_ctx *ctx, const double *pos);

/* Copies the state: pos (wrapped into [0, L)) and vel, host n x 3 each, either may be NULL. */
rbsog_status rbsog_get_state(rbsog_ctx *ctx, double *pos, double *vel);

/* Copies the near and far parts of the latest force evaluation (host n x 3
 * each, either may be NULL).  E_STATE if no evaluation has been made. */
rbsog_status rbsog_get_forces(rbsog_ctx *ctx, double *F_near, double *F_far);

/* The near and far parts of the latest force evaluation on m particles only,
 * named by their caller indices (host ids[m], 0 <= id < n), without copying
 * the whole system (sampled checks of large systems, observables of a few
 * particles): F_near, F_far host m x 3 each, either may be NULL.  E_ARG for an
 * index out of range, E_STATE if no evaluation has been made. */
rbsog_status rbsog_get_forces_subset(rbsog_ctx *ctx, int64_t m, const int64_t *ids, double *F_near,
                                     double *F_far);

/* Copies the latest energies (host 4 * n_sys doubles: U_N, U*, U_self, U of
 * each system) and the structure factors of system sys (host P doubles each
 * for rho_re, rho_im; either may be NULL). */
rbsog_status rbsog_get_energy(rbsog_ctx *ctx, double *E);
rbsog_status rbsog_get_rho(rbsog_ctx *ctx, int32_t sys, double *rho_re, double *rho_im);

/* Copies the wave vectors m of the latest evaluation's batch of system sys
 * (Algorithm 1, the P vectors of one step; host 3 * P int32, m_x m_y m_z per
 * vector) whether the host chain or the device chains drew them.  E_STATE if
 * no evaluation has been made. */
rbsog_status rbsog_get_kbatch(rbsog_ctx *ctx, int32_t sys, int32_t *m_out);

/* Scalars of system sys: S, V, number of cells, wave vectors left in its
 * sequence, evaluations made, its particle count and the number of systems. */
typedef struct {
    double S;
    double volume;
    int32_t ncell[3];
    int64_t k_remaining;
    int64_t evaluations;
    int64_t n;
    int32_t n_sys;
    int32_t rho_chunk;            /* launch shapes in use (see rbsog_autotune) */
    int32_t far_block;
    int32_t tuned;                /* 1 if the shapes come from tuning (now or cached) */
    int64_t list_capacity;        /* near-list entries per 64-particle item (64 x the pairs one home can hold) */
    int64_t list_builds;          /* near-list builds made by evaluations so far */
    double skin;                  /* skin in use: the caller's, or 0 while the steps build every time
                                     (rbsog_step checks every 32 steps: when lists last under two
                                     steps it builds at every step, with r_c-wide cells and no list,
                                     and tries the caller's skin again after 4 to 32 checks) */
    int32_t rho_ktile;            /* launch shapes in use (see rbsog_autotune): k tiles of 64 per
                                     structure-factor block (largest over the systems), */
    int32_t build_slots;          /* candidate slots of 64 per lane and test pass of the list build, */
    int32_t cell_slots;           /* and of the fused cell kernel of the build-every-step mode */
    int32_t list_home_major;      /* 1: the near list is kept home by home (lists of more than 128
                                     pairs of one home at sizing; one home per wave in the list
                                     pass), 0: in columns (one home per lane) */
} rbsog_info_t;
rbsog_status rbsog_info(rbsog_ctx *ctx, int32_t sys, rbsog_info_t *info);

/* Tunes the launch shapes of the batch on the data of the latest evaluation,
 * one phase after the other, each candidate timed over `reps` launches of its
 * kernels with HIP events (after one untimed launch); the fastest are kept:
 *   particles per structure-factor chunk (256..32768) and k tiles of 64 per
 *   structure-factor block (1..16; the block's other waves split the chunk),
 *   timed on the latest evaluation's wave vectors (left as they are when
 *   rbsog_set_k or rbsog_sample_k has since started a new sequence);
 *   particles per far block (64, 128, 256), timed on the far kernels of the
 *   near mode in use (after the near list, or beside the near part when every
 *   step builds);
 *   candidate slots of 64 per lane and test pass of the near kernel in use
 *   (the list build: 2..4; the fused cell kernel of the build-every-step
 *   mode: 2, 3), each trial a rebuild at the current positions.
 * The sequence is not consumed and the positions do not move; the near and
 * far forces are recomputed with the chosen shapes (same pairs, same data).
 * The choice is cached for the process under (GPU architecture, precision,
 * batch size, log2 n, P, log2 cells) and, if the environment variable
 * RBSOG_TUNE_CACHE names a file, appended to it; new contexts of the same
 * kind start from the cached shapes.  E_STATE before the first evaluation. */
rbsog_status rbsog_autotune(rbsog_ctx *ctx, int32_t reps);

/* Debug exports of system sys: the cell list of the latest near-list build
 * and a full neighbour list at the current positions built on the device
 * with the pair rule above (rows ascending i, columns ascending j).  Indices are local to the system (0 .. n_s - 1).
 *   cell_start  host ncell+1 int32;  order  host n_s int32 (ids by (cell, id))
 *   row_ptr     host n_s+1 int64;  cols  host cap int32
 * rbsog_debug_neighbors returns E_ARG if cap is smaller than the entry count
 * (row_ptr is still filled, so the call can be repeated). */
rbsog_status rbsog_debug_cells(rbsog_ctx *ctx, int32_t sys, int32_t *cell_start, int32_t *order);
rbsog_status rbsog_debug_neighbors(rbsog_ctx *ctx, int32_t sys, int64_t *row_ptr, int32_t *cols,
                                   int64_t cap);

/* Structure factor of one set of point charges, without a context (Sec. 3.1:
 * rho(k_e) = sum_j q_j e^{i k_e.r_j}, k_e = 2 pi (m_x/L_x, m_y/L_y, m_z/L_z);
 * Sec. 3.4: the one reduction of the method, which a run sharded over several
 * devices computes per device over its own particles and then sums).
 *   n          particles, 1 <= n <= 2^31-1
 *   x          device, n x 3 FP64 positions (row-major; wrapped into the box)
 *   q          device, n FP64 charges
 *   box        host, 3 side lengths > 0
 *   n_k        wave vectors, >= 1
 *   m          device, n_k x 3 int32 integer vectors m_e (k_e = 2 pi m_e / L)
 *   precision  RBSOG_FP64: FP64 fractional coordinates, FP64 sin/cos of the
 *              phase m.s - rint(m.s), FP64 sums; RBSOG_FP32C: the phase
 *              m.u mod 2^32 on the 32-bit fixed-point coordinates of the
 *              rule above, hardware FP32 sin/cos, FP32 sums over runs of 32
 *              particles added in FP64
 *   rho_re, rho_im  device, n_k doubles each, written
 *   stream     hipStream_t to launch on (NULL: the null stream)
 * Asynchronous on `stream`; the result is deterministic (partial sums over
 * particle chunks, added in a fixed order).  Non-finite positions or charges
 * give unspecified values.  The partial sums live in device memory allocated
 * and freed on `stream` for the call.  E_ARG for sizes out of range or a null
 * pointer, E_OOM if the partial sums cannot be allocated, E_DEVICE if a launch
 * fails; the message is at rbsog_last_error(NULL). */
rbsog_status rbsog_structure_factor(int64_t n, const double *x, const double *q, const double *box, int64_t n_k,
                                    const int32_t *m, int32_t precision, double *rho_re, double *rho_im,
                                    void *stream);

/* rbsog_structure_factor for callers that cannot allocate device memory
 * (work captured into a HIP graph, serving loops, harnesses that forbid
 * allocation): the same arguments, kernels and chunk plan, so the same
 * result bit for bit, with the partial sums in one library-held array of
 * 2^20 complex FP64 values (16 MiB on each device used, held until the
 * process ends); it calls no allocator.  n_k above 2^20 returns E_ARG.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (two streams, two threads) race and must not be made. */
rbsog_status rbsog_structure_factor_noalloc(int64_t n, const double *x, const double *q, const double *box,
                                            int64_t n_k, const int32_t *m, int32_t precision, double *rho_re,
                                            double *rho_im, void *stream);

/* Debug record of the pairs the near kernels accept: with cap > 0 (at most
 * 2^31-1) every later evaluation records, from the near kernel that evaluates
 * it (the list pass, which evaluates every evaluation with the near list, the
 * ones with a list build included, or the fused cell kernel of the
 * build-every-step mode), each pair that passes the pair rule of the header's
 * conventions, as the kernel evaluates it; rbsog_step then launches kernel by
 * kernel (no graphs).  cap = 0 stops recording and frees the record.
 * rbsog_debug_pairs returns the latest evaluation's record for system sys as
 * CSR over local ids (rows ascending i, columns ascending j; each pair in both
 * orders), and in *kinds which kernels recorded: bit 1 the list pass, bit 2
 * the fused cell kernel (bit 0 is not used).  E_STATE if recording is off or
 * the record overflowed; E_ARG (row_ptr filled) if cap is smaller than the
 * entry count.
 * rbsog_debug_list returns the near list of the latest build (the pairs within
 * r_c (1 + skin) by its FP32 test) in the same form; E_STATE at skin 0. */
rbsog_status rbsog_debug_record_pairs(rbsog_ctx *ctx, int64_t cap);
rbsog_status rbsog_debug_pairs(rbsog_ctx *ctx, int32_t sys, int32_t *kinds, int64_t *row_ptr, int32_t *cols,
                               int64_t cap);
rbsog_status rbsog_debug_list(rbsog_ctx *ctx, int32_t sys, int64_t *row_ptr, int32_t *cols, int64_t cap);

/* Per-kernel timing with HIP events; later steps launch kernel by kernel (no
 * graphs).  enable 1: every kernel alone on the context's stream (its time
 * with the whole device); enable 2: as in the steps, the structure factor (and
 * the far force when every step builds) on the second stream beside the
 * near part, each kernel timed on the stream it runs on (its time while it
 * shares the device); 0 stops; 1 and 2 clear the totals; other values E_ARG.
 * rbsog_profile_read returns the name, summed milliseconds and launch count
 * of kernel idx (E_ARG past the last one). */
rbsog_status rbsog_profile(rbsog_ctx *ctx, int32_t enable);
rbsog_status rbsog_profile_read(rbsog_ctx *ctx, int32_t idx, const char **name, double *ms,
                                int64_t *launches);

/* Checkpoint and resume: every quantity a later step reads, so that a run
 * resumed from a saved state continues bit for bit as the uninterrupted run
 * would (Algorithm 1 consumes the wave-vector sequence in order: the chain
 * states, the sequence and its cursor are part of the state): positions,
 * velocities and charges in the current cell order with the caller indices,
 * the fixed-point coordinates and those of the latest near-list build, the
 * cell starts (the near list itself is listed again from them on load), the
 * near and far forces of the latest evaluation, energies, structure factors
 * and the latest batch's wave-vector records, the host chain, sequence and
 * cursor of every system (or the
 * device chains and their batches), the Langevin step counter, the
 * Nose-Hoover xi and kinetic energies, the mean-square-displacement origin
 * and displacements, the skin in use with the adaptive-skin counters, the
 * thermostat settings and the launch shapes.
 * rbsog_save_state: with buf NULL only *size (bytes needed) is set; else
 * buf (host, cap bytes) receives the state and *size its length; E_ARG if
 * cap is too small.  The bytes are an opaque format of this library build.
 * rbsog_load_state: restores a state into a context created by the same
 * rbsog_init / rbsog_init_batch call (same systems, charges, boxes, cutoffs,
 * P, seeds and options; the positions given at creation are replaced);
 * E_ARG if the state belongs to a context of another shape or is truncated:
 * the context is unchanged unless only the near list at the end is cut short
 * (then it must be loaded again or destroyed). */
rbsog_status rbsog_save_state(rbsog_ctx *ctx, void *buf, int64_t cap, int64_t *size);
rbsog_status rbsog_load_state(rbsog_ctx *ctx, const void *buf, int64_t len);

/* Measured issue rates of the vector instructions the kernels are built
 * from (the peaks their instruction counts are priced against; no passage of
 * the paper: the method's work is stated per pair and per wave vector, the
 * rate at which a device retires it is measured here).  Probe i runs
 * independent chains of one instruction or mix on every lane of 16 waves per
 * SIMD; rbsog_probe_name(i) names it (NULL past the last), rbsog_probe_count()
 * gives how many there are.  rbsog_probe_rates times each probe reps times on
 * its own stream of `device` (HIP events, best of reps) and writes
 * lane-instructions per second (a mix counts each of its instructions) into
 * rates[0 .. count-1] (host, n >= count entries).  E_ARG for a short array or
 * reps < 1, E_DEVICE if a launch fails; messages at rbsog_last_error(NULL).
 * Allocates and frees 4 MiB of device memory. */
int32_t rbsog_probe_count(void);
const char *rbsog_probe_name(int32_t i);
rbsog_status rbsog_probe_rates(int32_t device, int32_t reps, double *rates, int32_t n);

/* Blocks until all work of the context has finished. */
rbsog_status rbsog_sync(rbsog_ctx *ctx);

const char *rbsog_last_error(const rbsog_ctx *ctx);
const char *rbsog_status_string(rbsog_status s);

/* Frees every resource of the context; NULL is ignored. */
void rbsog_destroy(rbsog_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* RBSOG_H */
