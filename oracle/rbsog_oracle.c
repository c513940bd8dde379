/*
 * Plain FP64 CPU oracle for the random batch sum-of-Gaussians (RBSOG) force
 * evaluation of Liang, Xu and Zhou, "Random batch sum-of-Gaussians method for
 * molecular dynamics simulations of particle systems" (arXiv 2205.13824).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, constant or table with
 * the GPU library.
 *
 * Every routine is written from the paper's definitions, in FP64, with no
 * blocking or fusion beyond what the definition states.  Where the printed
 * formula is garbled the corrected reading is stated at the routine (each one
 * was checked against a finite-difference gradient or a quadrature):
 *   - near force (Sec. 3.1, eq. "forcesplit", first line): the printed 1/(2r^3)
 *     and single Gaussian weight are half of -grad U_N; the oracle uses
 *     q_i q_j (1/r^3 - 2 sum_l omega_l/s_l^2 exp(-r^2/s_l^2)) r_ij;
 *   - far force (eq. "forcesplit" second line and eq. "approximateForce"):
 *     -grad U* carries a leading minus sign;
 *   - proposal pmf (Sec. 3.3): the erf argument is (m +- 1/2) pi s_0 / L.
 *
 * Conventions shared by definition (not by code) with the GPU library:
 *   fixed-point fractional coordinate  u_d = min(2^32-1, floor(frac(x_d/L_d) 2^32))
 *   neighbour rule   r2 = (dx*dx + dy*dy) + dz*dz < rc*rc  in FP64, no FMA
 *                    contraction, dx = (double)(int32)(u_j,d - u_i,d) * (L_d 2^-32)
 *   cell grid        n_d = floor(L_d / rc) if that is >= 3, else 1;
 *                    c_d = (u_d * n_d) >> 32; cell = c_x + n_x (c_y + n_y c_z)
 *   cell order       ascending (cell, particle id)
 * This file must be compiled with -ffp-contract=off.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define TWO32 4294967296.0

/* Neumaier compensated sum, used for structure factors and energies. */
typedef struct { double s, c; } nsum_t;
static inline void nadd(nsum_t *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum_t *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Sum-of-Gaussians coefficients, Sec. 2 (u-series split, eq. "SOGField" and
 * the coefficient formula after it):
 *   omega_l = (pi/2)^(-1/2) b^(-l) sigma^(-1) ln b,   s_l = sqrt(2) b^l sigma,
 * l = 0..M, with omega_0 multiplied by the continuity factor w0 (Table 1
 * gives w0 as that factor; eq. "omega0" defines the retuned omega_0). */
void orc_sog_coeffs(double b, double sigma, double w0, int M, double *omega, double *s) {
    for (int l = 0; l <= M; ++l) {
        double bl = pow(b, (double)l);
        omega[l] = log(b) / (sqrt(M_PI / 2.0) * bl * sigma);
        s[l] = sqrt(2.0) * bl * sigma;
    }
    omega[0] *= w0;
}

/* F(r) = sum_l omega_l exp(-r^2/s_l^2), eq. "SOGField". */
double orc_sog_F(double r, int M, const double *omega, const double *s) {
    double f = 0.0;
    for (int l = 0; l <= M; ++l) f += omega[l] * exp(-r * r / (s[l] * s[l]));
    return f;
}

/* ------------------------------------------------------------------------ */
/* Fixed-point fractional coordinates (the quantisation that decides cells and
 * neighbour inclusion) and the wrapped FP64 position x_w = frac(x/L) L. */
void orc_quantise(int64_t n, const double *pos, const double *box, uint32_t *u, double *xw) {
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            double t = pos[3 * i + d] / box[d];
            double f = t - floor(t);
            double v = floor(f * TWO32);
            if (v > TWO32 - 1.0) v = TWO32 - 1.0;
            u[3 * i + d] = (uint32_t)v;
            if (xw) xw[3 * i + d] = f * box[d];
        }
    }
}

/* Pair inclusion: r < r_c (strict, eq. "SOGDEcomp"), evaluated on the
 * fixed-point coordinates so that the decision is reproducible bit for bit. */
static int pair_within(const uint32_t *ui, const uint32_t *uj, const double *box, double rc2) {
    double dx = (double)(int32_t)(uj[0] - ui[0]) * (box[0] / TWO32);
    double dy = (double)(int32_t)(uj[1] - ui[1]) * (box[1] / TWO32);
    double dz = (double)(int32_t)(uj[2] - ui[2]) * (box[2] / TWO32);
    double r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    return r2 < rc2;
}

/* Minimum-image displacement r_i - r_j from wrapped FP64 positions. */
static void min_image(const double *xi, const double *xj, const double *box, double *d) {
    for (int k = 0; k < 3; ++k) {
        double t = xi[k] - xj[k];
        d[k] = t - box[k] * nearbyint(t / box[k]);
    }
}

void orc_cell_dims(const double *box, double rc, int32_t *nc) {
    for (int d = 0; d < 3; ++d) {
        int32_t k = (int32_t)floor(box[d] / rc);
        nc[d] = k >= 3 ? k : 1;
    }
}

/* Cell list by definition: cell of each particle, counts, exclusive prefix,
 * and the particle ids ordered by (cell, id). */
void orc_cell_list(int64_t n, const uint32_t *u, const int32_t *nc, int32_t *cell_of,
                   int32_t *cell_start, int32_t *order) {
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    for (int64_t c = 0; c <= ncell; ++c) cell_start[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) c[d] = (int64_t)(((uint64_t)u[3 * i + d] * (uint64_t)nc[d]) >> 32);
        cell_of[i] = (int32_t)(c[0] + nc[0] * (c[1] + nc[1] * c[2]));
        cell_start[cell_of[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) cell_start[c + 1] += cell_start[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncell);
    for (int64_t c = 0; c < ncell; ++c) fill[c] = cell_start[c];
    for (int64_t i = 0; i < n; ++i) order[fill[cell_of[i]]++] = (int32_t)i;
    free(fill);
}

/* Full neighbour list I(i) (Sec. 3.1) by brute force over all pairs, rows in
 * ascending i, columns ascending j.  Returns the number of entries, or -1 if
 * cap was too small (row_ptr is then still complete). */
int64_t orc_neighbors_brute(int64_t n, const uint32_t *u, const double *box, double rc,
                            int64_t *row_ptr, int32_t *cols, int64_t cap) {
    double rc2 = rc * rc;
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            if (pair_within(u + 3 * i, u + 3 * j, box, rc2)) {
                if (k < cap) cols[k] = (int32_t)j;
                ++k;
            }
        }
        row_ptr[i + 1] = k;
    }
    return k <= cap ? k : -1;
}

/* Pair kernel of the near part for one pair at displacement d = r_i - r_j:
 * force on i (eq. "forcesplit", corrected factor) and the pair energy
 * q_i q_j N(r), N(r) = 1/r - F(r) (eq. "SOGDEcomp"). */
static void near_pair(double qq, const double *d, int M, const double *omega, const double *s,
                      double *f, double *e) {
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r = sqrt(r2);
    double g = 0.0, phi = 0.0;
    for (int l = 0; l <= M; ++l) {
        double ex = exp(-r2 / (s[l] * s[l]));
        g += omega[l] / (s[l] * s[l]) * ex;
        phi += omega[l] * ex;
    }
    double coef = qq * (1.0 / (r2 * r) - 2.0 * g);
    f[0] = coef * d[0];
    f[1] = coef * d[1];
    f[2] = coef * d[2];
    *e = qq * (1.0 / r - phi);
}

/* Near part by brute force over unordered pairs: F_N (Newton's third law per
 * pair) and U_N = sum over pairs q_i q_j N(r_ij), eq. "U1" truncated at r_c. */
void orc_near_brute(int64_t n, const double *pos, const double *q, const double *box, double rc,
                    int M, const double *omega, const double *s, double *F, double *U) {
    uint32_t *u = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_quantise(n, pos, box, u, xw);
    double rc2 = rc * rc;
    nsum_t ue = {0, 0};
    memset(F, 0, sizeof(double) * 3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            if (!pair_within(u + 3 * i, u + 3 * j, box, rc2)) continue;
            double d[3], f[3], e;
            min_image(xw + 3 * i, xw + 3 * j, box, d);
            near_pair(q[i] * q[j], d, M, omega, s, f, &e);
            for (int k = 0; k < 3; ++k) { F[3 * i + k] += f[k]; F[3 * j + k] -= f[k]; }
            nadd(&ue, e);
        }
    }
    *U = nval(&ue);
    free(u);
    free(xw);
}

/* Near part through the cell list (same pairs as the brute-force routine; the
 * force on each i is summed over its full neighbour list).  per_i_energy[i]
 * receives (1/2) sum_j q_i q_j N(r_ij); U is their compensated sum. */
void orc_near_cells(int64_t n, const double *pos, const double *q, const double *box, double rc,
                    int M, const double *omega, const double *s, double *F, double *U) {
    uint32_t *u = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_quantise(n, pos, box, u, xw);
    int32_t nc[3];
    orc_cell_dims(box, rc, nc);
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *start = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    orc_cell_list(n, u, nc, cell_of, start, order);
    double *ei = (double *)malloc(sizeof(double) * (size_t)n);
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = cell_of[i];
        int32_t cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
        int rx = nc[0] >= 3 ? 1 : 0, ry = nc[1] >= 3 ? 1 : 0, rz = nc[2] >= 3 ? 1 : 0;
        double fi[3] = {0, 0, 0};
        double e_i = 0.0;
        for (int oz = -rz; oz <= rz; ++oz)
            for (int oy = -ry; oy <= ry; ++oy)
                for (int ox = -rx; ox <= rx; ++ox) {
                    int32_t jx = (cx + ox + nc[0]) % nc[0];
                    int32_t jy = (cy + oy + nc[1]) % nc[1];
                    int32_t jz = (cz + oz + nc[2]) % nc[2];
                    int32_t cj = jx + nc[0] * (jy + nc[1] * jz);
                    for (int32_t t = start[cj]; t < start[cj + 1]; ++t) {
                        int32_t j = order[t];
                        if (j == i) continue;
                        if (!pair_within(u + 3 * i, u + 3 * j, box, rc2)) continue;
                        double d[3], f[3], e;
                        min_image(xw + 3 * i, xw + 3 * j, box, d);
                        near_pair(q[i] * q[j], d, M, omega, s, f, &e);
                        fi[0] += f[0];
                        fi[1] += f[1];
                        fi[2] += f[2];
                        e_i += 0.5 * e;
                    }
                }
        F[3 * i] = fi[0];
        F[3 * i + 1] = fi[1];
        F[3 * i + 2] = fi[2];
        ei[i] = e_i;
    }
    nsum_t ue = {0, 0};
    for (int64_t i = 0; i < n; ++i) nadd(&ue, ei[i]);
    *U = nval(&ue);
    free(ei);
    free(order);
    free(start);
    free(cell_of);
    free(xw);
    free(u);
}

/* Near force on selected targets only, by brute force over every source j
 * (for sampled checks on systems too large for the pair loops above). */
void orc_near_targets(int64_t n, const double *pos, const double *q, const double *box, double rc,
                      int M, const double *omega, const double *s, int64_t nt,
                      const int64_t *targets, double *F) {
    uint32_t *u = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_quantise(n, pos, box, u, xw);
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets[t];
        double fi[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            if (!pair_within(u + 3 * i, u + 3 * j, box, rc2)) continue;
            double d[3], f[3], e;
            min_image(xw + 3 * i, xw + 3 * j, box, d);
            near_pair(q[i] * q[j], d, M, omega, s, f, &e);
            fi[0] += f[0];
            fi[1] += f[1];
            fi[2] += f[2];
        }
        F[3 * t] = fi[0];
        F[3 * t + 1] = fi[1];
        F[3 * t + 2] = fi[2];
    }
    free(xw);
    free(u);
}

/* ------------------------------------------------------------------------ */
/* Structure factor rho(k) = sum_j q_j exp(i k.r_j), k = 2 pi (m_x/L_x,
 * m_y/L_y, m_z/L_z) (Sec. 3.1, Fourier convention eq. "fourtrans"), for a
 * list of integer vectors m.  Compensated sums over particles. */
void orc_structure_factor(int64_t n, const double *pos, const double *q, const double *box,
                          int64_t nk, const int32_t *m, double *rho_re, double *rho_im) {
    double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double t = pos[3 * i + d] / box[d];
            xw[3 * i + d] = (t - floor(t)) * box[d];
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < nk; ++e) {
        double kx = 2.0 * M_PI * m[3 * e] / box[0];
        double ky = 2.0 * M_PI * m[3 * e + 1] / box[1];
        double kz = 2.0 * M_PI * m[3 * e + 2] / box[2];
        nsum_t re = {0, 0}, im = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double th = kx * xw[3 * j] + ky * xw[3 * j + 1] + kz * xw[3 * j + 2];
            nadd(&re, q[j] * cos(th));
            nadd(&im, q[j] * sin(th));
        }
        rho_re[e] = nval(&re);
        rho_im[e] = nval(&im);
    }
    free(xw);
}

/* Fourier-space force for a weighted k list (eq. "forcesplit" second line with
 * the corrected sign, and its random-batch form eq. "approximateForce"):
 *   F_i = - q_i sum_e w_e k_e Im( exp(-i k_e.r_i) rho(k_e) ).
 * w_e = F~(k_e)/V gives the full Fourier sum; w_e = S pi^{3/2}/(P V) gives
 * the random-batch estimator.  Targets: the particle positions/charges to
 * evaluate (need not be the sources). */
void orc_far_force(int64_t nt, const double *pos_t, const double *q_t, const double *box,
                   int64_t nk, const int32_t *m, const double *w, const double *rho_re,
                   const double *rho_im, double *F) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nt; ++i) {
        double x[3];
        for (int d = 0; d < 3; ++d) {
            double t = pos_t[3 * i + d] / box[d];
            x[d] = (t - floor(t)) * box[d];
        }
        double f[3] = {0, 0, 0};
        for (int64_t e = 0; e < nk; ++e) {
            double kx = 2.0 * M_PI * m[3 * e] / box[0];
            double ky = 2.0 * M_PI * m[3 * e + 1] / box[1];
            double kz = 2.0 * M_PI * m[3 * e + 2] / box[2];
            double th = kx * x[0] + ky * x[1] + kz * x[2];
            /* Im( (cos th - i sin th)(re + i im) ) = cos th * im - sin th * re */
            double imv = cos(th) * rho_im[e] - sin(th) * rho_re[e];
            f[0] += w[e] * kx * imv;
            f[1] += w[e] * ky * imv;
            f[2] += w[e] * kz * imv;
        }
        F[3 * i] = -q_t[i] * f[0];
        F[3 * i + 1] = -q_t[i] * f[1];
        F[3 * i + 2] = -q_t[i] * f[2];
    }
}

/* F~(k) = pi^{3/2} sum_l omega_l s_l^3 exp(-s_l^2 k^2 / 4), eq. "FourierSOG". */
double orc_sog_Ftilde(double k2, int M, const double *omega, const double *s) {
    double f = 0.0;
    for (int l = 0; l <= M; ++l) f += omega[l] * s[l] * s[l] * s[l] * exp(-s[l] * s[l] * k2 / 4.0);
    return pow(M_PI, 1.5) * f;
}

/* ------------------------------------------------------------------------ */
/* Far force of one Gaussian omega exp(-r^2/s^2) summed over periodic images in
 * real space (the Poisson-summation twin of its Fourier series; the k = 0
 * term is a constant and carries no force):
 *   F_i = sum_j sum_n' q_i q_j omega (2/s^2) exp(-|d|^2/s^2) d,  d = r_i - r_j + n L,
 * over |n_d| <= nimg.  Used only to cross-check the Fourier-space routine. */
void orc_gauss_realspace_force(int64_t n, const double *pos, const double *q, const double *box,
                               double omega, double s, int nimg, int64_t nt,
                               const int64_t *targets, double *F) {
    double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double t = pos[3 * i + d] / box[d];
            xw[3 * i + d] = (t - floor(t)) * box[d];
        }
    double s2 = s * s;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = targets[t];
        double f[3] = {0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double base[3];
            min_image(xw + 3 * i, xw + 3 * j, box, base);
            for (int nz = -nimg; nz <= nimg; ++nz)
                for (int ny = -nimg; ny <= nimg; ++ny)
                    for (int nx = -nimg; nx <= nimg; ++nx) {
                        if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
                        double d0 = base[0] + nx * box[0];
                        double d1 = base[1] + ny * box[1];
                        double d2 = base[2] + nz * box[2];
                        double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                        double c = q[i] * q[j] * omega * (2.0 / s2) * exp(-r2 / s2);
                        f[0] += c * d0;
                        f[1] += c * d1;
                        f[2] += c * d2;
                    }
        }
        F[3 * t] = f[0];
        F[3 * t + 1] = f[1];
        F[3 * t + 2] = f[2];
    }
    free(xw);
}

/* ------------------------------------------------------------------------ */
/* Far force on selected targets of the Gaussians l = 0..nl-1 (omega_l, s_l as
 * given) summed over periodic images in real space, each out to the radius
 * sqrt(tail) s_l, beyond which its terms are below exp(-tail) of its weight.
 * This is the real-space side of the Poisson identity
 *   sum_n exp(-|r + nL|^2/s^2) = (pi^{3/2} s^3/V) sum_k exp(-s^2 k^2/4) exp(i k.r)
 * (Sec. 3.3; the k = 0 term is a constant and carries no force):
 *   F_i = q_i sum_l omega_l sum_{(j, n): |d| < sqrt(tail) s_l} q_j (2/s_l^2) exp(-|d|^2/s_l^2) d,
 *   d = r_i - r_j + n L   (j = i with n = 0 gives d = 0 and adds nothing).
 * Candidates (j, n) come from a grid of cells of the box tiled periodically:
 * every image of every cell within the widest radius of the target's cell is
 * visited once.  Sums per target are compensated. */
static int64_t floor_div(int64_t a, int64_t b) {
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

void orc_far_realspace_cut(int64_t n, const double *pos, const double *q, const double *box, int nl,
                           const double *omega, const double *s, double tail, int64_t nt, const int64_t *targets,
                           double *F) {
    double smax = 0.0;
    for (int l = 0; l < nl; ++l) smax = s[l] > smax ? s[l] : smax;
    const double R = sqrt(tail) * smax, R2 = R * R;
    double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int32_t nc[3];
    double cw[3];
    for (int d = 0; d < 3; ++d) {
        int64_t k = (int64_t)floor(box[d] / (R / 16.0));
        nc[d] = (int32_t)(k < 1 ? 1 : (k > 256 ? 256 : k));
        cw[d] = box[d] / nc[d];
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *cell_of = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) {
            double t = pos[3 * i + d] / box[d];
            xw[3 * i + d] = (t - floor(t)) * box[d];
            int64_t cd = (int64_t)floor(xw[3 * i + d] / cw[d]);
            c[d] = cd < 0 ? 0 : (cd >= nc[d] ? nc[d] - 1 : cd);
        }
        cell_of[i] = c[0] + nc[0] * (c[1] + (int64_t)nc[1] * c[2]);
        start[cell_of[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
        memcpy(fill, start, sizeof(int64_t) * (size_t)ncell);
        for (int64_t i = 0; i < n; ++i) order[fill[cell_of[i]]++] = i;
        free(fill);
    }
    double lim[64];
    for (int l = 0; l < nl && l < 64; ++l) lim[l] = tail * s[l] * s[l];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = targets[t];
        const double *xi = xw + 3 * i;
        int64_t ci[3], K[3];
        for (int d = 0; d < 3; ++d) {
            int64_t cd = (int64_t)floor(xi[d] / cw[d]);
            ci[d] = cd < 0 ? 0 : (cd >= nc[d] ? nc[d] - 1 : cd);
            K[d] = (int64_t)ceil(R / cw[d]) + 1;
        }
        nsum_t f[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t oz = -K[2]; oz <= K[2]; ++oz) {
            const int64_t cz = ci[2] + oz, iz = floor_div(cz, nc[2]), mz = cz - iz * nc[2];
            for (int64_t oy = -K[1]; oy <= K[1]; ++oy) {
                const int64_t cy = ci[1] + oy, iy = floor_div(cy, nc[1]), my = cy - iy * nc[1];
                for (int64_t ox = -K[0]; ox <= K[0]; ++ox) {
                    const int64_t cx = ci[0] + ox, ix = floor_div(cx, nc[0]), mx = cx - ix * nc[0];
                    const double shift[3] = {ix * box[0], iy * box[1], iz * box[2]};
                    const int64_t cell = mx + nc[0] * (my + (int64_t)nc[1] * mz);
                    for (int64_t p = start[cell]; p < start[cell + 1]; ++p) {
                        const int64_t j = order[p];
                        const double d0 = xi[0] - (xw[3 * j] + shift[0]);
                        const double d1 = xi[1] - (xw[3 * j + 1] + shift[1]);
                        const double d2 = xi[2] - (xw[3 * j + 2] + shift[2]);
                        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                        if (r2 >= R2) continue;
                        double c = 0.0;
                        for (int l = 0; l < nl; ++l)
                            if (r2 < lim[l]) c += omega[l] * (2.0 / (s[l] * s[l])) * exp(-r2 / (s[l] * s[l]));
                        c *= q[j];
                        nadd(&f[0], c * d0);
                        nadd(&f[1], c * d1);
                        nadd(&f[2], c * d2);
                    }
                }
            }
        }
        for (int d = 0; d < 3; ++d) F[3 * t + d] = q[i] * nval(&f[d]);
    }
    free(order);
    free(start);
    free(cell_of);
    free(xw);
}

/* ------------------------------------------------------------------------ */
/* Classical Ewald summation (Sec. 2, eq. "splitting"), tinfoil boundary, used
 * only as an independent validator of the whole splitting on small systems.
 * Real-space part over images |n_d| <= nimg:
 *   U_r = 1/2 sum_{i,j,n}' q_i q_j erfc(alpha r)/r,
 *   F_i = q_i sum_{j,n}' q_j [erfc(alpha r)/r + 2 alpha/sqrt(pi) exp(-alpha^2 r^2)] d / r^2.
 * The reciprocal part is orc_structure_factor + orc_far_force with
 * w = 4 pi exp(-k^2/(4 alpha^2)) / (k^2 V), and the self term
 * -alpha/sqrt(pi) sum q_i^2. */
void orc_ewald_real(int64_t n, const double *pos, const double *q, const double *box, double alpha,
                    int nimg, double *F, double *U) {
    double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *ei = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double t = pos[3 * i + d] / box[d];
            xw[3 * i + d] = (t - floor(t)) * box[d];
        }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
        double f[3] = {0, 0, 0};
        nsum_t e = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            double base[3];
            min_image(xw + 3 * i, xw + 3 * j, box, base);
            for (int nz = -nimg; nz <= nimg; ++nz)
                for (int ny = -nimg; ny <= nimg; ++ny)
                    for (int nx = -nimg; nx <= nimg; ++nx) {
                        if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
                        double d0 = base[0] + nx * box[0];
                        double d1 = base[1] + ny * box[1];
                        double d2 = base[2] + nz * box[2];
                        double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                        double r = sqrt(r2);
                        double ec = erfc(alpha * r) / r;
                        double c = q[i] * q[j] * (ec + 2.0 * alpha / sqrt(M_PI) * exp(-alpha * alpha * r2)) / r2;
                        f[0] += c * d0;
                        f[1] += c * d1;
                        f[2] += c * d2;
                        nadd(&e, 0.5 * q[i] * q[j] * ec);
                    }
        }
        F[3 * i] = f[0];
        F[3 * i + 1] = f[1];
        F[3 * i + 2] = f[2];
        ei[i] = nval(&e);
    }
    nsum_t ue = {0, 0};
    for (int64_t i = 0; i < n; ++i) nadd(&ue, ei[i]);
    *U = nval(&ue);
    free(ei);
    free(xw);
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, written from its published
 * definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with
 * multipliers 0xD2511F53 and 0xCD9E8D57, the key bumped by the Weyl
 * increments 0x9E3779B9 and 0xBB67AE85 between rounds. */
void orc_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Two uniforms in [0,1) with 53 random bits each from one Philox block. */
static void philox_uniform2(uint64_t seed, uint32_t stream, uint64_t index, uint32_t lane,
                            double *a, double *b) {
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), stream, lane};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    uint64_t x = ((uint64_t)o[1] << 32) | o[0];
    uint64_t y = ((uint64_t)o[3] << 32) | o[2];
    *a = (double)(x >> 11) * 0x1.0p-53;
    *b = (double)(y >> 11) * 0x1.0p-53;
}

/* One 1-D factor of the proposal pmf (Sec. 3.3, corrected argument):
 * q(m) = 1/2 [erf((m+1/2) a) - erf((m-1/2) a)],  a = pi s_0 / L_d;
 * evaluated through erfc on |m| to avoid cancellation in the tails. */
static double proposal_pmf_1d(int32_t m, double a) {
    if (m == 0) return erf(0.5 * a);
    double am = fabs((double)m);
    return 0.5 * (erfc((am - 0.5) * a) - erfc((am + 0.5) * a));
}

double orc_proposal_pmf_1d(int32_t m, double a) { return proposal_pmf_1d(m, a); }

/* Unnormalised target p(m) proportional to F~(2 pi m / L) (eq. "distribution"). */
static double target_unnorm(const int32_t *m, const double *box, int M, const double *omega,
                            const double *s) {
    double k2 = 0.0;
    for (int d = 0; d < 3; ++d) {
        double k = 2.0 * M_PI * m[d] / box[d];
        k2 += k * k;
    }
    return orc_sog_Ftilde(k2, M, omega, s);
}

/* Metropolis-Hastings independence sampler of Sec. 3.3.
 * Proposal attempt t draws three normals z_d (Box-Muller on Philox uniforms,
 * block lanes 0 and 1) and the acceptance uniform (lane 2); the candidate is
 * m*_d = round(z_d L_d / (sqrt(2) pi s_0)), i.e. a normal of variance
 * (L_d/(s_0 pi))^2/2 rounded to the nearest integer.  A candidate m* = 0 is
 * discarded and the next attempt is drawn.  The first nonzero candidate
 * starts the chain; `burnin` transitions are then discarded and the next
 * nsamp chain states are written to m_out (a rejected move repeats the
 * current state).  Returns the acceptance rate of the recorded transitions
 * through acc_rate. */
int orc_mh_sample(const double *box, int M, const double *omega, const double *s, uint64_t seed,
                  uint32_t stream, int64_t burnin, int64_t nsamp, int32_t *m_out, double *acc_rate) {
    const double s0 = s[0];
    double sd[3], a[3];
    for (int d = 0; d < 3; ++d) {
        sd[d] = box[d] / (sqrt(2.0) * M_PI * s0);
        a[d] = M_PI * s0 / box[d];
    }
    uint64_t t = 0;
    int32_t cur[3] = {0, 0, 0};
    double pcur = 0.0, qcur = 0.0;
    int64_t accepted = 0;
    int started = 0;
    int64_t total = burnin + nsamp;
    int64_t step = 0;
    while (step < total) {
        double u1, u2, u3, u4, ua, ub;
        philox_uniform2(seed, stream, t, 0, &u1, &u2);
        philox_uniform2(seed, stream, t, 1, &u3, &u4);
        philox_uniform2(seed, stream, t, 2, &ua, &ub);
        ++t;
        double r1 = sqrt(-2.0 * log(1.0 - u1));
        double r2 = sqrt(-2.0 * log(1.0 - u3));
        double z[3] = {r1 * cos(2.0 * M_PI * u2), r1 * sin(2.0 * M_PI * u2), r2 * cos(2.0 * M_PI * u4)};
        int32_t cand[3];
        for (int d = 0; d < 3; ++d) cand[d] = (int32_t)round(z[d] * sd[d]);
        if (cand[0] == 0 && cand[1] == 0 && cand[2] == 0) continue;
        double pc = target_unnorm(cand, box, M, omega, s);
        double qc = proposal_pmf_1d(cand[0], a[0]) * proposal_pmf_1d(cand[1], a[1]) *
                    proposal_pmf_1d(cand[2], a[2]);
        if (!started) {
            for (int d = 0; d < 3; ++d) cur[d] = cand[d];
            pcur = pc;
            qcur = qc;
            started = 1;
            continue;
        }
        double ratio = (pc * qcur) / (pcur * qc);
        int acc = ua < ratio;
        if (acc) {
            for (int d = 0; d < 3; ++d) cur[d] = cand[d];
            pcur = pc;
            qcur = qc;
        }
        if (step >= burnin) {
            int64_t o = step - burnin;
            for (int d = 0; d < 3; ++d) m_out[3 * o + d] = cur[d];
            accepted += acc;
        }
        ++step;
    }
    if (acc_rate) *acc_rate = nsamp > 0 ? (double)accepted / (double)nsamp : 0.0;
    return 0;
}

/* Threads of the OpenMP loops above (used to time the oracle on one core and
 * on all cores; no arithmetic). */
int orc_max_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
