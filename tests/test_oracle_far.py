"""Pins of the oracle's Fourier part (Sec. 3.1-3.3) and of the whole split
(Ewald, Madelung).  CPU only."""
import math
import os

import numpy as np
import pytest

from paper_2205_13824_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROW2 = (1.62976708826776469, 3.633717409009413, 1.00780697934380681, 16)
ROW4 = (1.32070036405934420, 2.277149356440992, 1.00188914114811980, 64)
ROW5 = (1.21812525709410644, 1.774456369233284, 1.00090146156033341, 102)


def sog_at(orc, row, rc):
    return orc.SOG(row[0], row[1] * rc / 10.0, row[2], row[3])


def random_system(n, L, seed):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * L
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return pos, q, np.array([L, L, L])


def relrms(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))


def test_far_force_is_minus_gradient_of_ustar(orc):
    # Pins the sign of eq. "forcesplit" (second line).
    pos, q, box = random_system(20, 10.0, 0)
    sog = orc.sog_row2(3.0)
    F, _, _, _ = orc.far_full(pos, q, box, sog)
    h = 1e-6
    for i in (2, 11):
        for d in range(3):
            p = pos.copy(); p[i, d] += h
            up = orc.far_full(p, q, box, sog)[1]
            p = pos.copy(); p[i, d] -= h
            um = orc.far_full(p, q, box, sog)[1]
            assert abs(-(up - um) / (2 * h) - F[i, d]) < 1e-6 * max(1.0, abs(F[i, d]))


def test_far_force_sums_to_zero(orc):
    pos, q, box = random_system(200, 10.0, 1)
    sog = orc.sog_row2(3.0)
    F, _, _, _ = orc.far_full(pos, q, box, sog)
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).max() * 200
    # the random-batch force also sums to zero for any k list
    m = orc.exact_mixture_sample(sog, box, 50, np.random.default_rng(2))
    Fr, _, _, _ = orc.far_rb(pos, q, box, sog, m, 50)
    assert np.abs(Fr.sum(0)).max() < 1e-12 * np.abs(Fr).max() * 200


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_fourier_series_equals_real_space_image_sum(orc, l):
    # Poisson summation: the Fourier-space force of one Gaussian equals the
    # direct sum of its gradient over periodic images (two independent codes).
    pos, q, box = random_system(60, 10.0, 3)
    sog = orc.sog_row2(3.0)
    m = orc.kvectors_full(sog, box)
    k = 2 * math.pi * m / box
    k2 = (k * k).sum(1)
    w = math.pi ** 1.5 * sog.omega[l] * sog.s[l] ** 3 * np.exp(-sog.s[l] ** 2 * k2 / 4) / orc.volume(box)
    t = np.arange(0, 60, 6)
    Fk, _, _, _ = orc.far_kspace(pos, q, box, m, w, targets=t)
    nimg = int(math.ceil(6.1 * sog.s[l] / 10.0)) + 1
    Fr = orc.gauss_realspace_force(pos, q, box, sog.omega[l], sog.s[l], nimg, t)
    assert np.abs(Fk - Fr).max() < 1e-12 * np.abs(Fr).max()


@pytest.mark.parametrize("box,rc", [((10.0, 10.0, 10.0), 3.0), ((20.0, 14.0, 9.0), 3.5),
                                    ((144.225, 144.225, 144.225), 3.5)])
def test_S_three_ways(orc, box, rc):
    # eq. "S": product form == enumeration of sum_{k != 0} F~/pi^{3/2} == Poisson form of H.
    sog = orc.sog_row2(rc)
    S1 = orc.S_product(sog, box)
    S3 = orc.S_poisson(sog, box)
    # H1 H2 H3 - 1 cancels for wide Gaussians in the Poisson form: ~1e-12 rounding
    assert abs(S3 / S1 - 1) < 1e-10
    if box[0] < 50:
        S2 = orc.S_enumerated(sog, box)
        assert abs(S2 / S1 - 1) < 1e-12


def test_H_poisson_form_corrected_exponent(orc):
    # eq. "Hell": the two forms agree with exponent -m^2 L^2/s^2 (not -pi^2 m^2 L^2/s^2).
    for s, L in ((1.5, 10.0), (17.73, 10.0), (4.0, 6.0), (300.0, 144.0)):
        assert abs(orc.H_poisson(s, L) / orc.H_direct(s, L) - 1) < 1e-13


@pytest.mark.parametrize("row,ftol,utol", [(ROW2, 2e-3, 2e-3), (ROW4, 2e-6, 2e-6), (ROW5, 2e-9, 5e-8)])
def test_whole_split_agrees_with_ewald(orc, row, ftol, utol):
    # Near + full Fourier sum - self energy reproduces classical Ewald summation
    # to the split's own kernel error (row 2: ~1.6e-3 in the pair force just
    # beyond r_c; rows 4/5 far smaller).  Any dropped term, sign or factor in
    # either part shows up at O(1).
    pos, q, box = random_system(20, 10.0, 0)
    rc = 3.0
    sog = sog_at(orc, row, rc)
    F, U, _ = orc.rbsog_full(pos, q, box, rc, sog)
    Fe, Ue = orc.ewald(pos, q, box, alpha=0.8, nimg=2)
    assert relrms(F, Fe) < ftol
    assert abs(U - Ue) / abs(Ue) < utol


def test_ewald_validator_independent_of_alpha(orc):
    pos, q, box = random_system(16, 8.0, 4)
    F1, U1 = orc.ewald(pos, q, box, alpha=0.7, nimg=2)
    F2, U2 = orc.ewald(pos, q, box, alpha=1.1, nimg=2)
    assert relrms(F1, F2) < 1e-11 and abs(U1 - U2) < 1e-11 * abs(U1)


def test_madelung_energy_and_zero_lattice_forces(orc):
    # Rock-salt crystal (Fig. 2 setup): lattice energy -M/(2a) per ion, forces 0.
    with open(os.path.join(HERE, "golden", "madelung.txt")) as f:
        mad = float([ln for ln in f if not ln.startswith("#")][0])
    pos, q, box = W.nacl_lattice(8, 1.0)
    rc = 3.5
    F, U, _ = orc.rbsog_full(pos, q, box, rc, sog_at(orc, ROW5, rc))
    assert abs(U / len(q) / (-mad / 2) - 1) < 1e-8
    assert np.abs(F).max() < 1e-12
    F2, U2, _ = orc.rbsog_full(pos, q, box, rc, sog_at(orc, ROW2, rc))
    assert abs(U2 / len(q) / (-mad / 2) - 1) < 2e-3
    assert np.abs(F2).max() < 1e-12


def test_rb_estimator_unbiased_with_lemma1_variance(orc):
    # Lemma 1: E F* = F_F, and (corrected constant)
    #   E|Xi_i|^2 = (1/P) [ (pi^{3/2} S q_i^2 / V^2) sum_k F~ |k|^2 Im(e^{-ik.r_i} rho)^2 - |F_F,i|^2 ].
    pos, q, box = random_system(40, 10.0, 5)
    sog = orc.sog_row2(3.0)
    S = orc.S_product(sog, box)
    V = orc.volume(box)
    Ffull, _, re, im = orc.far_full(pos, q, box, sog)
    mk = orc.kvectors_full(sog, box)
    k = 2 * math.pi * mk / box
    Ft = sog.Ftilde_vec((k * k).sum(1))
    th = pos @ k.T
    imv = np.cos(th) * im[None, :] - np.sin(th) * re[None, :]
    P, R = 8, 3000
    var_pred = (math.pi ** 1.5 * S * q ** 2 / V ** 2
                * np.sum(Ft[None, :] * (k * k).sum(1)[None, :] * imv ** 2, axis=1)
                - (Ffull ** 2).sum(1)) / P
    rng = np.random.default_rng(6)
    draws = orc.exact_mixture_sample(sog, box, P * R, rng)
    acc = np.zeros((R, 40, 3))
    for r in range(R):
        acc[r] = orc.far_rb(pos, q, box, sog, draws[r * P:(r + 1) * P], P, S)[0]
    mean = acc.mean(0)
    sd = acc.std(0, ddof=1)
    z = (mean - Ffull) / (sd / math.sqrt(R))
    assert np.abs(z).max() < 5.0
    # The particles share the k draws, so their errors are correlated; the
    # total squared error of the mean is compared with its expectation
    # sum_i Var_i / R from Lemma 1 (a ratio above 6 has probability < 2 %
    # even if every component were perfectly correlated).
    ratio = float(((mean - Ffull) ** 2).sum()) / (float(var_pred.sum()) / R)
    assert ratio < 6.0
    var_emp = ((acc - Ffull[None]) ** 2).sum(2).mean(0)
    assert abs(var_emp.sum() / var_pred.sum() - 1) < 0.08


@pytest.mark.parametrize("box,rc,n", [((10.0, 10.0, 10.0), 3.0, 120), ((12.0, 9.0, 11.0), 2.9, 90),
                                      ((16.0, 16.0, 16.0), 3.5, 200)])
@pytest.mark.parametrize("n_real", [0, 1, 3, 5])
def test_poisson_split_far_field_equals_full_fourier_sum(orc, box, rc, n, n_real):
    # The large-system far field (Sec. 3.3, each Gaussian through the Poisson
    # identity: the narrowest in real space with a radius cutoff over a cell
    # grid of the periodically tiled box, the widest over half the k lattice)
    # against the plain Fourier sum over every k != 0: two independent codes.
    rng = np.random.default_rng(n + n_real)
    box = np.asarray(box)
    pos = rng.random((n, 3)) * box
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    sog = orc.sog_row2(rc)
    t = np.arange(0, n, 7)
    Ffull, _, _, _ = orc.far_full(pos, q, box, sog, targets=t)
    Fs = orc.far_split(pos, q, box, sog, t, n_real)
    assert relrms(Fs, Ffull) < 1e-12


def test_poisson_split_real_space_alone_equals_image_sum(orc):
    # The cutoff real-space sum of one Gaussian against the plain image sum
    # over every image within the same reach (no cells, no cutoff).
    pos, q, box = random_system(50, 9.0, 8)
    sog = orc.sog_row2(3.0)
    t = np.arange(0, 50, 5)
    for l in (0, 2, 4):
        Fc = orc.far_realspace_cut(pos, q, box, sog.omega[l:l + 1], sog.s[l:l + 1], t)
        nimg = int(math.ceil(6.1 * sog.s[l] / 9.0)) + 1
        Fi = orc.gauss_realspace_force(pos, q, box, sog.omega[l], sog.s[l], nimg, t)
        # rounding of the O(omega_l / s_l) terms that cancel to the total
        assert np.abs(Fc - Fi).max() < 1e-11 * np.abs(Fi).max() + 1e-12 * sog.omega[l] / sog.s[l]


def _truncation_error(orc, sog_full_row, rc, M, pos, q, box):
    """R^F(M) = |U_err^F / U*| of Theorem 1 summed directly: the Gaussians
    l > M (nominal omega_l) over every k != 0 against the far energy of the
    split truncated at M (Sec. 4.1, eqs. "UerrF" and "uF")."""
    b, sig10, w0, _ = sog_full_row
    sigma = sig10 * rc / 10.0
    sog = orc.SOG(b, sigma, w0, M)
    m = orc.kvectors_full(sog, box)
    k = 2 * math.pi * m / box
    k2 = (k * k).sum(1)
    re, im = orc.structure_factor(pos, q, box, m)
    rho2 = re * re + im * im
    tail = np.zeros_like(k2)
    for l in range(M + 1, M + 400):
        om = math.sqrt(2.0 / math.pi) * math.log(b) / (sigma * b ** l)
        s = math.sqrt(2.0) * b ** l * sigma
        term = om * s ** 3 * np.exp(-s * s * k2 / 4.0)
        tail += term
        if term.max() < 1e-300:
            break
    V = orc.volume(box)
    Uerr = math.pi ** 1.5 * float((tail * rho2).sum()) / (2 * V)
    Uf = float((sog.Ftilde_vec(k2) * rho2).sum()) / (2 * V)
    return abs(Uerr / Uf), orc.theorem1_bound(b, sigma, M, float(np.max(box)))


@pytest.mark.parametrize("L,rc,n", [(10.0, 3.0, 200), (20.0, 3.0, 400), (30.0, 3.5, 300)])
def test_theorem1_bound_holds_with_the_true_decay_rate(orc, L, rc, n):
    # Theorem 1: R^F(M) <= b^{2M} exp(-2 (b^{2M} - 1) (pi b sigma / L)^2).
    # Directly summed, the error stays below the bound for every M, and once
    # the first omitted Gaussian dominates (M >= 4) the ratio bound / R^F no
    # longer changes with M: the bound's exponent is the true decay rate (a
    # dropped factor b, 2 or pi in it would make the ratio run away or fall
    # below 1 within a few M).
    pos, q, box = random_system(n, L, 17)
    ratios = {}
    for M in range(1, 9):
        R, bound = _truncation_error(orc, ROW2, rc, M, pos, q, box)
        if R < 1e-290:
            break
        assert R <= bound, (M, R, bound)
        ratios[M] = bound / R
    assert 4 in ratios and 5 in ratios
    for M in sorted(ratios):
        if M >= 4 and M + 1 in ratios:
            assert abs(ratios[M + 1] / ratios[M] - 1.0) < 0.05, ratios
