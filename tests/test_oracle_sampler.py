"""Pins of the oracle's k sampling (Sec. 3.3): Philox known answers, proposal
pmf against quadrature, and chi-square tests of both samplers against the
enumerated target P_k = F~(k)/(pi^{3/2} S).  CPU only."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers(orc):
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            out = orc.philox4x32_10(v[0:4], v[4:6])
            assert [int(x) for x in out] == v[6:10]


@pytest.mark.parametrize("m", [0, 1, 2, 3, 7, -4])
def test_proposal_pmf_equals_quadrature(orc, m):
    # Sec. 3.3: q(m) = (sqrt(pi) s0/L) int_{m-1/2}^{m+1/2} exp(-(pi s0 x/L)^2) dx.
    L, s0 = 10.0, 1.5416
    a = math.pi * s0 / L
    quad = integrate.quad(lambda x: math.sqrt(math.pi) * s0 / L * math.exp(-(a * x) ** 2), m - 0.5, m + 0.5,
                          epsabs=1e-15, epsrel=1e-13)[0]
    assert abs(orc.proposal_pmf_1d(m, a) / quad - 1) < 1e-10


def _support(orc, sog, box, pmin):
    m = orc.kvectors_full(sog, box, tail=60.0)
    p = orc.target_pmf(sog, box, m)
    return m, p


def _chi2(orc, sog, box, draws, min_expected=8.0):
    m, p = _support(orc, sog, box, 0.0)
    n = draws.shape[0]
    assert abs(p.sum() - 1) < 1e-9  # the enumeration covers the distribution
    key = {tuple(v): i for i, v in enumerate(m.tolist())}
    idx = np.array([key.get(tuple(v), -1) for v in draws.tolist()])
    assert (idx >= 0).all()
    counts = np.bincount(idx, minlength=len(p)).astype(float)
    expected = p * n
    big = expected >= min_expected
    # pool the small-probability vectors into shells of |m|^2
    r2 = (m.astype(np.int64) ** 2).sum(1)
    obs, exp = list(counts[big]), list(expected[big])
    small = np.where(~big)[0]
    order = small[np.argsort(r2[small], kind="stable")]
    acc_o = acc_e = 0.0
    for i in order:
        acc_o += counts[i]
        acc_e += expected[i]
        if acc_e >= min_expected:
            obs.append(acc_o); exp.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0:
        obs[-1] += acc_o; exp[-1] += acc_e
    obs, exp = np.array(obs), np.array(exp)
    exp *= obs.sum() / exp.sum()
    return stats.chisquare(obs, exp).pvalue, len(obs)


@pytest.mark.parametrize("box,rc", [((10.0, 10.0, 10.0), 3.0), ((12.0, 8.0, 10.0), 3.5)])
def test_exact_mixture_sampler_chi_square(orc, box, rc):
    sog = orc.sog_row2(rc)
    draws = orc.exact_mixture_sample(sog, np.array(box), 30000, np.random.default_rng(21))
    pval, nbins = _chi2(orc, sog, np.array(box), draws)
    assert nbins > 50
    assert pval > 1e-3


@pytest.mark.parametrize("box,rc", [((10.0, 10.0, 10.0), 3.0), ((12.0, 8.0, 10.0), 3.5)])
def test_mh_sampler_chi_square(orc, box, rc):
    # Metropolis-Hastings independence chain, thinned to near-independent draws.
    sog = orc.sog_row2(rc)
    chain, acc = orc.mh_sample(sog, np.array(box), seed=77, stream=3, n=300000)
    assert 0.4 < acc < 0.9
    assert not (chain == 0).all(1).any()
    pval, nbins = _chi2(orc, sog, np.array(box), chain[::10])
    assert nbins > 50
    assert pval > 1e-3


def test_chi_square_has_power(orc):
    # The chi-square check sees a small distortion of the target: moving the
    # |m_x| = 1 draws to |m_x| = 2 must be rejected.
    sog = orc.sog_row2(3.0)
    box = np.array([10.0, 10.0, 10.0])
    draws = orc.exact_mixture_sample(sog, box, 30000, np.random.default_rng(5))
    bad = draws.copy()
    bad[:, 0] = np.where(np.abs(bad[:, 0]) == 1, 2 * np.sign(bad[:, 0]), bad[:, 0])
    pval, _ = _chi2(orc, sog, box, bad)
    assert pval < 1e-6


def test_mh_sampler_is_deterministic_per_seed_and_stream(orc):
    sog = orc.sog_row2(3.0)
    box = np.array([10.0, 10.0, 10.0])
    a, _ = orc.mh_sample(sog, box, seed=5, stream=0, n=500)
    b, _ = orc.mh_sample(sog, box, seed=5, stream=0, n=500)
    c, _ = orc.mh_sample(sog, box, seed=5, stream=1, n=500)
    assert (a == b).all() and not (a == c).all()
