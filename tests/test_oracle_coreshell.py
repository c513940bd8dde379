"""Pins of the oracle's core-shell near kernel (Sec. 3.4), against what the
mathematics fixes: the linear-interpolation error bound on every table
interval, the alternating-series remainder of the Taylor core, exact values
at table points, and the direct Gaussian sum for whole systems."""
import math

import numpy as np
import pytest

from oracle import coreshell as cs


@pytest.mark.parametrize("rc", [3.0, 3.5, 10.0])
def test_table_error_within_interpolation_bound(orc, rc):
    sog = orc.sog_row2(rc)
    t = cs.Table(sog, rc)
    x = np.linspace(t.rin ** 2, rc * rc * (1 - 1e-7), 200001)
    xf = x.astype(np.float32).astype(np.float64)  # the table is indexed by r^2 in FP32
    g, h = t.lookup(x)
    ge, he = cs.kernels_exact(xf, sog)
    bg, bh = t.interval_bound(x)
    assert np.all(np.abs(g - ge) <= bg * (1 + 1e-9) + 1e-15)
    assert np.all(np.abs(h - he) <= bh * (1 + 1e-9) + 1e-15)
    # and the bound is tight (a wrong node or slope would sit far above it)
    assert np.max(np.abs(g - ge) / bg) > 0.9


def test_table_points_are_exact(orc):
    sog = orc.sog_row2(3.5)
    t = cs.Table(sog, 3.5)
    rng = np.random.default_rng(3)
    for _ in range(200):
        x = rng.uniform(t.rin ** 2, 3.5 ** 2)
        bits = int(np.array([np.float32(x)], dtype=np.float32).view(np.uint32)[0])
        node = np.array([(bits >> t.shift) << t.shift], dtype=np.uint32).view(np.float32)[0]
        g, h = t.lookup(np.array([float(node)]))
        ge, he = cs.kernels_exact(np.array([float(node)]), sog)
        assert g[0] == ge[0] and h[0] == he[0]


def test_table_refuses_too_wide_a_range(orc):
    with pytest.raises(ValueError):
        cs.Table(orc.sog_row2(3.0), 3.0, rin=0.05)


@pytest.mark.parametrize("rc", [3.0, 10.0])
def test_taylor_core_within_remainder_bound(orc, rc):
    sog = orc.sog_row2(rc)
    A, B = cs.taylor_coefficients(sog, 4)
    rin = cs.RIN_FRACTION * rc
    x = np.linspace(1e-6, rin * rin, 5001)
    g, h = cs.core_kernels(x, A, B)
    ge, he = cs.kernels_exact(x, sog)
    # alternating series of e^{-y}, y = x/s^2 < 5: remainder at most y^Q/Q!
    bg = sum(2 * w / s ** 2 * (x / s ** 2) ** 4 / 24.0 for w, s in zip(sog.omega, sog.s))
    bh = sum(w * (x / s ** 2) ** 4 / 24.0 for w, s in zip(sog.omega, sog.s))
    # plus FP64 rounding of the 1/r^3 and 1/r terms, which dominate as r -> 0
    assert np.all(np.abs(g - ge) <= bg * (1 + 1e-9) + 1e-14 * np.abs(ge))
    assert np.all(np.abs(h - he) <= bh * (1 + 1e-9) + 1e-14 * np.abs(he))
    # the alternating sign matters: without it the core is off by orders of magnitude more
    A_bad = np.abs(A)
    g_bad, _ = cs.core_kernels(x, A_bad, B)
    assert np.max(np.abs(g_bad - ge)) > 100 * np.max(bg)


def test_core_and_shell_meet_at_rin(orc):
    sog = orc.sog_row2(3.5)
    t = cs.Table(sog, 3.5)
    A, B = cs.taylor_coefficients(sog, 4)
    x = np.array([np.nextafter(np.float32(t.rin ** 2), np.float32(10))], dtype=np.float64)
    gs, hs = t.lookup(x)
    gc, hc = cs.core_kernels(x, A, B)
    assert abs(gs[0] - gc[0]) / abs(gc[0]) < 1e-5 and abs(hs[0] - hc[0]) / abs(hc[0]) < 2e-5


def test_coreshell_forces_match_direct_sum(orc):
    rng = np.random.default_rng(12)
    L, n = 12.0, 800
    pos = rng.random((n, 3)) * L
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    box = np.array([L, L, L])
    rc = 3.5
    sog = orc.sog_row2(rc)
    nb = orc.neighbors_brute(pos, box, rc)
    F, U = cs.near_coreshell(pos, q, box, rc, sog, nb)
    Fo, Uo = orc.near_brute(pos, q, box, rc, sog)
    err = math.sqrt(float(np.sum((F - Fo) ** 2) / np.sum(Fo ** 2)))
    assert err < 5e-6
    assert abs(U - Uo) / abs(Uo) < 5e-6
