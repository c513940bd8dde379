"""Pins of the oracle's velocity-Verlet loop (Algorithm 1 with NVE
integration).  CPU only."""
import numpy as np

from paper_2205_13824_amd import workloads as W


def small_system(n=24, L=8.0, seed=3):
    rng = np.random.default_rng(seed)
    # keep ions apart so that a short run stays smooth
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.2, seed)
    v = W.maxwellian(n, 0.5, seed + 1)
    return pos, q, box, v


def test_vv_conserves_momentum_with_rb_forces(orc):
    pos, q, box, v = small_system()
    rc = 3.0
    sog = orc.sog_row2(rc)
    P = 20
    kseq = orc.exact_mixture_sample(sog, box, P * 21, np.random.default_rng(9))
    x, v1, F, _ = orc.vv_run(pos, v, q, box, rc, sog, P, kseq, 20, 2e-3)
    assert np.abs(v1.sum(0) - v.sum(0)).max() < 1e-12


def test_vv_conserves_energy_with_full_forces(orc):
    # With the deterministic far field (every k, weight F~/V) the discrete
    # energy fluctuates at O(dt^2): halving dt quarters the drift.  Table 1
    # row 5 is used because the truncated split's pair potential steps by
    # sum_{l>M} omega_l at r_c (2e-4 for row 2, 2e-9 for row 5), which would
    # otherwise hide the integrator's error whenever a pair crosses r_c.
    pos, q, box, v = small_system()
    rc = 3.0
    sog = orc.SOG(1.21812525709410644, 1.774456369233284 * rc / 10.0, 1.00090146156033341, 102)

    def run(dt, steps):
        x = pos.copy(); vv = v.copy()
        m = orc.kvectors_full(sog, box)
        w = orc.full_weights(sog, box, m)

        def force(xx):
            Fn, Un = orc.near_cells(xx, q, box, rc, sog)
            Ff, Us, _, _ = orc.far_kspace(xx, q, box, m, w)
            return Fn + Ff, Un + Us - orc.self_energy(sog, q)
        F, U = force(x)
        e0 = U + 0.5 * (vv * vv).sum()
        worst = 0.0
        for _ in range(steps):
            vv += 0.5 * dt * F
            x += dt * vv
            x -= box * np.floor(x / box)
            F, U = force(x)
            vv += 0.5 * dt * F
            worst = max(worst, abs(U + 0.5 * (vv * vv).sum() - e0))
        return worst

    d1 = run(4e-3, 50)
    d2 = run(2e-3, 100)
    assert d2 < 0.4 * d1


def test_vv_time_reversible(orc):
    pos, q, box, v = small_system()
    rc = 3.0
    sog = orc.sog_row2(rc)
    P = 16
    kseq = orc.exact_mixture_sample(sog, box, P * 11, np.random.default_rng(4))
    x1, v1, _, _ = orc.vv_run(pos, v, q, box, rc, sog, P, kseq, 10, 1e-3)
    # replay the same batches backwards with reversed velocities
    back = np.concatenate([kseq[(10 - e) * P:(11 - e) * P] for e in range(11)])
    x2, v2, _, _ = orc.vv_run(x1, -v1, q, box, rc, sog, P, back, 10, 1e-3)
    d = x2 - pos
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(v2 + v).max() < 1e-9
