"""Pins of the oracle's Langevin (BAOAB) thermostat: the noise is standard
normal, the O step alone drives free particles to the Maxwellian at T, and
with gamma = 0 a step is the velocity-Verlet step."""
import math

import numpy as np

from oracle import thermostat as th


def test_noise_is_standard_normal(orc):
    xi = np.concatenate([th.normals(orc, 500, s, 123) for s in range(8)])
    assert abs(xi.mean()) < 4 / math.sqrt(xi.size)
    assert abs(xi.var() - 1.0) < 4 * math.sqrt(2.0 / xi.size)
    # components and steps are independent
    assert abs(np.corrcoef(xi[:, 0], xi[:, 1])[0, 1]) < 0.05
    a, b = th.normals(orc, 500, 0, 123), th.normals(orc, 500, 1, 123)
    assert abs(np.corrcoef(a.ravel(), b.ravel())[0, 1]) < 0.05


def test_ou_step_reaches_target_temperature(orc):
    # free particles: v_{s+1} = c1 v_s + c2 xi_s is exact for the OU process, so
    # <v^2> tends to T/m whatever dt and gamma
    n, T, m, c1 = 400, 2.5, 1.7, math.exp(-0.5)
    c2 = math.sqrt((1 - c1 * c1) * T / m)
    v = np.zeros((n, 3))
    acc = []
    for s in range(60):
        v = c1 * v + c2 * th.normals(orc, n, s, 9)
        if s >= 20:
            acc.append((v * v).mean())
    assert abs(np.mean(acc) / (T / m) - 1.0) < 0.03


def test_zero_friction_is_velocity_verlet(orc):
    rng = np.random.default_rng(3)
    pos = rng.random((60, 3)) * 8.0
    q = np.where(np.arange(60) % 2 == 0, 1.0, -1.0)
    box = np.array([8.0, 8.0, 8.0])
    sog = orc.sog_row2(2.5)
    v0 = rng.standard_normal((60, 3)) * 0.3
    ks, _ = orc.mh_sample(sog, box, seed=4, stream=0, n=4 * 10)
    x1, v1 = th.baoab_run(orc, pos, v0, q, box, 2.5, sog, 10, ks, 3, 1e-3, 0.0, 1.0, 5)
    x2, v2, _, _ = orc.vv_run(pos, v0, q, box, 2.5, sog, 10, ks, 3, 1e-3)
    assert np.allclose(x1, x2, rtol=0, atol=1e-12) and np.allclose(v1, v2, rtol=0, atol=1e-12)


def _nh_system(orc, n=24, L=8.0, seed=3):
    from paper_2205_13824_amd import workloads as W
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.2, seed)
    v = W.maxwellian(n, 0.5, seed + 1)
    return pos, q, box, v


def test_nose_hoover_without_thermostat_mass_is_velocity_verlet(orc):
    pos, q, box, v = _nh_system(orc)
    rc, P = 3.0, 16
    sog = orc.sog_row2(rc)
    kseq = orc.exact_mixture_sample(sog, box, P * 9, np.random.default_rng(5))
    x1, v1, _, _ = orc.vv_run(pos, v, q, box, rc, sog, P, kseq, 8, 2e-3)
    x2, v2, xi, _, _ = th.nose_hoover_run(orc, pos, v, q, box, rc, sog, P, kseq, 8, 2e-3, T=1.0, tau=math.inf)
    assert xi == 0.0 and (x1 == x2).all() and (v1 == v2).all()


def test_nose_hoover_conserves_its_extended_energy(orc):
    # deterministic far field (every k, weight F~/V) and Table 1 row 5, as for
    # the velocity-Verlet energy pin: H = U + K + Q xi^2/2 + N_f T eta drifts
    # at O(dt^2) while K itself is driven towards N_f T / 2
    pos, q, box, v = _nh_system(orc)
    rc, T, tau = 3.0, 2.0, 0.05
    sog = orc.SOG(1.21812525709410644, 1.774456369233284 * rc / 10.0, 1.00090146156033341, 102)
    m = orc.kvectors_full(sog, box)
    w = orc.full_weights(sog, box, m)

    def force(xx, e):
        Fn, Un = orc.near_cells(xx, q, box, rc, sog)
        Ff, Us, _, _ = orc.far_kspace(xx, q, box, m, w)
        return Fn + Ff, Un + Us - orc.self_energy(sog, q)

    nf = 3 * len(q) - 3
    Q = nf * T * tau * tau

    def drift(dt, steps):
        _, _, _, _, hist = th.nose_hoover_run(orc, pos, v, q, box, rc, sog, 0, None, steps, dt, T, tau,
                                              force=force)
        H = [U + K + 0.5 * Q * xi * xi + nf * T * eta for U, K, xi, eta in hist]
        return max(abs(h - H[0]) for h in H), hist

    d1, h1 = drift(4e-3, 50)
    d2, _ = drift(2e-3, 100)
    assert d2 < 0.4 * d1
    # the thermostat acts: xi moved and K was pulled up from its start (T0 = 0.5 < T)
    assert max(abs(xi) for _, _, xi, _ in h1) > 1e-2
    assert max(K for _, K, _, _ in h1) > 1.2 * h1[0][1]


def test_nose_hoover_time_reversible(orc):
    pos, q, box, v = _nh_system(orc)
    rc, P, T, tau, steps = 3.0, 16, 1.5, 0.1, 10
    sog = orc.sog_row2(rc)
    kseq = orc.exact_mixture_sample(sog, box, P * (steps + 1), np.random.default_rng(4))
    x1, v1, xi1, _, _ = th.nose_hoover_run(orc, pos, v, q, box, rc, sog, P, kseq, steps, 1e-3, T, tau)
    back = np.concatenate([kseq[(steps - e) * P:(steps + 1 - e) * P] for e in range(steps + 1)])
    x2, v2, xi2, _, _ = th.nose_hoover_run(orc, x1, -v1, q, box, rc, sog, P, back, steps, 1e-3, T, tau, xi0=-xi1)
    d = x2 - pos
    d -= box * np.round(d / box)
    assert abs(xi1) > 1e-4
    assert np.abs(d).max() < 1e-9 and np.abs(v2 + v).max() < 1e-9 and abs(xi2) < 1e-12
