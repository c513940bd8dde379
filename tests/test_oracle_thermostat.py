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
