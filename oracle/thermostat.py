"""Langevin thermostat around the random-batch force (Algorithm 1 leaves the
thermostat open; Theorem 3's setting is Langevin dynamics) - test
infrastructure only.

One step is BAOAB: a half kick with the current force (B), a half drift (A),
the exact Ornstein-Uhlenbeck update v <- c1 v + c2 xi with c1 = e^{-gamma dt},
c2 = sqrt((1 - c1^2) T/m) (O), a half drift (A), the force at the new
positions, and a half kick (B).  xi are standard normals: for particle id i
at step s (s = 0 for the first thermostatted step of the context), Philox4x32-10
with key (seed_lo, seed_hi) and counter (i, s, 2, lane), lanes 0 and 1 each
giving two 53-bit uniforms (u1, u2), (u3, u4); xi = (r1 cos 2 pi u2,
r1 sin 2 pi u2, r2 cos 2 pi u4) with r = sqrt(-2 ln(1 - u)).
"""
from __future__ import annotations

import math

import numpy as np


def _uniform2(orc, seed: int, stream: int, index: int, lane: int):
    c = orc.philox4x32_10([index & 0xFFFFFFFF, (index >> 32) & 0xFFFFFFFF, stream, lane],
                          [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    w0 = (int(c[1]) << 32) | int(c[0])
    w1 = (int(c[3]) << 32) | int(c[2])
    return (w0 >> 11) * 2.0 ** -53, (w1 >> 11) * 2.0 ** -53


def normals(orc, n: int, step: int, seed: int) -> np.ndarray:
    xi = np.zeros((n, 3))
    for i in range(n):
        idx = (step << 32) | i
        u1, u2 = _uniform2(orc, seed, 2, idx, 0)
        u3, u4 = _uniform2(orc, seed, 2, idx, 1)
        r1 = math.sqrt(-2.0 * math.log(1.0 - u1))
        r2 = math.sqrt(-2.0 * math.log(1.0 - u3))
        xi[i] = (r1 * math.cos(2 * math.pi * u2), r1 * math.sin(2 * math.pi * u2), r2 * math.cos(2 * math.pi * u4))
    return xi


def baoab_run(orc, pos, vel, q, box, rc, sog, P: int, kseq, n_steps: int, dt: float, gamma: float, T: float,
              seed: int, mass: float = 1.0, step0: int = 0):
    """BAOAB steps; force evaluation e uses kseq[e*P:(e+1)*P] (evaluation 0 is the
    initial force).  Returns (pos, vel)."""
    box = np.asarray(box, dtype=np.float64)
    kseq = np.asarray(kseq, dtype=np.int32).reshape(-1, 3)
    S = orc.S_product(sog, box)
    x = np.array(pos, dtype=np.float64)
    x = x - box * np.floor(x / box)
    v = np.array(vel, dtype=np.float64)
    c1 = math.exp(-gamma * dt)
    c2 = math.sqrt((1.0 - c1 * c1) * T / mass)

    def force(e):
        m = kseq[e * P:(e + 1) * P]
        Fn, _ = orc.near_cells(x, q, box, rc, sog)
        Ff, _, _, _ = orc.far_rb(x, q, box, sog, m, P, S)
        return Fn + Ff

    F = force(0)
    for s in range(n_steps):
        v += 0.5 * dt * F / mass
        x += 0.5 * dt * v
        v = c1 * v + c2 * normals(orc, len(q), step0 + s, seed)
        x += 0.5 * dt * v
        x = x - box * np.floor(x / box)
        F = force(s + 1)
        v += 0.5 * dt * F / mass
    return x, v
