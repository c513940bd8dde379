"""Thermostats around the random-batch force (Algorithm 1 leaves the
thermostat open; Theorem 3's setting is Langevin dynamics, and Sec. 5's
water runs use a Nose-Hoover thermostat) - test infrastructure only.

Langevin:

One step is BAOAB: a half kick with the current force (B), a half drift (A),
the exact Ornstein-Uhlenbeck update v <- c1 v + c2 xi with c1 = e^{-gamma dt},
c2 = sqrt((1 - c1^2) T/m) (O), a half drift (A), the force at the new
positions, and a half kick (B).  xi are standard normals: for particle id i
at step s (s = 0 for the first thermostatted step of the context), Philox4x32-10
with key (seed_lo, seed_hi) and counter (i, s, 2, lane), lanes 0 and 1 each
giving two 53-bit uniforms (u1, u2), (u3, u4); xi = (r1 cos 2 pi u2,
r1 sin 2 pi u2, r2 cos 2 pi u4) with r = sqrt(-2 ln(1 - u)).

Nose-Hoover: see ``nose_hoover_run``; its pins are the tau = inf limit
(velocity Verlet), conservation of the extended energy
U + K + Q xi^2 / 2 + N_f T eta at O(dt^2) with deterministic forces, and
time reversibility.
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


def nose_hoover_run(orc, pos, vel, q, box, rc, sog, P: int, kseq, n_steps: int, dt: float, T: float, tau: float,
                    mass: float = 1.0, xi0: float = 0.0, eta0: float = 0.0, force=None):
    """Nose-Hoover dynamics (one thermostat variable xi per system, thermostat
    mass Q = N_f T tau^2 with N_f = 3n - 3 degrees of freedom, xi's time
    integral eta) in the symmetric splitting: xi moves half a step with the
    kinetic energy K at the step's start, velocities are scaled by
    exp(-xi dt/2), velocity-Verlet kick, drift, force, kick, scaled again by
    exp(-xi dt/2), and xi moves the second half step with the new K.
    tau = inf gives velocity Verlet.  Force evaluation e uses kseq[e*P:(e+1)*P]
    (evaluation 0 is the initial force) unless `force(x, e)` is given (it
    returns (F, U)).  Returns (pos, vel, xi, eta, list of (U, K, xi, eta) after
    each step, with the initial state first)."""
    box = np.asarray(box, dtype=np.float64)
    x = np.array(pos, dtype=np.float64)
    x = x - box * np.floor(x / box)
    v = np.array(vel, dtype=np.float64)
    n = len(q)
    nf = 3 * n - 3
    Q = nf * T * tau * tau
    if force is None:
        kseq = np.asarray(kseq, dtype=np.int32).reshape(-1, 3)
        S = orc.S_product(sog, box)

        def force(xx, e):
            m = kseq[e * P:(e + 1) * P]
            Fn, Un = orc.near_cells(xx, q, box, rc, sog)
            Ff, Us, _, _ = orc.far_rb(xx, q, box, sog, m, P, S)
            return Fn + Ff, Un + Us - orc.self_energy(sog, q)

    def kinetic(vv):
        return 0.5 * mass * float((vv * vv).sum())

    F, U = force(x, 0)
    xi, eta = float(xi0), float(eta0)
    K = kinetic(v)
    hist = [(U, K, xi, eta)]
    for s in range(n_steps):
        xi += 0.5 * dt * (2.0 * K - nf * T) / Q
        eta += 0.5 * dt * xi
        v *= math.exp(-0.5 * dt * xi)
        v += 0.5 * dt * F / mass
        x += dt * v
        x = x - box * np.floor(x / box)
        F, U = force(x, s + 1)
        v += 0.5 * dt * F / mass
        v *= math.exp(-0.5 * dt * xi)
        eta += 0.5 * dt * xi
        K = kinetic(v)
        xi += 0.5 * dt * (2.0 * K - nf * T) / Q
        hist.append((U, K, xi, eta))
    return x, v, xi, eta, hist
