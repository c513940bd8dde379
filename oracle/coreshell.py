"""Core-shell near kernel of Sec. 3.4, written out in FP64 (test infrastructure
only, like the rest of ``oracle/``).

Pairs with r < r_in (the core) take the Gaussians' Taylor series to Q terms
with 1/r and 1/r^3 computed directly; pairs with r_in <= r < r_c (the shell)
take a table indexed by bits of the FP32 representation of r^2 (the low
B_exp bits of the exponent and the high B_man bits of the mantissa) with
linear interpolation between consecutive table points.

Readings (Sec. 3.4; Sec. 4 for the parameters):
  * the Taylor coefficients carry the alternating sign of the exponential's
    series, A_i = sum_l omega_l (-1)^(i-1) / ((i-1)! s_l^2) (1/s_l^2)^(i-1)
    (the printed A_i omits it); the force uses the factor of the corrected
    eq. "forcesplit": 1/r^3 - 2 sum_i A_i r^(2i-2);
  * the energy takes the same construction for sum_l omega_l e^{-r^2/s_l^2}
    (B_i = sum_l omega_l (-1)^(i-1)/(i-1)! (1/s_l^2)^(i-1)); the paper tabulates
    only what the force needs and is silent on the energy;
  * Q = 4, r_in = 0.2 r_c (0.2 nm at r_c = 1 nm), B_exp = 3, B_man = 9;
  * the table's binades start at the one holding r_in^2; a table point's value
    is the exact kernel at that point, linear interpolation in r^2 between a
    point and the next representable point of the table grid.
"""
from __future__ import annotations

import math

import numpy as np

Q_DEFAULT = 4
RIN_FRACTION = 0.2
BEXP = 3
BMAN = 9


def kernels_exact(x, sog):
    """g(x) = x^{-3/2} - 2 sum_l omega_l/s_l^2 e^{-x/s_l^2} (force coefficient) and
    h(x) = x^{-1/2} - sum_l omega_l e^{-x/s_l^2} (pair potential), x = r^2 (Sec. 3.1)."""
    x = np.asarray(x, dtype=np.float64)
    g = x ** -1.5
    h = x ** -0.5
    for w, s in zip(sog.omega, sog.s):
        e = np.exp(-x / (s * s))
        g = g - 2.0 * w / (s * s) * e
        h = h - w * e
    return g, h


def taylor_coefficients(sog, Q: int = Q_DEFAULT):
    """A_i (force, Gaussian part before the factor 2) and B_i (energy), i = 1..Q."""
    A = np.zeros(Q)
    B = np.zeros(Q)
    for w, s in zip(sog.omega, sog.s):
        a = 1.0 / (s * s)
        for i in range(1, Q + 1):
            c = (-1.0) ** (i - 1) / math.factorial(i - 1) * a ** (i - 1)
            A[i - 1] += w * a * c
            B[i - 1] += w * c
    return A, B


def core_kernels(x, A, B):
    x = np.asarray(x, dtype=np.float64)
    pa = np.zeros_like(x)
    pb = np.zeros_like(x)
    for i in range(len(A) - 1, -1, -1):
        pa = pa * x + A[i]
        pb = pb * x + B[i]
    return x ** -1.5 - 2.0 * pa, x ** -0.5 - pb


class Table:
    """Bitmask-indexed table of g and h over [r_in^2, r_c^2)."""

    def __init__(self, sog, rc: float, rin: float | None = None, bexp: int = BEXP, bman: int = BMAN):
        self.rc = float(rc)
        self.rin = float(RIN_FRACTION * rc if rin is None else rin)
        self.bexp, self.bman = bexp, bman
        self.shift = 23 - bman
        self.size = 1 << (bexp + bman)
        x0 = np.float32(self.rin * self.rin)
        self.e0 = int((np.array([x0], dtype=np.float32).view(np.uint32)[0] >> 23) & 0xFF)  # biased exponent
        nb = 1 << bexp
        top = np.float32(self.rc * self.rc)
        etop = int((np.array([top], dtype=np.float32).view(np.uint32)[0] >> 23) & 0xFF)
        if etop - self.e0 > nb - 2:
            raise ValueError("r_c^2 / r_in^2 spans more binades than the table holds")
        # node value for every index: the binade e in [e0, e0 + nb) with (e mod nb) = index >> bman
        g = np.zeros(self.size)
        h = np.zeros(self.size)
        for idx in range(self.size):
            blk, mant = idx >> bman, idx & ((1 << bman) - 1)
            e = self.e0 + ((blk - self.e0) % nb)
            bits = np.uint32((e << 23) | (mant << self.shift))
            x = float(np.array([bits], dtype=np.uint32).view(np.float32)[0])
            g[idx], h[idx] = kernels_exact(x, sog)
        self.g, self.h = g, h
        self.sog = sog

    def lookup(self, x):
        """Linear interpolation of g and h at x = r^2 (indexed by x rounded to FP32)."""
        xf = np.asarray(x, dtype=np.float64).astype(np.float32)
        bits = xf.view(np.uint32).astype(np.int64)
        node = bits >> self.shift
        idx = node & (self.size - 1)
        nxt = (node + 1) & (self.size - 1)
        frac = (bits & ((1 << self.shift) - 1)).astype(np.float64) / float(1 << self.shift)
        g = self.g[idx] + frac * (self.g[nxt] - self.g[idx])
        h = self.h[idx] + frac * (self.h[nxt] - self.h[idx])
        return g, h

    def interval_bound(self, x):
        """Linear-interpolation error bound on the interval holding x: spacing^2/8 times
        the largest |g''| and |h''| on it (both decrease with x here: taken at the left point)."""
        xf = np.asarray(x, dtype=np.float64).astype(np.float32)
        bits = xf.view(np.uint32).astype(np.int64)
        left = ((bits >> self.shift) << self.shift).astype(np.uint32).view(np.float32).astype(np.float64)
        e = (bits >> 23) & 0xFF
        spacing = np.ldexp(1.0, (e - 127 - self.bman).astype(np.int64))
        g2 = 3.75 * left ** -3.5
        h2 = 0.75 * left ** -2.5
        for w, s in zip(self.sog.omega, self.sog.s):
            ex = np.exp(-left / (s * s))
            g2 = g2 + 2.0 * w / s ** 6 * ex
            h2 = h2 + w / s ** 4 * ex
        return spacing ** 2 / 8.0 * g2, spacing ** 2 / 8.0 * h2


def pair_kernels(x, table: Table, A, B):
    """Core-shell g and h for squared distances x (all below r_c^2)."""
    x = np.asarray(x, dtype=np.float64)
    core = x < table.rin * table.rin
    g = np.empty_like(x)
    h = np.empty_like(x)
    if core.any():
        g[core], h[core] = core_kernels(x[core], A, B)
    if (~core).any():
        g[~core], h[~core] = table.lookup(x[~core])
    return g, h


def near_coreshell(pos, q, box, rc: float, sog, neighbors, Q: int = Q_DEFAULT):
    """Near forces and U_N with the core-shell kernel over a full neighbour list
    (row_ptr, cols) of the pair rule; the displacement is the FP64 minimum image."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    row, cols = neighbors
    n = len(q)
    i = np.repeat(np.arange(n), np.diff(row))
    j = np.asarray(cols, dtype=np.int64)
    d = pos[i] - pos[j]
    d -= box * np.rint(d / box)
    x = np.sum(d * d, axis=1)
    table = Table(sog, rc)
    A, B = taylor_coefficients(sog, Q)
    g, h = pair_kernels(x, table, A, B)
    qq = q[i] * q[j]
    F = np.zeros((n, 3))
    np.add.at(F, i, (qq * g)[:, None] * d)
    U = 0.5 * float(np.sum(qq * h))
    return F, U
