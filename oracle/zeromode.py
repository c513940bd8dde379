"""Zero-frequency mode terms of Sec. 3.2 (test infrastructure only).

With tinfoil boundary conditions the k = 0 term vanishes.  For a periodic
system in a medium of unit permittivity summed in spherical order the term is
U^0 = (2 pi / 3V) |M|^2 (eq. "sperical"); for a slab geometry (planar
boundary along z) it is U^0 = (2 pi / V) M_z^2 (eq. "planar"); M = sum_i q_i r_i
over the positions as wrapped into the box (the paper is silent on the image
choice).  The forces are -grad U^0: -(4 pi / 3V) q_i M and -(4 pi / V) q_i M_z e_z.
"""
from __future__ import annotations

import math

import numpy as np

TINFOIL, SPHERICAL, SLAB = 0, 1, 2


def zero_mode(pos, q, box, mode: int):
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    xw = pos - box * np.floor(pos / box)
    M = (q[:, None] * xw).sum(0)
    F = np.zeros_like(pos)
    if mode == SPHERICAL:
        U = 2.0 * math.pi / (3.0 * V) * float(M @ M)
        F = -(4.0 * math.pi / (3.0 * V)) * q[:, None] * M[None, :]
    elif mode == SLAB:
        U = 2.0 * math.pi / V * float(M[2] ** 2)
        F[:, 2] = -(4.0 * math.pi / V) * q * M[2]
    else:
        U = 0.0
    return F, U, M


def image_sum(pos, q, box, cells):
    """Coulomb energy 1/2 sum_n sum_{i,j}' q_i q_j / |r_i - r_j + n L| over the image
    cells n given (the self term n = 0, i = j excluded)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    shift = np.asarray(cells, dtype=np.float64) * box
    E = 0.0
    for i in range(len(q)):
        for j in range(len(q)):
            d = pos[i] - pos[j] + shift
            r = np.sqrt(np.sum(d * d, axis=1))
            if i == j:
                r = r[r > 0]
            E += 0.5 * q[i] * q[j] * float(np.sum(1.0 / r))
    return E


def sphere_cells(R: int):
    g = np.arange(-R, R + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return n[(n * n).sum(1) <= R * R]


def plate_cells(R: int, H: int):
    g = np.arange(-R, R + 1)
    n = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    n = n[(n * n).sum(1) <= R * R]
    return np.concatenate([np.concatenate([n, np.full((len(n), 1), z)], 1) for z in range(-H, H + 1)])
