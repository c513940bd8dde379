"""Seeded synthetic systems shaped like the workloads the RBSOG paper runs.

This module holds no arithmetic of the method: it only places charges in a
periodic box (and draws initial velocities) from a seeded numpy generator, so
that the GPU library and the CPU oracle can be fed identical inputs.

Systems:
  * ``ions_uniform``   N ions, half +1 then half -1, uniform positions;
  * ``ions_rsa``       neutral +-1 electrolyte by random sequential addition
                       with a minimum separation (no overlapping ions);
  * ``water``          rigid 3-site water-shaped molecules (O at -0.8476, two
                       H at +0.4238, O-H 1 Angstrom, H-O-H 109.47 degrees) on a
                       jittered simple-cubic lattice with random orientations;
  * ``nacl_lattice``   rock-salt crystal (alternating +-1 on a cubic lattice);
  * ``ensemble_sizes`` log-uniform replica sizes for batched ensembles;
  * ``maxwellian``     velocities N(0, T/m) with the centre-of-mass drift removed.
"""
from __future__ import annotations

import math

import numpy as np


def ions_uniform(n: int, L: float, seed: int):
    """n ions in a cube of side L: ids [0, n/2) carry +1, the rest -1; x ~ U[0, L)^3."""
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * L
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return np.ascontiguousarray(pos), np.ascontiguousarray(q), np.array([L, L, L], dtype=np.float64)


def _rsa_accept(cand: np.ndarray, L: float, dmin: float) -> np.ndarray:
    """Random sequential addition in candidate order: candidate i is kept iff no
    earlier kept candidate lies within dmin (periodic minimum image)."""
    from scipy.spatial import cKDTree

    tree = cKDTree(cand, boxsize=L)
    pairs = tree.query_pairs(r=dmin, output_type="ndarray")
    n = cand.shape[0]
    if pairs.size == 0:
        return np.ones(n, dtype=bool)
    lo = np.minimum(pairs[:, 0], pairs[:, 1])
    hi = np.maximum(pairs[:, 0], pairs[:, 1])
    # state: 1 kept, 0 undecided, -1 dropped
    state = np.zeros(n, dtype=np.int8)
    has_lower = np.zeros(n, dtype=bool)
    has_lower[hi] = True
    state[~has_lower] = 1
    while True:
        und = state == 0
        if not und.any():
            break
        # dropped if an earlier neighbour is kept
        kill = np.zeros(n, dtype=bool)
        kill[hi[state[lo] == 1]] = True
        state[und & kill] = -1
        # kept if every earlier neighbour is dropped
        pending = np.zeros(n, dtype=bool)
        pending[hi[state[lo] != -1]] = True
        newly = (state == 0) & ~pending
        if not newly.any() and not (und & kill).any():
            raise RuntimeError("RSA resolution did not progress")
        state[newly] = 1
    return state == 1


def ions_rsa(n: int, density: float, dmin: float, seed: int):
    """Neutral +-1 electrolyte of n ions (n even) at the given number density in a
    cube, placed by random sequential addition with minimum separation dmin; the
    charges are shuffled over the particle ids."""
    if n % 2:
        raise ValueError("n must be even for a neutral +-1 system")
    L = (n / density) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    kept = np.zeros((0, 3))
    factor = 1.4
    while kept.shape[0] < n:
        cand = rng.random((int(n * factor) + 16, 3)) * L
        cand = np.concatenate([kept, cand])
        ok = _rsa_accept(cand, L, dmin)
        kept = cand[ok]
        factor *= 1.5
    pos = np.ascontiguousarray(kept[:n])
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    rng.shuffle(q)
    return pos, np.ascontiguousarray(q), np.array([L, L, L], dtype=np.float64)


def ions_lattice(n_side: int, density: float, seed: int, jitter: float = 0.25):
    """Neutral +-1 electrolyte of n_side^3 ions (even) at the given number density:
    a simple-cubic lattice of spacing a jittered by U(-jitter a, +jitter a) per
    axis, so that no two ions are closer than (1 - 2 jitter) a; charges shuffled.
    Used where random sequential addition of tens of millions of ions would
    dominate the set-up time."""
    n = n_side ** 3
    if n % 2:
        raise ValueError("n_side^3 must be even for a neutral +-1 system")
    L = (n / density) ** (1.0 / 3.0)
    a = L / n_side
    rng = np.random.default_rng(seed)
    g = (np.arange(n_side, dtype=np.float64) + 0.5) * a
    gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    pos += rng.uniform(-jitter * a, jitter * a, size=pos.shape)
    pos -= L * np.floor(pos / L)
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    rng.shuffle(q)
    return np.ascontiguousarray(pos), np.ascontiguousarray(q), np.array([L, L, L], dtype=np.float64)


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotation matrices from normalised Gaussian quaternions."""
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


WATER_Q = (-0.8476, 0.4238, 0.4238)


def water(n_side: int, density: float, seed: int, bond: float = 1.0, angle_deg: float = 109.47,
          jitter: float = 0.15):
    """n_side^3 rigid 3-site molecules at `density` molecules per unit volume, on a
    simple-cubic lattice of spacing a = L/n_side, the oxygen jittered by
    U(-jitter a, +jitter a) per axis and each molecule rotated uniformly at
    random.  Sites are ordered O, H, H per molecule; positions are wrapped."""
    nmol = n_side ** 3
    L = (nmol / density) ** (1.0 / 3.0)
    a = L / n_side
    rng = np.random.default_rng(seed)
    g = (np.arange(n_side) + 0.5) * a
    gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
    O = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    O = O + rng.uniform(-jitter * a, jitter * a, size=O.shape)
    half = math.radians(angle_deg) / 2.0
    ref = np.array([[0.0, 0.0, 0.0],
                    [bond * math.sin(half), bond * math.cos(half), 0.0],
                    [-bond * math.sin(half), bond * math.cos(half), 0.0]])
    R = _random_rotations(rng, nmol)
    sites = O[:, None, :] + np.einsum("nij,sj->nsi", R, ref)
    pos = sites.reshape(-1, 3)
    pos = pos - L * np.floor(pos / L)
    q = np.tile(np.array(WATER_Q), nmol)
    return np.ascontiguousarray(pos), np.ascontiguousarray(q), np.array([L, L, L], dtype=np.float64)


def nacl_lattice(n_side: int, a: float = 1.0):
    """Rock-salt crystal: n_side^3 sites (n_side even) of spacing a with charge
    (-1)^(i+j+k); box side n_side * a."""
    if n_side % 2:
        raise ValueError("n_side must be even for a periodic rock-salt crystal")
    idx = np.arange(n_side)
    gx, gy, gz = np.meshgrid(idx, idx, idx, indexing="ij")
    pos = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1).astype(np.float64) * a
    q = np.where((gx + gy + gz).ravel() % 2 == 0, 1.0, -1.0)
    L = n_side * a
    return np.ascontiguousarray(pos), np.ascontiguousarray(q), np.array([L, L, L], dtype=np.float64)


def ensemble_sizes(n_sys: int, nmin: int, nmax: int, seed: int) -> np.ndarray:
    """Even replica sizes 2 round(exp(U(ln nmin, ln nmax))/2)."""
    rng = np.random.default_rng(seed)
    x = np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=n_sys))
    return (2 * np.round(x / 2)).astype(np.int64)


def maxwellian(n: int, T: float, seed: int, mass: float = 1.0) -> np.ndarray:
    """Velocities N(0, T/m) per component with the centre-of-mass velocity removed."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3)) * math.sqrt(T / mass)
    v -= v.mean(axis=0, keepdims=True)
    return np.ascontiguousarray(v)


# Named workloads with the sizes the paper's experiments and the benchmark use.
def c1_small():
    """1,000 ions in L = 10 (uniform positions), r_c = 3.0, P = 100."""
    pos, q, box = ions_uniform(1000, 10.0, seed=1)
    return dict(pos=pos, q=q, box=box, rc=3.0, P=100)


def c2_electrolyte(n: int = 300_000):
    """300,000-ion +-1 electrolyte at density 0.1 (RSA, d_min = 1), r_c = 3.5, P = 200."""
    pos, q, box = ions_rsa(n, 0.1, 1.0, seed=2)
    return dict(pos=pos, q=q, box=box, rc=3.5, P=200)


def c3_water(n_side: int = 100):
    """n_side^3 water-shaped molecules at 0.0334 / A^3, r_c = 10 A, P = 500."""
    pos, q, box = water(n_side, 0.0334, seed=3)
    return dict(pos=pos, q=q, box=box, rc=10.0, P=500)


def c4_ensemble(n_sys: int = 256, nmin: int = 500, nmax: int = 50_000, seed: int = 4):
    """Replica ensemble: n_sys +-1 electrolytes at density 0.1 (RSA, d_min = 1)
    with log-uniform sizes in [nmin, nmax], r_c = 3.5, P = 100, seeds 1000 + r."""
    sizes = ensemble_sizes(n_sys, nmin, nmax, seed)
    systems = []
    for r, n in enumerate(sizes):
        pos, q, box = ions_rsa(int(n), 0.1, 1.0, seed=1000 + r)
        systems.append(dict(pos=pos, q=q, box=box))
    return dict(systems=systems, rc=3.5, P=100, seeds=[1000 + r for r in range(n_sys)])


def c5_large(n_side: int = 272):
    """About 2e7 ions (272^3 = 20,123,648) at density 0.1 on a jittered lattice
    (minimum separation 0.5 a = 1.08), r_c = 3.5, P = 1000."""
    pos, q, box = ions_lattice(n_side, 0.1, seed=5)
    return dict(pos=pos, q=q, box=box, rc=3.5, P=1000)
