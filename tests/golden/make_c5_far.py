"""Writes the stored expected far forces of the 2e7-ion system, calling only
the oracle (and the seeded input generator, which holds no arithmetic of the
method):

  c5_far_subset.txt  the far force on 1000 ions (ids drawn with seed 55) of
                     the 272^3-ion jittered lattice (seed 5, density 0.1,
                     r_c = 3.5, Table 1 row 2 scaled to r_c):
                       full  every k != 0 (Sec. 3.3: each Gaussian through the
                             Poisson identity, the 9 narrowest as real-space
                             image sums, the 8 widest as Fourier series;
                             oracle.far_split)
                       rb    the random-batch estimate (Sec. 3.3, eq.
                             "approximateForce") on the first batch of
                             P = 1000 wave vectors of the Metropolis-Hastings
                             chain keyed 55 (oracle.mh_sample), with the
                             structure factors over all ions
  c5_rb_batch.txt    that batch: m and rho(k) of each wave vector, and U*.

Run from the repository root: python tests/golden/make_c5_far.py
(about ten minutes on eight cores).
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2205_13824_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SUBSET_SEED = 55
CHAIN_SEED = 55
N_REAL = 9


def main():
    t0 = time.time()
    c = W.c5_large()
    pos, q, box, rc, P = c["pos"], c["q"], c["box"], c["rc"], c["P"]
    n = len(q)
    sog = oracle.sog_row2(rc)
    ids = np.sort(np.random.default_rng(SUBSET_SEED).choice(n, size=1000, replace=False))
    print(f"system of {n} ions built in {time.time() - t0:.1f} s", flush=True)

    t0 = time.time()
    m = oracle.mh_sample(sog, box, seed=CHAIN_SEED, stream=0, n=P)[0]
    S = oracle.S_product(sog, box)
    F_rb, U_rb, re, im = oracle.far_rb(pos, q, box, sog, m, P, S=S, targets=ids)
    print(f"random-batch far force: {time.time() - t0:.1f} s", flush=True)

    t0 = time.time()
    F_full = oracle.far_split(pos, q, box, sog, ids, N_REAL)
    print(f"full far force (Poisson split, {N_REAL} real-space Gaussians): {time.time() - t0:.1f} s", flush=True)

    with open(os.path.join(HERE, "c5_far_subset.txt"), "w") as f:
        f.write("# Far force on 1000 ions of the 272^3-ion jittered lattice (workloads.c5_large: seed 5,\n"
                "# density 0.1, r_c = 3.5, Table 1 row 2 scaled to r_c; ids: numpy default_rng(55)\n"
                "# .choice(n, 1000, replace=False), sorted), written by tests/golden/make_c5_far.py,\n"
                "# which calls only the oracle:\n"
                f"#   full  every k != 0 (Sec. 3.3, Poisson identity per Gaussian, the {N_REAL} narrowest\n"
                "#         in real space out to sqrt(37) s_l, the rest as Fourier series; oracle.far_split)\n"
                "#   rb    random-batch estimate (Sec. 3.3, eq. \"approximateForce\") on the first batch of\n"
                "#         P = 1000 vectors of the Metropolis-Hastings chain keyed 55 (c5_rb_batch.txt)\n"
                "# columns: id Fx_full Fy_full Fz_full Fx_rb Fy_rb Fz_rb\n")
        for i, ff, fr in zip(ids, F_full, F_rb):
            f.write(f"{int(i)} {ff[0]:.17e} {ff[1]:.17e} {ff[2]:.17e} {fr[0]:.17e} {fr[1]:.17e} {fr[2]:.17e}\n")
    with open(os.path.join(HERE, "c5_rb_batch.txt"), "w") as f:
        f.write("# The first batch of P = 1000 wave vectors of the Metropolis-Hastings chain (Sec. 3.3)\n"
                "# keyed 55, stream 0, 100 transitions discarded, for the system of c5_far_subset.txt,\n"
                "# and the structure factor rho(k) = sum_j q_j e^{i k.r_j} of every vector over all ions;\n"
                "# written by tests/golden/make_c5_far.py (oracle only).\n"
                f"# S = {S:.17e}\n"
                f"# Ustar = {U_rb:.17e}\n"
                "# columns: m_x m_y m_z rho_re rho_im\n")
        for mm, a, b in zip(m, re, im):
            f.write(f"{int(mm[0])} {int(mm[1])} {int(mm[2])} {a:.17e} {b:.17e}\n")
    rms = math.sqrt(float(np.mean(np.sum((F_rb - F_full) ** 2, axis=1))))
    print(f"written; rms |F_rb - F_full| = {rms:.3e}, rms |F_full| = "
          f"{math.sqrt(float(np.mean(np.sum(F_full ** 2, axis=1)))):.3e}", flush=True)


if __name__ == "__main__":
    main()
