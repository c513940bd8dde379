"""Pins of the oracle's near part (Sec. 3.1): pair rule, cell list, forces
against finite differences of U_N, Newton's third law, invariances.  CPU only."""
import numpy as np
import pytest

from paper_2205_13824_amd import workloads as W


def random_system(n, box, seed):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * np.asarray(box)
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    return pos, q


@pytest.mark.parametrize("box,rc", [((10.0, 10.0, 10.0), 3.0), ((12.0, 9.0, 15.0), 2.9),
                                    ((5.0, 5.0, 5.0), 2.4)])
def test_neighbour_list_matches_plain_distances(orc, box, rc):
    # The fixed-point rule includes exactly the pairs with minimum-image
    # distance < r_c, up to the 2^-32 quantisation band.
    box = np.array(box)
    pos, _ = random_system(300, box, 7)
    row, cols = orc.neighbors_brute(pos, box, rc)
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.round(d / box)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, np.inf)
    band = 1e-6
    inside = r < rc - band
    outside = r > rc + band
    listed = np.zeros_like(inside)
    for i in range(pos.shape[0]):
        listed[i, cols[row[i]:row[i + 1]]] = True
    assert not (inside & ~listed).any()
    assert not (outside & listed).any()
    # symmetric, sorted rows, no self pairs
    assert (listed == listed.T).all()
    for i in range(pos.shape[0]):
        c = cols[row[i]:row[i + 1]]
        assert (np.diff(c) > 0).all() and i not in c


@pytest.mark.parametrize("box,rc", [((10.0, 10.0, 10.0), 3.0), ((12.0, 9.0, 15.0), 2.9),
                                    ((5.0, 5.0, 5.0), 2.4)])
def test_cell_list_definition(orc, box, rc):
    box = np.array(box)
    pos, _ = random_system(500, box, 8)
    nc, cell_of, start, order = orc.cell_list(pos, box, rc)
    for d in range(3):
        k = int(np.floor(box[d] / rc))
        assert nc[d] == (k if k >= 3 else 1)
    # each particle lies inside the spatial extent of its cell
    frac = pos / box - np.floor(pos / box)
    c = np.stack([cell_of % nc[0], (cell_of // nc[0]) % nc[1], cell_of // (nc[0] * nc[1])], 1)
    lo, hi = c / nc, (c + 1) / nc
    assert ((frac >= lo - 1e-9) & (frac < hi + 1e-9)).all()
    # order is sorted by (cell, id) and start is the exclusive prefix of counts
    assert start[0] == 0 and start[-1] == pos.shape[0]
    key = cell_of[order].astype(np.int64) * pos.shape[0] + order
    assert (np.diff(key) > 0).all()
    assert (np.diff(start) == np.bincount(cell_of, minlength=len(start) - 1)).all()


@pytest.mark.parametrize("box,rc", [((10.0, 10.0, 10.0), 3.0), ((12.0, 9.0, 15.0), 2.9),
                                    ((5.0, 5.0, 5.0), 2.4)])
def test_near_cells_equals_brute_force(orc, box, rc):
    box = np.array(box)
    pos, q = random_system(400, box, 9)
    sog = orc.sog_row2(rc)
    Fb, Ub = orc.near_brute(pos, q, box, rc, sog)
    Fc, Uc = orc.near_cells(pos, q, box, rc, sog)
    assert np.abs(Fb - Fc).max() <= 1e-12 * np.abs(Fb).max()
    assert abs(Ub - Uc) <= 1e-12 * abs(Ub)
    Ft = orc.near_targets(pos, q, box, rc, sog, np.arange(0, 400, 7))
    assert np.abs(Ft - Fb[::7]).max() <= 1e-12 * np.abs(Fb).max()


def test_near_newton_third_law(orc):
    box = np.array([10.0, 10.0, 10.0])
    pos, q = random_system(300, box, 10)
    F, _ = orc.near_brute(pos, q, box, 3.0, orc.sog_row2(3.0))
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).max()


def test_near_force_is_minus_gradient_of_energy(orc):
    # Pins the corrected factor of eq. "forcesplit" (the printed one is half).
    box = np.array([10.0, 10.0, 10.0])
    pos, q = random_system(40, box, 11)
    rc = 3.0
    sog = orc.sog_row2(rc)
    F, _ = orc.near_brute(pos, q, box, rc, sog)
    h = 1e-6
    for i in (0, 5, 17):
        for d in range(3):
            p = pos.copy(); p[i, d] += h
            up = orc.near_brute(p, q, box, rc, sog)[1]
            p = pos.copy(); p[i, d] -= h
            um = orc.near_brute(p, q, box, rc, sog)[1]
            assert abs(-(up - um) / (2 * h) - F[i, d]) < 1e-6 * max(1.0, abs(F[i, d]))


def test_near_pair_potential_vanishes_smoothly_at_cutoff(orc):
    # N(r) = 1/r - F(r) is continuous in value (to the l > M tail) and slope at r_c.
    rc = 3.5
    sog = orc.sog_row2(rc)
    assert abs(1.0 / rc - sog.F(rc)) < 1e-3 / rc
    h = 1e-5
    dN = (-(1.0 / (rc + h) - sog.F(rc + h)) + (1.0 / (rc - h) - sog.F(rc - h))) / (2 * h)
    assert abs(dN) < 1e-9


def test_near_translation_invariance(orc):
    box = np.array([10.0, 10.0, 10.0])
    pos, q = random_system(200, box, 12)
    sog = orc.sog_row2(3.0)
    F0, U0 = orc.near_cells(pos, q, box, 3.0, sog)
    F1, U1 = orc.near_cells(pos + np.array([3.3, -7.1, 12.9]), q, box, 3.0, sog)
    assert np.abs(F0 - F1).max() < 1e-9 * np.abs(F0).max()
    assert abs(U0 - U1) < 1e-9 * abs(U0)


def test_config_c1_neighbour_count(orc):
    # 1000 ions in L = 10 with r_c = 3: about 4/3 pi r_c^3 n/V = 113 neighbours.
    c = W.c1_small()
    row, _ = orc.neighbors_brute(c["pos"], c["box"], c["rc"])
    mean = row[-1] / 1000.0
    assert 105 < mean < 121
