"""The pairs the near kernels actually evaluate, recorded by the kernels
themselves (rbsog_debug_record_pairs: the list build, the list pass and the
fused cell kernel append every pair that passes the pair rule), against the
oracle's brute-force neighbour list, bit for bit (Sec. 3.1, the neighbour set
I(i) of eq. "SOGDEcomp", strict r < r_c; the fixed-point rule of rbsog.h).

Hand-placed pairs put the decision at its edges.  In a cube of side 16 the
fixed-point step is h = 2^-28, so a displacement of integer steps (d_x, d_y,
d_z), each below 2^26, has r^2 = (d_x^2 + d_y^2 + d_z^2) 2^-56 exactly in
FP64, and r_c^2 = 0.09 (r_c = 0.3) is itself a multiple of 2^-56 (its unit in
the last place): a pair with d^2 = r_c^2 2^56 + k sits k ulps from the cutoff.
Such pairs are built for k = -8..8 (sums of three squares through a prime
p = 1 mod 4 written as a sum of two squares), at the FP32 band edges of the
kernels' fast test, at the list radius r_c (1 + skin) and at its widened FP32
edge, across the periodic seam, and in a box with one cell along an axis.
"""
import math

import numpy as np
import pytest

from paper_2205_13824_amd import rbsog as R

pytestmark = pytest.mark.gpu

L16 = 16.0
H = 2.0 ** -28          # fixed-point step of a side-16 box
RC = 0.3
RC2_UNITS = int(round(RC * RC * 2.0 ** 56))  # r_c^2 in units of 2^-56 (exact)
assert RC2_UNITS * 2.0 ** -56 == RC * RC


def is_prime(n):
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def two_squares_prime(p):
    """x^2 + y^2 = p for a prime p = 1 mod 4 (Hermite-Serret: Euclid on p and
    a square root of -1 mod p, stopped below sqrt(p))."""
    for a in range(2, 200):
        t = pow(a, (p - 1) // 4, p)
        if t * t % p == p - 1:
            break
    else:
        raise ValueError("no square root of -1 found")
    lim = math.isqrt(p)
    x, y = p, t
    while y > lim:
        x, y = y, x % y
    b = math.isqrt(p - y * y)
    assert y * y + b * b == p
    return y, b


def representable(T):
    """Legendre: T is a sum of three squares unless T = 4^a (8b + 7)."""
    while T % 4 == 0 and T > 0:
        T //= 4
    return T % 8 != 7


def three_squares(T, rng):
    """An integer vector with |d|^2 = T, components below 2^26 and random signs
    and order: factors of 4 taken out (they scale every component by 2), then
    z drawn until T - z^2 is a prime p = 1 mod 4 or twice one (2p = (a+b)^2 +
    (a-b)^2 when p = a^2 + b^2)."""
    s = 1
    while T % 4 == 0:
        T //= 4
        s *= 2
    top = math.isqrt(T)
    for _ in range(200000):
        z = int(rng.integers(int(0.45 * top), int(0.65 * top)))
        m = T - z * z
        if m % 4 == 1 and is_prime(m):
            x, y = two_squares_prime(m)
        elif m % 2 == 0 and (m // 2) % 4 == 1 and is_prime(m // 2):
            a, b = two_squares_prime(m // 2)
            x, y = a + b, abs(a - b)
        else:
            continue
        d = s * np.array([x, y, z], dtype=np.int64)
        if np.abs(d).max() >= 2 ** 26:
            continue
        d = d[rng.permutation(3)] * rng.choice([-1, 1], size=3)
        assert int((d * d).sum()) == T * s * s
        return d
    raise ValueError(f"no decomposition of {T}")


def place_pairs(targets, rng, seam=False, avoid=()):
    """One pair per target |d|^2 (in units of 2^-56) in the side-16 cube,
    anchored at distinct sites of a grid of spacing 1 (pairs far apart);
    positions are exact fixed-point values x = (u + 1/2) h.  With `seam` the
    anchor sits within 2^-8 of the x = 0 face and the partner wraps to the
    x = 16 face.  Returns positions (n x 3), charges, the sites used."""
    sites = [(i, j, k) for i in range(16) for j in range(16) for k in range(16)
             if (i, j, k) not in avoid and (not seam or i == 0)]
    order = rng.permutation(len(sites))
    pos, q, used = [], [], []
    for t, si in zip(targets, order):
        site = sites[si]
        d = three_squares(t, rng)
        ua = np.array([int((site[a] + 0.35) / H) for a in range(3)], dtype=np.int64)
        if seam:
            ua[0] = int(rng.integers(0, 2 ** 20))
            d[0] = -abs(d[0])
        ub = (ua + d) % 2 ** 32
        for u in (ua, ub):
            pos.append((u.astype(np.float64) + 0.5) * H)
        q += [1.0, -1.0]
        used.append(site)
    return np.array(pos), np.array(q), used


def offsets_near(center, ks):
    """The representable |d|^2 among center + k."""
    return [center + k for k in ks if representable(center + k)]


def band_units(rc, skin, box):
    """Thresholds of the kernels' FP32 fast test and list, in units of 2^-56
    (the library's constants for a cube of side 16)."""
    hmax = max(box) / 2.0 ** 32
    d32 = 32.0 * hmax / rc + 1e-12 + 3e-5
    rc2 = rc * rc
    lo = float(np.float32(rc2 * (1.0 - d32)))
    hi = float(np.float32(rc2 * (1.0 + d32)))
    rl = rc * (1.0 + skin)
    rl2f = float(np.float32(rl * rl * (1.0 + 1e-4) + 1e-30))
    u = 2.0 ** 56
    return int(lo * u), int(hi * u), int(rl * rl * u), int(rl2f * u)


def edge_system(seed, skin):
    rng = np.random.default_rng(seed)
    lo, hi, rl2, rl2f = band_units(RC, skin if skin > 0 else 0.0, (L16,) * 3)
    ks = list(range(-8, 9))
    targets = offsets_near(RC2_UNITS, ks) * 3                    # r_c^2 + k ulps, three orientations each
    targets += offsets_near(lo, (-3, -1, 0, 1, 3)) + offsets_near(hi, (-3, -1, 0, 1, 3))  # FP32 band edges
    if skin > 0:
        targets += offsets_near(rl2, (-4, -1, 0, 1, 4)) + offsets_near(rl2f, (-2000, -4, 0, 4, 2000))
    pos, q, used = place_pairs(targets, rng)
    # and pairs across the periodic seam
    pos2, q2, _ = place_pairs(offsets_near(RC2_UNITS, (-3, -1, 0, 1)) * 2, rng, seam=True, avoid=set(used))
    return np.concatenate([pos, pos2]), np.concatenate([q, q2]), np.array([L16] * 3)


def recorded_pairs(sysm):
    row, cols, kinds = R.rbsog_debug_pairs(sysm.ctx)
    return row, cols, kinds


def assert_same_csr(row, cols, row_o, cols_o, what):
    assert row.shape == row_o.shape, what
    bad = np.nonzero(row != row_o)[0]
    assert bad.size == 0 and np.array_equal(cols, cols_o), f"{what}: rows differ at {bad[:10]}"


CASES = [(R.RBSOG_FP64, False), (R.RBSOG_FP32C, False), (R.RBSOG_FP32C, True)]


@pytest.mark.parametrize("prec,table", CASES)
@pytest.mark.parametrize("skin", [0.1, 0.0])
def test_kernel_pairs_at_the_cutoff_edges_bit_exact(orc, prec, table, skin):
    pos, q, box = edge_system(11, skin)
    sysm = R.System(pos, q, box, RC, 4, seed=3, precision=prec, near_table=table, skin=skin)
    R.rbsog_debug_record_pairs(sysm.ctx, 1 << 16)
    sysm.sample_k(2)
    sysm.forces()
    row, cols, kinds = recorded_pairs(sysm)
    row_o, cols_o = orc.neighbors_brute(pos, box, RC)
    # the constructed ulp pairs: exactly those below r_c^2 are neighbours
    npairs = int(row_o[-1]) // 2
    print(f"prec={prec} table={table} skin={skin}: {npairs} neighbour pairs of {len(q) // 2} placed, "
          f"kernels {kinds}", flush=True)
    assert kinds == (2 if skin > 0 else 4)
    assert_same_csr(row, cols, row_o, cols_o, "first evaluation")
    if skin > 0:
        # the same positions again: the list pass evaluates the stored list
        # without a build
        nb = R.rbsog_info(sysm.ctx)["list_builds"]
        sysm.forces()
        assert R.rbsog_info(sysm.ctx)["list_builds"] == nb
        row2, cols2, kinds2 = recorded_pairs(sysm)
        assert kinds2 == 2
        assert_same_csr(row2, cols2, row_o, cols_o, "list pass")
        # the list holds every pair within r_c (1 + skin) and none beyond its widened edge
        lrow, lcols = R.rbsog_debug_list(sysm.ctx)
        rl = RC * (1.0 + skin)
        in_row, in_cols = orc.neighbors_brute(pos, box, rl)
        out_row, out_cols = orc.neighbors_brute(pos, box, rl * (1.0 + 1e-3))
        listed = {(i, j) for i in range(len(q)) for j in lcols[lrow[i]:lrow[i + 1]]}
        need = {(i, j) for i in range(len(q)) for j in in_cols[in_row[i]:in_row[i + 1]]}
        allow = {(i, j) for i in range(len(q)) for j in out_cols[out_row[i]:out_row[i + 1]]}
        # the list stores each pair once per home: both orders
        assert need <= listed <= allow
    sysm.close()


@pytest.mark.parametrize("prec", [R.RBSOG_FP64, R.RBSOG_FP32C])
@pytest.mark.parametrize("skin", [0.1, 0.0])
def test_kernel_pairs_in_single_cell_dimensions(orc, prec, skin):
    # floor(L_z / (r_c (1 + skin))) < 3: one cell along z, the stencil does not
    # reach across it; pairs placed at r_c (1 +- 1e-12 .. 1e-6) by scanning
    # integer x steps, random positions besides
    rng = np.random.default_rng(21)
    box = np.array([13.0, 11.0, 2.4])
    rc = 1.0
    h = box / 2.0 ** 32
    pos, q = [], []
    for t, rel in enumerate((-1e-6, -1e-9, -1e-12, 1e-12, 1e-9, 1e-6)):
        ua = np.array([int(rng.integers(0, 2 ** 32)) for _ in range(3)], dtype=np.int64)
        dx = int(round(rc * (1.0 + rel) / h[0]))
        ub = (ua + np.array([dx, 0, 0])) % 2 ** 32
        for u in (ua, ub):
            pos.append((u + 0.5) * h)
        q += [1.0, -1.0]
    extra = rng.random((200, 3)) * box
    pos = np.concatenate([np.array(pos), extra])
    q = np.concatenate([np.array(q), np.where(np.arange(200) % 2 == 0, 1.0, -1.0)])
    sysm = R.System(pos, q, box, rc, 4, seed=3, precision=prec, skin=skin)
    assert R.rbsog_info(sysm.ctx)["ncell"][2] == 1
    R.rbsog_debug_record_pairs(sysm.ctx, 1 << 16)
    sysm.sample_k(2)
    sysm.forces()
    row, cols, kinds = recorded_pairs(sysm)
    row_o, cols_o = orc.neighbors_brute(pos, box, rc)
    assert kinds == (2 if skin > 0 else 4)
    assert_same_csr(row, cols, row_o, cols_o, "single-cell z")
    sysm.close()


@pytest.mark.parametrize("prec", [R.RBSOG_FP64, R.RBSOG_FP32C])
@pytest.mark.parametrize("skin", [0.1, 0.0])
def test_kernel_pairs_along_a_trajectory(orc, prec, skin):
    # velocity-Verlet steps of a 3000-ion system with list builds and list
    # passes: after every step the kernel's record equals the neighbour list
    # of the library's debug kernel (plain loop over the cells, exact rule)
    # at the same fixed-point positions, and the first record equals the oracle's
    rng = np.random.default_rng(8)
    n, Lb = 3000, 16.0
    pos = rng.random((n, 3)) * Lb
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    box = np.array([Lb] * 3)
    sysm = R.System(pos, q, box, 1.6, 16, seed=5, precision=prec, skin=skin)
    R.rbsog_debug_record_pairs(sysm.ctx, 1 << 20)
    sysm.sample_k(40)
    sysm.forces()
    row, cols, _ = recorded_pairs(sysm)
    row_o, cols_o = orc.neighbors_brute(pos, box, 1.6)
    assert_same_csr(row, cols, row_o, cols_o, "step 0 vs oracle")
    R.rbsog_set_velocities(sysm.ctx, None, T=4.0, seed=9)
    seen = set()
    for s in range(30):
        sysm.step(1, 2e-3)
        row, cols, kinds = recorded_pairs(sysm)
        rowd, colsd = R.rbsog_debug_neighbors(sysm.ctx)
        assert_same_csr(row, cols, rowd, colsd, f"step {s + 1}")
        seen.add(kinds)
    print(f"prec={prec} skin={skin}: kernels seen {sorted(seen)}", flush=True)
    assert seen == ({2} if skin > 0 else {4})
    sysm.close()


@pytest.mark.parametrize("prec", [R.RBSOG_FP64, R.RBSOG_FP32C])
@pytest.mark.parametrize("dense", [False, True])
def test_list_layouts_pairs_and_forces(orc, prec, dense):
    # short lists are kept in columns (one home per lane in the list pass),
    # long ones home by home (one home per wave): both give the oracle's
    # neighbour set bit for bit and its near forces, at a build and after it
    rng = np.random.default_rng(31)
    n, Lb, rc = (1500, 10.0, 3.0) if dense else (3000, 30.0, 3.0)
    pos = rng.random((n, 3)) * Lb
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    box = np.array([Lb] * 3)
    sysm = R.System(pos, q, box, rc, 8, seed=5, precision=prec)
    assert R.rbsog_info(sysm.ctx)["list_home_major"] == dense
    R.rbsog_debug_record_pairs(sysm.ctx, 1 << 21)
    sysm.sample_k(4)
    row_o, cols_o = orc.neighbors_brute(pos, box, rc)
    s = sysm.sog
    Fo, _ = orc.near_brute(pos, q, box, rc, orc.SOG(s.b, s.sigma, s.w0, s.M))
    tol = 1e-11 if prec == R.RBSOG_FP64 else 1e-5
    for what in ("build", "list pass"):
        sysm.forces()
        row, cols, kinds = recorded_pairs(sysm)
        assert kinds == 2
        assert_same_csr(row, cols, row_o, cols_o, what)
        Fn, _ = sysm.components()
        err = np.sqrt(np.sum((Fn - Fo) ** 2) / np.sum(Fo ** 2))
        print(f"dense={dense} prec={prec} {what}: near relrms {err:.2e}", flush=True)
        assert err < tol
    sysm.close()
