"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: integer work (cells, neighbour lists, sampled wave vectors) bit-exact;
FP64 forces within 1e-11 relative RMS (per part: near, far, total) and
FP64 energies within 1e-11 relative; FP32C forces within 1e-5 relative RMS
of the FP64 oracle.  Random-batch forces are compared on the identical k
list.  Full-size checks compare sampled particles computed one by one by the
oracle."""
import math
import sys

import numpy as np
import pytest

from paper_2205_13824_amd import rbsog as R
from paper_2205_13824_amd import workloads as W

pytestmark = pytest.mark.gpu

F64_TOL = 1e-11
F32C_TOL = 1e-5


def relrms(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b ** 2)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(pos, q, box, rc, P, seed=11, prec=R.RBSOG_FP64, sog=None, **kw):
    say(f"[gpu] init n={len(q)} box={tuple(np.round(box, 3))} rc={rc} P={P} prec={prec} {kw}")
    return R.System(pos, q, box, rc, P, seed=seed, precision=prec, sog=sog, **kw)


def cell_width(rc, skin=None):
    """Cells of the near list are at least r_c (1 + skin) wide."""
    if skin is None:
        skin = R.rbsog_default_opts().skin
    return rc * (1.0 + skin)


def oracle_sog(orc, s: R.rbsog_sog):
    return orc.SOG(s.b, s.sigma, s.w0, s.M)


def check_eval(orc, sysm, pos, q, box, rc, m, tol, label):
    """One evaluation on the GPU vs the oracle's near (brute force) + RB far on list m."""
    sog = oracle_sog(orc, sysm.sog)
    F, E = sysm.forces()
    Fn, Ff = sysm.components()
    Fn_o, Un_o = orc.near_brute(pos, q, box, rc, sog)
    Ff_o, Us_o, _, _ = orc.far_rb(pos, q, box, sog, m, sysm.P)
    e_near, e_far, e_tot = relrms(Fn, Fn_o), relrms(Ff, Ff_o), relrms(F, Fn_o + Ff_o)
    say(f"[{label}] relrms near {e_near:.3e} far {e_far:.3e} total {e_tot:.3e}")
    assert e_near < tol and e_far < tol and e_tot < tol
    Uself = orc.self_energy(sog, q)
    for got, want, name in ((E[0], Un_o, "U_N"), (E[1], Us_o, "U*"), (E[2], Uself, "U_self"),
                            (E[3], Un_o + Us_o - Uself, "U")):
        err = abs(got - want) / max(abs(want), 1.0)
        say(f"[{label}] {name} gpu {got:.15g} oracle {want:.15g} rel {err:.2e}")
        assert err < tol * 10
    return F, E


def test_sampler_sequence_bit_exact(orc):
    c = W.c1_small()
    sysm = make(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=101)
    got = sysm.sample_k(5)
    want, _ = orc.mh_sample(oracle_sog(orc, sysm.sog), c["box"], seed=101, stream=0, n=5 * c["P"])
    assert got.shape == want.shape and (got == want).all()
    # the chain continues across calls
    more = sysm.sample_k(2)
    want2, _ = orc.mh_sample(oracle_sog(orc, sysm.sog), c["box"], seed=101, stream=0, n=7 * c["P"])
    assert (more == want2[5 * c["P"]:]).all()


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_c1_one_evaluation(orc, prec, tol):
    c = W.c1_small()
    sysm = make(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=101, prec=prec)
    m = sysm.sample_k(1)
    check_eval(orc, sysm, c["pos"], c["q"], c["box"], c["rc"], m, tol, f"C1 prec={prec}")
    info = R.rbsog_info(sysm.ctx)
    S_o = orc.S_product(oracle_sog(orc, sysm.sog), c["box"])
    assert abs(info["S"] / S_o - 1) < 1e-13


@pytest.mark.parametrize("prec", [R.RBSOG_FP64, R.RBSOG_FP32C])
@pytest.mark.parametrize("case,skin", [("c1", None), ("c1", 0.0), ("c1", 0.3), ("skew", None), ("tiny", None),
                                       ("manycells", None)])
def test_cell_and_neighbour_lists_bit_exact(orc, prec, case, skin):
    if case == "c1":
        c = W.c1_small()
        pos, q, box, rc = c["pos"], c["q"], c["box"], c["rc"]
    elif case == "skew":
        rng = np.random.default_rng(3)
        box = np.array([11.3, 9.7, 14.1])
        pos = rng.random((777, 3)) * box - 5.0  # unwrapped input
        q = np.where(np.arange(777) < 388, 1.0, -1.0)
        q[-1] = 0.0
        rc = 3.1
    elif case == "manycells":
        # 60^3 = 216,000 cells of width 1.1: the cell-count scan takes its multi-block path
        rng = np.random.default_rng(5)
        box = np.array([66.5, 66.5, 66.5])
        pos = rng.random((20000, 3)) * box
        q = np.where(np.arange(20000) % 2 == 0, 1.0, -1.0)
        rc = 1.0
    else:
        rng = np.random.default_rng(4)
        box = np.array([6.0, 6.0, 6.0])  # floor(L/rc) = 2 -> single cell per dimension
        pos = rng.random((64, 3)) * box
        q = np.where(np.arange(64) % 2 == 0, 1.0, -1.0)
        rc = 2.9
    sysm = make(pos, q, box, rc, 8, prec=prec, skin=skin)
    sysm.sample_k(1)
    sysm.forces()
    start, order = R.rbsog_debug_cells(sysm.ctx, len(q))
    nc, _, start_o, order_o = orc.cell_list(pos, box, cell_width(rc, skin))
    assert tuple(R.rbsog_info(sysm.ctx)["ncell"]) == tuple(int(v) for v in nc)
    assert (start == start_o).all() and (order == order_o).all()
    row, cols = R.rbsog_debug_neighbors(sysm.ctx, len(q))
    row_o, cols_o = orc.neighbors_brute(pos, box, rc)
    assert (row == row_o).all() and (cols == cols_o).all()


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
@pytest.mark.parametrize("n,box,rc,P", [
    (777, (11.3, 9.7, 14.1), 3.1, 37),     # ragged n, non-cubic box, odd P
    (64, (6.0, 6.0, 6.0), 2.9, 130),       # single-cell fallback, P spans 3 k tiles
    (5000, (20.0, 20.0, 20.0), 3.5, 1500),  # P above one block of k tiles
    (2, (10.0, 10.0, 10.0), 3.0, 1),       # smallest system
])
def test_ragged_shapes(orc, prec, tol, n, box, rc, P):
    rng = np.random.default_rng(n + P)
    box = np.array(box)
    pos = rng.random((n, 3)) * box
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    if n % 2:
        q[-1] = 0.0
    if n == 2:
        pos = np.array([[1.0, 1.0, 1.0], [2.2, 1.5, 0.4]])
    sysm = make(pos, q, box, rc, P, seed=n, prec=prec)
    m = sysm.sample_k(1)
    check_eval(orc, sysm, pos, q, box, rc, m, tol, f"ragged n={n} P={P} prec={prec}")


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_full_fourier_sum_mode(orc, prec, tol):
    # every k of the lattice with weight F~(k)/V: the deterministic far part
    rng = np.random.default_rng(7)
    L = 8.0
    box = np.array([L, L, L])
    n = 300
    pos = rng.random((n, 3)) * L
    q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
    rc = 3.0
    sog_c = R.rbsog_sog_table1(2, rc)
    sog = oracle_sog(orc, sog_c)
    mk = orc.kvectors_full(sog, box)
    w = orc.full_weights(sog, box, mk)
    sysm = make(pos, q, box, rc, len(mk), prec=prec, sog=sog_c)
    sysm.set_k(mk, w)
    F, E = sysm.forces()
    _, Ff = sysm.components()
    Ff_o, Us_o, _, _ = orc.far_full(pos, q, box, sog)
    err = relrms(Ff, Ff_o)
    say(f"[full-sum prec={prec}] P={len(mk)} far relrms {err:.3e} U* {E[1]:.15g} vs {Us_o:.15g}")
    assert err < tol
    assert abs(E[1] - Us_o) / abs(Us_o) < tol * 10


def test_repeat_evaluation_is_bitwise_identical(orc):
    c = W.c1_small()
    sysm = make(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=5)
    m = sysm.sample_k(1)
    sysm.set_k(np.concatenate([m, m]))
    F1, E1 = sysm.forces()
    F2, E2 = sysm.forces()
    assert (F1 == F2).all() and (E1 == E2).all()


def test_sequence_exhaustion_is_reported_and_recoverable(orc):
    c = W.c1_small()
    sysm = make(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=5)
    with pytest.raises(R.RbsogError) as e:
        sysm.forces()
    assert e.value.status == -8
    sysm.sample_k(1)
    sysm.forces()
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_step(sysm.ctx, 1, 1e-3)
    assert e.value.status == -8


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, 1e-10), (R.RBSOG_FP32C, 1e-5)])
def test_velocity_verlet_matches_oracle(orc, prec, tol):
    n, L = 200, 10.0
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 21)
    v0 = W.maxwellian(n, 1.0, 22)
    rc, P, steps, dt = 3.0, 40, 5, 1e-3
    sysm = make(pos, q, box, rc, P, seed=9, prec=prec)
    m = sysm.sample_k(steps + 1)
    R.rbsog_set_velocities(sysm.ctx, v0)
    sysm.step(steps, dt)
    x_g, v_g = R.rbsog_get_state(sysm.ctx, n)
    x_o, v_o, F_o, _ = orc.vv_run(pos, v0, q, box, rc, oracle_sog(orc, sysm.sog), P, m, steps, dt)
    dx = x_g - x_o
    dx -= box * np.round(dx / box)
    ex = float(np.abs(dx).max())
    ev = relrms(v_g - v0, v_o - v0)
    say(f"[vv prec={prec}] max|dx| {ex:.3e} velocity-change relrms {ev:.3e}")
    assert ex < tol * 10
    assert ev < tol * 10
    # total momentum: FP64 forces cancel to rounding; FP32C near/far sums cancel to ~1e-7 of |F|
    assert np.abs(v_g.sum(0) - v0.sum(0)).max() < (1e-9 if prec == R.RBSOG_FP64 else 1e-7)


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, 1e-10), (R.RBSOG_FP32C, 1e-5)])
def test_energies_after_a_run_of_steps(orc, prec, tol):
    # the steps of a run sum no energies but the last: after 21 steps (graphs
    # of several steps, then the last step alone) the energies are those of
    # the final positions and the last wave-vector batch
    n, L = 300, 12.0
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 23)
    rc, P, steps, dt = 3.0, 40, 21, 1e-3
    sysm = make(pos, q, box, rc, P, seed=12, prec=prec)
    m = sysm.sample_k(steps + 1)
    R.rbsog_set_velocities(sysm.ctx, None, T=1.0, seed=5)
    sysm.step(steps, dt)
    x, _ = R.rbsog_get_state(sysm.ctx, n)
    E = R.rbsog_get_energy(sysm.ctx)
    sog = oracle_sog(orc, sysm.sog)
    _, Un = orc.near_brute(x, q, box, rc, sog)
    _, Us, _, _ = orc.far_rb(x, q, box, sog, m[steps * P:], P)
    say(f"[energies after steps prec={prec}] U_N {E[0]:.12g} vs {Un:.12g}, U* {E[1]:.12g} vs {Us:.12g}")
    assert abs(E[0] - Un) < tol * abs(Un) and abs(E[1] - Us) < tol * abs(Us)
    assert abs(E[3] - (E[0] + E[1] - E[2])) < 1e-12 * abs(E[1])


def test_maxwellian_velocities_have_zero_momentum_and_temperature(orc):
    c = W.c1_small()
    sysm = make(c["pos"], c["q"], c["box"], c["rc"], c["P"])
    R.rbsog_set_velocities(sysm.ctx, None, T=2.0, seed=3)
    _, v = R.rbsog_get_state(sysm.ctx, 1000)
    assert np.abs(v.sum(0)).max() < 1e-10
    assert abs(float((v * v).mean()) / 2.0 - 1) < 0.1


@pytest.fixture(scope="module")
def c2():
    say("[gpu] building the 300,000-ion electrolyte")
    return W.c2_electrolyte()


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_c2_full_size_sampled(orc, c2, prec, tol):
    pos, q, box, rc, P = c2["pos"], c2["q"], c2["box"], c2["rc"], c2["P"]
    n = len(q)
    sysm = make(pos, q, box, rc, P, seed=202, prec=prec)
    m = sysm.sample_k(1)
    F, E = sysm.forces()
    Fn, Ff = sysm.components()
    re, im = R.rbsog_get_rho(sysm.ctx, P)
    sog = oracle_sog(orc, sysm.sog)
    targets = np.random.default_rng(55).choice(n, 400, replace=False)
    Fn_o = orc.near_targets(pos, q, box, rc, sog, targets)
    S = orc.S_product(sog, box)
    Ff_o, Us_o, re_o, im_o = orc.far_rb(pos, q, box, sog, m, P, S, targets=targets)
    e_rho = math.sqrt(float(np.sum((re - re_o) ** 2 + (im - im_o) ** 2) / np.sum(re_o ** 2 + im_o ** 2)))
    e_near, e_far = relrms(Fn[targets], Fn_o), relrms(Ff[targets], Ff_o)
    say(f"[C2 prec={prec}] rho {e_rho:.3e} near {e_near:.3e} far {e_far:.3e} U* rel "
        f"{abs(E[1] - Us_o) / abs(Us_o):.3e}")
    assert e_rho < tol and e_near < tol and e_far < tol
    assert abs(E[1] - Us_o) / abs(Us_o) < 10 * tol
    # properties at full size: Newton's third law and zero total far force
    assert np.abs(Fn.sum(0)).max() < (1e-9 if prec == R.RBSOG_FP64 else 1e-3) * np.abs(Fn).max() * math.sqrt(n)
    assert np.abs(Ff.sum(0)).max() < (1e-9 if prec == R.RBSOG_FP64 else 1e-3) * np.abs(Ff).max() * math.sqrt(n)


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_structure_factor_mixed_charges(orc, prec, tol):
    """Charges of both signs and several magnitudes, zeros included, in a
    random order over 30,000 ions: the FP32C structure factor pairs equal
    charges within each wave of a stage and sums the rest singly (odd
    counts per sign, unequal neighbours, a ragged last chunk and stage);
    rho(k) of the batch against the oracle's direct sum."""
    c = W.c2_electrolyte(30_000)
    n = len(c["q"])
    pattern = np.array([1.0, -1.0, 0.4238, 0.4238, -0.8476, 0.3, -0.3, 0.0])
    q = np.random.default_rng(77).permutation(np.tile(pattern, n // 8))
    sysm = make(c["pos"], q, c["box"], c["rc"], c["P"], seed=303, prec=prec)
    m = sysm.sample_k(1)
    sysm.forces()
    re, im = R.rbsog_get_rho(sysm.ctx, c["P"])
    re_o, im_o = orc.structure_factor(c["pos"], q, c["box"], m[: c["P"]])
    e = math.sqrt(float(np.sum((re - re_o) ** 2 + (im - im_o) ** 2) / np.sum(re_o ** 2 + im_o ** 2)))
    say(f"[mixed charges prec={prec}] rho relrms {e:.3e}")
    assert e < tol
    sysm.close()


@pytest.mark.parametrize("prec,nh,skin", [(R.RBSOG_FP64, False, None), (R.RBSOG_FP32C, False, None),
                                          (R.RBSOG_FP32C, True, None), (R.RBSOG_FP64, False, 0.0),
                                          (R.RBSOG_FP32C, True, 0.0)])
def test_graph_replay_equals_eager(orc, prec, nh, skin):
    # rbsog_step replays captured graphs of one and of several steps; interleave
    # replays with host reads (synchronisations) and compare with eager
    # launches bit for bit (also with the Nose-Hoover thermostat, whose
    # kinetic-energy sum runs inside every step, and building at every step,
    # where the far force runs on the second stream beside the near part)
    n, L = 500, 12.0
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 31)
    v0 = W.maxwellian(n, 1.0, 32)
    kw = {} if skin is None else {"skin": skin}
    out = []
    for graphs in (False, True):
        say(f"[gpu] graph replay check prec={prec} nh={nh} skin={skin} graphs={graphs}")
        sysm = R.System(pos, q, box, 3.0, 50, seed=3, precision=prec, graphs=graphs, **kw)
        sysm.sample_k(70)
        R.rbsog_set_velocities(sysm.ctx, v0)
        if nh:
            R.rbsog_set_nose_hoover(sysm.ctx, 1.2, 0.05)
        states = []
        # runs of 9 and 20 steps take the graphs of several steps
        for chunk in (5, 7, 3, 9, 20):
            sysm.step(chunk, 1e-3)
            states.append(R.rbsog_get_state(sysm.ctx, n))
        states.append(tuple(sysm.components()))
        states.append((R.rbsog_get_energy(sysm.ctx),))
        states.append(R.rbsog_get_kinetic(sysm.ctx))
        out.append(states)
        sysm.close()
    for a, b in zip(*out):
        for x, y in zip(a, b):
            assert (x == y).all()


@pytest.mark.parametrize("prec", [R.RBSOG_FP64, R.RBSOG_FP32C])
def test_fused_steps_equal_unfused(orc, prec):
    # with graphs, plain velocity-Verlet steps on a kept list are fused: the
    # far kernel opens the next step (its kick, drift, quantisation and
    # displacement check) and the next step stages its k records alone.
    # Eager launches are never fused: the two must agree bit for bit, with
    # list builds inside fused runs (dt large enough for the displacement
    # check to fire), runs that cross the build-rate check, fused graphs of
    # one and of several steps, and the mean-square displacement tracked.
    n, L = 500, 12.0
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 41)
    v0 = W.maxwellian(n, 1.0, 42)
    out = []
    for graphs in (False, True):
        say(f"[gpu] fused vs unfused steps prec={prec} graphs={graphs}")
        sysm = R.System(pos, q, box, 3.0, 50, seed=5, precision=prec, graphs=graphs)
        sysm.sample_k(200)
        R.rbsog_set_velocities(sysm.ctx, v0)
        R.rbsog_set_msd_origin(sysm.ctx)
        states = []
        for chunk in (2, 11, 17, 40, 1, 9):
            sysm.step(chunk, 5e-3)
            states.append(R.rbsog_get_state(sysm.ctx, n))
            states.append((np.asarray(R.rbsog_get_msd(sysm.ctx)),))
        states.append(tuple(sysm.components()))
        states.append((R.rbsog_get_energy(sysm.ctx),))
        states.append(R.rbsog_get_kinetic(sysm.ctx))
        info = R.rbsog_info(sysm.ctx)
        states.append((np.array([info["list_builds"]]),))
        say(f"[gpu]   list builds {info['list_builds']} skin {info['skin']}")
        assert info["list_builds"] >= 3
        out.append(states)
        sysm.close()
    for a, b in zip(*out):
        for x, y in zip(a, b):
            assert (np.asarray(x) == np.asarray(y)).all()


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
@pytest.mark.parametrize("skin", [None, 0.0])
def test_autotune_keeps_results(orc, prec, tol, skin):
    c = W.c1_small()
    sysm = make(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=101, prec=prec, skin=skin)
    m = sysm.sample_k(3)
    F0, E0 = sysm.forces()
    Fn0, Ff0 = sysm.components()
    info = R.rbsog_autotune(sysm.ctx, 2)
    say(f"[autotune prec={prec} skin={skin}] shapes chunk={info['rho_chunk']} ktile={info['rho_ktile']} "
        f"far_block={info['far_block']} slots={info['build_slots']}/{info['cell_slots']} tuned={info['tuned']}")
    assert info["tuned"] and info["k_remaining"] == 2 * c["P"]
    # the tuning recomputed the forces of the same positions with the chosen
    # shapes (the near kernel's slots per pass and the structure factor's
    # chunks order the FP32 sums)
    Fn1, Ff1 = sysm.components()
    rt = 1e-13 if prec == R.RBSOG_FP64 else 1e-6
    assert relrms(Fn1, Fn0) < rt and relrms(Ff1, Ff0) < rt
    # and later evaluations still match the oracle
    check_eval(orc, sysm, c["pos"], c["q"], c["box"], c["rc"], m[c["P"]:2 * c["P"]], tol, f"tuned prec={prec}")


@pytest.mark.parametrize("prec", [R.RBSOG_FP64, R.RBSOG_FP32C])
def test_autotune_after_new_sequence(orc, prec):
    # the structure factor reads the batch at the sequence cursor, and the
    # tuner times it on the latest evaluation's batch again; after set_k
    # that batch is gone: the tuner keeps the structure factor's shapes, the
    # forces stay those of the evaluation, and the next evaluation takes the
    # new sequence from its start
    c = W.c1_small()
    sysm = make(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=102, prec=prec)
    sysm.sample_k(2)
    sysm.forces()
    Fn0, Ff0 = sysm.components()
    shapes0 = R.rbsog_info(sysm.ctx)
    rng = np.random.default_rng(9)
    mnew = rng.integers(-4, 5, size=(3 * c["P"], 3)).astype(np.int32)
    mnew[np.all(mnew == 0, axis=1)] = (1, 0, 0)
    sysm.set_k(mnew)
    info = R.rbsog_autotune(sysm.ctx, 2)
    assert info["tuned"] and info["k_remaining"] == 3 * c["P"]
    assert info["rho_chunk"] == shapes0["rho_chunk"] and info["rho_ktile"] == shapes0["rho_ktile"]
    Fn1, Ff1 = sysm.components()
    rt = 1e-13 if prec == R.RBSOG_FP64 else 1e-6
    assert relrms(Fn1, Fn0) < rt and relrms(Ff1, Ff0) < rt
    tol = F64_TOL if prec == R.RBSOG_FP64 else F32C_TOL
    check_eval(orc, sysm, c["pos"], c["q"], c["box"], c["rc"], mnew[:c["P"]], tol, f"tuned after set_k prec={prec}")


def test_autotune_option_in_step():
    c = W.c1_small()
    runs = []
    for tune in (False, True):
        s = R.System(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=5, precision=R.RBSOG_FP64, autotune=tune)
        s.sample_k(6)
        R.rbsog_set_velocities(s.ctx, None, T=1.0, seed=2)
        s.step(4, 1e-3)
        runs.append(R.rbsog_get_state(s.ctx, 1000) + (R.rbsog_get_energy(s.ctx),))
        assert R.rbsog_info(s.ctx)["tuned"] == tune or tune is False
        s.close()
    for a, b in zip(*runs):
        assert np.allclose(a, b, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("case", ["c1", "ions5000", "water"])
def test_coreshell_table_near(orc, case):
    # core-shell near kernel (Sec. 3.4) in the FP32C form: against the oracle's
    # core-shell kernel (same table construction and Taylor core) and against
    # the direct Gaussian sum, both to the FP32C bar
    from oracle import coreshell as cs
    if case == "c1":
        c = W.c1_small()
        pos, q, box, rc, P = c["pos"], c["q"], c["box"], c["rc"], c["P"]
    elif case == "ions5000":
        pos, q, box = W.ions_rsa(5000, 0.1, 1.0, seed=21)
        rc, P = 3.5, 64
    else:
        pos, q, box = W.water(10, 0.0334, seed=22)
        rc, P = 10.0, 50
    say(f"[gpu] core-shell near, case {case}: n={len(q)} rc={rc}")
    sysm = R.System(pos, q, box, rc, P, seed=9, precision=R.RBSOG_FP32C, near_table=True)
    m = sysm.sample_k(1)
    F, E = sysm.forces()
    Fn, Ff = sysm.components()
    sog = oracle_sog(orc, sysm.sog)
    nb = orc.neighbors_brute(pos, box, rc)
    Fcs, Ucs = cs.near_coreshell(pos, q, box, rc, sog, nb)
    Fo, Uo = orc.near_brute(pos, q, box, rc, sog)
    Ffo, _, _, _ = orc.far_rb(pos, q, box, sog, m, P)
    e_cs, e_ex, e_far = relrms(Fn, Fcs), relrms(Fn, Fo), relrms(Ff, Ffo)
    e_u = abs(E[0] - Ucs) / abs(Ucs)
    say(f"[core-shell {case}] near vs oracle core-shell {e_cs:.3e}, vs direct sum {e_ex:.3e}; far {e_far:.3e}; "
        f"U_N rel {e_u:.2e}")
    assert e_cs < F32C_TOL and e_ex < F32C_TOL and e_far < F32C_TOL and e_u < F32C_TOL


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
@pytest.mark.parametrize("mode", [1, 2])
def test_zero_mode_terms(orc, prec, tol, mode):
    # spherical (1) and slab (2) zero-frequency mode terms of Sec. 3.2 on top of
    # the random-batch far force, in a 2-system batch (unwrapped input positions)
    from oracle import zeromode as zm
    systems = []
    for i, (n, L, rc, P) in enumerate(((777, 11.3, 3.1, 37), (1000, 10.0, 3.0, 100))):
        rng = np.random.default_rng(40 + i)
        box = np.array([L, L * 0.9, L * 1.1])
        pos = rng.random((n, 3)) * box * 1.5 - 2.0
        q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
        if n % 2:
            q[-1] = 0.0
        systems.append(dict(pos=pos, q=q, box=box, rc=rc, P=P))
    b = R.Batch([s["pos"] for s in systems], [s["q"] for s in systems], [s["box"] for s in systems],
                [s["rc"] for s in systems], [s["P"] for s in systems], [61, 62], precision=prec, zero_mode=mode)
    m_all = b.sample_k(1)
    F, E = b.forces()
    Fn, Ff = b.components()
    off = np.cumsum([0] + [len(s["q"]) for s in systems])
    ms = np.split(m_all, np.cumsum([s["P"] for s in systems])[:-1])
    for i, s in enumerate(systems):
        sl = slice(off[i], off[i + 1])
        sog = oracle_sog(orc, b.sogs[i])
        Ffo, Uso, _, _ = orc.far_rb(s["pos"], s["q"], s["box"], sog, ms[i], s["P"])
        Fz, Uz, _ = zm.zero_mode(s["pos"], s["q"], s["box"], mode)
        e_f = relrms(Ff[sl], Ffo + Fz)
        e_u = abs(E[i][1] - (Uso + Uz)) / abs(Uso + Uz)
        say(f"[zero mode {mode} prec={prec} sys {i}] far+zero-mode relrms {e_f:.3e}, U* rel {e_u:.2e}, "
            f"U0/U* {Uz / Uso:.3f}")
        assert e_f < tol and e_u < 10 * tol
    b.close()


def test_langevin_baoab_steps_match_oracle(orc):
    # three BAOAB steps in FP64 against the oracle's own Philox noise
    from oracle import thermostat as th
    n, L = 400, 16.0
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 71)
    v0 = W.maxwellian(n, 1.0, 72)
    rc, P, dt, gamma, T, seed = 3.5, 40, 2e-3, 3.0, 1.7, 1234
    out = []
    for graphs in (False, True):
        sysm = R.System(pos, q, box, rc, P, seed=8, precision=R.RBSOG_FP64, graphs=graphs)
        ks = sysm.sample_k(4)
        R.rbsog_set_velocities(sysm.ctx, v0)
        R.rbsog_set_thermostat(sysm.ctx, gamma, T, seed)
        sysm.step(3, dt)
        out.append(R.rbsog_get_state(sysm.ctx, n))
        sysm.close()
    assert (out[0][0] == out[1][0]).all() and (out[0][1] == out[1][1]).all()
    xo, vo = th.baoab_run(orc, pos, v0, q, box, rc, oracle_sog(orc, R.rbsog_sog_table1(2, rc)), P, ks, 3, dt,
                          gamma, T, seed)
    ex = float(np.abs(out[0][0] - xo).max())
    ev = relrms(out[0][1], vo)
    say(f"[baoab] max |x - x_oracle| {ex:.2e}, velocity relrms {ev:.2e}")
    assert ex < 1e-10 and ev < 1e-10


def test_langevin_thermostat_holds_temperature():
    # weak charges (+-0.1, Coulomb energy at contact well below kT): point ions
    # without a repulsive core would otherwise pair up and heat the system
    n = 512
    pos, q, box = W.ions_rsa(n, 0.1, 1.0, 73)
    q = 0.1 * q
    T, gamma = 1.5, 2.0
    sysm = R.System(pos, q, box, 3.5, 50, seed=9, precision=R.RBSOG_FP32C)
    sysm.sample_k(2 + 3000)
    R.rbsog_set_thermostat(sysm.ctx, gamma, T, 77)
    sysm.step(1000, 2e-3)
    temps = []
    for _ in range(40):
        sysm.step(50, 2e-3)
        _, v = R.rbsog_get_state(sysm.ctx, n)
        temps.append(float((v * v).sum()) / (3 * n))
    Tm = float(np.mean(temps))
    say(f"[thermostat] kinetic temperature {Tm:.4f} (target {T})")
    assert abs(Tm / T - 1.0) < 0.05


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_near_list_rebuilds_keep_pairs_exact(orc, prec, tol):
    # a hot system and a thin skin: the list is rebuilt many times during the
    # run; after every chunk of steps (graphs and single eager steps) the near
    # forces and the neighbour list at the current positions match the oracle
    n, L, rc, P = 500, 12.0, 3.0, 30
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 41)
    sysm = make(pos, q, box, rc, P, seed=5, prec=prec, skin=0.02)
    sysm.sample_k(140)
    R.rbsog_set_velocities(sysm.ctx, None, T=20.0, seed=8)
    sog = oracle_sog(orc, sysm.sog)
    builds = [R.rbsog_info(sysm.ctx)["list_builds"]]
    skins = []
    for chunk in (1, 6, 1, 9, 12, 1, 8, 40, 3, 50):
        sysm.step(chunk, 2e-3)
        x, _ = R.rbsog_get_state(sysm.ctx, n)
        Fn, _ = sysm.components()
        Fn_o, _ = orc.near_brute(x, q, box, rc, sog)
        err = relrms(Fn, Fn_o)
        row, cols = R.rbsog_debug_neighbors(sysm.ctx, n)
        row_o, cols_o = orc.neighbors_brute(x, box, rc)
        info = R.rbsog_info(sysm.ctx)
        builds.append(info["list_builds"])
        skins.append(info["skin"])
        say(f"[list rebuilds prec={prec}] after {chunk} steps: builds {builds[-1]} skin {skins[-1]} "
            f"near relrms {err:.3e}")
        assert err < tol
        assert (row == row_o).all() and (cols == cols_o).all()
    assert builds[-1] - builds[0] >= 5
    # lists this short-lived switch the steps to building every time
    assert 0.0 in skins


@pytest.mark.parametrize("prec,xtol,vtol", [(R.RBSOG_FP64, 1e-10, 1e-10), (R.RBSOG_FP32C, 1e-6, 1e-5)])
def test_near_list_skin_does_not_change_the_trajectory(orc, prec, xtol, vtol):
    # the skin only changes when the list is rebuilt, not which pairs are
    # evaluated: trajectories with skins 0, 0.1 and 0.5 agree to rounding
    # (skin 0 builds at every step, with the far force computed beside the
    # near part and taken back in the new order; FP32C near sums differ in
    # order between the two modes)
    n, L, rc, P, steps = 400, 11.0, 3.0, 40, 30
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 43)
    out = []
    for skin in (0.0, 0.1, 0.5):
        sysm = make(pos, q, box, rc, P, seed=6, prec=prec, skin=skin)
        sysm.sample_k(steps + 1)
        R.rbsog_set_velocities(sysm.ctx, None, T=5.0, seed=9)
        sysm.step(steps, 2e-3)
        x, v = R.rbsog_get_state(sysm.ctx, n)
        info = R.rbsog_info(sysm.ctx)
        say(f"[skin {skin}] list builds {info['list_builds']} capacity {info['list_capacity']}")
        out.append((x, v, info["list_builds"]))
        sysm.close()
    assert out[0][2] == steps + 1 and out[2][2] < out[1][2] < out[0][2]
    for x, v, _ in out[1:]:
        dx = x - out[0][0]
        dx -= box * np.round(dx / box)
        say(f"[skin trajectories prec={prec}] max |dx| {np.abs(dx).max():.3e} v relrms {relrms(v, out[0][1]):.3e}")
        assert np.abs(dx).max() < xtol and relrms(v, out[0][1]) < vtol


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
@pytest.mark.parametrize("L", [21.5, 39.1])
def test_fused_cell_kernel_with_paired_home_cells(orc, prec, tol, L):
    # skin 0: every evaluation builds with the fused cell kernel, which pairs
    # neighbouring home cells in rows of at least 6 cells (L = 21.5: 6 cells,
    # both seams of each row inside a pair's stencil; L = 39.1: 11 cells, an
    # odd row leaves one cell alone); forces and energies vs the oracle over a
    # few steps, and the neighbour list bit-exact
    n = int(0.1 * L ** 3) // 2 * 2
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 91)
    rc, P = 3.5, 30
    sysm = make(pos, q, box, rc, P, seed=4, prec=prec, skin=0.0)
    m = sysm.sample_k(4)
    check_eval(orc, sysm, pos, q, box, rc, m[:P], tol, f"paired cells L={L} prec={prec}")
    R.rbsog_set_velocities(sysm.ctx, None, T=1.0, seed=2)
    sysm.step(2, 1e-3)
    x, _ = R.rbsog_get_state(sysm.ctx, n)
    Fn, _ = sysm.components()
    Fn_o, _ = orc.near_brute(x, q, box, rc, oracle_sog(orc, sysm.sog))
    assert relrms(Fn, Fn_o) < tol
    row, cols = R.rbsog_debug_neighbors(sysm.ctx, n)
    row_o, cols_o = orc.neighbors_brute(x, box, rc)
    assert (row == row_o).all() and (cols == cols_o).all()
    assert R.rbsog_info(sysm.ctx)["ncell"][0] == int(box[0] // rc) >= 6


@pytest.mark.parametrize("prec", [R.RBSOG_FP64, R.RBSOG_FP32C])
def test_coincident_ions_report_nonfinite_and_context_recovers(prec):
    # two ions at one point: the pair term 1/r of the near part is infinite
    # (Eq. (6)), so both rbsog_forces and rbsog_step report E_NONFINITE
    n, L = 300, 10.0
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 41)
    bad = pos.copy()
    bad[7] = bad[3]
    sysm = make(bad, q, box, 3.0, 20, seed=2, prec=prec)
    sysm.sample_k(40)
    for want_F, want_E in ((True, False), (False, True)):
        with pytest.raises(R.RbsogError) as e:
            R.rbsog_forces(sysm.ctx, n, want_F, want_E)
        assert e.value.status == -7
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_step(sysm.ctx, 1, 1e-3)
    assert e.value.status == -7
    # the report is made once; finite positions run on with finite forces
    R.rbsog_set_positions(sysm.ctx, pos)
    R.rbsog_set_velocities(sysm.ctx, np.zeros((n, 3)))
    F, E = R.rbsog_forces(sysm.ctx, n)
    assert np.isfinite(F).all() and np.isfinite(E).all()
    R.rbsog_step(sysm.ctx, 2, 1e-3)
    x, v = R.rbsog_get_state(sysm.ctx, n)
    assert np.isfinite(x).all() and np.isfinite(v).all()
    sysm.close()
