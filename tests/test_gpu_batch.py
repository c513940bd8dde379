"""Batched contexts (several independent systems in one context, one launch
per kernel for the whole batch) against the FP64 oracle, system by system,
and against single-system contexts.

Bars as for single systems: lists and sampled sequences bit-exact, FP64
forces within 1e-11 and FP32C within 1e-5 relative RMS of the oracle."""
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


def mixed_systems():
    """Heterogeneous batch: cubic and skewed boxes, 1-cell and 3-cell grids,
    a ragged odd-sized system with a zero charge, different cutoffs and P."""
    out = []
    specs = [(1000, (10.0, 10.0, 10.0), 3.0, 100), (777, (11.3, 9.7, 14.1), 3.1, 37),
             (64, (6.0, 6.0, 6.0), 2.9, 130), (3000, (20.0, 18.0, 22.0), 3.5, 64), (2, (10.0, 10.0, 10.0), 3.0, 1)]
    for i, (n, box, rc, P) in enumerate(specs):
        rng = np.random.default_rng(100 + i)
        box = np.array(box)
        pos = rng.random((n, 3)) * box
        q = np.where(np.arange(n) < n // 2, 1.0, -1.0)
        if n % 2:
            q[-1] = 0.0
        if n == 2:
            pos = np.array([[1.0, 1.0, 1.0], [2.2, 1.5, 0.4]])
        out.append(dict(pos=pos, q=q, box=box, rc=rc, P=P, seed=500 + i))
    return out


def make_batch(systems, prec, **kw):
    say(f"[gpu] batch of {len(systems)} systems, n={[len(s['q']) for s in systems]} prec={prec} {kw}")
    return R.Batch([s["pos"] for s in systems], [s["q"] for s in systems], [s["box"] for s in systems],
                   [s["rc"] for s in systems], [s["P"] for s in systems], [s["seed"] for s in systems],
                   precision=prec, **kw)


def split(arr, sizes):
    return np.split(arr, np.cumsum(sizes)[:-1])


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
@pytest.mark.parametrize("skin", [None, 0.0])
def test_mixed_batch_vs_oracle(orc, prec, tol, skin):
    # skin 0: every evaluation builds (fused cell kernel, far force beside it
    # in the order before the re-sort, taken back through the permutation)
    systems = mixed_systems()
    b = make_batch(systems, prec, skin=skin)
    m_all = b.sample_k(1)
    F, E = b.forces()
    Fn, Ff = b.components()
    m_parts = split(m_all, [s["P"] for s in systems])
    for i, (s, m, Fi, Fni, Ffi, Ei) in enumerate(zip(systems, m_parts, split(F, b.sizes), split(Fn, b.sizes),
                                                     split(Ff, b.sizes), E)):
        sog = orc.SOG(b.sogs[i].b, b.sogs[i].sigma, b.sogs[i].w0, b.sogs[i].M)
        # each system samples its own chain
        want_m, _ = orc.mh_sample(sog, s["box"], seed=s["seed"], stream=0, n=s["P"])
        assert (m == want_m).all()
        Fn_o, Un_o = orc.near_brute(s["pos"], s["q"], s["box"], s["rc"], sog)
        Ff_o, Us_o, _, _ = orc.far_rb(s["pos"], s["q"], s["box"], sog, m, s["P"])
        e_n, e_f, e_t = relrms(Fni, Fn_o), relrms(Ffi, Ff_o), relrms(Fi, Fn_o + Ff_o)
        say(f"[batch sys {i}] relrms near {e_n:.3e} far {e_f:.3e} total {e_t:.3e}")
        assert e_n < tol and e_f < tol and e_t < tol
        Uself = orc.self_energy(sog, s["q"])
        for got, want in ((Ei[0], Un_o), (Ei[1], Us_o), (Ei[2], Uself), (Ei[3], Un_o + Us_o - Uself)):
            assert abs(got - want) / max(abs(want), 1.0) < tol * 10
        # cell and neighbour lists of the system, local indices, bit-exact
        start, order = R.rbsog_debug_cells(b.ctx, sys=i)
        width = s["rc"] * (1.0 + (R.rbsog_default_opts().skin if skin is None else skin))
        _, _, start_o, order_o = orc.cell_list(s["pos"], s["box"], width)
        assert (start == start_o).all() and (order == order_o).all()
        row, cols = R.rbsog_debug_neighbors(b.ctx, sys=i)
        row_o, cols_o = orc.neighbors_brute(s["pos"], s["box"], s["rc"])
        assert (row == row_o).all() and (cols == cols_o).all()
        re, im = R.rbsog_get_rho(b.ctx, s["P"], sys=i)
        info = R.rbsog_info(b.ctx, sys=i)
        assert info["n"] == len(s["q"]) and info["n_sys"] == len(systems)
    b.close()


def test_batch_matches_single_contexts():
    systems = mixed_systems()
    b = make_batch(systems, R.RBSOG_FP64)
    b.sample_k(4)
    b.step(2, 1e-3)
    Fb, Eb = b.forces()
    xb, vb = R.rbsog_get_state(b.ctx, b.n)
    for i, (s, Fi, Ei, xi, vi) in enumerate(zip(systems, split(Fb, b.sizes), Eb, split(xb, b.sizes),
                                                split(vb, b.sizes))):
        one = R.System(s["pos"], s["q"], s["box"], s["rc"], s["P"], seed=s["seed"], precision=R.RBSOG_FP64)
        one.sample_k(4)
        one.step(2, 1e-3)
        F1, E1 = one.forces()
        x1, v1 = R.rbsog_get_state(one.ctx, len(s["q"]))
        e = relrms(Fi, F1)
        say(f"[batch vs single {i}] force relrms {e:.3e}")
        # the same arithmetic per pair; only the grouping of partial sums differs
        assert e < 1e-12
        assert np.allclose(Ei, E1, rtol=1e-12, atol=1e-12)
        assert np.allclose(xi, x1, rtol=0, atol=1e-12) and np.allclose(vi, v1, rtol=0, atol=1e-12)
        one.close()
    b.close()


@pytest.mark.parametrize("prec", [R.RBSOG_FP64, R.RBSOG_FP32C])
@pytest.mark.parametrize("skin", [None, 0.0])
def test_batch_graph_replay_equals_eager(prec, skin):
    systems = mixed_systems()
    runs = []
    for graphs in (True, False):
        b = R.Batch([s["pos"] for s in systems], [s["q"] for s in systems], [s["box"] for s in systems],
                    [s["rc"] for s in systems], [s["P"] for s in systems], [s["seed"] for s in systems],
                    precision=prec, graphs=graphs, skin=skin)
        b.sample_k(12)
        R.rbsog_set_velocities(b.ctx, None, T=1.0, seed=9)
        states = []
        for _ in range(3):
            b.step(3, 1e-3)
            states.append(R.rbsog_get_state(b.ctx, b.n) + (R.rbsog_get_energy(b.ctx),))
        runs.append(states)
        b.close()
    for sg, se in zip(*runs):
        for a, c in zip(sg, se):
            assert (a == c).all()


def test_replica_ensemble_sampled(orc):
    # a 16-replica ensemble with log-uniform sizes, FP32C as in production
    ens = W.c4_ensemble(n_sys=16, nmin=500, nmax=5000, seed=44)
    systems = [dict(pos=s["pos"], q=s["q"], box=s["box"], rc=ens["rc"], P=ens["P"], seed=sd)
               for s, sd in zip(ens["systems"], ens["seeds"])]
    b = make_batch(systems, R.RBSOG_FP32C)
    m_all = b.sample_k(1)
    F, E = b.forces()
    for i, (s, m, Fi) in enumerate(zip(systems, split(m_all, [s["P"] for s in systems]), split(F, b.sizes))):
        sog = orc.SOG(b.sogs[i].b, b.sogs[i].sigma, b.sogs[i].w0, b.sogs[i].M)
        Fn_o, _ = orc.near_cells(s["pos"], s["q"], s["box"], s["rc"], sog)
        Ff_o, _, _, _ = orc.far_rb(s["pos"], s["q"], s["box"], sog, m, s["P"])
        e = relrms(Fi, Fn_o + Ff_o)
        say(f"[ensemble {i}] n={len(s['q'])} L={s['box'][0]:.2f} relrms {e:.3e}")
        assert e < F32C_TOL
    b.close()


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, 1e-10), (R.RBSOG_FP32C, 2e-5)])
def test_mixed_batch_steps_building_every_step(orc, prec, tol):
    # skin 0 over several velocity-Verlet steps: after every step the near
    # and far forces of each system match the oracle at the library's own
    # positions (the far force crosses the re-sort's permutation, which now
    # moves particles within every system's slot range)
    systems = mixed_systems()
    b = make_batch(systems, prec, skin=0.0)
    b.sample_k(8)
    b.forces()
    R.rbsog_set_velocities(b.ctx, None, T=3.0, seed=13)
    for step in range(3):
        b.step(1, 2e-3)
        x, _ = R.rbsog_get_state(b.ctx, b.n)
        Fn, Ff = b.components()
        # the batch of each system's latest evaluation (the sequences
        # themselves are checked bit for bit elsewhere)
        ms = [R.rbsog_get_kbatch(b.ctx, s["P"], sys=i) for i, s in enumerate(systems)]
        for i, (s, xi, Fni, Ffi, m) in enumerate(zip(systems, split(x, b.sizes), split(Fn, b.sizes),
                                                     split(Ff, b.sizes), ms)):
            sog = orc.SOG(b.sogs[i].b, b.sogs[i].sigma, b.sogs[i].w0, b.sogs[i].M)
            Fn_o, _ = orc.near_brute(xi, s["q"], s["box"], s["rc"], sog)
            Ff_o, _, _, _ = orc.far_rb(xi, s["q"], s["box"], sog, m, s["P"])
            e_n, e_f = relrms(Fni, Fn_o), relrms(Ffi, Ff_o)
            say(f"[batch skin 0 step {step + 1} sys {i}] near {e_n:.3e} far {e_f:.3e}")
            assert e_n < tol and e_f < tol
    b.close()
