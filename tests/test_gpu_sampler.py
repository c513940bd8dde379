"""On-device wave-vector sampler (lambda Metropolis-Hastings chains per system,
the parallel sampling of Sec. 3.4) against the oracle's chains.

Chain c of a system uses Philox stream 3 + c; evaluation e takes the P states
of chain e mod lambda that follow its (e div lambda) P earlier ones.  The
oracle's independent chain of the same stream and seed must give the same
integer vectors bit for bit, the forces of each evaluation match the oracle on
that batch to the usual bars, and a trajectory driven by the device chains
matches the oracle's velocity-Verlet run on the interleaved sequence."""
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


def oracle_sog(orc, s: R.rbsog_sog):
    return orc.SOG(s.b, s.sigma, s.w0, s.M)


def expected_batches(orc, sog, box, seed, P, lam, n_evals):
    """Batch e of the device sampler, from the oracle's chains."""
    rounds = (n_evals + lam - 1) // lam
    chains = [orc.mh_sample(sog, box, seed=seed, stream=3 + c, n=rounds * P)[0] for c in range(lam)]
    return [chains[e % lam][(e // lam) * P:(e // lam + 1) * P] for e in range(n_evals)]


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_device_chains_match_oracle(orc, prec, tol):
    c = W.c1_small()
    lam, evals, seed = 8, 19, 77
    say(f"[gpu] device chains lambda={lam} evals={evals} prec={prec}")
    sysm = R.System(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=seed, precision=prec, device_chains=lam)
    sog = oracle_sog(orc, sysm.sog)
    want = expected_batches(orc, sog, c["box"], seed, c["P"], lam, evals)
    Fn_o, Un_o = orc.near_brute(c["pos"], c["q"], c["box"], c["rc"], sog)
    for e in range(evals):
        F, E = sysm.forces()
        m = sysm.kbatch()
        assert m.shape == want[e].shape and (m == want[e]).all(), f"evaluation {e}"
        info = R.rbsog_info(sysm.ctx)
        assert info["k_remaining"] == (lam - 1 - e % lam) * c["P"]
        if e in (0, lam - 1, lam, evals - 1):
            Ff_o, Us_o, _, _ = orc.far_rb(c["pos"], c["q"], c["box"], sog, m, c["P"])
            err = relrms(F, Fn_o + Ff_o)
            say(f"[device chains e={e}] force relrms {err:.3e} U* {E[1]:.12g} oracle {Us_o:.12g}")
            assert err < tol
            assert abs(E[1] - Us_o) / max(abs(Us_o), 1.0) < 10 * tol


def test_device_chains_in_a_batch(orc):
    # every system runs its own lambda chains keyed by its own seed; P differs
    specs = [(1000, 10.0, 3.0, 100, 41), (500, 9.0, 2.9, 37, 42), (64, 6.0, 2.9, 1, 43)]
    lam, evals = 4, 9
    pos_l, q_l, boxes = [], [], []
    for n, L, rc, P, sd in specs:
        p_, q_, b_ = W.ions_uniform(n, L, sd)
        pos_l.append(p_), q_l.append(q_), boxes.append(b_)
    say(f"[gpu] batch with device chains lambda={lam}")
    b = R.Batch(pos_l, q_l, boxes, [s[2] for s in specs], [s[3] for s in specs], [s[4] for s in specs],
                precision=R.RBSOG_FP64, device_chains=lam)
    wants = [expected_batches(orc, oracle_sog(orc, b.sogs[i]), boxes[i], s[4], s[3], lam, evals)
             for i, s in enumerate(specs)]
    for e in range(evals):
        b.forces()
        for i, s in enumerate(specs):
            m = R.rbsog_get_kbatch(b.ctx, s[3], i)
            assert (m == wants[i][e]).all(), f"system {i} evaluation {e}"


def test_device_chains_reject_host_sequences():
    c = W.c1_small()
    sysm = R.System(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=1, device_chains=2)
    for call in (lambda: sysm.sample_k(1), lambda: sysm.set_k(np.array([[1, 0, 0]], dtype=np.int32))):
        with pytest.raises(R.RbsogError) as e:
            call()
        assert e.value.status == -9
    # no sequence to run out of
    sysm.step(7, 1e-3)
    assert R.rbsog_info(sysm.ctx)["evaluations"] == 8


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, 1e-10), (R.RBSOG_FP32C, 1e-5)])
def test_device_chains_trajectory_matches_oracle(orc, prec, tol):
    # velocity Verlet driven by the device chains across three refills, with
    # graphs, against the oracle's run on the interleaved chain sequence
    n, L = 200, 10.0
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 21)
    v0 = W.maxwellian(n, 1.0, 22)
    rc, P, steps, dt, lam, seed = 3.0, 40, 9, 1e-3, 3, 13
    say(f"[gpu] device-chain trajectory prec={prec}")
    sysm = R.System(pos, q, box, rc, P, seed=seed, precision=prec, device_chains=lam)
    sog = oracle_sog(orc, sysm.sog)
    m = np.concatenate(expected_batches(orc, sog, box, seed, P, lam, steps + 1))
    R.rbsog_set_velocities(sysm.ctx, v0)
    sysm.step(steps, dt)
    assert (sysm.kbatch() == m[steps * P:]).all()
    x_g, v_g = R.rbsog_get_state(sysm.ctx, n)
    x_o, v_o, _, _ = orc.vv_run(pos, v0, q, box, rc, sog, P, m, steps, dt)
    dx = x_g - x_o
    dx -= box * np.round(dx / box)
    ex = float(np.abs(dx).max())
    ev = relrms(v_g - v0, v_o - v0)
    say(f"[device-chain vv prec={prec}] max|dx| {ex:.3e} velocity-change relrms {ev:.3e}")
    assert ex < tol * 10 and ev < tol * 10


def test_device_chains_graph_replay_equals_eager():
    n, L = 500, 12.0
    pos, q, box = W.ions_rsa(n, n / L ** 3, 1.0, 31)
    v0 = W.maxwellian(n, 1.0, 32)
    out = []
    for graphs in (False, True):
        say(f"[gpu] device-chain graph replay graphs={graphs}")
        sysm = R.System(pos, q, box, 3.0, 50, seed=3, precision=R.RBSOG_FP32C, graphs=graphs, device_chains=5)
        R.rbsog_set_velocities(sysm.ctx, v0)
        states = []
        for chunk in (4, 7, 3, 9):
            sysm.step(chunk, 1e-3)
            states.append(R.rbsog_get_state(sysm.ctx, n) + (sysm.kbatch(),))
        out.append(states)
        sysm.close()
    for a, b in zip(*out):
        for x, y in zip(a, b):
            assert (x == y).all()
