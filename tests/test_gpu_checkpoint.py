"""Checkpoint and resume (rbsog_save_state / rbsog_load_state): a run saved
after 13 steps and resumed in a fresh context continues bit for bit as the
uninterrupted run of 33 steps does (Algorithm 1: the wave-vector sequence is
consumed in order, so its sampler state and cursor are part of the state).
Covered: the host chain and the device chains, velocity Verlet, the Langevin
and the Nose-Hoover thermostats, the mean-square displacement, the near list
(skin 0.1, list passes between builds) and building at every step (skin 0),
both precisions, and a batch of systems; 13 steps ends between graphs of
eight steps."""
import numpy as np
import pytest

from paper_2205_13824_amd import rbsog as R
from paper_2205_13824_amd import workloads as W

pytestmark = pytest.mark.gpu

DT = 2e-3


def system():
    pos, q, box = W.ions_rsa(2000, 0.1, 1.0, seed=31)
    return pos, q, box


def make(mode, prec, skin):
    pos, q, box = system()
    chains = 16 if mode in ("chains", "nh") else 0
    return R.System(pos, q, box, 3.5, 40, seed=77, precision=prec, skin=skin, device_chains=chains)


def setup(sysm, mode):
    if mode in ("host", "langevin", "msd"):
        sysm.sample_k(60)
    sysm.forces()
    R.rbsog_set_velocities(sysm.ctx, None, T=2.0, seed=5)
    if mode == "langevin":
        R.rbsog_set_thermostat(sysm.ctx, 2.0, 1.5, seed=9)
    if mode == "nh":
        R.rbsog_set_nose_hoover(sysm.ctx, 1.5, 0.2)
    if mode == "msd":
        R.rbsog_set_msd_origin(sysm.ctx)


def snapshot(sysm, mode):
    n = sysm.n
    x, v = R.rbsog_get_state(sysm.ctx, n)
    Fn, Ff = R.rbsog_get_forces(sysm.ctx, n)
    E = R.rbsog_get_energy(sysm.ctx)
    K, xi = R.rbsog_get_kinetic(sysm.ctx)
    info = R.rbsog_info(sysm.ctx)
    out = dict(x=x, v=v, Fn=Fn, Ff=Ff, E=E, K=K, xi=xi, kbatch=R.rbsog_get_kbatch(sysm.ctx, sysm.P),
               builds=info["list_builds"], evals=info["evaluations"], left=info["k_remaining"])
    if mode == "msd":
        out["msd"] = R.rbsog_get_msd(sysm.ctx)
    return out


def assert_identical(a, b, what):
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), f"{what}: {k} differs"


@pytest.mark.parametrize("mode,prec,skin", [
    ("host", R.RBSOG_FP64, 0.1), ("host", R.RBSOG_FP32C, 0.1), ("chains", R.RBSOG_FP32C, 0.1),
    ("chains", R.RBSOG_FP64, 0.0), ("langevin", R.RBSOG_FP32C, 0.1), ("nh", R.RBSOG_FP64, 0.1),
    ("msd", R.RBSOG_FP32C, 0.0)])
def test_resume_continues_bit_for_bit(mode, prec, skin):
    ref = make(mode, prec, skin)
    setup(ref, mode)
    ref.step(33, DT)
    want = snapshot(ref, mode)
    ref.close()

    a = make(mode, prec, skin)
    setup(a, mode)
    a.step(13, DT)
    state = R.rbsog_save_state(a.ctx)
    a.step(20, DT)
    assert_identical(snapshot(a, mode), want, "run split in 13 + 20 steps")
    a.close()

    b = make(mode, prec, skin)  # fresh context: its own initial positions, no velocities
    R.rbsog_load_state(b.ctx, state)
    b.step(20, DT)
    got = snapshot(b, mode)
    print(f"mode={mode} prec={prec} skin={skin}: state {len(state)} bytes, builds {got['builds']}", flush=True)
    assert_identical(got, want, "resumed run")
    # the same state loaded again into the same context rewinds it
    R.rbsog_load_state(b.ctx, state)
    b.step(20, DT)
    assert_identical(snapshot(b, mode), want, "second resume")
    b.close()


def test_resume_of_a_batch():
    ens = [W.ions_rsa(n, 0.1, 1.0, seed=40 + i) for i, n in enumerate((600, 1500, 900))]

    def mk():
        return R.Batch([e[0] for e in ens], [e[1] for e in ens], [e[2] for e in ens], 3.5, 30, [1, 2, 3],
                       precision=R.RBSOG_FP32C, device_chains=8)

    ref = mk()
    ref.forces()
    R.rbsog_set_velocities(ref.ctx, None, T=1.0, seed=4)
    ref.step(21, DT)
    want = R.rbsog_get_state(ref.ctx, ref.n)
    ref.close()
    a = mk()
    a.forces()
    R.rbsog_set_velocities(a.ctx, None, T=1.0, seed=4)
    a.step(9, DT)
    state = R.rbsog_save_state(a.ctx)
    a.close()
    b = mk()
    R.rbsog_load_state(b.ctx, state)
    b.step(12, DT)
    got = R.rbsog_get_state(b.ctx, b.n)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    b.close()


def test_state_of_another_context_is_refused():
    a = make("host", R.RBSOG_FP64, 0.1)
    setup(a, "host")
    state = R.rbsog_save_state(a.ctx)
    pos, q, box = W.ions_rsa(1000, 0.1, 1.0, seed=3)
    other = R.System(pos, q, box, 3.5, 40, seed=77)
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_load_state(other.ctx, state)
    assert e.value.status == -1
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_load_state(a.ctx, state[: len(state) // 2])
    assert e.value.status == -1
    with pytest.raises(R.RbsogError):
        R.rbsog_load_state(a.ctx, b"not a state")
    other.close()
    a.close()
