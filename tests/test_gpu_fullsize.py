"""Full-size workloads against the FP64 oracle on sampled outputs, and the
unbiasedness of the random-batch far force drawn by the library's sampler.

* 3,000,000-site water (10^6 rigid 3-site molecules, r_c = 10, P = 500): one
  evaluation in FP64 and FP32C; near and far forces of sampled sites computed
  one by one by the oracle (the far part with the oracle's own structure
  factors over all sites), U* from the oracle's rho.
* About 2e7 ions (r_c = 3.5, P = 1000): near forces of sampled ions, rho of
  sampled wave vectors, the exact zero sum of the random-batch far force, and
  momentum over velocity-Verlet steps.
* About 2e7 ions against stored oracle values (tests/golden/make_c5_far.py):
  the sampled wave vectors, every structure factor and the far force of
  1000 ions of one random batch; and the mean of many random batches drawn
  by the library against the oracle's full far field of those ions (every
  k != 0 through the Poisson identity): 300 batches here, 10,000 in the
  gpu_long test.
* Unbiasedness (Sec. 3.3, Lemma 1): the mean of many random-batch far forces
  drawn by the library equals the oracle's full Fourier sum."""
import os
import math
import sys
import time

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


def osog(orc, s):
    return orc.SOG(s.b, s.sigma, s.w0, s.M)


@pytest.fixture(scope="module")
def water():
    t0 = time.time()
    pos, q, box = W.water(100, 0.0334, seed=3)
    say(f"[water] {len(q)} sites, L={box[0]:.3f}, built in {time.time() - t0:.1f} s")
    return dict(pos=pos, q=q, box=box, rc=10.0, P=500)


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_water_3M_sampled_sites(orc, water, prec, tol):
    w = water
    n = len(w["q"])
    sysm = R.System(w["pos"], w["q"], w["box"], w["rc"], w["P"], seed=33, precision=prec)
    m = sysm.sample_k(1)
    t0 = time.time()
    F, E = sysm.forces()
    Fn, Ff = sysm.components()
    say(f"[water prec={prec}] evaluation + copies {time.time() - t0:.2f} s")
    rng = np.random.default_rng(30)
    tgt = np.sort(rng.choice(n, size=96, replace=False))
    sog = osog(orc, sysm.sog)
    Fn_o = orc.near_targets(w["pos"], w["q"], w["box"], w["rc"], sog, tgt)
    Ff_o, Us_o, _, _ = orc.far_rb(w["pos"], w["q"], w["box"], sog, m, w["P"], targets=tgt)
    e_n, e_f = relrms(Fn[tgt], Fn_o), relrms(Ff[tgt], Ff_o)
    e_u = abs(E[1] - Us_o) / abs(Us_o)
    say(f"[water prec={prec}] sampled relrms near {e_n:.3e} far {e_f:.3e}; U* rel {e_u:.3e}")
    assert e_n < tol and e_f < tol and e_u < 10 * tol
    sysm.close()


@pytest.fixture(scope="module")
def large():
    t0 = time.time()
    c = W.c5_large()
    say(f"[large] {len(c['q'])} ions, L={c['box'][0]:.3f}, built in {time.time() - t0:.1f} s")
    return c


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP32C, F32C_TOL), (R.RBSOG_FP64, F64_TOL)])
def test_20M_ions_sampled_and_invariants(orc, large, prec, tol):
    c = large
    n = len(c["q"])
    sysm = R.System(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=55, precision=prec)
    m = sysm.sample_k(6)
    t0 = time.time()
    F, E = sysm.forces()
    Fn, Ff = sysm.components()
    say(f"[large prec={prec}] evaluation + copies {time.time() - t0:.2f} s, E={E}")
    sog = osog(orc, sysm.sog)
    rng = np.random.default_rng(50)
    tgt = np.sort(rng.choice(n, size=48, replace=False))
    Fn_o = orc.near_targets(c["pos"], c["q"], c["box"], c["rc"], sog, tgt)
    e_n = relrms(Fn[tgt], Fn_o)
    # rho of sampled wave vectors of the batch
    ks = np.sort(rng.choice(c["P"], size=8, replace=False))
    re, im = R.rbsog_get_rho(sysm.ctx, c["P"])
    re_o, im_o = orc.structure_factor(c["pos"], c["q"], c["box"], m[:c["P"]][ks])
    e_rho = math.sqrt(float(np.sum((re[ks] - re_o) ** 2 + (im[ks] - im_o) ** 2))
                      / float(np.sum(re_o ** 2 + im_o ** 2)))
    # the random-batch far force sums to zero exactly: sum_i q_i Im(e^{-ik.r_i} rho) = Im(conj(rho) rho) = 0
    zsum = float(np.abs(Ff.sum(0)).max()) / float(np.abs(Ff).sum(0).max())
    say(f"[large prec={prec}] sampled near relrms {e_n:.3e}, rho relrms {e_rho:.3e}, far sum {zsum:.2e}")
    assert e_n < tol and e_rho < tol
    assert zsum < (1e-12 if prec == R.RBSOG_FP64 else 1e-6)
    # U_N over all 2e7 ions (the oracle's cell-list sum, pinned to brute
    # force on small systems): the near energies' partials are summed by
    # several blocks at this size
    t0 = time.time()
    _, Un_o = orc.near_cells(c["pos"], c["q"], c["box"], c["rc"], sog)
    e_un = abs(E[0] - Un_o) / abs(Un_o)
    say(f"[large prec={prec}] U_N rel {e_un:.3e} (oracle {time.time() - t0:.1f} s)")
    assert e_un < (1e-10 if prec == R.RBSOG_FP64 else 10 * tol)
    # velocity-Verlet: total momentum stays at its initial zero
    R.rbsog_set_velocities(sysm.ctx, None, T=1.0, seed=8)
    sysm.step(4, 1e-3)
    _, v = R.rbsog_get_state(sysm.ctx, n)
    p = float(np.abs(v.sum(0)).max()) / float(np.abs(v).sum(0).max())
    say(f"[large prec={prec}] momentum after 4 steps {p:.2e}")
    assert p < (1e-9 if prec == R.RBSOG_FP64 else 1e-6)
    # the kinetic energy the library sums (several blocks per system at this
    # size) against the host's sum of the returned velocities
    K, _ = R.rbsog_get_kinetic(sysm.ctx)
    K_h = 0.5 * float(np.sum(v * v))
    say(f"[large prec={prec}] kinetic rel {abs(K[0] - K_h) / K_h:.3e}")
    assert abs(K[0] - K_h) < 1e-11 * K_h
    sysm.close()


def test_random_batch_mean_is_full_sum(orc):
    # 1000 ions: the oracle's full Fourier sum (about 9,200 wave vectors) vs
    # the mean over 2000 random batches of P = 100 drawn by the library's chain
    c = W.c1_small()
    pos, q, box, rc, P = c["pos"], c["q"], c["box"], c["rc"], c["P"]
    sysm = R.System(pos, q, box, rc, P, seed=77, precision=R.RBSOG_FP64)
    sog = osog(orc, sysm.sog)
    Ffull, _, re, im = orc.far_full(pos, q, box, sog)
    B = 2000
    sysm.sample_k(B)
    acc = np.zeros((B, len(q), 3))
    t0 = time.time()
    for b in range(B):
        sysm.forces()
        acc[b] = sysm.components()[1]
    say(f"[unbiased] {B} random batches in {time.time() - t0:.1f} s")
    mean = acc.mean(0)
    sd = acc.std(0, ddof=1)
    z = (mean - Ffull) / (sd / math.sqrt(B))
    # Lemma 1 variance of one batch (independent draws) for comparison
    S = orc.S_product(sog, box)
    V = orc.volume(box)
    mk = orc.kvectors_full(sog, box)
    k = 2 * math.pi * mk / box
    Ft = sog.Ftilde_vec((k * k).sum(1))
    th = pos @ k.T
    imv = np.cos(th) * im[None, :] - np.sin(th) * re[None, :]
    var_pred = (math.pi ** 1.5 * S * q ** 2 / V ** 2 * np.sum(Ft[None, :] * (k * k).sum(1)[None, :] * imv ** 2, axis=1)
                - (Ffull ** 2).sum(1)) / P
    var_emp = ((acc - Ffull[None]) ** 2).sum(2).mean(0)
    ratio = float(((mean - Ffull) ** 2).sum()) / (float(var_emp.sum()) / B)
    vr = var_emp.sum() / var_pred.sum()
    say(f"[unbiased] max|z| {np.abs(z).max():.2f}, rms z {math.sqrt(float((z ** 2).mean())):.3f}, "
        f"error/expected {ratio:.2f}, batch variance / Lemma 1 (iid) {vr:.3f}")
    assert np.abs(z).max() < 5.5
    assert ratio < 6.0
    # the chain's states within a batch are correlated (repeated states after
    # rejections), which can only raise the variance above the iid value
    assert 0.9 < vr < 3.0
    sysm.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def c5_golden():
    """Stored oracle values of the 2e7-ion system (tests/golden/make_c5_far.py)."""
    sub = np.loadtxt(os.path.join(GOLDEN, "c5_far_subset.txt"))
    ids = sub[:, 0].astype(np.int64)
    batch_path = os.path.join(GOLDEN, "c5_rb_batch.txt")
    head = [ln for ln in open(batch_path) if ln.startswith("# Ustar")]
    batch = np.loadtxt(batch_path)
    return dict(ids=ids, F_full=sub[:, 1:4], F_rb=sub[:, 4:7], m=batch[:, :3].astype(np.int32),
                re=batch[:, 3], im=batch[:, 4], Ustar=float(head[0].split("=")[1]))


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_20M_far_force_of_one_batch_matches_stored_oracle(large, prec, tol):
    # the host chain keyed 55 gives the stored batch bit for bit; rho over
    # all 2e7 ions and the far force of the 1000 stored ions match the oracle
    c = large
    g = c5_golden()
    sysm = R.System(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=55, precision=prec)
    m = sysm.sample_k(1)
    assert np.array_equal(m, g["m"])
    _, E = R.rbsog_forces(sysm.ctx, len(c["q"]), want_forces=False)
    re, im = R.rbsog_get_rho(sysm.ctx, c["P"])
    e_rho = math.sqrt(float(np.sum((re - g["re"]) ** 2 + (im - g["im"]) ** 2))
                      / float(np.sum(g["re"] ** 2 + g["im"] ** 2)))
    _, Ff = R.rbsog_get_forces_subset(sysm.ctx, g["ids"])
    e_f = relrms(Ff, g["F_rb"])
    e_u = abs(E[1] - g["Ustar"]) / abs(g["Ustar"])
    say(f"[large prec={prec}] vs stored oracle: rho relrms {e_rho:.3e}, far force of 1000 ions {e_f:.3e}, "
        f"U* rel {e_u:.3e}")
    assert e_rho < tol and e_f < tol and e_u < 10 * tol
    sysm.close()


def mean_of_batches(c, g, draws, prec=R.RBSOG_FP32C):
    """Far force of the stored ions over `draws` random batches drawn by the
    library's device chains (64 chains: consecutive batches come from
    different chains), summed per batch on the host."""
    sysm = R.System(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=56, precision=prec, device_chains=64)
    acc = np.zeros((len(g["ids"]), 3))
    acc2 = np.zeros_like(acc)
    t0 = time.time()
    for b in range(draws):
        R.rbsog_forces(sysm.ctx, len(c["q"]), want_forces=False, want_energy=False)
        _, Ff = R.rbsog_get_forces_subset(sysm.ctx, g["ids"])
        acc += Ff
        acc2 += Ff * Ff
        if (b + 1) % 1000 == 0:
            say(f"[unbiased 2e7] {b + 1} batches, {time.time() - t0:.0f} s")
    sysm.close()
    mean = acc / draws
    var = (acc2 - draws * mean * mean) / (draws - 1)
    return mean, var


def check_unbiased(mean, var, draws, F_full, tag):
    se = np.sqrt(var / draws)
    z = (mean - F_full) / se
    rms_z = math.sqrt(float(np.mean(z * z)))
    err = math.sqrt(float(np.sum((mean - F_full) ** 2)))
    pred = math.sqrt(float(np.sum(var)) / draws)
    say(f"[{tag}] {draws} batches: rms z {rms_z:.3f}, max |z| {np.abs(z).max():.2f}, "
        f"|mean - full| / predicted standard error {err / pred:.2f}, relative error of the mean "
        f"{err / math.sqrt(float(np.sum(F_full ** 2))):.3e}")
    # C5 criteria: per-component z-scores with RMS in [0.8, 1.2] and max below
    # 5, and the error of the mean within 3 predicted standard errors
    assert 0.8 <= rms_z <= 1.2
    assert np.abs(z).max() < 5.0
    assert err <= 3.0 * pred


def test_20M_random_batch_mean_is_full_far_field(large):
    g = c5_golden()
    draws = 300
    mean, var = mean_of_batches(large, g, draws)
    check_unbiased(mean, var, draws, g["F_full"], "unbiased 2e7")
