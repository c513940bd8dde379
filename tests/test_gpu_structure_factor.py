"""The context-free structure factor (rbsog_structure_factor, Sec. 3.1 rho(k)
and the per-device reduction of Sec. 3.4) against the FP64 oracle, on device
arrays: ragged particle counts (one particle, a partial LDS batch, many
chunks), wave-vector counts that leave a partial tile, positions outside the
box (wrapped by the call), and agreement with the structure factors a context
computes for the same wave vectors."""
import math

import numpy as np
import pytest

from paper_2205_13824_amd import rbsog as R

from hipmem import DeviceArray
from paper_2205_13824_amd import workloads as W

pytestmark = pytest.mark.gpu

F64_TOL = 1e-11
F32C_TOL = 1e-5


def rho_err(re, im, re_o, im_o):
    return math.sqrt(float(np.sum((re - re_o) ** 2 + (im - im_o) ** 2)) / float(np.sum(re_o ** 2 + im_o ** 2)))


def device_sf(pos, q, box, m, prec):
    x = DeviceArray(np.ascontiguousarray(pos, dtype=np.float64))
    qd = DeviceArray(np.ascontiguousarray(q, dtype=np.float64))
    md = DeviceArray(np.ascontiguousarray(m, dtype=np.int32))
    nk = md.shape[0]
    re = DeviceArray(np.full(nk, np.nan))
    im = DeviceArray(np.full(nk, np.nan))
    R.rbsog_structure_factor(len(q), x.ptr, qd.ptr, box, nk, md.ptr, prec, re.ptr, im.ptr)
    return re.numpy(), im.numpy()


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
@pytest.mark.parametrize("n,nk,L", [(1, 1, 10.0), (2, 37, 10.0), (255, 256, 7.5), (257, 257, 12.0),
                                    (3001, 300, 20.0), (100_003, 1500, 46.0)])
def test_structure_factor_matches_oracle(orc, prec, tol, n, nk, L):
    rng = np.random.default_rng(n + nk)
    # positions partly outside [0, L): the call wraps them
    pos = rng.uniform(-1.5 * L, 2.5 * L, size=(n, 3))
    q = rng.choice([-1.0, 1.0, 0.4238, -0.8476], size=n)
    box = np.array([L, 0.9 * L, 1.1 * L])
    m = rng.integers(-40, 41, size=(nk, 3)).astype(np.int32)
    re, im = device_sf(pos, q, box, m, prec)
    re_o, im_o = orc.structure_factor(pos, q, box, m)
    err = rho_err(re, im, re_o, im_o)
    print(f"n={n} nk={nk} prec={prec}: rho relrms {err:.3e}", flush=True)
    assert np.all(np.isfinite(re)) and np.all(np.isfinite(im))
    assert err < tol


@pytest.mark.parametrize("prec,tol", [(R.RBSOG_FP64, F64_TOL), (R.RBSOG_FP32C, F32C_TOL)])
def test_structure_factor_matches_context(orc, prec, tol):
    c = W.c1_small()
    sysm = R.System(c["pos"], c["q"], c["box"], c["rc"], c["P"], seed=11, precision=prec)
    m = sysm.sample_k(1)
    sysm.forces()
    re_c, im_c = R.rbsog_get_rho(sysm.ctx, c["P"])
    re, im = device_sf(c["pos"], c["q"], c["box"], m, prec)
    err = rho_err(re, im, re_c, im_c)
    print(f"prec={prec}: stateless vs context rho relrms {err:.3e}", flush=True)
    assert err < tol
    sysm.close()


def test_structure_factor_rejects_bad_arguments():
    x = DeviceArray(np.zeros((4, 3)))
    q = DeviceArray(np.zeros(4))
    m = DeviceArray(np.ones((2, 3), dtype=np.int32))
    out = DeviceArray(np.zeros(2))
    for args, what in [((0, 2, [1.0, 1.0, 1.0], 0), "n"), ((4, 0, [1.0, 1.0, 1.0], 0), "n_k"),
                       ((4, 2, [1.0, 0.0, 1.0], 0), "box"), ((4, 2, [1.0, 1.0, 1.0], 7), "precision")]:
        n, nk, box, prec = args
        with pytest.raises(R.RbsogError) as e:
            R.rbsog_structure_factor(n, x.ptr, q.ptr, box, nk, m.ptr, prec, out.ptr, out.ptr)
        assert e.value.status == -1, what
