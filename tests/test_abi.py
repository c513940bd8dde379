"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/rbsog.h declares, and the host-side validation of rbsog_init returns
the documented status codes (these paths return before any device call)."""
import os
import re

import numpy as np
import pytest

from paper_2205_13824_amd import build as B
from paper_2205_13824_amd import rbsog as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(R.LIB_PATH):
        B.build()
    return R.lib()


def declared_functions():
    with open(os.path.join(ROOT, "include", "rbsog.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbsog_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(R.EXPORTS) == declared_functions()


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_table1_helper(lib):
    s = R.rbsog_sog_table1(2, 3.5)
    assert s.M == 16 and abs(s.sigma - 3.633717409009413 * 0.35) < 1e-15
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_sog_table1(6, 3.5)
    assert e.value.status == -1


def test_status_strings(lib):
    for code in R.STATUS:
        assert lib.rbsog_status_string(code)


def _system():
    pos = np.random.default_rng(0).random((8, 3)) * 10.0
    q = np.array([1, -1] * 4, dtype=np.float64)
    return pos, q, np.array([10.0, 10.0, 10.0])


@pytest.mark.parametrize("mutate,status", [
    (lambda a: a.update(q=np.array([1, -1] * 3 + [1, 0.5])), -2),        # not neutral
    (lambda a: a.update(rc=5.5), -3),                                      # rc > L/2
    (lambda a: a.update(rc=-1.0), -3),
    (lambda a: a.update(sog=R.rbsog_sog(1.0, 1.0, 1.0, 16)), -4),         # b <= 1
    (lambda a: a.update(sog=R.rbsog_sog(1.6, -1.0, 1.0, 16)), -4),        # sigma <= 0
    (lambda a: a.update(sog=R.rbsog_sog(1.6, 1.0, 1.0, -1)), -4),         # M < 0
    (lambda a: a.update(P=0), -1),
    (lambda a: a.update(box=np.array([10.0, 0.0, 10.0])), -1),
    (lambda a: a.update(pos=np.full((8, 3), np.nan)), -7),
    (lambda a: a.update(q=np.array([1, -1] * 3 + [np.inf, -1])), -7),
])
def test_init_validation(lib, mutate, status):
    pos, q, box = _system()
    a = dict(pos=pos, q=q, box=box, rc=3.0, P=10, sog=R.rbsog_sog_table1(2, 3.0))
    mutate(a)
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_init(a["pos"], a["q"], a["box"], a["sog"], a["rc"], a["P"], 1)
    assert e.value.status == status
    assert lib.rbsog_last_error(None)


def test_null_context_calls_fail_cleanly(lib):
    assert lib.rbsog_forces(None, None, None) == -1
    assert lib.rbsog_step(None, 1, 0.1) == -1
    lib.rbsog_destroy(None)


def test_option_and_batch_validation(lib):
    pos, q, box = _system()
    sog = R.rbsog_sog_table1(2, 3.0)
    # the core-shell table is an option of the FP32C form only
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_init(pos, q, box, sog, 3.0, 10, 1, precision=R.RBSOG_FP64, near_table=True)
    assert e.value.status == -1
    # a batch names the system that fails validation
    q_bad = np.array([1, -1] * 3 + [1, 0.5])
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_init_batch([pos, pos], [q, q_bad], [box, box], [sog, sog], [3.0, 3.0], [10, 10], [1, 2])
    assert e.value.status == -2 and "system 1" in str(e.value)
    with pytest.raises(R.RbsogError) as e:
        R.rbsog_init_batch([pos, pos[:1]], [q, q[:1]], [box, box], [sog, sog], [3.0, 3.0], [10, 10], [1, 2])
    assert e.value.status == -1
    # the near-list skin is a fraction of r_c in [0, 1]
    for skin in (-0.1, 1.5, float("nan")):
        with pytest.raises(R.RbsogError) as e:
            R.rbsog_init(pos, q, box, sog, 3.0, 10, 1, skin=skin)
        assert e.value.status == -1 and "skin" in str(e.value)
    assert R.rbsog_default_opts().skin == 0.1
    # the number of device chains is bounded
    for lam in (-1, 4097):
        with pytest.raises(R.RbsogError) as e:
            R.rbsog_init(pos, q, box, sog, 3.0, 10, 1, device_chains=lam)
        assert e.value.status == -1 and "device_chains" in str(e.value)
