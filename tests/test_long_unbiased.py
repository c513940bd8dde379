"""Lemma 1 (Sec. 3.3) at the configured scale of the 2e7-ion system: the mean
of 10^4 random batches of P = 1000 wave vectors, drawn by the library's
device chains, on 1000 ions against the oracle's full far field of those ions
(stored by tests/golden/make_c5_far.py).  About four minutes of GPU time, so
it sits outside the gpu set: run it with -m gpu_long."""
import time

import pytest

from paper_2205_13824_amd import workloads as W

from test_gpu_fullsize import c5_golden, check_unbiased, mean_of_batches, say

pytestmark = pytest.mark.gpu_long


@pytest.fixture(scope="module")
def large():
    t0 = time.time()
    c = W.c5_large()
    say(f"[large] {len(c['q'])} ions, built in {time.time() - t0:.1f} s")
    return c


def test_20M_random_batch_mean_of_10000_batches_is_full_far_field(large):
    g = c5_golden()
    draws = 10_000
    mean, var = mean_of_batches(large, g, draws)
    check_unbiased(mean, var, draws, g["F_full"], "unbiased 2e7, 10^4 batches")
