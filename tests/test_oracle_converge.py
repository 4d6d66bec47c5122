"""Pins of the convergence stop (Section 2: iterate until the L1 distance
between consecutive centres is below a threshold): a zero threshold never
stops early, the stopping iteration is the first whose residual, computed
here from independent fixed-count runs, is below the threshold, and the
residual itself is the exact quantised L1 sum."""
import numpy as np
import pytest

import oracle
import synth
from synth.configs import Workload


def _lab(w, h, seed):
    wl = Workload("conv", w, h, max(1, w * h // 500), 8.0, seed, 8)
    return oracle.rgb_to_lab(synth.image_for(wl))


def test_residual_is_the_quantised_l1_sum():
    rng = np.random.default_rng(0)
    a = rng.uniform(-50, 50, (7, 5)).astype(np.float32)
    b = (a + rng.normal(0, 0.3, a.shape)).astype(np.float32)
    want = sum(int(np.rint(abs(float(y) - float(x)) * 2 ** 18)) for x, y in zip(a.ravel(), b.ravel()))
    assert oracle.residual(a, b) == want
    assert oracle.residual(a, a) == 0


def test_zero_threshold_runs_every_iteration():
    lab = _lab(80, 60, 1)
    lb, cen, cnt, n = oracle.kmeans_converge(lab, 8, 10.0, True, 6, 0.0)
    lb6, cen6, cnt6 = oracle.kmeans(lab, 8, 10.0, True, 6)
    assert n == 6
    assert np.array_equal(lb, lb6) and np.array_equal(cen, cen6) and np.array_equal(cnt, cnt6)


@pytest.mark.parametrize("threshold", [0.05, 0.2, 1.0, 1e6])
def test_stop_is_the_first_iteration_below_threshold(threshold):
    lab = _lab(96, 72, 2)
    S, m = 8, 10.0
    K = 12 * 9
    limit = int(np.rint(threshold * 2 ** 18)) * K
    runs = [oracle.kmeans(lab, S, m, True, i) for i in range(0, 16)]
    want = 15
    for i in range(1, 16):
        prev, cur = runs[i - 1][1], runs[i][1]
        r = sum(int(np.rint(abs(float(y) - float(x)) * 2 ** 18))
                for x, y in zip(prev.ravel(), cur.ravel()))
        if r < limit:
            want = i
            break
    lb, cen, cnt, n = oracle.kmeans_converge(lab, S, m, True, 15, threshold)
    assert n == want
    assert np.array_equal(lb, runs[n][0]) and np.array_equal(cen, runs[n][1])
