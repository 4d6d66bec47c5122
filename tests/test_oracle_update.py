"""Pins of the oracle's centre update (Section 3, updating the cluster
centre: each centre becomes the mean [l a b x y] of its pixels) and of the
loop of Section 4's listing."""
from fractions import Fraction

import numpy as np
import pytest

import oracle

Q = oracle.qshift()


def _exact_centre(values, qshift):
    """Exact rational mean of the fixed-point colour values, rounded to
    FP64, scaled back and rounded to FP32; coordinates likewise."""
    q = [round(Fraction(float(v)) * 2 ** qshift) for v in values]  # half-to-even
    mean = float(Fraction(sum(q), len(q)))  # correctly rounded
    return np.float32(mean * 2.0 ** -qshift)


@pytest.mark.parametrize("seed", range(6))
def test_update_is_the_exact_mean(seed):
    rng = np.random.default_rng(seed)
    h, w, S = int(rng.integers(4, 20)), int(rng.integers(4, 20)), int(rng.integers(1, 6))
    lab = tuple(rng.normal(40, 30, (h, w)).astype(np.float32) for _ in range(3))
    _, nc, nr = oracle.grid(w, h, S)
    K = nc * nr
    labels = rng.integers(0, K, (h, w)).astype(np.int32)
    old = rng.normal(0, 1, (K, 5)).astype(np.float32)
    cen, cnt = oracle.update(lab, labels, old)
    assert cnt.sum() == h * w
    assert np.array_equal(cnt, np.bincount(labels.ravel(), minlength=K))
    y, x = np.mgrid[0:h, 0:w]
    for k in range(K):
        sel = labels == k
        if not sel.any():
            assert np.array_equal(cen[k], old[k]), "an empty cluster keeps its centre"
            continue
        for j in range(3):
            assert cen[k, j] == _exact_centre(lab[j][sel], Q)
        assert cen[k, 3] == np.float32(float(Fraction(int(x[sel].sum()), int(sel.sum()))))
        assert cen[k, 4] == np.float32(float(Fraction(int(y[sel].sum()), int(sel.sum()))))


@pytest.mark.parametrize("seed", range(3))
def test_update_over_voting_pixels_is_their_exact_mean(seed):
    """The warm start's first update: only pixels with a vote count; a
    cluster without one keeps its centre; all votes give the plain update."""
    rng = np.random.default_rng(50 + seed)
    h, w, S = 11, 14, 3
    lab = tuple(rng.normal(40, 30, (h, w)).astype(np.float32) for _ in range(3))
    _, nc, nr = oracle.grid(w, h, S)
    K = nc * nr
    labels = rng.integers(0, K, (h, w)).astype(np.int32)
    votes = rng.random((h, w)) < 0.4
    old = rng.normal(0, 1, (K, 5)).astype(np.float32)
    cen, cnt = oracle.update(lab, labels, old, votes)
    assert np.array_equal(cnt, np.bincount(labels[votes], minlength=K))
    y, x = np.mgrid[0:h, 0:w]
    for k in range(K):
        sel = (labels == k) & votes
        if not sel.any():
            assert np.array_equal(cen[k], old[k])
            continue
        for j in range(3):
            assert cen[k, j] == _exact_centre(lab[j][sel], Q)
        assert cen[k, 3] == np.float32(float(Fraction(int(x[sel].sum()), int(sel.sum()))))
        assert cen[k, 4] == np.float32(float(Fraction(int(y[sel].sum()), int(sel.sum()))))
    all_c, all_n = oracle.update(lab, labels, old, np.ones((h, w), bool))
    plain_c, plain_n = oracle.update(lab, labels, old)
    assert np.array_equal(all_c, plain_c) and np.array_equal(all_n, plain_n)
    none_c, none_n = oracle.update(lab, labels, old, np.zeros((h, w), bool))
    assert np.array_equal(none_c, old) and not none_n.any()


def test_fixed_point_rounds_half_to_even():
    # 2^-19 and 3*2^-19 are exactly halfway between fixed-point steps
    h, w = 1, 2
    half = np.float32(2.0 ** -(Q + 1))
    for vals, expect in [((half, half), 0.0), ((3 * half, 3 * half), 2.0 ** -Q * 2)]:
        lab = (np.array([vals], np.float32), np.zeros((h, w), np.float32),
               np.zeros((h, w), np.float32))
        cen, _ = oracle.update(lab, np.zeros((h, w), np.int32), np.zeros((1, 5), np.float32))
        assert cen[0, 0] == np.float32(expect)


@pytest.mark.parametrize("w,h,S", [(64, 48, 16), (40, 24, 8), (15, 9, 3), (7, 5, 7)])
def test_uniform_image_centres_land_on_cell_middles(w, h, S):
    """Closed form: on a flat image each full cell's centre becomes
    x0 + (S-1)/2 after the first update and then stays fixed."""
    lab = tuple(np.full((h, w), v, np.float32) for v in (60.0, 5.0, -5.0))
    for iters in (1, 2, 4):
        lb, cen, cnt = oracle.kmeans(lab, S, 10.0, True, iters)
        _, nc, nr = oracle.grid(w, h, S)
        for cy in range(nr):
            for cx in range(nc):
                x0, x1 = cx * S, min(cx * S + S, w)
                y0, y1 = cy * S, min(cy * S + S, h)
                c = cen[cy * nc + cx]
                assert c[3] == np.float32((x0 + x1 - 1) / 2) and c[4] == np.float32((y0 + y1 - 1) / 2)
                assert cnt[cy * nc + cx] == (x1 - x0) * (y1 - y0)
                assert tuple(c[:3]) == (60.0, 5.0, -5.0)


@pytest.mark.parametrize("a,b", [(0, 3), (2, 3), (4, 1)])
def test_loop_composes(a, b):
    """Section 4's listing: kmeans(a+b) equals kmeans(a) followed by b more
    (update, associate) rounds."""
    rng = np.random.default_rng(a * 10 + b)
    h, w, S, m = 30, 41, 6, 10.0
    lab = tuple(rng.normal(50, 20, (h, w)).astype(np.float32) for _ in range(3))
    lb, cen, cnt = oracle.kmeans(lab, S, m, True, a)
    for _ in range(b):
        cen, cnt = oracle.update(lab, lb, cen)
        lb = oracle.assign(lab, S, m, cen)
    lb2, cen2, cnt2 = oracle.kmeans(lab, S, m, True, a + b)
    assert np.array_equal(lb, lb2) and np.array_equal(cen, cen2) and np.array_equal(cnt, cnt2)


def test_zero_iterations_is_one_association_with_the_seeds():
    rng = np.random.default_rng(5)
    h, w, S = 20, 20, 5
    lab = tuple(rng.normal(50, 20, (h, w)).astype(np.float32) for _ in range(3))
    lb, cen, cnt = oracle.kmeans(lab, S, 10.0, True, 0)
    seeds = oracle.seed(lab, S, True)
    assert np.array_equal(cen, seeds) and not cnt.any()
    assert np.array_equal(lb, oracle.assign(lab, S, 10.0, seeds))
