"""The oracle's results do not depend on its thread count: the loops split
over OpenMP threads compute every value by the same operations, and the
centre sums are exact integers.  One thread and all threads must agree bit
for bit on the whole path, the update with votes and the net's logits."""
import os

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture
def all_threads():
    n = oracle.threads()
    yield max(2, os.cpu_count() or 2)
    oracle.threads(n)


def _both(fn, n):
    oracle.threads(1)
    one = fn()
    oracle.threads(n)
    many = fn()
    return one, many


@pytest.mark.parametrize("w,h,S,seed", [(320, 240, 16, 1), (203, 157, 7, 2)])
def test_segment_independent_of_threads(all_threads, w, h, S, seed):
    img = synth.voronoi_image(seed, w, h, 64, 8.0)
    one, many = _both(lambda: oracle.segment(img, S, 10.0, 4, True, True), all_threads)
    for k in ("labels", "centres", "counts", "seg_labels"):
        assert np.array_equal(one[k], many[k]), k
    for a, b in zip(one["lab"], many["lab"]):
        assert np.array_equal(a, b)
    assert one["energy"] == many["energy"] and one["n_segments"] == many["n_segments"]


def test_update_with_votes_independent_of_threads(all_threads):
    img = synth.voronoi_image(3, 160, 120, 32, 8.0)
    lab = oracle.rgb_to_lab(img)
    labels, cen, _ = oracle.kmeans(lab, 8, 10.0, True, 2)
    votes = (np.arange(labels.size).reshape(labels.shape) % 3 != 0).astype(np.uint8)
    one, many = _both(lambda: oracle.update(lab, labels, cen, votes), all_threads)
    assert np.array_equal(one[0], many[0]) and np.array_equal(one[1], many[1])


def test_net_forward_independent_of_threads(all_threads):
    rng = np.random.default_rng(4)
    S = 8
    lab = oracle.rgb_to_lab(synth.voronoi_image(4, 48, 40, 8, 8.0))
    p = rng.normal(0, 0.2, oracle.net_param_count(S))
    one, many = _both(lambda: oracle.net_forward(lab, p, S, True), all_threads)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)
