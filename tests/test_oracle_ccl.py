"""Pins of the oracle's connectivity clean-up (Section 2: connectivity is
enforced to clean up the final lattice) under the canonical merge rule, and
of its energy (mean Eq. 1 distance)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle

FOUR = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]])


def _reference_merge(labels, S, min_segment):
    """Independent statement of the rule: components from scipy's labelling,
    then the joins resolved by following them."""
    h, w = labels.shape
    comp = np.full((h, w), -1, np.int64)
    for v in np.unique(labels):
        cc, n = ndimage.label(labels == v, structure=FOUR)
        for j in range(1, n + 1):
            idx = np.flatnonzero(cc.ravel() == j)
            comp.ravel()[idx] = idx.min()
    flat = comp.ravel()
    roots = sorted(set(flat.tolist()))
    size = {r: int((flat == r).sum()) for r in roots}

    def small(r):
        return size[r] < min_segment if min_segment > 0 else 4 * size[r] < S * S

    def final(r):
        while r != 0 and small(r):
            r = int(flat[r - 1] if r % w else flat[r - w])
        return r

    fin = {r: final(r) for r in roots}
    kept = sorted(set(fin.values()))
    rank = {r: i for i, r in enumerate(kept)}
    out = np.array([rank[fin[int(r)]] for r in flat], np.int32).reshape(h, w)
    return out, len(kept)


def _random_labels(rng, h, w, n):
    # blobs plus speckle so that small components occur
    base = rng.integers(0, n, ((h + 3) // 4, (w + 3) // 4))
    lb = np.kron(base, np.ones((4, 4), np.int64))[:h, :w]
    speckle = rng.random((h, w)) < 0.15
    lb[speckle] = rng.integers(0, n, speckle.sum())
    return lb.astype(np.int32)


@pytest.mark.parametrize("seed", range(40))
def test_matches_independent_statement(seed):
    rng = np.random.default_rng(seed)
    h, w = int(rng.integers(1, 25)), int(rng.integers(1, 25))
    S = int(rng.integers(1, 9))
    ms = int(rng.choice([0, 0, 1, 3, 10]))
    lb = _random_labels(rng, h, w, int(rng.integers(1, 6)))
    out, ns, sc = oracle.connectivity(lb, S, ms)
    ref, nref = _reference_merge(lb, S, ms)
    assert ns == nref
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("seed", range(15))
def test_invariants(seed):
    rng = np.random.default_rng(1000 + seed)
    h, w, S = int(rng.integers(8, 40)), int(rng.integers(8, 40)), int(rng.integers(2, 8))
    lb = _random_labels(rng, h, w, 4)
    out, ns, sc = oracle.connectivity(lb, S, 0)
    assert out.min() == 0 and out.max() == ns - 1
    # numbered in order of first raster appearance
    _, first = np.unique(out.ravel(), return_index=True)
    assert np.all(np.diff(first) > 0)
    for s in range(ns):
        sel = out == s
        _, n = ndimage.label(sel, structure=FOUR)
        assert n == 1, "segment is not 4-connected"
        if not sel.ravel()[0]:
            assert 4 * sel.sum() >= S * S, "small segment survived"
        # the segment's cluster is the input label at its first pixel
        assert sc[s] == lb.ravel()[first[s]]


@pytest.mark.parametrize("w,h,S", [(64, 48, 16), (40, 24, 8), (9, 6, 3)])
def test_grid_labels_are_unchanged(w, h, S):
    y, x = np.mgrid[0:h, 0:w]
    lb = ((y // S) * (w // S) + x // S).astype(np.int32)
    out, ns, sc = oracle.connectivity(lb, S, 0)
    assert ns == (w // S) * (h // S) and np.array_equal(out, lb)


def test_single_pixel_and_all_small():
    out, ns, _ = oracle.connectivity(np.zeros((1, 1), np.int32), 4, 0)
    assert ns == 1 and out[0, 0] == 0
    checker = (np.indices((6, 6)).sum(0) % 2).astype(np.int32)
    out, ns, _ = oracle.connectivity(checker, 4, 0)  # every component has 1 pixel
    assert ns == 1 and not out.any()


@pytest.mark.parametrize("seed", range(5))
def test_energy_is_the_mean_eq1_distance(seed):
    rng = np.random.default_rng(seed)
    h, w, S, m = 17, 23, 5, 10.0
    lab = tuple(rng.normal(50, 20, (h, w)).astype(np.float32) for _ in range(3))
    lb, cen, cnt = oracle.kmeans(lab, S, m, True, 2)
    e = oracle.energy(lab, S, m, cen, lb)
    c = cen.astype(np.float64)[lb]
    y, x = np.mgrid[0:h, 0:w]
    dlab = np.sqrt(sum((c[..., j] - lab[j]) ** 2 for j in range(3)))
    dxy = np.sqrt((c[..., 3] - x) ** 2 + (c[..., 4] - y) ** 2)
    ref = float(np.mean(dlab + (m / S) * dxy))
    assert abs(e - ref) <= 1e-6 * ref
