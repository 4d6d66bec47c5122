"""Pins of the oracle's association step (Eq. 1; Section 3: each pixel
examines at most nine cluster centres)."""
import numpy as np
import pytest

import oracle


def _random_case(rng, jitter=True):
    h, w = int(rng.integers(5, 49)), int(rng.integers(5, 49))
    S = int(rng.integers(1, 9))
    lab = tuple(rng.normal(50, 25, (h, w)).astype(np.float32) for _ in range(3))
    _, nc, nr = oracle.grid(w, h, S)
    cen = np.empty((nc * nr, 5), np.float32)
    for cy in range(nr):
        for cx in range(nc):
            x0, x1 = cx * S, min(cx * S + S, w)
            y0, y1 = cy * S, min(cy * S + S, h)
            k = cy * nc + cx
            cen[k, :3] = rng.normal(50, 25, 3)
            if jitter:  # anywhere inside its own cell
                cen[k, 3] = rng.uniform(x0, x1 - 1) if x1 - x0 > 1 else x0
                cen[k, 4] = rng.uniform(y0, y1 - 1) if y1 - y0 > 1 else y0
            else:
                cen[k, 3], cen[k, 4] = x0, y0
    return lab, S, cen, nc, nr


def _bruteforce_d64(lab, S, m, cen, nc, x, y):
    """Eq. 1 in FP64 for every centre whose cell is within one cell of the
    pixel's cell; other centres get +inf."""
    L, A, B = (np.float64(v[y, x]) for v in lab)
    c = cen.astype(np.float64)
    k = np.arange(len(c))
    kx, ky = k % nc, k // nc
    near = (np.abs(kx - x // S) <= 1) & (np.abs(ky - y // S) <= 1)
    dlab = np.sqrt((c[:, 0] - L) ** 2 + (c[:, 1] - A) ** 2 + (c[:, 2] - B) ** 2)
    dxy = np.sqrt((c[:, 3] - x) ** 2 + (c[:, 4] - y) ** 2)
    d = dlab + (m / S) * dxy
    return np.where(near, d, np.inf)


@pytest.mark.parametrize("seed", range(20))
@pytest.mark.parametrize("m", [0.0, 1.0, 10.0, 40.0])
def test_assignment_bruteforce(seed, m):
    rng = np.random.default_rng(seed)
    lab, S, cen, nc, nr = _random_case(rng)
    lb = oracle.assign(lab, S, m, cen)
    h, w = lb.shape
    for y in range(h):
        for x in range(w):
            d = _bruteforce_d64(lab, S, m, cen, nc, x, y)
            k = lb[y, x]
            assert np.isfinite(d[k]), "label outside the 3x3 neighbouring cells"
            dmin = d.min()
            assert d[k] <= dmin + 1e-5 * (1 + dmin)
            # ties (within FP32 noise) go to the lowest index
            near_min = np.flatnonzero(d <= dmin + 1e-5 * (1 + dmin))
            if len(near_min) == 1:
                assert k == near_min[0]


@pytest.mark.parametrize("w,h,S", [(64, 48, 16), (40, 24, 8), (12, 12, 3), (6, 4, 2), (5, 5, 1)])
@pytest.mark.parametrize("iters", [0, 1, 3])
def test_uniform_image_gives_the_grid(w, h, S, iters):
    """A flat image with S dividing W and H: every iteration labels the
    pixel with its own cell (closed form)."""
    lab = tuple(np.full((h, w), v, np.float32) for v in (40.0, -3.0, 7.5))
    for perturb in (False, True):
        lb, cen, cnt = oracle.kmeans(lab, S, 10.0, perturb, iters)
        y, x = np.mgrid[0:h, 0:w]
        assert np.array_equal(lb, (y // S) * (w // S) + x // S)


def test_m_zero_is_pure_colour_argmin():
    rng = np.random.default_rng(7)
    lab, S, cen, nc, nr = _random_case(rng)
    lb = oracle.assign(lab, S, 0.0, cen)
    h, w = lb.shape
    for y in range(h):
        for x in range(w):
            c = cen.astype(np.float64)
            d = np.sqrt(sum((c[:, j] - lab[j][y, x]) ** 2 for j in range(3)))
            k = np.arange(len(c))
            near = (np.abs(k % nc - x // S) <= 1) & (np.abs(k // nc - y // S) <= 1)
            d = np.where(near, d, np.inf)
            assert d[lb[y, x]] <= d.min() * (1 + 1e-6) + 1e-6


def test_large_m_is_spatial_voronoi_and_window_coverage():
    """With m huge the colour term is negligible; and while every centre lies
    in its own cell, every centre within Chebyshev distance S of a pixel is
    among its candidates, so the label is the spatially nearest of those."""
    rng = np.random.default_rng(11)
    for _ in range(10):
        lab, S, cen, nc, nr = _random_case(rng)
        lab = tuple(np.full_like(v, 50.0) for v in lab)
        cen[:, :3] = 50.0
        lb = oracle.assign(lab, S, 1e6, cen)
        h, w = lb.shape
        for y in range(h):
            for x in range(w):
                dxy = np.hypot(cen[:, 3].astype(np.float64) - x, cen[:, 4].astype(np.float64) - y)
                cheb = np.maximum(np.abs(cen[:, 3] - x), np.abs(cen[:, 4] - y))
                k = np.arange(len(cen))
                near = (np.abs(k % nc - x // S) <= 1) & (np.abs(k // nc - y // S) <= 1)
                assert np.all(near[cheb <= S]), "a centre within S is not a candidate"
                best = dxy[near].min()
                assert dxy[lb[y, x]] <= best * (1 + 1e-6) + 1e-6


def test_exact_ties_go_to_lowest_index():
    # two centres at the same colour and mirrored positions around a pixel
    h, w, S = 4, 8, 4
    lab = tuple(np.full((h, w), 30.0, np.float32) for _ in range(3))
    cen = np.array([[30, 30, 30, 1.5, 1.5], [30, 30, 30, 5.5, 1.5]], np.float32)
    lb = oracle.assign(lab, S, 10.0, cen)
    # pixels x=3 and x=4 are 1.5 and 2.5 from the centres: no tie; make one
    cen2 = np.array([[30, 30, 30, 2.0, 1.5], [30, 30, 30, 5.0, 1.5]], np.float32)
    lb2 = oracle.assign(lab, S, 10.0, cen2)
    assert lb2[1, 3] == 0 and lb2[1, 4] == 1
    cen3 = np.array([[30, 30, 30, 2.5, 1.0], [30, 30, 30, 4.5, 1.0]], np.float32)
    lb3 = oracle.assign(lab, S, 10.0, cen3)
    assert lb3[1, 3] == 0 and lb3[1, 4] == 1  # (3,1) is 0.5 from 2.5 and 1.5 from 4.5
    cen4 = np.array([[30, 30, 30, 2.0, 1.0], [30, 30, 30, 4.0, 1.0]], np.float32)
    lb4 = oracle.assign(lab, S, 10.0, cen4)
    assert lb4[1, 3] == 0, "equidistant pixel (3,1) must take the lower index"
    assert lb.min() >= 0


@pytest.mark.parametrize("seed", range(5))
def test_label_invariants(seed):
    rng = np.random.default_rng(50 + seed)
    lab, S, cen, nc, nr = _random_case(rng, jitter=False)
    lb = oracle.assign(lab, S, 10.0, cen)
    h, w = lb.shape
    assert lb.min() >= 0 and lb.max() < nc * nr
    y, x = np.mgrid[0:h, 0:w]
    assert np.all(np.abs(lb % nc - x // S) <= 1) and np.all(np.abs(lb // nc - y // S) <= 1)
