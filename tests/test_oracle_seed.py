"""Pins of the oracle's grid (Section 2, S = sqrt(N/K); Section 3, the
ns_r x ns_c superpixel map) and seeding (Section 2, perturbation to the lowest
gradient position of a local neighbourhood)."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("w,h,S,K,expect", [
    (320, 240, 16, 0, (16, 20, 15)),
    (640, 480, 16, 0, (16, 40, 30)),
    (1920, 1080, 8, 0, (8, 240, 135)),
    (1920, 1080, 16, 0, (16, 120, 68)),
    (640, 480, 0, 1200, (16, 40, 30)),
    (1920, 1080, 0, 32400, (8, 240, 135)),
    (5, 3, 0, 1000, (1, 5, 3)),
    (7, 5, 100, 0, (100, 1, 1)),
])
def test_grid_closed_form(w, h, S, K, expect):
    assert oracle.grid(w, h, S, K) == expect


def test_grid_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.grid(0, 5, 4)
    with pytest.raises(ValueError):
        oracle.grid(5, 5, 0, 0)


def _uniform_lab(h, w, v=(50.0, 10.0, -20.0)):
    return tuple(np.full((h, w), c, np.float32) for c in v)


@pytest.mark.parametrize("w,h,S", [(64, 48, 16), (37, 29, 8), (5, 5, 2), (9, 4, 5)])
@pytest.mark.parametrize("perturb", [False, True])
def test_seeds_sit_in_cell_middles_on_a_flat_image(w, h, S, perturb):
    lab = _uniform_lab(h, w)
    cen = oracle.seed(lab, S, perturb)
    _, nc, nr = oracle.grid(w, h, S)
    for cy in range(nr):
        for cx in range(nc):
            x0, x1 = cx * S, min(cx * S + S, w)
            y0, y1 = cy * S, min(cy * S + S, h)
            c = cen[cy * nc + cx]
            assert c[3] == x0 + (x1 - x0 - 1) // 2 and c[4] == y0 + (y1 - y0 - 1) // 2
            assert tuple(c[:3]) == (50.0, 10.0, -20.0)


def _gradient64(lab, x, y):
    """Gradient of the cited SLIC paper, FP64, clamped coordinates."""
    L = np.stack(lab, -1).astype(np.float64)
    h, w = L.shape[:2]
    xl, xr = max(x - 1, 0), min(x + 1, w - 1)
    yu, yd = max(y - 1, 0), min(y + 1, h - 1)
    return float(((L[y, xr] - L[y, xl]) ** 2).sum() + ((L[yd, x] - L[yu, x]) ** 2).sum())


def test_planted_minimum_is_found():
    rng = np.random.default_rng(3)
    h, w, S = 32, 32, 8
    lab = tuple(rng.uniform(0, 100, (h, w)).astype(np.float32) for _ in range(3))
    # the seed of cell (1, 2) sits at (11, 19); make (12, 18) the only
    # flat spot of its window: its four neighbours share one colour
    for arr in lab:
        v = arr[18, 12]
        arr[18, 11] = arr[18, 13] = arr[17, 12] = arr[19, 12] = v
    assert oracle.gradient_at(lab, 12, 18) == 0.0
    cen = oracle.seed(lab, S, True)
    c = cen[2 * 4 + 1]
    assert (c[3], c[4]) == (12, 18)
    assert c[0] == lab[0][18, 12]
    assert tuple(oracle.seed(lab, S, False)[2 * 4 + 1][3:]) == (11, 19)


def test_gradient_definition_on_known_values():
    h, w = 4, 5
    L = np.arange(h * w, dtype=np.float32).reshape(h, w)
    A = np.zeros((h, w), np.float32)
    B = 2 * L
    # interior: horizontal difference 2 in L and 4 in B; vertical 10 and 20
    assert oracle.gradient_at((L, A, B), 2, 1) == pytest.approx(4 + 16 + 100 + 400)
    # clamped corner (0,0): horizontal L(1)-L(0) = 1, vertical L(5)-L(0) = 5
    assert oracle.gradient_at((L, A, B), 0, 0) == pytest.approx(1 + 4 + 25 + 100)


@pytest.mark.parametrize("seed", range(12))
def test_seed_perturbation_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    h, w = int(rng.integers(3, 30)), int(rng.integers(3, 30))
    S = int(rng.integers(1, 9))
    lab = tuple(rng.normal(50, 20, (h, w)).astype(np.float32) for _ in range(3))
    cen = oracle.seed(lab, S, True)
    _, nc, nr = oracle.grid(w, h, S)
    for cy in range(nr):
        for cx in range(nc):
            x0, x1 = cx * S, min(cx * S + S, w)
            y0, y1 = cy * S, min(cy * S + S, h)
            sx, sy = x0 + (x1 - x0 - 1) // 2, y0 + (y1 - y0 - 1) // 2
            win = [(sx + dx, sy + dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                   if 0 <= sx + dx < w and 0 <= sy + dy < h]
            g = {p: _gradient64(lab, *p) for p in win}
            gmin = min(g.values())
            c = cen[cy * nc + cx]
            pos = (int(c[3]), int(c[4]))
            assert pos in g
            assert g[pos] <= gmin * (1 + 1e-5) + 1e-3
            assert c[0] == lab[0][pos[1], pos[0]] and c[2] == lab[2][pos[1], pos[0]]
