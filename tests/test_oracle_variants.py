"""Pins of the colour-space and distance options (the listing's colour
space setting; the cited SLIC paper's squared-sum distance): XYZ of white,
black and grey from the matrix and the sRGB curve, additivity of XYZ over
the primaries, RGB as the bytes themselves; the squared-sum association
against brute force over all centres within reach, and its agreement with
Eq. 1 where the two reduce to the same ordering (m = 0)."""
import numpy as np
import pytest

import oracle
import synth
from synth.configs import Workload


def _px(*rgb):
    return np.array([[list(c) for c in rgb]], np.uint8)


def test_xyz_white_black_grey():
    X, Y, Z = oracle.rgb_to_space(_px((255, 255, 255), (0, 0, 0), (128, 128, 128)),
                                  oracle.COLOR_XYZ)
    for v in (X, Y, Z):
        assert v[0, 0] == pytest.approx(100.0, abs=1e-4)
        assert v[0, 1] == 0.0
        # sRGB 128/255 decodes to ((128/255 + 0.055)/1.055)^2.4
        assert v[0, 2] == pytest.approx(100 * ((128 / 255 + 0.055) / 1.055) ** 2.4, rel=1e-5)


def test_xyz_is_additive_over_the_primaries():
    X, Y, Z = oracle.rgb_to_space(_px((255, 0, 0), (0, 255, 0), (0, 0, 255), (255, 255, 255)),
                                  oracle.COLOR_XYZ)
    for v in (X, Y, Z):
        assert v[0, 0] + v[0, 1] + v[0, 2] == pytest.approx(v[0, 3], abs=1e-4)
    # the Y row of the matrix sums to one: Y of the primaries are its entries
    assert Y[0, 0] == pytest.approx(21.26, abs=1e-3)
    assert Y[0, 1] == pytest.approx(71.52, abs=1e-3)
    assert Y[0, 2] == pytest.approx(7.22, abs=1e-3)


def test_rgb_space_is_the_bytes():
    img = np.random.default_rng(0).integers(0, 256, (7, 5, 3)).astype(np.uint8)
    R, G, B = oracle.rgb_to_space(img, oracle.COLOR_RGB)
    assert np.array_equal(R, img[..., 0].astype(np.float32))
    assert np.array_equal(G, img[..., 1].astype(np.float32))
    assert np.array_equal(B, img[..., 2].astype(np.float32))


def _lab(w, h, seed):
    wl = Workload("var", w, h, max(1, w * h // 300), 8.0, seed, 8)
    return oracle.rgb_to_lab(synth.image_for(wl))


@pytest.mark.parametrize("m", [0.0, 10.0, 40.0])
def test_squared_association_is_the_nearest_candidate(m):
    S = 6
    lab = _lab(40, 31, 5)
    rng = np.random.default_rng(2)
    _, nc, nr = oracle.grid(40, 31, S)
    cen = oracle.seed(lab, S, True)
    cen[:, :3] += rng.normal(0, 3, (cen.shape[0], 3)).astype(np.float32)
    lb = oracle.assign(lab, S, m, cen, oracle.DIST_SQUARED)
    L, A, B = lab
    wgt = np.float64(np.float32(m) / np.float32(S))
    for y in range(31):
        for x in range(40):
            cands = [(cy * nc + cx) for cy in range(y // S - 1, y // S + 2)
                     for cx in range(x // S - 1, x // S + 2) if 0 <= cy < nr and 0 <= cx < nc]
            c = cen[cands].astype(np.float64)
            d2 = ((c[:, 0] - L[y, x]) ** 2 + (c[:, 1] - A[y, x]) ** 2 + (c[:, 2] - B[y, x]) ** 2
                  + wgt ** 2 * ((c[:, 3] - x) ** 2 + (c[:, 4] - y) ** 2))
            best = d2.min()
            chosen = d2[cands.index(lb[y, x])]
            assert chosen <= best * (1 + 1e-5) + 1e-6, (x, y)


def test_squared_and_eq1_agree_without_the_spatial_term():
    lab = _lab(48, 40, 6)
    cen = oracle.seed(lab, 8, True)
    a = oracle.assign(lab, 8, 0.0, cen, oracle.DIST_EQ1)
    b = oracle.assign(lab, 8, 0.0, cen, oracle.DIST_SQUARED)
    assert (a == b).mean() > 0.999  # only FP32 near-ties may differ


def test_squared_energy_is_the_mean_root():
    lab = _lab(32, 24, 7)
    lb, cen, _ = oracle.kmeans(lab, 8, 10.0, True, 2, oracle.DIST_SQUARED)
    L, A, B = lab
    yy, xx = np.mgrid[0:24, 0:32]
    c = cen[lb].astype(np.float64)
    wgt = np.float64(np.float32(10.0) / np.float32(8))
    d = np.sqrt((c[..., 0] - L) ** 2 + (c[..., 1] - A) ** 2 + (c[..., 2] - B) ** 2
                + wgt ** 2 * ((c[..., 3] - xx) ** 2 + (c[..., 4] - yy) ** 2))
    assert oracle.energy(lab, 8, 10.0, cen, lb, oracle.DIST_SQUARED) == pytest.approx(d.mean(),
                                                                                       rel=1e-5)
