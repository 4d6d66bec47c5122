"""Pins of the oracle's RGB -> CIELAB conversion (Section 3, image space
conversion; Section 2, CIELAB as the colour part of the 5-D space)."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "srgb_lab_published.txt")


def _lab_of(colours):
    px = np.asarray(colours, np.uint8).reshape(1, -1, 3)
    L, A, B = oracle.rgb_to_lab(px)
    return np.stack([L[0], A[0], B[0]], axis=-1)


def test_white_is_exactly_100_0_0():
    lab = _lab_of([[255, 255, 255]])[0]
    assert lab[0] == np.float32(100.0) and lab[1] == 0.0 and lab[2] == 0.0


def test_black():
    lab = _lab_of([[0, 0, 0]])[0]
    assert abs(lab[0]) <= 1e-6 and lab[1] == 0.0 and lab[2] == 0.0


def test_published_colorimetry():
    rows = np.loadtxt(GOLDEN, comments="#")
    lab = _lab_of(rows[:, :3].astype(np.uint8))
    np.testing.assert_allclose(lab, rows[:, 3:], atol=0.05, rtol=0)


def test_neutral_axis():
    """Greys have no chroma, and their lightness is the CIE lightness of the
    sRGB-decoded luminance (a special case with a textbook closed form)."""
    v = np.arange(256)
    lab = _lab_of(np.stack([v, v, v], -1))
    assert np.all(np.abs(lab[:, 1]) <= 1e-4) and np.all(np.abs(lab[:, 2]) <= 1e-4)
    assert np.all(np.diff(lab[:, 0]) > 0), "lightness must increase with grey level"
    c = v / 255.0
    Y = np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)
    eps, kap = 216 / 24389, 24389 / 27
    Lstar = np.where(Y > eps, 116 * np.cbrt(Y) - 16, kap * Y)
    np.testing.assert_allclose(lab[:, 0], Lstar, atol=1e-4, rtol=0)


def test_cbrt_newton_against_library():
    rng = np.random.default_rng(0)
    t = np.concatenate([rng.uniform(216 / 24389, 1.1, 20000), np.geomspace(1e-300, 1e300, 2000)])
    got = np.array([oracle.cbrt(x) for x in t])
    ref = np.cbrt(t)
    assert np.all(np.abs(got - ref) <= 4 * np.spacing(ref))
    assert oracle.cbrt(1.0) == 1.0
    for x, r in [(8.0, 2.0), (0.125, 0.5), (27.0, 3.0), (0.001, 0.1)]:
        assert abs(oracle.cbrt(x) - r) <= np.spacing(r)


def _fp64_lab(rgb):
    """The conversion's definition evaluated in FP64 with numpy's cube root."""
    c = rgb.astype(np.float64) / 255.0
    lin = np.where(c <= 0.04045, c / 12.92, ((c + 0.055) / 1.055) ** 2.4)
    M = np.array([[0.4124, 0.3576, 0.1805], [0.2126, 0.7152, 0.0722], [0.0193, 0.1192, 0.9505]])
    xyz = lin @ (M / M.sum(axis=1, keepdims=True)).T
    eps, kap = 216 / 24389, 24389 / 27
    f = np.where(xyz > eps, np.cbrt(xyz), (kap * xyz + 16) / 116)
    return np.stack([116 * f[:, 1] - 16, 500 * (f[:, 0] - f[:, 1]), 200 * (f[:, 1] - f[:, 2])], -1)


def test_full_gamut_within_1e4_of_fp64_and_range():
    """All 2^24 colours: the FP32 evaluation stays within 1e-4 of the exact
    (FP64) value, and Lab stays inside the range that bounds the fixed-point
    centre sums (|v| < 108)."""
    lo = np.full(3, np.inf)
    hi = np.full(3, -np.inf)
    worst = 0.0
    for r0 in range(0, 256, 32):
        r, g, b = np.meshgrid(np.arange(r0, r0 + 32), np.arange(256), np.arange(256), indexing="ij")
        rgb = np.stack([r.ravel(), g.ravel(), b.ravel()], -1).astype(np.uint8)
        L, A, B = oracle.rgb_to_lab(rgb.reshape(1, -1, 3))
        lab = np.stack([L[0], A[0], B[0]], -1).astype(np.float64)
        worst = max(worst, float(np.abs(lab - _fp64_lab(rgb)).max()))
        lo = np.minimum(lo, lab.min(0))
        hi = np.maximum(hi, lab.max(0))
    assert worst <= 1e-4, worst
    assert lo[0] >= 0.0 and hi[0] <= 100.0
    assert -86.3 <= lo[1] and hi[1] <= 98.3 and -108.0 <= lo[2] and hi[2] <= 94.5
    assert max(abs(lo).max(), abs(hi).max()) < 108.0


@pytest.mark.parametrize("channels", [3, 4])
def test_pitch_and_channels(channels):
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, (7, 11, 3), dtype=np.uint8)
    ref = oracle.rgb_to_lab(img)
    padded = np.zeros((7, 11 * channels + 5), np.uint8)
    for x in range(11):
        padded[:, x * channels: x * channels + 3] = img[:, x]
    L = np.empty((7, 11), np.float32)
    A = np.empty_like(L)
    B = np.empty_like(L)
    lib = oracle._load()
    rc = lib.orc_rgb_to_lab(padded.ctypes.data, 11, 7, padded.shape[1], channels, L.ctypes.data,
                            A.ctypes.data, B.ctypes.data)
    assert rc == 0
    for u, v in zip(ref, (L, A, B)):
        assert np.array_equal(u, v)
