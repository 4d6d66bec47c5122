"""Pins of the warm-start net oracle: its backward pass against central finite
differences (FP64), its forward pass against an independent evaluation built
on scipy's correlation, closed forms for zero weights and uniform logits,
bfloat16 rounding, and the class encoding of targets and decoded labels."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle


def _case(seed, w=7, h=6, S=4):
    rng = np.random.default_rng(seed)
    lab = (rng.uniform(0, 100, (h, w)).astype(np.float32),
           rng.uniform(-80, 80, (h, w)).astype(np.float32),
           rng.uniform(-80, 80, (h, w)).astype(np.float32))
    p = rng.normal(0, 0.3, oracle.net_param_count(S))
    target = rng.integers(0, 9, (h, w)).astype(np.int32)
    return lab, p, target, S


@pytest.mark.parametrize("seed", range(3))
def test_backward_matches_central_differences(seed):
    lab, p, target, S = _case(seed)
    origin = (5, 3)
    loss, g = oracle.net_loss_grad(lab, p, S, target, bf16_mode=False, origin=origin)
    off = oracle.net_offsets(S)
    rng = np.random.default_rng(100 + seed)
    idx = np.concatenate([rng.integers(off[a], off[b], 25) for a, b in
                          [("W1", "b1"), ("b1", "W2"), ("W2", "b2"), ("b2", "W3"), ("W3", "b3"),
                           ("b3", "P"), ("P", "end")]])
    gmax = np.abs(g).max()
    for i in idx:
        h = 1e-6
        q = p.copy()
        q[i] += h
        lp, _ = oracle.net_loss_grad(lab, q, S, target, False, origin, want_grad=False)
        q[i] -= 2 * h
        lm, _ = oracle.net_loss_grad(lab, q, S, target, False, origin, want_grad=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * gmax + 1e-9, (i, fd, g[i])


def _numpy_forward(lab, p, S, origin):
    """The net's forward in FP64 from scipy.ndimage.correlate (zero padding)."""
    off = oracle.net_offsets(S)
    L, A, B = lab
    h, w = L.shape
    x = np.stack([L / 100.0, A / 128.0, B / 128.0], 0).astype(np.float64)

    def conv(inp, W, b, cout):
        cin = inp.shape[0]
        W = W.reshape(9, cout, cin)
        out = np.zeros((cout, h, w))
        for o in range(cout):
            acc = np.full((h, w), b[o])
            for c in range(cin):
                k = W[:, o, c].reshape(3, 3)  # tap (dy+1)*3 + (dx+1)
                acc += ndimage.correlate(inp[c], k, mode="constant", cval=0.0)
            out[o] = acc
        return out

    a1 = np.maximum(conv(x, p[off["W1"]:off["b1"]], p[off["b1"]:off["W2"]], 32), 0)
    a2 = np.maximum(conv(a1, p[off["W2"]:off["b2"]], p[off["b2"]:off["W3"]], 32), 0)
    z = conv(a2, p[off["W3"]:off["b3"]], p[off["b3"]:off["P"]], 9)
    P = p[off["P"]:off["end"]].reshape(S * S, 9)
    yy, xx = np.mgrid[0:h, 0:w]
    ph = ((yy + origin[1]) % S) * S + (xx + origin[0]) % S
    return np.moveaxis(z, 0, -1) + P[ph]


@pytest.mark.parametrize("seed", range(3))
def test_forward_matches_scipy_correlation(seed):
    lab, p, _, S = _case(seed, w=9, h=5, S=3)
    origin = (2, 7)
    lg, _, _ = oracle.net_forward(lab, p, S, bf16_mode=False, origin=origin)
    ref = _numpy_forward(lab, p, S, origin)
    np.testing.assert_allclose(lg, ref, rtol=1e-12, atol=1e-12)


def test_bf16_rounding():
    assert oracle.bf16(1.0) == 1.0
    assert oracle.bf16(1.0 + 2 ** -8) == 1.0  # tie to even
    assert oracle.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert oracle.bf16(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    assert oracle.bf16(-2.5) == -2.5
    assert oracle.bf16(-(1.0 + 2 ** -7 + 2 ** -8)) == -(1.0 + 2 ** -6)  # tie to even


def test_zero_weights_give_bias_plus_phase():
    lab, p, _, S = _case(1, w=8, h=8, S=4)
    off = oracle.net_offsets(S)
    q = p.copy()
    q[off["W1"]:off["b1"]] = 0
    q[off["W2"]:off["b2"]] = 0
    q[off["W3"]:off["b3"]] = 0
    lg, _, _ = oracle.net_forward(lab, q, S, bf16_mode=True)
    P = q[off["P"]:off["end"]].reshape(S * S, 9)
    yy, xx = np.mgrid[0:8, 0:8]
    want = q[off["b3"]:off["P"]][None, None, :] + P[(yy % S) * S + xx % S]
    assert np.array_equal(lg, want)


def test_uniform_logits_give_log9():
    lab, p, target, S = _case(2)
    q = np.zeros_like(p)
    loss, g = oracle.net_loss_grad(lab, q, S, target)
    assert loss == pytest.approx(math.log(9), abs=1e-12)
    off = oracle.net_offsets(S)
    # d loss / d b3 = mean(softmax - onehot) = 1/9 - fraction of each class
    frac = np.bincount(target.ravel(), minlength=9) / target.size
    np.testing.assert_allclose(g[off["b3"]:off["P"]], 1 / 9 - frac, atol=1e-12)


def test_targets_and_decode_are_inverse():
    S, w, h = 4, 13, 10
    rng = np.random.default_rng(3)
    nc, nr = (w + S - 1) // S, (h + S - 1) // S
    yy, xx = np.mgrid[0:h, 0:w]
    cy = np.clip(yy // S + rng.integers(-1, 2, (h, w)), 0, nr - 1)
    cx = np.clip(xx // S + rng.integers(-1, 2, (h, w)), 0, nc - 1)
    labels = (cy * nc + cx).astype(np.int32)
    t = oracle.net_targets(labels, S)
    assert t.min() >= 0 and t.max() <= 8
    onehot = np.eye(9)[t]
    assert np.array_equal(oracle.net_decode(onehot, S), labels)
    grid = ((yy // S) * nc + xx // S).astype(np.int32)
    assert np.all(oracle.net_targets(grid, S) == 4)
    far = grid.copy()
    far[0, 0] = nc * nr - 1
    assert oracle.net_targets(far, S)[0, 0] == -1


def test_decode_clamps_at_the_border():
    S = 4
    lg = np.zeros((4, 4, 9))
    lg[..., 0] = 1.0  # up-left of cell (0, 0) does not exist
    assert np.all(oracle.net_decode(lg, S) == 0)


@pytest.mark.parametrize("tau", [0.2, 0.5, 0.7, 0.9])
def test_votes_closed_form(tau):
    """One class a above eight equal others: its softmax probability is
    e^a / (e^a + 8), at least tau exactly when a >= ln(8 tau / (1 - tau)),
    wherever the class sits and whatever the common offset."""
    edge = math.log(8 * tau / (1 - tau))
    rng = np.random.default_rng(int(tau * 10))
    h, w = 4, 9
    lg = np.zeros((h, w, 9))
    lg += rng.uniform(-3, 3, (h, w, 1))  # common offset: softmax ignores it
    best = rng.integers(0, 9, (h, w))
    lift = np.where(np.arange(w)[None, :] % 2 == 0, edge + 1e-7, edge - 1e-7) * np.ones((h, 1))
    lg[np.arange(h)[:, None], np.arange(w)[None, :], best] += lift
    want = np.arange(w)[None, :] % 2 == 0
    assert np.array_equal(oracle.net_votes(lg, tau), np.broadcast_to(want, (h, w)))


def test_votes_against_softmax():
    from scipy.special import softmax
    rng = np.random.default_rng(7)
    lg = rng.normal(0, 2, (30, 40, 9))
    pmax = softmax(lg, axis=-1).max(-1)
    for tau in (0.15, 0.3, 0.5, 0.8):
        got = oracle.net_votes(lg, tau)
        clear = np.abs(pmax - tau) > 1e-12
        assert np.array_equal(got[clear], pmax[clear] >= tau)
    assert oracle.net_votes(lg, 0.0).all()
    assert not oracle.net_votes(lg, 1.01).any()
