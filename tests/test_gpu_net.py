"""The warm-start net on the GPU against the oracle: forward logits and the
loss gradient (relative L2 error at most 1e-2, the scale of bfloat16
rounding of activations), training targets (exact), the Adam step (its
definition in float64), and the warm-started segmentation against the
oracle's composition of seeding, decoding, the confidence votes of the
first update and (update, associate) rounds (exact labels and centres)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth.configs import Workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1509_04232_amd as slic
    return slic


def _image(w, h, seed):
    wl = Workload("net", w, h, max(1, w * h // 600), 8.0, seed, 8)
    img = synth.image_for(wl)
    return img, oracle.rgb_to_lab(img)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _random_params(S, seed, conv_scale=1.0):
    """He-scaled random convolution weights, random biases and phase bias."""
    rng = np.random.default_rng(seed)
    off = oracle.net_offsets(S)
    p = rng.normal(0.0, 1.0, off["end"])
    p[off["W1"]:off["b1"]] *= np.sqrt(2 / 27) * conv_scale
    p[off["W2"]:off["b2"]] *= np.sqrt(2 / 288) * conv_scale
    p[off["W3"]:off["b3"]] *= np.sqrt(2 / 288) * conv_scale
    p[off["b1"]:off["W2"]] *= 0.1
    p[off["b2"]:off["W3"]] *= 0.1
    p[off["b3"]:off["P"]] *= 0.1
    p[off["P"]:off["end"]] *= 0.5
    return p.astype(np.float32)


def _rel_l2(got, want):
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-30))


# crops of 70 x 45 (two conv tiles across with a ragged tail, 12 tile rows,
# 2 x 2 weight-gradient strips, 3 loss blocks); the second runs past the
# image's right and bottom edges
CW, CH = 70, 45
CROPS = [(0, 0, 0), (0, 40, 30), (1, 13, 7)]


def _setup(slic, S, seed):
    imgs = [_image(97, 61, 11 + seed), _image(150, 90, 12 + seed)]
    dev = [tuple(_dev(v) for v in lab) for _, lab in imgs]
    crops = [slic.warm.crop(*dev[i], ox=ox, oy=oy) for i, ox, oy in CROPS]
    return imgs, dev, crops


def _region(lab, ox, oy):
    return tuple(v[oy:oy + CH, ox:ox + CW] for v in lab)


@pytest.mark.parametrize("S,seed", [(8, 0), (5, 1), (16, 2)])
def test_forward_matches_oracle(slic, S, seed):
    imgs, dev, crops = _setup(slic, S, seed)
    p = _random_params(S, 100 + seed)
    net = slic.warm.Net(S, len(crops), CW, CH, params=p)
    lg = net.forward(crops).cpu().numpy()
    for i, (j, ox, oy) in enumerate(CROPS):
        reg = _region(imgs[j][1], ox, oy)
        want, _, _ = oracle.net_forward(reg, p.astype(np.float64), S, True, origin=(ox, oy))
        rh, rw = reg[0].shape
        got = lg[i, :rh, :rw]
        assert _rel_l2(got, want) <= 1e-2, (i, _rel_l2(got, want))
        assert np.abs(got - want).max() <= 0.05 * np.abs(want).max()


@pytest.mark.parametrize("S,seed", [(8, 0), (16, 1)])
def test_loss_and_gradient_match_oracle(slic, S, seed):
    imgs, dev, crops = _setup(slic, S, seed)
    p = _random_params(S, 200 + seed)
    rng = np.random.default_rng(300 + seed)
    target = rng.integers(-1, 9, (len(CROPS), CH, CW)).astype(np.int32)
    for i, (j, ox, oy) in enumerate(CROPS):  # no targets beyond the image
        h, w = imgs[j][1][0].shape
        target[i, max(0, h - oy):, :] = -1
        target[i, :, max(0, w - ox):] = -1
    net = slic.warm.Net(S, len(crops), CW, CH, params=p)
    loss = float(net.loss_grad(crops, _dev(target)).cpu()[0])
    grad = net.grad.cpu().numpy().astype(np.float64)
    total, want_loss, want_grad = 0, 0.0, np.zeros(p.size)
    for i, (j, ox, oy) in enumerate(CROPS):
        reg = _region(imgs[j][1], ox, oy)
        rh, rw = reg[0].shape
        t = np.ascontiguousarray(target[i, :rh, :rw])
        n = int((t >= 0).sum())
        li, gi = oracle.net_loss_grad(reg, p.astype(np.float64), S, t, True, origin=(ox, oy))
        total += n
        want_loss += li * n
        want_grad += gi * n
    want_loss /= total
    want_grad /= total
    assert abs(loss - want_loss) <= 1e-2 * want_loss
    off = oracle.net_offsets(S)
    for a, b in [("W1", "b1"), ("b1", "W2"), ("W2", "b2"), ("b2", "W3"), ("W3", "b3"),
                 ("b3", "P"), ("P", "end")]:
        e = _rel_l2(grad[off[a]:off[b]], want_grad[off[a]:off[b]])
        assert e <= 1e-2, (a, e)


def test_gradient_is_deterministic(slic):
    imgs, dev, crops = _setup(slic, 8, 3)
    p = _random_params(8, 7)
    target = np.random.default_rng(8).integers(0, 9, (len(CROPS), CH, CW)).astype(np.int32)
    net = slic.warm.Net(8, len(crops), CW, CH, params=p)
    t = _dev(target)
    net.loss_grad(crops, t)
    g1 = net.grad.clone()
    net.loss_grad(crops, t)
    assert torch.equal(g1, net.grad)


def test_targets_match_oracle(slic):
    S = 8
    img, lab = _image(130, 77, 21)
    labels, _, _ = oracle.kmeans(lab, S, 10.0, True, 3)
    L, A, B = (_dev(v) for v in lab)
    lt = _dev(labels)
    spec = [(0, 0), (50, 40), (129, 76)]
    crops = [slic.warm.crop(L, A, B, ox=ox, oy=oy, labels=lt) for ox, oy in spec]
    net = slic.warm.Net(S, len(crops), 64, 48)
    got = net.targets(crops).cpu().numpy()
    full = oracle.net_targets(labels, S)
    for i, (ox, oy) in enumerate(spec):
        want = np.full((48, 64), -1, np.int32)
        reg = full[oy:oy + 48, ox:ox + 64]
        want[:reg.shape[0], :reg.shape[1]] = reg
        assert np.array_equal(got[i], want), i


def test_adam_step_matches_its_definition(slic):
    rng = np.random.default_rng(5)
    n = 1000
    p, g = rng.normal(0, 1, n), rng.normal(0, 1e-2, n)
    m, v = rng.normal(0, 1e-2, n), rng.uniform(0, 1e-4, n)
    lr, b1, b2, eps, step = 3e-3, 0.9, 0.999, 1e-8, 4
    t = [_dev(a.astype(np.float32)) for a in (p, g, m, v)]
    slic.slic_net_adam(t[0].data_ptr(), t[1].data_ptr(), t[2].data_ptr(), t[3].data_ptr(), n,
                       step, lr, b1, b2, eps, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    f = [a.astype(np.float32).astype(np.float64) for a in (p, g, m, v)]
    m2 = b1 * f[2] + (1 - b1) * f[1]
    v2 = b2 * f[3] + (1 - b2) * f[1] ** 2
    p2 = f[0] - lr * (m2 / (1 - b1 ** step)) / (np.sqrt(v2 / (1 - b2 ** step)) + eps)
    np.testing.assert_allclose(t[2].cpu().numpy(), m2, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(t[3].cpu().numpy(), v2, rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(t[0].cpu().numpy(), p2, rtol=1e-5, atol=1e-6)


def _decisive_params(S, seed):
    """Small random convolutions and a phase bias with one class 4 above the
    rest at every phase, so every pixel's argmax is far from a tie."""
    rng = np.random.default_rng(seed)
    p = _random_params(S, seed, conv_scale=0.05)
    off = oracle.net_offsets(S)
    P = rng.uniform(-1.0, 1.0, (S * S, 9))
    P[np.arange(S * S), rng.integers(0, 9, S * S)] = 5.0
    p[off["P"]:off["end"]] = P.ravel()
    p[off["b3"]:off["P"]] = 0.0
    return p


# S = 2 and 1: a tile's window of cells is too large for the input region, so
# the fused kernel keeps the decode bins in the first hidden layer's region
@pytest.mark.parametrize("w,h,S,perturb,iters", [
    (97, 61, 8, True, 2), (130, 77, 5, False, 3), (64, 64, 16, True, 1), (150, 90, 8, True, 0),
    (33, 17, 4, True, 4), (70, 45, 2, True, 2), (41, 23, 1, False, 1)])
def test_warm_segment_matches_oracle(slic, w, h, S, perturb, iters):
    img, lab = _image(w, h, 40 + S)
    p = _decisive_params(S, 50 + w)
    lg, _, _ = oracle.net_forward(lab, p.astype(np.float64), S, True)
    top2 = np.sort(lg, axis=-1)[..., -2:]
    assert (top2[..., 1] - top2[..., 0]).min() > 1.0  # no near-ties to break differently
    labels = oracle.net_decode(lg, S)
    cen = oracle.seed(lab, S, perturb)
    for _ in range(iters):
        cen, _ = oracle.update(lab, labels, cen)
        labels = oracle.assign(lab, S, 10.0, cen)
    energy = oracle.energy(lab, S, 10.0, cen, labels)

    prm = slic.Params(w, h, S=S, m=10.0, perturb=perturb)
    net = slic.warm.prepare(_dev(p), S)
    out = slic.warm.warm_segment(_dev(img.reshape(-1)), prm, net, iters, want_centres=True)
    torch.cuda.synchronize()
    assert np.array_equal(out["labels"].cpu().numpy(), labels)
    assert np.array_equal(out["centres"].cpu().numpy(), cen)
    assert float(out["energy"].cpu()[0]) == pytest.approx(energy, rel=1e-9)


@pytest.mark.parametrize("w,h,S,perturb,iters", [
    (97, 61, 8, True, 2), (130, 77, 5, False, 3), (64, 64, 16, True, 1), (150, 90, 8, True, 0),
    (70, 45, 2, True, 2)])
def test_warm_segment_with_connectivity_matches_oracle(slic, w, h, S, perturb, iters):
    """The warm start with the clean-up: with rounds its last association
    also finds the tile-local components; the labels after the clean-up
    equal the oracle's connectivity step on the oracle's composition."""
    img, lab = _image(w, h, 40 + S)
    p = _decisive_params(S, 50 + w)
    lg, _, _ = oracle.net_forward(lab, p.astype(np.float64), S, True)
    top2 = np.sort(lg, axis=-1)[..., -2:]
    assert (top2[..., 1] - top2[..., 0]).min() > 1.0
    labels = oracle.net_decode(lg, S)
    cen = oracle.seed(lab, S, perturb)
    for _ in range(iters):
        cen, _ = oracle.update(lab, labels, cen)
        labels = oracle.assign(lab, S, 10.0, cen)
    seg, n_seg, _ = oracle.connectivity(labels, S, 0)

    prm = slic.Params(w, h, S=S, m=10.0, perturb=perturb)
    net = slic.warm.prepare(_dev(p), S)
    out = slic.warm.warm_segment(_dev(img.reshape(-1)), prm, net, iters, enforce=True,
                                 want_centres=True)
    torch.cuda.synchronize()
    assert np.array_equal(out["labels"].cpu().numpy(), seg)
    assert int(out["n_segments"].cpu()[0]) == n_seg
    assert np.array_equal(out["centres"].cpu().numpy(), cen)


def _two_level_params(S, seed):
    """Like _decisive_params, but at every other phase the leading class is
    only 2.5 above the rest: those pixels' best class is far less probable,
    so a confidence threshold splits the pixels with a wide margin."""
    p = _decisive_params(S, seed)
    off = oracle.net_offsets(S)
    P = p[off["P"]:off["end"]].reshape(S * S, 9)
    P[1::2] = np.where(P[1::2] == 5.0, 2.5, P[1::2])
    return p


@pytest.mark.parametrize("w,h,S,perturb,iters", [
    (97, 61, 8, True, 2), (130, 77, 5, False, 3), (64, 64, 16, True, 1), (150, 90, 8, True, 0),
    (33, 17, 4, True, 4), (70, 45, 2, True, 2)])
def test_warm_segment_with_votes_matches_oracle(slic, w, h, S, perturb, iters):
    """A minimum confidence between the two levels: only the confident
    pixels vote in the first update, exactly as the oracle's composition
    (decode, votes, update over the voters, then plain rounds)."""
    img, lab = _image(w, h, 40 + S)
    p = _two_level_params(S, 50 + w)
    lg, _, _ = oracle.net_forward(lab, p.astype(np.float64), S, True)
    top2 = np.sort(lg, axis=-1)[..., -2:]
    assert (top2[..., 1] - top2[..., 0]).min() > 1.0
    log_se = np.log(np.exp(lg - lg.max(-1, keepdims=True)).sum(-1))
    cut = 0.2  # the votes' threshold in log-mass: tau = exp(-cut)
    assert np.abs(log_se - cut).min() > 0.05  # no pixel near it
    tau = float(np.exp(-cut))
    votes = oracle.net_votes(lg, tau)
    assert 0.2 < votes.mean() < 0.8
    labels = oracle.net_decode(lg, S)
    cen = oracle.seed(lab, S, perturb)
    for it in range(iters):
        cen, _ = oracle.update(lab, labels, cen, votes if it == 0 else None)
        labels = oracle.assign(lab, S, 10.0, cen)
    energy = oracle.energy(lab, S, 10.0, cen, labels)

    prm = slic.Params(w, h, S=S, m=10.0, perturb=perturb)
    net = slic.warm.prepare(_dev(p), S, tau)
    out = slic.warm.warm_segment(_dev(img.reshape(-1)), prm, net, iters, want_centres=True)
    torch.cuda.synchronize()
    assert np.array_equal(out["labels"].cpu().numpy(), labels)
    assert np.array_equal(out["centres"].cpu().numpy(), cen)
    assert float(out["energy"].cpu()[0]) == pytest.approx(energy, rel=1e-9)


@pytest.mark.parametrize("w,h,S,seed", [(97, 61, 8, 0), (200, 130, 16, 1), (45, 33, 3, 2)])
def test_warm_start_without_voters_is_plain_slic_one_round_shorter(slic, w, h, S, seed):
    """Above 1 no pixel is confident enough: the first update keeps every
    seed, so n warm rounds equal plain SLIC's n - 1 rounds exactly."""
    img, _ = _image(w, h, 70 + seed)
    rgb = _dev(img.reshape(-1))
    prm = slic.Params(w, h, S=S, m=10.0)
    net = slic.warm.prepare(_dev(_random_params(S, 75 + seed)), S, 1.5)
    for n in (1, 2, 3):
        warm = slic.warm.warm_segment(rgb, prm, net, n, want_centres=True)
        plain = slic.segment(rgb, prm, n - 1, want_centres=True, want_energy=True)
        assert torch.equal(warm["labels"], plain["labels"])
        assert torch.equal(warm["centres"], plain["centres"])
        assert torch.equal(warm["energy"], plain["energy"])


@pytest.mark.parametrize("w,h,S,seed", [(97, 61, 8, 0), (200, 130, 16, 1), (45, 33, 3, 2)])
def test_fused_decode_matches_oracle_away_from_ties(slic, w, h, S, seed):
    """Full random weights: the fused net's decoded labels (zero rounds)
    equal the oracle's wherever the oracle's best logit leads the second by
    more than the bf16 error scale; elsewhere they name one of its two best
    classes."""
    img, lab = _image(w, h, 80 + seed)
    p = _random_params(S, 90 + seed)
    lg, _, _ = oracle.net_forward(lab, p.astype(np.float64), S, True)
    order = np.argsort(-lg, axis=-1, kind="stable")
    top = np.take_along_axis(lg, order[..., :2], axis=-1)
    margin = top[..., 0] - top[..., 1]
    prm = slic.Params(w, h, S=S, m=10.0)
    net = slic.warm.prepare(_dev(p), S)
    got = slic.warm.warm_segment(_dev(img.reshape(-1)), prm, net, 0)["labels"].cpu().numpy()
    want = oracle.net_decode(lg, S)
    clear = margin > 0.02 * np.abs(lg).max()
    assert clear.mean() > 0.8
    assert np.array_equal(got[clear], want[clear])
    second = np.zeros_like(lg)
    second[np.arange(h)[:, None], np.arange(w)[None, :], order[..., 1]] = 1.0
    alt = oracle.net_decode(second, S)
    assert np.all((got == want) | (got == alt))


def test_warm_context_resumes_and_enforces(slic):
    w, h, S = 120, 80, 8
    img, lab = _image(w, h, 61)
    p = slic.warm.prepare(_dev(_decisive_params(S, 62)), S)
    prm = slic.Params(w, h, S=S, m=10.0)
    rgb = _dev(img.reshape(-1))
    one = slic.warm.warm_segment(rgb, prm, p, 3, enforce=True)
    ctx = slic.Context(prm, rgb, net=p)
    ctx.iterate(1).iterate(2)
    split = ctx.labels()
    n = ctx.enforce_connectivity()
    seg = ctx.labels()
    torch.cuda.synchronize()
    plain3 = slic.warm.warm_segment(rgb, prm, p, 3)["labels"]
    assert torch.equal(split, plain3)
    want, ns, _ = oracle.connectivity(split.cpu().numpy(), S)
    assert np.array_equal(seg.cpu().numpy(), want)
    assert int(n.cpu()[0]) == ns == int(one["n_segments"].cpu()[0])
    assert torch.equal(one["labels"], seg)
    ctx.close()


def test_net_rejects_bad_arguments(slic):
    from paper_1509_04232_amd import _abi
    with pytest.raises(_abi.SlicError):
        _abi.slic_net_param_count(33)
    with pytest.raises(_abi.SlicError):
        _abi.slic_net_workspace_bytes(33, 16, 16, 8)
    img, lab = _image(40, 30, 70)
    L, A, B = (_dev(v) for v in lab)
    net = slic.warm.Net(8, 1, 16, 16)
    with pytest.raises(_abi.SlicError):  # origin outside the image
        net.forward([slic.warm.crop(L, A, B, ox=40, oy=0)])
    with pytest.raises(_abi.SlicError):  # host memory
        host = torch.zeros(40 * 30, dtype=torch.float32)
        bad = _abi.SlicNetCrop(host.data_ptr(), A.data_ptr(), B.data_ptr(), None, 40, 30, 0, 0)
        net.forward([bad])
    with pytest.raises(_abi.SlicError):  # targets need labels
        net.targets([slic.warm.crop(L, A, B)])
    with pytest.raises(_abi.SlicError):  # the net's phase table stops at S = 32
        _abi.slic_warm_workspace_bytes(slic.Params(200, 200, S=40).c())
    prm = slic.Params(40, 30, S=8)
    rgb = _dev(img.reshape(-1))
    with pytest.raises(_abi.SlicError):  # prepared net in host memory
        slic.warm.warm_segment(rgb, prm, torch.zeros(_abi.slic_net_prepared_bytes(),
                                                     dtype=torch.uint8), 2)
    with pytest.raises(_abi.SlicError):  # S beyond the phase table
        _abi.slic_net_prepare(33, net.params.data_ptr(), 0.0, net.ws.data_ptr(), 0)
    with pytest.raises(ValueError):  # parameter count of another S
        slic.warm.prepare(net.params, 16)
    buf = torch.empty(_abi.slic_net_prepared_bytes(), dtype=torch.uint8, device="cuda")
    for bad in (-0.1, float("nan"), float("inf")):  # minimum confidence
        with pytest.raises(_abi.SlicError):
            slic.warm.prepare(net.params, 8, bad, out=buf)


def test_prepared_net_is_bound_to_its_step(slic):
    """A net prepared for one S is rejected for a frame of another S (its
    phase bias is indexed with the frame's S), and a buffer that
    slic_net_prepare never filled is rejected too; re-preparing the same
    buffer for the frame's S makes it valid."""
    from paper_1509_04232_amd import _abi
    img, _ = _image(96, 64, 72)
    rgb = _dev(img.reshape(-1))
    net16 = slic.warm.prepare(_dev(_random_params(16, 73)), 16)
    prm8 = slic.Params(96, 64, S=8, m=10.0)
    with pytest.raises(_abi.SlicError) as e:
        slic.warm.warm_segment(rgb, prm8, net16, 1)
    assert e.value.code == _abi.SLIC_EINVAL
    with pytest.raises(_abi.SlicError):
        slic.Context(prm8, rgb, net=net16)
    never = torch.zeros(_abi.slic_net_prepared_bytes(), dtype=torch.uint8, device="cuda")
    with pytest.raises(_abi.SlicError):
        slic.warm.warm_segment(rgb, prm8, never, 1)
    slic.warm.prepare(_dev(_random_params(8, 74)), 8, out=net16)
    out = slic.warm.warm_segment(rgb, prm8, net16, 1)
    torch.cuda.synchronize()
    assert int(out["labels"].min()) >= 0
