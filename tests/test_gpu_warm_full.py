"""The fused warm-start kernel at the sizes the warm start is evaluated on,
against the oracle's composition (seed, decode the oracle's logits, votes,
rounds of update and association).  At 640x480 the frame has 1,200 tiles
of 32x8 pixels and at 1920x1080 8,100, more than the persistent grid's
workgroups (two per compute unit), so every workgroup walks several tiles
and loads the next tile's input while it computes the current one, and the
last round of tiles is ragged."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth.configs import warm_eval_workload
from test_gpu_net import _decisive_params, _dev, _random_params, _two_level_params

pytestmark = pytest.mark.gpu

TILE_W, TILE_H, PER_CU = 32, 8, 2


@pytest.fixture(scope="module")
def slic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1509_04232_amd as slic
    return slic


def _tiles_per_workgroup(w, h):
    tiles = -(-w // TILE_W) * -(-h // TILE_H)
    grid = min(tiles, PER_CU * torch.cuda.get_device_properties(0).multi_processor_count)
    return tiles, grid


def _composition(lab, lg, S, perturb, iters, votes=None):
    labels = oracle.net_decode(lg, S)
    cen = oracle.seed(lab, S, perturb)
    for it in range(iters):
        cen, _ = oracle.update(lab, labels, cen, votes if it == 0 else None)
        labels = oracle.assign(lab, S, 10.0, cen)
    return labels, cen, oracle.energy(lab, S, 10.0, cen, labels)


def _check(out, labels, cen, energy):
    got = out["labels"].cpu().numpy()
    assert np.array_equal(got, labels), f"{(got != labels).sum()} labels differ"
    assert np.array_equal(out["centres"].cpu().numpy(), cen), "centres differ"
    assert float(out["energy"].cpu()[0]) == pytest.approx(energy, rel=1e-9)


@pytest.mark.parametrize("hd,iters", [(False, 2), (False, 0), (True, 1)])
def test_full_size_warm_segment_matches_oracle(slic, hd, iters):
    wl = warm_eval_workload(1, hd)
    w, h, S = wl.width, wl.height, wl.S
    tiles, grid = _tiles_per_workgroup(w, h)
    assert tiles > 2 * grid and tiles % grid != 0  # several tiles each, ragged last round
    print(f"warm full size {w}x{h} S={S} rounds={iters}: {tiles} tiles on {grid} workgroups",
          flush=True)
    img = synth.image_for(wl)
    lab = oracle.rgb_to_lab(img)
    p = _decisive_params(S, 500 + w)
    lg, _, _ = oracle.net_forward(lab, p.astype(np.float64), S, True)
    top2 = np.sort(lg, axis=-1)[..., -2:]
    assert (top2[..., 1] - top2[..., 0]).min() > 1.0  # no near-ties to break differently
    labels, cen, energy = _composition(lab, lg, S, True, iters)
    prm = slic.Params(w, h, S=S, m=10.0, perturb=True)
    net = slic.warm.prepare(_dev(p), S)
    out = slic.warm.warm_segment(_dev(img.reshape(-1)), prm, net, iters, want_centres=True)
    torch.cuda.synchronize()
    _check(out, labels, cen, energy)


def test_full_size_votes_match_oracle(slic):
    """640x480 with a minimum confidence between the two levels of the phase
    bias: only the confident pixels vote in the first update."""
    wl = warm_eval_workload(2)
    w, h, S = wl.width, wl.height, wl.S
    print(f"warm votes {w}x{h} S={S}", flush=True)
    img = synth.image_for(wl)
    lab = oracle.rgb_to_lab(img)
    p = _two_level_params(S, 600)
    lg, _, _ = oracle.net_forward(lab, p.astype(np.float64), S, True)
    top2 = np.sort(lg, axis=-1)[..., -2:]
    assert (top2[..., 1] - top2[..., 0]).min() > 1.0
    log_se = np.log(np.exp(lg - lg.max(-1, keepdims=True)).sum(-1))
    cut = 0.2
    assert np.abs(log_se - cut).min() > 0.05  # no pixel near the threshold
    tau = float(np.exp(-cut))
    votes = oracle.net_votes(lg, tau)
    assert 0.2 < votes.mean() < 0.8
    labels, cen, energy = _composition(lab, lg, S, True, 3, votes)
    prm = slic.Params(w, h, S=S, m=10.0, perturb=True)
    net = slic.warm.prepare(_dev(p), S, tau)
    out = slic.warm.warm_segment(_dev(img.reshape(-1)), prm, net, 3, want_centres=True)
    torch.cuda.synchronize()
    _check(out, labels, cen, energy)


@pytest.mark.parametrize("hd", [False, True])
def test_full_size_fused_decode_away_from_ties(slic, hd):
    """Random full-scale weights, zero rounds: the decoded labels equal the
    oracle's wherever its best logit leads the second by more than the bf16
    error scale, and name one of its two best classes elsewhere."""
    wl = warm_eval_workload(3, hd)
    w, h, S = wl.width, wl.height, wl.S
    print(f"warm decode {w}x{h} S={S}", flush=True)
    img = synth.image_for(wl)
    lab = oracle.rgb_to_lab(img)
    p = _random_params(S, 700 + w)
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
