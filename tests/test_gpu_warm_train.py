"""Training of the warm-start net on the GPU (targets from plain SLIC's
labels after 10 rounds, crops of c5 training images): the loss falls, the
trained net predicts the converged cells better than the best predictor
that sees only the grid phase (measured on the same image), its warm start
beats the untrained net's at equal rounds, and, with the first update over
its confident pixels, plain SLIC's after as many associations.  The gate falls back to
plain SLIC whenever the warm energy exceeds 1.01 times plain's."""
import numpy as np
import pytest
import torch

import synth
from synth.configs import warm_eval_workload, warm_train_workload

pytestmark = pytest.mark.gpu
S = 16


@pytest.fixture(scope="module")
def slic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1509_04232_amd as slic
    return slic


def _rgb(wl):
    return torch.from_numpy(synth.image_for(wl).reshape(-1)).cuda()


@pytest.fixture(scope="module")
def trained(slic):
    imgs = []
    for j in range(64):
        wl = warm_train_workload(j)
        imgs.append((_rgb(wl), slic.Params(wl.width, wl.height, S=S, m=wl.m)))
    data = slic.warm.TrainingSet(imgs, 10)
    net = slic.warm.Net(S, 32, 128, 128, seed=1)
    untrained = net.params.clone()
    log = slic.warm.train(net, data, 1500, seed=2, log_every=100)
    return net, untrained, log


def _accuracy(slic, params, rgb, p):
    ctx = slic.Context(p, rgb)
    L, A, B = ctx.lab()
    ctx.iterate(10)
    lb = ctx.labels()
    ev = slic.warm.Net(S, 1, p.width, p.height, params=params.cpu().numpy())
    c = [slic.warm.crop(L, A, B, 0, 0, lb)]
    t = ev.targets(c)
    pred = ev.forward(c).argmax(-1)
    ok = t >= 0
    acc = float((pred[ok] == t[ok]).float().mean())
    # best phase-only predictor, fitted on this very image
    tt = t[0].cpu().numpy()
    yy, xx = np.mgrid[0:p.height, 0:p.width]
    ph = ((yy % S) * S + xx % S).ravel()
    cnt = np.zeros((S * S, 9))
    np.add.at(cnt, (ph[tt.ravel() >= 0], tt.ravel()[tt.ravel() >= 0]), 1)
    return acc, cnt.max(1).sum() / cnt.sum()


def test_loss_falls(trained):
    _, _, log = trained
    first, last = log[0][1], np.mean([v for _, v in log[-3:]])
    assert last < 0.6 * first, log


def test_trained_net_beats_the_phase_prior(slic, trained):
    net, _, _ = trained
    for j in range(2):
        wl = warm_eval_workload(j)
        p = slic.Params(wl.width, wl.height, S=S, m=wl.m)
        acc, prior = _accuracy(slic, net.params, _rgb(wl), p)
        assert acc > prior + 0.03, (acc, prior)


def test_training_improves_the_warm_start(slic, trained):
    net, untrained, _ = trained
    for j in range(2):
        wl = warm_eval_workload(j)
        rgb = _rgb(wl)
        p = slic.Params(wl.width, wl.height, S=S, m=wl.m)
        trained_net = slic.warm.prepare(net.params, S)
        untrained_net = slic.warm.prepare(untrained, S)
        e_t = float(slic.warm.warm_segment(rgb, p, trained_net, 2)["energy"].cpu()[0])
        e_u = float(slic.warm.warm_segment(rgb, p, untrained_net, 2)["energy"].cpu()[0])
        assert e_t < e_u, (e_t, e_u)


def test_confident_warm_start_beats_the_grid_seeds(slic, trained):
    """What the trained net gains over plain SLIC: with the first update
    taken over its confident pixels (best class at least 70% probable), two
    warm rounds end below plain SLIC after the same number of associations
    (the seeds' association and one round), on images it never saw."""
    net, _, _ = trained
    prepared = slic.warm.prepare(net.params, S, 0.7)
    for j in range(2):
        wl = warm_eval_workload(j)
        rgb = _rgb(wl)
        p = slic.Params(wl.width, wl.height, S=S, m=wl.m, perturb=wl.perturb)
        e_w = float(slic.warm.warm_segment(rgb, p, prepared, 2)["energy"].cpu()[0])
        e_p = float(slic.segment(rgb, p, 1, want_energy=True)["energy"].cpu()[0])
        assert e_w < e_p, (e_w, e_p)


def test_gate_falls_back_to_plain(slic, trained):
    net, _, _ = trained
    wl = warm_eval_workload(3)
    rgb = _rgb(wl)
    p = slic.Params(wl.width, wl.height, S=S, m=wl.m)
    plain = slic.segment(rgb, p, 10, want_energy=True)
    warm = slic.warm.warm_segment(rgb, p, slic.warm.prepare(net.params, S), 2)
    ep, ew = float(plain["energy"].cpu()[0]), float(warm["energy"].cpu()[0])
    out = warm if slic.warm.passes_gate(ew, ep) else plain
    e = float(out["energy"].cpu()[0])
    assert e <= 1.01 * ep
    assert (out is warm) == (ew <= 1.01 * ep)
