"""Video warm start: a frame initialised from the previous frame's centres
(slic_init_from_centres) against the oracle's composition of association
and update rounds from the same centres (exact), and the energy a chain of
warm-started frames of a shaking camera reaches within two rounds."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth.configs import Workload, video_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1509_04232_amd as slic
    return slic


def _frames(w, h, n, shake, seed):
    canvas, origins = video_workload(n, w, h, shake, seed)
    img = synth.image_for(canvas)
    return [np.ascontiguousarray(img[oy:oy + h, ox:ox + w]) for ox, oy in origins]


@pytest.mark.parametrize("w,h,S,rounds", [(160, 120, 16, 0), (160, 120, 16, 1), (131, 77, 8, 3),
                                          (97, 45, 5, 2)])
def test_init_from_centres_matches_oracle(slic, w, h, S, rounds):
    f0, f1 = _frames(w, h, 2, 2, 600 + w)
    lab0, lab1 = oracle.rgb_to_lab(f0), oracle.rgb_to_lab(f1)
    _, prev, _ = oracle.kmeans(lab0, S, 10.0, True, 10)
    cen = prev.copy()
    labels = oracle.assign(lab1, S, 10.0, cen)
    for _ in range(rounds):
        cen, _ = oracle.update(lab1, labels, cen)
        labels = oracle.assign(lab1, S, 10.0, cen)
    p = slic.Params(w, h, S=S, m=10.0)
    ctx = slic.Context(p, torch.from_numpy(f1.reshape(-1)).cuda(),
                       centres=torch.from_numpy(prev).cuda())
    ctx.iterate(rounds)
    got_lb = ctx.labels()
    got_cen, _ = ctx.centres()
    torch.cuda.synchronize()
    assert np.array_equal(got_lb.cpu().numpy(), labels)
    assert np.array_equal(got_cen.cpu().numpy(), cen)
    ctx.close()


def test_shaking_sequence_reaches_plain_energy_in_two_rounds(slic):
    frames = _frames(640, 480, 8, 2, 5_000_000)
    p = slic.Params(640, 480, S=16, m=10.0)
    prev = None
    for t, f in enumerate(frames):
        rgb = torch.from_numpy(f.reshape(-1)).cuda()
        plain = slic.segment(rgb, p, 10, want_energy=True)
        if prev is None:
            ctx = slic.Context(p, rgb)
            ctx.iterate(10)
        else:
            ctx = slic.Context(p, rgb, centres=prev)
            ctx.iterate(2)
        e = float(ctx.energy().cpu()[0])
        prev, _ = ctx.centres()
        ctx.close()
        assert e <= 1.01 * float(plain["energy"].cpu()[0]), t


def test_init_from_centres_rejects_bad_arguments(slic):
    from paper_1509_04232_amd import _abi
    p = slic.Params(64, 48, S=16)
    rgb = torch.zeros(64 * 48 * 3, dtype=torch.uint8, device="cuda")
    ws = slic.workspace_for(p)
    host = torch.zeros((p.n_clusters, 5), dtype=torch.float32)
    with pytest.raises(_abi.SlicError):
        _abi.slic_init_from_centres(p.c(), rgb.data_ptr(), host.data_ptr(), 0, ws.data_ptr(),
                                    ws.numel())
    with pytest.raises(ValueError):
        slic.Context(p, rgb, centres=torch.zeros((p.n_clusters + 1, 5), device="cuda"))
