"""The colour-space and distance options on the GPU against the oracle:
colour planes, labels and centres bit-exact and the energy within 1e-9, for
every combination, every launch variant of the squared-sum association,
batches, and the argument checks (a batch shares one distance form; the
warm start needs CIELAB and Eq. 1)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from synth.configs import Workload

pytestmark = pytest.mark.gpu

SPACES = {"lab": oracle.COLOR_LAB, "xyz": oracle.COLOR_XYZ, "rgb": oracle.COLOR_RGB}


@pytest.fixture(scope="module")
def slic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1509_04232_amd as slic
    return slic


def _img(w, h, seed):
    return synth.image_for(Workload("var", w, h, max(1, w * h // 500), 10.0, seed, 8))


@pytest.mark.parametrize("color", ["lab", "xyz", "rgb"])
@pytest.mark.parametrize("squared", [False, True])
@pytest.mark.parametrize("w,h,S", [(160, 120, 16), (131, 77, 7)])
def test_options_match_oracle(slic, color, squared, w, h, S):
    img = _img(w, h, 30 + S)
    dist = oracle.DIST_SQUARED if squared else oracle.DIST_EQ1
    m = 10.0 if color != "rgb" else 25.0
    want = oracle.segment(img, S, m, 4, True, False, 0, SPACES[color], dist)
    p = slic.Params(w, h, S=S, m=m, color=color, squared_distance=squared)
    rgb = torch.from_numpy(img.reshape(-1)).cuda()
    ctx = slic.Context(p, rgb)
    planes = ctx.lab()
    ctx.iterate(4)
    lb = ctx.labels()
    cen, cnt = ctx.centres()
    e = ctx.energy()
    torch.cuda.synchronize()
    for got, ref in zip(planes, want["lab"]):
        assert np.array_equal(got.cpu().numpy(), ref)
    assert np.array_equal(lb.cpu().numpy(), want["labels"])
    assert np.array_equal(cen.cpu().numpy(), want["centres"])
    assert np.array_equal(cnt.cpu().numpy(), want["counts"])
    assert float(e.cpu()[0]) == pytest.approx(want["energy"], rel=1e-9)
    ctx.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7])
def test_every_variant_of_the_squared_association(slic, variant):
    w, h, S = 200, 130, 8
    img = _img(w, h, 41)
    want = oracle.segment(img, S, 10.0, 3, True, False, 0, oracle.COLOR_LAB, oracle.DIST_SQUARED)
    slic.slic_set_assign_variant(w, h, S, variant)
    try:
        p = slic.Params(w, h, S=S, m=10.0, squared_distance=True)
        out = slic.segment(torch.from_numpy(img.reshape(-1)).cuda(), p, 3)
        torch.cuda.synchronize()
        assert np.array_equal(out["labels"].cpu().numpy(), want["labels"])
    finally:
        slic.slic_set_assign_variant(w, h, S, 0)


def test_batch_with_the_squared_distance(slic):
    shapes = [(96, 64, 8, "lab"), (120, 90, 16, "xyz"), (64, 48, 4, "rgb")]
    imgs = [_img(w, h, 50 + i) for i, (w, h, _, _) in enumerate(shapes)]
    params = [slic.Params(w, h, S=S, m=10.0, color=c, squared_distance=True)
              for w, h, S, c in shapes]
    b = slic.Batch(params, [torch.from_numpy(i.reshape(-1)).cuda() for i in imgs], 3,
                   use_graph=True)
    b.run()
    torch.cuda.synchronize()
    for (w, h, S, c), img, got in zip(shapes, imgs, b.labels):
        want = oracle.segment(img, S, 10.0, 3, True, False, 0, SPACES[c], oracle.DIST_SQUARED)
        assert np.array_equal(got.cpu().numpy(), want["labels"])
    b.close()


def test_option_arguments_are_checked(slic):
    from paper_1509_04232_amd import _abi
    img = torch.zeros(64 * 48 * 3, dtype=torch.uint8, device="cuda")
    mixed = [slic.Params(64, 48, S=8), slic.Params(64, 48, S=8, squared_distance=True)]
    with pytest.raises(_abi.SlicError):
        slic.Batch(mixed, [img, img], 2)
    with pytest.raises(_abi.SlicError):
        _abi.slic_warm_workspace_bytes(slic.Params(64, 48, S=8, color="xyz").c())
    with pytest.raises(_abi.SlicError):
        _abi.slic_workspace_bytes(_abi.SlicParams(64, 48, 192, 3, 8, 0, 10.0,
                                                  _abi.SLIC_COLOR_XYZ | _abi.SLIC_COLOR_RGB, 0))
