"""slic_segment_noalloc (the entry point for callers that cannot allocate
device memory) against slic_segment through the C ABI: labels, centres,
energy and segment count identical bit for bit, on two calls in a row that
share the library's device array, the second with a smaller image; and the
size limit enforced before anything is enqueued."""
import numpy as np
import pytest
import torch

import synth
from paper_1509_04232_amd import _abi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1509_04232_amd as slic
    return slic


def _outputs(p, dev):
    K = p.n_clusters
    return {"labels": torch.full((p.height, p.width), -7, dtype=torch.int32, device=dev),
            "centres": torch.full((K, 5), float("nan"), dtype=torch.float32, device=dev),
            "energy": torch.full((1,), -1.0, dtype=torch.float64, device=dev),
            "n_segments": torch.full((1,), -1, dtype=torch.int32, device=dev)}


def _run(slic, p, rgb, iters, noalloc):
    out = _outputs(p, rgb.device)
    stream = torch.cuda.current_stream().cuda_stream
    args = (p.c(), rgb.data_ptr(), iters, 1, out["labels"].data_ptr(),
            out["centres"].data_ptr(), out["energy"].data_ptr(), out["n_segments"].data_ptr())
    if noalloc:
        _abi.slic_segment_noalloc(*args, stream)
    else:
        # a workspace full of garbage: the result must not depend on it
        ws = torch.randint(0, 256, (slic.slic_workspace_bytes(p.c()),), dtype=torch.uint8,
                           device=rgb.device)
        _abi.slic_segment(*args, stream, ws.data_ptr(), ws.numel())
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(got, want):
    for k in ("labels", "centres", "energy", "n_segments"):
        assert np.array_equal(got[k], want[k]), f"{k} differ"


# two calls in a row, the second smaller, so the second reads an array that
# still holds the first call's contents
CASES = [("1920x1080 S=8", 1920, 1080, 8, 1, 2048, 12.0, 10),
         ("320x240 S=16", 320, 240, 16, 2, 64, 8.0, 5)]


def test_noalloc_equals_segment_on_consecutive_calls(slic):
    dev = torch.device("cuda:0")
    for name, w, h, S, seed, regions, sigma, iters in CASES:
        print(f"noalloc case {name}", flush=True)
        img = synth.voronoi_image(seed, w, h, regions, sigma)
        rgb = torch.from_numpy(img.reshape(-1)).to(dev)
        p = slic.Params(w, h, S=S, m=10.0, perturb=True)
        assert slic.slic_workspace_bytes(p.c()) <= _abi.SLIC_NOALLOC_MAX_WORKSPACE
        got = _run(slic, p, rgb, iters, noalloc=True)
        want = _run(slic, p, rgb, iters, noalloc=False)
        _same(got, want)
        assert got["n_segments"][0] > 0 and got["labels"].min() >= 0


def test_noalloc_rejects_a_frame_beyond_its_array(slic):
    dev = torch.device("cuda:0")
    p = slic.Params(1920, 1080, S=6, m=10.0)
    assert slic.slic_workspace_bytes(p.c()) > _abi.SLIC_NOALLOC_MAX_WORKSPACE
    rgb = torch.zeros(1920 * 1080 * 3, dtype=torch.uint8, device=dev)
    labels = torch.full((1080, 1920), -7, dtype=torch.int32, device=dev)
    with pytest.raises(_abi.SlicError) as e:
        _abi.slic_segment_noalloc(p.c(), rgb.data_ptr(), 2, 1, labels.data_ptr(), None, None,
                                  None, torch.cuda.current_stream().cuda_stream)
    assert e.value.code == _abi.SLIC_EINVAL
    torch.cuda.synchronize()
    assert int(labels.min()) == -7 and int(labels.max()) == -7  # nothing was enqueued
