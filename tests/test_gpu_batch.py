"""Batched segmentation (many images of uneven sizes and steps through shared
launches, optionally one HIP graph) against per-image calls and the oracle."""
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


def _mixed_workloads():
    rng = np.random.default_rng(77)
    out = []
    for j in range(10):
        w, h = int(rng.integers(8, 200)), int(rng.integers(8, 150))
        S = int(rng.choice([3, 5, 8, 12, 16, 32]))
        out.append(Workload(f"mix{j}", w, h, max(1, w * h // 300), 8.0, 900 + j, S,
                            iters=4, perturb=bool(j % 2)))
    return out


def _device(img):
    return torch.from_numpy(img.reshape(-1)).cuda()


def _single(slic, wl, img, iters, enforce):
    p = slic.Params(wl.width, wl.height, S=wl.S, m=wl.m, perturb=wl.perturb,
                    min_segment=wl.min_segment)
    out = slic.segment(_device(img), p, iters, enforce=enforce)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("enforce", [False, True])
def test_batch_equals_single_calls(slic, use_graph, enforce):
    wls = _mixed_workloads()
    imgs = [synth.image_for(w) for w in wls]
    params = [slic.Params(w.width, w.height, S=w.S, m=w.m, perturb=w.perturb) for w in wls]
    b = slic.Batch(params, [_device(i) for i in imgs], 4, enforce=enforce, use_graph=use_graph)
    b.run()
    torch.cuda.synchronize()
    first = [t.cpu().numpy() for t in b.labels]
    for wl, img, got in zip(wls, imgs, first):
        want = _single(slic, wl, img, 4, enforce)
        assert np.array_equal(got, want["labels"].cpu().numpy()), wl.name
    if enforce:
        for wl, img, n in zip(wls, imgs, b.n_segments.cpu().numpy()):
            assert n == int(_single(slic, wl, img, 4, True)["n_segments"].cpu()[0])
    # replays, with other work in between, give the same bits every time
    for _ in range(3):
        junk = torch.randn(1 << 20, device="cuda").sum()
        b.run()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for got, ref in zip(b.labels, first):
            assert np.array_equal(got.cpu().numpy(), ref)
    b.close()


def test_batch_of_the_c4_images_matches_the_oracle(slic):
    """All 64 images of the c4 batch (46 Mpix, sizes 320x240 to 1920x1080,
    S of 8, 16 and 32), through one HIP graph with the autotuned variant, as
    the benchmark runs them (no connectivity) and with connectivity: every
    image's labels and segment count equal the oracle's."""
    wls = synth.batch_workload()
    assert len(wls) == 64
    imgs = [synth.image_for(w) for w in wls]
    devs = [_device(i) for i in imgs]
    params = [slic.Params(w.width, w.height, S=w.S, m=w.m, perturb=w.perturb) for w in wls]
    iters = wls[0].iters
    plain = slic.Batch(params, devs, iters, use_graph=True)
    variant, _ = plain.autotune(reps=1)
    plain.run()
    merged = slic.Batch(params, devs, iters, enforce=True, variant=variant, use_graph=True)
    merged.run()
    torch.cuda.synchronize()
    print(f"c4: 64 images, variant {variant}", flush=True)
    for j, (wl, img) in enumerate(zip(wls, imgs)):
        want = oracle.segment(img, wl.S, wl.m, wl.iters, wl.perturb, True)
        assert np.array_equal(plain.labels[j].cpu().numpy(), want["labels"]), wl.name
        assert np.array_equal(merged.labels[j].cpu().numpy(), want["seg_labels"]), wl.name
        assert int(merged.n_segments[j].cpu()) == want["n_segments"], wl.name
    plain.close()
    merged.close()


def test_batch_autotune_keeps_results(slic):
    wls = synth.batch_workload()[:8]
    imgs = [synth.image_for(w) for w in wls]
    params = [slic.Params(w.width, w.height, S=w.S, m=w.m) for w in wls]
    b = slic.Batch(params, [_device(i) for i in imgs], 3, use_graph=True)
    b.run()
    torch.cuda.synchronize()
    ref = [t.cpu().numpy() for t in b.labels]
    best, ms = b.autotune(reps=2)
    assert 1 <= best <= slic.slic_assign_variants() and ms > 0
    b.run()
    torch.cuda.synchronize()
    for got, r in zip(b.labels, ref):
        assert np.array_equal(got.cpu().numpy(), r)
    b.close()


def test_segment_batch_one_shot(slic):
    wls = _mixed_workloads()[:4]
    imgs = [synth.image_for(w) for w in wls]
    devs = [_device(i) for i in imgs]
    params = [slic.Params(w.width, w.height, S=w.S, m=w.m, perturb=w.perturb) for w in wls]
    cps = [p.c() for p in params]
    labels = [torch.empty((p.height, p.width), dtype=torch.int32, device="cuda") for p in params]
    ws = torch.empty(slic.slic_batch_workspace_bytes(cps), dtype=torch.uint8, device="cuda")
    slic.slic_segment_batch(cps, [d.data_ptr() for d in devs], 4, 0,
                            [t.data_ptr() for t in labels], None,
                            torch.cuda.current_stream().cuda_stream, ws.data_ptr(), ws.numel())
    torch.cuda.synchronize()
    for wl, img, got in zip(wls, imgs, labels):
        assert np.array_equal(got.cpu().numpy(), _single(slic, wl, img, 4, False)["labels"]
                              .cpu().numpy())


def test_batch_rejects_bad_arguments(slic):
    from paper_1509_04232_amd import _abi
    p = slic.Params(64, 48, S=8)
    img = torch.zeros(64 * 48 * 3, dtype=torch.uint8, device="cuda")
    lab = torch.empty((48, 64), dtype=torch.int32, device="cuda")
    ws = torch.empty(slic.slic_batch_workspace_bytes([p.c()]), dtype=torch.uint8, device="cuda")
    with pytest.raises(_abi.SlicError):  # workspace too small
        _abi.slic_batch_create([p.c()], [img.data_ptr()], [lab.data_ptr()], 2, 0, None, 0, 0,
                               ws.data_ptr(), ws.numel() - 1)
    with pytest.raises(_abi.SlicError):  # 4-wide variant with S = 6
        q = slic.Params(64, 48, S=6)
        ws2 = torch.empty(slic.slic_batch_workspace_bytes([q.c()]), dtype=torch.uint8,
                          device="cuda")
        _abi.slic_batch_create([q.c()], [img.data_ptr()], [lab.data_ptr()], 2, 0, None, 4, 0,
                               ws2.data_ptr(), ws2.numel())
    host = torch.zeros(64 * 48 * 3, dtype=torch.uint8)
    with pytest.raises(_abi.SlicError):  # host memory
        _abi.slic_batch_create([p.c()], [host.data_ptr()], [lab.data_ptr()], 2, 0, None, 0, 0,
                               ws.data_ptr(), ws.numel())


def test_batch_with_a_large_image_takes_the_per_image_connectivity(slic):
    """A 4.35 Mpix image's segment numbering does not fit the batched relabel
    pass's own scan (4096 runs of 1024 pixels), so the batch runs the
    connectivity image by image; the results equal single calls either way."""
    wls = [Workload("big", 2560, 1700, 400, 8.0, 4242, 32, iters=1),
           Workload("small", 120, 90, 30, 8.0, 4243, 8, iters=1)]
    imgs = [synth.image_for(w) for w in wls]
    params = [slic.Params(w.width, w.height, S=w.S, m=w.m, perturb=w.perturb) for w in wls]
    b = slic.Batch(params, [_device(i) for i in imgs], 1, enforce=True, use_graph=False)
    b.run()
    torch.cuda.synchronize()
    for wl, img, got, n in zip(wls, imgs, b.labels, b.n_segments.cpu().numpy()):
        want = _single(slic, wl, img, 1, True)
        assert np.array_equal(got.cpu().numpy(), want["labels"].cpu().numpy()), wl.name
        assert n == int(want["n_segments"].cpu()[0])
    b.close()


def test_batch_connectivity_with_per_image_thresholds(slic):
    """Each image's own merge threshold reaches the batched connectivity
    launches (min_segment from 0, the S*S/4 default, to large values)."""
    wls = _mixed_workloads()[:6]
    imgs = [synth.image_for(w) for w in wls]
    thresholds = [0, 1, 5, 30, 200, 10_000]
    params = [slic.Params(w.width, w.height, S=w.S, m=w.m, perturb=w.perturb, min_segment=ms)
              for w, ms in zip(wls, thresholds)]
    b = slic.Batch(params, [_device(i) for i in imgs], 3, enforce=True, use_graph=True)
    b.run()
    torch.cuda.synchronize()
    for wl, img, ms, got, n in zip(wls, imgs, thresholds, b.labels, b.n_segments.cpu().numpy()):
        want = oracle.segment(img, wl.S, wl.m, 3, wl.perturb, True, ms)
        assert np.array_equal(got.cpu().numpy(), want["seg_labels"]), (wl.name, ms)
        assert n == want["n_segments"]
    b.close()
