"""The one-call segmentation with connectivity (slic_segment and the warm
start's slic_warm_segment) ends its last association launch with the
clean-up's tile-local components on 32 x 32 tiles and then skips that
pass.  These cases compare the labels after the clean-up bit-exactly with
the oracle (Section 2's connectivity step under the canonical merge rule)
and with the context API, which runs every pass on its own: ragged images,
no rounds after the first association, both distances, and full-size
frames."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slic():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1509_04232_amd as slic
    return slic


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    # widths and heights on both sides of multiples of the 32-pixel tile
    w = int(rng.choice([1, 7, 31, 32, 33, 63, 64, 65, 97, 130]))
    h = int(rng.choice([1, 5, 31, 32, 33, 64, 70, 95]))
    kind = seed % 3
    if kind == 0:
        img = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    elif kind == 1:
        img = synth.voronoi_image(seed, w, h, int(rng.integers(1, 12)), 6.0)
    else:  # few colours: long runs and exact ties in colour distance
        pal = rng.integers(0, 256, (3, 3), dtype=np.uint8)
        img = pal[rng.integers(0, 3, (h, w))]
    S = int(rng.choice([1, 2, 4, 5, 8, 16, 32]))
    m = float(rng.choice([0.0, 10.0, 40.0]))
    iters = int(rng.integers(0, 4))
    ms = int(rng.choice([0, 3, 20]))
    squared = bool(seed % 4 == 3)
    return img, S, m, iters, ms, squared


def _segment(slic, img, S, m, iters, ms, squared):
    h, w, _ = img.shape
    p = slic.Params(w, h, S=S, m=m, min_segment=ms, squared_distance=squared)
    rgb = torch.from_numpy(np.ascontiguousarray(img).reshape(-1)).cuda()
    out = slic.segment(rgb, p, iters, enforce=True, want_centres=True)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("seed", range(40))
def test_fused_segment_matches_oracle(slic, seed):
    img, S, m, iters, ms, squared = _case(seed)
    print(f"case seed={seed} shape={img.shape} S={S} m={m} iters={iters} ms={ms} "
          f"squared={squared}", flush=True)
    out = _segment(slic, img, S, m, iters, ms, squared)
    S = oracle.grid(img.shape[1], img.shape[0], S, 0)[0]
    want = oracle.segment(img, S, m, iters, True, True, ms,
                          dist=oracle.DIST_SQUARED if squared else oracle.DIST_EQ1)
    got = out["labels"].cpu().numpy()
    assert np.array_equal(got, want["seg_labels"]), \
        f"{(got != want['seg_labels']).sum()} labels differ"
    assert int(out["n_segments"].cpu()[0]) == want["n_segments"]
    assert np.array_equal(out["centres"].cpu().numpy(), want["centres"])


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_fused_segment_equals_separate_passes(slic, name):
    """At the workloads' full sizes: the one-call path against the context
    path (association launches, then every connectivity pass)."""
    wl = synth.WORKLOADS[name]
    img = synth.image_for(wl)
    print(f"case {name} {wl.width}x{wl.height}", flush=True)
    rgb = torch.from_numpy(np.ascontiguousarray(img).reshape(-1)).cuda()
    p = slic.Params(wl.width, wl.height, S=wl.S, m=wl.m, min_segment=wl.min_segment)
    one = slic.segment(rgb, p, wl.iters, enforce=True)
    ctx = slic.Context(p, rgb)
    ctx.iterate(wl.iters)
    n = ctx.enforce_connectivity()
    torch.cuda.synchronize()
    assert torch.equal(one["labels"], ctx.labels())
    assert int(one["n_segments"].cpu()[0]) == int(n.cpu()[0])
    ctx.close()


@pytest.mark.parametrize("w,h,S,squared", [
    (96, 70, 8, False),    # four pixels of a row per thread (S and width multiples of 4)
    (128, 64, 16, True),
    (98, 70, 8, False),    # width not a multiple of 4: one pixel in each of four rows
    (96, 70, 6, False),    # step not a multiple of 4
    (33, 97, 4, False),
    (200, 150, 64, False),  # cells larger than the 32 x 32 tiles
    (70, 45, 1, False),     # S = 1: the window does not fit, the separate pass runs
])
def test_fused_segment_both_tile_shapes(slic, w, h, S, squared):
    img = synth.voronoi_image(w * 131 + h, w, h, 9, 8.0)
    print(f"case {w}x{h} S={S} squared={squared}", flush=True)
    out = _segment(slic, img, S, 10.0, 3, 5, squared)
    want = oracle.segment(img, S, 10.0, 3, True, True, 5,
                          dist=oracle.DIST_SQUARED if squared else oracle.DIST_EQ1)
    assert np.array_equal(out["labels"].cpu().numpy(), want["seg_labels"])
    assert int(out["n_segments"].cpu()[0]) == want["n_segments"]
    assert np.array_equal(out["centres"].cpu().numpy(), want["centres"])


@pytest.mark.parametrize("iters", [0, 1, 2, 5])
def test_one_call_labels_without_connectivity(slic, iters):
    """Only the last association launch of a one-call segmentation writes
    labels: the labels and centres after 0..5 rounds without the clean-up
    equal the oracle's."""
    w, h, S = 150, 90, 8
    img = synth.voronoi_image(77 + iters, w, h, 12, 8.0)
    p = slic.Params(w, h, S=S, m=10.0)
    rgb = torch.from_numpy(np.ascontiguousarray(img).reshape(-1)).cuda()
    print(f"case iters={iters}", flush=True)
    out = slic.segment(rgb, p, iters, enforce=False, want_centres=True)
    torch.cuda.synchronize()
    want = oracle.segment(img, S, 10.0, iters, True)
    assert np.array_equal(out["labels"].cpu().numpy(), want["labels"])
    assert np.array_equal(out["centres"].cpu().numpy(), want["centres"])
