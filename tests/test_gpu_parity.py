"""Parity of the HIP path (through the C ABI) with the CPU oracle: labels,
centres, counts and connectivity bit-exact, CIELAB bit-exact (the stated
bar is 1e-4), energy within 1e-9 relative."""
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


def _to_dev(img, channels=3, pad=0):
    """uint8 (H, W, 3) -> device buffer with `channels` bytes per pixel and
    `pad` extra bytes per row.  Returns (tensor, pitch)."""
    h, w, _ = img.shape
    pitch = w * channels + pad
    buf = np.zeros((h, pitch), np.uint8)
    for c in range(3):
        buf[:, c: w * channels: channels] = img[:, :, c]
    if channels == 4:
        buf[:, 3: w * 4: 4] = 77  # ignored fourth byte
    return torch.from_numpy(buf).cuda(), pitch


def gpu_run(slic, img, S, m, iters, perturb, enforce=False, min_segment=0, channels=3, pad=0,
            K=0):
    h, w, _ = img.shape
    rgb, pitch = _to_dev(img, channels, pad)
    p = slic.Params(w, h, S=S, K=K, m=m, perturb=perturb, min_segment=min_segment,
                    channels=channels, pitch=pitch)
    ctx = slic.Context(p, rgb)
    ctx.iterate(iters)
    lab = ctx.lab()
    labels = ctx.labels()
    cen, cnt = ctx.centres()
    energy = ctx.energy()
    res = {"lab": tuple(t.cpu().numpy() for t in lab), "labels": labels.cpu().numpy(),
           "centres": cen.cpu().numpy(), "counts": cnt.cpu().numpy(),
           "energy": float(energy.cpu()[0])}
    if enforce:
        n = ctx.enforce_connectivity()
        res["seg_labels"] = ctx.labels().cpu().numpy()
        res["n_segments"] = int(n.cpu()[0])
    ctx.close()
    torch.cuda.synchronize()
    return res


def oracle_run(img, S, m, iters, perturb, enforce=False, min_segment=0, K=0):
    h, w, _ = img.shape
    S = oracle.grid(w, h, S, K)[0]
    return oracle.segment(img, S, m, iters, perturb, enforce, min_segment)


def assert_parity(got, want, enforce=False):
    for g, o in zip(got["lab"], want["lab"]):
        assert np.abs(g - o).max() <= 1e-4
        assert np.array_equal(g, o), "CIELAB differs from the oracle in the last bits"
    assert np.array_equal(got["labels"], want["labels"]), \
        f"{(got['labels'] != want['labels']).sum()} labels differ"
    assert np.array_equal(got["centres"], want["centres"]), "centres differ"
    assert np.array_equal(got["counts"], want["counts"]), "counts differ"
    assert abs(got["energy"] - want["energy"]) <= 1e-9 * abs(want["energy"])
    if enforce:
        assert got["n_segments"] == want["n_segments"]
        assert np.array_equal(got["seg_labels"], want["seg_labels"])


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_workloads_full_size(slic, name):
    wl = synth.WORKLOADS[name]
    img = synth.image_for(wl)
    args = (wl.S, wl.m, wl.iters, wl.perturb)
    got = gpu_run(slic, img, *args, enforce=True, min_segment=wl.min_segment)
    want = oracle_run(img, *args, enforce=True, min_segment=wl.min_segment)
    assert_parity(got, want, enforce=True)


def _fuzz_case(seed):
    rng = np.random.default_rng(seed)
    h, w = int(rng.integers(1, 90)), int(rng.integers(1, 90))
    kind = seed % 3
    if kind == 0:
        img = rng.integers(0, 256, (h, w, 3), dtype=np.uint8)
    elif kind == 1:
        img = synth.voronoi_image(seed, w, h, int(rng.integers(1, 12)), 6.0)
    else:  # few colours: exact ties in colour distance
        pal = rng.integers(0, 256, (3, 3), dtype=np.uint8)
        img = pal[rng.integers(0, 3, (h, w))]
    S = int(rng.choice([1, 2, 3, 4, 5, 7, 8, 16, 32]))
    m = float(rng.choice([0.0, 1.0, 10.0, 40.0]))
    iters = int(rng.integers(0, 5))
    perturb = bool(rng.integers(0, 2))
    channels = int(rng.choice([3, 4]))
    pad = int(rng.choice([0, 0, 5]))
    ms = int(rng.choice([0, 0, 3, 20]))
    return img, dict(S=S, m=m, iters=iters, perturb=perturb), dict(channels=channels, pad=pad), ms


@pytest.mark.parametrize("seed", range(80))
def test_fuzz_tiny_images(slic, seed):
    img, args, layout, ms = _fuzz_case(seed)
    got = gpu_run(slic, img, **args, enforce=True, min_segment=ms, **layout)
    want = oracle_run(img, **args, enforce=True, min_segment=ms)
    assert_parity(got, want, enforce=True)


@pytest.mark.parametrize("w,h,S,K", [(1, 1, 1, 0), (1, 1, 16, 0), (5, 3, 16, 0), (3, 40, 2, 0),
                                     (77, 1, 4, 0), (200, 150, 0, 100), (64, 64, 1, 0),
                                     (300, 17, 0, 7)])
def test_edge_shapes(slic, w, h, S, K):
    img = synth.voronoi_image(w * 7 + h, w, h, 5, 10.0)
    got = gpu_run(slic, img, S, 10.0, 3, True, enforce=True, K=K)
    want = oracle_run(img, S, 10.0, 3, True, enforce=True, K=K)
    assert_parity(got, want, enforce=True)


@pytest.mark.parametrize("w,h", [(2048, 2048), (2560, 1700)])
def test_connectivity_numbering_both_scan_paths(slic, w, h):
    """The segment numbering sums per-workgroup survivor counts (1024 pixels
    per workgroup): inside the relabel pass up to 4096 workgroups
    (4,194,304 pixels, the first case exactly), with a separate scan launch
    beyond that (the second case, 4,352,000 pixels)."""
    img = synth.voronoi_image(w + h, w, h, 400, 8.0)
    got = gpu_run(slic, img, 32, 10.0, 1, True, enforce=True)
    want = oracle_run(img, 32, 10.0, 1, True, enforce=True)
    assert_parity(got, want, enforce=True)


@pytest.mark.parametrize("w,h,S,ms", [(640, 480, 16, 0), (640, 480, 16, 6), (333, 257, 8, 2)])
def test_connectivity_on_pure_noise(slic, w, h, S, ms):
    """Uniform random pixels: the label map breaks into tens of thousands of
    small components whose chains of joins run across many 32 x 32 tiles,
    the deepest case for the merge and relabel passes.  With the default
    threshold every component is small and all join pixel 0's (one segment);
    small explicit thresholds leave thousands of segments."""
    img = np.random.default_rng(w * h).integers(0, 256, (h, w, 3), dtype=np.uint8)
    got = gpu_run(slic, img, S, 10.0, 2, True, enforce=True, min_segment=ms)
    want = oracle_run(img, S, 10.0, 2, True, enforce=True, min_segment=ms)
    assert_parity(got, want, enforce=True)


@pytest.mark.parametrize("w,h,S", [(64, 48, 16), (40, 24, 8), (96, 96, 3)])
def test_uniform_image_closed_form(slic, w, h, S):
    img = np.full((h, w, 3), (90, 140, 200), np.uint8)
    got = gpu_run(slic, img, S, 10.0, 3, True, enforce=True)
    y, x = np.mgrid[0:h, 0:w]
    assert np.array_equal(got["labels"], (y // S) * (w // S) + x // S)
    assert got["n_segments"] == (w // S) * (h // S)
    assert np.array_equal(got["seg_labels"], got["labels"])


def test_full_gamut_lab(slic):
    """All 2^24 colours as one 4096 x 4096 image."""
    v = np.arange(1 << 24, dtype=np.uint32)
    img = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], -1).astype(np.uint8)
    img = img.reshape(4096, 4096, 3)
    rgb, pitch = _to_dev(img)
    p = slic.Params(4096, 4096, S=64, m=10.0)
    ctx = slic.Context(p, rgb)
    got = [t.cpu().numpy() for t in ctx.lab()]
    ctx.close()
    want = oracle.rgb_to_lab(img)
    for g, o in zip(got, want):
        assert np.array_equal(g, o)


@pytest.mark.parametrize("w,h,S,perturb", [
    (333, 257, 8, True),    # 32 x 16 conversion tiles, ragged on both sides
    (613, 397, 7, True),    # 40 x 30 tiles, ragged
    (640, 480, 16, False),  # 40 x 30 tiles, exact
    (1500, 900, 12, True),  # 64 x 32 tiles, ragged
])
def test_conversion_tile_shapes(slic, w, h, S, perturb):
    """Every conversion tile shape the library picks by frame size gives the
    oracle's CIELAB planes and seeds exactly, ragged tiles included."""
    img = synth.image_for(Workload("tiles", w, h, max(1, w * h // 2000), 10.0, w + h, S))
    rgb, pitch = _to_dev(img)
    p = slic.Params(w, h, S=S, m=10.0, perturb=perturb)
    ctx = slic.Context(p, rgb)
    got = [t.cpu().numpy() for t in ctx.lab()]
    cen, _ = ctx.centres()
    ctx.close()
    want = oracle.rgb_to_lab(img)
    for g, o in zip(got, want):
        assert np.array_equal(g, o)
    assert np.array_equal(cen.cpu().numpy(), oracle.seed(want, S, perturb))


def test_resume_equals_one_run(slic):
    wl = synth.WORKLOADS["c2"]
    img = synth.image_for(wl)
    rgb, _ = _to_dev(img)
    p = slic.Params(wl.width, wl.height, S=wl.S, m=wl.m)
    a = slic.Context(p, rgb).iterate(3).iterate(2)
    b = slic.Context(p, rgb).iterate(5)
    assert torch.equal(a.labels(), b.labels())
    ca, na = a.centres()
    cb, nb = b.centres()
    assert torch.equal(ca, cb) and torch.equal(na, nb)


def test_segment_entry_point_and_determinism(slic):
    wl = synth.WORKLOADS["c2"]
    img = synth.image_for(wl)
    rgb, _ = _to_dev(img)
    p = slic.Params(wl.width, wl.height, S=wl.S, m=wl.m)
    outs = [slic.segment(rgb, p, wl.iters, enforce=True, want_centres=True, want_energy=True)
            for _ in range(3)]
    torch.cuda.synchronize()
    want = oracle_run(img, wl.S, wl.m, wl.iters, True, enforce=True)
    for o in outs:
        assert np.array_equal(o["labels"].cpu().numpy(), want["seg_labels"])
        assert np.array_equal(o["centres"].cpu().numpy(), want["centres"])
        assert int(o["n_segments"].cpu()[0]) == want["n_segments"]
        assert float(o["energy"].cpu()[0]) == float(outs[0]["energy"].cpu()[0])


def test_error_paths(slic):
    from paper_1509_04232_amd import _abi
    img = synth.voronoi_image(1, 64, 48, 4, 5.0)
    rgb, _ = _to_dev(img)
    p = slic.Params(64, 48, S=8)
    host = torch.zeros(64 * 48 * 3, dtype=torch.uint8)
    ws = slic.workspace_for(p)
    with pytest.raises(_abi.SlicError) as e:
        _abi.slic_init(p.c(), host.data_ptr(), 0, ws.data_ptr(), ws.numel())
    assert e.value.code == _abi.SLIC_EINVAL
    with pytest.raises(_abi.SlicError) as e:
        _abi.slic_init(p.c(), rgb.data_ptr(), 0, ws.data_ptr(), ws.numel() - 1)
    assert e.value.code == _abi.SLIC_EINVAL
    ctx = slic.Context(p, rgb)
    ctx.enforce_connectivity()
    with pytest.raises(_abi.SlicError) as e:
        ctx.iterate(1)
    assert e.value.code == _abi.SLIC_ESTATE
    with pytest.raises(_abi.SlicError) as e:
        ctx.energy()
    assert e.value.code == _abi.SLIC_ESTATE
    ctx.close()
    torch.cuda.synchronize()


def _supported_variants(slic, w, h, S):
    out = []
    for v in range(1, slic.slic_assign_variants() + 1):
        try:
            slic.slic_set_assign_variant(w, h, S, v)
        except slic.SlicError:
            continue
        out.append(v)
    slic.slic_set_assign_variant(w, h, S, 0)
    return out


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_every_variant_is_bit_exact(slic, name):
    wl = synth.WORKLOADS[name]
    img = synth.image_for(wl)
    want = oracle_run(img, wl.S, wl.m, wl.iters, wl.perturb, enforce=True)
    variants = _supported_variants(slic, wl.width, wl.height, wl.S)
    assert 1 in variants and len(variants) >= 3
    try:
        for v in variants:
            slic.slic_set_assign_variant(wl.width, wl.height, wl.S, v)
            got = gpu_run(slic, img, wl.S, wl.m, wl.iters, wl.perturb, enforce=True)
            assert_parity(got, want, enforce=True)
    finally:
        slic.slic_set_assign_variant(wl.width, wl.height, wl.S, 0)


@pytest.mark.parametrize("seed", range(24))
def test_every_variant_on_ragged_images(slic, seed):
    rng = np.random.default_rng(500 + seed)
    w = int(rng.integers(1, 140)) * (4 if seed % 2 else 1)
    h = int(rng.integers(1, 90))
    S = int(rng.choice([1, 2, 3, 4, 8, 12, 16, 32]))
    img = synth.voronoi_image(seed, w, h, int(rng.integers(1, 20)), 8.0)
    want = oracle_run(img, S, 10.0, 2, True, enforce=True)
    try:
        for v in _supported_variants(slic, w, h, S):
            slic.slic_set_assign_variant(w, h, S, v)
            got = gpu_run(slic, img, S, 10.0, 2, True, enforce=True)
            assert_parity(got, want, enforce=True)
    finally:
        slic.slic_set_assign_variant(w, h, S, 0)


def test_autotune_records_a_supported_variant(slic):
    wl = synth.WORKLOADS["c1"]
    img = synth.image_for(wl)
    rgb, _ = _to_dev(img)
    p = slic.Params(wl.width, wl.height, S=wl.S, m=wl.m)
    ws = slic.workspace_for(p)
    # listing the supported variants sets and then clears the recorded
    # choice, so it comes before the autotuner records one
    supported = _supported_variants(slic, wl.width, wl.height, wl.S)
    try:
        best, ms = slic.slic_autotune(p.c(), rgb.data_ptr(), 3, 2, 0, ws.data_ptr(), ws.numel())
        assert best in supported
        assert ms > 0
        assert slic.slic_get_assign_variant(wl.width, wl.height, wl.S) == best
        got = gpu_run(slic, img, wl.S, wl.m, wl.iters, wl.perturb)
        assert_parity(got, oracle_run(img, wl.S, wl.m, wl.iters, wl.perturb))
    finally:
        slic.slic_set_assign_variant(wl.width, wl.height, wl.S, 0)
