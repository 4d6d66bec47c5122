"""The seeded input generator: determinism, pinned bytes, exact Voronoi
partition and the stated noise level."""
import hashlib
import json
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "synth_sha256.json")


def test_pinned_bytes():
    want = json.load(open(GOLDEN))
    for name, wl in synth.WORKLOADS.items():
        assert hashlib.sha256(synth.image_for(wl).tobytes()).hexdigest() == want[name], name
    for wl in synth.batch_workload()[:4]:
        assert hashlib.sha256(synth.image_for(wl).tobytes()).hexdigest() == want[wl.name]


@pytest.mark.parametrize("seed,w,h,n", [(1, 64, 48, 7), (2, 97, 33, 40), (3, 200, 150, 300),
                                        (4, 5, 5, 30)])
def test_bucketed_partition_matches_bruteforce(seed, w, h, n):
    _, reg = synth.voronoi_image(seed, w, h, n, 8.0, with_regions=True)
    assert np.array_equal(reg, synth.voronoi_regions_bruteforce(seed, w, h, n))


def test_noise_level_and_ramp_bounds():
    w, h, n = 320, 240, 16
    clean = synth.voronoi_image(9, w, h, n, 0.0).astype(np.float64)
    noisy = synth.voronoi_image(9, w, h, n, 8.0).astype(np.float64)
    inside = (clean > 40) & (clean < 215)  # far from the clamp
    d = (noisy - clean)[inside]
    assert abs(d.mean()) < 0.1 and abs(d.std() - 8.0) < 0.15
    flat = synth.voronoi_image(9, w, h, n, 0.0, ramp=0.0)
    _, reg = synth.voronoi_image(9, w, h, n, 0.0, ramp=0.0, with_regions=True)
    for r in range(n):  # no ramp, no noise: one colour per region
        assert len(np.unique(flat[reg == r].reshape(-1, 3), axis=0)) == 1
    spread = [np.ptp(clean[reg == r].reshape(-1, 3), axis=0).max() for r in range(n)]
    assert max(spread) <= 41  # base +- 20 levels, rounded


def test_batch_workload_is_stable():
    b = synth.batch_workload()
    assert len(b) == 64
    assert {(w.width, w.height) for w in b} <= {(320, 240), (640, 480), (1280, 720), (1920, 1080)}
    assert {w.S for w in b} <= {8, 16, 32}
    assert b == synth.batch_workload()
