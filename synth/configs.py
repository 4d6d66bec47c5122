"""The five benchmark workloads as concrete seeded inputs.

c1  320x240 single image, S=16, 5 iterations, grid seeds, no connectivity.
c2  640x480 single image (the paper's camera size), S=16, 10 iterations,
    gradient-perturbed seeds, connectivity (segments under S*S/4 merged).
c3  1920x1080 single image, S=8, 10 iterations, perturbed seeds, connectivity.
c4  64 images of uneven sizes with per-image S, 10 iterations.
c5  learned warm start: 640x480 training images, 32-image evaluation batches
    at 640x480 and 1920x1080, S=16.
"""
from __future__ import annotations

import dataclasses

_M64 = 0xFFFFFFFFFFFFFFFF


def _splitmix_at(key: int, n: int) -> int:
    z = (key + (n + 1) * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    width: int
    height: int
    regions: int
    sigma: float
    seed: int
    S: int
    m: float = 10.0
    iters: int = 10
    perturb: bool = True
    connectivity: bool = True
    min_segment: int = 0  # 0: the S*S/4 rule
    ramp: float = 20.0

    @property
    def n_pixels(self) -> int:
        return self.width * self.height


WORKLOADS = {
    "c1": Workload("c1", 320, 240, 64, 8.0, 1, 16, iters=5, perturb=False, connectivity=False),
    "c2": Workload("c2", 640, 480, 256, 8.0, 2, 16),
    "c3": Workload("c3", 1920, 1080, 2048, 12.0, 3, 8),
}

_SIZES = [(320, 240), (640, 480), (1280, 720), (1920, 1080)]
_STEPS = [8, 16, 32]


def batch_workload(n_images: int = 64, base_seed: int = 4000, key: int = 4):
    """Workload c4: image j has seed base_seed + j; its size and S are drawn
    from SplitMix64(key) so the batch is the same everywhere."""
    out = []
    for j in range(n_images):
        r = _splitmix_at(key, j)
        w, h = _SIZES[r % 4]
        s = _STEPS[(r >> 8) % 3]
        out.append(Workload(f"c4[{j}]", w, h, max(1, (w * h) // 1200), 8.0, base_seed + j, s,
                            iters=10, perturb=True, connectivity=False))
    return out


def warm_train_workload(j: int) -> Workload:
    """c5 training image j (the c2 generator)."""
    return Workload(f"c5.train[{j}]", 640, 480, 256, 8.0, 1_000_000 + j, 16)


def warm_eval_workload(j: int, hd: bool = False) -> Workload:
    """c5 evaluation image j at 640x480, or at 1920x1080 with the same region
    density (1728 regions) when ``hd``."""
    if hd:
        return Workload(f"c5.eval1080[{j}]", 1920, 1080, 1728, 8.0, 3_000_000 + j, 16)
    return Workload(f"c5.eval480[{j}]", 640, 480, 256, 8.0, 2_000_000 + j, 16)


def image_for(wl: Workload):
    from . import voronoi_image
    return voronoi_image(wl.seed, wl.width, wl.height, wl.regions, wl.sigma, wl.ramp)


def video_workload(n_frames: int = 32, width: int = 640, height: int = 480, shake: int = 2,
                   seed: int = 5_000_000):
    """A hand-held camera over one seeded Voronoi canvas: frame t is the
    width x height crop at (shake + dx_t, shake + dy_t), with dx_t, dy_t in
    [-shake, shake] drawn by SplitMix64 (key = seed), so the view shakes
    around a fixed point.  The canvas keeps c2's region density.  Returns
    (canvas workload, [(x, y) origin per frame])."""
    cw, ch = width + 2 * shake, height + 2 * shake
    regions = max(1, round(256 * cw * ch / (640 * 480)))
    canvas = Workload(f"video[{seed}]", cw, ch, regions, 8.0, seed, 16)
    origins = []
    for t in range(n_frames):
        r = _splitmix_at(seed, t)
        origins.append((int(r % (2 * shake + 1)), int((r >> 16) % (2 * shake + 1))))
    return canvas, origins
