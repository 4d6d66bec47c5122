"""SLIC superpixels (gSLICr, arXiv 1509.04232) on one AMD Instinct MI355X.

The work runs in libslic's hand-written HIP kernels behind the C ABI of
``include/slic.h``; this package only marshals torch tensors (device memory)
and the current torch stream into those calls.
"""
from __future__ import annotations

import dataclasses

import torch

from . import _abi
from ._abi import (EXPORTED, SLIC_COLOR_RGB, SLIC_COLOR_XYZ, SLIC_DISTANCE_SQUARED, SLIC_EHIP,
                   SLIC_EINVAL, SLIC_ENOMEM, SLIC_ESTATE, SLIC_OK, SLIC_PERTURB_SEEDS, SlicError, SlicParams, slic_assign_variant_info,
                   slic_assign_variants, slic_autotune, slic_batch_autotune, slic_batch_create,
                   slic_batch_destroy, slic_batch_run, slic_batch_workspace_bytes,
                   slic_destroy, slic_filter_stray, slic_segment_batch,
                   slic_enforce_connectivity, slic_energy, slic_get_assign_variant,
                   slic_get_centres, slic_get_lab, slic_get_labels, slic_grid, slic_init,
                   slic_init_from_centres, slic_init_from_labels,
                   slic_iterate, slic_iterate_converge, slic_segment, slic_segment_noalloc,
                   slic_set_assign_variant, SLIC_NOALLOC_MAX_WORKSPACE,
                   slic_strerror,
                   slic_timing_enable, slic_timing_read, slic_workspace_bytes,
                   SlicNetCrop, slic_net_adam, slic_net_forward, slic_net_loss_grad,
                   slic_net_param_count, slic_net_targets, slic_net_workspace_bytes,
                   slic_net_prepare, slic_net_prepared_bytes, slic_warm_init, slic_warm_segment,
                   slic_warm_workspace_bytes)

__all__ = [
    "Params", "Context", "Batch", "segment", "workspace_for", "SlicError", "SlicParams",
    "SlicNetCrop", "warm",
    *EXPORTED,
]


@dataclasses.dataclass
class Params:
    """Section 2's problem statement: image size, S (or K), compactness m."""
    width: int
    height: int
    S: int = 0
    K: int = 0
    m: float = 10.0
    perturb: bool = True
    min_segment: int = 0
    channels: int = 3
    pitch: int | None = None
    color: str = "lab"          # "lab", "xyz" or "rgb"
    squared_distance: bool = False

    def c(self) -> SlicParams:
        flags = SLIC_PERTURB_SEEDS if self.perturb else 0
        flags |= {"lab": 0, "xyz": SLIC_COLOR_XYZ, "rgb": SLIC_COLOR_RGB}[self.color]
        flags |= SLIC_DISTANCE_SQUARED if self.squared_distance else 0
        return SlicParams(self.width, self.height,
                          self.pitch if self.pitch is not None else self.width * self.channels,
                          self.channels, self.S, self.K, float(self.m), flags, self.min_segment)

    def grid(self):
        return slic_grid(self.c())

    @property
    def n_clusters(self) -> int:
        _, nc, nr = self.grid()
        return nc * nr


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_rgb(rgb: torch.Tensor, p: Params) -> None:
    if rgb.device.type != "cuda" or rgb.dtype != torch.uint8:
        raise ValueError("rgb must be a uint8 tensor on the GPU")
    pitch = p.pitch if p.pitch is not None else p.width * p.channels
    if not rgb.is_contiguous() or rgb.numel() < (p.height - 1) * pitch + p.width * p.channels:
        raise ValueError("rgb must be contiguous and hold height rows of `pitch` bytes")


def workspace_for(p: Params, device=None) -> torch.Tensor:
    n = slic_workspace_bytes(p.c())
    return torch.empty(n, dtype=torch.uint8, device=device or "cuda")


class Context:
    """A slic_ctx: slic_init on construction (slic_warm_init when a prepared
    net, ``warm.prepare``, is given; slic_init_from_centres with centres;
    slic_init_from_labels with a first association), then iterate / enforce
    / get."""

    def __init__(self, p: Params, rgb: torch.Tensor, stream=None, workspace=None,
                 net: torch.Tensor | None = None, centres: torch.Tensor | None = None,
                 labels: torch.Tensor | None = None):
        _check_rgb(rgb, p)
        self.params = p
        self._cp = p.c()
        self.stream = stream
        self._rgb = rgb  # kept alive until the conversion has run
        if labels is not None:  # a given first association
            if labels.dtype != torch.int32 or tuple(labels.shape) != (p.height, p.width) or \
                    not labels.is_contiguous() or labels.device != rgb.device:
                raise ValueError("labels must be a contiguous int32 (H, W) tensor on the image's "
                                 "device")
            self.ws = workspace if workspace is not None else workspace_for(p, rgb.device)
            self.ctx = slic_init_from_labels(self._cp, rgb.data_ptr(), labels.data_ptr(),
                                             _stream(stream), self.ws.data_ptr(), self.ws.numel())
        elif centres is not None:  # video warm start from a previous frame's centres
            if centres.dtype != torch.float32 or tuple(centres.shape) != (p.n_clusters, 5) or \
                    not centres.is_contiguous():
                raise ValueError("centres must be a contiguous float32 (K, 5) tensor")
            self.ws = workspace if workspace is not None else workspace_for(p, rgb.device)
            self.ctx = slic_init_from_centres(self._cp, rgb.data_ptr(), centres.data_ptr(),
                                              _stream(stream), self.ws.data_ptr(), self.ws.numel())
        elif net is None:
            self.ws = workspace if workspace is not None else workspace_for(p, rgb.device)
            self.ctx = slic_init(self._cp, rgb.data_ptr(), _stream(stream), self.ws.data_ptr(),
                                 self.ws.numel())
        else:
            self.ws = workspace if workspace is not None else torch.empty(
                slic_warm_workspace_bytes(self._cp), dtype=torch.uint8, device=rgb.device)
            self._net = net
            self.ctx = slic_warm_init(self._cp, rgb.data_ptr(), net.data_ptr(), _stream(stream),
                                      self.ws.data_ptr(), self.ws.numel())
        self.device = rgb.device

    def iterate(self, n: int) -> "Context":
        slic_iterate(self.ctx, n)
        return self

    def iterate_converge(self, max_iters: int, threshold: float) -> torch.Tensor:
        """Section 2's stopping rule; returns the rounds run (device int32)."""
        n = torch.empty(1, dtype=torch.int32, device=self.device)
        slic_iterate_converge(self.ctx, max_iters, threshold, n.data_ptr())
        return n

    def enforce_connectivity(self) -> torch.Tensor:
        n = torch.empty(1, dtype=torch.int32, device=self.device)
        slic_enforce_connectivity(self.ctx, n.data_ptr())
        return n

    def filter_stray(self, passes: int = 2) -> "Context":
        """Section 3's stray-pixel filter (the paper's two passes by default)."""
        slic_filter_stray(self.ctx, passes)
        return self

    def labels(self) -> torch.Tensor:
        out = torch.empty((self.params.height, self.params.width), dtype=torch.int32,
                          device=self.device)
        slic_get_labels(self.ctx, out.data_ptr())
        return out

    def centres(self):
        K = self.params.n_clusters
        cen = torch.empty((K, 5), dtype=torch.float32, device=self.device)
        cnt = torch.empty(K, dtype=torch.int32, device=self.device)
        slic_get_centres(self.ctx, cen.data_ptr(), cnt.data_ptr())
        return cen, cnt

    def lab(self):
        shape = (self.params.height, self.params.width)
        out = [torch.empty(shape, dtype=torch.float32, device=self.device) for _ in range(3)]
        slic_get_lab(self.ctx, *[t.data_ptr() for t in out])
        return tuple(out)

    def energy(self) -> torch.Tensor:
        e = torch.empty(1, dtype=torch.float64, device=self.device)
        slic_energy(self.ctx, e.data_ptr())
        return e

    def close(self) -> None:
        if getattr(self, "ctx", None):
            slic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()


def segment(rgb: torch.Tensor, p: Params, iters: int, enforce: bool = False,
            want_centres: bool = False, want_energy: bool = False, stream=None, workspace=None):
    """slic_segment: the whole listing in one call.  Returns a dict of device
    tensors: labels (H, W) int32, and optionally centres (K, 5), energy (1,)
    float64 and n_segments (1,) int32."""
    _check_rgb(rgb, p)
    dev = rgb.device
    ws = workspace if workspace is not None else workspace_for(p, dev)
    out = {"labels": torch.empty((p.height, p.width), dtype=torch.int32, device=dev)}
    if want_centres:
        out["centres"] = torch.empty((p.n_clusters, 5), dtype=torch.float32, device=dev)
    if want_energy:
        out["energy"] = torch.empty(1, dtype=torch.float64, device=dev)
    if enforce:
        out["n_segments"] = torch.empty(1, dtype=torch.int32, device=dev)
    ptr = lambda k: out[k].data_ptr() if k in out else None  # noqa: E731
    slic_segment(p.c(), rgb.data_ptr(), iters, 1 if enforce else 0, out["labels"].data_ptr(),
                 ptr("centres"), ptr("energy"), ptr("n_segments"), _stream(stream), ws.data_ptr(),
                 ws.numel())
    return out


class Batch:
    """A slic_batch: many images segmented by shared launches (optionally one
    HIP graph).  ``images`` are uint8 device tensors of H*W*channels bytes;
    the label tensors are allocated here and filled by every ``run``."""

    def __init__(self, params, images, iters: int, enforce: bool = False, variant: int = 0,
                 use_graph: bool = True, device=None):
        if len(params) != len(images) or not params:
            raise ValueError("one Params per image")
        for p, img in zip(params, images):
            _check_rgb(img, p)
        dev = device or images[0].device
        self.params = list(params)
        self._cp = [p.c() for p in params]
        self._images = list(images)
        self.labels = [torch.empty((p.height, p.width), dtype=torch.int32, device=dev)
                       for p in params]
        self.n_segments = torch.empty(len(params), dtype=torch.int32, device=dev) if enforce \
            else None
        n = slic_batch_workspace_bytes(self._cp)
        self.ws = torch.empty(n, dtype=torch.uint8, device=dev)
        self.batch = slic_batch_create(
            self._cp, [t.data_ptr() for t in images], [t.data_ptr() for t in self.labels], iters,
            1 if enforce else 0, self.n_segments.data_ptr() if enforce else None, variant,
            1 if use_graph else 0, self.ws.data_ptr(), self.ws.numel())

    def run(self, stream=None) -> "Batch":
        slic_batch_run(self.batch, _stream(stream))
        return self

    def autotune(self, reps: int = 3, stream=None):
        return slic_batch_autotune(self.batch, _stream(stream), reps)

    def close(self) -> None:
        if getattr(self, "batch", None):
            slic_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        self.close()


from . import warm  # noqa: E402  (uses Params and _check_rgb above)
