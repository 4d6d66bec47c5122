"""The learned warm start on the GPU: the net's parameters and Adam state as
torch device tensors, and the calls of libslic's net entry points
(``slic_net_forward``, ``slic_net_loss_grad``, ``slic_net_targets``,
``slic_net_adam``, ``slic_warm_segment``).  Every step of the arithmetic runs
in libslic's kernels; this module marshals arguments and sequences calls.

Training data: an image's targets are its plain-SLIC labels after the full
iteration count (grid-indexed, before connectivity), as the class of the
label's cell relative to the pixel's cell.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _abi
from ._abi import SlicNetCrop


def offsets(S: int) -> dict:
    """Start of each parameter block in the flat vector (and its end)."""
    o = {"W1": 0}
    o["b1"] = o["W1"] + 9 * 32 * 3
    o["W2"] = o["b1"] + 32
    o["b2"] = o["W2"] + 9 * 32 * 32
    o["W3"] = o["b2"] + 32
    o["b3"] = o["W3"] + 9 * 9 * 32
    o["P"] = o["b3"] + 9
    o["end"] = o["P"] + 9 * S * S
    assert o["end"] == _abi.slic_net_param_count(S)
    return o


def init_params(S: int, seed: int = 0) -> np.ndarray:
    """He-normal convolution weights (std sqrt(2 / (9 * fan_in))), zero
    biases, zero phase bias."""
    rng = np.random.default_rng(seed)
    o = offsets(S)
    p = np.zeros(o["end"], np.float32)
    for w, fan in (("W1", 3), ("W2", 32), ("W3", 32)):
        n = o[{"W1": "b1", "W2": "b2", "W3": "b3"}[w]] - o[w]
        p[o[w]:o[w] + n] = rng.normal(0.0, math.sqrt(2.0 / (9 * fan)), n)
    return p


def crop(L: torch.Tensor, A: torch.Tensor, B: torch.Tensor, ox: int = 0, oy: int = 0,
         labels: torch.Tensor | None = None) -> SlicNetCrop:
    """A crop descriptor over planar (H, W) float32 CIELAB device tensors
    (and optionally the image's int32 labels).  The tensors must outlive
    every call that uses the descriptor."""
    h, w = L.shape
    for t in (L, A, B):
        if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("L, A, B must be contiguous float32 GPU tensors")
    lp = 0
    if labels is not None:
        if labels.dtype != torch.int32 or labels.shape != L.shape or not labels.is_contiguous():
            raise ValueError("labels must be a contiguous int32 tensor of the image's shape")
        lp = labels.data_ptr()
    return SlicNetCrop(L.data_ptr(), A.data_ptr(), B.data_ptr(), lp or None, w, h, ox, oy)


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Net:
    """Parameters (FP32 master copy on the GPU), gradient, Adam moments and
    the workspace for batches of ``n_crops`` crops of ``crop_w x crop_h``."""

    def __init__(self, S: int, n_crops: int, crop_w: int, crop_h: int, params=None,
                 seed: int = 0, device="cuda"):
        self.S, self.n_crops, self.crop_w, self.crop_h = S, n_crops, crop_w, crop_h
        self.count = _abi.slic_net_param_count(S)
        p = init_params(S, seed) if params is None else np.asarray(params, np.float32)
        if p.size != self.count:
            raise ValueError(f"expected {self.count} parameters, got {p.size}")
        self.params = torch.from_numpy(p.copy()).to(device)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.ws = torch.empty(_abi.slic_net_workspace_bytes(n_crops, crop_w, crop_h, S),
                              dtype=torch.uint8, device=device)
        self.target = torch.empty((n_crops, crop_h, crop_w), dtype=torch.int32, device=device)
        self.steps = 0

    def forward(self, crops, stream=None) -> torch.Tensor:
        out = torch.empty((len(crops), self.crop_h, self.crop_w, 9), dtype=torch.float32,
                          device=self.params.device)
        _abi.slic_net_forward(crops, self.crop_w, self.crop_h, self.S, self.params.data_ptr(),
                              out.data_ptr(), _stream(stream), self.ws.data_ptr(), self.ws.numel())
        return out

    def targets(self, crops, stream=None) -> torch.Tensor:
        t = self.target[:len(crops)]
        _abi.slic_net_targets(crops, self.crop_w, self.crop_h, self.S, t.data_ptr(),
                              _stream(stream))
        return t

    def loss_grad(self, crops, target: torch.Tensor, stream=None) -> torch.Tensor:
        if target.dtype != torch.int32 or not target.is_contiguous() or \
                target.numel() < len(crops) * self.crop_w * self.crop_h:
            raise ValueError("target must be a contiguous int32 tensor of n x crop_h x crop_w")
        _abi.slic_net_loss_grad(crops, self.crop_w, self.crop_h, self.S, self.params.data_ptr(),
                                target.data_ptr(), self.grad.data_ptr(), self.loss.data_ptr(),
                                _stream(stream), self.ws.data_ptr(), self.ws.numel())
        return self.loss

    def adam(self, lr: float, betas=(0.9, 0.999), eps: float = 1e-8, stream=None) -> None:
        self.steps += 1
        _abi.slic_net_adam(self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(),
                           self.v.data_ptr(), self.count, self.steps, lr, betas[0], betas[1], eps,
                           _stream(stream))

    def train_step(self, crops, lr: float, stream=None) -> torch.Tensor:
        """Targets from the crops' labels, loss and gradient, one Adam step;
        returns the loss (device tensor, before the step)."""
        t = self.targets(crops, stream)
        loss = self.loss_grad(crops, t, stream)
        self.adam(lr, stream=stream)
        return loss


def prepare(params: torch.Tensor, S: int, min_confidence: float = 0.0, stream=None,
            out: torch.Tensor | None = None):
    """slic_net_prepare: the inference copy of a parameter vector (a uint8
    device tensor of slic_net_prepared_bytes()).  Only pixels whose best
    class has softmax probability >= min_confidence vote in the warm
    start's first centre update (0: all)."""
    if params.dtype != torch.float32 or params.device.type != "cuda":
        raise ValueError("params must be a float32 GPU tensor")
    if params.numel() != _abi.slic_net_param_count(S):
        raise ValueError(f"expected {_abi.slic_net_param_count(S)} parameters for S={S}")
    net = out if out is not None else torch.empty(_abi.slic_net_prepared_bytes(),
                                                  dtype=torch.uint8, device=params.device)
    _abi.slic_net_prepare(S, params.data_ptr(), float(min_confidence), net.data_ptr(),
                          _stream(stream))
    return net


def warm_segment(rgb: torch.Tensor, p, net: torch.Tensor, iters: int,
                 enforce: bool = False, want_centres: bool = False, want_energy: bool = True,
                 stream=None, workspace=None) -> dict:
    """slic_warm_segment: the prepared net's labels (``prepare``) as the
    first association, then ``iters`` rounds of (update, associate).
    Returns device tensors: labels, and optionally centres, energy,
    n_segments."""
    from . import _check_rgb
    _check_rgb(rgb, p)
    cp = p.c()
    dev = rgb.device
    ws = workspace if workspace is not None else torch.empty(
        _abi.slic_warm_workspace_bytes(cp), dtype=torch.uint8, device=dev)
    out = {"labels": torch.empty((p.height, p.width), dtype=torch.int32, device=dev)}
    if want_centres:
        out["centres"] = torch.empty((p.n_clusters, 5), dtype=torch.float32, device=dev)
    if want_energy:
        out["energy"] = torch.empty(1, dtype=torch.float64, device=dev)
    if enforce:
        out["n_segments"] = torch.empty(1, dtype=torch.int32, device=dev)
    ptr = lambda k: out[k].data_ptr() if k in out else None  # noqa: E731
    _abi.slic_warm_segment(cp, rgb.data_ptr(), net.data_ptr(), iters, 1 if enforce else 0,
                           out["labels"].data_ptr(), ptr("centres"), ptr("energy"),
                           ptr("n_segments"), _stream(stream), ws.data_ptr(), ws.numel())
    return out


def passes_gate(warm_energy: float, plain_energy: float, ratio: float = 1.01) -> bool:
    """The warm result replaces plain SLIC only if its energy is at most
    ``ratio`` times plain SLIC's."""
    return warm_energy <= ratio * plain_energy


class TrainingSet:
    """Training images on the GPU: CIELAB planes and the plain-SLIC labels
    after ``iters`` rounds (grid-indexed, before connectivity), all computed
    by libslic.  ``images``: (uint8 device tensor, Params) pairs with one
    common S."""

    def __init__(self, images, iters: int = 10, stream=None):
        from . import Context
        self.items = []
        self.S = None
        for rgb, p in images:
            S = p.grid()[0]
            if self.S is None:
                self.S = S
            elif S != self.S:
                raise ValueError("every training image needs the same grid step S")
            ctx = Context(p, rgb, stream=stream)
            ctx.iterate(iters)
            L, A, B = ctx.lab()
            labels = ctx.labels()
            ctx.close()
            self.items.append((L, A, B, labels))

    def __len__(self) -> int:
        return len(self.items)


def train(net: Net, data: TrainingSet, steps: int, lr: float = 3e-3, lr_final: float = 3e-4,
          seed: int = 0, log_every: int = 0, stream=None):
    """``steps`` Adam steps on batches of ``net.n_crops`` random crops (image
    and origin drawn from a seeded generator), learning rate decaying from
    ``lr`` to ``lr_final`` on a cosine.  Returns [(step, loss)] every
    ``log_every`` steps (each one synchronises the host)."""
    if data.S != net.S:
        raise ValueError(f"net built for S={net.S}, training images use S={data.S}")
    rng = np.random.default_rng(seed)
    log = []
    for s in range(steps):
        crops = []
        for _ in range(net.n_crops):
            L, A, B, lb = data.items[int(rng.integers(len(data)))]
            h, w = L.shape
            ox = int(rng.integers(0, max(1, w - net.crop_w + 1)))
            oy = int(rng.integers(0, max(1, h - net.crop_h + 1)))
            crops.append(crop(L, A, B, ox, oy, lb))
        f = 0.5 * (1.0 + math.cos(math.pi * s / max(1, steps - 1)))
        loss = net.train_step(crops, lr_final + (lr - lr_final) * f, stream)
        if log_every and (s % log_every == 0 or s == steps - 1):
            log.append((s, float(loss.cpu()[0])))
    return log
