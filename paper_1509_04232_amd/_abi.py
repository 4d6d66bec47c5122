"""ctypes binding of libslic's C ABI (``include/slic.h``).

Argument marshalling only: every function here forwards to the library of
the same name and raises :class:`SlicError` on a non-zero status.  There is
no fallback: importing this module fails if ``libslic.so`` is not built.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libslic.so")

SLIC_OK, SLIC_EINVAL, SLIC_ENOMEM, SLIC_EHIP, SLIC_ESTATE = 0, 1, 2, 3, 4
SLIC_PERTURB_SEEDS = 1
SLIC_COLOR_XYZ, SLIC_COLOR_RGB, SLIC_DISTANCE_SQUARED = 2, 4, 8

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; "
                      "g.build()'` (hipcc for gfx950) first")

lib = ctypes.CDLL(LIB_PATH)


class SlicParams(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("pitch", ctypes.c_int32),
        ("channels", ctypes.c_int32), ("S", ctypes.c_int32), ("K", ctypes.c_int32),
        ("m", ctypes.c_float), ("flags", ctypes.c_int32), ("min_segment", ctypes.c_int32),
    ]


class SlicNetCrop(ctypes.Structure):
    _fields_ = [
        ("d_L", ctypes.c_void_p), ("d_a", ctypes.c_void_p), ("d_b", ctypes.c_void_p),
        ("d_labels", ctypes.c_void_p), ("img_w", ctypes.c_int32), ("img_h", ctypes.c_int32),
        ("ox", ctypes.c_int32), ("oy", ctypes.c_int32),
    ]


class SlicError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lib.slic_strerror(code).decode()} (code {code})")


_P = ctypes.c_void_p
_I = ctypes.c_int32
_PP = ctypes.POINTER(SlicParams)
_CP = ctypes.POINTER(SlicNetCrop)

_SIGS = {
    "slic_workspace_bytes": ([_PP], ctypes.c_size_t),
    "slic_grid": ([_PP, _P, _P, _P], ctypes.c_int),
    "slic_init": ([ctypes.POINTER(_P), _PP, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "slic_init_from_centres": ([ctypes.POINTER(_P), _PP, _P, _P, _P, _P, ctypes.c_size_t],
                               ctypes.c_int),
    "slic_init_from_labels": ([ctypes.POINTER(_P), _PP, _P, _P, _P, _P, ctypes.c_size_t],
                              ctypes.c_int),
    "slic_iterate": ([_P, _I], ctypes.c_int),
    "slic_iterate_converge": ([_P, _I, ctypes.c_float, _P], ctypes.c_int),
    "slic_enforce_connectivity": ([_P, _P], ctypes.c_int),
    "slic_filter_stray": ([_P, _I], ctypes.c_int),
    "slic_get_labels": ([_P, _P], ctypes.c_int),
    "slic_get_centres": ([_P, _P, _P], ctypes.c_int),
    "slic_get_lab": ([_P, _P, _P, _P], ctypes.c_int),
    "slic_energy": ([_P, _P], ctypes.c_int),
    "slic_segment": ([_PP, _P, _I, _I, _P, _P, _P, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "slic_segment_noalloc": ([_PP, _P, _I, _I, _P, _P, _P, _P, _P], ctypes.c_int),
    "slic_destroy": ([_P], None),
    "slic_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "slic_assign_variants": ([], ctypes.c_int32),
    "slic_assign_variant_info": ([_I, _P, _P, _P, _P], ctypes.c_int),
    "slic_set_assign_variant": ([_I, _I, _I, _I], ctypes.c_int),
    "slic_get_assign_variant": ([_I, _I, _I, _P], ctypes.c_int),
    "slic_autotune": ([_PP, _P, _I, _I, _P, _P, ctypes.c_size_t, _P, _P], ctypes.c_int),
    "slic_batch_workspace_bytes": ([_PP, _I], ctypes.c_size_t),
    "slic_batch_create": ([ctypes.POINTER(_P), _PP, _I, _P, _P, _I, _I, _P, _I, _I, _P,
                           ctypes.c_size_t], ctypes.c_int),
    "slic_batch_run": ([_P, _P], ctypes.c_int),
    "slic_batch_autotune": ([_P, _P, _I, _P, _P], ctypes.c_int),
    "slic_batch_destroy": ([_P], None),
    "slic_segment_batch": ([_PP, _P, _I, _I, _I, _P, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "slic_net_param_count": ([_I], ctypes.c_int32),
    "slic_net_workspace_bytes": ([_I, _I, _I, _I], ctypes.c_size_t),
    "slic_net_forward": ([_CP, _I, _I, _I, _I, _P, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "slic_net_loss_grad": ([_CP, _I, _I, _I, _I, _P, _P, _P, _P, _P, _P, ctypes.c_size_t],
                           ctypes.c_int),
    "slic_net_targets": ([_CP, _I, _I, _I, _I, _P, _P], ctypes.c_int),
    "slic_net_adam": ([_P, _P, _P, _P, _I, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                       ctypes.c_float, _P], ctypes.c_int),
    "slic_net_prepared_bytes": ([], ctypes.c_size_t),
    "slic_net_prepare": ([_I, _P, ctypes.c_float, _P, _P], ctypes.c_int),
    "slic_warm_workspace_bytes": ([_PP], ctypes.c_size_t),
    "slic_warm_init": ([ctypes.POINTER(_P), _PP, _P, _P, _P, _P, ctypes.c_size_t], ctypes.c_int),
    "slic_warm_segment": ([_PP, _P, _P, _I, _I, _P, _P, _P, _P, _P, _P, ctypes.c_size_t],
                          ctypes.c_int),
    "slic_timing_enable": ([_I], ctypes.c_int),
    "slic_timing_read": ([ctypes.c_char_p, _P, _P], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTED = tuple(_SIGS)


def _check(rc: int, where: str) -> None:
    if rc != SLIC_OK:
        raise SlicError(rc, where)


def slic_workspace_bytes(p: SlicParams) -> int:
    n = lib.slic_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise SlicError(SLIC_EINVAL, "slic_workspace_bytes")
    return int(n)


def slic_grid(p: SlicParams):
    out = [ctypes.c_int32() for _ in range(3)]
    _check(lib.slic_grid(ctypes.byref(p), *[ctypes.byref(o) for o in out]), "slic_grid")
    return tuple(int(o.value) for o in out)


def slic_init(p: SlicParams, d_rgb: int, stream: int, d_ws: int, ws_bytes: int) -> int:
    ctx = _P()
    _check(lib.slic_init(ctypes.byref(ctx), ctypes.byref(p), d_rgb, stream, d_ws, ws_bytes),
           "slic_init")
    return int(ctx.value)


def slic_init_from_centres(p: SlicParams, d_rgb: int, d_centres: int, stream: int, d_ws: int,
                           ws_bytes: int) -> int:
    ctx = _P()
    _check(lib.slic_init_from_centres(ctypes.byref(ctx), ctypes.byref(p), d_rgb, d_centres, stream,
                                      d_ws, ws_bytes), "slic_init_from_centres")
    return int(ctx.value)


def slic_init_from_labels(p: SlicParams, d_rgb: int, d_labels0: int, stream: int, d_ws: int,
                          ws_bytes: int) -> int:
    ctx = _P()
    _check(lib.slic_init_from_labels(ctypes.byref(ctx), ctypes.byref(p), d_rgb, d_labels0, stream,
                                     d_ws, ws_bytes), "slic_init_from_labels")
    return int(ctx.value)


def slic_iterate(ctx: int, n_iters: int) -> None:
    _check(lib.slic_iterate(ctx, n_iters), "slic_iterate")


def slic_iterate_converge(ctx: int, max_iters: int, threshold: float,
                          d_iters_done: int | None) -> None:
    _check(lib.slic_iterate_converge(ctx, max_iters, threshold, d_iters_done),
           "slic_iterate_converge")


def slic_enforce_connectivity(ctx: int, d_n_segments: int | None) -> None:
    _check(lib.slic_enforce_connectivity(ctx, d_n_segments), "slic_enforce_connectivity")


def slic_filter_stray(ctx: int, passes: int) -> None:
    _check(lib.slic_filter_stray(ctx, passes), "slic_filter_stray")


def slic_get_labels(ctx: int, d_labels: int) -> None:
    _check(lib.slic_get_labels(ctx, d_labels), "slic_get_labels")


def slic_get_centres(ctx: int, d_centres: int, d_counts: int | None) -> None:
    _check(lib.slic_get_centres(ctx, d_centres, d_counts), "slic_get_centres")


def slic_get_lab(ctx: int, d_L: int, d_a: int, d_b: int) -> None:
    _check(lib.slic_get_lab(ctx, d_L, d_a, d_b), "slic_get_lab")


def slic_energy(ctx: int, d_out: int) -> None:
    _check(lib.slic_energy(ctx, d_out), "slic_energy")


def slic_segment(p: SlicParams, d_rgb: int, n_iters: int, enforce: int, d_labels: int,
                 d_centres: int | None, d_energy: int | None, d_n_segments: int | None,
                 stream: int, d_ws: int, ws_bytes: int) -> None:
    _check(lib.slic_segment(ctypes.byref(p), d_rgb, n_iters, enforce, d_labels, d_centres,
                            d_energy, d_n_segments, stream, d_ws, ws_bytes), "slic_segment")


def slic_segment_noalloc(p: SlicParams, d_rgb: int, n_iters: int, enforce: int, d_labels: int,
                         d_centres: int | None, d_energy: int | None, d_n_segments: int | None,
                         stream: int) -> None:
    _check(lib.slic_segment_noalloc(ctypes.byref(p), d_rgb, n_iters, enforce, d_labels,
                                    d_centres, d_energy, d_n_segments, stream),
           "slic_segment_noalloc")


SLIC_NOALLOC_MAX_WORKSPACE = 72 << 20


def slic_destroy(ctx: int) -> None:
    lib.slic_destroy(ctx)


def slic_strerror(code: int) -> str:
    return lib.slic_strerror(code).decode()


def slic_assign_variants() -> int:
    return int(lib.slic_assign_variants())


def slic_assign_variant_info(variant: int):
    """(vec, rows, tile_w, tile_h) of an association launch variant."""
    out = [ctypes.c_int32() for _ in range(4)]
    _check(lib.slic_assign_variant_info(variant, *[ctypes.byref(o) for o in out]),
           "slic_assign_variant_info")
    return tuple(int(o.value) for o in out)


def slic_set_assign_variant(width: int, height: int, S: int, variant: int) -> None:
    _check(lib.slic_set_assign_variant(width, height, S, variant), "slic_set_assign_variant")


def slic_get_assign_variant(width: int, height: int, S: int) -> int:
    v = ctypes.c_int32()
    _check(lib.slic_get_assign_variant(width, height, S, ctypes.byref(v)), "slic_get_assign_variant")
    return int(v.value)


def slic_autotune(p: SlicParams, d_rgb: int, n_iters: int, reps: int, stream: int, d_ws: int,
                  ws_bytes: int):
    """(best variant, milliseconds per iteration); records the choice."""
    best = ctypes.c_int32()
    ms = ctypes.c_float()
    _check(lib.slic_autotune(ctypes.byref(p), d_rgb, n_iters, reps, stream, d_ws, ws_bytes,
                             ctypes.byref(best), ctypes.byref(ms)), "slic_autotune")
    return int(best.value), float(ms.value)


def _params_array(params):
    arr = (SlicParams * len(params))(*params)
    return arr


def _ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*ptrs)


def slic_batch_workspace_bytes(params) -> int:
    arr = _params_array(params)
    n = lib.slic_batch_workspace_bytes(arr, len(params))
    if n == 0:
        raise SlicError(SLIC_EINVAL, "slic_batch_workspace_bytes")
    return int(n)


def slic_batch_create(params, d_rgb, d_labels, n_iters: int, enforce: int, d_n_segments,
                      variant: int, use_graph: int, d_ws: int, ws_bytes: int) -> int:
    b = _P()
    _check(lib.slic_batch_create(ctypes.byref(b), _params_array(params), len(params),
                                 _ptr_array(d_rgb), _ptr_array(d_labels), n_iters, enforce,
                                 d_n_segments, variant, use_graph, d_ws, ws_bytes),
           "slic_batch_create")
    return int(b.value)


def slic_batch_run(batch: int, stream: int) -> None:
    _check(lib.slic_batch_run(batch, stream), "slic_batch_run")


def slic_batch_autotune(batch: int, stream: int, reps: int):
    best = ctypes.c_int32()
    ms = ctypes.c_float()
    _check(lib.slic_batch_autotune(batch, stream, reps, ctypes.byref(best), ctypes.byref(ms)),
           "slic_batch_autotune")
    return int(best.value), float(ms.value)


def slic_batch_destroy(batch: int) -> None:
    lib.slic_batch_destroy(batch)


def slic_segment_batch(params, d_rgb, n_iters: int, enforce: int, d_labels, d_n_segments,
                       stream: int, d_ws: int, ws_bytes: int) -> None:
    _check(lib.slic_segment_batch(_params_array(params), _ptr_array(d_rgb), len(params), n_iters,
                                  enforce, _ptr_array(d_labels), d_n_segments, stream, d_ws,
                                  ws_bytes), "slic_segment_batch")


def slic_timing_enable(on: bool) -> None:
    _check(lib.slic_timing_enable(1 if on else 0), "slic_timing_enable")


def slic_timing_read(prefix: str | None = None):
    """(total milliseconds, launch count) of the recorded kernels matching
    prefix (records are kept until the next slic_timing_enable(True))."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib.slic_timing_read(prefix.encode() if prefix else None, ctypes.byref(ms),
                                ctypes.byref(n)), "slic_timing_read")
    return float(ms.value), int(n.value)


def _crops(crops):
    return (SlicNetCrop * len(crops))(*crops)


def slic_net_param_count(S: int) -> int:
    n = int(lib.slic_net_param_count(S))
    if n == 0:
        raise SlicError(SLIC_EINVAL, "slic_net_param_count")
    return n


def slic_net_workspace_bytes(n_crops: int, crop_w: int, crop_h: int, S: int) -> int:
    n = lib.slic_net_workspace_bytes(n_crops, crop_w, crop_h, S)
    if n == 0:
        raise SlicError(SLIC_EINVAL, "slic_net_workspace_bytes")
    return int(n)


def slic_net_forward(crops, crop_w: int, crop_h: int, S: int, d_params: int, d_logits: int,
                     stream: int, d_ws: int, ws_bytes: int) -> None:
    _check(lib.slic_net_forward(_crops(crops), len(crops), crop_w, crop_h, S, d_params, d_logits,
                                stream, d_ws, ws_bytes), "slic_net_forward")


def slic_net_loss_grad(crops, crop_w: int, crop_h: int, S: int, d_params: int, d_target: int,
                       d_grad: int, d_loss: int | None, stream: int, d_ws: int,
                       ws_bytes: int) -> None:
    _check(lib.slic_net_loss_grad(_crops(crops), len(crops), crop_w, crop_h, S, d_params, d_target,
                                  d_grad, d_loss, stream, d_ws, ws_bytes), "slic_net_loss_grad")


def slic_net_targets(crops, crop_w: int, crop_h: int, S: int, d_target: int, stream: int) -> None:
    _check(lib.slic_net_targets(_crops(crops), len(crops), crop_w, crop_h, S, d_target, stream),
           "slic_net_targets")


def slic_net_adam(d_params: int, d_grad: int, d_m: int, d_v: int, count: int, step: int,
                  lr: float, beta1: float, beta2: float, eps: float, stream: int) -> None:
    _check(lib.slic_net_adam(d_params, d_grad, d_m, d_v, count, step, lr, beta1, beta2, eps,
                             stream), "slic_net_adam")


def slic_net_prepared_bytes() -> int:
    return int(lib.slic_net_prepared_bytes())


def slic_net_prepare(S: int, d_params: int, min_confidence: float, d_net: int,
                     stream: int) -> None:
    _check(lib.slic_net_prepare(S, d_params, min_confidence, d_net, stream), "slic_net_prepare")


def slic_warm_workspace_bytes(p: SlicParams) -> int:
    n = lib.slic_warm_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise SlicError(SLIC_EINVAL, "slic_warm_workspace_bytes")
    return int(n)


def slic_warm_init(p: SlicParams, d_rgb: int, d_net: int, stream: int, d_ws: int,
                   ws_bytes: int) -> int:
    ctx = _P()
    _check(lib.slic_warm_init(ctypes.byref(ctx), ctypes.byref(p), d_rgb, d_net, stream,
                              d_ws, ws_bytes), "slic_warm_init")
    return int(ctx.value)


def slic_warm_segment(p: SlicParams, d_rgb: int, d_net: int, n_iters: int, enforce: int,
                      d_labels: int, d_centres: int | None, d_energy: int | None,
                      d_n_segments: int | None, stream: int, d_ws: int, ws_bytes: int) -> None:
    _check(lib.slic_warm_segment(ctypes.byref(p), d_rgb, d_net, n_iters, enforce, d_labels,
                                 d_centres, d_energy, d_n_segments, stream, d_ws, ws_bytes),
           "slic_warm_segment")
