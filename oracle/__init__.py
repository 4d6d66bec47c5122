"""CPU oracle for the SLIC superpixel path: numpy front end to ``slic_oracle.c``.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module.  It shares no code
with the GPU library.  Each function names the passage of the paper (gSLICr,
arXiv 1509.04232) that it follows; the C source states the readings taken
where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "slic_oracle.c"), os.path.join(_HERE, "net_oracle.c")]
# SLIC_ORACLE_LIB names another build of the same sources (the sanitizer
# test loads one built with AddressSanitizer and UBSan this way).
_LIB = os.environ.get("SLIC_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
SOURCES = list(_SRCS)

# Flags that make the oracle's FP32 evaluation order the one written in the
# source: no contraction into FMA, no fast-math reassociation.
# OpenMP splits the loops whose iterations are independent (results do not
# depend on the thread count).
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, *_SRCS, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int32
_F = ctypes.c_float
_D = ctypes.c_double


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    sig = {
        "orc_grid": [_I, _I, _I, _I, _P, _P, _P],
        "orc_rgb_to_lab": [_P, _I, _I, _I, _I, _P, _P, _P],
        "orc_seed": [_P, _P, _P, _I, _I, _I, _I, _P],
        "orc_assign": [_P, _P, _P, _I, _I, _I, _F, _P, _P],
        "orc_update": [_P, _P, _P, _I, _I, _P, _I, _P, _P],
        "orc_update_votes": [_P, _P, _P, _I, _I, _P, _P, _I, _P, _P],
        "orc_kmeans": [_P, _P, _P, _I, _I, _I, _F, _I, _I, _P, _P, _P],
        "orc_kmeans_ex": [_P, _P, _P, _I, _I, _I, _F, _I, _I, _I, _P, _P, _P],
        "orc_assign_ex": [_P, _P, _P, _I, _I, _I, _F, _I, _P, _P],
        "orc_energy_ex": [_P, _P, _P, _I, _I, _I, _F, _I, _P, _I, _P, _P],
        "orc_rgb_to_space": [_P, _I, _I, _I, _I, _I, _P, _P, _P],
        "orc_kmeans_converge": [_P, _P, _P, _I, _I, _I, _F, _I, _I, _F, _P, _P, _P, _P],
        "orc_residual": [_P, _P, _I],
        "orc_stray_filter": [_P, _I, _I, _I, _P],
        "orc_energy": [_P, _P, _P, _I, _I, _I, _F, _P, _I, _P, _P],
        "orc_connectivity": [_P, _I, _I, _I, _I, _P, _P, _P],
        "orc_lab_tables": [_P, _P],
        "orc_gradient_at": [_P, _P, _P, _I, _I, _I, _I],
        "orc_threads": [_I],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.orc_lab_tables.restype = None
    lib.orc_gradient_at.restype = ctypes.c_float
    lib.orc_cbrt_export.argtypes = [_D]
    lib.orc_cbrt_export.restype = _D
    lib.orc_weight.argtypes = [_F, _I]
    lib.orc_weight.restype = _F
    lib.orc_qshift.restype = ctypes.c_int
    lib.orc_residual.restype = ctypes.c_int64
    lib.orn_param_count.argtypes = [_I]
    lib.orn_param_count.restype = ctypes.c_int
    lib.orn_bf16.argtypes = [_D]
    lib.orn_bf16.restype = _D
    lib.orn_forward.argtypes = [_I, _I, _I, _I, _I, _P, _P, _P, _P, _I, _P, _P, _P]
    lib.orn_forward.restype = ctypes.c_int
    lib.orn_loss_grad.argtypes = [_I, _I, _I, _I, _I, _P, _P, _P, _P, _P, _I, _P, _P]
    lib.orn_loss_grad.restype = ctypes.c_int
    lib.orn_decode.argtypes = [_I, _I, _I, _P, _P]
    lib.orn_decode.restype = ctypes.c_int
    lib.orn_votes.argtypes = [_I, _I, _P, _D, _P]
    lib.orn_votes.restype = ctypes.c_int
    lib.orn_targets.argtypes = [_I, _I, _I, _P, _P]
    lib.orn_targets.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def threads(n: int = 0) -> int:
    """Threads of the oracle's parallel loops: n > 0 sets the count, 0 only
    queries it.  Results do not depend on it."""
    return int(_load().orc_threads(n))


def qshift() -> int:
    """Fixed-point scale exponent of the colour values in the centre sums."""
    return int(_load().orc_qshift())


def grid(width: int, height: int, S: int = 0, K: int = 0):
    """(S, ns_c, ns_r): Section 2's grid interval and Section 3's ns_r x ns_c map."""
    out = [ctypes.c_int32() for _ in range(3)]
    _check(_load().orc_grid(width, height, S, K, *[ctypes.byref(o) for o in out]), "grid")
    return tuple(int(o.value) for o in out)


def cbrt(t: float) -> float:
    """The oracle's Newton cube root (FP64)."""
    return float(_load().orc_cbrt_export(float(t)))


def lab_tables():
    lin = np.empty(256, np.float32)
    nm = np.empty(9, np.float32)
    _load().orc_lab_tables(_ptr(lin), _ptr(nm))
    return lin, nm.reshape(3, 3)


COLOR_LAB, COLOR_XYZ, COLOR_RGB = 0, 1, 2
DIST_EQ1, DIST_SQUARED = 0, 1


def rgb_to_space(rgb: np.ndarray, space: int):
    """The colour planes of another colour space (0 CIELAB, 1 XYZ x 100,
    2 the R, G, B bytes as floats)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    h, w, c = rgb.shape
    out = [np.empty((h, w), np.float32) for _ in range(3)]
    _check(_load().orc_rgb_to_space(_ptr(rgb), w, h, w * c, c, space, *[_ptr(o) for o in out]),
           "colour space")
    return tuple(out)


def rgb_to_lab(rgb: np.ndarray, pitch: int | None = None):
    """Section 3, image space conversion.  ``rgb``: uint8 (H, W, C), C in {3, 4},
    or a flat byte buffer with ``pitch``.  Returns planar float32 (L, a, b),
    each (H, W)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    h, w, c = rgb.shape
    if pitch is None:
        pitch = w * c
    L = np.empty((h, w), np.float32)
    A = np.empty((h, w), np.float32)
    B = np.empty((h, w), np.float32)
    _check(_load().orc_rgb_to_lab(_ptr(rgb), w, h, pitch, c, _ptr(L), _ptr(A), _ptr(B)), "lab")
    return L, A, B


def gradient_at(lab, x: int, y: int) -> float:
    L, A, B = (np.ascontiguousarray(v, np.float32) for v in lab)
    h, w = L.shape
    return float(_load().orc_gradient_at(_ptr(L), _ptr(A), _ptr(B), w, h, x, y))


def seed(lab, S: int, perturb: bool):
    """Section 2 seed perturbation, Section 3 centre initialisation.
    Returns float32 (K, 5) centres (L, a, b, x, y)."""
    L, A, B = (np.ascontiguousarray(v, np.float32) for v in lab)
    h, w = L.shape
    _, nc, nr = grid(w, h, S)
    cen = np.empty((nc * nr, 5), np.float32)
    _check(_load().orc_seed(_ptr(L), _ptr(A), _ptr(B), w, h, S, int(perturb), _ptr(cen)), "seed")
    return cen


def weight(m: float, S: int) -> float:
    return float(_load().orc_weight(float(m), S))


def assign(lab, S: int, m: float, centres: np.ndarray, dist: int = DIST_EQ1):
    """Eq. 1 (or, with dist=1, the squared-sum distance) and Section 3's
    nine-candidate association.  Returns int32 (H, W)."""
    L, A, B = (np.ascontiguousarray(v, np.float32) for v in lab)
    h, w = L.shape
    cen = np.ascontiguousarray(centres, np.float32)
    lab_out = np.empty((h, w), np.int32)
    _check(_load().orc_assign_ex(_ptr(L), _ptr(A), _ptr(B), w, h, S, float(m), int(dist),
                                 _ptr(cen), _ptr(lab_out)), "assign")
    return lab_out


def update(lab, labels: np.ndarray, centres: np.ndarray, votes: np.ndarray | None = None):
    """Section 3 centre update.  Returns (new centres (K,5), counts (K,)).
    With ``votes`` (bool (H,W)) only the pixels where it is true count."""
    L, A, B = (np.ascontiguousarray(v, np.float32) for v in lab)
    h, w = L.shape
    cen = np.array(centres, np.float32, copy=True, order="C")
    cnt = np.empty(cen.shape[0], np.int32)
    lb = np.ascontiguousarray(labels, np.int32)
    if votes is None:
        _check(_load().orc_update(_ptr(L), _ptr(A), _ptr(B), w, h, _ptr(lb), cen.shape[0],
                                  _ptr(cen), _ptr(cnt)), "update")
    else:
        vt = np.ascontiguousarray(votes, np.uint8)
        if vt.shape != lb.shape:
            raise ValueError("votes must have the labels' shape")
        _check(_load().orc_update_votes(_ptr(L), _ptr(A), _ptr(B), w, h, _ptr(lb), _ptr(vt),
                                        cen.shape[0], _ptr(cen), _ptr(cnt)), "update")
    return cen, cnt


def kmeans(lab, S: int, m: float, perturb: bool, iters: int, dist: int = DIST_EQ1):
    """Section 4's loop: seed, associate, iters x (update, associate).
    Returns (labels (H,W), centres (K,5), counts (K,))."""
    L, A, B = (np.ascontiguousarray(v, np.float32) for v in lab)
    h, w = L.shape
    _, nc, nr = grid(w, h, S)
    cen = np.empty((nc * nr, 5), np.float32)
    cnt = np.empty(nc * nr, np.int32)
    lb = np.empty((h, w), np.int32)
    _check(_load().orc_kmeans_ex(_ptr(L), _ptr(A), _ptr(B), w, h, S, float(m), int(dist),
                                 int(perturb), iters, _ptr(cen), _ptr(cnt), _ptr(lb)), "kmeans")
    return lb, cen, cnt


def kmeans_converge(lab, S: int, m: float, perturb: bool, max_iters: int, threshold: float):
    """Section 2's stopping rule: iterate until the summed L1 shift of the
    centres (exact in units of 2^-18) is below threshold * K, at most
    max_iters times.  Returns (labels, centres, counts, iterations run)."""
    L, A, B = (np.ascontiguousarray(v, np.float32) for v in lab)
    h, w = L.shape
    _, nc, nr = grid(w, h, S)
    cen = np.empty((nc * nr, 5), np.float32)
    cnt = np.empty(nc * nr, np.int32)
    lb = np.empty((h, w), np.int32)
    done = ctypes.c_int32()
    _check(_load().orc_kmeans_converge(_ptr(L), _ptr(A), _ptr(B), w, h, S, float(m), int(perturb),
                                       max_iters, float(threshold), _ptr(cen), _ptr(cnt), _ptr(lb),
                                       ctypes.byref(done)), "kmeans_converge")
    return lb, cen, cnt, int(done.value)


def residual(prev: np.ndarray, nxt: np.ndarray) -> int:
    """Summed L1 distance between two centre sets, in units of 2^-18."""
    a = np.ascontiguousarray(prev, np.float32)
    b = np.ascontiguousarray(nxt, np.float32)
    return int(_load().orc_residual(_ptr(a), _ptr(b), a.shape[0]))


def stray_filter(labels: np.ndarray, passes: int = 2) -> np.ndarray:
    """Section 3's stray-pixel filter, `passes` passes (the paper runs two)."""
    lb = np.ascontiguousarray(labels, np.int32)
    h, w = lb.shape
    out = np.empty_like(lb)
    _check(_load().orc_stray_filter(_ptr(lb), w, h, passes, _ptr(out)), "stray_filter")
    return out


def energy(lab, S: int, m: float, centres: np.ndarray, labels: np.ndarray,
           dist: int = DIST_EQ1) -> float:
    """Mean distance (Eq. 1, or the square root of the squared-sum form)
    between each pixel and its associated centre."""
    L, A, B = (np.ascontiguousarray(v, np.float32) for v in lab)
    h, w = L.shape
    cen = np.ascontiguousarray(centres, np.float32)
    lb = np.ascontiguousarray(labels, np.int32)
    out = ctypes.c_double()
    _check(_load().orc_energy_ex(_ptr(L), _ptr(A), _ptr(B), w, h, S, float(m), int(dist),
                                 _ptr(cen), cen.shape[0], _ptr(lb), ctypes.byref(out)), "energy")
    return float(out.value)


def connectivity(labels: np.ndarray, S: int, min_segment: int = 0):
    """Section 2's connectivity clean-up under the canonical merge rule.
    Returns (segment labels (H,W), n_segments, seg_cluster (n_segments,))."""
    lb = np.ascontiguousarray(labels, np.int32)
    h, w = lb.shape
    out = np.empty((h, w), np.int32)
    seg = np.empty(h * w, np.int32)
    ns = ctypes.c_int32()
    _check(_load().orc_connectivity(_ptr(lb), w, h, S, min_segment, _ptr(out), ctypes.byref(ns),
                                    _ptr(seg)), "connectivity")
    return out, int(ns.value), seg[: ns.value].copy()


def segment(rgb: np.ndarray, S: int, m: float, iters: int, perturb: bool = True,
            connectivity_on: bool = False, min_segment: int = 0, space: int = COLOR_LAB,
            dist: int = DIST_EQ1):
    """The whole path of Section 4's listing.  Returns a dict with lab, labels
    (after the k-means loop), centres, counts, energy and, when
    ``connectivity_on``, seg_labels / n_segments / seg_cluster."""
    lab = rgb_to_space(rgb, space) if space != COLOR_LAB else rgb_to_lab(rgb)
    labels, cen, cnt = kmeans(lab, S, m, perturb, iters, dist)
    res = {"lab": lab, "labels": labels, "centres": cen, "counts": cnt,
           "energy": energy(lab, S, m, cen, labels, dist)}
    if connectivity_on:
        seg, ns, sc = connectivity(labels, S, min_segment)
        res.update(seg_labels=seg, n_segments=ns, seg_cluster=sc)
    return res


# ---------------------------------------------------------------------------
# The learned warm start's net (see net_oracle.c).

NET_C1, NET_C2, NET_C3 = 32, 32, 9


def net_param_count(S: int) -> int:
    return int(_load().orn_param_count(S))


def net_offsets(S: int):
    """Offsets of W1, b1, W2, b2, W3, b3, P in the flat parameter vector."""
    w1 = 0
    b1 = w1 + 9 * NET_C1 * 3
    w2 = b1 + NET_C1
    b2 = w2 + 9 * NET_C2 * NET_C1
    w3 = b2 + NET_C2
    b3 = w3 + 9 * NET_C3 * NET_C2
    P = b3 + NET_C3
    return {"W1": w1, "b1": b1, "W2": w2, "b2": b2, "W3": w3, "b3": b3, "P": P,
            "end": P + S * S * NET_C3}


def bf16(v: float) -> float:
    return float(_load().orn_bf16(float(v)))


def _lab3(lab):
    return tuple(np.ascontiguousarray(v, np.float32) for v in lab)


def net_forward(lab, params, S: int, bf16_mode: bool = True, origin=(0, 0)):
    """Logits (H, W, 9) and the ReLU outputs a1, a2 (H, W, 32) of the net on
    a region whose top-left pixel is `origin` = (x, y) in the full image."""
    L, A, B = _lab3(lab)
    h, w = L.shape
    p = np.ascontiguousarray(params, np.float64)
    assert p.size == net_param_count(S)
    lg = np.empty((h, w, NET_C3), np.float64)
    a1 = np.empty((h, w, NET_C1), np.float64)
    a2 = np.empty((h, w, NET_C2), np.float64)
    _check(_load().orn_forward(w, h, origin[0], origin[1], S, _ptr(L), _ptr(A), _ptr(B), _ptr(p),
                               int(bf16_mode), _ptr(lg), _ptr(a1), _ptr(a2)), "net forward")
    return lg, a1, a2


def net_loss_grad(lab, params, S: int, target, bf16_mode: bool = True, origin=(0, 0),
                  want_grad: bool = True):
    """(mean cross-entropy, gradient or None)."""
    L, A, B = _lab3(lab)
    h, w = L.shape
    p = np.ascontiguousarray(params, np.float64)
    t = np.ascontiguousarray(target, np.int32)
    loss = ctypes.c_double()
    g = np.empty(p.size, np.float64) if want_grad else None
    _check(_load().orn_loss_grad(w, h, origin[0], origin[1], S, _ptr(L), _ptr(A), _ptr(B), _ptr(t),
                                 _ptr(p), int(bf16_mode), ctypes.byref(loss),
                                 _ptr(g) if want_grad else None), "net loss")
    return float(loss.value), g


def net_decode(logits, S: int):
    lg = np.ascontiguousarray(logits, np.float64)
    h, w, _ = lg.shape
    out = np.empty((h, w), np.int32)
    _check(_load().orn_decode(w, h, S, _ptr(lg), _ptr(out)), "net decode")
    return out


def net_votes(logits, min_confidence: float):
    """bool (H, W): the pixels whose best class has softmax probability at
    least min_confidence (they alone vote in the warm start's first update)."""
    lg = np.ascontiguousarray(logits, np.float64)
    h, w, _ = lg.shape
    out = np.empty((h, w), np.uint8)
    _check(_load().orn_votes(w, h, _ptr(lg), float(min_confidence), _ptr(out)), "net votes")
    return out.astype(bool)


def net_targets(labels, S: int):
    lb = np.ascontiguousarray(labels, np.int32)
    h, w = lb.shape
    out = np.empty((h, w), np.int32)
    _check(_load().orn_targets(w, h, S, _ptr(lb), _ptr(out)), "net targets")
    return out
