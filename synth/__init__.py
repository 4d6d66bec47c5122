"""Seeded synthetic Voronoi images: the inputs shared by the CPU oracle and
the GPU path (see ``synth.c`` for the recipe).  Holds none of the
segmentation arithmetic.

The paper's Table 1 photographs are not available; these images stand in
for them with the sizes and superpixel densities of the workloads below.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
# SLIC_SYNTH_LIB names another build of synth.c (see the sanitizer test).
_LIB = os.environ.get("SLIC_SYNTH_LIB") or os.path.join(_HERE, "libsynth.so")
SOURCE = _SRC


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` in place with gcc (no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math", _SRC, "-o", tmp, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.synth_voronoi.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_double, ctypes.c_double, ctypes.c_uint64]
        lib.synth_voronoi.restype = ctypes.c_int
        lib.synth_voronoi_sites_bruteforce.argtypes = [
            ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
        lib.synth_voronoi_sites_bruteforce.restype = ctypes.c_int
        _lib = lib
    return _lib


def voronoi_image(seed: int, width: int, height: int, regions: int, sigma: float,
                  ramp: float = 20.0, with_regions: bool = False):
    """uint8 array (height, width, 3), R,G,B.  With ``with_regions`` also
    returns the int32 (height, width) Voronoi region index map."""
    lib = _load()
    out = np.empty((height, width, 3), dtype=np.uint8)
    reg = np.empty((height, width), dtype=np.int32) if with_regions else None
    rc = lib.synth_voronoi(out.ctypes.data, reg.ctypes.data if with_regions else None,
                           width, height, regions, float(ramp), float(sigma),
                           ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF))
    if rc != 0:
        raise ValueError(f"synth_voronoi failed with code {rc}")
    return (out, reg) if with_regions else out


def voronoi_regions_bruteforce(seed: int, width: int, height: int, regions: int):
    lib = _load()
    reg = np.empty((height, width), dtype=np.int32)
    rc = lib.synth_voronoi_sites_bruteforce(reg.ctypes.data, width, height, regions,
                                            ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF))
    if rc != 0:
        raise ValueError(f"synth_voronoi_sites_bruteforce failed with code {rc}")
    return reg


from .configs import WORKLOADS, Workload, batch_workload, image_for  # noqa: E402

__all__ = ["build", "voronoi_image", "voronoi_regions_bruteforce", "WORKLOADS", "Workload",
           "batch_workload", "image_for"]
