"""Seeded synthetic stereo inputs.

Makes the left/right views, ground-truth disparity and occlusion mask that the tests
and the benchmark feed to both the CPU checker and the GPU library.  The arithmetic
lives in ``synth.c`` (built into ``libsynth.so`` next to this file); this module holds
no part of the stereo method itself.

The workload presets below describe the five synthetic configurations the library is
measured and tested on: their image sizes, disparity ranges, plane counts, NCC window,
hierarchy depth, half-steps per scale and smoothness parameters.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


class SynthSpec(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("num_disp", ctypes.c_int32),
        ("planes_min", ctypes.c_int32),
        ("planes_max", ctypes.c_int32),
        ("background", ctypes.c_int32),
        ("slabs", ctypes.c_int32),
        ("rgb", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')"
            )
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_pair.argtypes = [ctypes.POINTER(SynthSpec)] + [ctypes.c_void_p] * 4
        lib.synth_pair.restype = ctypes.c_int
        lib.synth_batch_shape.argtypes = [ctypes.c_uint64] + [ctypes.POINTER(ctypes.c_int32)] * 4
        lib.synth_batch_shape.restype = None
        _lib = lib
    return _lib


def make_pair(width, height, num_disp, planes=(4, 4), background=False, slabs=0, rgb=False, seed=1):
    """Return dict(left, right, gt, occ) as numpy arrays.

    left/right are uint8 [H, W] (or [H, W, 3] when rgb), gt is int16 [H, W] and occ is
    uint8 [H, W] (1 = the left pixel has no visible match in the right view).
    """
    lib = _load()
    spec = SynthSpec(int(width), int(height), int(num_disp), int(planes[0]), int(planes[1]),
                     1 if background else 0, int(slabs), 1 if rgb else 0, 0, int(seed) & (2**64 - 1))
    shape = (height, width, 3) if rgb else (height, width)
    left = np.empty(shape, np.uint8)
    right = np.empty(shape, np.uint8)
    gt = np.empty((height, width), np.int16)
    occ = np.empty((height, width), np.uint8)
    rc = lib.synth_pair(ctypes.byref(spec), left.ctypes.data, right.ctypes.data, gt.ctypes.data, occ.ctypes.data)
    if rc != 0:
        raise ValueError(f"bad synthetic spec {spec}")
    return {"left": left, "right": right, "gt": gt, "occ": occ}


def batch_shape(seed):
    """(width, height, num_disp, planes) of one pair of the uneven batch."""
    lib = _load()
    vals = [ctypes.c_int32() for _ in range(4)]
    lib.synth_batch_shape(ctypes.c_uint64(int(seed)), *[ctypes.byref(v) for v in vals])
    return tuple(v.value for v in vals)


# Workload presets.  lam/trunc: truncated-linear smoothness lam*min(|dp-dq|, trunc);
# iters: half-steps per scale (finest first); skip: 0 plain, 1 converged-pixel freeze.
WORKLOADS = {
    "tiny": dict(width=128, height=96, num_disp=16, planes=(4, 4), background=False, slabs=0, rgb=False,
                 seed=1, window=5, num_scales=3, iters=8, lam=64, trunc=4, skip=0,
                 cost_scale=256, cost_trunc=1024),
    "production": dict(width=384, height=288, num_disp=16, planes=(8, 12), background=True, slabs=0,
                       rgb=False, seed=2, window=7, num_scales=4, iters=10, lam=64, trunc=4, skip=1,
                       cost_scale=256, cost_trunc=1024),
    "large": dict(width=1920, height=1080, num_disp=128, planes=(40, 40), background=False, slabs=12,
                  rgb=True, seed=3, window=9, num_scales=5, iters=12, lam=64, trunc=4, skip=0,
                  cost_scale=256, cost_trunc=1024),
}

BATCH = dict(count=256, seed0=1000, window=7, num_scales=4, iters=10, lam=64, trunc=4, skip=0,
             cost_scale=256, cost_trunc=1024)


def workload_pair(name):
    """The synthetic pair of a named workload preset."""
    w = WORKLOADS[name]
    return make_pair(w["width"], w["height"], w["num_disp"], w["planes"], w["background"], w["slabs"],
                     w["rgb"], w["seed"])


def batch_pair(i, seed0=BATCH["seed0"]):
    """Pair i of the uneven batch (grey, no background, no slabs)."""
    seed = seed0 + i
    W, H, D, planes = batch_shape(seed)
    p = make_pair(W, H, D, (planes, planes), False, 0, False, seed)
    p["num_disp"] = D
    return p
