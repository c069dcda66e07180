"""ORACLE — test infrastructure only.

Python access to the plain CPU implementation in ``bp_oracle.c`` (built into
``liboracle.so`` beside this file by ``oracle.build.build()``).  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this package; the GPU
library never does, and the two share no code.

All functions take and return numpy arrays in the layouts of ``bp_oracle.h``:
images uint8 [H, W], cost int16 [H, W, D], messages int16 [4, H, W, D] with
direction k = 0 from-left, 1 from-right, 2 from-up, 3 from-down.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_i16p = ctypes.POINTER(ctypes.c_int16)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.c_int32


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("num_disp", ctypes.c_int32),
        ("num_scales", ctypes.c_int32),
        ("iters", ctypes.c_int32 * 8),
        ("lambda_", ctypes.c_int32),
        ("trunc", ctypes.c_int32),
        ("skip_mode", ctypes.c_int32),
        ("converge_iters", ctypes.c_int32),
        ("warm_msgs", ctypes.c_void_p),
    ]


class OracleStats(ctypes.Structure):
    _fields_ = [
        ("msg_updates", ctypes.c_int64),
        ("pixel_updates", ctypes.c_int64),
        ("n_halfsteps", ctypes.c_int32 * 8),
        ("active", (ctypes.c_int32 * 64) * 8),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.oracle_luma.argtypes = [_u8p, _i32, _i32, _u8p]
        lib.oracle_ncc_at.argtypes = [_u8p, _u8p, _i32, _i32, _i32, _i32, _i32, _i32]
        lib.oracle_ncc_at.restype = ctypes.c_double
        lib.oracle_cost_at.argtypes = [_u8p, _u8p] + [_i32] * 8
        lib.oracle_cost_at.restype = ctypes.c_int16
        lib.oracle_cost_volume.argtypes = [_u8p, _u8p] + [_i32] * 6 + [_i16p, _f64p]
        lib.oracle_pyramid_level.argtypes = [_i16p, _i32, _i32, _i32, _i16p]
        lib.oracle_message.argtypes = [_i32p, _i32, _i32, _i32, _i16p]
        lib.oracle_bp_solve.argtypes = [_i16p, _i32, _i32, ctypes.POINTER(OracleParams), _i16p, _i16p,
                                        ctypes.POINTER(OracleStats)]
        lib.oracle_bp_solve.restype = ctypes.c_int32
        for fn in (lib.oracle_bp_flat_checkerboard, lib.oracle_bp_flat_jacobi):
            fn.argtypes = [_i16p, _i32, _i32, _i32, _i32, _i32, _i32, _i16p, _i16p]
            fn.restype = ctypes.c_int32
        lib.oracle_wta.argtypes = [_i16p, _i16p, _i32, _i32, _i32, _i16p]
        lib.oracle_message_at.argtypes = [_i16p, _i16p] + [_i32] * 8 + [_i16p]
        lib.oracle_message_at.restype = ctypes.c_int32
        lib.oracle_wta_at.argtypes = [_i16p, _i16p] + [_i32] * 5
        lib.oracle_wta_at.restype = ctypes.c_int32
        lib.oracle_bp_energy.argtypes = [_i16p, _i16p, _i32, _i32, _i32, _i32, _i32]
        lib.oracle_bp_energy.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def luma(rgb):
    rgb = _c(rgb, np.uint8)
    H, W, _ = rgb.shape
    out = np.empty((H, W), np.uint8)
    _load().oracle_luma(_p(rgb, _u8p), W, H, _p(out, _u8p))
    return out


def ncc_at(left, right, window, x, y, d):
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    H, W = left.shape
    return _load().oracle_ncc_at(_p(left, _u8p), _p(right, _u8p), W, H, window, x, y, d)


def cost_at(left, right, window, x, y, d, cost_scale=256, cost_trunc=1024):
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    H, W = left.shape
    return int(_load().oracle_cost_at(_p(left, _u8p), _p(right, _u8p), W, H, window, x, y, d,
                                      cost_scale, cost_trunc))


def cost_volume(left, right, num_disp, window, cost_scale=256, cost_trunc=1024, want_ncc=False):
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    H, W = left.shape
    cost = np.empty((H, W, num_disp), np.int16)
    ncc = np.empty((H, W, num_disp), np.float64) if want_ncc else None
    _load().oracle_cost_volume(_p(left, _u8p), _p(right, _u8p), W, H, num_disp, window, cost_scale,
                               cost_trunc, _p(cost, _i16p), _p(ncc, _f64p) if want_ncc else None)
    return (cost, ncc) if want_ncc else cost


def pyramid_level(cost):
    cost = _c(cost, np.int16)
    H, W, D = cost.shape
    out = np.empty(((H + 1) // 2, (W + 1) // 2, D), np.int16)
    _load().oracle_pyramid_level(_p(cost, _i16p), W, H, D, _p(out, _i16p))
    return out


def message(h, lam, trunc):
    h = _c(h, np.int32)
    out = np.empty(h.shape[0], np.int16)
    _load().oracle_message(_p(h, _i32p), h.shape[0], lam, trunc, _p(out, _i16p))
    return out


def make_params(num_disp, num_scales, iters, lam, trunc, skip_mode=0, converge_iters=2, warm_msgs=None):
    p = OracleParams()
    p.num_disp = num_disp
    p.num_scales = num_scales
    its = list(iters) if hasattr(iters, "__len__") else [iters] * num_scales
    for i in range(8):
        p.iters[i] = its[i] if i < len(its) else 0
    p.lambda_ = lam
    p.trunc = trunc
    p.skip_mode = skip_mode
    p.converge_iters = converge_iters
    p.warm_msgs = warm_msgs.ctypes.data if warm_msgs is not None else None
    return p


def bp_solve(cost, num_scales, iters, lam, trunc, skip_mode=0, converge_iters=2, warm_msgs=None,
             want_msgs=True):
    """Hierarchical solve.  Returns (disparity int16 [H,W], msgs [4,H,W,D] or None, stats dict)."""
    cost = _c(cost, np.int16)
    H, W, D = cost.shape
    if warm_msgs is not None:
        warm_msgs = _c(warm_msgs, np.int16)
    p = make_params(D, num_scales, iters, lam, trunc, skip_mode, converge_iters, warm_msgs)
    disp = np.empty((H, W), np.int16)
    msgs = np.empty((4, H, W, D), np.int16) if want_msgs else None
    st = OracleStats()
    rc = _load().oracle_bp_solve(_p(cost, _i16p), W, H, ctypes.byref(p), _p(disp, _i16p),
                                 _p(msgs, _i16p) if want_msgs else None, ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle_bp_solve rejected its arguments")
    stats = {
        "msg_updates": st.msg_updates,
        "pixel_updates": st.pixel_updates,
        "n_halfsteps": list(st.n_halfsteps),
        "active": np.array([[st.active[l][t] for t in range(64)] for l in range(8)], np.int64),
    }
    return disp, msgs, stats


def _flat(fn, cost, lam, trunc, n, init):
    cost = _c(cost, np.int16)
    H, W, D = cost.shape
    init = np.zeros((4, H, W, D), np.int16) if init is None else _c(init, np.int16)
    out = np.empty((4, H, W, D), np.int16)
    rc = fn(_p(cost, _i16p), W, H, D, lam, trunc, n, _p(init, _i16p), _p(out, _i16p))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def flat_checkerboard(cost, lam, trunc, halfsteps, init=None):
    return _flat(_load().oracle_bp_flat_checkerboard, cost, lam, trunc, halfsteps, init)


def flat_jacobi(cost, lam, trunc, iterations, init=None):
    return _flat(_load().oracle_bp_flat_jacobi, cost, lam, trunc, iterations, init)


def wta(cost, msgs):
    cost, msgs = _c(cost, np.int16), _c(msgs, np.int16)
    H, W, D = cost.shape
    out = np.empty((H, W), np.int16)
    _load().oracle_wta(_p(cost, _i16p), _p(msgs, _i16p), W, H, D, _p(out, _i16p))
    return out


def energy(cost, disparity, lam, trunc):
    cost, disparity = _c(cost, np.int16), _c(disparity, np.int16)
    H, W, D = cost.shape
    return int(_load().oracle_bp_energy(_p(cost, _i16p), _p(disparity, _i16p), W, H, D, lam, trunc))


def message_at(cost, msgs, lam, trunc, x, y, k):
    """Message pixel (x, y) sends to its neighbour on side k, from the state (cost, msgs)."""
    cost, msgs = _c(cost, np.int16), _c(msgs, np.int16)
    H, W, D = cost.shape
    out = np.empty(D, np.int16)
    rc = _load().oracle_message_at(_p(cost, _i16p), _p(msgs, _i16p), W, H, D, lam, trunc, x, y, k, _p(out, _i16p))
    return out if rc == 0 else None


def wta_at(cost, msgs, x, y):
    cost, msgs = _c(cost, np.int16), _c(msgs, np.int16)
    H, W, D = cost.shape
    return int(_load().oracle_wta_at(_p(cost, _i16p), _p(msgs, _i16p), W, H, D, x, y))
