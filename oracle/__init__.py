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
        lib.oracle_ncc_rgb_at.argtypes = [_u8p, _u8p, _i32, _i32, _i32, _i32, _i32, _i32]
        lib.oracle_ncc_rgb_at.restype = ctypes.c_double
        lib.oracle_cost_rgb_at.argtypes = [_u8p, _u8p] + [_i32] * 8
        lib.oracle_cost_rgb_at.restype = ctypes.c_int16
        lib.oracle_cost_volume_rgb.argtypes = [_u8p, _u8p] + [_i32] * 6 + [_i16p, _f64p]
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
        _u16p = ctypes.POINTER(ctypes.c_uint16)
        _f32p = ctypes.POINTER(ctypes.c_float)
        lib.oracle_bf16.argtypes = [ctypes.c_float]
        lib.oracle_bf16.restype = ctypes.c_uint16
        lib.oracle_warm_input.argtypes = [_u8p, _u8p, _i32, _i32, _i32, _i16p, _i32, _i32, _u16p]
        lib.oracle_conv3x3.argtypes = [_f64p, _i32, _i32, _i32, _f64p, _f64p, _i32, _f64p]
        lib.oracle_conv3x3_backward.argtypes = [_f64p, _i32, _i32, _i32, _f64p, _i32, _f64p, _f64p, _f64p, _f64p]
        lib.oracle_warm_messages.argtypes = [_f32p, _i32, _i32, _i32, _i32, _i16p]
        lib.oracle_warm_l1.argtypes = [_f32p, _i16p, _i32, _i32, _i32, _i32, _f64p]
        lib.oracle_warm_l1.restype = ctypes.c_double
        lib.oracle_adam.argtypes = [_f64p, _f64p, _f64p, _f64p, ctypes.c_int64, _i32, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.oracle_bp_energy.argtypes = [_i16p, _i16p, _i32, _i32, _i32, _i32, _i32]
        lib.oracle_lr_check.argtypes = [_i16p, _i16p, _i32, _i32, _i32, _i32, _i16p]
        lib.oracle_lr_check.restype = None
        lib.oracle_bp_energy.restype = ctypes.c_int64
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int32
        lib.oracle_set_threads.argtypes = [_i32]
        lib.oracle_set_threads.restype = None
        _lib = lib
    return _lib


def threads():
    """Host threads the oracle's row loops use."""
    return int(_load().oracle_threads())


def set_threads(n):
    """Use n host threads (n >= 1) in the oracle's row loops; results do not depend on n."""
    _load().oracle_set_threads(int(n))


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


def ncc_rgb_at(left, right, window, x, y, d):
    """Colour correlation of interleaved RGB views [H, W, 3] (channels pooled)."""
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    H, W, _ = left.shape
    return _load().oracle_ncc_rgb_at(_p(left, _u8p), _p(right, _u8p), W, H, window, x, y, d)


def cost_rgb_at(left, right, window, x, y, d, cost_scale=256, cost_trunc=1024):
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    H, W, _ = left.shape
    return int(_load().oracle_cost_rgb_at(_p(left, _u8p), _p(right, _u8p), W, H, window, x, y, d,
                                          cost_scale, cost_trunc))


def cost_volume_rgb(left, right, num_disp, window, cost_scale=256, cost_trunc=1024, want_ncc=False):
    """Colour cost volume int16 [H, W, D] from interleaved RGB views [H, W, 3]."""
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    H, W, C = left.shape
    if C != 3 or right.shape != left.shape:
        raise ValueError("views must be interleaved RGB [H, W, 3] of one shape")
    cost = np.empty((H, W, num_disp), np.int16)
    ncc = np.empty((H, W, num_disp), np.float64) if want_ncc else None
    _load().oracle_cost_volume_rgb(_p(left, _u8p), _p(right, _u8p), W, H, num_disp, window, cost_scale,
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


def lr_check(disp_left, disp_right, num_disp, tol):
    """Left disparities kept where the right view agrees within tol, -1 elsewhere."""
    dl, dr = _c(disp_left, np.int16), _c(disp_right, np.int16)
    H, W = dl.shape
    out = np.empty((H, W), np.int16)
    _load().oracle_lr_check(_p(dl, _i16p), _p(dr, _i16p), W, H, num_disp, tol, _p(out, _i16p))
    return out


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


# ---------------------------------------------------------------- learned warm start
_f32 = np.float32


def bf16(a):
    """bf16 bit patterns (uint16) of float32 values, round to nearest even."""
    a = np.ascontiguousarray(a, dtype=np.float32).ravel()
    lib = _load()
    out = np.array([lib.oracle_bf16(float(v)) for v in a], dtype=np.uint16)
    return out


def bf16_value(bits):
    """float32 values of bf16 bit patterns."""
    b = np.ascontiguousarray(bits, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


def warm_input(left, right, s, coarse, cin_p):
    """CNN input [Hs, Ws, cin_p] (bf16 bits) at scale s from the views and the scale-(s+1) cost."""
    left, right, coarse = _c(left, np.uint8), _c(right, np.uint8), _c(coarse, np.int16)
    H, W = left.shape
    D = coarse.shape[2]
    Ws, Hs = W, H
    for _ in range(s):
        Ws, Hs = (Ws + 1) // 2, (Hs + 1) // 2
    out = np.empty((Hs, Ws, cin_p), np.uint16)
    _load().oracle_warm_input(_p(left, _u8p), _p(right, _u8p), W, H, s, _p(coarse, _i16p), D, cin_p,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)))
    return out


def conv3x3(x, w, b):
    """x [H, W, Cin] float64, w [Cout, 9, Cin], b [Cout] -> z [H, W, Cout] (zero padding)."""
    x = _c(x, np.float64)
    w = _c(w, np.float64)
    H, W, Cin = x.shape
    Cout = w.shape[0]
    b = _c(b, np.float64) if b is not None else None
    z = np.empty((H, W, Cout), np.float64)
    _load().oracle_conv3x3(_p(x, _f64p), H, W, Cin, _p(w, _f64p), _p(b, _f64p) if b is not None else None, Cout,
                           _p(z, _f64p))
    return z


def conv3x3_backward(x, w, dz, want_dx=True):
    x, w, dz = _c(x, np.float64), _c(w, np.float64), _c(dz, np.float64)
    H, W, Cin = x.shape
    Cout = w.shape[0]
    dx = np.empty_like(x) if want_dx else None
    dw = np.empty_like(w)
    db = np.empty(Cout, np.float64)
    _load().oracle_conv3x3_backward(_p(x, _f64p), H, W, Cin, _p(w, _f64p), Cout, _p(dz, _f64p),
                                    _p(dx, _f64p) if want_dx else None, _p(dw, _f64p), _p(db, _f64p))
    return dx, dw, db


def warm_messages(y, D, lam_t):
    """Initial messages [4, Hs, Ws, D] int16 from the CNN output y [Hs, Ws, 4D] float32."""
    y = _c(y, np.float32)
    Hs, Ws, _ = y.shape
    out = np.empty((4, Hs, Ws, D), np.int16)
    _load().oracle_warm_messages(y.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), Ws, Hs, D, lam_t,
                                 _p(out, _i16p))
    return out


def warm_l1(y, label, lam_t, want_grad=True):
    y, label = _c(y, np.float32), _c(label, np.int16)
    Hs, Ws, C = y.shape
    D = C // 4
    dy = np.empty((Hs, Ws, C), np.float64) if want_grad else None
    loss = _load().oracle_warm_l1(y.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _p(label, _i16p), Ws, Hs, D,
                                  lam_t, _p(dy, _f64p) if want_grad else None)
    return loss, dy


def adam(w, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (w, m, v, g):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().oracle_adam(_p(w, _f64p), _p(m, _f64p), _p(v, _f64p), _p(g, _f64p), w.size, step, lr, b1, b2, eps)
