"""Python binding of the C ABI in include/bpstereo.h (libbpstereo.so, built in-tree).

Argument marshalling only: tensors are checked for device, dtype, layout and shape,
outputs and workspaces are allocated with PyTorch on the current device, and each call
goes straight to the library on torch's current stream.  Every step of the method runs
in the library's HIP kernels; if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbpstereo.so")

BP_OK, BP_E_INVAL, BP_E_NOMEM, BP_E_HIP, BP_E_UNSUPPORTED, BP_E_WORKSPACE = 0, -1, -2, -3, -4, -5


class BPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bpstereo error {code}: {msg}")
        self.code = code


class BPParams(ctypes.Structure):
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


class BPStats(ctypes.Structure):
    _fields_ = [
        ("msg_updates", ctypes.c_int64),
        ("pixel_updates", ctypes.c_int64),
        ("n_halfsteps", ctypes.c_int32 * 8),
        ("active", (ctypes.c_int32 * 64) * 8),
    ]


class BPTiming(ctypes.Structure):
    _fields_ = [
        ("halfstep_ms", ctypes.c_double),
        ("halfstep_launches", ctypes.c_int64),
        ("halfstep_pixel_updates_max", ctypes.c_int64),
        ("scale_ms", ctypes.c_double * 8),
        ("scale_launches", ctypes.c_int64 * 8),
    ]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(LIB_PATH)
        lib.bp_last_error.restype = ctypes.c_char_p
        lib.bp_context_create.argtypes = [ctypes.POINTER(_vp)]
        lib.bp_context_destroy.argtypes = [_vp]
        lib.bp_context_set_timing.argtypes = [_vp, _i32]
        lib.bp_context_set_graphs.argtypes = [_vp, _i32]
        lib.bp_context_set_fused.argtypes = [_vp, _i32]
        lib.bp_context_graph_counts.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
        lib.bp_context_take_timing.argtypes = [_vp, ctypes.POINTER(BPTiming)]
        lib.stereo_luma.argtypes = [_vp, _i32, _i32, _vp, _vp]
        lib.stereo_cost_volume.argtypes = [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp]
        lib.stereo_cost_volume_rgb.argtypes = [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp]
        lib.bp_workspace_bytes.argtypes = [_i32, _i32, ctypes.POINTER(BPParams)]
        lib.bp_workspace_bytes.restype = ctypes.c_size_t
        lib.bp_message_bits.argtypes = [_i32, _i32, ctypes.POINTER(BPParams)]
        lib.bp_message_bits.restype = ctypes.c_int32
        lib.bp_hierarchical_solve.argtypes = [_vp, _vp, _i32, _i32, ctypes.POINTER(BPParams), _vp, ctypes.c_size_t,
                                              _vp, _vp, ctypes.POINTER(BPStats), _vp]
        lib.bp_hierarchical_solve_noalloc.argtypes = [_vp, _vp, _i32, _i32, ctypes.POINTER(BPParams), _vp, _vp,
                                                      ctypes.POINTER(BPStats), _vp]
        lib.bp_noalloc_scratch_bytes.argtypes = []
        lib.bp_noalloc_scratch_bytes.restype = ctypes.c_size_t
        lib.bp_energy_workspace_bytes.argtypes = [_i32, _i32]
        lib.bp_energy_workspace_bytes.restype = ctypes.c_size_t
        lib.bp_energy.argtypes = [_vp, _vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp, ctypes.c_size_t, _vp]
        lib.bp_lr_check.argtypes = [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp]
        lib.bp_jacobi_workspace_bytes.argtypes = [_i32, _i32, _i32]
        lib.bp_jacobi_workspace_bytes.restype = ctypes.c_size_t
        lib.bp_jacobi_iterations.argtypes = [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, ctypes.c_size_t,
                                             _vp]
        for name in ("bp_context_create", "bp_context_destroy", "bp_context_set_timing", "bp_context_take_timing",
                     "bp_context_set_graphs", "bp_context_set_fused", "bp_context_graph_counts",
                     "stereo_luma", "stereo_cost_volume", "stereo_cost_volume_rgb", "bp_hierarchical_solve", "bp_hierarchical_solve_noalloc",
                     "bp_energy",
                     "bp_jacobi_iterations", "bp_lr_check"):
            getattr(lib, name).restype = ctypes.c_int32
        _lib = lib
    return _lib


def library():
    """The loaded ctypes library (loads it on first use)."""
    return _load()


def _check(rc):
    if rc != BP_OK:
        raise BPError(rc, _load().bp_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, ndim, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owner of a bp_context (timing events); one per stream."""

    def __init__(self):
        h = _vp()
        _check(_load().bp_context_create(ctypes.byref(h)))
        self.handle = h

    def set_timing(self, on=True):
        """Event timing of the message-update launches: True or 1 per launch, 2 per scale's
        run of launches, False or 0 off."""
        _check(_load().bp_context_set_timing(self.handle, int(on)))

    def set_graphs(self, on=True):
        _check(_load().bp_context_set_graphs(self.handle, 1 if on else 0))

    def set_fused(self, mode):
        """Half-steps per launch on small scales: 0 one each, 1 several wherever they fit, 2 by size."""
        _check(_load().bp_context_set_fused(self.handle, int(mode)))

    def graph_counts(self):
        c = (ctypes.c_int64 * 3)()
        _check(_load().bp_context_graph_counts(self.handle, c))
        return {"captures": c[0], "replays": c[1], "fallbacks": c[2]}

    def take_timing(self):
        t = BPTiming()
        _check(_load().bp_context_take_timing(self.handle, ctypes.byref(t)))
        return {"halfstep_ms": t.halfstep_ms, "halfstep_launches": t.halfstep_launches,
                "halfstep_pixel_updates_max": t.halfstep_pixel_updates_max,
                "scale_ms": list(t.scale_ms), "scale_launches": list(t.scale_launches)}

    def close(self):
        if self.handle:
            _check(_load().bp_context_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stereo_luma(rgb, out=None, stream=None):
    H, W, C = rgb.shape
    if C != 3:
        raise ValueError("rgb must be [H, W, 3]")
    p = _dev(rgb, torch.uint8, 3, "rgb")
    out = torch.empty((H, W), dtype=torch.uint8, device=rgb.device) if out is None else out
    _check(_load().stereo_luma(p, W, H, _dev(out, torch.uint8, 2, "out"), _stream(stream)))
    return out


def stereo_cost_volume(left, right, num_disp, window, cost_scale=256, cost_trunc=1024, want_ncc=False, out=None,
                       stream=None):
    """Quantised NCC cost volume int16 [H, W, D] (and the float NCC if want_ncc)."""
    H, W = left.shape
    if tuple(right.shape) != (H, W):
        raise ValueError("left and right must have the same shape")
    lp, rp = _dev(left, torch.uint8, 2, "left"), _dev(right, torch.uint8, 2, "right")
    cost = torch.empty((H, W, num_disp), dtype=torch.int16, device=left.device) if out is None else out
    if tuple(cost.shape) != (H, W, num_disp):
        raise ValueError("out has the wrong shape")
    ncc = torch.empty((H, W, num_disp), dtype=torch.float32, device=left.device) if want_ncc else None
    _check(_load().stereo_cost_volume(lp, rp, W, H, num_disp, window, cost_scale, cost_trunc,
                                      _dev(cost, torch.int16, 3, "cost"),
                                      _dev(ncc, torch.float32, 3, "ncc") if want_ncc else None, _stream(stream)))
    return (cost, ncc) if want_ncc else cost


def stereo_cost_volume_rgb(left, right, num_disp, window, cost_scale=256, cost_trunc=1024, want_ncc=False, out=None,
                           stream=None):
    """Quantised colour NCC cost volume int16 [H, W, D] of interleaved RGB views [H, W, 3]."""
    H, W, C = left.shape
    if C != 3 or tuple(right.shape) != (H, W, 3):
        raise ValueError("left and right must be [H, W, 3] of one shape")
    lp, rp = _dev(left, torch.uint8, 3, "left"), _dev(right, torch.uint8, 3, "right")
    cost = torch.empty((H, W, num_disp), dtype=torch.int16, device=left.device) if out is None else out
    if tuple(cost.shape) != (H, W, num_disp):
        raise ValueError("out has the wrong shape")
    ncc = torch.empty((H, W, num_disp), dtype=torch.float32, device=left.device) if want_ncc else None
    _check(_load().stereo_cost_volume_rgb(lp, rp, W, H, num_disp, window, cost_scale, cost_trunc,
                                          _dev(cost, torch.int16, 3, "cost"),
                                          _dev(ncc, torch.float32, 3, "ncc") if want_ncc else None, _stream(stream)))
    return (cost, ncc) if want_ncc else cost


def make_params(num_disp, num_scales, iters, lam, trunc, skip_mode=0, converge_iters=2, warm_msgs=None):
    p = BPParams()
    p.num_disp = num_disp
    p.num_scales = num_scales
    its = list(iters) if hasattr(iters, "__len__") else [int(iters)] * num_scales
    for i in range(8):
        p.iters[i] = its[i] if i < len(its) else 0
    p.lambda_ = lam
    p.trunc = trunc
    p.skip_mode = skip_mode
    p.converge_iters = converge_iters
    p.warm_msgs = _dev(warm_msgs, torch.int16, 4, "warm_msgs").value if warm_msgs is not None else None
    return p


def bp_workspace_bytes(width, height, params):
    return int(_load().bp_workspace_bytes(width, height, ctypes.byref(params)))


def bp_message_bits(width, height, params):
    """Bits per label of the solve's stored messages (12 or 16; 0 for invalid arguments)."""
    return int(_load().bp_message_bits(width, height, ctypes.byref(params)))


def bp_hierarchical_solve(cost, num_scales, iters, lam, trunc, skip_mode=0, converge_iters=2, warm_msgs=None,
                          want_msgs=False, want_stats=False, ctx=None, workspace=None, disparity=None, stream=None):
    """Returns (disparity int16 [H, W], messages int16 [4, H, W, D] or None, stats dict or None)."""
    H, W, D = cost.shape
    cp = _dev(cost, torch.int16, 3, "cost")
    if warm_msgs is not None:
        hs, ws = H, W
        for _ in range(num_scales - 2):
            hs, ws = (hs + 1) // 2, (ws + 1) // 2
        if tuple(warm_msgs.shape) != (4, hs, ws, D):
            raise ValueError(f"warm_msgs must be [4, {hs}, {ws}, {D}] (scale {num_scales - 2}), got "
                             f"{tuple(warm_msgs.shape)}")
    p = make_params(D, num_scales, iters, lam, trunc, skip_mode, converge_iters, warm_msgs)
    need = bp_workspace_bytes(W, H, p)
    if need == 0:
        raise BPError(BP_E_INVAL, "invalid solve parameters")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=cost.device)
    disp = torch.empty((H, W), dtype=torch.int16, device=cost.device) if disparity is None else disparity
    msgs = torch.empty((4, H, W, D), dtype=torch.int16, device=cost.device) if want_msgs else None
    st = BPStats() if want_stats else None
    _check(_load().bp_hierarchical_solve(ctx.handle if ctx is not None else None, cp, W, H, ctypes.byref(p),
                                         ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                         _dev(disp, torch.int16, 2, "disparity"),
                                         _dev(msgs, torch.int16, 4, "msgs") if want_msgs else None,
                                         ctypes.byref(st) if want_stats else None, _stream(stream)))
    stats = None
    if want_stats:
        stats = {"msg_updates": st.msg_updates, "pixel_updates": st.pixel_updates,
                 "n_halfsteps": list(st.n_halfsteps),
                 "active": [[st.active[l][t] for t in range(64)] for l in range(8)]}
    return disp, msgs, stats


def bp_noalloc_scratch_bytes():
    """Bytes of the library's static per-device scratch (the largest solve workspace the
    allocation-free solve accepts)."""
    return int(_load().bp_noalloc_scratch_bytes())


def bp_hierarchical_solve_noalloc(cost, num_scales, iters, lam, trunc, skip_mode=0, converge_iters=2, warm_msgs=None,
                                  want_msgs=False, want_stats=False, ctx=None, disparity=None, msgs=None, stream=None):
    """As bp_hierarchical_solve, with the library's static device scratch as its workspace
    (the C call allocates no device memory).  Pass `disparity` (and `msgs`) to have this
    wrapper allocate nothing either.  Returns (disparity, messages or None, stats or None)."""
    H, W, D = cost.shape
    cp = _dev(cost, torch.int16, 3, "cost")
    p = make_params(D, num_scales, iters, lam, trunc, skip_mode, converge_iters, warm_msgs)
    disp = torch.empty((H, W), dtype=torch.int16, device=cost.device) if disparity is None else disparity
    if want_msgs and msgs is None:
        msgs = torch.empty((4, H, W, D), dtype=torch.int16, device=cost.device)
    st = BPStats() if want_stats else None
    _check(_load().bp_hierarchical_solve_noalloc(ctx.handle if ctx is not None else None, cp, W, H, ctypes.byref(p),
                                                 _dev(disp, torch.int16, 2, "disparity"),
                                                 _dev(msgs, torch.int16, 4, "msgs") if want_msgs else None,
                                                 ctypes.byref(st) if want_stats else None, _stream(stream)))
    stats = None
    if want_stats:
        stats = {"msg_updates": st.msg_updates, "pixel_updates": st.pixel_updates,
                 "n_halfsteps": list(st.n_halfsteps),
                 "active": [[st.active[l][t] for t in range(64)] for l in range(8)]}
    return disp, (msgs if want_msgs else None), stats


def bp_energy_workspace_bytes(width, height):
    return int(_load().bp_energy_workspace_bytes(width, height))


def bp_energy(cost, disparity, lam, trunc, workspace=None, out=None, stream=None):
    """E(d) as an int64 GPU tensor of one element (INT64_MIN if a disparity is out of range)."""
    H, W, D = cost.shape
    if tuple(disparity.shape) != (H, W):
        raise ValueError("disparity must be [H, W]")
    need = bp_energy_workspace_bytes(W, H)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=cost.device)
    out = torch.empty(1, dtype=torch.int64, device=cost.device) if out is None else out
    _check(_load().bp_energy(_dev(cost, torch.int16, 3, "cost"), _dev(disparity, torch.int16, 2, "disparity"), W, H,
                             D, lam, trunc, _dev(out, torch.int64, 1, "energy"),
                             ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream(stream)))
    return out


def bp_lr_check(disp_left, disp_right, num_disp, tol, out=None, stream=None):
    """Left disparities kept where the right-reference map agrees within tol, -1 elsewhere."""
    H, W = disp_left.shape
    if tuple(disp_right.shape) != (H, W):
        raise ValueError("disp_right must be [H, W] like disp_left")
    out = torch.empty((H, W), dtype=torch.int16, device=disp_left.device) if out is None else out
    _check(_load().bp_lr_check(_dev(disp_left, torch.int16, 2, "disp_left"), _dev(disp_right, torch.int16, 2, "disp_right"),
                               W, H, num_disp, tol, _dev(out, torch.int16, 2, "out"), _stream(stream)))
    return out


def bp_jacobi_workspace_bytes(width, height, num_disp):
    return int(_load().bp_jacobi_workspace_bytes(width, height, num_disp))


def bp_jacobi_iterations(cost, lam, trunc, iterations, init=None, workspace=None, out=None, stream=None):
    """Flat Jacobi min-sum iterations on one scale: the int16 messages [4, H, W, D] after
    `iterations` iterations from `init` (zeros if None)."""
    H, W, D = cost.shape
    need = bp_jacobi_workspace_bytes(W, H, D)
    if need == 0:
        raise ValueError("bad sizes")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=cost.device)
    out = torch.empty((4, H, W, D), dtype=torch.int16, device=cost.device) if out is None else out
    ip = None if init is None else _dev(init, torch.int16, 4, "init")
    _check(_load().bp_jacobi_iterations(_dev(cost, torch.int16, 3, "cost"), W, H, D, lam, trunc, iterations, ip,
                                        _dev(out, torch.int16, 4, "out"), ctypes.c_void_p(workspace.data_ptr()),
                                        workspace.numel(), _stream(stream)))
    return out


# ---------------------------------------------------------------------------------------- batched solve
class PairDesc(ctypes.Structure):
    _fields_ = [("left", ctypes.c_void_p), ("right", ctypes.c_void_p), ("cost", ctypes.c_void_p),
                ("disparity", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("num_disp", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class BatchParams(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("cost_scale", ctypes.c_int32), ("cost_trunc", ctypes.c_int32),
                ("num_scales", ctypes.c_int32), ("iters", ctypes.c_int32 * 8), ("lambda_", ctypes.c_int32),
                ("trunc", ctypes.c_int32), ("skip_mode", ctypes.c_int32), ("converge_iters", ctypes.c_int32)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32), ("schedule", ctypes.c_int32 * 16), ("blocks_per_cu", ctypes.c_int32 * 16),
                ("order", ctypes.c_int32 * 16), ("ms", ctypes.c_float * 16), ("best", ctypes.c_int32)]


def _batch_sigs(lib):
    if getattr(lib, "_batch_ready", False):
        return
    lib.bp_batch_workspace_bytes.argtypes = [ctypes.POINTER(PairDesc), _i32, ctypes.POINTER(BatchParams)]
    lib.bp_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.bp_batch_message_bits.argtypes = [ctypes.POINTER(PairDesc), _i32, ctypes.POINTER(BatchParams)]
    lib.bp_batch_message_bits.restype = ctypes.c_int32
    lib.bp_solve_batched.argtypes = [_vp, ctypes.POINTER(PairDesc), _i32, ctypes.POINTER(BatchParams), _vp,
                                     ctypes.c_size_t, _vp]
    lib.bp_solve_batched.restype = ctypes.c_int32
    lib.bp_batch_status.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_int32)]
    lib.bp_batch_status.restype = ctypes.c_int32
    lib.bp_autotune_batched.argtypes = [_vp, ctypes.POINTER(PairDesc), _i32, ctypes.POINTER(BatchParams), _vp,
                                        ctypes.c_size_t, _vp, ctypes.POINTER(BatchTuning)]
    lib.bp_autotune_batched.restype = ctypes.c_int32
    lib.bp_context_set_batch_schedule.argtypes = [_vp, _i32, _i32, _i32]
    lib.bp_context_set_batch_schedule.restype = ctypes.c_int32
    lib._batch_ready = True


def make_batch_params(window, num_scales, iters, lam, trunc, skip_mode=0, converge_iters=2, cost_scale=256,
                      cost_trunc=1024):
    p = BatchParams()
    p.window, p.cost_scale, p.cost_trunc, p.num_scales = window, cost_scale, cost_trunc, num_scales
    its = list(iters) if hasattr(iters, "__len__") else [int(iters)] * num_scales
    for i in range(8):
        p.iters[i] = its[i] if i < len(its) else 0
    p.lambda_, p.trunc, p.skip_mode, p.converge_iters = lam, trunc, skip_mode, converge_iters
    return p


class Batch:
    """A batch of pairs with its GPU buffers: per-pair cost volumes and disparities and the
    workspace of bp_solve_batched.  lefts/rights: lists of uint8 [H, W] GPU tensors."""

    def __init__(self, lefts, rights, num_disps, params):
        if not (len(lefts) == len(rights) == len(num_disps)) or not lefts:
            raise ValueError("lefts, rights and num_disps must be non-empty lists of one length")
        lib = _load()
        _batch_sigs(lib)
        self.params = params
        self.lefts, self.rights = list(lefts), list(rights)
        self.costs, self.disps = [], []
        n = len(lefts)
        self.descs = (PairDesc * n)()
        for i, (l, r, D) in enumerate(zip(lefts, rights, num_disps)):
            H, W = l.shape
            if tuple(r.shape) != (H, W):
                raise ValueError(f"pair {i}: left and right differ in shape")
            c = torch.empty((H, W, D), dtype=torch.int16, device=l.device)
            d = torch.empty((H, W), dtype=torch.int16, device=l.device)
            self.costs.append(c)
            self.disps.append(d)
            self.descs[i] = PairDesc(_dev(l, torch.uint8, 2, "left").value, _dev(r, torch.uint8, 2, "right").value,
                                     c.data_ptr(), d.data_ptr(), W, H, D, 0)
        need = int(lib.bp_batch_workspace_bytes(self.descs, n, ctypes.byref(params)))
        if need == 0:
            raise BPError(BP_E_INVAL, "invalid or unsupported batch")
        self.workspace = torch.empty(need, dtype=torch.uint8, device=lefts[0].device)

    def message_bits(self):
        """Bits per label of the batch's stored messages (12 or 16)."""
        return int(_load().bp_batch_message_bits(self.descs, len(self.descs), ctypes.byref(self.params)))

    def solve(self, ctx, stream=None):
        _check(_load().bp_solve_batched(ctx.handle, self.descs, len(self.descs), ctypes.byref(self.params),
                                        ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                        _stream(stream)))
        return self.disps

    def status(self, stream=None):
        s = ctypes.c_int32()
        _check(_load().bp_batch_status(ctypes.c_void_p(self.workspace.data_ptr()), _stream(stream), ctypes.byref(s)))
        return s.value

    def autotune(self, ctx, stream=None):
        t = BatchTuning()
        _check(_load().bp_autotune_batched(ctx.handle, self.descs, len(self.descs), ctypes.byref(self.params),
                                           ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                           _stream(stream), ctypes.byref(t)))
        return {"candidates": [{"schedule": t.schedule[i], "blocks_per_cu": t.blocks_per_cu[i], "order": t.order[i],
                                "ms": t.ms[i]}
                               for i in range(t.n_candidates)], "best": t.best}


def set_batch_schedule(ctx, schedule, blocks_per_cu=1, order=0):
    """Force the schedule of later batched solves on ctx (-1: back to tuned/default)."""
    lib = _load()
    _batch_sigs(lib)
    _check(lib.bp_context_set_batch_schedule(ctx.handle, schedule, blocks_per_cu, order))
