"""Python binding of the learned warm-start entry points of libbpstereo.so.

Argument marshalling only: every computation (input preparation, convolutions, loss,
gradients, Adam, quantisation) runs in the library's HIP kernels.  Tensors are torch GPU
tensors; bf16 tensors are carried as torch.uint16 bit patterns.
"""
from __future__ import annotations

import ctypes

import torch

from . import bpstereo as B

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_ready = False


def _lib():
    global _ready
    lib = B.library()
    if not _ready:
        lib.bp_cnn_param_count.argtypes = [_i32]
        lib.bp_cnn_param_count.restype = ctypes.c_int64
        lib.bp_cnn_layer.argtypes = [_i32, _i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
        lib.bp_cnn_workspace_bytes.argtypes = [_i32, _i32, _i32]
        lib.bp_cnn_workspace_bytes.restype = ctypes.c_size_t
        lib.bp_conv3x3_forward.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp]
        lib.bp_conv3x3_data_grad.argtypes = [_vp, _i32, _i32, _i32, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]
        lib.bp_conv3x3_wgrad_workspace_bytes.argtypes = [_i32, _i32, _i32, _i32]
        lib.bp_conv3x3_wgrad_workspace_bytes.restype = ctypes.c_size_t
        lib.bp_conv3x3_weight_grad.argtypes = [_vp, _vp, _i32, _i32, _i32, _i32, _vp, ctypes.c_size_t, _vp, _vp, _vp]
        lib.bp_cnn_forward.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp, _vp, ctypes.c_size_t, _vp, _vp]
        lib.bp_cnn_backward.argtypes = [_vp, _i32, _i32, _i32, _vp, _vp, ctypes.c_size_t, _vp, _vp, _i32, _vp, _vp,
                                        _vp]
        lib.bp_adam_step.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int64, _i32, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, _vp]
        lib.bp_cnn_to_bf16.argtypes = [_vp, ctypes.c_int64, _vp, _vp]
        lib.bp_warmstart_input.argtypes = [_vp, _vp, _vp, _i32, _i32, ctypes.POINTER(B.BPParams), _vp,
                                           ctypes.c_size_t, _vp, _vp]
        lib.bp_warmstart_messages.argtypes = [_vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp]
        lib.bp_pyramid_level.argtypes = [_vp, _i32, _i32, ctypes.POINTER(B.BPParams), _i32, _vp, ctypes.c_size_t,
                                         _vp, _vp]
        lib.bp_warmstart_solve.argtypes = [_vp, _vp, _vp, _vp, _i32, _i32, ctypes.POINTER(B.BPParams), _vp, _vp, _vp,
                                           ctypes.c_size_t, _vp, _vp, _vp, _vp]
        for n in ("bp_cnn_layer", "bp_conv3x3_forward", "bp_conv3x3_data_grad", "bp_conv3x3_weight_grad",
                  "bp_cnn_forward", "bp_cnn_backward", "bp_adam_step", "bp_cnn_to_bf16", "bp_warmstart_input",
                  "bp_warmstart_messages", "bp_pyramid_level", "bp_warmstart_solve"):
            getattr(lib, n).restype = ctypes.c_int32
        _ready = True
    return lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _s(stream):
    return B._stream(stream)


class Layout:
    """Parameter layout of the network for D disparity levels."""

    def __init__(self, num_disp):
        lib = _lib()
        self.D = num_disp
        self.count = int(lib.bp_cnn_param_count(num_disp))
        if self.count < 0:
            raise B.BPError(B.BP_E_INVAL, "num_disp must be in 1..256")
        self.layers = []
        for l in range(6):
            dims = (ctypes.c_int32 * 5)()
            offs = (ctypes.c_int64 * 2)()
            B._check(lib.bp_cnn_layer(num_disp, l, dims, offs))
            self.layers.append(dict(cin=dims[0], cin_p=dims[1], cout=dims[2], cout_p=dims[3], relu=dims[4],
                                    w_off=offs[0], b_off=offs[1]))

    def init_params(self, seed, device="cuda"):
        """He-normal weights on the real channels (the last layer 10x smaller), zero padding
        and biases; drawn with torch's CPU generator from `seed`."""
        gen = torch.Generator().manual_seed(int(seed))
        p = torch.zeros(self.count, dtype=torch.float32)
        for i, L in enumerate(self.layers):
            std = (2.0 / (9 * L["cin"])) ** 0.5 * (0.1 if i == 5 else 1.0)
            w = torch.zeros(L["cout_p"], 9, L["cin_p"])
            w[:L["cout"], :, :L["cin"]] = torch.randn(L["cout"], 9, L["cin"], generator=gen) * std
            p[L["w_off"]:L["w_off"] + w.numel()] = w.reshape(-1)
        return p.to(device)

    def weights(self, params, layer):
        L = self.layers[layer]
        return params[L["w_off"]:L["w_off"] + L["cout_p"] * 9 * L["cin_p"]].view(L["cout_p"], 9, L["cin_p"])

    def bias(self, params, layer):
        L = self.layers[layer]
        return params[L["b_off"]:L["b_off"] + L["cout_p"]]


def to_bf16(params, out=None, stream=None):
    out = torch.empty(params.numel(), dtype=torch.uint16, device=params.device) if out is None else out
    B._check(_lib().bp_cnn_to_bf16(_p(params), params.numel(), _p(out), _s(stream)))
    return out


def workspace(Ws, Hs, num_disp, device="cuda"):
    n = int(_lib().bp_cnn_workspace_bytes(Ws, Hs, num_disp))
    if n == 0:
        raise B.BPError(B.BP_E_INVAL, "bad CNN size")
    return torch.empty(n, dtype=torch.uint8, device=device)


def conv3x3_forward(x, w, bias, cout, relu=False, mask=None, want_bf16=True, want_f32=True, stream=None):
    H, W, cin_p = x.shape
    cout_p = w.shape[0]
    ob = torch.empty((H, W, cout_p), dtype=torch.uint16, device=x.device) if want_bf16 else None
    of = torch.empty((H, W, cout_p), dtype=torch.float32, device=x.device) if want_f32 else None
    B._check(_lib().bp_conv3x3_forward(_p(x), H, W, cin_p, _p(w), _p(bias), cout, cout_p, 1 if relu else 0, _p(mask),
                                       _p(ob), _p(of), _s(stream)))
    return ob, of


def conv3x3_data_grad(g, w, cin, mask=None, stream=None):
    H, W, cout_p = g.shape
    cin_p = w.shape[2]
    scratch = torch.empty(cin_p * 9 * cout_p, dtype=torch.uint16, device=g.device)
    ob = torch.empty((H, W, cin_p), dtype=torch.uint16, device=g.device)
    of = torch.empty((H, W, cin_p), dtype=torch.float32, device=g.device)
    B._check(_lib().bp_conv3x3_data_grad(_p(g), H, W, cout_p, _p(w), cin, cin_p, _p(mask), _p(scratch), _p(ob),
                                         _p(of), _s(stream)))
    return ob, of


def conv3x3_weight_grad(x, g, stream=None):
    H, W, cin_p = x.shape
    cout_p = g.shape[2]
    lib = _lib()
    ws = torch.empty(int(lib.bp_conv3x3_wgrad_workspace_bytes(H, W, cin_p, cout_p)), dtype=torch.uint8,
                     device=x.device)
    dw = torch.empty((cout_p, 9, cin_p), dtype=torch.float32, device=x.device)
    db = torch.empty(cout_p, dtype=torch.float32, device=x.device)
    B._check(lib.bp_conv3x3_weight_grad(_p(x), _p(g), H, W, cin_p, cout_p, _p(ws), ws.numel(), _p(dw), _p(db),
                                        _s(stream)))
    return dw, db


def forward(x, layout, params, w16, ws, y=None, stream=None):
    Hs, Ws, _ = x.shape
    cout_p = layout.layers[5]["cout_p"]
    y = torch.empty((Hs, Ws, cout_p), dtype=torch.float32, device=x.device) if y is None else y
    B._check(_lib().bp_cnn_forward(_p(x), Ws, Hs, layout.D, _p(params), _p(w16), _p(ws), ws.numel(), _p(y),
                                   _s(stream)))
    return y


def backward(x, layout, w16, ws, y, label, lam_t, grads=None, loss=None, stream=None):
    Hs, Ws, _ = x.shape
    grads = torch.empty(layout.count, dtype=torch.float32, device=x.device) if grads is None else grads
    loss = torch.empty(1, dtype=torch.float32, device=x.device) if loss is None else loss
    B._check(_lib().bp_cnn_backward(_p(x), Ws, Hs, layout.D, _p(w16), _p(ws), ws.numel(), _p(y), _p(label), lam_t,
                                    _p(grads), _p(loss), _s(stream)))
    return grads, loss


def adam_step(params, m, v, grads, w16, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    B._check(_lib().bp_adam_step(_p(params), _p(m), _p(v), _p(grads), _p(w16), params.numel(), step, lr, beta1, beta2,
                                 eps, _s(stream)))


def warmstart_input(left, right, cost, num_scales, iters, lam, trunc, workspace=None, out=None, stream=None):
    H, W, D = cost.shape
    p = B.make_params(D, num_scales, iters, lam, trunc)
    need = B.bp_workspace_bytes(W, H, p)
    workspace = torch.empty(need, dtype=torch.uint8, device=cost.device) if workspace is None else workspace
    cin_p = Layout(D).layers[0]["cin_p"]
    hs, ws_ = H, W
    for _ in range(num_scales - 2):
        hs, ws_ = (hs + 1) // 2, (ws_ + 1) // 2
    out = torch.empty((hs, ws_, cin_p), dtype=torch.uint16, device=cost.device) if out is None else out
    B._check(_lib().bp_warmstart_input(_p(left), _p(right), _p(cost), W, H, ctypes.byref(p), _p(workspace),
                                       workspace.numel(), _p(out), _s(stream)))
    return out


def warmstart_messages(y, num_disp, lam, trunc, out=None, stream=None):
    Hs, Ws, _ = y.shape
    out = torch.empty((4, Hs, Ws, num_disp), dtype=torch.int16, device=y.device) if out is None else out
    B._check(_lib().bp_warmstart_messages(_p(y), Ws, Hs, num_disp, lam, trunc, _p(out), _s(stream)))
    return out


def pyramid_level(cost, num_scales, level, workspace=None, out=None, stream=None):
    H, W, D = cost.shape
    p = B.make_params(D, num_scales, 0, 0, 0)
    need = B.bp_workspace_bytes(W, H, p)
    workspace = torch.empty(need, dtype=torch.uint8, device=cost.device) if workspace is None else workspace
    h, w = H, W
    for _ in range(level):
        h, w = (h + 1) // 2, (w + 1) // 2
    out = torch.empty((h, w, D), dtype=torch.int16, device=cost.device) if out is None else out
    B._check(_lib().bp_pyramid_level(_p(cost), W, H, ctypes.byref(p), level, _p(workspace), workspace.numel(), _p(out),
                                     _s(stream)))
    return out


def warmstart_solve(left, right, cost, num_scales, iters, lam, trunc, params, w16, skip_mode=0, converge_iters=2,
                    want_msgs=False, want_stats=False, ctx=None, workspace=None, disparity=None, stream=None):
    """The warm-started solve in one library call (the network as one launch inside the solve):
    the same results as warmstart_input, forward, warmstart_messages and the solve with those
    messages.  Returns (disparity, messages or None, stats or None) as bp_hierarchical_solve."""
    H, W, D = cost.shape
    for t, name in ((left, "left"), (right, "right")):
        if tuple(t.shape) != (H, W):
            raise ValueError(f"{name} must be [{H}, {W}]")
    p = B.make_params(D, num_scales, iters, lam, trunc, skip_mode, converge_iters)
    need = B.bp_workspace_bytes(W, H, p)
    if need == 0:
        raise B.BPError(B.BP_E_INVAL, "invalid solve parameters")
    workspace = torch.empty(need, dtype=torch.uint8, device=cost.device) if workspace is None else workspace
    disp = torch.empty((H, W), dtype=torch.int16, device=cost.device) if disparity is None else disparity
    msgs = torch.empty((4, H, W, D), dtype=torch.int16, device=cost.device) if want_msgs else None
    st = B.BPStats() if want_stats else None
    B._check(_lib().bp_warmstart_solve(ctx.handle if ctx is not None else None, B._dev(left, torch.uint8, 2, "left"),
                                       B._dev(right, torch.uint8, 2, "right"), B._dev(cost, torch.int16, 3, "cost"),
                                       W, H, ctypes.byref(p), B._dev(params, torch.float32, 1, "params"),
                                       B._dev(w16, torch.uint16, 1, "w16"), _p(workspace), workspace.numel(),
                                       B._dev(disp, torch.int16, 2, "disparity"), _p(msgs),
                                       ctypes.byref(st) if want_stats else None, _s(stream)))
    stats = None
    if want_stats:
        stats = {"msg_updates": st.msg_updates, "pixel_updates": st.pixel_updates,
                 "n_halfsteps": list(st.n_halfsteps),
                 "active": [[st.active[l][t] for t in range(64)] for l in range(8)]}
    return disp, msgs, stats
