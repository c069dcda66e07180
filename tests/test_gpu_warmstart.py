"""GPU parity of the learned warm start (network input, 3x3 convolutions on MFMA and their
gradients, L1 loss, Adam, message quantisation, cost pyramid export) against the CPU oracle.

Integer and bf16-bit results are compared bit for bit.  fp32 sums of bf16 products are
compared with the fp64 oracle fed the same bf16 operands, within the recursive-summation
bound n * 2^-23 * sum|terms| (twice the textbook gamma_n = n * 2^-24), where n is the number
of terms one output adds and sum|terms| is the oracle's result on |operands|.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1709_06509_amd import bpstereo as B
from paper_1709_06509_amd import synth
from paper_1709_06509_amd import warmstart as WS

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bf16_array(rng, shape, scale=1.0, real=None):
    """Random bf16 bits of N(0, scale^2) values; channels >= real (last axis) are 0."""
    v = (rng.standard_normal(shape) * scale).astype(np.float32)
    if real is not None:
        v[..., real:] = 0.0
    return oracle.bf16(v).reshape(shape)


def val(bits):
    return oracle.bf16_value(bits).astype(np.float64)


def within(got, ref, mag, n, what):
    tol = n * 2.0**-23 * mag + 1e-30
    err = np.abs(got.astype(np.float64) - ref)
    bad = err > tol
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {bad.size} outside the bound, worst "
                           f"{float(np.max(err - tol)):.3g} at {np.unravel_index(np.argmax(err - tol), err.shape)}")


# (H, W, cin, cin_p, cout, cout_p, relu): every layer shape of D = 10, 16 and 64, images with a
# ragged 64-pixel tail and more than one 512-pixel weight-gradient chunk
CONV_CASES = [
    (13, 37, 12, 16, 32, 32, True),
    (13, 37, 32, 32, 40, 64, False),
    (30, 40, 18, 32, 32, 32, True),
    (30, 40, 32, 32, 64, 64, False),
    (21, 29, 66, 80, 32, 32, True),
    (21, 29, 32, 32, 32, 32, True),
    (9, 70, 32, 32, 256, 256, False),
    (1, 1, 32, 32, 32, 32, True),
    (1, 50, 12, 16, 32, 32, False),
]


def conv_operands(case, seed):
    H, W, cin, cin_p, cout, cout_p, relu = case
    rng = np.random.default_rng(seed)
    x = bf16_array(rng, (H, W, cin_p), 1.0, real=cin)
    w = bf16_array(rng, (cout_p, 9, cin_p), (2.0 / (9 * cin)) ** 0.5, real=cin)
    w[cout:] = oracle.bf16(rng.standard_normal((cout_p - cout) * 9 * cin_p).astype(np.float32)).reshape(
        cout_p - cout, 9, cin_p)  # rows past cout must not reach the output
    b = (rng.standard_normal(cout_p) * 0.1).astype(np.float32)
    return x, w, b


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_forward_matches_oracle(case):
    H, W, cin, cin_p, cout, cout_p, relu = case
    say(f"conv forward {case}")
    x, w, b = conv_operands(case, 11)
    ob, of = WS.conv3x3_forward(gpu(x), gpu(w), gpu(b), cout, relu=relu)
    got_f, got_b = host(of), host(ob)
    xv, wv = val(x)[..., :cin], val(w)[:cout, :, :cin]
    z = oracle.conv3x3(xv, wv, b[:cout].astype(np.float64))
    mag = oracle.conv3x3(np.abs(xv), np.abs(wv), np.abs(b[:cout]).astype(np.float64))
    ref = np.maximum(z, 0.0) if relu else z
    within(got_f[..., :cout], ref, mag, 9 * cin_p + 1, "forward fp32")
    assert not got_f[..., cout:].any() and not got_b[..., cout:].any(), "padded output channels not zero"
    assert np.array_equal(got_b, oracle.bf16(got_f).reshape(got_b.shape)), "bf16 output is not the rounded fp32"


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_gradients_match_oracle(case):
    H, W, cin, cin_p, cout, cout_p, relu = case
    say(f"conv gradients {case}")
    x, w, _ = conv_operands(case, 12)
    rng = np.random.default_rng(13)
    g = bf16_array(rng, (H, W, cout_p), 1e-2, real=cout)
    xv, wv, gv = val(x)[..., :cin], val(w)[:cout, :, :cin], val(g)[..., :cout]
    dx, dw, db = oracle.conv3x3_backward(xv, wv, gv)
    mx, mw, mb = oracle.conv3x3_backward(np.abs(xv), np.abs(wv), np.abs(gv))
    P = H * W
    # weight and bias gradients
    gdw, gdb = WS.conv3x3_weight_grad(gpu(x), gpu(g))
    gdw, gdb = host(gdw), host(gdb)
    within(gdw[:cout, :, :cin], dw, mw, P + 64, "weight gradient")
    within(gdb[:cout], db, mb, P + 64, "bias gradient")
    assert not gdw[cout:].any() and not gdw[:, :, cin:].any() and not gdb[cout:].any()
    # data gradient (layers after the first have cin_p a multiple of 32), masked by the input's ReLU
    if cin_p % 32 == 0:
        ob, of = WS.conv3x3_data_grad(gpu(g), gpu(w), cin, mask=gpu(x))
        got_f, got_b = host(of), host(ob)
        keep = xv > 0
        within(got_f[..., :cin], dx * keep, mx * keep, 9 * cout_p, "data gradient")
        assert not got_f[..., cin:].any()
        assert np.array_equal(got_b, oracle.bf16(got_f).reshape(got_b.shape))
        ob2, of2 = WS.conv3x3_data_grad(gpu(g), gpu(w), cin)
        within(host(of2)[..., :cin], dx, mx, 9 * cout_p, "data gradient without mask")


def small_network(D, Hs, Ws, seed):
    layout = WS.Layout(D)
    params = layout.init_params(seed)
    # non-zero biases so that their path is exercised
    gen = torch.Generator().manual_seed(seed + 1)
    for l, L in enumerate(layout.layers):
        layout.bias(params, l)[:L["cout"]] = (torch.randn(L["cout"], generator=gen) * 0.05).cuda()
    w16 = WS.to_bf16(params)
    rng = np.random.default_rng(seed)
    x = bf16_array(rng, (Hs, Ws, layout.layers[0]["cin_p"]), 0.5, real=layout.layers[0]["cin"])
    return layout, params, w16, gpu(x)


def chain_forward(layout, params, w16, x):
    acts = [x]
    y = None
    for l, L in enumerate(layout.layers):
        last = l == len(layout.layers) - 1
        ob, of = WS.conv3x3_forward(acts[-1], layout.weights(w16, l), layout.bias(params, l), L["cout"],
                                    relu=bool(L["relu"]), want_bf16=not last, want_f32=last)
        if last:
            y = of
        else:
            acts.append(ob)
    return acts, y


@pytest.mark.parametrize("D,Hs,Ws", [(16, 12, 20), (64, 18, 24), (10, 7, 33)])
def test_network_forward_backward(D, Hs, Ws):
    say(f"network D={D} {Hs}x{Ws}")
    layout, params, w16, x = small_network(D, Hs, Ws, 21)
    ws = WS.workspace(Ws, Hs, D)
    y = WS.forward(x, layout, params, w16, ws)
    acts, y_chain = chain_forward(layout, params, w16, x)
    assert torch.equal(y, y_chain), "network forward differs from its layers run one by one"
    yh = host(y)
    assert not yh[..., 4 * D:].any()

    lam_t = 64 * min(4, D)
    rng = np.random.default_rng(22)
    label = rng.integers(0, lam_t + 1, (4, Hs, Ws, D)).astype(np.int16)
    # labels within rounding of y*lam_t: the residual's sign decides the gradient there
    label[1, 0, 0, :] = np.clip(np.round(yh[0, 0, D:2 * D] * lam_t), -32768, 32767).astype(np.int16)
    grads, loss = WS.backward(x, layout, w16, ws, y, gpu(label), lam_t)
    grads_h, loss_h = host(grads), float(host(loss)[0])
    ref_loss, dy = oracle.warm_l1(yh[..., :4 * D], label, lam_t)
    assert abs(loss_h - ref_loss) <= 1e-5 * ref_loss, (loss_h, ref_loss)

    # walk the layers backwards from the oracle's output gradient, each checked on the GPU's own
    # inputs (activations of the forward, gradient of the layer above)
    cout_p5 = layout.layers[-1]["cout_p"]
    g = np.zeros((Hs, Ws, cout_p5), np.float32)
    g[..., :4 * D] = dy
    g = gpu(oracle.bf16(g).reshape(Hs, Ws, cout_p5))
    for l in range(len(layout.layers) - 1, -1, -1):
        L = layout.layers[l]
        a = host(acts[l])
        gb = host(g)
        av = val(a)[..., :L["cin"]]
        wv = val(host(layout.weights(w16, l)))[:L["cout"], :, :L["cin"]]
        gv = val(gb)[..., :L["cout"]]
        _, dw, db = oracle.conv3x3_backward(av, wv, gv, want_dx=False)
        _, mw, mb = oracle.conv3x3_backward(np.abs(av), np.abs(wv), np.abs(gv), want_dx=False)
        n = Hs * Ws + 64
        gw = grads_h[L["w_off"]:L["w_off"] + L["cout_p"] * 9 * L["cin_p"]].reshape(L["cout_p"], 9, L["cin_p"])
        within(gw[:L["cout"], :, :L["cin"]], dw, mw, n, f"layer {l} weight gradient")
        within(grads_h[L["b_off"]:L["b_off"] + L["cout"]], db, mb, n, f"layer {l} bias gradient")
        assert not gw[L["cout"]:].any() and not gw[:, :, L["cin"]:].any()
        if l > 0:
            g, _ = WS.conv3x3_data_grad(g, layout.weights(w16, l), L["cin"], mask=acts[l])

    # deterministic: a second backward gives the same bits
    grads2, loss2 = WS.backward(x, layout, w16, ws, y, gpu(label), lam_t)
    assert torch.equal(grads, grads2) and torch.equal(loss, loss2)


def test_adam_matches_oracle():
    say("adam")
    rng = np.random.default_rng(31)
    n = 100003
    w = (rng.standard_normal(n) * 0.1).astype(np.float32)
    wg, mg, vg = gpu(w.copy()), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    w16 = torch.empty(n, dtype=torch.uint16, device="cuda")
    wo, mo, vo = w.astype(np.float64), np.zeros(n), np.zeros(n)
    lr = 1e-3
    for step in range(1, 5):
        g = (rng.standard_normal(n) * 10.0**rng.integers(-4, 1, n)).astype(np.float32)
        g[:7] = 0.0
        WS.adam_step(wg, mg, vg, gpu(g), w16, step, lr)
        oracle.adam(wo, mo, vo, g.astype(np.float64), step, lr)
    got = host(wg)
    # each step moves w by at most lr*(1 + rounding); the fp32 state carries about 2^-22 of |w| per step
    err = np.abs(got - wo)
    tol = 4 * 2.0**-22 * np.abs(wo) + 1e-3 * lr
    assert np.all(err <= tol), float(np.max(err - tol))
    assert np.array_equal(host(w16), oracle.bf16(got))


def test_to_bf16_bits():
    say("to_bf16")
    rng = np.random.default_rng(32)
    v = (rng.standard_normal(5000) * 10.0**rng.integers(-30, 30, 5000)).astype(np.float32)
    ties = np.array([1.0 + 2**-8, 1.0 + 3 * 2**-8, -(1.0 + 2**-8), 0.0, -0.0, 3.0e38, 1e-40], np.float32)
    v = np.concatenate([v, ties])
    got = host(WS.to_bf16(gpu(v)))
    assert np.array_equal(got, oracle.bf16(v))


@pytest.mark.parametrize("W,H,D,L", [(96, 64, 16, 3), (101, 77, 24, 4), (40, 30, 64, 2), (53, 9, 10, 3)])
def test_warmstart_input_and_pyramid(W, H, D, L):
    say(f"warm input {W}x{H} D={D} L={L}")
    p = synth.make_pair(W, H, D, (3, 5), False, 0, False, seed=40 + W)
    cost = oracle.cost_volume(p["left"], p["right"], D, 5)
    levels = [cost]
    for _ in range(L - 1):
        levels.append(oracle.pyramid_level(levels[-1]))
    for lvl in range(L):
        got = host(WS.pyramid_level(gpu(cost), L, lvl))
        assert np.array_equal(got, levels[lvl]), f"pyramid level {lvl}"
    cin_p = WS.Layout(D).layers[0]["cin_p"]
    got = host(WS.warmstart_input(gpu(p["left"]), gpu(p["right"]), gpu(cost), L, 5, 64, 4))
    ref = oracle.warm_input(p["left"], p["right"], L - 2, levels[L - 1], cin_p)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("Ws,Hs,D", [(20, 12, 16), (33, 7, 64), (1, 5, 10), (6, 1, 8)])
def test_warmstart_messages(Ws, Hs, D):
    say(f"warm messages {Ws}x{Hs} D={D}")
    lam, T = 64, 4
    lam_t = lam * min(T, D)
    cout_p = WS.Layout(D).layers[-1]["cout_p"]
    rng = np.random.default_rng(50)
    y = rng.uniform(-0.2, 1.2, (Hs, Ws, cout_p)).astype(np.float32)
    # exact halves of 1/lam_t: rounding ties go to even
    y.reshape(-1)[::7] = ((rng.integers(0, lam_t, y.size)[::7] + 0.5) / lam_t).astype(np.float32)
    got = host(WS.warmstart_messages(gpu(y), D, lam, T))
    ref = oracle.warm_messages(y[..., :4 * D], D, lam_t)
    assert np.array_equal(got, ref)


def test_training_steps_reduce_loss():
    """Library-only training on one small pair: the loss after 60 Adam steps is below the first."""
    from paper_1709_06509_amd import warmstart_train as T
    cfg = dict(T.DEFAULT, num_disp=16, num_scales=3, iters=6)
    say("training steps")
    pair = synth.make_pair(64, 48, 16, (3, 5), False, 0, False, seed=77)
    sample = T.Sample(pair, cfg)
    tr = T.Trainer(cfg, seed=3)
    first = float(host(tr.train_step(sample))[0])
    for _ in range(59):
        tr.train_step(sample)
    last = float(host(tr.train_step(sample))[0])
    say(f"loss {first:.3f} -> {last:.3f}")
    assert last < first
    # checkpoint round trip resumes bit for bit
    st = tr.state()
    tr2 = T.Trainer(cfg, seed=99)
    tr2.load(st)
    a = tr.train_step(sample).clone()
    b = tr2.train_step(sample).clone()
    assert torch.equal(a, b) and torch.equal(tr.params, tr2.params)


def test_warm_solve_matches_oracle_end_to_end():
    """Network messages fed to the solve: the GPU result equals the oracle solve given the same
    messages, and the warm hierarchy skips the coarsest scale."""
    from paper_1709_06509_amd import warmstart_train as T
    cfg = dict(T.DEFAULT, num_disp=16, num_scales=3, iters=6)
    say("warm solve end to end")
    pair = synth.make_pair(70, 45, 16, (3, 5), False, 0, False, seed=78)
    sample = T.Sample(pair, cfg, with_label=False)
    tr = T.Trainer(cfg, seed=4)
    msgs = tr.predict(sample)
    d = T.solve_warm(sample, cfg, msgs, (4, 4))
    cost = host(sample.cost)
    ref, _, _ = oracle.bp_solve(cost, 3, [4, 4, 0], 64, 4, warm_msgs=host(msgs), want_msgs=False)
    assert np.array_equal(host(d), ref)


@pytest.mark.parametrize("D,L,size", [(16, 3, (96, 72)), (64, 4, (160, 120))])
@pytest.mark.parametrize("skip", [0, 1])
def test_warm_solve_parity_learned_shapes(D, L, size, skip):
    """The warm solve in the learned configuration's shape (D = 64, 4 scales: network messages
    at scale 2, scale 3 skipped) and a smaller one, plain BP and the freeze rule: disparities,
    messages and counters equal the oracle's solve from the same messages."""
    from paper_1709_06509_amd import warmstart_train as T
    cfg = dict(T.DEFAULT, num_disp=D, num_scales=L, iters=6)
    say(f"warm solve parity D={D} L={L} size={size} skip={skip}")
    pair = synth.make_pair(size[0], size[1], D, (3, 5), True, 0, False, seed=79 + D)
    sample = T.Sample(pair, cfg, with_label=False)
    msgs = T.Trainer(cfg, seed=6).predict(sample)
    iters = [5, 4, 4, 0][:L]
    d, m, st = B.bp_hierarchical_solve(sample.cost, L, iters, 64, 4, skip, 2, warm_msgs=msgs, want_msgs=True,
                                       want_stats=True)
    rd, rm, rs = oracle.bp_solve(host(sample.cost), L, iters, 64, 4, skip, 2, warm_msgs=host(msgs))
    assert np.array_equal(host(d), rd) and np.array_equal(host(m), rm)
    assert st["pixel_updates"] == rs["pixel_updates"] and st["msg_updates"] == rs["msg_updates"]


def test_trained_network_gain_over_no_network():
    """What the trained network gains over the method without it, at equal schedule (the same
    reduced half-steps from the warm scale down, the network's messages against the zero
    start the hierarchy would otherwise have there), on held-out pairs.  With few half-steps
    the start decides much of the result and the network must win on energy; with the
    deployable schedule (8 half-steps a scale) the finest scale decides the energy and the two
    starts come out within the 0.5 % judge of plain BP, which is all asserted there."""
    from paper_1709_06509_amd import warmstart_train as T
    cfg = dict(T.DEFAULT, num_disp=16, num_scales=3, iters=8, train_size=(128, 96), eval_size=(128, 96))
    say("training gain")
    tr = T.Trainer(cfg, seed=5)
    T.train(tr, cfg, [cfg["train_seed0"] + i for i in range(400)], log=say)
    held = [T.Sample(T.gen_pair(cfg["train_size"], 300000 + i, cfg), cfg) for i in range(8)]
    losses = [tr.heldout_loss(s) for s in held]
    net, zero = float(np.mean([l[0] for l in losses])), float(np.mean([l[1] for l in losses]))
    res = {}
    for sched in [(1, 1), (8, 8)]:
        rows = []
        for s in held:
            ep = T.energy(s.cost, T.solve_plain(s, cfg), cfg)
            ew = T.energy(s.cost, T.solve_warm(s, cfg, tr.predict(s), sched), cfg)
            ez = T.energy(s.cost, T.solve_warm(s, cfg, torch.zeros_like(s.label), sched), cfg)
            rows.append((ew / ep, ez / ep))
        res[sched] = np.array(rows)
        say(f"schedule {sched}: energy / plain, network start {res[sched][:, 0].mean():.5f}, zero start "
            f"{res[sched][:, 1].mean():.5f}, network lower on {int((res[sched][:, 0] < res[sched][:, 1]).sum())} of 8")
    say(f"held-out L1: network {net:.2f}, zero start {zero:.2f}")
    assert net < 0.5 * zero
    short = res[(1, 1)]
    assert short[:, 0].mean() < short[:, 1].mean()
    assert (short[:, 0] < short[:, 1]).sum() >= 6
    assert all(r <= 1.005 for r in res[(8, 8)][:, 0])


def spread_network(D, seed):
    """Parameters whose messages spread over the whole quantisation range: the layout's
    initial weights, the last layer 10x larger with biases uniform in [0, 1] (and every bias
    of the hidden layers small but non-zero, so bias addition is exercised)."""
    lay = WS.Layout(D)
    params = lay.init_params(seed)
    gen = torch.Generator().manual_seed(seed + 1)
    for i, L in enumerate(lay.layers):
        b = lay.bias(params, i)
        if i == 5:
            w = lay.weights(params, i)
            w.mul_(10.0)
            b[:L["cout"]] = torch.rand(L["cout"], generator=gen).cuda()
        else:
            b[:L["cout"]] = (torch.rand(L["cout"], generator=gen) * 0.1 - 0.05).cuda()
    return lay, params, WS.to_bf16(params)


def layer_path(left, right, cost, L, iters, lam, T, skip, lay, params, w16):
    """The warm-started solve through the layer-level calls: network input, forward, messages,
    then the solve with those messages."""
    H, W, D = cost.shape
    x = WS.warmstart_input(left, right, cost, L, iters, lam, T)
    Hs, Ws, _ = x.shape
    y = WS.forward(x, lay, params, w16, WS.workspace(Ws, Hs, D))
    msgs = WS.warmstart_messages(y, D, lam, T)
    d, m, st = B.bp_hierarchical_solve(cost, L, iters, lam, T, skip, 2, warm_msgs=msgs, want_msgs=True,
                                       want_stats=True)
    return msgs, d, m, st


# (W, H, D, L): scale-(L-2) sizes with ragged and whole 10 x 8 tiles, smaller than one tile,
# one pixel wide or high, the learned configuration (640 x 480, D = 64, 4 scales: 160 x 120),
# and five scales (the network at scale 3, the views averaged over 8 x 8 blocks)
ONE_LAUNCH_CASES = [
    (70, 45, 16, 3),
    (33, 29, 32, 2),
    (96, 72, 48, 3),
    (5, 3, 16, 2),
    (1, 9, 32, 2),
    (130, 1, 16, 2),
    (200, 150, 64, 4),
    (640, 480, 64, 4),
    (160, 96, 16, 5),  # scale 3: the views averaged over 8 x 8 blocks
    (97, 53, 32, 5),
]


@pytest.mark.parametrize("case", ONE_LAUNCH_CASES)
@pytest.mark.parametrize("skip", [0, 1, 2])
def test_warmstart_solve_equals_layer_path(case, skip):
    """bp_warmstart_solve (the network as one launch inside the solve) against the layer-level
    calls on the same pair and parameters: with no half-steps the scale-(L-2) start itself
    (L = 2: the finest scale's exported messages are the network's messages), else the
    disparities, finest messages and counters of the whole solve, bit for bit."""
    W, H, D, L = case
    say(f"one-launch warm solve W={W} H={H} D={D} L={L} skip={skip}")
    pair = synth.make_pair(W, H, D, (3, 6), True, 0, False, seed=500 + W + D + skip)
    left, right = gpu(pair["left"]), gpu(pair["right"])
    cost = B.stereo_cost_volume(left, right, D, 5)
    lay, params, w16 = spread_network(D, 40 + D)
    lam, T = 64, 4
    for iters in ([0] * L, ([4, 3, 3, 0][:L] if L <= 4 else [4, 3, 3, 3, 0]) if L > 2 else [5, 0]):
        msgs, d_ref, m_ref, st_ref = layer_path(left, right, cost, L, iters, lam, T, skip, lay, params, w16)
        d, m, st = WS.warmstart_solve(left, right, cost, L, iters, lam, T, params, w16, skip, want_msgs=True,
                                      want_stats=True)
        if L == 2 and not any(iters):
            assert torch.equal(m, msgs), "network messages differ from the layer path's"
            q = host(msgs)
            assert q.min() == 0 and q.max() > lam  # spread over the range (not all clamped or zero)
        assert torch.equal(d, d_ref), f"disparities differ (iters {iters})"
        assert torch.equal(m, m_ref), f"finest messages differ (iters {iters})"
        assert st["msg_updates"] == st_ref["msg_updates"] and st["pixel_updates"] == st_ref["pixel_updates"]
        assert st["active"] == st_ref["active"] and st["n_halfsteps"] == st_ref["n_halfsteps"]


def test_warmstart_solve_trained_network_and_graph_replays():
    """A trained network (a short run) through the one-call solve equals the layer path, also
    when the call is captured in a HIP graph and replayed with new views in place."""
    from paper_1709_06509_amd import warmstart_train as T
    cfg = dict(T.DEFAULT, num_disp=32, num_scales=3, iters=6)
    say("one-launch warm solve with a trained network")
    tr = T.Trainer(cfg, seed=8)
    for i in range(20):
        tr.train_step(T.Sample(synth.make_pair(96, 72, 32, (3, 5), True, 0, False, seed=900 + i), cfg))
    W, H, D, L = 150, 110, 32, 3
    iters = [4, 4, 0]
    pairs = [synth.make_pair(W, H, D, (3, 6), True, 0, False, seed=950 + i) for i in range(3)]
    left = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    right = torch.empty_like(left)
    cost = torch.empty((H, W, D), dtype=torch.int16, device="cuda")
    disp = torch.empty((H, W), dtype=torch.int16, device="cuda")
    ws = torch.empty(B.bp_workspace_bytes(W, H, B.make_params(D, L, iters, 64, 4)), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()

    def step():
        B.stereo_cost_volume(left, right, D, cfg["window"], out=cost)
        WS.warmstart_solve(left, right, cost, L, iters, 64, 4, tr.params, tr.w16, 1, workspace=ws, disparity=disp)

    left.copy_(gpu(pairs[0]["left"]))
    right.copy_(gpu(pairs[0]["right"]))
    with torch.cuda.stream(stream):
        step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            step()
    torch.cuda.synchronize()
    for p in pairs + pairs[:1]:
        left.copy_(gpu(p["left"]))
        right.copy_(gpu(p["right"]))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            g.replay()
        torch.cuda.synchronize()
        _, d_ref, _, _ = layer_path(left, right, cost, L, iters, 64, 4, 1, tr.layout, tr.params, tr.w16)
        assert torch.equal(disp, d_ref)
