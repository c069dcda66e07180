"""Pins of the CPU oracle's warm-start pieces (CNN convolution, its gradients, the message
quantisation, the L1 loss and Adam) against closed forms, hand-worked cases and finite
differences."""
import numpy as np

import oracle


def test_bf16_round_to_nearest_even():
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 2**-9, -2.5, 0.0, 65280.0], np.float32)
    bits = oracle.bf16(vals)
    # 1+2^-8 is halfway between 1 and 1+2^-7: ties to the even mantissa (1.0); 1+3*2^-8 ties up
    assert bits.tolist() == [0x3F80, 0x3F80, 0x3F82, 0x3F80, 0xC020, 0x0000, 0x477F]
    assert oracle.bf16_value(bits).tolist() == [1.0, 1.0, 1.0 + 2**-6, 1.0, -2.5, 0.0, 65280.0]


def test_conv_identity_kernel_and_border_counts():
    rng = np.random.default_rng(0)
    H, W, C = 5, 6, 3
    x = rng.standard_normal((H, W, C))
    w = np.zeros((C, 9, C))
    for c in range(C):
        w[c, 4, c] = 1.0  # centre tap
    b = np.array([0.5, -1.0, 2.0])
    assert np.allclose(oracle.conv3x3(x, w, b), x + b, atol=0, rtol=0)
    # all-ones kernel on all-ones input counts the in-bounds neighbours times Cin
    z = oracle.conv3x3(np.ones((H, W, C)), np.ones((1, 9, C)), None)[..., 0]
    cnt = np.full((H, W), 9.0)
    cnt[0, :] = cnt[-1, :] = 6
    cnt[:, 0] = cnt[:, -1] = 6
    cnt[0, 0] = cnt[0, -1] = cnt[-1, 0] = cnt[-1, -1] = 4
    assert np.array_equal(z, cnt * C)
    # a single off-centre tap shifts the image (tap (dy, dx) = (0, 2) reads x[y-1][x+1])
    w = np.zeros((1, 9, 1))
    w[0, 2, 0] = 1.0
    img = rng.standard_normal((H, W, 1))
    z = oracle.conv3x3(img, w, None)
    ref = np.zeros((H, W, 1))
    ref[1:, :-1] = img[:-1, 1:]
    assert np.array_equal(z, ref)


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    H, W, Cin, Cout = 4, 5, 3, 2
    x = rng.standard_normal((H, W, Cin))
    w = rng.standard_normal((Cout, 9, Cin))
    b = rng.standard_normal(Cout)
    r = rng.standard_normal((H, W, Cout))  # loss = sum(z * r), so dz = r

    def loss(x_, w_, b_):
        return float(np.sum(oracle.conv3x3(x_, w_, b_) * r))

    dx, dw, db = oracle.conv3x3_backward(x, w, r)
    h = 1e-3  # the conv is linear in each argument: central differences are exact up to rounding
    for idx in [(0, 0, 0), (2, 3, 1), (3, 4, 2), (1, 2, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (loss(x + e, w, b) - loss(x - e, w, b)) / (2 * h)
        assert abs(fd - dx[idx]) <= 1e-9 * max(1.0, abs(fd))
    for idx in [(0, 0, 0), (1, 4, 2), (0, 8, 1), (1, 3, 0)]:
        e = np.zeros_like(w)
        e[idx] = h
        fd = (loss(x, w + e, b) - loss(x, w - e, b)) / (2 * h)
        assert abs(fd - dw[idx]) <= 1e-9 * max(1.0, abs(fd))
    for i in range(Cout):
        e = np.zeros_like(b)
        e[i] = h
        fd = (loss(x, w, b + e) - loss(x, w, b - e)) / (2 * h)
        assert abs(fd - db[i]) <= 1e-9 * max(1.0, abs(fd))
    assert np.allclose(db, r.sum(axis=(0, 1)))


def test_warm_messages_hand_case():
    # one 2x1 image (two pixels in a row), D = 3, lambda*T = 10
    D, lam_t = 3, 10
    y = np.zeros((1, 2, 4 * D), np.float32)
    # pixel 0, side 1 (from-right, the neighbour exists): y*10 = [2.5, 3.5, 12.0] -> rint [2, 4, 10]
    # (ties to even, clamp at 10) -> minus min 2 -> [0, 2, 8]
    y[0, 0, 1 * D:2 * D] = [0.25, 0.35, 1.2]
    # pixel 1, side 0 (from-left): y*10 = [-3, 7.4, 5.5] -> [0, 7, 6] -> minus 0 -> [0, 7, 6]
    y[0, 1, 0:D] = [-0.3, 0.74, 0.55]
    # a side without a neighbour is zero whatever y says
    y[0, 0, 0:D] = [0.9, 0.1, 0.5]
    m = oracle.warm_messages(y, D, lam_t)
    assert m[1, 0, 0].tolist() == [0, 2, 8]
    assert m[0, 0, 1].tolist() == [0, 7, 6]
    assert not m[0, 0, 0].any() and not m[2].any() and not m[3].any()


def test_warm_l1_hand_case_and_gradient():
    D, lam_t = 2, 4
    y = np.zeros((1, 2, 4 * D), np.float32)
    lab = np.zeros((4, 1, 2, D), np.int16)
    y[0, 0, 1 * D:2 * D] = [1.0, 0.5]  # pixel 0 from-right: [4, 2] vs label [3, 2]
    lab[1, 0, 0] = [3, 2]
    y[0, 1, 0:D] = [0.0, 2.0]  # pixel 1 from-left: [0, 8] vs label [1, 1]
    lab[0, 0, 1] = [1, 1]
    loss, dy = oracle.warm_l1(y, lab, lam_t)
    # |4-3| + |2-2| + |0-1| + |8-1| = 9 over 4 valid entries
    assert loss == 9 / 4
    assert dy[0, 0, 1 * D:2 * D].tolist() == [lam_t / 4, 0.0]
    assert dy[0, 1, 0:D].tolist() == [-lam_t / 4, lam_t / 4]
    assert not dy[0, 0, 0:D].any()


def test_warm_input_hand_case():
    # 4x2 image, s = 1: two blocks of 2x2 pixels; coarse scale has 1 pixel, D = 2
    L = np.array([[0, 255, 10, 20], [255, 0, 30, 40]], np.uint8)
    R = np.array([[51, 51, 0, 0], [51, 51, 0, 255]], np.uint8)
    coarse = np.array([[[512, 1024]]], np.int16)
    x = oracle.warm_input(L, R, 1, coarse, 8)
    v = oracle.bf16_value(x)
    assert x.shape == (1, 2, 8)
    assert v[0, 0, 0] == oracle.bf16_value(oracle.bf16(np.float32(0.5)))[0]     # (0+255+255+0)/4/255
    assert v[0, 0, 1] == oracle.bf16_value(oracle.bf16(np.float32(0.2)))[0]     # 51/255
    assert v[0, 1, 0] == oracle.bf16_value(oracle.bf16(np.float32(100 / 1020)))[0]
    assert v[0, 1, 1] == oracle.bf16_value(oracle.bf16(np.float32(255 / 1020)))[0]
    assert v[0, 0, 2:4].tolist() == [0.5, 1.0] and v[0, 1, 2:4].tolist() == [0.5, 1.0]
    assert not x[..., 4:].any()


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    w0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    oracle.adam(w, m, v, g.copy(), 1, 1e-3)
    # first step: bias-corrected m = g and v = g^2, so the update is lr * g / (|g| + eps)
    assert np.allclose(w, w0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
