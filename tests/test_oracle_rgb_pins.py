"""Pins of the oracle's colour correlation (views from a regular RGB camera, the paper's
Abstract) against hand-worked cases and what the definition fixes: grey views give the
one-channel correlation, a common gain with per-channel offsets changes nothing, inverting
every channel negates it, and flat channels drop out."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


@pytest.mark.parametrize("case", GOLDEN["ncc_rgb"], ids=lambda c: c["name"])
def test_rgb_hand_cases(case):
    L = np.array(case["left"], np.uint8)
    R = np.array(case["right"], np.uint8)
    v = oracle.ncc_rgb_at(L, R, case["window"], case["x"], case["y"], case["d"])
    assert abs(v - case["ncc"]) <= 1e-15
    assert oracle.cost_rgb_at(L, R, case["window"], case["x"], case["y"], case["d"]) == case["cost"]


def grey_pair(H, W, seed, hi=256):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, hi, (H, W), dtype=np.uint8)
    R = np.clip(np.roll(L, -3, axis=1).astype(int) + rng.integers(-25, 26, (H, W)), 0, hi - 1).astype(np.uint8)
    R[:, : W // 5] = 40  # flat band: zero-variance windows
    return L, R


@pytest.mark.parametrize("win", [1, 3, 5, 9])
def test_grey_views_give_the_one_channel_correlation(win):
    L, R = grey_pair(7, 23, win)
    L3, R3 = np.repeat(L[..., None], 3, 2), np.repeat(R[..., None], 3, 2)
    c3, n3 = oracle.cost_volume_rgb(L3, R3, 9, win, want_ncc=True)
    c1, n1 = oracle.cost_volume(L, R, 9, win, want_ncc=True)
    assert np.array_equal(c3, c1)  # exact: every pooled sum is three times the grey one
    assert np.max(np.abs(n3 - n1)) <= 1e-12


def test_common_gain_and_channel_offsets_are_ignored():
    rng = np.random.default_rng(2)
    L = rng.integers(0, 60, (6, 19, 3), dtype=np.uint8)
    R = rng.integers(0, 60, (6, 19, 3), dtype=np.uint8)
    base_c, base_n = oracle.cost_volume_rgb(L, R, 7, 5, want_ncc=True)
    for a, offs in [(2, (3, 60, 17)), (4, (0, 11, 5))]:
        L2 = (a * L.astype(int) + np.array(offs)).astype(np.uint8)  # no clipping: values stay below 256
        R2 = (a * R.astype(int) + np.array(offs[::-1])).astype(np.uint8)
        c, n = oracle.cost_volume_rgb(L2, R2, 7, 5, want_ncc=True)
        assert np.array_equal(c, base_c)
        assert np.max(np.abs(n - base_n)) <= 1e-12


def test_inverting_every_channel_negates():
    rng = np.random.default_rng(3)
    L = rng.integers(0, 256, (5, 17, 3), dtype=np.uint8)
    R = rng.integers(0, 256, (5, 17, 3), dtype=np.uint8)
    for (x, y, d) in [(8, 2, 3), (16, 4, 0), (5, 0, 5)]:
        a = oracle.ncc_rgb_at(L, R, 5, x, y, d)
        b = oracle.ncc_rgb_at(L, (255 - R.astype(int)).astype(np.uint8), 5, x, y, d)
        assert abs(a + b) <= 1e-12


@pytest.mark.parametrize("channel", [0, 1, 2])
def test_flat_channels_drop_out(channel):
    """Two channels flat in both views: the colour correlation is the grey one of the third
    (each channel in turn, so a channel left out of the sums fails here)."""
    L, R = grey_pair(6, 21, 4 + channel)
    L3 = np.stack([np.full_like(L, 9), np.full_like(L, 100), np.full_like(L, 200)], -1)
    R3 = np.stack([np.full_like(R, 31), np.full_like(R, 55), np.full_like(R, 77)], -1)
    L3[..., channel], R3[..., channel] = L, R
    c3, n3 = oracle.cost_volume_rgb(L3, R3, 6, 3, want_ncc=True)
    c1, n1 = oracle.cost_volume(L, R, 6, 3, want_ncc=True)
    assert np.array_equal(c3, c1)
    assert np.max(np.abs(n3 - n1)) <= 1e-12


def test_identical_views_and_invalid_columns():
    rng = np.random.default_rng(5)
    L = rng.integers(0, 256, (5, 12, 3), dtype=np.uint8)
    c, n = oracle.cost_volume_rgb(L, L, 4, 3, want_ncc=True)
    assert np.all(c[:, :, 0] == 0) and np.all(np.abs(n[:, :, 0] - 1.0) <= 1e-12)
    for x in range(3):
        for d in range(x + 1, 4):
            assert np.all(c[:, x, d] == 1024) and np.all(n[:, x, d] == -2.0)
