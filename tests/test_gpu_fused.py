"""GPU parity of the fused half-steps (several half-steps of a scale per launch, from LDS).

The solve with fused launches forced on, and with interior tiles forced small so that even
small images are cut into many tiles with halos, must equal the CPU oracle bit for bit
(final messages and disparities), for plain BP and the freeze rule, odd and even half-step
counts, every lanes-per-pixel width the fused kernel has, and a warm start.
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1709_06509_amd import bpstereo as B
from paper_1709_06509_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture
def fused_ctx():
    ctx = B.Context()
    ctx.set_fused(1)
    yield ctx
    os.environ.pop("BPSTEREO_FUSED_TILE", None)
    ctx.close()


def cost_of(W, H, D, seed, window=5):
    p = synth.make_pair(W, H, D, (3, 5), True, 0, False, seed)
    return oracle.cost_volume(p["left"], p["right"], D, window)


CASES = [
    # W, H, D, L, iters, skip, tile
    (40, 30, 16, 3, [10, 10, 10], 0, "6x4"),
    (40, 30, 16, 3, [10, 10, 10], 1, "6x4"),
    (37, 23, 16, 3, [7, 5, 3], 1, "5x7"),
    (33, 21, 8, 3, [9, 6, 4], 0, "4x4"),
    (33, 21, 8, 3, [9, 6, 4], 1, "8x3"),
    (29, 17, 24, 2, [6, 6], 1, "7x5"),
    (24, 20, 32, 3, [6, 6, 6], 0, "5x5"),
    (26, 19, 64, 2, [5, 4], 1, "3x3"),
    (30, 22, 5, 3, [1, 3, 2], 1, "4x6"),
    (64, 48, 16, 4, [10, 10, 10, 10], 1, None),
    (17, 1, 9, 2, [6, 6], 1, "4x1"),
    (1, 19, 9, 2, [6, 6], 0, "1x5"),
]


@pytest.mark.parametrize("case", CASES)
def test_fused_matches_oracle(case, fused_ctx):
    W, H, D, L, iters, skip, tile = case
    say(f"fused {W}x{H} D={D} L={L} iters={iters} skip={skip} tile={tile}")
    if tile:
        os.environ["BPSTEREO_FUSED_TILE"] = tile
    else:
        os.environ.pop("BPSTEREO_FUSED_TILE", None)
    cost = cost_of(W, H, D, 900 + W + H + D)
    d, m, _ = B.bp_hierarchical_solve(gpu(cost), L, iters, 64, 4, skip, 2, want_msgs=True, ctx=fused_ctx)
    rd, rm, _ = oracle.bp_solve(cost, L, iters, 64, 4, skip, 2)
    assert np.array_equal(host(m), rm), "messages differ"
    assert np.array_equal(host(d), rd), "disparities differ"


@pytest.mark.parametrize("compact", ["0", "1"])
@pytest.mark.parametrize("case", [CASES[1], CASES[2], CASES[4], CASES[5], CASES[7], CASES[9]])
def test_fused_listing_forced(case, compact, fused_ctx):
    """Freeze-rule half-steps in fused launches with the listing of active pixels forced on
    or off (by default it is used only where a compute unit holds more than a wave per SIMD)."""
    W, H, D, L, iters, skip, tile = case
    say(f"fused {W}x{H} D={D} tile={tile}, listing {compact}")
    if tile:
        os.environ["BPSTEREO_FUSED_TILE"] = tile
    else:
        os.environ.pop("BPSTEREO_FUSED_TILE", None)
    os.environ["BPSTEREO_FUSED_COMPACT"] = compact
    try:
        cost = cost_of(W, H, D, 900 + W + H + D)
        d, m, _ = B.bp_hierarchical_solve(gpu(cost), L, iters, 64, 4, skip, 2, want_msgs=True, ctx=fused_ctx)
        torch.cuda.synchronize()
    finally:
        os.environ.pop("BPSTEREO_FUSED_COMPACT", None)
    rd, rm, _ = oracle.bp_solve(cost, L, iters, 64, 4, skip, 2)
    assert np.array_equal(host(m), rm), "messages differ"
    assert np.array_equal(host(d), rd), "disparities differ"


def test_fused_warm_start_matches_oracle(fused_ctx):
    W, H, D, L = 36, 28, 16, 3
    os.environ["BPSTEREO_FUSED_TILE"] = "5x4"
    say("fused warm start")
    cost = cost_of(W, H, D, 77)
    hs, ws = H, W
    for _ in range(L - 2):
        hs, ws = (hs + 1) // 2, (ws + 1) // 2
    warm = np.random.default_rng(3).integers(0, 257, (4, hs, ws, D)).astype(np.int16)
    for skip in (0, 1):
        d, m, _ = B.bp_hierarchical_solve(gpu(cost), L, [6, 5, 0], 64, 4, skip, 2, warm_msgs=gpu(warm),
                                          want_msgs=True, ctx=fused_ctx)
        rd, rm, _ = oracle.bp_solve(cost, L, [6, 5, 0], 64, 4, skip, 2, warm_msgs=warm)
        assert np.array_equal(host(m), rm) and np.array_equal(host(d), rd)


def test_fused_modes_agree_on_production_pair():
    """Production workload: one launch per half-step, fused wherever it fits, and the default
    size rule give the same disparities and messages, eager and replayed from a graph."""
    w = synth.WORKLOADS["production"]
    p = synth.workload_pair("production")
    cost = B.stereo_cost_volume(gpu(p["left"]), gpu(p["right"]), w["num_disp"], w["window"])
    L, iters = w["num_scales"], w["iters"]
    outs = []
    for mode in (0, 1, 2):
        ctx = B.Context()
        ctx.set_fused(mode)
        say(f"production, fused mode {mode}")
        d, m, _ = B.bp_hierarchical_solve(cost, L, iters, w["lam"], w["trunc"], w["skip"], 2, want_msgs=True, ctx=ctx)
        outs.append((host(d), host(m)))
        if mode == 2:
            ctx.set_graphs(True)
            ws = torch.empty(B.bp_workspace_bytes(w["width"], w["height"],
                                                  B.make_params(w["num_disp"], L, iters, w["lam"], w["trunc"],
                                                                w["skip"])), dtype=torch.uint8, device="cuda")
            disp = torch.empty((w["height"], w["width"]), dtype=torch.int16, device="cuda")
            stream = torch.cuda.Stream()  # the context captures graphs on a non-default stream
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                for _ in range(3):
                    B.bp_hierarchical_solve(cost, L, iters, w["lam"], w["trunc"], w["skip"], 2, ctx=ctx,
                                            workspace=ws, disparity=disp)
                    assert np.array_equal(host(disp), outs[0][0])
            counts = ctx.graph_counts()
            assert counts["captures"] == 1 and counts["replays"] == 2
        ctx.close()
    for d, m in outs[1:]:
        assert np.array_equal(d, outs[0][0]) and np.array_equal(m, outs[0][1])


# The packed 16-bit message sums (scales above the finest, capv <= 10922): at the limit the
# sums reach 32767 + 3 * 10922 = 65533, one past it the int32 path runs instead.
@pytest.mark.parametrize("lam,T", [(10922, 1), (10923, 1), (5461, 2), (64, 4)])
def test_fused_packed_sums_at_the_limit(lam, T, fused_ctx):
    os.environ["BPSTEREO_FUSED_TILE"] = "5x4"
    rng = np.random.default_rng(lam + T)
    cost = rng.integers(20000, 32768, (27, 35, 16)).astype(np.int16)  # coarse costs saturate
    say(f"fused packed-sum limit lam={lam} T={T}")
    for skip in (0, 1):
        d, m, _ = B.bp_hierarchical_solve(gpu(cost), 4, [6, 6, 6, 6], lam, T, skip, 2, want_msgs=True, ctx=fused_ctx)
        rd, rm, _ = oracle.bp_solve(cost, 4, [6, 6, 6, 6], lam, T, skip, 2)
        assert np.array_equal(host(m), rm) and np.array_equal(host(d), rd)


@pytest.mark.parametrize("warm_iters", [0, 1, 2])
def test_fused_warm_values_beyond_capv(warm_iters, fused_ctx):
    """Warm messages far above capv: the warm scale reads them on the int32 path, and with
    fewer than two half-steps there they also reach the finer scales, which then stay off the
    packed path."""
    os.environ["BPSTEREO_FUSED_TILE"] = "4x4"
    W, H, D, L = 34, 26, 16, 4
    cost = cost_of(W, H, D, 91)
    hs, ws = H, W
    for _ in range(L - 2):
        hs, ws = (hs + 1) // 2, (ws + 1) // 2
    warm = np.random.default_rng(warm_iters).integers(0, 32768, (4, hs, ws, D)).astype(np.int16)
    iters = [5, 4, warm_iters, 0]
    say(f"fused warm start, warm-scale half-steps {warm_iters}")
    for skip in (0, 1):
        d, m, _ = B.bp_hierarchical_solve(gpu(cost), L, iters, 64, 4, skip, 2, warm_msgs=gpu(warm), want_msgs=True,
                                          ctx=fused_ctx)
        rd, rm, _ = oracle.bp_solve(cost, L, iters, 64, 4, skip, 2, warm_msgs=warm)
        assert np.array_equal(host(m), rm) and np.array_equal(host(d), rd)


def test_fused_negative_finest_costs(fused_ctx):
    os.environ["BPSTEREO_FUSED_TILE"] = "6x5"
    rng = np.random.default_rng(17)
    cost = rng.integers(-32768, 32768, (23, 31, 16)).astype(np.int16)
    say("fused, negative finest costs")
    for skip in (0, 1):
        d, m, _ = B.bp_hierarchical_solve(gpu(cost), 3, [6, 6, 6], 64, 4, skip, 2, want_msgs=True, ctx=fused_ctx)
        rd, rm, _ = oracle.bp_solve(cost, 3, [6, 6, 6], 64, 4, skip, 2)
        assert np.array_equal(host(m), rm) and np.array_equal(host(d), rd)


@pytest.mark.parametrize("tail", ["2", "4", "7"])
def test_fused_tail_on_production_pair(tail):
    """Under the freeze rule, the half-steps of a scale from t = k on in fused launches after
    one launch each before (the tail hook), on the production pair: equal to the oracle."""
    w = synth.WORKLOADS["production"]
    p = synth.workload_pair("production")
    cost = oracle.cost_volume(p["left"], p["right"], w["num_disp"], w["window"])
    L, iters = w["num_scales"], [w["iters"]] * w["num_scales"]
    os.environ["BPSTEREO_FUSED_TAIL"] = tail
    try:
        ctx = B.Context()
        say(f"production pair, fused tail from t = {tail}")
        d, m, _ = B.bp_hierarchical_solve(gpu(cost), L, iters, w["lam"], w["trunc"], w["skip"], 2, want_msgs=True,
                                          ctx=ctx)
        dm = (host(d), host(m))
        ctx.close()
    finally:
        os.environ.pop("BPSTEREO_FUSED_TAIL", None)
    rd, rm, _ = oracle.bp_solve(cost, L, iters, w["lam"], w["trunc"], w["skip"], 2)
    assert np.array_equal(dm[1], rm) and np.array_equal(dm[0], rd)
