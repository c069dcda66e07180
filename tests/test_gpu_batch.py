"""GPU parity of the batched persistent solve.

Every pair of a batch must come out bit-identical to the CPU oracle (small pairs) and to
its own solo GPU solve (larger pairs); reordering the batch or changing the tuned launch
shape must not change any pair's result.
"""
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


def small_pairs():
    shapes = [(40, 32, 16), (64, 48, 32), (33, 21, 64), (48, 40, 8), (17, 29, 16), (70, 22, 5), (24, 24, 24)]
    out = []
    for i, (W, H, D) in enumerate(shapes):
        p = synth.make_pair(W, H, D, (3, 5), False, 0, False, seed=500 + i)
        out.append((p["left"], p["right"], D))
    return out


# (lambda, T) with messages kept in 12 bits (lambda T <= 4095), in 16 bits with the packed
# 16-bit sums available (<= 16383), and in 16 bits on the int32 path only
STORAGES = [(64, 4, 12), (1500, 4, 16), (5000, 4, 16)]


@pytest.mark.parametrize("lam,trunc,bits", STORAGES)
@pytest.mark.parametrize("skip", [0, 1, 2])
def test_batch_matches_oracle(skip, lam, trunc, bits):
    pairs = small_pairs()
    params = B.make_batch_params(5, 3, [6, 5, 4], lam, trunc, skip_mode=skip)
    say(f"batch of {len(pairs)} small pairs, skip={skip}, lambda={lam}, T={trunc}")
    batch = B.Batch([gpu(l) for l, _, _ in pairs], [gpu(r) for _, r, _ in pairs], [D for _, _, D in pairs], params)
    assert batch.message_bits() == bits
    ctx = B.Context()
    batch.solve(ctx)
    assert batch.status() == 0
    for i, (l, r, D) in enumerate(pairs):
        c = oracle.cost_volume(l, r, D, 5)
        assert np.array_equal(host(batch.costs[i]), c), f"pair {i} cost"
        d, _, _ = oracle.bp_solve(c, 3, [6, 5, 4], lam, trunc, skip, 2, want_msgs=False)
        assert np.array_equal(host(batch.disps[i]), d), f"pair {i} disparity"


def batch_of_generator_pairs(n, seed0):
    pairs = [synth.batch_pair(i, seed0) for i in range(n)]
    return [gpu(p["left"]) for p in pairs], [gpu(p["right"]) for p in pairs], [p["num_disp"] for p in pairs]


def solo(left, right, D, w):
    cost = B.stereo_cost_volume(left, right, D, w["window"])
    d, _, _ = B.bp_hierarchical_solve(cost, w["num_scales"], w["iters"], w["lam"], w["trunc"], w["skip"])
    return cost, d


def test_batch_matches_solo_solves_and_permutation():
    w = dict(synth.BATCH)
    lefts, rights, Ds = batch_of_generator_pairs(12, w["seed0"])
    say("batch of 12 generator pairs vs solo solves")
    params = B.make_batch_params(w["window"], w["num_scales"], w["iters"], w["lam"], w["trunc"], w["skip"])
    batch = B.Batch(lefts, rights, Ds, params)
    ctx = B.Context()
    batch.solve(ctx)
    assert batch.status() == 0
    for i in range(len(lefts)):
        c, d = solo(lefts[i], rights[i], Ds[i], w)
        assert torch.equal(batch.costs[i], c), f"pair {i} cost"
        assert torch.equal(batch.disps[i], d), f"pair {i} disparity"
    perm = [5, 0, 11, 3, 7, 1, 9, 2, 10, 4, 8, 6]
    say("permuted batch")
    b2 = B.Batch([lefts[j] for j in perm], [rights[j] for j in perm], [Ds[j] for j in perm], params)
    b2.solve(ctx)
    assert b2.status() == 0
    for k, j in enumerate(perm):
        assert torch.equal(b2.disps[k], batch.disps[j])


def test_batch_autotune_and_graph_replay():
    w = dict(synth.BATCH)
    lefts, rights, Ds = batch_of_generator_pairs(8, 2000)
    params = B.make_batch_params(w["window"], w["num_scales"], w["iters"], w["lam"], w["trunc"], 1)
    batch = B.Batch(lefts, rights, Ds, params)
    ctx = B.Context()
    batch.solve(ctx)
    ref = [d.clone() for d in batch.disps]
    say("autotune 8 pairs")
    tune = batch.autotune(ctx)
    assert tune["candidates"] and all(c["ms"] < 1e29 for c in tune["candidates"])
    assert all(torch.equal(a, b) for a, b in zip(batch.disps, ref))
    ctx.set_graphs(True)
    s = torch.cuda.Stream()
    say("graph replays of the batch")
    with torch.cuda.stream(s):
        for rep in range(3):
            for d in batch.disps:
                d.fill_(-1)
            batch.solve(ctx, stream=s)
            torch.cuda.synchronize()
            assert batch.status(stream=s) == 0
            assert all(torch.equal(a, b) for a, b in zip(batch.disps, ref)), f"replay {rep}"
    counts = ctx.graph_counts()
    assert counts["captures"] == 1 and counts["replays"] == 2


@pytest.mark.parametrize("skip", [0, 1])
def test_every_schedule_gives_the_same_result(skip):
    w = dict(synth.BATCH)
    lefts, rights, Ds = batch_of_generator_pairs(10, 3000)
    params = B.make_batch_params(w["window"], w["num_scales"], w["iters"], w["lam"], w["trunc"], skip)
    batch = B.Batch(lefts, rights, Ds, params)
    ctx = B.Context()
    ref = None
    for sched, bpc, order in [(1, 1, 0), (2, 1, 0), (0, 1, 0), (0, 1, 1), (0, 2, 0), (0, 3, 1)]:
        say(f"schedule {sched} bpc {bpc} order {order} skip {skip}")
        B.set_batch_schedule(ctx, sched, bpc, order)
        for d in batch.disps:
            d.fill_(-1)
        batch.solve(ctx)
        assert batch.status() == 0
        got = [d.clone() for d in batch.disps]
        if ref is None:
            ref = got
            for i in range(len(lefts)):
                c, d = solo(lefts[i], rights[i], Ds[i], dict(w, skip=skip))
                assert torch.equal(batch.costs[i], c) and torch.equal(got[i], d), f"pair {i}"
        else:
            assert all(torch.equal(a, b) for a, b in zip(got, ref))


@pytest.mark.parametrize("lam,trunc", [(64, 4), (1500, 4)])
@pytest.mark.parametrize("skip", [0, 1, 2])
def test_batch_narrow_schedule_matches_oracle(skip, lam, trunc):
    """Schedule 2 (one launch per phase, packed 16-bit message sums where a pair's pixel
    spans at most 8 lanes and messages are kept in 16 bits: lambda T = 6000) against the
    oracle, with pairs of every lane width: D = 5 and 8 (one lane), 16 and 24 (two, four), 64
    (eight) and 128 (sixteen lanes: the int32 path); with lambda T = 256 (12-bit messages)
    schedule 2 runs as schedule 1."""
    shapes = [(40, 32, 16), (33, 21, 64), (48, 40, 8), (70, 22, 5), (24, 24, 24), (26, 18, 128)]
    pairs = []
    for i, (W, H, D) in enumerate(shapes):
        p = synth.make_pair(W, H, D, (3, 5), False, 0, False, seed=700 + i)
        pairs.append((p["left"], p["right"], D))
    params = B.make_batch_params(5, 3, [6, 5, 4], lam, trunc, skip_mode=skip)
    say(f"narrow schedule, batch of {len(pairs)} small pairs, skip={skip}, lambda={lam}, T={trunc}")
    batch = B.Batch([gpu(l) for l, _, _ in pairs], [gpu(r) for _, r, _ in pairs], [D for _, _, D in pairs], params)
    ctx = B.Context()
    B.set_batch_schedule(ctx, 2)
    batch.solve(ctx)
    assert batch.status() == 0
    for i, (l, r, D) in enumerate(pairs):
        c = oracle.cost_volume(l, r, D, 5)
        assert np.array_equal(host(batch.costs[i]), c), f"pair {i} cost"
        d, _, _ = oracle.bp_solve(c, 3, [6, 5, 4], lam, trunc, skip, 2, want_msgs=False)
        assert np.array_equal(host(batch.disps[i]), d), f"pair {i} disparity"


@pytest.mark.parametrize("lam", [64, 1500])
@pytest.mark.parametrize("sched", [0, 1, 2])
def test_batch_plain_odd_finest_halfsteps(sched, lam):
    """Plain BP with an odd number of finest half-steps: the last one updates the other
    colour, whose winners it writes itself (int32 path), the WTA phase covering the rest."""
    shapes = [(40, 32, 16), (33, 21, 64), (70, 22, 5), (26, 18, 128), (31, 17, 100)]
    pairs = []
    for i, (W, H, D) in enumerate(shapes):
        p = synth.make_pair(W, H, D, (3, 5), False, 0, False, seed=900 + i)
        pairs.append((p["left"], p["right"], D))
    params = B.make_batch_params(5, 3, [5, 4, 3], lam, 4, skip_mode=0)
    say(f"plain batch, 5 finest half-steps, schedule {sched}, lambda={lam}")
    batch = B.Batch([gpu(l) for l, _, _ in pairs], [gpu(r) for _, r, _ in pairs], [D for _, _, D in pairs], params)
    ctx = B.Context()
    B.set_batch_schedule(ctx, sched, 1, 0)
    batch.solve(ctx)
    assert batch.status() == 0
    for i, (l, r, D) in enumerate(pairs):
        c = oracle.cost_volume(l, r, D, 5)
        d, _, _ = oracle.bp_solve(c, 3, [5, 4, 3], lam, 4, 0, 2, want_msgs=False)
        assert np.array_equal(host(batch.disps[i]), d), f"pair {i} disparity"


def test_full_benchmark_batch():
    """The 256-pair batch the benchmark times, autotuned and replayed from a graph: sampled
    pairs equal their solo solves bit for bit (costs and disparities), and the smallest pair
    equals the oracle."""
    w = dict(synth.BATCH)
    n = w["count"]
    pairs = [synth.batch_pair(i, w["seed0"]) for i in range(n)]
    L, iters = w["num_scales"], [w["iters"]] * w["num_scales"]
    params = B.make_batch_params(w["window"], L, iters, w["lam"], w["trunc"], w["skip"], 2, w["cost_scale"],
                                 w["cost_trunc"])
    say("full benchmark batch, 256 pairs")
    batch = B.Batch([gpu(p["left"]) for p in pairs], [gpu(p["right"]) for p in pairs],
                    [p["num_disp"] for p in pairs], params)
    ctx = B.Context()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        batch.autotune(ctx, s)
        ctx.set_graphs(True)
        for d in batch.disps:
            d.fill_(-1)
        batch.solve(ctx, s)
        batch.solve(ctx, s)  # a replay of the captured graph
    torch.cuda.synchronize()
    assert batch.status(stream=s) == 0
    rng = np.random.default_rng(5)
    for i in sorted(set(rng.integers(0, n, 8).tolist())):
        c, d = solo(batch.lefts[i], batch.rights[i], pairs[i]["num_disp"], dict(w, iters=iters))
        assert torch.equal(batch.costs[i], c) and torch.equal(batch.disps[i], d), f"pair {i}"
    small = min(range(n), key=lambda i: pairs[i]["left"].size * pairs[i]["num_disp"])
    p = pairs[small]
    c = oracle.cost_volume(p["left"], p["right"], p["num_disp"], w["window"])
    assert np.array_equal(host(batch.costs[small]), c)
    rd, _, _ = oracle.bp_solve(c, L, iters, w["lam"], w["trunc"], w["skip"], 2, want_msgs=False)
    assert np.array_equal(host(batch.disps[small]), rd), f"pair {small} vs oracle"
