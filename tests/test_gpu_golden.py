"""Full-size parity: every element of the GPU results on the 1920x1080 RGB pair (D = 128,
5 scales x 12 half-steps) and on all 256 pairs of the uneven batch, against the oracle.

The oracle's results at these sizes take minutes of CPU time, so tests/golden/make_golden.py
(which calls only oracle/ and the seeded generator) stored their SHA-256 digests once; a GPU
array matches when the digest of its raw little-endian bytes does.  Each run also checks the
digests of the generated inputs, so a generator that drifted fails here first, not as a
parity failure.  The GPU path runs in the launch configuration the benchmark times.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest
import torch

from paper_1709_06509_amd import bpstereo as B
from paper_1709_06509_amd import synth
from paper_1709_06509_amd import warmstart as WS

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def digest(a):
    if isinstance(a, torch.Tensor):
        torch.cuda.synchronize()
        a = a.cpu().numpy()
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def large():
    g = load("large_1920x1080_d128.json")
    w = synth.WORKLOADS["large"]
    p = synth.workload_pair("large")
    assert digest(p["left"]) == g["left_rgb"] and digest(p["right"]) == g["right_rgb"], "generator drifted"
    say("large pair: luma and cost volume on the GPU")
    lg = B.stereo_luma(torch.from_numpy(p["left"]).cuda())
    rg = B.stereo_luma(torch.from_numpy(p["right"]).cuda())
    cost = B.stereo_cost_volume(lg, rg, w["num_disp"], w["window"], w["cost_scale"], w["cost_trunc"])
    return g, w, lg, rg, cost


def test_large_luma_cost_and_pyramid(large):
    g, w, lg, rg, cost = large
    assert digest(lg) == g["left_luma"] and digest(rg) == g["right_luma"]
    assert digest(cost) == g["cost"], "cost volume differs from the oracle's"
    L = w["num_scales"]
    for l in range(1, L):
        say(f"large pair: pyramid scale {l}")
        assert digest(WS.pyramid_level(cost, L, l)) == g["pyramid"][l], f"pyramid scale {l}"


def test_large_colour_cost_volume(large):
    """The colour correlation volume of the same RGB pair (channels pooled), every element."""
    g, w, _, _, _ = large
    p = synth.workload_pair("large")
    say("large pair: colour cost volume on the GPU")
    c = B.stereo_cost_volume_rgb(torch.from_numpy(p["left"]).cuda(), torch.from_numpy(p["right"]).cuda(),
                                 w["num_disp"], w["window"], w["cost_scale"], w["cost_trunc"])
    assert digest(c) == g["cost_rgb"], "colour cost volume differs from the oracle's"


def test_large_plain_solve_every_element(large):
    """The finest messages and disparities of the whole 5 x 12 solve, the messages each
    coarser scale ends with, and the energy."""
    g, w, _, _, cost = large
    L, iters, lam, T = w["num_scales"], [w["iters"]] * w["num_scales"], w["lam"], w["trunc"]
    say("large pair: plain solve, 5 scales x 12 half-steps")
    d, m, _ = B.bp_hierarchical_solve(cost, L, iters, lam, T, 0, 2, want_msgs=True, ctx=B.Context())
    assert digest(d) == g["plain"]["disparity"], "disparity differs from the oracle's"
    assert digest(m) == g["plain"]["messages"], "finest messages differ from the oracle's"
    del m
    assert int(B.bp_energy(cost, d, lam, T).cpu()[0]) == g["plain"]["energy"]
    for l in range(1, L):
        say(f"large pair: the hierarchy's messages at scale {l}")
        cl = WS.pyramid_level(cost, L, l)
        dl, ml, _ = B.bp_hierarchical_solve(cl, L - l, iters[l:], lam, T, 0, 2, want_msgs=True)
        assert digest(ml) == g["plain_scales"][str(l)]["messages"], f"scale {l} messages"
        assert digest(dl) == g["plain_scales"][str(l)]["disparity"], f"scale {l} disparity"


def test_large_freeze_rule_every_element(large):
    g, w, _, _, cost = large
    L, iters, lam, T = w["num_scales"], [w["iters"]] * w["num_scales"], w["lam"], w["trunc"]
    say("large pair: freeze rule, 5 scales x 12 half-steps")
    d, m, _ = B.bp_hierarchical_solve(cost, L, iters, lam, T, 1, 2, want_msgs=True, ctx=B.Context())
    assert digest(d) == g["freeze"]["disparity"], "disparity differs from the oracle's"
    assert digest(m) == g["freeze"]["messages"], "finest messages differ from the oracle's"
    del m
    _, _, st = B.bp_hierarchical_solve(cost, L, iters, lam, T, 1, 2, want_stats=True)
    assert st["pixel_updates"] == g["freeze"]["pixel_updates"]
    assert st["msg_updates"] == g["freeze"]["msg_updates"]
    for l in range(L):
        assert st["active"][l][: len(g["freeze"]["active"][l])] == g["freeze"]["active"][l], f"scale {l} active"


def test_full_batch_every_pair():
    """All 256 pairs of the uneven batch through one autotuned batched solve: every pair's
    cost volume and disparity against the oracle's."""
    g = load("batch_256.json")
    b = dict(synth.BATCH)
    n = g["count"]
    pairs = [synth.batch_pair(i, g["seed0"]) for i in range(n)]
    for i, (p, ref) in enumerate(zip(pairs, g["pairs"])):
        assert digest(p["left"]) == ref["left"] and digest(p["right"]) == ref["right"], f"generator drifted, pair {i}"
    lefts = [torch.from_numpy(p["left"]).cuda() for p in pairs]
    rights = [torch.from_numpy(p["right"]).cuda() for p in pairs]
    params = B.make_batch_params(b["window"], b["num_scales"], b["iters"], b["lam"], b["trunc"], b["skip"], 2,
                                 b["cost_scale"], b["cost_trunc"])
    batch = B.Batch(lefts, rights, [p["num_disp"] for p in pairs], params)
    ctx = B.Context()
    say(f"batch of {n} pairs: autotune, then solve")
    batch.autotune(ctx)
    batch.solve(ctx)
    assert batch.status() == 0
    bad = [i for i in range(n) if digest(batch.costs[i]) != g["pairs"][i]["cost"]]
    assert not bad, f"cost volumes differ from the oracle's for pairs {bad[:10]}"
    bad = [i for i in range(n) if digest(batch.disps[i]) != g["pairs"][i]["disparity"]]
    assert not bad, f"disparities differ from the oracle's for pairs {bad[:10]}"
