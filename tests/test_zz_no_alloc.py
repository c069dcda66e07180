"""The allocation-free solve (bp_hierarchical_solve_noalloc) against the solve with a
caller workspace (bp_hierarchical_solve), through the C ABI: bit-identical disparities,
messages and counters on consecutive calls that share the library's static scratch (the
second smaller than the first, then larger again), its rejection of shapes that do not fit
the scratch, and graph replays of a captured call with eager work in between."""
import sys

import numpy as np
import pytest
import torch

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


def both(cost, L, iters, lam, T, skip, K=2):
    a = B.bp_hierarchical_solve(cost, L, iters, lam, T, skip, K, want_msgs=True, want_stats=True)
    b = B.bp_hierarchical_solve_noalloc(cost, L, iters, lam, T, skip, K, want_msgs=True, want_stats=True)
    return a, b


def assert_same(a, b):
    assert np.array_equal(host(a[0]), host(b[0])), "disparities differ"
    assert np.array_equal(host(a[1]), host(b[1])), "messages differ"
    assert a[2] == b[2], "counters differ"


def test_noalloc_matches_workspace_solve_on_consecutive_calls():
    w = synth.WORKLOADS["production"]
    p = synth.workload_pair("production")
    cost_big = B.stereo_cost_volume(gpu(p["left"]), gpu(p["right"]), w["num_disp"], w["window"])
    rng = np.random.default_rng(3)
    cost_small = gpu(rng.integers(0, 800, (37, 51, 24)).astype(np.int16))
    # D = 128: messages in 12 bits, the finest scale reading the caller's cost
    cost_wide = gpu(rng.integers(-2000, 2000, (33, 40, 128)).astype(np.int16))
    L, iters = w["num_scales"], [w["iters"]] * w["num_scales"]
    for name, cost, LL, its, skip in [("production 384x288 D=16 freeze", cost_big, L, iters, 1),
                                      ("random 51x37 D=24 plain", cost_small, 3, [7, 6, 5], 0),
                                      ("random 40x33 D=128 plain", cost_wide, 3, [6, 5, 4], 0),
                                      ("production 384x288 D=16 exact skip", cost_big, L, iters, 2),
                                      ("random 40x33 D=128 freeze", cost_wide, 3, [7, 5, 4], 1),
                                      ("random 51x37 D=24 freeze", cost_small, 3, [9, 4, 4], 1)]:
        say(f"noalloc vs workspace solve: {name}")
        a, b = both(cost, LL, its, w["lam"], w["trunc"], skip)
        assert_same(a, b)


def test_noalloc_rejects_shapes_beyond_the_scratch():
    cost = torch.zeros((480, 640, 64), dtype=torch.int16, device="cuda")
    params = B.make_params(64, 4, 10, 64, 4)
    assert B.bp_workspace_bytes(640, 480, params) > B.bp_noalloc_scratch_bytes()
    say("noalloc: a 640x480 D=64 solve does not fit the scratch")
    with pytest.raises(B.BPError) as e:
        B.bp_hierarchical_solve_noalloc(cost, 4, 10, 64, 4)
    assert e.value.code == B.BP_E_WORKSPACE


def test_noalloc_graph_replays():
    rng = np.random.default_rng(4)
    costs = [gpu(rng.integers(0, 700, (45, 61, 16)).astype(np.int16)) for _ in range(2)]
    refs = [host(B.bp_hierarchical_solve(c, 3, [6, 6, 6], 64, 4, 1)[0]) for c in costs]
    disp = torch.empty((45, 61), dtype=torch.int16, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    say("noalloc: capture into a graph, replay with eager calls in between")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        B.bp_hierarchical_solve_noalloc(costs[0], 3, [6, 6, 6], 64, 4, 1, disparity=disp, stream=s)
    for rep in range(3):
        disp.fill_(-7)
        g.replay()
        assert np.array_equal(host(disp), refs[0]), f"replay {rep}"
        other = B.bp_hierarchical_solve_noalloc(costs[1], 3, [6, 6, 6], 64, 4, 1)[0]
        assert np.array_equal(host(other), refs[1]), f"eager call after replay {rep}"
