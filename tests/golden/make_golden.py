"""Writes the oracle's full-size results as SHA-256 digests, for the GPU parity tests.

Calls only the CPU oracle (``oracle/``) and the seeded input generator; nothing here
touches the GPU library.  Run once on the CPU (OpenMP uses every host core):

    python tests/golden/make_golden.py large      # -> tests/golden/large_1920x1080_d128.json
    python tests/golden/make_golden.py large_rgb  # adds the colour cost volume's digest to it
    python tests/golden/make_golden.py batch      # -> tests/golden/batch_256.json

Digests are of the arrays' raw little-endian bytes in the library's layouts: images uint8
[H][W] (or [H][W][3]), cost int16 [H][W][D], disparity int16 [H][W], messages int16
[4][H][W][D].  A GPU result matches when its digest does, which makes the comparison
bit-exact over every element without storing gigabytes of expected values.
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1709_06509_amd import synth  # noqa: E402


def digest(a):
    a = np.ascontiguousarray(a)
    if a.dtype.byteorder == ">":
        a = a.byteswap().view(a.dtype.newbyteorder("<"))
    return hashlib.sha256(a.tobytes()).hexdigest()


def log(*a):
    print(*a, flush=True)


def solve_record(cost, L, iters, lam, trunc, skip):
    t = time.time()
    disp, msgs, st = oracle.bp_solve(cost, L, iters, lam, trunc, skip, 2)
    log(f"  solve L={L} iters={iters} skip={skip}: {time.time() - t:.1f} s")
    return {
        "disparity": digest(disp),
        "messages": digest(msgs),
        "energy": oracle.energy(cost, disp, lam, trunc),
        "pixel_updates": int(st["pixel_updates"]),
        "msg_updates": int(st["msg_updates"]),
        "active": [[int(v) for v in st["active"][l][: min(iters[l], 64)]] for l in range(L)],
    }


def make_large(out):
    w = synth.WORKLOADS["large"]
    D, win, L, iters = w["num_disp"], w["window"], w["num_scales"], [w["iters"]] * w["num_scales"]
    lam, trunc = w["lam"], w["trunc"]
    log(f"large: {w['width']}x{w['height']} D={D}, oracle threads {oracle.threads()}")
    p = synth.workload_pair("large")
    lg, rg = oracle.luma(p["left"]), oracle.luma(p["right"])
    t = time.time()
    cost = oracle.cost_volume(lg, rg, D, win, w["cost_scale"], w["cost_trunc"])
    log(f"  cost volume: {time.time() - t:.1f} s")
    rec = {
        "_doc": "SHA-256 digests of the oracle's results on the 1920x1080 RGB pair (D=128, 9x9 NCC, "
                "5 scales x 12 half-steps, lambda 64, T 4), written by tests/golden/make_golden.py from "
                "oracle/ and the seeded generator only",
        "workload": "large", "width": w["width"], "height": w["height"], "num_disp": D, "window": win,
        "num_scales": L, "iters": iters, "lam": lam, "trunc": trunc,
        "left_rgb": digest(p["left"]), "right_rgb": digest(p["right"]),
        "left_luma": digest(lg), "right_luma": digest(rg), "cost": digest(cost),
    }
    # every scale of the pyramid, and the hierarchy's messages at every scale: the solve
    # restricted to scales l..L-1 of the same pyramid ends at scale l with exactly the
    # messages the full hierarchy has there after its half-steps of scale l
    levels = [cost]
    for _ in range(1, L):
        levels.append(oracle.pyramid_level(levels[-1]))
    rec["pyramid"] = [digest(c) for c in levels]
    rec["plain"] = solve_record(cost, L, iters, lam, trunc, 0)
    rec["plain_scales"] = {}
    for l in range(1, L):
        r = solve_record(levels[l], L - l, iters[l:], lam, trunc, 0)
        rec["plain_scales"][str(l)] = {"disparity": r["disparity"], "messages": r["messages"]}
    rec["freeze"] = solve_record(cost, L, iters, lam, trunc, 1)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    log(f"wrote {out}")


def add_large_rgb(out):
    """The colour correlation volume of the same pair (9x9 window, channels pooled)."""
    w = synth.WORKLOADS["large"]
    p = synth.workload_pair("large")
    with open(out) as f:
        rec = json.load(f)
    assert rec["left_rgb"] == digest(p["left"]) and rec["right_rgb"] == digest(p["right"])
    t = time.time()
    cost = oracle.cost_volume_rgb(p["left"], p["right"], w["num_disp"], w["window"], w["cost_scale"], w["cost_trunc"])
    log(f"  colour cost volume: {time.time() - t:.1f} s")
    rec["cost_rgb"] = digest(cost)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    log(f"updated {out}")


def make_batch(out, n):
    b = synth.BATCH
    L, iters = b["num_scales"], [b["iters"]] * b["num_scales"]
    pairs = []
    t0 = time.time()
    for i in range(n):
        p = synth.batch_pair(i, b["seed0"])
        H, W = p["left"].shape
        D = p["num_disp"]
        cost = oracle.cost_volume(p["left"], p["right"], D, b["window"], b["cost_scale"], b["cost_trunc"])
        disp, _, _ = oracle.bp_solve(cost, L, iters, b["lam"], b["trunc"], b["skip"], 2, want_msgs=False)
        pairs.append({"width": W, "height": H, "num_disp": D, "left": digest(p["left"]), "right": digest(p["right"]),
                      "cost": digest(cost), "disparity": digest(disp),
                      "energy": oracle.energy(cost, disp, b["lam"], b["trunc"])})
        if i % 16 == 15:
            log(f"  batch pair {i + 1}/{n}: {time.time() - t0:.0f} s")
    rec = {"_doc": "SHA-256 digests of the oracle's results on every pair of the uneven batch (grey, 7x7 NCC, "
                   "4 scales x 10 half-steps, plain BP, lambda 64, T 4), written by tests/golden/make_golden.py "
                   "from oracle/ and the seeded generator only",
           "seed0": b["seed0"], "count": n, "window": b["window"], "num_scales": L, "iters": iters,
           "lam": b["lam"], "trunc": b["trunc"], "skip": b["skip"], "pairs": pairs}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    log(f"wrote {out}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["large", "large_rgb", "batch"])
    ap.add_argument("--pairs", type=int, default=synth.BATCH["count"])
    a = ap.parse_args()
    if a.what == "large":
        make_large(os.path.join(HERE, "large_1920x1080_d128.json"))
    elif a.what == "large_rgb":
        add_large_rgb(os.path.join(HERE, "large_1920x1080_d128.json"))
    else:
        make_batch(os.path.join(HERE, "batch_256.json"), a.pairs)


if __name__ == "__main__":
    main()
