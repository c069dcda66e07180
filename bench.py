"""Benchmark: stereo pairs/s of the whole GPU path on the largest single-pair workload.

One step = one synthetic 1920x1080 RGB pair (luma of both views, D = 128, 9x9 NCC window)
through the correlation volume, the 5-scale x 12-half-step hierarchical solve (plain BP),
winner-take-all and the energy.  Inputs are resident in HBM before timing.  Other
workloads (--workload production | tiny | batched | jacobi | live) are the smaller and
batched configurations.

Prints one JSON line.  Besides the headline pairs/s it reports message updates/s, the
energy against plain BP on the same pair, the roofline of the dominant kernel (the
half-step message update, timed with HIP events on its launch stream inside the timed
region), the run time against the number of half-steps, and the CPU oracle's throughput
on a bounded sample of the same workload, single-threaded and on every host core.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "stereo pairs/s and Gmsg-updates/s at equal energy vs plain BP; % HBM peak"
HBM_PEAK_GBS = 8000.0
# sources that define the half-step kernel; measured traffic counts only while they are unchanged
HALFSTEP_SOURCES = ["paper_1709_06509_amd/csrc/bp_device.h", "paper_1709_06509_amd/csrc/bp_kernels.hip",
                    "paper_1709_06509_amd/csrc/fused_kernels.hip", "paper_1709_06509_amd/csrc/internal.h",
                    "paper_1709_06509_amd/csrc/api.cpp", "paper_1709_06509_amd/csrc/batch_kernels.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "halfstep_traffic.json")


def halfstep_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in HALFSTEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per half-step launch from the profiler's counters (profiles/halfstep_traffic.json),
    or None when there is no record for the workload or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    w = rec.get("workloads", {}).get(workload)
    if not w or rec.get("source_sha256") != halfstep_source_hash():
        return None
    return w["traffic_bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="large", choices=["large", "production", "tiny", "batched", "jacobi", "live", "warm"])
    ap.add_argument("--batch-pairs", type=int, default=256, help="pairs of the batched workload")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU-oracle sample (small workloads)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the step only: no event-free rerun, graph replay or half-step sweep (for profiling)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB device-to-device 3 times (a kernel of "
                         "known traffic, for scaling profiler byte counters)")
    return ap.parse_args()


def halfstep_bytes(stats, D, levels, skip, msg_bits=16):
    """Algorithmic bytes of the half-step launches of one solve per pixel update: the data
    term (int16, 2*D) and 4 incoming messages read and 4 outgoing written, each D labels of
    msg_bits / 8 bytes (18*D in all with 16-bit messages, 14*D with 12-bit ones), plus the 4
    previous outgoing messages read where the freeze rule or the exact skip compares them."""
    mb = msg_bits / 8.0
    total = 0
    for l in range(levels):
        for t in range(min(stats["n_halfsteps"][l], 64)):
            n = stats["active"][l][t]
            total += (2 + 8 * mb) * D * n
            if (skip == 1 and t >= 2) or skip == 2:
                total += 4 * mb * D * n
    return int(total)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_pair_time(left, right, w, threads):
    """Seconds the CPU oracle takes for one pair on `threads` host threads: luma (RGB),
    cost volume, hierarchical solve, energy."""
    import oracle

    oracle.set_threads(threads)
    t0 = time.perf_counter()
    if w["rgb"]:
        left, right = oracle.luma(left), oracle.luma(right)
    cost = oracle.cost_volume(left, right, w["num_disp"], w["window"], w["cost_scale"], w["cost_trunc"])
    d, _, _ = oracle.bp_solve(cost, w["num_scales"], [w["iters"]] * w["num_scales"], w["lam"], w["trunc"], w["skip"], 2,
                              want_msgs=False)
    oracle.energy(cost, d, w["lam"], w["trunc"])
    return time.perf_counter() - t0


def cpu_baseline(w, seconds):
    """The CPU oracle (test infrastructure, never on the GPU path) timed on this host.

    Small workloads: whole pairs, repeated for about `seconds`.  The large pair: a bounded
    sample of it, full-width strips of its top rows (same D, window and schedule, the same
    share of columns with x - d < 0), whose time scales with the pixel count; pairs/s is
    extrapolated from the strip's pixels to the whole pair's.  Both single-threaded and on
    every host thread the oracle's OpenMP loops use."""
    import numpy as np

    import oracle
    from paper_1709_06509_amd import synth

    p = synth.workload_pair(w["name"])
    H, W = w["height"], w["width"]
    threads = oracle.threads()
    if w["name"] == "large":
        runs = {}
        for nthr, rows in ((1, 8), (threads, min(H, 8 * threads))):
            lc = np.ascontiguousarray(p["left"][:rows])
            rc = np.ascontiguousarray(p["right"][:rows])
            el = oracle_pair_time(lc, rc, w, nthr)
            runs[nthr] = (rows, el, (rows * W) / (H * W) / el)
        oracle.set_threads(threads)
        rows, el, v = runs[threads]
        rows1, el1, v1 = runs[1]
        return {"value": v, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                "sample": f"the top {rows} rows (full width {W}) of the {W}x{H} RGB pair: luma, cost volume, "
                          f"{w['num_scales']}x{w['iters']} solve, energy; {el:.1f} s on {threads} threads, "
                          f"extrapolated by pixel count to the whole pair",
                "single_core_value": v1,
                "single_core_sample": f"the top {rows1} rows, {el1:.1f} s on 1 thread",
                "nproc": os.cpu_count(), "cpu_model": cpu_model()}
    res = {}
    for nthr in (1, threads):
        n, t0 = 0, time.perf_counter()
        while True:
            oracle_pair_time(p["left"], p["right"], w, nthr)
            n += 1
            el = time.perf_counter() - t0
            if el >= seconds or n >= 1000:
                break
        res[nthr] = (n, el)
    oracle.set_threads(threads)
    n, el = res[threads]
    n1, el1 = res[1]
    return {"value": n / el, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full {w['width']}x{w['height']} pairs (cost volume + {w['num_scales']}x{w['iters']} "
                      f"solve, skip={w['skip']} + energy) on {threads} threads, {el:.1f} s",
            "single_core_value": n1 / el1, "single_core_sample": f"{n1} pairs on 1 thread, {el1:.1f} s",
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def plain_counts(W, H, levels, iters):
    """Pixel and directed-message updates of plain BP on a W x H pair (no skipping): half-step t
    updates the pixels of one colour and sends one message along every 4-edge."""
    pix = msg = 0
    for l in range(levels):
        w, h = W, H
        for _ in range(l):
            w, h = (w + 1) // 2, (h + 1) // 2
        edges = (w - 1) * h + w * (h - 1)
        n0 = (w * h + 1) // 2
        for t in range(iters[l]):
            pix += n0 if t % 2 == 0 else w * h - n0
            msg += edges
    return pix, msg


def run_batched(args):
    import torch

    from paper_1709_06509_amd import bpstereo as B
    from paper_1709_06509_amd import synth

    w = dict(synth.BATCH)
    n = args.batch_pairs
    dev = torch.device("cuda:0")
    pairs = [synth.batch_pair(i, w["seed0"]) for i in range(n)]
    lefts = [torch.from_numpy(p["left"]).to(dev) for p in pairs]
    rights = [torch.from_numpy(p["right"]).to(dev) for p in pairs]
    Ds = [p["num_disp"] for p in pairs]
    L, iters = w["num_scales"], [w["iters"]] * w["num_scales"]
    params = B.make_batch_params(w["window"], L, iters, w["lam"], w["trunc"], w["skip"], 2, w["cost_scale"],
                                 w["cost_trunc"])
    batch = B.Batch(lefts, rights, Ds, params)
    ctx = B.Context()
    if args.calib_copy_mib:
        # a plain copy of known size: the scale of the profiler's byte counters
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch.solve(ctx, stream)
        tune = batch.autotune(ctx, stream)
        ctx.set_graphs(True)
        for _ in range(max(1, args.warmup // 10)):
            batch.solve(ctx, stream)
        torch.cuda.synchronize()
        steps = max(1, args.steps // 20)
        t0 = time.perf_counter()
        for _ in range(steps):
            batch.solve(ctx, stream)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        status = batch.status(stream)
        best = tune["candidates"][tune["best"]]
        timing = None
        if best["schedule"] in (1, 2):
            # the dominant kernel's own time: the same batch launched eagerly, a HIP event pair
            # on the launch stream around every half-step phase
            ctx.set_graphs(False)
            ctx.set_timing(True)
            n_timed = 3
            for _ in range(n_timed):
                batch.solve(ctx, stream)
            torch.cuda.synchronize()
            timing = ctx.take_timing()
            timing["solves"] = n_timed
            ctx.set_timing(False)
    msgs = byts = 0
    bits = batch.message_bits()  # a pixel update moves its cost (2 D bytes) and 8 messages
    for p, D in zip(pairs, Ds):
        H, W = p["left"].shape
        pix, m = plain_counts(W, H, L, iters)
        msgs += m
        byts += (2 + bits) * D * pix
    per_batch = elapsed / steps
    if timing and timing["halfstep_launches"]:
        launches = timing["halfstep_launches"] // timing["solves"]
        avg_launch_s = timing["halfstep_ms"] / 1e3 / timing["halfstep_launches"]
        per_launch = byts / launches
        kernel = ("k_batch_phase, half-step phases (one launch per phase, every pair's tiles"
                  + ("; packed sums on scales that fit the caches)" if best["schedule"] == 2 else ")"))
    else:
        launches, avg_launch_s, per_launch = 1, best["ms"] / 1e3, byts
        kernel = (f"k_batch_solve (one persistent launch, {best['blocks_per_cu']} workgroups/CU; "
                  "half-step bytes over the whole solve part)")
    achieved = per_launch / avg_launch_s / 1e9
    # profiler-measured HBM bytes per half-step phase launch (the default batch, per-phase schedules)
    traffic = measured_traffic("batched") if timing and n == 256 else None
    return {
        "metric": METRIC, "value": n / per_batch, "unit": "pairs/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": per_batch * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int16", "data": "synthetic",
        "config": {"workload": f"batched: {n} pairs, W 160..640, H 128..480 (step 16), D in {{16,32,64}}, "
                               f"{w['window']}x{w['window']} NCC, {L} scales x {w['iters']} half-steps, skip={w['skip']}, "
                               f"seeds {w['seed0']}..{w['seed0'] + n - 1}", "pairs_per_step": n},
        "gmsg_updates_per_s": msgs / per_batch / 1e9,
        "batch_status": status,
        "roofline": {"bound": "hbm", "kernel": kernel,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_us": avg_launch_s * 1e6, "algorithmic_bytes_per_launch": per_launch,
                     "launches_per_step": launches, "message_bits": bits},
        "autotune": tune,
    }


def run_jacobi(args):
    """The Jacobi schedule (two sets of four message volumes) on the large pair's cost
    volume: 12 iterations of 1920x1080, D = 128, from zero messages."""
    import torch

    from paper_1709_06509_amd import bpstereo as B
    from paper_1709_06509_amd import synth

    w = dict(synth.WORKLOADS["large"])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = synth.workload_pair("large")
    D, H, W, n = w["num_disp"], w["height"], w["width"], w["iters"]
    gl, gr = B.stereo_luma(torch.from_numpy(p["left"]).to(dev)), B.stereo_luma(torch.from_numpy(p["right"]).to(dev))
    cost = B.stereo_cost_volume(gl, gr, D, w["window"])
    ws = torch.empty(B.bp_jacobi_workspace_bytes(W, H, D), dtype=torch.uint8, device=dev)
    out = torch.empty((4, H, W, D), dtype=torch.int16, device=dev)
    stream = torch.cuda.Stream()

    def timed(iterations, reps):
        with torch.cuda.stream(stream):
            for _ in range(2):
                B.bp_jacobi_iterations(cost, w["lam"], w["trunc"], iterations, workspace=ws, out=out, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                B.bp_jacobi_iterations(cost, w["lam"], w["trunc"], iterations, workspace=ws, out=out, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    steps = max(1, args.steps // 20)
    per_call = timed(n, steps)
    # one iteration = two half-step launches (one per colour); their time is the difference
    # between calls of n and 2 iterations, which share the conversions in and out
    per_iter = (per_call - timed(2, steps)) / (n - 2)
    msgs = 4 * W * H - 2 * W - 2 * H  # directed messages an iteration recomputes
    byts = 2 * D * W * H + 4 * D * msgs  # the cost once, every message read once and written once
    achieved = byts / per_iter / 1e9
    return {
        "metric": METRIC, "value": n * msgs / per_call / 1e9, "unit": "Gmsg-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": 2, "ms_per_step": per_call * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int16", "data": "synthetic",
        "config": {"workload": f"jacobi: {n} Jacobi iterations (two sets of four message volumes) on the "
                               f"{W}x{H}, D={D} synthetic pair's {w['window']}x{w['window']} NCC cost volume, "
                               "from zero messages, with the conversions in and out"},
        "roofline": {"bound": "hbm", "kernel": "k_halfstep<16, 0, 0, 4> (streamed), two launches an iteration",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "avg_launch_us": per_iter / 2 * 1e6, "algorithmic_bytes_per_launch": byts / 2,
                     "launches_per_step": 2 * n},
    }


def run_live(args, frames=16, live_halfsteps=4):
    """A live sequence of the production pair (a static scene, fresh sensor noise per frame):
    frame 0 through the full hierarchy, every later frame through the finest scale alone,
    warm-started from the previous frame's final messages.  Each frame: cost volume, solve,
    energy; the plain hierarchy on the same frames is timed and judged beside it."""
    import numpy as np
    import torch

    from paper_1709_06509_amd import bpstereo as B
    from paper_1709_06509_amd import synth

    w = dict(synth.WORKLOADS["production"])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = synth.workload_pair("production")
    D, L, n = w["num_disp"], w["num_scales"], w["iters"]
    lam, T, skip = w["lam"], w["trunc"], w["skip"]

    def frame(img, seed):
        rng = np.random.default_rng(seed)
        return np.clip(img.astype(np.float64) + rng.normal(0.0, 2.0, img.shape), 0, 255).round().astype(np.uint8)

    views = [(torch.from_numpy(frame(p["left"], 100 + f)).to(dev), torch.from_numpy(frame(p["right"], 200 + f)).to(dev))
             for f in range(frames)]
    costs = [B.stereo_cost_volume(lv, rv, D, w["window"]) for lv, rv in views]

    def plain(f):
        d, _, _ = B.bp_hierarchical_solve(costs[f], L, [n] * L, lam, T, skip, 2)
        return d, B.bp_energy(costs[f], d, lam, T)

    def live(f, prev):
        if prev is None:
            d, m, _ = B.bp_hierarchical_solve(costs[f], L, [n] * L, lam, T, skip, 2, want_msgs=True)
        else:
            d, m, _ = B.bp_hierarchical_solve(costs[f], 2, [live_halfsteps, 0], lam, T, skip, 2, warm_msgs=prev,
                                              want_msgs=True)
        return d, m, B.bp_energy(costs[f], d, lam, T)

    def sequence(kind, reps):
        for _ in range(2):  # warm-up
            prev = None
            for f in range(frames):
                if kind == "plain":
                    plain(f)
                else:
                    _, prev, _ = live(f, prev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            prev = None
            for f in range(frames):
                if kind == "plain":
                    plain(f)
                else:
                    _, prev, _ = live(f, prev)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps / frames

    reps = max(1, args.steps // 40)
    t_plain, t_live = sequence("plain", reps), sequence("live", reps)
    ratios, prev = [], None
    for f in range(frames):
        _, ep = plain(f)
        _, prev, el = live(f, prev)
        ratios.append(int(el.item()) / int(ep.item()))
    later = ratios[1:]
    return {
        "metric": METRIC, "value": 1.0 / t_live, "unit": "frames/s", "n_gpus": 1, "steps": reps * frames,
        "warmup": 2 * frames, "ms_per_step": t_live * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int16", "data": "synthetic",
        "config": {"workload": f"live: {frames} frames of the {w['width']}x{w['height']}, D={D} pair (a static "
                               f"scene, fresh noise sigma 2 per frame); frame 0 through {L} scales x {n} half-steps, "
                               f"later frames through the finest scale alone, {live_halfsteps} half-steps from the "
                               f"previous frame's final messages; skip={skip}; eager launches, cost volume + solve "
                               "+ energy per frame"},
        "plain_frames_per_s": 1.0 / t_plain, "speedup_vs_plain": t_plain / t_live,
        "energy_ratio_live_vs_plain_mean": float(np.mean(later)), "energy_ratio_live_vs_plain_max": float(max(later)),
        "frames_within_0.5pct": int(sum(r <= 1.005 for r in later)), "frames_judged": len(later),
    }


def run_warm(args, schedule=(8, 6, 6)):
    """The learned warm start's step at its evaluation size (640x480, D = 64, 4 scales): cost
    volume plus the warm-started solve with the network as one launch inside it
    (bp_warmstart_solve), against the same step through the layer-level calls and against
    plain BP.  The network is freshly initialised: the kernels' time does not depend on the
    weights (its accuracy is the warm-start experiment's subject, not this one's)."""
    import torch

    from paper_1709_06509_amd import bpstereo as B
    from paper_1709_06509_amd import synth
    from paper_1709_06509_amd import warmstart as WS

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W, H, D, L, win, lam, T, its = 640, 480, 64, 4, 7, 64, 4, 10
    p = synth.make_pair(W, H, D, (8, 12), True, 0, False, 200000)
    left, right = torch.from_numpy(p["left"]).to(dev), torch.from_numpy(p["right"]).to(dev)
    cost = torch.empty((H, W, D), dtype=torch.int16, device=dev)
    disp = torch.empty((H, W), dtype=torch.int16, device=dev)
    warm_iters = list(schedule) + [0]
    ws = torch.empty(B.bp_workspace_bytes(W, H, B.make_params(D, L, its, lam, T)), dtype=torch.uint8, device=dev)
    lay = WS.Layout(D)
    params = lay.init_params(1)
    w16 = WS.to_bf16(params)
    x = WS.warmstart_input(left, right, B.stereo_cost_volume(left, right, D, win), L, warm_iters, lam, T)
    Hs, Ws_, _ = x.shape
    cnn_ws = WS.workspace(Ws_, Hs, D)
    y = torch.empty((Hs, Ws_, lay.layers[-1]["cout_p"]), dtype=torch.float32, device=dev)
    msgs = torch.empty((4, Hs, Ws_, D), dtype=torch.int16, device=dev)

    def plain():
        B.stereo_cost_volume(left, right, D, win, out=cost)
        B.bp_hierarchical_solve(cost, L, [its] * L, lam, T, 0, 2, workspace=ws, disparity=disp)

    def one_call():
        B.stereo_cost_volume(left, right, D, win, out=cost)
        WS.warmstart_solve(left, right, cost, L, warm_iters, lam, T, params, w16, 0, workspace=ws, disparity=disp)

    def layers():
        B.stereo_cost_volume(left, right, D, win, out=cost)
        WS.warmstart_input(left, right, cost, L, warm_iters, lam, T, workspace=ws, out=x)
        WS.forward(x, lay, params, w16, cnn_ws, y=y)
        WS.warmstart_messages(y, D, lam, T, out=msgs)
        B.bp_hierarchical_solve(cost, L, warm_iters, lam, T, 0, 2, warm_msgs=msgs, workspace=ws, disparity=disp)

    def timed(f):
        for _ in range(args.warmup):
            f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    t_one, t_layers, t_plain = timed(one_call), timed(layers), timed(plain)
    return {
        "metric": METRIC, "value": 1.0 / t_one, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_one * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int16+bf16", "data": "synthetic",
        "config": {"workload": f"warm: {W}x{H} grey pair, D={D}, {win}x{win} NCC, {L} scales; the network's "
                               f"messages start scale {L - 2}, half-steps {list(schedule)} at scales 0..{L - 2}; "
                               "network as one launch inside the solve; eager launches, cost volume + solve"},
        "layer_path_pairs_per_s": 1.0 / t_layers, "plain_pairs_per_s": 1.0 / t_plain,
        "plain_config": f"{L} scales x {its} half-steps, plain BP",
        "network_note": "freshly initialised weights: timing only",
    }


def time_vs_halfsteps(B, cost, ws, w, stream, counts=(2, 4, 6, 8, 10, 12), reps=5):
    """Run time of the solve against the number of half-steps per scale (the paper's claim:
    plain BP's time is linear in its iterations), for plain BP and the freeze rule: the
    median device time of `reps` solves at each count, and a least-squares line for plain
    BP with its R^2.  Every scale runs the same count.  (Below two half-steps a scale's
    initial messages are written by a separate pass, a different launch sequence, so the
    line starts at two.)"""
    import numpy as np
    import torch

    D, L, lam, T = w["num_disp"], w["num_scales"], w["lam"], w["trunc"]
    H, W = cost.shape[0], cost.shape[1]
    disp = torch.empty((H, W), dtype=torch.int16, device=cost.device)
    res = {"halfsteps_per_scale": list(counts)}
    for name, skip in (("plain", 0), ("freeze", 1)):
        ms = []
        for n in counts:
            its = [n] * L
            B.bp_hierarchical_solve(cost, L, its, lam, T, skip, 2, workspace=ws, disparity=disp, stream=stream)
            times = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                B.bp_hierarchical_solve(cost, L, its, lam, T, skip, 2, workspace=ws, disparity=disp, stream=stream)
                e1.record(stream)
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
            ms.append(float(np.median(times)))
        res[f"{name}_ms"] = ms
    x = np.array(counts, np.float64)
    y = np.array(res["plain_ms"])
    slope, icpt = np.polyfit(x, y, 1)
    pred = slope * x + icpt
    res["plain_fit"] = {"slope_ms_per_halfstep": float(slope), "intercept_ms": float(icpt),
                        "r2": float(1.0 - np.sum((y - pred) ** 2) / np.sum((y - y.mean()) ** 2))}
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        print(json.dumps(run_batched(args)))
        return
    if args.workload == "jacobi":
        print(json.dumps(run_jacobi(args)))
        return
    if args.workload == "live":
        print(json.dumps(run_live(args)))
        return
    if args.workload == "warm":
        print(json.dumps(run_warm(args)))
        return
    import numpy as np
    import torch

    from paper_1709_06509_amd import bpstereo as B
    from paper_1709_06509_amd import synth

    w = dict(synth.WORKLOADS[args.workload])
    w["name"] = args.workload
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    p = synth.workload_pair(args.workload)
    D, L, iters = w["num_disp"], w["num_scales"], [w["iters"]] * w["num_scales"]
    H, W = w["height"], w["width"]
    rgb = w["rgb"]
    left = torch.from_numpy(p["left"]).to(dev)
    right = torch.from_numpy(p["right"]).to(dev)
    gl = torch.empty((H, W), dtype=torch.uint8, device=dev)
    gr = torch.empty((H, W), dtype=torch.uint8, device=dev)
    cost = torch.empty((H, W, D), dtype=torch.int16, device=dev)
    disp = torch.empty((H, W), dtype=torch.int16, device=dev)
    energy = torch.empty(1, dtype=torch.int64, device=dev)
    params = B.make_params(D, L, iters, w["lam"], w["trunc"], w["skip"], 2)
    ws = torch.empty(B.bp_workspace_bytes(W, H, params), dtype=torch.uint8, device=dev)
    ews = torch.empty(B.bp_energy_workspace_bytes(W, H), dtype=torch.uint8, device=dev)
    ctx = B.Context()

    def step(skip=w["skip"], wsp=ws):
        if rgb:
            B.stereo_luma(left, gl)
            B.stereo_luma(right, gr)
            a, b = gl, gr
        else:
            a, b = left, right
        B.stereo_cost_volume(a, b, D, w["window"], w["cost_scale"], w["cost_trunc"], out=cost)
        B.bp_hierarchical_solve(cost, L, iters, w["lam"], w["trunc"], skip, 2, ctx=ctx, workspace=wsp,
                                disparity=disp)
        B.bp_energy(cost, disp, w["lam"], w["trunc"], workspace=ews, out=energy)

    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # The timed region launches every kernel of each step eagerly on one stream (the host
        # stays ahead of the GPU), with the context's timing mode on: a HIP event pair on the
        # launch stream around each scale's run of message-update launches, so the roofline
        # below comes from the very launches the headline times.  (An event pair around every
        # launch costs about 5 % of the step on this stack; five pairs a step cost about 0.5 %.)
        ctx.set_timing(2)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        timing = ctx.take_timing()
        ctx.set_timing(False)
        n_timed = args.steps
        # for the record: the same steps without events, and replayed as one HIP graph
        reps = 0 if args.no_extras else max(1, min(args.steps, 50))
        no_event_elapsed = graph_elapsed = scaling = freeze_elapsed = None
        if reps:
            t0 = time.perf_counter()
            for _ in range(reps):
                step()
            torch.cuda.synchronize()
            no_event_elapsed = (time.perf_counter() - t0) / reps
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                step()
            for _ in range(3):
                graph.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                graph.replay()
            torch.cuda.synchronize()
            graph_elapsed = (time.perf_counter() - t0) / reps
            del graph
            scaling = time_vs_halfsteps(B, cost, ws, w, stream)
            # the same whole step under the paper's fast-converging rule (freeze rule, K = 2)
            if w["skip"] != 1:
                ws_frz = torch.empty(B.bp_workspace_bytes(W, H, B.make_params(D, L, iters, w["lam"], w["trunc"], 1, 2)),
                                     dtype=torch.uint8, device=dev)
                for _ in range(3):
                    step(1, ws_frz)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    step(1, ws_frz)
                torch.cuda.synchronize()
                freeze_elapsed = (time.perf_counter() - t0) / reps
                del ws_frz

    # counters and energies (outside the timed region; the solve is deterministic)
    _, _, st = B.bp_hierarchical_solve(cost, L, iters, w["lam"], w["trunc"], w["skip"], 2, want_stats=True)
    e_run = int(B.bp_energy(cost, disp, w["lam"], w["trunc"]).cpu()[0])
    d_plain, _, st_plain = B.bp_hierarchical_solve(cost, L, iters, w["lam"], w["trunc"], 0, 2, want_stats=True)
    e_plain = int(B.bp_energy(cost, d_plain, w["lam"], w["trunc"]).cpu()[0])
    d_frz, _, st_frz = B.bp_hierarchical_solve(cost, L, iters, w["lam"], w["trunc"], 1, 2, want_stats=True)
    e_frz = int(B.bp_energy(cost, d_frz, w["lam"], w["trunc"]).cpu()[0])

    ms_per_step = 1000.0 * elapsed / args.steps
    pairs_per_s = args.steps / elapsed
    msg_bits = B.bp_message_bits(W, H, B.make_params(D, L, iters, w["lam"], w["trunc"], w["skip"]))
    hs_bytes = halfstep_bytes(st, D, L, w["skip"], msg_bits)
    n_launch = timing["halfstep_launches"] // n_timed if n_timed else 0
    avg_launch_s = timing["halfstep_ms"] / 1000.0 / max(1, timing["halfstep_launches"])
    halfstep_ms_per_step = timing["halfstep_ms"] / max(1, n_timed)
    if halfstep_ms_per_step > ms_per_step:
        raise RuntimeError(f"half-step time {halfstep_ms_per_step:.3f} ms exceeds the step {ms_per_step:.3f} ms")
    bytes_per_launch = hs_bytes / max(1, n_launch)
    achieved = bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    traffic = measured_traffic(args.workload)  # profiler-measured HBM bytes per launch, or None
    # pixels of each colour at the finest scale: the freeze rule's active fraction per half-step
    n0 = (W * H + 1) // 2
    frz_active = [st_frz["active"][0][t] / (n0 if t % 2 == 0 else W * H - n0) for t in range(min(iters[0], 64))]
    out = {
        "metric": METRIC,
        "value": pairs_per_s,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} {W}x{H}{' RGB->luma' if rgb else ''} D={D}, "
                               f"{w['window']}x{w['window']} NCC, {L} scales x {w['iters']} half-steps, "
                               f"lambda={w['lam']} T={w['trunc']}, skip={w['skip']} (K=2), seed={w['seed']}",
                   "pairs_per_step": 1},
        "gmsg_updates_per_s": st["msg_updates"] * pairs_per_s / 1e9,
        "effective_gmsg_updates_per_s": st_plain["msg_updates"] * pairs_per_s / 1e9,
        "energy": e_run,
        "energy_plain": e_plain,
        "energy_ratio_vs_plain": e_run / e_plain if e_plain else None,
        "msg_updates_per_pair": st["msg_updates"],
        "msg_updates_per_pair_plain": st_plain["msg_updates"],
        "roofline": {
            "bound": "hbm",
            "kernel": "message-update launches of all scales: k_halfstep (one half-step) and k_fused (several "
                      "half-steps of a small scale from LDS)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_gbs": traffic / avg_launch_s / 1e9 if traffic and avg_launch_s > 0 else None,
            "avg_launch_us": avg_launch_s * 1e6,
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "message_bits": msg_bits,
            "launches_per_step": n_launch,
        },
        "halfstep_ms_per_step": halfstep_ms_per_step,
        "halfstep_ms_per_scale": [timing["scale_ms"][l] / max(1, n_timed) for l in range(L)],
        "halfstep_launches_per_scale": [timing["scale_launches"][l] // max(1, n_timed) for l in range(L)],
        "pairs_per_s_without_events": 1.0 / no_event_elapsed if no_event_elapsed else None,
        "graph_replay_pairs_per_s": 1.0 / graph_elapsed if graph_elapsed else None,
        "time_vs_halfsteps": scaling,
        "freeze_rule": {"energy_ratio_vs_plain": e_frz / e_plain if e_plain else None,
                        "msg_updates_per_pair": st_frz["msg_updates"],
                        "active_fraction_finest": frz_active,
                        "pairs_per_s": 1.0 / freeze_elapsed if freeze_elapsed else None,
                        "speedup_vs_plain_without_events": (no_event_elapsed / freeze_elapsed
                                                            if freeze_elapsed and no_event_elapsed else None)},
        "timing_note": "value: the whole step launched eagerly, steps back to back, with a HIP event pair on the "
                       "launch stream around each scale's run of message-update launches (the roofline's average "
                       "launch duration is their summed time over the launch count); pairs_per_s_without_events "
                       "and graph_replay_pairs_per_s: the same steps without the events and as one replayed HIP graph",
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
