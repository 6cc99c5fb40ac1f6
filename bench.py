#!/usr/bin/env python3
"""Throughput of the MSGPM hot path on one MI355X.

One step = one whole pipeline run (libmsgpm msgpm_solve) over a frame pair
already resident in HBM: features, random initial NNF, PatchMatch initial
pass, three plane-fit levels (two RANSAC stages, assignment, plane symmetry,
forward-backward check, NNF update, restricted PatchMatch pass) and the
outputs (flow, occlusion mask, plane table) of both directions.

Workload: a synthetic 1024x436 piecewise-planar pair (seed 0) standing in for
the MPI-Sintel frames of the paper's experiments; 9x9 patches over RGB + luma
gradients, windows 64/32/16, 8 PatchMatch iterations per pass, 256 RANSAC
hypotheses per window, FP32 patch costs, FP64 plane fits.

Prints one JSON line: flow Mpix/s of the timed steps (each step one launch of
the pipeline captured as a HIP graph, msgpm_solve_graph; --no-graph: eager
launches); per PatchMatch kernel (identity patches of the initial pass and of
the restricted passes, distorted patches) its own time (an equal number of
eager steps with the restricted launches in sequence on one stream, HIP events
around each launch) against the chip's FP32 ALU, HBM and LDS peaks and against
the measured gather ceiling of its access pattern (libmsgpm_ceiling); the
dominant kernel's entry as the roofline; and the FP64 CPU oracle (its OpenMP
build, all of this host's cores) timed on the same 1024x436 pair.

Other workloads: --fp16 (FP16 feature storage), --cues (occlusion cues 2 and
3 on), --fill N (N half-sweeps of filling by model propagation), --histeq
(HSV value equalisation of the frames), --strict (strict level priority),
--independent (every quad moving on its own by up to 100 px), --seed,
--batched (uneven
pairs per msgpm_solve_batch), --serving (Poisson arrivals, continuous
batching).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

W, H = 1024, 436
PARAMS = dict(C=5, r=4, blocks=(64, 32, 16), iters=8, hyps=256, tau=1.0, eps=0.1, tau_fb=1.0, seed=0)
# MI355X peaks: vector FP32 with packed (dual-issue) FMA 157.3 TFLOP/s (256 CU x
# 2.4 GHz x 256 flop/clk); without packing 78.6 (the kernels are built without
# packed FP32 instructions); HBM3E 8 TB/s; LDS 160 KB per CU at 128 B/clk
# (256 x 2.4 GHz x 128 B = 78.6 TB/s).
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PEAK_LDS_GBS = 78643.2

# Bytes beyond L2 per launch of each PatchMatch kernel on the 1024x436 workload,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch, scaled by 2.0 and
# 1.0: what the counters read for a plain 256 MiB copy), averaged over the
# dispatches of one pipeline run (identity: the initial pass's and the
# restricted ones'); keyed by storage.  None where not measured for the
# kernels as they are now.
TRAFFIC = {
    # profiles/k_pm_halfsweep_1024x436_traffic.md
    ("k_pm_halfsweep (identity patches, initial pass)", False): 1.9691e9,
    ("k_pm_halfsweep (identity patches, restricted)", False): 4.9611e8,
    ("k_pm_halfsweep (distorted patches)", False): 3.3862e8,
    ("k_pm_halfsweep (identity patches, initial pass)", True): 5.9985e8,
    ("k_pm_halfsweep (identity patches, restricted)", True): 1.9960e8,
    ("k_pm_halfsweep (distorted patches)", True): 1.5155e8,
}


def gather_ceiling(W: int, H: int, r: int, record_words: int, bilinear: bool, patches: int = 15,
                   reps: int = 5) -> float:
    """Patches per second of libmsgpm_ceiling's gather kernel: the PatchMatch
    kernels' gathers (lane groups per pixel of one colour, each gathering the
    patches of a candidate stream of 4 propagations and one target per search
    radius) with none of their arithmetic, on a W x H frame of records of
    record_words words; the best of `reps` launches."""
    import ctypes

    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1804_03787_amd", "libmsgpm_ceiling.so"))
    lib.msgpm_ceiling_blocks.argtypes = [ctypes.c_int] * 3
    lib.msgpm_ceiling_gather.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_void_p, ctypes.c_void_p]
    nb = lib.msgpm_ceiling_blocks(W, H, r)
    if nb <= 0:
        raise RuntimeError("gather ceiling: frame size or radius out of range")
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    feat = torch.rand((W * H + 1) * record_words, device="cuda", generator=g)
    sink = torch.empty(nb * 256, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    best = None
    for k in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        st = lib.msgpm_ceiling_gather(ctypes.c_void_p(feat.data_ptr()), W, H, record_words, r, int(bilinear),
                                      patches, 1234 + k, ctypes.c_void_p(sink.data_ptr()), stream)
        b.record()
        if st != 0:
            raise RuntimeError(f"gather ceiling launch failed ({st})")
        b.synchronize()
        if k:  # the first launch warms up
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
    groups = ((W + 1) // 2) * H
    return groups * patches / (best * 1e-3)


def flops_per_eval(kind: str, r: int, C: int) -> int:
    """Algorithmic FP32 flops of one patch-cost evaluation (FMA = 2).
    Identity patch: per tap and channel a difference and a multiply-add (3),
    gradient channels one more multiply for their weight.  Distorted patch:
    each value is bilinear (3 lerps = 3 x (sub + FMA) = 9 flops) before that."""
    taps = (2 * r + 1) ** 2
    extra = 2 if C == 5 else 0
    if kind == "identity":
        return taps * (3 * C + extra)
    return taps * (12 * C + extra)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cues: bool = False, fill: int = 0, histeq: bool = False, full: bool = True,
                 seed: int = 0, fp16: bool = False, strict: bool = False, independent: bool = False) -> dict:
    """The FP64 oracle over the whole pipeline, both directions, in its OpenMP
    build (the phase loops shared among all the host's cores; the same bits as
    the single-threaded build).  full: the 1024x436 pair itself (about 30 s
    with 16 threads); otherwise a 512x218 instance of the 1024x436 scene
    generator (lengths x1/2) with the same method parameters and a first
    random-search radius of 1024, as in the full workload, so that a pixel does
    the same work."""
    import oracle
    from paper_1804_03787_amd import synth
    sw, sh = (W, H) if full else (W // 2, H // 2)
    pair = synth.planar_pair(sw, sh, seed=seed, scale=sw / W, independent=independent)
    cores = oracle.set_threads(os.cpu_count() or 1)
    o = oracle.Oracle(pair.frame1, pair.frame2, variant="omp", R0=max(W, H),
                      **dict(PARAMS, cue_overlap=cues, cue_unique=cues, fill_sweeps=fill, histeq=histeq, fp16=fp16,
                             merge_strict=strict))
    t0 = time.perf_counter()
    o.solve()
    dt = time.perf_counter() - t0
    what = "the 1024x436 pair itself" if full else f"a {sw}x{sh} instance of the 1024x436 scene generator (lengths x1/2)"
    return {"value": round(sw * sh / dt / 1e6, 6), "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "sample": f"whole pipeline, both directions, on {what}, same parameters, R0=1024; {dt:.1f} s with "
                      f"{cores} threads (OpenMP build of the FP64 oracle) on {_cpu_model()}"}


BATCH_SIZES = [(320, 240), (640, 360), (1024, 436), (1280, 544)]


def _batch_pair(i: int):
    """Pair i of the batched workload: size uniform over BATCH_SIZES, 12-30
    quads, displacements up to about 120 px (camera translation up to 40 px at
    1024 width, lengths scaled with the width), occlusion by foreground quads
    targeted uniformly in 3-8 %; scene seed 1000 + i."""
    import numpy as np

    from paper_1804_03787_amd import synth
    rng = np.random.default_rng(1000 + i)
    W, H = BATCH_SIZES[int(rng.integers(len(BATCH_SIZES)))]
    occ = float(rng.uniform(0.03, 0.08))
    pr = synth.planar_pair(W, H, seed=1000 + i, n_quads=int(rng.integers(12, 31)), cam_t=40.0,
                           fg_occ=(occ - 0.005, occ + 0.005), scale=W / 1024)
    return W, H, pr.frame1, pr.frame2


def run_batched(args) -> int:
    """Batched workload: n pairs of uneven sizes in one msgpm_solve_batch per
    step (FP16 feature storage), against the same pairs solved one at a time in
    the FP16 and the plain FP32 forms."""
    import multiprocessing as mp

    # scenes first, in worker processes started before this process touches the GPU
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
        scenes = pool.map(_batch_pair, range(args.pairs))
    print(f"bench: {args.pairs} scenes generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    import torch

    from paper_1804_03787_amd import msgpm
    msgpm.lib()
    full = dict(C=5, r=4, blocks=(64, 32, 16), iters=8, hyps=256, tau=1.0, eps=0.1, tau_fb=1.0)
    f1 = [torch.from_numpy(a).cuda() for _, _, a, _ in scenes]
    f2 = [torch.from_numpy(b).cuda() for _, _, _, b in scenes]
    mpix = sum(W * H for W, H, _, _ in scenes) / 1e6

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / args.steps

    if args.tuning:
        msgpm.tuning_set(r=4, C=5, fp16=True, **json.loads(args.tuning))
    pairs16 = [msgpm.Pair(W, H, **dict(full, seed=1000 + i, fp16=True)) for i, (W, H, _, _) in enumerate(scenes)]
    batch = msgpm.Batch(pairs16)
    t_eager = timed(lambda: batch.solve(f1, f2))
    t_batch = timed(lambda: batch.solve(f1, f2, graph=True))
    print(f"bench: batched {t_eager * 1e3:.1f} ms eager, {t_batch * 1e3:.1f} ms as one graph launch "
          f"(tuning {msgpm.tuning_get(4, 5, True)})", file=sys.stderr, flush=True)
    if args.batched_only:
        print(json.dumps({"metric": "flow Mpix/s (batched)", "value": round(mpix / t_batch, 4), "unit": "Mpix/s",
                          "eager_mpix_s": round(mpix / t_eager, 4), "tuning": msgpm.tuning_get(4, 5, True)}))
        return 0
    t_one16 = timed(lambda: [g.solve(a, b) for g, a, b in zip(pairs16, f1, f2)])
    del batch, pairs16
    pairs32 = [msgpm.Pair(W, H, **dict(full, seed=1000 + i)) for i, (W, H, _, _) in enumerate(scenes)]
    t_one32 = timed(lambda: [g.solve(a, b) for g, a, b in zip(pairs32, f1, f2)])
    line = {
        "metric": "flow Mpix/s (batched, sum of W*H / makespan)",
        "value": round(mpix / t_batch, 4),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_batch * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32",
        "data": "synthetic",
        "config": {"workload": f"{args.pairs} pairs, sizes uniform over 320x240/640x360/1024x436/1280x544, "
                               "12-30 quads, 3-8% occlusion, patch 9x9, C=5, windows 64/32/16, 8 PM iterations, "
                               "256 RANSAC hypotheses, FP16 feature storage",
                   "pairs": args.pairs, "mpix_per_step": round(mpix, 4)},
        "launch": "one HIP graph per step (msgpm_solve_batch_graph), persistent kernels",
        "eager_mpix_s": round(mpix / t_eager, 4),
        "tuning_wg_per_cu": msgpm.tuning_get(4, 5, True),
        "one_at_a_time_fp16_mpix_s": round(mpix / t_one16, 4),
        "one_at_a_time_fp32_mpix_s": round(mpix / t_one32, 4),
        "speedup_vs_fp32_one_at_a_time": round(t_one32 / t_batch, 3),
    }
    print(json.dumps(line))
    return 0


SERVE_SIZES = [((1024, 436), 0.5, (64, 32, 16)), ((640, 360), 0.3, (64, 32, 16)),
               ((2048, 872), 0.2, (128, 64, 32, 16))]
SERVE_SCENES = [6, 4, 3]  # distinct scenes per size class


def _serve_scene(job):
    """Scene j of size class c of the serving workload (seed 2000 + 100 c + j)."""
    from paper_1804_03787_amd import synth
    c, j = job
    (W, H), _, _ = SERVE_SIZES[c]
    pr = synth.planar_pair(W, H, seed=2000 + 100 * c + j, scale=W / 1024)
    return c, j, pr.frame1, pr.frame2


def run_serving(args) -> int:
    """Serving workload: Poisson arrivals, sizes 50 % 1024x436, 30 % 640x360,
    20 % 2048x872 (4 window scales), FP16 feature storage, continuous batching
    (msgpm_server_*).  First the capacity (every request submitted at once),
    then the arrival trace at --rate and at 60 % of the capacity, then the
    same trace served one pair at a time in the plain FP32 form.  Frames come
    from a pool of distinct scenes per size class (every request is solved in
    full; nothing is cached between requests)."""
    import multiprocessing as mp

    import numpy as np
    t0 = time.perf_counter()
    jobs = [(c, j) for c, k in enumerate(SERVE_SCENES) for j in range(k)]
    with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
        scenes = pool.map(_serve_scene, jobs)
    print(f"bench: {len(scenes)} scenes generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    import torch

    from paper_1804_03787_amd import msgpm
    msgpm.lib()
    frames = {(c, j): (torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for c, j, a, b in scenes}
    full = dict(C=5, r=4, iters=8, hyps=256, tau=1.0, eps=0.1, tau_fb=1.0)

    def trace(rate, duration, seed):
        rng = np.random.default_rng(seed)
        t, out = 0.0, []
        while True:
            t += rng.exponential(1.0 / rate)
            if t > duration:
                return out
            c = int(rng.choice(len(SERVE_SIZES), p=[w for _, w, _ in SERVE_SIZES]))
            out.append((t, c, int(rng.integers(SERVE_SCENES[c]))))

    def make_pair(c, fp16):
        (W, H), _, blocks = SERVE_SIZES[c]
        return msgpm.Pair(W, H, **dict(full, blocks=blocks, fp16=fp16))

    def serve(reqs, max_active=64, budget=200 << 30):
        """Returns (latencies in s, makespan in s, Mpix)."""
        srv = msgpm.Server(budget, max_active)
        srv.set_cohorts(args.cohorts)
        lat, out, cls = [], {}, []
        mpix = sum(SERVE_SIZES[c][0][0] * SERVE_SIZES[c][0][1] for _, c, _ in reqs) / 1e6
        torch.cuda.synchronize()
        start = time.perf_counter()
        k = 0
        shown = start
        while k < len(reqs) or out:
            now = time.perf_counter() - start
            if time.perf_counter() - shown > 20.0:
                shown = time.perf_counter()
                print(f"bench: serving {now:.0f} s: {k} of {len(reqs)} submitted, {len(lat)} done",
                      file=sys.stderr, flush=True)
            while k < len(reqs) and reqs[k][0] <= now:
                t, c, j = reqs[k]
                a, b = frames[(c, j)]
                out[srv.submit(make_pair(c, True), a, b)] = (t, c)
                k += 1
            if out:
                srv.step()
                now = time.perf_counter() - start
                for tk in [tk for tk in out if srv.poll(tk)]:
                    t0, c0 = out.pop(tk)
                    lat.append(now - t0)
                    cls.append(c0)
                    srv.result(tk)
            elif k < len(reqs):
                time.sleep(max(0.0, reqs[k][0] - (time.perf_counter() - start)))
        span = time.perf_counter() - start
        srv.close()
        return np.array(lat), span, mpix, np.array(cls)

    def one_at_a_time(reqs):
        pairs = {c: make_pair(c, False) for c in range(len(SERVE_SIZES))}
        lat = []
        torch.cuda.synchronize()
        start = time.perf_counter()
        shown = start
        for t, c, j in reqs:
            now = time.perf_counter() - start
            if time.perf_counter() - shown > 20.0:
                shown = time.perf_counter()
                print(f"bench: one at a time {now:.0f} s: {len(lat)} of {len(reqs)} done", file=sys.stderr, flush=True)
            if now < t:
                time.sleep(t - now)
            a, b = frames[(c, j)]
            pairs[c].solve(a, b)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - start - t)
        return np.array(lat), time.perf_counter() - start, np.array([c for _, c, _ in reqs])

    def per_class(lat, cls):
        out = {}
        for c, ((W, H), _, _) in enumerate(SERVE_SIZES):
            sel = lat[cls == c]
            if len(sel):
                out[f"{W}x{H}"] = {"pairs": int(len(sel)), "p50_ms": round(float(np.median(sel)) * 1e3, 1),
                                   "p99_ms": round(float(np.quantile(sel, 0.99)) * 1e3, 1)}
        return out

    # capacity: every request of a trace submitted at time 0
    cap_reqs = [(0.0, c, j) for _, c, j in trace(args.rate, args.duration / 2, 4)]
    serve(cap_reqs[:8])  # warm-up
    _, span, mpix, _ = serve(cap_reqs)
    capacity = mpix / span
    print(f"bench: capacity {capacity:.2f} Mpix/s ({len(cap_reqs)} pairs in {span:.2f} s)", file=sys.stderr,
          flush=True)

    # the same requests as lock-step batches (msgpm_solve_batch_graph), one per
    # schedule (3-level and 4-level pairs), the second run timed
    groups = {}
    for _, c, j in cap_reqs:
        groups.setdefault(len(SERVE_SIZES[c][2]), []).append((c, j))
    batches = []
    for g in groups.values():
        b = msgpm.Batch([make_pair(c, True) for c, _ in g])
        batches.append((b, [frames[k][0] for k in g], [frames[k][1] for k in g]))
    span_b = 0.0
    for _ in range(2):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for b, a1, a2 in batches:
            b.solve(a1, a2, graph=True)
        torch.cuda.synchronize()
        span_b = time.perf_counter() - tb
    batched_same = mpix / span_b
    del batches
    print(f"bench: the same requests as lock-step batches {batched_same:.2f} Mpix/s", file=sys.stderr, flush=True)
    mean_mpix = sum(SERVE_SIZES[c][0][0] * SERVE_SIZES[c][0][1] * w for c, (_, w, _) in enumerate(SERVE_SIZES)) / 1e6
    runs = {}
    for label, rate in (("offered", args.rate), ("stable", 0.6 * capacity / mean_mpix)):
        reqs = trace(rate, args.duration, 4)
        lat, span, mpix, cls = serve(reqs)
        offered = rate * mean_mpix
        runs[label] = {"rate_pairs_s": round(rate, 2), "offered_mpix_s": round(offered, 2), "pairs": len(reqs),
                       "throughput_mpix_s": round(mpix / span, 3), "p50_ms": round(float(np.median(lat)) * 1e3, 1),
                       "p99_ms": round(float(np.quantile(lat, 0.99)) * 1e3, 1),
                       "queue_stable": bool(offered < capacity), "by_size": per_class(lat, cls)}
        print(f"bench: {label} {runs[label]}", file=sys.stderr, flush=True)
    reqs = trace(runs["stable"]["rate_pairs_s"], args.duration, 4)
    lat1, span1, cls1 = one_at_a_time(reqs)
    mpix1 = sum(SERVE_SIZES[c][0][0] * SERVE_SIZES[c][0][1] for _, c, _ in reqs) / 1e6
    runs["stable_one_at_a_time_fp32"] = {"throughput_mpix_s": round(mpix1 / span1, 3),
                                         "p50_ms": round(float(np.median(lat1)) * 1e3, 1),
                                         "p99_ms": round(float(np.quantile(lat1, 0.99)) * 1e3, 1),
                                         "by_size": per_class(lat1, cls1)}
    line = {
        "metric": "serving: flow Mpix/s and p50/p99 pair latency",
        "value": runs["stable"]["throughput_mpix_s"],
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16-storage/f32",
        "data": "synthetic",
        "config": {"workload": "Poisson arrivals; sizes 50% 1024x436, 30% 640x360, 20% 2048x872 (windows "
                               "128/64/32/16); patch 9x9, C=5, 8 PM iterations, 256 RANSAC hypotheses; FP16 "
                               "storage; continuous batching",
                   "duration_s": args.duration, "cohorts": args.cohorts},
        "capacity_mpix_s": round(capacity, 3),
        "batched_same_requests_mpix_s": round(batched_same, 3),
        "runs": runs,
    }
    print(json.dumps(line))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches only (default: the pipeline as one captured HIP graph per step, "
                         "plus an eager pass with HIP events around every launch for the per-kernel figures)")
    ap.add_argument("--fp16", action="store_true", help="FP16 feature storage (FP32 accumulation)")
    ap.add_argument("--two-streams", action="store_true",
                    help="restricted half-sweeps' two launches side by side on two streams (library default) "
                         "instead of in sequence on one")
    ap.add_argument("--seed", type=int, default=0, help="scene seed of the 1024x436 generator")
    ap.add_argument("--cues", action="store_true", help="occlusion cues 2 (uniqueness) and 3 (overlap) on")
    ap.add_argument("--fill", type=int, default=0, help="half-sweeps of filling by model propagation (0 = none)")
    ap.add_argument("--histeq", action="store_true", help="equalise the frames' HSV value channel first")
    ap.add_argument("--strict", action="store_true", help="strict level priority (MSGPM_FLAG_MERGE_STRICT)")
    ap.add_argument("--independent", action="store_true",
                    help="scene with every quad moving on its own (up to 100 px, scale 0.9-1.1, 10 degrees)")
    ap.add_argument("--cpu-sample", action="store_true",
                    help="time the CPU oracle on a 512x218 instance instead of the 1024x436 pair itself")
    ap.add_argument("--batched", action="store_true",
                    help="batched workload: --pairs pairs of uneven sizes per msgpm_solve_batch")
    ap.add_argument("--pairs", type=int, default=48)
    ap.add_argument("--tuning", type=str, default="", help="batched: JSON of wg_per_cu per class for r=4, C=5, FP16")
    ap.add_argument("--batched-only", action="store_true", help="batched: skip the one-at-a-time comparisons")
    ap.add_argument("--serving", action="store_true", help="serving workload: Poisson arrivals, continuous batching")
    ap.add_argument("--rate", type=float, default=40.0, help="serving: arrivals per second")
    ap.add_argument("--duration", type=float, default=10.0, help="serving: seconds of arrivals")
    ap.add_argument("--cohorts", type=int, default=4, help="serving: cohorts in flight at most (1..4)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the pipeline runs on one GPU; --gpus {args.gpus} is not supported "
              "(frame pairs are independent, so more GPUs would serve more pairs side by side)", file=sys.stderr)
        return 2
    if args.batched:
        return run_batched(args)
    if args.serving:
        return run_serving(args)

    import numpy as np
    import torch

    from paper_1804_03787_amd import msgpm, synth

    msgpm.lib()  # fails loudly if the HIP library is missing
    pair = synth.planar_pair(W, H, seed=args.seed, independent=args.independent)
    f1 = torch.from_numpy(pair.frame1).cuda()
    f2 = torch.from_numpy(pair.frame2).cuda()
    params = dict(PARAMS, fp16=args.fp16, cue_overlap=args.cues, cue_unique=args.cues, fill_sweeps=args.fill,
                  histeq=args.histeq, merge_strict=args.strict, one_stream=not args.two_streams)
    g = msgpm.Pair(W, H, **params)
    flows = [torch.empty((H, W, 2), dtype=torch.float32, device="cuda") for _ in range(2)]
    occs = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(2)]
    use_graph = not args.no_graph
    for _ in range(args.warmup):
        g.solve(f1, f2, out=(flows, occs))
        if use_graph:
            g.solve(f1, f2, out=(flows, occs), graph=True)
    torch.cuda.synchronize()
    print(f"bench: warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    msgpm.timing_enable(True)
    msgpm.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.solve(f1, f2, out=(flows, occs))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = msgpm.timing_read()
    msgpm.timing_enable(False)
    eager_ms = (t1 - t0) * 1e3 / args.steps
    ms_per_step = eager_ms
    if use_graph:
        # the timed steps: the same pipeline launched as one captured HIP graph each
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            g.solve(f1, f2, out=(flows, occs), graph=True)
        torch.cuda.synchronize()
        ms_per_step = (time.perf_counter() - tg) * 1e3 / args.steps
        print(f"bench: eager {eager_ms:.2f} ms/step, graph {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)
    print(f"bench: timed {args.steps} eager steps with per-launch events", file=sys.stderr, flush=True)

    value = W * H / (ms_per_step / 1e3) / 1e6

    # not the headline: the same steps with the frames coming from pinned host
    # memory and the flow and masks going back to it (PCIe included)
    f1h, f2h = torch.from_numpy(pair.frame1).pin_memory(), torch.from_numpy(pair.frame2).pin_memory()
    flows_h = [torch.empty((H, W, 2), dtype=torch.float32).pin_memory() for _ in range(2)]
    occs_h = [torch.empty((H, W), dtype=torch.uint8).pin_memory() for _ in range(2)]
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for _ in range(args.steps):
        f1.copy_(f1h, non_blocking=True)
        f2.copy_(f2h, non_blocking=True)
        g.solve(f1, f2, out=(flows, occs), graph=use_graph)
        for d in range(2):
            flows_h[d].copy_(flows[d], non_blocking=True)
            occs_h[d].copy_(occs[d], non_blocking=True)
    torch.cuda.synchronize()
    pcie_ms = (time.perf_counter() - tp) * 1e3 / args.steps
    print(f"bench: with host transfers {pcie_ms:.2f} ms/step", file=sys.stderr, flush=True)

    # evaluations of the last step (every step is identical: same inputs and seed);
    # a candidate rejected early by its partial sum counts for the rows it computed
    cnt = g.counters()
    taps_rows = 2 * PARAMS["r"] + 1
    ev = {k: sum(cnt[k]) for k in ("pm_init", "pm_restricted", "pm_restricted_ident", "eval_cost")}
    full = {k: sum(cnt[k + "_rows"]) / taps_rows for k in ("pm_init", "pm_restricted", "pm_restricted_ident")}
    occ0 = (occs[0] != 0).float().mean().item()  # no plane of its own (filled pixels included)
    filled0 = (occs[0] == 2).float().mean().item()
    kernel_ms = {k: v[0] / args.steps for k, v in timing.items()}
    launches = {k: v[1] / args.steps for k, v in timing.items()}
    r, C = params["r"], params["C"]

    # each PatchMatch kernel on its own: by default the restricted half-sweeps'
    # two launches run in sequence on one stream (MSGPM_FLAG_ONE_STREAM), so the
    # timed eager steps give each kernel's own time; with --two-streams they
    # run side by side there, and an equal number of one-stream steps is timed
    alone_ms, alone_n = kernel_ms, launches
    if args.two_streams:
        g1 = msgpm.Pair(W, H, **dict(params, one_stream=True))
        g1.solve(f1, f2)
        torch.cuda.synchronize()
        msgpm.timing_enable(True)
        msgpm.timing_read()
        for _ in range(args.steps):
            g1.solve(f1, f2)
        torch.cuda.synchronize()
        alone = msgpm.timing_read()
        msgpm.timing_enable(False)
        del g1
        alone_ms = {k: v[0] / args.steps for k, v in alone.items()}
        alone_n = {k: v[1] / args.steps for k, v in alone.items()}
        print("bench: timed the steps with one stream", file=sys.stderr, flush=True)

    words = (3 if C == 5 else 2) if args.fp16 else C
    ceil_ident = gather_ceiling(W, H, r, words, False)
    ceil_bilin = gather_ceiling(W, H, r, words, True)
    print(f"bench: gather ceiling {ceil_ident / 1e9:.2f} G identity patches/s, {ceil_bilin / 1e9:.2f} G bilinear",
          file=sys.stderr, flush=True)

    # per kernel: tap rows computed (a candidate dropped by early rejection
    # counts the rows it gathered) as full-patch equivalents; flops of those
    # rows; bytes beyond L2 from the counters; LDS none (no kernel stages tiles)
    kernels = {}
    for name, kind, ck, ident, ceil in (
            ("k_pm_halfsweep (identity patches, initial pass)", "pm_init", "pm_init", True, ceil_ident),
            ("k_pm_halfsweep (identity patches, restricted)", "pm_restricted_ident", "pm_restricted_ident", True,
             ceil_ident),
            ("k_pm_halfsweep (distorted patches)", "pm_restricted", "pm_restricted", False, ceil_bilin)):
        ms, n = alone_ms.get(kind, 0.0), alone_n.get(kind, 0.0)
        if ms <= 0 or n <= 0:
            continue
        patches = full[ck]
        flops = patches * flops_per_eval("identity" if ident else "warped", r, C)
        tflops = flops / (ms * 1e-3) / 1e12
        # the counter figures are those of the default workload (scene seed 0, no options)
        default_workload = (args.seed == 0 and not (args.cues or args.fill or args.histeq or args.strict
                                                    or args.independent))
        traffic = TRAFFIC.get((name, bool(args.fp16))) if default_workload else None
        launch_s = ms * 1e-3 / n
        hbm_gbs = traffic / launch_s / 1e9 if traffic else None
        kernels[name] = {
            "ms_per_step": round(ms, 3), "launches_per_step": n, "avg_launch_us": round(launch_s * 1e6, 2),
            "evals_per_s": round(ev[ck] / (ms * 1e-3), 1),
            "full_patch_equiv_per_s": round(patches / (ms * 1e-3), 1),
            "gather_ceiling_patches_per_s": round(ceil, 1), "gather_frac": round(patches / (ms * 1e-3) / ceil, 4),
            "alu_tflops": round(tflops, 3), "alu_frac": round(tflops / PEAK_FP32_TFLOPS, 4),
            "alu_frac_nonpacked": round(tflops / PEAK_FP32_NONPACKED_TFLOPS, 4),
            "hbm_bytes_per_launch": traffic, "hbm_gbs": round(hbm_gbs, 1) if hbm_gbs else None,
            "hbm_frac": round(hbm_gbs / PEAK_HBM_GBS, 4) if hbm_gbs else None,
            "lds_bytes_per_launch": 0, "lds_frac": 0.0,
        }
    dominant = max(kernels, key=lambda k: kernels[k]["ms_per_step"]) if kernels else None
    roofline = None
    if dominant:
        k = kernels[dominant]
        roofline = {"bound": "alu", "achieved": k["alu_tflops"], "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                    "frac": k["alu_frac"], "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                    "frac_nonpacked": k["alu_frac_nonpacked"],
                    "traffic": k["hbm_bytes_per_launch"], "traffic_unit": "bytes per launch (beyond L2)",
                    "kernel": dominant, "ms_per_step": k["ms_per_step"], "avg_launch_us": k["avg_launch_us"],
                    "gather_frac": k["gather_frac"], "hbm_frac": k["hbm_frac"], "lds_frac": 0.0}
    warped = kernels.get("k_pm_halfsweep (distorted patches)")
    target = None
    if warped:
        best = max(warped["hbm_frac"] or 0.0, warped["lds_frac"])
        target = {"kernel": "k_pm_halfsweep (distorted patches)", "hbm_lds_frac": best, "target": 0.5,
                  "met": best >= 0.5, "gather_frac": warped["gather_frac"],
                  "note": "the warped-SSD kernel moves its bytes through L1/L2 gathers; beyond-L2 traffic is "
                          "the HBM figure, and it stages nothing in LDS"}

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args.cues, args.fill, args.histeq, full=not args.cpu_sample, seed=args.seed, fp16=args.fp16,
                           strict=args.strict, independent=args.independent)

    line = {
        "metric": "flow Mpix/s (full pipeline)",
        "value": round(value, 4),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if not args.fp16 else "f16-storage/f32",
        "data": "synthetic",
        "config": {"workload": "piecewise-planar pair 1024x436, fwd+bwd, patch 9x9, C=5, windows 64/32/16, "
                               "8 PM iterations, 256 RANSAC hypotheses",
                   "width": W, "height": H, "seed": args.seed, "fp16_storage": bool(args.fp16),
                   "occlusion_cues_2_3": bool(args.cues), "fill_sweeps": args.fill, "histeq": bool(args.histeq),
                   "merge_strict": bool(args.strict), "independent_quads": bool(args.independent),
                   "restricted_launches": "two streams" if args.two_streams else "one stream"},
        "patch_evals_per_s": round((ev["pm_init"] + ev["pm_restricted"] + ev["pm_restricted_ident"])
                                   / (ms_per_step * 1e-3), 1),
        # the initial pass alone: its evaluations over its kernel time, beside the
        # count without skipped duplicates (every pixel, 4 neighbours + every radius)
        "patch_evals_per_s_initial_pass": round(ev["pm_init"] / (kernel_ms["pm_init"] * 1e-3), 1)
        if kernel_ms.get("pm_init") else None,
        "evals_upper_bound_initial_pass": PARAMS["iters"] * W * H * 2 * (4 + (max(W, H)).bit_length()),
        "pcie_inclusive_ms_per_step": round(pcie_ms, 3),
        "pcie_inclusive_mpix_s": round(W * H / (pcie_ms / 1e3) / 1e6, 4),
        "evals_per_step": {**ev, **{k + "_full_equiv": round(v) for k, v in full.items()}},
        "kernel_ms_per_step": {k: round(v, 3) for k, v in kernel_ms.items()},
        "occluded_fraction_dir0": round(occ0, 4),
        "filled_fraction_dir0": round(filled0, 4),
        "launch": "hip graph per step" if use_graph else "eager",
        "eager_ms_per_step": round(eager_ms, 3),
        "roofline": roofline,
        "roofline_kernels": kernels,
        "warped_ssd_hbm_lds_target": target,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
