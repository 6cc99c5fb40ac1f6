"""Autotuner of the launch shape of the batched and served forms.

Their kernels are persistent: a launch runs wg_per_cu x (compute units)
resident workgroups that take the launch's work items (pixel tiles, windows)
in turn, per class of kernel (identity-patch PatchMatch, distorted-patch
PatchMatch, RANSAC, other per-pixel kernels).  The results do not depend on
the shape; the time does.  This script times the batched pipeline (one graph
launch per step, msgpm_solve_batch_graph) on a synthetic batch of uneven pairs
for candidate shapes, one class at a time (coordinate descent from the
library's defaults, twice over the classes), and stores the best shape per
kernel instantiation (patch radius, channel count, storage) in tuning.json
next to the library, where the Python binding installs it.

    python -m paper_1804_03787_amd.autotune [--pairs 16] [--steps 2]

Needs the GPU; run it after building the library.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SIZES = [(320, 240), (640, 360), (1024, 436), (1280, 544)]
FULL = dict(C=5, r=4, blocks=(64, 32, 16), iters=8, hyps=256, tau=1.0, eps=0.1, tau_fb=1.0)
# 0: one workgroup per work item (for the PatchMatch classes the kernel form
# without the persistent loop)
CANDIDATES = {
    "pm_identity": [0, 2, 3, 4, 6, 8, 16, 64],
    "pm_distorted": [0, 2, 3, 4, 6, 8, 16, 64],
    "ransac": [0, 1, 2, 3, 4, 8, 16],
    "pixel": [0, 2, 4, 8, 16, 32, 64],
}


def scenes(n: int, seed: int = 3000):
    from paper_1804_03787_amd import synth
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W, H = SIZES[int(rng.integers(len(SIZES)))]
        pr = synth.planar_pair(W, H, seed=seed + i, n_quads=int(rng.integers(12, 31)), scale=W / 1024)
        out.append((W, H, pr.frame1, pr.frame2))
    return out


def tune(batch, f1, f2, key: dict, steps: int, log) -> tuple:
    import torch

    from paper_1804_03787_amd import msgpm

    def measure(shape: dict) -> float:
        msgpm.tuning_set(**key, **shape)
        batch.solve(f1, f2, graph=True)  # captures the graph of this shape
        torch.cuda.synchronize()
        ts = []
        for _ in range(steps):
            t = time.perf_counter()
            batch.solve(f1, f2, graph=True)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)) * 1e3

    best = msgpm.tuning_get(**key)
    default_ms = best_ms = measure(best)
    log({"shape": dict(best), "ms": round(best_ms, 2), "note": "start"})
    for _ in range(2):
        for cls, values in CANDIDATES.items():
            for v in values:
                if v == best[cls]:
                    continue
                trial = dict(best, **{cls: v})
                ms = measure(trial)
                log({"shape": trial, "ms": round(ms, 2)})
                if ms < best_ms:
                    best, best_ms = trial, ms
    msgpm.tuning_set(**key, **best)
    return best, best_ms, default_ms


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--pairs", type=int, default=16)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    args = ap.parse_args()
    sc = scenes(args.pairs)
    import torch

    from paper_1804_03787_amd import msgpm
    msgpm.lib()
    f1 = [torch.from_numpy(a).cuda() for _, _, a, _ in sc]
    f2 = [torch.from_numpy(b).cuda() for _, _, _, b in sc]
    mpix = sum(W * H for W, H, _, _ in sc) / 1e6
    result = {"device": torch.cuda.get_device_name(0), "pairs": args.pairs, "mpix": round(mpix, 4),
              "workload": "uneven pairs over 320x240/640x360/1024x436/1280x544, patch 9x9, C=5, windows 64/32/16, "
                          "8 PM iterations, 256 RANSAC hypotheses; batched pipeline, one graph launch per step",
              "choices": {}, "trials": {}}
    for fp16 in (True, False):
        key = dict(r=FULL["r"], C=FULL["C"], fp16=fp16)
        name = msgpm.tuning_key(**key)
        pairs = [msgpm.Pair(W, H, **dict(FULL, seed=3000 + i, fp16=fp16)) for i, (W, H, _, _) in enumerate(sc)]
        batch = msgpm.Batch(pairs)
        trials = []

        def log(rec, name=name, trials=trials):
            trials.append(rec)
            print(f"autotune {name}: {rec}", flush=True)

        best, best_ms, default_ms = tune(batch, f1, f2, key, args.steps, log)
        result["choices"][name] = {"r": key["r"], "C": key["C"], "fp16": fp16, "wg_per_cu": best,
                                   "ms": round(best_ms, 2), "mpix_s": round(mpix / best_ms * 1e3, 3),
                                   "default_ms": round(default_ms, 2)}
        result["trials"][name] = trials
        del batch, pairs
        msgpm.graph_cache_clear()
    with open(args.out, "w") as f:
        json.dump(result, f, indent=1)
        f.write("\n")
    print(json.dumps(result["choices"]))
    return 0


if __name__ == "__main__":
    sys.exit(main())
