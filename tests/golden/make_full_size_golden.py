"""Writes tests/golden/oracle_1024x436_<case>.npz: whole oracle solves of the
1024x436 workload, for the free-running full-size parity test.

Cases: "fp32_seed0" (scene seed 0, FP32 features: the benchmark's pair) and
"fp16_seed1" (scene seed 1, features rounded to FP16, as the FP16-storage form
consumes them).  Both use 9x9 patches over RGB + luma gradients, windows
64/32/16, 8 PatchMatch iterations per pass, 256 RANSAC hypotheses, random
stream key 0.

The script calls nothing but oracle/ (its OpenMP build, which gives the
single-threaded build's bits) and the scene generator; a run takes a few
minutes on 8 cores.  Stored per direction: the flow (float32), the occlusion
mask, the final NNF, the per-pixel near-tie flags; plus the frames' SHA-256 so
that a test can tell that the generator reproduced the same input.  Run it
again (python tests/golden/make_full_size_golden.py [case ...]) only when the
oracle's arithmetic changes on purpose.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

W, H = 1024, 436
PARAMS = dict(C=5, r=4, blocks=(64, 32, 16), iters=8, hyps=256, tau=1.0, eps=0.1, tau_fb=1.0, seed=0)
CASES = {
    "fp32_seed0": dict(scene_seed=0, fp16=False),
    "fp16_seed1": dict(scene_seed=1, fp16=True),
}


def path(case: str) -> str:
    return os.path.join(HERE, f"oracle_1024x436_{case}.npz")


def frames(case: str):
    from paper_1804_03787_amd import synth
    pair = synth.planar_pair(W, H, seed=CASES[case]["scene_seed"])
    return pair


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def make(case: str) -> str:
    import oracle
    pair = frames(case)
    print(f"{case}: threads {oracle.set_threads(os.cpu_count() or 1)}", flush=True)
    o = oracle.Oracle(pair.frame1, pair.frame2, variant="omp", **dict(PARAMS, fp16=CASES[case]["fp16"]))
    t0 = time.perf_counter()
    flows, occs = o.solve()
    dt = time.perf_counter() - t0
    print(f"{case}: oracle solve {dt:.1f} s, {o.evals} evaluations", flush=True)
    out = path(case)
    np.savez_compressed(
        out, flow0=flows[0], flow1=flows[1], occ0=occs[0], occ1=occs[1], nnf0=o.nnf[0], nnf1=o.nnf[1],
        pflag0=o.pflag[0], pflag1=o.pflag[1], evals=np.int64(o.evals), seconds=np.float64(dt),
        frames_sha256=np.array([digest(pair.frame1), digest(pair.frame2)]))
    return out


if __name__ == "__main__":
    for case in (sys.argv[1:] or list(CASES)):
        print(make(case), os.path.getsize(path(case)), "bytes", flush=True)
