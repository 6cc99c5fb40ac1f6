"""Writes tests/golden/oracle_small_solve.json: a regression anchor for the FP64
oracle (not a pin: the paper prints no worked example for this path).

The input is built with exactly rounded operations only (integer textures from
numpy's PCG64, integer box sums, one division, integer shifts), so it is the
same on every x86-64 host; the script calls nothing but oracle/ on it.  Run it
again (python tests/golden/make_oracle_golden.py) only when the oracle's
arithmetic changes on purpose, and say which reading justifies the change.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

W, H = 56, 40
PARAMS = dict(C=5, r=2, blocks=(16,), iters=3, hyps=32, tau=1.0, eps=0.1, tau_fb=1.0, seed=9)
# one level; two levels (windows 24 and 12, so the second level's merge, its
# restricted pass and the label carried over from the first all take part),
# with the default merge key and with the strict level priority
CASES = {
    "one_level": PARAMS,
    "two_levels": dict(PARAMS, blocks=(24, 12)),
    "two_levels_strict": dict(PARAMS, blocks=(24, 12), merge_strict=True),
}


def _texture(rng, h, w, k=5):
    raw = rng.integers(0, 256, (h + k - 1, w + k - 1, 3)).astype(np.int64)
    c = np.cumsum(np.cumsum(raw, axis=0), axis=1)
    c = np.pad(c, ((1, 0), (1, 0), (0, 0)))
    box = c[k:, k:] - c[:-k, k:] - c[k:, :-k] + c[:-k, :-k]
    return box.astype(np.float64) / float(255 * k * k)


def frames():
    """Background shifted by (+3, +1), a 16x14 foreground block shifted by (-2, +2)."""
    rng = np.random.default_rng(20260)
    bg = _texture(rng, H + 16, W + 16)
    fg = _texture(rng, H + 16, W + 16)
    f1 = bg[8:8 + H, 8:8 + W].copy()
    f2 = bg[8 - 1:8 - 1 + H, 8 - 3:8 - 3 + W].copy()   # frame2(x + 3, y + 1) = frame1(x, y)
    y0, x0 = 12, 20
    f1[y0:y0 + 14, x0:x0 + 16] = fg[y0:y0 + 14, x0:x0 + 16]
    f2[y0 + 2:y0 + 16, x0 - 2:x0 + 14] = fg[y0:y0 + 14, x0:x0 + 16]
    return f1.astype(np.float32), f2.astype(np.float32)


def summary():
    return {name: case_summary(p) for name, p in CASES.items()}


def case_summary(params):
    import oracle
    f1, f2 = frames()
    o = oracle.Oracle(f1, f2, **params)
    flows, occs = o.solve()
    digest = lambda a: hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
    valid = o.pinfo[:, oracle.PI["valid"]]
    return {
        "frames_sha256": [digest(f1), digest(f2)],
        "flow_sha256": [digest(flows[d]) for d in range(2)],
        "occ_sha256": [digest(occs[d]) for d in range(2)],
        "planes_sha256": digest(o.pH) + ":" + digest(o.pinfo),
        "occluded": [int(occs[d].sum()) for d in range(2)],
        "valid_planes": int(valid.sum()),
        "params": {k: (list(v) if isinstance(v, tuple) else v) for k, v in params.items()},
        "size": [W, H],
    }


if __name__ == "__main__":
    out = os.path.join(HERE, "oracle_small_solve.json")
    with open(out, "w") as f:
        json.dump(summary(), f, indent=1, sort_keys=True)
        f.write("\n")
    print(open(out).read())
