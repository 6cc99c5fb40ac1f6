"""Helpers that move state between the oracle and the GPU library and compare
them (test infrastructure)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from oracle import PI_FIELDS
from paper_1804_03787_amd import msgpm


def cost_tol(o_cost, r, C):
    """Tolerance of an FP32-accumulated patch cost against the FP64 value."""
    return 1e-5 * np.abs(o_cost) + 1e-7 * (2 * r + 1) ** 2 * C


def planes_to_gpu(o: oracle.Oracle) -> np.ndarray:
    arr = np.zeros(len(o.pinfo), msgpm.PLANE_DTYPE)
    arr["H"] = o.pH
    for i, f in enumerate(PI_FIELDS):
        arr[f] = o.pinfo[:, i]
    return arr


def push_state(o: oracle.Oracle, g: msgpm.Pair):
    dev = g.device
    for d in range(2):
        g.nnf(d).copy_(torch.from_numpy(o.nnf[d]).to(dev))
        g.cost(d).copy_(torch.from_numpy(o.cost[d].astype(np.float32)).to(dev))
        g.win(d).copy_(torch.from_numpy(o.win[d]).to(dev))
        g.loss(d).copy_(torch.from_numpy(o.loss[d]).to(dev))
        g.hlabel(d).copy_(torch.from_numpy(o.hlabel[d]).to(dev))
        g.twin(d).copy_(torch.from_numpy(o.twin[d]).to(dev))
        g.tloss(d).copy_(torch.from_numpy(o.tloss[d]).to(dev))
    g.set_planes(planes_to_gpu(o))
    torch.cuda.synchronize()


def poison_refresh(o: oracle.Oracle, g: msgpm.Pair, colour: int, mode: int) -> int:
    """After push_state: sets to zero, on the GPU, the costs that a cost refresh
    of `mode` (0: every pixel, 1: the unassigned ones) sets on the pixels of
    `colour`.  No candidate beats a zero cost, so a half-sweep that read them
    would keep every offset: a sweep with PM_FRESH must compute them itself.
    Returns the number of costs replaced."""
    H, W = o.Hh, o.Ww
    ys, xs = np.mgrid[0:H, 0:W]
    n = 0
    for d in range(2):
        sel = ((xs + ys) % 2).ravel() == colour
        if mode == 1:
            sel &= o.win[d] < 0
        c = o.cost[d].astype(np.float32)
        c[sel] = 0.0
        n += int(sel.sum())
        g.cost(d).copy_(torch.from_numpy(c).to(g.device))
    torch.cuda.synchronize()
    return n


def pull_state(g: msgpm.Pair) -> dict:
    torch.cuda.synchronize()
    s = {}
    for name in ("nnf", "cost", "win", "loss", "hlabel", "twin", "tloss"):
        s[name] = [getattr(g, name)(d).cpu().numpy().copy() for d in range(2)]
    s["planes"] = g.planes()
    return s


def compare_planes(o: oracle.Oracle, gp: np.ndarray, sel=None, exact=True):
    """Returns a list of mismatch descriptions (empty = identical)."""
    ref = planes_to_gpu(o)
    if sel is not None:
        ref, gp = ref[sel], gp[sel]
    bad = []
    for f in PI_FIELDS:
        m = ref[f] != gp[f]
        if m.any():
            bad.append(f"{f}: {int(m.sum())} differ, first at {int(np.nonzero(m)[0][0])}")
    if exact:
        m = ~np.all(ref["H"] == gp["H"], axis=1)
    else:
        num = np.linalg.norm(ref["H"] - gp["H"], axis=1)
        den = np.maximum(np.linalg.norm(ref["H"], axis=1), 1e-300)
        m = num > 1e-6 * den
    if m.any():
        bad.append(f"H: {int(m.sum())} differ, first at {int(np.nonzero(m)[0][0])}")
    return bad
