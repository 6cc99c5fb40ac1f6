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


# Near-tie flags of the oracle that excuse a different decision at a pixel:
# PatchMatch cost comparisons, rounding, colour threshold or loss argmin,
# forward-backward distance, image bounds.  TWO_BEST is the narrower PatchMatch
# rule (the two best costs over distinct targets within the band) in place of
# the running-best comparison.
PIXEL_FLAGS = oracle.F_COST | oracle.F_ROUND | oracle.F_COLOUR | oracle.F_FB | oracle.F_BOUNDS
TWO_BEST_FLAGS = oracle.F_TWOBEST | oracle.F_ROUND | oracle.F_COLOUR | oracle.F_FB | oracle.F_BOUNDS


def free_run_compare(nnf_o, occ_o, flow_o, pflag_o, nnf_g, occ_g, flow_g) -> dict:
    """One direction of a free-running solve against the oracle's.  Counts the
    pixels whose NNF offset or mask differ, how many of them the oracle flags
    as near-ties (under either rule), and the mean flow difference over the
    pixels assigned on both sides (EPE delta)."""
    nnf_o, nnf_g = nnf_o.reshape(-1), nnf_g.reshape(-1)
    occ_o, occ_g = occ_o.reshape(-1), occ_g.reshape(-1)
    pf = pflag_o.reshape(-1)
    flag_any = (pf & PIXEL_FLAGS) != 0
    flag_two = (pf & TWO_BEST_FLAGS) != 0
    nd = nnf_o != nnf_g
    od = occ_o != occ_g
    both = (occ_o == 0) & (occ_g == 0)
    fo, fg = flow_o.reshape(-1, 2), flow_g.reshape(-1, 2)
    epe = float(np.linalg.norm(fg[both] - fo[both], axis=-1).mean()) if both.any() else 0.0
    return {
        "pixels": int(nnf_o.size),
        "flagged": int(flag_any.sum()), "flagged_two_best": int(flag_two.sum()),
        "nnf_differ": int(nd.sum()), "nnf_unexplained": int((nd & ~flag_any).sum()),
        "nnf_unexplained_two_best": int((nd & ~flag_two).sum()),
        "occ_differ": int(od.sum()), "occ_unexplained": int((od & ~flag_any).sum()),
        "occ_unexplained_two_best": int((od & ~flag_two).sum()),
        "assigned_both": int(both.sum()), "epe_delta": epe,
    }
