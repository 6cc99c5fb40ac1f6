"""GPU parity at the size and parameters of the benchmark workload (a
1024x436 pair, 9x9 patches over 5 channels, windows 64/32/16, 256 RANSAC
hypotheses): the same launch configuration as bench.py, phases fed the
oracle's exact state and compared as in the small lock-step tests.

The oracle needs about 25 s per PatchMatch half-sweep at this size, so these
tests cover single steps of each kind rather than the whole pipeline:
  * features, the random initial NNF, the cost refresh and the first
    half-sweep of the initial pass (identity patches, every pixel of a colour);
  * starting from an initial NNF made of the generator's ground-truth flow in
    both directions with 20 % of the offsets perturbed, every plane phase of
    the three levels (RANSAC stages 1 and 2, assignment, plane symmetry, FB,
    NNF update), one restricted half-sweep after the first level (both the
    distorted-patch kernel over pixels with a region plane and the
    identity-patch kernel over those without), and the outputs.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_03787_amd import synth
from tests import parity
from tests.test_gpu_parity import _check_step, _gpu_params, _gpu_step, _need_gpu

pytestmark = pytest.mark.gpu

W, H = 1024, 436
FULL = dict(C=5, r=4, blocks=(64, 32, 16), iters=8, hyps=256, tau=1.0, eps=0.1, tau_fb=1.0, seed=0)


@pytest.fixture(scope="module")
def pair():
    return synth.planar_pair(W, H, seed=0)


def _lockstep(o, g, steps, p):
    report = dict(pm_flagged=0, pm_flagged_diff=0, pm_unexplained=0, ransac_nonexact=0, steps=0)
    for name, args in steps:
        for d in range(2):
            o.pflag[d][:] = 0
        o.bflag[:] = 0
        parity.push_state(o, g)
        o.run_step(name, args)
        _gpu_step(g, name, args)
        got = parity.pull_state(g)
        _check_step(name, args, o, got, None, p, report)
        report["steps"] += 1
    return report


def _start(msgpm, pair):
    o = oracle.Oracle(pair.frame1, pair.frame2, **FULL)
    g = msgpm.Pair(W, H, **_gpu_params(FULL))
    g.set_features(pair.frame1, pair.frame2)
    for f in range(2):
        assert np.array_equal(g.features(f).view(np.uint32), o.feat[f].view(np.uint32))
    return o, g


def test_full_size_initial_pass_step(pair):
    msgpm = _need_gpu()
    o, g = _start(msgpm, pair)
    g.init_state()
    for d in range(2):
        o.nnf_init(d)
        assert np.array_equal(g.nnf(d).cpu().numpy(), o.nnf[d])
    report = _lockstep(o, g, [("eval_cost", (0,)), ("pm_halfsweep", (0, 0, 0, 0))], FULL)
    assert report["steps"] == 2 and report["pm_unexplained"] == 0
    print("full-size initial pass", report)


def _perturbed_nnf(flow, seed, frac=0.2, amp=16):
    dx = np.rint(flow[..., 0]).astype(np.int64).reshape(-1)
    dy = np.rint(flow[..., 1]).astype(np.int64).reshape(-1)
    rng = np.random.default_rng(seed)
    m = rng.random(dx.size) < frac
    dx[m] += rng.integers(-amp, amp + 1, int(m.sum()))
    dy[m] += rng.integers(-amp, amp + 1, int(m.sum()))
    return oracle.pack(dx, dy)


def test_full_size_plane_phases(pair):
    msgpm = _need_gpu()
    o, g = _start(msgpm, pair)
    init = [_perturbed_nnf(pair.flow, 1), _perturbed_nnf(synth.ground_truth_backward(pair.layers, W, H), 2)]
    g.init_state(torch.from_numpy(init[0]), torch.from_numpy(init[1]))
    for d in range(2):
        o.set_nnf(d, init[d])
        assert np.array_equal(g.nnf(d).cpu().numpy(), o.nnf[d])
    steps = []
    for lv in range(3):
        for stage in (1, 2):
            steps += [("ransac", (lv, stage)), ("assign", (lv, stage, 1)), ("symmetry", (lv, stage)),
                      ("assign", (lv, stage, 0))]
        steps += [("fb_unassign", ()), ("nnf_update", (lv,))]
        if lv == 0:
            steps += [("eval_cost", (1,)), ("pm_halfsweep", (0, 0, 1, 1))]
    report = _lockstep(o, g, steps, FULL)
    assert report["pm_unexplained"] == 0
    # the steps did real work: most pixels end up on a plane, some windows needed stage 2
    pl = parity.planes_to_gpu(o)
    assert (o.win[0] >= 0).mean() > 0.5 and (o.win[1] >= 0).mean() > 0.5
    assert pl["valid"][pl["stage"] == 1].sum() > 100 and pl["detected"][pl["stage"] == 2].sum() > 0
    parity.push_state(o, g)
    flows_g, occs_g = g.finalize()
    for d in range(2):
        fo, oo = o.finalize(d)
        assert np.array_equal(occs_g[d].cpu().numpy(), oo)
        assert np.array_equal(flows_g[d].cpu().numpy(), fo)
        c = g.cost(d).cpu().numpy()
        asg = o.win[d] >= 0
        tol = parity.cost_tol(o.cost[d], FULL["r"], FULL["C"])
        assert (np.abs(c - o.cost[d])[asg] <= tol[asg]).all()
    print("full-size plane phases", report, "assigned", float((o.win[0] >= 0).mean()))
