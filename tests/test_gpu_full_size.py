"""GPU parity at the size and parameters of the benchmark workload (a
1024x436 pair, 9x9 patches over 5 channels, windows 64/32/16, 256 RANSAC
hypotheses), in its plain FP32 form (scene seed 0) and its FP16-storage form
(scene seed 1): the same launch configuration as bench.py, phases fed the
oracle's exact state and compared as in the small lock-step tests.

The oracle needs about 25 s per PatchMatch half-sweep at this size, so these
tests cover single steps of each kind rather than the whole pipeline:
  * features, the random initial NNF, the cost refresh and the first
    half-sweep of the initial pass (identity patches, every pixel of a colour),
    then the first half-sweep of the other colour in the fused form the
    pipeline runs (the refresh computed inside the sweep);
  * starting from an initial NNF made of the generator's ground-truth flow in
    both directions with 20 % of the offsets perturbed, every plane phase of
    the three levels (RANSAC stages 1 and 2, assignment, plane symmetry, FB,
    NNF update), one restricted half-sweep after the first level in the fused
    form (the pass's cost refresh inside it; both the distorted-patch kernel
    over pixels with a region plane and the identity-patch kernel over those
    without), and the outputs; a third form
    (scene seed 2) adds occlusion cues 2 and 3 and the filling.
"""
import ctypes

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
# (scene seed, FP16 feature storage, further parameters): the plain FP32 workload, its FP16-storage
# precision form, and the FP32 form with occlusion cues 2 and 3 and 64 half-sweeps of filling
FORMS = {"fp32_seed0": (0, False, {}), "fp16_seed1": (1, True, {}),
         "fp32_seed2_cues_fill": (2, False, dict(cue_overlap=True, cue_unique=True, fill_sweeps=64))}
_pairs = {}


def _pair(seed):
    if seed not in _pairs:
        _pairs[seed] = synth.planar_pair(W, H, seed=seed)
    return _pairs[seed]


def _lockstep(o, g, steps, p):
    """Runs the steps on both sides from the oracle's state, comparing after
    each.  ("fresh", (colour, iter, slot, restricted)) is a half-sweep that
    computes its pixels' costs itself, as the whole pipeline runs the first
    half-sweep of each colour: the oracle runs the cost refresh (unless an
    ("eval_cost", ...) step already did) and the plain half-sweep, the GPU the
    fused sweep with those costs zeroed beforehand."""
    from paper_1804_03787_amd import msgpm
    report = dict(pm_flagged=0, pm_flagged_diff=0, pm_unexplained=0, ransac_nonexact=0, steps=0)
    refreshed = False
    for name, args in steps:
        for d in range(2):
            o.pflag[d][:] = 0
        o.bflag[:] = 0
        if name == "fresh":
            colour, it, slot, restricted = args
            if not refreshed:
                o.run_step("eval_cost", (restricted,))
            parity.push_state(o, g)
            assert parity.poison_refresh(o, g, colour, restricted) > 0
            o.run_step("pm_halfsweep", args)
            g.pm_halfsweep(colour, it, slot, restricted | msgpm.PM_FRESH)
            name = "pm_halfsweep"
        else:
            refreshed = name == "eval_cost"
            parity.push_state(o, g)
            o.run_step(name, args)
            _gpu_step(g, name, args)
        got = parity.pull_state(g)
        if name == "pm_halfsweep":
            for d in range(2):
                assert np.array_equal(np.isfinite(got["cost"][d]), np.isfinite(o.cost[d])), (name, args, d)
        _check_step(name, args, o, got, None, p, report)
        report["steps"] += 1
    return report


def _start(msgpm, pair, p):
    o = oracle.Oracle(pair.frame1, pair.frame2, **p)
    g = msgpm.Pair(W, H, **_gpu_params(p))
    g.set_features(pair.frame1, pair.frame2)
    for f in range(2):
        assert np.array_equal(g.features(f).view(np.uint32), o.feat[f].view(np.uint32))
    return o, g


@pytest.mark.parametrize("form", ["fp32_seed0", "fp16_seed1"])
def test_full_size_initial_pass_step(form):
    msgpm = _need_gpu()
    seed, fp16, _ = FORMS[form]
    pair = _pair(seed)
    p = dict(FULL, fp16=fp16)
    o, g = _start(msgpm, pair, p)
    g.init_state()
    for d in range(2):
        o.nnf_init(d)
        assert np.array_equal(g.nnf(d).cpu().numpy(), o.nnf[d])
    report = _lockstep(o, g, [("eval_cost", (0,))], p)
    if fp16:
        # precision of the FP16 storage: the same costs from the oracle on the FP32 features
        o32 = oracle.Oracle(pair.frame1, pair.frame2, **FULL)
        for d in range(2):
            o32.set_nnf(d, o.nnf[d])
            o32.eval_cost(d, 0)
            got = g.cost(d).cpu().numpy().astype(np.float64)
            rel = np.abs(got - o32.cost[d]) / np.maximum(np.abs(o32.cost[d]), 1e-12)
            q = np.quantile(rel, [0.5, 0.99, 1.0])
            print(f"FP16 storage, cost relative error against FP32 features, dir {d}: "
                  f"median {q[0]:.2e}, p99 {q[1]:.2e}, max {q[2]:.2e}")
            assert q[0] < 1e-3
    # the first half-sweep of colour 0 after the refresh, then that of colour 1
    # with the refresh folded in, as the pipeline runs it
    report = _lockstep(o, g, [("pm_halfsweep", (0, 0, 0, 0)), ("fresh", (1, 0, 0, 0))], p)
    assert report["pm_unexplained"] == 0
    print("full-size initial pass", form, report)


def _perturbed_nnf(flow, seed, frac=0.2, amp=16):
    dx = np.rint(flow[..., 0]).astype(np.int64).reshape(-1)
    dy = np.rint(flow[..., 1]).astype(np.int64).reshape(-1)
    rng = np.random.default_rng(seed)
    m = rng.random(dx.size) < frac
    dx[m] += rng.integers(-amp, amp + 1, int(m.sum()))
    dy[m] += rng.integers(-amp, amp + 1, int(m.sum()))
    return oracle.pack(dx, dy)


@pytest.mark.parametrize("form", list(FORMS))
def test_full_size_plane_phases(form):
    msgpm = _need_gpu()
    seed, fp16, extra = FORMS[form]
    pair = _pair(seed)
    p = dict(FULL, fp16=fp16, **extra)
    o, g = _start(msgpm, pair, p)
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
        steps += [("fb_unassign", ())] + ([("unique", ())] if p.get("cue_unique") else [])
        steps += [("nnf_update", (lv,))]
        if lv == 0:
            # the restricted pass's cost refresh folded into its first half-sweep
            steps += [("fresh", (0, 0, 1, 1))]
    if p.get("fill_sweeps"):
        steps += [("fill", ())]
    report = _lockstep(o, g, steps, p)
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
        assert (np.abs(c[asg] - o.cost[d][asg]) <= tol[asg]).all()
    if p.get("fill_sweeps"):
        assert (o.win[0] <= -2).sum() > 1000
    print("full-size plane phases", form, report, "assigned", float((o.win[0] >= 0).mean()),
          "filled", float((o.win[0] <= -2).mean()))


def test_full_size_fp16_storage_against_fp32_form():
    """Whole pipeline at full size, scene seed 1: the FP16-storage form against
    the plain FP32 GPU form (the oracle needs tens of minutes for a whole
    pipeline at this size; its parity is covered step by step above)."""
    msgpm = _need_gpu()
    pair = _pair(1)
    out = {}
    for fp16 in (False, True):
        g = msgpm.Pair(W, H, **_gpu_params(dict(FULL, fp16=fp16)))
        flows, occs = g.solve(pair.frame1, pair.frame2)
        torch.cuda.synchronize()
        out[fp16] = (flows[0].cpu().numpy(), occs[0].cpu().numpy())
    (f32, o32), (f16, o16) = out[False], out[True]
    vis = pair.occ == 0
    both = (o16 == 0) & (o32 == 0)
    delta = np.linalg.norm(f16 - f32, axis=-1)[both].mean()
    epe16 = np.linalg.norm(f16 - pair.flow, axis=-1)[vis & (o16 == 0)].mean()
    epe32 = np.linalg.norm(f32 - pair.flow, axis=-1)[vis & (o32 == 0)].mean()
    agree = (o16 == o32).mean()
    print(f"full size, FP16 storage vs FP32 form: mean flow delta {delta:.4f} px, EPE to ground truth "
          f"{epe16:.4f} vs {epe32:.4f} px, occlusion agreement {agree:.4f}")
    assert abs(epe16 - epe32) < 0.05 and agree > 0.95


def _project(Hm, x, y):
    qx, qy = ctypes.c_double(), ctypes.c_double()
    h = np.ascontiguousarray(Hm, dtype=np.float64).reshape(9)
    ok = oracle.lib().orc_project(h.ctypes.data_as(ctypes.c_void_p), float(x), float(y), ctypes.byref(qx),
                                  ctypes.byref(qy))
    return bool(ok), qx.value, qy.value


def test_full_size_graph_solve_sampled_outputs():
    """The whole pipeline at full size, launched as bench.py launches it (one HIP
    graph per pair, a replay), checked pixel by pixel on a sample: an assigned
    pixel's flow is its plane's projection (bit for bit), its colour error is
    below eps^2 and its cost is the oracle's cost of its offset under that
    plane; an unassigned pixel's flow is its NNF offset and its cost the
    oracle's cost under its region plane (or the identity)."""
    msgpm = _need_gpu()
    pair = _pair(0)
    g = msgpm.Pair(W, H, **_gpu_params(FULL))
    f1, f2 = torch.from_numpy(pair.frame1).cuda(), torch.from_numpy(pair.frame2).cuda()
    out = ([torch.empty((H, W, 2), device="cuda") for _ in range(2)],
           [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(2)])
    for _ in range(2):
        flows, occs = g.solve(f1, f2, out=out, graph=True)
    torch.cuda.synchronize()
    o = oracle.Oracle(pair.frame1, pair.frame2, **FULL)
    planes = g.planes()
    rng = np.random.default_rng(77)
    eps2 = FULL["eps"] ** 2
    for d in range(2):
        flow = flows[d].cpu().numpy().reshape(-1, 2)
        occ = occs[d].cpu().numpy().ravel()
        win = g.win(d).cpu().numpy()
        nnf = g.nnf(d).cpu().numpy()
        cost = g.cost(d).cpu().numpy()
        hl = g.hlabel(d).cpu().numpy()
        dx, dy = oracle.unpack(nnf)
        assigned = np.nonzero(win >= 0)[0]
        free = np.nonzero(win < 0)[0]
        assert len(assigned) > 0.5 * W * H and len(free) > 1000
        for p in np.concatenate([rng.choice(assigned, 200, replace=False), rng.choice(free, 200, replace=False)]):
            x, y = int(p % W), int(p // W)
            tx, ty = x + int(dx[p]), y + int(dy[p])
            j = int(win[p])
            if j >= 0:
                Hm = planes["H"][j]
                ok, qx, qy = _project(Hm, x, y)
                assert ok and occ[p] == 0
                assert flow[p, 0] == np.float32(qx - x) and flow[p, 1] == np.float32(qy - y), (d, p)
                assert o.colour_err(d, x, y, Hm) < eps2
            else:
                Hm = planes["H"][hl[p]] if hl[p] >= 0 else None
                assert occ[p] == 1
                assert flow[p, 0] == dx[p] and flow[p, 1] == dy[p]
            ref = o.cost_at(d, x, y, tx, ty, Hm)
            if not np.isfinite(ref):
                assert not np.isfinite(cost[p])
                continue
            tol = parity.cost_tol(np.array([ref]), FULL["r"], FULL["C"])[0]
            assert abs(float(cost[p]) - ref) <= tol, (d, p, float(cost[p]), ref)


def _golden(case):
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_full_size_golden", os.path.join(here, "make_full_size_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod, np.load(mod.path(case))


@pytest.mark.parametrize("case", ["fp32_seed0", "fp16_seed1"])
def test_full_size_free_running_against_oracle_solve(case):
    """The whole pipeline at full size, free-running and launched as bench.py
    launches it (a replay of the captured graph), against the oracle's whole
    solve of the same pair (stored by tests/golden/make_full_size_golden.py
    from oracle/ alone): FP32 on scene seed 0, FP16 storage on scene seed 1.
    NNF offsets and masks must be bit-exact outside the pixels the oracle flags
    as near-ties under the two-best rule (the two best PatchMatch costs over
    distinct targets within the band, or a rounding, colour, forward-backward
    or bounds decision within its band), and the flow EPE delta over pixels
    assigned on both sides must stay <= 0.01 px.  A flipped near-tie could
    cascade into unflagged pixels; none does on these pairs (measured on
    MI355X: one differing NNF offset in 892 928, flagged, and no differing
    mask pixel, EPE delta 0)."""
    msgpm = _need_gpu()
    mod, ref = _golden(case)
    seed, fp16, _ = FORMS[case]
    pair = _pair(seed)
    assert [mod.digest(pair.frame1), mod.digest(pair.frame2)] == [str(s) for s in ref["frames_sha256"]]
    g = msgpm.Pair(W, H, **_gpu_params(dict(FULL, fp16=fp16)))
    f1, f2 = torch.from_numpy(pair.frame1).cuda(), torch.from_numpy(pair.frame2).cuda()
    out = ([torch.empty((H, W, 2), device="cuda") for _ in range(2)],
           [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(2)])
    for _ in range(2):
        flows, occs = g.solve(f1, f2, out=out, graph=True)
    torch.cuda.synchronize()
    for d in range(2):
        rep = parity.free_run_compare(ref[f"nnf{d}"], ref[f"occ{d}"], ref[f"flow{d}"], ref[f"pflag{d}"],
                                      g.nnf(d).cpu().numpy(), occs[d].cpu().numpy(), flows[d].cpu().numpy())
        print(case, "dir", d, rep, flush=True)
        assert rep["epe_delta"] <= 0.01, rep
        assert rep["nnf_unexplained_two_best"] == 0 and rep["occ_unexplained_two_best"] == 0, rep


def _others():
    """Two pairs of other sizes and scenes that share the batch or the server
    with the full-size pair (same instantiation and schedule: windows 64/32/16)."""
    return [(synth.planar_pair(640, 360, seed=21, scale=0.625), 21), (synth.planar_pair(320, 240, seed=22, scale=0.3125), 22)]


def _check_against_golden(ref, g, flows, occs, label):
    for d in range(2):
        rep = parity.free_run_compare(ref[f"nnf{d}"], ref[f"occ{d}"], ref[f"flow{d}"], ref[f"pflag{d}"],
                                      g.nnf(d).cpu().numpy(), occs[d].cpu().numpy(), flows[d].cpu().numpy())
        print(label, "dir", d, rep, flush=True)
        assert rep["epe_delta"] <= 0.01, rep
        assert rep["nnf_unexplained_two_best"] == 0 and rep["occ_unexplained_two_best"] == 0, rep


def test_full_size_batched_fp16_against_oracle_solve():
    """The batched FP16-storage form at full size against the oracle: the scene
    seed 1 1024x436 pair in one batch with a 640x360 and a 320x240 pair of other
    scenes, the whole batch launched as one graph (msgpm_solve_batch_graph, as
    bench.py --batched launches it), the full-size pair's NNF and masks bit-exact
    against the stored whole oracle solve outside two-best near-ties, EPE delta
    <= 0.01 px."""
    msgpm = _need_gpu()
    mod, ref = _golden("fp16_seed1")
    pair = _pair(1)
    assert [mod.digest(pair.frame1), mod.digest(pair.frame2)] == [str(s) for s in ref["frames_sha256"]]
    scenes = [(pair, 0)] + _others()
    gs = [msgpm.Pair(pr.shape[1], pr.shape[0], **_gpu_params(dict(FULL, fp16=True, seed=s))) for pr, s in scenes]
    batch = msgpm.Batch(gs)
    res = batch.solve([pr.frame1 for pr, _ in scenes], [pr.frame2 for pr, _ in scenes], graph=True)
    torch.cuda.synchronize()
    flows, occs = res[0]
    _check_against_golden(ref, gs[0], flows, occs, "batched fp16_seed1")


def test_full_size_served_fp16_against_oracle_solve():
    """The served FP16-storage form at full size against the oracle: continuous
    batching with the 1024x436 pair (scene seed 1) submitted while a 640x360
    pair is in flight and before a 320x240 one, its result checked against the
    stored whole oracle solve as in the batched test."""
    msgpm = _need_gpu()
    mod, ref = _golden("fp16_seed1")
    pair = _pair(1)
    others = _others()
    srv = msgpm.Server(hbm_budget=1 << 34, max_active=8)
    order = [(others[0][0], others[0][1]), (pair, 0), (others[1][0], others[1][1])]
    tickets, done = {}, {}
    for k, (pr, s) in enumerate(order):
        g = msgpm.Pair(pr.shape[1], pr.shape[0], **_gpu_params(dict(FULL, fp16=True, seed=s)))
        tickets[srv.submit(g, pr.frame1, pr.frame2)] = k
        srv.step()
    rounds = 0
    while tickets:
        srv.step()
        for t, k in list(tickets.items()):
            if srv.poll(t):
                done[k] = srv.result(t)
                del tickets[t]
        rounds += 1
        assert rounds < 1000000
    srv.close()
    g, flows, occs = done[1]
    torch.cuda.synchronize()
    _check_against_golden(ref, g, flows, occs, "served fp16_seed1")
