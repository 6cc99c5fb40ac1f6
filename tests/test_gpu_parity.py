"""GPU parity: the HIP library against the FP64 oracle on the same seeded
inputs, through the C ABI.

Phase-isolated ("lock-step") tests feed the oracle's exact state to each GPU
phase and compare the phase's outputs:
  * integer, index and FP64 outputs (features, initial NNF, RANSAC plane
    records, assignments, symmetry counts, FB, NNF update, flow of assigned
    pixels) must be bit-exact;
  * PatchMatch offsets must be bit-exact except at pixels the oracle flags as
    near-ties (a cost comparison within 1e-5 relative); FP32 costs must agree
    within 1e-5 relative plus 1e-7 (2r+1)^2 C absolute.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_03787_amd import synth
from tests import parity
from tests.conftest import TINY_PARAMS

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1804_03787_amd import msgpm
    msgpm.lib()
    return msgpm


def _gpu_params(p):
    keys = ("C", "r", "blocks", "iters", "hyps", "R0", "tau", "eps", "tau_fb", "mu", "m_min_abs", "eta", "seed",
            "fp16", "grad_weight", "cue_overlap", "cue_unique", "fill_sweeps", "histeq", "merge_strict")
    full = dict(oracle.DEFAULTS)
    full.update(p)
    return {k: full[k] for k in keys}


RAGGED = dict(C=3, r=2, grad_weight=0.0, blocks=(20, 12), iters=2, hyps=48, seed=7)


def _ragged_pair():
    W, H = 77, 53
    rng = np.random.default_rng(31)
    bg = synth.Layer(H=synth.similarity_about(38, 26, 1.02, 2.0, 3.0, -2.0))
    fg = synth.Layer(H=synth.translation(-4, 3), poly=np.array([[20.0, 10], [50, 14], [46, 40], [18, 36]]))
    return synth.render([bg, fg], W, H, rng)


def _two_layer_pair(W, H, seed):
    """A zoomed and rotated background with one translated foreground quad."""
    rng = np.random.default_rng(seed)
    bg = synth.Layer(H=synth.similarity_about(W / 2, H / 2, 1.02, 2.0, 4.0, -3.0))
    fg = synth.Layer(H=synth.translation(-6, 4),
                     poly=np.array([[0.2 * W, 0.2 * H], [0.55 * W, 0.25 * H], [0.5 * W, 0.7 * H], [0.25 * W, 0.65 * H]]))
    return synth.render([bg, fg], W, H, rng)


CASES = {
    "tiny_c5": (lambda: synth.tiny_pair(0), TINY_PARAMS),
    "tiny_c3": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, C=3, grad_weight=0.0)),
    "ragged": (_ragged_pair, RAGGED),
    # FP16 feature storage with FP32 accumulation, against the oracle on the
    # same FP16-rounded features
    "tiny_c5_fp16": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, fp16=True)),
    # occlusion cues 2 and 3 on: on this pair the uniqueness step unassigns
    # several hundred pixels and the overlap test rejects about twenty planes
    "tiny_cues": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, cue_overlap=True, cue_unique=True)),
    # filling by model propagation, 64 half-sweeps: on this pair about half of
    # the unassigned pixels are filled
    "tiny_fill": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, fill_sweeps=64)),
    # two levels with the strict level priority: the 16-pixel level assigns
    # only what the 32-pixel level left unassigned
    "tiny_strict": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, blocks=(32, 16), merge_strict=True)),
    # the same two levels with the default merge key, for comparison
    "tiny_two_levels": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, blocks=(32, 16))),
    # frames equalised in HSV value before the features
    "tiny_histeq": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, histeq=True)),
    # no plane levels at all: PatchMatch alone, every pixel occluded, an empty
    # plane table (and a filling with nothing to propagate)
    "no_levels": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, blocks=(), fill_sweeps=4)),
    # random-search start radii of 16 and 32: 5 and 6 radii, so the last
    # identity-patch batch holds 1 and 2 candidates (the other cases leave 0 or 3)
    "tiny_r0_16": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, R0=16)),
    "tiny_r0_32": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, R0=32)),
    # no PatchMatch iterations: the passes are their cost refreshes alone (run on
    # their own, not folded into a first half-sweep), the planes are fitted to
    # the random initial NNF
    "no_sweeps": (lambda: synth.tiny_pair(0), dict(TINY_PARAMS, iters=0)),
    # a frame smaller than the patch and the window (9x7, 9x9 patches, 8-pixel
    # windows): every gather clamps, one wave holds the whole frame
    "minimal": (lambda: _two_layer_pair(9, 7, 43),
                dict(C=5, r=4, blocks=(8,), iters=2, hyps=16, tau=1.0, eps=0.1, tau_fb=1.0, seed=6)),
    # 128-pixel windows (as the fourth level of 2048-wide frames): point lists of
    # up to 16384 points, more than 64 KB of LDS, 8 points per lane in the scoring
    "big_windows": (lambda: _two_layer_pair(224, 160, 41),
                    dict(C=5, r=3, blocks=(128, 64), iters=3, hyps=128, tau=1.0, eps=0.1, tau_fb=1.0, seed=4)),
    # the paper's own preset: two levels of 81 and 41 pixel windows (strides 40
    # and 20), 7x7 patches over RGB
    "paper_preset": (lambda: synth.planar_pair(200, 144, seed=11, scale=0.08),
                     dict(C=3, r=3, grad_weight=0.0, blocks=(81, 41), iters=4, hyps=128, tau=1.0, eps=0.1,
                          tau_fb=1.0, seed=2)),
}


@pytest.mark.parametrize("histeq", [False, True])
@pytest.mark.parametrize("fp16", [False, True])
@pytest.mark.parametrize("C", [3, 5])
def test_features_bitexact(C, fp16, histeq):
    """Features of the ragged 77x53 pair, bit for bit; with histeq, of the
    equalised frames (frame 2 darkened by a gain of 0.6 first)."""
    msgpm = _need_gpu()
    pair = _ragged_pair()
    f2 = pair.frame2 * np.float32(0.6) if histeq else pair.frame2
    g = msgpm.Pair(77, 53, **_gpu_params(dict(C=C, fp16=fp16, blocks=(16,), histeq=histeq)))
    g.set_features(pair.frame1, f2)
    for f, frame in enumerate((pair.frame1, f2)):
        ref = oracle.features(oracle.histeq(frame) if histeq else frame, C=C, fp16=fp16)
        got = g.features(f)
        assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))


def test_histeq_features_edge_frames():
    """Equalisation on frames that take its special paths: a single-level frame
    (left as it is), a frame with black and negative pixels (value <= 0) and
    values above 1 (clamped levels); features bit-exact against the oracle."""
    msgpm = _need_gpu()
    rng = np.random.default_rng(61)
    W, H = 45, 31
    flat = np.full((H, W, 3), 0.4, np.float32)
    flat[..., 2] = 0.1
    odd = rng.random((H, W, 3)).astype(np.float32) * 1.6 - 0.2
    odd[:5, :7] = 0.0
    odd[10:12, 3:9] = -0.05
    for C in (3, 5):
        g = msgpm.Pair(W, H, **_gpu_params(dict(C=C, blocks=(16,), histeq=True)))
        g.set_features(flat, odd)
        for f, frame in enumerate((flat, odd)):
            ref = oracle.features(oracle.histeq(frame), C=C)
            assert np.array_equal(g.features(f).view(np.uint32), ref.view(np.uint32)), (C, f)
    assert np.array_equal(oracle.histeq(flat), flat)


def test_init_nnf_bitexact_and_given_nnf_clamped():
    msgpm = _need_gpu()
    pair = synth.tiny_pair(0)
    o = oracle.Oracle(pair.frame1, pair.frame2, **TINY_PARAMS)
    g = msgpm.Pair(128, 96, **_gpu_params(TINY_PARAMS))
    g.set_features(pair.frame1, pair.frame2)
    g.init_state()
    for d in range(2):
        o.nnf_init(d)
        assert np.array_equal(g.nnf(d).cpu().numpy(), o.nnf[d])
        assert (g.win(d).cpu().numpy() == -1).all() and (g.hlabel(d).cpu().numpy() == -1).all()
    rng = np.random.default_rng(3)
    given = [oracle.pack(rng.integers(-300, 300, 128 * 96), rng.integers(-300, 300, 128 * 96)) for _ in range(2)]
    g.init_state(torch.from_numpy(given[0]), torch.from_numpy(given[1]))
    for d in range(2):
        o.set_nnf(d, given[d])
        assert np.array_equal(g.nnf(d).cpu().numpy(), o.nnf[d])


def _check_step(name, args, o, got, before, p, report):
    r, C = p.get("r", 4), p.get("C", 5)
    if name == "eval_cost":
        for d in range(2):
            tol = parity.cost_tol(o.cost[d], r, C)
            fin = np.isfinite(o.cost[d])
            assert np.array_equal(np.isfinite(got["cost"][d]), fin), (name, args, d)
            err = np.abs(got["cost"][d][fin] - o.cost[d][fin])
            assert (err <= tol[fin]).all(), (name, args, d, float(err.max()))
    elif name == "pm_halfsweep":
        for d in range(2):
            flagged = (o.pflag[d] & (oracle.F_COST | oracle.F_ROUND)) != 0
            diff = got["nnf"][d] != o.nnf[d]
            report["pm_flagged"] += int(flagged.sum())
            report["pm_flagged_diff"] += int((diff & flagged).sum())
            report["pm_unexplained"] += int((diff & ~flagged).sum())
            same = ~diff & np.isfinite(o.cost[d])
            tol = parity.cost_tol(o.cost[d][same], r, C)
            err = np.abs(got["cost"][d][same] - o.cost[d][same])
            assert (err <= tol).all(), (name, args, d, float(err.max()))
        assert report["pm_unexplained"] == 0, (name, args, report)
    elif name == "ransac":
        bad = parity.compare_planes(o, got["planes"])
        if bad:
            flagged = np.nonzero(o.bflag)[0]
            bad_loose = parity.compare_planes(o, got["planes"], sel=~(o.bflag > 0), exact=True)
            report["ransac_nonexact"] += 1
            assert not bad_loose, (name, args, bad, "unflagged:", bad_loose, len(flagged))
    elif name == "assign":
        tent = args[2]
        wk, lk = ("twin", "tloss") if tent else ("win", "loss")
        for d in range(2):
            ow = (o.twin if tent else o.win)[d]
            ol = (o.tloss if tent else o.loss)[d]
            assert np.array_equal(got[wk][d], ow), (name, args, d, int((got[wk][d] != ow).sum()))
            assert np.array_equal(got[lk][d], ol), (name, args, d)
    elif name == "symmetry":
        bad = parity.compare_planes(o, got["planes"])
        assert not bad, (name, args, bad)
    elif name in ("fb_unassign", "unique", "fill"):
        for d in range(2):
            assert np.array_equal(got["win"][d], o.win[d]), (name, d)
            assert np.array_equal(got["loss"][d], o.loss[d]), (name, d)
    elif name == "nnf_update":
        for d in range(2):
            assert np.array_equal(got["nnf"][d], o.nnf[d]), (name, args, d)
            assert np.array_equal(got["hlabel"][d], o.hlabel[d]), (name, args, d)


def _gpu_step(g, name, args):
    if name == "eval_cost":
        g.eval_cost(*args)
    else:
        getattr(g, name)(*args)


@pytest.mark.parametrize("case", list(CASES))
def test_lockstep_pipeline(case):
    """Every phase of the pipeline, GPU fed the oracle's state, outputs compared."""
    msgpm = _need_gpu()
    make, p = CASES[case]
    pair = make()
    H, W = pair.shape
    o = oracle.Oracle(pair.frame1, pair.frame2, **p)
    g = msgpm.Pair(W, H, **_gpu_params(p))
    g.set_features(pair.frame1, pair.frame2)
    for f in range(2):
        assert np.array_equal(g.features(f).view(np.uint32), o.feat[f].view(np.uint32))
    g.init_state()
    for d in range(2):
        o.nnf_init(d)
    report = dict(pm_flagged=0, pm_flagged_diff=0, pm_unexplained=0, ransac_nonexact=0, steps=0)
    for name, args in o.schedule():
        for d in range(2):
            o.pflag[d][:] = 0
        o.bflag[:] = 0
        parity.push_state(o, g)
        before = None
        o.run_step(name, args)
        _gpu_step(g, name, args)
        got = parity.pull_state(g)
        _check_step(name, args, o, got, before, p, report)
        report["steps"] += 1
    # outputs
    parity.push_state(o, g)
    flows_g, occs_g = g.finalize()
    for d in range(2):
        fo, oo = o.finalize(d)
        assert np.array_equal(occs_g[d].cpu().numpy(), oo)
        assert np.array_equal(flows_g[d].cpu().numpy(), fo)
        c = g.cost(d).cpu().numpy()
        asg = o.win[d] >= 0
        tol = parity.cost_tol(o.cost[d], p.get("r", 4), p.get("C", 5))
        assert (np.abs(c[asg] - o.cost[d][asg]) <= tol[asg]).all()
    print(case, report)


@pytest.mark.parametrize("case", ["tiny_c5", "tiny_c5_fp16", "ragged", "paper_preset"])
def test_lockstep_fresh_halfsweeps(case):
    """The cost refresh folded into the first half-sweep of each colour
    (PM_FRESH, as the whole pipeline runs it).  The GPU is fed the oracle's
    state with the costs the refresh would set replaced by zeros (a cost no
    candidate beats, so a sweep that read them would keep every offset); its
    fused sweep must give what the oracle's refresh followed by its plain
    half-sweep gives, to the bar of the plain half-sweep."""
    msgpm = _need_gpu()
    make, p = CASES[case]
    pair = make()
    H, W = pair.shape
    o = oracle.Oracle(pair.frame1, pair.frame2, **p)
    g = msgpm.Pair(W, H, **_gpu_params(p))
    g.set_features(pair.frame1, pair.frame2)
    g.init_state()
    for d in range(2):
        o.nnf_init(d)
    report = dict(pm_flagged=0, pm_flagged_diff=0, pm_unexplained=0, ransac_nonexact=0, steps=0)
    pending, fused, poisoned_total = {}, 0, 0
    for name, args in o.schedule():
        for d in range(2):
            o.pflag[d][:] = 0
        o.bflag[:] = 0
        if name == "eval_cost":
            o.run_step(name, args)  # the GPU folds it into the next two half-sweeps
            pending = {0: args[0], 1: args[0]}
            continue
        parity.push_state(o, g)
        if name == "pm_halfsweep" and args[0] in pending:
            colour, it, slot, restricted = args
            mode = pending.pop(colour)
            assert it == 0 and restricted == mode
            poisoned_total += parity.poison_refresh(o, g, colour, mode)
            o.run_step(name, args)
            g.pm_halfsweep(colour, it, slot, restricted | msgpm.PM_FRESH)
            fused += 1
            got = parity.pull_state(g)
            for d in range(2):
                assert np.array_equal(np.isfinite(got["cost"][d]), np.isfinite(o.cost[d])), (args, d)
        else:
            o.run_step(name, args)
            _gpu_step(g, name, args)
            got = parity.pull_state(g)
        _check_step(name, args, o, got, None, p, report)
        report["steps"] += 1
    assert fused == 2 * (1 + len(p["blocks"])) and poisoned_total > 0
    print(case, report, "fused sweeps", fused, "poisoned costs", poisoned_total)


@pytest.mark.parametrize("case", ["tiny_c5", "tiny_c5_fp16", "tiny_cues", "tiny_fill", "tiny_histeq", "no_sweeps",
                                  "tiny_strict", "tiny_two_levels"])
def test_solve_end_to_end(case):
    """Free-running whole pipeline against the oracle's whole solve: NNF
    offsets and occlusion masks bit-exact outside the pixels the oracle flags
    as near-ties, flow EPE delta <= 0.01 px over the pixels assigned on both
    sides; where both leave a pixel occluded with the same offset, the flow is
    that offset."""
    msgpm = _need_gpu()
    make, p = CASES[case]
    pair = make()
    H, W = pair.shape
    o = oracle.Oracle(pair.frame1, pair.frame2, **p)
    fo, oo = o.solve()
    g = msgpm.Pair(W, H, **_gpu_params(p))
    fg, og = g.solve(pair.frame1, pair.frame2)
    torch.cuda.synchronize()
    for d in range(2):
        og_ = og[d].cpu().numpy()
        fg_ = fg[d].cpu().numpy()
        occ_agree = (og_ == oo[d]).mean()
        both = (og_ == 0) & (oo[d] == 0)
        epe_delta = np.linalg.norm(fg_ - fo[d], axis=-1)[both].mean() if both.any() else 0.0
        nnf_same = g.nnf(d).cpu().numpy() == o.nnf[d]
        rep = parity.free_run_compare(o.nnf[d], oo[d], fo[d], o.pflag[d], g.nnf(d).cpu().numpy(), og_, fg_)
        print(case, d, "occ agree", occ_agree, "nnf agree", nnf_same.mean(), "EPE delta", epe_delta,
              "assigned", both.mean(), rep)
        assert rep["nnf_unexplained"] == 0 and rep["occ_unexplained"] == 0, rep
        assert epe_delta <= 0.01
        # occluded on both sides with the same offset: the flow is that offset
        none = ((og_ == 1) & (oo[d] == 1)).reshape(-1) & nnf_same
        assert np.array_equal(fg_.reshape(-1, 2)[none], fo[d].reshape(-1, 2)[none])


def test_solve_is_deterministic():
    msgpm = _need_gpu()
    pair = synth.tiny_pair(0)
    outs = []
    for _ in range(2):
        g = msgpm.Pair(128, 96, **_gpu_params(TINY_PARAMS))
        fg, og = g.solve(pair.frame1, pair.frame2)
        torch.cuda.synchronize()
        outs.append((fg[0].cpu().numpy(), og[0].cpu().numpy(), g.planes()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2].view(np.uint8), outs[1][2].view(np.uint8))


def test_one_stream_flag_gives_the_same_result():
    """MSGPM_FLAG_ONE_STREAM (both restricted launches in sequence on the
    caller's stream) against the default two-stream issue: flow, masks, plane
    table and NNF bit-identical, eager and as a captured graph, and the
    restricted kinds are timed on their own."""
    msgpm = _need_gpu()
    pair = synth.planar_pair(160, 120, seed=3, scale=0.15)
    outs = []
    for one, graph in ((False, False), (True, False), (True, True)):
        g = msgpm.Pair(160, 120, **_gpu_params(TINY_PARAMS), one_stream=one)
        msgpm.timing_enable(not graph)
        msgpm.timing_read()
        fg, og = g.solve(pair.frame1, pair.frame2, graph=graph)
        torch.cuda.synchronize()
        tm = msgpm.timing_read()
        msgpm.timing_enable(False)
        if not graph:
            assert tm["pm_restricted"][1] > 0 and tm["pm_restricted_ident"][1] > 0
        outs.append(([f.cpu().numpy() for f in fg], [o.cpu().numpy() for o in og], g.planes(),
                     [g.nnf(d).cpu().numpy() for d in range(2)]))
    for other in outs[1:]:
        for d in range(2):
            assert np.array_equal(outs[0][0][d].view(np.uint32), other[0][d].view(np.uint32))
            assert np.array_equal(outs[0][1][d], other[1][d])
            assert np.array_equal(outs[0][3][d], other[3][d])
        assert np.array_equal(outs[0][2].view(np.uint8), other[2].view(np.uint8))


def test_fp16_mixed_precision_arithmetic_equals_widening_first():
    """msgpm_check_fp16_arith: every mixed-precision form the FP16 kernels use
    (f - h, h - h', h - v, h * w + a, h * w + 0, with halves widened inside one
    FMA) gives the bits of an exact conversion followed by FP32 arithmetic,
    over all 65536 FP16 patterns in both halves of a word."""
    msgpm = _need_gpu()
    bad, total = msgpm.check_fp16_arith(256)
    assert total == 65536 * 256 * 12
    assert bad == 0, f"{bad} of {total} results differ"
    with pytest.raises(msgpm.MsgpmError):
        msgpm.check_fp16_arith(0)


def test_invalid_arguments_raise():
    msgpm = _need_gpu()
    with pytest.raises(msgpm.MsgpmError):
        msgpm.Pair(128, 96, r=7)
    g = msgpm.Pair(64, 48, **_gpu_params(dict(blocks=(16,), r=2, C=3)))
    with pytest.raises(msgpm.MsgpmError):
        g.ransac(3, 1)
    with pytest.raises(msgpm.MsgpmError):
        g.pm_halfsweep(2, 0, 0, 0)
    with pytest.raises(msgpm.MsgpmError):
        g.pm_halfsweep(0, 0, 0, 4)


def test_fp16_storage_precision_report():
    """What FP16 feature storage costs in the flow: the GPU's FP16-storage
    solve against the oracle on the FP32 features and against the GPU's FP32
    form (the FP16 form against the oracle on the same FP16 features is held to
    the parity bar above).  Reported; bounded loosely."""
    msgpm = _need_gpu()
    pair = synth.tiny_pair(0)
    p16 = dict(TINY_PARAMS, fp16=True)
    fo32, oo32 = oracle.Oracle(pair.frame1, pair.frame2, **TINY_PARAMS).solve()
    g16 = msgpm.Pair(128, 96, **_gpu_params(p16))
    fg16, og16 = g16.solve(pair.frame1, pair.frame2)
    g32 = msgpm.Pair(128, 96, **_gpu_params(TINY_PARAMS))
    fg32, og32 = g32.solve(pair.frame1, pair.frame2)
    torch.cuda.synchronize()
    gt = pair.flow
    vis = pair.occ == 0
    for name, (fr, orr) in {"oracle FP32 features": (fo32[0], oo32[0]),
                            "GPU FP32 form": (fg32[0].cpu().numpy(), og32[0].cpu().numpy())}.items():
        f16, o16 = fg16[0].cpu().numpy(), og16[0].cpu().numpy()
        both = (o16 == 0) & (orr == 0)
        delta = np.linalg.norm(f16 - fr, axis=-1)[both].mean()
        epe16 = np.linalg.norm(f16 - gt, axis=-1)[vis & (o16 == 0)].mean()
        eperef = np.linalg.norm(fr - gt, axis=-1)[vis & (orr == 0)].mean()
        agree = (o16 == orr).mean()
        print(f"FP16 storage vs {name}: mean flow delta {delta:.4f} px, EPE to ground truth "
              f"{epe16:.4f} vs {eperef:.4f} px, occlusion agreement {agree:.4f}")
        assert delta < 0.25 and abs(epe16 - eperef) < 0.25 and agree > 0.95
