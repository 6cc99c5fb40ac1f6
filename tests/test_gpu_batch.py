"""Batched solves (msgpm_solve_batch): pairs of uneven sizes share one launch
per phase, and each pair's outputs (flow, occlusion, plane table, NNF) are
bit-identical to a msgpm_solve of that pair alone.  GPU against GPU: the
single-pair path is held to the oracle by the parity tests, and one batch of
FP16-storage pairs is also compared with the oracle directly."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1804_03787_amd import synth
from tests.conftest import TINY_PARAMS
from tests.test_gpu_parity import _gpu_params, _need_gpu

pytestmark = pytest.mark.gpu


def _outputs(g, flows, occs):
    torch.cuda.synchronize()
    return ([f.cpu().numpy() for f in flows], [o.cpu().numpy() for o in occs], g.planes(),
            [g.nnf(d).cpu().numpy() for d in range(2)])


def _same(a, b):
    fa, oa, pa, na = a
    fb, ob, pb, nb = b
    for d in range(2):
        assert np.array_equal(fa[d].view(np.uint32), fb[d].view(np.uint32))
        assert np.array_equal(oa[d], ob[d])
        assert np.array_equal(na[d], nb[d])
    assert np.array_equal(pa.view(np.uint8), pb.view(np.uint8))


def _run(msgpm, pairs, params, inits=None):
    """Each pair alone, then the batch three ways: eager launches, one graph
    launch (twice: capture, then a replay), and eager with every persistent
    launch at one resident workgroup per compute unit; all bit-identical."""
    alone = []
    for i, (pr, p) in enumerate(zip(pairs, params)):
        H, W = pr.shape
        g = msgpm.Pair(W, H, **p)
        init = (None, None) if inits is None or inits[i] is None else inits[i]
        flows, occs = g.solve(pr.frame1, pr.frame2, *init)
        alone.append(_outputs(g, flows, occs))
    gs = [msgpm.Pair(pr.shape[1], pr.shape[0], **p) for pr, p in zip(pairs, params)]
    batch = msgpm.Batch(gs)
    f1, f2 = [pr.frame1 for pr in pairs], [pr.frame2 for pr in pairs]
    key = dict(r=params[0]["r"], C=params[0]["C"], fp16=bool(params[0]["fp16"]))
    saved = msgpm.tuning_get(**key)
    try:
        for graph, tune in ((False, None), (True, None), (True, None), (False, 1)):
            if tune is not None:
                msgpm.tuning_set(**key, **{k: tune for k in saved})
            for g in gs:
                g.ws.zero_()
            res = batch.solve(f1, f2, inits, graph=graph)
            for i, g in enumerate(gs):
                _same(alone[i], _outputs(g, *res[i]))
    finally:
        msgpm.tuning_set(**key, **saved)
    return gs


def test_batch_uneven_small_pairs_match_single_solves():
    msgpm = _need_gpu()
    pairs = [synth.tiny_pair(0), synth.planar_pair(160, 120, seed=3, scale=0.15),
             synth.planar_pair(97, 61, seed=4, scale=0.1), synth.tiny_pair(0)]
    base = _gpu_params(TINY_PARAMS)
    params = [dict(base), dict(base, seed=5), dict(base, seed=6, blocks=(20,)), dict(base, fp16=False, seed=9)]
    rng = np.random.default_rng(8)
    H, W = pairs[1].shape
    given = rng.integers(-40, 40, (2, H * W)).astype(np.int32)
    inits = [None, (torch.from_numpy((given[0] & 0xffff) | (given[1] << 16)), None), None, None]
    _run(msgpm, pairs, params, inits)


def test_batch_paper_sizes_match_single_solves():
    """Sizes of the batched workload (320x240 ... 1280x544), full parameters."""
    msgpm = _need_gpu()
    sizes = [(320, 240), (640, 360), (1024, 436), (1280, 544)]
    pairs = [synth.planar_pair(W, H, seed=100 + i, scale=W / 1024) for i, (W, H) in enumerate(sizes)]
    full = dict(C=5, r=4, blocks=(64, 32, 16), iters=8, hyps=256, tau=1.0, eps=0.1, tau_fb=1.0)
    params = [_gpu_params(dict(full, seed=100 + i, fp16=True)) for i in range(len(sizes))]
    _run(msgpm, pairs, params)


def test_batch_graph_serves_other_pairs_with_the_same_schedule():
    """The batched graph depends on the schedule and the table address only: a
    graph captured for one batch, replayed for a batch of other pairs (other
    sizes and number) through the same table buffer, gives each pair's lone
    result."""
    msgpm = _need_gpu()
    base = _gpu_params(TINY_PARAMS)
    first = [(synth.tiny_pair(0), dict(base)), (synth.planar_pair(160, 120, seed=3, scale=0.15), dict(base, seed=5))]
    second = [(synth.planar_pair(97, 61, seed=4, scale=0.1), dict(base, seed=6)),
              (synth.planar_pair(200, 144, seed=7, scale=0.1), dict(base, seed=7)),
              (synth.tiny_pair(0), dict(base, seed=8))]
    batches = []
    for scenes in (first, second):
        gs = [msgpm.Pair(pr.shape[1], pr.shape[0], **p) for pr, p in scenes]
        batches.append((scenes, gs, msgpm.Batch(gs)))
    big = max(b.scratch.numel() for _, _, b in batches)
    shared = torch.empty(big + 256, dtype=torch.uint8, device="cuda")
    ptr = ctypes.c_void_p(shared.data_ptr() + (-shared.data_ptr()) % 256)
    for scenes, gs, b in batches:
        b.scratch, b.scratch_ptr = shared, ptr
        res = b.solve([pr.frame1 for pr, _ in scenes], [pr.frame2 for pr, _ in scenes], graph=True)
        for (pr, p), g, r in zip(scenes, gs, res):
            alone = msgpm.Pair(pr.shape[1], pr.shape[0], **p)
            _same(_outputs(alone, *alone.solve(pr.frame1, pr.frame2)), _outputs(g, *r))


def test_batch_rejects_mixed_shapes():
    msgpm = _need_gpu()
    base = _gpu_params(TINY_PARAMS)
    gs = [msgpm.Pair(128, 96, **base), msgpm.Pair(128, 96, **dict(base, r=2))]
    with pytest.raises(msgpm.MsgpmError):
        msgpm.Batch(gs)


def test_batch_with_cues_filling_and_equalisation_matches_single_solves():
    msgpm = _need_gpu()
    pairs = [synth.tiny_pair(0), synth.planar_pair(97, 61, seed=4, scale=0.1)]
    base = _gpu_params(dict(TINY_PARAMS, cue_overlap=True, cue_unique=True, fill_sweeps=24, histeq=True))
    _run(msgpm, pairs, [dict(base), dict(base, seed=6, blocks=(20,))])


def test_batch_without_sweeps_matches_single_solves():
    """No PatchMatch iterations: the batch runs the passes' cost refreshes as
    launches of their own, as the single solve does."""
    msgpm = _need_gpu()
    pairs = [synth.tiny_pair(0), synth.planar_pair(97, 61, seed=4, scale=0.1)]
    base = _gpu_params(dict(TINY_PARAMS, iters=0))
    _run(msgpm, pairs, [dict(base), dict(base, seed=6, blocks=(20,))])


def test_batch_rejects_mixed_options():
    msgpm = _need_gpu()
    base = _gpu_params(TINY_PARAMS)
    for other in (dict(base, cue_unique=True), dict(base, fill_sweeps=8), dict(base, histeq=True)):
        gs = [msgpm.Pair(128, 96, **base), msgpm.Pair(128, 96, **other)]
        with pytest.raises(msgpm.MsgpmError):
            msgpm.Batch(gs)


def _against_oracle(pr, p, g, flows, occs):
    """A pair's free-running result against the oracle's whole solve of it: NNF
    and masks bit-exact outside flagged near-ties, EPE delta <= 0.01 px."""
    import oracle
    from tests import parity
    o = oracle.Oracle(pr.frame1, pr.frame2, variant="omp", **p)
    fo, oo = o.solve()
    torch.cuda.synchronize()
    for d in range(2):
        rep = parity.free_run_compare(o.nnf[d], oo[d], fo[d], o.pflag[d], g.nnf(d).cpu().numpy(),
                                      occs[d].cpu().numpy(), flows[d].cpu().numpy())
        print(d, rep)
        assert rep["nnf_unexplained"] == 0 and rep["occ_unexplained"] == 0 and rep["epe_delta"] <= 0.01, rep


def test_batch_fp16_pairs_against_oracle():
    """The batched FP16-storage form against the FP64 oracle directly (on the
    same FP16-rounded features): a 128x96 pair and a 160x120 pair of another
    scene, batched together."""
    msgpm = _need_gpu()
    scenes = [(synth.tiny_pair(0), dict(TINY_PARAMS, fp16=True)),
              (synth.planar_pair(160, 120, seed=3, scale=0.15), dict(TINY_PARAMS, fp16=True, seed=5))]
    gs = [msgpm.Pair(pr.shape[1], pr.shape[0], **_gpu_params(p)) for pr, p in scenes]
    res = msgpm.Batch(gs).solve([pr.frame1 for pr, _ in scenes], [pr.frame2 for pr, _ in scenes])
    for (pr, p), g, (flows, occs) in zip(scenes, gs, res):
        _against_oracle(pr, p, g, flows, occs)
