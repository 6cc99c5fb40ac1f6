"""Serving (msgpm_server_*): pairs submitted while others are in flight are
admitted within an HBM budget and co-batched step by step with pairs at other
steps; each pair's outputs are bit-identical to a msgpm_solve of that pair
alone (GPU against GPU)."""
import numpy as np
import pytest
import torch

from paper_1804_03787_amd import synth
from tests.conftest import TINY_PARAMS
from tests.test_gpu_batch import _outputs, _same
from tests.test_gpu_parity import _gpu_params, _need_gpu

pytestmark = pytest.mark.gpu


def _scenes():
    base = _gpu_params(TINY_PARAMS)
    return [
        (synth.tiny_pair(0), dict(base)),
        (synth.planar_pair(160, 120, seed=3, scale=0.15), dict(base, seed=5)),
        (synth.planar_pair(97, 61, seed=4, scale=0.1), dict(base, seed=6, blocks=(20, 10))),
        (synth.planar_pair(200, 144, seed=7, scale=0.1), dict(base, seed=7, iters=3)),
        (synth.tiny_pair(0), dict(base, seed=8, blocks=(24, 12), cue_overlap=True, cue_unique=True,
                                  fill_sweeps=32)),
        (synth.planar_pair(128, 200, seed=9, scale=0.12), dict(base, seed=9, histeq=True)),
    ]


def test_serving_mix_matches_single_solves():
    msgpm = _need_gpu()
    scenes = _scenes()
    alone = []
    for pr, p in scenes:
        H, W = pr.shape
        g = msgpm.Pair(W, H, **p)
        alone.append(_outputs(g, *g.solve(pr.frame1, pr.frame2)))
    srv = msgpm.Server(hbm_budget=1 << 34, max_active=3)
    arrivals = {0: [0, 1], 5: [2, 3], 12: [4], 30: [5]}   # round -> scenes submitted before it
    tickets, done = {}, {}
    rnd = 0
    while len(done) < len(scenes):
        for k in arrivals.get(rnd, []):
            pr, p = scenes[k]
            H, W = pr.shape
            tickets[srv.submit(msgpm.Pair(W, H, **p), pr.frame1, pr.frame2)] = k
        srv.step()
        for t, k in list(tickets.items()):
            if srv.poll(t):
                g, flows, occs = srv.result(t)
                done[k] = _outputs(g, flows, occs)
                del tickets[t]
        rnd += 1
        assert rnd < 100000
    srv.close()
    for k in range(len(scenes)):
        _same(alone[k], done[k])


def test_serving_admission_by_budget_and_errors():
    msgpm = _need_gpu()
    scenes = _scenes()[:3]
    pairs = [msgpm.Pair(pr.shape[1], pr.shape[0], **p) for pr, p in scenes]
    sizes = [int(g.L.total_bytes) for g in pairs]
    # room for the largest pair only: the pairs run one after another
    srv = msgpm.Server(hbm_budget=max(sizes), max_active=8)
    ts = [srv.submit(g, pr.frame1, pr.frame2) for g, (pr, _) in zip(pairs, scenes)]
    pend = srv.step()
    assert pend == len(ts)
    finished = set()
    for _ in range(100000):
        srv.step()
        finished |= {t for t in ts if t not in finished and srv.poll(t)}
        if len(finished) == len(ts):
            break
    assert len(finished) == len(ts)
    for t in ts:
        srv.result(t)
    small = msgpm.Server(hbm_budget=min(sizes) - 1, max_active=2)
    pr, p = scenes[0]
    with pytest.raises(msgpm.MsgpmError):
        small.submit(msgpm.Pair(pr.shape[1], pr.shape[0], **p), pr.frame1, pr.frame2)
    other = dict(p, r=2)
    with pytest.raises(msgpm.MsgpmError):
        srv.submit(msgpm.Pair(pr.shape[1], pr.shape[0], **other), pr.frame1, pr.frame2)
    small.close()
    srv.close()
