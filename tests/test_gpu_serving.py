"""Serving (msgpm_server_*): pairs submitted while others are in flight are
admitted within an HBM budget and co-batched step by step with pairs at other
steps; each pair's outputs are bit-identical to a msgpm_solve of that pair
alone (GPU against GPU); one served FP16-storage mix is also compared with
the oracle directly."""
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


@pytest.mark.parametrize("cohorts", [4, 1])
def test_serving_mix_matches_single_solves(cohorts):
    """Also with one cohort in flight at a time (msgpm_server_set_cohorts)."""
    msgpm = _need_gpu()
    scenes = _scenes()
    alone = []
    for pr, p in scenes:
        H, W = pr.shape
        g = msgpm.Pair(W, H, **p)
        alone.append(_outputs(g, *g.solve(pr.frame1, pr.frame2)))
    srv = msgpm.Server(hbm_budget=1 << 34, max_active=3)
    srv.set_cohorts(cohorts)
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


def test_serving_cancel_queued_and_in_flight():
    """A queued pair cancelled before admission is gone at once; an in-flight
    pair cancelled after its cohort was enqueued runs to its end, is reported
    done and returns its budget; the pair left running still matches its lone
    solve."""
    msgpm = _need_gpu()
    scenes = _scenes()[:3]
    alone = []
    for pr, p in scenes:
        g = msgpm.Pair(pr.shape[1], pr.shape[0], **p)
        alone.append(_outputs(g, *g.solve(pr.frame1, pr.frame2)))
    pairs = [msgpm.Pair(pr.shape[1], pr.shape[0], **p) for pr, p in scenes]
    srv = msgpm.Server(hbm_budget=1 << 34, max_active=2)
    ts = [srv.submit(g, pr.frame1, pr.frame2) for g, (pr, _) in zip(pairs, scenes)]
    assert srv.cancel(ts[2])            # third pair never admitted (two slots)
    with pytest.raises(msgpm.MsgpmError):
        srv.poll(ts[2])
    for _ in range(5):
        srv.step()
    assert not srv.cancel(ts[1])        # in flight: its enqueued work completes
    done = {}
    for _ in range(100000):
        pend = srv.step()
        for t in ts[:2]:
            if t not in done and srv.poll(t):
                done[t] = True
        if len(done) == 2:
            break
    # a step after both polls (the work may finish between a step and the polls)
    pend = srv.step()
    assert len(done) == 2 and pend == 0
    g, flows, occs = srv.result(ts[0])
    _same(alone[0], _outputs(g, flows, occs))
    srv.result(ts[1])
    # the cancelled pairs' budget is free again: the third pair now runs alone
    t = srv.submit(pairs[2], scenes[2][0].frame1, scenes[2][0].frame2)
    for _ in range(100000):
        srv.step()
        if srv.poll(t):
            break
    g, flows, occs = srv.result(t)
    _same(alone[2], _outputs(g, flows, occs))
    srv.close()


def test_served_fp16_pairs_against_oracle():
    """Pairs served with continuous batching (FP16 storage, the second
    submitted while the first is in flight) against the FP64 oracle directly."""
    from tests.test_gpu_batch import _against_oracle
    msgpm = _need_gpu()
    scenes = [(synth.tiny_pair(0), dict(TINY_PARAMS, fp16=True)),
              (synth.planar_pair(160, 120, seed=3, scale=0.15), dict(TINY_PARAMS, fp16=True, seed=5))]
    srv = msgpm.Server(hbm_budget=1 << 34, max_active=4)
    tickets, done = {}, {}
    rnd = 0
    while len(done) < len(scenes):
        if rnd in (0, 7):
            k = 0 if rnd == 0 else 1
            pr, p = scenes[k]
            tickets[srv.submit(msgpm.Pair(pr.shape[1], pr.shape[0], **_gpu_params(p)), pr.frame1, pr.frame2)] = k
        srv.step()
        for t, k in list(tickets.items()):
            if srv.poll(t):
                done[k] = srv.result(t)
                del tickets[t]
        rnd += 1
        assert rnd < 100000
    srv.close()
    for k, (pr, p) in enumerate(scenes):
        g, flows, occs = done[k]
        _against_oracle(pr, p, g, flows, occs)


def test_serving_wait_status_codes():
    """msgpm_server_wait: E_TIMEOUT while a pair is still being launched (the
    ticket stays valid), OK once its work has completed (outputs equal to the
    pair solved alone), E_CANCELLED for a pair cancelled in flight; the budget
    of both returns."""
    msgpm = _need_gpu()
    pr, p = _scenes()[0]
    H, W = pr.shape
    alone_g = msgpm.Pair(W, H, **p)
    alone = _outputs(alone_g, *alone_g.solve(pr.frame1, pr.frame2))
    srv = msgpm.Server(hbm_budget=1 << 34, max_active=4)
    keep = srv.submit(msgpm.Pair(W, H, **p), pr.frame1, pr.frame2)
    drop = srv.submit(msgpm.Pair(W, H, **dict(p, seed=3)), pr.frame1, pr.frame2)
    with pytest.raises(msgpm.MsgpmError) as e:
        srv.wait(keep, 1000)             # queued: not admitted before a step
    assert e.value.status == msgpm.E_TIMEOUT
    assert not srv.poll(keep)
    srv.step()                           # both admitted, their pipeline enqueued
    assert not srv.cancel(drop)          # in flight: runs to its end, reported cancelled
    while srv.step():
        pass
    srv.wait(keep, 10_000_000)
    g, flows, occs = srv.result(keep)
    _same(alone, _outputs(g, flows, occs))
    with pytest.raises(msgpm.MsgpmError) as e:
        srv.wait(drop, 10_000_000)
    assert e.value.status == msgpm.E_CANCELLED
    srv.jobs.pop(drop, None)
    srv.close()
