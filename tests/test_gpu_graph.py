"""msgpm_solve_graph: the whole pipeline captured once into a HIP graph and
replayed.  Every replay, with eager work of the program in between, must give
the eager msgpm_solve result bit for bit (GPU against GPU)."""
import numpy as np
import pytest
import torch

from paper_1804_03787_amd import synth
from tests.conftest import TINY_PARAMS
from tests.test_gpu_batch import _outputs, _same
from tests.test_gpu_parity import _gpu_params, _need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("size", ["tiny", "tiny_options", "1024x436"])
def test_graph_replays_match_eager(size):
    msgpm = _need_gpu()
    if size == "tiny":
        pr, p = synth.tiny_pair(0), _gpu_params(TINY_PARAMS)
    elif size == "tiny_options":
        pr, p = synth.tiny_pair(0), _gpu_params(dict(TINY_PARAMS, cue_overlap=True, cue_unique=True, fill_sweeps=48,
                                                      histeq=True))
    else:
        pr = synth.planar_pair(1024, 436, seed=0)
        p = _gpu_params(dict(C=5, r=4, blocks=(64, 32, 16), iters=8, hyps=256, tau=1.0, eps=0.1, tau_fb=1.0))
    H, W = pr.shape
    f1 = torch.from_numpy(pr.frame1).cuda()
    f2 = torch.from_numpy(pr.frame2).cuda()
    g = msgpm.Pair(W, H, **p)
    ref = _outputs(g, *g.solve(f1, f2))
    out = ([torch.empty((H, W, 2), device="cuda") for _ in range(2)],
           [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(2)])
    other = msgpm.Pair(128, 96, **_gpu_params(TINY_PARAMS))
    tiny = synth.tiny_pair(1)
    for rep in range(4):
        for d in range(2):
            out[0][d].fill_(float(rep) + 7.0)
            out[1][d].fill_(255)
        flows, occs = g.solve(f1, f2, out=out, graph=True)
        _same(ref, _outputs(g, flows, occs))
        # eager work of the program between the replays
        other.solve(tiny.frame1, tiny.frame2)
        torch.cuda.synchronize()
        _ = (f1 * 2.0).sum().item()
    msgpm.lib().msgpm_graph_cache_clear()
