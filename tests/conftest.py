import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def tiny_pair():
    from paper_1804_03787_amd import synth
    return synth.tiny_pair(0)


TINY_PARAMS = dict(C=5, r=3, blocks=(16,), iters=4, hyps=64, tau=1.0, eps=0.1, tau_fb=1.0, seed=0)
