"""CPU checks of the C-ABI library and of the oracle's regression anchor.

No GPU work: the library is loaded and its host-only entry points (parameter
validation, workspace layout, scratch sizes) are called; every function that
include/msgpm.h declares must be exported."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from paper_1804_03787_amd import msgpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "msgpm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:msgpm_status|const char\s*\*)\s*(msgpm_\w+)\s*\(", text, flags=re.M)))


def test_binding_constants_match_the_header():
    """Flag bits and status codes of the Python binding are the header's."""
    text = open(os.path.join(ROOT, "include", "msgpm.h")).read()
    flags = dict(re.findall(r"#define MSGPM_FLAG_(\w+) (\d+)u", text))
    assert flags, "no flags found"
    for name, v in flags.items():
        assert getattr(msgpm, "FLAG_" + name) == int(v), name
    codes = dict(re.findall(r"MSGPM_(OK|E_\w+) = (\d+)", text))
    assert len(codes) == 8
    for name, v in codes.items():
        assert msgpm.STATUS[int(v)] == name, name
    assert int(re.search(r"#define MSGPM_SERVER_MAX_COHORTS (\d+)", text).group(1)) == msgpm.SERVER_MAX_COHORTS


def test_one_stream_flag_is_accepted():
    p = msgpm.make_params(1024, 436, one_stream=True)
    assert p.flags & msgpm.FLAG_ONE_STREAM
    assert msgpm.layout(p).total_bytes == msgpm.layout(msgpm.make_params(1024, 436)).total_bytes


def test_library_exports_every_declared_function():
    names = _declared()
    assert len(names) >= 28, names
    lib = ctypes.CDLL(msgpm.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _layout(**kw):
    W = kw.pop("width", 1024)
    H = kw.pop("height", 436)
    n_levels = kw.pop("n_levels", None)
    p = msgpm.make_params(W, H, **kw)
    if n_levels is not None:
        p.n_levels = n_levels
    L = msgpm.Layout()
    st = msgpm.lib().msgpm_layout_query(ctypes.byref(p), ctypes.byref(L))
    return st, L


@pytest.mark.parametrize("bad", [
    dict(width=1), dict(height=40000), dict(C=4), dict(r=0), dict(r=5), dict(blocks=(3,)), dict(blocks=(129,)),
    dict(n_levels=9), dict(iters=-1), dict(hyps=0), dict(hyps=1025), dict(eta=(1, 0)), dict(tau=0.0),
    dict(eps=float("nan")), dict(fill_sweeps=-1), dict(fill_sweeps=70000),
])
def test_layout_query_rejects_bad_parameters(bad):
    st, _ = _layout(**bad)
    assert st != 0
    assert msgpm.lib().msgpm_last_error().decode()


def test_layout_query_rejects_unknown_flags():
    p = msgpm.make_params(64, 48)
    p.flags = 1 << 7
    assert msgpm.lib().msgpm_layout_query(ctypes.byref(p), ctypes.byref(msgpm.Layout())) != 0
    p.flags = msgpm.FLAG_MERGE_STRICT
    assert msgpm.lib().msgpm_layout_query(ctypes.byref(p), ctypes.byref(msgpm.Layout())) == 0
    p.flags = msgpm.FLAG_ONE_STREAM
    assert msgpm.lib().msgpm_layout_query(ctypes.byref(p), ctypes.byref(msgpm.Layout())) == 0
    p.flags = 1 << 6
    assert msgpm.lib().msgpm_layout_query(ctypes.byref(p), ctypes.byref(msgpm.Layout())) != 0
    assert b"flags" in msgpm.lib().msgpm_last_error()


@pytest.mark.parametrize("fp16,r,h_max", [(False, 4, 3272), (True, 1, 5460)])
def test_feature_offsets_limit_includes_patch_rows_past_the_frame(fp16, r, h_max):
    """Feature byte offsets are 32-bit and the identity-patch rows are offset
    before their clamp, up to r rows past the last: a 32767-wide frame is
    accepted up to the largest height with (W (H + r) + 1) * record bytes
    < 2^31 and refused (unsupported) one row above it."""
    W = 32767
    rec = 12 if fp16 else 20
    assert (W * (h_max + r) + 1) * rec <= 2**31 - 1 < (W * (h_max + 1 + r) + 1) * rec
    p = msgpm.make_params(W, h_max, fp16=fp16, r=r)
    assert msgpm.lib().msgpm_layout_query(ctypes.byref(p), ctypes.byref(msgpm.Layout())) == 0
    p = msgpm.make_params(W, h_max + 1, fp16=fp16, r=r)
    assert msgpm.lib().msgpm_layout_query(ctypes.byref(p), ctypes.byref(msgpm.Layout())) == msgpm.E_UNSUPPORTED
    assert b"exceed 2 GiB" in msgpm.lib().msgpm_last_error()


REGIONS = ["feat", "nnf", "cost", "win", "loss", "hlabel", "twin", "tloss", "planes", "counters", "histeq", "active"]


@pytest.mark.parametrize("kw", [dict(), dict(fp16=True), dict(C=3, grad_weight=0.0), dict(width=77, height=53,
                                blocks=(20, 12), r=2), dict(width=2048, height=872, blocks=(128, 64, 32, 16))])
def test_layout_regions_aligned_and_disjoint(kw):
    W, H = kw.get("width", 1024), kw.get("height", 436)
    st, L = _layout(**kw)
    assert st == 0, msgpm.lib().msgpm_last_error()
    C, fp16 = kw.get("C", 5), kw.get("fp16", False)
    rec = (8 if C == 3 else 12) if fp16 else 4 * C
    assert L.feat_bytes == (W * H + 1) * rec
    spans = []
    for name in REGIONS:
        v = getattr(L, name)
        offs = list(v) if hasattr(v, "__len__") else [v]
        for o in offs:
            assert o % 256 == 0, (name, o)
            spans.append((o, name))
    spans.sort()
    for (a, na), (b, nb) in zip(spans, spans[1:]):
        assert a < b, (na, nb)
    assert spans[-1][0] < L.total_bytes
    # plane records: two directions, two stages, every window of every level
    blocks = kw.get("blocks", (64, 32, 16))

    def count(n, B):
        return 1 if n <= B else (n - B) // (B // 2) + 1 + (1 if (n - B) % (B // 2) else 0)
    assert L.n_planes == 4 * sum(count(W, B) * count(H, B) for B in blocks)
    assert [L.level_blocks[i] for i in range(len(blocks))] == [count(W, B) * count(H, B) for B in blocks]


def test_server_scratch_bytes():
    nb = ctypes.c_uint64()
    assert msgpm.lib().msgpm_server_scratch_bytes(64, ctypes.byref(nb)) == 0
    assert nb.value > 0 and nb.value % 256 == 0
    assert msgpm.lib().msgpm_server_scratch_bytes(0, ctypes.byref(nb)) != 0


def test_oracle_matches_its_regression_anchor():
    """The oracle's whole solves on the exactly reproducible small input (one
    level; two levels with the default and the strict merge) equal the stored
    fixture (tests/golden/make_oracle_golden.py wrote it from oracle/)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_oracle_golden",
                                                  os.path.join(ROOT, "tests", "golden", "make_oracle_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    want = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_small_solve.json")))
    got = json.loads(json.dumps(mod.summary()))
    assert set(got) == set(want) == {"one_level", "two_levels", "two_levels_strict"}
    for case in want:
        assert got[case]["frames_sha256"] == want[case]["frames_sha256"]
        assert got[case] == want[case], case


def test_gather_ceiling_library_host_checks():
    """libmsgpm_ceiling (the benchmark's gather-ceiling kernel): grid size and
    argument checks run on the host; bad arguments launch nothing."""
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1804_03787_amd", "libmsgpm_ceiling.so"))
    lib.msgpm_ceiling_blocks.argtypes = [ctypes.c_int] * 3
    # one 9-lane group per pixel of one colour, 7 groups per wave, 4 waves per workgroup
    assert lib.msgpm_ceiling_blocks(1024, 436, 4) == -(-(512 * 436) // 28)
    assert lib.msgpm_ceiling_blocks(77, 53, 2) == -(-(39 * 53) // 48)
    assert lib.msgpm_ceiling_blocks(1, 436, 4) == -1 and lib.msgpm_ceiling_blocks(64, 64, 5) == -1
    lib.msgpm_ceiling_gather.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(0x10000000)
    assert lib.msgpm_ceiling_gather(fake, 64, 48, 4, 2, 0, 15, 1, fake, None) == -1  # 4-word records
    assert lib.msgpm_ceiling_gather(fake, 64, 48, 5, 2, 0, 0, 1, fake, None) == -1   # no patches
    assert lib.msgpm_ceiling_gather(None, 64, 48, 5, 2, 0, 15, 1, fake, None) == -1
