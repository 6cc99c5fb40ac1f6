"""Python binding of libmsgpm (C ABI in include/msgpm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libmsgpm.so.  PyTorch supplies device memory (the workspace and frame
buffers) and the current HIP stream.  There is no fallback: if the library is
not built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsgpm.so")
MAX_LEVELS = 8
FLAG_FP16 = 1
FLAG_CUE_OVERLAP = 2  # occlusion cue 3: plane kept only if its consistent pixels mostly match its RANSAC test
FLAG_CUE_UNIQUE = 4   # occlusion cue 2: one assigned pixel per target
FLAG_HISTEQ = 8       # equalise the frames' HSV value channel before the features
FLAG_MERGE_STRICT = 16  # strict level priority: a later level assigns only unassigned pixels
FLAG_ONE_STREAM = 32  # restricted half-sweeps' two launches in sequence on the caller's stream
SERVER_MAX_COHORTS = 4  # cohorts a server runs side by side at most (msgpm_server_set_cohorts)
PM_FRESH = 2          # pm_halfsweep: compute each swept pixel's current cost first (folds the cost refresh in)

STATUS = {0: "OK", 1: "E_INVALID", 2: "E_OOM", 3: "E_DEVICE", 4: "E_UNSUPPORTED", 5: "E_BUSY", 6: "E_CANCELLED",
          7: "E_TIMEOUT"}
E_INVALID, E_OOM, E_DEVICE, E_UNSUPPORTED, E_BUSY, E_CANCELLED, E_TIMEOUT = 1, 2, 3, 4, 5, 6, 7


class MsgpmError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("channels", ctypes.c_int32),
        ("patch_radius", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("block", ctypes.c_int32 * MAX_LEVELS),
        ("pm_iters", ctypes.c_int32), ("ransac_hyps", ctypes.c_int32), ("search_radius0", ctypes.c_int32),
        ("min_support_abs", ctypes.c_int32), ("eta_num", ctypes.c_int32), ("eta_den", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("fill_sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("grad_weight", ctypes.c_double), ("inlier_px", ctypes.c_double), ("eps_color", ctypes.c_double),
        ("fb_px", ctypes.c_double), ("min_support_frac", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


class Layout(ctypes.Structure):
    _fields_ = [
        ("total_bytes", ctypes.c_uint64), ("feat", ctypes.c_uint64 * 2), ("feat_bytes", ctypes.c_uint64),
        ("nnf", ctypes.c_uint64 * 2), ("cost", ctypes.c_uint64 * 2), ("win", ctypes.c_uint64 * 2),
        ("loss", ctypes.c_uint64 * 2), ("hlabel", ctypes.c_uint64 * 2), ("twin", ctypes.c_uint64 * 2),
        ("tloss", ctypes.c_uint64 * 2), ("planes", ctypes.c_uint64), ("counters", ctypes.c_uint64),
        ("histeq", ctypes.c_uint64), ("active", ctypes.c_uint64),
        ("n_planes", ctypes.c_int32), ("n_levels", ctypes.c_int32),
        ("level_blocks", ctypes.c_int32 * MAX_LEVELS), ("level_nbx", ctypes.c_int32 * MAX_LEVELS),
    ]


PLANE_INT_FIELDS = ["dir", "level", "stage", "block", "x0", "y0", "bw", "bh", "support", "count", "hyp",
                    "hyp_count", "refit", "detected", "rk", "pass", "valid", "rin"]
PLANE_DTYPE = np.dtype([("H", "<f8", (9,))] + [(f, "<i4") for f in PLANE_INT_FIELDS])
assert PLANE_DTYPE.itemsize == 144
assert ctypes.sizeof(Params) == 136

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1804_03787_amd.build` "
                               "(the HIP library is required: there is no CPU path)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(Params)
        vp, i = ctypes.c_void_p, ctypes.c_int
        sigs = {
            "msgpm_layout_query": [P, ctypes.POINTER(Layout)],
            "msgpm_solve": [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
            "msgpm_solve_graph": [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
            "msgpm_features": [P, vp, vp, vp, vp],
            "msgpm_init_state": [P, vp, vp, vp, vp],
            "msgpm_eval_cost": [P, vp, i, vp],
            "msgpm_pm_halfsweep": [P, vp, i, i, i, i, vp],
            "msgpm_ransac": [P, vp, i, i, vp],
            "msgpm_assign": [P, vp, i, i, i, vp],
            "msgpm_symmetry": [P, vp, i, i, vp],
            "msgpm_fb_unassign": [P, vp, vp],
            "msgpm_unique": [P, vp, vp],
            "msgpm_fill": [P, vp, vp],
            "msgpm_nnf_update": [P, vp, i, vp],
            "msgpm_finalize": [P, vp, vp, vp, vp, vp, vp],
            "msgpm_solve_static": [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.msgpm_batch_query.argtypes = [i, P, ctypes.POINTER(ctypes.c_uint64)]
        L.msgpm_batch_query.restype = ctypes.c_int
        L.msgpm_solve_batch.argtypes = [i, P] + [vp] * 11
        L.msgpm_solve_batch.restype = ctypes.c_int
        L.msgpm_solve_batch_graph.argtypes = [i, P] + [vp] * 11
        L.msgpm_solve_batch_graph.restype = ctypes.c_int
        L.msgpm_tuning_set.argtypes = [ctypes.POINTER(Tuning)]
        L.msgpm_tuning_set.restype = ctypes.c_int
        L.msgpm_tuning_get.argtypes = [ctypes.POINTER(Tuning)]
        L.msgpm_tuning_get.restype = ctypes.c_int
        u64, pu64 = ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)
        for name, args in {
            "msgpm_server_create": [u64, i, ctypes.POINTER(vp)],
            "msgpm_server_destroy": [vp],
            "msgpm_server_scratch_bytes": [i, pu64],
            "msgpm_server_submit": [vp, P] + [vp] * 9 + [pu64],
            "msgpm_server_step": [vp, vp, vp, ctypes.POINTER(i)],
            "msgpm_server_poll": [vp, u64, ctypes.POINTER(i)],
            "msgpm_server_cancel": [vp, u64, ctypes.POINTER(i)],
            "msgpm_server_wait": [vp, u64, ctypes.c_int64],
            "msgpm_server_set_queue_limit": [vp, i],
            "msgpm_server_set_cohorts": [vp, i],
            "msgpm_debug_fail_allocations": [i],
            "msgpm_check_fp16_arith": [i, vp, vp],
        }.items():
            getattr(L, name).argtypes = args
            getattr(L, name).restype = ctypes.c_int
        L.msgpm_graph_cache_clear.argtypes = []
        L.msgpm_graph_cache_clear.restype = ctypes.c_int
        L.msgpm_timing_enable.argtypes = [ctypes.c_int]
        L.msgpm_timing_enable.restype = ctypes.c_int
        L.msgpm_timing_read.argtypes = [vp, vp]
        L.msgpm_timing_read.restype = ctypes.c_int
        L.msgpm_last_error.restype = ctypes.c_char_p
        L.msgpm_last_error.argtypes = []
        _install_tuning(L)
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        raise MsgpmError(name, st, lib().msgpm_last_error().decode())


TIMER_KINDS = ["features", "init", "eval_cost", "pm_init", "pm_restricted", "ransac", "assign", "symmetry", "fb",
               "nnf_update", "finalize", "pm_list", "pm_restricted_ident", "fill"]


def graph_cache_clear():
    """Drops every cached HIP graph (msgpm_graph_cache_clear)."""
    _call("msgpm_graph_cache_clear")


def timing_enable(on: bool = True):
    _call("msgpm_timing_enable", int(on))


def timing_read() -> dict:
    """Milliseconds and launch counts per kernel kind since the last read."""
    ms = np.zeros(len(TIMER_KINDS), np.float64)
    n = np.zeros(len(TIMER_KINDS), np.int64)
    _call("msgpm_timing_read", ms.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(TIMER_KINDS)}


def make_params(width: int, height: int, *, C: int = 5, r: int = 4, blocks=(64, 32, 16), iters: int = 8,
                hyps: int = 256, R0: int = 0, tau: float = 1.0, eps: float = 0.1, tau_fb: float = 1.0,
                mu: float = 0.25, m_min_abs: int = 8, eta=(1, 2), seed: int = 0, fp16: bool = False,
                grad_weight: float = 1.0, cue_overlap: bool = False, cue_unique: bool = False,
                fill_sweeps: int = 0, histeq: bool = False, merge_strict: bool = False,
                one_stream: bool = False) -> Params:
    p = Params()
    p.width, p.height, p.channels, p.patch_radius = width, height, C, r
    blocks = list(blocks)
    p.n_levels = len(blocks)
    for k, b in enumerate(blocks):
        p.block[k] = b
    p.pm_iters, p.ransac_hyps, p.search_radius0, p.min_support_abs = iters, hyps, R0, m_min_abs
    p.eta_num, p.eta_den = eta
    p.flags = ((FLAG_FP16 if fp16 else 0) | (FLAG_CUE_OVERLAP if cue_overlap else 0) |
               (FLAG_CUE_UNIQUE if cue_unique else 0) | (FLAG_HISTEQ if histeq else 0) |
               (FLAG_MERGE_STRICT if merge_strict else 0) | (FLAG_ONE_STREAM if one_stream else 0))
    p.grad_weight, p.inlier_px, p.eps_color, p.fb_px, p.min_support_frac = grad_weight, tau, eps, tau_fb, mu
    p.seed = seed
    p.fill_sweeps = fill_sweeps
    return p


def layout(p: Params) -> Layout:
    L = Layout()
    _call("msgpm_layout_query", ctypes.byref(p), ctypes.byref(L))
    return L


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Pair:
    """Device state of one frame pair (one workspace) and the phase calls on it."""

    def __init__(self, width: int, height: int, device="cuda", **params):
        self.W, self.H = width, height
        self.p = make_params(width, height, **params)
        self.L = layout(self.p)
        self.device = torch.device(device)
        self.ws = torch.zeros(int(self.L.total_bytes), dtype=torch.uint8, device=self.device)
        assert self.ws.data_ptr() % 256 == 0
        self.n_planes = int(self.L.n_planes)

    # ---- views of the workspace -------------------------------------------
    def _view(self, off, count, dtype):
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.ws[int(off):int(off) + nbytes].view(dtype)

    def nnf(self, d):
        return self._view(self.L.nnf[d], self.W * self.H, torch.int32)

    def cost(self, d):
        return self._view(self.L.cost[d], self.W * self.H, torch.float32)

    def win(self, d):
        return self._view(self.L.win[d], self.W * self.H, torch.int32)

    def loss(self, d):
        return self._view(self.L.loss[d], self.W * self.H, torch.float64)

    def hlabel(self, d):
        return self._view(self.L.hlabel[d], self.W * self.H, torch.int32)

    def twin(self, d):
        return self._view(self.L.twin[d], self.W * self.H, torch.int32)

    def tloss(self, d):
        return self._view(self.L.tloss[d], self.W * self.H, torch.float64)

    def feat_bytes(self, f):
        return self.ws[int(self.L.feat[f]):int(self.L.feat[f]) + int(self.L.feat_bytes)]

    def planes_bytes(self):
        return self.ws[int(self.L.planes):int(self.L.planes) + self.n_planes * PLANE_DTYPE.itemsize]

    def planes(self) -> np.ndarray:
        return self.planes_bytes().cpu().numpy().view(PLANE_DTYPE).copy()

    def set_planes(self, arr: np.ndarray):
        assert arr.dtype == PLANE_DTYPE and len(arr) == self.n_planes
        self.planes_bytes().copy_(torch.from_numpy(arr.view(np.uint8).copy()).to(self.device))

    def counters(self) -> dict:
        """Warped-patch evaluations of the last pipeline run, per direction."""
        c = self._view(self.L.counters, 16 * 64, torch.int64).cpu().numpy().reshape(16, 64).sum(axis=1)
        return {"pm_init": c[0:2].tolist(), "eval_cost": c[2:4].tolist(), "pm_restricted": c[4:6].tolist(),
                "pm_init_rows": c[6:8].tolist(), "pm_restricted_rows": c[8:10].tolist(),
                "pm_restricted_ident": c[10:12].tolist(), "pm_restricted_ident_rows": c[12:14].tolist()}

    def features(self, f) -> np.ndarray:
        """Features of frame f as (H, W, C) float32 on the host."""
        n = self.W * self.H
        C = self.p.channels
        raw = self.feat_bytes(f)
        if self.p.flags & FLAG_FP16:
            S = 4 if C == 3 else 6
            h = raw[:n * S * 2].view(torch.float16).reshape(n, S).float().cpu().numpy()
            return np.ascontiguousarray(h[:, :C]).reshape(self.H, self.W, C)
        return raw[:n * C * 4].view(torch.float32).reshape(self.H, self.W, C).cpu().numpy().copy()

    # ---- phases --------------------------------------------------------------
    def _frame(self, f):
        t = torch.as_tensor(f)
        assert t.shape == (self.H, self.W, 3)
        return t.to(self.device, torch.float32).contiguous()

    def set_features(self, rgb1, rgb2):
        a, b = self._frame(rgb1), self._frame(rgb2)
        self._keep = (a, b)
        _call("msgpm_features", ctypes.byref(self.p), _ptr(a), _ptr(b), _ptr(self.ws), _stream())

    def init_state(self, init0=None, init1=None):
        i0 = None if init0 is None else torch.as_tensor(init0).to(self.device, torch.int32).contiguous()
        i1 = None if init1 is None else torch.as_tensor(init1).to(self.device, torch.int32).contiguous()
        _call("msgpm_init_state", ctypes.byref(self.p), _ptr(i0), _ptr(i1), _ptr(self.ws), _stream())

    def eval_cost(self, mode):
        _call("msgpm_eval_cost", ctypes.byref(self.p), _ptr(self.ws), mode, _stream())

    def pm_halfsweep(self, colour, it, slot, restricted):
        _call("msgpm_pm_halfsweep", ctypes.byref(self.p), _ptr(self.ws), colour, it, slot, int(restricted),
              _stream())

    def ransac(self, level, stage):
        _call("msgpm_ransac", ctypes.byref(self.p), _ptr(self.ws), level, stage, _stream())

    def assign(self, level, stage, tentative):
        _call("msgpm_assign", ctypes.byref(self.p), _ptr(self.ws), level, stage, int(tentative), _stream())

    def symmetry(self, level, stage):
        _call("msgpm_symmetry", ctypes.byref(self.p), _ptr(self.ws), level, stage, _stream())

    def fb_unassign(self):
        _call("msgpm_fb_unassign", ctypes.byref(self.p), _ptr(self.ws), _stream())

    def unique(self):
        _call("msgpm_unique", ctypes.byref(self.p), _ptr(self.ws), _stream())

    def fill(self):
        _call("msgpm_fill", ctypes.byref(self.p), _ptr(self.ws), _stream())

    def nnf_update(self, level):
        _call("msgpm_nnf_update", ctypes.byref(self.p), _ptr(self.ws), level, _stream())

    def finalize(self):
        flows = [torch.empty((self.H, self.W, 2), dtype=torch.float32, device=self.device) for _ in range(2)]
        occs = [torch.empty((self.H, self.W), dtype=torch.uint8, device=self.device) for _ in range(2)]
        _call("msgpm_finalize", ctypes.byref(self.p), _ptr(self.ws), _ptr(flows[0]), _ptr(flows[1]),
              _ptr(occs[0]), _ptr(occs[1]), _stream())
        return flows, occs

    def solve(self, rgb1, rgb2, init0=None, init1=None, out=None, graph=False):
        """Whole pipeline; returns ([flow0, flow1], [occ0, occ1]) as device tensors.
        graph: launch through a cached HIP graph of the whole sequence
        (msgpm_solve_graph; the frames, initial NNF and outputs must then be the
        same device buffers on every call for the cache to hit)."""
        a, b = self._frame(rgb1), self._frame(rgb2)
        i0 = None if init0 is None else torch.as_tensor(init0).to(self.device, torch.int32).contiguous()
        i1 = None if init1 is None else torch.as_tensor(init1).to(self.device, torch.int32).contiguous()
        if out is None:
            flows = [torch.empty((self.H, self.W, 2), dtype=torch.float32, device=self.device) for _ in range(2)]
            occs = [torch.empty((self.H, self.W), dtype=torch.uint8, device=self.device) for _ in range(2)]
        else:
            flows, occs = out
        _call("msgpm_solve_graph" if graph else "msgpm_solve", ctypes.byref(self.p), _ptr(a), _ptr(b), _ptr(i0),
              _ptr(i1), _ptr(self.ws),
              _ptr(flows[0]), _ptr(flows[1]), _ptr(occs[0]), _ptr(occs[1]), _stream())
        self._keep = (a, b, i0, i1)
        return flows, occs


STATIC_WS_BYTES = 64 << 20  # MSGPM_STATIC_WS_BYTES


def solve_static(p: Params, rgb1, rgb2, flows, occs, planes=None, init0=None, init1=None):
    """msgpm_solve_static: the whole pipeline in the library's static workspace
    (no allocation, no stream or event created).  rgb1, rgb2: device HWC
    float32 frames; flows, occs: device outputs as for Pair.solve; planes:
    optional device uint8 tensor of n_planes * 144 bytes for the plane table;
    init0/init1: optional device int32 initial NNFs.  Every argument is a
    caller-owned device tensor; nothing is allocated here."""
    _call("msgpm_solve_static", ctypes.byref(p), _ptr(rgb1), _ptr(rgb2), _ptr(init0), _ptr(init1),
          _ptr(flows[0]), _ptr(flows[1]), _ptr(occs[0]), _ptr(occs[1]), _ptr(planes), _stream())


class Tuning(ctypes.Structure):
    _fields_ = [("patch_radius", ctypes.c_int32), ("channels", ctypes.c_int32), ("fp16", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32 * 4)]


TUNE_CLASSES = ["pm_identity", "pm_distorted", "ransac", "pixel"]
TUNING_PATH = os.path.join(_HERE, "tuning.json")


def tuning_key(r: int, C: int, fp16: bool) -> str:
    return f"r{r}_C{C}_{'fp16' if fp16 else 'fp32'}"


def tuning_get(r: int = 0, C: int = 0, fp16=None) -> dict:
    """Resident workgroups per compute unit of the persistent batched launches
    that apply to instantiation (r, C, storage); 0 / 0 / None: the default."""
    t = Tuning()
    t.patch_radius, t.channels, t.fp16 = r, C, -1 if fp16 is None else int(fp16)
    _call("msgpm_tuning_get", ctypes.byref(t))
    return {k: int(t.wg_per_cu[i]) for i, k in enumerate(TUNE_CLASSES)}


def tuning_set(r: int = 0, C: int = 0, fp16=None, **wg_per_cu):
    """Stores a shape for instantiation (r, C, storage) (0 / 0 / None: the
    default); classes not given keep the value that applied so far."""
    cur = tuning_get(r, C, fp16)
    cur.update(wg_per_cu)
    t = Tuning()
    t.patch_radius, t.channels, t.fp16 = r, C, -1 if fp16 is None else int(fp16)
    for i, k in enumerate(TUNE_CLASSES):
        t.wg_per_cu[i] = int(cur[k])
    _call("msgpm_tuning_set", ctypes.byref(t))


def _install_tuning(L):
    """Installs the autotuner's stored choices (paper_1804_03787_amd/tuning.json,
    written by autotune.py), one entry per instantiation."""
    if not os.path.exists(TUNING_PATH):
        return
    import json
    for key, entry in json.load(open(TUNING_PATH)).get("choices", {}).items():
        t = Tuning()
        t.patch_radius, t.channels, t.fp16 = entry["r"], entry["C"], int(entry["fp16"])
        for i, k in enumerate(TUNE_CLASSES):
            t.wg_per_cu[i] = int(entry["wg_per_cu"][k])
        if L.msgpm_tuning_set(ctypes.byref(t)) != 0:
            raise MsgpmError("msgpm_tuning_set", 1, f"{TUNING_PATH}: entry {key}")


def check_fp16_arith(rounds: int = 256) -> tuple:
    """msgpm_check_fp16_arith on the current device: (differing results, results
    compared).  0 differing: the FP16 form's mixed-precision arithmetic gives
    the values of widening first."""
    import torch
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    _call("msgpm_check_fp16_arith", int(rounds), _ptr(out), _stream())
    torch.cuda.synchronize()
    return int(out.item()), 65536 * int(rounds) * 12


def debug_fail_allocations(n: int):
    """Test hook: the library's next n own allocations fail (E_OOM)."""
    _call("msgpm_debug_fail_allocations", int(n))


def solve(frame1, frame2, **params):
    """One-shot solve of a frame pair (numpy or torch HWC float32 frames)."""
    H, W = frame1.shape[:2]
    pair = Pair(W, H, **params)
    flows, occs = pair.solve(frame1, frame2)
    return pair, flows, occs


class Batch:
    """Several frame pairs solved together (msgpm_solve_batch): one launch per
    phase covers every pair.  pairs: Pair objects (their parameters and
    workspaces); they must share patch radius, channels, storage, iteration
    and level counts."""

    def __init__(self, pairs):
        self.pairs = list(pairs)
        n = len(self.pairs)
        self.params = (Params * n)(*[q.p for q in self.pairs])
        nbytes = ctypes.c_uint64()
        _call("msgpm_batch_query", n, self.params, ctypes.byref(nbytes))
        dev = self.pairs[0].device
        self.scratch = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
        off = (-self.scratch.data_ptr()) % 256
        self.scratch_ptr = ctypes.c_void_p(self.scratch.data_ptr() + off)
        self.flows = [[torch.empty((q.H, q.W, 2), dtype=torch.float32, device=dev) for _ in range(2)]
                      for q in self.pairs]
        self.occs = [[torch.empty((q.H, q.W), dtype=torch.uint8, device=dev) for _ in range(2)] for q in self.pairs]

    def solve(self, frames1, frames2, inits=None, graph=False):
        """Returns per pair ([flow0, flow1], [occ0, occ1]) as device tensors.
        graph: one HIP graph launch (msgpm_solve_batch_graph)."""
        n = len(self.pairs)
        a = [q._frame(f) for q, f in zip(self.pairs, frames1)]
        b = [q._frame(f) for q, f in zip(self.pairs, frames2)]
        arr = lambda ts: (ctypes.c_void_p * n)(*[None if t is None else t.data_ptr() for t in ts])
        i0 = i1 = None
        keep = [a, b]
        if inits is not None:
            t0 = [None if v is None or v[0] is None else torch.as_tensor(v[0]).to(q.device, torch.int32).contiguous()
                  for q, v in zip(self.pairs, inits)]
            t1 = [None if v is None or v[1] is None else torch.as_tensor(v[1]).to(q.device, torch.int32).contiguous()
                  for q, v in zip(self.pairs, inits)]
            i0, i1 = arr(t0), arr(t1)
            keep += [t0, t1]
        ws = arr([q.ws for q in self.pairs])
        _call("msgpm_solve_batch_graph" if graph else "msgpm_solve_batch", n, self.params, arr(a), arr(b), i0, i1, ws,
              arr([f[0] for f in self.flows]), arr([f[1] for f in self.flows]),
              arr([o[0] for o in self.occs]), arr([o[1] for o in self.occs]), self.scratch_ptr, _stream())
        self._keep = keep
        return list(zip(self.flows, self.occs))


class Server:
    """Continuous batching (msgpm_server_*): pairs submitted at any time are
    admitted within an HBM budget; each step admits the waiting pairs that fit
    as one cohort, whose whole batched pipeline is enqueued as one graph
    launch on one of the server's streams, beside the cohorts still running."""

    def __init__(self, hbm_budget: int, max_active: int, device="cuda"):
        self.device = torch.device(device)
        h = ctypes.c_void_p()
        _call("msgpm_server_create", int(hbm_budget), int(max_active), ctypes.byref(h))
        self.h = h
        nbytes = ctypes.c_uint64()
        _call("msgpm_server_scratch_bytes", int(max_active), ctypes.byref(nbytes))
        self.scratch = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        self.scratch_ptr = ctypes.c_void_p(self.scratch.data_ptr() + (-self.scratch.data_ptr()) % 256)
        self.jobs = {}

    def submit(self, pair: "Pair", rgb1, rgb2, init0=None, init1=None) -> int:
        a, b = pair._frame(rgb1), pair._frame(rgb2)
        i0 = None if init0 is None else torch.as_tensor(init0).to(self.device, torch.int32).contiguous()
        i1 = None if init1 is None else torch.as_tensor(init1).to(self.device, torch.int32).contiguous()
        flows = [torch.empty((pair.H, pair.W, 2), dtype=torch.float32, device=self.device) for _ in range(2)]
        occs = [torch.empty((pair.H, pair.W), dtype=torch.uint8, device=self.device) for _ in range(2)]
        t = ctypes.c_uint64()
        _call("msgpm_server_submit", self.h, ctypes.byref(pair.p), _ptr(a), _ptr(b), _ptr(i0), _ptr(i1),
              _ptr(pair.ws), _ptr(flows[0]), _ptr(flows[1]), _ptr(occs[0]), _ptr(occs[1]), ctypes.byref(t))
        self.jobs[t.value] = (pair, flows, occs, (a, b, i0, i1))
        return t.value

    def step(self) -> int:
        n = ctypes.c_int()
        _call("msgpm_server_step", self.h, self.scratch_ptr, _stream(), ctypes.byref(n))
        return n.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _call("msgpm_server_poll", self.h, int(ticket), ctypes.byref(d))
        return bool(d.value)

    def wait(self, ticket: int, timeout_us: int = -1):
        """msgpm_server_wait: returns once the pair is done (ticket retired);
        raises MsgpmError with status E_TIMEOUT (ticket still valid) or
        E_CANCELLED (retired)."""
        _call("msgpm_server_wait", self.h, int(ticket), int(timeout_us))

    def set_queue_limit(self, max_queued: int):
        _call("msgpm_server_set_queue_limit", self.h, int(max_queued))

    def set_cohorts(self, cohorts: int):
        """Largest number of cohorts in flight (msgpm_server_set_cohorts)."""
        _call("msgpm_server_set_cohorts", self.h, int(cohorts))

    def cancel(self, ticket: int) -> bool:
        """Cancels a pair; True if it was still queued and is gone already (an
        in-flight pair is reported done by poll once its enqueued work passed;
        its outputs are then undefined)."""
        r = ctypes.c_int()
        _call("msgpm_server_cancel", self.h, int(ticket), ctypes.byref(r))
        if r.value:
            self.jobs.pop(ticket, None)
        return bool(r.value)

    def result(self, ticket: int):
        """(pair, [flow0, flow1], [occ0, occ1]) of a finished ticket; forgets it."""
        pair, flows, occs, _ = self.jobs.pop(ticket)
        return pair, flows, occs

    def close(self):
        if self.h:
            _call("msgpm_server_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
