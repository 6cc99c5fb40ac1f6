"""Python handle on the FP64 CPU oracle (oracle/msgpm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  Argument marshalling
only; every step of the method runs in the C oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "msgpm_oracle.c")
HDR = os.path.join(_HERE, "msgpm_oracle.h")
LIB = os.path.join(_HERE, "libmsgpm_oracle.so")
LIB_OMP = os.path.join(_HERE, "libmsgpm_oracle_omp.so")
# Single-threaded build: the parity authority.  An OpenMP build of the same
# source (LIB_OMP) shares the phase loops among threads and gives the same
# bits.  MSGPM_ORACLE_LIB names another single-threaded build to load instead
# (the mutation test points it at deliberately broken copies).
_LIB_ENV = "MSGPM_ORACLE_LIB"

PI_FIELDS = ["dir", "level", "stage", "block", "x0", "y0", "bw", "bh", "support", "count", "hyp",
             "hyp_count", "refit", "detected", "rk", "pass", "valid", "rin"]
PI = {n: i for i, n in enumerate(PI_FIELDS)}

F_COST, F_ROUND, F_COLOUR, F_FB, F_BOUNDS, F_RANSAC, F_TWOBEST = 1, 2, 4, 8, 16, 32, 64
B_RCOUNT, B_SYMCOUNT = 64, 128

DEFAULTS = dict(C=5, r=4, grad_weight=1.0, blocks=(64, 32, 16), iters=8, hyps=256, R0=0, tau=1.0, eps=0.1,
                tau_fb=1.0, mu=0.25, m_min_abs=8, eta=(1, 2), seed=0, fp16=False, cue_overlap=False,
                cue_unique=False, fill_sweeps=0, histeq=False, merge_strict=False)
CUE_OVERLAP, CUE_UNIQUE = 1, 2


def compile_oracle(src: str, out: str, openmp: bool = False, extra=(), verbose: bool = False) -> str:
    """Compiles one oracle source file into a shared library."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall", "-Wextra", "-Wno-unknown-pragmas", "-fPIC",
           "-shared", *(["-fopenmp"] if openmp else []), *extra, "-I", _HERE, "-o", out, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return out


def build(verbose: bool = False) -> str:
    compile_oracle(SRC, LIB, verbose=verbose)
    compile_oracle(SRC, LIB_OMP, openmp=True, verbose=verbose)
    return LIB


_libs = {}


def _stale(path: str) -> bool:
    return not os.path.exists(path) or os.path.getmtime(path) < max(os.path.getmtime(SRC), os.path.getmtime(HDR))


def lib(variant: str = "serial"):
    """The oracle library: "serial" (the parity authority) or "omp"."""
    if variant not in _libs:
        if variant == "serial" and os.environ.get(_LIB_ENV):
            path = os.environ[_LIB_ENV]
        else:
            path = LIB if variant == "serial" else LIB_OMP
            if _stale(path):
                compile_oracle(SRC, path, openmp=(variant == "omp"))
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(_Pair)
        vp = ctypes.c_void_p
        i = ctypes.c_int
        sig = {
            "orc_philox4x64": (None, [vp, vp, vp]),
            "orc_draw": (ctypes.c_uint32, [ctypes.c_uint64, ctypes.c_uint32]),
            "orc_features": (None, [vp, i, i, i, i, vp]),
            "orc_histeq": (None, [vp, i, i, vp]),
            "orc_round_fp16": (ctypes.c_float, [ctypes.c_float]),
            "orc_project": (i, [vp, ctypes.c_double, ctypes.c_double, vp, vp]),
            "orc_cost": (ctypes.c_double, [P, i, i, i, i, i, vp]),
            "orc_cost_all": (None, [P, i, vp]),
            "orc_block_count": (i, [i, i]),
            "orc_block_origin": (i, [i, i, i]),
            "orc_plane_capacity": (i, [P]),
            "orc_plane_index": (i, [P, i, i, i, i]),
            "orc_m_min": (i, [P, i, i]),
            "orc_planes_init": (None, [P]),
            "orc_nnf_init": (None, [P, i]),
            "orc_eval_cost": (None, [P, i, i]),
            "orc_pm_halfsweep": (None, [P, i, i, i, i, i]),
            "orc_ransac": (None, [P, i, i, i]),
            "orc_dlt4": (i, [vp, vp, vp, vp, vp]),
            "orc_refit": (i, [vp, vp, vp, vp, i, vp]),
            "orc_gauss_solve": (i, [vp, vp, i, vp]),
            "orc_colour_err": (ctypes.c_double, [P, i, i, i, vp, vp]),
            "orc_assign": (None, [P, i, i, i, i]),
            "orc_symmetry": (None, [P, i, i]),
            "orc_fb_test": (i, [P, i, i, i, vp, vp, vp]),
            "orc_fb_unassign": (None, [P]),
            "orc_unique": (None, [P]),
            "orc_fill": (None, [P]),
            "orc_nnf_update": (None, [P, i, i]),
            "orc_finalize": (None, [P, i, vp, vp]),
            "orc_solve": (None, [P, vp, vp, vp, vp, vp, vp]),
            "orc_set_threads": (i, [i]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _libs[variant] = L
    return _libs[variant]


def set_threads(n: int) -> int:
    """Threads of the OpenMP build's phase loops; returns the count in use."""
    return int(lib("omp").orc_set_threads(n))


class _Pair(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("C", ctypes.c_int32), ("r", ctypes.c_int32),
        ("wc", ctypes.c_double * 5),
        ("F", ctypes.c_void_p * 2),
        ("n_levels", ctypes.c_int32), ("block", ctypes.c_int32 * 8),
        ("iters", ctypes.c_int32), ("hyps", ctypes.c_int32), ("R0", ctypes.c_int32), ("m_min_abs", ctypes.c_int32),
        ("eta_num", ctypes.c_int32), ("eta_den", ctypes.c_int32),
        ("tau", ctypes.c_double), ("eps", ctypes.c_double), ("tau_fb", ctypes.c_double), ("mu", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("nnf", ctypes.c_void_p * 2), ("cost", ctypes.c_void_p * 2), ("win", ctypes.c_void_p * 2),
        ("loss", ctypes.c_void_p * 2), ("hlabel", ctypes.c_void_p * 2), ("twin", ctypes.c_void_p * 2),
        ("tloss", ctypes.c_void_p * 2), ("pflag", ctypes.c_void_p * 2),
        ("P", ctypes.c_int32), ("pH", ctypes.c_void_p), ("pinfo", ctypes.c_void_p), ("bflag", ctypes.c_void_p),
        ("evals", ctypes.c_int64), ("cues", ctypes.c_int32), ("fill_sweeps", ctypes.c_int32),
        ("merge_strict", ctypes.c_int32),
    ]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x64(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(word: int, n: int) -> int:
    return int(lib().orc_draw(ctypes.c_uint64(word), n))


def features(rgb: np.ndarray, C: int = 5, fp16: bool = False) -> np.ndarray:
    rgb = np.ascontiguousarray(rgb, dtype=np.float32)
    H, W, _ = rgb.shape
    out = np.zeros((H, W, C), dtype=np.float32)
    lib().orc_features(_ptr(rgb), W, H, C, int(fp16), _ptr(out))
    return out


def histeq(rgb: np.ndarray) -> np.ndarray:
    """HSV value-channel histogram equalisation of one HWC RGB frame."""
    rgb = np.ascontiguousarray(rgb, dtype=np.float32)
    H, W, _ = rgb.shape
    out = np.empty_like(rgb)
    lib().orc_histeq(_ptr(rgb), W, H, _ptr(out))
    return out


def round_fp16(x: float) -> float:
    return float(lib().orc_round_fp16(x))


def dlt4(src, dst):
    src = np.ascontiguousarray(src, dtype=np.float64)
    dst = np.ascontiguousarray(dst, dtype=np.float64)
    Hm = np.zeros(9)
    ok = lib().orc_dlt4(_ptr(np.ascontiguousarray(src[:, 0])), _ptr(np.ascontiguousarray(src[:, 1])),
                        _ptr(np.ascontiguousarray(dst[:, 0])), _ptr(np.ascontiguousarray(dst[:, 1])), _ptr(Hm))
    return Hm.reshape(3, 3) if ok else None


def refit(src, dst):
    src = np.ascontiguousarray(src, dtype=np.float64)
    dst = np.ascontiguousarray(dst, dtype=np.float64)
    cols = [np.ascontiguousarray(a) for a in (src[:, 0], src[:, 1], dst[:, 0], dst[:, 1])]
    Hm = np.zeros(9)
    ok = lib().orc_refit(*[_ptr(c) for c in cols], len(src), _ptr(Hm))
    return Hm.reshape(3, 3) if ok else None


def gauss_solve(A, b):
    A = np.ascontiguousarray(A, dtype=np.float64).copy()
    b = np.ascontiguousarray(b, dtype=np.float64).copy()
    x = np.zeros(len(b))
    ok = lib().orc_gauss_solve(_ptr(A), _ptr(b), len(b), _ptr(x))
    return x if ok else None


def pack(dx, dy) -> np.ndarray:
    dx = np.asarray(dx, dtype=np.int64)
    dy = np.asarray(dy, dtype=np.int64)
    return ((dx & 0xFFFF) | ((dy & 0xFFFF) << 16)).astype(np.uint32).view(np.int32)


def unpack(v):
    v = np.asarray(v).astype(np.int32).view(np.uint32)
    dx = (v & 0xFFFF).astype(np.uint16).view(np.int16).astype(np.int32)
    dy = (v >> 16).astype(np.uint16).view(np.int16).astype(np.int32)
    return dx, dy


class Oracle:
    """One frame pair with its full per-direction state, driven phase by phase
    or end to end.  Arrays are numpy and may be read or overwritten between
    phases (to feed identical state to another implementation).  variant
    "omp" runs the phases on the OpenMP build (same results, see lib())."""

    def __init__(self, frame1: np.ndarray, frame2: np.ndarray, variant: str = "serial", **params):
        p = dict(DEFAULTS)
        p.update(params)
        self._L = lib(variant)
        self.params = p
        self.Hh, self.Ww = frame1.shape[:2]
        H, W = self.Hh, self.Ww
        C = p["C"]
        if p["histeq"]:
            frame1, frame2 = histeq(frame1), histeq(frame2)
        self.feat = [features(frame1, C, p["fp16"]), features(frame2, C, p["fp16"])]
        n = W * H
        self.nnf = [np.zeros(n, np.int32) for _ in range(2)]
        self.cost = [np.zeros(n, np.float64) for _ in range(2)]
        self.win = [np.full(n, -1, np.int32) for _ in range(2)]
        self.loss = [np.full(n, np.inf) for _ in range(2)]
        self.hlabel = [np.full(n, -1, np.int32) for _ in range(2)]
        self.twin = [np.full(n, -1, np.int32) for _ in range(2)]
        self.tloss = [np.full(n, np.inf) for _ in range(2)]
        self.pflag = [np.zeros(n, np.uint8) for _ in range(2)]
        s = _Pair()
        s.W, s.H, s.C, s.r = W, H, C, p["r"]
        g = p["grad_weight"]
        for i, v in enumerate([1.0, 1.0, 1.0, g, g]):
            s.wc[i] = v
        blocks = list(p["blocks"])
        s.n_levels = len(blocks)
        for i, b in enumerate(blocks):
            s.block[i] = b
        s.iters, s.hyps, s.R0, s.m_min_abs = p["iters"], p["hyps"], p["R0"], p["m_min_abs"]
        s.eta_num, s.eta_den = p["eta"]
        s.tau, s.eps, s.tau_fb, s.mu = p["tau"], p["eps"], p["tau_fb"], p["mu"]
        s.seed = p["seed"]
        s.cues = (CUE_OVERLAP if p["cue_overlap"] else 0) | (CUE_UNIQUE if p["cue_unique"] else 0)
        s.fill_sweeps = p["fill_sweeps"]
        s.merge_strict = int(bool(p["merge_strict"]))
        self.s = s
        self._bind()
        P = self._L.orc_plane_capacity(ctypes.byref(s))
        s.P = P
        self.pH = np.zeros((P, 9), np.float64)
        self.pinfo = np.zeros((P, len(PI_FIELDS)), np.int32)
        self.bflag = np.zeros(P, np.uint8)
        s.pH, s.pinfo, s.bflag = _ptr(self.pH), _ptr(self.pinfo), _ptr(self.bflag)
        self._L.orc_planes_init(ctypes.byref(s))

    def _bind(self):
        s = self.s
        s.F[0], s.F[1] = _ptr(self.feat[0]), _ptr(self.feat[1])
        for d in range(2):
            s.nnf[d] = _ptr(self.nnf[d])
            s.cost[d] = _ptr(self.cost[d])
            s.win[d] = _ptr(self.win[d])
            s.loss[d] = _ptr(self.loss[d])
            s.hlabel[d] = _ptr(self.hlabel[d])
            s.twin[d] = _ptr(self.twin[d])
            s.tloss[d] = _ptr(self.tloss[d])
            s.pflag[d] = _ptr(self.pflag[d])

    @property
    def ref(self):
        self._bind()
        return ctypes.byref(self.s)

    @property
    def evals(self) -> int:
        return int(self.s.evals)

    # -- helpers ---------------------------------------------------------
    def plane_index(self, d, level, stage, block):
        return self._L.orc_plane_index(self.ref, d, level, stage, block)

    def block_grid(self, level):
        B = self.params["blocks"][level]
        return self._L.orc_block_count(self.Ww, B), self._L.orc_block_count(self.Hh, B)

    def m_min(self, bw, bh):
        return self._L.orc_m_min(self.ref, bw, bh)

    def cost_at(self, d, px, py, tx, ty, Hm=None):
        h = None if Hm is None else _ptr(np.ascontiguousarray(Hm, dtype=np.float64).reshape(9))
        return self._L.orc_cost(self.ref, d, px, py, tx, ty, h)

    def cost_all(self, d):
        n = self.Ww * self.Hh
        out = np.zeros(n * n)
        self._L.orc_cost_all(self.ref, d, _ptr(out))
        return out.reshape(n, n)

    def colour_err(self, d, px, py, Hm):
        h = np.ascontiguousarray(Hm, dtype=np.float64).reshape(9)
        nb = ctypes.c_int(0)
        return self._L.orc_colour_err(self.ref, d, px, py, _ptr(h), ctypes.byref(nb))

    # -- phases ----------------------------------------------------------
    def nnf_init(self, d):
        self._L.orc_nnf_init(self.ref, d)

    def set_nnf(self, d, nnf):
        """Install a caller-supplied NNF, clamping targets into the frame."""
        W, H = self.Ww, self.Hh
        dx, dy = unpack(np.asarray(nnf).reshape(-1))
        x = np.arange(W * H) % W
        y = np.arange(W * H) // W
        tx = np.clip(x + dx, 0, W - 1)
        ty = np.clip(y + dy, 0, H - 1)
        self.nnf[d][:] = pack(tx - x, ty - y)

    def eval_cost(self, d, mode):
        self._L.orc_eval_cost(self.ref, d, mode)

    def pm_halfsweep(self, d, colour, it, slot, restricted):
        self._L.orc_pm_halfsweep(self.ref, d, colour, it, slot, restricted)

    def pm_pass(self, slot, restricted):
        for it in range(self.params["iters"]):
            for colour in range(2):
                for d in range(2):
                    self.pm_halfsweep(d, colour, it, slot, restricted)

    def ransac(self, d, level, stage):
        self._L.orc_ransac(self.ref, d, level, stage)

    def assign(self, d, level, stage, tentative):
        self._L.orc_assign(self.ref, d, level, stage, int(tentative))

    def symmetry(self, level, stage):
        self._L.orc_symmetry(self.ref, level, stage)

    def fb_unassign(self):
        self._L.orc_fb_unassign(self.ref)

    def unique(self):
        self._L.orc_unique(self.ref)

    def fill(self):
        self._L.orc_fill(self.ref)

    def nnf_update(self, d, level):
        self._L.orc_nnf_update(self.ref, d, level)

    def finalize(self, d):
        W, H = self.Ww, self.Hh
        flow = np.zeros((H, W, 2), np.float32)
        occ = np.zeros((H, W), np.uint8)
        self._L.orc_finalize(self.ref, d, _ptr(flow), _ptr(occ))
        return flow, occ

    def reset_state(self):
        for d in range(2):
            self.win[d][:] = -1
            self.loss[d][:] = np.inf
            self.hlabel[d][:] = -1
            self.pflag[d][:] = 0
        self._L.orc_planes_init(self.ref)

    def solve(self, init_nnf=(None, None)):
        W, H = self.Ww, self.Hh
        flows = [np.zeros((H, W, 2), np.float32) for _ in range(2)]
        occs = [np.zeros((H, W), np.uint8) for _ in range(2)]
        inits = []
        for a in init_nnf:
            inits.append(None if a is None else np.ascontiguousarray(a, dtype=np.int32).reshape(-1))
        self._L.orc_solve(self.ref, None if inits[0] is None else _ptr(inits[0]),
                        None if inits[1] is None else _ptr(inits[1]), _ptr(flows[0]), _ptr(flows[1]),
                        _ptr(occs[0]), _ptr(occs[1]))
        return flows, occs

    def schedule(self):
        """Every phase of the pipeline after the initial state, in order, as
        (name, args) pairs covering both directions; run_step executes one."""
        p = self.params
        yield ("eval_cost", (0,))
        for it in range(p["iters"]):
            for colour in range(2):
                yield ("pm_halfsweep", (colour, it, 0, 0))
        for lv in range(len(p["blocks"])):
            for stage in (1, 2):
                yield ("ransac", (lv, stage))
                yield ("assign", (lv, stage, 1))
                yield ("symmetry", (lv, stage))
                yield ("assign", (lv, stage, 0))
            yield ("fb_unassign", ())
            if p["cue_unique"]:
                yield ("unique", ())
            yield ("nnf_update", (lv,))
            yield ("eval_cost", (1,))
            for it in range(p["iters"]):
                for colour in range(2):
                    yield ("pm_halfsweep", (colour, it, lv + 1, 1))
        if p["fill_sweeps"] > 0:
            yield ("fill", ())

    def run_step(self, name, args):
        if name in ("symmetry", "fb_unassign", "unique", "fill"):
            getattr(self, name)(*args)
            return
        for d in range(2):
            getattr(self, name)(d, *args)
