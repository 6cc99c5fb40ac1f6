"""Seeded synthetic frame pairs: piecewise-planar scenes with ground truth.

Stand-in for the MPI-Sintel frames the paper evaluates on (Sec. 4, 1024x436
frames), which are not available here.  A scene is a stack of textured planar
layers; each layer has a support region in frame 1 and a homography that moves
it to frame 2 (the piecewise-homography scene model of Sec. 3.1.1, Eq. 1).

Rendering rules:
  * texture: i.i.d. N(0, 1) per channel, separable Gaussian blur sigma = 2 px
    (radius 8, reflect), then per-channel min-max scaling to [0, 1];
  * frame 1 at pixel p takes the top layer whose support contains p;
  * frame 2 at pixel q takes the first layer (top first) whose inverse-mapped
    point H^-1 q lies in its support, sampled bilinearly in FP64;
  * ground-truth flow is H_layer(p) - p for the top layer at p; a pixel is
    occluded when its target leaves the frame or a higher layer covers it.

This module holds input synthesis only (no step of the matching method) and is
shared by the tests, the smoke check and the benchmark.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import ndimage


def translation(tx: float, ty: float) -> np.ndarray:
    return np.array([[1.0, 0.0, tx], [0.0, 1.0, ty], [0.0, 0.0, 1.0]])


def similarity_about(cx: float, cy: float, scale: float, theta_deg: float, tx: float = 0.0, ty: float = 0.0,
                     h6: float = 0.0, h7: float = 0.0) -> np.ndarray:
    """Scale + rotation about (cx, cy), optional perspective row, then translation."""
    t = math.radians(theta_deg)
    A = np.array([[scale * math.cos(t), -scale * math.sin(t), 0.0],
                  [scale * math.sin(t), scale * math.cos(t), 0.0],
                  [h6, h7, 1.0]])
    return translation(cx + tx, cy + ty) @ A @ translation(-cx, -cy)


@dataclasses.dataclass
class Layer:
    H: np.ndarray                       # frame 1 -> frame 2, 3x3
    rect: tuple | None = None           # (x0, y0, x1, y1) half-open, or None
    poly: np.ndarray | None = None      # convex polygon, counter-clockwise (y down), (k, 2)
    tex: np.ndarray | None = None       # texture canvas (h, w, 3) in frame-1 coordinates
    tex_origin: tuple = (0, 0)          # frame-1 coordinate of tex[0, 0]

    def inside(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        if self.rect is None and self.poly is None:
            return np.ones(np.shape(x), dtype=bool)
        if self.rect is not None:
            x0, y0, x1, y1 = self.rect
            return (x >= x0) & (x < x1) & (y >= y0) & (y < y1)
        P = self.poly
        ok = np.ones(np.shape(x), dtype=bool)
        for i in range(len(P)):
            ax, ay = P[i]
            bx, by = P[(i + 1) % len(P)]
            ok &= (bx - ax) * (y - ay) - (by - ay) * (x - ax) >= 0
        return ok

    def bbox(self, W: int, H: int, pad: int) -> tuple:
        if self.rect is None and self.poly is None:
            return (-pad, -pad, W + pad, H + pad)
        if self.rect is not None:
            x0, y0, x1, y1 = self.rect
        else:
            x0, y0 = self.poly.min(axis=0)
            x1, y1 = self.poly.max(axis=0)
        x0 = max(math.floor(x0) - 2, -pad)
        y0 = max(math.floor(y0) - 2, -pad)
        x1 = min(math.ceil(x1) + 3, W + pad)
        y1 = min(math.ceil(y1) + 3, H + pad)
        return (x0, y0, x1, y1)

    def sample(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        ox, oy = self.tex_origin
        u = x - ox
        v = y - oy
        h, w, _ = self.tex.shape
        u = np.clip(u, 0, w - 1)
        v = np.clip(v, 0, h - 1)
        u0 = np.clip(np.floor(u).astype(np.int64), 0, w - 2)
        v0 = np.clip(np.floor(v).astype(np.int64), 0, h - 2)
        fu = (u - u0)[..., None]
        fv = (v - v0)[..., None]
        T = self.tex
        return ((1 - fv) * ((1 - fu) * T[v0, u0] + fu * T[v0, u0 + 1]) +
                fv * ((1 - fu) * T[v0 + 1, u0] + fu * T[v0 + 1, u0 + 1]))


def make_texture(rng: np.random.Generator, h: int, w: int, sigma: float = 2.0) -> np.ndarray:
    noise = rng.standard_normal((h, w, 3))
    out = np.empty_like(noise)
    for c in range(3):
        out[..., c] = ndimage.gaussian_filter(noise[..., c], sigma=sigma, truncate=4.0, mode="reflect")
        lo, hi = out[..., c].min(), out[..., c].max()
        out[..., c] = (out[..., c] - lo) / (hi - lo)
    return out


@dataclasses.dataclass
class Pair:
    frame1: np.ndarray      # (H, W, 3) float32
    frame2: np.ndarray
    flow: np.ndarray        # (H, W, 2) float32 ground truth, frame 1 -> frame 2
    occ: np.ndarray         # (H, W) uint8 ground-truth occlusion
    layers: list
    gain: float = 1.0

    @property
    def shape(self):
        return self.frame1.shape[:2]


def _apply(Hm: np.ndarray, x: np.ndarray, y: np.ndarray):
    w = Hm[2, 0] * x + Hm[2, 1] * y + Hm[2, 2]
    return ((Hm[0, 0] * x + Hm[0, 1] * y + Hm[0, 2]) / w,
            (Hm[1, 0] * x + Hm[1, 1] * y + Hm[1, 2]) / w, w)


def render(layers: list, W: int, H: int, rng: np.random.Generator, pad: int = 256, gain: float = 1.0,
           textures: bool = True) -> Pair:
    """layers[0] is the background, later layers are higher in z-order."""
    if textures:
        for L in layers:
            x0, y0, x1, y1 = L.bbox(W, H, pad)
            L.tex = make_texture(rng, y1 - y0, x1 - x0)
            L.tex_origin = (x0, y0)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    top1 = _top_layer_frame1(layers, xs, ys)
    frame1 = np.zeros((H, W, 3))
    for i, L in enumerate(layers):
        m = top1 == i
        if m.any():
            frame1[m] = L.sample(xs[m], ys[m])
    top2, pre = _top_layer_frame2(layers, xs, ys)
    frame2 = np.zeros((H, W, 3))
    for i, L in enumerate(layers):
        m = top2 == i
        if m.any():
            frame2[m] = L.sample(pre[i][0][m], pre[i][1][m])
    frame2 *= gain
    flow, occ = ground_truth(layers, W, H, top1)
    return Pair(frame1.astype(np.float32), frame2.astype(np.float32), flow, occ, layers, gain)


def _top_layer_frame1(layers, xs, ys):
    top = np.zeros(xs.shape, dtype=np.int32)
    for i, L in enumerate(layers):
        top[L.inside(xs, ys)] = i
    return top


def _top_layer_frame2(layers, xs, ys):
    top = np.full(xs.shape, -1, dtype=np.int32)
    pre = {}
    for i in range(len(layers) - 1, -1, -1):
        L = layers[i]
        Hi = np.linalg.inv(L.H)
        px, py, w = _apply(Hi, xs, ys)
        pre[i] = (px, py)
        m = (top < 0) & (w > 0) & L.inside(px, py)
        top[m] = i
    top[top < 0] = 0
    return top, pre


def ground_truth(layers, W, H, top1=None, return_cover=False, step=1):
    ys, xs = np.mgrid[0:H:step, 0:W:step].astype(np.float64)
    if top1 is None:
        top1 = _top_layer_frame1(layers, xs, ys)
    flow = np.zeros(xs.shape + (2,))
    occ = np.zeros(xs.shape, dtype=np.uint8)
    qx = np.zeros(xs.shape)
    qy = np.zeros(xs.shape)
    for i, L in enumerate(layers):
        m = top1 == i
        if not m.any():
            continue
        a, b, _ = _apply(L.H, xs[m], ys[m])
        qx[m] = a
        qy[m] = b
    flow[..., 0] = qx - xs
    flow[..., 1] = qy - ys
    out = (qx < 0) | (qx > W - 1) | (qy < 0) | (qy > H - 1)
    # a pixel is visible in frame 2 only if its own layer is the top one at its target
    top_at_q = np.full(xs.shape, -1, dtype=np.int32)
    for i in range(len(layers) - 1, -1, -1):
        L = layers[i]
        px, py, w = _apply(np.linalg.inv(L.H), qx, qy)
        m = (top_at_q < 0) & (w > 0) & L.inside(px, py)
        top_at_q[m] = i
    occ[(top_at_q != top1) | out] = 1
    if return_cover:
        return flow.astype(np.float32), occ, top1, top_at_q, out
    return flow.astype(np.float32), occ


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def ground_truth_backward(layers, W, H):
    """Ground-truth flow from frame 2 to frame 1: a frame-2 pixel q belongs to
    the top layer whose pre-image H^-1 q lies in its support (the background
    otherwise), and moves to that pre-image."""
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    top2, pre = _top_layer_frame2(layers, xs, ys)
    flow = np.zeros((H, W, 2))
    for i in range(len(layers)):
        m = top2 == i
        flow[m, 0] = pre[i][0][m] - xs[m]
        flow[m, 1] = pre[i][1][m] - ys[m]
    return flow.astype(np.float32)


def tiny_pair(seed: int = 0) -> Pair:
    """128x96: background translated by (+5, +3); right half (x >= 64) zoomed by
    5 % and rotated by 3 degrees about (96, 48); a 20x20 occluder over
    [54, 74) x [38, 58) translated by (+12, 0)."""
    W, H = 128, 96
    rng = np.random.default_rng(seed)
    bg = Layer(H=translation(5, 3))
    right = Layer(H=similarity_about(96, 48, 1.05, 3.0), rect=(64, -10_000, 10_000, 10_000))
    occl = Layer(H=translation(12, 0), rect=(54, 38, 74, 58))
    return render([bg, right, occl], W, H, rng)


def _random_convex_quad(rng, W, H, rmin, rmax):
    while True:
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        rad = rng.uniform(rmin, rmax)
        ang = [(k + rng.uniform(0.0, 1.0)) * (math.pi / 2) for k in range(4)]
        pts = np.array([[cx + rad * rng.uniform(0.7, 1.0) * math.cos(a),
                         cy + rad * rng.uniform(0.7, 1.0) * math.sin(a)] for a in ang])
        # counter-clockwise in a y-down frame means the cross products are >= 0
        cr = []
        for i in range(4):
            a, b, c = pts[i], pts[(i + 1) % 4], pts[(i + 2) % 4]
            cr.append((b[0] - a[0]) * (c[1] - b[1]) - (b[1] - a[1]) * (c[0] - b[0]))
        if all(v > 0 for v in cr):
            return pts


def _random_motion(rng, cx, cy, tmax, persp=2e-5):
    return similarity_about(cx, cy, rng.uniform(0.9, 1.1), rng.uniform(-10, 10),
                            rng.uniform(-tmax, tmax), rng.uniform(-tmax, tmax),
                            rng.uniform(-persp, persp), rng.uniform(-persp, persp))


def planar_pair(W: int = 1024, H: int = 436, seed: int = 0, n_quads: int = 20, cam_t: float = 30.0,
                rel_t: float = 12.0, fg_t: float = 40.0, fg_occ: tuple = (0.045, 0.055),
                gain_range: tuple = (0.8, 1.2), max_tries: int = 400, scale: float = 1.0,
                independent: bool = False) -> Pair:
    """Piecewise-planar scene shaped like the paper's 1024x436 frames.

    * camera: a perspective similarity of the whole frame about its centre
      (translation up to cam_t px, scale 0.95-1.05, rotation up to 5 degrees,
      perspective terms up to 2e-5) applied to the background;
    * n_quads convex quads (radius 40-160 px) in random z-order, each moving
      with the camera composed with its own similarity about its centroid
      (translation up to rel_t px, scale 0.97-1.03, rotation up to 3 degrees):
      absolute displacements reach about 100 px at the frame border;
    * foreground quads (radius 20-80 px, own translation up to fg_t px) on
      top, added until the share of pixels hidden in frame 2 by a foreground
      quad lies in fg_occ;
    * frame 2 multiplied by a global gain drawn from gain_range.
    scale multiplies every length (radii, translations) for smaller instances.

    independent: the ranges written per quad instead, each motion drawn on its
    own and not relative to the camera: the background and every quad get a
    perspective similarity about their centre with translation up to 100 px,
    scale 0.9-1.1, rotation up to 10 degrees and perspective terms up to 2e-5
    (quads moving apart or across each other occlude far more of the frame
    than the foreground quads alone).
    """
    cam_t, rel_t, fg_t = cam_t * scale, rel_t * scale, fg_t * scale
    rng = np.random.default_rng(seed)
    if independent:
        cam = _random_motion(rng, W / 2, H / 2, 100.0 * scale)
    else:
        cam = similarity_about(W / 2, H / 2, rng.uniform(0.95, 1.05), rng.uniform(-5, 5),
                               rng.uniform(-cam_t, cam_t), rng.uniform(-cam_t, cam_t), rng.uniform(-2e-5, 2e-5),
                               rng.uniform(-2e-5, 2e-5))
    layers = [Layer(H=cam)]
    for _ in range(n_quads):
        q = _random_convex_quad(rng, W, H, 40 * scale, 160 * scale)
        c = q.mean(axis=0)
        if independent:
            layers.append(Layer(H=_random_motion(rng, c[0], c[1], 100.0 * scale), poly=q))
            continue
        rel = similarity_about(c[0], c[1], rng.uniform(0.97, 1.03), rng.uniform(-3, 3), rng.uniform(-rel_t, rel_t),
                               rng.uniform(-rel_t, rel_t))
        layers.append(Layer(H=cam @ rel, poly=q))
    n_base = len(layers)
    lo, hi = fg_occ

    def hidden_by_fg(ls):  # on every second pixel in x and y
        _, _, top1, top_q, out = ground_truth(ls, W, H, return_cover=True, step=2)
        return float(((top1 < n_base) & (top_q >= n_base) & ~out).mean())

    frac = 0.0
    tries = 0
    while frac < lo and tries < max_tries:
        tries += 1
        q = _random_convex_quad(rng, W, H, 20 * scale, 80 * scale)
        c = q.mean(axis=0)
        rel = similarity_about(c[0], c[1], 1.0, rng.uniform(-3, 3), rng.uniform(-fg_t, fg_t), rng.uniform(-fg_t, fg_t))
        cand = Layer(H=cam @ rel, poly=q)
        f = hidden_by_fg(layers + [cand])
        if f <= hi:
            layers.append(cand)
            frac = f
    gain = rng.uniform(*gain_range)
    return render(layers, W, H, rng, gain=gain)


def smooth_pair(W: int, H: int, seed: int, shift=(3, 2)) -> Pair:
    """Single textured plane translated by an integer shift (tests)."""
    rng = np.random.default_rng(seed)
    return render([Layer(H=translation(*shift))], W, H, rng)
