"""Pins of the oracle's restricted PatchMatch pass (Sec. 3.3.2) and of its
multi-level loop (Sec. 3.3: merge across levels, region plane carried from one
level to the next, random streams keyed by level), against closed forms,
constructed scenes and independent re-derivations.  CPU only.

Every expectation here comes from the scene's construction or from numpy
(its Philox generator, integer arithmetic), never from the GPU library."""
import numpy as np
import pytest

import oracle
from oracle import PI
from paper_1804_03787_amd import synth


def _minus_one(ctr):
    c = [int(v) for v in ctr]
    for i in range(4):
        if c[i] == 0:
            c[i] = 2**64 - 1
        else:
            c[i] -= 1
            break
    return np.array(c, dtype=np.uint64)


def _philox_block(ctr, seed):
    """Philox4x64-10 block of `ctr` under key (seed, 0), from numpy's own
    implementation (its counter advances before each block)."""
    bg = np.random.Philox(counter=_minus_one(ctr), key=np.array([seed, 0], dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def _draw(word, n):
    """Integer in [0, n) from the top 32 bits of a 64-bit word."""
    return ((word >> 32) * n) >> 32


def _search_offset(seed, p, k, it, d, slot, R):
    """Random-search offset of radius R: counter (pixel, radius index,
    iteration, phase 2 | direction | slot | stage 0)."""
    u = _philox_block([p, k, it, (2 << 24) | (d << 16) | (slot << 8)], seed)
    return _draw(u[0], 2 * R + 1) - R, _draw(u[1], 2 * R + 1) - R


def _shift_scene(W=48, H=40, s=(3, 2), **kw):
    """Frame 2 is frame 1 moved by the integer shift s: F2(p + s) = F1(p)."""
    pair = synth.smooth_pair(W, H, seed=81, shift=s)
    p = dict(C=3, r=2, grad_weight=0.0, blocks=(16,), iters=1, hyps=8, seed=5, R0=2)
    p.update(kw)
    return pair, oracle.Oracle(pair.frame1, pair.frame2, **p)


def _interior(W, H, r, s):
    ys, xs = np.divmod(np.arange(W * H), W)
    return (xs >= r) & (xs + s[0] + r <= W - 1) & (ys >= r) & (ys + s[1] + r <= H - 1)


# --------------------------------------------------------------------------
# Restricted pass (Sec. 3.3.2, readings R14-R16)
# --------------------------------------------------------------------------

def test_restricted_plane_candidate_takes_exact_match():
    """Every unassigned pixel carries a region plane equal to the scene's exact
    translation, and every offset starts 11 px off (so propagation offers only
    that wrong target).  The plane candidate is the exact match, whose cost is
    0, so after one restricted half-sweep each interior pixel of the colour
    holds the true offset with cost 0; the other colour is untouched."""
    s = (3, 2)
    W, H, r = 48, 40, 2
    pair, o = _shift_scene(W, H, s)
    k0 = o.plane_index(0, 0, 1, 0)
    o.pH[k0] = synth.translation(*s).ravel()
    o.hlabel[0][:] = k0
    o.set_nnf(0, oracle.pack(np.full(W * H, s[0] + 11), np.full(W * H, s[1] + 7)))
    o.eval_cost(0, 1)
    before = o.nnf[0].copy()
    o.pm_halfsweep(0, 0, 0, 1, 1)
    ys, xs = np.divmod(np.arange(W * H), W)
    sel = _interior(W, H, r, s) & ((xs + ys) % 2 == 0)
    dx, dy = oracle.unpack(o.nnf[0])
    assert sel.sum() > 300
    assert (dx[sel] == s[0]).all() and (dy[sel] == s[1]).all()
    assert (o.cost[0][sel] == 0.0).all()
    other = (xs + ys) % 2 == 1
    assert np.array_equal(o.nnf[0][other], before[other])


@pytest.mark.parametrize("slot", [1, 2])
def test_restricted_random_search_centred_after_plane_candidate(slot):
    """Random search is centred on the best offset after the plane candidate.
    A lone unassigned pixel p whose region plane sends it one draw away from the
    true match, (p + s) - o, where o is p's radius-1 random-search offset of
    this iteration and slot, taken from numpy's Philox: the plane candidate
    beats the wrong incumbent, and the random candidate centred on it lands
    exactly on p + s (cost 0).  Centred on the incumbent it would not.  The
    pass after level l uses slot l + 1; both slots are checked."""
    s = (3, 2)
    W, H, r, seed, it = 48, 40, 2, 5, 1
    pair, o = _shift_scene(W, H, s, R0=1, seed=seed)
    J = (s[0] + 9, s[1] - 6)
    o.set_nnf(0, oracle.pack(np.full(W * H, J[0]), np.full(W * H, J[1])))
    o.win[0][:] = 0                      # every pixel assigned but the test pixels
    interior = _interior(W, H, r, s)
    tested = []
    nwin = o.block_grid(0)[0] * o.block_grid(0)[1]
    for p in np.nonzero(interior)[0][::7]:
        x, y = int(p % W), int(p // W)
        if (x + y) % 2 or len(tested) == nwin:
            continue
        ox, oy = _search_offset(seed, int(p), 0, it, 0, slot, 1)
        if (ox, oy) == (0, 0):
            continue
        k = o.plane_index(0, 0, 1, len(tested))
        Hk = synth.translation(s[0] - ox, s[1] - oy)
        # precondition of the construction: the plane candidate beats the incumbent
        if not o.cost_at(0, x, y, x + s[0] - ox, y + s[1] - oy, Hk) < o.cost_at(0, x, y, x + J[0], y + J[1], Hk):
            continue
        o.pH[k] = Hk.ravel()
        o.hlabel[0][p] = k
        o.win[0][p] = -1
        tested.append(int(p))
    assert len(tested) >= 10
    o.eval_cost(0, 1)
    o.pm_halfsweep(0, 0, it, slot, 1)
    dx, dy = oracle.unpack(o.nnf[0])
    for p in tested:
        assert (dx[p], dy[p]) == s, p
        assert o.cost[0][p] == 0.0


def _ramp(W, H, a, b, c, t0=(0, 0), zoom=1):
    """Per-channel linear ramp F(x, y) = a x + b y + c seen through the map
    q = zoom p + t0: F2(q) = F1((q - t0) / zoom).  Dyadic coefficients keep every
    value exact in FP32."""
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    X, Y = (xs - t0[0]) / zoom, (ys - t0[1]) / zoom
    return np.stack([a[k] * X + b[k] * Y + c[k] for k in range(3)], axis=-1).astype(np.float32)


def test_restricted_incumbent_costed_under_region_plane():
    """Frame 2 is frame 1 (a linear ramp) zoomed by 2: the region plane
    H = 2p + t0 maps every tap to an integer pixel whose value is F1(p + d), so
    the incumbent offset Hp - p costs 0 under H (and 12.5 sum(a^2 + b^2) as a
    square patch, r = 2).  The refresh of the restricted pass costs the
    incumbent under H, so nothing beats it and no interior offset changes; a
    refresh under the identity would let the neighbour's target Hp - (1, 0),
    6.25 sum(a^2) under H, replace it."""
    W, H, r = 64, 48, 2
    t0 = (-10, -6)
    a = np.array([0.0078125, 0.01171875, -0.005859375])
    b = np.array([0.00390625, -0.0078125, 0.009765625])
    c = np.array([0.25, 0.5, 0.625])
    f1 = _ramp(W, H, a, b, c)
    f2 = _ramp(W, H, a, b, c, t0=t0, zoom=2)
    o = oracle.Oracle(f1, f2, C=3, r=r, grad_weight=0.0, blocks=(16,), iters=1, hyps=8, seed=3, R0=1)
    k0 = o.plane_index(0, 0, 1, 0)
    Hz = np.array([[2.0, 0, t0[0]], [0, 2.0, t0[1]], [0, 0, 1]])
    o.pH[k0] = Hz.ravel()
    o.hlabel[0][:] = k0
    ys, xs = np.divmod(np.arange(W * H), W)
    o.set_nnf(0, oracle.pack(xs + t0[0], ys + t0[1]))
    o.eval_cost(0, 1)
    inner = (xs >= 7) & (xs <= 34) & (ys >= 5) & (ys <= 24)
    assert (o.cost[0][inner] == 0.0).all()
    # the closed forms of the construction
    x, y = 20, 12
    t = (2 * x + t0[0], 2 * y + t0[1])
    ident = o.cost_at(0, x, y, t[0], t[1], None)
    assert ident == pytest.approx(12.5 * (a @ a + b @ b), rel=1e-12)
    left = o.cost_at(0, x, y, t[0] - 1, t[1], Hz)
    assert left == pytest.approx(6.25 * (a @ a), rel=1e-12)
    before = o.nnf[0].copy()
    for colour in range(2):
        o.pm_halfsweep(0, colour, 0, 1, 1)
    assert np.array_equal(o.nnf[0][inner], before[inner])
    assert (o.cost[0][inner] == 0.0).all()


# --------------------------------------------------------------------------
# Multi-level merge (Sec. 3.3, reading R11 and its strict form)
# --------------------------------------------------------------------------

def _layered_two_planes():
    """Integer-translation layers: left (+4, +2), right (-3, +1) for x >= 32."""
    W, H = 64, 48
    rng = np.random.default_rng(18)
    bg = synth.Layer(H=synth.translation(4, 2))
    right = synth.Layer(H=synth.translation(-3, 1), rect=(32, -1000, 1000, 1000))
    return synth.render([bg, right], W, H, rng)


def _two_level_oracle(pair, **kw):
    p = dict(C=3, r=2, grad_weight=0.0, blocks=(32, 16), iters=4, hyps=64, eps=0.1, seed=8)
    p.update(kw)
    return oracle.Oracle(pair.frame1, pair.frame2, **p)


def _exact_nnf(o, pair):
    H, W = pair.frame1.shape[:2]
    ys, xs = np.mgrid[0:H, 0:W]
    tx = np.floor(xs + pair.flow[..., 0] + 0.5).astype(int)
    ty = np.floor(ys + pair.flow[..., 1] + 0.5).astype(int)
    o.set_nnf(0, oracle.pack((tx - xs).ravel(), (ty - ys).ravel()))


def _covering(o, level, stage, x, y):
    nbx, nby = o.block_grid(level)
    out = []
    for b in range(nbx * nby):
        k = o.plane_index(0, level, stage, b)
        I = o.pinfo[k]
        if I[PI["x0"]] <= x < I[PI["x0"]] + I[PI["bw"]] and I[PI["y0"]] <= y < I[PI["y0"]] + I[PI["bh"]]:
            out.append(k)
    return out


@pytest.mark.parametrize("strict", [False, True])
def test_merge_across_levels(strict):
    """Level-0 plane A holds the left layer's pixels with a stored loss of 0.003
    (some with exactly 0); the level-1 fit on the exact NNF gives planes with
    loss 0 there.  Default key (L, level, stage, window): a level-1 plane
    replaces A exactly where its loss is strictly smaller, and at an exact tie
    the coarser level keeps the pixel.  Strict: an assigned pixel never
    changes; unassigned pixels take the minimum key either way."""
    pair = _layered_two_planes()
    W, H = 64, 48
    o = _two_level_oracle(pair, merge_strict=strict)
    _exact_nnf(o, pair)
    o.ransac(0, 1, 1)
    nb1 = o.block_grid(1)[0] * o.block_grid(1)[1]
    for b in range(nb1):
        k = o.plane_index(0, 1, 1, b)
        o.pinfo[k, PI["valid"]] = o.pinfo[k, PI["detected"]]
    kA = o.plane_index(0, 0, 1, 0)
    o.pH[kA] = synth.translation(4, 2).ravel()
    rng = np.random.default_rng(83)
    ys, xs = np.divmod(np.arange(W * H), W)
    held = (xs < 30) & (rng.random(W * H) < 0.8)
    tie = held & (rng.random(W * H) < 0.25)
    o.win[0][:] = np.where(held, kA, -1)
    o.loss[0][:] = np.where(tie, 0.0, np.where(held, 0.003, np.inf))
    win0, loss0 = o.win[0].copy(), o.loss[0].copy()
    o.assign(0, 1, 1, 0)
    eps2 = 0.1 * 0.1
    changed = 0
    for p in range(W * H):
        x, y = p % W, p // W
        best, bl = int(win0[p]), float(loss0[p])
        if not (strict and best >= 0):
            for k in _covering(o, 1, 1, x, y):     # window order: equal losses keep the earlier
                if not o.pinfo[k, PI["valid"]]:
                    continue
                e = o.colour_err(0, x, y, o.pH[k])
                if not e < eps2:
                    continue
                # an equal loss keeps the incumbent: a level-0 plane or an earlier window
                if best < 0 or e < bl:
                    best, bl = k, e
        assert o.win[0][p] == best, (p, o.win[0][p], best)
        changed += int(win0[p] >= 0 and best != win0[p])
    if strict:
        assert changed == 0
        assert np.array_equal(o.win[0][held], win0[held])
    else:
        assert changed > 100                       # the loss-0.003 pixels moved to level 1
        assert (o.win[0][tie] == kA).all()         # exact ties stay with the coarser level


@pytest.mark.parametrize("strict", [False, True])
def test_two_level_layered_solve(strict):
    """Whole two-level pipeline (windows 32 and 16) on two integer-translation
    layers, phase by phase, from the exact NNF of both directions.  Every
    pixel at least 6 px inside its layer and the frame, and not occluded, ends
    assigned, with a plane flow within half a pixel of its layer's motion
    (RANSAC keeps the first hypothesis of maximal count, which on these points
    need only be within the 1 px inlier threshold), so its NNF offset is the
    exact integer motion.  Strict: the level-1
    assignment changes no pixel assigned when it starts; default: a pixel
    leaves its level-0 plane only for a level-1 plane with a strictly smaller
    loss."""
    pair = _layered_two_planes()
    W, H = 64, 48
    o = _two_level_oracle(pair, merge_strict=strict, iters=2)
    _exact_nnf(o, pair)
    ys, xs = np.divmod(np.arange(W * H), W)
    right2 = xs >= 29                     # the right layer covers x >= 29 in frame 2
    o.set_nnf(1, oracle.pack(np.where(right2, 3, -4), np.where(right2, -1, -2)))
    moved = 0
    for name, args in o.schedule():
        if name == "assign" and args[0] == 1 and args[2] == 0:
            win0, loss0 = [w.copy() for w in o.win], [l.copy() for l in o.loss]
            o.run_step(name, args)
            for d in range(2):
                was, now = win0[d], o.win[d]
                kept = (was >= 0) & (now == was)
                if strict:
                    assert ((was < 0) | kept).all()
                else:
                    sw = (was >= 0) & (now != was)
                    moved += int(sw.sum())
                    assert (o.loss[d][sw] < loss0[d][sw]).all()
                    assert (o.pinfo[now[sw], PI["level"]] == 1).all()
            continue
        o.run_step(name, args)
    flows = [o.finalize(d) for d in range(2)]
    ys, xs = np.mgrid[0:H, 0:W]
    left = (xs >= 6) & (xs < 26) & (ys >= 6) & (ys < H - 6)
    right = (xs >= 38) & (xs < W - 6) & (ys >= 6) & (ys < H - 6)
    flow, occ = flows[0]
    ok = pair.occ == 0
    dx, dy = (v.reshape(H, W) for v in oracle.unpack(o.nnf[0]))
    for region, t in ((left, (4, 2)), (right, (-3, 1))):
        sel = region & ok
        assert sel.sum() > 300
        assert (occ[sel] == 0).all()
        assert np.abs(flow[sel] - np.array(t, np.float32)).max() < 0.5
        assert (dx[sel] == t[0]).all() and (dy[sel] == t[1]).all()
    if not strict:
        assert moved > 0


def test_region_label_inherited_across_levels():
    """After level 1's NNF update each pixel's region plane is, among the valid
    level-1 planes of both stages whose window contains it, the one with the
    largest count (ties: stage 1, then the lower window); where level 1 has
    none, the plane chosen at level 0 stays."""
    pair = _layered_two_planes()
    W, H = 64, 48
    o = _two_level_oracle(pair)
    _exact_nnf(o, pair)
    rng = np.random.default_rng(84)
    for lv in range(2):
        for st in (1, 2):
            nb = o.block_grid(lv)[0] * o.block_grid(lv)[1]
            for b in range(nb):
                k = o.plane_index(0, lv, st, b)
                o.pinfo[k, PI["valid"]] = int(rng.random() < (0.7 if lv == 0 else 0.35))
                o.pinfo[k, PI["count"]] = int(rng.integers(10, 14))
    o.hlabel[0][:] = -1
    o.nnf_update(0, 0)
    lab0 = o.hlabel[0].copy()
    assert (lab0 >= 0).mean() > 0.5
    o.nnf_update(0, 1)
    none = 0
    for p in range(W * H):
        x, y = p % W, p // W
        best, bc = int(lab0[p]), -1
        for st in (1, 2):
            for k in _covering(o, 1, st, x, y):
                if o.pinfo[k, PI["valid"]] and o.pinfo[k, PI["count"]] > bc:
                    best, bc = k, o.pinfo[k, PI["count"]]
        none += int(bc < 0)
        assert o.hlabel[0][p] == best, p
    assert none > 50


def _sample4(u, n):
    """Partial Fisher-Yates: four positions of a virtual identity permutation."""
    perm = {}
    sel = []
    for j in range(4):
        rj = j + _draw(u[j], n - j)
        vj, vr = perm.get(j, j), perm.get(rj, rj)
        perm[j], perm[rj] = vr, vj
        sel.append(vr)
    return sel


def _collinear(X, Y):
    for a, b, c in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
        if (X[b] - X[a]) * (Y[c] - Y[a]) - (Y[b] - Y[a]) * (X[c] - X[a]) == 0:
            return True
    return False


@pytest.mark.parametrize("level,stage", [(0, 1), (1, 1), (1, 2)])
def test_ransac_hypotheses_keyed_by_level_and_stage(level, stage):
    """The winning hypothesis of a window is the first of maximal inlier count
    among K draws, hypothesis h using the counter (window, h, 0, phase 3 |
    direction | slot level + 1 | stage).  Re-derived here with numpy's Philox,
    the Fisher-Yates rule and an inlier count in integers and FP64 (points on
    the grid, one exact plane and random outliers, 12 points per window)."""
    W = H = 16
    seed, K = 11, 24
    f = np.zeros((H, W, 3), np.float32)
    o = oracle.Oracle(f, f, C=3, r=1, blocks=(16, 16), iters=1, hyps=K, seed=seed, mu=0.0, m_min_abs=4)
    rng = np.random.default_rng(85 + 3 * level + stage)
    ys, xs = np.mgrid[0:H, 0:W]
    tx, ty = xs + 3, ys - 1
    # outliers at least 3 px from the plane, so no inlier decision is near the
    # threshold (where the rounding of the test, not the sampling, would decide)
    rx, ry = rng.integers(0, W, (H, W)), rng.integers(0, H, (H, W))
    bad = (rng.random((H, W)) < 0.5) & ((np.abs(rx - tx) >= 3) | (np.abs(ry - ty) >= 3))
    tx, ty = np.where(bad, rx, tx), np.where(bad, ry, ty)
    o.nnf[0][:] = oracle.pack((tx - xs).ravel(), (ty - ys).ravel())
    keep = np.sort(rng.choice(W * H, 12, replace=False))
    if stage == 2:
        o.win[0][:] = 3
        o.win[0][keep] = -1
        pts = keep
    else:
        pts = np.arange(W * H)
    o.ransac(0, level, stage)
    k = o.plane_index(0, level, stage, 0)
    src = np.stack([pts % W, pts // W], 1)
    dst = np.stack([tx.ravel()[pts], ty.ravel()[pts]], 1)
    n = len(pts)
    best, bestc = -1, -1
    for h in range(K):
        u = _philox_block([0, h, 0, (3 << 24) | (0 << 16) | ((level + 1) << 8) | stage], seed)
        sel = _sample4(u, n)
        S, D = src[sel], dst[sel]
        if _collinear(S[:, 0], S[:, 1]) or _collinear(D[:, 0], D[:, 1]):
            continue
        Hh = oracle.dlt4(S.astype(float), D.astype(float))
        if Hh is None:
            continue
        w = src @ Hh[2, :2] + Hh[2, 2]
        uv = src @ Hh[:2, :2].T + Hh[:2, 2]
        e2 = ((uv - w[:, None] * dst) ** 2).sum(1)
        c = int(((w > 0) & (e2 < w * w)).sum())
        if c > bestc:
            best, bestc = h, c
    assert o.pinfo[k, PI["support"]] == n
    assert o.pinfo[k, PI["hyp"]] == best
    assert o.pinfo[k, PI["hyp_count"]] == bestc


def test_solve_follows_the_documented_schedule():
    """The C driver of the whole pipeline (init pass, then per level the two
    plane stages, the FB check, the NNF update and the restricted pass keyed by
    slot level + 1) gives the same bits as the phase schedule run one step at
    a time, on two levels."""
    pair = synth.tiny_pair(0)
    p = dict(C=5, r=3, blocks=(32, 16), iters=2, hyps=32, seed=4)
    a = oracle.Oracle(pair.frame1, pair.frame2, **p)
    fa, oa = a.solve()
    b = oracle.Oracle(pair.frame1, pair.frame2, **p)
    b.nnf_init(0)
    b.nnf_init(1)
    for name, args in b.schedule():
        b.run_step(name, args)
    for d in range(2):
        fb, ob = b.finalize(d)
        assert np.array_equal(fa[d].view(np.uint32), fb.view(np.uint32))
        assert np.array_equal(oa[d], ob)
        assert np.array_equal(a.nnf[d], b.nnf[d]) and np.array_equal(a.hlabel[d], b.hlabel[d])
    assert np.array_equal(a.pH.view(np.uint64), b.pH.view(np.uint64))
    assert np.array_equal(a.pinfo, b.pinfo)


def test_openmp_build_is_bit_identical():
    """The OpenMP build of the oracle (phase loops shared among threads) gives
    the single-threaded build's bits: flows, masks, NNF, costs, labels, plane
    table, near-tie flags and the evaluation count, on two levels with both
    occlusion cues, the strict merge and the filling."""
    pair = synth.tiny_pair(0)
    p = dict(C=5, r=3, blocks=(32, 16), iters=3, hyps=48, seed=2, cue_overlap=True, cue_unique=True,
             fill_sweeps=16)
    for strict in (False, True):
        runs = []
        for variant in ("serial", "omp"):
            if variant == "omp":
                assert oracle.set_threads(4) == 4
            o = oracle.Oracle(pair.frame1, pair.frame2, variant=variant, merge_strict=strict, **p)
            flows, occs = o.solve()
            runs.append((flows, occs, o))
        (fa, oa, a), (fb, ob, b) = runs
        for d in range(2):
            assert np.array_equal(fa[d].view(np.uint32), fb[d].view(np.uint32))
            assert np.array_equal(oa[d], ob[d])
            for name in ("nnf", "win", "hlabel", "pflag"):
                assert np.array_equal(getattr(a, name)[d], getattr(b, name)[d]), name
            for name in ("cost", "loss"):
                assert np.array_equal(getattr(a, name)[d].view(np.uint64), getattr(b, name)[d].view(np.uint64)), name
        assert np.array_equal(a.pH.view(np.uint64), b.pH.view(np.uint64))
        assert np.array_equal(a.pinfo, b.pinfo) and np.array_equal(a.bflag, b.bflag)
        assert a.evals == b.evals
