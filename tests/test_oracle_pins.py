"""Pins of the FP64 oracle against what the mathematics fixes: library routines,
closed forms, special cases, invariants and brute force.  CPU only."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import PI
from paper_1804_03787_amd import synth
from tests.conftest import TINY_PARAMS


# --------------------------------------------------------------------------
# RNG: Philox4x64-10 against numpy's independent implementation
# --------------------------------------------------------------------------

def _minus_one(ctr):
    c = [int(v) for v in ctr]
    for i in range(4):
        if c[i] == 0:
            c[i] = 2**64 - 1
        else:
            c[i] -= 1
            break
    return np.array(c, dtype=np.uint64)


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 2, 3, 4], [5, 6]),
    ([12288, 7, 3, (2 << 24) | (1 << 16) | (1 << 8)], [0, 0]),
    ([2**64 - 1] * 4, [2**64 - 1] * 2),
    ([0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89],
     [0x452821E638D01377, 0xBE5466CF34E90C6C]),
])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox bit generator advances its counter before each block
    bg = np.random.Philox(counter=_minus_one(ctr), key=np.array(key, dtype=np.uint64))
    assert np.array_equal(bg.random_raw(4), oracle.philox4x64(ctr, key))


def test_philox_many_counters():
    rng = np.random.default_rng(1)
    for _ in range(200):
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        bg = np.random.Philox(counter=_minus_one(ctr), key=key)
        assert np.array_equal(bg.random_raw(4), oracle.philox4x64(ctr, key))


def test_draw_range_and_power_of_two():
    rng = np.random.default_rng(2)
    words = rng.integers(0, 2**64, size=2000, dtype=np.uint64)
    for k in range(0, 12):
        n = 1 << k
        for w in words[:200]:
            # n = 2^k: the draw is the top k bits of the word
            assert oracle.draw(int(w), n) == (int(w) >> (64 - k) if k else 0)
    for n in (1, 3, 7, 2049, 1024 * 2 + 1):
        d = [oracle.draw(int(w), n) for w in words]
        assert min(d) >= 0 and max(d) < n


def test_draw_uniformity_chi2():
    # 2R+1 buckets as used by the random search, from Philox words
    n = 33
    counts = np.zeros(n)
    for i in range(3000):
        u = oracle.philox4x64([i, 0, 0, 2 << 24], [7, 0])
        for w in u:
            counts[oracle.draw(int(w), n)] += 1
    exp = counts.sum() / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 80  # 32 dof: P(chi2 > 80) < 1e-5


# --------------------------------------------------------------------------
# Features
# --------------------------------------------------------------------------

def test_fp16_rounding_matches_numpy():
    rng = np.random.default_rng(3)
    vals = np.concatenate([
        rng.uniform(-2, 2, 5000), rng.uniform(-1e-4, 1e-4, 2000), rng.uniform(-7e4, 7e4, 1000),
        np.array([0.0, -0.0, 65504.0, 65519.0, 65520.0, 6.1e-5, 5.96e-8, 2.98e-8, 2.99e-8, 1.0 + 2**-11,
                  1.0 + 3 * 2**-11, 0.5 + 2**-12]),
    ]).astype(np.float32)
    with np.errstate(over='ignore'):
        ref = vals.astype(np.float16).astype(np.float32)
    got = np.array([oracle.round_fp16(float(v)) for v in vals], dtype=np.float32)
    assert np.array_equal(ref.view(np.uint32), got.view(np.uint32))


def test_features_rgb_passthrough_and_gradients():
    rng = np.random.default_rng(4)
    rgb = rng.uniform(0, 1, (13, 17, 3)).astype(np.float32)
    f3 = oracle.features(rgb, C=3)
    assert np.array_equal(f3, rgb)
    # grey image: luma equals the grey value (weights sum to one) to 1 ulp
    grey = np.repeat(rng.uniform(0, 1, (13, 17, 1)), 3, axis=2).astype(np.float32)
    f5 = oracle.features(grey, C=5)
    Y = grey[..., 0]
    # interior central differences equal numpy.gradient (same float32 arithmetic up to the luma ulp)
    gx = np.gradient(Y.astype(np.float64), axis=1)
    gy = np.gradient(Y.astype(np.float64), axis=0)
    assert np.allclose(f5[:, 1:-1, 3], gx[:, 1:-1], atol=2e-7)
    assert np.allclose(f5[1:-1, :, 4], gy[1:-1, :], atol=2e-7)
    # replicate border: one-sided difference halved
    assert np.allclose(f5[:, 0, 3], 0.5 * gx[:, 0], atol=2e-7)
    assert np.allclose(f5[-1, :, 4], 0.5 * gy[-1, :], atol=2e-7)
    # pure red image: luma is 0.299 R
    red = np.zeros((5, 6, 3), np.float32)
    red[..., 0] = np.arange(6, dtype=np.float32)[None, :] * 0.25
    f = oracle.features(red, C=5)
    assert np.allclose(f[:, 2, 3], 0.299 * 0.25, rtol=1e-6)


# --------------------------------------------------------------------------
# Warped-patch SSD
# --------------------------------------------------------------------------

def _oracle_for(f1, f2, **kw):
    p = dict(C=3, r=3, grad_weight=0.0, blocks=(16,), iters=1, hyps=8)
    p.update(kw)
    return oracle.Oracle(f1, f2, **p)


def _square_ssd(F1, F2, p, t, r, w):
    P1 = np.pad(F1, ((r, r), (r, r), (0, 0)), mode="edge")
    P2 = np.pad(F2, ((r, r), (r, r), (0, 0)), mode="edge")
    (px, py), (tx, ty) = p, t
    a = P1[py:py + 2 * r + 1, px:px + 2 * r + 1]
    b = P2[ty:ty + 2 * r + 1, tx:tx + 2 * r + 1]
    return float(((a.astype(np.float64) - b) ** 2 * np.asarray(w)).sum())


def test_identity_cost_is_square_ssd():
    pair = synth.tiny_pair(0)
    o = _oracle_for(pair.frame1, pair.frame2, C=5, grad_weight=0.7)
    rng = np.random.default_rng(5)
    w = [1, 1, 1, 0.7, 0.7]
    for _ in range(300):
        px, tx = rng.integers(0, 128, 2)
        py, ty = rng.integers(0, 96, 2)
        c = o.cost_at(0, px, py, tx, ty)
        ref = _square_ssd(o.feat[0], o.feat[1], (px, py), (tx, ty), 3, w)
        assert abs(c - ref) <= 1e-12 * max(1.0, ref)
        # a translation has the same local distortion as the identity: bit-exact
        assert o.cost_at(0, px, py, tx, ty, synth.translation(3.0, -7.0)) == c


def test_integer_shift_zero_cost():
    pair = synth.smooth_pair(48, 40, seed=6, shift=(3, 2))
    o = _oracle_for(pair.frame1, pair.frame2)
    for y in range(5, 30):
        for x in range(5, 40):
            assert o.cost_at(0, x, y, x + 3, y + 2) == 0.0
            assert o.cost_at(1, x + 3, y + 2, x, y) == 0.0


def _ramp(W, H, alpha, beta, gamma):
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    return np.stack([a * xs + b * ys + g for a, b, g in zip(alpha, beta, gamma)], axis=-1).astype(np.float32)


def test_linear_ramp_closed_form_affine():
    W, H = 96, 80
    al, be, ga = (0.01, -0.004, 0.002), (0.003, 0.007, -0.005), (0.2, 0.5, 0.6)
    F = _ramp(W, H, al, be, ga)
    o = _oracle_for(F, F, r=4)
    rng = np.random.default_rng(7)
    f64 = F.astype(np.float64)
    for _ in range(60):
        A = np.eye(2) + rng.uniform(-0.15, 0.15, (2, 2))
        Hm = np.eye(3)
        Hm[:2, :2] = A
        Hm[:2, 2] = rng.uniform(-20, 20, 2)
        px, py = rng.integers(10, 80), rng.integers(10, 64)
        tx, ty = rng.integers(12, 80), rng.integers(12, 66)
        c = o.cost_at(0, px, py, tx, ty, Hm)
        # bilinear sampling reproduces a linear function exactly: cost is a closed form in A d
        ref = 0.0
        for dy in range(-4, 5):
            for dx in range(-4, 5):
                sx, sy = np.array([tx, ty]) + A @ np.array([dx, dy])
                for ch in range(3):
                    f1 = f64[py + dy, px + dx, ch]
                    f2 = al[ch] * sx + be[ch] * sy + ga[ch]
                    ref += (f1 - f2) ** 2
        # features are float32-rounded ramps: compare to a rounding-level tolerance
        assert abs(c - ref) <= 1e-9 + 1e-6 * ref


def test_projective_cost_matches_direct_sampling():
    """For a projective H the taps sit at t + pi(H(p+d)) - pi(Hp); on a linear
    ramp this gives the closed form with the projective displacement."""
    W, H = 96, 80
    al, be, ga = (0.02, 0.0, -0.01), (0.0, 0.015, 0.01), (0.1, 0.2, 0.9)
    F = _ramp(W, H, al, be, ga)
    o = _oracle_for(F, F, r=3)
    Hm = np.array([[1.02, 0.03, 4.0], [-0.02, 0.98, -3.0], [2e-4, -1e-4, 1.0]])
    f64 = F.astype(np.float64)

    def proj(x, y):
        v = Hm @ np.array([x, y, 1.0])
        return v[:2] / v[2]

    for (px, py, tx, ty) in [(40, 30, 44, 28), (20, 50, 25, 47), (60, 20, 58, 25)]:
        c = o.cost_at(0, px, py, tx, ty, Hm)
        base = proj(px, py)
        ref = 0.0
        for dy in range(-3, 4):
            for dx in range(-3, 4):
                s = np.array([tx, ty]) + (proj(px + dx, py + dy) - base)
                for ch in range(3):
                    ref += (f64[py + dy, px + dx, ch] - (al[ch] * s[0] + be[ch] * s[1] + ga[ch])) ** 2
        assert abs(c - ref) <= 1e-9 + 1e-6 * ref


def test_cost_nonnegative_and_infinite_behind_camera():
    pair = synth.tiny_pair(0)
    o = _oracle_for(pair.frame1, pair.frame2)
    Hm = np.array([[1, 0, 0], [0, 1, 0], [-0.02, 0, 1.0]])  # w <= 0 for x >= 50
    assert math.isinf(o.cost_at(0, 60, 40, 10, 10, Hm))
    assert o.cost_at(0, 10, 40, 10, 10, Hm) >= 0


def test_border_targets_replicate():
    pair = synth.tiny_pair(0)
    o = _oracle_for(pair.frame1, pair.frame2, r=3)
    for (p, t) in [((0, 0), (127, 95)), ((127, 0), (0, 95)), ((64, 95), (2, 1))]:
        ref = _square_ssd(o.feat[0], o.feat[1], p, t, 3, [1, 1, 1])
        assert abs(o.cost_at(0, *p, *t) - ref) <= 1e-12 * max(1, ref)


# --------------------------------------------------------------------------
# Homography estimation
# --------------------------------------------------------------------------

def _random_H(rng):
    Hm = np.eye(3)
    Hm[:2, :2] += rng.uniform(-0.2, 0.2, (2, 2))
    Hm[:2, 2] = rng.uniform(-30, 30, 2)
    Hm[2, :2] = rng.uniform(-3e-4, 3e-4, 2)
    return Hm


def _apply(Hm, pts):
    v = np.c_[pts, np.ones(len(pts))] @ Hm.T
    return v[:, :2] / v[:, 2:]


def test_dlt4_recovers_exact_homography():
    rng = np.random.default_rng(8)
    for _ in range(200):
        Hm = _random_H(rng)
        src = rng.uniform(0, 64, (4, 2))
        dst = _apply(Hm, src)
        got = oracle.dlt4(src, dst)
        assert got is not None
        assert np.abs(got - Hm / Hm[2, 2]).max() <= 1e-9 * np.abs(Hm).max()


def _square_to_quad(q):
    """Projective map of the unit square onto quad q (corners in order
    (0,0),(1,0),(1,1),(0,1)) by the textbook basis construction."""
    (x0, y0), (x1, y1), (x2, y2), (x3, y3) = q
    sx = x0 - x1 + x2 - x3
    sy = y0 - y1 + y2 - y3
    dx1, dx2, dy1, dy2 = x1 - x2, x3 - x2, y1 - y2, y3 - y2
    den = dx1 * dy2 - dx2 * dy1
    g = (sx * dy2 - dx2 * sy) / den
    h = (dx1 * sy - sx * dy1) / den
    return np.array([[x1 - x0 + g * x1, x3 - x0 + h * x3, x0],
                     [y1 - y0 + g * y1, y3 - y0 + h * y3, y0],
                     [g, h, 1.0]])


def test_dlt4_matches_projective_basis_construction():
    rng = np.random.default_rng(9)
    for _ in range(200):
        base = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
        src = base * 40 + rng.uniform(-6, 6, (4, 2)) + 10
        dst = base * 40 + rng.uniform(-6, 6, (4, 2)) + rng.uniform(0, 50, 2)
        ref = _square_to_quad(dst) @ np.linalg.inv(_square_to_quad(src))
        ref /= ref[2, 2]
        got = oracle.dlt4(src, dst)
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_dlt4_matches_numpy_solve():
    rng = np.random.default_rng(10)
    for _ in range(100):
        src = rng.uniform(0, 64, (4, 2))
        dst = src + rng.uniform(-5, 5, (4, 2)) + 10
        A = []
        b = []
        for (x, y), (u, v) in zip(src, dst):
            A.append([x, y, 1, 0, 0, 0, -x * u, -y * u])
            b.append(u)
            A.append([0, 0, 0, x, y, 1, -x * v, -y * v])
            b.append(v)
        h = np.linalg.solve(np.array(A), np.array(b))
        ref = np.append(h, 1.0).reshape(3, 3)
        got = oracle.dlt4(src, dst)
        assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_dlt4_rejects_degenerate():
    dst = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    same = np.array([[3, 3]] * 4, float)          # zero spread: normalisation fails
    assert oracle.dlt4(same, dst) is None
    line = np.array([[0, 0], [1, 1], [2, 2], [3, 3]], float)  # rank-deficient system
    assert oracle.dlt4(line, dst) is None


def _normalised(pts):
    c = pts - pts.mean(axis=0)
    return c * (math.sqrt(2) / np.sqrt((c ** 2).sum(1)).mean())


def test_refit_exact_and_lstsq():
    rng = np.random.default_rng(11)
    for _ in range(50):
        Hm = _random_H(rng)
        Hm /= Hm[2, 2]
        src = rng.uniform(0, 64, (30, 2))
        dst = _apply(Hm, src)
        got = oracle.refit(src, dst)
        assert np.abs(got - Hm).max() <= 1e-9 * np.abs(Hm).max()
    for _ in range(50):
        # on point sets that are already Hartley-normalised the refit is the
        # plain algebraic least-squares solution
        src = _normalised(rng.uniform(0, 64, (30, 2)))
        dst = _normalised(_apply(_random_H(rng), src * 20) + rng.normal(0, 0.3, (30, 2)))
        A, b = [], []
        for (x, y), (u, v) in zip(src, dst):
            A.append([x, y, 1, 0, 0, 0, -x * u, -y * u])
            b.append(u)
            A.append([0, 0, 0, x, y, 1, -x * v, -y * v])
            b.append(v)
        h = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)[0]
        ref = np.append(h, 1.0).reshape(3, 3)
        got = oracle.refit(src, dst)
        assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


def test_refit_similarity_equivariant():
    """Hartley normalisation makes the estimate commute with similarities of
    either image: refit(S1 x, S2 y) = S2 refit(x, y) S1^-1."""
    rng = np.random.default_rng(22)
    for _ in range(30):
        src = rng.uniform(0, 64, (40, 2))
        dst = _apply(_random_H(rng), src) + rng.normal(0, 0.5, (40, 2))
        S1 = synth.similarity_about(0, 0, rng.uniform(0.5, 2), rng.uniform(-90, 90), *rng.uniform(-50, 50, 2))
        S2 = synth.similarity_about(0, 0, rng.uniform(0.5, 2), rng.uniform(-90, 90), *rng.uniform(-50, 50, 2))
        base = oracle.refit(src, dst)
        moved = oracle.refit(_apply(S1, src), _apply(S2, dst))
        ref = S2 @ base @ np.linalg.inv(S1)
        ref /= ref[2, 2]
        pts = _apply(S1, src)
        assert np.abs(_apply(moved, pts) - _apply(ref, pts)).max() < 1e-7


def test_gauss_solve_matches_numpy():
    rng = np.random.default_rng(12)
    for n in (1, 2, 5, 8):
        for _ in range(30):
            A = rng.normal(size=(n, n)) + n * np.eye(n) * rng.uniform(0, 1)
            b = rng.normal(size=n)
            x = oracle.gauss_solve(A, b)
            assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-9)
    assert oracle.gauss_solve(np.zeros((3, 3)), np.ones(3)) is None


# --------------------------------------------------------------------------
# Blocks
# --------------------------------------------------------------------------

def test_block_grid_counts():
    o = oracle.Oracle(np.zeros((436, 1024, 3), np.float32), np.zeros((436, 1024, 3), np.float32), C=3,
                      blocks=(64, 32, 16), iters=1, hyps=1)
    assert o.block_grid(0) == (31, 13)
    assert o.block_grid(1) == (63, 27)
    assert o.block_grid(2) == (127, 54)
    t = synth.tiny_pair(0)
    o2 = oracle.Oracle(t.frame1, t.frame2, **TINY_PARAMS)
    assert o2.block_grid(0) == (15, 11)
    # last origin is flush with the border, origins cover every pixel
    lib = oracle.lib()
    for n, B in [(436, 64), (100, 16), (17, 16), (16, 16), (10, 16)]:
        m = lib.orc_block_count(n, B)
        origins = [lib.orc_block_origin(n, B, i) for i in range(m)]
        bw = min(B, n)
        assert origins[-1] + bw == n
        covered = np.zeros(n, bool)
        for o_ in origins:
            covered[o_:o_ + bw] = True
        assert covered.all()


# --------------------------------------------------------------------------
# RANSAC
# --------------------------------------------------------------------------

def _ransac_oracle(W, H, B, nnf_fn, hyps=64, seed=0, mu=0.25):
    f = np.zeros((H, W, 3), np.float32)
    o = oracle.Oracle(f, f, C=3, r=1, blocks=(B,), iters=1, hyps=hyps, seed=seed, mu=mu)
    ys, xs = np.mgrid[0:H, 0:W]
    tx, ty = nnf_fn(xs, ys)
    o.nnf[0][:] = oracle.pack((tx - xs).ravel(), (ty - ys).ravel())
    return o


@pytest.mark.parametrize("Hm", [
    np.array([[1, 0, 7], [0, 1, -3], [0, 0, 1]], float),
    np.array([[1, 1, 2], [0, 1, 5], [0, 0, 1]], float),        # integer shear
    np.array([[0, -1, 40], [1, 0, -2], [0, 0, 1]], float),      # 90 degree rotation
])
def test_ransac_exact_plane(Hm):
    W = H = 48

    def fn(xs, ys):
        return Hm[0, 0] * xs + Hm[0, 1] * ys + Hm[0, 2], Hm[1, 0] * xs + Hm[1, 1] * ys + Hm[1, 2]

    o = _ransac_oracle(W, H, 16, fn)
    o.ransac(0, 0, 1)
    nb = o.block_grid(0)[0] * o.block_grid(0)[1]
    for b in range(nb):
        k = o.plane_index(0, 0, 1, b)
        assert o.pinfo[k, PI["count"]] == 256
        assert np.abs(o.pH[k].reshape(3, 3) - Hm).max() <= 1e-9 * np.abs(Hm).max()


@pytest.mark.parametrize("exact", [True, False])
def test_ransac_half_outliers(exact):
    """50 % uniform outliers: with an integer-preserving plane every all-inlier
    sample recovers H exactly (P(no such sample in 256) ~ (15/16)^256 ~ 7e-8);
    with a rounded non-integer plane the fit stays within rounding error."""
    W = H = 64
    if exact:
        Hm = np.array([[1.0, 1.0, 6.0], [0.0, 1.0, 4.0], [0, 0, 1]])
    else:
        Hm = np.array([[1.03, 0.02, 6.0], [-0.02, 0.97, 4.0], [0, 0, 1]])
    rng = np.random.default_rng(13)
    bad = rng.random((H, W)) < 0.5
    rx, ry = rng.integers(0, W, (H, W)), rng.integers(0, H, (H, W))

    def fn(xs, ys):
        u = np.floor(Hm[0, 0] * xs + Hm[0, 1] * ys + Hm[0, 2] + 0.5).astype(int)
        v = np.floor(Hm[1, 0] * xs + Hm[1, 1] * ys + Hm[1, 2] + 0.5).astype(int)
        if exact:
            # outliers at least 3 px from the plane, so none is an accidental inlier
            far = (np.abs(rx - u) >= 3) | (np.abs(ry - v) >= 3)
            return np.where(bad & far, rx, np.where(bad, u + 5, u)), np.where(bad, ry, v)
        return np.where(bad, rx, u), np.where(bad, ry, v)

    o = _ransac_oracle(W, H, 32, fn, hyps=256)
    o.ransac(0, 0, 1)
    for b in range(9):
        k = o.plane_index(0, 0, 1, b)
        assert o.pinfo[k, PI["detected"]] == 1
        got = o.pH[k].reshape(3, 3)
        x0, y0 = o.pinfo[k, PI["x0"]], o.pinfo[k, PI["y0"]]
        if exact:
            good = ~bad[y0:y0 + 32, x0:x0 + 32]
            assert np.abs(got - Hm).max() <= 1e-9 * np.abs(Hm).max()
            assert o.pinfo[k, PI["count"]] >= good.sum()
        else:
            pts = np.array([[x, y] for x in range(x0, x0 + 32, 2) for y in range(y0, y0 + 32, 2)], float)
            err = np.linalg.norm(_apply(got, pts) - _apply(Hm, pts), axis=1)
            assert err.mean() < 0.5 and err.max() < 1.5


def test_ransac_brute_force_tiny():
    """On point sets of <= 10 points the hypothesis count never exceeds the best
    4-subset, and K = 256 draws reach it."""
    W = H = 16
    rng = np.random.default_rng(14)
    for trial in range(6):
        f = np.zeros((H, W, 3), np.float32)
        o = oracle.Oracle(f, f, C=3, r=1, blocks=(16,), iters=1, hyps=256, seed=trial, mu=0.0, m_min_abs=4)
        tx = rng.integers(0, W, (H, W))
        ty = rng.integers(0, H, (H, W))
        ys, xs = np.mgrid[0:H, 0:W]
        # some points on a plane
        tx[:4, :] = xs[:4, :] + 2
        ty[:4, :] = ys[:4, :] + 1
        o.nnf[0][:] = oracle.pack((tx - xs).ravel(), (ty - ys).ravel())
        keep = rng.choice(W * H, size=9, replace=False)
        o.win[0][:] = 7  # everything assigned ...
        o.win[0][keep] = -1  # ... except a residual of 9 pixels
        o.ransac(0, 0, 2)
        k = o.plane_index(0, 0, 2, 0)
        pts = [(int(p % W), int(p // W)) for p in sorted(keep)]
        src = np.array(pts, float)
        dst = np.array([(x + oracle.unpack(o.nnf[0][y * W + x])[0], y + oracle.unpack(o.nnf[0][y * W + x])[1])
                        for x, y in pts], float)
        best = 0
        for sub in itertools.combinations(range(len(pts)), 4):
            Hs = oracle.dlt4(src[list(sub)], dst[list(sub)])
            if Hs is None:
                continue
            w = src @ Hs[2, :2] + Hs[2, 2]
            uv = src @ Hs[:2, :2].T + Hs[:2, 2]
            e2 = ((uv - w[:, None] * dst) ** 2).sum(1)
            c = int(((w > 0) & (e2 < w * w)).sum())
            best = max(best, c)
        assert o.pinfo[k, PI["hyp_count"]] <= best
        assert o.pinfo[k, PI["hyp_count"]] == best
        assert o.pinfo[k, PI["count"]] >= o.pinfo[k, PI["hyp_count"]] or o.pinfo[k, PI["refit"]] == 0


def test_ransac_deterministic():
    pair = synth.tiny_pair(0)
    runs = []
    for _ in range(2):
        o = oracle.Oracle(pair.frame1, pair.frame2, **TINY_PARAMS)
        o.nnf_init(0)
        o.ransac(0, 0, 1)
        runs.append((o.pH.copy(), o.pinfo.copy()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])


# --------------------------------------------------------------------------
# PatchMatch
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shift,noise", [((0, 0), 0.0), ((2, 1), 0.01), ((-3, 2), 0.02)])
def test_patchmatch_converges_to_exhaustive_search(shift, noise):
    """32x32: iterating the init pass reaches the global minimum of the
    square-patch SSD found by exhaustive search, wherever the true match lies in
    the frame (border pixels whose match left the frame have isolated minima
    that random search need not hit)."""
    pair = synth.smooth_pair(32, 32, seed=15, shift=shift)
    f2 = pair.frame2 + np.random.default_rng(23).normal(0, noise, pair.frame2.shape).astype(np.float32)
    o = oracle.Oracle(pair.frame1, f2, C=3, r=2, grad_weight=0.0, blocks=(16,), iters=32, hyps=8, seed=3)
    o.nnf_init(0)
    o.eval_cost(0, 0)
    for it in range(32):
        for colour in range(2):
            o.pm_halfsweep(0, colour, it, 0, 0)
    allc = o.cost_all(0)
    best = allc.min(axis=1)
    n = 32 * 32
    xs, ys = np.arange(n) % 32, np.arange(n) // 32
    inside = (xs + shift[0] >= 0) & (xs + shift[0] < 32) & (ys + shift[1] >= 0) & (ys + shift[1] < 32)
    assert np.array_equal(o.cost[0][inside], best[inside])
    assert (o.cost[0] == best).mean() > 0.98
    assert (o.cost[0] >= best).all()
    dx, dy = oracle.unpack(o.nnf[0])
    t = (ys + dy) * 32 + (xs + dx)
    unique = (allc == best[:, None]).sum(1) == 1
    sel = unique & inside
    assert np.array_equal(t[sel], allc.argmin(axis=1)[sel])


def test_halfsweep_reads_only_other_colour():
    pair = synth.tiny_pair(0)
    o = oracle.Oracle(pair.frame1, pair.frame2, **TINY_PARAMS)
    o.nnf_init(0)
    o.eval_cost(0, 0)
    nnf0, cost0 = o.nnf[0].copy(), o.cost[0].copy()
    o.pm_halfsweep(0, 0, 0, 0, 0)
    out_a = o.nnf[0].copy()
    # scramble colour-0 pixels (the ones being updated) except a probe set
    W = 128
    rng = np.random.default_rng(16)
    o.nnf[0][:] = nnf0
    o.cost[0][:] = cost0
    ys, xs = np.divmod(np.arange(W * 96), W)
    col0 = ((xs + ys) & 1) == 0
    probe = col0 & (rng.random(W * 96) < 0.2)
    scr = col0 & ~probe
    o.nnf[0][scr] = np.roll(nnf0, 17)[scr]
    o.cost[0][scr] = np.inf
    o.pm_halfsweep(0, 0, 0, 0, 0)
    assert np.array_equal(o.nnf[0][probe], out_a[probe])


def test_costs_never_increase_and_restricted_mask():
    pair = synth.tiny_pair(0)
    o = oracle.Oracle(pair.frame1, pair.frame2, **TINY_PARAMS)
    o.nnf_init(0)
    o.eval_cost(0, 0)
    for it in range(3):
        for colour in range(2):
            before = o.cost[0].copy()
            o.pm_halfsweep(0, colour, it, 0, 0)
            assert (o.cost[0] <= before).all()
    # restricted: assigned pixels never change
    rng = np.random.default_rng(17)
    assigned = rng.random(128 * 96) < 0.6
    o.win[0][:] = np.where(assigned, 0, -1)
    before = o.nnf[0].copy()
    o.eval_cost(0, 1)
    for colour in range(2):
        o.pm_halfsweep(0, colour, 0, 1, 1)
    assert np.array_equal(o.nnf[0][assigned], before[assigned])


# --------------------------------------------------------------------------
# Assignment, symmetry, FB, end to end
# --------------------------------------------------------------------------

def _layered_two_planes():
    """Integer-translation layers: left (+4, +2), right (-3, +1)."""
    W, H = 64, 48
    rng = np.random.default_rng(18)
    bg = synth.Layer(H=synth.translation(4, 2))
    right = synth.Layer(H=synth.translation(-3, 1), rect=(32, -1000, 1000, 1000))
    return synth.render([bg, right], W, H, rng)


def _plane_oracle(pair, **kw):
    p = dict(C=3, r=2, grad_weight=0.0, blocks=(16,), iters=4, hyps=64, eps=0.1)
    p.update(kw)
    o = oracle.Oracle(pair.frame1, pair.frame2, **p)
    W, H = pair.frame1.shape[1], pair.frame1.shape[0]
    ys, xs = np.mgrid[0:H, 0:W]
    for d in range(2):
        f = pair.flow if d == 0 else None
        if d == 0:
            tx = np.floor(xs + pair.flow[..., 0] + 0.5).astype(int)
            ty = np.floor(ys + pair.flow[..., 1] + 0.5).astype(int)
            o.set_nnf(0, oracle.pack((tx - xs).ravel(), (ty - ys).ravel()))
    return o


def test_assign_exact_layers_zero_loss():
    pair = _layered_two_planes()
    o = _plane_oracle(pair)
    o.ransac(0, 0, 1)
    o.assign(0, 0, 1, 0)
    W = 64
    ys, xs = np.divmod(np.arange(W * 48), W)
    # rows >= 32 share a block with the rows whose targets leave the frame
    inner = (xs >= 4) & (xs < 26) & (ys >= 2) & (ys < 32) & (pair.occ.ravel() == 0)
    assert (o.win[0][inner] >= 0).all()
    assert (o.loss[0][inner] <= 1e-20).all()  # zero up to the rounding of the fitted H
    for p in np.nonzero(inner)[0]:
        Hk = o.pH[o.win[0][p]].reshape(3, 3)
        assert np.abs(Hk - synth.translation(4, 2)).max() < 1e-9


def test_assign_infinite_eps_takes_min_loss():
    pair = synth.tiny_pair(0)
    o = oracle.Oracle(pair.frame1, pair.frame2, **dict(TINY_PARAMS, eps=1e6))
    o.nnf_init(0)
    o.ransac(0, 0, 1)
    o.assign(0, 0, 1, 0)
    lib = oracle.lib()
    rng = np.random.default_rng(19)
    for p in rng.choice(128 * 96, 200, replace=False):
        x, y = p % 128, p // 128
        best, bestk = np.inf, -1
        for b in range(15 * 11):
            k = o.plane_index(0, 0, 1, b)
            I = o.pinfo[k]
            if not I[PI["valid"]]:
                continue
            if not (I[PI["x0"]] <= x < I[PI["x0"]] + I[PI["bw"]] and I[PI["y0"]] <= y < I[PI["y0"]] + I[PI["bh"]]):
                continue
            e = o.colour_err(0, x, y, o.pH[k])
            if e < best:
                best, bestk = e, k
        assert o.win[0][p] == bestk
        if bestk >= 0:
            assert o.loss[0][p] == best


def test_assign_ties_prefer_lower_block():
    pair = _layered_two_planes()
    o = _plane_oracle(pair)
    o.ransac(0, 0, 1)
    # make two overlapping blocks carry the same exact plane
    k0, k1 = o.plane_index(0, 0, 1, 0), o.plane_index(0, 0, 1, 1)
    o.pH[k0] = o.pH[k1] = synth.translation(4, 2).ravel()
    o.pinfo[[k0, k1], PI["valid"]] = 1
    o.pinfo[[k0, k1], PI["detected"]] = 1
    o.assign(0, 0, 1, 0)
    # pixel (10, 3) is covered by blocks 0 and 1
    assert o.win[0][3 * 64 + 10] == k0


def test_fb_occlusion_free_global_warp():
    """A single global integer translation: interior pixels pass FB and stay
    unoccluded; every block whose NNF is exact yields the exact plane, and the
    forward and backward planes there invert each other."""
    pair = synth.smooth_pair(96, 72, seed=20, shift=(3, 2))
    o = oracle.Oracle(pair.frame1, pair.frame2, C=3, r=2, grad_weight=0.0, blocks=(16,), iters=8, hyps=64, seed=1)
    o.nnf_init(0)
    o.nnf_init(1)
    o.eval_cost(0, 0)
    o.eval_cost(1, 0)
    o.pm_pass(0, 0)
    nnf_after_init = [o.nnf[0].copy(), o.nnf[1].copy()]
    o.reset_state()
    W, H = 96, 72
    # continue the pipeline from the converged init pass
    for stage in (1, 2):
        for d in range(2):
            o.ransac(d, 0, stage)
        for d in range(2):
            o.assign(d, 0, stage, 1)
        o.symmetry(0, stage)
        for d in range(2):
            o.assign(d, 0, stage, 0)
    o.fb_unassign()
    ys, xs = np.mgrid[0:H, 0:W]
    inner = (xs + 3 <= W - 4) & (ys + 2 <= H - 4) & (xs >= 3) & (ys >= 3)
    assert (o.win[0].reshape(H, W)[inner] >= 0).all()
    shifts = [(3, 2), (-3, -2)]
    n_exact = 0
    for d in range(2):
        dx, dy = oracle.unpack(nnf_after_init[d])
        ok = ((dx == shifts[d][0]) & (dy == shifts[d][1])).reshape(H, W)
        for b in range(o.block_grid(0)[0] * o.block_grid(0)[1]):
            k = o.plane_index(d, 0, 1, b)
            I = o.pinfo[k]
            if ok[I[PI["y0"]]:I[PI["y0"]] + 16, I[PI["x0"]]:I[PI["x0"]] + 16].all():
                n_exact += 1
                assert I[PI["count"]] == 256
                assert np.abs(o.pH[k].reshape(3, 3) - synth.translation(*shifts[d])).max() < 1e-9
    assert n_exact >= 20, n_exact
    # forward plane at p and backward plane at its target invert each other
    for (x, y) in [(20, 20), (30, 12), (40, 25)]:
        jf = o.win[0][y * W + x]
        jb = o.win[1][(y + 2) * W + x + 3]
        Hf, Hb = o.pH[jf].reshape(3, 3), o.pH[jb].reshape(3, 3)
        if np.abs(Hf - synth.translation(3, 2)).max() < 1e-9 and np.abs(Hb - synth.translation(-3, -2)).max() < 1e-9:
            Hp = Hb @ Hf
            assert np.abs(Hp / Hp[2, 2] - np.eye(3)).max() < 1e-9


def test_fb_translated_occluder_band():
    W, H = 64, 48
    rng = np.random.default_rng(21)
    bg = synth.Layer(H=synth.translation(0, 0))
    occl = synth.Layer(H=synth.translation(8, 0), rect=(20, 14, 44, 34))
    pair = synth.render([bg, occl], W, H, rng)
    o = oracle.Oracle(pair.frame1, pair.frame2, C=3, r=2, grad_weight=0.0, blocks=(16,), iters=6, hyps=128, seed=2)
    flows, occs = o.solve()
    ys, xs = np.mgrid[0:H, 0:W]
    # background pixels covered in frame 2 by the moved occluder: the band [44, 52) x [14, 34)
    band = (xs >= 46) & (xs < 50) & (ys >= 17) & (ys < 31)
    visible_bg = (pair.occ == 0) & ((xs < 18) | (xs > 54)) & (ys > 3) & (ys < 44) & (xs > 3) & (xs < 60)
    assert occs[0][band].mean() == 1.0
    assert occs[0][visible_bg].mean() < 0.02


@pytest.mark.slow
def test_end_to_end_sanity_tiny(tiny_pair):
    o = oracle.Oracle(tiny_pair.frame1, tiny_pair.frame2, **TINY_PARAMS)
    flows, occs = o.solve()
    vis = tiny_pair.occ == 0
    assigned = occs[0] == 0
    epe = np.linalg.norm(flows[0] - tiny_pair.flow, axis=-1)
    assert epe[vis & assigned].mean() < 0.5
    assert occs[0][tiny_pair.occ == 1].mean() > 0.8
    assert assigned[vis].mean() > 0.8


def test_luma_weights_per_channel():
    for ch, wgt in [(0, 0.299), (1, 0.587), (2, 0.114)]:
        img = np.zeros((5, 6, 3), np.float32)
        img[..., ch] = np.arange(6, dtype=np.float32)[None, :] * 0.5
        f = oracle.features(img, C=5)
        assert np.allclose(f[:, 2, 3], wgt * 0.5, rtol=1e-6), ch
        assert np.allclose(f[:, 2, 4], 0.0)


def test_ransac_ties_keep_lowest_hypothesis():
    """On an exact plane every accepted hypothesis has the full count, so the
    winner is the first hypothesis that is not rejected; the draw of
    hypothesis h does not depend on K, so that index is found by growing K."""
    W = H = 16

    def fn(xs, ys):
        return xs + 3, ys - 2

    first = None
    for K in range(1, 40):
        o = _ransac_oracle(W, H, 16, fn, hyps=K, seed=5)
        o.ransac(0, 0, 1)
        k = o.plane_index(0, 0, 1, 0)
        if o.pinfo[k, PI["hyp"]] >= 0:
            first = K - 1
            break
    assert first is not None
    o = _ransac_oracle(W, H, 16, fn, hyps=256, seed=5)
    o.ransac(0, 0, 1)
    assert o.pinfo[o.plane_index(0, 0, 1, 0), PI["hyp"]] == first


# --------------------------------------------------------------------------
# Occlusion cues 2 (many-to-one matches) and 3 (plane / colour-region overlap)
# --------------------------------------------------------------------------

def _project(Hm, x, y):
    """pi(H p) with the oracle's operation order (w <= 0: no target)."""
    w = Hm[6] * x + Hm[7] * y + Hm[8]
    if not w > 0:
        return 0.0, 0.0, w
    return (Hm[0] * x + Hm[1] * y + Hm[2]) / w, (Hm[3] * x + Hm[4] * y + Hm[5]) / w, w


def test_unique_matches_brute_force():
    """Cue 2 against its definition evaluated pixel by pixel: among the
    assigned pixels sent to one in-frame target, only the smallest (loss,
    index) keeps its plane."""
    W, H = 40, 30
    pair = synth.smooth_pair(W, H, seed=31)
    o = oracle.Oracle(pair.frame1, pair.frame2, C=3, r=2, grad_weight=0.0, blocks=(16,), cue_unique=True)
    rng = np.random.default_rng(32)
    planes = [synth.translation(2.25, -1.3), synth.translation(1.0, 0.0), synth.translation(-3.4, 2.2),
              synth.similarity_about(20, 15, 1.05, 4.0, 0.3, 0.2),
              np.array([[1.0, 0, 0.2], [0, 1.0, 0.1], [-0.04, 0, 1.0]])]   # w <= 0 right of x = 25
    ks = [o.plane_index(d, 0, 1, b) for d in range(2) for b in range(len(planes))]
    for d in range(2):
        for b, Hm in enumerate(planes):
            o.pH[o.plane_index(d, 0, 1, b)] = (Hm / Hm[2, 2]).ravel()
    before = []
    for d in range(2):
        pick = rng.integers(-1, len(planes), W * H)
        o.win[d][:] = np.where(pick >= 0, [o.plane_index(d, 0, 1, max(b, 0)) for b in pick], -1)
        o.loss[d][:] = np.where(pick >= 0, rng.choice([1e-4, 2e-4, 3e-4], W * H), np.inf)
        before.append((o.win[d].copy(), o.loss[d].copy()))
    o.unique()
    for d in range(2):
        win0, loss0 = before[d]
        best = {}
        targets = {}
        for p in range(W * H):
            if win0[p] < 0:
                continue
            qx, qy, w = _project(o.pH[win0[p]], p % W, p // W)
            if not w > 0:
                continue
            rx, ry = np.floor(qx + 0.5), np.floor(qy + 0.5)
            if not (0 <= rx <= W - 1 and 0 <= ry <= H - 1):
                continue
            q = int(ry) * W + int(rx)
            targets[p] = q
            if q not in best or (loss0[p], p) < (loss0[best[q]], best[q]):
                best[q] = p
        exp_win, exp_loss = win0.copy(), loss0.copy()
        for p, q in targets.items():
            if best[q] != p:
                exp_win[p], exp_loss[p] = -1, np.inf
        assert np.array_equal(o.win[d], exp_win)
        assert np.array_equal(o.loss[d], exp_loss)
        assert (exp_win < 0).sum() > (win0 < 0).sum() + 50     # the cue did remove pixels


def test_overlap_cue_counts_and_decision():
    """Cue 3 on an exact translation (the window's plane set to it) whose NNF
    is right on 40 % of the window, exactly one pixel off on 20 % (not an
    inlier: the test is strict) and far off elsewhere: the colour-consistent
    region is the whole in-frame window and only the right 40 % of it are
    inliers, so the plane is dropped when the cue is on and kept when off."""
    W, H, B = 64, 48, 16
    pair = synth.smooth_pair(W, H, seed=33, shift=(3, 2))
    rng = np.random.default_rng(34)
    ys, xs = np.mgrid[0:H, 0:W]
    u = rng.random((H, W))
    good, one_off = u < 0.4, (u >= 0.4) & (u < 0.6)
    side = rng.integers(0, 4, (H, W))
    dx = np.where(good, 3, rng.integers(10, 20, (H, W)))
    dy = np.where(good, 2, rng.integers(-20, -10, (H, W)))
    dx = np.where(one_off, 3 + np.array([1, -1, 0, 0])[side], dx)
    dy = np.where(one_off, 2 + np.array([0, 0, 1, -1])[side], dy)
    for cue in (False, True):
        o = oracle.Oracle(pair.frame1, pair.frame2, C=3, r=2, grad_weight=0.0, blocks=(B,), seed=3, cue_overlap=cue)
        o.set_nnf(0, oracle.pack(dx.ravel(), dy.ravel()))
        k = o.plane_index(0, 0, 1, 0)
        o.pH[k] = synth.translation(3, 2).ravel()
        o.pinfo[k, PI["detected"]] = 1
        kb = o.plane_index(1, 0, 1, 0)
        o.pH[kb] = synth.translation(-3, -2).ravel()
        o.twin[1][:] = kb
        o.symmetry(0, 1)
        win = (xs < B) & (ys < B)
        region = win & (xs + 3 <= W - 1) & (ys + 2 <= H - 1)
        assert o.pinfo[k, PI["rk"]] == region.sum()
        assert o.pinfo[k, PI["rin"]] == (region & good).sum()
        assert o.pinfo[k, PI["pass"]] == region.sum()
        assert o.pinfo[k, PI["valid"]] == (0 if cue else 1)


# --------------------------------------------------------------------------
# Filling by homography-model propagation
# --------------------------------------------------------------------------

def _rgb_err_at(f1, f2, x, y, tx, ty):
    """Colour error of pixel (x, y) against the integer target (tx, ty): the
    mean over R, G, B of the squared difference, summed in channel order."""
    d = [float(f1[y, x, c]) - float(f2[ty, tx, c]) for c in range(3)]
    return (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) / 3.0


@pytest.mark.parametrize("sources", ["random", "one_colour0"])
def test_fill_reach_matches_red_black_distance(sources):
    """Every candidate accepted (large epsilon, identity plane): a red-black
    propagation fills pixel p at half-sweep min over sources s of
    d(s, p) - 1 + [s has colour 0] (d = 4-neighbour distance), so after K
    half-sweeps exactly the pixels with that time below K are filled, each
    with the sources' plane and its own colour error as loss.  A single
    source of colour 0 leaves the first half-sweep with nothing to fill."""
    W, H, K = 40, 30, 7
    pair = synth.smooth_pair(W, H, seed=41)
    o = oracle.Oracle(pair.frame1, pair.frame2, C=3, r=2, grad_weight=0.0, blocks=(16,), eps=10.0, fill_sweeps=K)
    rng = np.random.default_rng(42)
    k = o.plane_index(0, 0, 1, 1)
    o.pH[k] = np.eye(3).ravel()
    ys, xs = np.divmod(np.arange(W * H), W)
    src = rng.random(W * H) < 0.02 if sources == "random" else (xs == 12) & (ys == 14)
    o.win[0][:] = np.where(src, k, -1)
    o.win[1][:] = -1
    o.loss[0][:] = np.where(src, 0.5, np.inf)
    o.fill()
    sx, sy = xs[src], ys[src]
    d = np.abs(xs[:, None] - sx[None, :]) + np.abs(ys[:, None] - sy[None, :])
    t = (d - 1 + ((sx + sy) % 2 == 0)[None, :]).min(axis=1)
    filled = ~src & (t < K)
    assert filled.sum() > (100 if sources == "random" else 40) and (~src & ~filled).sum() > 100
    assert np.array_equal(o.win[0], np.where(src, k, np.where(filled, -2 - k, -1)))
    f1, f2 = o.feat[0], o.feat[1]
    exp = [_rgb_err_at(f1, f2, x, y, x, y) for x, y in zip(xs[filled], ys[filled])]
    assert np.array_equal(o.loss[0][filled], np.array(exp))
    assert (o.win[1] == -1).all()


def test_fill_stops_at_colour_inconsistent_pixels():
    """Backward direction of an exact translation, plane sources on one
    column, a two-column wall of pixels whose colour was changed: the fill
    covers everything reachable without crossing the wall or the pixels the
    plane sends out of the frame, and nothing beyond the wall although those
    pixels are consistent.  The filled pixels' flow is the plane's and their
    mask value is 2."""
    W, H = 48, 24
    pair = synth.smooth_pair(W, H, seed=43, shift=(3, 2))
    f2 = pair.frame2.copy()
    f2[:, 20:22] = np.clip(1.0 - f2[:, 20:22], 0, 1) + 0.3
    o = oracle.Oracle(pair.frame1, f2, C=3, r=2, grad_weight=0.0, blocks=(16,), fill_sweeps=200)
    k = o.plane_index(1, 0, 2, 0)
    o.pH[k] = synth.translation(-3, -2).ravel()
    ys, xs = np.divmod(np.arange(W * H), W)
    src = xs == 5
    o.win[1][:] = np.where(src, k, -1)
    o.loss[1][:] = np.where(src, 0.0, np.inf)
    o.fill()
    consistent = np.array([xx >= 3 and yy >= 2 and _rgb_err_at(o.feat[1], o.feat[0], xx, yy, xx - 3, yy - 2) < 0.01
                           for xx, yy in zip(xs, ys)])
    assert not consistent[(xs >= 20) & (xs < 22)].any()
    assert consistent[(xs >= 22) & (ys >= 2)].all()
    filled = ~src & (xs >= 3) & (xs < 20) & (ys >= 2)
    assert np.array_equal(o.win[1], np.where(src, k, np.where(filled, -2 - k, -1)))
    assert (o.loss[1][filled] == 0.0).all()
    flow, occ = o.finalize(1)
    fl = flow.reshape(-1, 2)
    assert (fl[filled] == np.array([-3.0, -2.0], np.float32)).all()
    assert (occ.ravel()[filled] == 2).all() and (occ.ravel()[src] == 0).all()
    assert (occ.ravel()[~filled & ~src] == 1).all()


def test_fill_takes_smallest_error_then_smallest_index():
    """A one-pixel gap between a region of plane A (left) and plane B (right):
    one half-sweep fills the gap pixels of its colour with whichever plane has
    the smaller colour error there (errors computed here by direct lookup,
    the planes being integer translations); with B a copy of A stored at a
    smaller index, the tie goes to B."""
    W, H, c = 40, 30, 17
    pair = synth.smooth_pair(W, H, seed=44, shift=(2, 1))
    ys, xs = np.divmod(np.arange(W * H), W)
    # gap pixels on rows 1, 5, 9, ... copy plane B's target, so B wins there
    f1 = pair.frame1.copy()
    for y in range(1, H - 2, 4):
        f1[y, c] = pair.frame2[y + 2, c - 1]
    for tie in (False, True):
        o = oracle.Oracle(f1, pair.frame2, C=3, r=2, grad_weight=0.0, blocks=(16,), eps=10.0, fill_sweeps=1)
        ka, kb = o.plane_index(0, 0, 1, 2), o.plane_index(0, 0, 1, 0)
        ta, tb = (2, 1), ((2, 1) if tie else (-1, 2))
        o.pH[ka] = synth.translation(*ta).ravel()
        o.pH[kb] = synth.translation(*tb).ravel()
        o.win[0][:] = np.where(xs < c, ka, np.where(xs > c, kb, -1))
        o.loss[0][:] = np.where(xs != c, 0.0, np.inf)
        o.fill()
        f1s, f2s = o.feat[0], o.feat[1]
        n_a = n_b = 0
        for y in range(H):
            p = y * W + c
            if (c + y) % 2 == 1:
                assert o.win[0][p] == -1
                continue
            ea = _rgb_err_at(f1s, f2s, c, y, c + ta[0], y + ta[1]) if 0 <= y + ta[1] < H else np.inf
            eb = _rgb_err_at(f1s, f2s, c, y, c + tb[0], y + tb[1]) if 0 <= y + tb[1] < H else np.inf
            if not min(ea, eb) < 100.0:
                assert o.win[0][p] == -1
                continue
            best = kb if (eb < ea or (eb == ea and kb < ka)) else ka
            n_a += best == ka
            n_b += best == kb
            assert o.win[0][p] == -2 - best, (tie, y)
            assert o.loss[0][p] == min(ea, eb)
        if tie:
            assert n_b > 10 and n_a == 0
        else:
            assert n_a > 3 and n_b > 3


# --------------------------------------------------------------------------
# HSV histogram equalisation
# --------------------------------------------------------------------------

def _grey(values, W, H, seed):
    rng = np.random.default_rng(seed)
    v = np.array(values, np.float32)
    v = v[rng.permutation(v.size)].reshape(H, W)
    return np.repeat(v[..., None], 3, axis=2)


def test_histeq_equal_counts_map_to_even_steps():
    """A grey frame whose k occupied levels are equally frequent: the i-th
    level maps to i / (k - 1).  Levels are the nearest of 256 steps, so values
    0.3/255 and 0.7/255 fall in different levels."""
    rng = np.random.default_rng(51)
    k = 17
    lv = np.sort(rng.choice(256, k, replace=False))
    vals = np.repeat(lv.astype(np.float32) / np.float32(255), 40)
    out = oracle.histeq(_grey(vals, 34, 20, 52))
    src = _grey(vals, 34, 20, 52)
    idx = np.searchsorted(lv.astype(np.float32) / np.float32(255), src[..., 0])
    assert np.allclose(out[..., 0], idx / (k - 1), rtol=3e-7, atol=0)
    assert (out[..., 0] == out[..., 1]).all() and (out[..., 1] == out[..., 2]).all()
    vals = np.repeat(np.array([0.3, 0.7, 255.0], np.float32) / np.float32(255), 10)
    out = oracle.histeq(_grey(vals, 6, 5, 53))
    src = _grey(vals, 6, 5, 53)
    exp = np.where(src < 0.5 / 255, 0.0, np.where(src < 0.9, 0.5, 1.0))
    assert np.allclose(out, exp, rtol=3e-7, atol=1e-30)


def test_histeq_is_the_empirical_value_distribution():
    """A colour frame: the new value of a pixel equals the share of pixels
    whose value level is at or below its own, rescaled so that the lowest
    occupied level goes to 0 and the highest to 1; the output spans [0, 1]
    and depends on the value levels only through their order."""
    rng = np.random.default_rng(54)
    H, W = 30, 41
    rgb = (rng.random((H, W, 3)) ** 1.7).astype(np.float32)
    out = oracle.histeq(rgb)
    V = rgb.max(axis=2)
    Vn = out.max(axis=2)
    lvl = np.floor(V.astype(np.float64) * 255 + 0.5).astype(np.int64).ravel()
    srt = np.sort(lvl)
    n = lvl.size
    at_or_below = np.searchsorted(srt, lvl, side="right")
    lowest = np.searchsorted(srt, srt[0], side="right")
    exp = (at_or_below - lowest) / (n - lowest)
    assert np.allclose(Vn.ravel(), exp, rtol=1e-6, atol=1e-7)
    assert abs(Vn.min()) < 1e-7 and abs(Vn.max() - 1) < 1e-6
    # an order-preserving change of the levels leaves the output unchanged
    grey = np.repeat(np.sort(rng.choice(np.arange(20, 120), 12, replace=False)), 20)
    a = oracle.histeq(_grey(grey.astype(np.float32) / np.float32(255), 24, 10, 55))
    b = oracle.histeq(_grey((2 * grey + 7).astype(np.float32) / np.float32(255), 24, 10, 55))
    assert np.allclose(a, b, rtol=3e-7, atol=0)


def test_histeq_keeps_hue_and_saturation():
    """HSV round trip by an independent library: hue and saturation of every
    pixel are unchanged; black pixels stay black (the lowest level maps to 0);
    a frame on a single level is returned as it is."""
    from matplotlib.colors import rgb_to_hsv
    rng = np.random.default_rng(56)
    rgb = rng.random((20, 30, 3)).astype(np.float32)
    rgb[3, 4] = 0.0
    rgb[7, 9] = 0.0
    out = oracle.histeq(rgb)
    hi, ho = rgb_to_hsv(rgb.astype(np.float64)), rgb_to_hsv(out.astype(np.float64))
    live = rgb.max(axis=2) > 0
    assert np.allclose(hi[live][:, 1], ho[live][:, 1], atol=2e-6)
    dh = np.abs(hi[live][:, 0] - ho[live][:, 0])
    assert (np.minimum(dh, 1 - dh)[hi[live][:, 1] > 1e-3] < 2e-6).all()
    assert (out[3, 4] == out[3, 4, 0]).all() and out[3, 4, 0] == 0.0   # lowest level maps to 0
    flat = np.full((8, 9, 3), 0.25, np.float32)
    flat[..., 1] = 0.1
    assert np.array_equal(oracle.histeq(flat), flat)


# --------------------------------------------------------------------------
# NNF update and region plane
# --------------------------------------------------------------------------

def test_nnf_update_rounds_half_up_and_picks_region_plane():
    """Assigned pixels move to where their plane sends them, rounded half up
    and clamped into the frame (a translation by (0.5, -1.5) gives the offset
    (1, -1), which rounding half to even would not); unassigned pixels keep
    their offset.  The region plane of every pixel is, among the valid planes
    of both stages whose window contains it, the one with the largest count,
    ties to stage 1 and then to the lower window; with none the old label
    stays."""
    W, H = 48, 32
    pair = synth.smooth_pair(W, H, seed=71)
    o = oracle.Oracle(pair.frame1, pair.frame2, C=3, r=2, grad_weight=0.0, blocks=(16,))
    rng = np.random.default_rng(72)
    k0 = o.plane_index(0, 0, 1, 0)
    o.pH[k0] = synth.translation(0.5, -1.5).ravel()
    assigned = rng.random(W * H) < 0.7
    old = oracle.pack(rng.integers(-5, 6, W * H), rng.integers(-5, 6, W * H))
    o.set_nnf(0, old)
    old = o.nnf[0].copy()        # as stored: targets clamped into the frame
    o.win[0][:] = np.where(assigned, k0, -1)
    nwin = o.block_grid(0)[0] * o.block_grid(0)[1]
    recs = [o.plane_index(0, 0, st, b) for st in (1, 2) for b in range(nwin)]
    for k in recs:
        o.pinfo[k, PI["valid"]] = int(rng.random() < 0.5)
        o.pinfo[k, PI["count"]] = int(rng.integers(5, 9))   # few values: many ties
    o.hlabel[0][:] = -7
    o.nnf_update(0, 0)
    ys, xs = np.divmod(np.arange(W * H), W)
    ex = np.where(xs == W - 1, 0, 1)
    ey = np.where(ys == 0, 0, -1)
    dx, dy = oracle.unpack(o.nnf[0])
    odx, ody = oracle.unpack(old)
    assert np.array_equal(dx, np.where(assigned, ex, odx))
    assert np.array_equal(dy, np.where(assigned, ey, ody))
    expect = np.full(W * H, -7)
    for p in range(W * H):
        best, bestc = -7, -1
        for k in recs:           # stage 1 windows first, each stage in window order
            I = o.pinfo[k]
            if not I[PI["valid"]]:
                continue
            if not (I[PI["x0"]] <= xs[p] < I[PI["x0"]] + I[PI["bw"]] and I[PI["y0"]] <= ys[p] < I[PI["y0"]] + I[PI["bh"]]):
                continue
            if I[PI["count"]] > bestc:
                best, bestc = k, I[PI["count"]]
        expect[p] = best
    assert np.array_equal(o.hlabel[0], expect)
    assert (expect == -7).any() and (expect != -7).any()
