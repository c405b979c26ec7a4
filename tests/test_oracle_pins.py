"""Pins for the CPU oracle: each test ties it to something other than itself
(printed constants, textbook routines, closed forms, invariants, brute force).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.stats

from paper_1501_04140_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def np_iso(block, t):
    """The 8 isometries from numpy's own rotate/flip (independent of the oracle's table)."""
    rot = [block, np.rot90(block, -1), np.rot90(block, 2), np.rot90(block, 1)][t % 4]
    return np.fliplr(rot) if t >= 4 else rot


# ----------------------------------------------------------------- printed constants (P11, counts)
def test_paper_constants(orc):
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert list(orc.LEVEL_SIDES) == g["level_sides"]["value"]
    assert orc.N_ISO == g["n_isometries"]["value"]
    assert [[k / orc.Q for k in ks] for ks in orc.PAPER_K] == g["predefined_s"]["value"]
    lo, hi = g["plain_s_range"]["value"]
    assert [k / orc.Q for k in orc.PLAIN_K] == [pytest.approx(lo + 0.1 * i) for i in range(11)]
    assert orc.PLAIN_K[-1] / orc.Q == hi


def test_counts_section1(orc):
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))["count_examples"]
    for case in g["cases"]:
        N, n = case["N"], case["n"]
        gy, gx = orc.range_grid(N, N, n)
        assert gy * gx == case["ranges"]
        dy, dx = orc.domain_grid(N, N, n, 1)
        assert dy * dx == case["domains_step1"]
    # the single-level workload's 841 domains (step 4) and the quadtree's per-level grids
    assert orc.domain_grid(128, 128, 8, 4) == (29, 29)
    assert [orc.domain_grid(512, 512, B, max(B // 2, 1))[0] for B in (16, 8, 4, 2)] == \
        [61, 125, 253, 509]


# ----------------------------------------------------------------- isometries (P6)
@pytest.mark.parametrize("B", [2, 4, 8, 16])
def test_isometry_table_is_numpy_d4(orc, B):
    rng = np.random.default_rng(B)
    blk = rng.integers(0, 1000, size=(B, B))
    for t in range(8):
        assert np.array_equal(orc.isometry(blk, t), np_iso(blk, t)), t


def test_isometry_group_laws(orc):
    B = 4
    idx = np.arange(B * B).reshape(B, B)
    maps = [tuple(orc.isometry(idx, t).ravel()) for t in range(8)]
    assert len(set(maps)) == 8
    x = idx
    for _ in range(4):
        x = orc.isometry(x, 1)
    assert np.array_equal(x, idx)                       # rot^4 = id
    for t in range(4, 8):
        assert np.array_equal(orc.isometry(orc.isometry(idx, t), t), idx)  # reflections
    for a in range(8):                                  # closure
        for b in range(8):
            comp = tuple(orc.isometry(orc.isometry(idx, b), a).ravel())
            assert comp in maps


def test_decimation_commutes_and_sums_invariant(orc):
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(8, 8)).astype(np.uint8)
    dd = orc.decimate(img, 0, 0, 4)
    assert dd.max() <= 1020
    for t in range(8):
        # decimating an isometric copy of the 2B x 2B block = isometry of the decimation
        timg = np.ascontiguousarray(np_iso(img, t))
        assert np.array_equal(orc.decimate(timg, 0, 0, 4), orc.isometry(dd, t))
        c = orc.isometry(dd, t)
        assert c.sum() == dd.sum() and (c.astype(np.int64) ** 2).sum() == (dd.astype(np.int64) ** 2).sum()


# ----------------------------------------------------------------- eq. (1) with eq. (3)
def test_candidate_equals_least_squares_residual(orc):
    """For a fixed s the o of eq. (3) is the least-squares offset, so E = n * var(r - s*d)."""
    rng = np.random.default_rng(7)
    for B in (2, 4, 8):
        n = B * B
        for _ in range(20):
            r = rng.integers(0, 256, size=(B, B))
            dd = rng.integers(0, 1021, size=(B, B))
            for t in range(8):
                d = np_iso(dd, t) / 4.0
                for k in range(11):
                    e = orc.eval_candidate(r, dd, t, k)
                    assert e >= 0 and e % n == 0
                    E = e / (4.0 * orc.Q * n) ** 2
                    ref = n * np.var(r - (k / 10.0) * d)
                    assert E == pytest.approx(ref, rel=1e-12, abs=1e-9)


def test_offset_eq3_minimises(orc):
    """Moving o away from eq. (3) never lowers E (literal eq. (1) in Fractions)."""
    rng = np.random.default_rng(11)
    for _ in range(30):
        r = [int(v) for v in rng.integers(0, 256, size=4)]
        d = [Fraction(int(v), 4) for v in rng.integers(0, 1021, size=4)]
        s = Fraction(int(rng.integers(0, 11)), 10)
        o3 = Fraction(sum(r), 4) - s * sum(d) / 4

        def E(o):
            return sum((s * di + o - ri) ** 2 for di, ri in zip(d, r))

        for delta in (Fraction(1, 7), Fraction(-3, 5), Fraction(2)):
            assert E(o3 + delta) > E(o3)


def test_closed_form_s_by_dense_grid():
    """Eq. (2): the unconstrained optimum; clamped to [0,1] it is the minimum over a dense s grid."""
    rng = np.random.default_rng(5)
    grid = np.linspace(0.0, 1.0, 100001)
    for n in (4, 16):
        for _ in range(20):
            r = rng.integers(0, 256, size=n).astype(np.float64)
            d = rng.integers(0, 1021, size=n) / 4.0
            rc, dc = r - r.mean(), d - d.mean()
            sdd = (dc * dc).sum()
            if sdd == 0:
                continue
            s_star = (rc * dc).sum() / sdd                      # eq. (2)
            E_grid = ((rc * rc).sum() - 2 * grid * (rc * dc).sum() + grid * grid * sdd)
            s_c = min(max(s_star, 0.0), 1.0)
            E_c = ((s_c * dc - rc) ** 2).sum()
            assert E_grid.min() == pytest.approx(E_c, abs=sdd * (0.5e-5) ** 2 + 1e-9)
            if 0 <= s_star <= 1:
                assert E_c == pytest.approx((rc * rc).sum() - (rc * dc).sum() ** 2 / sdd, abs=1e-7)


def test_grid_best_bounded_by_continuous_optimum(orc):
    img = synth.gradients_blobs(32, seed=2)
    B, L = 4, 4
    m = orc.match_level(img, B, L)
    n = B * B
    gy, gx = orc.domain_grid(32, 32, B, L)
    for q, (ry, rx) in enumerate(orc.full_ranges(32, 32, B)):
        r = img[ry:ry + B, rx:rx + B].astype(np.float64)
        best = m["e_lit"][q] / (4.0 * orc.Q * n) ** 2
        lo = np.inf
        for j in range(gy * gx):
            dy, dx = orc.domain_yx(j, gx, L)
            dd = orc.decimate(img, int(dy), int(dx), B) / 4.0
            for t in range(8):
                A = np.stack([np_iso(dd, t).ravel(), np.ones(n)], axis=1)
                # least squares over s in [0,1] with free o: unconstrained, then clamp
                res = np.linalg.lstsq(A, r.ravel(), rcond=None)
                s = min(max(res[0][0], 0.0), 1.0)
                e = n * np.var(r.ravel() - s * A[:, 0])
                lo = min(lo, e)
        assert best >= lo - 1e-7
        assert best <= n * np.var(r) + 1e-9                     # k = 0 is a candidate


# ----------------------------------------------------------------- exact copies (P2)
def _copy_image(k, o, t, B=4, seed=0):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(48, 48)).astype(np.int64)
    m = rng.integers(0, 26, size=(B, B))                        # cell means 10*m, d' = 40*m
    while len({tuple(np_iso(m, u).ravel()) for u in range(8)}) < 8:
        m = rng.integers(0, 26, size=(B, B))
    dy, dx = 24, 24
    img[dy:dy + 2 * B, dx:dx + 2 * B] = np.kron(10 * m, np.ones((2, 2), dtype=np.int64))
    ry, rx = 4, 8
    img[ry:ry + B, rx:rx + B] = k * np_iso(m, t) + o            # s*d = (k/10)*(10 m) = k m
    assert img.min() >= 0 and img.max() <= 255
    return img.astype(np.uint8), (dy, dx), (ry, rx)


@pytest.mark.parametrize("t", range(8))
def test_isometric_copy_found_exactly(orc, t):
    img, (dy, dx), (ry, rx) = _copy_image(10, 3, t, seed=t)
    B, L = 4, 4
    m = orc.match_level(img, B, L, ranges=np.array([[ry, rx]]))
    gy, gx = orc.domain_grid(48, 48, B, L)
    assert m["e_lit"][0] == 0 and m["second"][0] > 0
    assert (m["dom"][0], m["iso"][0], m["k"][0], m["q_o"][0]) == ((dy // L) * gx + dx // L, t, 10, 3)


@pytest.mark.parametrize("k,o", [(3, 40), (7, 5), (5, 100)])
def test_scaled_copy_found_exactly(orc, k, o):
    img, (dy, dx), (ry, rx) = _copy_image(k, o, 5, seed=k)
    m = orc.match_level(img, 4, 4, ranges=np.array([[ry, rx]]))
    gy, gx = orc.domain_grid(48, 48, 4, 4)
    assert m["e_lit"][0] == 0
    assert (m["dom"][0], m["iso"][0], m["k"][0], m["q_o"][0]) == ((dy // 4) * gx + dx // 4, 5, k, o)


# ----------------------------------------------------------------- brute force on tiny inputs
def _brute(img, B, L, ks, pool=None):
    """Pure-Python exhaustive search in Fractions with numpy isometries."""
    H, W = img.shape
    gy, gx = (H - 2 * B) // L + 1, (W - 2 * B) // L + 1
    pool = range(gy * gx) if pool is None else pool
    out = []
    for ry in range(0, H - B + 1, B):
        for rx in range(0, W - B + 1, B):
            r = [int(v) for v in img[ry:ry + B, rx:rx + B].ravel()]
            n = len(r)
            cands = []
            for j in pool:
                y, x = (j // gx) * L, (j % gx) * L
                blk = img[y:y + 2 * B, x:x + 2 * B].astype(np.int64)
                dm = (blk[0::2, 0::2] + blk[0::2, 1::2] + blk[1::2, 0::2] + blk[1::2, 1::2])
                for t in range(8):
                    d = [Fraction(int(v), 4) for v in np_iso(dm, t).ravel()]
                    for si, k in enumerate(ks):
                        s = Fraction(k, 10)
                        o = Fraction(sum(r), n) - s * sum(d) / n
                        E = sum((s * di + o - ri) ** 2 for di, ri in zip(d, r))
                        cands.append((E, j, t, si, o))
            cands.sort(key=lambda c: c[:4])
            E, j, t, si, o = cands[0]
            out.append((E, j, t, si, math.floor(o + Fraction(1, 2)), cands[1][0]))
    return out


@pytest.mark.parametrize("kind", ["noise", "constant", "replicated", "blobs"])
def test_bruteforce_tiny(orc, kind):
    rng = np.random.default_rng(1)
    if kind == "noise":
        img = rng.integers(0, 256, size=(12, 12)).astype(np.uint8)
    elif kind == "constant":
        img = np.full((12, 12), 77, dtype=np.uint8)
    elif kind == "replicated":
        img = np.kron(rng.integers(0, 256, size=(6, 6)), np.ones((2, 2))).astype(np.uint8)
    else:
        img = synth.gradients_blobs(12, seed=4)
    for B, L, ks in [(2, 2, orc.PLAIN_K), (2, 1, (2, 4)), (4, 2, orc.PLAIN_K)]:
        m = orc.match_level(img, B, L, ks)
        ref = _brute(img, B, L, ks)
        n = B * B
        for q, (E, j, t, si, qo, E2) in enumerate(ref):
            assert Fraction(int(m["e_lit"][q]), (4 * orc.Q * n) ** 2) == E
            assert (m["dom"][q], m["iso"][q], m["s_idx"][q], m["q_o"][q]) == (j, t, si, qo)
            assert Fraction(int(m["second"][q]), (4 * orc.Q * n) ** 2) == E2


def test_constant_range_special_case(orc):
    rng = np.random.default_rng(9)
    img = rng.integers(0, 256, size=(32, 32)).astype(np.uint8)
    img[0:4, 0:4] = 200
    pool = np.array([5, 9, 30], dtype=np.int32)
    m = orc.match_level(img, 4, 4, pool=pool, ranges=np.array([[0, 0]]))
    assert (m["e_lit"][0], m["dom"][0], m["iso"][0], m["k"][0], m["q_o"][0]) == (0, 5, 0, 0, 200)


# ----------------------------------------------------------------- entropy (P7)
def test_entropy_special_cases(orc):
    assert orc.entropy_bits([16, 0, 0, 0, 0, 0, 0, 0]) == 0.0
    assert not orc.entropy_above([16, 0, 0, 0, 0, 0, 0, 0], 0.0)
    assert orc.entropy_bits([2] * 8) == pytest.approx(3.0)
    assert orc.entropy_above([2] * 8, 2.5)
    assert not orc.entropy_above([2] * 8, 3.0)               # strict: H = 3 is not > 3
    tie = [4, 4, 2, 2, 2, 2, 0, 0]
    assert orc.entropy_bits(tie) == pytest.approx(2.5)
    assert not orc.entropy_above(tie, 2.5)                    # exactly 2.5 is excluded
    assert orc.entropy_above([3, 3, 2, 2, 2, 2, 1, 1], 2.5)
    assert not orc.entropy_above([4, 4, 3, 2, 2, 1, 0, 0], 2.5)      # 2.45 bits


def test_entropy_decision_matches_scipy(orc):
    rng = np.random.default_rng(2)
    for nw in (16, 64, 256, 1024):
        for _ in range(300):
            c = rng.multinomial(nw, rng.dirichlet(np.ones(8) * 0.7))
            h = scipy.stats.entropy(c, base=2)
            if abs(h - 2.5) > 1e-9:
                assert orc.entropy_above(c, 2.5) == (h > 2.5)


def test_pool_floor_by_bruteforce(orc):
    img = synth.power_law(48, beta=2.0, seed=3)
    B, L = 4, 2
    pool, n_pass = orc.entropy_pool(img, B, L, 2.5, min_pool=40)
    gy, gx = orc.domain_grid(48, 48, B, L)
    H = []
    for j in range(gy * gx):
        y, x = orc.domain_yx(j, gx, L)
        c = np.bincount((img[y:y + 2 * B, x:x + 2 * B] >> 5).ravel(), minlength=8)
        H.append(scipy.stats.entropy(c, base=2))
    H = np.array(H)
    assert n_pass == int((H > 2.5 + 1e-12).sum())
    if n_pass >= 40:
        assert np.array_equal(pool, np.flatnonzero(H > 2.5 + 1e-12))
    else:
        order = sorted(range(len(H)), key=lambda j: (-round(H[j], 9), j))[:40]
        assert np.array_equal(pool, np.sort(order))


# ----------------------------------------------------------------- subset monotonicity (P10)
def test_subset_monotonicity(orc):
    img = synth.power_law(64, beta=2.0, seed=1, n_rect=1)
    B, L = 4, 2
    full = orc.match_level(img, B, L)
    pool, _ = orc.entropy_pool(img, B, L, 2.5, min_pool=64)
    filt = orc.match_level(img, B, L, pool=pool)
    pres = orc.match_level(img, B, L, s_k=(3, 8))
    assert np.all(filt["e_lit"] >= full["e_lit"])
    assert np.all(pres["e_lit"] >= full["e_lit"])


# ----------------------------------------------------------------- quadtree invariants
def test_quadtree_invariants(orc):
    img = synth.power_law(64, beta=2.0, seed=0, n_rect=3)
    codes, stats = orc.encode_image(img, s_sets=orc.PAPER_K, rms=8.0, min_pool=32)
    cover = np.zeros((64, 64), dtype=np.int32)
    for c in codes:
        cover[c["y"]:c["y"] + c["B"], c["x"]:c["x"] + c["B"]] += 1
        n = int(c["B"]) ** 2
        if c["level"] < 3:
            assert c["e_lit"] <= 64 * n * (40 * n) ** 2
    assert np.all(cover == 1)
    # every range that was split had error above the threshold
    for lv in range(1, 4):
        B = orc.LEVEL_SIDES[lv - 1]
        parents = {(int(c["y"]) // B * B, int(c["x"]) // B * B) for c in codes if c["level"] >= lv}
        if not parents:
            continue
        pool, _ = orc.entropy_pool(img, B, max(B // 2, 1), 2.5, 32)
        m = orc.match_level(img, B, max(B // 2, 1), orc.PAPER_K[lv - 1], pool,
                            np.array(sorted(parents), dtype=np.int32))
        assert np.all(m["e_lit"] > 64 * B * B * (40 * B * B) ** 2)
    assert sum(s["accepted"] for s in stats) == len(codes)


# ----------------------------------------------------------------- decoder (P8)
def _continuous_decode(codes, H, W, iters):
    x = np.full((H, W), 128.0)
    for _ in range(iters):
        nxt = np.empty_like(x)
        for c in codes:
            B = int(c["B"])
            blk = x[c["dy"]:c["dy"] + 2 * B, c["dx"]:c["dx"] + 2 * B]
            d = (blk[0::2, 0::2] + blk[0::2, 1::2] + blk[1::2, 0::2] + blk[1::2, 1::2]) / 4.0
            v = (int(c["k"]) / 10.0) * np_iso(d, int(c["iso"])) + int(c["q_o"])
            nxt[c["y"]:c["y"] + B, c["x"]:c["x"] + B] = np.clip(v, 0, 255)
        x = nxt
    return x


def test_decode_contraction_and_rounding_bound(orc):
    img = synth.power_law(32, beta=2.0, seed=5, n_rect=1)
    codes, _ = orc.encode_image(img, s_sets=orc.PAPER_K, rms=8.0, min_pool=16)
    s_max = max(int(c["k"]) for c in codes) / 10.0
    assert s_max <= 0.9
    xi = orc.decode(codes, 32, 32, iters=64).astype(np.float64)
    xc = _continuous_decode(codes, 32, 32, 150)
    # each integer step is W(x) rounded (error <= 1/2) and W contracts by s_max in the
    # max norm, so the integer iterate stays within 1/2 / (1 - s_max) of the attractor
    slack = 255.0 * s_max ** 64 + 255.0 * s_max ** 150
    assert np.abs(xi - xc).max() <= 0.5 / (1 - s_max) + slack + 1e-9


def test_decode_collage_bound(orc):
    img = synth.power_law(32, beta=2.0, seed=6)
    codes, _ = orc.encode_image(img, s_sets=orc.PAPER_K, rms=8.0, min_pool=16)
    s_max = max(int(c["k"]) for c in codes) / 10.0
    x_inf = _continuous_decode(codes, 32, 32, 200)
    f = img.astype(np.float64)
    Wf = np.empty_like(f)
    for c in codes:
        B = int(c["B"])
        blk = f[c["dy"]:c["dy"] + 2 * B, c["dx"]:c["dx"] + 2 * B]
        d = (blk[0::2, 0::2] + blk[0::2, 1::2] + blk[1::2, 0::2] + blk[1::2, 1::2]) / 4.0
        Wf[c["y"]:c["y"] + B, c["x"]:c["x"] + B] = np.clip(
            (int(c["k"]) / 10.0) * np_iso(d, int(c["iso"])) + int(c["q_o"]), 0, 255)
    assert np.abs(f - x_inf).max() <= np.abs(f - Wf).max() / (1 - s_max) + 1e-6


def test_decode_exact_image(orc):
    img = np.full((32, 32), 93, dtype=np.uint8)
    codes, _ = orc.encode_image(img, s_sets=orc.PAPER_K, rms=8.0, min_pool=8)
    assert np.all(codes["e_lit"] == 0) and np.all(codes["level"] == 0)
    out = orc.decode(codes, 32, 32, iters=8)
    assert np.array_equal(out, img) and orc.psnr(out, img) == float("inf")


def test_psnr_definition(orc):
    a = np.zeros((4, 4), np.uint8)
    b = a.copy()
    b[0, 0] = 4
    assert orc.psnr(a, b) == pytest.approx(10 * math.log10(255 ** 2 / (16 / 16)))


# --------------------------------------------------------------------------- variance pool
import oracle  # noqa: E402


def _window_vars(img, side, step):
    win = np.lib.stride_tricks.sliding_window_view(img.astype(np.float64), (side, side))[::step, ::step]
    return win.reshape(win.shape[0] * win.shape[1], -1).var(axis=1)


@pytest.mark.parametrize("B,L,vmin", [(4, 2, 150.0), (8, 4, 400.0), (2, 1, 30.5)])
def test_variance_pool_threshold_matches_numpy_var(B, L, vmin):
    img = synth.power_law(64, beta=1.6, seed=3)
    pool, n_pass = oracle.variance_pool(img, B, L, vmin, min_pool=1)
    v = _window_vars(img, 2 * B, L)
    clear = np.abs(v - vmin) > 1e-6
    keep = np.zeros(len(v), dtype=bool)
    keep[pool] = True
    assert n_pass == len(pool) and n_pass > 0
    assert np.array_equal(keep[clear], (v > vmin)[clear])


def test_variance_pool_floor_is_a_stable_sort():
    rng = np.random.default_rng(0)
    img = (rng.integers(0, 4, size=(40, 40)) * 60).astype(np.uint8)  # few distinct variances
    pool, n_pass = oracle.variance_pool(img, 4, 2, 1e9, min_pool=37)
    v = _window_vars(img, 8, 2)
    order = sorted(range(len(v)), key=lambda j: (-round(v[j] * 64 * 64), j))[:37]
    assert n_pass == 0 and list(pool) == sorted(order)


def test_variance_pool_constant_image():
    img = np.full((32, 32), 90, np.uint8)
    pool, n = oracle.variance_pool(img, 4, 4, 0.0, min_pool=5)
    assert n == 0 and list(pool) == [0, 1, 2, 3, 4]
    pool, n = oracle.variance_pool(img, 4, 4, -1.0, min_pool=5)
    assert n == len(pool) == 49  # (32 - 8) / 4 + 1 = 7 domains per side


# --------------------------------------------------------------------------- contrast histograms
def test_s_histogram_counts_kept_leaves():
    img = synth.power_law(64, beta=2.0, seed=5, n_rect=2)
    hist = oracle.s_histogram(img)
    codes, stats = oracle.encode_image(img, s_sets=(oracle.PLAIN_K,) * 4, entropy=False)
    assert [int(v) for v in hist.sum(axis=1)] == [s["accepted"] for s in stats] + [0] * (4 - len(stats))
    low = oracle.s_histogram(img, low_only=True)
    assert (low <= hist).all()
    # the mean of the low-entropy histogram is the calibrated value
    cal = oracle.calibrate_s(img)
    for l in range(4):
        if low[l].sum():
            mean = Fraction(int((low[l] * np.arange(11)).sum()), int(low[l].sum()))
            assert cal[l] == (math.floor(mean + Fraction(1, 2)),)


def test_select_s_rule():
    h = np.zeros((4, 11), dtype=np.int64)
    h[0, 3] = 10; h[0, 7] = 5; h[0, 1] = 4          # second at exactly half
    h[1, 9] = 10; h[1, 2] = 4                         # second below half
    h[2, 4] = 6; h[2, 6] = 6                          # tie: smaller k first
    assert oracle.select_s(h, 0.5) == ((3, 7), (9,), (4, 6), ())
    assert oracle.select_s(h, 0.0)[1] == (2, 9)
    assert oracle.select_s(h, 1.0)[0] == (3,)


# --------------------------------------------------------------------------- calibrated contrast values
def _calibration_image(k):
    """8 x 16 image for the levels (4, 2), fixed by construction.

    Left half: the 4 x 4 range at (0, 0) holds six grey levels, one per 8-bin
    histogram bin 0..5, with counts {4, 4, 2, 2, 2, 2} (entropy exactly 2.5
    bits); the other three left ranges are constant (200). Right half: the one
    domain at x = 8 whose 2 x 2 cells are constant with R = (k/10) d + 16, so
    the range at (0, 0) is an exact scaled copy (E = 0, contrast k). The four
    right ranges are two-tone checkers of 2 x 2 cells (1 bit each) that no
    domain matches within RMS 8, so they split into constant 2 x 2 children.
    """
    v = np.array([16, 48, 80, 112, 144, 176])
    q = lambda a, b: np.array([[a, b], [b, a]])
    r6 = np.block([[q(v[0], v[1]), q(v[0], v[2])], [q(v[1], v[3]), q(v[4], v[5])]])
    img = np.full((8, 16), 200, np.int64)
    img[0:4, 0:4] = r6
    d = (r6 - 16) * 10 // k
    assert ((d * k) == (r6 - 16) * 10).all()
    img[0:8, 8:16] = np.kron(d, np.ones((2, 2), np.int64))
    return img.astype(np.uint8)


def _brute_best(img, ry, rx, B, L):
    """Literal eq. (1) in Fractions over every (domain, isometry, k of the 11-value grid)."""
    H, W = img.shape
    gx = (W - 2 * B) // L + 1
    r = [int(v) for v in img[ry:ry + B, rx:rx + B].ravel()]
    n = len(r)
    cands = []
    for j in range(((H - 2 * B) // L + 1) * gx):
        y, x = (j // gx) * L, (j % gx) * L
        blk = img[y:y + 2 * B, x:x + 2 * B].astype(np.int64)
        dm = blk[0::2, 0::2] + blk[0::2, 1::2] + blk[1::2, 0::2] + blk[1::2, 1::2]
        for t in range(8):
            d = [Fraction(int(v), 4) for v in np_iso(dm, t).ravel()]
            for k in range(11):
                s = Fraction(k, 10)
                o = Fraction(sum(r), n) - s * sum(d) / n
                cands.append((sum((s * di + o - ri) ** 2 for di, ri in zip(d, r)), j, t, k))
    return min(cands)


@pytest.mark.parametrize("k,expect,all_active", [(10, 3, 2), (8, 2, 3)])
def test_calibrate_s_constructed(orc, k, expect, all_active):
    """The abstract's "mean optimal s of low-entropy ranges", on an image whose answer is fixed
    by construction. Level 0 keeps the exact copy (contrast k, entropy exactly 2.5 bits, so it
    is low: H <= 2.5) and three constant ranges (contrast 0, the first candidate); the four
    checkers split. Mean k/4, rounded half up: 10/4 -> 3 and 8/4 -> 2. The three plausible
    misreadings give other values: a strict H < 2.5 drops the copy (0), rounding half down gives
    2 for 2.5, and averaging every active range instead of the kept ones gives ``all_active``.
    Level 1 holds only constant children: 0."""
    img = _calibration_image(k)
    # the construction, checked by brute force
    assert _brute_best(img, 0, 0, 4, 2) == (0, 4, 0, k)
    assert scipy.stats.entropy(orc.hist8(img[0:4, 0:4]), base=2) == pytest.approx(2.5)
    for ry, rx in [(0, 4), (4, 0), (4, 4)]:
        assert _brute_best(img, ry, rx, 4, 2) == (0, 0, 0, 0)
    split_k = []
    for ry, rx in [(0, 8), (0, 12), (4, 8), (4, 12)]:
        E, _, _, kk = _brute_best(img, ry, rx, 4, 2)
        assert E > 64 * 16 and len(np.unique(img[ry:ry + 4, rx:rx + 4] >> 5)) == 2
        split_k.append(kk)
    assert math.floor(Fraction(k + sum(split_k), 8) + Fraction(1, 2)) == all_active != expect
    assert orc.calibrate_s(img, levels=(4, 2)) == ((expect,), (0,))


def test_calibrate_s_fallback(orc):
    """A level with no kept low-entropy range keeps the printed value of Section 3.1: a
    constant image is kept whole at the first level, so the second level is empty."""
    img = np.full((16, 16), 90, np.uint8)
    assert orc.calibrate_s(img, levels=(4, 2)) == ((0,), orc.PAPER_K[1])
    assert orc.calibrate_s(img, levels=(4, 2), fallback=((1,), (7,))) == ((0,), (7,))
