"""CPU oracle for the fractal encoder's hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never loads it, and the two share no code.

It is a plain, slow, obviously correct CPU version of what the encoder
computes, written from the paper (Miar Naimi & Salarian, "A Fast Fractal Image
Compression Algorithm Using Predefined Values for Contrast Scaling"):

* range/domain geometry and the 8 isometries (Section 2);
* the distance E of eq. (1) with the offset of eq. (3), evaluated literally in
  exact integers by ``fic_oracle.c`` (exhaustive search, Section 2);
* the entropy of eqs. (4)-(5), computed exactly with big integers and used to
  keep only high-entropy domains (Section 3);
* the quadtree that splits badly matched ranges 16 -> 8 -> 4 -> 2 (Section 2,
  and the three cases at the end of Section 3.1);
* the per-step predefined contrast values (Section 3.1) and their estimate
  from low-entropy ranges (abstract, Section 3.1);
* a decoder and PSNR for the reconstructions the paper reports (Section 4).

Where the paper is silent the readings are fixed here and listed in the
design notes: 2x2-mean decimation kept exact, s = k/10, 8-bin (p >> 5)
histogram entropy in bits with a strict threshold, a floor of ``min_pool``
highest-entropy domains, split iff RMS error > T, round-half-up offsets, and
an integer decoder.

The calibrated contrast values (``calibrate_s``) are pinned on an image built
so that its kept low-entropy ranges, their best contrasts and their rounded
mean are known by construction (and checked by a Fraction brute force).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from fractions import Fraction

import numpy as np

Q = 10                                   # s = k / Q
LEVEL_SIDES = (16, 8, 4, 2)              # range sides of the four steps (Section 2)
PLAIN_K = tuple(range(11))               # s in {0, 0.1, ..., 1.0}
PAPER_K = ((1,), (2, 4), (3, 8), (5, 9))  # Section 3.1: {0.1}, {0.2,0.4}, {0.3,0.8}, {0.5,0.9}
N_ISO = 8

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fic_oracle.c")
_SO = os.path.join(_HERE, "_fic_oracle.so")
_lib = None


# --------------------------------------------------------------------------- build / load
def build(force: bool = True) -> str:
    """Compile the C part of the oracle (gcc, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        i32p, i64p = P(ctypes.c_int32), P(ctypes.c_int64)
        lib.orc_match_level.argtypes = [P(ctypes.c_uint8)] + [ctypes.c_int] * 5 + [
            i32p, ctypes.c_int, i32p, ctypes.c_int, i32p, ctypes.c_int,
            i64p, i32p, i32p, i32p, i64p]
        lib.orc_match_level.restype = ctypes.c_int
        lib.orc_eval.argtypes = [i32p, i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_eval.restype = ctypes.c_int64
        lib.orc_isometry.argtypes = [i32p, ctypes.c_int, ctypes.c_int, i32p]
        lib.orc_isometry.restype = None
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Thread count of the C search (OpenMP); timing only, results do not depend on it."""
    _load().orc_set_threads(int(n))


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# --------------------------------------------------------------------------- geometry (Section 2)
def range_grid(H: int, W: int, B: int):
    """Number of B x B range blocks per column and row; (N/n)^2 of them (Section 1)."""
    return H // B, W // B


def domain_grid(H: int, W: int, B: int, L: int):
    """Top-left corners of the 2B x 2B domains at step L: ((N-2B)/L + 1) per side.
    At L = 1 this is the (N - 2n + 1)^2 count of Section 1."""
    return (H - 2 * B) // L + 1, (W - 2 * B) // L + 1


def domain_yx(j, gx: int, L: int):
    j = np.asarray(j)
    return (j // gx) * L, (j % gx) * L


def full_ranges(H: int, W: int, B: int) -> np.ndarray:
    gy, gx = range_grid(H, W, B)
    yy, xx = np.mgrid[0:gy, 0:gx]
    return np.stack([yy.ravel() * B, xx.ravel() * B], axis=1).astype(np.int32)


def decimate(img: np.ndarray, y: int, x: int, B: int) -> np.ndarray:
    """Four times the 2x2 mean of the 2B x 2B block at (y, x): integers 0..1020."""
    blk = img[y:y + 2 * B, x:x + 2 * B].astype(np.int64)
    return blk[0::2, 0::2] + blk[0::2, 1::2] + blk[1::2, 0::2] + blk[1::2, 1::2]


def isometry(block: np.ndarray, t: int) -> np.ndarray:
    """T_t of a square block (C oracle's table, run through ctypes)."""
    b = np.ascontiguousarray(block, dtype=np.int32)
    B = b.shape[0]
    out = np.empty_like(b)
    _load().orc_isometry(_ptr(b, ctypes.c_int32), B, int(t), _ptr(out, ctypes.c_int32))
    return out


def eval_candidate(r: np.ndarray, dd: np.ndarray, t: int, k: int) -> int:
    """E * (4 Q n)^2 of eq. (1) for one candidate (range r, decimated domain dd)."""
    r = np.ascontiguousarray(r, dtype=np.int32)
    dd = np.ascontiguousarray(dd, dtype=np.int32)
    return int(_load().orc_eval(_ptr(r, ctypes.c_int32), _ptr(dd, ctypes.c_int32),
                                r.shape[0], int(t), int(k)))


# --------------------------------------------------------------------------- entropy (Section 3, eqs. 4-5)
def hist8(pixels: np.ndarray) -> np.ndarray:
    """Counts of the 8 grey-level bins of width 32 (bin = p >> 5)."""
    return np.bincount((np.asarray(pixels).ravel() >> 5).astype(np.int64), minlength=8)


def _plogp_product(counts) -> int:
    """prod_b c_b^c_b as an exact integer; log2 of it is sum_b c_b log2 c_b."""
    v = 1
    for c in counts:
        c = int(c)
        if c > 1:
            v *= c ** c
    return v


def entropy_bits(counts) -> float:
    """Shannon entropy in bits of a histogram (eq. 5 with log base 2), for reporting."""
    c = np.asarray(counts, dtype=np.float64)
    nw = c.sum()
    p = c[c > 0] / nw
    return float(-(p * np.log2(p)).sum())


def entropy_above(counts, theta: float) -> bool:
    """Exactly decide entropy(counts) > theta bits.

    H = log2 Nw - (1/Nw) sum c log2 c, so H > theta  <=>  sum c log2 c < m with
    m = Nw log2 Nw - Nw theta  <=>  prod c^c < 2^m, compared in big integers.
    """
    nw = int(np.sum(counts))
    lg = nw.bit_length() - 1
    if (1 << lg) != nw:
        raise ValueError("window size must be a power of two")
    m = Fraction(nw * lg) - nw * Fraction(theta)
    v = _plogp_product(counts)
    # v < 2^(p/q)  <=>  v^q < 2^p
    p, q = m.numerator, m.denominator
    if p < 0:
        return False
    return v ** q < (1 << p)


def _window_hists(img: np.ndarray, side: int, step: int):
    """8-bin histograms of every side x side window with top-left on the step grid."""
    bins = (np.asarray(img) >> 5).astype(np.uint8)
    win = np.lib.stride_tricks.sliding_window_view(bins, (side, side))[::step, ::step]
    gy, gx = win.shape[:2]
    out = np.empty((gy * gx, 8), dtype=np.int64)
    for b in range(8):
        out[:, b] = (win == b).sum(axis=(2, 3)).reshape(-1)
    return out


def entropy_pool(img: np.ndarray, B: int, L: int, theta: float = 2.5, min_pool: int = 256):
    """Domain pool of one level after the entropy filter of Section 3.

    Keep every 2B x 2B domain whose 8-bin entropy exceeds ``theta`` bits. If
    fewer than ``min_pool`` pass, the pool is instead the ``min_pool``
    highest-entropy domains (ties to the lower index). Returns (ascending
    index array, number that passed the threshold).
    """
    H, W = img.shape
    gy, gx = domain_grid(H, W, B, L)
    hists = _window_hists(img, 2 * B, L)
    uniq, inv = np.unique(hists, axis=0, return_inverse=True)
    inv = np.asarray(inv).ravel()
    keep_u = np.array([entropy_above(h, theta) for h in uniq], dtype=bool)
    keep = keep_u[inv]
    n_pass = int(keep.sum())
    if n_pass >= min_pool:
        return np.flatnonzero(keep).astype(np.int32), n_pass
    total = gy * gx
    if total <= min_pool:
        return np.arange(total, dtype=np.int32), n_pass
    # rank unique histograms by the exact value prod c^c (lower = higher entropy)
    vals = [_plogp_product(h) for h in uniq]
    order = sorted(range(len(uniq)), key=lambda u: vals[u])
    rank_u = np.empty(len(uniq), dtype=np.int64)
    r = 0
    for pos, u in enumerate(order):
        if pos > 0 and vals[u] != vals[order[pos - 1]]:
            r = pos
        rank_u[u] = r
    rank = rank_u[inv]
    idx = np.lexsort((np.arange(total), rank))[:min_pool]
    return np.sort(idx).astype(np.int32), n_pass


def variance_pool(img: np.ndarray, B: int, L: int, vmin: float, min_pool: int = 256):
    """Domain pool of one level by pixel variance (the classical alternative the paper
    cites to the entropy filter): keep every 2B x 2B domain whose variance exceeds
    ``vmin`` (strictly, the float32 value compared exactly); if fewer than ``min_pool``
    pass, the ``min_pool`` highest-variance domains, ties to the lower index.
    Returns (ascending index array, number that passed)."""
    H, W = img.shape
    gy, gx = domain_grid(H, W, B, L)
    side = 2 * B
    N = side * side
    win = np.lib.stride_tricks.sliding_window_view(np.asarray(img, dtype=np.int64),
                                                   (side, side))[::L, ::L]
    s1 = win.sum(axis=(2, 3)).reshape(-1)
    s2 = (win * win).sum(axis=(2, 3)).reshape(-1)
    vp = N * s2 - s1 * s1                      # N^2 * variance, exact
    t = Fraction(float(np.float32(vmin))) * N * N
    keep = np.array([Fraction(int(v)) > t for v in vp], dtype=bool)
    n_pass = int(keep.sum())
    total = gy * gx
    if n_pass >= min_pool:
        return np.flatnonzero(keep).astype(np.int32), n_pass
    if total <= min_pool:
        return np.arange(total, dtype=np.int32), n_pass
    idx = np.lexsort((np.arange(total), -vp))[:min_pool]
    return np.sort(idx).astype(np.int32), n_pass


def range_entropy_low(img: np.ndarray, y: int, x: int, B: int, theta: float = 2.5) -> bool:
    """True iff the B x B range block's 8-bin entropy is <= theta bits (a low-activity range)."""
    return not entropy_above(hist8(img[y:y + B, x:x + B]), theta)


# --------------------------------------------------------------------------- matching (Section 2)
MATCH_DTYPE = np.dtype([("e_lit", np.int64), ("second", np.int64), ("dom", np.int32),
                        ("iso", np.int32), ("s_idx", np.int32), ("k", np.int32),
                        ("q_o", np.int32), ("dy", np.int32), ("dx", np.int32)])


def quantise_o(sum_r: int, sum_dd: int, k: int, n: int) -> int:
    """Offset of eq. (3), o = (4Q sumR - k sumDD) / (4Q n), rounded half up to an integer."""
    num = 2 * (4 * Q * sum_r - k * sum_dd) + 4 * Q * n
    return num // (8 * Q * n)


def match_level(img: np.ndarray, B: int, L: int, s_k=PLAIN_K, pool=None, ranges=None):
    """Exhaustive argmin of eq. (1) for every range block at one level.

    ``pool``: ascending domain indices (default: the whole grid).
    ``ranges``: (n, 2) int32 top-left corners (default: the whole range grid).
    Returns a structured array (MATCH_DTYPE); e_lit = E * (4 Q n)^2 exactly.
    """
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    gy, gx = domain_grid(H, W, B, L)
    if pool is None:
        pool = np.arange(gy * gx, dtype=np.int32)
    if ranges is None:
        ranges = full_ranges(H, W, B)
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    ranges = np.ascontiguousarray(ranges, dtype=np.int32).reshape(-1, 2)
    sk = np.ascontiguousarray(s_k, dtype=np.int32)
    nr = ranges.shape[0]
    out = np.zeros(nr, dtype=MATCH_DTYPE)
    if nr == 0:
        return out
    be = np.empty(nr, np.int64)
    se = np.empty(nr, np.int64)
    bj = np.empty(nr, np.int32)
    bt = np.empty(nr, np.int32)
    bs = np.empty(nr, np.int32)
    rc = _load().orc_match_level(_ptr(img, ctypes.c_uint8), H, W, W, B, L,
                                 _ptr(sk, ctypes.c_int32), len(sk), _ptr(pool, ctypes.c_int32),
                                 len(pool), _ptr(ranges, ctypes.c_int32), nr,
                                 _ptr(be, ctypes.c_int64), _ptr(bj, ctypes.c_int32),
                                 _ptr(bt, ctypes.c_int32), _ptr(bs, ctypes.c_int32),
                                 _ptr(se, ctypes.c_int64))
    if rc != 0:
        raise ValueError("orc_match_level rejected its arguments")
    n = B * B
    out["e_lit"], out["second"], out["dom"], out["iso"], out["s_idx"] = be, se, bj, bt, bs
    out["k"] = sk[bs]
    dy, dx = domain_yx(bj, gx, L)
    out["dy"], out["dx"] = dy, dx
    for q in range(nr):
        ry, rx = ranges[q]
        sr = int(img[ry:ry + B, rx:rx + B].astype(np.int64).sum())
        sd = int(decimate(img, int(dy[q]), int(dx[q]), B).sum())
        out["q_o"][q] = quantise_o(sr, sd, int(out["k"][q]), n)
    return out


# --------------------------------------------------------------------------- quadtree (Sections 2, 3.1)
CODE_DTYPE = np.dtype([("level", np.int32), ("y", np.int32), ("x", np.int32), ("B", np.int32),
                       ("dom", np.int32), ("dy", np.int32), ("dx", np.int32), ("iso", np.int32),
                       ("s_idx", np.int32), ("k", np.int32), ("q_o", np.int32),
                       ("e_lit", np.int64)])


def default_steps(levels=LEVEL_SIDES):
    """Domain step L = B/2 (1 at B = 2)."""
    return tuple(max(B // 2, 1) for B in levels)


def accept(e_lit: int, n: int, rms: float) -> bool:
    """Keep a transform iff its RMS error sqrt(E/n) <= rms, i.e. E <= rms^2 n."""
    t2 = Fraction(rms) ** 2
    return Fraction(e_lit) <= t2 * n * (4 * Q * n) ** 2


def encode_image(img: np.ndarray, s_sets=PAPER_K, levels=LEVEL_SIDES, steps=None,
                 rms: float = 8.0, entropy: bool = True, theta: float = 2.5,
                 min_pool: int = 256, variance: float | None = None):
    """Quadtree encoder: match every active range, keep it if its RMS error is at most
    ``rms`` (always at the last level), else split it into TL, TR, BL, BR children.

    Returns (codes, stats). Codes are in level order; within a level they follow the
    active list, which is raster order at the first level and, below it, the four
    children of each rejected range in the order of their parents. With ``variance``
    set, the pool filter is the variance filter with that threshold instead of the
    entropy filter.
    """
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    steps = default_steps(levels) if steps is None else steps
    if H % levels[0] or W % levels[0]:
        raise ValueError("image sides must be multiples of the first range size")
    active = full_ranges(H, W, levels[0])
    codes = []
    stats = []
    for lv, (B, L) in enumerate(zip(levels, steps)):
        gy, gx = domain_grid(H, W, B, L)
        if variance is not None:
            pool, n_pass = variance_pool(img, B, L, variance, min_pool)
        elif entropy:
            pool, n_pass = entropy_pool(img, B, L, theta, min_pool)
        else:
            pool, n_pass = np.arange(gy * gx, dtype=np.int32), gy * gx
        ks = s_sets[lv]
        m = match_level(img, B, L, ks, pool, active)
        n = B * B
        last = lv == len(levels) - 1
        children = []
        n_acc = 0
        split = np.zeros(len(active), dtype=bool)
        for q in range(len(active)):
            y, x = (int(v) for v in active[q])
            if last or accept(int(m["e_lit"][q]), n, rms):
                n_acc += 1
                codes.append((lv, y, x, B, m["dom"][q], m["dy"][q], m["dx"][q], m["iso"][q],
                              m["s_idx"][q], m["k"][q], m["q_o"][q], m["e_lit"][q]))
            else:
                split[q] = True
                h = B // 2
                children += [(y, x), (y, x + h), (y + h, x), (y + h, x + h)]
        stats.append(dict(B=B, L=L, pool=len(pool), passed=n_pass, active=len(active),
                          accepted=n_acc, matches=len(active) * len(pool) * N_ISO,
                          n_s=len(ks), pool_list=np.asarray(pool, np.int32), split=split,
                          filtered=bool(entropy or variance is not None), grid=gy * gx))
        active = np.array(children, dtype=np.int32).reshape(-1, 2)
        if len(active) == 0:
            break
    return np.array(codes, dtype=CODE_DTYPE), stats


def calibrate_s(img: np.ndarray, levels=LEVEL_SIDES, steps=None, rms: float = 8.0,
                theta: float = 2.5, fallback=PAPER_K):
    """Per-level contrast estimate from low-entropy ranges (abstract; Section 3.1).

    Runs the plain method (all 11 values of s, unfiltered pool) through the quadtree;
    at each level takes the ranges that were accepted and whose 8-bin entropy is
    <= ``theta`` bits, and rounds the mean of their best k half up. A level with no
    such range keeps ``fallback``. Returns one 1-tuple of k per level.
    """
    codes, _ = encode_image(img, s_sets=[PLAIN_K] * len(levels), levels=levels, steps=steps,
                            rms=rms, entropy=False)
    out = []
    for lv, B in enumerate(levels):
        ks = [int(c["k"]) for c in codes if c["level"] == lv
              and range_entropy_low(img, int(c["y"]), int(c["x"]), B, theta)]
        if ks:
            tot, cnt = sum(ks), len(ks)
            out.append(((2 * tot + cnt) // (2 * cnt),))
        else:
            out.append(tuple(fallback[lv]))
    return tuple(out)


# --------------------------------------------------------------------------- decoder (Section 4)
def s_histogram(img: np.ndarray, levels=LEVEL_SIDES, steps=None, rms: float = 8.0,
                low_only: bool = False, theta: float = 2.5) -> np.ndarray:
    """Counts [len(levels), 11] of the optimal contrast numerator k over the kept leaves
    of the plain quadtree (11 values, no pool filter) -- Section 3.1's Fig. 3 -- over
    all leaves, or only those whose range has 8-bin entropy <= theta."""
    codes, _ = encode_image(img, s_sets=(PLAIN_K,) * len(levels), levels=levels, steps=steps,
                            rms=rms, entropy=False)
    hist = np.zeros((len(levels), 11), dtype=np.int64)
    for c in codes:
        if low_only and not range_entropy_low(img, int(c["y"]), int(c["x"]), int(c["B"]), theta):
            continue
        hist[int(c["level"]), int(c["k"])] += 1
    return hist


def select_s(hist, second_frac: float = 0.5):
    """Per level: the most frequent k, and the second most frequent too when its count is at
    least ``second_frac`` of the first (ties to the smaller k). Empty levels give ()."""
    out = []
    for h in np.asarray(hist):
        order = sorted((k for k in range(11) if h[k] > 0), key=lambda k: (-h[k], k))
        if not order:
            out.append(())
        elif len(order) > 1 and h[order[1]] >= second_frac * h[order[0]]:
            out.append(tuple(sorted(order[:2])))
        else:
            out.append((order[0],))
    return tuple(out)


def decode(codes, H: int, W: int, iters: int = 64) -> np.ndarray:
    """Iterate the code's map from a mid-grey image, all in integers.

    One iteration rebuilds every leaf block from the previous image x:
    value = (k/Q) * (2x2 mean of the domain, isometry applied) + q_o, rounded
    half up and clamped to 0..255. All blocks read the previous image.
    """
    x = np.full(H * W, 128, dtype=np.int64)
    if len(codes) == 0:
        return x.reshape(H, W).astype(np.uint8)
    dst, src, kk, oo = [], [], [], []
    for B in sorted(set(int(b) for b in codes["B"])):
        ii, cc = np.mgrid[0:B, 0:B]
        for t in range(N_ISO):
            sel = codes[(codes["B"] == B) & (codes["iso"] == t)]
            if len(sel) == 0:
                continue
            # position inside the decimated domain that T_t moves to (i, c)
            smap = isometry(np.arange(B * B).reshape(B, B), t).ravel()
            si, sc = smap // B, smap % B
            ys = sel["y"][:, None] + ii.ravel()[None, :]
            xs = sel["x"][:, None] + cc.ravel()[None, :]
            dst.append((ys * W + xs).ravel())
            sy = sel["dy"][:, None] + 2 * si[None, :]
            sx = sel["dx"][:, None] + 2 * sc[None, :]
            base = sy * W + sx
            src.append(np.stack([base, base + 1, base + W, base + W + 1], axis=-1).reshape(-1, 4))
            kk.append(np.repeat(sel["k"].astype(np.int64), B * B))
            oo.append(np.repeat(sel["q_o"].astype(np.int64), B * B))
    dst, src = np.concatenate(dst), np.concatenate(src)
    kk, oo = np.concatenate(kk), np.concatenate(oo)
    if np.unique(dst).size != H * W or dst.size != H * W:
        raise ValueError("codes do not tile the image")
    for _ in range(iters):
        dd = x[src].sum(axis=1)
        v = (kk * dd + 4 * Q * oo + 2 * Q) // (4 * Q)
        nxt = np.empty_like(x)
        nxt[dst] = np.clip(v, 0, 255)
        x = nxt
    return x.reshape(H, W).astype(np.uint8)


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    """10 log10(255^2 / MSE) between two uint8 images (inf when equal)."""
    d = a.astype(np.int64) - b.astype(np.int64)
    sse = int((d * d).sum())
    if sse == 0:
        return float("inf")
    return 10.0 * math.log10(255.0 ** 2 * d.size / sse)
