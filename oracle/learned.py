"""Learned domain proposal, plain fp64 definition -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the GPU library never loads it and shares no code with it.

The exhaustive search of Section 2 compares every range with every domain in
all eight isometries. This extension lets a small network propose, per 8 x 8
range, the ``k`` domains most likely to hold the argmin; the exact distance of
eq. (1) (offset of eq. (3), contrast s = k/10) is then evaluated over those
domains only, and a range whose best proposed match would be split by the
RMS test of Section 2 falls back to the exhaustive search over every domain.

Definitions used here (each written out in fp64 with numpy matrix products as
the only library step):

* block vector: the 64 values of a block (range pixels, or the 2x2 sums of a
  domain), mean removed, scaled to unit Euclidean norm; the zero vector for a
  constant block;
* network f: 64 -> 256 -> 256 -> 64, ReLU after the first two layers, weights
  stored as in a linear map y = W x + b with W of shape (out, in);
* embedding g(x) = S / |S| with S = sum over the 8 isometries T_t of f(T_t x)
  (0 if S = 0). Summing over the isometry group makes g invariant under them;
* similarity of a range and a domain: the dot product of the int8 codes of
  their embeddings, q = rint(x s) with one scale s = 127 / max |x| over the
  ranges' and the domains' embeddings together, evaluated in fp32 (one
  correctly rounded division, one rounded product per value, ties to even):
  an integer. Proposal = the ``k`` most similar domains, ties to the lower
  domain index. (The proposal is this extension's own choice; it does not
  change what the exact rescoring and the fallback compute.);
* training loss: mean over ranges of the softmax cross-entropy of the
  similarities / tau over all domains of the image, against the exhaustive
  argmin domain; gradients by hand-derived back-propagation;
* optimiser: Adam (Kingma & Ba) with bias correction.
"""
from __future__ import annotations

import numpy as np

from . import PLAIN_K, Q, accept, domain_grid, full_ranges, isometry, match_level

D_IN, D_HID, D_OUT = 64, 256, 64
SHAPES = (("W1", (D_HID, D_IN)), ("b1", (D_HID,)), ("W2", (D_HID, D_HID)), ("b2", (D_HID,)),
          ("W3", (D_OUT, D_HID)), ("b3", (D_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
BLOCK = 8  # range side of the learned form


def unpack(theta):
    """Flat parameter vector -> dict of views (W1, b1, W2, b2, W3, b3 in that order)."""
    theta = np.asarray(theta)
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    return out


def _perms():
    base = np.arange(BLOCK * BLOCK, dtype=np.int32).reshape(BLOCK, BLOCK)
    return np.stack([isometry(base, t).ravel() for t in range(8)])


_PERM = None


def iso_perms() -> np.ndarray:
    """Row t: source index of each output element of T_t on an 8 x 8 block."""
    global _PERM
    if _PERM is None:
        _PERM = _perms()
    return _PERM


# --------------------------------------------------------------------------- block vectors
def block_vectors(blocks) -> np.ndarray:
    """Mean-removed, unit-norm rows (zero row for a constant block)."""
    v = np.asarray(blocks, dtype=np.float64).reshape(-1, BLOCK * BLOCK)
    c = v - v.mean(axis=1, keepdims=True)
    nrm = np.sqrt((c * c).sum(axis=1, keepdims=True))
    return np.where(nrm > 0, c / np.where(nrm > 0, nrm, 1.0), 0.0)


def range_blocks(img: np.ndarray, yx) -> np.ndarray:
    """Pixels of the 8 x 8 ranges at the given corners, [n, 64]."""
    img = np.asarray(img, dtype=np.int64)
    yx = np.asarray(yx, dtype=np.int64).reshape(-1, 2)
    ii, cc = np.mgrid[0:BLOCK, 0:BLOCK]
    return img[yx[:, 0, None, None] + ii, yx[:, 1, None, None] + cc].reshape(-1, 64)


def domain_blocks(img: np.ndarray, L: int, idx=None) -> np.ndarray:
    """2x2 sums (0..1020) of the 16 x 16 domains with raster index idx on the step-L grid."""
    img = np.asarray(img, dtype=np.int64)
    H, W = img.shape
    gy, gx = domain_grid(H, W, BLOCK, L)
    idx = np.arange(gy * gx) if idx is None else np.asarray(idx, dtype=np.int64)
    s2 = img[:-1, :-1] + img[:-1, 1:] + img[1:, :-1] + img[1:, 1:]
    y0, x0 = (idx // gx) * L, (idx % gx) * L
    ii, cc = np.mgrid[0:BLOCK, 0:BLOCK]
    return s2[y0[:, None, None] + 2 * ii, x0[:, None, None] + 2 * cc].reshape(-1, 64)


# --------------------------------------------------------------------------- network
def mlp_forward(p: dict, U: np.ndarray):
    a1 = U @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (U, a1, h1, a2, h2)


def embed(theta, X: np.ndarray):
    """g(x) for each row of X ([n, 64] block vectors). Returns (G [n, 64], cache)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64).reshape(-1, 64)
    n = X.shape[0]
    U = X[:, iso_perms()].reshape(n * 8, 64)  # row 8 q + t = T_t x_q
    y, cache = mlp_forward(p, U)
    S = y.reshape(n, 8, D_OUT).sum(axis=1)
    nrm = np.sqrt((S * S).sum(axis=1, keepdims=True))
    G = np.where(nrm > 0, S / np.where(nrm > 0, nrm, 1.0), 0.0)
    return G, (p, cache, S, nrm)


def _embed_backward(dG, ecache, grads):
    p, (U, a1, h1, a2, h2), S, nrm = ecache
    safe = np.where(nrm > 0, nrm, 1.0)
    G = S / safe
    dS = np.where(nrm > 0, (dG - G * (G * dG).sum(axis=1, keepdims=True)) / safe, 0.0)
    dy = np.repeat(dS, 8, axis=0)  # every isometry's output feeds S with weight 1
    grads["W3"] += dy.T @ h2
    grads["b3"] += dy.sum(axis=0)
    da2 = (dy @ p["W3"]) * (a2 > 0)
    grads["W2"] += da2.T @ h1
    grads["b2"] += da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (a1 > 0)
    grads["W1"] += da1.T @ U
    grads["b1"] += da1.sum(axis=0)


def loss_and_grad(theta, XR, XD, labels, tau: float):
    """Mean softmax cross-entropy of (g(r) . g(d_j)) / tau over all domains j against
    the label domain of each range, and its gradient (flat, same layout as theta)."""
    labels = np.asarray(labels, dtype=np.int64)
    GR, cR = embed(theta, XR)
    GD, cD = embed(theta, XD)
    nr = GR.shape[0]
    Z = GR @ GD.T / tau
    zmax = Z.max(axis=1, keepdims=True)
    ez = np.exp(Z - zmax)
    se = ez.sum(axis=1, keepdims=True)
    lse = zmax[:, 0] + np.log(se[:, 0])
    loss = float(np.mean(lse - Z[np.arange(nr), labels]))
    P = ez / se
    P[np.arange(nr), labels] -= 1.0
    P /= nr
    dGR = P @ GD / tau
    dGD = P.T @ GR / tau
    grads = {name: np.zeros(shape) for name, shape in SHAPES}
    _embed_backward(dGR, cR, grads)
    _embed_backward(dGD, cD, grads)
    flat = np.concatenate([grads[name].ravel() for name, _ in SHAPES])
    return loss, flat


def adam_step(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1). Returns (theta, m, v)."""
    theta = np.asarray(theta, np.float64)
    grad = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------- proposals
def quantize(*sets):
    """int8 codes (as int64 arrays) of embedding rows and their common scale:
    q = rint(x s), s = 127 / max |x| over every value of every set (0 when all
    are 0), in fp32 arithmetic."""
    xs = [np.asarray(x, np.float32) for x in sets]
    m = max((float(np.abs(x).max()) for x in xs if x.size), default=0.0)
    s = np.float32(127.0) / np.float32(m) if m > 0 else np.float32(0.0)
    return [np.rint(x * s).astype(np.int64) for x in xs], s


def similarity(GR, GD) -> np.ndarray:
    """Integer similarities [ranges, domains]: dot products of the int8 codes."""
    (qr, qd), _ = quantize(GR, GD)
    return qr @ qd.T


def topk(GR, GD, k: int) -> np.ndarray:
    """Indices of the k most similar domains per row, best first; ties to the lower index."""
    S = similarity(GR, GD)
    k = min(k, S.shape[1])
    out = np.empty((S.shape[0], k), dtype=np.int32)
    cols = np.arange(S.shape[1])
    for q in range(S.shape[0]):
        order = np.lexsort((cols, -S[q]))
        out[q] = order[:k]
    return out


def learned_match(img: np.ndarray, theta, L: int, k: int, s_k=PLAIN_K, rms: float = 8.0,
                  ranges=None, proposals=None):
    """Proposal encoder at one level with 8 x 8 ranges.

    Each range is matched exactly (eq. 1, exhaustive over isometries and s) against
    its k proposed domains; if that best match fails the RMS test (E > rms^2 n), the
    range is matched against every domain instead. ``proposals`` replaces the
    network's top-k lists (for checking another implementation's lists).
    Returns (matches, fallback flags, proposal lists).
    """
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    ranges = full_ranges(H, W, BLOCK) if ranges is None else np.asarray(ranges, np.int32).reshape(-1, 2)
    if proposals is None:
        GR, _ = embed(theta, block_vectors(range_blocks(img, ranges)))
        GD, _ = embed(theta, block_vectors(domain_blocks(img, L)))
        proposals = topk(GR, GD, k)
    n = BLOCK * BLOCK
    out = []
    fb = np.zeros(len(ranges), dtype=bool)
    for q in range(len(ranges)):
        pool = np.unique(np.asarray(proposals[q], np.int32))
        m = match_level(img, BLOCK, L, s_k, pool, ranges[q:q + 1])
        if not accept(int(m["e_lit"][0]), n, rms):
            fb[q] = True
            m = match_level(img, BLOCK, L, s_k, None, ranges[q:q + 1])
        out.append(m)
    return np.concatenate(out), fb, np.asarray(proposals)


def recall(proposals, labels) -> float:
    """Fraction of ranges whose exhaustive argmin domain is among its proposals."""
    proposals = np.asarray(proposals)
    labels = np.asarray(labels).reshape(-1, 1)
    return float((proposals == labels).any(axis=1).mean())


__all__ = ["N_PARAMS", "SHAPES", "unpack", "iso_perms", "block_vectors", "range_blocks", "quantize", "similarity",
           "domain_blocks", "mlp_forward", "embed", "loss_and_grad", "adam_step", "topk",
           "learned_match", "recall", "Q"]
