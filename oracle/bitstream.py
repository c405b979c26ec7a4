"""Bitstream of a quadtree encode, plain reference writer and reader -- TEST
INFRASTRUCTURE ONLY (imported by the tests, never by the GPU library).

The paper reports compression ratios (Section 4, Tables 1-2) but gives no bit
allocation; this fixed-length format is the reading used here. Bit b of the
stream is bit (b mod 8) of byte b // 8 (least significant first).

  header   magic 0xF1C5 (16), version 1 (8), H (16), W (16), B0 (5), n_levels (3);
           per level: L (16), n_s (4), the n_s contrast numerators k (4 each),
           listed (1); if listed: pool size P (24) and the P ascending grid
           indices of the pool (g bits each, g = bits for the grid size).
           A level is listed iff a pool filter is on, it has leaves, and the
           list makes the level shorter: 24 + P g + leaves bits(P) < leaves g.
  flags    for every level but the last, one bit per active range in
           active-list order: 1 = split into TL, TR, BL, BR.
  leaves   in code order (level by level, active-list order): the domain's
           position in the level's pool (bits for P; the grid index when the
           level is not listed), isometry (3), contrast index (bits for n_s),
           offset q_o (9, two's complement).

"bits for x" is ceil(log2 x) for x >= 2 and 0 otherwise.
"""
from __future__ import annotations

import numpy as np

from . import CODE_DTYPE, domain_grid

MAGIC = 0xF1C5
VERSION = 1


def bits_for(x: int) -> int:
    return 0 if x <= 1 else int(x - 1).bit_length()


def _listed(st, H, W, B, L) -> bool:
    if st is None or not st["filtered"] or st["active"] == 0 or st["accepted"] == 0:
        return False
    gy, gx = domain_grid(H, W, B, L)
    g = bits_for(gy * gx)
    P = len(st["pool_list"])
    return 24 + P * g + st["accepted"] * bits_for(P) < st["accepted"] * g


class _Writer:
    def __init__(self):
        self.bits = []

    def put(self, value: int, width: int):
        for i in range(width):
            self.bits.append((int(value) >> i) & 1)

    def tobytes(self) -> bytes:
        out = bytearray((len(self.bits) + 7) // 8)
        for i, b in enumerate(self.bits):
            if b:
                out[i >> 3] |= 1 << (i & 7)
        return bytes(out)


class _Reader:
    def __init__(self, data: bytes):
        self.data = data
        self.pos = 0

    def get(self, width: int) -> int:
        v = 0
        for i in range(width):
            p = self.pos + i
            v |= ((self.data[p >> 3] >> (p & 7)) & 1) << i
        self.pos += width
        return v


def pack(codes, stats, H: int, W: int, levels, steps, s_sets) -> bytes:
    """Stream of the encode (codes, stats) returned by ``encode_image``."""
    w = _Writer()
    w.put(MAGIC, 16)
    w.put(VERSION, 8)
    w.put(H, 16)
    w.put(W, 16)
    w.put(levels[0], 5)
    w.put(len(levels), 3)
    for lv, (B, L) in enumerate(zip(levels, steps)):
        w.put(L, 16)
        w.put(len(s_sets[lv]), 4)
        for k in s_sets[lv]:
            w.put(k, 4)
        st = stats[lv] if lv < len(stats) else None
        listed = _listed(st, H, W, B, L)
        w.put(int(listed), 1)
        if listed:
            gy, gx = domain_grid(H, W, B, L)
            g = bits_for(gy * gx)
            w.put(len(st["pool_list"]), 24)
            for j in st["pool_list"]:
                w.put(int(j), g)
    for lv in range(len(levels) - 1):
        if lv < len(stats):
            for f in stats[lv]["split"]:
                w.put(int(f), 1)
    for c in codes:
        lv = int(c["level"])
        st = stats[lv]
        B, L = levels[lv], steps[lv]
        gy, gx = domain_grid(H, W, B, L)
        if _listed(st, H, W, B, L):
            pos = int(np.searchsorted(st["pool_list"], int(c["dom"])))
            assert st["pool_list"][pos] == c["dom"]
            w.put(pos, bits_for(len(st["pool_list"])))
        else:
            w.put(int(c["dom"]), bits_for(gy * gx))
        w.put(int(c["iso"]), 3)
        w.put(int(c["s_idx"]), bits_for(len(s_sets[lv])))
        w.put(int(c["q_o"]) & 0x1FF, 9)
    return w.tobytes()


def unpack(data: bytes):
    """(codes, H, W) from a stream; e_lit is -1 (not stored)."""
    r = _Reader(data)
    if r.get(16) != MAGIC or r.get(8) != VERSION:
        raise ValueError("not a stream of this format")
    H, W = r.get(16), r.get(16)
    B0, nl = r.get(5), r.get(3)
    levels = [B0 >> l for l in range(nl)]
    steps, ksets, pools = [], [], []
    for lv in range(nl):
        steps.append(r.get(16))
        ns = r.get(4)
        ksets.append([r.get(4) for _ in range(ns)])
        if r.get(1):
            gy, gx = domain_grid(H, W, levels[lv], steps[lv])
            P = r.get(24)
            g = bits_for(gy * gx)
            pools.append([r.get(g) for _ in range(P)])
        else:
            pools.append(None)
    # flags: rebuild the active lists
    active = [[(y * B0, x * B0) for y in range(H // B0) for x in range(W // B0)]]
    splits = []
    for lv in range(nl - 1):
        f = [r.get(1) for _ in active[lv]]
        splits.append(f)
        h = levels[lv] // 2
        nxt = []
        for (y, x), s in zip(active[lv], f):
            if s:
                nxt += [(y, x), (y, x + h), (y + h, x), (y + h, x + h)]
        active.append(nxt)
    splits.append([0] * len(active[nl - 1]))
    out = []
    for lv in range(nl):
        B, L = levels[lv], steps[lv]
        gy, gx = domain_grid(H, W, B, L)
        for (y, x), s in zip(active[lv], splits[lv]):
            if s:
                continue
            if pools[lv] is not None:
                dom = pools[lv][r.get(bits_for(len(pools[lv])))]
            else:
                dom = r.get(bits_for(gy * gx))
            iso = r.get(3)
            si = r.get(bits_for(len(ksets[lv])))
            q = r.get(9)
            q = q - 512 if q >= 256 else q
            out.append((lv, y, x, B, dom, (dom // gx) * L, (dom % gx) * L, iso, si,
                        ksets[lv][si], q, -1))
    return np.array(out, dtype=CODE_DTYPE), H, W


def stream_bits(stats, H: int, W: int, levels, steps, s_sets) -> int:
    """Length of the stream in bits, from the encode's counts alone."""
    n = 16 + 8 + 32 + 8
    for lv, (B, L) in enumerate(zip(levels, steps)):
        n += 16 + 4 + 4 * len(s_sets[lv]) + 1
        st = stats[lv] if lv < len(stats) else None
        if _listed(st, H, W, B, L):
            gy, gx = domain_grid(H, W, B, L)
            n += 24 + len(st["pool_list"]) * bits_for(gy * gx)
    for lv, st in enumerate(stats):
        if lv < len(levels) - 1:
            n += st["active"]
        gy, gx = domain_grid(H, W, levels[lv], steps[lv])
        P = len(st["pool_list"]) if _listed(st, H, W, levels[lv], steps[lv]) else gy * gx
        n += st["accepted"] * (bits_for(P) + 3 + bits_for(len(s_sets[lv])) + 9)
    return n
