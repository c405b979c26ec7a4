"""Pins of the reference bitstream: hand-counted sizes, field positions,
round trips through the reader, and decodes of the round-tripped codes."""
import numpy as np
import pytest

import oracle
from oracle import bitstream as bs
from paper_1501_04140_amd import synth


def test_bits_for():
    assert [bs.bits_for(x) for x in (0, 1, 2, 3, 4, 5, 256, 257, 259081)] == [0, 0, 1, 2, 2, 3, 8, 9, 18]


def test_hand_counted_single_level_stream():
    img = synth.power_law(32, beta=2.0, seed=0)
    codes, stats = oracle.encode_image(img, s_sets=((1,),), levels=(16,), steps=(8,), entropy=False)
    data = bs.pack(codes, stats, 32, 32, (16,), (8,), ((1,),))
    # header 16+8+16+16+5+3 = 64, level 16+4+4+1 = 25; 4 leaves x (0 domain bits, the grid
    # has one domain) + 3 + 0 + 9
    assert bs.stream_bits(stats, 32, 32, (16,), (8,), ((1,),)) == 64 + 25 + 4 * 12
    assert len(data) == (64 + 25 + 48 + 7) // 8
    assert data[0] == 0xC5 and data[1] == 0xF1 and data[2] == 1
    assert data[3] | (data[4] << 8) == 32 and data[5] | (data[6] << 8) == 32
    assert data[7] & 31 == 16 and data[7] >> 5 == 1


@pytest.mark.parametrize("size,kw", [(64, dict(min_pool=64)), (96, dict(min_pool=32, variance=150.0)),
                                     (64, dict(entropy=False, s_sets=(oracle.PLAIN_K,) * 4))])
def test_round_trip_and_decode(size, kw):
    img = synth.power_law(size, beta=2.0, seed=1, n_rect=2)
    s_sets = kw.pop("s_sets", oracle.PAPER_K)
    codes, stats = oracle.encode_image(img, s_sets=s_sets, **kw)
    steps = oracle.default_steps()
    data = bs.pack(codes, stats, size, size, oracle.LEVEL_SIDES, steps, s_sets)
    assert len(data) * 8 - 8 < bs.stream_bits(stats, size, size, oracle.LEVEL_SIDES, steps, s_sets) <= len(data) * 8
    got, H, W = bs.unpack(data)
    assert (H, W) == (size, size) and len(got) == len(codes)
    for f in ("level", "y", "x", "B", "dom", "dy", "dx", "iso", "s_idx", "k", "q_o"):
        assert np.array_equal(got[f], codes[f]), f
    assert np.array_equal(oracle.decode(got, H, W, iters=8), oracle.decode(codes, H, W, iters=8))


def test_signed_offsets_round_trip():
    codes = np.zeros(2, dtype=oracle.CODE_DTYPE)
    codes["level"] = 0
    codes["y"], codes["x"], codes["B"] = [0, 0], [0, 16], 16
    codes["q_o"] = [-255, 255]
    codes["iso"] = [7, 3]
    stats = [dict(active=2, accepted=2, filtered=False, split=np.zeros(2, bool), pool_list=np.arange(1))]
    data = bs.pack(codes, stats, 16, 32, (16,), (8,), ((5,),))
    got, _, _ = bs.unpack(data)
    assert list(got["q_o"]) == [-255, 255] and list(got["iso"]) == [7, 3] and list(got["k"]) == [5, 5]
