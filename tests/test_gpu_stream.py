"""Bitstream packed on the GPU: byte-identical to the reference writer on the
oracle's own encode, and round-trips through the library's reader."""
import numpy as np
import pytest

import oracle
from oracle import bitstream as bs
from paper_1501_04140_amd import fic, synth

from test_gpu_parity import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fic.load()
    return torch.device("cuda:0")


CASES = [
    (64, dict(s_sets=oracle.PAPER_K, min_pool=64), {}),
    (96, dict(s_sets=oracle.PAPER_K, min_pool=32, entropy_mode=2, entropy_bits=150.0), dict(variance=150.0)),
    (64, dict(s_sets=(oracle.PLAIN_K,) * 4, entropy_mode=0), dict(entropy=False)),
    (128, dict(s_sets=((1,), (3,), (9,), (9,)), min_pool=256), {}),
    (512, dict(s_sets=oracle.PAPER_K, min_pool=256), {}),
]


@pytest.mark.parametrize("size,pk,ok", CASES)
def test_gpu_stream_equals_reference(dev, size, pk, ok):
    img = synth.quadtree_image(0) if size == 512 else synth.power_law(size, beta=2.0, seed=size, n_rect=3)
    params = fic.EncoderParams(**pk)
    say(f"[stream] size={size} params={pk}")
    data, codes, n, _ = fic.encode_image_stream(torch.from_numpy(img).to(dev), params)
    ref_codes, stats = oracle.encode_image(img, s_sets=pk["s_sets"], min_pool=pk.get("min_pool", 256), **ok)
    ref = bs.pack(ref_codes, stats, size, size, oracle.LEVEL_SIDES, oracle.default_steps(), pk["s_sets"])
    assert bytes(data) == ref
    got, H, W = fic.unpack_stream(data)
    gpu = fic.codes_numpy(codes, n)
    assert (H, W) == (size, size) and len(got) == len(gpu)
    for f in ("level", "y", "x", "dom", "dy", "dx", "iso", "s_idx", "k", "q_o", "log2B"):
        assert np.array_equal(got[f], gpu[f]), f
    ratio = size * size * 8 / (len(data) * 8)
    say(f"[stream] {len(data)} bytes, {len(data) * 8 / (size * size):.3f} bpp, ratio {ratio:.2f}")
    # decoding the unpacked codes gives the decode of the encoder's codes
    gd = torch.from_numpy(got.view(np.uint8).reshape(-1, 32)).to(dev)
    a = fic.decode(gd, len(got), size, size, iters=8)
    b = fic.decode(codes, int(n.item()), size, size, iters=8)
    assert torch.equal(a, b)
