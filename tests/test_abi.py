"""C-ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before any device call (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1501_04140_amd import fic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fic.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fic_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return fic.load()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert {"fic_encode_level", "fic_encode_image", "fic_decode", "fic_last_error"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert lib.fic_version() == 100


def test_struct_layouts_match_header():
    assert fic.MATCH_DTYPE.itemsize == 24
    assert fic.CODE_DTYPE.itemsize == 32
    assert fic.STATS_DTYPE.itemsize == 24
    assert ctypes.sizeof(fic.Params) == 4 + 4 + 16 + 16 + 48 + 4 + 4 + 4 + 4


def _level(lib, **kw):
    a = dict(img=1, H=64, W=64, pitch=64, B=8, L=4, s_k=(0, 1, 2), n_s=None, mode=0, bits=2.5,
             min_pool=1, ranges=None, n_ranges=None, out=1)
    a.update(kw)
    ks = (ctypes.c_int8 * 16)(*a["s_k"])
    n_s = len(a["s_k"]) if a["n_s"] is None else a["n_s"]
    n_r = (a["H"] // max(a["B"], 1)) * (a["W"] // max(a["B"], 1)) if a["n_ranges"] is None else a["n_ranges"]
    rc = lib.fic_encode_level(a["img"], a["H"], a["W"], a["pitch"], a["B"], a["L"], ks, n_s,
                              a["mode"], a["bits"], a["min_pool"], a["ranges"], n_r, a["out"],
                              None, None, None)
    return rc, lib.fic_last_error().decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(img=None), "image pointer"),
    (dict(B=3), "range side"),
    (dict(B=32), "range side"),
    (dict(H=60), "multiple"),
    (dict(H=8, W=8), "smaller than a domain"),
    (dict(pitch=32), "pitch"),
    (dict(L=0), "step"),
    (dict(s_k=(2, 1)), "increasing"),
    (dict(s_k=(0, 11)), "not in 0..10"),
    (dict(s_k=tuple(range(11)) + (0,), n_s=12), "size"),
    (dict(n_s=0), "size"),
    (dict(mode=3), "entropy_mode"),
    (dict(mode=-1), "entropy_mode"),
    (dict(min_pool=0), "min_pool"),
    (dict(n_ranges=5), "n_ranges"),
    (dict(out=None), "out is NULL"),
    (dict(H=32768, W=64), "above"),
])
def test_encode_level_rejects(lib, kw, frag):
    rc, msg = _level(lib, **kw)
    assert rc == fic.FIC_EINVAL and frag in msg


def test_encode_level_noalloc_checks_on_the_host(lib):
    """The same argument checks as fic_encode_level, and a level whose buffers
    exceed the fixed scratch is refused (with the bytes it needs) before any
    device call."""
    ks = (ctypes.c_int8 * 16)(*range(11))
    f = lib.fic_encode_level_noalloc
    assert f(None, 64, 64, 64, 8, 4, ks, 11, 0, 2.5, 1, None, 64, 1, None, None, None) == fic.FIC_EINVAL
    assert "image pointer" in lib.fic_last_error().decode()
    assert f(1, 64, 64, 64, 3, 4, ks, 11, 0, 2.5, 1, None, 64, 1, None, None, None) == fic.FIC_EINVAL
    assert "range side" in lib.fic_last_error().decode()
    for side, B, L in ((2048, 2, 1), (1024, 8, 2)):
        rc = f(1, side, side, side, B, L, ks, 11, 0, 2.5, 1, None, (side // B) ** 2, 1, None, None, None)
        msg = lib.fic_last_error().decode()
        assert rc == fic.FIC_EINVAL and "scratch" in msg, msg
        need = int(re.search(r"needs (\d+) bytes", msg).group(1))
        assert need > (64 << 20)


def _params(**kw):
    p = fic.EncoderParams(**{k: v for k, v in kw.items() if k in fic.EncoderParams.__dataclass_fields__})
    c = p.to_c()
    for k, v in kw.items():
        if k not in fic.EncoderParams.__dataclass_fields__:
            setattr(c, k, v)
    return c


@pytest.mark.parametrize("kw,code,frag", [
    (dict(n_levels=0), fic.FIC_EINVAL, "n_levels"),
    (dict(n_levels=5), fic.FIC_EINVAL, "n_levels"),
    (dict(B0=12), fic.FIC_EINVAL, "B0"),
    (dict(B0=4), fic.FIC_EINVAL, "last level"),
    (dict(rms=-1.0), fic.FIC_EINVAL, "rms_thresh"),
    (dict(rms=float("inf")), fic.FIC_EINVAL, "rms_thresh"),
    (dict(entropy_mode=3), fic.FIC_EINVAL, "entropy_mode"),
    (dict(min_pool=0), fic.FIC_EINVAL, "min_pool"),
    (dict(s_sets=((1,), (2, 2), (3,), (5,))), fic.FIC_EINVAL, "increasing"),
])
def test_encode_image_rejects(lib, kw, code, frag):
    c = _params(**kw)
    n = ctypes.c_int32(0)
    rc = lib.fic_encode_image(1, 64, 64, 64, ctypes.byref(c), 1, 4096, 1, None, None)
    assert rc == code and frag in lib.fic_last_error().decode()


def test_encode_image_capacity_lower_bound(lib):
    c = _params()
    rc = lib.fic_encode_image(1, 64, 64, 64, ctypes.byref(c), 1, 15, 1, None, None)
    assert rc == fic.FIC_ECAPACITY and "capacity" in lib.fic_last_error().decode()


def test_encode_level_ex_rejects_variants(lib):
    ks = (ctypes.c_int8 * 16)(*range(11))
    def call(B, n_s, variant):
        return lib.fic_encode_level_ex(1, 64, 64, 64, B, 4, ks, n_s, 0, 2.5, 1, None,
                                       (64 // B) ** 2, 1, None, None, variant, None)
    assert call(8, 11, 5) == fic.FIC_EINVAL and "variant" in lib.fic_last_error().decode()
    assert call(8, 11, -1) == fic.FIC_EINVAL
    for v in (fic.MATCH_MFMA_I8, fic.MATCH_MFMA_F16):
        assert call(4, 11, v) == fic.FIC_EINVAL and "B = 8" in lib.fic_last_error().decode()
    assert call(8, 2, fic.MATCH_MFMA_I8) == fic.FIC_EINVAL
    # the FP16 form also takes one or two values at B = 4, 8 and 16, one of them nonzero
    assert call(2, 2, fic.MATCH_MFMA_F16) == fic.FIC_EINVAL
    assert call(16, 11, fic.MATCH_MFMA_F16) == fic.FIC_EINVAL
    assert call(8, 1, fic.MATCH_MFMA_F16) == fic.FIC_EINVAL  # {0}: nothing to screen
    assert call(16, 11, fic.MATCH_FP32) == fic.FIC_EINVAL
    # the small-set form indexes fewer than 2^21 grid domains: 1456^2 at B = 8, L = 1
    # is (1456 - 16 + 1)^2 = 2076481 < 2^21 = 2097152, 1464^2 gives 2099601
    small = (ctypes.c_int8 * 16)(3, 8)
    side = 1464
    rc = lib.fic_encode_level_ex(1, side, side, side, 8, 1, small, 2, 0, 2.5, 1, None,
                                 (side // 8) ** 2, 1, None, None, fic.MATCH_MFMA_F16, None)
    assert rc == fic.FIC_EINVAL and "2097152" in lib.fic_last_error().decode()


def test_decode_and_sse_reject(lib):
    assert lib.fic_decode(1, 4, 16, 16, 4, None, 16, None) == fic.FIC_EINVAL
    assert lib.fic_decode(1, 0, 16, 16, 4, 1, 16, None) == fic.FIC_EINVAL
    assert lib.fic_decode(1, 4, 16, 16, -1, 1, 16, None) == fic.FIC_EINVAL
    assert lib.fic_decode(1, 4, 16, 16, 4, 1, 8, None) == fic.FIC_EINVAL
    assert lib.fic_sse(None, 4, 1, 4, 4, 4, 1, None) == fic.FIC_EINVAL
    assert lib.fic_sse(1, 2, 1, 4, 4, 4, 1, None) == fic.FIC_EINVAL


def test_calibrate_rejects(lib):
    c = _params(n_levels=0)
    out = (ctypes.c_int8 * 4)()
    assert lib.fic_calibrate_s(1, 64, 64, 64, ctypes.byref(c), out, None) == fic.FIC_EINVAL
    c = _params()
    assert lib.fic_calibrate_s(1, 64, 64, 64, ctypes.byref(c), None, None) == fic.FIC_EINVAL


def test_params_marshalling():
    c = fic.EncoderParams(s_sets=fic.PAPER_K).to_c()
    assert (c.n_levels, c.B0) == (4, 16)
    assert list(c.L) == [8, 4, 2, 1]
    assert list(c.n_s) == [1, 2, 2, 2]
    assert [list(c.s_k[l])[:c.n_s[l]] for l in range(4)] == [[1], [2, 4], [3, 8], [5, 9]]


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        fic.encode_level(torch.zeros((16, 16), dtype=torch.uint8), 4, 2)
    with pytest.raises(TypeError):
        fic.encode_level(np.zeros((16, 16), np.uint8), 4, 2)


def _batch(lib, n=1, H=(64,), W=(64,), pitch=None, off=None, params=None, codes=1, ncodes=1, out=True):
    pitch = W if pitch is None else pitch
    c = params or _params()
    imgs = (ctypes.c_void_p * max(n, 1))(*([1] * max(n, 1)))
    Ha = (ctypes.c_int32 * max(n, 1))(*H)
    Wa = (ctypes.c_int32 * max(n, 1))(*W)
    Pa = (ctypes.c_int32 * max(n, 1))(*pitch)
    off = off or [0] + list(np.cumsum([(h // 2) * (w // 2) for h, w in zip(H, W)]))
    Oa = (ctypes.c_int64 * (len(off)))(*[int(v) for v in off])
    h = ctypes.c_void_p()
    rc = lib.fic_batch_create(n, imgs, Ha, Wa, Pa, ctypes.byref(c), codes, Oa, ncodes, None,
                              ctypes.byref(h) if out else None)
    return rc, lib.fic_last_error().decode()


@pytest.mark.parametrize("kw,code,frag", [
    (dict(n=0), fic.FIC_EINVAL, "batch size"),
    (dict(out=False), fic.FIC_EINVAL, "out is NULL"),
    (dict(codes=None), fic.FIC_EINVAL, "codes"),
    (dict(H=(60,)), fic.FIC_EINVAL, "image 0"),
    (dict(n=2, H=(64, 64), W=(64, 40)), fic.FIC_EINVAL, "image 1"),
    (dict(n=2, H=(64, 64), W=(64, 64), off=[0, 1024, 1030]), fic.FIC_ECAPACITY, "image 1"),
    (dict(params=_params(n_levels=0)), fic.FIC_EINVAL, "n_levels"),
])
def test_batch_create_rejects(lib, kw, code, frag):
    rc, msg = _batch(lib, **kw)
    assert rc == code and frag in msg


def test_batch_calls_reject_null(lib):
    assert lib.fic_batch_run(None, None) == fic.FIC_EINVAL
    assert lib.fic_batch_set_chunks(None, None) == fic.FIC_EINVAL
    assert lib.fic_batch_get_chunks(None, None) == fic.FIC_EINVAL
    assert lib.fic_batch_autotune(None, None, 1, None, None) == fic.FIC_EINVAL
    assert lib.fic_batch_destroy(None) == fic.FIC_OK


# ------------------------------------------------------------------ bitstream reader (host code)
@pytest.mark.parametrize("size,kw", [(64, dict(min_pool=64)), (96, dict(min_pool=32, variance=150.0)),
                                     (64, dict(entropy=False, s_sets=("plain",) * 4))])
def test_library_reader_parses_reference_streams(size, kw):
    """The library's host reader against streams written by the reference writer."""
    import oracle
    from oracle import bitstream as bs
    from paper_1501_04140_amd import synth
    img = synth.power_law(size, beta=2.0, seed=3, n_rect=2)
    s_sets = kw.pop("s_sets", oracle.PAPER_K)
    if s_sets[0] == "plain":
        s_sets = (oracle.PLAIN_K,) * 4
    codes, stats = oracle.encode_image(img, s_sets=s_sets, **kw)
    data = bs.pack(codes, stats, size, size, oracle.LEVEL_SIDES, oracle.default_steps(), s_sets)
    got, H, W = fic.unpack_stream(data)
    assert (H, W) == (size, size) and len(got) == len(codes)
    for f in ("level", "y", "x", "dom", "dy", "dx", "iso", "s_idx", "k", "q_o"):
        assert np.array_equal(got[f].astype(np.int64), codes[f].astype(np.int64)), f
    assert np.array_equal(1 << got["log2B"].astype(np.int64), codes["B"])
    assert (got["e_num"] == -1).all()


def test_library_reader_rejects_bad_streams(lib):
    import oracle
    from oracle import bitstream as bs
    from paper_1501_04140_amd import synth
    img = synth.power_law(64, beta=2.0, seed=0)
    codes, stats = oracle.encode_image(img, min_pool=16)
    data = bs.pack(codes, stats, 64, 64, oracle.LEVEL_SIDES, oracle.default_steps(), oracle.PAPER_K)
    n = ctypes.c_int32(0)
    buf = (ctypes.c_uint8 * len(data)).from_buffer_copy(data)
    assert lib.fic_unpack_stream(buf, len(data) // 2, None, 0, ctypes.byref(n), None, None) == fic.FIC_EINVAL
    bad = bytearray(data)
    bad[0] ^= 1
    buf2 = (ctypes.c_uint8 * len(bad)).from_buffer_copy(bytes(bad))
    assert lib.fic_unpack_stream(buf2, len(bad), None, 0, ctypes.byref(n), None, None) == fic.FIC_EINVAL
    assert lib.fic_unpack_stream(buf, len(data), None, 0, ctypes.byref(n), None, None) == fic.FIC_ECAPACITY
    assert n.value == len(codes)


def test_select_s_matches_reference_rule():
    import oracle
    rng = np.random.default_rng(0)
    for trial in range(50):
        h = rng.integers(0, 5, size=(4, 11)) * rng.integers(0, 2, size=(4, 11))
        for frac in (0.0, 0.3, 0.5, 1.0):
            assert fic.select_s(h, 4, frac) == oracle.select_s(h, frac), (trial, frac)
