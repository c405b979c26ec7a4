"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by
element. Every integer field must match exactly; e_num (1600 n E) times n must
equal the oracle's exact (40 n)^2 E."""
import numpy as np
import pytest

import oracle
from paper_1501_04140_amd import fic, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fic.load()
    return torch.device("cuda:0")


def gpu_level(dev, img, B, L, ks, entropy=0, bits=2.5, min_pool=256, ranges=None,
              variant=fic.MATCH_AUTO):
    x = torch.from_numpy(np.ascontiguousarray(img)).to(dev)
    r = None if ranges is None else torch.from_numpy(np.asarray(ranges, np.int32)).to(dev)
    out, pool, pc = fic.encode_level(x, B, L, ks, entropy, bits, min_pool, ranges=r, return_pool=True,
                                     variant=variant)
    torch.cuda.synchronize()
    return fic.matches_numpy(out), pool.cpu().numpy()[:int(pc.item())]


def assert_level_equal(got, ref, B):
    n = B * B
    assert len(got) == len(ref)
    assert np.array_equal(got["dom"], ref["dom"])
    assert np.array_equal(got["iso"].astype(np.int32), ref["iso"])
    assert np.array_equal(got["s_idx"].astype(np.int32), ref["s_idx"])
    assert np.array_equal(got["k"].astype(np.int32), ref["k"])
    assert np.array_equal(got["q_o"].astype(np.int32), ref["q_o"])
    assert np.array_equal(got["e_num"] * n, ref["e_lit"])
    E_ref = ref["e_lit"] / (40.0 * n) ** 2
    assert np.allclose(got["E"], E_ref, rtol=1e-6, atol=1e-6)


def check_level(dev, img, B, L, ks, entropy=0, min_pool=256, ranges=None, bits=2.5,
                variant=fic.MATCH_AUTO):
    say(f"[level] shape={img.shape} B={B} L={L} ks={ks} entropy={entropy} min_pool={min_pool} "
        f"variant={variant}")
    got, gpool = gpu_level(dev, img, B, L, ks, entropy, bits, min_pool, ranges, variant)
    if entropy == 2:
        pool, _ = oracle.variance_pool(img, B, L, bits, min_pool)
        assert np.array_equal(gpool, pool)
    elif entropy:
        pool, _ = oracle.entropy_pool(img, B, L, bits, min_pool)
        assert np.array_equal(gpool, pool)
    else:
        gy, gx = oracle.domain_grid(*img.shape, B, L)
        pool = None
        assert len(gpool) == gy * gx
    ref = oracle.match_level(img, B, L, ks, pool, ranges)
    assert_level_equal(got, ref, B)
    return got


# ------------------------------------------------------------------ single level
def test_single_level_workload_full(dev):
    """128x128 gradients + blobs + noise, 8x8 ranges, step 4 (841 domains), s = 0..1."""
    img = synth.single_level_image(0)
    check_level(dev, img, 8, 4, oracle.PLAIN_K)


@pytest.mark.parametrize("B,L,ks", [
    (2, 1, oracle.PLAIN_K), (2, 3, (5, 9)), (4, 2, oracle.PLAIN_K), (4, 5, (2, 4)),
    (8, 3, (3, 8)), (8, 8, (0,)), (16, 8, (1,)), (16, 5, oracle.PLAIN_K),
    (4, 1, (10,)), (8, 2, (1, 5, 9)), (2, 2, (3, 4, 5, 6)),
])
def test_level_shapes_and_sets(dev, B, L, ks):
    img = synth.power_law(64, 96, beta=2.0, seed=B * 100 + L, n_rect=2)
    check_level(dev, img, B, L, ks)


@pytest.mark.parametrize("kind", ["constant", "replicated", "noise", "two_tone"])
def test_level_adversarial(dev, kind):
    rng = np.random.default_rng(5)
    if kind == "constant":
        img = np.full((48, 48), 131, np.uint8)
    elif kind == "replicated":
        img = np.kron(rng.integers(0, 256, size=(24, 24)), np.ones((2, 2))).astype(np.uint8)
    elif kind == "noise":
        img = rng.integers(0, 256, size=(48, 48)).astype(np.uint8)
    else:
        img = (rng.integers(0, 2, size=(48, 48)) * 255).astype(np.uint8)
    for B, L in ((2, 1), (4, 2), (8, 4)):
        check_level(dev, img, B, L, oracle.PLAIN_K)
        check_level(dev, img, B, L, (2, 4))


def test_isometric_copies(dev):
    rng = np.random.default_rng(0)
    for t in range(8):
        img = rng.integers(0, 256, size=(48, 48)).astype(np.int64)
        m = rng.integers(0, 26, size=(4, 4))
        img[24:32, 24:32] = np.kron(10 * m, np.ones((2, 2), dtype=np.int64))
        rot = [m, np.rot90(m, -1), np.rot90(m, 2), np.rot90(m, 1)][t % 4]
        rot = np.fliplr(rot) if t >= 4 else rot
        img[4:8, 8:12] = 10 * rot + 3
        img = img.astype(np.uint8)
        got = check_level(dev, img, 4, 4, oracle.PLAIN_K, ranges=np.array([[4, 8], [0, 0]]))
        assert got["e_num"][0] == 0 and got["iso"][0] == t and got["k"][0] == 10


def test_range_subset_and_invalid_corner(dev):
    img = synth.power_law(64, beta=1.8, seed=2)
    ranges = np.array([[8, 16], [0, 0], [56, 56], [3, 4], [64, 0], [24, 8]], np.int32)
    say("[level] invalid corners")
    got, _ = gpu_level(dev, img, 8, 4, oracle.PLAIN_K, ranges=ranges)
    assert got["dom"][3] == -1 and got["dom"][4] == -1
    ok = [0, 1, 2, 5]
    ref = oracle.match_level(img, 8, 4, oracle.PLAIN_K, None, ranges[ok])
    assert_level_equal(got[ok], ref, 8)


# ------------------------------------------------------------------ entropy filter (Section 3)
@pytest.mark.parametrize("B,L,min_pool", [(2, 1, 256), (4, 2, 256), (8, 4, 64), (16, 8, 32),
                                          (4, 2, 5000), (2, 1, 10 ** 6)])
def test_entropy_pool_floor_and_pass(dev, B, L, min_pool):
    img = synth.power_law(96, beta=2.0, seed=1, n_rect=3)
    check_level(dev, img, B, L, (2, 4), entropy=1, min_pool=min_pool)


def test_entropy_pool_many_pass(dev):
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(64, 64)).astype(np.uint8)   # near-uniform bins: high entropy
    img[:32, :32] = 100
    for B, L in ((2, 1), (4, 2), (8, 4)):
        check_level(dev, img, B, L, (3, 8), entropy=1, min_pool=16)


def test_entropy_threshold_variants(dev):
    img = synth.power_law(64, beta=1.5, seed=4)
    for bits in (0.0, 1.0, 1.75, 2.0):
        check_level(dev, img, 4, 2, (1,), entropy=1, min_pool=8, bits=bits)


@pytest.mark.parametrize("B,L,H,W", [(2, 1, 200, 300), (4, 2, 392, 520), (8, 4, 760, 776),
                                     (16, 8, 1488, 1520)])
def test_entropy_pool_large_grids(dev, B, L, H, W):
    """Grids of 32768 domains or more, whose entropy keys come from cell histograms;
    both grid sides leave a partial tile. Threshold mode (most domains pass at 1 bit)
    and floor mode (the 5000 lowest keys, nothing passing at 2.5 bits)."""
    img = synth.power_law(max(H, W), beta=2.0, seed=7, n_rect=3)[:H, :W].copy()
    gy, gx = oracle.domain_grid(H, W, B, L)
    assert gy * gx >= 32768 and gx % 64 and gy % 4
    x = torch.from_numpy(img).to(dev)
    corner = torch.tensor([[0, 0]], dtype=torch.int32, device=dev)
    for bits, min_pool in ((1.0, 16), (2.5, 5000)):
        say(f"[entropy] {H}x{W} B={B} L={L} bits={bits} min_pool={min_pool}")
        _, pool, pc = fic.encode_level(x, B, L, (2, 4), 1, bits, min_pool, ranges=corner,
                                       return_pool=True)
        torch.cuda.synchronize()
        ref, _ = oracle.entropy_pool(img, B, L, bits, min_pool)
        assert np.array_equal(pool.cpu().numpy()[:int(pc.item())], ref)


@pytest.mark.parametrize("L,H,W", [(2, 188, 188), (2, 204, 308), (4, 516, 516)])
def test_direct_select_mid_grids(dev, L, H, W):
    """Grids of 8193..16384 domains (B = 4: 8281 and 14949 at L = 2, exactly 16384 at L = 4), which
    the pool select takes in one launch with only the keys staged: threshold mode, floor
    mode (nothing passes at 9 bits), a floor that the passers may or may not reach, the
    whole grid, and the variance filter's threshold and floor; a three-valued image puts many equal keys at the
    cut, whose first ones in index order must be kept."""
    B = 4
    gy, gx = oracle.domain_grid(H, W, B, L)
    assert 8192 < gy * gx <= 16384
    img = synth.power_law(max(H, W), beta=1.8, seed=11, n_rect=3)[:H, :W].copy()
    rng = np.random.default_rng(3)
    ties = (rng.integers(0, 3, size=(H, W)) * 100).astype(np.uint8)
    corner = torch.tensor([[0, 0]], dtype=torch.int32, device=dev)
    for name, im in (("power_law", img), ("three_valued", ties)):
        x = torch.from_numpy(np.ascontiguousarray(im)).to(dev)
        for entropy, bits, min_pool in ((1, 1.0, 16), (1, 2.5, 700), (1, 9.0, 5000),
                                        (1, 2.5, 10 ** 6), (2, 300.0, 4096), (2, 1e9, 4096)):
            say(f"[direct select] {name} {H}x{W} entropy={entropy} bits={bits} min_pool={min_pool}")
            _, pool, pc = fic.encode_level(x, B, L, (2, 4), entropy, bits, min_pool, ranges=corner,
                                           return_pool=True)
            torch.cuda.synchronize()
            if entropy == 2:
                ref, _ = oracle.variance_pool(im, B, L, bits, min_pool)
            else:
                ref, _ = oracle.entropy_pool(im, B, L, bits, min_pool)
            assert np.array_equal(pool.cpu().numpy()[:int(pc.item())], ref)


@pytest.mark.parametrize("B,L,vmin,min_pool", [(2, 1, 50.0, 256), (4, 2, 300.0, 64), (8, 4, 900.0, 16),
                                               (16, 8, 1e9, 32), (4, 2, -1.0, 8), (2, 1, 0.0, 10 ** 6)])
def test_variance_pool_levels(dev, B, L, vmin, min_pool):
    """Variance filter (threshold and floor) against the oracle, then the matcher on that pool."""
    img = synth.power_law(96, beta=1.8, seed=6, n_rect=2)
    check_level(dev, img, B, L, (2, 4), entropy=2, min_pool=min_pool, bits=vmin)


def test_variance_pool_ties(dev):
    rng = np.random.default_rng(1)
    img = (rng.integers(0, 4, size=(64, 64)) * 60).astype(np.uint8)  # few distinct variances
    for B, L in ((2, 1), (4, 2)):
        check_level(dev, img, B, L, (1,), entropy=2, min_pool=100, bits=1e9)


# ------------------------------------------------------------------ quadtree
def gpu_image(dev, img, params):
    x = torch.from_numpy(np.ascontiguousarray(img)).to(dev)
    codes, n, stats = fic.encode_image(x, params)
    torch.cuda.synchronize()
    return codes, n, fic.codes_numpy(codes, n), fic.stats_numpy(stats)


def assert_codes_equal(got, ref):
    assert len(got) == len(ref)
    for f in ("level", "y", "x", "dom", "dy", "dx", "iso", "s_idx", "k", "q_o"):
        assert np.array_equal(got[f].astype(np.int64), ref[f].astype(np.int64)), f
    assert np.array_equal(1 << got["log2B"].astype(np.int64), ref["B"])
    n = (1 << got["log2B"].astype(np.int64)) ** 2
    assert np.array_equal(got["e_num"] * n, ref["e_lit"])


@pytest.mark.parametrize("size,seed,min_pool,sets", [
    (64, 0, 64, "paper"), (96, 1, 128, "paper"), (128, 2, 256, "paper"), (64, 3, 16, "plain"),
])
def test_quadtree_matches_oracle(dev, size, seed, min_pool, sets):
    img = synth.power_law(size, beta=2.0, seed=seed, n_rect=3)
    ks = oracle.PAPER_K if sets == "paper" else (oracle.PLAIN_K,) * 4
    say(f"[quadtree] size={size} seed={seed} min_pool={min_pool} sets={sets}")
    codes, n, got, st = gpu_image(dev, img, fic.EncoderParams(s_sets=ks, min_pool=min_pool))
    ref, rst = oracle.encode_image(img, s_sets=ks, min_pool=min_pool)
    assert_codes_equal(got, ref)
    for l, s in enumerate(rst):
        assert (st["pool"][l], st["active"][l], st["accepted"][l], st["matches"][l]) == (
            s["pool"], s["active"], s["accepted"], s["matches"])
        assert st["passed"][l] == s["passed"]
    rec = fic.decode(codes, int(n.item()), size, size, iters=24)
    assert np.array_equal(rec.cpu().numpy(), oracle.decode(ref, size, size, iters=24))


@pytest.mark.parametrize("steps", [(8, 8, 2, 1), (4, 4, 2, 2)])
def test_quadtree_other_steps(dev, steps):
    """Steps other than L = B/2: those levels are scored window by window,
    not from cells, so the one-image encode sets up level 0 another way (its
    keys by cells without the other levels, or level 0 not by cells)."""
    img = synth.power_law(96, beta=3.0, seed=5, n_rect=4)  # smooth: levels 1-3 keep ranges
    say(f"[quadtree] steps {steps}")
    params = fic.EncoderParams(s_sets=oracle.PAPER_K, min_pool=64, steps=steps)
    _, _, got, st = gpu_image(dev, img, params)
    ref, rst = oracle.encode_image(img, s_sets=oracle.PAPER_K, min_pool=64, steps=steps)
    assert_codes_equal(got, ref)
    for l, s in enumerate(rst):
        assert (st["pool"][l], st["passed"][l], st["accepted"][l]) == (s["pool"], s["passed"], s["accepted"])


def test_quadtree_alternating_arguments(dev):
    """The encoder keeps a device copy of each image's level arguments and
    rewrites it only when they change: alternating images, sizes and
    parameters on one stream must each give the oracle's codes, also when an
    earlier argument set comes back (same buffers, same image)."""
    a = synth.power_law(96, beta=2.0, seed=7, n_rect=2)
    b = synth.power_law(128, beta=1.6, seed=8, n_rect=1)
    pa = fic.EncoderParams(s_sets=oracle.PAPER_K, min_pool=64)
    pb = fic.EncoderParams(s_sets=((3,), (2, 4), (9,), (5, 9)), min_pool=100)
    xa = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    xb = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    ref = {}
    for key, img, p in (("a", a, pa), ("b", b, pb), ("ab", a, pb)):
        ref[key], _ = oracle.encode_image(img, s_sets=p.s_sets, min_pool=p.min_pool)
    out_a = fic.encode_image(xa, pa)
    for key, x, p in (("a", xa, pa), ("b", xb, pb), ("a", xa, pa), ("ab", xa, pb), ("a", xa, pa)):
        say(f"[quadtree] alternating arguments: {key}")
        codes, n, _ = fic.encode_image(x, p, out=out_a if key == "a" else None)
        torch.cuda.synchronize()
        assert_codes_equal(fic.codes_numpy(codes, n), ref[key])


def test_quadtree_variance_pool(dev):
    img = synth.power_law(96, beta=2.0, seed=2, n_rect=3)
    params = fic.EncoderParams(s_sets=oracle.PAPER_K, entropy_mode=2, entropy_bits=200.0, min_pool=48)
    say("[quadtree] variance pool 96")
    codes, n, got, st = gpu_image(dev, img, params)
    ref, rst = oracle.encode_image(img, s_sets=oracle.PAPER_K, min_pool=48, variance=200.0)
    assert_codes_equal(got, ref)
    for l, s in enumerate(rst):
        assert (st["pool"][l], st["passed"][l], st["accepted"][l]) == (s["pool"], s["passed"], s["accepted"])


def test_quadtree_unfiltered_plain(dev):
    img = synth.gradients_blobs(64, seed=7)
    params = fic.EncoderParams(s_sets=(oracle.PLAIN_K,) * 4, entropy_mode=0)
    say("[quadtree] unfiltered plain 64")
    _, _, got, _ = gpu_image(dev, img, params)
    ref, _ = oracle.encode_image(img, s_sets=(oracle.PLAIN_K,) * 4, entropy=False)
    assert_codes_equal(got, ref)


def test_quadtree_capacity_overflow_reports_required(dev):
    img = synth.power_law(64, beta=2.0, seed=0, n_rect=3)
    x = torch.from_numpy(img).to(dev)
    params = fic.EncoderParams(min_pool=64)
    say("[quadtree] capacity overflow")
    full, nfull, _ = fic.encode_image(x, params)
    small, nsmall, _ = fic.encode_image(x, params, capacity=16)
    torch.cuda.synchronize()
    need = int(nfull.item())
    assert int(nsmall.item()) == need and need > 16
    assert np.array_equal(small.cpu().numpy()[:16], full.cpu().numpy()[:16])


def test_quadtree_full_size_paper_preset(dev):
    """512x512 1/f^2 + rectangles with the predefined s of Section 3.1, whole image."""
    img = synth.quadtree_image(0)
    say("[quadtree] 512 paper preset")
    codes, n, got, st = gpu_image(dev, img, fic.EncoderParams(s_sets=oracle.PAPER_K))
    ref, _ = oracle.encode_image(img, s_sets=oracle.PAPER_K)
    assert_codes_equal(got, ref)
    rec = fic.decode(codes, int(n.item()), 512, 512, iters=8)
    assert np.array_equal(rec.cpu().numpy(), oracle.decode(ref, 512, 512, iters=8))


def test_quadtree_full_size_calibrated(dev):
    """The default workload: 512x512 1/f^2 + rectangles with one contrast value per level,
    {1}, {3}, {9}, {9}. With one value the B = 2 level takes the single-value branch of the
    VALU matcher (the largest kernel of that encode), which the printed preset (two values)
    does not reach at full size."""
    img = synth.quadtree_image(0)
    ks = ((1,), (3,), (9,), (9,))
    say("[quadtree] 512 calibrated sets")
    codes, n, got, st = gpu_image(dev, img, fic.EncoderParams(s_sets=ks))
    ref, rst = oracle.encode_image(img, s_sets=ks)
    assert_codes_equal(got, ref)
    for l, s in enumerate(rst):
        assert (st["pool"][l], st["active"][l], st["accepted"][l]) == (s["pool"], s["active"], s["accepted"])
    rec = fic.decode(codes, int(n.item()), 512, 512, iters=8)
    assert np.array_equal(rec.cpu().numpy(), oracle.decode(ref, 512, 512, iters=8))


def _big_b2_image(N=2944):
    """Uniform noise with three 2 x 2 ranges planted as exact scaled copies of domains near
    the end of the B = 2, L = 1 grid ((N - 3)^2 = 8,649,481 domains at N = 2944, above 2^23),
    so the winners sit at pool positions 6.5M-8.6M."""
    rng = np.random.default_rng(23)
    img = rng.integers(0, 256, size=(N, N)).astype(np.int64)
    yx = []
    for (ry, rx), (dy, dx), k, o, t in [((0, 0), (N - 4, N - 4), 5, 30, 3),
                                        ((100, 2000), (2500, 1777), 9, 7, 6),
                                        ((2940, 10), (2200, 2939), 10, 0, 0)]:
        m = rng.integers(0, 26, size=(2, 2))
        img[dy:dy + 4, dx:dx + 4] = np.kron(10 * m, np.ones((2, 2), np.int64))
        rot = [m, np.rot90(m, -1), np.rot90(m, 2), np.rot90(m, 1)][t % 4]
        img[ry:ry + 2, rx:rx + 2] = k * (np.fliplr(rot) if t >= 4 else rot) + o
        yx.append((ry, rx))
    return img.astype(np.uint8), np.array(yx + [(500, 500), (N - 2, N - 2)], np.int32)


@pytest.mark.parametrize("ks", [(5,), (5, 9), (10,)])
def test_b2_pool_beyond_2_23(dev, ks):
    """The B = 2 small-set matcher over an unfiltered grid of 8.6M domains: its exact 24-bit
    multiply-add must not depend on the pool position."""
    img, yx = _big_b2_image()
    say(f"[level] B=2 L=1 grid above 2^23, ks={ks}")
    got = check_level(dev, img, 2, 1, ks, ranges=yx)
    # a winner beyond 2^23 - 4 * 1020 * 765 (about 5.26M), where a dot product seeded with
    # the pool position would leave the 24-bit multiplier's range
    assert got["dom"].max() > (1 << 23) - 4 * 1020 * 765


def test_calibration_matches_oracle(dev):
    img = synth.power_law(64, beta=2.0, seed=0, n_rect=3)
    say("[calibrate] 64")
    x = torch.from_numpy(img).to(dev)
    ks = fic.calibrate_s(x, fic.EncoderParams())
    ref = oracle.calibrate_s(img, fallback=((-1,),) * 4)
    assert ks == [r[0] for r in ref]


def test_sse_psnr(dev):
    rng = np.random.default_rng(0)
    a = rng.integers(0, 256, size=(37, 53)).astype(np.uint8)
    b = rng.integers(0, 256, size=(37, 53)).astype(np.uint8)
    ta, tb = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
    assert int(fic.sse(ta, tb).item()) == int(((a.astype(np.int64) - b) ** 2).sum())
    assert fic.psnr(ta, tb) == pytest.approx(oracle.psnr(a, b), rel=1e-12)


def test_decode_rejects_bad_codes(dev):
    img = synth.power_law(32, beta=2.0, seed=0)
    x = torch.from_numpy(img).to(dev)
    codes, n, _ = fic.encode_image(x, fic.EncoderParams(min_pool=8))
    torch.cuda.synchronize()
    k = int(n.item())
    with pytest.raises(fic.FicError):
        fic.decode(codes, k - 1, 32, 32, iters=2)          # a hole
    bad = codes.clone()
    bad[0, 16:18] = torch.tensor([30, 0], dtype=torch.uint8)  # dy = 30: domain leaves the image
    with pytest.raises(fic.FicError):
        fic.decode(bad, k, 32, 32, iters=2)


# ------------------------------------------------------------------ large sizes, sampled
def test_precision_workload_sampled(dev):
    """1024x1024 1/f^1.8, 8x8 ranges, step 2 (505^2 domains), s = 0..1: the whole
    image on the GPU, a deterministic sample of ranges through the oracle."""
    img = synth.precision_image(0)
    say("[level] 1024 precision workload")
    got, _ = gpu_level(dev, img, 8, 2, oracle.PLAIN_K)
    idx = np.arange(0, 16384, 1031)[:12]
    ranges = oracle.full_ranges(1024, 1024, 8)[idx]
    ref = oracle.match_level(img, 8, 2, oracle.PLAIN_K, None, ranges)
    assert_level_equal(got[idx], ref, 8)


# ------------------------------------------------------------------ precision form (B = 8)
MFMA_FORMS = [fic.MATCH_MFMA_I8, fic.MATCH_MFMA_F16]


@pytest.mark.parametrize("variant", [fic.MATCH_VALU] + MFMA_FORMS)
def test_single_level_workload_variants(dev, variant):
    img = synth.single_level_image(0)
    check_level(dev, img, 8, 4, oracle.PLAIN_K, variant=variant)


@pytest.mark.parametrize("variant", MFMA_FORMS)
@pytest.mark.parametrize("kind", ["constant", "half_flat", "replicated", "noise", "two_tone", "blobs",
                                  "copy"])
@pytest.mark.parametrize("ks", [oracle.PLAIN_K, (0, 1, 2), (0, 1, 2, 3, 4, 5)])
def test_mfma_exact_on_adversarial(dev, kind, ks, variant):
    rng = np.random.default_rng(11)
    if kind == "constant":
        img = np.full((72, 88), 201, np.uint8)
    elif kind == "half_flat":
        # constant ranges and constant domains beside textured ones (F = 0 ties)
        img = rng.integers(0, 256, size=(72, 88)).astype(np.uint8)
        img[:, :44] = 77
        img[:16, 60:] = 3
    elif kind == "replicated":
        img = np.kron(rng.integers(0, 256, size=(36, 44)), np.ones((2, 2))).astype(np.uint8)
    elif kind == "noise":
        img = rng.integers(0, 256, size=(72, 88)).astype(np.uint8)
    elif kind == "two_tone":
        img = (rng.integers(0, 2, size=(72, 88)) * 255).astype(np.uint8)
    elif kind == "blobs":
        img = synth.gradients_blobs(88, seed=3)[:72]
    else:
        img = rng.integers(0, 256, size=(72, 88)).astype(np.int64)
        m = rng.integers(0, 26, size=(8, 8))
        img[40:56, 56:72] = np.kron(10 * m, np.ones((2, 2), dtype=np.int64))
        img[0:8, 8:16] = 10 * np.fliplr(np.rot90(m, -1)) + 5
        img = img.astype(np.uint8)
    for L in (1, 3):
        check_level(dev, img, 8, L, ks, variant=variant)


@pytest.mark.parametrize("variant", MFMA_FORMS)
def test_mfma_ragged_ranges_and_pool(dev, variant):
    img = synth.power_law(120, 136, beta=1.8, seed=9)
    rng = np.random.default_rng(2)
    corners = oracle.full_ranges(120, 136, 8)
    sub = corners[np.sort(rng.choice(len(corners), 37, replace=False))]
    check_level(dev, img, 8, 5, oracle.PLAIN_K, ranges=sub, variant=variant)
    check_level(dev, img, 8, 2, oracle.PLAIN_K, entropy=1, min_pool=300, variant=variant)


# ------------------------------------------------------------------ FP16 MFMA, small sets (B = 4, 8, 16)
SMALL_SETS = [(1,), (3,), (2, 4), (5, 9), (0, 7), (9,)]


@pytest.mark.parametrize("B", [4, 8, 16])
@pytest.mark.parametrize("kind", ["constant", "half_flat", "noise", "two_tone", "blobs"])
def test_mfq_small_sets_adversarial(dev, B, kind):
    """The small-set FP16 MFMA matcher against the oracle: constant ranges and
    domains (F = 0 ties, B' = 0), saturated noise, and every preset shape of set
    (one value, two values, a set holding 0)."""
    rng = np.random.default_rng(5)
    if kind == "constant":
        img = np.full((80, 96), 201, np.uint8)
    elif kind == "half_flat":
        img = rng.integers(0, 256, size=(80, 96)).astype(np.uint8)
        img[:, :48] = 77
        img[:32, 64:] = 3
    elif kind == "noise":
        img = rng.integers(0, 256, size=(80, 96)).astype(np.uint8)
    elif kind == "two_tone":
        img = (rng.integers(0, 2, size=(80, 96)) * 255).astype(np.uint8)
    else:
        img = synth.gradients_blobs(96, seed=4)[:80]
    for ks in SMALL_SETS:
        check_level(dev, img, B, 3, ks, variant=fic.MATCH_MFMA_F16)


@pytest.mark.parametrize("B", [4, 8, 16])
def test_mfq_ragged_ranges_and_pool(dev, B):
    img = synth.power_law(144, 160, beta=1.8, seed=9)
    rng = np.random.default_rng(3)
    corners = oracle.full_ranges(144, 160, B)
    sub = corners[np.sort(rng.choice(len(corners), min(37, len(corners) - 3), replace=False))]
    check_level(dev, img, B, 5, (2, 4), ranges=sub, variant=fic.MATCH_MFMA_F16)
    check_level(dev, img, B, 2, (3,), entropy=1, min_pool=200, variant=fic.MATCH_MFMA_F16)
    check_level(dev, img, B, 1, (0, 9), entropy=1, min_pool=3000, variant=fic.MATCH_MFMA_F16)


@pytest.mark.parametrize("B,L,ks", [(16, 8, (1,)), (16, 4, (5, 9)), (8, 4, (3,)), (8, 2, (2, 4)),
                                    (8, 4, (0, 5)), (4, 2, (9,)), (4, 2, (3, 8)), (4, 1, (0, 4))])
def test_mfq_equals_valu_at_512(dev, B, L, ks):
    """The quadtree image at full size: the FP16 small-set matcher equals the dot4
    VALU matcher on every range, with the whole grid and with the entropy pool."""
    img = synth.quadtree_image(0)
    for entropy in (0, 1):
        say(f"[level] 512 B={B} L={L} ks={ks} entropy={entropy}: FP16 MFMA vs VALU")
        got, _ = gpu_level(dev, img, B, L, ks, entropy=entropy, variant=fic.MATCH_MFMA_F16)
        valu, _ = gpu_level(dev, img, B, L, ks, entropy=entropy, variant=fic.MATCH_VALU)
        for f in ("e_num", "dom", "iso", "s_idx", "k", "q_o"):
            assert np.array_equal(got[f], valu[f]), f


def test_mfma_in_quadtree_unfiltered(dev):
    img = synth.power_law(96, beta=2.0, seed=5, n_rect=2)
    say("[quadtree] plain grid, MFMA level")
    _, _, got, _ = gpu_image(dev, img, fic.EncoderParams(s_sets=(oracle.PLAIN_K,) * 4,
                                                         entropy_mode=0))
    ref, _ = oracle.encode_image(img, s_sets=(oracle.PLAIN_K,) * 4, entropy=False)
    assert_codes_equal(got, ref)


@pytest.mark.parametrize("variant", MFMA_FORMS)
def test_precision_workload_mfma_sampled(dev, variant):
    """1024x1024 1/f^1.8, 8x8 ranges, step 2: int8 or FP16 MFMA over the whole
    image, equal to the VALU matcher everywhere, a deterministic sample of ranges
    through the oracle."""
    img = synth.precision_image(0)
    say(f"[level] 1024 precision workload, MFMA variant {variant}")
    got, _ = gpu_level(dev, img, 8, 2, oracle.PLAIN_K, variant=variant)
    valu, _ = gpu_level(dev, img, 8, 2, oracle.PLAIN_K, variant=fic.MATCH_VALU)
    for f in ("e_num", "dom", "iso", "k", "q_o"):
        assert np.array_equal(got[f], valu[f]), f
    idx = np.arange(0, 16384, 1301)[:12]
    ranges = oracle.full_ranges(1024, 1024, 8)[idx]
    ref = oracle.match_level(img, 8, 2, oracle.PLAIN_K, None, ranges)
    assert_level_equal(got[idx], ref, 8)


def test_fp32_comparator_error_is_reported(dev):
    """The FP32 comparator: its e_num is the exact value of the candidate it picked,
    never below the exact optimum; its FP32 E is close to that exact value."""
    img = synth.single_level_image(0)
    say("[level] FP32 comparator")
    f32, _ = gpu_level(dev, img, 8, 4, oracle.PLAIN_K, variant=fic.MATCH_FP32)
    ref = oracle.match_level(img, 8, 4, oracle.PLAIN_K)
    n = 64
    exact_pick = f32["e_num"] * n
    assert np.all(exact_pick >= ref["e_lit"])
    E_exact = ref["e_lit"] / (40.0 * n) ** 2
    E_pick = f32["e_num"] / (1600.0 * n)
    same = (f32["dom"] == ref["dom"]) & (f32["iso"] == ref["iso"]) & (f32["k"] == ref["k"])
    rel = np.abs(f32["E"] - E_pick) / np.maximum(E_pick, 1.0)
    say(f"[fp32] argmin agrees on {same.mean():.4f} of ranges; max rel E error "
        f"{rel.max():.3e}; max E excess {np.max(E_pick - E_exact):.3e}")
    assert same.mean() > 0.9
    assert np.all(E_pick - E_exact <= 1e-3 * np.maximum(E_exact, 1.0) + 1.0)


# ------------------------------------------------------------------ contrast histograms (Fig. 3)
@pytest.mark.parametrize("low_only", [False, True])
def test_s_histogram_matches_oracle(dev, low_only):
    imgs = [synth.power_law(64, beta=2.0, seed=s, n_rect=2) for s in (0, 1)] + [synth.gradients_blobs(96, 2)]
    hist = None
    ref = np.zeros((4, 11), dtype=np.int64)
    for im in imgs:
        hist = fic.s_histogram(torch.from_numpy(im).to(dev), fic.EncoderParams(), low_only, hist)
        ref += oracle.s_histogram(im, low_only=low_only)
    torch.cuda.synchronize()
    say(f"[s-hist] low_only={low_only}: {hist.cpu().numpy().tolist()}")
    assert np.array_equal(hist.cpu().numpy(), ref)
    assert fic.select_s(hist.cpu().numpy()) == oracle.select_s(ref)
