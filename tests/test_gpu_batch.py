"""Batched quadtree encoder (one captured hipGraph for many images) against the
oracle on small mixed sizes, and against the single-image path, with sampled
oracle checks, on images of the 64-image batch workload."""
import numpy as np
import pytest

import oracle
from paper_1501_04140_amd import fic, synth

from test_gpu_parity import assert_codes_equal, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fic.load()
    return torch.device("cuda:0")


MIXED = [((64, 64), 2.0, 0), ((96, 128), 1.6, 1), ((128, 64), 2.4, 2), ((48, 80), 2.0, 3),
         ((32, 32), 1.8, 4)]


def mixed_images():
    return [synth.power_law(h, w, beta=b, seed=s, n_rect=2) for (h, w), b, s in MIXED]


@pytest.mark.parametrize("min_pool,sets", [(64, "paper"), (16, "plain")])
def test_batch_mixed_sizes_match_oracle_over_replays(dev, min_pool, sets):
    imgs = mixed_images()
    ks = oracle.PAPER_K if sets == "paper" else (oracle.PLAIN_K,) * 4
    params = fic.EncoderParams(s_sets=ks, min_pool=min_pool)
    refs = [oracle.encode_image(im, s_sets=ks, min_pool=min_pool) for im in imgs]
    xs = [torch.from_numpy(im).to(dev) for im in imgs]
    say(f"[batch] mixed sizes min_pool={min_pool} sets={sets}")
    b = fic.Batch(xs, params)
    try:
        for rep in range(3):
            b.codes.fill_(0xAB)  # eager work between replays; stale codes must not survive
            b.run()
            torch.cuda.synchronize()
            say(f"[batch] replay {rep}")
            for i, (ref, rst) in enumerate(refs):
                got = fic.codes_numpy(b.image_codes(i), int(b.n_codes[i].item()))
                assert_codes_equal(got, ref)
                st = fic.stats_numpy(b.stats[i])
                for l, s in enumerate(rst):
                    assert (st["pool"][l], st["active"][l], st["accepted"][l], st["matches"][l],
                            st["passed"][l]) == (s["pool"], s["active"], s["accepted"],
                                                 s["matches"], s["passed"])
            # a single-image encode on the torch stream in between
            fic.encode_image(xs[0], params)
            torch.cuda.synchronize()
    finally:
        b.close()


def test_batch_chunk_choices_do_not_change_codes(dev):
    imgs = mixed_images()[:3]
    params = fic.EncoderParams(min_pool=32)
    xs = [torch.from_numpy(im).to(dev) for im in imgs]
    b = fic.Batch(xs, params)
    try:
        b.run()
        torch.cuda.synchronize()
        base = [b.image_codes(i).cpu().numpy().copy() for i in range(len(xs))]
        for chunks in ([32, 64, 128, 256], [4096, 4096, 4096, 4096], [0, 0, 0, 0]):
            say(f"[batch] chunks {chunks}")
            b.set_chunks(chunks)
            if all(chunks):
                assert b.chunks() == chunks
            else:  # 0 = library default, reported as the value in use
                assert all(c > 0 for c in b.chunks())
            b.run()
            torch.cuda.synchronize()
            for i in range(len(xs)):
                assert np.array_equal(b.image_codes(i).cpu().numpy(), base[i])
    finally:
        b.close()


def test_batch_autotune_cache_roundtrip(dev, tmp_path):
    imgs = mixed_images()[:2]
    xs = [torch.from_numpy(im).to(dev) for im in imgs]
    params = fic.EncoderParams(min_pool=32)
    cache = str(tmp_path / "tune.jsonl")
    b = fic.Batch(xs, params)
    try:
        say("[batch] autotune")
        ms = b.autotune(reps=1, cache_path=cache)
        chosen = b.chunks()
        assert ms > 0 and all(c > 0 for c in chosen)
        b.run()
        torch.cuda.synchronize()
        ref = [oracle.encode_image(im, min_pool=32)[0] for im in imgs]
        for i in range(2):
            assert_codes_equal(fic.codes_numpy(b.image_codes(i), int(b.n_codes[i].item())), ref[i])
    finally:
        b.close()
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and '"chunks": [' in lines[0]
    b2 = fic.Batch(xs, params)
    try:
        b2.autotune(reps=1, cache_path=cache)  # applies the cached entry
        assert b2.chunks() == chosen
    finally:
        b2.close()
    assert len(open(cache).read().splitlines()) == 1


def test_batch_workload_images_match_single_path_and_sampled_oracle(dev):
    """Eight images of the 64-image batch (sides 256..2048): batch == single-image
    path bit for bit; sampled level-0 codes against the oracle's matcher."""
    imgs = synth.batch_images(8)
    xs = [torch.from_numpy(im).to(dev) for im in imgs]
    params = fic.EncoderParams(s_sets=fic.PAPER_K)
    say("[batch] workload sides", [im.shape[0] for im in imgs])
    b = fic.Batch(xs, params)
    try:
        b.run()
        torch.cuda.synchronize()
        rng = np.random.default_rng(5)
        for i, x in enumerate(xs):
            codes, n, stats = fic.encode_image(x, params)
            torch.cuda.synchronize()
            single = fic.codes_numpy(codes, n)
            got = fic.codes_numpy(b.image_codes(i), int(b.n_codes[i].item()))
            assert int(n.item()) == int(b.n_codes[i].item())
            assert np.array_equal(got, single)
            assert np.array_equal(b.stats[i].cpu().numpy(), stats.cpu().numpy())
            if i >= 3:
                continue
            # sampled oracle check of level-0 codes
            img = imgs[i]
            pool, _ = oracle.entropy_pool(img, 16, 8, 2.5, 256)
            lv0 = got[got["level"] == 0]
            pick = rng.choice(len(lv0), size=min(12, len(lv0)), replace=False)
            ranges = np.stack([lv0["y"][pick], lv0["x"][pick]], 1).astype(np.int32)
            ref = oracle.match_level(img, 16, 8, oracle.PAPER_K[0], pool, ranges)
            say(f"[batch] image {i} side {img.shape[0]}: {len(pick)} sampled ranges")
            for f in ("dom", "iso", "s_idx", "k", "q_o"):
                assert np.array_equal(lv0[f][pick].astype(np.int64), ref[f].astype(np.int64)), f
            assert np.array_equal(lv0["e_num"][pick].astype(np.int64) * 256, ref["e_lit"])
    finally:
        b.close()


@pytest.mark.parametrize("min_pool,sets", [(64, "paper"), (16, "plain"), (32, "calibrated")])
def test_persistent_form_matches_oracle_and_level_form_over_replays(dev, min_pool, sets):
    """The persistent form (one kernel draining a device queue of range tiles)
    gives the level form's codes, counts and statistics bit for bit, and the
    oracle's, on mixed sizes, over replays with eager work in between."""
    imgs = mixed_images()
    ks = {"paper": oracle.PAPER_K, "plain": (oracle.PLAIN_K,) * 4, "calibrated": ((1,), (3,), (9,), (9,))}[sets]
    params = fic.EncoderParams(s_sets=ks, min_pool=min_pool)
    refs = [oracle.encode_image(im, s_sets=ks, min_pool=min_pool) for im in imgs]
    xs = [torch.from_numpy(im).to(dev) for im in imgs]
    say(f"[persistent] mixed sizes min_pool={min_pool} sets={sets}")
    lv = fic.Batch(xs, params)
    pq = fic.Batch(xs, params)
    try:
        lv.set_form(fic.FORM_LEVELS)
        lv.run()
        pq.set_form(fic.FORM_PERSISTENT)
        form, tiles, wgs = pq.form()
        say(f"[persistent] tiles {tiles} workgroups {wgs}")
        assert form == fic.FORM_PERSISTENT and all(t > 0 for t in tiles) and wgs > 0
        torch.cuda.synchronize()
        for rep in range(3):
            pq.codes.fill_(0xAB)
            pq.n_codes.fill_(-1)
            pq.stats.fill_(0)
            pq.run()
            torch.cuda.synchronize()
            say(f"[persistent] replay {rep}")
            assert torch.equal(pq.n_codes, lv.n_codes)
            assert torch.equal(pq.stats, lv.stats)
            for i, (ref, rst) in enumerate(refs):
                got = fic.codes_numpy(pq.image_codes(i), int(pq.n_codes[i].item()))
                assert np.array_equal(pq.image_codes(i).cpu().numpy(), lv.image_codes(i).cpu().numpy())
                assert_codes_equal(got, ref)
            fic.encode_image(xs[0], params)  # other work on the torch stream in between
            torch.cuda.synchronize()
    finally:
        lv.close()
        pq.close()


@pytest.mark.parametrize("tiles,wgs", [([8, 16, 16, 64], 1), ([16, 64, 128, 256], 7), ([8, 128, 256, 256], 0)])
def test_persistent_tile_shapes_do_not_change_codes(dev, tiles, wgs):
    """Ranges per tile and the number of resident workgroups change only the
    schedule (one workgroup runs every tile itself; seven share them)."""
    imgs = mixed_images()[:4]
    params = fic.EncoderParams(s_sets=oracle.PAPER_K, min_pool=32)
    xs = [torch.from_numpy(im).to(dev) for im in imgs]
    b = fic.Batch(xs, params)
    try:
        b.set_form(fic.FORM_LEVELS)
        b.run()
        torch.cuda.synchronize()
        base = [b.image_codes(i).cpu().numpy().copy() for i in range(len(xs))]
        nb = b.n_codes.clone()
        say(f"[persistent] tiles {tiles} workgroups {wgs}")
        b.set_form(fic.FORM_PERSISTENT, tiles, wgs)
        f, t, w = b.form()
        assert t == tiles and (w == wgs if wgs else w > 0)
        for _ in range(2):
            b.run()
            torch.cuda.synchronize()
            assert torch.equal(b.n_codes, nb)
            for i in range(len(xs)):
                assert np.array_equal(b.image_codes(i).cpu().numpy(), base[i])
    finally:
        b.close()


def test_persistent_form_workload_images_match_level_form(dev):
    """Eight images of the 64-image batch workload (sides 256..2048), paper's
    preset: persistent form == level form bit for bit (the level form is
    oracle-checked on the same images above)."""
    imgs = synth.batch_images(8)
    xs = [torch.from_numpy(im).to(dev) for im in imgs]
    params = fic.EncoderParams(s_sets=fic.PAPER_K)
    b = fic.Batch(xs, params)
    try:
        b.set_form(fic.FORM_LEVELS)
        b.run()
        torch.cuda.synchronize()
        base = [b.image_codes(i).cpu().numpy().copy() for i in range(len(xs))]
        nb, sb = b.n_codes.clone(), b.stats.clone()
        b.set_form(fic.FORM_PERSISTENT)
        b.run()
        torch.cuda.synchronize()
        assert torch.equal(b.n_codes, nb) and torch.equal(b.stats, sb)
        for i in range(len(xs)):
            assert np.array_equal(b.image_codes(i).cpu().numpy(), base[i])
    finally:
        b.close()
