"""Writes workload_sha256.json: the SHA-256 of every seeded workload image the
benchmarks and tests draw (shape, then the uint8 pixels in row order). A change
to the generators, or to numpy's generator or FFT, changes a digest, and
tests/test_synth_pins.py fails instead of every workload changing silently.
Run from the repository root: python tests/golden/make_workload_pins.py"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_1501_04140_amd import synth  # noqa: E402


def digest(img) -> str:
    h = hashlib.sha256()
    h.update(("%dx%d:" % img.shape).encode())
    h.update(img.tobytes())
    return h.hexdigest()


def workloads():
    """(name, image) of each pinned input: the single-level, quadtree and precision
    images, the first 8 images of the 64-image batch, 4 training images and the first
    evaluation image of the learned form."""
    yield "single_level_128_seed0", synth.single_level_image(0)
    yield "quadtree_512_seed0", synth.quadtree_image(0)
    yield "precision_1024_seed0", synth.precision_image(0)
    for i, im in enumerate(synth.batch_images(8)):
        yield f"batch_{i}", im
    for i in range(4):
        yield f"learned_train_{i}", synth.learned_train_image(i)
    yield "learned_eval_0", synth.learned_eval_image(0)


if __name__ == "__main__":
    pins = {name: {"shape": list(im.shape), "sha256": digest(im)} for name, im in workloads()}
    with open(os.path.join(HERE, "workload_sha256.json"), "w") as f:
        json.dump(pins, f, indent=1, sort_keys=True)
        f.write("\n")
    print(len(pins), "pins written")
