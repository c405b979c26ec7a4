"""The seeded workload images are the ones pinned by SHA-256 (shape and pixels):
the workloads cannot change without this test failing."""
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PINS = json.load(open(os.path.join(HERE, "golden", "workload_sha256.json")))


def _workloads():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_workload_pins",
                                                  os.path.join(HERE, "golden", "make_workload_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MOD = _workloads()


@pytest.mark.parametrize("name,img", list(MOD.workloads()), ids=lambda v: v if isinstance(v, str) else "")
def test_workload_image_matches_its_pin(name, img):
    pin = PINS[name]
    assert list(img.shape) == pin["shape"]
    assert MOD.digest(img) == pin["sha256"], name


def test_every_pin_is_checked():
    assert sorted(PINS) == sorted(n for n, _ in MOD.workloads())
