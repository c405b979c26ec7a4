"""Fractal image encoding on AMD Instinct MI355X.

Exhaustive range-domain matching with the entropy-filtered domain pool and
predefined contrast values of Miar Naimi & Salarian (arXiv 1501.04140), in
hand-written gfx950 HIP kernels behind the C ABI of include/fic.h.
The binding lives in ``paper_1501_04140_amd.fic``.
"""
from . import synth  # noqa: F401
