"""Python binding of libfic (include/fic.h): argument marshalling only.

Every step of the encoder runs in the library's HIP kernels. PyTorch only
provides device memory and the current stream. The binding refuses to run
when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfic.so")

FIC_OK, FIC_EINVAL, FIC_ECAPACITY, FIC_EDEVICE, FIC_ENOMEM = 0, -1, -2, -3, -4
MATCH_AUTO, MATCH_VALU, MATCH_MFMA_I8, MATCH_FP32, MATCH_MFMA_F16 = 0, 1, 2, 3, 4
MAX_S = 11
PLAIN_K = tuple(range(11))                   # s = 0, 0.1, ..., 1.0 (Section 2)
PAPER_K = ((1,), (2, 4), (3, 8), (5, 9))     # predefined s per step (Section 3.1)
LEVELS = (16, 8, 4, 2)                       # range sides of the four steps (Section 2)

MATCH_DTYPE = np.dtype([("e_num", "<i8"), ("dom", "<i4"), ("iso", "u1"), ("s_idx", "u1"),
                        ("k", "u1"), ("flags", "u1"), ("q_o", "<i2"), ("pad_", "<i2"),
                        ("E", "<f4")])
CODE_DTYPE = np.dtype([("e_num", "<i8"), ("dom", "<i4"), ("y", "<i2"), ("x", "<i2"),
                       ("dy", "<i2"), ("dx", "<i2"), ("q_o", "<i2"), ("log2B", "u1"),
                       ("iso", "u1"), ("k", "u1"), ("s_idx", "u1"), ("level", "u1"),
                       ("pad_", "u1", (5,))])
STATS_DTYPE = np.dtype([("matches", "<i8"), ("pool", "<i4"), ("passed", "<i4"),
                        ("active", "<i4"), ("accepted", "<i4")])
KTIME_DTYPE = np.dtype([("name", "S24"), ("launches", "<i4"), ("pad_", "<i4"),
                        ("total_ms", "<f8")])
assert MATCH_DTYPE.itemsize == 24 and CODE_DTYPE.itemsize == 32 and STATS_DTYPE.itemsize == 24
assert KTIME_DTYPE.itemsize == 40


class FicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfic error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("B0", ctypes.c_int32), ("L", ctypes.c_int32 * 4),
                ("n_s", ctypes.c_int32 * 4), ("s_k", (ctypes.c_int8 * 12) * 4),
                ("rms_thresh", ctypes.c_float), ("entropy_mode", ctypes.c_int32),
                ("entropy_bits", ctypes.c_float), ("min_pool", ctypes.c_int32)]


@dataclass
class EncoderParams:
    """Quadtree encoder settings (fic_params)."""
    levels: tuple = LEVELS
    steps: tuple | None = None                 # default: L = B/2 (1 at B = 2)
    s_sets: tuple = PAPER_K
    rms: float = 8.0
    entropy_mode: int = 1
    entropy_bits: float = 2.5
    min_pool: int = 256
    extra: dict = field(default_factory=dict)

    def to_c(self) -> Params:
        p = Params()
        n = len(self.levels)
        p.n_levels = n
        p.B0 = int(self.levels[0])
        steps = self.steps or tuple(max(int(B) // 2, 1) for B in self.levels)
        for l in range(n):
            p.L[l] = int(steps[l])
            ks = tuple(int(k) for k in self.s_sets[l])
            p.n_s[l] = len(ks)
            for i, k in enumerate(ks):
                p.s_k[l][i] = k
        p.rms_thresh = float(self.rms)
        p.entropy_mode = int(self.entropy_mode)
        p.entropy_bits = float(self.entropy_bits)
        p.min_pool = int(self.min_pool)
        return p


_lib = None


def load():
    """Load libfic.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FicError(FIC_EDEVICE, f"{LIB_PATH} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
    lib.fic_encode_level.argtypes = [vp, i32, i32, i32, i32, i32, vp, i32, i32, f32, i32, vp, i32,
                                     vp, vp, vp, vp]
    lib.fic_encode_level_ex.argtypes = [vp, i32, i32, i32, i32, i32, vp, i32, i32, f32, i32, vp,
                                        i32, vp, vp, vp, i32, vp]
    lib.fic_encode_level_noalloc.argtypes = [vp, i32, i32, i32, i32, i32, vp, i32, i32, f32, i32, vp,
                                             i32, vp, vp, vp, vp]
    lib.fic_encode_image.argtypes = [vp, i32, i32, i32, ctypes.POINTER(Params), vp, i32, vp, vp, vp]
    lib.fic_decode.argtypes = [vp, i32, i32, i32, i32, vp, i32, vp]
    lib.fic_sse.argtypes = [vp, i32, vp, i32, i32, i32, vp, vp]
    lib.fic_calibrate_s.argtypes = [vp, i32, i32, i32, ctypes.POINTER(Params), vp, vp]
    lib.fic_profile_end.argtypes = [vp, i32, vp]
    lib.fic_batch_create.argtypes = [i32, vp, vp, vp, vp, ctypes.POINTER(Params), vp, vp, vp, vp,
                                     ctypes.POINTER(vp)]
    lib.fic_batch_run.argtypes = [vp, vp]
    lib.fic_batch_run_eager.argtypes = [vp, vp]
    lib.fic_batch_set_chunks.argtypes = [vp, vp]
    lib.fic_batch_get_chunks.argtypes = [vp, vp]
    lib.fic_batch_autotune.argtypes = [vp, vp, i32, ctypes.c_char_p, ctypes.POINTER(f32)]
    lib.fic_batch_destroy.argtypes = [vp]
    lib.fic_batch_set_form.argtypes = [vp, i32, vp, i32]
    lib.fic_peak_probe.argtypes = [i32, vp, ctypes.POINTER(ctypes.c_double)]
    lib.fic_batch_get_form.argtypes = [vp, vp, vp, vp]
    lib.fic_mlp_create.argtypes = [vp, f32, ctypes.POINTER(vp)]
    lib.fic_mlp_destroy.argtypes = [vp]
    lib.fic_mlp_get_params.argtypes = [vp, vp]
    lib.fic_mlp_embed.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, i32, vp, vp]
    lib.fic_mlp_loss_grad.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, i32, vp, vp, vp]
    lib.fic_mlp_adam.argtypes = [vp, vp, f32, f32, f32, f32, vp]
    lib.fic_mlp_train_step.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, i32, f32, vp, vp]
    lib.fic_topk_similar.argtypes = [vp, i32, vp, i32, i32, vp, vp, vp, vp]
    lib.fic_encode_level_learned.argtypes = [vp, vp, i32, i32, i32, i32, vp, i32, i32, f32, vp, vp,
                                             vp, vp]
    lib.fic_level_codes.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    lib.fic_encode_image_ex.argtypes = [vp, i32, i32, i32, ctypes.POINTER(Params), vp, i32, vp, vp, vp,
                                        vp, vp]
    lib.fic_s_histogram.argtypes = [vp, i32, i32, i32, ctypes.POINTER(Params), i32, vp, vp]
    lib.fic_select_s.argtypes = [vp, i32, f32, vp, vp]
    lib.fic_stream_bound.argtypes = [i32, i32, ctypes.POINTER(Params)]
    lib.fic_stream_bound.restype = ctypes.c_int64
    lib.fic_pack_stream.argtypes = [vp, i32, i32, i32, ctypes.POINTER(Params), vp, vp, vp, vp,
                                    ctypes.c_int64, vp, vp]
    lib.fic_unpack_stream.argtypes = [vp, ctypes.c_int64, vp, i32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.fic_last_error.restype = ctypes.c_char_p
    for name in ("fic_encode_level", "fic_encode_level_ex", "fic_encode_level_noalloc", "fic_encode_image", "fic_decode", "fic_sse",
                 "fic_calibrate_s", "fic_version", "fic_profile_begin", "fic_profile_end",
                 "fic_batch_create", "fic_batch_run", "fic_batch_run_eager", "fic_batch_set_chunks", "fic_batch_get_chunks",
                 "fic_batch_autotune", "fic_batch_destroy", "fic_batch_set_form", "fic_batch_get_form", "fic_peak_probe", "fic_mlp_create", "fic_mlp_destroy",
                 "fic_mlp_get_params", "fic_mlp_embed", "fic_mlp_loss_grad", "fic_mlp_adam",
                 "fic_mlp_train_step", "fic_topk_similar", "fic_encode_level_learned",
                 "fic_level_codes", "fic_encode_image_ex", "fic_pack_stream", "fic_unpack_stream",
                 "fic_s_histogram", "fic_select_s"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != FIC_OK:
        raise FicError(rc, load().fic_last_error().decode())


def _stream(stream):
    """The HIP stream to queue on: `stream` (a torch stream), else torch's current
    stream of the current device, read as a raw handle where torch offers that
    (building the Stream object costs a few microseconds per call)."""
    import torch
    if stream is None:
        raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
        if raw is not None:
            return ctypes.c_void_p(raw(torch._C._cuda_getDevice()))
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_u8_image(img):
    import torch
    if not isinstance(img, torch.Tensor) or img.dtype != torch.uint8 or img.dim() != 2:
        raise TypeError("image must be a 2-D torch.uint8 tensor")
    if not img.is_cuda:
        raise TypeError("image must be on the GPU")
    if img.stride(1) != 1:
        raise ValueError("image rows must be contiguous")
    return img


def encode_level(img, B: int, L: int, s_k=PLAIN_K, entropy_mode: int = 0,
                 entropy_bits: float = 2.5, min_pool: int = 256, ranges=None,
                 return_pool: bool = False, stream=None, variant: int = MATCH_AUTO):
    """fic_encode_level_ex. Returns a uint8 tensor [n_ranges, 24] of fic_match records
    (and, with return_pool, the pool index tensor and a 1-element pool-count tensor)."""
    import torch
    img = _dev_u8_image(img)
    H, W = img.shape
    lib = load()
    ks = (ctypes.c_int8 * max(1, len(s_k)))(*[int(k) for k in s_k])
    if ranges is not None:
        ranges = ranges.to(device=img.device, dtype=torch.int32).contiguous().reshape(-1, 2)
        n = ranges.shape[0]
    else:
        n = (H // B) * (W // B) if B > 0 else 0
    out = torch.empty((max(n, 1), 24), dtype=torch.uint8, device=img.device)
    gx = (W - 2 * B) // L + 1 if L > 0 else 1
    gy = (H - 2 * B) // L + 1 if L > 0 else 1
    pool = torch.empty(max(gx * gy, 1), dtype=torch.int32, device=img.device) if return_pool else None
    pcount = torch.zeros(1, dtype=torch.int32, device=img.device) if return_pool else None
    rc = lib.fic_encode_level_ex(img.data_ptr(), H, W, img.stride(0), B, L, ks, len(s_k),
                                 entropy_mode, entropy_bits, min_pool,
                                 ranges.data_ptr() if ranges is not None else None, n,
                                 out.data_ptr(), pool.data_ptr() if pool is not None else None,
                                 pcount.data_ptr() if pcount is not None else None, variant,
                                 _stream(stream))
    _check(rc)
    out = out[:n]
    return (out, pool, pcount) if return_pool else out


def encode_level_noalloc(img, B: int, L: int, s_k=PLAIN_K, entropy_mode: int = 0,
                         entropy_bits: float = 2.5, min_pool: int = 256, ranges=None, out=None,
                         pool=None, pcount=None, stream=None):
    """fic_encode_level_noalloc: fic_encode_level with the library's workspace in
    its fixed device scratch. The caller may pass the output tensors in (out:
    uint8 [n_ranges, 24]; pool: int32 [grid domains]; pcount: int32 [1]); those
    it leaves as None are not written, except `out`, which is created here."""
    import torch
    img = _dev_u8_image(img)
    H, W = img.shape
    lib = load()
    ks = (ctypes.c_int8 * max(1, len(s_k)))(*[int(k) for k in s_k])
    if ranges is not None:
        ranges = ranges.to(device=img.device, dtype=torch.int32).contiguous().reshape(-1, 2)
        n = ranges.shape[0]
    else:
        n = (H // B) * (W // B) if B > 0 else 0
    if out is None:
        out = torch.empty((max(n, 1), 24), dtype=torch.uint8, device=img.device)
    rc = lib.fic_encode_level_noalloc(img.data_ptr(), H, W, img.stride(0), B, L, ks, len(s_k),
                                      entropy_mode, entropy_bits, min_pool,
                                      ranges.data_ptr() if ranges is not None else None, n,
                                      out.data_ptr(), pool.data_ptr() if pool is not None else None,
                                      pcount.data_ptr() if pcount is not None else None,
                                      _stream(stream))
    _check(rc)
    return out[:n]


PEAK_PROBES = {"valu_fma_ops": 0, "dot2_ops": 1, "mfma_f16_flops": 2, "mfma_i8_ops": 3, "hbm_copy_bytes": 4}


def peak_probe(stream=None) -> dict:
    """fic_peak_probe for every probe: measured rates per second of this device."""
    out = {}
    for name, what in PEAK_PROBES.items():
        v = ctypes.c_double(0.0)
        _check(load().fic_peak_probe(what, _stream(stream), ctypes.byref(v)))
        out[name] = v.value
    return out


def code_capacity(H: int, W: int, levels=LEVELS) -> int:
    """Most codes a quadtree with these levels can emit."""
    return (H // levels[-1]) * (W // levels[-1])


def encode_image(img, params: EncoderParams | None = None, capacity: int | None = None,
                 stream=None, out=None):
    """fic_encode_image. Returns (codes uint8 [capacity, 32], n_codes int32 [1],
    stats uint8 [n_levels, 24]) as device tensors. ``out`` may pass that triple
    back in to reuse its buffers."""
    import torch
    img = _dev_u8_image(img)
    params = params or EncoderParams()
    H, W = img.shape
    if out is not None:
        codes, ncodes, stats = out
        cap = codes.shape[0]
    else:
        cap = code_capacity(H, W, params.levels) if capacity is None else capacity
        codes = torch.empty((max(cap, 1), 32), dtype=torch.uint8, device=img.device)
        ncodes = torch.zeros(1, dtype=torch.int32, device=img.device)
        stats = torch.zeros((len(params.levels), 24), dtype=torch.uint8, device=img.device)
    p = params.to_c()
    rc = load().fic_encode_image(img.data_ptr(), H, W, img.stride(0), ctypes.byref(p),
                                 codes.data_ptr(), cap, ncodes.data_ptr(), stats.data_ptr(),
                                 _stream(stream))
    _check(rc)
    return codes, ncodes, stats


FORM_LEVELS = 0
FORM_PERSISTENT = 1


class Batch:
    """fic_batch_*: n images (any sizes the encoder accepts) encoded by one
    captured hipGraph. The images must stay alive and in place; ``codes`` holds
    every image's codes back to back (``offsets[i]`` .. ``offsets[i+1]``)."""

    def __init__(self, images, params: EncoderParams | None = None):
        import torch
        self.images = [_dev_u8_image(im) for im in images]
        if not self.images:
            raise ValueError("empty batch")
        self.params = params or EncoderParams()
        n = len(self.images)
        dev = self.images[0].device
        caps = [max(code_capacity(im.shape[0], im.shape[1], self.params.levels), 1) for im in self.images]
        self.offsets = np.concatenate([[0], np.cumsum(caps)]).astype(np.int64)
        self.codes = torch.empty((int(self.offsets[-1]), 32), dtype=torch.uint8, device=dev)
        self.n_codes = torch.zeros(n, dtype=torch.int32, device=dev)
        self.stats = torch.zeros((n, len(self.params.levels), 24), dtype=torch.uint8, device=dev)
        ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in self.images])
        H = (ctypes.c_int32 * n)(*[im.shape[0] for im in self.images])
        W = (ctypes.c_int32 * n)(*[im.shape[1] for im in self.images])
        pitch = (ctypes.c_int32 * n)(*[im.stride(0) for im in self.images])
        off = (ctypes.c_int64 * (n + 1))(*[int(v) for v in self.offsets])
        self._p = self.params.to_c()
        self._h = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(load().fic_batch_create(n, ptrs, H, W, pitch, ctypes.byref(self._p),
                                       self.codes.data_ptr(), off, self.n_codes.data_ptr(),
                                       self.stats.data_ptr(), ctypes.byref(self._h)))

    def run(self, stream=None):
        _check(load().fic_batch_run(self._h, _stream(stream)))
        return self.codes, self.n_codes, self.stats

    def run_eager(self, stream=None):
        """Same kernels, launched one by one (for per-kernel timing)."""
        _check(load().fic_batch_run_eager(self._h, _stream(stream)))
        return self.codes, self.n_codes, self.stats

    def chunks(self) -> list:
        out = (ctypes.c_int32 * len(self.params.levels))()
        _check(load().fic_batch_get_chunks(self._h, out))
        return list(out)

    def set_chunks(self, chunks):
        arr = (ctypes.c_int32 * len(self.params.levels))(*[int(c) for c in chunks])
        _check(load().fic_batch_set_chunks(self._h, arr))

    def set_form(self, form: int, tiles=None, workgroups: int = 0):
        """fic_batch_set_form: FORM_LEVELS or FORM_PERSISTENT, with the persistent
        form's ranges per tile per level (None or 0 = default) and resident
        workgroups (0 = every one that fits)."""
        nl = len(self.params.levels)
        arr = None if tiles is None else (ctypes.c_int32 * nl)(*[int(t) for t in tiles])
        _check(load().fic_batch_set_form(self._h, int(form), arr, int(workgroups)))

    def form(self):
        """(form, ranges per tile per level, workgroups) in use."""
        nl = len(self.params.levels)
        f = ctypes.c_int32(0)
        w = ctypes.c_int32(0)
        t = (ctypes.c_int32 * nl)()
        _check(load().fic_batch_get_form(self._h, ctypes.byref(f), t, ctypes.byref(w)))
        return f.value, list(t), w.value

    def autotune(self, reps: int = 3, cache_path: str | None = None, stream=None) -> float:
        ms = ctypes.c_float(0.0)
        path = cache_path.encode() if cache_path else None
        _check(load().fic_batch_autotune(self._h, _stream(stream), reps, path, ctypes.byref(ms)))
        return ms.value

    def image_codes(self, i: int):
        """Codes of image i (device uint8 [n, 32]); call after run() has finished."""
        n = int(self.n_codes[i].item())
        return self.codes[int(self.offsets[i]):int(self.offsets[i]) + n]

    def close(self):
        if self._h:
            load().fic_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_PARAMS = 98880
FLAG_FALLBACK = 1


def _ptr(t):
    return None if t is None else t.data_ptr()


class Mlp:
    """fic_mlp_*: the learned domain proposal network (64-256-256-64) with its
    Adam state. ``init`` is a flat float32 parameter vector (see include/fic.h)."""

    def __init__(self, init, tau: float = 0.1):
        init = np.ascontiguousarray(init, dtype=np.float32)
        if init.size != MLP_PARAMS:
            raise ValueError(f"init must hold {MLP_PARAMS} values")
        self.tau = tau
        self._init = init
        self._h = ctypes.c_void_p()
        _check(load().fic_mlp_create(init.ctypes.data, tau, ctypes.byref(self._h)))

    def params(self) -> np.ndarray:
        out = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(load().fic_mlp_get_params(self._h, out.ctypes.data))
        return out

    def embed(self, img, kind: int, L: int = 4, idx=None, stream=None):
        """fp16 [n, 64] embeddings of ranges (kind 0; idx = [n, 2] corners) or domains
        (kind 1; idx = [n] indices); idx None = all of them."""
        import torch
        img = _dev_u8_image(img)
        H, W = img.shape
        if idx is not None:
            idx = idx.to(device=img.device, dtype=torch.int32).contiguous()
            n = idx.shape[0]
        elif kind == 0:
            n = (H // 8) * (W // 8)
        else:
            n = ((H - 16) // L + 1) * ((W - 16) // L + 1)
        out = torch.empty((max(n, 1), 64), dtype=torch.float16, device=img.device)
        _check(load().fic_mlp_embed(self._h, img.data_ptr(), H, W, img.stride(0), kind, L, _ptr(idx),
                                    n, out.data_ptr(), _stream(stream)))
        return out[:n]

    def loss_grad(self, img, L: int, labels, ranges=None, stream=None):
        """(mean loss [1], gradient [MLP_PARAMS]) as float32 device tensors."""
        import torch
        img = _dev_u8_image(img)
        H, W = img.shape
        labels = labels.to(device=img.device, dtype=torch.int32).contiguous()
        if ranges is not None:
            ranges = ranges.to(device=img.device, dtype=torch.int32).contiguous()
        loss = torch.zeros(1, dtype=torch.float32, device=img.device)
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=img.device)
        _check(load().fic_mlp_loss_grad(self._h, img.data_ptr(), H, W, img.stride(0), L, _ptr(ranges),
                                        labels.data_ptr(), labels.shape[0], loss.data_ptr(),
                                        grad.data_ptr(), _stream(stream)))
        return loss, grad

    def adam(self, grad=None, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8, stream=None):
        _check(load().fic_mlp_adam(self._h, _ptr(grad), lr, beta1, beta2, eps, _stream(stream)))

    def train_step(self, img, L: int, labels, ranges=None, lr: float = 1e-3, loss=None, stream=None):
        import torch
        img = _dev_u8_image(img)
        H, W = img.shape
        if ranges is not None:
            ranges = ranges.to(device=img.device, dtype=torch.int32).contiguous()
        loss = torch.zeros(1, dtype=torch.float32, device=img.device) if loss is None else loss
        _check(load().fic_mlp_train_step(self._h, img.data_ptr(), H, W, img.stride(0), L, _ptr(ranges),
                                         labels.data_ptr(), labels.shape[0], lr, loss.data_ptr(),
                                         _stream(stream)))
        return loss

    def topk(self, q, keys, k: int, stream=None):
        """(idx int32 [nq, k], score float32 [nq, k]) of fp16 [n, 64] device tensors: the
        k keys of largest int8-code similarity per query (fic_topk_similar)."""
        import torch
        q = q.contiguous()
        keys = keys.contiguous()
        idx = torch.empty((max(q.shape[0], 1), k), dtype=torch.int32, device=q.device)
        score = torch.empty((max(q.shape[0], 1), k), dtype=torch.float32, device=q.device)
        _check(load().fic_topk_similar(q.data_ptr(), q.shape[0], keys.data_ptr(), keys.shape[0], k,
                                       idx.data_ptr(), score.data_ptr(), self._h, _stream(stream)))
        return idx[:q.shape[0]], score[:q.shape[0]]

    def encode_level(self, img, L: int = 4, s_k=PLAIN_K, topk: int = 32, rms: float = 8.0,
                     return_proposals: bool = False, stream=None):
        """fic_encode_level_learned: (matches uint8 [nr, 24], n_fallback int32 [1][, proposals])."""
        import torch
        img = _dev_u8_image(img)
        H, W = img.shape
        nr = (H // 8) * (W // 8)
        ks = (ctypes.c_int8 * max(1, len(s_k)))(*[int(k) for k in s_k])
        out = torch.empty((max(nr, 1), 24), dtype=torch.uint8, device=img.device)
        nfb = torch.zeros(1, dtype=torch.int32, device=img.device)
        props = torch.empty((max(nr, 1), topk), dtype=torch.int32, device=img.device) if return_proposals else None
        _check(load().fic_encode_level_learned(self._h, img.data_ptr(), H, W, img.stride(0), L, ks, len(s_k),
                                               topk, rms, out.data_ptr(), _ptr(props), nfb.data_ptr(),
                                               _stream(stream)))
        return (out[:nr], nfb, props[:nr]) if return_proposals else (out[:nr], nfb)

    def close(self):
        if self._h:
            load().fic_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def level_codes(matches, H: int, W: int, B: int, L: int, stream=None):
    """fic_level_codes: uint8 [nr, 32] codes of a full range grid's matches."""
    import torch
    nr = (H // B) * (W // B)
    codes = torch.empty((max(nr, 1), 32), dtype=torch.uint8, device=matches.device)
    _check(load().fic_level_codes(matches.data_ptr(), H, W, B, L, codes.data_ptr(), _stream(stream)))
    return codes[:nr]


def s_histogram(img, params: EncoderParams | None = None, low_entropy_only: bool = False, hist=None,
                stream=None):
    """fic_s_histogram: adds the image's optimal-contrast counts to ``hist`` (device int64
    [4, 11], created zeroed when None) and returns it."""
    import torch
    img = _dev_u8_image(img)
    H, W = img.shape
    p = (params or EncoderParams()).to_c()
    if hist is None:
        hist = torch.zeros((4, 11), dtype=torch.int64, device=img.device)
    _check(load().fic_s_histogram(img.data_ptr(), H, W, img.stride(0), ctypes.byref(p),
                                  int(low_entropy_only), hist.data_ptr(), _stream(stream)))
    return hist


def select_s(hist, n_levels: int = 4, second_frac: float = 0.5):
    """fic_select_s (host): predefined contrast sets (tuples of k) from histograms."""
    h = np.ascontiguousarray(np.asarray(hist, dtype=np.uint64).reshape(-1, 11)[:n_levels])
    sk = np.zeros((4, 2), dtype=np.int8)
    ns = np.zeros(4, dtype=np.int32)
    _check(load().fic_select_s(h.ctypes.data, n_levels, second_frac, sk.ctypes.data, ns.ctypes.data))
    return tuple(tuple(int(v) for v in sk[l, :ns[l]]) for l in range(n_levels))


def stream_bound(H: int, W: int, params: EncoderParams | None = None) -> int:
    p = (params or EncoderParams()).to_c()
    n = load().fic_stream_bound(H, W, ctypes.byref(p))
    if n < 0:
        raise FicError(FIC_EINVAL, "parameters do not fit the image")
    return int(n)


def encode_image_stream(img, params: EncoderParams | None = None, stream=None):
    """fic_encode_image_ex then fic_pack_stream. Returns (stream bytes as a host numpy
    uint8 array, codes, n_codes, stats) -- the last three as in encode_image."""
    import torch
    img = _dev_u8_image(img)
    params = params or EncoderParams()
    H, W = img.shape
    p = params.to_c()
    cap = code_capacity(H, W, params.levels)
    dev = img.device
    codes = torch.empty((max(cap, 1), 32), dtype=torch.uint8, device=dev)
    ncodes = torch.zeros(1, dtype=torch.int32, device=dev)
    stats = torch.zeros((len(params.levels), 24), dtype=torch.uint8, device=dev)
    nflag = sum((H // B) * (W // B) for B in params.levels[:-1])
    flags = torch.zeros(max((nflag + 31) // 32, 1), dtype=torch.int32, device=dev)
    steps = params.steps or tuple(max(int(B) // 2, 1) for B in params.levels)
    ngrid = sum(((H - 2 * B) // L + 1) * ((W - 2 * B) // L + 1) for B, L in zip(params.levels, steps))
    pools = torch.zeros(max(ngrid, 1), dtype=torch.int32, device=dev)
    lib = load()
    st = _stream(stream)
    _check(lib.fic_encode_image_ex(img.data_ptr(), H, W, img.stride(0), ctypes.byref(p), codes.data_ptr(),
                                   cap, ncodes.data_ptr(), stats.data_ptr(), flags.data_ptr(),
                                   pools.data_ptr(), st))
    n = int(ncodes.item())
    bound = stream_bound(H, W, params)
    out = torch.zeros(bound, dtype=torch.uint8, device=dev)
    nbytes = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib.fic_pack_stream(codes.data_ptr(), min(n, cap), H, W, ctypes.byref(p), stats.data_ptr(),
                               flags.data_ptr(), pools.data_ptr(), out.data_ptr(), bound,
                               nbytes.data_ptr(), st))
    nb = int(nbytes.item())
    return out[:nb].cpu().numpy(), codes, ncodes, stats


def unpack_stream(data):
    """fic_unpack_stream (host): (codes numpy CODE_DTYPE, H, W); e_num is -1."""
    buf = np.ascontiguousarray(np.frombuffer(bytes(data), dtype=np.uint8))
    n = ctypes.c_int32(0)
    H = ctypes.c_int32(0)
    W = ctypes.c_int32(0)
    lib = load()
    rc = lib.fic_unpack_stream(buf.ctypes.data, buf.size, None, 0, ctypes.byref(n), ctypes.byref(H),
                               ctypes.byref(W))
    if rc not in (FIC_OK, FIC_ECAPACITY):
        _check(rc)
    codes = np.zeros(max(n.value, 1), dtype=CODE_DTYPE)
    _check(lib.fic_unpack_stream(buf.ctypes.data, buf.size, codes.ctypes.data, n.value, ctypes.byref(n),
                                 ctypes.byref(H), ctypes.byref(W)))
    return codes[:n.value], H.value, W.value


def decode(codes, n_codes: int, H: int, W: int, iters: int = 64, stream=None):
    """fic_decode (synchronous). Returns a uint8 [H, W] device tensor."""
    import torch
    out = torch.empty((H, W), dtype=torch.uint8, device=codes.device)
    rc = load().fic_decode(codes.data_ptr(), int(n_codes), H, W, iters, out.data_ptr(), W,
                           _stream(stream))
    _check(rc)
    return out


def sse(a, b, stream=None):
    """fic_sse: sum of squared differences of two uint8 images, as an int64 device tensor."""
    import torch
    a, b = _dev_u8_image(a), _dev_u8_image(b)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    out = torch.zeros(1, dtype=torch.int64, device=a.device)
    rc = load().fic_sse(a.data_ptr(), a.stride(0), b.data_ptr(), b.stride(0), a.shape[0],
                        a.shape[1], out.data_ptr(), _stream(stream))
    _check(rc)
    return out


def psnr(a, b) -> float:
    """10 log10(255^2 / MSE) with the SSE from the GPU."""
    import math
    s = int(sse(a, b).item())
    return float("inf") if s == 0 else 10.0 * math.log10(255.0 ** 2 * a.numel() / s)


def calibrate_s(img, params: EncoderParams | None = None, stream=None):
    """fic_calibrate_s: per-level mean best k of kept low-entropy ranges (-1 = none)."""
    img = _dev_u8_image(img)
    params = params or EncoderParams()
    p = params.to_c()
    out = (ctypes.c_int8 * 4)()
    rc = load().fic_calibrate_s(img.data_ptr(), img.shape[0], img.shape[1], img.stride(0),
                                ctypes.byref(p), out, _stream(stream))
    _check(rc)
    return [int(out[i]) for i in range(len(params.levels))]


def calibrated_sets(ks, fallback=PAPER_K):
    """Per-level 1-element contrast sets from calibrate_s output (fallback where -1)."""
    return tuple((k,) if k >= 0 else tuple(fallback[l]) for l, k in enumerate(ks))


def profile_begin():
    """Start bracketing every library kernel launch with HIP events."""
    _check(load().fic_profile_begin())


def profile_end(max_labels: int = 64) -> dict:
    """Stop profiling; returns {label: (launches, total_ms)} from the HIP events."""
    buf = np.zeros(max_labels, dtype=KTIME_DTYPE)
    n = ctypes.c_int32(0)
    _check(load().fic_profile_end(buf.ctypes.data, max_labels, ctypes.byref(n)))
    return {r["name"].decode(): (int(r["launches"]), float(r["total_ms"]))
            for r in buf[:min(n.value, max_labels)]}


# ------------------------------------------------------------------ host views
def matches_numpy(t) -> np.ndarray:
    return t.cpu().numpy().reshape(-1).view(MATCH_DTYPE)


def codes_numpy(codes, n_codes) -> np.ndarray:
    n = int(n_codes.item()) if hasattr(n_codes, "item") else int(n_codes)
    n = min(n, codes.shape[0])
    return codes[:n].cpu().numpy().reshape(-1).view(CODE_DTYPE)


def stats_numpy(stats) -> np.ndarray:
    return stats.cpu().numpy().reshape(-1).view(STATS_DTYPE)
