"""Python binding of libkripke.so (argument marshalling only).

Every function named kripke_* forwards to the C entry point of the same name
(include/kripke.h).  PyTorch supplies device memory and streams; all
evaluation runs in the library's HIP kernels.  There is no CPU fallback: if
the library is missing the first call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkripke.so")

KRIPKE_K, KRIPKE_T, KRIPKE_S4, KRIPKE_S5 = 0, 1, 2, 3
CLASS_NAMES = ("K", "T", "S4", "S5")
KRIPKE_COUNT, KRIPKE_DECIDE = 0, 1
KRIPKE_PLAN_PLAIN = 0x10
NO_KEY = (1 << 64) - 1

_lib = None


class KripkeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"kripke status {status}: {msg}")
        self.status = status


def lib():
    """Load libkripke.so (built by __graft_entry__.build() or paper_2606_15437_amd/build.py)."""
    global _lib
    if _lib is None:
        # PyTorch brings its own HIP runtime; loading it first lets this library bind to
        # the same runtime instead of starting a second one that may not see the device
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g;"
                               " g.build()'` first")
        L = C.CDLL(LIB_PATH)
        u8p, u32p, u64p, vp = (C.POINTER(C.c_uint8), C.POINTER(C.c_uint32),
                               C.POINTER(C.c_uint64), C.c_void_p)
        u32, u64 = C.c_uint32, C.c_uint64
        sig = {
            "kripke_census": [u8p, u32p, u32, u32, u32, u32, vp, vp],
            "kripke_census_range": [u8p, u32p, u32, u32, u32, u32, u64, u64, u32, vp, vp],
            "kripke_census_range_static": [u8p, u32p, u32, u32, u32, u32, u64, u64, u32, vp,
                                           vp],
            "kripke_split": [u8p, u32, u8p, u32, vp, u64, u32, u32, vp, vp],
            "kripke_frame_validity": [u8p, u32p, u32, u32, u32, vp, vp],
            "kripke_split_batch": [u8p, u32p, u32, vp, u64, u32, u32, vp, vp],
            "kripke_plan_create": [u8p, u32p, u32, u32, u32, u32, C.c_char_p, C.POINTER(vp)],
            "kripke_plan_launch": [vp, vp, vp],
            "kripke_plan_destroy": [vp],
            "kripke_version": [],
            "kripke_program_stats": [u8p, u32p, u32, u32, C.POINTER(C.c_int32)],
            "kripke_calibrate_int32": [C.POINTER(C.c_double), vp],
            "kripke_signatures": [u8p, u32p, u32, u32, u64p, u32, vp, vp],
            "kripke_knn_pairs": [vp, u32, u32, u32, vp, vp, vp],
            "kripke_pair_hamming": [vp, u32, vp, u64, vp, vp],
            "kripke_select_top": [vp, u64, u64, vp, vp],
            "kripke_mlp_create": [u64, u32, C.POINTER(vp)],
            "kripke_mlp_destroy": [vp],
            "kripke_mlp_get_params": [vp, C.POINTER(C.c_float)],
            "kripke_mlp_set_params": [vp, C.POINTER(C.c_float)],
            "kripke_mlp_get_grads": [vp, C.POINTER(C.c_float)],
            "kripke_mlp_forward": [vp, vp, u32, vp, u64, vp, vp],
            "kripke_mlp_gradients": [vp, vp, u32, vp, vp, u32, C.c_float, vp, vp],
            "kripke_mlp_adam_step": [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.kripke_last_error.argtypes = []
        L.kripke_last_error.restype = C.c_char_p
        L.kripke_key_decode.argtypes = [u64, u32, u32, u64p, u64p, u32p]
        L.kripke_key_decode.restype = None
        L.kripke_frame_decode.argtypes = [u64, u32, u32p]
        L.kripke_frame_decode.restype = None
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise KripkeError(rc, lib().kripke_last_error().decode())


def _host_u8(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint8))
    return a, a.ctypes.data_as(C.POINTER(C.c_uint8))


def _host_u32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return a, a.ctypes.data_as(C.POINTER(C.c_uint32))


def _ptr(t) -> int:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device buffers must be contiguous CUDA tensors")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


# ------------------------------------------------------------ C entry points
def kripke_census(code, offsets, n, cls, nvars, d_out, stream=None):
    """d_out: CUDA int64 tensor [B, 2] (first_key, fail_count), overwritten."""
    c, cp = _host_u8(code)
    o, op = _host_u32(offsets)
    _check(lib().kripke_census(cp, op, len(o) - 1, n, cls, nvars, _ptr(d_out), _stream(stream)))


def kripke_census_range(code, offsets, n, cls, nvars, frame_begin, frame_end, flags, d_out,
                        stream=None):
    c, cp = _host_u8(code)
    o, op = _host_u32(offsets)
    _check(lib().kripke_census_range(cp, op, len(o) - 1, n, cls, nvars, frame_begin, frame_end,
                                     flags, _ptr(d_out), _stream(stream)))


def kripke_census_range_static(code, offsets, n, cls, nvars, frame_begin, frame_end, flags,
                               d_out, stream=None):
    """kripke_census_range without device allocation (fixed static scratch; K and T)."""
    c, cp = _host_u8(code)
    o, op = _host_u32(offsets)
    _check(lib().kripke_census_range_static(cp, op, len(o) - 1, n, cls, nvars, frame_begin,
                                            frame_end, flags, _ptr(d_out), _stream(stream)))


def kripke_frame_validity(code, offsets, n, nvars, d_bits, stream=None):
    """d_bits: CUDA int32 tensor [B, ceil(2^(n*n) / 32)], overwritten with validity maps."""
    c, cp = _host_u8(code)
    o, op = _host_u32(offsets)
    _check(lib().kripke_frame_validity(cp, op, len(o) - 1, n, nvars, _ptr(d_bits),
                                       _stream(stream)))


def kripke_split(phi, psi, d_frames, n, nvars, d_first_key, stream=None):
    a, ap = _host_u8(phi)
    b, bp = _host_u8(psi)
    nframes = d_frames.shape[0] if d_frames is not None else 0
    _check(lib().kripke_split(ap, len(a), bp, len(b), _ptr(d_frames), nframes, n, nvars,
                              _ptr(d_first_key), _stream(stream)))


def kripke_split_batch(code, offsets, d_frames, n, nvars, d_first_key, stream=None):
    c, cp = _host_u8(code)
    o, op = _host_u32(offsets)
    nframes = d_frames.shape[0] if d_frames is not None else 0
    _check(lib().kripke_split_batch(cp, op, (len(o) - 1) // 2, _ptr(d_frames), nframes, n, nvars,
                                    _ptr(d_first_key), _stream(stream)))


def kripke_plan_create(code, offsets, n, class_mask, nvars, tune_cache=None):
    c, cp = _host_u8(code)
    o, op = _host_u32(offsets)
    plan = C.c_void_p()
    tc = tune_cache.encode() if tune_cache else None
    _check(lib().kripke_plan_create(cp, op, len(o) - 1, n, class_mask, nvars, tc, C.byref(plan)))
    return plan


def kripke_plan_launch(plan, d_out, stream=None):
    _check(lib().kripke_plan_launch(plan, _ptr(d_out), _stream(stream)))


def kripke_plan_destroy(plan):
    _check(lib().kripke_plan_destroy(plan))


def kripke_key_decode(key, n, nvars):
    if key == NO_KEY:
        return None
    f, v, w = C.c_uint64(), C.c_uint64(), C.c_uint32()
    lib().kripke_key_decode(key, n, nvars, C.byref(f), C.byref(v), C.byref(w))
    return f.value, v.value, w.value


def kripke_frame_decode(frame, n):
    out = (C.c_uint32 * n)()
    lib().kripke_frame_decode(frame, n, out)
    return list(out)


def kripke_version():
    return lib().kripke_version()


def kripke_program_stats(code, offsets, nvars):
    """int32[B][6]: modal, binary, loads, saves, stack slots, constant (-1/0/1) per compiled
    program (host-only)."""
    c, cp = _host_u8(code)
    o, op = _host_u32(offsets)
    out = np.zeros((len(o) - 1, 6), dtype=np.int32)
    _check(lib().kripke_program_stats(cp, op, len(o) - 1, nvars,
                                      out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def kripke_calibrate_int32(stream=None):
    """Measured plain 32-bit bitwise VALU rate of the device, lane-operations per second."""
    r = C.c_double()
    _check(lib().kripke_calibrate_int32(C.byref(r), _stream(stream)))
    return r.value


MLP_PARAMS = 4326401
MLP_SHAPES = (("W1", (512, 8192)), ("b1", (512,)), ("W2", (256, 512)), ("b2", (256,)),
              ("w3", (256,)), ("b3", (1,)))


def kripke_signatures(code, offsets, nvars, samples, d_sig, stream=None):
    """d_sig: CUDA int64 tensor [B][nsamples/64]; samples: host uint64 packed models."""
    c, cp = _host_u8(code)
    o, op = _host_u32(offsets)
    smp = np.ascontiguousarray(np.asarray(samples, dtype=np.uint64))
    _check(lib().kripke_signatures(cp, op, len(o) - 1, nvars,
                                   smp.ctypes.data_as(C.POINTER(C.c_uint64)), len(smp),
                                   _ptr(d_sig), _stream(stream)))


def kripke_knn_pairs(d_sig, k, d_pairs, d_npairs, stream=None):
    nf, words = d_sig.shape
    _check(lib().kripke_knn_pairs(_ptr(d_sig), nf, words, k, _ptr(d_pairs), _ptr(d_npairs),
                                  _stream(stream)))


def kripke_pair_hamming(d_sig, d_pairs, npairs, d_dist, stream=None):
    _check(lib().kripke_pair_hamming(_ptr(d_sig), d_sig.shape[1], _ptr(d_pairs), npairs,
                                     _ptr(d_dist), _stream(stream)))


def kripke_select_top(d_scores, budget, d_idx, stream=None):
    _check(lib().kripke_select_top(_ptr(d_scores), d_scores.numel(), budget, _ptr(d_idx),
                                   _stream(stream)))


def kripke_mlp_create(seed, max_batch):
    h = C.c_void_p()
    _check(lib().kripke_mlp_create(seed, max_batch, C.byref(h)))
    return h


def kripke_mlp_destroy(h):
    _check(lib().kripke_mlp_destroy(h))


def _fbuf(n):
    a = np.zeros(n, dtype=np.float32)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def kripke_mlp_get_params(h):
    a, p = _fbuf(MLP_PARAMS)
    _check(lib().kripke_mlp_get_params(h, p))
    return a


def kripke_mlp_set_params(h, params):
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    assert a.size == MLP_PARAMS
    _check(lib().kripke_mlp_set_params(h, a.ctypes.data_as(C.POINTER(C.c_float))))


def kripke_mlp_get_grads(h):
    a, p = _fbuf(MLP_PARAMS)
    _check(lib().kripke_mlp_get_grads(h, p))
    return a


def kripke_mlp_forward(h, d_sig, d_pairs, d_logits, stream=None):
    _check(lib().kripke_mlp_forward(h, _ptr(d_sig), d_sig.shape[1], _ptr(d_pairs), d_pairs.numel(),
                                    _ptr(d_logits), _stream(stream)))


def kripke_mlp_gradients(h, d_sig, d_pairs, d_labels, pos_weight, d_loss, stream=None):
    _check(lib().kripke_mlp_gradients(h, _ptr(d_sig), d_sig.shape[1], _ptr(d_pairs), _ptr(d_labels),
                                      d_pairs.numel(), pos_weight, _ptr(d_loss), _stream(stream)))


def kripke_mlp_adam_step(h, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().kripke_mlp_adam_step(h, lr, beta1, beta2, eps, _stream(stream)))


def split_params(flat):
    """Named views of the flat FP32 parameter (or gradient) vector."""
    out, at = {}, 0
    for name, shape in MLP_SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[at:at + n].reshape(shape)
        at += n
    return out


# ---------------------------------------------------------------- helpers
def as_u64(t) -> np.ndarray:
    """Host uint64 view of a CUDA int64 tensor."""
    return t.detach().cpu().numpy().view(np.uint64)


def census(formulas, n, cls=KRIPKE_K, nvars=2, frame_begin=None, frame_end=None, decide=False,
           device="cuda"):
    """Census of a list of postfix programs; returns (first_keys, fail_counts) as uint64 arrays."""
    import torch
    from .inputs import pack
    code, offs = pack(formulas)
    out = torch.empty((len(formulas), 2), dtype=torch.int64, device=device)
    if frame_begin is None and frame_end is None and not decide and n <= 5:
        kripke_census(code, offs, n, cls, nvars, out)
    else:
        fb = 0 if frame_begin is None else frame_begin
        fe = (1 << (n * n)) if frame_end is None else frame_end
        kripke_census_range(code, offs, n, cls, nvars, fb, fe,
                            KRIPKE_DECIDE if decide else KRIPKE_COUNT, out)
    torch.cuda.synchronize()
    r = as_u64(out)
    return r[:, 0].copy(), r[:, 1].copy()


def split(pairs, frames, n, nvars=2, device="cuda"):
    """First separating key per (phi, psi) pair over a uint32[nframes][n] frame list."""
    import torch
    from .inputs import pack
    progs = [p for pair in pairs for p in pair]
    code, offs = pack(progs)
    d_frames = torch.as_tensor(np.ascontiguousarray(frames, dtype=np.uint32).view(np.int32),
                               device=device)
    out = torch.empty(len(pairs), dtype=torch.int64, device=device)
    kripke_split_batch(code, offs, d_frames, n, nvars, out)
    torch.cuda.synchronize()
    return as_u64(out).copy()
