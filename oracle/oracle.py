"""ctypes wrapper over the plain-C oracle (test infrastructure only).

Every function here forwards to oracle/kripke_oracle.c, which evaluates the
recursive Kripke satisfaction definition (Section 2) over explicit boolean
arrays.  Keys are packed as frame << (nvars*n + 4) | valuation << 4 | world.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CLASS_K, CLASS_T, CLASS_S4, CLASS_S5, CLASS_K4 = 0, 1, 2, 3, 4
NONE = (1 << 64) - 1


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        u8p, u32p, u64p = C.POINTER(C.c_uint8), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
        L.orc_census.restype = C.c_int
        L.orc_census.argtypes = [u8p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                 C.c_uint64, C.c_uint64, C.c_int, C.c_int, u64p, u64p]
        L.orc_class_size.restype = C.c_int64
        L.orc_class_size.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_in_class.restype = C.c_int
        L.orc_in_class.argtypes = [u32p, C.c_uint32, C.c_uint32]
        L.orc_truth_set.restype = C.c_int
        L.orc_truth_set.argtypes = [u8p, C.c_uint32, C.c_uint32, u32p, C.c_uint32, C.c_uint64, u8p]
        L.orc_sat_at.restype = C.c_int
        L.orc_sat_at.argtypes = [u8p, C.c_uint32, C.c_uint32, u32p, C.c_uint32, C.c_uint64,
                                 C.c_uint32]
        L.orc_check_certificate.restype = C.c_int
        L.orc_check_certificate.argtypes = [u8p, C.c_uint32, C.c_uint32, u32p, C.c_uint32,
                                            C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_split.restype = C.c_int
        L.orc_split.argtypes = [u8p, C.c_uint32, u8p, C.c_uint32, u32p, C.c_uint64, C.c_uint32,
                                C.c_uint32, u64p]
        L.orc_signatures.restype = C.c_int
        L.orc_signatures.argtypes = [u8p, u32p, C.c_uint32, C.c_uint32, u64p, C.c_uint32, u64p]
        L.orc_hardware_threads.restype = C.c_int
        _lib = L
    return _lib


def _u8(code):
    a = np.ascontiguousarray(np.asarray(code, dtype=np.uint8))
    return a, a.ctypes.data_as(C.POINTER(C.c_uint8))


def _u32(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint32))
    return a, a.ctypes.data_as(C.POINTER(C.c_uint32))


def census(code, n, cls=CLASS_K, nvars=2, frame_begin=0, frame_end=None, stop_at_first=False,
           threads=1):
    """(first_key, fail_count, threads_used) of one formula over a frame range of the class."""
    if frame_end is None:
        frame_end = 1 << (n * n)
    a, p = _u8(code)
    key, cnt = C.c_uint64(), C.c_uint64()
    rc = lib().orc_census(p, len(a), n, cls, nvars, frame_begin, frame_end, int(stop_at_first),
                          threads, C.byref(key), C.byref(cnt))
    if rc < 0:
        raise ValueError(f"oracle census rejected input (status {rc})")
    return key.value, cnt.value, rc


def class_size(n, cls):
    return lib().orc_class_size(n, cls)


def in_class(succ, cls):
    a, p = _u32(succ)
    return bool(lib().orc_in_class(p, len(a), cls))


def truth_set(code, succ, nvars, val):
    a, p = _u8(code)
    s, sp = _u32(succ)
    out = np.zeros(len(s), dtype=np.uint8)
    rc = lib().orc_truth_set(p, len(a), len(s), sp, nvars, val,
                             out.ctypes.data_as(C.POINTER(C.c_uint8)))
    if rc < 0:
        raise ValueError(f"oracle rejected input (status {rc})")
    return [int(x) for x in out]


def sat_at(code, succ, nvars, val, world):
    a, p = _u8(code)
    s, sp = _u32(succ)
    rc = lib().orc_sat_at(p, len(a), len(s), sp, nvars, val, world)
    if rc < 0:
        raise ValueError(f"oracle rejected input (status {rc})")
    return bool(rc)


def check_certificate(code, succ, nvars, val, world, cls=CLASS_K):
    a, p = _u8(code)
    s, sp = _u32(succ)
    rc = lib().orc_check_certificate(p, len(a), len(s), sp, nvars, val, world, cls)
    if rc < 0:
        raise ValueError(f"oracle rejected input (status {rc})")
    return bool(rc)


def split(phi, psi, frames, nvars=2):
    """First (position, valuation, world) key where phi and psi differ on the frame list."""
    fr = np.ascontiguousarray(np.asarray(frames, dtype=np.uint32))
    nframes, n = fr.shape
    a, pa = _u8(phi)
    b, pb = _u8(psi)
    key = C.c_uint64()
    rc = lib().orc_split(pa, len(a), pb, len(b), fr.ctypes.data_as(C.POINTER(C.c_uint32)),
                         nframes, n, nvars, C.byref(key))
    if rc < 0:
        raise ValueError(f"oracle split rejected input (status {rc})")
    return key.value


def signatures(formulas, samples, nvars=2):
    """uint64[len(formulas)][ceil(len(samples)/64)] truth bits at pointed models."""
    from paper_2606_15437_amd.inputs import pack
    code, offs = pack(formulas)
    a, pa = _u8(code)
    o, po = _u32(offs)
    smp = np.ascontiguousarray(np.asarray(samples, dtype=np.uint64))
    words = (len(smp) + 63) // 64
    sig = np.zeros((len(formulas), words), dtype=np.uint64)
    rc = lib().orc_signatures(pa, po, len(formulas), nvars,
                              smp.ctypes.data_as(C.POINTER(C.c_uint64)), len(smp),
                              sig.ctypes.data_as(C.POINTER(C.c_uint64)))
    if rc < 0:
        raise ValueError(f"oracle signatures rejected input (status {rc})")
    return sig


def decode_key(key, n, nvars):
    """(frame, valuation, world) from a packed key."""
    if key == NONE:
        return None
    sh = nvars * n + 4
    return key >> sh, (key >> 4) & ((1 << (nvars * n)) - 1), key & 15


def hardware_threads():
    return lib().orc_hardware_threads()
