"""Plain CPU oracle for the Group codecs -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never links, loads
or calls it, and it shares no code with the HIP implementation.

The codecs live in plain C (``gc_oracle.c``, bit-at-a-time, written from the
paper's sections); this module compiles that file with gcc on first use and
wraps it with ctypes.  The learned-selector reference (``mlp_ref``) is numpy in
float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "gc_oracle.c")]
_lock = threading.Lock()
_lib = None

SIMPLE, SCHEME, AFOR, PFD, VSE = 0, 1, 2, 3, 4
LD_BINARY, LD_CU, LD_IU = 0, 1, 2
PFD_LINKED, PFD_BITMAP = 0, 1
OK, EINVAL, ENOSPC, ECORRUPT = 0, -1, -2, -3


class Params(ctypes.Structure):
    _fields_ = [("codec", ctypes.c_int), ("k", ctypes.c_int), ("cg", ctypes.c_int),
                ("ld", ctypes.c_int), ("delta", ctypes.c_int), ("pfd_pos", ctypes.c_int),
                ("zeta_num", ctypes.c_int), ("zeta_den", ctypes.c_int)]


def build(force: bool = False) -> str:
    """Compiles liboracle.so with gcc (plain C99, -O2)."""
    srcs = [s for s in _SRCS if os.path.exists(s)]
    if not force and os.path.exists(_SO):
        so_t = os.path.getmtime(_SO)
        if all(os.path.getmtime(s) <= so_t for s in srcs + [os.path.join(_HERE, "gc_oracle.h")]):
            return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-Wall", "-fPIC", "-shared", *srcs,
                           "-o", tmp])
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_SO)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            u8p = ctypes.POINTER(ctypes.c_uint8)
            sz = ctypes.c_size_t
            L.or_bw.argtypes = [ctypes.c_uint32]
            L.or_bw.restype = ctypes.c_int
            L.or_tuple_max.argtypes = [u32p, sz, ctypes.c_int, u32p]
            L.or_dgap.argtypes = [u32p, sz, u32p]
            L.or_prefix_sum.argtypes = [u32p, sz, u32p]
            L.or_gsim_table.argtypes = [ctypes.POINTER(ctypes.c_int)] * 2
            L.or_gsim_select.argtypes = [u32p, sz, u8p]
            L.or_gsim_select.restype = sz
            L.or_parse_header.argtypes = [ctypes.c_uint32, ctypes.POINTER(Params)]
            L.or_gsc_units.argtypes = [ctypes.c_uint32, ctypes.c_int]
            L.or_afor_partition.argtypes = [u32p, sz, ctypes.c_int, u8p]
            L.or_afor_partition.restype = sz
            L.or_vse_partition.argtypes = [u32p, sz, ctypes.c_int, u8p]
            L.or_vse_partition.restype = sz
            L.or_pfd_width.argtypes = [u32p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
            L.or_encode.argtypes = [u32p, sz, ctypes.POINTER(Params), u32p, sz]
            L.or_encode.restype = ctypes.c_long
            L.or_gsim_encode_with.argtypes = [u32p, sz, ctypes.POINTER(Params), u8p, sz, u32p, sz]
            L.or_gsim_encode_with.restype = ctypes.c_long
            L.or_afor_encode_with.argtypes = [u32p, sz, ctypes.POINTER(Params), u8p, sz, u32p, sz]
            L.or_afor_encode_with.restype = ctypes.c_long
            L.or_decode.argtypes = [u32p, sz, u32p, sz]
            L.or_decode.restype = ctypes.c_long
            _bind_blocks(L)
            _lib = L
    return _lib


def _bind_blocks(L):
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    sz = ctypes.c_size_t
    L.or_block_class_params.argtypes = [ctypes.c_int, ctypes.POINTER(Params)]
    L.or_block_encode.argtypes = [u32p, ctypes.c_int, u32p, sz, u32p]
    L.or_block_encode.restype = ctypes.c_long
    L.or_block_size.argtypes = [u32p, ctypes.c_int]
    L.or_block_size.restype = ctypes.c_long
    L.or_block_best.argtypes = [u32p, ctypes.POINTER(ctypes.c_long)]
    L.or_block_decode.argtypes = [ctypes.c_uint32, u32p, sz, u32p]
    L.or_block_features.argtypes = [u32p, ctypes.POINTER(ctypes.c_double)]
    L.or_blockmix_encode.argtypes = [u32p, sz, u8p, u32p, sz, u8p]
    L.or_blockmix_encode.restype = ctypes.c_long
    L.or_blockmix_decode.argtypes = [u32p, sz, u32p, sz]
    L.or_blockmix_decode.restype = ctypes.c_long


def _u32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def params(codec, k=4, cg=1, ld=LD_CU, delta=False, pfd_pos=PFD_LINKED, zeta=(1, 10)):
    return Params(int(codec), int(k), int(cg), int(ld), int(bool(delta)), int(pfd_pos),
                  int(zeta[0]), int(zeta[1]))


def bw(x: int) -> int:
    return lib().or_bw(ctypes.c_uint32(int(x) & 0xFFFFFFFF))


def tuple_max(x, k=4):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    T = x.size // k
    out = np.zeros(T, np.uint32)
    lib().or_tuple_max(_u32(x), T, k, _u32(out))
    return out


def dgap(d):
    d = np.ascontiguousarray(d, dtype=np.uint32)
    g = np.zeros_like(d)
    lib().or_dgap(_u32(d), d.size, _u32(g))
    return g


def prefix_sum(g):
    g = np.ascontiguousarray(g, dtype=np.uint32)
    d = np.zeros_like(g)
    lib().or_prefix_sum(_u32(g), g.size, _u32(d))
    return d


def gsim_table():
    num = (ctypes.c_int * 10)()
    bwt = (ctypes.c_int * 10)()
    lib().or_gsim_table(num, bwt)
    return list(num), list(bwt)


def gsim_select(qmax):
    q = np.ascontiguousarray(qmax, dtype=np.uint32)
    sel = np.zeros(max(q.size, 1), np.uint8)
    S = lib().or_gsim_select(_u32(q), q.size, _u8(sel))
    return sel[:S].copy()


def gsc_units(qmax: int, cg: int) -> int:
    return lib().or_gsc_units(ctypes.c_uint32(int(qmax)), cg)


def afor_partition(qmax, k=4):
    q = np.ascontiguousarray(qmax, dtype=np.uint32)
    F = np.zeros(q.size // 8 + 1, np.uint8)
    nf = lib().or_afor_partition(_u32(q), q.size, k, _u8(F))
    return [int(f) for f in F[:nf]]


def vse_partition(qmax, k=4):
    q = np.ascontiguousarray(qmax, dtype=np.uint32)
    F = np.zeros(q.size // 8 + 1, np.uint8)
    nf = lib().or_vse_partition(_u32(q), q.size, k, _u8(F))
    return [int(f) for f in F[:nf]]


def pfd_width(qmax, zeta=(1, 10)):
    q = np.ascontiguousarray(qmax, dtype=np.uint32)
    return lib().or_pfd_width(_u32(q), q.size, zeta[0], zeta[1])


def _cap(n, k):
    T = (n + k - 1) // k + 64
    return 64 + 4 * T * k + 8 * T + 4 * (T // 32 + 1) * (k + 2)


def encode(x, p: Params):
    """Encodes a uint32 list into one self-describing stream (uint32 words)."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    cap = _cap(x.size, p.k)
    out = np.zeros(cap, np.uint32)
    r = lib().or_encode(_u32(x), x.size, ctypes.byref(p), _u32(out), cap)
    if r < 0:
        raise ValueError("oracle encode failed: %d" % r)
    return out[:r].copy()


def gsim_encode_with(x, sel, p: Params):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    s = np.ascontiguousarray(sel, dtype=np.uint8)
    cap = _cap(x.size, p.k) + 8 * s.size
    out = np.zeros(cap, np.uint32)
    r = lib().or_gsim_encode_with(_u32(x), x.size, ctypes.byref(p), _u8(s), s.size,
                                  _u32(out), cap)
    if r < 0:
        raise ValueError("invalid selector sequence: %d" % r)
    return out[:r].copy()


def afor_encode_with(x, frames, p: Params):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    F = np.ascontiguousarray(frames, dtype=np.uint8)
    cap = _cap(x.size, p.k) + 8 * F.size
    out = np.zeros(cap, np.uint32)
    r = lib().or_afor_encode_with(_u32(x), x.size, ctypes.byref(p), _u8(F), F.size,
                                  _u32(out), cap)
    if r < 0:
        raise ValueError("invalid partition: %d" % r)
    return out[:r].copy()


def decode(stream, cap=None):
    """Decodes one stream; returns the uint32 list or raises on corruption."""
    s = np.ascontiguousarray(stream, dtype=np.uint32)
    if cap is None:
        cap = int(s[1]) if s.size >= 2 else 0
    out = np.zeros(max(cap, 1), np.uint32)
    r = lib().or_decode(_u32(s), s.size, _u32(out), cap)
    if r < 0:
        raise CorruptStream(r)
    return out[:r].copy()


def decode_status(stream):
    s = np.ascontiguousarray(stream, dtype=np.uint32)
    cap = int(s[1]) if s.size >= 2 else 0
    out = np.zeros(max(cap, 1), np.uint32)
    r = lib().or_decode(_u32(s), s.size, _u32(out), cap)
    return min(int(r), 0)


def parse_header(w0: int):
    p = Params()
    ok = lib().or_parse_header(ctypes.c_uint32(int(w0)), ctypes.byref(p))
    return p if ok else None


class CorruptStream(ValueError):
    pass


# ---------------------------------------------------------------------------
# Per-block container of the learned selector.

BLOCK_INTS = 128
NCLASS = 16


def block_class_params(kappa: int) -> Params:
    p = Params()
    if not lib().or_block_class_params(int(kappa), ctypes.byref(p)):
        raise ValueError(kappa)
    return p


def _block(x):
    x = np.ascontiguousarray(x, dtype=np.uint32)
    assert x.size == BLOCK_INTS
    return x


def block_encode(x, kappa: int):
    """(block word, payload words) of one 128-integer block coded with class kappa."""
    x = _block(x)
    buf = np.zeros(4 * BLOCK_INTS + 64, np.uint32)
    bw = ctypes.c_uint32()
    w = lib().or_block_encode(_u32(x), int(kappa), _u32(buf), buf.size, ctypes.byref(bw))
    if w <= 0:
        raise ValueError("block encode failed")
    return int(bw.value), buf[:w].copy()


def block_size(x, kappa: int) -> int:
    return int(lib().or_block_size(_u32(_block(x)), int(kappa)))


def block_best(x):
    """(exhaustive class, sizes of all classes in words)."""
    sizes = (ctypes.c_long * NCLASS)()
    best = lib().or_block_best(_u32(_block(x)), sizes)
    return int(best), np.array(sizes[:], dtype=np.int64)


def block_decode(blockword: int, payload):
    payload = np.ascontiguousarray(payload, dtype=np.uint32)
    out = np.zeros(BLOCK_INTS, np.uint32)
    rc = lib().or_block_decode(ctypes.c_uint32(int(blockword)), _u32(payload), payload.size, _u32(out))
    if rc != OK:
        raise CorruptStream(rc)
    return out


def block_features(x):
    f = (ctypes.c_double * 40)()
    lib().or_block_features(_u32(_block(x)), f)
    return np.array(f[:], dtype=np.float64)


def blockmix_encode(x, kappas=None):
    """(container words, classes used); kappas None = exhaustive choice."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    nb = (x.size + BLOCK_INTS - 1) // BLOCK_INTS
    cap = 4 + nb * (4 * BLOCK_INTS + 64) + 64
    out = np.zeros(cap, np.uint32)
    used = np.zeros(max(nb, 1), np.uint8)
    kp = None
    if kappas is not None:
        kappas = np.ascontiguousarray(kappas, dtype=np.uint8)
        assert kappas.size == nb
        kp = _u8(kappas)
    w = lib().or_blockmix_encode(_u32(x), x.size, kp, _u32(out), cap, _u8(used))
    if w < 0:
        raise ValueError("blockmix encode failed: %d" % w)
    return out[:w].copy(), used[:nb].copy()


def blockmix_decode(s):
    s = np.ascontiguousarray(s, dtype=np.uint32)
    n = int(s[1]) if s.size >= 2 else 0
    out = np.zeros(max(n, 1), np.uint32)
    r = lib().or_blockmix_decode(_u32(s), s.size, _u32(out), n)
    if r < 0:
        raise CorruptStream(r)
    return out[:n]
