"""Host-side checks of libgc that need no GPU: the library loads and exports
every symbol include/gc.h declares, its host encoder writes streams
byte-identical to the oracle's, argument validation, and the batch encoder."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1502_01916_amd import gc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "gc.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = gc.lib()
    names = header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert gc.version().startswith("libgc")


VARIANTS = [
    (O.SIMPLE, {}), (O.SCHEME, dict(cg=1, ld=O.LD_CU)), (O.SCHEME, dict(cg=2, ld=O.LD_CU)),
    (O.SCHEME, dict(cg=4, ld=O.LD_CU)), (O.SCHEME, dict(cg=8, ld=O.LD_CU)),
    (O.SCHEME, dict(cg=4, ld=O.LD_IU)), (O.SCHEME, dict(cg=8, ld=O.LD_IU)),
    (O.SCHEME, dict(cg=1, ld=O.LD_BINARY)), (O.SCHEME, dict(cg=2, ld=O.LD_BINARY)),
    (O.SCHEME, dict(cg=4, ld=O.LD_BINARY)), (O.SCHEME, dict(cg=8, ld=O.LD_BINARY)),
    (O.AFOR, {}), (O.PFD, {}), (O.PFD, dict(pfd_pos=O.PFD_BITMAP)), (O.PFD, dict(zeta=(1, 32))),
    (O.PFD, dict(zeta=(3, 10))), (O.VSE, {}),
]


def both_params(codec, k, delta, kw):
    op = O.params(codec, k=k, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU), delta=delta,
                  pfd_pos=kw.get("pfd_pos", 0), zeta=kw.get("zeta", (1, 10)))
    gp = gc.params(k=k, cg=kw.get("cg", 1), ld=kw.get("ld", gc.LD_CU), pfd_pos=kw.get("pfd_pos", 0),
                   zeta=kw.get("zeta", (1, 10)), delta=delta)
    return op, gp


def inputs(rng, n):
    yield np.sort(rng.choice(1 << 27, n, replace=False)).astype(np.uint32), True
    yield (rng.integers(0, 1 << 32, n, dtype=np.uint64)
           >> rng.integers(0, 33, n).astype(np.uint64)).astype(np.uint32), False
    x = rng.geometric(0.3, n).astype(np.uint32)
    if n:
        x[rng.integers(0, n, max(1, n // 30))] = 1 << 21
    yield x, False


@pytest.mark.parametrize("k", [4, 8, 64])
@pytest.mark.parametrize("vi", range(len(VARIANTS)))
def test_host_encoder_is_byte_identical_to_oracle(vi, k):
    codec, kw = VARIANTS[vi]
    rng = np.random.default_rng(300 + vi)
    for n in (0, 1, 3, 4, 5, 127, 128, 129, 1000, 4099):
        for x, delta in inputs(rng, n):
            op, gp = both_params(codec, k, delta, kw)
            a = gc.encode(x, codec, gp)
            b = O.encode(x, op)
            assert a.size == b.size and np.array_equal(a, b), (n, delta)


def test_encode_lists_matches_single_encodes():
    rng = np.random.default_rng(7)
    lengths = rng.integers(0, 3000, 60)
    flat = np.concatenate([np.sort(rng.choice(1 << 25, int(L), replace=False)).astype(np.uint32)
                           for L in lengths])
    codecs = rng.integers(0, 4, lengths.size)
    plist = [gc.params(k=4, cg=8, ld=gc.LD_IU, delta=True) if c == 1 else gc.params(delta=True)
             for c in codecs]
    s, offs = gc.encode_lists(flat, lengths, codecs, plist, nthreads=4)
    lo = np.concatenate([[0], np.cumsum(lengths)])
    for i in range(lengths.size):
        ref = gc.encode(flat[lo[i]:lo[i + 1]], int(codecs[i]), plist[i])
        assert np.array_equal(s[int(offs[i]):int(offs[i + 1])], ref)
        assert int(offs[i]) % 4 == 0


def test_encode_rejects_bad_parameters():
    x = np.arange(100, dtype=np.uint32)
    for codec, p in [(gc.SCHEME, gc.params(cg=3)), (gc.SCHEME, gc.params(cg=2, ld=gc.LD_IU)),
                     (gc.PFD, gc.params(zeta=(0, 10))), (gc.PFD, gc.params(zeta=(10, 10))),
                     (gc.SIMPLE, gc.params(k=6)), (gc.SIMPLE, gc.params(k=128)), (7, gc.params()),
                     (5, gc.params())]:
        with pytest.raises(gc.GcError) as e:
            gc.encode(x, codec, p)
        assert e.value.code == gc.EINVAL


def test_encode_reports_small_capacity():
    L = gc.lib()
    x = np.arange(1000, dtype=np.uint32)
    out = np.zeros(8, np.uint32)
    w = ctypes.c_size_t()
    p = gc.params()
    rc = L.gc_encode(x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), x.size, gc.SIMPLE,
                     ctypes.byref(p), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), out.size,
                     ctypes.byref(w))
    assert rc == gc.ENOSPC


def test_device_entry_points_validate_arguments_without_touching_a_gpu():
    L = gc.lib()
    assert L.gc_decode(None, None, 0, None, None, None) == gc.EINVAL
    assert L.gc_decode_noalloc(None, None, 0, None, None, None) == gc.EINVAL
    assert L.gc_plan_destroy(None) == gc.EINVAL
    assert L.gc_decode_batch(None, None, None, None) == gc.EINVAL
    assert L.gc_sync_status(None, None, None) == gc.EINVAL
    assert L.gc_ctx_destroy(None) == gc.EINVAL
