"""gc_decode_noalloc (the single-list decode on the library's fixed device
scratch) against gc_decode, through the C ABI: two calls in a row, the
second with a smaller list, for every codec class, element by element; a
list above the fixed scratch's limit is refused."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1502_01916_amd import gc

pytestmark = pytest.mark.gpu

CODECS = [(O.SIMPLE, {}), (O.SCHEME, dict(cg=1, ld=O.LD_CU)), (O.SCHEME, dict(cg=8, ld=O.LD_IU)),
          (O.SCHEME, dict(cg=2, ld=O.LD_BINARY)), (O.AFOR, {}), (O.PFD, {}),
          (O.PFD, dict(pfd_pos=O.PFD_BITMAP, k=64))]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return torch


def run(torch, ctx, fn, s, n):
    d_s = gc.to_device(s)
    d_o = torch.full((n + 64,), -1, dtype=torch.int32, device="cuda")
    fn(d_s, s.size, s[:4], d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, (rc, det)
    out = gc.to_host(d_o)
    assert np.all(out[n:] == 0xFFFFFFFF), "write past the end of the output"
    return out[:n]


def test_noalloc_matches_gc_decode_twice(torch_cuda):
    """Per codec: a multi-tile list (docIDs prefix-summed, or TFs), then a
    smaller one, each decoded by gc_decode_noalloc and by gc_decode."""
    torch = torch_cuda
    rng = np.random.default_rng(4242)
    ctx = gc.Context(0)
    try:
        for ci, (codec, kw) in enumerate(CODECS):
            for n, delta in ((700001 + 1111 * ci, True), (9000 + 37 * ci, ci % 2 == 0)):
                if delta:
                    x = np.sort(rng.choice(1 << 30, n, replace=False)).astype(np.uint32)
                else:
                    x = rng.geometric(0.3, n).astype(np.uint32)
                s = O.encode(x, O.params(codec, delta=delta, **kw))
                say("noalloc", codec, kw, n, delta)
                got = run(torch, ctx, ctx.decode_noalloc, s, n)
                ref = run(torch, ctx, ctx.decode, s, n)
                assert np.array_equal(got, ref), (codec, kw, n)
                assert np.array_equal(got, x), (codec, kw, n)
    finally:
        ctx.close()


def test_noalloc_limit(torch_cuda):
    """A list of 2^22 + 1 integers is refused with GC_ENOSPC before any
    launch; one of 2^22 decodes exactly."""
    torch = torch_cuda
    ctx = gc.Context(0)
    try:
        for n, ok in (((1 << 22) + 1, False), (1 << 22, True)):
            x = np.arange(n, dtype=np.uint32) * 3
            s = gc.encode(x, gc.SIMPLE, gc.params(delta=True))
            d_s = gc.to_device(s)
            d_o = torch.full((n + 64,), -1, dtype=torch.int32, device="cuda")
            rc = gc.lib().gc_decode_noalloc(ctx._h, gc._ptr(d_s), int(s.size), gc._u32(np.ascontiguousarray(s[:4])),
                                            gc._ptr(d_o), None)
            say("noalloc limit", n, rc)
            if ok:
                assert rc == gc.OK
                rc2, det = ctx.sync_status()
                assert rc2 == gc.OK, det
                assert np.array_equal(gc.to_host(d_o)[:n], x)
            else:
                assert rc == gc.ENOSPC
    finally:
        ctx.close()
