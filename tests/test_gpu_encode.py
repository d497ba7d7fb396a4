"""GPU list encoders (gc_encode_lists_gpu) against the host encoder, whose
streams equal the oracle's (tests/test_capi_cpu.py): every codec variant at
several layout widths, lists of every length class (empty, ragged, one
chunk, many chunks), docID and TF-like values; then the full cfg2 lists of
the five benchmark codecs at k = 4 and 64.  Streams must be identical word
for word."""
import sys
import zlib

import numpy as np
import pytest

from paper_1502_01916_amd import gc, synth

pytestmark = pytest.mark.gpu

VARIANTS = [
    ("gsim", gc.SIMPLE, {}), ("gsc1cu", gc.SCHEME, dict(cg=1, ld=gc.LD_CU)),
    ("gsc2cu", gc.SCHEME, dict(cg=2, ld=gc.LD_CU)), ("gsc4cu", gc.SCHEME, dict(cg=4, ld=gc.LD_CU)),
    ("gsc8cu", gc.SCHEME, dict(cg=8, ld=gc.LD_CU)), ("gsc4iu", gc.SCHEME, dict(cg=4, ld=gc.LD_IU)),
    ("gsc8iu", gc.SCHEME, dict(cg=8, ld=gc.LD_IU)), ("gsc1b", gc.SCHEME, dict(cg=1, ld=gc.LD_BINARY)),
    ("gsc2b", gc.SCHEME, dict(cg=2, ld=gc.LD_BINARY)), ("gsc4b", gc.SCHEME, dict(cg=4, ld=gc.LD_BINARY)),
    ("gsc8b", gc.SCHEME, dict(cg=8, ld=gc.LD_BINARY)), ("afor", gc.AFOR, {}),
    ("pfd", gc.PFD, {}), ("pfdbitmap", gc.PFD, dict(pfd_pos=gc.PFD_BITMAP)),
    ("bp128", gc.PFD, dict(zeta=(1, 32))),
]

LENGTHS = [0, 1, 3, 4, 5, 31, 32, 33, 127, 128, 129, 1000, 8191, 8192, 8193, 70001, 0, 2]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return torch


def make_lists(rng, kind, lengths):
    out = []
    for n in lengths:
        if kind == "docids":
            out.append(np.sort(rng.choice(1 << 30, n, replace=False)).astype(np.uint32))
        elif kind == "spiky":
            x = rng.geometric(0.3, n).astype(np.uint32)
            m = max(1, n // 40) if n else 0
            if m:
                x[rng.integers(0, n, m)] = rng.integers(1 << 9, 1 << 31, m).astype(np.uint32)
            out.append(x)
        elif kind == "runs":
            # long runs of small values with sudden wide ones (exercises
            # Group-PFD's compulsory exceptions and long Group-Simple chains)
            x = np.ones(n, np.uint32)
            if n:
                x[rng.integers(0, n, max(1, n // 300))] = np.uint32(1 << 20)
            out.append(x)
        else:
            out.append((rng.integers(0, 1 << 32, n, dtype=np.uint64)
                        >> rng.integers(0, 33, n).astype(np.uint64)).astype(np.uint32))
    return out


def compare(torch, lists, codec, p):
    lengths = np.array([x.size for x in lists], np.int64)
    flat = np.concatenate(lists) if lists else np.zeros(0, np.uint32)
    want, woffs = gc.encode_lists(flat, lengths, codec, p)
    d_flat = gc.to_device(flat) if flat.size else torch.zeros(1, dtype=torch.int32, device="cuda")
    got_d, goffs = gc.encode_lists_gpu(d_flat, lengths, codec, p)
    torch.cuda.synchronize()
    assert np.array_equal(goffs, woffs), "stream offsets differ"
    got = gc.to_host(got_d)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        li = int(np.searchsorted(woffs, bad[0], side="right")) - 1
        pytest.fail("%d words differ, first at %d (list %d, n=%d, word %d of its stream): got %#x want %#x"
                    % (bad.size, bad[0], li, lengths[li], bad[0] - int(woffs[li]), got[bad[0]], want[bad[0]]))


@pytest.mark.parametrize("k", [4, 8, 64])
@pytest.mark.parametrize("name,codec,kw", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_gpu_encoder_matches_host(torch_cuda, name, codec, kw, k):
    rng = np.random.default_rng(zlib.crc32(name.encode()) + k)
    for kind, delta in (("docids", True), ("spiky", False), ("runs", False), ("widths", False)):
        lists = make_lists(rng, kind, LENGTHS)
        say(name, "k", k, kind)
        compare(torch_cuda, lists, codec, gc.params(k=k, delta=delta, **kw))


def test_gpu_encoder_long_lists(torch_cuda):
    """Lists of many chunks (2^20 and 300,001 integers): the chunk summaries
    and each list's walk over them."""
    rng = np.random.default_rng(99)
    lists = [np.sort(rng.choice(1 << 28, 1 << 20, replace=False)).astype(np.uint32),
             np.sort(rng.choice(1 << 26, 300001, replace=False)).astype(np.uint32)]
    for name, codec, kw in VARIANTS:
        for k in (4, 64):
            say("long", name, k)
            compare(torch_cuda, lists, codec, gc.params(k=k, delta=True, **kw))


def test_gpu_encoder_capacity(torch_cuda):
    """Too small an output: GC_ENOSPC, with the stream sizes reported."""
    torch = torch_cuda
    x = np.arange(1000, dtype=np.uint32) * 7
    d = gc.to_device(x)
    small = torch.zeros(8, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError):
        gc.encode_lists_gpu(d, np.array([1000]), gc.SIMPLE, gc.params(delta=True), d_out=small)


def test_gpu_encoder_refuses_vse(torch_cuda):
    """Group-VSEncoding streams come from the host encoder only: the GPU
    encoder returns GC_EINVAL for that codec."""
    x = np.arange(1000, dtype=np.uint32) * 7
    d = gc.to_device(x)
    with pytest.raises(gc.GcError) as e:
        gc.encode_lists_gpu(d, np.array([1000]), gc.VSE, gc.params(delta=True))
    assert e.value.code == gc.EINVAL


@pytest.mark.parametrize("k", [4, 64])
def test_gpu_encoder_cfg2(torch_cuda, k):
    """The full cfg2 lists (10,000 docID lists of 2^26 docIDs and their TF
    lists) in the five benchmark codecs: identical to the host encoder."""
    torch = torch_cuda
    lengths, docs, tfs = synth.cfg2()
    codecs = [("gsim", gc.SIMPLE, {}), ("gsc1cu", gc.SCHEME, dict(cg=1, ld=gc.LD_CU)),
              ("gsc8iu", gc.SCHEME, dict(cg=8, ld=gc.LD_IU)), ("afor", gc.AFOR, {}), ("pfd", gc.PFD, {})]
    d_docs, d_tfs = gc.to_device(docs), gc.to_device(tfs)
    for name, codec, kw in codecs:
        for what, flat, d_flat, delta in (("docids", docs, d_docs, True), ("tf", tfs, d_tfs, False)):
            say("cfg2", name, what, "k", k)
            p = gc.params(k=k, delta=delta, **kw)
            want, woffs = gc.encode_lists(flat, lengths, codec, p)
            got_d, goffs = gc.encode_lists_gpu(d_flat, lengths, codec, p)
            assert np.array_equal(goffs, woffs), (name, what)
            assert np.array_equal(gc.to_host(got_d), want), (name, what)
            del got_d


def test_gpu_encoder_threads_and_kept_scratch(torch_cuda):
    """The encoder keeps its scratch per device across calls: four host
    threads encode different list sets on one device at once (each on its
    own stream; the calls take the device's scratch in turn), then a small
    call runs in the grown scratch.  Every stream set equals the host
    encoder's."""
    import threading
    torch = torch_cuda
    rng = np.random.default_rng(77)
    picks = [VARIANTS[0], VARIANTS[11], VARIANTS[12], VARIANTS[6]]
    sets = []
    for i, (name, codec, kw) in enumerate(picks):
        lists = make_lists(rng, "docids", [100000 + 1000 * i, 5000, 0, 70001, 33])
        lengths = np.array([x.size for x in lists], np.int64)
        flat = np.concatenate(lists)
        sets.append((name, lengths, flat, gc.to_device(flat), codec, gc.params(k=4, delta=True, **kw)))
    torch.cuda.synchronize()
    got = [None] * len(sets)
    errors = []

    def work(i):
        try:
            name, lengths, flat, d_flat, codec, p = sets[i]
            st = torch.cuda.Stream()
            d, offs = gc.encode_lists_gpu(d_flat, lengths, codec, p, stream=st.cuda_stream)
            st.synchronize()
            got[i] = (gc.to_host(d), offs)
        except Exception as e:   # reported below, in the test's thread
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(sets))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for (name, lengths, flat, _, codec, p), (streams, offs) in zip(sets, got):
        say("threads", name)
        want, woffs = gc.encode_lists(flat, lengths, codec, p)
        assert np.array_equal(offs, woffs), name
        assert np.array_equal(streams, want), name
    small = [np.arange(1, 300, 3, dtype=np.uint32), np.arange(7, dtype=np.uint32)]
    say("small call after the threads")
    compare(torch, small, gc.PFD, gc.params(k=4, delta=True))
