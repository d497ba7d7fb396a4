"""GPU parity: libgc's HIP decode path (through the C ABI) against the CPU
oracle, element by element and bit-exact.  Streams are written by the oracle;
outputs are compared with the oracle's decode of the same stream and with the
original list."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1502_01916_amd import gc, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = gc.Context(0)
    yield c
    c.close()


def gpu_decode(torch, ctx, stream, n):
    d_s = gc.to_device(stream)
    d_o = torch.full((max(n, 1) + 64,), -1, dtype=torch.int32, device="cuda")
    ctx.decode(d_s, stream.size, stream[:4], d_o)
    rc, detail = ctx.sync_status()
    out = gc.to_host(d_o)
    assert rc == gc.OK, "device status %d detail %d" % (rc, detail)
    assert np.all(out[max(n, 1):] == 0xFFFFFFFF), "write past the end of the output"
    return out[:n]


VARIANTS = [
    ("gsim", O.SIMPLE, {}), ("gsc1cu", O.SCHEME, dict(cg=1, ld=O.LD_CU)),
    ("gsc2cu", O.SCHEME, dict(cg=2, ld=O.LD_CU)), ("gsc4cu", O.SCHEME, dict(cg=4, ld=O.LD_CU)),
    ("gsc8cu", O.SCHEME, dict(cg=8, ld=O.LD_CU)), ("gsc4iu", O.SCHEME, dict(cg=4, ld=O.LD_IU)),
    ("gsc8iu", O.SCHEME, dict(cg=8, ld=O.LD_IU)), ("gsc1b", O.SCHEME, dict(cg=1, ld=O.LD_BINARY)),
    ("gsc2b", O.SCHEME, dict(cg=2, ld=O.LD_BINARY)), ("gsc4b", O.SCHEME, dict(cg=4, ld=O.LD_BINARY)),
    ("gsc8b", O.SCHEME, dict(cg=8, ld=O.LD_BINARY)), ("afor", O.AFOR, {}),
    ("pfd", O.PFD, {}), ("pfdbitmap", O.PFD, dict(pfd_pos=O.PFD_BITMAP)),
    ("bp128", O.PFD, dict(zeta=(1, 32))), ("vse", O.VSE, {}),
]

LENGTHS = [1, 3, 4, 5, 127, 128, 129, 4095, 4096, 4097, 3 * 4096 + 17, 70001]


def gen_inputs(rng, n):
    yield "docids", np.sort(rng.choice(1 << 27, n, replace=False)).astype(np.uint32), True
    yield "widths", (rng.integers(0, 1 << 32, n, dtype=np.uint64)
                     >> rng.integers(0, 33, n).astype(np.uint64)).astype(np.uint32), False
    x = rng.geometric(0.3, n).astype(np.uint32)
    x[rng.integers(0, n, max(1, n // 40))] = rng.integers(1 << 9, 1 << 31, max(1, n // 40)).astype(np.uint32)
    yield "spiky", x, False


@pytest.mark.parametrize("k", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("vi", range(len(VARIANTS)))
def test_single_list_parity(torch_cuda, ctx, vi, k):
    name, codec, kw = VARIANTS[vi]
    rng = np.random.default_rng(1000 + 17 * vi + k)
    for n in LENGTHS:
        for kind, x, delta in gen_inputs(rng, n):
            say("case", name, "k", k, "n", n, kind)
            p = O.params(codec, k=k, delta=delta, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU),
                         pfd_pos=kw.get("pfd_pos", 0), zeta=kw.get("zeta", (1, 10)))
            s = O.encode(x, p)
            ref = O.decode(s)
            got = gpu_decode(torch_cuda, ctx, s, n)
            if not np.array_equal(got, ref):
                bad = np.nonzero(got != ref)[0]
                pytest.fail("%s k=%d n=%d %s: %d mismatches, first at %d: got %d want %d"
                            % (name, k, n, kind, bad.size, bad[0], got[bad[0]], ref[bad[0]]))
            assert np.array_equal(ref, x)


def test_degenerate_lists(torch_cuda, ctx):
    for name, codec, kw in VARIANTS:
        for x in (np.zeros(9000, np.uint32), np.full(9000, 0xFFFFFFFF, np.uint32),
                  np.full(8193, 1, np.uint32)):
            say("degenerate", name, x[0], x.size)
            p = O.params(codec, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU),
                         pfd_pos=kw.get("pfd_pos", 0), zeta=kw.get("zeta", (1, 10)))
            s = O.encode(x, p)
            assert np.array_equal(gpu_decode(torch_cuda, ctx, s, x.size), x)
        # docIDs that wrap past 2^32 (gaps near 2^31)
        g = np.full(5000, (1 << 31) - 1, np.uint32)
        d = O.prefix_sum(g)
        s = O.encode(d, O.params(codec, delta=True, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU),
                                 pfd_pos=kw.get("pfd_pos", 0), zeta=kw.get("zeta", (1, 10))))
        assert np.array_equal(gpu_decode(torch_cuda, ctx, s, d.size), d)


def test_cfg1_group_simple(torch_cuda, ctx):
    d = synth.cfg1()
    s = O.encode(d, O.params(O.SIMPLE, delta=True))
    say("cfg1", d.size, s.size)
    got = gpu_decode(torch_cuda, ctx, s, d.size)
    assert np.array_equal(got, O.decode(s))
    assert np.array_equal(got, d)


@pytest.mark.parametrize("codec,kw", [(O.SIMPLE, {}), (O.SCHEME, dict(cg=1, ld=O.LD_CU)), (O.PFD, {})])
def test_single_list_carry_modes(torch_cuda, ctx, codec, kw):
    """A list decoded alone finds its carries by look-back up to 2048 tiles
    and by the tile-sum pass beyond: lists just inside and just past that
    size (tiles of 2048 integers, 4096 for Group-PFD)."""
    rng = np.random.default_rng(11 + codec)
    tile = 4096 if codec == O.PFD else 2048
    for n in (2048 * tile - 5, 2048 * tile + 77):
        d = np.sort(rng.choice(1 << 27, n, replace=False)).astype(np.uint32)
        s = O.encode(d, O.params(codec, delta=True, **kw))
        say("single list", codec, kw, n)
        got = gpu_decode(torch_cuda, ctx, s, n)
        assert np.array_equal(got, d)
        assert np.array_equal(got, O.decode(s))


def make_batch(rng, nlists, kmix=(4,), maxlen=40000):
    """nlists lists cycling through the variants; each pass over them takes
    the next layout width of kmix, and delta and TF lists alternate between
    passes, so every (variant, k, delta) combination occurs once nlists
    reaches 2 * len(kmix) * len(VARIANTS)."""
    lengths = np.clip(np.round(np.exp(rng.normal(np.log(800), 1.6, nlists))), 0, maxlen).astype(np.int64)
    streams, lists, plist = [], [], []
    for i, L in enumerate(lengths):
        name, codec, kw = VARIANTS[i % len(VARIANTS)]
        k = kmix[(i // len(VARIANTS)) % len(kmix)]
        delta = (i // len(VARIANTS)) % 2 == 0
        x = (np.sort(rng.choice(1 << 28, int(L), replace=False)).astype(np.uint32) if delta
             else rng.geometric(0.2, int(L)).astype(np.uint32))
        p = O.params(codec, k=k, delta=delta, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU),
                     pfd_pos=kw.get("pfd_pos", 0), zeta=kw.get("zeta", (1, 10)))
        streams.append(O.encode(x, p))
        lists.append(x)
    offs = np.concatenate([[0], np.cumsum([s.size for s in streams])]).astype(np.int64)
    flat = np.concatenate(streams) if streams else np.zeros(0, np.uint32)
    return flat, offs, lengths, lists


@pytest.mark.parametrize("tiles", [(1024, 2048), (2048, 4096), (4096, 4096)])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("carry", [gc.CARRY_DEFAULT, gc.CARRY_SUM_PASS, gc.CARRY_LOOKBACK])
def test_batch_parity(torch_cuda, ctx, tiles, graph, carry):
    torch = torch_cuda
    tile, pfd_tile = tiles
    rng = np.random.default_rng(50 + tile + int(graph))
    flat, offs, lengths, lists = make_batch(rng, 300, kmix=(4, 8, 16, 32, 64))
    align = 4 if graph else 1        # 16-byte aligned lists take the vector-store path
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=align)
    d_s = gc.to_device(flat)
    total = int(out_offs[-1])
    d_o = torch.full((total + 64,), -1, dtype=torch.int32, device="cuda")
    say("batch tile", tile, "graph", graph, "carry", carry, "lists", len(descs), "ints", total)
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, tile_ints=tile, pfd_tile_ints=pfd_tile, use_graph=graph,
                   carry_pass=carry)
    want = np.concatenate(lists)
    for rep in range(3):
        d_o.fill_(-1)
        plan.decode_batch(d_s, d_o)
        rc, det = ctx.sync_status()
        assert rc == gc.OK, det
        got = gc.to_host(d_o)
        assert np.all(got[total:] == 0xFFFFFFFF)
        assert np.array_equal(gc.unpad(got, out_offs, lengths), want), "replay %d" % rep
        torch.cuda.synchronize()
        _ = (d_o[:16].sum() + 1).item()     # unrelated eager work between replays
    d_o.fill_(-1)
    plan.decode_each(d_s, d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), want)
    plan.close()


@pytest.mark.parametrize("carry", [gc.CARRY_DEFAULT, gc.CARRY_SUM_PASS, gc.CARRY_LOOKBACK])
def test_pfd_1024_tiles(torch_cuda, ctx, carry):
    """Group-PFD in tiles of 1024 integers (whole 32-tuple blocks up to
    k = 32): linked and bitmap exceptions and the no-exception form, k = 4 to
    32, ragged lengths, d-gap lists (carried across tiles) and lists of
    exception-heavy widths; then with one k = 64 list added, which raises the
    class's tile to 2048."""
    torch = torch_cuda
    rng = np.random.default_rng(300 + carry)
    pv = [(dict(), 0), (dict(pfd_pos=O.PFD_BITMAP), 0), (dict(zeta=(1, 32)), 0)]
    streams, lists = [], []
    i = 0
    for k in (4, 8, 16, 32):
        for kw, _ in pv:
            for n in (1, 127, 1023, 1024, 1025, 5000, 70001):
                delta = i % 2 == 0
                x = (np.sort(rng.choice(1 << 28, n, replace=False)).astype(np.uint32) if delta else
                     (rng.integers(0, 1 << 32, n, dtype=np.uint64) >> rng.integers(0, 33, n).astype(np.uint64))
                     .astype(np.uint32))
                streams.append(O.encode(x, O.params(O.PFD, k=k, delta=delta, **kw)))
                lists.append(x)
                i += 1
    wide = np.sort(rng.choice(1 << 28, 9000, replace=False)).astype(np.uint32)
    for extra in (False, True):
        ss = streams + ([O.encode(wide, O.params(O.PFD, k=64, delta=True))] if extra else [])
        ls = lists + ([wide] if extra else [])
        flat = np.concatenate(ss)
        offs = np.concatenate([[0], np.cumsum([x.size for x in ss])]).astype(np.int64)
        lengths = np.array([x.size for x in ls], np.int64)
        descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=4)
        d_s = gc.to_device(flat)
        total = int(out_offs[-1])
        d_o = torch.full((total + 64,), -1, dtype=torch.int32, device="cuda")
        say("pfd 1024 tiles: carry", carry, "k=64 list", extra, "lists", len(descs), "ints", total)
        plan = gc.Plan(ctx, descs, headers, d_s, d_o, pfd_tile_ints=1024, use_graph=True, carry_pass=carry)
        assert plan.config()["pfd_tile_ints"] == (2048 if extra else 1024)
        want = np.concatenate(ls)
        for rep in range(2):
            d_o.fill_(-1)
            plan.decode_batch(d_s, d_o)
            rc, det = ctx.sync_status()
            assert rc == gc.OK, det
            got = gc.to_host(d_o)
            assert np.all(got[total:] == 0xFFFFFFFF)
            assert np.array_equal(gc.unpad(got, out_offs, lengths), want), "replay %d" % rep
        plan.close()


@pytest.mark.parametrize("codec,kw", [(gc.SIMPLE, {}), (gc.SCHEME, dict(cg=8, ld=gc.LD_IU)), (gc.PFD, {})])
def test_lookback_long_lists(torch_cuda, ctx, codec, kw):
    """Single-pass carries over lists of hundreds of tiles, so that a look-back
    crosses several 64-tile windows, next to short lists; replayed from a
    graph (each replay a new epoch of flags) and checked every time; then the
    same plan with the two-pass carry, and with the mixed one (look-back for
    the lists of up to 64 tiles, the tile-sum pass for the longer ones, in
    the same launches)."""
    torch = torch_cuda
    rng = np.random.default_rng(int(codec) + 900)
    # 64 and 65 tiles of 1024: the two sides of the mixed mode's threshold
    lengths = np.array([700 * 1024 + 333, 5, 2048, 300 * 1024, 1, 129 * 1024 + 1, 64 * 1024, 64 * 1024 + 1],
                       np.int64)
    lists = [np.sort(rng.choice(1 << 31, int(n), replace=False)).astype(np.uint32) for n in lengths]
    lists[3] = O.prefix_sum(np.full(int(lengths[3]), (1 << 31) - 1, np.uint32))   # wrapping sums
    p = O.params(codec, delta=True, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU))
    streams = [O.encode(x, p) for x in lists]
    offs = np.concatenate([[0], np.cumsum([x.size for x in streams])]).astype(np.int64)
    flat = np.concatenate(streams)
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=4)
    d_s = gc.to_device(flat)
    d_o = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    want = np.concatenate(lists)
    for carry in (gc.CARRY_LOOKBACK, gc.CARRY_SUM_PASS, gc.CARRY_HYBRID):
        say("look-back long lists codec", codec, "carry", carry)
        plan = gc.Plan(ctx, descs, headers, d_s, d_o, tile_ints=1024, pfd_tile_ints=2048, use_graph=True,
                       carry_pass=carry)
        for rep in range(4):
            d_o.fill_(-1)
            plan.decode_batch(d_s, d_o)
            rc, det = ctx.sync_status()
            assert rc == gc.OK, det
            assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), want), (carry, rep)
        plan.close()


def test_lookback_bounded_wait(torch_cuda, ctx, monkeypatch):
    """The look-back's wait is bounded.  With the plan's tiles withholding
    their flags (a condition only this test sets, from the host), every
    look-back gives up after its limit, the kernels finish, and the device
    reports the expiry (detail 12).  A plan made without it afterwards decodes
    the same batch exactly."""
    torch = torch_cuda
    rng = np.random.default_rng(1212)
    lengths = np.array([3 * 1024 + 5, 7 * 1024, 40 * 1024 + 1, 2 * 1024], np.int64)
    lists = [np.sort(rng.choice(1 << 30, int(n), replace=False)).astype(np.uint32) for n in lengths]
    streams = [O.encode(x, O.params(O.SIMPLE, delta=True)) for x in lists]
    offs = np.concatenate([[0], np.cumsum([x.size for x in streams])]).astype(np.int64)
    flat = np.concatenate(streams)
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=4)
    d_s = gc.to_device(flat)
    d_o = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    say("look-back bounded wait")
    monkeypatch.setenv("GC_TEST_LOOKBACK_STALL", "20000")   # 200 us per look-back
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, tile_ints=1024, carry_pass=gc.CARRY_LOOKBACK)
    plan.decode_batch(d_s, d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.ECORRUPT and det == 12, (rc, det)
    plan.close()
    monkeypatch.delenv("GC_TEST_LOOKBACK_STALL")
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, tile_ints=1024, carry_pass=gc.CARRY_LOOKBACK)
    d_o.fill_(-1)
    plan.decode_batch(d_s, d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), np.concatenate(lists))
    plan.close()


def test_widest_tiles_full_width(torch_cuda, ctx):
    """4096-integer tiles whose values are all 32 bits wide (gaps of 2^31 and
    more, plus a TF list of 2^32 - 1): the bit offsets of a tile's tuples then
    run up to 1024 * 32, the largest a tuple record holds.  Every codec, one
    batch, both carry modes."""
    torch = torch_cuda
    rng = np.random.default_rng(4096)
    streams, lists = [], []
    for i, (name, codec, kw) in enumerate(VARIANTS):
        n = 3 * 4096 + 100 + 37 * i
        if i % 2 == 0:
            g = rng.integers(1 << 31, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
            x, delta = O.prefix_sum(g), True
        else:
            x, delta = np.full(n, 0xFFFFFFFF, np.uint32), False
        p = O.params(codec, delta=delta, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU),
                     pfd_pos=kw.get("pfd_pos", 0), zeta=kw.get("zeta", (1, 10)))
        streams.append(O.encode(x, p))
        lists.append(x)
    lengths = np.array([x.size for x in lists], np.int64)
    offs = np.concatenate([[0], np.cumsum([x.size for x in streams])]).astype(np.int64)
    flat = np.concatenate(streams)
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=4)
    d_s = gc.to_device(flat)
    d_o = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    want = np.concatenate(lists)
    for carry in (gc.CARRY_SUM_PASS, gc.CARRY_LOOKBACK, gc.CARRY_HYBRID):
        say("full-width 4096 tiles carry", carry)
        plan = gc.Plan(ctx, descs, headers, d_s, d_o, tile_ints=4096, pfd_tile_ints=4096, carry_pass=carry)
        d_o.fill_(-1)
        plan.decode_batch(d_s, d_o)
        rc, det = ctx.sync_status()
        assert rc == gc.OK, det
        assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), want), carry
        plan.close()


@pytest.mark.parametrize("class_tiles", [[1024, 4096, 2048, 4096, 2048], [4096, 1024, 4096, 1024, 4096]])
def test_mixed_class_tiles(torch_cuda, ctx, class_tiles):
    """A different tile size for the codec classes of one batch (the
    autotuner's per-class choice), replayed from a graph, every carry mode."""
    torch = torch_cuda
    rng = np.random.default_rng(515)
    flat, offs, lengths, lists = make_batch(rng, 200, kmix=(4, 4, 8))
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=4)
    d_s = gc.to_device(flat)
    d_o = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    want = np.concatenate(lists)
    for carry in (gc.CARRY_DEFAULT, gc.CARRY_SUM_PASS, gc.CARRY_LOOKBACK):
        say("class tiles", class_tiles, "carry", carry)
        plan = gc.Plan(ctx, descs, headers, d_s, d_o, class_tiles=class_tiles, use_graph=True, carry_pass=carry)
        assert plan.config()["class_tiles"] == class_tiles
        for rep in range(2):
            d_o.fill_(-1)
            plan.decode_batch(d_s, d_o)
            rc, det = ctx.sync_status()
            assert rc == gc.OK, det
            assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), want), (carry, rep)
        plan.close()


def test_autotuned_plan(torch_cuda, ctx, tmp_path, monkeypatch):
    torch = torch_cuda
    monkeypatch.setenv("GC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    rng = np.random.default_rng(77)
    flat, offs, lengths, lists = make_batch(rng, 120)
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths)
    d_s = gc.to_device(flat)
    d_o = torch.zeros(int(out_offs[-1]) + 4, dtype=torch.int32, device="cuda")
    say("autotune")
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, autotune=True, use_graph=True)
    cfg = plan.config()
    assert cfg["tile_ints"] in (1024, 2048, 4096) and cfg["pfd_tile_ints"] in (1024, 2048, 4096)
    ct = cfg["class_tiles"]        # one size per codec class
    assert all(t in (1024, 2048, 4096) for t in ct)
    assert 1 <= cfg["tiles"] and cfg["sum_tiles"] <= cfg["tiles"]
    plan.decode_batch(d_s, d_o)
    assert ctx.sync_status()[0] == gc.OK
    assert np.array_equal(gc.to_host(d_o)[:int(out_offs[-1])], np.concatenate(lists))
    assert (tmp_path / "tune.json").exists()
    plan2 = gc.Plan(ctx, descs, headers, d_s, d_o, autotune=True)   # served from the cache
    assert plan2.config()["class_tiles"] == ct


@pytest.mark.parametrize("locate_stream", [False, True])
def test_timed_plan(torch_cuda, ctx, locate_stream):
    """A plan with timing slots launches its kernels directly (the locate
    kernels on a second stream with locate_stream); its output equals the
    oracle's, and every class present reports positive phase times on every
    run."""
    torch = torch_cuda
    rng = np.random.default_rng(31)
    flat, offs, lengths, lists = make_batch(rng, 160, kmix=(4, 4, 8))
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=4)
    d_s = gc.to_device(flat)
    d_o = torch.full((int(out_offs[-1]) + 16,), -1, dtype=torch.int32, device="cuda")
    say("timed plan locate_stream", locate_stream)
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, timing_slots=4, locate_stream=locate_stream)
    want = np.concatenate(lists)
    for rep in range(6):
        plan.decode_batch(d_s, d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), want)
    tm = plan.timings(10)
    assert tm["total"].shape == (4,) and tm["decode"].shape == (4, gc.CLASSES)
    present = {gc.CLS_SIMPLE, gc.CLS_SCHEME_UNARY, gc.CLS_SCHEME_BINARY, gc.CLS_AFOR, gc.CLS_PFD}
    assert np.all(tm["total"] > 0)
    for c in present:
        assert np.all(tm["decode"][:, c] > 0), c
        assert np.all(tm["sum"][:, c] > 0), c
        assert np.all(tm["decode"][:, c] <= tm["total"] + 1e-3)
    if locate_stream:
        for c in present:
            assert np.all(tm["locate"][:, c] > 0), c
    else:
        # one locate pass for every class, timed in the first class's column
        assert np.all(tm["locate"][:, gc.CLS_SIMPLE] > 0)
        assert not np.any(tm["locate"][:, 1:])
    plan.close()


def test_corrupt_streams_latch_status(torch_cuda, ctx):
    torch = torch_cuda
    rng = np.random.default_rng(9)
    d = np.sort(rng.choice(1 << 26, 20000, replace=False)).astype(np.uint32)
    cases = []
    s = O.encode(d, O.params(O.SIMPLE, delta=True))
    bad = s.copy()
    bad[4 + 3] = 0xCCCCCCCC                          # selectors 12
    cases.append(("gsim selector", bad))
    s = O.encode(d, O.params(O.AFOR, delta=True))
    bad = s.copy()
    bad[4 + 1] |= 0xC0C0C0C0                         # frame class 3
    cases.append(("afor class", bad))
    s = O.encode(d, O.params(O.VSE, delta=True))
    bad = s.copy()
    bad[4 + 1] = 0xE8E8E8E8                          # 12-tuple frames of width 40
    assert O.decode_status(bad) == O.ECORRUPT
    cases.append(("vse width", bad))
    s = O.encode(d, O.params(O.PFD, delta=True))
    bad = s.copy()
    bad[4 + 2] = (int(bad[4 + 2]) & ~63) | 45        # b = 45
    cases.append(("pfd width", bad))
    s = O.encode(d, O.params(O.SCHEME, cg=1, ld=O.LD_CU, delta=True))
    bad = s.copy()
    bad[4 + 5] = 0xFFFFFFFF
    bad[4 + 6] = 0xFFFFFFFF                          # a code longer than 32 units
    cases.append(("gsc unary", bad))
    for name, b in cases:
        say("corrupt", name)
        d_s = gc.to_device(b)
        d_o = torch.full((d.size + 64,), -1, dtype=torch.int32, device="cuda")
        ctx.decode(d_s, b.size, b[:4], d_o)
        rc, detail = ctx.sync_status()
        assert rc == gc.ECORRUPT, name
        assert np.all(gc.to_host(d_o)[d.size:] == 0xFFFFFFFF)
    # the context keeps working after an error
    s = O.encode(d, O.params(O.SIMPLE, delta=True))
    assert np.array_equal(gpu_decode(torch, ctx, s, d.size), d)


def test_host_rejects_bad_headers(torch_cuda, ctx):
    d = np.arange(1000, dtype=np.uint32)
    s = O.encode(d, O.params(O.SIMPLE))
    descs, headers, _ = gc.batch_layout(s, np.array([0, s.size]), np.array([d.size]))
    headers = headers.copy()
    headers[0, 0] |= 1 << 30
    with pytest.raises(gc.GcError) as e:
        gc.Plan(ctx, descs, headers)
    assert e.value.code == gc.ECORRUPT
    descs[0].stream_words = 3
    with pytest.raises(gc.GcError):
        gc.Plan(ctx, descs, headers)


def test_cfg2_full_size_batch(torch_cuda, ctx):
    """The benchmark workload at full size, in the launch configuration the
    benchmark times: every cfg2 list (docIDs and TFs) through one hipGraph
    launch per codec; outputs equal the generator's lists (the
    lossless-codec property at any size) and, on sampled lists, the oracle."""
    torch = torch_cuda
    lengths, docs, tfs = synth.cfg2()
    lo = np.concatenate([[0], np.cumsum(lengths)])
    sample = np.random.default_rng(0).choice(lengths.size, 12, replace=False)
    codecs = [("gsim", gc.SIMPLE, {}), ("gsc1cu", gc.SCHEME, dict(cg=1, ld=gc.LD_CU)),
              ("gsc8iu", gc.SCHEME, dict(cg=8, ld=gc.LD_IU)), ("afor", gc.AFOR, {}),
              ("pfd", gc.PFD, {})]
    for name, codec, kw in codecs:
        for what, flat, delta in (("docids", docs, True), ("tf", tfs, False)):
            say("cfg2", name, what)
            p = gc.params(delta=delta, **kw)
            s, offs = gc.encode_lists(flat, lengths, codec, p)
            descs, headers, out_offs = gc.batch_layout(s, offs, lengths)
            d_s = gc.to_device(s)
            d_o = torch.empty(int(out_offs[-1]), dtype=torch.int32, device="cuda")
            plan = gc.Plan(ctx, descs, headers, d_s, d_o, use_graph=True)
            plan.decode_batch(d_s, d_o)
            rc, det = ctx.sync_status()
            assert rc == gc.OK, det
            got = gc.to_host(d_o)
            assert np.array_equal(got, flat), (name, what)
            op = O.params(codec, delta=delta, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU))
            for i in sample:
                seg = s[int(offs[i]):int(offs[i + 1])]
                assert np.array_equal(seg, O.encode(flat[lo[i]:lo[i + 1]], op))
                assert np.array_equal(got[lo[i]:lo[i + 1]], O.decode(seg))
            plan.close()
            del d_s, d_o


def test_single_lists_of_different_classes(torch_cuda):
    """One context decodes multi-tile delta lists of different codec classes
    in turn (its single-list tables, look-back flags included, are shared by
    every class): each output equals the oracle's, on a fresh context so the
    classes' run counts stay level."""
    torch = torch_cuda
    c = gc.Context(0)
    rng = np.random.default_rng(4242)
    order = [(O.SIMPLE, {}), (O.SCHEME, dict(cg=1, ld=O.LD_CU)), (O.SCHEME, dict(cg=2, ld=O.LD_BINARY)),
             (O.AFOR, {}), (O.PFD, {})]
    for rnd in range(3):
        for codec, kw in order:
            n = int(rng.integers(20000, 60000))
            d = np.sort(rng.choice(1 << 28, n, replace=False)).astype(np.uint32)
            s = O.encode(d, O.params(codec, delta=True, **kw))
            say("cross-class round", rnd, codec, kw, n)
            got = gpu_decode(torch, c, s, n)
            assert np.array_equal(got, O.decode(s)), (rnd, codec, kw)
    c.close()


def test_decode_captured_in_graph(torch_cuda, ctx):
    """gc_decode allocates nothing and never synchronises, so it can be
    captured in a hipGraph: the captured decode of a multi-tile delta list is
    replayed several times, with eager work between the replays, and every
    replay equals the oracle's decode."""
    torch = torch_cuda
    rng = np.random.default_rng(808)
    for codec, kw in ((O.SIMPLE, {}), (O.PFD, {}), (O.SCHEME, dict(cg=8, ld=O.LD_IU))):
        n = 300001
        d = np.sort(rng.choice(1 << 28, n, replace=False)).astype(np.uint32)
        s = O.encode(d, O.params(codec, delta=True, **kw))
        want = O.decode(s)
        d_s = gc.to_device(s)
        d_o = torch.full((n + 64,), -1, dtype=torch.int32, device="cuda")
        ctx.decode(d_s, s.size, s[:4], d_o)          # eager warm-up
        torch.cuda.synchronize()
        say("graph capture of gc_decode", codec, kw)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            ctx.decode(d_s, s.size, s[:4], d_o)
        for rep in range(4):
            d_o.fill_(-1)
            g.replay()
            rc, det = ctx.sync_status()
            assert rc == gc.OK, det
            out = gc.to_host(d_o)
            assert np.array_equal(out[:n], want), rep
            assert np.all(out[n:] == 0xFFFFFFFF)
            _ = (d_o[:16].sum() + 1).item()     # unrelated eager work between replays
        del g


def test_decode_over_context_limit(torch_cuda):
    """A list longer than the context's max_list_ints is refused with
    GC_ENOSPC (nothing is launched or allocated); lists within it decode."""
    torch = torch_cuda
    c = gc.Context(0, max_list_ints=4096)
    d = np.arange(5000, dtype=np.uint32) * 3
    s = O.encode(d, O.params(O.SIMPLE, delta=True))
    d_s = gc.to_device(s)
    d_o = torch.full((5064,), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(gc.GcError) as e:
        c.decode(d_s, s.size, s[:4], d_o)
    assert e.value.code == gc.ENOSPC
    assert np.all(gc.to_host(d_o) == 0xFFFFFFFF)
    s2 = O.encode(d[:4096], O.params(O.SIMPLE, delta=True))
    assert np.array_equal(gpu_decode(torch, c, s2, 4096), d[:4096])
    c.close()


@pytest.mark.parametrize("graph", [False, True])
def test_autotuned_plan_with_locate_stream(torch_cuda, ctx, tmp_path, monkeypatch, graph):
    """Autotuning a plan whose locate kernels run on a second stream: the
    candidate runs and the final plan agree on whose locate epoch tags the
    tile starts, so every run decodes (status OK) and matches the oracle."""
    torch = torch_cuda
    monkeypatch.setenv("GC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    rng = np.random.default_rng(78 + int(graph))
    flat, offs, lengths, lists = make_batch(rng, 150, kmix=(4, 8))
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=4)
    d_s = gc.to_device(flat)
    d_o = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    want = np.concatenate(lists)
    say("autotune with locate stream, graph", graph)
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, autotune=True, locate_stream=True, use_graph=graph)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det        # the autotuner's own runs
    for rep in range(3):
        d_o.fill_(-1)
        plan.decode_batch(d_s, d_o)
        rc, det = ctx.sync_status()
        assert rc == gc.OK, det
        assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), want), rep
    d_o.fill_(-1)
    plan.decode_each(d_s, d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), want)
    plan.close()
