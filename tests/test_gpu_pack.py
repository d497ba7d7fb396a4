"""GPU parity of the pack kernels, which decode up to 32 short lists of one
stream format per wave (their streams staged in LDS together, their control
units parsed and their integers unpacked together): element by element
against the oracle, for every codec variant and layout width, ragged and
aligned outputs, replayed from a graph, beside lists that stay on the class
passes, and with the kernel's grid capped so that each wave decodes many
packs in turn."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1502_01916_amd import gc

pytestmark = pytest.mark.gpu

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


def values(rng, n, kind):
    if kind == "docids":
        return np.sort(rng.choice(1 << 28, n, replace=False)).astype(np.uint32), True
    if kind == "spiky":
        x = rng.geometric(0.3, n).astype(np.uint32)
        m = max(1, n // 30)
        x[rng.integers(0, n, m)] = rng.integers(1 << 9, 1 << 31, m).astype(np.uint32)
        return x, False
    return (rng.integers(0, 1 << 32, n, dtype=np.uint64) >> rng.integers(0, 33, n).astype(np.uint64)
            ).astype(np.uint32), False


def short_batch(rng, nlists, ks, lengths):
    """nlists lists cycling through the variants and the layout widths ks,
    lengths drawn from `lengths`, docIDs / spiky / random-width values."""
    streams, lists = [], []
    kinds = ("docids", "spiky", "widths")
    for i in range(nlists):
        name, codec, kw = VARIANTS[i % len(VARIANTS)]
        k = ks[(i // len(VARIANTS)) % len(ks)]
        n = int(lengths[i])
        x, delta = values(rng, n, kinds[(i // (len(VARIANTS) * len(ks))) % 3])
        p = O.params(codec, k=k, delta=delta, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU),
                     pfd_pos=kw.get("pfd_pos", 0), zeta=kw.get("zeta", (1, 10)))
        streams.append(O.encode(x, p))
        lists.append(x)
    offs = np.concatenate([[0], np.cumsum([s.size for s in streams])]).astype(np.int64)
    return np.concatenate(streams), offs, np.array([x.size for x in lists], np.int64), lists


def check_plan(torch, ctx, flat, offs, lengths, lists, align, graph, pack_ints, reps=2, expect_packed=True,
               pack_groups=0):
    descs, headers, out_offs = gc.batch_layout(flat, offs, lengths, align=align)
    d_s = gc.to_device(flat)
    total = int(out_offs[-1])
    d_o = torch.full((total + 64,), -1, dtype=torch.int32, device="cuda")
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, use_graph=graph, pack_ints=pack_ints, pack_groups=pack_groups)
    cfg = plan.config()
    say("  plan", cfg)
    if expect_packed:
        assert cfg["packed_lists"] > 0 and cfg["packs"] > 0
    for rep in range(reps):
        d_o.fill_(-1)
        plan.decode_batch(d_s, d_o)
        rc, det = ctx.sync_status()
        assert rc == gc.OK, det
        got = gc.to_host(d_o)
        assert np.all(got[total:] == 0xFFFFFFFF), "write past the end"
        for i, x in enumerate(lists):
            o = int(out_offs[i])
            if not np.array_equal(got[o:o + x.size], x):
                bad = np.nonzero(got[o:o + x.size] != x)[0]
                pytest.fail("list %d (%s, n=%d): %d mismatches, first at %d: got %d want %d"
                            % (i, VARIANTS[i % len(VARIANTS)][0], x.size, bad.size, bad[0], got[o + bad[0]],
                               x[bad[0]]))
        _ = (d_o[:16].sum() + 1).item()     # unrelated eager work between replays
    d_o.fill_(-1)
    plan.decode_each(d_s, d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), np.concatenate(lists))
    plan.close()
    return cfg


@pytest.mark.parametrize("ks", [(4,), (64,), (8, 16, 32)])
@pytest.mark.parametrize("graph,align", [(False, 1), (True, 4)])
def test_short_lists_every_variant(torch_cuda, ctx, ks, graph, align):
    """Lists of 1 to 300 integers of every variant (docIDs prefix-summed, and
    values of mixed widths), each against the oracle's input."""
    rng = np.random.default_rng(7000 + 10 * len(ks) + ks[0] + int(graph))
    n = 3 * len(VARIANTS) * len(ks) * 2
    lengths = np.concatenate([[1, 2, 3, 4, 5, 7, 8, 9], rng.integers(1, 301, n - 8)])
    flat, offs, L, lists = short_batch(rng, n, ks, lengths)
    say("short lists ks", ks, "graph", graph, "align", align, "lists", n, "ints", int(L.sum()))
    check_plan(torch_cuda, ctx, flat, offs, L, lists, align, graph, 2048)


@pytest.mark.parametrize("pack_ints", [1024, 2048])
def test_pack_boundaries(torch_cuda, ctx, pack_ints):
    """Lists at and around the pack kernels' tile sizes (1024: 1023..1025,
    2048: 2047, 2048, 2049) and the staging limit, with the threshold at
    1024 and 2048: lists above it, or whose streams do not fit a pack, take
    the class passes in the same batch."""
    rng = np.random.default_rng(8100 + pack_ints)
    base = [1023, 1024, 1025, 2047, 2048, 2049, 4096, 1, 600, 5000]
    lengths = np.array([base[i % len(base)] for i in range(3 * len(VARIANTS))], np.int64)
    flat, offs, L, lists = short_batch(rng, lengths.size, (4, 8, 64), lengths)
    say("pack boundaries", pack_ints, int(L.sum()))
    check_plan(torch_cuda, ctx, flat, offs, L, lists, 1, False, pack_ints)


def test_pack_off_and_mixed_batch(torch_cuda, ctx):
    """A lognormal batch of short and long lists: packing on (default) and
    off give the oracle's output; with it off no list is packed."""
    rng = np.random.default_rng(8300)
    lengths = np.clip(np.round(np.exp(rng.normal(np.log(300), 1.5, 400))), 1, 60000).astype(np.int64)
    flat, offs, L, lists = short_batch(rng, lengths.size, (4, 4, 64), lengths)
    say("mixed batch", int(L.sum()))
    cfg = check_plan(torch_cuda, ctx, flat, offs, L, lists, 4, True, 0)
    assert cfg["pack_ints"] == 2048
    cfg = check_plan(torch_cuda, ctx, flat, offs, L, lists, 4, True, gc.PACK_OFF, expect_packed=False)
    assert cfg["packed_lists"] == 0 and cfg["packs"] == 0


def test_pack_incompressible_lists(torch_cuda, ctx):
    """32-bit values: a 2048-integer list's stream (8 KB) exceeds a pack's
    staging buffer and stays on the class passes, shorter ones are packed;
    all decode exactly."""
    rng = np.random.default_rng(8400)
    streams, lists = [], []
    for i, n in enumerate([2048, 1000, 200, 2048, 17, 999]):
        x = (rng.integers(1 << 31, 1 << 32, n, dtype=np.uint64)).astype(np.uint32)
        name, codec, kw = VARIANTS[(3 * i) % len(VARIANTS)]
        streams.append(O.encode(x, O.params(codec, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU),
                                            pfd_pos=kw.get("pfd_pos", 0))))
        lists.append(x)
    offs = np.concatenate([[0], np.cumsum([s.size for s in streams])]).astype(np.int64)
    L = np.array([x.size for x in lists], np.int64)
    cfg = check_plan(torch_cuda, ctx, np.concatenate(streams), offs, L, lists, 1, False, 2048)
    assert 0 < cfg["packed_lists"] < len(lists)


def test_pack_autotuned(torch_cuda, ctx, tmp_path, monkeypatch):
    """The autotuner chooses a threshold among none, 1024, 2048 and 4096
    (cached with the tile sizes); the plan decodes exactly."""
    torch = torch_cuda
    monkeypatch.setenv("GC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    rng = np.random.default_rng(8500)
    lengths = np.clip(np.round(np.exp(rng.normal(np.log(256), 1.2, 300))), 1, 20000).astype(np.int64)
    flat, offs, L, lists = short_batch(rng, lengths.size, (4, 64), lengths)
    descs, headers, out_offs = gc.batch_layout(flat, offs, L, align=4)
    d_s = gc.to_device(flat)
    d_o = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, autotune=True, use_graph=True)
    cfg = plan.config()
    say("autotuned pack", cfg)
    assert cfg["pack_ints"] in (0, 1024, 2048, 4096)
    assert cfg["pack_groups"] in (5, gc.PACK_GROUPS_ALL)
    plan.decode_batch(d_s, d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, L), np.concatenate(lists))
    plan2 = gc.Plan(ctx, descs, headers, d_s, d_o, autotune=True)      # from the cache
    assert plan2.config()["pack_ints"] == cfg["pack_ints"]
    assert plan2.config()["pack_groups"] == cfg["pack_groups"]
    assert plan2.config()["class_tiles"] == cfg["class_tiles"]
    plan.close()
    plan2.close()


@pytest.mark.parametrize("pack_groups", [1, 5, gc.PACK_GROUPS_ALL])
@pytest.mark.parametrize("name", ["pfd", "afor", "gsc8iu"])
def test_pack_groups(torch_cuda, ctx, name, pack_groups):
    """20,000 lists of 1 to 700 integers in one format (about 8,000 packs):
    with one pack workgroup per CU every wave decodes several packs in
    turn, with five fewer, with GC_PACK_GROUPS_ALL one each; all decode
    exactly, replayed from a graph."""
    rng = np.random.default_rng(8600 + len(name))
    _, codec, kw = next(v for v in VARIANTS if v[0] == name)
    lengths = rng.integers(1, 701, 20000)
    streams, lists = [], []
    for i, n in enumerate(lengths):
        x, delta = values(rng, int(n), "docids" if i % 3 else "spiky")
        p = O.params(codec, k=4, delta=delta, cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU))
        streams.append(O.encode(x, p))
        lists.append(x)
    offs = np.concatenate([[0], np.cumsum([s.size for s in streams])]).astype(np.int64)
    say("pack groups", name, pack_groups, int(lengths.sum()))
    cfg = check_plan(torch_cuda, ctx, np.concatenate(streams), offs, lengths.astype(np.int64), lists, 4, True,
                     1024, reps=2, pack_groups=pack_groups)
    assert cfg["pack_groups"] == pack_groups
    assert cfg["packs"] > 4 * 256
