"""GPU parity of the per-block container kernels (through the C ABI) against
the oracle: features, all sixteen class sizes and the exhaustive choice, and
the container itself, word for word."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1502_01916_amd import gc, synth

from test_blocks_oracle import blocks

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


def corpus(seed, nb):
    """Blocks of the d-gap/TF corpus plus the synthetic width mixes."""
    _, vals = synth.block_corpus(seed, 128 * (nb - nb // 4))
    x = np.concatenate([vals, blocks(seed, nb // 4).reshape(-1)])
    x = np.concatenate([x, np.zeros(128 * nb - x.size, np.uint32)])
    x[:128] = 0                       # an all-zero block
    x[128:256] = 0xFFFFFFFF           # an all-32-bit block
    return x.reshape(nb, 128)


def oracle_rows(x):
    feat = np.array([O.block_features(b) for b in x])
    best, sizes = zip(*[O.block_best(b) for b in x])
    return feat, np.array(sizes), np.array(best)


@pytest.mark.parametrize("nb", [1, 5, 300, 2049])
def test_block_features_sizes(torch_cuda, ctx, nb):
    torch = torch_cuda
    say("block features/sizes nb=%d" % nb)
    x = corpus(nb, nb)
    feat, sizes, best = oracle_rows(x)
    d_in = gc.to_device(x.reshape(-1))
    d_feat = torch.full((nb, 40), -1.0, dtype=torch.float32, device="cuda")
    d_sizes = torch.full((nb, 16), -1, dtype=torch.int32, device="cuda")
    d_best = torch.full((nb,), 255, dtype=torch.uint8, device="cuda")
    d_cost = torch.full((nb, 16), -1.0, dtype=torch.float32, device="cuda")
    ctx.block_features(d_in, nb, d_feat)
    ctx.block_sizes(d_in, nb, d_sizes, d_best, d_cost)
    torch.cuda.synchronize()
    g_feat = d_feat.cpu().numpy().astype(np.float64)
    # every feature is a multiple of 1/128 or 1/32: exact in fp32
    assert np.array_equal(g_feat, feat)
    assert np.array_equal(d_sizes.cpu().numpy().astype(np.int64), sizes)
    assert np.array_equal(d_best.cpu().numpy().astype(np.int64), best)
    # relative excess: an exact integer difference over the least size, one fp32 rounding
    smin = sizes.min(axis=1, keepdims=True)
    want = (sizes - smin).astype(np.float32) / smin.astype(np.float32)
    assert np.array_equal(d_cost.cpu().numpy(), want)
    # best alone
    d_best2 = torch.full((nb,), 255, dtype=torch.uint8, device="cuda")
    ctx.block_sizes(d_in, nb, None, d_best2)
    torch.cuda.synchronize()
    assert torch.equal(d_best, d_best2)


@pytest.mark.parametrize("n", [1, 127, 128, 129, 5000, 128 * 2048 + 77])
@pytest.mark.parametrize("mode", ["best", "random", "fixed"])
def test_blockmix_encode(torch_cuda, ctx, n, mode):
    torch = torch_cuda
    say("blockmix encode n=%d mode=%s" % (n, mode))
    nb = (n + 127) // 128
    x = corpus(n, nb).reshape(-1)
    x[n:] = 0
    rng = np.random.default_rng(n)
    if mode == "best":
        k = np.array([O.block_best(b)[0] for b in x.reshape(nb, 128)], np.uint8)
    elif mode == "random":
        k = rng.integers(0, 16, nb).astype(np.uint8)
    else:
        k = np.full(nb, 12, np.uint8)
    want, _ = O.blockmix_encode(x[:n], k)
    d_in = gc.to_device(x)
    d_k = torch.from_numpy(k).cuda()
    cap = gc.blockmix_bound_words(n)
    d_out = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    used = ctx.blockmix_encode(d_in, n, d_k, d_out)
    got = gc.to_host(d_out)
    assert used == want.size
    assert np.array_equal(got[:used], want)
    assert np.all(got[used:] == 0xFFFFFFFF)
    assert np.array_equal(O.blockmix_decode(got[:used]), x[:n])


def test_blockmix_errors(torch_cuda, ctx):
    torch = torch_cuda
    say("blockmix errors")
    x = corpus(1, 4).reshape(-1)
    d_in = gc.to_device(x)
    d_k = torch.tensor([0, 3, 16, 1], dtype=torch.uint8, device="cuda")
    d_out = torch.zeros(gc.blockmix_bound_words(512), dtype=torch.int32, device="cuda")
    with pytest.raises(gc.GcError) as e:
        ctx.blockmix_encode(d_in, 512, d_k, d_out)
    assert e.value.code == gc.EINVAL
    d_k[2] = 5
    small = torch.zeros(10, dtype=torch.int32, device="cuda")
    with pytest.raises(gc.GcError) as e:
        ctx.blockmix_encode(d_in, 512, d_k, small)
    assert e.value.code == gc.ENOSPC
    # capacities between the block words and the whole container: nothing
    # is written past the capacity
    need = ctx.blockmix_encode(d_in, 512, d_k, d_out)
    assert need > 8
    for cap in (8, 9, need - 1):
        big = torch.full((need + 64,), -7, dtype=torch.int32, device="cuda")
        with pytest.raises(gc.GcError) as e:
            ctx.blockmix_encode(d_in, 512, d_k, big[:cap])
        assert e.value.code == gc.ENOSPC
        torch.cuda.synchronize()
        assert torch.all(big[cap:] == -7), cap
    assert ctx.blockmix_encode(d_in, 512, d_k, d_out) == need
