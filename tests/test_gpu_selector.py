"""The learned per-block codec selector at full size: trained on the GPU by
the library's own kernels on 2^26 integers of the d-gap/TF corpus (seed 4)
with labels from the exhaustive search, evaluated on 2^27 held-out integers
(seed 5).  Checks: the labels agree with the oracle's exhaustive search,
the learned container is within 1% of the exhaustive one, it is word for
word the oracle's container for the same classes and decodes exactly, it
beats the methods without the network (the best single class, an untrained
network), and the learned encoder is faster than the exhaustive one."""
import sys
import time

import numpy as np
import pytest

import oracle as O
from paper_1502_01916_amd import gc, selector, synth

pytestmark = pytest.mark.gpu

TRAIN_INTS, EVAL_INTS = 1 << 26, 1 << 27
TRAIN = dict(epochs=400, batch=4096, lr=1e-2, lr_final=1e-3, lam=16.0, seed=0)


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
    c = gc.Context(0, max_list_ints=EVAL_INTS)
    yield c
    c.close()


@pytest.fixture(scope="module")
def data(torch_cuda, ctx):
    say("selector corpora: train 2^26 (seed 4), eval 2^27 (seed 5)")
    _, tr = synth.block_corpus(4, TRAIN_INTS)
    _, ev = synth.block_corpus(5, EVAL_INTS)
    d_tr, d_ev = gc.to_device(tr), gc.to_device(ev)
    T = selector.Targets(ctx, d_tr, tr.size // gc.BLOCK_INTS)
    return tr, ev, d_tr, d_ev, T


@pytest.fixture(scope="module")
def trained(data, ctx):
    _, _, _, _, T = data
    say("selector training %s" % TRAIN)
    model, losses, secs = selector.train(ctx, T, **TRAIN)
    say("trained in %.2f s, loss %.4f -> %.4f" % (secs, losses[0], losses[-1]))
    yield model
    model.close()


def test_labels_are_the_oracle_search(data):
    tr, _, _, _, T = data
    rng = np.random.default_rng(0)
    pick = rng.choice(T.n, 3000, replace=False)
    best = T.best.cpu().numpy()
    cost = T.cost.cpu().numpy()
    feat = T.feat.cpu().numpy()
    x = tr.reshape(-1, 128)
    for b in pick:
        kb, sizes = O.block_best(x[b])
        assert best[b] == kb
        smin = sizes.min()
        assert np.array_equal(cost[b], (sizes - smin).astype(np.float32) / np.float32(smin))
        assert np.array_equal(feat[b].astype(np.float64), O.block_features(x[b]))


def test_learned_within_one_percent(torch_cuda, ctx, data, trained):
    torch = torch_cuda
    _, ev, _, d_ev, _ = data
    d_out, used_l, cls = selector.encode(ctx, d_ev, ev.size, gc.SELECT_LEARNED, model=trained, with_classes=True)
    _, used_e = selector.encode(ctx, d_ev, ev.size, gc.SELECT_EXHAUSTIVE)
    ratio = used_l / used_e
    say("learned %d words, exhaustive %d words: ratio %.5f (%.3f bits/int learned)" %
        (used_l, used_e, ratio, 32.0 * used_l / ev.size))
    assert ratio <= 1.01
    # the same container as the oracle writes for these classes, and it decodes exactly
    k = cls.cpu().numpy()
    got = gc.to_host(d_out)[:used_l]
    want, _ = O.blockmix_encode(ev, k)
    assert np.array_equal(got, want)
    assert np.array_equal(O.blockmix_decode(got), ev)


def test_gain_over_no_network(torch_cuda, ctx, data, trained):
    """Without the network: one class for every block (the best of the 16 in
    hindsight), or the untrained network's choices."""
    _, ev, _, d_ev, _ = data
    _, used_l = selector.encode(ctx, d_ev, ev.size, gc.SELECT_LEARNED, model=trained)
    fixed = [selector.encode(ctx, d_ev, ev.size, gc.SELECT_FIXED, fixed_class=k)[1] for k in range(16)]
    best_fixed = min(fixed)
    untrained = gc.Mlp(ctx, 4096)
    untrained.set_params(selector.init_params(TRAIN["seed"]))
    _, used_u = selector.encode(ctx, d_ev, ev.size, gc.SELECT_LEARNED, model=untrained)
    untrained.close()
    say("learned %d, best fixed class %d (class %d, %.4fx), untrained network %d (%.4fx)" %
        (used_l, best_fixed, int(np.argmin(fixed)), best_fixed / used_l, used_u, used_u / used_l))
    assert used_l * 1.05 < best_fixed
    assert used_l * 1.05 < used_u


def test_learned_encoder_faster(torch_cuda, ctx, data, trained):
    torch = torch_cuda
    _, ev, _, d_ev, _ = data

    def best_time(mode):
        times = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            selector.encode(ctx, d_ev, ev.size, mode, model=trained)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return min(times)

    t_l, t_e = best_time(gc.SELECT_LEARNED), best_time(gc.SELECT_EXHAUSTIVE)
    say("encode 2^27 ints: learned %.2f ms (%.1f Gints/s), exhaustive %.2f ms (%.1f Gints/s)" %
        (t_l * 1e3, ev.size / t_l / 1e9, t_e * 1e3, ev.size / t_e / 1e9))
    assert t_l < t_e
