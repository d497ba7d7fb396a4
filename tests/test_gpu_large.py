"""Full-size batched decoding of the two large workloads, in the launch
configuration of the benchmark (one hipGraph-captured plan per batch):

* 100,000 lognormal-length lists (about 2^28 docIDs, cfg2 gap model), each
  with one of five codecs, decoded in one batch and with one launch sequence
  per list;
* 1,000,000 lognormal-length lists (about 2^29 docIDs) of heavy-tailed
  Pareto d-gaps, Group-PFD and Group-AFOR in the 4-way and the 64-way layouts.

Every decoded list equals the generated list (the lossless-codec property,
checkable at any size); on sampled lists the stream equals the oracle's
encoding and the output the oracle's decoding."""
import sys
import time

import numpy as np
import pytest

import oracle as O
from paper_1502_01916_amd import gc, synth

pytestmark = pytest.mark.gpu

CFG2_CODECS = [(gc.SIMPLE, {}), (gc.SCHEME, dict(cg=1, ld=gc.LD_CU)), (gc.SCHEME, dict(cg=8, ld=gc.LD_IU)),
               (gc.AFOR, {}), (gc.PFD, {})]


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


def oracle_params(codec, kw):
    return O.params(codec, k=kw.get("k", 4), cg=kw.get("cg", 1), ld=kw.get("ld", O.LD_CU), delta=True,
                    pfd_pos=kw.get("pfd_pos", O.PFD_LINKED))


def check_sample(flat, lengths, s, offs, got_flat, params_of, nsample, seed):
    lo = np.concatenate([[0], np.cumsum(lengths)])
    pick = np.random.default_rng(seed).choice(lengths.size, nsample, replace=False)
    pick = np.concatenate([pick, [int(np.argmax(lengths))]])     # the longest list too
    for i in pick:
        seg = s[int(offs[i]):int(offs[i + 1])]
        lst = flat[lo[i]:lo[i + 1]]
        assert np.array_equal(seg, O.encode(lst, params_of(i))), i
        assert np.array_equal(got_flat[lo[i]:lo[i + 1]], O.decode(seg)), i


def test_cfg3_batched_and_per_list(torch_cuda, ctx):
    torch = torch_cuda
    say("cfg3: generating 100,000 lists")
    lengths, docs, cidx = synth.cfg3()
    codecs = np.array([CFG2_CODECS[c][0] for c in cidx], np.int32)
    plist = [gc.params(delta=True, **CFG2_CODECS[c][1]) for c in cidx]
    s, offs = gc.encode_lists(docs, lengths, codecs, plist)
    descs, headers, out_offs = gc.batch_layout(s, offs, lengths, align=4)
    say("cfg3: %d ints, %.3f bits/int" % (docs.size, 32.0 * s.size / docs.size))
    d_s = gc.to_device(s)
    d_o = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, use_graph=True, autotune=True)
    say("cfg3: plan %s" % plan.config())
    plan.decode_batch(d_s, d_o)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    got = gc.unpad(gc.to_host(d_o), out_offs, lengths)
    assert np.array_equal(got, docs)
    check_sample(docs, lengths, s, offs, got, lambda i: oracle_params(*CFG2_CODECS[cidx[i]]), 25, 3)
    del got
    # timing: one batched replay against one launch sequence per list
    for _ in range(3):
        plan.decode_batch(d_s, d_o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        plan.decode_batch(d_s, d_o)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / 10
    d_o.fill_(-1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.decode_each(d_s, d_o)
    torch.cuda.synchronize()
    t_each = time.perf_counter() - t0
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    assert np.array_equal(gc.unpad(gc.to_host(d_o), out_offs, lengths), docs)
    say("cfg3: batched %.2f ms (%.1f Gints/s), per-list %.1f ms (%.2f Gints/s): %.1fx" %
        (t_batch * 1e3, docs.size / t_batch / 1e9, t_each * 1e3, docs.size / t_each / 1e9, t_each / t_batch))
    assert t_each >= 3 * t_batch
    plan.close()


@pytest.fixture(scope="module")
def cfg5_data():
    say("cfg5: generating 1,000,000 lists")
    return synth.cfg5()


@pytest.mark.parametrize("name,codec,kw", [
    ("pfd-k4", gc.PFD, dict(k=4)),
    ("afor-k4", gc.AFOR, dict(k=4)),
    ("pfd-k64", gc.PFD, dict(k=64, pfd_pos=gc.PFD_BITMAP)),
    ("afor-k64", gc.AFOR, dict(k=64)),
])
def test_cfg5_full_size(torch_cuda, ctx, cfg5_data, name, codec, kw):
    torch = torch_cuda
    lengths, docs = cfg5_data
    say("cfg5 %s: encoding %d ints" % (name, docs.size))
    s, offs = gc.encode_lists(docs, lengths, codec, gc.params(delta=True, **kw))
    descs, headers, out_offs = gc.batch_layout(s, offs, lengths, align=4)
    d_s = gc.to_device(s)
    d_o = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, use_graph=True, autotune=True)
    say("cfg5 %s: %.3f bits/int, plan %s" % (name, 32.0 * s.size / docs.size, plan.config()))
    plan.decode_batch(d_s, d_o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        plan.decode_batch(d_s, d_o)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    got = gc.unpad(gc.to_host(d_o), out_offs, lengths)
    assert np.array_equal(got, docs)
    say("cfg5 %s: %.2f ms per batch, %.1f Gints/s" % (name, dt * 1e3, docs.size / dt / 1e9))
    op = oracle_params(codec, kw)
    check_sample(docs, lengths, s, offs, got, lambda i: op, 20, 6)
    plan.close()
    del got, d_s, d_o
