"""AND queries with BM25 top-k on the GPU (gc_query_plan_create /
gc_query_run) over lists decoded by the batched decode path, against the
float64 reference (oracle/query_ref.py).  Scores are single precision on the
GPU: the number of results must match exactly, every returned document must
be in the intersection, and the score at every rank must match the
reference's within a relative 2e-5 (so near-ties may swap documents, but only
between documents whose reference scores agree to that tolerance)."""
import sys

import numpy as np
import pytest

from oracle import query_ref as Q
from paper_1502_01916_amd import gc, synth

pytestmark = pytest.mark.gpu
RTOL = 2e-5


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
def index(torch_cuda):
    """A 2,000-term collection (cfg2 model, 2^22 postings) coded with
    Group-PFD (docIDs) and Group-Simple (TFs), decoded on the GPU by one
    batched plan into docID and TF arenas with equal offsets."""
    torch = torch_cuda
    lengths, docs, tfs = synth.cfg2(seed=12, nlists=2000, total=1 << 22)
    s_d, o_d = gc.encode_lists(docs, lengths, gc.PFD, gc.params(delta=True))
    s_t, o_t = gc.encode_lists(tfs, lengths, gc.SIMPLE, gc.params())
    streams = np.concatenate([s_d, s_t])
    offs = np.concatenate([o_d[:-1], o_t + o_d[-1]]).astype(np.int64)
    L2 = np.concatenate([lengths, lengths])
    descs, headers, out_offs = gc.batch_layout(streams, offs, L2, align=4)
    ctx = gc.Context(0)
    d_s = gc.to_device(streams)
    arena = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    plan = gc.Plan(ctx, descs, headers, d_s, arena, use_graph=True)
    plan.decode_batch(d_s, arena)
    rc, det = ctx.sync_status()
    assert rc == gc.OK, det
    n = lengths.size
    half = int(out_offs[n])
    assert np.array_equal(out_offs[n:2 * n] - half, out_offs[:n])
    term_off = torch.from_numpy(out_offs[:n].astype(np.int64)).cuda()
    doclen = synth.doc_lengths(ndocs=synth.U25)
    d_doclen = torch.from_numpy(doclen.view(np.int16)).cuda()
    lo = np.concatenate([[0], np.cumsum(lengths)])
    doc_lists = [docs[lo[i]:lo[i + 1]] for i in range(n)]
    tf_lists = [tfs[lo[i]:lo[i + 1]] for i in range(n)]
    # the decoded arenas hold the generated lists
    got = gc.to_host(arena)
    assert np.array_equal(gc.unpad(got, out_offs[:n + 1], lengths), docs)
    assert np.array_equal(gc.unpad(got[half:], out_offs[n:] - half, lengths), tfs)
    yield dict(lengths=lengths, doc_lists=doc_lists, tf_lists=tf_lists, arena=arena, half=half,
               term_off=term_off, doclen=doclen, d_doclen=d_doclen, avgdl=float(doclen.mean()))
    plan.close()
    ctx.close()


def run_queries(torch, ix, queries, topk, k1=1.2, b=0.75):
    qp = gc.QueryPlan(ix["lengths"], queries, ix.get("ndocs", synth.U25), ix["avgdl"], topk=topk, k1=k1, b=b)
    nq = queries.shape[0]
    d_doc = torch.empty(nq * topk, dtype=torch.int32, device="cuda")
    d_sc = torch.empty(nq * topk, dtype=torch.float32, device="cuda")
    qp.run(ix["arena"], ix["arena"][ix["half"]:], ix["term_off"], ix["d_doclen"], d_doc, d_sc)
    torch.cuda.synchronize()
    qp.close()
    return gc.to_host(d_doc).reshape(nq, topk), d_sc.cpu().numpy().reshape(nq, topk)


def check(ix, queries, docs, scores, topk, k1=1.2, b=0.75):
    ndocs = ix.get("ndocs", synth.U25)
    for q in range(queries.shape[0]):
        want = Q.and_topk(ix["doc_lists"], ix["tf_lists"], queries[q], ix["doclen"], ndocs, ix["avgdl"],
                          k=topk, k1=k1, b=b)
        n = len(want)
        got_d = docs[q]
        assert np.all(got_d[n:] == 0xFFFFFFFF), (q, "extra results")
        assert np.all(got_d[:n] != 0xFFFFFFFF), (q, "missing results")
        if not n:
            continue
        ws = np.array([s for s, _ in want])
        assert np.allclose(scores[q, :n], ws, rtol=RTOL, atol=0), (q, scores[q, :n], ws)
        # every returned document is in the intersection, with the score of its rank
        terms = [int(t) for t in queries[q] if t >= 0]
        full = {d: s for s, d in Q.and_topk(ix["doc_lists"], ix["tf_lists"], terms, ix["doclen"], ndocs,
                                            ix["avgdl"], k=1 << 30, k1=k1, b=b)}
        for r in range(n):
            d = int(got_d[r])
            assert d in full, (q, r, d)
            assert full[d] == pytest.approx(ws[r], rel=RTOL), (q, r, d)


def test_queries_top10(torch_cuda, index):
    """300 queries of 2 to 4 terms drawn by list length, top-10."""
    queries = synth.queries(index["lengths"], seed=7, nq=300)
    say("queries", queries.shape)
    docs, scores = run_queries(torch_cuda, index, queries, 10)
    check(index, queries, docs, scores, 10)
    hits = int(np.sum(docs != 0xFFFFFFFF))
    say("results", hits)
    assert hits > 300      # the queries are not all empty


def test_queries_edge_cases(torch_cuda, index):
    """Single-term queries (the whole list ranked), empty queries, terms
    that never meet, repeated terms; top-1 and top-64; other BM25
    parameters."""
    L = index["lengths"]
    big = np.argsort(L)[::-1]
    small = np.argsort(L)[:4]
    queries = np.array([[big[0], -1, -1, -1], [small[0], -1, -1, -1], [-1, -1, -1, -1],
                        [big[0], big[1], big[2], big[3]], [small[0], small[1], -1, -1],
                        [big[5], big[0], -1, -1], [big[1], -1, big[7], -1], [big[2], big[2], -1, -1]], np.int64)
    for topk, k1, b in ((1, 1.2, 0.75), (64, 1.2, 0.75), (10, 0.9, 0.4)):
        say("edge topk", topk, k1, b)
        docs, scores = run_queries(torch_cuda, index, queries, topk, k1, b)
        check(index, queries, docs, scores, topk, k1, b)


def test_queries_list_shapes(torch_cuda):
    """A small collection (2^18 documents) of lists shaped to reach every
    search path: empty and one-posting lists, lengths at the 64-docID round
    and 2048-docID segment boundaries, equal lengths (the pivot is the first
    term), a dense run of consecutive docIDs, lists packed at the front or
    the back of the collection (the first probe stride overshoots or falls
    short), every docID (ranges longer than the LDS buffer, searched in
    global memory); every ordered pair of lists, then triples and quads."""
    torch = torch_cuda
    rng = np.random.default_rng(31)
    nd = 1 << 18

    def spread(n, lo=0, hi=nd):
        return np.sort(rng.choice(np.arange(lo, hi), n, replace=False)).astype(np.uint32)

    doc_lists = [np.zeros(0, np.uint32), np.array([5], np.uint32), spread(64), spread(65), spread(1025),
                 spread(1025), spread(8193), np.arange(100000, 116384, dtype=np.uint32), spread(120000),
                 np.arange(nd, dtype=np.uint32), spread(3000, 0, 5000), spread(3000, nd - 12000, nd),
                 spread(8192), spread(8191), spread(2048), spread(2049)]
    # a list of clusters: runs of 40 consecutive docIDs
    starts = np.sort(rng.choice(nd // 64, 300, replace=False)) * 64
    doc_lists.append((starts[:, None] + np.arange(40)).ravel().astype(np.uint32))
    tf_lists = [rng.integers(1, 21, x.size).astype(np.uint32) for x in doc_lists]
    lengths = np.array([x.size for x in doc_lists], np.int64)
    offs = np.concatenate([[0], np.cumsum(lengths)])
    arena_d = gc.to_device(np.concatenate(doc_lists))
    arena_t = gc.to_device(np.concatenate(tf_lists))
    doclen = synth.doc_lengths(seed=9, ndocs=nd)
    ix = dict(lengths=lengths, doc_lists=doc_lists, tf_lists=tf_lists, arena=None, ndocs=nd,
              doclen=doclen, avgdl=float(doclen.mean()))
    n = lengths.size
    qs = [[i, j, -1, -1] for i in range(n) for j in range(n) if i != j]
    qs += [list(rng.choice(n, 3, replace=False)) + [-1] for _ in range(40)]
    qs += [list(rng.choice(n, 4, replace=False)) for _ in range(40)]
    qs += [[9, 9, 8, -1], [8, 9, 7, 6], [-1, 9, -1, 4], [0, 9, -1, -1], [9, -1, -1, -1], [16, 9, 8, 12],
           [14, 15, 9, -1], [15, 14, 6, -1]]
    queries = np.array(qs, np.int64)
    term_off = torch.from_numpy(offs[:-1].astype(np.int64)).cuda()
    d_doclen = torch.from_numpy(doclen.view(np.int16)).cuda()
    for topk in (10, 64):
        say("shapes topk", topk, "queries", queries.shape)
        qp = gc.QueryPlan(lengths, queries, nd, ix["avgdl"], topk=topk)
        nq = queries.shape[0]
        d_doc = torch.empty(nq * topk, dtype=torch.int32, device="cuda")
        d_sc = torch.empty(nq * topk, dtype=torch.float32, device="cuda")
        qp.run(arena_d, arena_t, term_off, d_doclen, d_doc, d_sc)
        torch.cuda.synchronize()
        qp.close()
        docs = gc.to_host(d_doc).reshape(nq, topk)
        scores = d_sc.cpu().numpy().reshape(nq, topk)
        check(ix, queries, docs, scores, topk)
