"""Pins of the AND / BM25 top-k reference (oracle/query_ref.py): special
cases of BM25 that reduce to closed forms, its monotonicity and limit, the
intersection against a brute-force scan of every document, and the ranking
rule (score, then smaller docID)."""
import math

import numpy as np
import pytest

from oracle import query_ref as Q


def test_idf_closed_form_and_sign():
    # N = 10, df = 2: ln(1 + 8.5 / 2.5) = ln(4.4)
    assert Q.idf(2, 10) == pytest.approx(math.log(4.4), rel=1e-15)
    # never negative, even for a term in every document; decreasing in df
    assert Q.idf(10, 10) > 0
    assert Q.idf(1, 1000) > Q.idf(2, 1000) > Q.idf(500, 1000)


def test_weight_special_cases():
    i = 2.5
    # b = 0: no length normalisation, tf (k1 + 1) / (tf + k1)
    assert Q.term_weight(3, 123.0, i, 500.0, k1=1.2, b=0.0) == pytest.approx(i * 3 * 2.2 / (3 + 1.2))
    # a document of average length with tf = 1 weighs exactly idf
    assert Q.term_weight(1, 500.0, i, 500.0, k1=1.2, b=0.75) == pytest.approx(i)
    # k1 = 0: the term frequency is ignored
    assert Q.term_weight(7, 80.0, i, 500.0, k1=0.0, b=0.75) == pytest.approx(i)
    # increasing in tf towards idf (k1 + 1); longer documents weigh less
    w = [Q.term_weight(t, 300.0, i, 250.0) for t in (1, 2, 5, 50, 5000)]
    assert all(a < b for a, b in zip(w, w[1:])) and w[-1] < i * 2.2 and w[-1] == pytest.approx(i * 2.2, rel=1e-3)
    assert Q.term_weight(3, 100.0, i, 250.0) > Q.term_weight(3, 900.0, i, 250.0)


def test_intersection_and_scores_against_brute_force():
    rng = np.random.default_rng(5)
    ndocs = 400
    doclen = rng.integers(1, 1000, ndocs).astype(np.uint16)
    docs = [np.sort(rng.choice(ndocs, n, replace=False)) for n in (150, 220, 90, 300)]
    tfs = [rng.integers(1, 9, d.size) for d in docs]
    avgdl = float(doclen.mean())
    for terms in ([0, 1], [0, 1, 2], [3, 2, 1, 0], [2]):
        got = Q.and_topk(docs, tfs, terms, doclen, ndocs, avgdl, k=400)
        # brute force: every document, every term, in plain loops
        want = []
        for d in range(ndocs):
            s = 0.0
            hit = True
            for t in terms:
                pos = [j for j, x in enumerate(docs[t]) if x == d]
                if not pos:
                    hit = False
                    break
                df = len(docs[t])
                idf = math.log(1 + (ndocs - df + 0.5) / (df + 0.5))
                tf = float(tfs[t][pos[0]])
                s += idf * tf * 2.2 / (tf + 1.2 * (0.25 + 0.75 * float(doclen[d]) / avgdl))
            if hit:
                want.append((s, d))
        want.sort(key=lambda x: (-x[0], x[1]))
        assert [d for _, d in got] == [d for _, d in want]
        assert np.allclose([s for s, _ in got], [s for s, _ in want], rtol=1e-12)


def test_ranking_ties_and_truncation():
    # two documents with identical postings and lengths tie: the smaller
    # docID ranks first; k cuts the list
    docs = [np.array([3, 8, 12]), np.array([3, 8, 12, 40])]
    tfs = [np.array([2, 2, 5]), np.array([1, 1, 1, 1])]
    doclen = np.full(64, 100, np.uint16)
    r = Q.and_topk(docs, tfs, [0, 1], doclen, 64, 100.0, k=2)
    assert [d for _, d in r] == [12, 3]
    assert Q.and_topk(docs, tfs, [0, 1], doclen, 64, 100.0, k=10)[1:] == [
        (r[1][0], 3), (r[1][0], 8)]
    assert Q.and_topk(docs, tfs, [], doclen, 64, 100.0) == []
    assert Q.and_topk([np.array([1]), np.array([2])], [np.array([1]), np.array([1])], [0, 1], doclen, 64, 100.0) == []
