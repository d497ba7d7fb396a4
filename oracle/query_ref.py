"""Plain CPU reference for AND queries with BM25 top-k -- TEST
INFRASTRUCTURE ONLY (imported by the tests and bench.py's checks, never by
the library).

Query processing as Section 7.4 describes it: an AND query keeps the
documents that appear in every one of its terms' posting lists; each is
scored with Okapi BM25 and the k best are returned (k = 10 in the paper).
Written in float64 numpy, term by term, so it can be read against the
definitions:

  idf(t)       = ln(1 + (N - df_t + 0.5) / (df_t + 0.5))
  w(t, d)      = idf(t) * tf * (k1 + 1) / (tf + k1 * (1 - b + b * dl_d / avgdl))
  score(q, d)  = sum over the terms t of q of w(t, d)

with df_t the length of t's list, tf the term frequency of t in d (its TF
list, aligned with the docID list), dl_d the document length and N the
number of documents.  The paper gives no BM25 parameters: k1 = 1.2 and
b = 0.75 (Robertson's usual values) unless stated.  Ranking: higher score
first, then smaller docID.
"""
from __future__ import annotations

import math

import numpy as np


def idf(df, ndocs):
    return math.log(1.0 + (ndocs - df + 0.5) / (df + 0.5))


def term_weight(tf, dl, idf_t, avgdl, k1=1.2, b=0.75):
    return idf_t * tf * (k1 + 1.0) / (tf + k1 * (1.0 - b + b * dl / avgdl))


def and_topk(doc_lists, tf_lists, terms, doclen, ndocs, avgdl, k=10, k1=1.2, b=0.75):
    """One AND query: `terms` are indices into doc_lists / tf_lists (sorted
    docID lists without repeats, and their TF lists).  Returns [(score,
    docid), ...], best first, at most k entries.  The intersection is a
    library set operation (numpy.intersect1d); the scores are float64."""
    terms = [int(t) for t in terms if t >= 0]
    if not terms:
        return []
    common = np.asarray(doc_lists[terms[0]], dtype=np.int64)
    for t in terms[1:]:
        common = np.intersect1d(common, np.asarray(doc_lists[t], dtype=np.int64), assume_unique=True)
    if common.size == 0:
        return []
    score = np.zeros(common.size, np.float64)
    dl = np.asarray(doclen, dtype=np.float64)[common]
    for t in terms:
        docs = np.asarray(doc_lists[t], dtype=np.int64)
        where = np.searchsorted(docs, common)
        tf = np.asarray(tf_lists[t], dtype=np.float64)[where]
        i = idf(docs.size, ndocs)
        score += i * tf * (k1 + 1.0) / (tf + k1 * (1.0 - b + b * dl / avgdl))
    order = np.lexsort((common, -score))[:k]
    return [(float(score[j]), int(common[j])) for j in order]
