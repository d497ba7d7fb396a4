"""Seeded synthetic posting-list generators.

The paper measures on GOV2, ClueWeb09B, Wikipedia and Twitter posting lists
(Section 7.1); none is available here, so these generators stand in for them.
They reproduce the character the paper reports -- over 90% of d-gaps and TFs
fit in 8 bits, per-term list lengths are heavily skewed -- with fixed seeds.

This module holds no codec arithmetic: it only draws lists.  Both the oracle
tests and the GPU path take their inputs from here.
"""
from __future__ import annotations

import numpy as np

U25 = 1 << 25
MAX_LIST = 1 << 22


def _seg_labels(rng, total, mean_a, mean_b):
    """Alternating segment labels (0 = kind a, 1 = kind b) covering `total`
    positions, segment lengths geometric with the given means, starting with a."""
    lab = np.empty(total, np.uint8)
    pos = 0
    kind = 0
    while pos < total:
        need = max(64, int((total - pos) / (mean_a + mean_b) * 2.2) + 64)
        la = rng.geometric(1.0 / mean_a, need)
        lb = rng.geometric(1.0 / mean_b, need)
        lens = np.empty(2 * need, np.int64)
        kinds = np.empty(2 * need, np.uint8)
        if kind == 0:
            lens[0::2], lens[1::2] = la, lb
            kinds[0::2], kinds[1::2] = 0, 1
        else:
            lens[0::2], lens[1::2] = lb, la
            kinds[0::2], kinds[1::2] = 1, 0
        cum = np.cumsum(lens)
        stop = int(np.searchsorted(cum, total - pos)) + 1
        seg = np.repeat(kinds[:stop], lens[:stop])[: total - pos]
        lab[pos:pos + seg.size] = seg
        pos += seg.size
        kind = int(kinds[stop - 1]) ^ 1
    return lab


def _segmented_cumsum(g, lengths):
    """docIDs per list: cumulative sums restarted at each list start (mod 2^32)."""
    c = np.cumsum(g.astype(np.uint64))
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    base = np.where(starts > 0, c[np.maximum(starts - 1, 0)], 0)
    d = c - np.repeat(base, lengths)
    return (d & 0xFFFFFFFF).astype(np.uint32)


def mixed_gaps(rng, lengths, universe=U25, sparse_frac=0.7, cluster_mean=32):
    """d-gaps for lists of the given lengths: sparse segments (uniform gaps in
    [1, 2m-1], m chosen so a list spans about 90% of the universe) alternate
    with clustered runs (gaps uniform in {1,2,3}, run length geometric with
    mean `cluster_mean`); clustered gaps make up 1 - sparse_frac of the total.
    Lists whose last docID would reach the universe are redrawn."""
    lengths = np.asarray(lengths, np.int64)
    total = int(lengths.sum())
    sparse_mean = cluster_mean * sparse_frac / (1.0 - sparse_frac)
    lab = _seg_labels(rng, total, sparse_mean, cluster_mean)
    Lrep = np.repeat(lengths, lengths).astype(np.float64)
    m = (0.9 * universe - 2.0 * (1 - sparse_frac) * Lrep) / (sparse_frac * Lrep)
    hi = np.maximum(np.floor(2 * m - 1), 1.0)
    u = rng.random(total)
    sparse = 1 + np.floor(u * hi)
    clustered = rng.integers(1, 4, total)
    g = np.where(lab == 0, sparse, clustered).astype(np.uint32)
    # redraw any list whose docIDs would leave the universe
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    for _ in range(200):
        sums = np.add.reduceat(g.astype(np.uint64), starts) if total else np.zeros(0)
        bad = np.nonzero((sums >= universe) & (lengths > 0))[0]
        if bad.size == 0:
            break
        for li in bad:
            s, L = starts[li], lengths[li]
            mm = m[s] if L else 1.0
            gg = 1 + np.floor(rng.random(L) * max(np.floor(2 * mm - 1), 1.0))
            gg = np.where(lab[s:s + L] == 0, gg, rng.integers(1, 4, L))
            if gg.sum() >= universe:
                gg = np.maximum(np.floor(gg * (0.9 * universe / gg.sum())), 1)
            g[s:s + L] = gg.astype(np.uint32)
    return g


def split(flat, lengths):
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    return [flat[offs[i]:offs[i + 1]] for i in range(len(lengths))]


# ---------------------------------------------------------------------------
# Workloads.

def cfg1(seed=1, n=1 << 20, universe=1 << 24):
    """One list of n distinct docIDs drawn uniformly from [0, universe), sorted
    (mean d-gap universe/n = 16)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(universe, n, replace=False)).astype(np.uint32)


def zipf_lengths(nlists, total, lo, hi, rng):
    """Rank-Zipf(s=1) list lengths L_r = clip(round(Cz/r), lo, hi), with Cz
    solved so the lengths sum to about `total`, assigned in shuffled order."""
    r = np.arange(1, nlists + 1, dtype=np.float64)
    a, b = 1.0, float(total) * 4
    for _ in range(100):
        c = 0.5 * (a + b)
        s = np.clip(np.round(c / r), lo, hi).sum()
        if s < total:
            a = c
        else:
            b = c
    L = np.clip(np.round(c / r), lo, hi).astype(np.int64)
    rng.shuffle(L)
    return L


def lognormal_lengths(nlists, median, sigma, hi, rng):
    return np.clip(np.round(np.exp(rng.normal(np.log(median), sigma, nlists))), 1,
                   hi).astype(np.int64)


def cfg2(seed=2, nlists=10_000, total=1 << 26):
    """10,000 docID lists (Zipf lengths in [128, 2^22], about 2^26 postings,
    universe 2^25, 70% sparse / 30% clustered gaps) plus matching TF lists
    (geometric, p = 0.4, values >= 1).  Returns (lengths, docids_flat, tfs_flat)."""
    rng = np.random.default_rng(seed)
    L = zipf_lengths(nlists, total, 128, MAX_LIST, rng)
    g = mixed_gaps(rng, L)
    d = _segmented_cumsum(g, L)
    tf = rng.geometric(0.4, int(L.sum())).astype(np.uint32)
    return L, d, tf


def cfg3(seed=3, nlists=100_000, median=1024, sigma=1.388, ncodecs=5):
    """100,000 docID lists with lognormal lengths (median 1024, about 2^28
    postings in total), the cfg2 gap model, one codec index per list drawn
    uniformly from `ncodecs`.  Returns (lengths, docids_flat, codec_idx)."""
    rng = np.random.default_rng(seed)
    L = lognormal_lengths(nlists, median, sigma, MAX_LIST, rng)
    g = mixed_gaps(rng, L)
    d = _segmented_cumsum(g, L)
    codec = rng.integers(0, ncodecs, nlists)
    return L, d, codec


def block_corpus(seed, total_ints, nlists_hint=10_000):
    """Integers for the learned block selector: lists drawn from the cfg2 model
    (d-gaps and TFs in equal proportion) until `total_ints` values.  Returns
    (lengths, values_flat) where each list is a d-gap list or a TF list."""
    rng = np.random.default_rng(seed)
    per = total_ints // 2
    L = zipf_lengths(nlists_hint, per, 128, MAX_LIST, rng)
    if L.sum() < per:                 # the Zipf fit lands a few values short
        L[np.argmin(L)] += per - L.sum()
    g = mixed_gaps(rng, L)
    tf = rng.geometric(0.4, int(L.sum())).astype(np.uint32)
    lengths = np.concatenate([L, L])
    vals = np.concatenate([g, tf])
    # cut to exactly total_ints values
    cum = np.cumsum(lengths)
    keep = int(np.searchsorted(cum, total_ints)) + 1
    lengths = lengths[:keep].copy()
    excess = int(lengths.sum()) - total_ints
    if excess > 0:
        lengths[-1] -= excess
    vals = vals[:total_ints].copy()
    return lengths, vals


def pareto_gaps(rng, total, alpha=1.2, dense_frac=0.2, dense_mean=128):
    """Heavy-tailed d-gaps: floor(1 + Pareto(alpha)) capped at 2^31 - 1,
    interleaved with dense runs of gap 1 (run length geometric, mean
    `dense_mean`) making up `dense_frac` of all gaps."""
    other_mean = dense_mean * (1 - dense_frac) / dense_frac
    lab = _seg_labels(rng, total, other_mean, dense_mean)
    p = np.floor(1.0 + rng.pareto(alpha, total))
    p = np.minimum(p, float((1 << 31) - 1))
    return np.where(lab == 0, p, 1.0).astype(np.uint32)


def cfg5(seed=6, nlists=1_000_000, median=256, sigma=1.217):
    """1,000,000 lists (lognormal lengths, median 256, about 2^29 postings) of
    heavy-tailed d-gaps; docIDs are wrapping cumulative sums.
    Returns (lengths, docids_flat)."""
    rng = np.random.default_rng(seed)
    L = lognormal_lengths(nlists, median, sigma, MAX_LIST, rng)
    g = pareto_gaps(rng, int(L.sum()))
    d = _segmented_cumsum(g, L)
    return L, d


def doc_lengths(seed=8, ndocs=U25, median=300, sigma=0.8):
    """Length of every document of the collection (for BM25's length
    normalisation): lognormal, median 300 terms, in [1, 65535], uint16."""
    rng = np.random.default_rng(seed)
    x = np.exp(rng.normal(np.log(median), sigma, ndocs))
    return np.clip(np.round(x), 1, 65535).astype(np.uint16)


def queries(lengths, seed=7, nq=1000, min_terms=2, max_terms=4):
    """AND queries over the lists of a collection: 2 to 4 distinct terms
    each, a term drawn with probability proportional to its list's length
    (frequent terms are queried more, as in query logs).  Returns an
    (nq, max_terms) int64 array of list indices, padded with -1."""
    rng = np.random.default_rng(seed)
    p = np.asarray(lengths, np.float64)
    p = p / p.sum()
    out = np.full((nq, max_terms), -1, np.int64)
    for q in range(nq):
        m = int(rng.integers(min_terms, max_terms + 1))
        out[q, :m] = rng.choice(p.size, m, replace=False, p=p)
    return out
