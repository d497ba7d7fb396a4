// query.hip -- AND queries with Okapi BM25 top-k over decoded posting lists.
//
// The consumer of the decoded lists (Section 7.4): an AND query keeps the
// documents present in every one of its terms' lists, scores each with
// BM25 and returns the k best.  The lists are decoded by the batched decode
// path (docIDs prefix-summed, TFs) into device arenas.  A query plan cuts
// every query's shortest list (the pivot) into segments of 2048 docIDs, one
// work item each, so long queries spread over many waves:
//   - a wave takes the pivot's docIDs of its segment 64 at a time, one per
//     lane;
//   - the other terms are taken shortest list first (the most selective
//     first), and a term is skipped once no lane's docID is left;
//   - each other term finds where its postings of the round's docIDs end,
//     galloping from where the previous round's ended (the pivot's docIDs
//     increase) by 64 parallel probes a step, with a first stride set by
//     the two lists' length ratio; a range of up to 1024 postings is copied
//     to LDS and each lane searches it there, a longer one is searched in
//     global memory, first over its block heads, one every 512 postings
//     (the paper's skip pointers), then inside the block;
//   - a document found in every list is scored (single precision; its
//     length and the pivot's TF are read only then) and
//     offered to the wave's top-k, kept sorted in LDS (higher score first,
//     then the smaller docID);
// then the segments' top-k lists of each query are merged as a tree, up
// to 64 lists a node, one wave per node.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "gc.h"

namespace gcq {

typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) uint16_t gu16;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kMaxTerms = 8;
constexpr uint32_t kMaxTopk = 64;
constexpr uint32_t kSkip = 512;     // postings between skip pointers
constexpr uint32_t kSeg = 2048;     // pivot docIDs per work item
constexpr uint32_t kLdsRange = 1024; // postings of one term's range searched in LDS

// A work item: pivot docIDs [s0, s1) of query q.
struct QItem {
    uint32_t q, s0, s1, pad;
};

struct QArgs {
    const uint32_t *docs, *tfs;
    const uint64_t *term_off;
    const uint32_t *term_len;
    const int32_t *qterms;
    const uint16_t *doclen;
    const QItem *items;
    const uint32_t *first;      // per query: its first item (nq + 1 entries)
    uint32_t *part_doc;         // per item: topk docIDs, then its count at [nitems * topk + item]
    float *part_score;
    uint32_t *out_doc;
    float *out_score;
    uint32_t tpq, nq, nitems, ndocs, topk;
    float avgdl, k1, b;
};

__device__ __forceinline__ float bm25_weight(uint32_t tf, uint32_t dl, float idf, const QArgs &a) {
    const float t = (float)tf;
    return idf * t * (a.k1 + 1.0f) / (t + a.k1 * (1.0f - a.b + a.b * (float)dl / a.avgdl));
}

// First index p in [lo, n) with v[p] >= key (n if none): the block heads
// v[512 j] inside [lo, n) first, then the postings of one block.
__device__ __forceinline__ uint32_t skip_lower_bound(const gu32 *v, uint32_t lo, uint32_t n, uint32_t key) {
    uint32_t l = lo, r = n;
    const uint32_t j0 = (l + kSkip - 1u) / kSkip;
    uint32_t jl = j0, jr = (r + kSkip - 1u) / kSkip;   // heads kSkip * j, j in [jl, jr), lie in [l, r)
    while (jl < jr) {
        const uint32_t m = (jl + jr) >> 1;
        if (v[kSkip * m] < key) jl = m + 1u;
        else jr = m;
    }
    if (jl > j0) l = max(l, kSkip * (jl - 1u) + 1u);    // heads before jl are below the key
    if (kSkip * jl < r) r = kSkip * jl;                  // head jl is not
    while (l < r) {
        const uint32_t m = (l + r) >> 1;
        if (v[m] < key) l = m + 1u;
        else r = m;
    }
    return l;
}

// For a wave-uniform key, the first index p in [lo, hi) with v[p] >= key
// (hi if none), or, once some e with p <= e has e - lo <= span, that e:
// each step probes 64 positions and keeps the gap between the last probe
// below the key and the first at or above it, so a range of 2^20 postings
// takes four dependent loads.  The first step's stride is at most
// `stride0`: a caller that expects the answer near lo gallops from it.
__device__ __forceinline__ uint32_t probe_lower_bound(const gu32 *v, const uint32_t lo, uint32_t hi, uint32_t key,
                                                      uint32_t lane, uint32_t stride0, uint32_t span = 0u) {
    uint32_t l = lo;
    uint32_t stride = min(stride0, (hi - l + 63u) >> 6);
    while (hi - l > 64u) {
        if (hi - lo <= span) return hi;
        const uint32_t pos = l + lane * stride;
        // a probe past the range counts as at or above the key
        const uint64_t b = __ballot(pos >= hi || v[pos] >= key);
        // lane 0 probes inside the range; with no lane at or above the key
        // the answer lies after lane 63's probe
        const uint32_t f = b ? (uint32_t)__builtin_ctzll(b) : 64u;
        const uint32_t nl = f ? l + (f - 1u) * stride + 1u : l;
        hi = f < 64u ? min(l + f * stride, hi) : hi;
        l = nl;
        stride = (hi - l + 63u) >> 6;
    }
    if (hi - lo <= span) return hi;
    const uint32_t pos = l + lane;
    const uint64_t b = __ballot(pos < hi && v[pos] >= key);
    return b ? l + (uint32_t)__builtin_ctzll(b) : hi;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Offers (s, d) to a sorted top-k of `count` entries (lane 0 writes):
// after the entries of equal or higher score, since documents are offered
// in increasing docID order.  Returns the new count.
__device__ __forceinline__ uint32_t topk_insert(float *sc, uint32_t *dc, uint32_t count, uint32_t topk, float s,
                                                uint32_t d, uint32_t lane) {
    if (lane == 0) {
        uint32_t pos = count;
        while (pos > 0 && s > sc[pos - 1]) pos--;
        const uint32_t lim = min(count, topk - 1u);
        for (uint32_t r = lim; r > pos; r--) {
            sc[r] = sc[r - 1];
            dc[r] = dc[r - 1];
        }
        if (pos < topk) {
            sc[pos] = s;
            dc[pos] = d;
        }
    }
    wave_sync_lds();
    return min(count + 1u, topk);
}

// One wave per work item: its pivot docIDs found in every other list,
// scored, into the item's top-k.  The kernel waits on chains of dependent
// loads, so it is held to at least five waves per SIMD (it takes 78 VGPRs
// and runs six; with four it ran 20% slower).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_and_topk(QArgs a) {
    __shared__ float s_sc[kWaves][kMaxTopk];
    __shared__ uint32_t s_dc[kWaves][kMaxTopk];
    __shared__ uint32_t s_rng[kWaves][kLdsRange];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t w = blockIdx.x * (uint32_t)kWaves + wave;
    if (w >= a.nitems) return;
    float *sc = s_sc[wave];
    uint32_t *dc = s_dc[wave];
    uint32_t *rng = s_rng[wave];
    const QItem it = a.items[w];
    // lane i < tpq: term i of the query
    const int32_t t = lane < a.tpq ? a.qterms[(uint64_t)it.q * a.tpq + lane] : -1;
    const bool valid = t >= 0;
    const uint32_t len = valid ? a.term_len[t] : 0u;
    const uint64_t off = valid ? a.term_off[t] : 0u;
    const float idf = valid ? logf(1.0f + ((float)a.ndocs - (float)len + 0.5f) / ((float)len + 0.5f)) : 0.0f;
    const uint64_t vb = __ballot(valid);
    const uint32_t nterms = (uint32_t)__builtin_popcountll(vb);
    // the terms by increasing list length (the first of equal lengths
    // first): the shortest is the pivot, and the next shortest, the most
    // selective, is searched first
    uint32_t rank = 0;
#pragma unroll
    for (uint32_t i = 0; i < kMaxTerms; i++) {
        const uint32_t li = (uint32_t)__shfl((int)len, (int)i);
        rank += ((vb >> i) & 1ull) && (li < len || (li == len && i < lane)) ? 1u : 0u;
    }
    uint32_t ord[kMaxTerms];
#pragma unroll
    for (uint32_t r = 0; r < kMaxTerms; r++) {
        const uint64_t b = __ballot(valid && rank == r);
        ord[r] = b ? (uint32_t)__builtin_ctzll(b) : 0u;
    }
    const uint32_t piv = ord[0];
    const uint32_t mlen = (uint32_t)__shfl((int)len, (int)piv);
    const uint64_t offp = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(off >> 32), (int)piv) << 32) |
                          (uint32_t)__shfl((int)(uint32_t)off, (int)piv);
    const float idfp = __shfl(idf, (int)piv);
    const uint32_t s1 = nterms ? min(it.s1, mlen) : 0u;
    // per other term (by rank): where the next round's range starts, and
    // the stride of the first probe for its end, twice the postings
    // expected between two pivot docIDs
    uint32_t from[kMaxTerms], hint[kMaxTerms];
    float idfr[kMaxTerms];
#pragma unroll
    for (uint32_t r = 0; r < kMaxTerms; r++) {
        const uint64_t lj = (uint32_t)__shfl((int)len, (int)ord[r]), ml = max(mlen, 1u);
        idfr[r] = __shfl(idf, (int)ord[r]);
        from[r] = 0;
        hint[r] = (uint32_t)max<uint64_t>(1u, (2u * lj + ml - 1u) / ml);
    }
    // terms whose `from` may lie before the round's first docID (all at
    // first; later the terms skipped in a round)
    uint32_t lag = ~0u;
    uint32_t count = 0;
    float thr = -1.0f;
    for (uint32_t base = it.s0; base < s1; base += 64u) {
        const uint32_t i = base + lane;
        const bool in = i < s1;
        const uint32_t d = in ? ((const gu32 *)a.docs)[offp + i] : 0xFFFFFFFFu;
        bool ok = in && d < a.ndocs;
        const uint32_t last = min(63u, s1 - base - 1u);
        const uint32_t d0 = (uint32_t)__shfl((int)d, 0), dlast = (uint32_t)__shfl((int)d, (int)last);
        uint32_t tfr[kMaxTerms];
#pragma unroll
        for (uint32_t r = 1; r < kMaxTerms; r++) {
            tfr[r] = 0;
            if (r >= nterms) break;
            if (!__ballot(ok)) {   // no candidate left in the round
                lag |= 1u << r;
                continue;
            }
            const uint32_t j = ord[r];
            const uint32_t lj = (uint32_t)__shfl((int)len, (int)j);
            const uint64_t oj = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(off >> 32), (int)j) << 32) |
                                (uint32_t)__shfl((int)(uint32_t)off, (int)j);
            const gu32 *v = (const gu32 *)a.docs + oj;
            // the postings of list j from the round's first docID to its
            // last (inclusive) hold each lane's docID or not at all: they
            // start at lo and end at or before hi, and are searched in LDS
            // if up to kLdsRange postings reach them
            uint32_t lo = min(from[r], lj);
            if ((lag >> r) & 1u) {
                lo = probe_lower_bound(v, lo, lj, d0, lane, 0xFFFFFFFFu);
                lag &= ~(1u << r);
            }
            const uint32_t hi =
                dlast == 0xFFFFFFFFu ? lj : probe_lower_bound(v, lo, lj, dlast + 1u, lane, hint[r], kLdsRange);
            const uint32_t n = hi - lo;
            uint32_t p;
            bool found;
            if (n <= kLdsRange) {
                for (uint32_t x = lane; x < n; x += 64u) rng[x] = v[lo + x];
                wave_sync_lds();
                uint32_t l = 0, cnt = n;   // first l with rng[l] >= d
                while (cnt) {
                    const uint32_t half = cnt >> 1;
                    const bool below = rng[l + half] < d;
                    l = below ? l + half + 1u : l;
                    cnt = below ? cnt - half - 1u : half;
                }
                found = l < n && rng[l] == d;
                p = lo + l;
                // the next round starts past the last lane's docID
                from[r] = lo + (uint32_t)__shfl((int)(l + (found ? 1u : 0u)), (int)last);
                found = found && ok;
                wave_sync_lds();   // the buffer is refilled for the next term
            } else {
                p = ok ? skip_lower_bound(v, lo, hi, d) : hi;
                found = ok && p < hi && v[p] == d;
                from[r] = hi;
            }
            if (found) tfr[r] = ((const gu32 *)a.tfs)[oj + p];
            ok = found;
        }
        // documents in every list: BM25 over the pivot and the other terms
        float score = 0.0f;
        if (ok) {
            const uint32_t dl = ((const gu16 *)a.doclen)[d];
            score = bm25_weight(((const gu32 *)a.tfs)[offp + i], dl, idfp, a);
#pragma unroll
            for (uint32_t r = 1; r < kMaxTerms; r++)
                if (r < nterms) score += bm25_weight(tfr[r], dl, idfr[r], a);
        }
        // offer the round's documents to the top-k, in docID order
        const float cand = ok ? score : -1.0f;
        uint64_t m = __ballot(ok && cand > thr);
        while (m) {
            const uint32_t l = (uint32_t)__builtin_ctzll(m);
            count = topk_insert(sc, dc, count, a.topk, __shfl(cand, (int)l), (uint32_t)__shfl((int)d, (int)l), lane);
            thr = count == a.topk ? sc[a.topk - 1u] : -1.0f;
            m &= m - 1u;
            m &= __ballot(ok && cand > thr);
        }
    }
    for (uint32_t r = lane; r < a.topk; r += 64u) {
        a.part_doc[(uint64_t)w * a.topk + r] = r < count ? dc[r] : 0xFFFFFFFFu;
        a.part_score[(uint64_t)w * a.topk + r] = r < count ? sc[r] : 0.0f;
    }
    if (lane == 0) a.part_doc[(uint64_t)a.nitems * a.topk + w] = count;
}

// Whether (s1, d1) ranks before (s2, d2): the higher score, then the
// smaller docID.
__device__ __forceinline__ bool ranks_before(float s1, uint32_t d1, float s2, uint32_t d2) {
    return s1 > s2 || (s1 == s2 && d1 < d2);
}

constexpr uint32_t kMergeBuf = 1024;   // list entries a wave holds in LDS

// Lists merged by one wave: up to 64, at most 1024 entries.
__host__ __device__ constexpr uint32_t merge_group(uint32_t topk) {
    return 64u < kMergeBuf / topk ? 64u : kMergeBuf / topk;
}

// One level of the merge of a query's item lists (each sorted), as a tree:
// the lists stand at the query's item slots first, first + stride, ...; the
// wave of a group's first slot w merges the group's lists (slots w, w +
// stride, ..., up to merge_group(topk) of them, copied to LDS) and writes
// the result to slot w.  Lane l follows list l, and each of the next top-k
// is the best of the lanes' heads (a wave-wide arg-max).
__global__ __launch_bounds__(kThreads) void k_merge_level(QArgs a, uint32_t stride) {
    __shared__ float s_ns[kWaves][kMaxTopk];
    __shared__ uint32_t s_nd[kWaves][kMaxTopk];
    __shared__ float s_bs[kWaves][kMergeBuf];
    __shared__ uint32_t s_bd[kWaves][kMergeBuf];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t w = blockIdx.x * (uint32_t)kWaves + wave;
    if (w >= a.nitems) return;
    const uint32_t topk = a.topk, G = merge_group(topk);
    const uint32_t q = a.items[w].q, f0 = a.first[q], f1 = a.first[q + 1];
    if ((w - f0) % (stride * G) != 0u) return;   // not a group's first slot
    const uint32_t ng = min(G, (f1 - w + stride - 1u) / stride);
    if (ng < 2u) return;   // a lone list stays as it is
    float *bs = s_bs[wave], *ns = s_ns[wave];
    uint32_t *bd = s_bd[wave], *nd = s_nd[wave];
    // all of the group's loads issued before the first is waited for
#pragma unroll
    for (uint32_t r = 0; r < kMergeBuf / 64u; r++) {
        const uint32_t x = 64u * r + lane;
        if (x < ng * topk) {
            const uint32_t l = x / topk, j = x - l * topk;
            const uint64_t at = (uint64_t)(w + l * stride) * topk + j;
            bs[x] = a.part_score[at];
            bd[x] = a.part_doc[at];
        }
    }
    const uint32_t n = lane < ng ? a.part_doc[(uint64_t)a.nitems * topk + w + lane * stride] : 0u;
    wave_sync_lds();
    uint32_t h = 0, out = 0;
    while (out < topk) {
        // the best head over the lanes; a lane whose list is exhausted ranks
        // last (cl: the lane holding the best)
        uint32_t cv = h < n ? 1u : 0u, cl = lane;
        float cs = cv ? bs[lane * topk + h] : 0.0f;
        uint32_t cd = cv ? bd[lane * topk + h] : 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t m = 1; m < 64u; m <<= 1) {
            const float os = __shfl_xor(cs, (int)m);
            const uint32_t od = (uint32_t)__shfl_xor((int)cd, (int)m), ol = (uint32_t)__shfl_xor((int)cl, (int)m);
            const uint32_t ov = (uint32_t)__shfl_xor((int)cv, (int)m);
            const bool take =
                ov > cv || (ov == cv && (ranks_before(os, od, cs, cd) || (os == cs && od == cd && ol < cl)));
            cs = take ? os : cs;
            cd = take ? od : cd;
            cl = take ? ol : cl;
            cv = take ? ov : cv;
        }
        if (!cv) break;   // every list is exhausted
        if (lane == 0) {
            ns[out] = cs;
            nd[out] = cd;
        }
        h += lane == cl ? 1u : 0u;
        out++;
    }
    wave_sync_lds();
    for (uint32_t r = lane; r < out; r += 64u) {
        a.part_score[(uint64_t)w * topk + r] = ns[r];
        a.part_doc[(uint64_t)w * topk + r] = nd[r];
    }
    if (lane == 0) a.part_doc[(uint64_t)a.nitems * topk + w] = out;
}

// One wave per query: its merged list (at its first item slot) to the
// output, padded with empty entries.
__global__ __launch_bounds__(kThreads) void k_topk_out(QArgs a) {
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t q = blockIdx.x * (uint32_t)kWaves + wave;
    if (q >= a.nq) return;
    const uint32_t f0 = a.first[q], topk = a.topk;
    const uint32_t count = f0 < a.first[q + 1] ? a.part_doc[(uint64_t)a.nitems * topk + f0] : 0u;
    for (uint32_t r = lane; r < topk; r += 64u) {
        a.out_doc[(uint64_t)q * topk + r] = r < count ? a.part_doc[(uint64_t)f0 * topk + r] : 0xFFFFFFFFu;
        a.out_score[(uint64_t)q * topk + r] = r < count ? a.part_score[(uint64_t)f0 * topk + r] : 0.0f;
    }
}

}  // namespace gcq

using namespace gcq;

struct gc_query_plan {
    QArgs a;
    uint32_t max_items = 0;   // the most work items of one query
    int device = 0;
    void *mem[6] = {};
};

namespace {

template <typename T>
bool qalloc(gc_query_plan *p, int slot, T **ptr, size_t n) {
    void *m = nullptr;
    if (hipMalloc(&m, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    p->mem[slot] = m;
    *ptr = static_cast<T *>(m);
    return true;
}

void qfree(gc_query_plan *p) {
    for (void *&m : p->mem)
        if (m) (void)hipFree(m), m = nullptr;
}

}  // namespace

extern "C" {

gc_status gc_query_plan_create(const uint32_t *h_term_len, size_t nterms, const int32_t *h_query_terms,
                               uint32_t terms_per_query, uint32_t nq, const gc_bm25_params *bp,
                               gc_query_plan **plan) {
    if (!plan) return GC_EINVAL;
    *plan = nullptr;
    if (!bp || !h_term_len || (nq && !h_query_terms) || nterms > 0x7FFFFFFFu) return GC_EINVAL;
    if (terms_per_query == 0 || terms_per_query > kMaxTerms || bp->topk == 0 || bp->topk > kMaxTopk ||
        bp->ndocs == 0 || !(bp->avgdl > 0.0f) || !(bp->k1 >= 0.0f) || !(bp->b >= 0.0f && bp->b <= 1.0f) ||
        bp->reserved[0] || bp->reserved[1])
        return GC_EINVAL;
    // work items: every query's pivot (its shortest list) in segments
    std::vector<QItem> items;
    std::vector<uint32_t> first(nq + 1u, 0u);
    for (uint32_t q = 0; q < nq; q++) {
        first[q] = (uint32_t)items.size();
        uint32_t piv = 0xFFFFFFFFu;
        bool any = false;
        for (uint32_t i = 0; i < terms_per_query; i++) {
            const int32_t t = h_query_terms[(size_t)q * terms_per_query + i];
            if (t < -1 || t >= (int64_t)nterms) return GC_EINVAL;
            if (t < 0) continue;
            any = true;
            piv = std::min(piv, h_term_len[t]);
        }
        if (!any) continue;
        for (uint32_t s0 = 0; s0 < piv; s0 += kSeg) items.push_back(QItem{q, s0, std::min(piv, s0 + kSeg), 0u});
    }
    first[nq] = (uint32_t)items.size();
    gc_query_plan *p = new (std::nothrow) gc_query_plan();
    if (!p) return GC_ENOMEM;
    for (uint32_t q = 0; q < nq; q++) p->max_items = std::max(p->max_items, first[q + 1] - first[q]);
    (void)hipGetDevice(&p->device);
    std::memset(&p->a, 0, sizeof(p->a));
    QArgs &a = p->a;
    a.tpq = terms_per_query;
    a.nq = nq;
    a.nitems = (uint32_t)items.size();
    a.ndocs = bp->ndocs;
    a.topk = bp->topk;
    a.avgdl = bp->avgdl;
    a.k1 = bp->k1;
    a.b = bp->b;
    uint32_t *tl = nullptr, *fi = nullptr, *pd = nullptr;
    int32_t *qt = nullptr;
    QItem *it = nullptr;
    float *ps = nullptr;
    const size_t nit = items.size();
    bool ok = qalloc(p, 0, &tl, nterms) && qalloc(p, 1, &qt, (size_t)nq * terms_per_query) &&
              qalloc(p, 2, &it, nit) && qalloc(p, 3, &fi, (size_t)nq + 1u) &&
              qalloc(p, 4, &pd, nit * bp->topk + nit) && qalloc(p, 5, &ps, nit * bp->topk);
    ok = ok && hipMemcpy(tl, h_term_len, nterms * 4, hipMemcpyHostToDevice) == hipSuccess &&
         (!nq || hipMemcpy(qt, h_query_terms, (size_t)nq * terms_per_query * 4, hipMemcpyHostToDevice) == hipSuccess) &&
         (!nit || hipMemcpy(it, items.data(), nit * sizeof(QItem), hipMemcpyHostToDevice) == hipSuccess) &&
         hipMemcpy(fi, first.data(), first.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        qfree(p);
        delete p;
        return GC_ENOMEM;
    }
    a.term_len = tl;
    a.qterms = qt;
    a.items = it;
    a.first = fi;
    a.part_doc = pd;
    a.part_score = ps;
    *plan = p;
    return GC_OK;
}

gc_status gc_query_run(gc_query_plan *plan, const uint32_t *d_docs, const uint32_t *d_tfs,
                       const uint64_t *d_term_off, const uint16_t *d_doclen, uint32_t *d_top_doc,
                       float *d_top_score, void *hip_stream) {
    if (!plan || !d_docs || !d_tfs || !d_term_off || !d_doclen || !d_top_doc || !d_top_score) return GC_EINVAL;
    QArgs a = plan->a;
    if (!a.nq) return GC_OK;
    a.docs = d_docs;
    a.tfs = d_tfs;
    a.term_off = d_term_off;
    a.doclen = d_doclen;
    a.out_doc = d_top_doc;
    a.out_score = d_top_score;
    const hipStream_t s = (hipStream_t)hip_stream;
    if (a.nitems) hipLaunchKernelGGL(k_and_topk, dim3((a.nitems + kWaves - 1) / kWaves), dim3(kThreads), 0, s, a);
    // the items' lists merged per query as a tree, merge_group(topk) lists a node
    const uint32_t G = merge_group(a.topk);
    for (uint64_t stride = 1; stride < plan->max_items; stride *= G)
        hipLaunchKernelGGL(k_merge_level, dim3((a.nitems + kWaves - 1) / kWaves), dim3(kThreads), 0, s, a,
                           (uint32_t)stride);
    hipLaunchKernelGGL(k_topk_out, dim3((a.nq + kWaves - 1) / kWaves), dim3(kThreads), 0, s, a);
    return hipGetLastError() == hipSuccess ? GC_OK : GC_EDEVICE;
}

gc_status gc_query_plan_destroy(gc_query_plan *plan) {
    if (!plan) return GC_EINVAL;
    (void)hipSetDevice(plan->device);
    (void)hipDeviceSynchronize();
    qfree(plan);
    delete plan;
    return GC_OK;
}

}  // extern "C"
