// encode_gpu.hip -- Group-codec encoders on the GPU (index build).
//
// Writes the same streams as the host encoder (include/gc.h, byte for byte)
// for many lists at once, with one codec and one parameter set:
//
//   widths   one pass over the input: the d-gaps of docID lists and the bit
//            width of every tuple (the width of the OR of its k integers,
//            Section 4.4).
//   sizing   per codec, the control, data and exception words of every list;
//            the host turns them into stream offsets.
//   emit     the header, control area, data rows and exception area of every
//            stream, into an output area cleared first (unary Group-Scheme
//            control areas are set to ones and their terminators cleared).
//
// Group-Simple's selectors (Algorithm 1, Section 4.2) and Group-AFOR's
// frames (Section 6.1) form chains: where the next unit starts depends on
// where this one did.  The incomplete-unary Group-Scheme control stream
// (Section 5.2.1) carries a state too, its position within a byte.  These
// run in three steps over chunks of a list: every chunk computes, for each
// state it may be entered in (the tuple or octet offset where the chain
// enters it, or the bit position mod 8), the state it leaves in and what it
// emitted (units, bits); one lane per list then walks its chunks and finds
// each chunk's true entry state and the counts before it; every chunk then
// runs once more from its entry state and writes its units.  A chunk runs
// on one wave: each lane tabulates its 32 tuples (or 4 octets) for every
// entry state, one lane chains the tables, and each lane then walks its own
// part from its true entry.  Group-AFOR's frame sizes come from the exact
// dynamic programme of Section 6.1, run backwards: a stretch of octets maps
// the costs at its end to the costs at its start by a 4 x 4 min-plus
// matrix (its four columns from four runs, each with one end state at cost
// 0 and the others unreachable); the products are associative, so a wave
// combines its lanes' matrices, and each list's chunk matrices, by reverse
// scans, and each lane then runs the programme once over its octets with
// its true end costs and keeps its choices.  Group-PFD codes 32-tuple
// blocks independently (Section 6.2): half a wave per block.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "gc.h"
#include "gc_format.h"

namespace gcenc {

typedef __attribute__((address_space(1))) uint32_t gu32;

constexpr int kThreads = 256;
constexpr uint32_t kTupChunk = 2048;   // tuples per chunk (Group-Simple, Group-Scheme)
constexpr uint32_t kOctChunk = 256;    // octets (8 tuples) per chunk (Group-AFOR)
constexpr uint64_t kInf = 1ull << 62;  // an unreachable cost

// Group-Simple (Table III): NUM and BW of selectors 0..9.
__constant__ uint8_t kNum[10] = {32, 16, 10, 8, 6, 5, 4, 3, 2, 1};
__constant__ uint8_t kBw[10] = {1, 2, 3, 4, 5, 6, 8, 10, 16, 32};

// One list of the call.
struct EList {
    uint64_t in_off;    // first input integer
    uint64_t out_off;   // first stream word (set once the streams are sized)
    uint64_t t0;        // first tuple in the per-tuple arrays (padded tuples)
    uint32_t n, T, M;   // integers, tuples, padded tuples (to the codec's unit)
    uint32_t c0, nch;   // first chunk, chunks
    uint32_t b0;        // first Group-PFD block
};

// A chunk: units [u0, u0 + nu) of list `list` (tuples, or octets for
// Group-AFOR).
struct EChunk {
    uint32_t list, u0, nu, pad;
};

struct EArgs {
    const uint32_t *in;
    const EList *lists;
    const EChunk *chunks;
    uint32_t nlists, nchunks;
    uint64_t ntup;          // padded tuples of all lists
    uint32_t k, lk, cg, ld, delta, pfd_pos, zn, zd, nblocks, pad;
    uint8_t *W;             // width of every padded tuple
    uint32_t *sizes;        // per list: C, D, E (words)
    uint32_t *out;          // the streams
    uint64_t out_words;
    // per codec scratch
    uint32_t *chs;          // chunk summaries
    uint32_t *chb;          // per chunk: entry state and bases
    uint32_t *tw;           // per tuple words (positions, offsets, selector info)
    uint32_t *tw2;
    uint8_t *ob;            // per octet bytes (Group-AFOR: omax, then frame widths)
    uint8_t *och;           // Group-AFOR: frame choice per octet
    uint64_t *mat;          // Group-AFOR: chunk matrices (16) and end costs (4)
    const uint32_t *tl;     // per 256 tuples: the list of the first (tiles + 1 entries)
    const uint32_t *wl;     // per 256 stream words: the list of the first (tiles + 1 entries)
    uint32_t *blk;          // Group-PFD: per block desc, exception words, row base, exception base
    uint32_t *slot;         // Group-PFD: slot of every integer
    uint32_t *xbit;         // Group-PFD: exception bitmap of every integer
};

__device__ __forceinline__ uint32_t width_of(uint32_t x) { return x ? 32u - (uint32_t)__builtin_clz(x) : 0u; }

// Integer i of list L as coded: its d-gap for a docID list, 0 past the end.
__device__ __forceinline__ uint32_t coded(const EArgs &a, const EList &L, uint64_t i) {
    if (i >= L.n) return 0u;
    const uint32_t *x = a.in + L.in_off;
    return a.delta ? x[i] - (i ? x[i - 1] : 0u) : x[i];
}

// Orders a wave's LDS accesses before and after it (lanes of one wave).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr uint32_t kTileShift = 8;   // list tables per 256 tuples or stream words

// List of global tuple g: a binary search over the lists' first tuples,
// between those of g's 256-tuple tile and the next.
__device__ __forceinline__ uint32_t list_of_tuple(const EArgs &a, uint64_t g) {
    const uint64_t tile = g >> kTileShift;
    // invariant: lists[lo].t0 <= g < lists[hi].t0 (hi: end)
    uint32_t lo = a.tl[tile], hi = min(a.tl[tile + 1u] + 1u, a.nlists);
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.lists[mid].t0 <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---- widths ----------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_widths(EArgs a) {
    const uint64_t g = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= a.ntup) return;
    const EList L = a.lists[list_of_tuple(a, g)];
    const uint64_t t = g - L.t0;
    uint32_t o = 0;
    for (uint32_t c = 0; c < a.k; c++) o |= coded(a, L, t * a.k + c);
    a.W[g] = (uint8_t)width_of(o);
}

// ---- Group-Scheme (Section 5) --------------------------------------------------
// unary code length u of a tuple of width w (eq. (1)); its width is cg * u (eq. (2))
__device__ __forceinline__ uint32_t gsc_units(uint32_t w, uint32_t cg) { return max(1u, (w + cg - 1u) / cg); }

// One tuple's step of the control stream: the position of its terminator
// and the position after it (incomplete units do not cross a byte).
__device__ __forceinline__ uint32_t gsc_step(uint32_t pos, uint32_t u, bool iu, uint32_t &z) {
    if (iu) {
        const uint32_t left = 8u - (pos & 7u);
        if (u > left) pos += left;
    }
    z = pos + u - 1u;
    return pos + u;
}

// A chunk's walks on one wave: lane l takes tuples [32 l, 32 l + 32) of
// the chunk.  The units of the lane's tuples, four to a word (0 past the
// chunk's end), and their data bits.
constexpr uint32_t kSegUnits = 32;   // units of a chunk per lane
static_assert(kTupChunk == 64u * kSegUnits, "a chunk is 64 lane segments");

__device__ __forceinline__ void gsc_seg_units(const EArgs &a, const uint8_t *W, uint32_t nu, uint32_t lane,
                                              uint32_t (&pu)[8], uint32_t &dbits) {
    dbits = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8u; i++) {
        uint32_t w = 0;
#pragma unroll
        for (uint32_t q = 0; q < 4u; q++) {
            const uint32_t t = kSegUnits * lane + 4u * i + q;
            const uint32_t u = t < nu ? gsc_units(W[t], a.cg) : 0u;
            dbits += a.cg * u;
            w |= u << (8u * q);
        }
        pu[i] = w;
    }
}

// The control position after the lane's tuples, entered at pos.
__device__ __forceinline__ uint32_t gsc_seg_walk(uint32_t pos, const uint32_t (&pu)[8], bool iu) {
#pragma unroll
    for (uint32_t i = 0; i < kSegUnits; i++) {
        const uint32_t u = (pu[i >> 2] >> (8u * (i & 3u))) & 0xFFu;
        uint32_t z;
        if (u) pos = gsc_step(pos, u, iu, z);
    }
    return pos;
}

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v, uint32_t lane) {
#pragma unroll
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)v, d);
        v += lane >= d ? u : 0u;
    }
    return v;
}

// Step A, one wave per chunk: for every entry state s (IU enters at bit
// s mod 8; the other layouts have one state), exit state | control bits
// << 3, from the lanes' advances per state chained in LDS; plus the
// chunk's data bits.
__global__ __launch_bounds__(kThreads) void k_gsc_chunkA(EArgs a) {
    __shared__ uint32_t s_adv[kThreads / 64u][64][8];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t ch = blockIdx.x * (kThreads / 64u) + wave;
    if (ch >= a.nchunks) return;
    const EChunk C = a.chunks[ch];
    const EList L = a.lists[C.list];
    const bool iu = a.ld == GC_LD_IU;
    const uint32_t ns = iu ? 8u : 1u;
    uint32_t pu[8], db;
    gsc_seg_units(a, a.W + L.t0 + C.u0, C.nu, lane, pu, db);
    // the control bits the lane's tuples take, entered at bit s mod 8
    for (uint32_t st = 0; st < ns; st++) s_adv[wave][lane][st] = gsc_seg_walk(st, pu, iu) - st;
    db = (uint32_t)__shfl((int)wave_incl_sum(db, lane), 63);
    wave_lds_fence();
    if (lane < ns) {
        uint32_t pos = lane;
        for (uint32_t l = 0; l < 64u; l++) pos += s_adv[wave][l][iu ? pos & 7u : 0u];
        a.chs[2u * (ch * 8u + lane)] = ((pos - lane) << 3) | (pos & 7u);
        if (lane == 0) a.chs[2u * (ch * 8u) + 1u] = db;
    }
}

// Step B, one lane per list: every chunk's entry control bit and data bit;
// the list's C and D.
__global__ __launch_bounds__(kThreads) void k_gsc_listB(EArgs a) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.nlists) return;
    const EList L = a.lists[i];
    uint32_t pos = 0, dbits = 0;
    for (uint32_t c = L.c0; c < L.c0 + L.nch; c++) {
        a.chb[2u * c] = pos;
        a.chb[2u * c + 1u] = dbits;
        const uint32_t s = a.ld == GC_LD_IU ? pos & 7u : 0u;
        pos += a.chs[2u * (c * 8u + s)] >> 3;
        dbits += a.chs[2u * (c * 8u) + 1u];
    }
    uint32_t cbits = pos;
    if (a.ld == GC_LD_BINARY) {
        const uint32_t fields = a.cg == 1u ? 3u : a.cg == 8u ? 4u : 2u, ubits = a.cg == 1u ? 16u : 8u;
        cbits = L.T ? ((L.T - 1u) / fields + 1u) * ubits : 0u;
    }
    a.sizes[3u * i] = ((cbits + 31u) / 32u + 3u) / 4u * 4u;
    a.sizes[3u * i + 1u] = a.k * ((dbits + 31u) / 32u);
    a.sizes[3u * i + 2u] = 0u;
}

// Step C, one wave per chunk: every tuple's terminator (unary) and data
// bit.  Lane 0 chains the lanes' advances from the chunk's entry bit; each
// lane then walks its own tuples from its entry.
__global__ __launch_bounds__(kThreads) void k_gsc_chunkC(EArgs a) {
    __shared__ uint32_t s_adv[kThreads / 64u][64][8];
    __shared__ uint32_t s_pos[kThreads / 64u][64];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t ch = blockIdx.x * (kThreads / 64u) + wave;
    if (ch >= a.nchunks) return;
    const EChunk C = a.chunks[ch];
    const EList L = a.lists[C.list];
    const bool iu = a.ld == GC_LD_IU;
    const uint32_t ns = iu ? 8u : 1u;
    uint32_t pu[8], db;
    gsc_seg_units(a, a.W + L.t0 + C.u0, C.nu, lane, pu, db);
    for (uint32_t st = 0; st < ns; st++) s_adv[wave][lane][st] = gsc_seg_walk(st, pu, iu) - st;
    uint32_t dbits = a.chb[2u * ch + 1u] + wave_incl_sum(db, lane) - db;
    wave_lds_fence();
    if (lane == 0) {
        uint32_t pos = a.chb[2u * ch];
        for (uint32_t l = 0; l < 64u; l++) {
            s_pos[wave][l] = pos;
            pos += s_adv[wave][l][iu ? pos & 7u : 0u];
        }
    }
    wave_lds_fence();
    uint32_t pos = s_pos[wave][lane];
    const uint64_t g0 = (uint64_t)L.t0 + C.u0 + kSegUnits * lane;
#pragma unroll
    for (uint32_t i = 0; i < kSegUnits; i++) {
        const uint32_t u = (pu[i >> 2] >> (8u * (i & 3u))) & 0xFFu;
        if (u) {
            uint32_t z;
            pos = gsc_step(pos, u, iu, z);
            a.tw[g0 + i] = z;
            a.tw2[g0 + i] = dbits;
            dbits += a.cg * u;
        }
    }
}

// ---- Group-Simple (Section 4, Algorithm 1) -------------------------------------
// From tuple j: the first selector whose NUM next tuples -- or all that
// remain -- fit its width; code = selector | tuples covered << 4.
// The workgroup's widths, and the 32 after them, are read into LDS first.
__global__ __launch_bounds__(kThreads) void k_sim_cover(EArgs a) {
    __shared__ uint8_t s_w[kThreads + 32u];
    const uint64_t gb = (uint64_t)blockIdx.x * kThreads;
    for (uint32_t x = threadIdx.x; x < kThreads + 32u; x += kThreads)
        if (gb + x < a.ntup) s_w[x] = a.W[gb + x];
    __syncthreads();
    const uint64_t g = gb + threadIdx.x;
    if (g >= a.ntup) return;
    const EList L = a.lists[list_of_tuple(a, g)];
    const uint32_t j = (uint32_t)(g - L.t0);
    const uint8_t *W = s_w + threadIdx.x;   // W[p]: tuple j + p
    const uint32_t left = L.T - j;
    uint32_t pick = 9, cover = 1;
    for (uint32_t i = 0; i < 10u; i++) {
        const uint32_t num = kNum[i], lim = min(num, left);
        uint32_t p = 0;
        while (p < lim && W[p] <= kBw[i]) p++;
        if (p == num || p == left) {
            pick = i;
            cover = p;
            break;
        }
    }
    a.tw[g] = pick | (cover << 4);
}

// The selector chain over a chunk on one wave: lane l takes tuples
// [32 l, 32 l + 32) of the chunk, and for every entry offset p < 32 into
// them finds, by a backward pass, where the chain entered at p leaves
// (offset x from the lane's first tuple, x >= 32 into the next lane's; a
// chain that ends at the chunk's end, or the list's, stops there) and the
// selectors it starts: tab[p] = x | selectors << 6, in LDS.
__device__ __forceinline__ void sim_seg_table(const uint32_t *cv, uint32_t base, uint32_t end, uint16_t *tab) {
    for (uint32_t p = kSegUnits; p-- > 0u;) {
        if (base + p >= end) {
            tab[p] = (uint16_t)p;   // no chain starts here
            continue;
        }
        const uint32_t q = p + (cv[base + p] >> 4);
        tab[p] = (uint16_t)(q >= kSegUnits || base + q >= end ? q | (1u << 6) : tab[q] + (1u << 6));
    }
}

// Follows the lanes' tables from entry offset e into lane 0's tuples; with
// `in`, notes each lane's entry offset and first selector (or 0xFFFF: the
// chain does not reach it).  Returns the tuple where the chain leaves the
// chunk (relative to u0) and adds its selectors to *sel.
__device__ __forceinline__ uint32_t sim_chain(const uint16_t (*tab)[kSegUnits], uint32_t e, uint32_t nu, uint32_t &sel,
                                              uint32_t *in) {
    uint32_t l = 0;
    for (;;) {
        const uint32_t j = kSegUnits * l + e;
        if (j >= nu) return j;
        if (in) in[l] = e | (sel << 5);
        const uint32_t v = tab[l][e], x = v & 63u;
        sel += v >> 6;
        if (x < kSegUnits || l == 63u) return kSegUnits * l + x;
        l++;
        e = x - kSegUnits;
    }
}

// Step A, one wave per chunk: for every entry offset e < 32, the chain
// entering the chunk at tuple u0 + e; summary: exit offset | selectors << 5.
__global__ __launch_bounds__(kThreads) void k_sim_chainA(EArgs a) {
    __shared__ uint16_t s_tab[kThreads / 64u][64][kSegUnits];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t ch = blockIdx.x * (kThreads / 64u) + wave;
    if (ch >= a.nchunks) return;
    const EChunk C = a.chunks[ch];
    const EList L = a.lists[C.list];
    sim_seg_table(a.tw + L.t0 + C.u0, kSegUnits * lane, C.nu, s_tab[wave][lane]);
    wave_lds_fence();
    if (lane < kSegUnits) {
        uint32_t sel = 0;
        const uint32_t j = sim_chain(s_tab[wave], lane, C.nu, sel, nullptr);
        a.chs[ch * 32u + lane] = (j - C.nu) | (sel << 5);
    }
}

// Step B, one lane per list: entry offset and first selector of every
// chunk; C and D.
__global__ __launch_bounds__(kThreads) void k_sim_listB(EArgs a) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.nlists) return;
    const EList L = a.lists[i];
    uint32_t e = 0, sel = 0;
    for (uint32_t c = L.c0; c < L.c0 + L.nch; c++) {
        a.chb[2u * c] = e;
        a.chb[2u * c + 1u] = sel;
        const uint32_t v = a.chs[c * 32u + e];
        e = v & 31u;
        sel += v >> 5;
    }
    a.sizes[3u * i] = ((sel * 4u + 31u) / 32u + 3u) / 4u * 4u;
    a.sizes[3u * i + 1u] = a.k * sel;
    a.sizes[3u * i + 2u] = 0u;
}

// Step C, one wave per chunk: every tuple's selector index << 10 |
// selector << 5 | its place in the selector; selectors to the control
// area.  Lane 0 follows the tables from the chunk's entry; each lane then
// walks the selectors that start in its tuples.
__global__ __launch_bounds__(kThreads) void k_sim_chainC(EArgs a) {
    __shared__ uint16_t s_tab[kThreads / 64u][64][kSegUnits];
    __shared__ uint32_t s_in[kThreads / 64u][64];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t ch = blockIdx.x * (kThreads / 64u) + wave;
    if (ch >= a.nchunks) return;
    const EChunk C = a.chunks[ch];
    const EList L = a.lists[C.list];
    const uint32_t *cv = a.tw + L.t0 + C.u0;
    sim_seg_table(cv, kSegUnits * lane, C.nu, s_tab[wave][lane]);
    s_in[wave][lane] = 0xFFFFFFFFu;
    wave_lds_fence();
    if (lane == 0) {
        uint32_t sel = a.chb[2u * ch + 1u];
        (void)sim_chain(s_tab[wave], a.chb[2u * ch], C.nu, sel, s_in[wave]);
    }
    wave_lds_fence();
    const uint32_t in = s_in[wave][lane];
    if (in == 0xFFFFFFFFu) return;
    uint32_t *info = a.tw2 + L.t0 + C.u0;
    gu32 *ctrl = (gu32 *)(a.out + L.out_off + 4u);
    const uint32_t lim = min(C.nu, kSegUnits * (lane + 1u));
    uint32_t j = kSegUnits * lane + (in & 31u), s = in >> 5;
    while (j < lim) {
        const uint32_t v = cv[j], sel = v & 15u, cover = v >> 4;
        atomicOr((uint32_t *)&ctrl[s >> 3], sel << (4u * (s & 7u)));
        for (uint32_t jj = 0; jj < cover; jj++) info[j + jj] = (s << 10) | (sel << 5) | jj;
        j += cover;
        s++;
    }
}

// ---- Group-AFOR (Section 6.1) ---------------------------------------------------
// Octet o (8 tuples): the widest tuple.
__global__ __launch_bounds__(kThreads) void k_afor_omax(EArgs a) {
    const uint64_t o = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o >= a.ntup / 8u) return;
    uint32_t m = 0;
    for (int t = 0; t < 8; t++) m = max(m, (uint32_t)a.W[8u * o + t]);
    a.ob[o] = (uint8_t)m;
}

// The backward programme over octets [o0, o1) of a list of `oct` octets
// (global octet o of the list at om[o]), from the costs v[0..3] of octets
// o1 .. o1 + 3; returns the costs of o0 .. o0 + 3 in v; with `ch`, writes
// every octet's choice (frame of 32, 16 or 8 tuples; ties keep the larger).
__device__ __forceinline__ void afor_dp(const uint8_t *om, uint32_t oct, uint32_t o0, uint32_t o1, uint32_t k,
                                        uint64_t (&v)[4], uint8_t *ch) {
    uint64_t c1 = v[0], c2 = v[1], c3 = v[2], c4 = v[3];   // cost[o + 1 .. o + 4]
    for (uint32_t o = o1; o-- > o0;) {
        uint64_t best = kInf;
        uint32_t bf = 8;
        uint32_t b = 0;
        const uint32_t F[3] = {32u, 16u, 8u};
        for (int fi = 0; fi < 3; fi++) {
            const uint32_t no = F[fi] / 8u;
            if (o + no > oct) continue;
            b = 0;
            for (uint32_t q = o; q < o + no; q++) b = max(b, (uint32_t)om[q]);
            const uint64_t next = no == 4u ? c4 : no == 2u ? c2 : c1;
            const uint64_t c = next >= kInf ? kInf : 8ull + (uint64_t)k * F[fi] * b + next;
            if (c < best) {
                best = c;
                bf = F[fi];
            }
        }
        if (ch) ch[o] = (uint8_t)bf;
        c4 = c3;
        c3 = c2;
        c2 = c1;
        c1 = best;
    }
    v[0] = c1;
    v[1] = c2;
    v[2] = c3;
    v[3] = c4;
}

// Min-plus sum with an unreachable cost absorbing.
__device__ __forceinline__ uint64_t mp_add(uint64_t x, uint64_t y) { return x >= kInf || y >= kInf ? kInf : x + y; }

__device__ __forceinline__ uint64_t mp_ident(uint32_t x) { return x % 5u == 0u ? 0ull : kInf; }

// P_l = M_l (x) M_{l+1} (x) ... (x) M_63 over the wave's lanes (min-plus
// products of 4 x 4 matrices, row-major).
__device__ __forceinline__ void mp_suffix_scan(uint64_t (&P)[16], uint32_t lane) {
#pragma unroll
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        uint64_t Q[16];
#pragma unroll
        for (uint32_t x = 0; x < 16u; x++) {
            const uint64_t q = __shfl(P[x], (int)min(lane + d, 63u));
            Q[x] = lane + d < 64u ? q : mp_ident(x);
        }
        uint64_t R[16];
#pragma unroll
        for (uint32_t r = 0; r < 4u; r++)
#pragma unroll
            for (uint32_t q = 0; q < 4u; q++) {
                uint64_t best = kInf;
#pragma unroll
                for (uint32_t t = 0; t < 4u; t++) best = min(best, mp_add(P[4u * r + t], Q[4u * t + q]));
                R[4u * r + q] = best;
            }
#pragma unroll
        for (uint32_t x = 0; x < 16u; x++) P[x] = R[x];
    }
}

// The product of the lanes after this one, applied to e (e itself for
// lane 63), from the scanned P.
__device__ __forceinline__ void mp_after(const uint64_t (&P)[16], const uint64_t (&e)[4], uint32_t lane,
                                         uint64_t (&out)[4]) {
#pragma unroll
    for (uint32_t r = 0; r < 4u; r++) {
        uint64_t best = kInf;
#pragma unroll
        for (uint32_t q = 0; q < 4u; q++) {
            const uint64_t n = __shfl(P[4u * r + q], (int)min(lane + 1u, 63u));
            best = min(best, mp_add(lane < 63u ? n : mp_ident(4u * r + q), e[q]));
        }
        out[r] = best;
    }
}

// A chunk's costs on one wave: lane l takes octets [4 l, 4 l + 4) of the
// chunk; its min-plus matrix (start costs from end costs), column j from
// the programme run with end state j at cost 0 and the others unreachable.
constexpr uint32_t kSegOct = 4;   // octets of a chunk per lane
static_assert(kOctChunk == 64u * kSegOct, "a chunk is 64 lane segments");

__device__ __forceinline__ void afor_seg_matrix(const uint8_t *om, uint32_t oct, uint32_t s0, uint32_t s1, uint32_t k,
                                                uint64_t (&P)[16]) {
#pragma unroll
    for (uint32_t j = 0; j < 4u; j++) {
        uint64_t v[4] = {kInf, kInf, kInf, kInf};
        v[j] = 0;
        afor_dp(om, oct, s0, s1, k, v, nullptr);
#pragma unroll
        for (uint32_t i = 0; i < 4u; i++) P[4u * i + j] = v[i];
    }
}

// Step A of the costs, one wave per chunk: the chunk's min-plus matrix, the
// product of its lanes' matrices.
__global__ __launch_bounds__(kThreads) void k_afor_dpA(EArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t ch = blockIdx.x * (kThreads / 64u) + (threadIdx.x >> 6);
    if (ch >= a.nchunks) return;
    const EChunk C = a.chunks[ch];
    const EList L = a.lists[C.list];
    const uint32_t end = C.u0 + C.nu, s0 = min(C.u0 + kSegOct * lane, end), s1 = min(s0 + kSegOct, end);
    uint64_t P[16];
    afor_seg_matrix(a.ob + L.t0 / 8u, L.M / 8u, s0, s1, a.k, P);
    mp_suffix_scan(P, lane);
    if (lane == 0) {
#pragma unroll
        for (uint32_t x = 0; x < 16u; x++) a.mat[20ull * ch + x] = P[x];
    }
}

// Step B of the costs, one wave per list: the true costs at every chunk's
// end.  The end costs of chunk c are M_{c+1} (x) ... (x) M_last applied to
// the costs past the last octet; lane l takes chunk l of a group of 64, and
// the groups run from the last back, each starting from the costs at its
// end.
__global__ __launch_bounds__(kThreads) void k_afor_dpB(EArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t i = blockIdx.x * (kThreads / 64u) + (threadIdx.x >> 6);
    if (i >= a.nlists) return;
    const EList L = a.lists[i];
    uint64_t e[4] = {0, kInf, kInf, kInf};   // costs at the group's end (past the last octet at first)
    for (uint32_t gend = L.nch; gend > 0u;) {
        const uint32_t gbeg = gend > 64u ? gend - 64u : 0u;
        const bool valid = gbeg + lane < gend;
        const uint64_t *m = a.mat + 20ull * (L.c0 + gbeg + lane);
        uint64_t P[16];
#pragma unroll
        for (uint32_t x = 0; x < 16u; x++) P[x] = valid ? m[x] : mp_ident(x);
        mp_suffix_scan(P, lane);
        uint64_t end[4];
        mp_after(P, e, lane, end);
        if (valid) {
            uint64_t *me = a.mat + 20ull * (L.c0 + gbeg + lane) + 16u;
#pragma unroll
            for (uint32_t r = 0; r < 4u; r++) me[r] = end[r];
        }
        // the costs at the previous group's end: the whole group applied to e
        uint64_t ne[4];
#pragma unroll
        for (uint32_t r = 0; r < 4u; r++) {
            uint64_t best = kInf;
#pragma unroll
            for (uint32_t q = 0; q < 4u; q++) best = min(best, mp_add(__shfl(P[4u * r + q], 0), e[q]));
            ne[r] = best;
        }
#pragma unroll
        for (uint32_t r = 0; r < 4u; r++) e[r] = ne[r];
        gend = gbeg;
    }
}

// Step C of the costs, one wave per chunk: each lane's end costs from the
// chunk's true end costs and the lanes after it; the lane then runs the
// programme over its octets and keeps its choices.
__global__ __launch_bounds__(kThreads) void k_afor_dpC(EArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t ch = blockIdx.x * (kThreads / 64u) + (threadIdx.x >> 6);
    if (ch >= a.nchunks) return;
    const EChunk C = a.chunks[ch];
    const EList L = a.lists[C.list];
    const uint32_t end = C.u0 + C.nu, s0 = min(C.u0 + kSegOct * lane, end), s1 = min(s0 + kSegOct, end);
    const uint8_t *om = a.ob + L.t0 / 8u;
    uint64_t P[16];
    afor_seg_matrix(om, L.M / 8u, s0, s1, a.k, P);
    mp_suffix_scan(P, lane);
    uint64_t e[4], v[4];
#pragma unroll
    for (uint32_t r = 0; r < 4u; r++) e[r] = a.mat[20ull * ch + 16u + r];
    mp_after(P, e, lane, v);
    afor_dp(om, L.M / 8u, s0, s1, a.k, v, a.och + L.t0 / 8u);
}

// width of the frame of F tuples from octet o
__device__ __forceinline__ uint32_t afor_b(const uint8_t *om, uint32_t o, uint32_t F) {
    uint32_t b = 0;
    for (uint32_t q = o; q < o + F / 8u; q++) b = max(b, (uint32_t)om[q]);
    return b;
}

// The frame chain over a chunk on one wave: lane l takes octets
// [4 l, 4 l + 4) of the chunk, and for every entry offset p < 4 into them
// finds, by a backward pass, where the chain entered at p leaves (offset x
// from the lane's first octet, x >= 4 into the next lane's; a chain that
// reaches the chunk's end stops there), the frames it starts and their data
// bits: tab[p] = x | frames << 3 | bits << 6, in LDS.
// Octets before the chunk's entry may already hold the previous chunk's
// frame widths (step C rewrites them); their entries are never followed, and
// a value that is no frame size starts no chain.
__device__ __forceinline__ void afor_seg_table(const uint8_t *om, const uint8_t *cho, uint32_t oct, uint32_t s0,
                                               uint32_t end, uint32_t *tab) {
    for (uint32_t p = kSegOct; p-- > 0u;) {
        const uint32_t o = s0 + p;
        const uint32_t F = o < end ? cho[o] : 0u;
        if ((F != 8u && F != 16u && F != 32u) || o + F / 8u > oct) {
            tab[p] = p;   // no chain starts here
            continue;
        }
        const uint32_t q = p + F / 8u, fb = F * afor_b(om, o, F);
        tab[p] = q >= kSegOct || s0 + q >= end ? q | (1u << 3) | (fb << 6) : tab[q] + (1u << 3) + (fb << 6);
    }
}

// Follows the lanes' tables from entry offset e into lane 0's octets,
// adding frames and bits; with `in`, notes each lane's entry (e, frames,
// bits before it; e = 0xFFFFFFFF: the chain does not reach the lane).
// Returns the octet where the chain leaves the chunk (relative to u0).
__device__ __forceinline__ uint32_t afor_chain(const uint32_t (*tab)[kSegOct], uint32_t e, uint32_t nu, uint32_t &frames,
                                               uint32_t &bits, uint32_t (*in)[3]) {
    uint32_t l = 0;
    for (;;) {
        const uint32_t o = kSegOct * l + e;
        if (o >= nu) return o;
        if (in) {
            in[l][0] = e;
            in[l][1] = frames;
            in[l][2] = bits;
        }
        const uint32_t v = tab[l][e], x = v & 7u;
        frames += (v >> 3) & 7u;
        bits += v >> 6;
        if (x < kSegOct || l == 63u) return kSegOct * l + x;
        l++;
        e = x - kSegOct;
    }
}

// Step A of the frames, one wave per chunk: for every entry octet e < 4,
// exit octet, frames and data bits of the chain.
__global__ __launch_bounds__(kThreads) void k_afor_chainA(EArgs a) {
    __shared__ uint32_t s_tab[kThreads / 64u][64][kSegOct];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t ch = blockIdx.x * (kThreads / 64u) + wave;
    if (ch >= a.nchunks) return;
    const EChunk C = a.chunks[ch];
    const EList L = a.lists[C.list];
    afor_seg_table(a.ob + L.t0 / 8u, a.och + L.t0 / 8u, L.M / 8u, C.u0 + kSegOct * lane, C.u0 + C.nu, s_tab[wave][lane]);
    wave_lds_fence();
    if (lane < 4u) {
        uint32_t frames = 0, bits = 0;
        const uint32_t o = afor_chain(s_tab[wave], lane, C.nu, frames, bits, nullptr);
        a.chs[3u * (ch * 4u + lane)] = o - C.nu;
        a.chs[3u * (ch * 4u + lane) + 1u] = frames;
        a.chs[3u * (ch * 4u + lane) + 2u] = bits;
    }
}

// Step B of the frames, one lane per list.
__global__ __launch_bounds__(kThreads) void k_afor_chainB(EArgs a) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.nlists) return;
    const EList L = a.lists[i];
    uint32_t e = 0, frames = 0, bits = 0;
    for (uint32_t c = L.c0; c < L.c0 + L.nch; c++) {
        a.chb[3u * c] = e;
        a.chb[3u * c + 1u] = frames;
        a.chb[3u * c + 2u] = bits;
        const uint32_t *s = a.chs + 3u * (c * 4u + e);
        e = s[0];
        frames += s[1];
        bits += s[2];
    }
    a.sizes[3u * i] = ((frames * 8u + 31u) / 32u + 3u) / 4u * 4u;
    a.sizes[3u * i + 1u] = a.k * ((bits + 31u) / 32u);
    a.sizes[3u * i + 2u] = 0u;
}

// Step C of the frames, one wave per chunk: frame bytes to the control
// area; every octet's data bit and width (octet words in tw, widths in
// och).  Lane 0 follows the tables from the chunk's entry; each lane then
// writes the frames that start in its octets.
__global__ __launch_bounds__(kThreads) void k_afor_chainC(EArgs a) {
    __shared__ uint32_t s_tab[kThreads / 64u][64][kSegOct];
    __shared__ uint32_t s_in[kThreads / 64u][64][3];
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t ch = blockIdx.x * (kThreads / 64u) + wave;
    if (ch >= a.nchunks) return;
    const EChunk C = a.chunks[ch];
    const EList L = a.lists[C.list];
    const uint8_t *om = a.ob + L.t0 / 8u;
    uint8_t *cho = a.och + L.t0 / 8u;
    const uint32_t s0 = C.u0 + kSegOct * lane, end = C.u0 + C.nu;
    afor_seg_table(om, cho, L.M / 8u, s0, end, s_tab[wave][lane]);
    s_in[wave][lane][0] = 0xFFFFFFFFu;
    wave_lds_fence();
    if (lane == 0) {
        uint32_t frames = a.chb[3u * ch + 1u], bits = a.chb[3u * ch + 2u];
        (void)afor_chain(s_tab[wave], a.chb[3u * ch], C.nu, frames, bits, s_in[wave]);
    }
    wave_lds_fence();
    if (s_in[wave][lane][0] == 0xFFFFFFFFu) return;
    uint32_t *ooff = a.tw + L.t0 / 8u;
    gu32 *ctrl = (gu32 *)(a.out + L.out_off + 4u);
    const uint32_t lim = min(end, s0 + kSegOct);
    uint32_t o = s0 + s_in[wave][lane][0], f = s_in[wave][lane][1], bits = s_in[wave][lane][2];
    while (o < lim) {
        const uint32_t F = cho[o], b = afor_b(om, o, F);
        const uint32_t cls = F == 8u ? 0u : F == 16u ? 1u : 2u;
        atomicOr((uint32_t *)&ctrl[f >> 2], (b | (cls << 6)) << (8u * (f & 3u)));
        for (uint32_t q = 0; q < F / 8u; q++) {
            ooff[o + q] = bits + q * 8u * b;
            cho[o + q] = (uint8_t)b;   // the choice is no longer needed past here
        }
        bits += F * b;
        f++;
        o += F / 8u;
    }
}

// ---- data rows of Group-Simple, Group-Scheme and Group-AFOR ------------------------
// Where tuple t of list L goes: its first data word wi (component c at word
// wi * k + c), the bit shift sh there and its width bw (its bits run into
// word wi + 1 if sh + bw > 32); for Group-Scheme, the control word cw and
// the bits to clear there (unary: the terminator) or to set (binary: the
// length field) in cm.
struct TuplePlace {
    uint32_t wi, sh, bw, cw, cm;
};

__device__ __forceinline__ TuplePlace tuple_place(const EArgs &a, const EList &L, uint64_t g, uint32_t t, int codec) {
    TuplePlace P{0u, 0u, 0u, 0u, 0u};
    if (codec == GC_SIMPLE) {
        // a selector's row holds its tuples side by side (NUM * BW <= 32)
        const uint32_t v = a.tw2[g], sel = (v >> 5) & 15u;
        P.bw = kBw[sel];
        P.wi = v >> 10;
        P.sh = (v & 31u) * P.bw;
        return P;
    }
    uint32_t O;
    if (codec == GC_SCHEME) {
        P.bw = a.cg * gsc_units(a.W[g], a.cg);
        O = a.tw2[g];
        const uint32_t u = P.bw / a.cg;
        if (a.ld == GC_LD_BINARY) {
            const uint32_t fields = a.cg == 1u ? 3u : a.cg == 8u ? 4u : 2u, ubits = a.cg == 1u ? 16u : 8u;
            const uint32_t fb = a.cg == 1u ? 5u : a.cg == 2u ? 4u : a.cg == 4u ? 3u : 2u;
            const uint32_t pos = (t / fields) * ubits + (t % fields) * fb;
            P.cw = pos >> 5;
            P.cm = (u - 1u) << (pos & 31u);
        } else {
            const uint32_t z = a.tw[g];
            P.cw = z >> 5;
            P.cm = 1u << (z & 31u);
        }
    } else {
        const uint32_t o = t >> 3;
        P.bw = a.och[L.t0 / 8u + o];
        O = a.tw[L.t0 / 8u + o] + (t & 7u) * P.bw;
    }
    P.wi = O >> 5;
    P.sh = O & 31u;
    return P;
}

// A tile's span of data words per component, and of control words, held in
// LDS: 256 tuples of at most 32 bits (plus one word for the first's
// offset); incomplete-unary control adds under 8 bits per tuple.
constexpr uint32_t kEmitSpan = kThreads + 1u;
constexpr uint32_t kCtrlSpan = 320u;

// One lane per tuple: its k integers at their component bit offset, and its
// Group-Scheme control bits.  The tuples of the workgroup's first list
// gather their words in LDS: words only they touch are stored whole, the
// first and last (which neighbouring workgroups may share) merged by
// atomics.  Tuples of later lists in the tile (a list starting inside it),
// and tiles whose words exceed the LDS span (k = 64), use global atomics.
// Dynamic LDS: kEmitSpan * k words when k <= 32.
__global__ __launch_bounds__(kThreads) void k_emit_tuples(EArgs a, int codec) {
    extern __shared__ uint32_t s_data[];
    __shared__ uint32_t s_ctrl[kCtrlSpan];
    __shared__ uint32_t s_list, s_lo, s_hi, s_clo, s_chi;
    const uint64_t g0 = (uint64_t)blockIdx.x * kThreads;
    const uint64_t g = g0 + threadIdx.x;
    const uint32_t k = a.k, lk = a.lk;
    const bool unary = codec == GC_SCHEME && a.ld != GC_LD_BINARY;
    if (threadIdx.x == 0) {
        s_list = list_of_tuple(a, g0);
        s_lo = s_clo = 0xFFFFFFFFu;
        s_hi = s_chi = 0u;
    }
    __syncthreads();
    const uint32_t li0 = s_list;
    const uint64_t t00 = a.lists[li0].t0;
    bool act = g < a.ntup;
    const bool first = !act || g - t00 < a.lists[li0].M;
    const EList L = a.lists[first ? li0 : list_of_tuple(a, g)];
    const uint32_t t = act ? (uint32_t)(g - L.t0) : 0u;
    act = act && t < L.T;
    TuplePlace P{0u, 0u, 0u, 0u, 0u};
    if (act) P = tuple_place(a, L, g, t, codec);
    const bool cross = P.sh + P.bw > 32u;
    const bool gather = k <= 32u && act && first;
    if (gather && P.bw) {
        atomicMin(&s_lo, P.wi);
        atomicMax(&s_hi, P.wi + (cross ? 1u : 0u));
    }
    if (gather && codec == GC_SCHEME) {
        atomicMin(&s_clo, P.cw);
        atomicMax(&s_chi, P.cw);
    }
    __syncthreads();
    const uint32_t lo = s_lo, hi = s_hi, clo = s_clo, chi = s_chi;
    const uint32_t span = lo <= hi ? hi - lo + 1u : 0u, cspan = clo <= chi ? chi - clo + 1u : 0u;
    // uniform over the workgroup: gather in LDS, or every lane by atomics
    const bool lds = k <= 32u && span <= kEmitSpan && cspan <= kCtrlSpan;
    for (uint32_t x = threadIdx.x; lds && x < (span << lk); x += kThreads) s_data[x] = 0u;
    for (uint32_t x = threadIdx.x; lds && x < cspan; x += kThreads) s_ctrl[x] = unary ? 0xFFFFFFFFu : 0u;
    __syncthreads();
    uint32_t *base = a.out + L.out_off;
    gu32 *ctrl = (gu32 *)(base + 4u);
    gu32 *data = (gu32 *)(base + 4u + base[2]);
    const bool here = lds && gather;
    if (act && codec == GC_SCHEME) {
        if (here) {
            if (unary) atomicAnd(&s_ctrl[P.cw - clo], ~P.cm);
            else atomicOr(&s_ctrl[P.cw - clo], P.cm);
        } else {
            if (unary) atomicAnd((uint32_t *)&ctrl[P.cw], ~P.cm);
            else atomicOr((uint32_t *)&ctrl[P.cw], P.cm);
        }
    }
    if (act && P.bw) {
        for (uint32_t c = 0; c < k; c++) {
            const uint32_t x = coded(a, L, (uint64_t)t * k + c);
            const uint32_t v0 = x << P.sh, v1 = cross ? x >> (32u - P.sh) : 0u;
            if (here) {
                atomicOr(&s_data[((P.wi - lo) << lk) + c], v0);
                if (cross) atomicOr(&s_data[((P.wi + 1u - lo) << lk) + c], v1);
            } else {
                atomicOr((uint32_t *)&data[P.wi * k + c], v0);
                if (cross) atomicOr((uint32_t *)&data[(P.wi + 1u) * k + c], v1);
            }
        }
    }
    if (!lds) return;
    __syncthreads();
    // the first list's words, out of LDS
    uint32_t *base0 = a.out + a.lists[li0].out_off;
    gu32 *data0 = (gu32 *)(base0 + 4u + base0[2]);
    for (uint32_t x = threadIdx.x; x < (span << lk); x += kThreads) {
        const uint32_t w = lo + (x >> lk), v = s_data[x];
        gu32 *dst = data0 + ((uint64_t)lo << lk) + x;
        if (w != lo && w != hi) *dst = v;
        else if (v) atomicOr((uint32_t *)dst, v);
    }
    gu32 *ctrl0 = (gu32 *)(base0 + 4u);
    for (uint32_t x = threadIdx.x; x < cspan; x += kThreads) {
        const uint32_t w = clo + x, v = s_ctrl[x];
        if (w != clo && w != chi) ctrl0[w] = v;
        else if (unary && v != 0xFFFFFFFFu) atomicAnd((uint32_t *)&ctrl0[w], v);
        else if (!unary && v) atomicOr((uint32_t *)&ctrl0[w], v);
    }
}

// ---- Group-PFD (Section 6.2) -------------------------------------------------------
// Half a wave per 32-tuple block, lane t on tuple t: b (Step 2) by ballots
// over the tuple widths, the exceptions (Step 3) and their value width
// (Step 4), every slot and the exception bitmap (gathered in LDS) to
// scratch; for the linked layout one lane then walks the exceptions in
// order and adds the compulsory ones; the block's descriptor and exception
// words.
__global__ __launch_bounds__(kThreads) void k_pfd_blocks(EArgs a) {
    __shared__ uint32_t s_xb[kThreads / 32u][64];   // each block's bitmap (k words, k <= 64)
    const uint32_t lane = threadIdx.x & 63u, h = threadIdx.x >> 5, t = threadIdx.x & 31u;
    const uint32_t bi = blockIdx.x * (kThreads / 32u) + h;
    const bool valid = bi < a.nblocks;
    const uint64_t hm = lane < 32u ? 0xFFFFFFFFull : 0xFFFFFFFF00000000ull;
    const uint32_t k = a.k;
    const bool linked = a.pfd_pos == GC_PFD_LINKED;
    uint32_t *xbl = s_xb[h];
    for (uint32_t w = t; w < k; w += 32u) xbl[w] = 0u;
    const uint64_t g0 = 32ull * (valid ? bi : 0u);   // first tuple
    const EList L = a.lists[list_of_tuple(a, g0)];
    const uint32_t t0 = (uint32_t)(g0 - L.t0);
    const uint32_t Wt = valid ? a.W[g0 + t] : 0u;
    // the smallest b leaving fewer than the fraction zn / zd of the tuples wider
    uint32_t b = 0;
    for (;;) {
        const uint32_t wider = (uint32_t)__builtin_popcountll(__ballot(Wt > b) & hm);
        const bool more = valid && b < 32u && (uint64_t)wider * a.zd >= (uint64_t)a.zn * 32u;
        if (!__ballot(more)) break;
        b += more ? 1u : 0u;
    }
    const uint32_t M = b >= 32u ? 0xFFFFFFFFu : (1u << b) - 1u;
    const uint64_t x0 = (uint64_t)t0 * k;   // first integer of the block in its list
    uint32_t *slot = a.slot + g0 * k;
    const bool wide = Wt > b;
    uint32_t nxl = 0, mwl = 0;
    wave_lds_fence();
    if (valid) {
        for (uint32_t c = 0; c < k; c++) {
            const uint32_t p = t * k + c;
            const uint32_t x = coded(a, L, x0 + p);
            const uint32_t w = width_of(x);
            const bool e = wide && w > b;
            slot[p] = e && !linked ? x & M : x;
            if (e) {
                atomicOr(&xbl[p >> 5], 1u << (p & 31u));
                nxl++;
                mwl = max(mwl, w);
            }
        }
    }
    uint32_t nx = nxl, maxw = mwl;
#pragma unroll
    for (uint32_t m = 1; m < 32u; m <<= 1) {
        nx += (uint32_t)__shfl_xor((int)nx, (int)m);
        maxw = max(maxw, (uint32_t)__shfl_xor((int)maxw, (int)m));
    }
    const uint32_t nt = (uint32_t)__builtin_popcountll(__ballot(nxl > 0u) & hm);
    wave_lds_fence();
    uint32_t nexc = nx, first = nt;
    if (linked) {
        // the chain through the slots, with a compulsory exception wherever
        // the gap to the next one does not fit b bits
        nexc = first = 0;
        if (valid && t == 0u) {
            __threadfence_block();   // the slots above are stored before the chain's
            const uint64_t lim = b >= 32u ? ~0ull : (1ull << b) - 1u;
            int64_t prev = -1;
            for (uint32_t w = 0; w < k; w++) {
                uint32_t bits = xbl[w];
                while (bits) {
                    const uint32_t p = 32u * w + (uint32_t)__builtin_ctz(bits);
                    bits &= bits - 1u;
                    if (prev >= 0) {
                        while ((uint64_t)((int64_t)p - prev - 1) > lim) {
                            const uint32_t cp = (uint32_t)(prev + (int64_t)(1ull << b));
                            xbl[cp >> 5] |= 1u << (cp & 31u);
                            slot[(uint32_t)prev] = cp - (uint32_t)prev - 1u;
                            prev = cp;
                            nexc++;
                        }
                        slot[(uint32_t)prev] = p - (uint32_t)prev - 1u;
                    } else {
                        first = p;
                    }
                    prev = p;
                    nexc++;
                }
            }
            if (prev >= 0) slot[(uint32_t)prev] = 0u;
        }
        nexc = (uint32_t)__shfl((int)nexc, (int)(lane & 32u));
        first = (uint32_t)__shfl((int)first, (int)(lane & 32u));
        wave_lds_fence();
    }
    if (!valid) return;
    uint32_t *xb = a.xbit + g0 * k / 32u;
    for (uint32_t w = t; w < k; w += 32u) xb[w] = xbl[w];
    if (t == 0u) {
        const uint32_t wcode = nx == 0 ? 0u : maxw <= 8u ? 1u : maxw <= 16u ? 2u : 3u;
        const uint32_t ew = wcode ? 4u << wcode : 0u;
        const uint32_t vals = nexc ? (nexc * ew + 31u) / 32u : 0u;
        const uint32_t xw = !nexc ? 0u : a.pfd_pos == GC_PFD_BITMAP ? 1u + (first * k + 31u) / 32u + vals : vals;
        uint32_t *bk = a.blk + 4u * bi;
        bk[0] = b | (wcode << 6) | (first << 8) | (nexc << 20);
        bk[1] = xw;
    }
}

// Per list, one wave: every block's data-row base and exception-word base
// (exclusive sums over the list's blocks, eight consecutive blocks a lane,
// 512 a step), and the list's C, D and E.
constexpr uint32_t kPfdPer = 8;

__global__ __launch_bounds__(kThreads) void k_pfd_listB(EArgs a) {
    const uint32_t i = blockIdx.x * (kThreads / 64u) + (threadIdx.x >> 6), lane = threadIdx.x & 63u;
    if (i >= a.nlists) return;
    const EList L = a.lists[i];
    const uint32_t nb = L.M / 32u;
    uint32_t rows = 0, xw = 0;   // over the blocks before the step (uniform)
    for (uint32_t j0 = 0; j0 < nb; j0 += 64u * kPfdPer) {
        const uint32_t j1 = j0 + lane * kPfdPer;
        uint32_t r[kPfdPer], x[kPfdPer], sr = 0, sx = 0;
#pragma unroll
        for (uint32_t q = 0; q < kPfdPer; q++) {
            const uint2 bk = j1 + q < nb ? *reinterpret_cast<const uint2 *>(a.blk + 4u * (L.b0 + j1 + q)) : make_uint2(0u, 0u);
            r[q] = bk.x & 63u;
            x[q] = bk.y;
            sr += r[q];
            sx += x[q];
        }
        uint32_t ir = sr, ix = sx;   // inclusive sums over the lanes
#pragma unroll
        for (uint32_t d = 1; d < 64u; d <<= 1) {
            const uint32_t ur = (uint32_t)__shfl_up((int)ir, d), ux = (uint32_t)__shfl_up((int)ix, d);
            ir += lane >= d ? ur : 0u;
            ix += lane >= d ? ux : 0u;
        }
        uint32_t pr = rows + ir - sr, px = xw + ix - sx;
#pragma unroll
        for (uint32_t q = 0; q < kPfdPer; q++) {
            if (j1 + q < nb) *reinterpret_cast<uint2 *>(a.blk + 4u * (L.b0 + j1 + q) + 2u) = make_uint2(pr, px);
            pr += r[q];
            px += x[q];
        }
        rows += (uint32_t)__shfl((int)ir, 63);
        xw += (uint32_t)__shfl((int)ix, 63);
    }
    if (lane == 0) {
        a.sizes[3u * i] = (nb + 3u) / 4u * 4u;
        a.sizes[3u * i + 1u] = a.k * rows;
        a.sizes[3u * i + 2u] = xw;
    }
}

// Appends v (nb bits) to a word stream at out[*w], bit position *acc_n of
// the 64-bit accumulator.
struct WordSink {
    gu32 *out;
    uint32_t stride, w, n;
    uint64_t acc;
    __device__ __forceinline__ void put(uint32_t v, uint32_t nb) {
        if (!nb) return;
        acc |= (uint64_t)(nb >= 32u ? v : (v & ((1u << nb) - 1u))) << n;
        n += nb;
        while (n >= 32u) {
            out[(uint64_t)w * stride] = (uint32_t)acc;
            w++;
            acc >>= 32;
            n -= 32u;
        }
    }
    __device__ __forceinline__ void flush() {
        if (n) out[(uint64_t)w * stride] = (uint32_t)acc;
        if (n) w++;
        acc = 0;
        n = 0;
    }
};

// Half a wave per block, the descriptor to the control area, data rows and
// exception words to their places: lane t assembles whole row words
// (component c of row r at word k*r + c) from the slots they hold; lane 0
// writes the exception area (a block has few exceptions), walking the set
// bits of the bitmap.
__global__ __launch_bounds__(kThreads) void k_pfd_emit(EArgs a) {
    const uint32_t lane = threadIdx.x & 63u, t = threadIdx.x & 31u;
    const uint32_t bi = blockIdx.x * (kThreads / 32u) + (threadIdx.x >> 5);
    if (bi >= a.nblocks) return;
    const uint64_t g0 = 32ull * bi;
    const EList L = a.lists[list_of_tuple(a, g0)];
    const uint32_t j = (uint32_t)((g0 - L.t0) / 32u);
    const uint32_t k = a.k, lk = a.lk;
    const uint32_t *bk = a.blk + 4u * bi;
    const uint32_t desc = bk[0], b = desc & 63u, wcode = (desc >> 6) & 3u, nexc = desc >> 20;
    uint32_t *base = a.out + L.out_off;
    const uint32_t C = base[2], D = base[3];
    if (t == 0u) ((gu32 *)(base + 4u))[j] = desc;
    const uint32_t *slot = a.slot + g0 * k;
    const uint32_t *xb = a.xbit + g0 * k / 32u;
    gu32 *rows = (gu32 *)(base + 4u + C) + (uint64_t)bk[2] * k;
    const uint32_t M = b >= 32u ? 0xFFFFFFFFu : (1u << b) - 1u;
    // tuple tt of component c holds bits [tt*b, tt*b + b) of the
    // component's b words
    for (uint32_t idx = t; idx < (b << lk); idx += 32u) {
        const uint32_t r = idx >> lk, c = idx & (k - 1u), lo = 32u * r;
        const uint32_t ta = lo / b, tb = min(31u, (lo + 31u) / b);
        uint32_t v = 0;
        for (uint32_t tt = ta; tt <= tb; tt++) {
            const uint32_t x = slot[tt * k + c] & M, off = tt * b;
            v |= off >= lo ? x << (off - lo) : x >> (lo - off);
        }
        rows[idx] = v;
    }
    // the tuples with an exception (for the bitmap layout)
    const uint32_t kmask = k >= 32u ? 0xFFFFFFFFu : (1u << k) - 1u;
    const bool any = k <= 32u ? ((xb[(t * k) >> 5] >> ((t * k) & 31u)) & kmask) != 0u
                              : (xb[2u * t] | xb[2u * t + 1u]) != 0u;
    const uint32_t tm = (uint32_t)(__ballot(any) >> (lane & 32u));
    if (t != 0u || !nexc) return;
    WordSink e{(gu32 *)(base + 4u + C + D) + bk[3], 1u, 0u, 0u, 0ull};
    if (a.pfd_pos == GC_PFD_BITMAP) {
        // the tuple mask, then each marked tuple's k exception bits
        e.put(tm, 32u);
        for (uint32_t m = tm; m; m &= m - 1u) {
            const uint32_t tt = (uint32_t)__builtin_ctz(m);
            if (k <= 32u) {
                e.put(xb[(tt * k) >> 5] >> ((tt * k) & 31u), k);
            } else {
                e.put(xb[2u * tt], 32u);
                e.put(xb[2u * tt + 1u], 32u);
            }
        }
        e.flush();
    }
    const uint32_t ew = 4u << wcode;
    const uint64_t x0 = (uint64_t)(j * 32u) * k;
    for (uint32_t w = 0; w < k; w++)
        for (uint32_t m = xb[w]; m; m &= m - 1u) e.put(coded(a, L, x0 + 32u * w + (uint32_t)__builtin_ctz(m)), ew);
    e.flush();
}

// ---- output area -------------------------------------------------------------------------
// One lane per output word: 0, or 1s over a unary Group-Scheme control
// area; the four header words of every stream.
__global__ __launch_bounds__(kThreads) void k_fill(EArgs a, uint32_t w0h, int unary) {
    const uint64_t w = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (w >= a.out_words) return;
    uint32_t lo = a.wl[w >> kTileShift], hi = min(a.wl[(w >> kTileShift) + 1u] + 1u, a.nlists);
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a.lists[mid].out_off <= w) lo = mid;
        else hi = mid;
    }
    const EList L = a.lists[lo];
    const uint64_t r = w - L.out_off;
    const uint32_t C = a.sizes[3u * lo];
    uint32_t v = 0;
    if (r == 0) v = w0h;
    else if (r == 1) v = L.n;
    else if (r == 2) v = C;
    else if (r == 3) v = a.sizes[3u * lo + 1u];
    else if (unary && r < 4u + C) v = 0xFFFFFFFFu;
    a.out[w] = v;
}

}  // namespace gcenc

using namespace gcenc;

namespace {

// Device scratch and pinned host staging, kept per device from one call to
// the next and grown when a call needs more; a call holds its device's
// lock throughout (it returns with its stream synchronised).
struct EncCache {
    std::mutex m;
    char *dev = nullptr, *host = nullptr;
    size_t dev_cap = 0, host_cap = 0;
};
constexpr int kMaxDevices = 64;
EncCache g_cache[kMaxDevices];

constexpr size_t align256(size_t n) { return (n + 255u) & ~(size_t)255u; }

// Carves the call's buffers out of a cached area in order.
struct Bump {
    char *base;
    size_t cap, used;
    template <typename T>
    T *take(size_t n) {
        const size_t bytes = align256(std::max<size_t>(n, 1) * sizeof(T));
        if (used + bytes > cap) return nullptr;
        T *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return p;
    }
};

template <typename T>
gc_status dalloc(T **p, size_t n, Bump &b) {
    *p = b.take<T>(n);
    return *p ? GC_OK : GC_ENOMEM;
}

// Grows a cached area to at least `need` bytes (its old contents are not kept).
gc_status grow(char **area, size_t *cap, size_t need, bool host) {
    if (need <= *cap) return GC_OK;
    if (*area) (void)(host ? hipHostFree(*area) : hipFree(*area));
    *area = nullptr;
    *cap = 0;
    void *q = nullptr;
    if ((host ? hipHostMalloc(&q, need, hipHostMallocDefault) : hipMalloc(&q, need)) != hipSuccess) {
        (void)hipGetLastError();
        return GC_ENOMEM;
    }
    *area = static_cast<char *>(q);
    *cap = need;
    return GC_OK;
}

unsigned grid(uint64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }
// one wave per item
unsigned wave_grid(uint64_t n) { return (unsigned)((n + kThreads / 64 - 1) / (kThreads / 64)); }

#define ENC_OK(x)                                \
    do {                                         \
        if ((x) != hipSuccess) {                 \
            (void)hipGetLastError();             \
            rc = GC_EDEVICE;                     \
            goto done;                           \
        }                                        \
    } while (0)

}  // namespace

extern "C" gc_status gc_encode_lists_gpu(const uint32_t *d_in, const uint64_t *h_in_offs, size_t nlists,
                                         gc_codec codec, const gc_params *p, uint32_t *d_out,
                                         size_t out_cap_words, uint64_t *h_out_offs, void *hip_stream) {
    if (!d_in || !h_in_offs || !p || !d_out || !h_out_offs || nlists == 0 || nlists > 0x0FFFFFFFu)
        return GC_EINVAL;
    if ((int)codec < 0 || (int)codec > 3 || p->k < 4 || p->k > 64 || (p->k & (p->k - 1)) || (p->flags & ~GC_DELTA))
        return GC_EINVAL;
    if (codec == GC_SCHEME && ((p->cg != 1 && p->cg != 2 && p->cg != 4 && p->cg != 8) || p->ld > 2 ||
                               (p->ld == GC_LD_IU && p->cg < 4)))
        return GC_EINVAL;
    if (codec == GC_PFD && (p->zeta_num == 0 || p->zeta_den == 0 || p->zeta_num >= p->zeta_den || p->pfd_pos > 1))
        return GC_EINVAL;
    const uint32_t k = p->k;
    uint32_t lk = 0;
    while ((1u << lk) < k) lk++;
    const uint32_t unit = codec == GC_AFOR ? 8u : codec == GC_PFD ? 32u : 1u;
    // lists, chunks
    std::vector<EList> L(nlists);
    std::vector<EChunk> CH;
    uint64_t ntup = 0;
    uint32_t nblocks = 0;
    for (size_t i = 0; i < nlists; i++) {
        if (h_in_offs[i + 1] < h_in_offs[i]) return GC_EINVAL;
        const uint64_t n = h_in_offs[i + 1] - h_in_offs[i];
        if (n > (1ull << 28)) return GC_EINVAL;   // component bit offsets stay below 2^32
        EList &e = L[i];
        e.in_off = h_in_offs[i];
        e.out_off = 0;
        e.t0 = ntup;
        e.n = (uint32_t)n;
        e.T = (uint32_t)((n + k - 1) / k);
        e.M = (e.T + unit - 1) / unit * unit;
        e.b0 = nblocks;
        if (codec == GC_PFD) nblocks += e.M / 32u;
        const uint32_t units = codec == GC_AFOR ? e.M / 8u : e.T;
        const uint32_t per = codec == GC_AFOR ? kOctChunk : kTupChunk;
        e.c0 = (uint32_t)CH.size();
        e.nch = codec == GC_PFD ? 0u : (units + per - 1u) / per;
        for (uint32_t c = 0; c < e.nch; c++) CH.push_back(EChunk{(uint32_t)i, c * per, std::min(per, units - c * per), 0u});
        ntup += e.M;
    }
    if (ntup * k > (1ull << 34)) return GC_EINVAL;
    // per 256 tuples, the list of the first (the last list with t0 at or
    // before it), and one entry past the last tile
    auto tile_lists = [&](uint64_t units, bool words) {
        std::vector<uint32_t> t((size_t)((units + (1u << kTileShift) - 1) >> kTileShift) + 1u);
        size_t i = 0;
        for (size_t x = 0; x < t.size(); x++) {
            const uint64_t at = (uint64_t)x << kTileShift;
            while (i + 1 < nlists && (words ? L[i + 1].out_off : L[i + 1].t0) <= at) i++;
            t[x] = (uint32_t)i;
        }
        return t;
    };
    const std::vector<uint32_t> TL = tile_lists(ntup, false);
    std::vector<uint32_t> WL;
    const uint32_t nch = (uint32_t)CH.size();
    // the stream-word tile table, sized for streams of up to twice the
    // input words (a larger one takes an allocation of its own)
    const size_t nwl_guess = (size_t)((2u * ntup * k + 16u * nlists) >> kTileShift) + 2u;
    // device scratch in allocation order below, and host staging
    size_t need = align256(nlists * sizeof(EList)) + align256(std::max<size_t>(nch, 1) * sizeof(EChunk)) +
                  align256(TL.size() * 4) + align256(std::max<uint64_t>(ntup, 1)) + align256(12 * nlists) +
                  align256(nwl_guess * 4);
    if (codec == GC_SCHEME || codec == GC_SIMPLE)
        need += align256((codec == GC_SCHEME ? 64ull : 128ull) * std::max(nch, 1u)) + align256(8ull * std::max(nch, 1u)) +
                2 * align256(4 * std::max<uint64_t>(ntup, 1));
    else if (codec == GC_AFOR)
        need += 2 * align256(std::max<uint64_t>(ntup / 8u, 1)) + align256(160ull * std::max(nch, 1u)) +
                align256(48ull * std::max(nch, 1u)) + align256(12ull * std::max(nch, 1u)) +
                align256(4 * std::max<uint64_t>(ntup / 8u, 1));
    else
        need += align256(16ull * std::max(nblocks, 1u)) + align256(4 * std::max<uint64_t>(ntup * k, 1)) +
                align256(4 * (ntup * k / 32u + 1u));
    const size_t hneed = align256(nlists * sizeof(EList)) + align256(std::max<size_t>(nch, 1) * sizeof(EChunk)) +
                         align256(TL.size() * 4) + align256(12 * nlists) + align256(nwl_guess * 4);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return GC_EDEVICE;
    }
    EncCache &cache = g_cache[dev];
    std::lock_guard<std::mutex> lock(cache.m);
    const hipStream_t s = (hipStream_t)hip_stream;
    gc_status rc = GC_OK;
    if ((rc = grow(&cache.dev, &cache.dev_cap, need, false)) || (rc = grow(&cache.host, &cache.host_cap, hneed, true)))
        return rc;
    Bump b{cache.dev, cache.dev_cap, 0};
    Bump hb{cache.host, cache.host_cap, 0};
    EList *h_lists = hb.take<EList>(nlists);
    EChunk *h_chunks = hb.take<EChunk>(nch);
    uint32_t *h_tl = hb.take<uint32_t>(TL.size());
    uint32_t *h_sizes = hb.take<uint32_t>(3 * nlists);
    uint32_t *h_wl = hb.take<uint32_t>(nwl_guess);
    void *wl_own = nullptr;   // the stream-word table, if larger than the guess
    EArgs a;
    std::memset(&a, 0, sizeof(a));
    uint64_t total = 0;
    EList *d_lists = nullptr;
    EChunk *d_chunks = nullptr;
    uint32_t *d_tl = nullptr, *d_wl = nullptr;
    std::memcpy(h_lists, L.data(), nlists * sizeof(EList));
    if (nch) std::memcpy(h_chunks, CH.data(), nch * sizeof(EChunk));
    std::memcpy(h_tl, TL.data(), TL.size() * 4);
    if ((rc = dalloc(&d_lists, nlists, b)) || (rc = dalloc(&d_chunks, nch, b)) || (rc = dalloc(&d_tl, TL.size(), b)))
        goto done;
    ENC_OK(hipMemcpyAsync(d_lists, h_lists, nlists * sizeof(EList), hipMemcpyHostToDevice, s));
    ENC_OK(hipMemcpyAsync(d_tl, h_tl, TL.size() * 4, hipMemcpyHostToDevice, s));
    if (nch) ENC_OK(hipMemcpyAsync(d_chunks, h_chunks, nch * sizeof(EChunk), hipMemcpyHostToDevice, s));
    a.in = d_in;
    a.lists = d_lists;
    a.chunks = d_chunks;
    a.tl = d_tl;
    a.nlists = (uint32_t)nlists;
    a.nchunks = nch;
    a.ntup = ntup;
    a.k = k;
    a.lk = lk;
    a.cg = codec == GC_SCHEME ? p->cg : 1u;
    a.ld = codec == GC_SCHEME ? p->ld : 0u;
    a.delta = (p->flags & GC_DELTA) ? 1u : 0u;
    a.pfd_pos = codec == GC_PFD ? p->pfd_pos : 0u;
    a.zn = p->zeta_num;
    a.zd = p->zeta_den;
    a.nblocks = nblocks;
    a.out = d_out;
    if ((rc = dalloc(&a.W, ntup, b)) || (rc = dalloc(&a.sizes, 3 * nlists, b)) || (rc = dalloc(&d_wl, nwl_guess, b)))
        goto done;
    if (ntup) hipLaunchKernelGGL(k_widths, dim3(grid(ntup)), dim3(kThreads), 0, s, a);
    // sizing
    if (codec == GC_SCHEME) {
        if ((rc = dalloc(&a.chs, 16ull * nch, b)) || (rc = dalloc(&a.chb, 2ull * nch, b)) ||
            (rc = dalloc(&a.tw, ntup, b)) || (rc = dalloc(&a.tw2, ntup, b)))
            goto done;
        if (nch) hipLaunchKernelGGL(k_gsc_chunkA, dim3(wave_grid(nch)), dim3(kThreads), 0, s, a);
        hipLaunchKernelGGL(k_gsc_listB, dim3(grid(nlists)), dim3(kThreads), 0, s, a);
        if (nch) hipLaunchKernelGGL(k_gsc_chunkC, dim3(wave_grid(nch)), dim3(kThreads), 0, s, a);
    } else if (codec == GC_SIMPLE) {
        if ((rc = dalloc(&a.chs, 32ull * nch, b)) || (rc = dalloc(&a.chb, 2ull * nch, b)) ||
            (rc = dalloc(&a.tw, ntup, b)) || (rc = dalloc(&a.tw2, ntup, b)))
            goto done;
        if (ntup) hipLaunchKernelGGL(k_sim_cover, dim3(grid(ntup)), dim3(kThreads), 0, s, a);
        if (nch) hipLaunchKernelGGL(k_sim_chainA, dim3(wave_grid(nch)), dim3(kThreads), 0, s, a);
        hipLaunchKernelGGL(k_sim_listB, dim3(grid(nlists)), dim3(kThreads), 0, s, a);
    } else if (codec == GC_AFOR) {
        if ((rc = dalloc(&a.ob, ntup / 8u, b)) || (rc = dalloc(&a.och, ntup / 8u, b)) ||
            (rc = dalloc(&a.mat, 20ull * nch, b)) || (rc = dalloc(&a.chs, 12ull * nch, b)) ||
            (rc = dalloc(&a.chb, 3ull * nch, b)) || (rc = dalloc(&a.tw, ntup / 8u, b)))
            goto done;
        if (ntup) hipLaunchKernelGGL(k_afor_omax, dim3(grid(ntup / 8u)), dim3(kThreads), 0, s, a);
        if (nch) hipLaunchKernelGGL(k_afor_dpA, dim3(wave_grid(nch)), dim3(kThreads), 0, s, a);
        hipLaunchKernelGGL(k_afor_dpB, dim3(wave_grid(nlists)), dim3(kThreads), 0, s, a);
        if (nch) hipLaunchKernelGGL(k_afor_dpC, dim3(wave_grid(nch)), dim3(kThreads), 0, s, a);
        if (nch) hipLaunchKernelGGL(k_afor_chainA, dim3(wave_grid(nch)), dim3(kThreads), 0, s, a);
        hipLaunchKernelGGL(k_afor_chainB, dim3(grid(nlists)), dim3(kThreads), 0, s, a);
    } else {
        if ((rc = dalloc(&a.blk, 4ull * nblocks, b)) || (rc = dalloc(&a.slot, ntup * k, b)) ||
            (rc = dalloc(&a.xbit, ntup * k / 32u + 1u, b)))
            goto done;
        if (nblocks) hipLaunchKernelGGL(k_pfd_blocks, dim3((nblocks + kThreads / 32 - 1) / (kThreads / 32)), dim3(kThreads), 0, s, a);
        hipLaunchKernelGGL(k_pfd_listB, dim3(wave_grid(nlists)), dim3(kThreads), 0, s, a);
    }
    ENC_OK(hipGetLastError());
    ENC_OK(hipMemcpyAsync(h_sizes, a.sizes, 12 * nlists, hipMemcpyDeviceToHost, s));
    ENC_OK(hipStreamSynchronize(s));
    for (size_t i = 0; i < nlists; i++) {
        L[i].out_off = total;
        h_out_offs[i] = total;
        const uint64_t e4 = ((uint64_t)h_sizes[3 * i + 2] + 3u) / 4u * 4u;
        total += 4ull + h_sizes[3 * i] + h_sizes[3 * i + 1] + e4;
    }
    h_out_offs[nlists] = total;
    if (total > out_cap_words) {
        rc = GC_ENOSPC;
        goto done;
    }
    a.out_words = total;
    WL = tile_lists(total, true);
    if (WL.size() <= nwl_guess) {
        std::memcpy(h_wl, WL.data(), WL.size() * 4);
        ENC_OK(hipMemcpyAsync(d_wl, h_wl, WL.size() * 4, hipMemcpyHostToDevice, s));
    } else {
        if (hipMalloc(&wl_own, WL.size() * 4) != hipSuccess) {
            (void)hipGetLastError();
            rc = GC_ENOMEM;
            goto done;
        }
        d_wl = static_cast<uint32_t *>(wl_own);
        ENC_OK(hipMemcpyAsync(d_wl, WL.data(), WL.size() * 4, hipMemcpyHostToDevice, s));
    }
    a.wl = d_wl;
    std::memcpy(h_lists, L.data(), nlists * sizeof(EList));
    ENC_OK(hipMemcpyAsync(d_lists, h_lists, nlists * sizeof(EList), hipMemcpyHostToDevice, s));
    {
        const uint32_t w0h = header_word0((int)codec, (int)k, codec == GC_SCHEME ? p->cg : 1,
                                          codec == GC_SCHEME ? p->ld : 0, a.delta, codec == GC_PFD ? p->pfd_pos : 0);
        hipLaunchKernelGGL(k_fill, dim3(grid(total)), dim3(kThreads), 0, s, a, w0h,
                           codec == GC_SCHEME && p->ld != GC_LD_BINARY ? 1 : 0);
    }
    if (codec == GC_SIMPLE && nch) hipLaunchKernelGGL(k_sim_chainC, dim3(wave_grid(nch)), dim3(kThreads), 0, s, a);
    if (codec == GC_AFOR && nch) hipLaunchKernelGGL(k_afor_chainC, dim3(wave_grid(nch)), dim3(kThreads), 0, s, a);
    if (codec == GC_PFD) {
        if (nblocks) hipLaunchKernelGGL(k_pfd_emit, dim3((nblocks + kThreads / 32 - 1) / (kThreads / 32)), dim3(kThreads), 0, s, a);
    } else if (ntup) {
        const size_t lds = a.k <= 32u ? sizeof(uint32_t) * kEmitSpan * a.k : 0;
        hipLaunchKernelGGL(k_emit_tuples, dim3(grid(ntup)), dim3(kThreads), lds, s, a, (int)codec);
    }
    ENC_OK(hipGetLastError());
    ENC_OK(hipStreamSynchronize(s));
done:
    (void)hipStreamSynchronize(s);
    if (wl_own) (void)hipFree(wl_own);
    return rc;
}
