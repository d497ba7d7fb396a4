// decode.hip -- gfx950 kernels that decode Group-codec streams and restore
// docIDs by prefix sum.
//
//   locate  Scans the control areas of multi-tile lists, one wave per chunk
//           of 256 control words (128 for a list decoded alone), and records
//           where every decode tile starts: the control unit, the tuples of
//           it that belong to the previous tile, the component data bit
//           offset of the tile's first tuple and (Group-PFD) the exception
//           word offset.  Three kernels: chunk aggregates, their scan within
//           each list, tile starts.
//
//   decode  One kernel per codec class, one tile per wave64 (Group-Simple,
//           Group-Scheme with unary or binary descriptors, Group-AFOR,
//           Group-PFD).  A tile's control words and data rows are loaded
//           first, together; its control units are then parsed into
//           per-tuple records (component bit offset, width) in LDS, the rows
//           are staged in LDS, and each lane produces four consecutive
//           integers per round from two 16-byte rows with a 64-bit funnel
//           shift (v_alignbit_b32) and a mask.  Group-PFD marks its
//           exceptions in an LDS bitmap (linked chains, or the block's tuple
//           and component masks) and patches them by rank.
//
//   carry   A delta list of more than one tile is prefix-summed across its
//           tiles.  A short list (in a batch, one window of 64 tiles; a
//           list decoded alone, up to 2048 tiles) does it in the decode
//           pass: each tile sums its staged rows, publishes the sum and
//           reads its carry from the flags of the tiles before it
//           (decoupled look-back, a bounded wait).  A longer list takes a
//           sum pass that stores the sum of each tile's gaps, one workgroup
//           per list that scans those sums into exclusive carries, and the
//           decode pass that adds the carry to its in-tile scan.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gc.h"
#include "gc_device.h"
#include "gc_format.h"
#include "gc_wave.h"

namespace gcdev {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Pointers into global memory, so accesses compile to global_* rather than
// flat_* instructions.
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) u32x4 gu32x4;

// ---------------------------------------------------------------------------
// Small helpers.

constexpr uint32_t kEpochMask = 0x3FFFFFFFu;

// Epochs of codec class c run c + 1, c + 1 + kClasses, ... (never 0, the
// value of a flag or tile start no run has written), so the epochs of two
// classes never meet: a flag or tile start that one class's run left in a
// scratch slot cannot pass for another class's, whatever the tile ranges of
// later runs (a plan re-tiled by the autotuner, a context's single-list
// scratch shared by every class).
__device__ __forceinline__ uint32_t epoch_next(uint32_t e) {
    const uint32_t n = e + (uint32_t)kClasses;
    return n <= kEpochMask ? n : (e - 1u) % (uint32_t)kClasses + 1u;
}

// Exclusive scan over the workgroup; `tmp` holds kWaves words of LDS.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t *tmp, uint32_t &total) {
    const uint32_t inc = wave_incl_scan(x);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) tmp[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; i++) {
        const uint32_t v = tmp[i];
        pre += i < w ? v : 0u;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return pre + inc - x;
}

__device__ __forceinline__ void latch(Status *st, uint32_t detail) {
    if (atomicCAS(&st->code, 0u, (uint32_t)(int32_t)GC_ECORRUPT) == 0u)
        __hip_atomic_store(&st->detail, detail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Group-Simple selector -> (NUM, BW), Table III, packed as 5-bit fields
// holding NUM-1 and BW-1.
constexpr uint64_t kSimNumM1 = 31ull | 15ull << 5 | 9ull << 10 | 7ull << 15 | 5ull << 20 | 4ull << 25 |
                               3ull << 30 | 2ull << 35 | 1ull << 40 | 0ull << 45;
constexpr uint64_t kSimBwM1 = 0ull | 1ull << 5 | 2ull << 10 | 3ull << 15 | 4ull << 20 | 5ull << 25 |
                              7ull << 30 | 9ull << 35 | 15ull << 40 | 31ull << 45;
__device__ __forceinline__ uint32_t sim_num(uint32_t sel) { return (uint32_t)((kSimNumM1 >> ((5 * sel) & 63u)) & 31u) + 1u; }
__device__ __forceinline__ uint32_t sim_bw(uint32_t sel) { return (uint32_t)((kSimBwM1 >> ((5 * sel) & 63u)) & 31u) + 1u; }

// Group-Scheme binary descriptor units (Table IV widths; 16-bit units of
// three fields at 1-bit CG, 8-bit units otherwise).
struct BinUnit {
    uint32_t fpu, ub, fb, fpw;
};
__device__ __forceinline__ BinUnit bin_unit(int cg) {
    BinUnit u;
    u.fb = cg == 1 ? 5u : cg == 2 ? 4u : cg == 4 ? 3u : 2u;
    u.fpu = cg == 1 ? 3u : cg == 8 ? 4u : 2u;
    u.ub = cg == 1 ? 16u : 8u;
    u.fpw = u.fpu * (32u / u.ub);
    return u;
}
__device__ __forceinline__ uint32_t bin_field_bit(uint32_t t, const BinUnit &u) {
    return (t / u.fpu) * u.ub + (t % u.fpu) * u.fb;
}

// Useful (non-padding) bits of an incomplete-unary control word: in every
// byte, the bits up to and including its last 0.
__device__ __forceinline__ uint32_t iu_useful(uint32_t word) {
    const uint32_t z = ~word;
    uint32_t s = 0;
#pragma unroll
    for (int b = 0; b < 4; b++) {
        const uint32_t zb = (z >> (8 * b)) & 0xFFu;
        s += zb ? 32u - (uint32_t)__builtin_clz(zb) : 0u;
    }
    return s;
}

// Exception words of one Group-PFD block descriptor.
__device__ __forceinline__ uint32_t pfd_exc_words(uint32_t desc, int k, int bitmap) {
    const uint32_t wcode = (desc >> 6) & 3u, first = (desc >> 8) & 0xFFFu, nexc = desc >> 20;
    if (nexc == 0) return 0;
    const uint32_t w = wcode ? (4u << wcode) : 0u;
    const uint32_t vals = (nexc * w + 31u) >> 5;
    return bitmap ? 1u + ((first * (uint32_t)k + 31u) >> 5) + vals : vals;
}


// ===========================================================================
// Locate kernels: reduce -> scan -> emit.

// Position of the k-th (from 0) set bit of x (k < popcount(x)).
__device__ __forceinline__ uint32_t select_bit(uint32_t x, uint32_t k) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t h = 16u; h; h >>= 1) {
        const uint32_t c = (uint32_t)__builtin_popcount(x & ((1u << h) - 1u));
        const bool up = k >= c;
        k = up ? k - c : k;
        x = up ? x >> h : x;
        pos = up ? pos + h : pos;
    }
    return pos;
}


// Tuples of the first ns selectors of a Group-Simple control word, without
// a branch; *bad is set when one of them is not a selector (10..15, that is
// bit 3 and bit 2 or 1 set).
__device__ __forceinline__ uint32_t sim_word_tuples(uint32_t wd, uint32_t ns, bool &bad) {
    const uint32_t valid = ns >= 8u ? 0xFFFFFFFFu : (1u << (4u * ns)) - 1u;
    bad |= ((wd >> 3) & ((wd >> 2) | (wd >> 1)) & 0x11111111u & valid) != 0u;
    uint32_t wt = 0;
#pragma unroll
    for (uint32_t i = 0; i < 8u; i++) wt += i < ns ? sim_num((wd >> (4u * i)) & 15u) : 0u;
    return wt;
}

// Tuples and component data bits of the four frames of a Group-AFOR (vse:
// Group-VSEncoding) control word, without a branch; *bad is set for a width
// above 32 or, in Group-AFOR, a class-3 byte.
__device__ __forceinline__ void afor_word(uint32_t wd, bool vse, uint32_t &wt, uint32_t &wbits, bool &bad) {
    wt = wbits = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint32_t byte = (wd >> (8 * i)) & 0xFFu, b = byte & 63u, cls = byte >> 6;
        bad |= (cls == 3u && !vse) || b > 32u;
        const uint32_t F = frame_tuples(cls);
        wt += F;
        wbits += F * b;
    }
}

__device__ __forceinline__ uint32_t locate_words(const HeaderFields &h, uint32_t T, uint32_t C, uint32_t D) {
    switch (h.codec) {
    case 0: return min(C, ((D >> h.lk) + 7u) >> 3);          // selectors / 8
    case 1:
        if (h.ld == GC_LD_BINARY) {
            const BinUnit u = bin_unit(h.cg);
            return min(C, (T + u.fpw - 1u) / u.fpw);
        }
        return C;
    case 2:
    case 4: return C;
    default: return min(C, (T + 31u) >> 5);                  // one descriptor per block
    }
}

// One lane's view of a control chunk of 64 * W words (one wave per chunk):
// its W consecutive words and their aggregate (tuples, exception words,
// component data bits).
template <int W>
struct LocThread {
    HeaderFields h;
    bool ok, bad;
    uint32_t k, T, TT, D, nwords, wbase;
    uint32_t word[W];
    uint32_t wt[W], wb[W];   // per word: tuples, and component data bits (Group-AFOR, incomplete unary)
    uint32_t vt, ve, vd;
};

// The header comes from the host's copy in the list descriptor (validated
// when the plan was made): the decode tiles compare the stream's own header
// with it, so the locate pass does not wait for that load.
template <int W>
__device__ __forceinline__ void locate_thread(const ListDesc &L, uint32_t chunk, uint32_t lane, LocThread<W> &t) {
    const uint32_t *S = L.stream;
    const uint32_t n = L.n, C = L.C, D = L.D;
    t.ok = header_fields(L.w0, t.h);
    t.k = (uint32_t)t.h.k;
    t.T = t.ok ? (n + t.k - 1u) >> t.h.lk : 0u;
    t.TT = L.tile_ints >> t.h.lk;
    t.D = D;
    t.nwords = t.ok ? locate_words(t.h, t.T, C, D) : 0u;
    t.wbase = (chunk * 64u + lane) * (uint32_t)W;
    t.bad = !t.ok;
    t.vt = t.ve = t.vd = 0;
    const uint32_t *ctrl = S + 4;
    const HeaderFields &h = t.h;
    // 16-byte (8-byte at W = 2) loads, inside the control area (a whole
    // number of 16-byte groups), with no branch between them; a group past
    // the chunk's words reads the header
    static_assert(W == 2 || W % 4 == 0, "words per lane");
    if constexpr (W == 2) {
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        typedef __attribute__((address_space(1))) u32x2 gu32x2;
        const uint32_t w = t.wbase;
        const u32x2 v = *(const gu32x2 *)(w < t.nwords ? ctrl + w : S);
        t.word[0] = w < t.nwords ? v.x : 0u;
        t.word[1] = w + 1u < t.nwords ? v.y : 0u;
    } else {
#pragma unroll
        for (int g = 0; g < W; g += 4) {
            const uint32_t w = t.wbase + (uint32_t)g;
            const u32x4 v = *(const gu32x4 *)(w < t.nwords ? ctrl + w : S);
            t.word[g] = w < t.nwords ? v.x : 0u;
            t.word[g + 1] = w + 1u < t.nwords ? v.y : 0u;
            t.word[g + 2] = w + 2u < t.nwords ? v.z : 0u;
            t.word[g + 3] = w + 3u < t.nwords ? v.w : 0u;
        }
    }
#pragma unroll
    for (int q = 0; q < W; q++) {
        t.wt[q] = t.wb[q] = 0u;
        const uint32_t w = t.wbase + (uint32_t)q;
        if (w >= t.nwords) continue;
        const uint32_t wd = t.word[q];
        switch (h.codec) {
        case 0:   // w < nwords: at least one of the word's selectors exists
            t.wt[q] = sim_word_tuples(wd, min(8u, (D >> h.lk) - 8u * w), t.bad);
            t.vt += t.wt[q];
            break;
        case 1:
            if (h.ld == GC_LD_BINARY) {
                const BinUnit u = bin_unit(h.cg);
                for (uint32_t f = 0; f < u.fpw; f++) {
                    const uint32_t tt = w * u.fpw + f;
                    if (tt >= t.T) break;
                    const uint32_t bit = bin_field_bit(tt, u) & 31u;
                    t.vt += 1u;
                    t.vd += (uint32_t)h.cg * (((wd >> bit) & mask_of(u.fb)) + 1u);
                }
            } else {
                t.wt[q] = (uint32_t)__builtin_popcount(~wd);
                t.vt += t.wt[q];
                if (h.ld == GC_LD_IU) {
                    t.wb[q] = (uint32_t)h.cg * iu_useful(wd);
                    t.vd += t.wb[q];
                }
            }
            break;
        case 2:
        case 4: {
            afor_word(wd, h.codec == 4, t.wt[q], t.wb[q], t.bad);
            t.vt += t.wt[q];
            t.vd += t.wb[q];
            break;
        }
        default: {
            const uint32_t b = wd & 63u;
            if (b > 32u) t.bad = true;
            t.vt += 32u;
            t.vd += 32u * min(b, 32u);
            t.ve += pfd_exc_words(wd, (int)t.k, h.pfd_pos);
            break;
        }
        }
    }
}

// The list and chunk of a locate work item.  Loaded through global-address
// pointers before the kernel stores anything, so the wave-uniform loads
// stay scalar.
__device__ __forceinline__ bool locate_item(const LocateArgs &a, uint32_t item, ListDesc &L, uint32_t &chunk,
                                            uint32_t &list) {
    if (item >= a.total_items) return false;
    if (a.lists) {
        list = ((const gu32 *)a.item_list)[a.item_lo + item];
        const gu32x4 *g = (const gu32x4 *)(a.lists + list);
        union {
            u32x4 v[4];
            ListDesc d;
        } u;
        u.v[0] = g[0];
        u.v[1] = g[1];
        u.v[2] = g[2];
        u.v[3] = g[3];
        L = u.d;
        chunk = a.item_lo + item - L.chunk_base;
    } else {
        L = a.single;
        chunk = item;
        list = 0;
    }
    return true;
}

// Aggregate of every control chunk (a wave per chunk).
template <int W>
__global__ __launch_bounds__(kThreads) void gc_locate_reduce(LocateArgs a) {
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t item = blockIdx.x * (uint32_t)kWaves + wave;
    ListDesc L;
    uint32_t chunk, list;
    // a list of one chunk needs no aggregate (its prefix is zero); the emit
    // kernel checks its words
    if (locate_item(a, item, L, chunk, list) && L.nchunks > 1u) {
        LocThread<W> t;
        locate_thread<W>(L, chunk, lane, t);
        const uint32_t tt = wave_sum(t.vt), te = wave_sum(t.ve), td = wave_sum(t.vd);
        if (t.bad) latch(a.status, kErrLocate);
        if (lane == 0) {
            LocVal v;
            v.tup = tt;
            v.exc = te;
            v.data = td;
            a.agg[L.chunk_base + chunk] = v;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // a new locate run: later kernels of this launch sequence tag and
        // check tile starts with the advanced epoch (stored last, so the
        // loads above stay scalar)
        const uint32_t e = __hip_atomic_load(&a.state->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.state->epoch, epoch_next(e), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Exclusive prefix of the chunk aggregates of one list per wave (lists of
// more than one chunk; a batch lists only those).
__global__ __launch_bounds__(kThreads) void gc_locate_scan(LocateArgs a) {
    const uint32_t item = blockIdx.x * (uint32_t)kWaves + (threadIdx.x >> 6);
    if (item >= a.total_scan) return;
    const ListDesc L = a.lists ? a.lists[a.scan_list[item]] : a.single;
    if (L.nchunks <= 1u) return;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t ct = 0, ce = 0;
    uint64_t cd = 0;
    for (uint32_t c0 = 0; c0 < L.nchunks; c0 += 64u) {
        const uint32_t c = c0 + lane;
        LocVal v;
        v.tup = 0;
        v.exc = 0;
        v.data = 0;
        if (c < L.nchunks) v = a.agg[L.chunk_base + c];
        const uint32_t d = (uint32_t)v.data;   // a chunk holds < 2^23 data bits
        const uint32_t it = wave_incl_scan(v.tup), ie = wave_incl_scan(v.exc), id = wave_incl_scan(d);
        if (c < L.nchunks) {
            LocVal p;
            p.tup = ct + it - v.tup;
            p.exc = ce + ie - v.exc;
            p.data = cd + (id - d);
            a.pre[L.chunk_base + c] = p;
        }
        ct += (uint32_t)__builtin_amdgcn_readlane((int)it, 63);
        ce += (uint32_t)__builtin_amdgcn_readlane((int)ie, 63);
        cd += (uint32_t)__builtin_amdgcn_readlane((int)id, 63);
    }
}

// Tile starts from the chunk prefixes, tagged with this run's epoch (a
// wave per chunk).
template <int W>
__global__ __launch_bounds__(kThreads) void gc_locate_emit(LocateArgs a) {
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t item = blockIdx.x * (uint32_t)kWaves + wave;
    ListDesc L;
    uint32_t chunk, list;
    if (locate_item(a, item, L, chunk, list)) {
        const uint32_t epoch = *(const gu32 *)&a.state->epoch;   // advanced by the reduce kernel
        LocThread<W> t;
        locate_thread<W>(L, chunk, lane, t);
        const uint32_t xt = wave_incl_scan(t.vt) - t.vt;
        const uint32_t xe = wave_incl_scan(t.ve) - t.ve;
        const uint32_t xd = wave_incl_scan(t.vd) - t.vd;
        // a list of one chunk: no aggregate was taken, its prefix is zero
        // and its words are checked here
        LocVal pre;
        if (L.nchunks > 1u) {
            pre = a.pre[L.chunk_base + chunk];
        } else {
            pre.tup = pre.exc = 0u;
            pre.data = 0ull;
            if (t.bad) latch(a.status, kErrLocate);
        }
        const uint32_t TT = t.TT, ntiles = L.ntiles, D = t.D;
        const HeaderFields &h = t.h;
        uint32_t base_t = pre.tup + xt;
        uint64_t base_d = pre.data + xd;
        uint32_t base_e = pre.exc + xe;
        TileInfo *tiles = a.tiles + L.tile_base;
        auto emit = [&](uint32_t m, uint32_t unit, uint32_t sub, uint64_t data, uint32_t exc) {
            TileInfo ti;
            ti.unit = unit;
            ti.sub = sub;
            ti.exc = exc;
            ti.tag = epoch;
            ti.data = data;
            ti.list = list;
            ti.pad = 0;
            tiles[m] = ti;
        };
        if (!t.bad) {
            // Tile m (m >= 1) starts at tuple m * TT.  A unit (selector,
            // frame, control word of unary codes, field, block) holds at
            // most 32 tuples and a tile at least 32, so a unit holds at most
            // one tile start: the lane keeps the next one, m, found with one
            // division, and its walk only compares.
            const bool unary = h.codec == 1 && h.ld != GC_LD_BINARY;
            const uint32_t t0 = h.codec == 1 ? t.wbase * bin_unit(h.cg).fpw : h.codec == 3 ? 32u * t.wbase : base_t;
            // unary codes: the tile starts after the terminator of rank m * TT - 1
            uint32_t m = unary ? base_t / TT + 1u : max(1u, (t0 + TT - 1u) / TT);
            uint32_t B = m * TT;
#pragma unroll
            for (int q = 0; q < W; q++) {
                const uint32_t w = t.wbase + (uint32_t)q;
                if (w >= t.nwords) break;
                const uint32_t wd = t.word[q];
                switch (h.codec) {
                case 0: {
                    // the word's selectors are walked only when a tile starts among them
                    const uint32_t ns = min(8u, (D >> h.lk) - 8u * w);
                    const uint32_t wt = t.wt[q];
                    if (!(m < ntiles && B < base_t + wt)) {
                        base_t += wt;
                        break;
                    }
                    for (uint32_t i = 0; i < ns; i++) {
                        const uint32_t s = 8u * w + i;
                        const uint32_t num = sim_num((wd >> (4u * i)) & 15u);
                        if (m < ntiles && B < base_t + num) {
                            emit(m, s, B - base_t, 32ull * s, 0);
                            m++;
                            B += TT;
                        }
                        base_t += num;
                    }
                    break;
                }
                case 1:
                    if (h.ld == GC_LD_BINARY) {
                        const BinUnit u = bin_unit(h.cg);
                        for (uint32_t f = 0; f < u.fpw; f++) {
                            const uint32_t tt2 = w * u.fpw + f;
                            if (tt2 >= t.T) break;
                            if (tt2 == B && m < ntiles) {
                                emit(m, tt2, 0, base_d, 0);
                                m++;
                                B += TT;
                            }
                            const uint32_t bit = bin_field_bit(tt2, u) & 31u;
                            base_d += (uint32_t)h.cg * (((wd >> bit) & mask_of(u.fb)) + 1u);
                        }
                    } else {
                        // terminators (0 bits) of ranks base_t .. base_t + cnt - 1 end
                        // in this word
                        const uint32_t z = ~wd;
                        const uint32_t cnt = t.wt[q];
                        if (m < ntiles && B - 1u < base_t + cnt) {
                            // (a tile start is rarely more than a few terminators into a word)
                            uint32_t zz = z;
                            for (uint32_t i = 0; i < B - 1u - base_t; i++) zz &= zz - 1u;
                            const uint32_t bit = (uint32_t)__builtin_ctz(zz);
                            const uint32_t pos = 32u * w + bit + 1u;
                            uint64_t d;
                            if (h.ld == GC_LD_CU) {
                                d = (uint64_t)h.cg * pos;
                            } else {
                                // bits above `bit` read as padding: only bytes up to it count
                                const uint32_t upto = bit == 31u ? wd : (wd | ~((2u << bit) - 1u));
                                d = base_d + (uint64_t)h.cg * iu_useful(upto);
                            }
                            emit(m, pos, 0, d, 0);
                            m++;
                            B += TT;
                        }
                        base_t += cnt;
                        base_d += t.wb[q];
                    }
                    break;
                case 2:
                case 4: {
                    // the word's frames are walked only when a tile starts among them
                    const uint32_t wt = t.wt[q], wbits = t.wb[q];
                    if (!(m < ntiles && B < base_t + wt)) {
                        base_t += wt;
                        base_d += wbits;
                        break;
                    }
                    for (int i = 0; i < 4; i++) {
                        const uint32_t byte = (wd >> (8 * i)) & 0xFFu;
                        const uint32_t b = byte & 63u, F = frame_tuples(byte >> 6);
                        if (m < ntiles && B < base_t + F) {
                            const uint32_t sub = B - base_t;
                            emit(m, 4u * w + (uint32_t)i, sub, base_d + (uint64_t)sub * b, 0);
                            m++;
                            B += TT;
                        }
                        base_t += F;
                        base_d += (uint64_t)F * b;
                    }
                    break;
                }
                default: {
                    if (32u * w == B && m < ntiles) {
                        emit(m, w, 0, base_d, base_e);
                        m++;
                        B += TT;
                    }
                    base_d += 32u * min(wd & 63u, 32u);
                    base_e += pfd_exc_words(wd, (int)t.k, h.pfd_pos);
                    break;
                }
                }
            }
        }
    }
}
// ===========================================================================
// Decode kernels.

enum : int { kClsSim = 0, kClsGscU = 1, kClsGscB = 2, kClsAfor = 3, kClsPfd = 4 };

// Decode kernel class of a header word 0 (-1 for a word no decoder accepts).
__device__ __forceinline__ int codec_class_dev(uint32_t w0) {
    HeaderFields h;
    if (!header_fields(w0, h)) return -1;
    return h.codec == 0 ? kClsSim : h.codec == 1 ? (h.ld == GC_LD_BINARY ? kClsGscB : kClsGscU)
                                                 : h.codec == 3 ? kClsPfd : kClsAfor;
}

struct TileCtx {
    const uint32_t *S;
    const uint32_t *ctrl;
    const uint32_t *data;
    HeaderFields h;
    uint32_t n, C, D, k, lk, T, TT, t0, i0, ntup, nint;
    bool has_en;
    TileInfo st, en;
};


// Fills the tile context of tile m (global tile gi) of list L from the
// host's copy of the header (validated when the plan was made; the stream's
// own header is compared with it at the end of the tile's set-up); false if
// the locate pass did not reach the tile in this run.
__device__ __forceinline__ bool tile_ctx(const ListDesc &L, uint32_t m, const TileInfo &s0, const TileInfo &s1,
                                         uint32_t tile, uint32_t loc_tag, TileCtx &c) {
    c.S = L.stream;
    c.n = L.n;
    c.C = L.C;
    c.D = L.D;
    bool ok = header_fields(L.w0, c.h);
    c.k = (uint32_t)c.h.k;
    c.lk = (uint32_t)c.h.lk;
    c.T = (c.n + c.k - 1u) >> c.lk;
    c.TT = tile >> c.lk;
    c.t0 = m * c.TT;
    c.i0 = m * tile;
    ok = ok && c.i0 < c.n;
    c.ntup = ok ? min(c.TT, c.T - c.t0) : 0u;
    c.nint = ok ? min(tile, c.n - c.i0) : 0u;
    c.ctrl = c.S + 4;
    c.data = c.S + 4 + c.C;
    c.has_en = m + 1u < L.ntiles;
    c.st = TileInfo{};
    c.en = TileInfo{};
    if (m > 0u) {
        c.st = s0;
        ok = ok && c.st.tag == loc_tag;
    }
    if (c.has_en) {
        c.en = s1;
        ok = ok && c.en.tag == loc_tag;
    }
    return ok;
}

// The tile starts of tile gi and gi + 1 and the carry of tile gi, loaded
// before the list descriptor (the tile arrays hold one spare entry).
struct TilePre {
    TileInfo s0, s1;
    uint32_t carry;
};

__device__ __forceinline__ TilePre tile_pre(const DecodeArgs &a, uint32_t gi) {
    typedef __attribute__((address_space(1))) const TileInfo gTileInfo;
    const gTileInfo *t = (const gTileInfo *)a.tiles;
    TilePre p;
    p.s0.unit = t[gi].unit;
    p.s0.sub = t[gi].sub;
    p.s0.exc = t[gi].exc;
    p.s0.tag = t[gi].tag;
    p.s0.data = t[gi].data;
    p.s0.list = t[gi].list;
    p.s1.unit = t[gi + 1u].unit;
    p.s1.sub = t[gi + 1u].sub;
    p.s1.exc = t[gi + 1u].exc;
    p.s1.tag = t[gi + 1u].tag;
    p.s1.data = t[gi + 1u].data;
    p.carry = ((const gu32 *)a.carry)[gi];
    return p;
}

// Wave-uniform value, so the compiler keeps what depends on it in scalar
// registers.
__device__ __forceinline__ uint32_t uniform(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }

// The list of a tile, named by its start entry (from global memory in a
// batch, so the wave-uniform loads stay scalar).
__device__ __forceinline__ ListDesc tile_list(const DecodeArgs &a, const TilePre &pre) {
    if (!a.lists) return a.single;
    const gu32x4 *g = (const gu32x4 *)(a.lists + pre.s0.list);
    union {
        u32x4 v[4];
        ListDesc d;
    } u;
    u.v[0] = g[0];
    u.v[1] = g[1];
    u.v[2] = g[2];
    u.v[3] = g[3];
    return u.d;
}

// ===========================================================================
// Wave-tile decode kernels (Group-Simple, Group-Scheme, Group-AFOR, Group-PFD).
//
// Every wave64 decodes its own tile of TW integers with no workgroup
// barrier: a workgroup is only a container of four independent waves, each
// with its own slice of LDS for its tuple records.

template <int TW, int CLS>
struct WaveSmem {
    static constexpr int TTM = TW / 4;
    static constexpr int NCTRL = CLS == kClsSim ? TTM / 8 + 8 : CLS == kClsGscU ? TTM + 8 : 1;
    // 16-byte chunks: the unit records of the Group-Simple / Group-AFOR prologues
    static constexpr int NINFO = CLS == kClsSim ? (TTM + 2) / 2 : CLS == kClsAfor ? (TTM / 8 + 3) / 2 : 0;
    static constexpr int NDATA = TW / 8;   // data rows staged: 16 bits per integer
    static constexpr int cmax(int a, int b) { return a > b ? a : b; }
    // + one chunk: a tile stages its rows when the row after its last fits too
    // (the second row read of a quad may touch it; its bits are masked off)
    static constexpr int NB = cmax(cmax(NDATA + 1, (NCTRL + 3) / 4), NINFO);
    static_assert(NB == NDATA + 1, "staged rows are copied up to NDATA chunks");
    // control words or per-unit record bases while the records are built,
    // then the tile's data rows
    union {
        u32x4 data[NB];
        uint32_t ctrl[4 * NB];
    };
    // tuple records: bit offset (from the tile's first row, < 2^16) and width;
    // the offsets hold unit markers (Group-Simple, Group-AFOR) or terminator
    // positions + 1 (unary Group-Scheme) while the records are built.
    // Group-PFD computes its records from its block words instead.
    static constexpr int NREC = CLS == kClsPfd ? 16 : TTM + 16;
    uint16_t rel[NREC];
    uint8_t bwid[NREC];
    // Group-PFD only: block descriptors, data row and exception word offsets
    // of the tile's blocks and their record words (row offset | width); the
    // exception bitmap of the tile's integers, per bitmap word the
    // exceptions before it (tile-wide) and the bit offset | width code of
    // its first exception value.  The tile's exception words and its
    // exception values in tile order go to the data buffer after the rows,
    // when they fit there.
    static constexpr int NBLK = CLS == kClsPfd ? TW / 128 : 1;
    static constexpr int NBM = CLS == kClsPfd ? TW / 32 : 1;
    uint32_t bdesc[NBLK], brow[NBLK], bxw[NBLK], brec[NBLK];
    uint32_t bmap[NBM], xcnt[NBM], vbit[NBM];
};

// Record of tuple t (bit offset O from the tile's first row, width b): from
// the record arrays, or, for a Group-PFD tile, from the record word (row
// offset << 6 | width) of its 32-tuple block.
struct RecArr {
    const uint16_t *rel;
    const uint8_t *bw;
    __device__ __forceinline__ void operator()(uint32_t t, uint32_t &O, uint32_t &b) const {
        O = rel[t];
        b = bw[t];
    }
};
struct RecBlk {
    const uint32_t *brec;
    __device__ __forceinline__ void operator()(uint32_t t, uint32_t &O, uint32_t &b) const {
        const uint32_t w = brec[t >> 5];
        b = w & 63u;
        O = ((w >> 6) << 5) + __umul24(t & 31u, b);
    }
};


// Tuple records from unit starts.  A unit (selector, frame) u of the tile
// covers the tuples from start_u on; info[u] = {base, bw} such that tuple t
// of it has its component bit offset at base + t * bw.  The unit marks its
// start with u + 1 in the zeroed record array; a running maximum over the
// tuples (in-lane, then across the wave) names every tuple's unit.  Lane l
// owns tuples [l * TPL, (l + 1) * TPL).
template <int TTM>
__device__ __forceinline__ void zero_markers(uint16_t *mk, uint32_t lane) {
    constexpr int W = TTM / 128;   // 32-bit words (two markers) per lane
    uint32_t *p = reinterpret_cast<uint32_t *>(mk) + lane * W;
#pragma unroll
    for (int w = 0; w < W; w++) p[w] = 0u;
}

// Writes lane l's TPL records (tuples l*TPL ..): offsets two to a word,
// widths four to a word.
template <int TPL>
__device__ __forceinline__ void put_records(uint16_t *rel, uint8_t *bwa, uint32_t lane, const uint32_t *r,
                                            const uint32_t *b) {
    uint32_t *pr = reinterpret_cast<uint32_t *>(rel) + lane * (TPL / 2);
#pragma unroll
    for (int w = 0; w < TPL / 2; w++) pr[w] = (r[2 * w] & 0xFFFFu) | (r[2 * w + 1] << 16);
    uint32_t *pb = reinterpret_cast<uint32_t *>(bwa) + lane * (TPL / 4);
#pragma unroll
    for (int w = 0; w < TPL / 4; w++)
        pb[w] = b[4 * w] | (b[4 * w + 1] << 8) | (b[4 * w + 2] << 16) | (b[4 * w + 3] << 24);
}

template <int TTM>
__device__ __forceinline__ void expand_records(uint16_t *rel, uint8_t *bwa, const uint2 *info, uint32_t lane) {
    constexpr int TPL = TTM / 64;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(rel) + lane * (TPL / 2);
    uint32_t mk[TPL];
#pragma unroll
    for (int w = 0; w < TPL / 2; w++) {
        const uint32_t x = src[w];
        mk[2 * w] = x & 0xFFFFu;
        mk[2 * w + 1] = x >> 16;
    }
#pragma unroll
    for (int u = 1; u < TPL; u++) mk[u] = max(mk[u], mk[u - 1]);
    const uint32_t before = wave_shr1(wave_incl_max(mk[TPL - 1]));
    const uint32_t t0 = lane * (uint32_t)TPL;
    uint32_t r[TPL], b[TPL];
#pragma unroll
    for (int u = 0; u < TPL; u++) {
        const uint32_t m = max(max(mk[u], before), 1u) - 1u;
        const uint2 in = info[m];
        r[u] = in.x + (t0 + (uint32_t)u) * in.y;
        b[u] = in.y;
    }
    put_records<TPL>(rel, bwa, lane, r, b);
    wave_lds_sync();
}

// ---- Group-Simple ---------------------------------------------------------
// Selectors are dealt to the lanes 64 at a time (selector i to lane i mod
// 64), read straight from the control words; a wave scan of their tuple
// counts per round places them, and each scatters its unit marker and record
// base for expand_records.
template <int TW, int CE>
__device__ uint32_t wprologue_sim(const TileCtx &c, WaveSmem<TW, kClsSim> &sm, uint32_t lane, uint32_t &dbase,
                                  const uint32_t (&ce)[CE], bool cok) {
    using SM = WaveSmem<TW, kClsSim>;
    const uint32_t S_total = c.D >> c.lk;
    const uint32_t s_first = c.st.unit, sub0 = c.st.sub;
    const uint32_t s_end = c.has_en ? c.en.unit + (c.en.sub ? 1u : 0u) : S_total;
    const uint32_t nsel = s_end - s_first;
    const uint32_t cw0 = s_first >> 3, cw1 = (s_end + 7u) >> 3;
    if (!(s_end <= S_total && s_end > s_first && nsel <= c.TT + 1u && cw1 <= c.C && cok)) return kErrRange;
    static_assert(64 * CE * 4 <= SM::NREC, "the selector words are staged in the width array");
    zero_markers<SM::TTM>(sm.rel, lane);
    // the selector words, loaded before the prologue, staged in the width
    // array (written only once the records are expanded)
    uint32_t *cws = reinterpret_cast<uint32_t *>(sm.bwid);
#pragma unroll
    for (int v = 0; v < CE; v++) {
        const uint32_t i = (uint32_t)v * 64u + lane;
        if (i < cw1 - cw0) cws[i] = ce[v];
    }
    dbase = s_first;
    uint2 *info = reinterpret_cast<uint2 *>(sm.data);
    bool bad = false;
    uint32_t base = 0;   // tuples of the tile before this round's selectors
    wave_lds_sync();     // markers zeroed and words staged before the scatter
    for (uint32_t i0 = 0; i0 < nsel; i0 += 64u) {
        const uint32_t i = i0 + lane;
        const bool in = i < nsel;
        const uint32_t g = s_first + i;
        const uint32_t sel = in ? (cws[(g >> 3) - cw0] >> (4u * (g & 7u))) & 15u : 0u;
        const uint32_t j0 = i == 0u ? sub0 : 0u;
        const uint32_t num = sim_num(sel);
        const bool okj = sel < 10u && num > j0;
        bad |= in && !okj;
        const uint32_t cnt = (in && okj) ? num - j0 : 0u;
        const uint32_t bw = sim_bw(sel);
        const uint32_t inc = wave_incl_scan(cnt);
        const uint32_t start = base + inc - cnt;
        if (cnt) {
            info[i] = make_uint2(32u * i - (start - j0) * bw, bw);
            if (start < c.ntup) sm.rel[start] = (uint16_t)(i + 1u);
        }
        base += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    }
    if (wave_any(bad)) return kErrSelector;
    if (base < c.ntup) return kErrCount;
    wave_lds_sync();
    expand_records<SM::TTM>(sm.rel, sm.bwid, info, lane);
    return 0;
}

// ---- Group-Scheme, unary descriptors ----------------------------------------
// Every 0 bit of the control area ends one tuple's code (bits outside the
// tile's [p0, p1) read as 1).  Terminator r (r-th zero bit of the tile) is
// found in two steps.  A pass over the staged words (64 per round, one per
// lane) counts each word's zeros; their exclusive prefix ZE[w] is the rank
// of word w's first terminator, and each word with zeros leaves its index
// + 1 as a marker at that rank.  Lane l owns tuples t0 = l*TPL .. t0+TPL-1:
// a running maximum over the markers of ranks up to t0 + i (in-lane, then
// across the wave) names the word of terminator t0 + i.  The lane selects
// terminator t0 in its word (rank t0 - ZE[w] among the word's zeros) and
// steps through the next ones with ctz; terminator t0 - 1 comes from the
// lane before (lane 0: the position just before the tile).  A code spans
// the bits after the previous terminator up to its own (incomplete units:
// not across a byte, so it starts at the byte boundary at the latest), and
// its data follow the data of the codes before it.

template <int TW, int CE>
__device__ uint32_t wprologue_gscu(const TileCtx &c, WaveSmem<TW, kClsGscU> &sm, uint32_t lane, uint32_t &dbase,
                                   const uint32_t (&ce)[CE], bool cok) {
    using SM = WaveSmem<TW, kClsGscU>;
    constexpr int TPL = SM::TTM / 64;
    const uint32_t cg = (uint32_t)c.h.cg, umax = 32u / cg;
    const bool iu = c.h.ld == GC_LD_IU;
    const uint32_t p0 = c.st.unit;
    const uint32_t p1 = c.has_en ? c.en.unit : 32u * c.C;
    const uint32_t cw0 = p0 >> 5, cw1 = (p1 + 31u) >> 5;
    const uint32_t nctrl = cw1 - cw0;
    if (!(p1 >= p0 && cw1 <= c.C && nctrl <= (uint32_t)SM::NCTRL && cok)) return kErrRange;
    // the rank markers, in the record offsets until the records are written
    uint16_t *mk = sm.rel;
    zero_markers<SM::TTM>(mk, lane);
    // bits outside the tile's [p0, p1) read as 1
    auto put = [&](uint32_t i, uint32_t v) {
        const uint32_t gw = cw0 + i;
        if (gw == cw0 && (p0 & 31u)) v |= (1u << (p0 & 31u)) - 1u;
        if (gw == (p1 >> 5) && (p1 & 31u)) v |= ~((1u << (p1 & 31u)) - 1u);
        sm.ctrl[i] = v;
    };
    // the first 64 * CE words were loaded before the prologue
#pragma unroll
    for (int v = 0; v < CE; v++) {
        const uint32_t i = (uint32_t)v * 64u + lane;
        if (i < nctrl) put(i, ce[v]);
    }
    const gu32 *ctrl = (const gu32 *)c.ctrl;
    for (uint32_t i = 64u * CE + lane; i < nctrl; i += 64u) put(i, ctrl[cw0 + i]);
    const uint64_t abs0 = iu ? c.st.data : (uint64_t)cg * p0;
    dbase = (uint32_t)(abs0 >> 5);
    const uint32_t p0r = p0 & 31u;   // bit positions count from 32 * cw0
    wave_lds_sync();
    // ZE[w] (16 bits) after the largest control area, and the markers
    static_assert(SM::NCTRL + (SM::NCTRL + 1) / 2 <= 4 * SM::NB, "the word ranks fit the staging buffer");
    uint16_t *ZE = reinterpret_cast<uint16_t *>(sm.ctrl + SM::NCTRL);
    uint32_t run = 0;
    for (uint32_t w0 = 0; w0 < nctrl; w0 += 64u) {
        const uint32_t w = w0 + lane;
        const bool in = w < nctrl;
        const uint32_t cnt = in ? (uint32_t)__builtin_popcount(~sm.ctrl[w]) : 0u;
        const uint32_t inc = wave_incl_scan(cnt);
        const uint32_t ze = run + inc - cnt;
        if (in) ZE[w] = (uint16_t)ze;
        if (cnt && ze < c.ntup) mk[ze] = (uint16_t)(w + 1u);
        run += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    }
    if (run < c.ntup) return kErrCount;
    wave_lds_sync();
    const uint32_t t0 = lane * (uint32_t)TPL;
    // the word of terminator t0 + i: running maximum of the markers
    uint32_t wd[TPL];
    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(mk) + lane * (TPL / 2);
#pragma unroll
        for (int h = 0; h < TPL / 2; h++) {
            const uint32_t x = src[h];
            wd[2 * h] = x & 0xFFFFu;
            wd[2 * h + 1] = x >> 16;
        }
#pragma unroll
        for (int i = 1; i < TPL; i++) wd[i] = max(wd[i], wd[i - 1]);
        const uint32_t before = wave_shr1(wave_incl_max(wd[TPL - 1]));
        // (rank 0's word always holds a marker, so every word index is >= 0;
        // a lane past the tile's tuples repeats the last word with zeros)
#pragma unroll
        for (int i = 0; i < TPL; i++) wd[i] = max(max(wd[i], before), 1u) - 1u;
    }
    // positions of terminators t0 .. t0 + TPL - 1 (garbage past the tile's
    // tuples, which no record uses)
    uint32_t zr[TPL + 1];
    {
        uint32_t m = ~sm.ctrl[wd[0]];
        const uint32_t p = select_bit(m, t0 - (uint32_t)ZE[wd[0]]);
        zr[1] = 32u * wd[0] + p;
        m &= ~(0xFFFFFFFFu >> (31u - p));   // the zeros after it
#pragma unroll
        for (int i = 1; i < TPL; i++) {
            const uint32_t nw = ~sm.ctrl[wd[i]];
            m = wd[i] != wd[i - 1] ? nw : m;
            zr[i + 1] = 32u * wd[i] + (uint32_t)__builtin_ctz(m | 0x80000000u);
            m &= m - 1u;
        }
        const uint32_t prev = wave_shr1(zr[TPL]);
        zr[0] = lane ? prev : p0r - 1u;
    }
    uint32_t st[TPL], un[TPL];
    uint32_t usum = 0;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < TPL; i++) {
        const bool in = t0 + (uint32_t)i < c.ntup;
        const uint32_t zp = zr[i + 1];
        const uint32_t start = iu ? max(zr[i] + 1u, zp & ~7u) : zr[i] + 1u;
        const uint32_t u = zp - start + 1u;
        bad |= in && (u > umax || zp < start);
        st[i] = start;
        un[i] = in ? min(u, umax) : 0u;
        usum += un[i];
    }
    if (wave_any(bad)) return kErrUnary;
    uint32_t us = iu ? wave_incl_scan(usum) - usum : 0u;
    const uint32_t rel0 = (uint32_t)(abs0 & 31u);
    uint32_t ro[TPL], bo[TPL];
#pragma unroll
    for (int i = 0; i < TPL; i++) {
        ro[i] = iu ? rel0 + cg * us : rel0 + cg * (st[i] - p0r);
        bo[i] = cg * un[i];
        us += un[i];
    }
    put_records<TPL>(sm.rel, sm.bwid, lane, ro, bo);
    wave_lds_sync();
    return 0;
}

// Word i (< 64 * CE) of the control words loaded before the prologue, which
// lane i % 64 holds in register i / 64 (every lane takes part).
template <int CE>
__device__ __forceinline__ uint32_t early_word(const uint32_t (&ce)[CE], uint32_t i) {
    uint32_t w = 0;
#pragma unroll
    for (int v = 0; v < CE; v++) {
        const uint32_t x = (uint32_t)__shfl((int)ce[v], (int)(i & 63u));
        w = (i >> 6) == (uint32_t)v ? x : w;
    }
    return w;
}

// ---- Group-Scheme, binary descriptors ---------------------------------------
// The words of the tile's length fields (from the first tuple's on) were
// loaded before the prologue; cok: they lie inside the control area.
template <int TW, int CE>
__device__ uint32_t wprologue_gscb(const TileCtx &c, WaveSmem<TW, kClsGscB> &sm, uint32_t lane, uint32_t &dbase,
                                   const uint32_t (&ce)[CE], bool cok) {
    using SM = WaveSmem<TW, kClsGscB>;
    const uint32_t cg = (uint32_t)c.h.cg;
    const BinUnit bu = bin_unit(c.h.cg);
    constexpr int TPT = SM::TTM / 64;
    static_assert(64 * CE >= SM::TTM / 6 + 2, "the length fields fit the early words");
    if (c.ntup && !cok) return kErrRange;
    const uint32_t w0 = bin_field_bit(c.t0, bu) >> 5;
    uint32_t bw[TPT];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < TPT; j++) {
        const uint32_t tt = lane * TPT + (uint32_t)j;
        const uint32_t bit = bin_field_bit(c.t0 + tt, bu);
        const uint32_t word = early_word<CE>(ce, (bit >> 5) - w0);
        const uint32_t b = tt < c.ntup ? cg * (((word >> (bit & 31u)) & mask_of(bu.fb)) + 1u) : 0u;
        bw[j] = b;
        sum += b;
    }
    const uint64_t abs0 = c.st.data;
    dbase = (uint32_t)(abs0 >> 5);
    uint32_t run = wave_incl_scan(sum) - sum + (uint32_t)(abs0 & 31u);
    uint32_t ro[TPT];
#pragma unroll
    for (int j = 0; j < TPT; j++) {
        ro[j] = run;
        run += bw[j];
    }
    put_records<TPT>(sm.rel, sm.bwid, lane, ro, bw);
    wave_lds_sync();
    return 0;
}

// ---- Group-AFOR ---------------------------------------------------------------
// The frame bytes of the tile (control words from f0 / 4 on) were loaded
// before the prologue.
template <int TW, int CE>
__device__ uint32_t wprologue_afor(const TileCtx &c, WaveSmem<TW, kClsAfor> &sm, uint32_t lane, uint32_t &dbase,
                                   const uint32_t (&ce)[CE]) {
    using SM = WaveSmem<TW, kClsAfor>;
    const uint32_t f0 = c.st.unit, sub0 = c.st.sub;
    const bool vse = c.h.codec == 4;   // Group-VSEncoding: class 3 is a 12-tuple frame
    // frames hold at least 8 tuples, so a tile meets at most TT / 8 + 2 of them
    const uint32_t nfr = min(c.TT / 8u + 2u, 4u * c.C > f0 ? 4u * c.C - f0 : 0u);
    constexpr int FPT = (SM::TTM / 8 + 2 + 63) / 64;
    static_assert(64 * CE * 4 >= SM::TTM / 8 + 2 + 3, "the frame bytes fit the early words");
    uint32_t cnt[FPT], bb[FPT];
    uint32_t csum = 0, bsum = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < FPT; j++) {
        const uint32_t i = lane * FPT + (uint32_t)j;
        const uint32_t f = f0 + i;
        const uint32_t word = early_word<CE>(ce, (f >> 2) - (f0 >> 2));
        cnt[j] = bb[j] = 0u;
        if (i < nfr) {
            const uint32_t byte = (word >> (8u * (f & 3u))) & 0xFFu;
            uint32_t b = byte & 63u;
            const uint32_t cls = byte >> 6;
            if ((cls == 3u && !vse) || b > 32u) {
                bad = true;
                b = 0;
            }
            const uint32_t F = frame_tuples(cls);
            const uint32_t j0 = i == 0u ? sub0 : 0u;
            if (j0 >= F) bad = true;
            else cnt[j] = F - j0;
            bb[j] = b;
            csum += cnt[j];
            bsum += F * b;
        }
    }
    const uint32_t ic = wave_incl_scan(csum), ib = wave_incl_scan(bsum);
    const uint32_t tc = (uint32_t)__builtin_amdgcn_readlane((int)ic, 63);
    if (wave_any(bad)) return kErrFrame;
    if (tc < c.ntup) return kErrCount;
    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)bb[0]);   // frame f0 is lane 0's first
    // the tile start holds the bit offset of its first tuple, sub0 tuples into frame f0
    if ((uint64_t)sub0 * b0 > c.st.data) return kErrFrame;
    const uint64_t fdata0 = c.st.data - (uint64_t)sub0 * b0;
    dbase = (uint32_t)(c.st.data >> 5);
    const uint32_t frel0 = (uint32_t)(fdata0 - 32ull * dbase);
    // frame i of the tile marks its first tuple with i + 1 and records
    // {base, b} with base + t * b the bit offset of tile tuple t of it
    zero_markers<SM::TTM>(sm.rel, lane);
    wave_lds_sync();
    uint2 *info = reinterpret_cast<uint2 *>(sm.data);
    uint32_t st_t = ic - csum, off = ib - bsum;
#pragma unroll
    for (int j = 0; j < FPT; j++) {
        const uint32_t i = lane * FPT + (uint32_t)j;
        const uint32_t b = bb[j];
        const uint32_t j0 = i == 0u ? sub0 : 0u;
        if (cnt[j]) {
            info[i] = make_uint2(frel0 + off + j0 * b - st_t * b, b);
            if (st_t < c.ntup) sm.rel[st_t] = (uint16_t)(i + 1u);
        }
        st_t += cnt[j];
        off += (cnt[j] ? cnt[j] + j0 : 0u) * b;
    }
    wave_lds_sync();
    expand_records<SM::TTM>(sm.rel, sm.bwid, info, lane);
    return 0;
}

// ---- Group-PFD (Section 6.2) --------------------------------------------------
// A tile is a whole number of blocks of 32 tuples.  The prologue reads the
// tile's block descriptors, scans their data rows and exception words, stages
// the tile's exception words in LDS when they fit, and makes the tuple
// records: tuple t of block j has width b_j, at row offset 32 * (the rows of
// the blocks before j) + (t mod 32) * b_j.  Once the data rows are staged,
// pfd_marks sets a bitmap of the tile's exception positions -- from the
// linked chain (the slot of an exception holds the distance to the next
// one) or from the tuple and component masks -- and the unpack replaces the
// values at marked positions with their exception values.

// Exception words of a tile: staged in LDS, or read from the stream.
struct ExcSrc {
    const uint32_t *lds;
    const gu32 *g;
    uint32_t n;
    bool staged;
    __device__ __forceinline__ uint32_t at(uint32_t i) const {
        if (i >= n) return 0u;
        return staged ? lds[i] : g[i];
    }
};

// The tile's block descriptors (lane j: block j) were loaded before the
// prologue; cok: they lie inside the control area.
template <int TW>
__device__ uint32_t wprologue_pfd(const TileCtx &c, WaveSmem<TW, kClsPfd> &sm, uint32_t lane, uint32_t &dbase,
                                  uint64_t stream_words, ExcSrc &xs, uint32_t ce0, bool cok) {
    const uint32_t k = c.k;
    const uint32_t nb = (c.ntup + 31u) >> 5;   // <= NBLK <= 32
    const int bitmap = c.h.pfd_pos;
    uint32_t desc = 0, b = 0, ew = 0;
    bool bad_desc = false;
    if (nb && !cok) return kErrRange;
    if (lane < nb) {
        desc = ce0;
        b = desc & 63u;
        const uint32_t nexc = desc >> 20, wcode = (desc >> 6) & 3u;
        const uint32_t first = (desc >> 8) & 0xFFFu;
        if (b > 32u || nexc > 32u * k || (nexc && !wcode) || (bitmap && first > 32u)) {
            bad_desc = true;
            b = 0;
            desc = 0;
        }
        ew = pfd_exc_words(desc, (int)k, bitmap);
    }
    if (wave_any(bad_desc)) return kErrPfdDesc;
    const uint32_t ib = wave_incl_scan(b), ie = wave_incl_scan(ew);
    const uint32_t xwords = (uint32_t)__builtin_amdgcn_readlane((int)ie, 63);
    if (lane < nb) {
        sm.bdesc[lane] = desc;
        sm.brow[lane] = ib - b;
        sm.bxw[lane] = ie - ew;
        sm.brec[lane] = ((ib - b) << 6) | b;
    }
    dbase = (uint32_t)(c.st.data >> 5);
    const uint64_t ex0 = 4ull + c.C + c.D + c.st.exc;
    if (ex0 + xwords > stream_words) return kErrRange;
    xs.lds = nullptr;   // staged by the tile set-up when they fit
    xs.g = (const gu32 *)c.S + ex0;
    xs.n = xwords;
    xs.staged = false;
    wave_lds_sync();
    return 0;
}

template <int TW, typename W>
__device__ uint32_t pfd_marks(const TileCtx &c, WaveSmem<TW, kClsPfd> &sm, uint32_t lane, W rows, uint32_t nrow,
                              const ExcSrc &xs, uint32_t *xv, uint32_t xv_cap, uint32_t &nexc_tile) {
    // rows staged in LDS, or read from global memory
    constexpr bool STAGED = __is_same(W, const uint32_t *);
    const uint32_t k = c.k, lk = c.lk;
    const uint32_t nb = (c.ntup + 31u) >> 5;
    const uint32_t BI = 32u * k;        // positions per block
    const uint32_t nbw = nb * k;        // bitmap words of the tile's blocks (k per block)
    const bool linked = c.h.pfd_pos == GC_PFD_LINKED;
    for (uint32_t w = lane; w < nbw; w += 64u) sm.bmap[w] = 0u;
    wave_lds_sync();
    bool bad = false;
    if (linked && STAGED) {
        // one lane walks the chain of one block; position p is component
        // p mod k of the block's tuple p / k, at bit (p / k) * b of its rows,
        // and sets its bit in the block's k bitmap words.  The row is
        // clamped to the staged span, whose padding row follows it, so the
        // second read needs no test.
        const uint32_t km1 = k - 1u, rlast = nrow ? nrow - 1u : 0u;
        for (uint32_t j = lane; j < nb; j += 64u) {
            const uint32_t desc = sm.bdesc[j], nexc = desc >> 20, b = desc & 63u, M = mask_of(b);
            const uint32_t o0 = 32u * sm.brow[j];
            uint32_t *bw = sm.bmap + j * k;
            uint32_t p = (desc >> 8) & 0xFFFu;
            for (uint32_t e = 0; e < nexc; e++) {
                if (p >= BI) {
                    bad = true;
                    break;
                }
                const uint32_t O = o0 + __umul24(p >> lk, b);
                const uint32_t at = (min(O >> 5, rlast) << lk) | (p & km1);
                const uint32_t slot = funnel(rows[at + k], rows[at], O) & M;
                atomicOr(bw + (p >> 5), 1u << (p & 31u));
                p += 1u + min(slot, BI);
            }
        }
    } else if (linked) {
        // the same walk over rows in global memory, with clamped reads; at
        // k = 4 the block's four bitmap words stay in registers
        for (uint32_t j = lane; j < nb; j += 64u) {
            const uint32_t desc = sm.bdesc[j], nexc = desc >> 20, b = desc & 63u, M = mask_of(b);
            const uint32_t o0 = 32u * sm.brow[j];
            const uint32_t rlast = nrow ? nrow - 1u : 0u;
            uint32_t p = (desc >> 8) & 0xFFFu;
            uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
            for (uint32_t e = 0; e < nexc; e++) {
                if (p >= BI) {
                    bad = true;
                    break;
                }
                uint32_t slot = 0;
                if (b && nrow) {
                    const uint32_t O = o0 + (p >> lk) * b;
                    const uint32_t row = min(O >> 5, rlast), sh = O & 31u;
                    const uint32_t at = row * k + (p & (k - 1u));
                    const uint32_t lo = rows[at];
                    const uint32_t hi = row < rlast ? rows[at + k] : 0u;
                    slot = funnel(hi, lo, sh) & M;
                }
                const uint32_t bit = 1u << (p & 31u);
                if (k == 4u) {
                    const uint32_t wq = p >> 5;
                    m0 |= wq == 0u ? bit : 0u;
                    m1 |= wq == 1u ? bit : 0u;
                    m2 |= wq == 2u ? bit : 0u;
                    m3 |= wq == 3u ? bit : 0u;
                } else {
                    atomicOr(&sm.bmap[(j * BI + p) >> 5], bit);
                }
                p = slot < BI ? p + slot + 1u : BI;
            }
            if (k == 4u) {
                sm.bmap[4u * j] = m0;
                sm.bmap[4u * j + 1u] = m1;
                sm.bmap[4u * j + 2u] = m2;
                sm.bmap[4u * j + 3u] = m3;
            }
        }
    } else {
        // one lane per tuple: its component mask, if the tuple mask names it
        for (uint32_t x = lane; x < 32u * nb; x += 64u) {
            const uint32_t j = x >> 5, t = x & 31u;
            if (!(sm.bdesc[j] >> 20)) continue;
            const uint32_t xb = sm.bxw[j];
            const uint32_t tm = xs.at(xb);
            if (!((tm >> t) & 1u)) continue;
            const uint32_t r = (uint32_t)__builtin_popcount(tm & ((1u << t) - 1u));
            const uint32_t base = j * BI + t * k;
            if (k < 32u) {
                const uint32_t bit = r * k;
                const uint32_t m = (xs.at(xb + 1u + (bit >> 5)) >> (bit & 31u)) & mask_of(k);
                atomicOr(&sm.bmap[base >> 5], m << (base & 31u));
            } else {
                for (uint32_t h = 0; h < (k >> 5); h++) sm.bmap[(base >> 5) + h] = xs.at(xb + 1u + r * (k >> 5) + h);
            }
        }
    }
    if (wave_any(bad)) return kErrPfdChain;
    wave_lds_sync();
    // exceptions before every bitmap word, tile-wide
    uint32_t run = 0;
    for (uint32_t w0 = 0; w0 < nbw; w0 += 64u) {
        const uint32_t w = w0 + lane;
        const uint32_t cnt = w < nbw ? (uint32_t)__builtin_popcount(sm.bmap[w]) : 0u;
        const uint32_t inc = wave_incl_scan(cnt);
        if (w < nbw) sm.xcnt[w] = run + inc - cnt;
        run += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    }
    wave_lds_sync();
    // per word: bit offset of its first value in the tile's exception words
    // | width code; every block must mark exactly its exception count
    for (uint32_t w = lane; w < nbw; w += 64u) {
        const uint32_t j = w >> lk, desc = sm.bdesc[j], nexc = desc >> 20, wcode = (desc >> 6) & 3u;
        const uint32_t first_w = j << lk, last_w = first_w + k - 1u;
        const uint32_t before = sm.xcnt[w] - sm.xcnt[first_w];
        const uint32_t xb = sm.bxw[j];
        uint32_t vb = xb;
        if (!linked) {
            const uint32_t nt = (desc >> 8) & 0xFFFu;
            vb = xb + 1u + ((nt * k + 31u) >> 5);
            if (w == first_w && nexc && (uint32_t)__builtin_popcount(xs.at(xb)) != nt) bad = true;
        }
        if (w == last_w) {
            const uint32_t total = sm.xcnt[w] + (uint32_t)__builtin_popcount(sm.bmap[w]) - sm.xcnt[first_w];
            if (total != nexc) bad = true;
        }
        const uint32_t ewb = 4u << wcode;
        sm.vbit[w] = ((32u * vb + before * ewb) << 2) | wcode;
        // the word's exception values, in order, to xv when the tile's fit
        if (run <= xv_cap) {
            uint32_t bm = sm.bmap[w], r = sm.xcnt[w], bit = 32u * vb + before * ewb;
            const uint32_t M = mask_of(ewb);
            while (bm) {
                xv[r++] = (xs.at(bit >> 5) >> (bit & 31u)) & M;
                bit += ewb;
                bm &= bm - 1u;
            }
        }
    }
    if (wave_any(bad)) return linked ? kErrPfdChain : kErrBitmap;
    nexc_tile = run;
    wave_lds_sync();
    return 0;
}

// Replaces the marked integers of quad q (tile integers 4q .. 4q + 3): from
// the values in tile order (xv) when the tile's exceptions fit there,
// otherwise from the exception words.
struct PatchSrc {
    const uint32_t *bmap, *vbit, *xcnt, *xv;
    ExcSrc xs;
    bool in_lds;
};

__device__ __forceinline__ void pfd_patch(u32x4 &v, uint32_t q, const PatchSrc &ps) {
    const uint32_t wi = q >> 3, sh4 = (q & 7u) << 2;
    const uint32_t bm = ps.bmap[wi];
    const uint32_t nib = (bm >> sh4) & 15u;
    if (nib) {
        const uint32_t below = (uint32_t)__builtin_popcount(bm & ((1u << sh4) - 1u));
        uint32_t o[4] = {v.x, v.y, v.z, v.w};
        if (ps.in_lds) {
            uint32_t r = ps.xcnt[wi] + below;
#pragma unroll
            for (int j = 0; j < 4; j++)
                if ((nib >> j) & 1u) o[j] = ps.xv[r++];
        } else {
            const uint32_t code = ps.vbit[wi];
            const uint32_t ew = 4u << (code & 3u), M = mask_of(ew);
            uint32_t bit = (code >> 2) + below * ew;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if ((nib >> j) & 1u) {
                    o[j] = (ps.xs.at(bit >> 5) >> (bit & 31u)) & M;
                    bit += ew;
                }
            }
        }
        v = u32x4{o[0], o[1], o[2], o[3]};
    }
}

// Four consecutive integers of quad q from the tuple records and data rows
// (in global memory, or staged in LDS).
template <typename RowPtr>
__device__ __forceinline__ u32x4 extract_quad(uint32_t O, uint32_t bw, uint32_t q, uint32_t kq, RowPtr rows,
                                              uint32_t nrow) {
    u32x4 v = {0u, 0u, 0u, 0u};
    if (bw && nrow) {
        const uint32_t cq = q & (kq - 1u);
        const uint32_t wi = min(O >> 5, nrow - 1u), sh = O & 31u;
        const uint32_t M = mask_of(bw);
        const u32x4 lo = rows[(size_t)wi * kq + cq];
        u32x4 hi = {0u, 0u, 0u, 0u};
        if (sh + bw > 32u) hi = rows[(size_t)min(wi + 1u, nrow - 1u) * kq + cq];
        v.x = funnel(hi.x, lo.x, sh) & M;
        v.y = funnel(hi.y, lo.y, sh) & M;
        v.z = funnel(hi.z, lo.z, sh) & M;
        v.w = funnel(hi.w, lo.w, sh) & M;
    }
    return v;
}

// Copies n 16-byte chunks of data rows into the wave's LDS buffer, four
// loads per lane in flight at a time (all of them at 2048-integer tiles):
// more raised the register count of the larger tiles.
template <int N>
__device__ __forceinline__ void stage_rows(u32x4 *dst, const gu32x4 *src, uint32_t n, uint32_t lane) {
    constexpr int PL = N / 64;
    constexpr int BATCH = PL < 4 ? PL : 4;   // four 16-byte loads in flight per lane
#pragma unroll
    for (int j0 = 0; j0 < PL; j0 += BATCH) {
        u32x4 t[BATCH];
#pragma unroll
        for (int j = 0; j < BATCH; j++) {
            const uint32_t i = (uint32_t)(j0 + j) * 64u + lane;
            if (i < n) t[j] = src[i];
        }
#pragma unroll
        for (int j = 0; j < BATCH; j++) {
            const uint32_t i = (uint32_t)(j0 + j) * 64u + lane;
            if (i < n) dst[i] = t[j];
        }
    }
    wave_lds_sync();
}

__device__ __forceinline__ void store_quad(uint32_t *out, uint32_t ii, uint32_t nint, bool vec, u32x4 o) {
    if (ii >= nint) return;
    if (vec && ii + 4u <= nint) {
        __builtin_nontemporal_store(o, reinterpret_cast<u32x4 *>(out + ii));
    } else {
        out[ii] = o.x;
        if (ii + 1u < nint) out[ii + 1u] = o.y;
        if (ii + 2u < nint) out[ii + 2u] = o.z;
        if (ii + 3u < nint) out[ii + 3u] = o.w;
    }
}

// Sums (SUM) or writes the tile's integers: lane l handles quads l, l + 64,
// ...; a delta tile is scanned in-lane, across the wave with DPP, and from
// the carry of the previous rounds.
template <int R, bool SUM, bool PATCH, typename Rec, typename RowPtr>
__device__ __forceinline__ uint32_t tile_quads(Rec rec, uint32_t tsh, uint32_t kq, RowPtr rows,
                                               uint32_t nrow, uint32_t nint, uint32_t lane, bool delta,
                                               uint32_t carry, uint32_t *out, bool vec, const PatchSrc &ps) {
    uint32_t s = 0;
    const int nr = min(R, (int)((nint + 255u) >> 8));   // rounds that hold integers (wave-uniform)
#pragma unroll 4
    for (int r = 0; r < R; r++) {
        if (r >= nr) continue;
        const uint32_t q = (uint32_t)r * 64u + lane;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (4u * q < nint) {
            uint32_t O, bw;
            rec(q >> tsh, O, bw);
            v = extract_quad(O, bw, q, kq, rows, nrow);
            if constexpr (PATCH) pfd_patch(v, q, ps);
        }
        if constexpr (SUM) {
            s += v.x + v.y + v.z + v.w;
        } else if (delta) {
            v.y += v.x;
            v.z += v.y;
            v.w += v.z;
            const uint32_t inc = wave_incl_scan(v.w);
            const uint32_t add = carry + inc - v.w;
            store_quad(out, 4u * q, nint, vec, u32x4{v.x + add, v.y + add, v.z + add, v.w + add});
            carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        } else {
            store_quad(out, 4u * q, nint, vec, v);
        }
    }
    return s;
}

// The tile's integers from records and LDS-staged rows, lane l taking quads
// l, l + 64, ...: SUM returns the lane's sum of them; otherwise they are
// written (a delta tile scanned in-lane, across the wave with DPP, and from
// the carry of the earlier rounds).  FULL: a whole tile with a 16-byte
// aligned output, so no quad needs a bounds check.  Rows are read without a
// clamp: the row after the last holds padding, and its bits are masked off.
template <int R, bool SUM, bool FULL, bool DELTA, bool PATCH, bool K4, typename Rec>
__device__ __forceinline__ uint32_t quads_lds(Rec rec, const u32x4 *data, uint32_t tsh, uint32_t kq,
                                              uint32_t nint, uint32_t lane, uint32_t carry, uint32_t *out,
                                              bool vec, const PatchSrc &ps) {
    uint32_t s = 0;
    constexpr int U = PATCH ? 2 : (R < 4 ? R : 4);   // deeper unrolling only raised register use
    // rounds that hold integers (wave-uniform; all of them in a full tile)
    const int nr = FULL ? R : min(R, (int)((nint + 255u) >> 8));
#pragma unroll U
    for (int r = 0; r < R; r++) {
        if (r >= nr) continue;
        const uint32_t q = (uint32_t)r * 64u + lane;
        uint32_t O, bw;
        rec(K4 ? q : q >> tsh, O, bw);
        if constexpr (!FULL) {
            const bool in = 4u * q < nint;
            O = in ? O : 0u;
            bw = in ? bw : 0u;
        }
        const uint32_t sh = O & 31u;
        const uint32_t idx = K4 ? O >> 5 : (O >> 5) * kq + (q & (kq - 1u));
        const u32x4 lo = data[idx], hi = data[idx + (K4 ? 1u : kq)];
        const uint32_t M = (uint32_t)(0xFFFFFFFFull >> (32u - bw));
        u32x4 v;
        v.x = funnel(hi.x, lo.x, sh) & M;
        v.y = funnel(hi.y, lo.y, sh) & M;
        v.z = funnel(hi.z, lo.z, sh) & M;
        v.w = funnel(hi.w, lo.w, sh) & M;
        if constexpr (PATCH) {
            if (FULL || 4u * q < nint) pfd_patch(v, q, ps);
        }
        if constexpr (SUM) {
            s += v.x + v.y + v.z + v.w;
        } else {
            if constexpr (DELTA) {
                v.y += v.x;
                v.z += v.y;
                v.w += v.z;
                const uint32_t inc = wave_incl_scan(v.w);
                const uint32_t add = carry + inc - v.w;
                v += add;
                carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
            }
            if constexpr (FULL) __builtin_nontemporal_store(v, (gu32x4 *)out + q);
            else store_quad(out, 4u * q, nint, vec, v);
        }
    }
    return s;
}

// Everything of one tile up to its unpack: context, prologue, staged rows
// and (Group-PFD) exception marks.
template <int TW, int CLS>
struct TileRun {
    TileCtx c;
    PatchSrc ps;
    const u32x4 *rows;
    uint32_t *out;
    uint32_t nint, nrow, kq, tsh;
    bool staged, vec;
};

template <int TW, int CLS>
__device__ __forceinline__ auto tile_recs(const WaveSmem<TW, CLS> &sm) {
    if constexpr (CLS == kClsPfd) return RecBlk{sm.brec};
    else return RecArr{sm.rel, sm.bwid};
}

// Control words [w0, w0 + nw) that the prologue of a tile reads, from the
// tile starts at its two ends: Group-Simple, the words of its selectors;
// Group-Scheme, the words of its unary codes or binary length fields;
// Group-AFOR, the words of its frame bytes; Group-PFD, its block
// descriptors.  CE words per lane of them are loaded before the prologue.
template <int TW, int CLS>
constexpr int ctrl_early_words() {
    return CLS == kClsSim    ? (TW / 32 + 2 + 63) / 64
           : CLS == kClsGscU ? 3
           : CLS == kClsGscB ? (TW / 4 / 6 + 2 + 63) / 64
           : CLS == kClsAfor ? 1
                             : 1;   // Group-PFD: one descriptor per block
}

template <int CLS>
__device__ __forceinline__ void tile_ctrl_words(const TileCtx &c, uint32_t &w0, uint32_t &nw) {
    w0 = nw = 0;
    if constexpr (CLS == kClsSim) {
        const uint32_t s_end = c.has_en ? c.en.unit + (c.en.sub ? 1u : 0u) : c.D >> c.lk;
        w0 = c.st.unit >> 3;
        const uint32_t w1 = (s_end + 7u) >> 3;
        nw = s_end > c.st.unit && w1 > w0 ? w1 - w0 : 0u;
    } else if constexpr (CLS == kClsGscU) {
        const uint32_t p1 = c.has_en ? c.en.unit : 32u * c.C;
        w0 = c.st.unit >> 5;
        const uint32_t w1 = (p1 + 31u) >> 5;
        nw = p1 >= c.st.unit && w1 > w0 ? w1 - w0 : 0u;
    } else if constexpr (CLS == kClsGscB) {   // the words of its tuples' length fields
        if (c.ntup) {
            const BinUnit bu = bin_unit(c.h.cg);
            w0 = bin_field_bit(c.t0, bu) >> 5;
            nw = (bin_field_bit(c.t0 + c.ntup - 1u, bu) >> 5) + 1u - w0;
        }
    } else if constexpr (CLS == kClsAfor) {   // its frame bytes, four to a word
        const uint32_t f0 = c.st.unit;
        const uint32_t nfr = min(c.TT / 8u + 2u, 4u * c.C > f0 ? 4u * c.C - f0 : 0u);
        w0 = f0 >> 2;
        nw = nfr ? ((f0 + nfr + 3u) >> 2) - w0 : 0u;
    } else {   // Group-PFD: the descriptors of its blocks
        w0 = c.t0 >> 5;
        nw = (c.ntup + 31u) >> 5;
    }
}

// Data rows [r0, r1) of a tile, from the tile starts at its two ends (a
// list's last tile runs to the end of the data area).
template <int CLS>
__device__ __forceinline__ void tile_rows(const TileCtx &c, uint32_t Dk, uint32_t &r0, uint32_t &r1) {
    if constexpr (CLS == kClsSim) {   // one row per selector
        r0 = c.st.unit;
        r1 = c.has_en ? c.en.unit + (c.en.sub ? 1u : 0u) : Dk;
    } else {
        r0 = (uint32_t)min(c.st.data >> 5, (uint64_t)Dk);
        r1 = c.has_en ? (uint32_t)min((c.en.data + 31u) >> 5, (uint64_t)Dk) : Dk;
    }
    r1 = min(r1, Dk);
}

template <int TW, int CLS>
__device__ __forceinline__ void tile_setup(const DecodeArgs &a, const ListDesc &L, uint32_t m, const TilePre &pre,
                                           uint32_t loc_tag, WaveSmem<TW, CLS> &sm, uint32_t lane,
                                           TileRun<TW, CLS> &t) {
    using SM = WaveSmem<TW, CLS>;
    TileCtx &c = t.c;
    // the stream's header, loaded now and compared once the prologue's own
    // loads are under way; a vector load (its index a register the compiler
    // cannot see through), so that waiting on scalar loads does not wait
    // for it
    uint32_t vzero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
    const u32x4 hd = ((const gu32x4 *)L.stream)[vzero];
    const bool ok = tile_ctx(L, m, pre.s0, pre.s1, (uint32_t)TW, loc_tag, c);
    // The prologue's control words are loaded first, all at once (no branch
    // between the loads and their wait), so that the prologue waits for
    // them alone; a word past the range reads the stream header.
    constexpr int CE = ctrl_early_words<TW, CLS>();
    uint32_t ce[CE > 0 ? CE : 1];
    bool cok = false;
    if constexpr (CE > 0) {
        uint32_t w0, nw;
        tile_ctrl_words<CLS>(c, w0, nw);
        cok = ok && nw > 0u && w0 + nw <= c.C;
        const gu32 *g = cok ? (const gu32 *)c.ctrl + w0 : (const gu32 *)L.stream;
#pragma unroll
        for (int v = 0; v < CE; v++) {
            const uint32_t i = (uint32_t)v * 64u + lane;
            ce[v] = g[cok && i < nw ? i : 0u];
        }
    }
    // The data rows are loaded into registers before the prologue reads the
    // control words, so that the two loads wait together; they go to LDS
    // once the prologue no longer needs it.  Tiles whose rows do not fit
    // the registers (or whose records end past them) stage after the
    // prologue instead.
    constexpr int EV = SM::NDATA / 64;
    constexpr bool EARLY = EV <= 4;
    const uint32_t Dk = c.D >> c.lk;
    uint32_t r0 = 0, r1 = 0;
    tile_rows<CLS>(c, Dk, r0, r1);
    const uint32_t nch = r1 >= r0 ? (r1 - r0) * (c.k >> 2) : 0u;
    const bool early = EARLY && ok && r1 >= r0 && nch <= (uint32_t)SM::NDATA;
    u32x4 ev[EARLY ? EV : 1];
    if constexpr (EARLY) {
        // unconditional loads (no branch between them and their wait):
        // lanes past the rows, and every lane of a tile that does not load
        // early, read the stream's header instead
        const gu32x4 *g = early ? (const gu32x4 *)c.data + (size_t)r0 * (c.k >> 2) : (const gu32x4 *)L.stream;
#pragma unroll
        for (int v = 0; v < EV; v++) {
            const uint32_t i = (uint32_t)v * 64u + lane;
            ev[v] = g[early && i < nch ? i : 0u];
        }
    }
    // Group-PFD: the tile's exception words likewise (the tile starts give
    // their range; the last tile's run to the end of the stream)
    constexpr int XE = CLS == kClsPfd ? 4 : 1;   // words per lane
    uint32_t xe[XE];
    uint32_t xn = 0;
    if constexpr (CLS == kClsPfd) {
        const uint64_t ex0 = 4ull + c.C + c.D + c.st.exc;
        const uint64_t ex1 = c.has_en ? 4ull + c.C + c.D + c.en.exc : L.stream_words;
        const bool xok = ok && ex0 <= ex1 && ex1 <= L.stream_words && ex1 - ex0 <= 64ull * XE;
        xn = xok ? (uint32_t)(ex1 - ex0) : 0u;
        const gu32 *g = xok ? (const gu32 *)c.S + ex0 : (const gu32 *)L.stream;
#pragma unroll
        for (int v = 0; v < XE; v++) {
            const uint32_t i = (uint32_t)v * 64u + lane;
            xe[v] = g[i < xn ? i : 0u];
        }
    }
    uint32_t dbase = 0, err = ok ? 0u : kErrLocate;
    t.ps = PatchSrc{sm.bmap, sm.vbit, sm.xcnt, nullptr, ExcSrc{nullptr, nullptr, 0u, false}, false};
    if (!err) {
        if constexpr (CLS == kClsSim) err = wprologue_sim<TW, CE>(c, sm, lane, dbase, ce, cok);
        else if constexpr (CLS == kClsGscU) err = wprologue_gscu<TW, CE>(c, sm, lane, dbase, ce, cok);
        else if constexpr (CLS == kClsGscB) err = wprologue_gscb<TW, CE>(c, sm, lane, dbase, ce, cok);
        else if constexpr (CLS == kClsAfor) err = wprologue_afor<TW, CE>(c, sm, lane, dbase, ce);
        else err = wprologue_pfd<TW>(c, sm, lane, dbase, L.stream_words, t.ps.xs, ce[0], cok);
    }
    t.nrow = Dk > dbase ? Dk - dbase : 0u;
    t.kq = c.k >> 2;
    t.rows = reinterpret_cast<const u32x4 *>(c.data) + (size_t)dbase * t.kq;
    t.tsh = c.lk - 2u;
    t.nint = err ? 0u : c.nint;
    // the tile's data rows end with its last record (offsets grow with the tuple)
    uint32_t span = 0;
    if (t.nint) {
        uint32_t lo_bit, lw;
        tile_recs(sm)(c.ntup - 1u, lo_bit, lw);
        span = min(t.nrow, (lo_bit + lw + 31u) >> 5);
    }
    t.staged = (span + 1u) * t.kq <= (uint32_t)SM::NB;
    bool wrote = false;
    if (t.staged && span) {
        if (EARLY && early && dbase == r0 && span * t.kq <= nch) {
#pragma unroll
            for (int v = 0; v < (EARLY ? EV : 1); v++) {
                const uint32_t i = (uint32_t)v * 64u + lane;
                if (i < nch) sm.data[i] = ev[v];
            }
            wrote = true;
        } else {
            stage_rows<SM::NDATA>(sm.data, (const gu32x4 *)t.rows, span * t.kq, lane);
        }
    }
    if constexpr (CLS == kClsPfd) {
        // after the staged rows: the exception words, then the values in tile order
        uint32_t *buf = reinterpret_cast<uint32_t *>(sm.data);
        constexpr uint32_t kBufWords = 4u * (uint32_t)SM::NB;
        uint32_t used = t.staged ? 4u * span * t.kq : 0u;
        ExcSrc &xs = t.ps.xs;
        if (!err && xs.n <= xn && used + xs.n <= kBufWords) {
#pragma unroll
            for (int v = 0; v < XE; v++) {
                const uint32_t i = (uint32_t)v * 64u + lane;
                if (i < xs.n) buf[used + i] = xe[v];
            }
            xs.lds = buf + used;
            xs.staged = true;
            used += xs.n;
            wrote = true;
        }
        if (wrote) wave_lds_sync();
        if (!err) {
            uint32_t nx = 0;
            t.ps.xv = buf + used;
            const uint32_t cap = kBufWords - used;
            err = t.staged ? pfd_marks<TW>(c, sm, lane, reinterpret_cast<const uint32_t *>(sm.data), span, xs,
                                           buf + used, cap, nx)
                           : pfd_marks<TW>(c, sm, lane, (const gu32 *)t.rows, t.nrow, xs, buf + used, cap, nx);
            t.ps.in_lds = nx <= cap;
            if (err) t.nint = 0u;
        }
    } else {
        if (wrote) wave_lds_sync();
    }
    if (!err && (hd.x != L.w0 || hd.y != L.n || hd.z != L.C || hd.w != L.D)) {
        err = kErrHeader;
        t.nint = 0u;
    }
    if (err && lane == 0) latch(a.status, err);
    t.out = L.out + c.i0;
    t.vec = (reinterpret_cast<uintptr_t>(t.out) & 15u) == 0u;
}

// The sum of a set-up tile's integers (wave-uniform).
template <int TW, int CLS>
__device__ __forceinline__ uint32_t tile_total(const TileRun<TW, CLS> &t, WaveSmem<TW, CLS> &sm, uint32_t lane) {
    constexpr int R = TW / 256;
    constexpr bool PATCH = CLS == kClsPfd;
    uint32_t s;
    if (t.staged) {
        const bool full = t.nint == (uint32_t)TW && t.vec;
        const auto rc = tile_recs(sm);
        const u32x4 *d = sm.data;
        if (t.kq == 1u)   // 4-way layout: a quad per tuple
            s = full ? quads_lds<R, true, true, true, PATCH, true>(rc, d, t.tsh, 1u, t.nint, lane, 0u, t.out, t.vec, t.ps)
                     : quads_lds<R, true, false, true, PATCH, true>(rc, d, t.tsh, 1u, t.nint, lane, 0u, t.out, t.vec, t.ps);
        else
            s = full ? quads_lds<R, true, true, true, PATCH, false>(rc, d, t.tsh, t.kq, t.nint, lane, 0u, t.out, t.vec, t.ps)
                     : quads_lds<R, true, false, true, PATCH, false>(rc, d, t.tsh, t.kq, t.nint, lane, 0u, t.out, t.vec, t.ps);
    } else {
        s = tile_quads<R, true, PATCH>(tile_recs(sm), t.tsh, t.kq, t.rows, t.nrow, t.nint, lane, false, 0u, t.out, t.vec,
                                       t.ps);
    }
    return wave_sum(s);
}

// MODE: 0 decode (a delta tile adds carry[gi], the exclusive prefix of the
// tile sums of its list), 1 the tile's sum to carry[gi], 2 decode with the
// carry found in the same pass (decoupled look-back over the flags).
enum : int { kModeDecode = 0, kModeSum = 1, kModeFused = 2 };

// Single-pass carry of tile gi, the m-th of a delta list, with tile sum s
// (wave-uniform).  Every tile but the list's last publishes a flag
// epoch:30 | state:2 | value:32: state 1 with its sum as soon as it has it,
// state 2 with its inclusive prefix once it has its carry.  The carry is
// read from the flags before it, 64 at a time (lane l reads tile
// gi - 1 - l): the nearest inclusive prefix plus the sums after it.  The
// list's first tile publishes its sum as an inclusive prefix, so the
// look-back never leaves the list.  Flags of an earlier run carry another
// epoch and count as not yet written.  A tile waits only for tiles of lower
// index, which every workgroup dispatcher starts first; the wait is bounded
// all the same, and on expiry the error is latched.
constexpr uint64_t kLookbackTicks = 2000000ull;   // 20 ms of the 100 MHz real-time counter
// (a.lb_stall_ticks, set only by tests of the bounded wait, stops the tiles
// from publishing and replaces the limit, so that every look-back expires)

__device__ __forceinline__ void flag_store(unsigned long long *f, unsigned long long v) {
    __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The first window of flags before tile gi (m > 0), read before the tile's
// own sum is ready so that its latency overlaps the sum.
__device__ __forceinline__ unsigned long long lookback_first(const DecodeArgs &a, uint32_t gi, uint32_t m,
                                                             uint32_t lane) {
    const uint32_t first = gi - m;
    const uint32_t j = gi >= first + 1u + lane ? gi - 1u - lane : first;
    return __hip_atomic_load(a.flags + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ uint32_t tile_carry(const DecodeArgs &a, uint32_t gi, uint32_t m, uint32_t ntiles, uint32_t s,
                               uint32_t epoch, uint32_t lane, unsigned long long f0) {
    unsigned long long *flags = a.flags;
    const uint32_t ep = epoch & kEpochMask;
    const unsigned long long tag = (unsigned long long)ep << 34;
    const bool stall = a.lb_stall_ticks != 0u;
    const uint64_t limit = stall ? (uint64_t)a.lb_stall_ticks : kLookbackTicks;
    const bool last = m + 1u >= ntiles || stall;
    if (m == 0u) {
        if (!last && lane == 0) flag_store(flags + gi, tag | (2ull << 32) | s);
        return 0u;
    }
    if (!last && lane == 0) flag_store(flags + gi, tag | (1ull << 32) | s);
    const uint32_t first = gi - m;
    uint32_t acc = 0, base = gi;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (bool fresh = true;; fresh = false) {
        const bool in = base >= first + 1u + lane;
        const uint32_t j = in ? base - 1u - lane : first;
        const unsigned long long f =
            fresh ? f0 : __hip_atomic_load(flags + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t st = (uint32_t)(f >> 34) == ep ? (uint32_t)(f >> 32) & 3u : 0u;
        const uint64_t incl = __ballot(in && st == 2u), wait = __ballot(in && st == 0u);
        if (incl) {
            const uint32_t p = (uint32_t)__builtin_ctzll(incl);
            const uint64_t upto = p == 63u ? ~0ull : (2ull << p) - 1ull;
            if (!(wait & upto)) {
                acc += wave_sum(lane <= p ? (uint32_t)f : 0u);
                break;
            }
        } else if (!wait) {
            // 64 sums and no prefix yet: every lane is inside the list (its
            // first tile never holds a bare sum)
            acc += wave_sum((uint32_t)f);
            base -= 64u;
            continue;
        }
        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
            if (lane == 0) latch(a.status, kErrTimeout);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    if (!last && lane == 0) flag_store(flags + gi, tag | (2ull << 32) | (acc + s));
    return acc;
}

template <int TW, int CLS, int MODE>
__device__ void wave_tile(const DecodeArgs &a, const ListDesc &L, uint32_t m, uint32_t gi, const TilePre &pre,
                          uint32_t loc_tag, WaveSmem<TW, CLS> &sm, uint32_t lane) {
    constexpr int R = TW / 256;
    constexpr bool PATCH = CLS == kClsPfd;
    // no carry needs the sum of a list's last tile
    if constexpr (MODE == kModeSum)
        if (m + 1u >= L.ntiles) return;
    TileRun<TW, CLS> t;
    tile_setup<TW, CLS>(a, L, m, pre, loc_tag, sm, lane, t);
    if constexpr (MODE == kModeSum) {
        const uint32_t s = tile_total<TW, CLS>(t, sm, lane);
        if (lane == 0) a.carry[gi] = s;
        return;
    }
    HeaderFields hl;
    const bool delta = header_fields(L.w0, hl) && hl.delta;
    uint32_t carry0 = 0;
    if (delta && L.ntiles > 1u) {
        if constexpr (MODE == kModeFused) {
            if (L.ntiles <= a.lb_max_tiles) {
                const unsigned long long f0 = m ? lookback_first(a, gi, m, lane) : 0ull;
                // a list's last tile publishes no flag, so it needs no sum
                const uint32_t s = m + 1u < L.ntiles ? tile_total<TW, CLS>(t, sm, lane) : 0u;
                carry0 = tile_carry(a, gi, m, L.ntiles, s, loc_tag, lane, f0);
            } else {
                carry0 = pre.carry;
            }
        } else {
            carry0 = pre.carry;
        }
    }
    const uint32_t nint = t.nint;
    if (t.staged) {
        const u32x4 *d = sm.data;
        const bool full = nint == (uint32_t)TW && t.vec;
        const auto rc = tile_recs(sm);
        const uint32_t kq = t.kq, tsh = t.tsh;
        if (t.c.h.delta) {
            if (kq == 1u) {   // 4-way layout: a quad per tuple
                if (full) quads_lds<R, false, true, true, PATCH, true>(rc, d, tsh, 1u, nint, lane, carry0, t.out, t.vec, t.ps);
                else quads_lds<R, false, false, true, PATCH, true>(rc, d, tsh, 1u, nint, lane, carry0, t.out, t.vec, t.ps);
            } else {
                if (full) quads_lds<R, false, true, true, PATCH, false>(rc, d, tsh, kq, nint, lane, carry0, t.out, t.vec, t.ps);
                else quads_lds<R, false, false, true, PATCH, false>(rc, d, tsh, kq, nint, lane, carry0, t.out, t.vec, t.ps);
            }
        } else {
            if (kq == 1u) {
                if (full) quads_lds<R, false, true, false, PATCH, true>(rc, d, tsh, 1u, nint, lane, 0u, t.out, t.vec, t.ps);
                else quads_lds<R, false, false, false, PATCH, true>(rc, d, tsh, 1u, nint, lane, 0u, t.out, t.vec, t.ps);
            } else {
                if (full) quads_lds<R, false, true, false, PATCH, false>(rc, d, tsh, kq, nint, lane, 0u, t.out, t.vec, t.ps);
                else quads_lds<R, false, false, false, PATCH, false>(rc, d, tsh, kq, nint, lane, 0u, t.out, t.vec, t.ps);
            }
        }
    } else {
        (void)tile_quads<R, false, PATCH>(tile_recs(sm), t.tsh, t.kq, t.rows, t.nrow, nint, lane, t.c.h.delta, carry0, t.out,
                                          t.vec, t.ps);
    }
}

template <int TW, int CLS, int MODE>
// (The Group-PFD tile sums are held to seven waves per SIMD, the LDS limit:
// left alone they took 82 VGPRs and ran five.)
__global__ __launch_bounds__(kThreads, (MODE == kModeSum && CLS == kClsPfd) ? 7 : 1) void gc_wave_kernel(DecodeArgs a) {
    __shared__ WaveSmem<TW, CLS> sm[kWaves];
    const uint32_t wave = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    const uint32_t w = blockIdx.x * (uint32_t)kWaves + wave;
    if (w >= a.count) return;
    const uint32_t gi = a.lo + w;
    const uint32_t loc_tag = *(const gu32 *)&a.loc_state->epoch;   // written by an earlier kernel
    const TilePre pre = tile_pre(a, gi);
    const ListDesc L = tile_list(a, pre);
    // These scalar loads would otherwise be sunk past the set-up's branches,
    // a memory round trip later than the list descriptor; taken here, they
    // arrive with it, before the set-up issues its vector loads.
    asm volatile("" ::"s"(loc_tag), "s"(pre.s0.unit), "s"(pre.s0.sub), "s"(pre.s0.exc), "s"(pre.s0.tag),
                 "s"(pre.s0.data), "s"(pre.s1.unit), "s"(pre.s1.sub), "s"(pre.s1.exc), "s"(pre.s1.tag),
                 "s"(pre.s1.data), "s"(pre.carry));
    wave_tile<TW, CLS, MODE>(a, L, gi - L.tile_base, gi, pre, loc_tag, sm[wave], lane);
}

// ===========================================================================
// Pack kernel: many short lists per wave, decoded together.
//
// A list of one tile still pays a tile's whole chain of dependent loads and
// its prologue for a few hundred integers.  Here a wave takes a pack of up
// to 32 short lists that share one stream format (codec, layout width and
// codec parameters; docID and TF lists mix): lane j loads list j's
// descriptor, wave scans place the lists' streams one after another in the
// wave's LDS staging buffer (16-byte loads, every list's at once) and their
// tuples one after another in the pack's tuple space (each list's first
// tuple at a multiple of 32 / k tuples, so every list -- and every Group-PFD
// block -- starts at a 32-integer boundary of the pack's integer space).
// The control units of all the lists (selectors, unary code words, length
// fields, frame bytes, block descriptors) are then parsed together, lane by
// lane, with scans that restart at each list's first unit; they give one
// record per tuple of the pack: list, data row (a 16-byte chunk of the
// staging buffer), bit shift and width (Group-PFD: computed in the unpack
// from the tuple's block, which a table of the block of every 32 integers
// names).  The unpack walks the pack's quads 64 at a time: each lane makes
// four integers from its tuple's record and two staged rows, Group-PFD
// patches them from a bitmap of the pack's exception positions, and docID
// lists are prefix-summed by a wave scan that restarts at each list's first
// quad.

constexpr uint32_t kPackLists = 32;   // lists per pack (lanes 0 .. 31 hold their descriptors)

// Records of the pack's tuples: list:6 | row chunk:12 | shift:5 | width:6.
__device__ __forceinline__ uint32_t pack_rec(uint32_t j, uint32_t chunk, uint32_t sh, uint32_t bw) {
    return (j << 23) | ((chunk & 0xFFFu) << 11) | (sh << 6) | bw;
}
// The record of a tuple O bits into the column that starts at row chunk c0
// (row O / 32 of the column is chunk c0 + (O / 32) * k/4; chunks and shifts
// in range, as the record builders check, so the fields do not spill).
__device__ __forceinline__ uint32_t pack_rec_at(uint32_t j, uint32_t c0, uint32_t kq, uint32_t O, uint32_t bw) {
    return ((j << 23) | (c0 << 11) | bw) + (O << 6) + (((O >> 5) * (kq - 1u)) << 11);
}

// Capacities of one pack: PI integers of tuple space (PI / 4 tuples), SW
// staged stream words, kPackLists lists.
template <int PI, int SW>
struct PackSmem {
    static constexpr int TUP = PI / 4;
    static constexpr int TPL = TUP / 64;                       // tuples per lane in the record expansion
    static constexpr int NU = SW / 4 > TUP / 8 + (int)kPackLists ? SW / 4 : TUP / 8 + (int)kPackLists;   // selector / frame records
    static constexpr int NBLK = TUP / 32 + (int)kPackLists;    // Group-PFD blocks
    static constexpr int NBM = PI / 32;                        // exception bitmap words
    u32x4 stage[SW / 4 + 16];     // the streams (+ one row of the widest layout, read past a list's last row)
    uint32_t rec[TUP];            // tuple records (unit markers while the records are built);
                                  // Group-PFD: the block of each 32 integers (16 bits)
    u32x4 lst[kPackLists];        // list j: tuple base | delta << 31, n, output pointer (low, high word)
    uint16_t so[kPackLists + 1];  // staging chunk of list j (the pack's total from the last list on)
    uint16_t tb[kPackLists + 1];  // tuple base of list j (likewise)
    uint16_t ub[kPackLists + 1];  // first control unit of list j (likewise)
    // list j: tuples, stage word of its control area, control words, data
    // words, stream words, chunk of its data area (all below 2^16)
    uint16_t lt[6][kPackLists];
    union {
        uint2 info[NU];           // Group-Simple, Group-AFOR: unit {tuple start | bit << 16, record base}
        uint16_t z[TUP];          // unary Group-Scheme: terminator position of each tuple's code
        struct {
            // Group-PFD block: descriptor, first row chunk, exception word,
            // list | first tuple << 8
            u32x4 blk[NBLK];
            uint32_t bmap[NBM], vbit[NBM];
        } p;
    } u;
};

// The list of unit x: the last j with base[j] <= x (base[j] holds the
// pack's total for the lists after its last, so those are never chosen).
__device__ __forceinline__ uint32_t pack_list_of(const uint16_t *base, uint32_t x) {
    uint32_t j = 0;
#pragma unroll
    for (uint32_t step = kPackLists / 2u; step; step >>= 1) j = base[j + step] <= x ? j + step : j;
    return j;
}

// Exclusive scan of x over the lanes of one round, by segment: h is the
// lane (of this round) where the lane's segment starts, negative for a
// segment that began in an earlier round, whose lanes continue the running
// total `carry` of the previous rounds; `carry` is advanced to the total of
// the segment lane 63 belongs to.
__device__ __forceinline__ uint32_t seg_excl_scan(uint32_t x, int h, uint32_t &carry) {
    const uint32_t inc = wave_incl_scan(x);
    const uint32_t hx = (uint32_t)__shfl((int)inc, max(h, 1) - 1);   // the scan just before the segment
    const uint32_t e = inc - x + (h < 0 ? carry : h > 0 ? 0u - hx : 0u);
    carry = (uint32_t)__builtin_amdgcn_readlane((int)(e + x), 63);
    return e;
}
// The lane of round g0 where the segment starting at unit `first` begins.
__device__ __forceinline__ int seg_head(uint32_t first, uint32_t g0) { return (int)first - (int)g0; }

// Unit records (Group-Simple selectors, Group-AFOR frames) to tuple
// records: every unit marked its first tuple with its index + 1; a running
// maximum over the tuples names each tuple's unit.  Lane l owns tuples
// [l * TPL, (l + 1) * TPL).
template <int PI, int SW>
__device__ __forceinline__ void pack_expand(PackSmem<PI, SW> &sm, uint32_t lane, uint32_t kq) {
    using SM = PackSmem<PI, SW>;
    constexpr int TPL = SM::TPL;
    const uint32_t t0 = lane * (uint32_t)TPL;
    uint32_t mk[TPL];
#pragma unroll
    for (int i = 0; i < TPL; i++) mk[i] = sm.rec[t0 + (uint32_t)i];
#pragma unroll
    for (int i = 1; i < TPL; i++) mk[i] = max(mk[i], mk[i - 1]);
    const uint32_t before = wave_shr1(wave_incl_max(mk[TPL - 1]));
#pragma unroll
    for (int i = 0; i < TPL; i++) {
        const uint32_t m = max(max(mk[i], before), 1u) - 1u;
        const uint2 in = sm.u.info[m];
        const uint32_t t = t0 + (uint32_t)i;
        const uint32_t bw = in.y & 63u;
        const uint32_t O = (in.x >> 16) + (t - (in.x & 0xFFFFu)) * bw;
        sm.rec[t] = in.y + (((O >> 5) * kq) << 11) + ((O & 31u) << 6);
    }
    wave_lds_sync();
}

// ---- Group-Simple: one selector per data row --------------------------------
template <int PI, int SW>
__device__ __forceinline__ uint32_t pack_units_sim(PackSmem<PI, SW> &sm, const uint32_t *sw, uint32_t lane, uint32_t U,
                                   uint32_t kq, const uint16_t *Tl, const uint16_t *cwl, const uint16_t *Cl,
                                   const uint16_t *d0l) {
    using SM = PackSmem<PI, SW>;
    uint32_t carry = 0, nu = 0;
    bool bad = false, cnt_bad = false, rng = false;
    for (uint32_t g0 = 0; g0 < U; g0 += 64u) {
        const uint32_t g = g0 + lane;
        const bool in = g < U;
        const uint32_t j = in ? pack_list_of(sm.ub, g) : 0u;
        const uint32_t s = g - sm.ub[j];
        const uint32_t Tj = Tl[j], cw = cwl[j];
        const bool wok = (s >> 3) < Cl[j];
        rng |= in && !wok;
        const uint32_t sel = in && wok ? (sw[cw + (s >> 3)] >> (4u * (s & 7u))) & 15u : 15u;
        const uint32_t num = in && sel < 10u ? sim_num(sel) : 0u;
        const uint32_t st = seg_excl_scan(num, seg_head(sm.ub[j], g0), carry);
        const bool valid = in && st < Tj;
        bad |= valid && sel >= 10u;
        // the list's last selector: its selectors cover its tuples
        if (in && g + 1u == sm.ub[j + 1u] && st + num < Tj) cnt_bad = true;
        const uint64_t ball = __ballot(valid);
        const uint32_t uid = nu + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(ball >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)ball, 0u));
        if (valid && uid < (uint32_t)SM::NU) {
            const uint32_t t = sm.tb[j] + st;
            sm.u.info[uid] = make_uint2(t, pack_rec(j, d0l[j] + s * kq, 0u, sim_bw(sel)));
            sm.rec[t] = uid + 1u;
        }
        nu += (uint32_t)__builtin_popcountll(ball);
    }
    if (wave_any(rng)) return kErrRange;
    if (wave_any(bad)) return kErrSelector;
    if (wave_any(cnt_bad)) return kErrCount;
    if (nu > (uint32_t)SM::NU) return kErrPack;
    return 0;
}

// ---- Group-AFOR / Group-VSEncoding (vse): frame bytes -----------------------
template <int PI, int SW>
__device__ __forceinline__ uint32_t pack_units_afor(PackSmem<PI, SW> &sm, const uint32_t *sw, uint32_t lane, uint32_t U,
                                    uint32_t kq, uint32_t lk, bool vse, const uint16_t *Tl, const uint16_t *cwl,
                                    const uint16_t *Dl, const uint16_t *d0l) {
    using SM = PackSmem<PI, SW>;
    uint32_t c_t = 0, c_b = 0, nu = 0;
    bool bad = false, cnt_bad = false, rng = false;
    for (uint32_t g0 = 0; g0 < U; g0 += 64u) {
        const uint32_t g = g0 + lane;
        const bool in = g < U;
        const uint32_t j = in ? pack_list_of(sm.ub, g) : 0u;
        const uint32_t s = g - sm.ub[j];
        const uint32_t Tj = Tl[j];
        const uint32_t byte = in ? (sw[cwl[j] + (s >> 2)] >> (8u * (s & 3u))) & 0xFFu : 0u;
        const uint32_t cls = byte >> 6, b = byte & 63u;
        const bool fok = (cls != 3u || vse) && b <= 32u;
        const uint32_t F = in ? frame_tuples(fok ? cls : 0u) : 0u;
        const uint32_t bb = fok ? b : 0u;
        const int head = seg_head(sm.ub[j], g0);
        const uint32_t st = seg_excl_scan(F, head, c_t);
        const uint32_t fb = seg_excl_scan(F * bb, head, c_b);
        const bool valid = in && st < Tj;
        bad |= valid && !fok;
        rng |= valid && fb + F * bb > 32u * (Dl[j] >> lk);   // the frame's data inside the data area
        if (in && g + 1u == sm.ub[j + 1u] && st + F < Tj) cnt_bad = true;
        const uint64_t ball = __ballot(valid);
        const uint32_t uid = nu + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(ball >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)ball, 0u));
        if (valid && uid < (uint32_t)SM::NU) {
            const uint32_t t = sm.tb[j] + st;
            sm.u.info[uid] = make_uint2(t | ((fb & 31u) << 16), pack_rec(j, d0l[j] + (fb >> 5) * kq, 0u, bb));
            sm.rec[t] = uid + 1u;
        }
        nu += (uint32_t)__builtin_popcountll(ball);
    }
    if (wave_any(bad)) return kErrFrame;
    if (wave_any(rng)) return kErrRange;
    if (wave_any(cnt_bad)) return kErrCount;
    if (nu > (uint32_t)SM::NU) return kErrPack;
    return 0;
}

// ---- Group-Scheme, binary descriptors: one length field per tuple ----------
template <int PI, int SW>
__device__ __forceinline__ uint32_t pack_recs_gscb(PackSmem<PI, SW> &sm, const uint32_t *sw, uint32_t lane, uint32_t TT,
                                   uint32_t kq, uint32_t lk, uint32_t cg, const uint16_t *Tl,
                                   const uint16_t *cwl, const uint16_t *Cl, const uint16_t *Dl,
                                   const uint16_t *d0l) {
    const BinUnit bu = bin_unit((int)cg);
    uint32_t carry = 0;
    bool bad = false;
    for (uint32_t g0 = 0; g0 < TT; g0 += 64u) {
        const uint32_t g = g0 + lane;
        const bool in = g < TT;
        const uint32_t j = in ? pack_list_of(sm.tb, g) : 0u;
        const uint32_t u = g - sm.tb[j];
        const bool real = in && u < Tl[j];
        const uint32_t bit = bin_field_bit(u, bu);
        const bool wok = (bit >> 5) < Cl[j];
        bad |= real && !wok;
        const uint32_t word = real && wok ? sw[cwl[j] + (bit >> 5)] : 0u;
        const uint32_t b = real && wok ? cg * (((word >> (bit & 31u)) & mask_of(bu.fb)) + 1u) : 0u;
        const uint32_t O = seg_excl_scan(b, seg_head(sm.tb[j], g0), carry);
        bad |= real && O + b > 32u * (Dl[j] >> lk);   // the tuple's data inside the data area
        if (in) sm.rec[g] = pack_rec_at(j, d0l[j], kq, O, b);
    }
    return wave_any(bad) ? kErrRange : 0u;
}

// ---- Group-Scheme, unary descriptors: every 0 bit ends one tuple's code ------
template <int PI, int SW>
__device__ __forceinline__ uint32_t pack_recs_gscu(PackSmem<PI, SW> &sm, const uint32_t *sw, uint32_t lane, uint32_t U,
                                   uint32_t TT, uint32_t kq, uint32_t lk, uint32_t cg, bool iu,
                                   const uint16_t *Tl, const uint16_t *cwl, const uint16_t *Dl,
                                   const uint16_t *d0l) {
    uint32_t carry = 0;
    bool cnt_bad = false;
    // terminator r of list j at z[tb[j] + r] (for r < the list's tuples)
    for (uint32_t g0 = 0; g0 < U; g0 += 64u) {
        const uint32_t g = g0 + lane;
        const bool in = g < U;
        const uint32_t j = in ? pack_list_of(sm.ub, g) : 0u;
        const uint32_t s = g - sm.ub[j];
        const uint32_t Tj = Tl[j];
        uint32_t z = in ? ~sw[cwl[j] + s] : 0u;
        const uint32_t cnt = (uint32_t)__builtin_popcount(z);
        uint32_t r = seg_excl_scan(cnt, seg_head(sm.ub[j], g0), carry);
        if (in && g + 1u == sm.ub[j + 1u] && r + cnt < Tj) cnt_bad = true;
        const uint32_t base = sm.tb[j];
        while (z && r < Tj) {
            sm.u.z[base + r] = (uint16_t)(32u * s + (uint32_t)__builtin_ctz(z));
            z &= z - 1u;
            r++;
        }
    }
    if (wave_any(cnt_bad)) return kErrCount;
    wave_lds_sync();
    const uint32_t umax = 32u / cg;
    uint32_t c_u = 0;
    bool bad = false, rng = false;
    for (uint32_t g0 = 0; g0 < TT; g0 += 64u) {
        const uint32_t g = g0 + lane;
        const bool in = g < TT;
        const uint32_t j = in ? pack_list_of(sm.tb, g) : 0u;
        const uint32_t u = g - sm.tb[j];
        const bool real = in && u < Tl[j];
        const uint32_t zp = real ? (uint32_t)sm.u.z[g] : 0u;
        const uint32_t p1 = real && u ? (uint32_t)sm.u.z[g - 1u] + 1u : 0u;   // just after the previous code
        const uint32_t start = iu ? max(p1, zp & ~7u) : p1;
        const uint32_t un = zp + 1u - start;
        bad |= real && (zp < start || un > umax);
        const uint32_t units = real ? min(un, umax) : 0u;
        const uint32_t us = iu ? seg_excl_scan(units, seg_head(sm.tb[j], g0), c_u) : 0u;
        const uint32_t O = cg * (iu ? us : start);
        rng |= real && O + cg * units > 32u * (Dl[j] >> lk);   // the tuple's data inside the data area
        if (in) sm.rec[g] = pack_rec_at(j, d0l[j], kq, O, cg * units);
    }
    if (wave_any(bad)) return kErrUnary;
    return wave_any(rng) ? kErrRange : 0u;
}

// ---- Group-PFD (Section 6.2): block descriptors, records, exception marks ----
template <int PI, int SW>
__device__ __forceinline__ uint32_t pack_recs_pfd(PackSmem<PI, SW> &sm, const uint32_t *sw, uint32_t lane, uint32_t U,
                                  uint32_t TT, uint32_t k, uint32_t lk, bool bitmap, const uint16_t *Tl,
                                  const uint16_t *cwl, const uint16_t *Cl, const uint16_t *Dl,
                                  const uint16_t *Wl, const uint16_t *d0l) {
    const uint32_t kq = k >> 2;
    const uint32_t BI = 32u * k;
    uint32_t c_r = 0, c_x = 0;
    bool bad = false, rng = false;
    for (uint32_t g0 = 0; g0 < U; g0 += 64u) {
        const uint32_t g = g0 + lane;
        const bool in = g < U;
        const uint32_t j = in ? pack_list_of(sm.ub, g) : 0u;
        const uint32_t s = g - sm.ub[j];
        const uint32_t Cj = Cl[j], Dj = Dl[j];
        const bool sok = s < Cj;
        uint32_t desc = in && sok ? sw[cwl[j] + s] : 0u;
        uint32_t b = desc & 63u;
        const uint32_t nexc = desc >> 20, wcode = (desc >> 6) & 3u, first = (desc >> 8) & 0xFFFu;
        if (b > 32u || nexc > BI || (nexc && !wcode) || (bitmap && first > 32u)) {
            bad |= in;
            desc = 0u;
            b = 0u;
        }
        rng |= in && !sok;
        const uint32_t ew = pfd_exc_words(desc, (int)k, bitmap ? 1 : 0);
        const int head = seg_head(sm.ub[j], g0);
        const uint32_t rows = seg_excl_scan(b, head, c_r);
        const uint32_t xw = seg_excl_scan(ew, head, c_x);
        rng |= in && ((rows + b) << lk > Dj || 4u + Cj + Dj + xw + ew > Wl[j]);
        if (in) {
            // no per-tuple records: the unpack finds a tuple's block by its
            // 32 integers (a list starts at a 32-integer boundary and a
            // block holds 32k integers, so each 32 belong to one block) and
            // its bit offset from the block's first tuple
            const uint32_t c0 = d0l[j] + rows * kq;
            const uint32_t tb = sm.tb[j] + 32u * s;
            sm.u.p.blk[g] = u32x4{desc, c0, cwl[j] + Cj + Dj + xw, j | (tb << 8)};
            const uint32_t nt = min(32u, sm.tb[j + 1u] - min(sm.tb[j + 1u], tb));
            const uint32_t g0i = (tb << lk) >> 5, g1i = ((tb + nt) << lk) >> 5;
            uint16_t *gb = reinterpret_cast<uint16_t *>(sm.rec);
            for (uint32_t x = g0i; x < g1i; x++) gb[x] = (uint16_t)g;
        }
    }
    if (wave_any(bad)) return kErrPfdDesc;
    if (wave_any(rng)) return kErrRange;
    // The exception bitmap over the pack's integers, block by block: a
    // block starts at a 32-integer boundary, so the bitmap words of its
    // integers are its own.  One lane per block marks its exceptions (the
    // linked chain through the slots, or the tuple and component masks) and
    // writes, for each of its words, the staged bit offset of the word's
    // first exception value | width code, from the block's count so far.
    bool chain_bad = false;
    for (uint32_t g = lane; g < U; g += 64u) {
        const u32x4 bk = sm.u.p.blk[g];
        const uint32_t desc = bk.x, c0 = bk.y, xb = bk.z, j = bk.w & 0xFFu;
        const uint32_t s = g - sm.ub[j];
        const uint32_t nexc = desc >> 20, b = desc & 63u, M = mask_of(b), wcode = (desc >> 6) & 3u;
        const uint32_t real_t = min(32u, Tl[j] - 32u * s);       // real tuples of the block (> 0)
        const uint32_t wfirst = ((sm.tb[j] + 32u * s) << lk) >> 5;   // its first bitmap word
        const uint32_t nw = ((real_t << lk) + 31u) >> 5;             // words holding its integers
        const uint32_t ew = 4u << wcode;
        const uint32_t first = (desc >> 8) & 0xFFFu;
        const uint32_t v0 = bitmap ? xb + 1u + ((first * k + 31u) >> 5) : xb;   // its first exception value
        uint32_t *bm = sm.u.p.bmap + wfirst;
        uint32_t *vb = sm.u.p.vbit + wfirst;
        if (!nexc) {
            for (uint32_t w = 0; w < nw; w++) bm[w] = 0u;
            continue;
        }
        if (!bitmap && k == 4u) {
            // 128 positions: each exception's bit goes into the block's
            // words by an LDS or; the words are read back for their counts.
            // A block with b = 0 reads its first data row (masked off).
            for (uint32_t w = 0; w < nw; w++) bm[w] = 0u;
            uint32_t p = first;
            const uint32_t lim = real_t << 2;
            for (uint32_t e = 0; e < nexc; e++) {
                if (p >= lim) {
                    chain_bad = true;
                    break;
                }
                atomicOr(bm + (p >> 5), 1u << (p & 31u));
                const uint32_t O = (p >> 2) * b;
                const uint32_t at = ((c0 + (O >> 5)) << 2) | (p & 3u);
                const uint32_t slot = funnel(sw[at + 4u], sw[at], O) & M;
                p += 1u + min(slot, 128u);
            }
            uint32_t before = 0;
            for (uint32_t w = 0; w < nw; w++) {
                vb[w] = ((32u * v0 + before * ew) << 2) | wcode;
                before += (uint32_t)__builtin_popcount(bm[w]);
            }
            continue;
        }
        for (uint32_t w = 0; w < nw; w++) bm[w] = 0u;
        uint32_t marked = 0;
        if (!bitmap) {
            const uint32_t BI = 32u * k, lim = real_t << lk;
            uint32_t p = first;
            for (uint32_t e = 0; e < nexc; e++) {
                if (p >= lim) {
                    chain_bad = true;
                    break;
                }
                bm[p >> 5] |= 1u << (p & 31u);
                const uint32_t O = (p >> lk) * b, c = p & (k - 1u);
                const uint32_t at = 4u * (c0 + (O >> 5) * kq) + c;
                const uint32_t slot = b ? funnel(sw[at + k], sw[at], O & 31u) & M : 0u;
                p = slot < BI ? p + slot + 1u : BI;
            }
            marked = nexc;
        } else {
            const uint32_t tm = sw[xb];
            if ((uint32_t)__builtin_popcount(tm) != first || (real_t < 32u && (tm >> real_t))) {
                chain_bad = true;
                continue;
            }
            uint32_t m = tm, r = 0;
            while (m) {
                const uint32_t t = (uint32_t)__builtin_ctz(m);
                m &= m - 1u;
                const uint32_t bit = r * k, q = t * k;
                if (k < 32u) {
                    const uint32_t cm = (sw[xb + 1u + (bit >> 5)] >> (bit & 31u)) & mask_of(k);
                    bm[q >> 5] |= cm << (q & 31u);
                    marked += (uint32_t)__builtin_popcount(cm);
                } else {
                    for (uint32_t h = 0; h < (k >> 5); h++) {
                        const uint32_t cm = sw[xb + 1u + (bit >> 5) + h];
                        bm[(q >> 5) + h] = cm;
                        marked += (uint32_t)__builtin_popcount(cm);
                    }
                }
                r++;
            }
        }
        if (marked != nexc) chain_bad = true;
        uint32_t before = 0;
        for (uint32_t w = 0; w < nw; w++) {
            vb[w] = ((32u * v0 + before * ew) << 2) | wcode;
            before += (uint32_t)__builtin_popcount(bm[w]);
        }
    }
    if (wave_any(chain_bad)) return bitmap ? kErrBitmap : kErrPfdChain;
    wave_lds_sync();
    return 0;
}

// The pack's quads, 64 per round: lane l takes quad r * 64 + l of the pack
// (tuple q >> tsh, component quad q mod k/4; K4: k = 4, a quad per tuple).
// A docID list's scan starts at its first quad: lanes of a list that began
// in an earlier round add the running total `carry`, lanes of one that
// begins in this round subtract the scan at the lane before its first.
template <bool PATCH, bool K4, int PI, int SW>
__device__ __forceinline__ void pack_unpack(PackSmem<PI, SW> &sm, uint32_t lane, uint32_t NQ, uint32_t tsh,
                                            uint32_t kq, uint32_t lk, const PatchSrc &ps) {
    uint32_t carry = 0;
    for (uint32_t g0 = 0; g0 < NQ; g0 += 64u) {
        const uint32_t q = g0 + lane;
        const bool in = q < NQ;
        const uint32_t t = K4 ? q : q >> tsh, cq = K4 ? 0u : q & (kq - 1u);
        uint32_t rc;
        if constexpr (PATCH) {
            // Group-PFD: the record from the tuple's block
            const u32x4 bk = sm.u.p.blk[in ? reinterpret_cast<const uint16_t *>(sm.rec)[q >> 3] : 0u];
            const uint32_t b = bk.x & 63u;
            const uint32_t O = __umul24(t - (bk.w >> 8), b);
            rc = in ? pack_rec_at(bk.w & 0xFFu, bk.y, kq, O, b) : 0u;
        } else {
            rc = in ? sm.rec[t] : 0u;
        }
        const u32x4 L = sm.lst[(rc >> 23) & (kPackLists - 1u)];
        const uint32_t tb = L.x & 0x7FFFFFFFu;
        const uint32_t li = K4 ? (t - tb) << 2 : ((t - tb) << lk) + 4u * cq;   // the quad's first integer in its list
        const bool valid = in && li < L.y;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (valid) {
            const uint32_t c = (rc >> 11) & 0xFFFu, sh = (rc >> 6) & 31u, bw = rc & 63u;
            const u32x4 lo = sm.stage[c + cq], hi = sm.stage[c + (K4 ? 1u : kq) + cq];
            const uint32_t M = (uint32_t)(0xFFFFFFFFull >> (32u - bw));
            v.x = funnel(hi.x, lo.x, sh) & M;
            v.y = funnel(hi.y, lo.y, sh) & M;
            v.z = funnel(hi.z, lo.z, sh) & M;
            v.w = funnel(hi.w, lo.w, sh) & M;
            if constexpr (PATCH) pfd_patch(v, q, ps);
        }
        const bool delta = valid && (L.x >> 31);
        if (wave_any(delta)) {
            if (delta) {
                v.y += v.x;
                v.z += v.y;
                v.w += v.z;
            }
            // the list's first quad is its segment's start
            const uint32_t e = seg_excl_scan(delta ? v.w : 0u, seg_head(K4 ? tb : tb * kq, g0), carry);
            if (delta) v += e;
        } else {
            carry = 0u;   // no docID list continues into the next round
        }
        if (valid) {
            gu32 *out = (gu32 *)(((uint64_t)L.w << 32) | L.z) + li;
            const uint32_t n = L.y;
            if ((L.z & 15u) == 0u && li + 4u <= n) {
                __builtin_nontemporal_store(v, (gu32x4 *)out);
            } else {
                out[0] = v.x;
                if (li + 1u < n) out[1] = v.y;
                if (li + 2u < n) out[2] = v.z;
                if (li + 3u < n) out[3] = v.w;
            }
        }
    }
}

// Pack p, decoded by one wave; false after latching an error.
template <int PI, int SW>
__device__ __forceinline__ bool pack_one(const PackArgs &a, PackSmem<PI, SW> &sm, uint32_t p, uint32_t lane) {
    using SM = PackSmem<PI, SW>;
    const uint32_t f0 = ((const gu32 *)a.first)[p], f1 = ((const gu32 *)a.first)[p + 1u];
    const uint32_t np = f1 - f0;
    if (np == 0u || np > kPackLists) {
        if (lane == 0) latch(a.status, kErrPack);
        return false;
    }
    // lane j: list j's descriptor
    union {
        u32x4 v[2];
        PackDesc d;
    } ud;
    ud.v[0] = u32x4{0u, 0u, 0u, 0u};
    ud.v[1] = u32x4{0u, 0u, 0u, 0u};
    const bool mine = lane < np;
    if (mine) {
        const gu32x4 *g = (const gu32x4 *)(a.descs + f0 + lane);
        ud.v[0] = g[0];
        ud.v[1] = g[1];
    }
    const PackDesc d = ud.d;
    // every list of a pack has the stream format of the first (delta aside)
    const uint32_t w0 = uniform(d.w0) & ~(1u << 19);
    HeaderFields h;
    const bool hok = header_fields(w0, h);
    const uint32_t C = d.cd & 0xFFFFu, D = d.cd >> 16;
    const bool same = !mine || (d.w0 & ~(1u << 19)) == w0;
    const uint32_t k = (uint32_t)h.k, lk = (uint32_t)h.lk, kq = k >> 2;
    const uint32_t T = mine ? (d.n + k - 1u) >> lk : 0u;
    const uint32_t tpu = lk >= 5u ? 1u : 32u >> lk;   // tuples per 32 integers
    const uint32_t Tp = (T + tpu - 1u) & ~(tpu - 1u);
    const uint32_t ch = mine ? d.words >> 2 : 0u;
    const bool dok = !mine || (d.n >= 1u && (d.words & 3u) == 0u && (C & 3u) == 0u && 4u + C + D <= d.words &&
                               (D & (k - 1u)) == 0u);
    const int cls = hok ? (h.codec == 0 ? kClsSim : h.codec == 1 ? (h.ld == GC_LD_BINARY ? kClsGscB : kClsGscU)
                                        : h.codec == 3 ? kClsPfd : kClsAfor) : -1;
    // control units of the list
    const uint32_t units = !mine ? 0u
                         : cls == kClsSim  ? D >> lk
                         : cls == kClsAfor ? 4u * C
                         : cls == kClsGscU ? C
                         : cls == kClsPfd  ? (T + 31u) >> 5
                                           : 0u;
    const uint32_t i_ch = wave_incl_scan(ch), i_t = wave_incl_scan(Tp), i_u = wave_incl_scan(units);
    const uint32_t tot_ch = (uint32_t)__builtin_amdgcn_readlane((int)i_ch, 63);
    const uint32_t TT = (uint32_t)__builtin_amdgcn_readlane((int)i_t, 63);
    const uint32_t U = (uint32_t)__builtin_amdgcn_readlane((int)i_u, 63);
    if (wave_any(!same || !dok) || !hok || cls < 0) {
        if (lane == 0) latch(a.status, kErrHeader);
        return false;
    }
    // a list with tuples but no control units (Group-Simple, unary
    // Group-Scheme, Group-AFOR) would leave its tuples unclaimed
    if (wave_any(mine && T && !units && cls != kClsGscB)) {
        if (lane == 0) latch(a.status, kErrCount);
        return false;
    }
    if (tot_ch > (uint32_t)SW / 4u || TT > (uint32_t)SM::TUP || (TT << lk) > (uint32_t)PI ||
        (cls == kClsPfd && U > (uint32_t)SM::NBLK)) {
        if (lane == 0) latch(a.status, kErrPack);
        return false;
    }
    const uint32_t so = i_ch - ch, tbase = i_t - Tp;
    if (lane <= kPackLists) {
        sm.so[lane] = (uint16_t)(mine ? so : tot_ch);
        sm.tb[lane] = (uint16_t)(mine ? tbase : TT);
        sm.ub[lane] = (uint16_t)(mine ? i_u - units : U);
    }
    // (lanes past the pack's lists: no integers, so nothing is ever stored for them)
    const uint64_t op = reinterpret_cast<uint64_t>(d.out);
    if (lane < kPackLists)
        sm.lst[lane] = mine ? u32x4{tbase | ((d.w0 >> 19) & 1u) << 31, d.n, (uint32_t)op, (uint32_t)(op >> 32)}
                            : u32x4{0u, 0u, 0u, 0u};
    wave_lds_sync();
    // the pack's streams, chunk c to stage[c]: the list of a chunk by binary
    // search over the offsets, its stream pointer from that list's lane;
    // four 16-byte loads per lane in flight
    const uint64_t sp = reinterpret_cast<uint64_t>(d.stream);
    constexpr int RNDS = (SW / 4 + 63) / 64;
    constexpr int BATCH = RNDS < 4 ? RNDS : 4;
#pragma unroll
    for (int r0 = 0; r0 < RNDS; r0 += BATCH) {
        if ((uint32_t)r0 * 64u >= tot_ch) break;
        u32x4 t[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; b++) {
            const uint32_t cidx = (uint32_t)(r0 + b) * 64u + lane;
            const uint32_t j = pack_list_of(sm.so, cidx);
            const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)sp, (int)j);
            const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(sp >> 32), (int)j);
            const gu32x4 *src = reinterpret_cast<const gu32x4 *>(((uint64_t)hi << 32) | lo);
            if (cidx < tot_ch) t[b] = src[cidx - sm.so[j]];
        }
#pragma unroll
        for (int b = 0; b < BATCH; b++) {
            const uint32_t cidx = (uint32_t)(r0 + b) * 64u + lane;
            if (cidx < tot_ch) sm.stage[cidx] = t[b];
        }
    }
    wave_lds_sync();
    const uint32_t *sw = reinterpret_cast<const uint32_t *>(sm.stage);
    // every list's staged header against its descriptor
    const uint32_t cwo = 4u * so + 4u;   // stage word of the control area
    bool hbad = false;
    if (mine) hbad = sw[4u * so] != d.w0 || sw[4u * so + 1u] != d.n || sw[4u * so + 2u] != C || sw[4u * so + 3u] != D;
    if (wave_any(hbad)) {
        if (lane == 0) latch(a.status, kErrHeader);
        return false;
    }
    // per-list values for the record builders
    uint16_t *Tl = sm.lt[0], *cwl = sm.lt[1], *Cl = sm.lt[2], *Dl = sm.lt[3], *Wl = sm.lt[4], *d0l = sm.lt[5];
    if (lane < kPackLists) {
        Tl[lane] = (uint16_t)T;
        cwl[lane] = (uint16_t)cwo;
        Cl[lane] = (uint16_t)C;
        Dl[lane] = (uint16_t)D;
        Wl[lane] = (uint16_t)(mine ? d.words : 0u);
        d0l[lane] = (uint16_t)(so + 1u + (C >> 2));   // chunk of the data area
    }
    wave_lds_sync();
    uint32_t err = 0;
    if (cls == kClsSim || cls == kClsAfor) {
        for (uint32_t t = lane; t < (uint32_t)SM::TUP; t += 64u) sm.rec[t] = 0u;
        wave_lds_sync();
        err = cls == kClsSim ? pack_units_sim(sm, sw, lane, U, kq, Tl, cwl, Cl, d0l)
                             : pack_units_afor(sm, sw, lane, U, kq, lk, h.codec == 4, Tl, cwl, Dl, d0l);
        wave_lds_sync();
        if (!err) pack_expand(sm, lane, kq);
    } else if (cls == kClsGscB) {
        err = pack_recs_gscb(sm, sw, lane, TT, kq, lk, (uint32_t)h.cg, Tl, cwl, Cl, Dl, d0l);
    } else if (cls == kClsGscU) {
        err = pack_recs_gscu(sm, sw, lane, U, TT, kq, lk, (uint32_t)h.cg, h.ld == GC_LD_IU, Tl, cwl, Dl, d0l);
    } else {
        err = pack_recs_pfd(sm, sw, lane, U, TT, k, lk, h.pfd_pos != 0, Tl, cwl, Cl, Dl, Wl, d0l);
    }
    if (err) {
        if (lane == 0) latch(a.status, err);
        return false;
    }
    wave_lds_sync();
    const uint32_t NQ = TT * kq;
    if (cls == kClsPfd) {
        PatchSrc ps{sm.u.p.bmap, sm.u.p.vbit, nullptr, nullptr, ExcSrc{sw, nullptr, (uint32_t)SW, true}, false};
        if (k == 4u) pack_unpack<true, true>(sm, lane, NQ, 0u, 1u, 2u, ps);
        else pack_unpack<true, false>(sm, lane, NQ, lk - 2u, kq, lk, ps);
    } else {
        PatchSrc ps{nullptr, nullptr, nullptr, nullptr, ExcSrc{nullptr, nullptr, 0u, false}, false};
        if (k == 4u) pack_unpack<false, true>(sm, lane, NQ, 0u, 1u, 2u, ps);
        else pack_unpack<false, false>(sm, lane, NQ, lk - 2u, kq, lk, ps);
    }
    return true;
}

// A wave per pack, the grid striding over the packs when it is smaller
// than their number (the launch caps it, so that the packs, which depend on
// nothing else, leave room on every CU for the passes beside them).
template <int PI, int SW>
__global__ __launch_bounds__(kThreads) void gc_pack_kernel(PackArgs a) {
    __shared__ PackSmem<PI, SW> smem[kWaves];
    const uint32_t wave = uniform(threadIdx.x >> 6), lane = threadIdx.x & 63u;
    const uint32_t stride = gridDim.x * (uint32_t)kWaves;
    for (uint32_t p = blockIdx.x * (uint32_t)kWaves + wave; p < a.npacks; p += stride) {
        if (!pack_one<PI, SW>(a, smem[wave], p, lane)) return;
        wave_lds_sync();
    }
}

// ===========================================================================
// Carry scan: the tile sums of one delta list become exclusive carries, in
// place, 1024 tiles per round (the last tile's sum is never read: the sum
// pass skips it).

__global__ __launch_bounds__(kThreads) void gc_carry_scan(CarryArgs a) {
    __shared__ uint32_t s_tmp[kWaves];
    if (blockIdx.x >= a.count) return;
    const ListDesc L = a.lists ? a.lists[a.scan_list[blockIdx.x]] : a.single;
    uint32_t *cy = a.carry + L.tile_base;
    uint32_t run = 0;
    for (uint32_t b = 0; b < L.ntiles; b += 4u * kThreads) {
        const uint32_t i = b + 4u * threadIdx.x;
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; j++) v[j] = i + j + 1u < L.ntiles ? cy[i + j] : 0u;   // no tile follows the last
        uint32_t total;
        uint32_t p = run + block_excl_scan(v[0] + v[1] + v[2] + v[3], s_tmp, total);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (i + j < L.ntiles) cy[i + j] = p;
            p += v[j];
        }
        run += total;
    }
}

// ===========================================================================
// Launchers.

int codec_class(uint32_t w0) {
    HeaderFields h;
    if (!header_fields(w0, h)) return -1;
    switch (h.codec) {
    case 0: return kClsSim;
    case 1: return h.ld == GC_LD_BINARY ? kClsGscB : kClsGscU;
    case 3: return kClsPfd;
    default: return kClsAfor;   // Group-AFOR, Group-VSEncoding
    }
}

// chunk_words: kChunkWords or kChunkWordsSmall, as the items were counted.
int launch_locate(const LocateArgs &a, int chunk_words, hipStream_t s) {
    if (!a.total_items) return 0;
    if (chunk_words != kChunkWords && chunk_words != kChunkWordsSmall) return -2;
    const dim3 grid((a.total_items + kWaves - 1) / kWaves);
    if (chunk_words == kChunkWords) hipLaunchKernelGGL(gc_locate_reduce<kChunkWords / 64>, grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL(gc_locate_reduce<kChunkWordsSmall / 64>, grid, dim3(kThreads), 0, s, a);
    if (a.total_scan)   // lists of one chunk need no scan
        hipLaunchKernelGGL(gc_locate_scan, dim3((a.total_scan + kWaves - 1) / kWaves), dim3(kThreads), 0, s, a);
    if (chunk_words == kChunkWords) hipLaunchKernelGGL(gc_locate_emit<kChunkWords / 64>, grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL(gc_locate_emit<kChunkWordsSmall / 64>, grid, dim3(kThreads), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_carry_scan(const CarryArgs &a, hipStream_t s) {
    if (!a.count) return 0;
    hipLaunchKernelGGL(gc_carry_scan, dim3(a.count), dim3(kThreads), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int TW, int MODE>
static const void *wave_fn(int cls) {
    switch (cls) {
    case kClsSim: return reinterpret_cast<const void *>(gc_wave_kernel<TW, kClsSim, MODE>);
    case kClsGscU: return reinterpret_cast<const void *>(gc_wave_kernel<TW, kClsGscU, MODE>);
    case kClsGscB: return reinterpret_cast<const void *>(gc_wave_kernel<TW, kClsGscB, MODE>);
    case kClsAfor: return reinterpret_cast<const void *>(gc_wave_kernel<TW, kClsAfor, MODE>);
    case kClsPfd: return reinterpret_cast<const void *>(gc_wave_kernel<TW, kClsPfd, MODE>);
    default: return nullptr;
    }
}

template <int MODE>
static const void *decode_fn(int tile, int cls) {
    switch (tile) {
    case 1024: return wave_fn<1024, MODE>(cls);
    case 2048: return wave_fn<2048, MODE>(cls);
    case 4096: return wave_fn<4096, MODE>(cls);
    default: return nullptr;
    }
}

// Launches the pack kernel of capacity pi integers (2048 or 4096) over
// a.npacks packs, with at most max_groups workgroups (0: one wave per pack).
int launch_pack(int pi, const PackArgs &a, hipStream_t s, uint32_t max_groups) {
    if (!a.npacks) return 0;
    uint32_t groups = (a.npacks + kWaves - 1) / kWaves;
    if (max_groups && groups > max_groups) groups = max_groups;
    const dim3 grid(groups);
    if (pi == 2048) hipLaunchKernelGGL((gc_pack_kernel<2048, 512>), grid, dim3(kThreads), 0, s, a);
    else if (pi == 4096) hipLaunchKernelGGL((gc_pack_kernel<4096, 1024>), grid, dim3(kThreads), 0, s, a);
    else return -2;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Launches a pass over a.count tiles: mode 0 decode, 1 tile sums, 2 decode
// with the single-pass carry.
int launch_decode(int tile, int cls, int mode, const DecodeArgs &a, hipStream_t s) {
    if (!a.count) return 0;
    const void *fn = mode == 1   ? decode_fn<kModeSum>(tile, cls)
                     : mode == 2 ? decode_fn<kModeFused>(tile, cls)
                                 : decode_fn<kModeDecode>(tile, cls);
    if (!fn) return -2;
    const uint32_t per = (uint32_t)kWaves;
    DecodeArgs arg = a;
    void *params[] = {&arg};
    if (hipLaunchKernel(fn, dim3((a.count + per - 1) / per), dim3(kThreads), params, 0, s) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return 0;
}

}  // namespace gcdev
