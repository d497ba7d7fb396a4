// decode.hip -- gfx950 kernels that decode Group-codec streams and restore
// docIDs by prefix sum.
//
// Two persistent kernels per launch sequence:
//
//   locate  Scans the control areas of multi-tile lists, 256 control words
//           per work item, and records where every decode tile starts: the
//           control unit, the tuples of it already consumed, the component
//           data bit offset and (Group-PFD) the exception word offset.  The
//           scan across work items uses decoupled look-back.
//
//   decode  One work item = one tile of `TILE` output integers.  Control
//           units of the tile are parsed into per-tuple (bit offset, mask)
//           records in LDS; the tile's data words are staged HBM -> LDS with
//           16-byte loads; every thread then produces four consecutive
//           integers per round with a 64-bit funnel shift
//           (v_alignbit_b32) and a mask.  Group-PFD patches exceptions in
//           LDS (linked chains, or bitmap ranks by ballot/mbcnt).  Delta
//           lists are prefix-summed: in-thread, DPP wave scan, workgroup scan
//           through LDS, and a cross-tile carry by decoupled look-back.
//           Stores are 16-byte and coalesced (one wave writes 1 KiB).
//
// Both kernels pop work items from an atomic counter in list/tile order, so
// every look-back predecessor is already owned by a running workgroup, and
// both reset their own counters when the last workgroup retires.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gc.h"
#include "gc_device.h"
#include "gc_format.h"

namespace gcdev {

// ---------------------------------------------------------------------------
// Small helpers.

constexpr uint32_t kEpochMask = 0x3FFFFFFFu;
constexpr uint64_t kTimeoutTicks = 200000000ull;   // 2 s of the 100 MHz clock

__device__ __forceinline__ uint32_t epoch_next(uint32_t e) { return (e + 1u) & kEpochMask ? (e + 1u) & kEpochMask : 1u; }
__device__ __forceinline__ uint32_t epoch_prev(uint32_t e) { return e > 1u ? e - 1u : kEpochMask; }

__device__ __forceinline__ uint32_t mask_of(uint32_t b) { return b >= 32u ? 0xFFFFFFFFu : ((1u << b) - 1u); }

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh) {
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

template <int CTRL, int ROWS, bool BC>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, BC);
}

// Inclusive scan across a wave64 with DPP row shifts and row broadcasts.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += dpp<0x111, 0xF, true>(x);    // row_shr:1
    x += dpp<0x112, 0xF, true>(x);    // row_shr:2
    x += dpp<0x114, 0xF, true>(x);    // row_shr:4
    x += dpp<0x118, 0xF, true>(x);    // row_shr:8
    x += dpp<0x142, 0xA, false>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp<0x143, 0xC, false>(x);   // row_bcast:31 into rows 2 and 3
    return x;
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

__device__ __forceinline__ uint32_t load_acq(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long load_acq64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_rel(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_rel64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Group-Simple selector -> (NUM, BW), Table III, packed as 5-bit fields
// holding NUM-1 and BW-1.
constexpr uint64_t kSimNumM1 = 31ull | 15ull << 5 | 9ull << 10 | 7ull << 15 | 5ull << 20 | 4ull << 25 |
                               3ull << 30 | 2ull << 35 | 1ull << 40 | 0ull << 45;
constexpr uint64_t kSimBwM1 = 0ull | 1ull << 5 | 2ull << 10 | 3ull << 15 | 4ull << 20 | 5ull << 25 |
                              7ull << 30 | 9ull << 35 | 15ull << 40 | 31ull << 45;
__device__ __forceinline__ uint32_t sim_num(uint32_t sel) { return (uint32_t)((kSimNumM1 >> (5 * sel)) & 31u) + 1u; }
__device__ __forceinline__ uint32_t sim_bw(uint32_t sel) { return (uint32_t)((kSimBwM1 >> (5 * sel)) & 31u) + 1u; }

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
    uint32_t z = ~word, s = 0;
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

__device__ __forceinline__ bool header_ok(const ListDesc &L, uint32_t w0, uint32_t n, uint32_t C,
                                          uint32_t D, HeaderFields &h) {
    if (!header_fields(w0, h)) return false;
    if (n != L.n || (C & 3u) != 0u || (D & (uint32_t)(h.k - 1)) != 0u) return false;
    return 4ull + C + D <= L.stream_words;
}

__device__ __forceinline__ void finish_run(RunState *rs, uint32_t epoch) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t d = __hip_atomic_fetch_add(&rs->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (d == gridDim.x - 1) {
            __hip_atomic_store(&rs->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&rs->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&rs->epoch, epoch_next(epoch), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ===========================================================================
// Locate kernel.

// Control words the locate pass scans for one list (codec-specific).
__device__ __forceinline__ uint32_t locate_words(const HeaderFields &h, uint32_t T, uint32_t C, uint32_t D) {
    switch (h.codec) {
    case 0: return min(C, ((D >> h.lk) + 7u) >> 3);          // selectors / 8
    case 1:
        if (h.ld == GC_LD_BINARY) {
            const BinUnit u = bin_unit(h.cg);
            return min(C, (T + u.fpw - 1u) / u.fpw);
        }
        return C;
    case 2: return C;
    default: return min(C, (T + 31u) >> 5);                  // one descriptor per block
    }
}

__device__ void locate_chunk(const LocateArgs &a, const ListDesc &L, uint32_t chunk, uint32_t epoch,
                             LocVal &s_pre, uint32_t *s_tmp, uint32_t &s_bad) {
    const int tid = threadIdx.x;
    const uint32_t *S = L.stream;
    const uint32_t w0 = S[0], n = S[1], C = S[2], D = S[3];
    HeaderFields h;
    bool ok = header_ok(L, w0, n, C, D, h);
    const uint32_t k = (uint32_t)h.k;
    const uint32_t T = ok ? (n + k - 1u) >> h.lk : 0u;
    const uint32_t TT = a.tile_ints >> h.lk;
    const uint32_t nwords = ok ? locate_words(h, T, C, D) : 0u;
    const uint32_t *ctrl = S + 4;
    const uint32_t w = chunk * (uint32_t)kChunkWords + (uint32_t)tid;
    const bool valid = w < nwords;
    const uint32_t word = valid ? ctrl[w] : 0u;
    bool bad = false;

    // per-thread aggregate of its control word
    uint32_t vt = 0, ve = 0, vd = 0;
    if (valid) {
        switch (h.codec) {
        case 0: {
            const uint32_t S_total = D >> h.lk;
            for (uint32_t i = 0; i < 8u; i++) {
                const uint32_t s = 8u * w + i;
                if (s >= S_total) break;
                const uint32_t sel = (word >> (4u * i)) & 15u;
                if (sel >= 10u) { bad = true; continue; }
                vt += sim_num(sel);
            }
            break;
        }
        case 1:
            if (h.ld == GC_LD_BINARY) {
                const BinUnit u = bin_unit(h.cg);
                for (uint32_t f = 0; f < u.fpw; f++) {
                    const uint32_t t = w * u.fpw + f;
                    if (t >= T) break;
                    const uint32_t bit = bin_field_bit(t, u) & 31u;
                    vt += 1u;
                    vd += (uint32_t)h.cg * (((word >> bit) & mask_of(u.fb)) + 1u);
                }
            } else {
                vt = (uint32_t)__builtin_popcount(~word);
                if (h.ld == GC_LD_IU) vd = (uint32_t)h.cg * iu_useful(word);
            }
            break;
        case 2:
            for (int i = 0; i < 4; i++) {
                const uint32_t byte = (word >> (8 * i)) & 0xFFu;
                const uint32_t b = byte & 63u, cls = byte >> 6;
                if (cls == 3u || b > 32u) { bad = true; continue; }
                const uint32_t F = 8u << cls;
                vt += F;
                vd += F * b;
            }
            break;
        default: {
            const uint32_t b = word & 63u;
            if (b > 32u) bad = true;
            vt = 32u;
            vd = 32u * min(b, 32u);
            ve = pfd_exc_words(word, (int)k, h.pfd_pos);
            break;
        }
        }
    }
    if (!ok && tid == 0) bad = true;
    if (bad) s_bad = 1u;

    uint32_t tt, te, td;
    const uint32_t xt = block_excl_scan(vt, s_tmp, tt);
    const uint32_t xe = block_excl_scan(ve, s_tmp, te);
    const uint32_t xd = block_excl_scan(vd, s_tmp, td);

    if (tid == 0) {
        const uint32_t gi = L.chunk_base + chunk;
        LocVal agg;
        agg.tup = tt;
        agg.exc = te;
        agg.data = td;
        LocVal pre;
        pre.tup = 0;
        pre.exc = 0;
        pre.data = 0;
        if (chunk > 0) {
            a.agg[gi] = agg;
            store_rel(&a.flags[gi], (epoch << 2) | 1u);
            uint32_t j = gi - 1;
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            for (;;) {
                const uint32_t f = load_acq(&a.flags[j]);
                if ((f >> 2) == epoch && (f & 3u)) {
                    const LocVal v = (f & 3u) == 2u ? a.incl[j] : a.agg[j];
                    pre.tup += v.tup;
                    pre.exc += v.exc;
                    pre.data += v.data;
                    if ((f & 3u) == 2u) break;
                    j--;
                } else {
                    __builtin_amdgcn_s_sleep(2);
                    if (__builtin_amdgcn_s_memrealtime() - t0 > kTimeoutTicks) {
                        latch(a.status, kErrTimeout);
                        break;
                    }
                }
            }
        }
        LocVal inc;
        inc.tup = pre.tup + tt;
        inc.exc = pre.exc + te;
        inc.data = pre.data + td;
        a.incl[gi] = inc;
        store_rel(&a.flags[gi], (epoch << 2) | 2u);
        s_pre = pre;
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) latch(a.status, kErrLocate);
        return;
    }
    if (!valid) return;
    const uint32_t ntiles = L.ntiles;
    const uint32_t base_t = s_pre.tup + xt;
    const uint64_t base_d = s_pre.data + xd;
    const uint32_t base_e = s_pre.exc + xe;
    TileInfo *tiles = a.tiles + L.tile_base;

    auto emit = [&](uint32_t m, uint32_t unit, uint32_t sub, uint64_t data, uint32_t exc) {
        TileInfo ti;
        ti.unit = unit;
        ti.sub = sub;
        ti.exc = exc;
        ti.tag = epoch;
        ti.data = data;
        ti.pad = 0;
        tiles[m] = ti;
    };
    // the tile boundary m*TT (m >= 1) that falls in tuples [t, t + cnt)
    auto boundary = [&](uint32_t t, uint32_t cnt, uint32_t &m) -> bool {
        m = (t + TT - 1u) / TT;
        if (m == 0u) m = 1u;
        return m < ntiles && (uint64_t)m * TT < (uint64_t)t + cnt;
    };

    switch (h.codec) {
    case 0: {
        const uint32_t S_total = D >> h.lk;
        uint32_t t = base_t;
        for (uint32_t i = 0; i < 8u; i++) {
            const uint32_t s = 8u * w + i;
            if (s >= S_total) break;
            const uint32_t num = sim_num((word >> (4u * i)) & 15u);
            uint32_t m;
            if (boundary(t, num, m)) emit(m, s, m * TT - t, 32ull * s, 0);
            t += num;
        }
        break;
    }
    case 1:
        if (h.ld == GC_LD_BINARY) {
            const BinUnit u = bin_unit(h.cg);
            uint64_t d = base_d;
            for (uint32_t f = 0; f < u.fpw; f++) {
                const uint32_t t = w * u.fpw + f;
                if (t >= T) break;
                if (t > 0u && t % TT == 0u && t / TT < ntiles) emit(t / TT, t, 0, d, 0);
                const uint32_t bit = bin_field_bit(t, u) & 31u;
                d += (uint32_t)h.cg * (((word >> bit) & mask_of(u.fb)) + 1u);
            }
        } else {
            // terminators (0 bits) of ranks base_t .. base_t + z - 1 end in this
            // word; the tile starting at tuple m*TT starts after the terminator
            // of rank m*TT - 1
            const uint32_t z = ~word;
            const uint32_t cnt = (uint32_t)__builtin_popcount(z);
            if (cnt == 0u) break;
            uint32_t m = (base_t + TT) / TT;   // smallest m with m*TT - 1 >= base_t
            if (m < ntiles && m * TT - 1u < base_t + cnt) {
                uint32_t r = m * TT - 1u - base_t, zz = z;
                for (uint32_t i = 0; i < r; i++) zz &= zz - 1u;
                const uint32_t bit = (uint32_t)__builtin_ctz(zz);
                const uint32_t pos = 32u * w + bit + 1u;
                uint64_t d;
                if (h.ld == GC_LD_CU) {
                    d = (uint64_t)h.cg * pos;
                } else {
                    const uint32_t upto = bit == 31u ? word : (word | ~((2u << bit) - 1u));
                    // bits above `bit` read as padding 1s: keep only the bytes up to it
                    uint32_t u = 0;
                    for (uint32_t b = 0; b <= bit / 8u; b++) {
                        const uint32_t zb = (~upto >> (8u * b)) & 0xFFu;
                        u += zb ? 32u - (uint32_t)__builtin_clz(zb) : 0u;
                    }
                    d = base_d + (uint64_t)h.cg * u;
                }
                emit(m, pos, 0, d, 0);
            }
        }
        break;
    case 2: {
        uint32_t t = base_t;
        uint64_t d = base_d;
        for (int i = 0; i < 4; i++) {
            const uint32_t byte = (word >> (8 * i)) & 0xFFu;
            const uint32_t b = byte & 63u, F = 8u << (byte >> 6);
            uint32_t m;
            if (boundary(t, F, m)) emit(m, 4u * w + (uint32_t)i, m * TT - t, d, 0);
            t += F;
            d += (uint64_t)F * b;
        }
        break;
    }
    default: {
        const uint32_t t = 32u * w;
        if (t > 0u && t % TT == 0u && t / TT < ntiles) emit(t / TT, w, 0, base_d, base_e);
        break;
    }
    }
}

__global__ __launch_bounds__(kThreads) void gc_locate_kernel(LocateArgs a) {
    __shared__ uint32_t s_item;
    __shared__ LocVal s_pre;
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint32_t s_bad;
    const uint32_t epoch = __hip_atomic_load(&a.state->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0) {
            s_item = atomicAdd(&a.state->counter, 1u);
            s_bad = 0u;
        }
        __syncthreads();
        const uint32_t item = s_item;
        ListDesc L;
        uint32_t chunk;
        if (a.lists) {
            if (item >= a.total_items) break;
            L = a.lists[a.item_list[item]];
            chunk = item - L.chunk_base;
        } else {
            L = a.single;
            const uint32_t *S = L.stream;
            HeaderFields h;
            uint32_t nw = 0;
            if (header_ok(L, S[0], S[1], S[2], S[3], h)) {
                const uint32_t T = (S[1] + (uint32_t)h.k - 1u) >> h.lk;
                nw = locate_words(h, T, S[2], S[3]);
            }
            const uint32_t nchunks = (nw + kChunkWords - 1u) / kChunkWords;
            if (item >= (nchunks ? nchunks : 1u)) break;
            chunk = item;
        }
        locate_chunk(a, L, chunk, epoch, s_pre, s_tmp, s_bad);
        __syncthreads();
    }
    finish_run(a.state, epoch);
}

// ===========================================================================
// Decode kernel.

template <int TILE>
struct DecSmem {
    static constexpr int TTM = TILE / 4;            // tuples per tile at k = 4
    static constexpr int DATAW = TILE + 2 * 64 + 8;  // staged data words (+1 row)
    static constexpr int EXCW = TILE / 2;            // staged exception words
    static constexpr int R = TILE / (4 * kThreads);  // output rounds
    uint32_t data[DATAW];
    union {
        struct {
            uint32_t recO[TTM];
            uint32_t recM[TTM];
            uint32_t ctrl[TTM + 8];
        } r;
        struct {
            uint32_t gaps[TILE];
            uint32_t exc[EXCW];
        } p;
    } u;
    uint32_t blk_b[64], blk_off[64], blk_exc[64], blk_desc[64];
    uint32_t wtot[R * kWaves];
    uint32_t wpre[R * kWaves];
    uint32_t tmp[kWaves];
    uint32_t item, bad, prefix, rel_end, dbase, nw, b0, excw, exc_staged;
};

template <int TILE>
__device__ void decode_tile(const DecodeArgs &a, const ListDesc &L, uint32_t m, uint32_t epoch,
                            uint32_t loc_tag, DecSmem<TILE> &sm) {
    using SM = DecSmem<TILE>;
    constexpr int R = SM::R;
    constexpr int TTM = SM::TTM;
    const int tid = threadIdx.x;
    const uint32_t *S = L.stream;
    const uint32_t w0 = S[0], n = S[1], C = S[2], D = S[3];
    HeaderFields h;
    bool ok = header_ok(L, w0, n, C, D, h);
    const uint32_t k = (uint32_t)h.k, lk = (uint32_t)h.lk;
    const uint32_t T = (n + k - 1u) >> lk;
    const uint32_t TT = (uint32_t)TILE >> lk;
    const uint32_t t0 = m * TT;
    const uint32_t i0 = m * (uint32_t)TILE;
    ok = ok && i0 < n;
    const uint32_t ntup = ok ? min(TT, T - t0) : 0u;
    const uint32_t nint = ok ? min((uint32_t)TILE, n - i0) : 0u;
    const uint32_t *ctrl = S + 4;
    const uint32_t *data = S + 4 + C;
    const bool has_en = m + 1u < L.ntiles;
    TileInfo st{}, en{};
    if (ok && m > 0u) {
        st = a.tiles[L.tile_base + m];
        ok = ok && st.tag == loc_tag;
    }
    if (ok && has_en) {
        en = a.tiles[L.tile_base + m + 1u];
        ok = ok && en.tag == loc_tag;
    }
    if (tid == 0) {
        sm.bad = ok ? 0u : kErrLocate;
        sm.rel_end = 0u;
    }
    __syncthreads();

    // ---- control parse: per-tuple (bit offset, mask) records ----------------
    const int codec = h.codec;
    if (!sm.bad) {
        if (codec == 0) {
            const uint32_t S_total = D >> lk;
            const uint32_t s_first = st.unit, sub0 = st.sub;
            const uint32_t s_end = has_en ? en.unit + (en.sub ? 1u : 0u) : S_total;
            const uint32_t nsel = s_end - s_first;
            const uint32_t cw0 = s_first >> 3, cw1 = (s_end + 7u) >> 3;
            const bool rng_ok = s_end <= S_total && s_end > s_first && nsel <= TT + 1u && cw1 <= C;
            if (!rng_ok) {
                if (tid == 0) sm.bad = kErrRange;
            } else {
                for (uint32_t i = (uint32_t)tid; i < cw1 - cw0; i += kThreads) sm.u.r.ctrl[i] = ctrl[cw0 + i];
            }
            __syncthreads();
            constexpr int SPT = (TTM + 1 + kThreads - 1) / kThreads;
            uint32_t cnt[SPT];
            uint32_t sum = 0;
#pragma unroll
            for (int j = 0; j < SPT; j++) {
                const uint32_t i = (uint32_t)tid * SPT + (uint32_t)j;
                uint32_t c = 0;
                if (!sm.bad && i < nsel) {
                    const uint32_t s = s_first + i;
                    const uint32_t sel = (sm.u.r.ctrl[(s >> 3) - cw0] >> ((s & 7u) * 4u)) & 15u;
                    const uint32_t num = sel < 10u ? sim_num(sel) : 0u;
                    const uint32_t j0 = i == 0u ? sub0 : 0u;
                    if (sel >= 10u || num <= j0) sm.bad = kErrSelector;
                    else c = num - j0;
                }
                cnt[j] = c;
                sum += c;
            }
            uint32_t total;
            uint32_t run = block_excl_scan(sum, sm.tmp, total);
            if (!sm.bad && total < ntup && tid == 0) sm.bad = kErrCount;
#pragma unroll
            for (int j = 0; j < SPT; j++) {
                const uint32_t i = (uint32_t)tid * SPT + (uint32_t)j;
                if (cnt[j] && i < nsel) {
                    const uint32_t s = s_first + i;
                    const uint32_t sel = (sm.u.r.ctrl[(s >> 3) - cw0] >> ((s & 7u) * 4u)) & 15u;
                    const uint32_t bw = sim_bw(sel), msk = mask_of(bw);
                    const uint32_t j0 = i == 0u ? sub0 : 0u;
                    for (uint32_t jj = 0; jj < cnt[j]; jj++) {
                        const uint32_t t = run + jj;
                        if (t < ntup) {
                            sm.u.r.recO[t] = 32u * i + (j0 + jj) * bw;
                            sm.u.r.recM[t] = msk;
                        }
                    }
                }
                run += cnt[j];
            }
            if (tid == 0) {
                sm.dbase = s_first;
                sm.nw = nsel;
            }
        } else if (codec == 1 && h.ld != GC_LD_BINARY) {
            const uint32_t cg = (uint32_t)h.cg, umax = 32u / cg;
            const bool iu = h.ld == GC_LD_IU;
            const uint32_t p0 = st.unit;
            const uint32_t p1 = has_en ? en.unit : 32u * C;
            const uint32_t cw0 = p0 >> 5, cw1 = (p1 + 31u) >> 5;
            const uint32_t nctrl = cw1 - cw0;
            const bool rng_ok = p1 >= p0 && cw1 <= C && nctrl <= (uint32_t)TTM + 8u;
            if (!rng_ok) {
                if (tid == 0) sm.bad = kErrRange;
            } else {
                for (uint32_t i = (uint32_t)tid; i < nctrl; i += kThreads) {
                    // only bits in [p0, p1) belong to the tile: others read as 1
                    const uint32_t gw = cw0 + i;
                    uint32_t v = ctrl[gw];
                    if (gw == cw0) v |= (p0 & 31u) ? ((1u << (p0 & 31u)) - 1u) : 0u;
                    if (gw == (p1 >> 5) && (p1 & 31u)) v |= ~((1u << (p1 & 31u)) - 1u);
                    if (gw > (p1 >> 5) || (gw == (p1 >> 5) && !(p1 & 31u))) v = 0xFFFFFFFFu;
                    sm.u.r.ctrl[i] = v;
                }
            }
            __syncthreads();
            const uint32_t wpt = (nctrl + kThreads - 1u) / kThreads;
            const uint32_t wl0 = (uint32_t)tid * wpt, wl1 = min(wl0 + wpt, sm.bad ? 0u : nctrl);
            // where the first code of this thread's words starts: after the last
            // terminator of the earlier words of the tile, else at p0
            uint32_t start0 = p0;
            if (!sm.bad && wl0 < wl1)
                for (uint32_t wl = min(wl0, nctrl); wl-- > 0u;) {
                    const uint32_t z = ~sm.u.r.ctrl[wl];
                    if (z) {
                        start0 = 32u * (cw0 + wl) + 32u - (uint32_t)__builtin_clz(z);
                        break;
                    }
                }
            uint32_t cnt = 0, usum = 0;
            {
                uint32_t nxt = start0;
                for (uint32_t wl = wl0; wl < wl1; wl++) {
                    uint32_t z = ~sm.u.r.ctrl[wl];
                    while (z) {
                        const uint32_t zp = 32u * (cw0 + wl) + (uint32_t)__builtin_ctz(z);
                        z &= z - 1u;
                        const uint32_t start = iu ? max(nxt, zp & ~7u) : nxt;
                        const uint32_t u = zp - start + 1u;
                        if (u > umax) sm.bad = kErrUnary;
                        cnt++;
                        usum += u;
                        nxt = zp + 1u;
                    }
                }
            }
            uint32_t tcnt, tus;
            const uint32_t xc = block_excl_scan(cnt, sm.tmp, tcnt);
            const uint32_t xu = block_excl_scan(usum, sm.tmp, tus);
            if (tid == 0 && !sm.bad && tcnt < ntup) sm.bad = kErrCount;
            const uint64_t abs0 = iu ? st.data : (uint64_t)cg * p0;
            const uint32_t dbase = (uint32_t)(abs0 >> 5);
            if (!sm.bad) {
                uint32_t nxt = start0, t = xc, us = xu;
                for (uint32_t wl = wl0; wl < wl1; wl++) {
                    uint32_t z = ~sm.u.r.ctrl[wl];
                    while (z) {
                        const uint32_t zp = 32u * (cw0 + wl) + (uint32_t)__builtin_ctz(z);
                        z &= z - 1u;
                        const uint32_t start = iu ? max(nxt, zp & ~7u) : nxt;
                        const uint32_t u = zp - start + 1u;
                        const uint64_t abs = iu ? abs0 + (uint64_t)cg * us : (uint64_t)cg * start;
                        const uint32_t rel = (uint32_t)(abs - 32ull * dbase);
                        if (t < ntup) {
                            sm.u.r.recO[t] = rel;
                            sm.u.r.recM[t] = mask_of(cg * u);
                            if (t == ntup - 1u) sm.rel_end = rel + cg * u;
                        }
                        t++;
                        us += u;
                        nxt = zp + 1u;
                    }
                }
            }
            if (tid == 0) sm.dbase = dbase;
            __syncthreads();
            if (tid == 0) sm.nw = (sm.rel_end + 31u) >> 5;
        } else if (codec == 1) {
            const uint32_t cg = (uint32_t)h.cg;
            const BinUnit bu = bin_unit(h.cg);
            constexpr int TPT = TTM / kThreads;
            uint32_t bw[TPT];
            uint32_t sum = 0;
            bool bad = false;
#pragma unroll
            for (int j = 0; j < TPT; j++) {
                const uint32_t tt = (uint32_t)tid * TPT + (uint32_t)j;
                uint32_t b = 0;
                if (tt < ntup) {
                    const uint32_t bit = bin_field_bit(t0 + tt, bu);
                    if ((bit >> 5) >= C) bad = true;
                    else b = cg * (((ctrl[bit >> 5] >> (bit & 31u)) & mask_of(bu.fb)) + 1u);
                }
                bw[j] = b;
                sum += b;
            }
            if (bad) sm.bad = kErrRange;
            uint32_t total;
            uint32_t run = block_excl_scan(sum, sm.tmp, total);
            const uint64_t abs0 = st.data;
            const uint32_t dbase = (uint32_t)(abs0 >> 5);
            const uint32_t rel0 = (uint32_t)(abs0 & 31u);
#pragma unroll
            for (int j = 0; j < TPT; j++) {
                const uint32_t tt = (uint32_t)tid * TPT + (uint32_t)j;
                if (tt < ntup) {
                    sm.u.r.recO[tt] = rel0 + run;
                    sm.u.r.recM[tt] = mask_of(bw[j]);
                }
                run += bw[j];
            }
            if (tid == 0) {
                sm.dbase = dbase;
                sm.nw = (rel0 + total + 31u) >> 5;
            }
        } else if (codec == 2) {
            const uint32_t f0 = st.unit, sub0 = st.sub;
            const uint32_t nfr = min(TT / 8u + 2u, 4u * C > f0 ? 4u * C - f0 : 0u);
            constexpr int FPT = (TTM / 8 + 2 + kThreads - 1) / kThreads;
            uint32_t c[FPT], bits[FPT], bb[FPT];
            uint32_t csum = 0, bsum = 0;
#pragma unroll
            for (int j = 0; j < FPT; j++) {
                const uint32_t i = (uint32_t)tid * FPT + (uint32_t)j;
                c[j] = bits[j] = bb[j] = 0u;
                if (i < nfr) {
                    const uint32_t f = f0 + i;
                    const uint32_t byte = (ctrl[f >> 2] >> (8u * (f & 3u))) & 0xFFu;
                    uint32_t b = byte & 63u;
                    const uint32_t cls = byte >> 6;
                    if (cls == 3u || b > 32u) {
                        sm.bad = kErrFrame;
                        b = 0;
                    }
                    const uint32_t F = cls == 0u ? 8u : cls == 1u ? 16u : 32u;
                    const uint32_t j0 = i == 0u ? sub0 : 0u;
                    if (j0 >= F) sm.bad = kErrFrame;
                    else c[j] = F - j0;
                    bits[j] = F * b;
                    bb[j] = b;
                    if (i == 0u) sm.b0 = b;
                }
                csum += c[j];
                bsum += bits[j];
            }
            uint32_t tc, tb;
            uint32_t st_t = block_excl_scan(csum, sm.tmp, tc);
            uint32_t off = block_excl_scan(bsum, sm.tmp, tb);
            if (tid == 0 && !sm.bad && tc < ntup) sm.bad = kErrCount;
            const uint64_t fdata0 = st.data;
            const uint64_t first_abs = fdata0 + (uint64_t)sub0 * sm.b0;
            const uint32_t dbase = (uint32_t)(first_abs >> 5);
#pragma unroll
            for (int j = 0; j < FPT; j++) {
                const uint32_t i = (uint32_t)tid * FPT + (uint32_t)j;
                if (!sm.bad && c[j]) {
                    const uint32_t j0 = i == 0u ? sub0 : 0u;
                    const uint32_t b = bb[j];
                    const uint32_t frel = (uint32_t)(fdata0 + off - 32ull * dbase);
                    const uint32_t msk = mask_of(b);
                    for (uint32_t jj = 0; jj < c[j]; jj++) {
                        const uint32_t t = st_t + jj;
                        if (t < ntup) {
                            const uint32_t rel = frel + (j0 + jj) * b;
                            sm.u.r.recO[t] = rel;
                            sm.u.r.recM[t] = msk;
                            if (t == ntup - 1u) sm.rel_end = rel + b;
                        }
                    }
                }
                st_t += c[j];
                off += bits[j];
            }
            if (tid == 0) sm.dbase = dbase;
            __syncthreads();
            if (tid == 0) sm.nw = (sm.rel_end + 31u) >> 5;
        } else {
            const uint32_t nb = (ntup + 31u) >> 5;
            const uint32_t beta0 = t0 >> 5;
            const int bitmap = h.pfd_pos;
            if (tid < 64) {
                uint32_t desc = 0, b = 0, ew = 0;
                if ((uint32_t)tid < nb) {
                    if (beta0 + (uint32_t)tid >= C) {
                        sm.bad = kErrRange;
                    } else {
                        desc = ctrl[beta0 + (uint32_t)tid];
                        b = desc & 63u;
                        const uint32_t nexc = desc >> 20, wcode = (desc >> 6) & 3u;
                        const uint32_t first = (desc >> 8) & 0xFFFu;
                        if (b > 32u || nexc > 32u * k || (nexc && !wcode) || (bitmap && first > 32u)) {
                            sm.bad = kErrPfdDesc;
                            b = 0;
                            desc = 0;
                        }
                        ew = pfd_exc_words(desc, (int)k, bitmap);
                    }
                }
                const uint32_t ib = wave_incl_scan(b), ie = wave_incl_scan(ew);
                if ((uint32_t)tid < nb) {
                    sm.blk_b[tid] = b;
                    sm.blk_off[tid] = ib - b;
                    sm.blk_exc[tid] = ie - ew;
                    sm.blk_desc[tid] = desc;
                }
                if (tid == 63) {
                    sm.dbase = (uint32_t)(st.data >> 5);
                    sm.nw = ib;
                    sm.excw = ie;
                }
            }
        }
    }
    __syncthreads();

    // ---- stage the tile's data words HBM -> LDS -----------------------------
    if (!sm.bad) {
        const uint32_t dbase = sm.dbase, nw = sm.nw;
        const uint32_t Dk = D >> lk;
        if ((uint64_t)dbase + nw > Dk || (nw + 1u) * k > (uint32_t)SM::DATAW) {
            if (tid == 0) sm.bad = kErrRange;
        } else {
            const uint32_t g0 = dbase * k;
            const uint32_t nq = ((nw + 1u) * k) >> 2;
            const uint4 *src = reinterpret_cast<const uint4 *>(data + g0);
            uint4 *dst = reinterpret_cast<uint4 *>(sm.data);
            const uint32_t avail_q = (D - g0) >> 2;
            for (uint32_t q = (uint32_t)tid; q < nq; q += kThreads)
                dst[q] = q < avail_q ? src[q] : make_uint4(0u, 0u, 0u, 0u);
            if (codec == 3) {
                // exception words of the tile's blocks
                const uint64_t ex0 = 4ull + C + D + (m > 0u ? st.exc : 0u);
                const uint32_t excw = sm.excw;
                const bool fits = excw <= (uint32_t)SM::EXCW;
                if (ex0 + excw > L.stream_words) {
                    if (tid == 0) sm.bad = kErrRange;
                } else if (fits) {
                    for (uint32_t q = (uint32_t)tid; q < excw; q += kThreads) sm.u.p.exc[q] = S[ex0 + q];
                }
                if (tid == 0) sm.exc_staged = fits ? 1u : 0u;
            }
        }
    }
    __syncthreads();

    // ---- unpack: four consecutive integers per thread and round ------------
    const bool bad = sm.bad != 0u;
    uint32_t v[R][4];
    const uint32_t nwc = sm.nw;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t q = (uint32_t)(r * kThreads + tid);
        v[r][0] = v[r][1] = v[r][2] = v[r][3] = 0u;
        if (!bad && 4u * q < nint) {
            const uint32_t t = q >> (lk - 2u);
            const uint32_t c0 = (q << 2) & (k - 1u);
            uint32_t O, M;
            if (codec == 3) {
                const uint32_t bi = t >> 5, b = sm.blk_b[bi];
                O = 32u * sm.blk_off[bi] + (t & 31u) * b;
                M = mask_of(b);
            } else {
                O = sm.u.r.recO[t];
                M = sm.u.r.recM[t];
            }
            const uint32_t wi = min(O >> 5, nwc ? nwc - 1u : 0u);
            const uint32_t sh = O & 31u;
            const uint4 lo = *reinterpret_cast<const uint4 *>(&sm.data[wi * k + c0]);
            const uint4 hi = *reinterpret_cast<const uint4 *>(&sm.data[(wi + 1u) * k + c0]);
            v[r][0] = funnel(hi.x, lo.x, sh) & M;
            v[r][1] = funnel(hi.y, lo.y, sh) & M;
            v[r][2] = funnel(hi.z, lo.z, sh) & M;
            v[r][3] = funnel(hi.w, lo.w, sh) & M;
        }
    }

    // ---- Group-PFD: exceptions replace their slots -------------------------
    if (codec == 3) {
        __syncthreads();   // the exception words may overlap nothing, but gaps alias recO
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t q = (uint32_t)(r * kThreads + tid);
            *reinterpret_cast<uint4 *>(&sm.u.p.gaps[4u * q]) = make_uint4(v[r][0], v[r][1], v[r][2], v[r][3]);
        }
        __syncthreads();
        if (!bad) {
            const uint32_t nb = (ntup + 31u) >> 5;
            const uint32_t BI = 32u * k;
            const uint64_t ex0 = 4ull + C + D + (m > 0u ? st.exc : 0u);
            const bool staged = sm.exc_staged != 0u;
            auto exw = [&](uint32_t idx) -> uint32_t { return staged ? sm.u.p.exc[idx] : S[ex0 + idx]; };
            if (h.pfd_pos == GC_PFD_LINKED) {
                for (uint32_t bi = (uint32_t)tid; bi < nb; bi += kThreads) {
                    const uint32_t desc = sm.blk_desc[bi];
                    const uint32_t nexc = desc >> 20;
                    if (!nexc) continue;
                    const uint32_t w = 4u << ((desc >> 6) & 3u), wm = mask_of(w);
                    const uint32_t xb = sm.blk_exc[bi];
                    uint32_t p = (desc >> 8) & 0xFFFu;
                    uint32_t *g = &sm.u.p.gaps[bi * BI];
                    for (uint32_t e = 0; e < nexc; e++) {
                        if (p >= BI) {
                            sm.bad = kErrPfdChain;
                            break;
                        }
                        const uint32_t slot = g[p];
                        const uint32_t bit = e * w;
                        g[p] = (exw(xb + (bit >> 5)) >> (bit & 31u)) & wm;
                        p = slot < BI ? p + slot + 1u : BI;
                    }
                }
            } else {
                const int wave = tid >> 6, lane = tid & 63;
                for (uint32_t bi = (uint32_t)wave; bi < nb; bi += kWaves) {
                    const uint32_t desc = sm.blk_desc[bi];
                    const uint32_t nexc = desc >> 20;
                    if (!nexc) continue;
                    const uint32_t w = 4u << ((desc >> 6) & 3u), wm = mask_of(w);
                    const uint32_t nt = (desc >> 8) & 0xFFFu;
                    const uint32_t xb = sm.blk_exc[bi];
                    const uint32_t tm = exw(xb);
                    const uint32_t vbase = xb + 1u + ((nt * k + 31u) >> 5);
                    uint32_t run = 0;
                    if ((uint32_t)__builtin_popcount(tm) != nt) {
                        if (lane == 0) sm.bad = kErrBitmap;
                        continue;
                    }
                    for (uint32_t p0 = 0; p0 < BI; p0 += 64u) {
                        const uint32_t p = p0 + (uint32_t)lane;
                        const uint32_t t = p >> lk, c = p & (k - 1u);
                        bool isx = false;
                        if ((tm >> t) & 1u) {
                            const uint32_t rank = (uint32_t)__builtin_popcount(tm & ((1u << t) - 1u));
                            const uint32_t bit = rank * k + c;
                            isx = (exw(xb + 1u + (bit >> 5)) >> (bit & 31u)) & 1u;
                        }
                        const uint64_t bal = __ballot(isx);
                        const uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                        if (isx) {
                            const uint32_t e = run + before;
                            const uint32_t bitv = e * w;
                            if (e < nexc)
                                sm.u.p.gaps[bi * BI + p] = (exw(vbase + (bitv >> 5)) >> (bitv & 31u)) & wm;
                        }
                        run += (uint32_t)__builtin_popcountll(bal);
                    }
                    if (lane == 0 && run != nexc) sm.bad = kErrBitmap;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t q = (uint32_t)(r * kThreads + tid);
            const uint4 g = *reinterpret_cast<const uint4 *>(&sm.u.p.gaps[4u * q]);
            v[r][0] = g.x;
            v[r][1] = g.y;
            v[r][2] = g.z;
            v[r][3] = g.w;
        }
    }

    // ---- prefix sum (delta lists) -------------------------------------------
    const int wave = tid >> 6, lane = tid & 63;
    uint32_t add[R];
#pragma unroll
    for (int r = 0; r < R; r++) add[r] = 0u;
    if (h.delta) {
        uint32_t wex[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            v[r][1] += v[r][0];
            v[r][2] += v[r][1];
            v[r][3] += v[r][2];
            const uint32_t inc = wave_incl_scan(v[r][3]);
            wex[r] = inc - v[r][3];
            if (lane == 63) sm.wtot[r * kWaves + wave] = inc;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            for (int i = 0; i < R * kWaves; i++) {
                const uint32_t x = sm.wtot[i];
                sm.wpre[i] = acc;
                acc += x;
            }
            const uint32_t gi = L.tile_base + m;
            const unsigned long long tag = (unsigned long long)(epoch & kEpochMask) << 34;
            uint32_t pre = 0;
            if (m == 0u) {
                store_rel64(&a.flags[gi], tag | (2ull << 32) | acc);
            } else {
                store_rel64(&a.flags[gi], tag | (1ull << 32) | acc);
                uint32_t j = gi - 1u;
                const uint64_t tstart = __builtin_amdgcn_s_memrealtime();
                for (;;) {
                    const unsigned long long f = load_acq64(&a.flags[j]);
                    const uint32_t stt = (uint32_t)(f >> 32) & 3u;
                    if ((uint32_t)(f >> 34) == (epoch & kEpochMask) && stt) {
                        pre += (uint32_t)f;
                        if (stt == 2u) break;
                        j--;
                    } else {
                        __builtin_amdgcn_s_sleep(1);
                        if (__builtin_amdgcn_s_memrealtime() - tstart > kTimeoutTicks) {
                            latch(a.status, kErrTimeout);
                            break;
                        }
                    }
                }
                store_rel64(&a.flags[gi], tag | (2ull << 32) | (uint32_t)(pre + acc));
            }
            sm.prefix = pre;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; r++) add[r] = sm.prefix + sm.wpre[r * kWaves + wave] + wex[r];
    }
    if (tid == 0 && sm.bad) latch(a.status, sm.bad);

    // ---- store ---------------------------------------------------------------
    uint32_t *out = L.out + i0;
    const bool vec = (reinterpret_cast<uintptr_t>(out) & 15u) == 0u;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t q = (uint32_t)(r * kThreads + tid);
        const uint32_t ii = 4u * q;
        if (ii >= nint) continue;
        const uint4 o = make_uint4(v[r][0] + add[r], v[r][1] + add[r], v[r][2] + add[r], v[r][3] + add[r]);
        if (vec && ii + 4u <= nint) {
            *reinterpret_cast<uint4 *>(out + ii) = o;
        } else {
            out[ii] = o.x;
            if (ii + 1u < nint) out[ii + 1u] = o.y;
            if (ii + 2u < nint) out[ii + 2u] = o.z;
            if (ii + 3u < nint) out[ii + 3u] = o.w;
        }
    }
}

template <int TILE>
__global__ __launch_bounds__(kThreads) void gc_decode_kernel(DecodeArgs a) {
    __shared__ DecSmem<TILE> sm;
    const uint32_t epoch = __hip_atomic_load(&a.state->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t loc_tag =
        epoch_prev(__hip_atomic_load(&a.loc_state->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    for (;;) {
        if (threadIdx.x == 0) sm.item = atomicAdd(&a.state->counter, 1u);
        __syncthreads();
        const uint32_t item = sm.item;
        __syncthreads();
        ListDesc L;
        uint32_t m;
        if (a.lists) {
            if (item >= a.total_items) break;
            L = a.lists[a.item_list[item]];
            m = item - L.tile_base;
        } else {
            L = a.single;
            if (item >= L.ntiles) break;
            m = item;
        }
        decode_tile<TILE>(a, L, m, epoch, loc_tag, sm);
    }
    finish_run(a.state, epoch);
}

// ===========================================================================
// Launchers.

int launch_locate(const LocateArgs &a, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(gc_locate_kernel, dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_decode(int tile, const DecodeArgs &a, uint32_t grid, hipStream_t s) {
    switch (tile) {
    case 2048: hipLaunchKernelGGL(gc_decode_kernel<2048>, dim3(grid), dim3(kThreads), 0, s, a); break;
    case 4096: hipLaunchKernelGGL(gc_decode_kernel<4096>, dim3(grid), dim3(kThreads), 0, s, a); break;
    case 8192: hipLaunchKernelGGL(gc_decode_kernel<8192>, dim3(grid), dim3(kThreads), 0, s, a); break;
    default: return -2;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int decode_occupancy(int tile, int *blocks_per_cu) {
    hipError_t e;
    switch (tile) {
    case 2048: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gc_decode_kernel<2048>, kThreads, 0); break;
    case 4096: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gc_decode_kernel<4096>, kThreads, 0); break;
    case 8192: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gc_decode_kernel<8192>, kThreads, 0); break;
    default: return -2;
    }
    return e == hipSuccess ? 0 : -1;
}

int locate_occupancy(int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gc_locate_kernel, kThreads, 0) == hipSuccess ? 0 : -1;
}

}  // namespace gcdev
