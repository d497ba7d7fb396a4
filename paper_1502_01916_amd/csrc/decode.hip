// decode.hip -- gfx950 kernels that decode Group-codec streams and restore
// docIDs by prefix sum.
//
//   locate  Scans the control areas of multi-tile lists (1024 control words
//           per work item) and records where every decode tile starts: the
//           control unit, the tuples of it that belong to the previous tile,
//           the component data bit offset and (Group-PFD) the exception word
//           offset.  The scan across work items uses decoupled look-back.
//
//   decode  One persistent kernel per codec class (Group-Simple, Group-Scheme
//           unary, Group-Scheme binary, Group-AFOR, Group-PFD), so each keeps
//           only its own registers and LDS.  A work item is one tile of TILE
//           output integers.  The tile's control units are parsed into
//           per-tuple records (component bit offset, width) in LDS; each
//           thread then produces four consecutive integers per round from two
//           16-byte data rows read through the vector cache, with a 64-bit
//           funnel shift (v_alignbit_b32) and a mask.  Group-PFD patches
//           exceptions in LDS (linked chains, or bitmap ranks by ballot and
//           mbcnt).  Delta lists are prefix-summed in-thread, across the wave
//           with DPP, across the workgroup through LDS, and across tiles by a
//           decoupled look-back that inspects 64 predecessors per probe.
//
// Work items are popped from an atomic counter in list/tile order, so every
// look-back predecessor is owned by a running workgroup; each kernel resets
// its counters when its last workgroup retires, so a run needs no memset and
// can be replayed from a captured graph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gc.h"
#include "gc_device.h"
#include "gc_format.h"

namespace gcdev {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Small helpers.

constexpr uint32_t kEpochMask = 0x3FFFFFFFu;
constexpr uint64_t kTimeoutTicks = 200000000ull;   // 2 s of the 100 MHz clock
constexpr int kLocWords = kChunkWords / kThreads;  // control words per thread

__device__ __forceinline__ uint32_t epoch_next(uint32_t e) {
    return ((e + 1u) & kEpochMask) ? ((e + 1u) & kEpochMask) : 1u;
}
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

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(x), 63);
}

// 64-bit wave sum from 32-bit scans (16-bit halves of the low word cannot
// overflow across 64 lanes).
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    return (uint64_t)wave_sum(lo & 0xFFFFu) + ((uint64_t)wave_sum(lo >> 16) << 16) + ((uint64_t)wave_sum(hi) << 32);
}

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
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

// Decoupled look-back run by one whole wave: lane l inspects predecessor
// gi-1-l; the nearest inclusive prefix and every aggregate after it are
// summed into the probe.  `first` is the list's first entry, which always
// publishes an inclusive prefix.
template <typename Probe>
__device__ __forceinline__ void wave_lookback(uint32_t gi, uint32_t first, Probe &probe, Status *st) {
    const uint32_t lane = lane_id();
    uint32_t base = gi;                       // this window covers base-1-lane
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        const bool in = base >= first + 1u + lane;
        const uint32_t j = in ? base - 1u - lane : first;
        const int state = in ? probe.state(j) : 2;   // 0 not ready, 1 aggregate, 2 inclusive
        const uint64_t pmask = __ballot(state == 2);
        const uint64_t nready = __ballot(state == 0);
        if (pmask) {
            const uint32_t p = (uint32_t)__builtin_ctzll(pmask);
            const uint64_t need = (p == 63u) ? ~0ull : ((2ull << p) - 1ull);
            if ((nready & need) == 0ull) {
                probe.accumulate(in && lane <= p, j);
                return;
            }
        } else if (nready == 0ull) {
            probe.accumulate(true, j);
            base -= 64u;
            continue;
        }
        __builtin_amdgcn_s_sleep(1);
        if (__builtin_amdgcn_s_memrealtime() - t0 > kTimeoutTicks) {
            if (lane == 0) latch(st, kErrTimeout);
            return;
        }
    }
}

// ===========================================================================
// Locate kernel.

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

struct LocProbe {
    const uint32_t *flags;
    const LocVal *agg, *incl;
    uint32_t epoch;
    uint32_t tup, exc;
    uint64_t data;
    uint32_t st;
    __device__ int state(uint32_t j) {
        const uint32_t f = load_acq(&flags[j]);
        st = ((f >> 2) == epoch) ? (f & 3u) : 0u;
        return (int)st;
    }
    __device__ void accumulate(bool take, uint32_t j) {
        LocVal v;
        v.tup = 0;
        v.exc = 0;
        v.data = 0;
        if (take) v = st == 2u ? incl[j] : agg[j];
        tup += wave_sum(v.tup);
        exc += wave_sum(v.exc);
        data += wave_sum64(v.data);
    }
};

__device__ void locate_chunk(const LocateArgs &a, const ListDesc &L, uint32_t chunk, uint32_t epoch,
                             LocVal &s_pre, uint32_t *s_tmp, uint32_t &s_bad) {
    const int tid = threadIdx.x;
    const uint32_t *S = L.stream;
    const uint32_t w0 = S[0], n = S[1], C = S[2], D = S[3];
    HeaderFields h;
    const bool ok = header_ok(L, w0, n, C, D, h);
    const uint32_t k = (uint32_t)h.k;
    const uint32_t T = ok ? (n + k - 1u) >> h.lk : 0u;
    const uint32_t TT = a.tile_ints >> h.lk;
    const uint32_t nwords = ok ? locate_words(h, T, C, D) : 0u;
    const uint32_t *ctrl = S + 4;
    const uint32_t wbase = (chunk * (uint32_t)kThreads + (uint32_t)tid) * (uint32_t)kLocWords;
    uint32_t word[kLocWords];
    bool bad = !ok && tid == 0;

    uint32_t vt = 0, ve = 0, vd = 0;
#pragma unroll
    for (int q = 0; q < kLocWords; q++) {
        const uint32_t w = wbase + (uint32_t)q;
        word[q] = w < nwords ? ctrl[w] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kLocWords; q++) {
        const uint32_t w = wbase + (uint32_t)q;
        if (w >= nwords) continue;
        const uint32_t wd = word[q];
        switch (h.codec) {
        case 0: {
            const uint32_t S_total = D >> h.lk;
            for (uint32_t i = 0; i < 8u; i++) {
                if (8u * w + i >= S_total) break;
                const uint32_t sel = (wd >> (4u * i)) & 15u;
                if (sel >= 10u) {
                    bad = true;
                    continue;
                }
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
                    vd += (uint32_t)h.cg * (((wd >> bit) & mask_of(u.fb)) + 1u);
                }
            } else {
                vt += (uint32_t)__builtin_popcount(~wd);
                if (h.ld == GC_LD_IU) vd += (uint32_t)h.cg * iu_useful(wd);
            }
            break;
        case 2:
            for (int i = 0; i < 4; i++) {
                const uint32_t byte = (wd >> (8 * i)) & 0xFFu;
                const uint32_t b = byte & 63u, cls = byte >> 6;
                if (cls == 3u || b > 32u) {
                    bad = true;
                    continue;
                }
                const uint32_t F = 8u << cls;
                vt += F;
                vd += F * b;
            }
            break;
        default: {
            const uint32_t b = wd & 63u;
            if (b > 32u) bad = true;
            vt += 32u;
            vd += 32u * min(b, 32u);
            ve += pfd_exc_words(wd, (int)k, h.pfd_pos);
            break;
        }
        }
    }
    if (bad) s_bad = 1u;

    uint32_t tt, te, td;
    const uint32_t xt = block_excl_scan(vt, s_tmp, tt);
    const uint32_t xe = block_excl_scan(ve, s_tmp, te);
    const uint32_t xd = block_excl_scan(vd, s_tmp, td);

    if (tid < 64) {
        const uint32_t gi = L.chunk_base + chunk;
        LocProbe pr{a.flags, a.agg, a.incl, epoch, 0u, 0u, 0ull, 0u};
        if (chunk > 0) {
            if (tid == 0) {
                LocVal agg;
                agg.tup = tt;
                agg.exc = te;
                agg.data = td;
                a.agg[gi] = agg;
                store_rel(&a.flags[gi], (epoch << 2) | 1u);
            }
            wave_lookback(gi, L.chunk_base, pr, a.status);
        }
        if (tid == 0) {
            LocVal pre;
            pre.tup = pr.tup;
            pre.exc = pr.exc;
            pre.data = pr.data;
            LocVal inc;
            inc.tup = pre.tup + tt;
            inc.exc = pre.exc + te;
            inc.data = pre.data + td;
            a.incl[gi] = inc;
            store_rel(&a.flags[gi], (epoch << 2) | 2u);
            s_pre = pre;
        }
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) latch(a.status, kErrLocate);
        return;
    }
    const uint32_t ntiles = L.ntiles;
    uint32_t base_t = s_pre.tup + xt;
    uint64_t base_d = s_pre.data + xd;
    uint32_t base_e = s_pre.exc + xe;
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

#pragma unroll
    for (int q = 0; q < kLocWords; q++) {
        const uint32_t w = wbase + (uint32_t)q;
        if (w >= nwords) break;
        const uint32_t wd = word[q];
        switch (h.codec) {
        case 0: {
            const uint32_t S_total = D >> h.lk;
            for (uint32_t i = 0; i < 8u; i++) {
                const uint32_t s = 8u * w + i;
                if (s >= S_total) break;
                const uint32_t num = sim_num((wd >> (4u * i)) & 15u);
                uint32_t m;
                if (boundary(base_t, num, m)) emit(m, s, m * TT - base_t, 32ull * s, 0);
                base_t += num;
            }
            break;
        }
        case 1:
            if (h.ld == GC_LD_BINARY) {
                const BinUnit u = bin_unit(h.cg);
                for (uint32_t f = 0; f < u.fpw; f++) {
                    const uint32_t t = w * u.fpw + f;
                    if (t >= T) break;
                    if (t > 0u && t % TT == 0u && t / TT < ntiles) emit(t / TT, t, 0, base_d, 0);
                    const uint32_t bit = bin_field_bit(t, u) & 31u;
                    base_d += (uint32_t)h.cg * (((wd >> bit) & mask_of(u.fb)) + 1u);
                }
            } else {
                // terminators (0 bits) of ranks base_t .. base_t + cnt - 1 end in
                // this word; the tile starting at tuple m*TT begins right after
                // the terminator of rank m*TT - 1
                const uint32_t z = ~wd;
                const uint32_t cnt = (uint32_t)__builtin_popcount(z);
                const uint32_t m = (base_t + TT) / TT;
                if (cnt && m < ntiles && m * TT - 1u < base_t + cnt) {
                    uint32_t zz = z;
                    for (uint32_t i = 0; i < m * TT - 1u - base_t; i++) zz &= zz - 1u;
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
                }
                base_t += cnt;
                if (h.ld == GC_LD_IU) base_d += (uint32_t)h.cg * iu_useful(wd);
            }
            break;
        case 2:
            for (int i = 0; i < 4; i++) {
                const uint32_t byte = (wd >> (8 * i)) & 0xFFu;
                const uint32_t b = byte & 63u, F = 8u << (byte >> 6);
                uint32_t m;
                if (boundary(base_t, F, m)) emit(m, 4u * w + (uint32_t)i, m * TT - base_t, base_d, 0);
                base_t += F;
                base_d += (uint64_t)F * b;
            }
            break;
        default: {
            const uint32_t t = 32u * w;
            if (t > 0u && t % TT == 0u && t / TT < ntiles) emit(t / TT, w, 0, base_d, base_e);
            base_d += 32u * min(wd & 63u, 32u);
            base_e += pfd_exc_words(wd, (int)k, h.pfd_pos);
            break;
        }
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
// Decode kernels.

enum : int { kClsSim = 0, kClsGscU = 1, kClsGscB = 2, kClsAfor = 3, kClsPfd = 4 };

template <int TILE, int CLS>
struct DecSmem {
    static constexpr int TTM = TILE / 4;                    // tuples per tile at k = 4
    static constexpr int R = TILE / (4 * kThreads);          // output rounds
    static constexpr int NREC = CLS == kClsPfd ? 1 : TTM;
    static constexpr int NCTRL = CLS == kClsSim ? TTM / 8 + 8 : CLS == kClsGscU ? TTM + 8 : 1;
    static constexpr int NGAP = CLS == kClsPfd ? TILE : 1;
    static constexpr int NEXC = CLS == kClsPfd ? TILE / 4 : 1;
    static constexpr int NBLK = CLS == kClsPfd ? 64 : 1;
    uint32_t rec[NREC];      // per tuple: component bit offset << 6 | width
    uint32_t ctrl[NCTRL];
    uint32_t gaps[NGAP];
    uint32_t exc[NEXC];
    uint32_t blk_off[NBLK], blk_exc[NBLK], blk_desc[NBLK];
    uint32_t wtot[R * kWaves];
    uint32_t wpre[R * kWaves];
    uint32_t tmp[kWaves];
    uint32_t item, bad, prefix, dbase, b0, excw, exc_staged;
};

struct TileCtx {
    const uint32_t *S;
    const uint32_t *ctrl;
    const uint32_t *data;
    HeaderFields h;
    uint32_t n, C, D, k, lk, T, TT, t0, i0, ntup, nint;
    bool has_en;
    TileInfo st, en;
};

__device__ __forceinline__ uint32_t rec_pack(uint32_t rel, uint32_t bw) { return (rel << 6) | bw; }

// ---- Group-Simple: selector-stationary record scatter --------------------
template <int TILE>
__device__ void prologue_sim(const TileCtx &c, DecSmem<TILE, kClsSim> &sm) {
    using SM = DecSmem<TILE, kClsSim>;
    const int tid = threadIdx.x;
    const uint32_t S_total = c.D >> c.lk;
    const uint32_t s_first = c.st.unit, sub0 = c.st.sub;
    const uint32_t s_end = c.has_en ? c.en.unit + (c.en.sub ? 1u : 0u) : S_total;
    const uint32_t nsel = s_end - s_first;
    const uint32_t cw0 = s_first >> 3, cw1 = (s_end + 7u) >> 3;
    const bool rng_ok = s_end <= S_total && s_end > s_first && nsel <= c.TT + 1u && cw1 <= c.C &&
                        cw1 - cw0 <= (uint32_t)SM::NCTRL;
    if (!rng_ok) {
        if (tid == 0) sm.bad = kErrRange;
    } else {
        for (uint32_t i = (uint32_t)tid; i < cw1 - cw0; i += kThreads) sm.ctrl[i] = c.ctrl[cw0 + i];
    }
    if (tid == 0) sm.dbase = s_first;
    __syncthreads();
    constexpr int SPT = (SM::TTM + 1 + kThreads - 1) / kThreads;
    uint32_t sel[SPT];
    uint32_t sum = 0;
    const bool go = !sm.bad;
#pragma unroll
    for (int j = 0; j < SPT; j++) {
        const uint32_t i = (uint32_t)tid * SPT + (uint32_t)j;
        uint32_t s = 15u, cnt = 0;
        if (go && i < nsel) {
            const uint32_t g = s_first + i;
            s = (sm.ctrl[(g >> 3) - cw0] >> ((g & 7u) * 4u)) & 15u;
            const uint32_t j0 = i == 0u ? sub0 : 0u;
            const uint32_t num = s < 10u ? sim_num(s) : 0u;
            if (s >= 10u || num <= j0) {
                sm.bad = kErrSelector;
                s = 15u;
            } else {
                cnt = num - j0;
            }
        }
        sel[j] = s;
        sum += cnt;
    }
    uint32_t total;
    uint32_t run = block_excl_scan(sum, sm.tmp, total);
    if (tid == 0 && go && total < c.ntup) sm.bad = kErrCount;
#pragma unroll
    for (int j = 0; j < SPT; j++) {
        const uint32_t i = (uint32_t)tid * SPT + (uint32_t)j;
        if (sel[j] < 10u) {
            const uint32_t bw = sim_bw(sel[j]);
            const uint32_t j0 = i == 0u ? sub0 : 0u;
            const uint32_t cnt = sim_num(sel[j]) - j0;
            const uint32_t lim = min(cnt, max(c.ntup, run) - run);   // 0 once run >= ntup
            for (uint32_t jj = 0; jj < lim; jj++) sm.rec[run + jj] = rec_pack(32u * i + (j0 + jj) * bw, bw);
            run += cnt;
        }
    }
}

// ---- Group-Scheme with unary descriptors (complete or incomplete) --------
template <int TILE>
__device__ void prologue_gscu(const TileCtx &c, DecSmem<TILE, kClsGscU> &sm) {
    using SM = DecSmem<TILE, kClsGscU>;
    const int tid = threadIdx.x;
    const uint32_t cg = (uint32_t)c.h.cg, umax = 32u / cg;
    const bool iu = c.h.ld == GC_LD_IU;
    const uint32_t p0 = c.st.unit;
    const uint32_t p1 = c.has_en ? c.en.unit : 32u * c.C;
    const uint32_t cw0 = p0 >> 5, cw1 = (p1 + 31u) >> 5;
    const uint32_t nctrl = cw1 - cw0;
    const bool rng_ok = p1 >= p0 && cw1 <= c.C && nctrl <= (uint32_t)SM::NCTRL;
    if (!rng_ok) {
        if (tid == 0) sm.bad = kErrRange;
    } else {
        for (uint32_t i = (uint32_t)tid; i < nctrl; i += kThreads) {
            // only bits in [p0, p1) belong to the tile: the others read as 1
            const uint32_t gw = cw0 + i;
            uint32_t v = c.ctrl[gw];
            if (gw == cw0 && (p0 & 31u)) v |= (1u << (p0 & 31u)) - 1u;
            if (gw == (p1 >> 5) && (p1 & 31u)) v |= ~((1u << (p1 & 31u)) - 1u);
            sm.ctrl[i] = v;
        }
    }
    const uint64_t abs0 = iu ? c.st.data : (uint64_t)cg * p0;
    const uint32_t dbase = (uint32_t)(abs0 >> 5);
    if (tid == 0) sm.dbase = dbase;
    __syncthreads();
    const uint32_t nw = sm.bad ? 0u : nctrl;
    const uint32_t wpt = (nw + kThreads - 1u) / kThreads;
    const uint32_t wl0 = min((uint32_t)tid * wpt, nw), wl1 = min(wl0 + wpt, nw);
    // where this thread's first code starts: after the last terminator of the
    // tile's earlier words, else at p0
    uint32_t start0 = p0;
    if (wl0 < wl1)
        for (uint32_t wl = wl0; wl-- > 0u;) {
            const uint32_t z = ~sm.ctrl[wl];
            if (z) {
                start0 = 32u * (cw0 + wl) + 32u - (uint32_t)__builtin_clz(z);
                break;
            }
        }
    uint32_t cnt = 0, usum = 0;
    {
        uint32_t nxt = start0;
        for (uint32_t wl = wl0; wl < wl1; wl++) {
            uint32_t z = ~sm.ctrl[wl];
            cnt += (uint32_t)__builtin_popcount(z);
            while (z) {
                const uint32_t zp = 32u * (cw0 + wl) + (uint32_t)__builtin_ctz(z);
                z &= z - 1u;
                const uint32_t start = iu ? max(nxt, zp & ~7u) : nxt;
                const uint32_t u = zp - start + 1u;
                if (u > umax) sm.bad = kErrUnary;
                usum += u;
                nxt = zp + 1u;
            }
        }
    }
    uint32_t tcnt, tus;
    const uint32_t xc = block_excl_scan(cnt, sm.tmp, tcnt);
    const uint32_t xu = block_excl_scan(iu ? usum : 0u, sm.tmp, tus);
    if (tid == 0 && !sm.bad && tcnt < c.ntup) sm.bad = kErrCount;
    uint32_t nxt = start0, t = xc, us = xu;
    const uint32_t rel0 = (uint32_t)(abs0 & 31u);
    for (uint32_t wl = wl0; wl < wl1 && t < c.ntup; wl++) {
        uint32_t z = ~sm.ctrl[wl];
        while (z && t < c.ntup) {
            const uint32_t zp = 32u * (cw0 + wl) + (uint32_t)__builtin_ctz(z);
            z &= z - 1u;
            const uint32_t start = iu ? max(nxt, zp & ~7u) : nxt;
            const uint32_t u = min(zp - start + 1u, umax);
            const uint32_t rel = iu ? rel0 + cg * us : (uint32_t)((uint64_t)cg * start - 32ull * dbase);
            sm.rec[t] = rec_pack(rel, cg * u);
            t++;
            us += u;
            nxt = zp + 1u;
        }
    }
}

// ---- Group-Scheme with binary descriptors ---------------------------------
template <int TILE>
__device__ void prologue_gscb(const TileCtx &c, DecSmem<TILE, kClsGscB> &sm) {
    using SM = DecSmem<TILE, kClsGscB>;
    const int tid = threadIdx.x;
    const uint32_t cg = (uint32_t)c.h.cg;
    const BinUnit bu = bin_unit(c.h.cg);
    constexpr int TPT = SM::TTM / kThreads;
    uint32_t bw[TPT];
    uint32_t sum = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < TPT; j++) {
        const uint32_t tt = (uint32_t)tid * TPT + (uint32_t)j;
        uint32_t b = 0;
        if (tt < c.ntup) {
            const uint32_t bit = bin_field_bit(c.t0 + tt, bu);
            if ((bit >> 5) >= c.C) bad = true;
            else b = cg * (((c.ctrl[bit >> 5] >> (bit & 31u)) & mask_of(bu.fb)) + 1u);
        }
        bw[j] = b;
        sum += b;
    }
    if (bad) sm.bad = kErrRange;
    const uint64_t abs0 = c.st.data;
    if (tid == 0) sm.dbase = (uint32_t)(abs0 >> 5);
    uint32_t total;
    uint32_t run = block_excl_scan(sum, sm.tmp, total) + (uint32_t)(abs0 & 31u);
#pragma unroll
    for (int j = 0; j < TPT; j++) {
        const uint32_t tt = (uint32_t)tid * TPT + (uint32_t)j;
        if (tt < c.ntup) sm.rec[tt] = rec_pack(run, bw[j]);
        run += bw[j];
    }
}

// ---- Group-AFOR: frame-stationary record scatter ---------------------------
template <int TILE>
__device__ void prologue_afor(const TileCtx &c, DecSmem<TILE, kClsAfor> &sm) {
    using SM = DecSmem<TILE, kClsAfor>;
    const int tid = threadIdx.x;
    const uint32_t f0 = c.st.unit, sub0 = c.st.sub;
    const uint32_t nfr = min(c.TT / 8u + 2u, 4u * c.C > f0 ? 4u * c.C - f0 : 0u);
    constexpr int FPT = (SM::TTM / 8 + 2 + kThreads - 1) / kThreads;
    uint32_t cnt[FPT], bb[FPT];
    uint32_t csum = 0, bsum = 0;
#pragma unroll
    for (int j = 0; j < FPT; j++) {
        const uint32_t i = (uint32_t)tid * FPT + (uint32_t)j;
        cnt[j] = bb[j] = 0u;
        if (i < nfr) {
            const uint32_t f = f0 + i;
            const uint32_t byte = (c.ctrl[f >> 2] >> (8u * (f & 3u))) & 0xFFu;
            uint32_t b = byte & 63u;
            const uint32_t cls = byte >> 6;
            if (cls == 3u || b > 32u) {
                sm.bad = kErrFrame;
                b = 0;
            }
            const uint32_t F = cls == 0u ? 8u : cls == 1u ? 16u : 32u;
            const uint32_t j0 = i == 0u ? sub0 : 0u;
            if (j0 >= F) sm.bad = kErrFrame;
            else cnt[j] = F - j0;
            bb[j] = b;
            if (i == 0u) sm.b0 = b;
            csum += cnt[j];
            bsum += F * b;
        }
    }
    uint32_t tc, tb;
    uint32_t st_t = block_excl_scan(csum, sm.tmp, tc);
    uint32_t off = block_excl_scan(bsum, sm.tmp, tb);
    if (tid == 0 && !sm.bad && tc < c.ntup) sm.bad = kErrCount;
    const uint64_t fdata0 = c.st.data;
    const uint32_t dbase = (uint32_t)((fdata0 + (uint64_t)sub0 * sm.b0) >> 5);
    if (tid == 0) sm.dbase = dbase;
    const uint32_t frel0 = (uint32_t)(fdata0 - 32ull * dbase);
#pragma unroll
    for (int j = 0; j < FPT; j++) {
        const uint32_t i = (uint32_t)tid * FPT + (uint32_t)j;
        const uint32_t b = bb[j];
        const uint32_t j0 = i == 0u ? sub0 : 0u;
        const uint32_t frel = frel0 + off + j0 * b;
        const uint32_t lim = min(cnt[j], max(c.ntup, st_t) - st_t);   // 0 once st_t >= ntup
        for (uint32_t jj = 0; jj < lim; jj++) sm.rec[st_t + jj] = rec_pack(frel + jj * b, b);
        st_t += cnt[j];
        off += (cnt[j] ? cnt[j] + j0 : 0u) * b;
    }
}

// ---- Group-PFD: per-block descriptors, exceptions staged in LDS ------------
template <int TILE>
__device__ void prologue_pfd(const TileCtx &c, DecSmem<TILE, kClsPfd> &sm, uint64_t stream_words) {
    using SM = DecSmem<TILE, kClsPfd>;
    const int tid = threadIdx.x;
    const uint32_t k = c.k;
    const uint32_t nb = (c.ntup + 31u) >> 5;
    const uint32_t beta0 = c.t0 >> 5;
    const int bitmap = c.h.pfd_pos;
    if (tid < 64) {
        uint32_t desc = 0, b = 0, ew = 0;
        if ((uint32_t)tid < nb) {
            if (beta0 + (uint32_t)tid >= c.C) {
                sm.bad = kErrRange;
            } else {
                desc = c.ctrl[beta0 + (uint32_t)tid];
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
            sm.blk_off[tid] = ib - b;
            sm.blk_exc[tid] = ie - ew;
            sm.blk_desc[tid] = desc;
        }
        if (tid == 63) {
            sm.dbase = (uint32_t)(c.st.data >> 5);
            sm.excw = ie;
        }
    }
    __syncthreads();
    // exception words of the tile's blocks
    const uint64_t ex0 = 4ull + c.C + c.D + c.st.exc;
    const uint32_t excw = sm.excw;
    const bool fits = excw <= (uint32_t)SM::NEXC;
    if (!sm.bad) {
        if (ex0 + excw > stream_words) {
            if (tid == 0) sm.bad = kErrRange;
        } else if (fits) {
            for (uint32_t q = (uint32_t)tid; q < excw; q += kThreads) sm.exc[q] = c.S[ex0 + q];
        }
    }
    if (tid == 0) sm.exc_staged = fits ? 1u : 0u;
}

template <int TILE>
__device__ void patch_pfd(const TileCtx &c, DecSmem<TILE, kClsPfd> &sm) {
    const int tid = threadIdx.x;
    const uint32_t k = c.k, lk = c.lk;
    const uint32_t nb = (c.ntup + 31u) >> 5;
    const uint32_t BI = 32u * k;
    const uint64_t ex0 = 4ull + c.C + c.D + c.st.exc;
    const bool staged = sm.exc_staged != 0u;
    auto exw = [&](uint32_t idx) -> uint32_t { return staged ? sm.exc[idx] : c.S[ex0 + idx]; };
    if (c.h.pfd_pos == GC_PFD_LINKED) {
        for (uint32_t bi = (uint32_t)tid; bi < nb; bi += kThreads) {
            const uint32_t desc = sm.blk_desc[bi];
            const uint32_t nexc = desc >> 20;
            if (!nexc) continue;
            const uint32_t w = 4u << ((desc >> 6) & 3u), wm = mask_of(w);
            const uint32_t xb = sm.blk_exc[bi];
            uint32_t p = (desc >> 8) & 0xFFFu;
            uint32_t *g = &sm.gaps[bi * BI];
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
        const int wave = tid >> 6;
        const uint32_t lane = (uint32_t)(tid & 63);
        for (uint32_t bi = (uint32_t)wave; bi < nb; bi += kWaves) {
            const uint32_t desc = sm.blk_desc[bi];
            const uint32_t nexc = desc >> 20;
            if (!nexc) continue;
            const uint32_t w = 4u << ((desc >> 6) & 3u), wm = mask_of(w);
            const uint32_t nt = (desc >> 8) & 0xFFFu;
            const uint32_t xb = sm.blk_exc[bi];
            const uint32_t tm = exw(xb);
            if ((uint32_t)__builtin_popcount(tm) != nt) {
                if (lane == 0) sm.bad = kErrBitmap;
                continue;
            }
            const uint32_t vbase = xb + 1u + ((nt * k + 31u) >> 5);
            uint32_t run = 0;
            for (uint32_t p0 = 0; p0 < BI; p0 += 64u) {
                const uint32_t p = p0 + lane;
                const uint32_t t = p >> lk, cc = p & (k - 1u);
                bool isx = false;
                if ((tm >> t) & 1u) {
                    const uint32_t rank = (uint32_t)__builtin_popcount(tm & ((1u << t) - 1u));
                    const uint32_t bit = rank * k + cc;
                    isx = (exw(xb + 1u + (bit >> 5)) >> (bit & 31u)) & 1u;
                }
                const uint64_t bal = __ballot(isx);
                const uint32_t before =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                const uint32_t e = run + before;
                if (isx && e < nexc) {
                    const uint32_t bitv = e * w;
                    sm.gaps[bi * BI + p] = (exw(vbase + (bitv >> 5)) >> (bitv & 31u)) & wm;
                }
                run += (uint32_t)__builtin_popcountll(bal);
            }
            if (lane == 0 && run != nexc) sm.bad = kErrBitmap;
        }
    }
}

struct DecProbe {
    const unsigned long long *flags;
    uint32_t epoch;
    unsigned long long f;
    uint32_t acc;
    __device__ int state(uint32_t j) {
        f = load_acq64(&flags[j]);
        const uint32_t stt = (uint32_t)(f >> 32) & 3u;
        return ((uint32_t)(f >> 34) == epoch) ? (int)stt : 0;
    }
    __device__ void accumulate(bool take, uint32_t) { acc += wave_sum(take ? (uint32_t)f : 0u); }
};

template <int TILE, int CLS>
__device__ void decode_tile(const DecodeArgs &a, const ListDesc &L, uint32_t m, uint32_t epoch,
                            uint32_t loc_tag, DecSmem<TILE, CLS> &sm) {
    using SM = DecSmem<TILE, CLS>;
    constexpr int R = SM::R;
    const int tid = threadIdx.x;
    TileCtx c;
    c.S = L.stream;
    const uint32_t w0 = c.S[0];
    c.n = c.S[1];
    c.C = c.S[2];
    c.D = c.S[3];
    bool ok = header_ok(L, w0, c.n, c.C, c.D, c.h);
    c.k = (uint32_t)c.h.k;
    c.lk = (uint32_t)c.h.lk;
    c.T = (c.n + c.k - 1u) >> c.lk;
    c.TT = (uint32_t)TILE >> c.lk;
    c.t0 = m * c.TT;
    c.i0 = m * (uint32_t)TILE;
    ok = ok && c.i0 < c.n;
    c.ntup = ok ? min(c.TT, c.T - c.t0) : 0u;
    c.nint = ok ? min((uint32_t)TILE, c.n - c.i0) : 0u;
    c.ctrl = c.S + 4;
    c.data = c.S + 4 + c.C;
    c.has_en = m + 1u < L.ntiles;
    c.st = TileInfo{};
    c.en = TileInfo{};
    if (m > 0u) {
        c.st = a.tiles[L.tile_base + m];
        ok = ok && c.st.tag == loc_tag;
    }
    if (c.has_en) {
        c.en = a.tiles[L.tile_base + m + 1u];
        ok = ok && c.en.tag == loc_tag;
    }
    if (tid == 0) sm.bad = ok ? 0u : kErrLocate;
    __syncthreads();

    if (!sm.bad) {
        if constexpr (CLS == kClsSim) prologue_sim<TILE>(c, sm);
        else if constexpr (CLS == kClsGscU) prologue_gscu<TILE>(c, sm);
        else if constexpr (CLS == kClsGscB) prologue_gscb<TILE>(c, sm);
        else if constexpr (CLS == kClsAfor) prologue_afor<TILE>(c, sm);
        else prologue_pfd<TILE>(c, sm, L.stream_words);
    }
    __syncthreads();

    // ---- unpack: four consecutive integers per thread and round ------------
    const bool bad = sm.bad != 0u;
    const uint32_t Dk = c.D >> c.lk;
    const uint32_t dbase = sm.dbase;
    const uint32_t nrow = Dk > dbase ? Dk - dbase : 0u;   // data rows from dbase on
    const uint32_t kq = c.k >> 2;                          // 16-byte chunks per row
    const u32x4 *rows = reinterpret_cast<const u32x4 *>(c.data) + (size_t)dbase * kq;
    uint32_t v[R][4];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t q = (uint32_t)(r * kThreads + tid);
        v[r][0] = v[r][1] = v[r][2] = v[r][3] = 0u;
        if (!bad && 4u * q < c.nint) {
            const uint32_t t = q >> (c.lk - 2u);
            const uint32_t cq = q & (kq - 1u);
            uint32_t O, bw;
            if constexpr (CLS == kClsPfd) {
                const uint32_t bi = t >> 5, desc = sm.blk_desc[bi];
                bw = desc & 63u;
                O = 32u * sm.blk_off[bi] + (t & 31u) * bw;
            } else {
                const uint32_t rc = sm.rec[t];
                O = rc >> 6;
                bw = rc & 63u;
            }
            if (bw && nrow) {
                const uint32_t wi = min(O >> 5, nrow - 1u), sh = O & 31u;
                const uint32_t M = mask_of(bw);
                const u32x4 lo = rows[(size_t)wi * kq + cq];
                u32x4 hi = {0u, 0u, 0u, 0u};
                if (sh + bw > 32u) hi = rows[(size_t)min(wi + 1u, nrow - 1u) * kq + cq];
                v[r][0] = funnel(hi.x, lo.x, sh) & M;
                v[r][1] = funnel(hi.y, lo.y, sh) & M;
                v[r][2] = funnel(hi.z, lo.z, sh) & M;
                v[r][3] = funnel(hi.w, lo.w, sh) & M;
            }
        }
    }

    // ---- Group-PFD: exceptions replace their slots -------------------------
    if constexpr (CLS == kClsPfd) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t q = (uint32_t)(r * kThreads + tid);
            *reinterpret_cast<u32x4 *>(&sm.gaps[4u * q]) = u32x4{v[r][0], v[r][1], v[r][2], v[r][3]};
        }
        __syncthreads();
        if (!bad) patch_pfd<TILE>(c, sm);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; r++) {
            const uint32_t q = (uint32_t)(r * kThreads + tid);
            const u32x4 g = *reinterpret_cast<const u32x4 *>(&sm.gaps[4u * q]);
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
    if (c.h.delta) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            v[r][1] += v[r][0];
            v[r][2] += v[r][1];
            v[r][3] += v[r][2];
            const uint32_t inc = wave_incl_scan(v[r][3]);
            add[r] = inc - v[r][3];
            if (lane == 63) sm.wtot[r * kWaves + wave] = inc;
        }
        __syncthreads();
        if (tid < 64) {
            const uint32_t x = (uint32_t)tid < (uint32_t)(R * kWaves) ? sm.wtot[tid] : 0u;
            const uint32_t inc = wave_incl_scan(x);
            if ((uint32_t)tid < (uint32_t)(R * kWaves)) sm.wpre[tid] = inc - x;
            const uint32_t tile_sum = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
            const uint32_t gi = L.tile_base + m;
            const unsigned long long tag = (unsigned long long)(epoch & kEpochMask) << 34;
            DecProbe pr{a.flags, epoch & kEpochMask, 0ull, 0u};
            if (m == 0u) {
                if (tid == 0) store_rel64(&a.flags[gi], tag | (2ull << 32) | tile_sum);
            } else {
                if (tid == 0) store_rel64(&a.flags[gi], tag | (1ull << 32) | tile_sum);
                wave_lookback(gi, L.tile_base, pr, a.status);
                if (tid == 0) store_rel64(&a.flags[gi], tag | (2ull << 32) | (uint32_t)(pr.acc + tile_sum));
            }
            if (tid == 0) sm.prefix = pr.acc;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; r++) add[r] += sm.prefix + sm.wpre[r * kWaves + wave];
    }
    if (tid == 0 && sm.bad) latch(a.status, sm.bad);

    // ---- store ---------------------------------------------------------------
    uint32_t *out = L.out + c.i0;
    const bool vec = (reinterpret_cast<uintptr_t>(out) & 15u) == 0u;
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t q = (uint32_t)(r * kThreads + tid);
        const uint32_t ii = 4u * q;
        if (ii >= c.nint) continue;
        const u32x4 o = {v[r][0] + add[r], v[r][1] + add[r], v[r][2] + add[r], v[r][3] + add[r]};
        if (vec && ii + 4u <= c.nint) {
            __builtin_nontemporal_store(o, reinterpret_cast<u32x4 *>(out + ii));
        } else {
            out[ii] = o.x;
            if (ii + 1u < c.nint) out[ii + 1u] = o.y;
            if (ii + 2u < c.nint) out[ii + 2u] = o.z;
            if (ii + 3u < c.nint) out[ii + 3u] = o.w;
        }
    }
}

template <int TILE, int CLS>
__global__ __launch_bounds__(kThreads) void gc_decode_kernel(DecodeArgs a) {
    __shared__ DecSmem<TILE, CLS> sm;
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
            m = item - L.cls_base;
        } else {
            L = a.single;
            if (item >= L.ntiles) break;
            m = item;
        }
        decode_tile<TILE, CLS>(a, L, m, epoch, loc_tag, sm);
    }
    finish_run(a.state, epoch);
}

// ===========================================================================
// Launchers.

int codec_class(uint32_t w0) {
    HeaderFields h;
    if (!header_fields(w0, h)) return -1;
    switch (h.codec) {
    case 0: return kClsSim;
    case 1: return h.ld == GC_LD_BINARY ? kClsGscB : kClsGscU;
    case 2: return kClsAfor;
    default: return kClsPfd;
    }
}

int launch_locate(const LocateArgs &a, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL(gc_locate_kernel, dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int TILE>
static const void *decode_fn(int cls) {
    switch (cls) {
    case kClsSim: return reinterpret_cast<const void *>(gc_decode_kernel<TILE, kClsSim>);
    case kClsGscU: return reinterpret_cast<const void *>(gc_decode_kernel<TILE, kClsGscU>);
    case kClsGscB: return reinterpret_cast<const void *>(gc_decode_kernel<TILE, kClsGscB>);
    case kClsAfor: return reinterpret_cast<const void *>(gc_decode_kernel<TILE, kClsAfor>);
    case kClsPfd: return reinterpret_cast<const void *>(gc_decode_kernel<TILE, kClsPfd>);
    default: return nullptr;
    }
}

static const void *decode_fn(int tile, int cls) {
    switch (tile) {
    case 2048: return decode_fn<2048>(cls);
    case 4096: return decode_fn<4096>(cls);
    case 8192: return decode_fn<8192>(cls);
    default: return nullptr;
    }
}

int launch_decode(int tile, int cls, const DecodeArgs &a, uint32_t grid, hipStream_t s) {
    const void *fn = decode_fn(tile, cls);
    if (!fn) return -2;
    DecodeArgs arg = a;
    void *params[] = {&arg};
    if (hipLaunchKernel(fn, dim3(grid), dim3(kThreads), params, 0, s) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return 0;
}

int decode_occupancy(int tile, int cls, int *blocks_per_cu) {
    const void *fn = decode_fn(tile, cls);
    if (!fn) return -2;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, kThreads, 0) == hipSuccess ? 0 : -1;
}

int locate_occupancy(int *blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gc_locate_kernel, kThreads, 0) == hipSuccess
               ? 0
               : -1;
}

}  // namespace gcdev
