// blocks.hip -- gfx950 kernels of the encode side of the learned per-block
// codec selector: the 40 features of a block, the coded size of a block in
// every codec class (the exhaustive choice), and the per-block container
// encoder.  A block is 128 integers, i.e. 32 tuples of the 4-way layout, and
// every codec rule below is the whole-list rule of its section applied to
// those 32 tuples:
//   Group-Simple        Algorithm 1 and Table III (Section 4)
//   Group-Scheme        eq. (1)-(2), unary CU/IU and binary descriptors (Section 5.2)
//   Group-AFOR          optimal frames of 8/16/32 tuples (Section 6.1)
//   Group-PFD           width, exceptions and linked positions (Section 6.2)
// One wave64 codes one block; lane t < 32 holds tuple t.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gc.h"
#include "gc_blocks.h"
#include "gc_format.h"
#include "gc_wave.h"

namespace gcblk {

using gcdev::funnel;
using gcdev::wave_incl_max;
using gcdev::wave_incl_scan;
using gcdev::wave_lds_sync;
using gcdev::wave_sum;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) u32x4 gu32x4;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ uint32_t bitw(uint32_t x) { return x ? 32u - (uint32_t)__builtin_clz(x) : 0u; }

__device__ __forceinline__ uint32_t ballot32(bool b) { return (uint32_t)__ballot(b); }

// Table III: selector -> NUM - 1 and BW - 1, 5 bits each.
constexpr uint64_t kNumM1 = 31ull | 15ull << 5 | 9ull << 10 | 7ull << 15 | 5ull << 20 | 4ull << 25 | 3ull << 30 |
                            2ull << 35 | 1ull << 40 | 0ull << 45;
constexpr uint64_t kBwM1 = 0ull | 1ull << 5 | 2ull << 10 | 3ull << 15 | 4ull << 20 | 5ull << 25 | 7ull << 30 |
                           9ull << 35 | 15ull << 40 | 31ull << 45;
__device__ __forceinline__ uint32_t sim_num(uint32_t s) { return (uint32_t)((kNumM1 >> (5 * s)) & 31u) + 1u; }
__device__ __forceinline__ uint32_t sim_bw(uint32_t s) { return (uint32_t)((kBwM1 >> (5 * s)) & 31u) + 1u; }

// Codec class kappa: codec, log2 CG, length descriptor, PFD exception
// threshold zeta = zn / zd.
struct ClassDef {
    uint32_t codec, lcg, ld, zn, zd;
};

__device__ __forceinline__ ClassDef class_def(uint32_t kappa) {
    ClassDef d = {0u, 0u, 0u, 1u, 10u};
    if (kappa == 0u) {
        d.codec = GC_SIMPLE;
    } else if (kappa <= 10u) {
        d.codec = GC_SCHEME;
        if (kappa <= 4u) {
            d.ld = GC_LD_BINARY;
            d.lcg = kappa - 1u;
        } else if (kappa <= 8u) {
            d.ld = GC_LD_CU;
            d.lcg = kappa - 5u;
        } else {
            d.ld = GC_LD_IU;
            d.lcg = kappa - 7u;   // CG 4, 8
        }
    } else if (kappa == 11u) {
        d.codec = GC_AFOR;
    } else {
        d.codec = GC_PFD;
        d.zn = kappa == 12u ? 1u : kappa - 12u;
        d.zd = kappa == 12u ? 64u : 10u;
    }
    return d;
}

// LDS of one wave while it codes one block.
struct BlockSmem {
    uint32_t x[kBlockInts];        // the block
    uint32_t slot[kBlockInts];     // PFD normal slots
    uint32_t epos[kBlockInts + 1]; // PFD exception positions, in order
    uint32_t ctrl[kMaxCtrlWords];
    uint32_t data[kMaxDataWords];
    uint32_t exc[kMaxExcWords];
};

struct BlockLayout {
    uint32_t Cw, D, E;   // control, data and exception words of the payload
};

// ORs value v (width w <= 32) into component c of the data area at bit O.
__device__ __forceinline__ void put_comp(uint32_t *data, uint32_t c, uint32_t O, uint32_t v, uint32_t w) {
    if (!w) return;
    const uint32_t sh = O & 31u, wi = O >> 5;
    atomicOr(&data[4u * wi + c], v << sh);
    if (sh + w > 32u) atomicOr(&data[4u * (wi + 1u) + c], v >> (32u - sh));
}

// Codes block `sm.x` (lane t < 32 holds tuple t in v[], tuple width W) with
// class kappa.  Returns the payload layout; with EMIT the payload is built
// in sm.ctrl / sm.data / sm.exc (which the caller zeroed).
template <bool EMIT>
__device__ BlockLayout code_block(uint32_t kappa, uint32_t lane, const uint32_t (&v)[4], uint32_t W,
                                  BlockSmem &sm) {
    const bool valid = lane < (uint32_t)kTuples;
    const ClassDef d = class_def(kappa);
    BlockLayout L = {0u, 0u, 0u};
    if (d.codec == GC_SIMPLE) {
        // Algorithm 1 on fit masks: bit t of fm[s] says tuple t fits selector s
        const uint32_t smin = W <= 6u ? (W ? W - 1u : 0u) : W <= 8u ? 6u : W <= 10u ? 7u : W <= 16u ? 8u : 9u;
        uint32_t fm[10];
#pragma unroll
        for (int s = 0; s < 10; s++) fm[s] = ballot32(valid && smin <= (uint32_t)s);
        uint32_t j = 0, S = 0, starts = 0, nib[4] = {0u, 0u, 0u, 0u};
        while (j < (uint32_t)kTuples) {
            uint32_t s = 0, cnt = 0;
            for (; s < 9u; s++) {
                cnt = min(sim_num(s), (uint32_t)kTuples - j);
                const uint32_t m = (cnt >= 32u ? ~0u : ((1u << cnt) - 1u)) << j;
                if ((fm[s] & m) == m) break;
            }
            cnt = min(sim_num(s), (uint32_t)kTuples - j);
            starts |= 1u << j;
            nib[S >> 3] |= s << (4u * (S & 7u));
            S++;
            j += cnt;
        }
        L.Cw = (4u * S + 31u) >> 5;
        L.D = 4u * S;
        if (EMIT) {
            if (lane < L.Cw) sm.ctrl[lane] = lane == 0u ? nib[0] : lane == 1u ? nib[1] : lane == 2u ? nib[2] : nib[3];
            if (valid) {
                const uint32_t below = starts & (lane == 31u ? ~0u : ((2u << lane) - 1u));
                const uint32_t si = (uint32_t)__builtin_popcount(below) - 1u;
                const uint32_t st = 31u - (uint32_t)__builtin_clz(below);
                const uint32_t nw = si >> 3;
                const uint32_t word = nw == 0u ? nib[0] : nw == 1u ? nib[1] : nw == 2u ? nib[2] : nib[3];
                const uint32_t bw = sim_bw((word >> (4u * (si & 7u))) & 15u);
#pragma unroll
                for (int c = 0; c < 4; c++) atomicOr(&sm.data[4u * si + c], v[c] << ((lane - st) * bw));
            }
        }
    } else if (d.codec == GC_SCHEME) {
        const uint32_t cg = 1u << d.lcg;
        const uint32_t u = valid ? max(1u, (W + cg - 1u) >> d.lcg) : 0u;   // eq. (1)
        const uint32_t bw = u << d.lcg;                                     // eq. (2)
        const uint32_t ib = wave_incl_scan(bw);
        const uint32_t O = ib - bw;
        const uint32_t sumbw = (uint32_t)__builtin_amdgcn_readlane((int)ib, 63);
        L.D = 4u * ((sumbw + 31u) >> 5);
        uint32_t term = 0;   // bit of this tuple's terminating 0 (unary)
        if (d.ld == GC_LD_BINARY) {
            const uint32_t F = cg == 1u ? 3u : cg == 8u ? 4u : 2u;
            const uint32_t U = cg == 1u ? 16u : 8u;
            const uint32_t Lb = 5u - d.lcg;   // Table IV
            L.Cw = ((((uint32_t)kTuples + F - 1u) / F) * U + 31u) >> 5;
            if (EMIT && valid) {
                const uint32_t bit = (lane / F) * U + (lane % F) * Lb;
                atomicOr(&sm.ctrl[bit >> 5], (u - 1u) << (bit & 31u));
            }
        } else {
            uint32_t bits = 0;
            if (d.ld == GC_LD_CU) {
                const uint32_t iu = wave_incl_scan(u);
                term = iu - 1u;
                bits = (uint32_t)__builtin_amdgcn_readlane((int)iu, 63);
            } else {
                // codes never cross a byte: a code that does not fit the rest
                // of the byte starts at the next one (the gap reads as 1s)
                uint32_t pos = 0;
                for (uint32_t t = 0; t < (uint32_t)kTuples; t++) {
                    const uint32_t ut = (uint32_t)__builtin_amdgcn_readlane((int)u, (int)t);
                    const uint32_t left = 8u - (pos & 7u);
                    if (ut > left) pos += left;
                    if (lane == t) term = pos + ut - 1u;
                    pos += ut;
                }
                bits = pos;
            }
            L.Cw = (bits + 31u) >> 5;
            if (EMIT) {
                for (uint32_t w = lane; w < L.Cw; w += 64u) sm.ctrl[w] = ~0u;
                wave_lds_sync();
                if (valid) atomicAnd(&sm.ctrl[term >> 5], ~(1u << (term & 31u)));
            }
        }
        if (EMIT && valid) {
#pragma unroll
            for (int c = 0; c < 4; c++) put_comp(sm.data, (uint32_t)c, O, v[c], bw);
        }
    } else if (d.codec == GC_AFOR) {
        // widths of the four octets of tuples, then the dynamic programme
        // from the end with frames of 32, 16, 8 tuples (ties keep the larger)
        uint32_t om[4];
#pragma unroll
        for (int o = 0; o < 4; o++) {
            const uint32_t mo = wave_incl_max(valid && (lane >> 3) == (uint32_t)o ? W : 0u);
            om[o] = (uint32_t)__builtin_amdgcn_readlane((int)mo, 63);
        }
        uint32_t cost[5] = {0u, 0u, 0u, 0u, 0u}, choice[4] = {8u, 8u, 8u, 8u};
        for (int o = 3; o >= 0; o--) {
            uint32_t best = 0xFFFFFFFFu;
            for (uint32_t F = 32u; F >= 8u; F >>= 1) {
                const uint32_t no = F >> 3;
                if ((uint32_t)o + no > 4u) continue;
                uint32_t b = 0;
                for (uint32_t q = (uint32_t)o; q < (uint32_t)o + no; q++) b = max(b, om[q]);
                const uint32_t c = 8u + 4u * F * b + cost[o + no];
                if (c < best) {
                    best = c;
                    choice[o] = F;
                }
            }
            cost[o] = best;
        }
        uint32_t nf = 0, fo = 0, ctrl = 0, my_off = 0, my_b = 0;
        for (uint32_t o = 0; o < 4u;) {
            const uint32_t F = choice[o], no = F >> 3;
            uint32_t b = 0;
            for (uint32_t q = o; q < o + no; q++) b = max(b, om[q]);
            ctrl |= (b | ((F == 8u ? 0u : F == 16u ? 1u : 2u) << 6)) << (8u * nf);
            if ((lane >> 3) >= o && (lane >> 3) < o + no) {
                my_off = fo + (lane - 8u * o) * b;
                my_b = b;
            }
            fo += F * b;
            nf++;
            o += no;
        }
        L.Cw = (8u * nf + 31u) >> 5;
        L.D = 4u * ((fo + 31u) >> 5);
        if (EMIT) {
            if (lane == 0u) sm.ctrl[0] = ctrl;
            if (valid) {
#pragma unroll
                for (int c = 0; c < 4; c++) put_comp(sm.data, (uint32_t)c, my_off, v[c], my_b);
            }
        }
    } else {
        // Step 2: the smallest b with fewer than zeta of the tuples wider
        uint32_t b = 0;
        while (b < 32u && (uint32_t)__builtin_popcount(ballot32(valid && W > b)) * d.zd >= d.zn * 32u) b++;
        // Step 3: exceptions are the integers wider than b
        uint32_t nib = 0, mw = 0;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const uint32_t w = bitw(v[c]);
            if (valid && w > b) {
                nib |= 1u << c;
                mw = max(mw, w);
            }
        }
        const uint32_t maxw = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_max(mw), 63);
        // positions p = 4t + c of the exceptions, as four 32-bit masks
        uint32_t M[4] = {0u, 0u, 0u, 0u};
        for (uint32_t t = 0; t < (uint32_t)kTuples; t++) {
            const uint32_t nt = (uint32_t)__builtin_amdgcn_readlane((int)nib, (int)t);
            M[t >> 3] |= nt << (4u * (t & 7u));
        }
        const uint32_t nx = (uint32_t)(__builtin_popcount(M[0]) + __builtin_popcount(M[1]) +
                                       __builtin_popcount(M[2]) + __builtin_popcount(M[3]));
        // Step 4: 8, 16 or 32-bit exception values
        const uint32_t wcode = nx == 0u ? 0u : maxw <= 8u ? 1u : maxw <= 16u ? 2u : 3u;
        const uint32_t ew = wcode ? 4u << wcode : 0u;
        // linked positions: each slot of an exception holds the distance to
        // the next one; a distance beyond 2^b - 1 needs compulsory stops
        const uint32_t lim = b >= 32u ? 0xFFFFFFFFu : (1u << b) - 1u;
        uint32_t ne = 0, prev = 0xFFFFFFFFu;
        for (uint32_t q = 0; q < 4u; q++) {
            uint32_t m = M[q];
            while (m) {
                const uint32_t p = 32u * q + (uint32_t)__builtin_ctz(m);
                m &= m - 1u;
                if (prev != 0xFFFFFFFFu) {
                    while (p - prev - 1u > lim) {
                        prev += 1u << b;
                        if (EMIT && lane == 0u) sm.epos[ne] = prev;
                        ne++;
                    }
                }
                if (EMIT && lane == 0u) sm.epos[ne] = p;
                ne++;
                prev = p;
            }
        }
        L.Cw = 1u;
        L.D = 4u * b;
        L.E = (ne * ew + 31u) >> 5;
        if (EMIT) {
            for (uint32_t p = lane; p < (uint32_t)kBlockInts; p += 64u) sm.slot[p] = sm.x[p];
            wave_lds_sync();
            for (uint32_t e = lane; e < ne; e += 64u) {
                const uint32_t p = sm.epos[e];
                sm.slot[p] = e + 1u < ne ? sm.epos[e + 1u] - p - 1u : 0u;
                atomicOr(&sm.exc[(e * ew) >> 5], sm.x[p] << ((e * ew) & 31u));
            }
            wave_lds_sync();
            if (lane == 0u) sm.ctrl[0] = b | (wcode << 6) | ((ne ? sm.epos[0] : 0u) << 8) | (ne << 20);
            if (valid) {
#pragma unroll
                for (int c = 0; c < 4; c++) put_comp(sm.data, (uint32_t)c, lane * b, sm.slot[4u * lane + c], b);
            }
        }
    }
    return L;
}

// Loads block blk into registers (tuple per lane) and LDS.
// Lane t < 32 loads tuple t of the block (issued apart from its use, so
// that the kernels' other loads can be in flight with it).
__device__ __forceinline__ u32x4 block_tuple(const uint32_t *in, size_t blk, uint32_t lane) {
    const gu32x4 *src = (const gu32x4 *)(in + blk * (size_t)kBlockInts);
    u32x4 q = {0u, 0u, 0u, 0u};
    if (lane < (uint32_t)kTuples) q = src[lane];
    return q;
}

// The tuple's integers and width in registers, the block in LDS.
__device__ __forceinline__ void stage_block(u32x4 q, uint32_t lane, uint32_t (&v)[4], uint32_t &W, BlockSmem &sm) {
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
    W = bitw(q.x | q.y | q.z | q.w);
    if (lane < (uint32_t)kTuples) reinterpret_cast<u32x4 *>(sm.x)[lane] = q;
    wave_lds_sync();
}

// ---- features ---------------------------------------------------------------
// The largest bit width / 32; the histogram of the 32 tuple widths (0..32)
// / 32, a tuple's width being that of its widest integer; and the integers
// wider than maxw - t for t = 1..6 (all of them when maxw - t < 0) / 128.
// Two blocks per wave: lane 32h + t holds tuple t of block 2w + h.

// x reduced over the 32 lanes of each half wave
__device__ __forceinline__ uint32_t half_max(uint32_t x) {
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o));
    return x;
}
__device__ __forceinline__ uint32_t half_sum(uint32_t x) {
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) x += (uint32_t)__shfl_xor((int)x, o);
    return x;
}

__global__ __launch_bounds__(kThreads) void gc_block_features_kernel(const uint32_t *in, size_t nblocks,
                                                                     float *feat) {
    const uint32_t lane = threadIdx.x & 63u, h = lane >> 5, t = lane & 31u;
    const size_t pair = (size_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (2u * pair >= nblocks) return;
    const size_t blk = 2u * pair + h;
    const bool valid = blk < nblocks;   // the pair's second block may be missing
    u32x4 q = {0u, 0u, 0u, 0u};
    if (valid) q = ((const gu32x4 *)(in + blk * (size_t)kBlockInts))[t];
    const uint32_t tw = bitw(q.x | q.y | q.z | q.w);
    const uint32_t maxw = half_max(tw);
    // the tuple-width histogram of each block in LDS: one atomic add per tuple
    __shared__ uint32_t hist[kWaves][2][33];
    uint32_t *hw = hist[threadIdx.x >> 6][h];
    hw[t] = 0u;
    if (t == 0u) hw[32] = 0u;
    gcdev::wave_lds_sync();
    if (valid) atomicAdd(&hw[tw], 1u);
    gcdev::wave_lds_sync();
    const uint32_t ha = t ? hw[t - 1u] : 0u;      // bin t - 1: feature t >= 1
    const uint32_t hb = t < 2u ? hw[31u + t] : 0u;  // bins 31, 32: features 32, 33
    // integers by d = maxw - width, for d = 0..5, eight bits per count
    uint32_t n03 = 0, n45 = 0;
    const uint32_t v[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const uint32_t d = maxw - bitw(v[j]);
        n03 += d < 4u ? 1u << (8u * d) : 0u;
        n45 += d - 4u < 2u ? 1u << (8u * (d - 4u)) : 0u;
    }
    if (!valid) n03 = n45 = 0u;
    n03 = half_sum(n03);
    n45 = half_sum(n45);
    // wider than maxw - u: the integers with d < u
    uint32_t wider = 0;
#pragma unroll
    for (uint32_t d = 0; d < 6u; d++) {
        const uint32_t nd = d < 4u ? (n03 >> (8u * d)) & 255u : (n45 >> (8u * (d - 4u))) & 255u;
        wider += d + 2u <= t ? nd : 0u;   // lane t = 2..7 takes u = t - 1
    }
    if (!valid) return;
    float *f = feat + blk * (size_t)kFeatures;
    f[t] = t == 0u ? (float)maxw / 32.0f : (float)ha / 32.0f;
    if (t < 8u) f[32u + t] = t < 2u ? (float)hb / 32.0f : (float)wider / 128.0f;
}

// ---- sizes of every class, exhaustive choice -----------------------------------
__global__ __launch_bounds__(kThreads) void gc_block_sizes_kernel(const uint32_t *in, size_t nblocks,
                                                                  uint32_t *sizes, uint8_t *best, float *cost) {
    __shared__ BlockSmem smem[kWaves];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const size_t blk = (size_t)blockIdx.x * kWaves + wave;
    if (blk >= nblocks) return;
    BlockSmem &sm = smem[wave];
    uint32_t v[4], W;
    stage_block(block_tuple(in, blk, lane), lane, v, W, sm);
    uint32_t bsize = 0xFFFFFFFFu, bk = 0, mine = 0;
    for (uint32_t kappa = 0; kappa < (uint32_t)kClasses; kappa++) {
        const BlockLayout L = code_block<false>(kappa, lane, v, W, sm);
        const uint32_t sz = 1u + L.Cw + L.D + L.E;
        if (lane == kappa) mine = sz;
        if (sz < bsize) {
            bsize = sz;
            bk = kappa;
        }
    }
    if (sizes && lane < (uint32_t)kClasses) sizes[blk * (size_t)kClasses + lane] = mine;
    if (best && lane == 0u) best[blk] = (uint8_t)bk;
    // relative size excess over the least size: the selector's training cost
    if (cost && lane < (uint32_t)kClasses) cost[blk * (size_t)kClasses + lane] = (float)(mine - bsize) / (float)bsize;
}

// ---- container encode ----------------------------------------------------------
// Pass 1: the payload words of every block for its class; a class out of
// range counts no words and sets *bad.
__global__ __launch_bounds__(kThreads) void gc_blockmix_size_kernel(const uint32_t *in, size_t nblocks,
                                                                    const uint8_t *cls, uint32_t *words,
                                                                    uint32_t *bad) {
    __shared__ BlockSmem smem[kWaves];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const size_t blk = (size_t)blockIdx.x * kWaves + wave;
    if (blk >= nblocks) return;
    BlockSmem &sm = smem[wave];
    const u32x4 q = block_tuple(in, blk, lane);   // in flight with the class load
    const uint32_t kappa = (uint32_t)__builtin_amdgcn_readfirstlane((int)cls[blk]);
    uint32_t w = 0u;
    if (kappa < (uint32_t)kClasses) {
        uint32_t v[4], W;
        stage_block(q, lane, v, W, sm);
        const BlockLayout L = code_block<false>(kappa, lane, v, W, sm);
        w = L.Cw + L.D + L.E;
    } else if (lane == 0u) {
        *bad = 1u;
    }
    if (lane == 0u) words[blk] = w;
}

// Exclusive scan of u32 values, 1024 per workgroup round: per-chunk sums,
// one workgroup scanning them, then the in-chunk scans.
__device__ __forceinline__ uint32_t block_scan(uint32_t x, uint32_t *tmp, uint32_t &total) {
    const uint32_t inc = wave_incl_scan(x);
    const uint32_t w = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 63u) tmp[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; i++) {
        const uint32_t t = tmp[i];
        pre += (uint32_t)i < w ? t : 0u;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return pre + inc - x;
}

__global__ __launch_bounds__(kThreads) void gc_scan_chunks_kernel(const uint32_t *x, size_t n, uint32_t *csum) {
    __shared__ uint32_t tmp[kWaves];
    const size_t i = ((size_t)blockIdx.x * kThreads + threadIdx.x) * 4u;
    uint32_t s = 0;
    for (int j = 0; j < 4; j++) s += i + j < n ? x[i + j] : 0u;
    uint32_t total;
    (void)block_scan(s, tmp, total);
    if (threadIdx.x == 0) csum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void gc_scan_top_kernel(uint32_t *csum, size_t nchunks, uint32_t *total_out) {
    __shared__ uint32_t tmp[kWaves];
    uint32_t run = 0;
    for (size_t b = 0; b < nchunks; b += kThreads) {
        const size_t i = b + threadIdx.x;
        const uint32_t v = i < nchunks ? csum[i] : 0u;
        uint32_t total;
        const uint32_t p = block_scan(v, tmp, total);
        if (i < nchunks) csum[i] = run + p;
        run += total;
    }
    if (threadIdx.x == 0) *total_out = run;
}

__global__ __launch_bounds__(kThreads) void gc_scan_apply_kernel(const uint32_t *x, size_t n, const uint32_t *cpre,
                                                                 uint32_t *out) {
    __shared__ uint32_t tmp[kWaves];
    const size_t i = ((size_t)blockIdx.x * kThreads + threadIdx.x) * 4u;
    uint32_t v[4], s = 0;
    for (int j = 0; j < 4; j++) {
        v[j] = i + j < n ? x[i + j] : 0u;
        s += v[j];
    }
    uint32_t total;
    uint32_t p = cpre[blockIdx.x] + block_scan(s, tmp, total);
    for (int j = 0; j < 4; j++) {
        if (i + j < n) out[i + j] = p;
        p += v[j];
    }
}

// Pass 2: block words and payloads at their offsets (after the header and
// the block words); the header itself is written by the host side.
// Writes every block at its offset and, from the first block's wave, the
// container header; a block of an invalid class, or whose payload would end
// past cap_words, writes no payload (the host reports either from the
// sizing pass's flag and total).
__global__ __launch_bounds__(kThreads) void gc_blockmix_emit_kernel(const uint32_t *in, size_t nblocks,
                                                                    const uint8_t *cls, const uint32_t *offs,
                                                                    uint32_t *out, size_t cap_words, uint32_t n,
                                                                    const uint32_t *total) {
    __shared__ BlockSmem smem[kWaves];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const size_t blk = (size_t)blockIdx.x * kWaves + wave;
    if (blk >= nblocks) return;
    BlockSmem &sm = smem[wave];
    // the block, its class and its offset, loaded together
    const u32x4 q = block_tuple(in, blk, lane);
    const uint32_t kappa = (uint32_t)__builtin_amdgcn_readfirstlane((int)cls[blk]);
    const uint32_t off = (uint32_t)__builtin_amdgcn_readfirstlane((int)offs[blk]);
    for (uint32_t w = lane; w < (uint32_t)kMaxCtrlWords; w += 64u) sm.ctrl[w] = 0u;
    for (uint32_t w = lane; w < (uint32_t)kMaxDataWords; w += 64u) sm.data[w] = 0u;
    for (uint32_t w = lane; w < (uint32_t)kMaxExcWords; w += 64u) sm.exc[w] = 0u;
    if (blk == 0u && lane < 4u) {
        const uint32_t t = *total;   // written by the scan
        out[lane] = lane == 0u ? GC_FMT_VERSION | (4u << 8) | (2u << 12) : lane == 1u ? n : lane == 2u ? (uint32_t)nblocks : t;
    }
    if (kappa >= (uint32_t)kClasses) return;
    uint32_t v[4], W;
    stage_block(q, lane, v, W, sm);
    const BlockLayout L = code_block<true>(kappa, lane, v, W, sm);
    wave_lds_sync();
    const size_t pay = 4u + nblocks + (size_t)off;
    if (pay + L.Cw + L.D + L.E <= cap_words) {
        uint32_t *p = out + pay;
        for (uint32_t w = lane; w < L.Cw; w += 64u) p[w] = sm.ctrl[w];
        for (uint32_t w = lane; w < L.D; w += 64u) p[L.Cw + w] = sm.data[w];
        for (uint32_t w = lane; w < L.E; w += 64u) p[L.Cw + L.D + w] = sm.exc[w];
    }
    if (lane == 0u) out[4 + blk] = kappa | (L.Cw << 5) | (L.D << 14) | (L.E << 23);
}

// ---- launchers -------------------------------------------------------------------

static dim3 grid_for(size_t nblocks) { return dim3((unsigned)((nblocks + kWaves - 1) / kWaves)); }

int launch_block_features(const uint32_t *in, size_t nblocks, float *feat, hipStream_t s) {
    if (!nblocks) return 0;
    // two blocks per wave
    hipLaunchKernelGGL(gc_block_features_kernel, grid_for((nblocks + 1) / 2), dim3(kThreads), 0, s, in, nblocks, feat);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_block_sizes(const uint32_t *in, size_t nblocks, uint32_t *sizes, uint8_t *best, float *cost,
                       hipStream_t s) {
    if (!nblocks) return 0;
    hipLaunchKernelGGL(gc_block_sizes_kernel, grid_for(nblocks), dim3(kThreads), 0, s, in, nblocks, sizes, best,
                       cost);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

size_t scan_chunks(size_t n) { return (n + 4 * kThreads - 1) / (4 * kThreads); }

// Sizes of every block for its class, their exclusive scan into offs, the
// total into result[0] and a bad-class flag into result[1] (device memory);
// csum holds scan_chunks(nblocks) words.
int launch_blockmix_plan(const uint32_t *in, size_t nblocks, const uint8_t *cls, uint32_t *words, uint32_t *offs,
                         uint32_t *csum, uint32_t *result, hipStream_t s) {
    if (!nblocks) return 0;
    const size_t nc = scan_chunks(nblocks);
    uint32_t *total = result;
    if (hipMemsetAsync(result + 1, 0, sizeof(uint32_t), s) != hipSuccess) return -1;
    hipLaunchKernelGGL(gc_blockmix_size_kernel, grid_for(nblocks), dim3(kThreads), 0, s, in, nblocks, cls, words,
                       result + 1);
    hipLaunchKernelGGL(gc_scan_chunks_kernel, dim3((unsigned)nc), dim3(kThreads), 0, s, words, nblocks, csum);
    hipLaunchKernelGGL(gc_scan_top_kernel, dim3(1), dim3(kThreads), 0, s, csum, nc, total);
    hipLaunchKernelGGL(gc_scan_apply_kernel, dim3((unsigned)nc), dim3(kThreads), 0, s, words, nblocks, csum, offs);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_blockmix_emit(const uint32_t *in, size_t nblocks, const uint8_t *cls, const uint32_t *offs,
                         uint32_t *out, size_t cap_words, uint32_t n, const uint32_t *total, hipStream_t s) {
    if (!nblocks) return 0;
    hipLaunchKernelGGL(gc_blockmix_emit_kernel, grid_for(nblocks), dim3(kThreads), 0, s, in, nblocks, cls, offs,
                       out, cap_words, n, total);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gcblk
