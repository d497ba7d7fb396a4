// encode.cpp -- host-side Group-codec encoders of libgc (index build).
//
// Writes the stream format declared in include/gc.h.  Encoding happens once,
// when an index is built, so it runs on the host cores; gc_encode_lists
// spreads many lists over std::threads.  Packing is word-level: a value of b
// bits at component bit offset o is OR-ed into at most two words.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "gc.h"
#include "gc_format.h"

namespace gcfmt {

namespace {

inline int width_of(uint32_t x) { return x ? 32 - __builtin_clz(x) : 0; }

// Group-Simple patterns (Section 4.1.2, Table III): (NUM, BW) per selector.
constexpr int kSimNum[10] = {32, 16, 10, 8, 6, 5, 4, 3, 2, 1};
constexpr int kSimBw[10] = {1, 2, 3, 4, 5, 6, 8, 10, 16, 32};

struct Areas {
    std::vector<uint32_t> ctrl, data, exc;
    uint64_t ctrl_bits = 0;
};

// Control stream: LSB-first bits over little-endian words.
struct BitWriter {
    std::vector<uint32_t> &w;
    uint64_t pos = 0;
    explicit BitWriter(std::vector<uint32_t> &v) : w(v) {}
    void put(uint32_t v, int nb) {
        if (nb == 0) return;
        const uint64_t end = pos + (uint64_t)nb;
        if ((end + 31) / 32 > w.size()) w.resize((end + 31) / 32 + 64, 0u);
        const uint64_t wi = pos >> 5;
        const int sh = (int)(pos & 31);
        w[wi] |= v << sh;
        if (sh + nb > 32) w[wi + 1] |= v >> (32 - sh);
        pos = end;
    }
    void ones(int nb) {
        while (nb > 0) {
            int c = nb > 32 ? 32 : nb;
            put(c == 32 ? 0xFFFFFFFFu : ((1u << c) - 1u), c);
            nb -= c;
        }
    }
};

// Writes v (nb <= 32 bits, already < 2^nb) at bit offset o of component c.
inline void put_comp(std::vector<uint32_t> &D, int k, int c, uint64_t o, uint32_t v, int nb) {
    if (nb == 0) return;
    const uint64_t wi = o >> 5;
    const int sh = (int)(o & 31);
    D[(size_t)(wi * (uint64_t)k) + (size_t)c] |= v << sh;
    if (sh + nb > 32) D[(size_t)((wi + 1) * (uint64_t)k) + (size_t)c] |= v >> (32 - sh);
}

inline uint32_t low_bits(uint32_t v, int b) { return b >= 32 ? v : (v & ((1u << b) - 1u)); }

// ---- Group-Simple -------------------------------------------------------
void enc_simple(const uint32_t *x, size_t T, int k, const std::vector<uint8_t> &W, Areas &a) {
    // Algorithm 1: from the current tuple, the smallest selector whose NUM
    // next tuples (or all that remain) fit in its width.
    std::vector<uint8_t> sel;
    sel.reserve(T / 4 + 1);
    size_t j = 0;
    while (j < T) {
        const size_t left = T - j;
        int pick = 9;
        size_t cover = 1;
        for (int i = 0; i < 10; i++) {
            const size_t lim = std::min<size_t>((size_t)kSimNum[i], left);
            size_t p = 0;
            while (p < lim && W[j + p] <= kSimBw[i]) p++;
            if (p == (size_t)kSimNum[i] || p == left) {
                pick = i;
                cover = p;
                break;
            }
        }
        sel.push_back((uint8_t)pick);
        j += cover;
    }
    const size_t S = sel.size();
    BitWriter cw(a.ctrl);
    for (size_t s = 0; s < S; s++) cw.put(sel[s], 4);
    a.ctrl_bits = cw.pos;
    a.data.assign((size_t)k * S, 0u);
    size_t t0 = 0;
    for (size_t s = 0; s < S; s++) {
        const int bw = kSimBw[sel[s]];
        const size_t cnt = std::min<size_t>((size_t)kSimNum[sel[s]], T - t0);
        uint32_t *vec = &a.data[s * (size_t)k];
        for (size_t jj = 0; jj < cnt; jj++) {
            const uint32_t *tp = x + (t0 + jj) * (size_t)k;
            const int sh = (int)jj * bw;
            for (int c = 0; c < k; c++) vec[c] |= tp[c] << sh;   // bw * NUM <= 32
        }
        t0 += cnt;
    }
}

// ---- Group-Scheme -------------------------------------------------------
void binary_unit(int cg, int &fields, int &unit_bits, int &field_bits) {
    field_bits = cg == 1 ? 5 : cg == 2 ? 4 : cg == 4 ? 3 : 2;   // Table IV
    fields = cg == 1 ? 3 : cg == 8 ? 4 : 2;
    unit_bits = cg == 1 ? 16 : 8;
}

void enc_scheme(const uint32_t *x, size_t T, int k, int cg, int ld, const std::vector<uint8_t> &W,
                Areas &a) {
    BitWriter cw(a.ctrl);
    int fields = 0, unit_bits = 0, field_bits = 0;
    if (ld == GC_LD_BINARY) binary_unit(cg, fields, unit_bits, field_bits);
    std::vector<uint8_t> bwv(T);
    uint64_t O = 0;
    for (size_t t = 0; t < T; t++) {
        int u = (W[t] + cg - 1) / cg;            // eq. (1), unary form
        if (u < 1) u = 1;
        bwv[t] = (uint8_t)(cg * u);              // eq. (2)
        O += (uint64_t)(cg * u);
        if (ld == GC_LD_CU) {
            cw.ones(u - 1);
            cw.put(0, 1);
        } else if (ld == GC_LD_IU) {
            const int left = 8 - (int)(cw.pos & 7);
            if (u > left) cw.ones(left);
            cw.ones(u - 1);
            cw.put(0, 1);
        } else {
            const uint64_t unit = t / (size_t)fields, f = t % (size_t)fields;
            cw.pos = unit * (uint64_t)unit_bits + f * (uint64_t)field_bits;
            cw.put((uint32_t)(u - 1), field_bits);
            if (f + 1 == (uint64_t)fields || t + 1 == T) cw.pos = (unit + 1) * (uint64_t)unit_bits;
        }
    }
    a.ctrl_bits = cw.pos;
    if (ld != GC_LD_BINARY) {
        // unary areas: 1 bits to the end of the (4-word rounded) control area
        const uint64_t C = ((cw.pos + 31) / 32 + 3) / 4 * 4;
        cw.ones((int)(C * 32 - cw.pos));
    }
    a.data.assign((size_t)k * (size_t)((O + 31) / 32) + (size_t)k, 0u);
    O = 0;
    for (size_t t = 0; t < T; t++) {
        const int b = bwv[t];
        const uint32_t *tp = x + t * (size_t)k;
        for (int c = 0; c < k; c++) put_comp(a.data, k, c, O, tp[c], b);
        O += (uint64_t)b;
    }
    a.data.resize((size_t)k * (size_t)((O + 31) / 32));
}

// ---- Group-AFOR and Group-VSEncoding ----------------------------------------
// vse: Group-VSEncoding, frames of 8, 12, 16 or 32 tuples starting at multiples
// of 4 tuples (VSEncoding's frame lengths that fit a group frame; class 3 of
// the control byte is the 12-tuple frame); otherwise Group-AFOR's 8, 16, 32.
void enc_afor(const uint32_t *x, size_t M, int k, const std::vector<uint8_t> &W, Areas &a, bool vse) {
    // exact minimum of sum over frames of (8 + k*F*b) by dynamic programming
    // from the end, over groups of g tuples; frame sizes tried largest first
    // with strict improvement, so ties keep the larger frame (Section 6.1)
    const size_t g = vse ? 4 : 8;
    const size_t oct = M / g;
    std::vector<uint64_t> cost(oct + 1, 0);
    std::vector<uint8_t> choice(oct + 1, 0);
    std::vector<uint8_t> omax(oct + 1, 0);   // max width per group of tuples
    for (size_t o = 0; o < oct; o++) {
        uint8_t m = 0;
        for (size_t t = g * o; t < g * o + g; t++) m = std::max(m, W[t]);
        omax[o] = m;
    }
    static const int kAfor[3] = {32, 16, 8}, kVse[4] = {32, 16, 12, 8};
    const int *Fs = vse ? kVse : kAfor;
    const int nF = vse ? 4 : 3;
    for (size_t o = oct; o-- > 0;) {
        uint64_t best = UINT64_MAX;
        uint8_t bf = 0;
        for (int i = 0; i < nF; i++) {
            const int F = Fs[i];
            const size_t no = (size_t)F / g;
            if (o + no > oct || cost[o + no] == UINT64_MAX) continue;   // the rest cannot be tiled
            uint8_t b = 0;
            for (size_t q = o; q < o + no; q++) b = std::max(b, omax[q]);
            const uint64_t c = 8 + (uint64_t)k * (uint64_t)F * b + cost[o + no];
            if (c < best) {
                best = c;
                bf = (uint8_t)F;
            }
        }
        cost[o] = best;
        choice[o] = bf;
    }
    BitWriter cw(a.ctrl);
    uint64_t O = 0;
    std::vector<std::pair<uint8_t, uint8_t>> frames;
    for (size_t o = 0; o < oct; o += choice[o] / g) {
        const int F = choice[o];
        uint8_t b = 0;
        for (size_t q = o; q < o + (size_t)F / g; q++) b = std::max(b, omax[q]);
        const uint32_t cls = F == 8 ? 0u : F == 16 ? 1u : F == 32 ? 2u : 3u;
        cw.put((uint32_t)b | (cls << 6), 8);
        frames.emplace_back((uint8_t)F, b);
        O += (uint64_t)F * b;
    }
    a.ctrl_bits = cw.pos;
    a.data.assign((size_t)k * (size_t)((O + 31) / 32) + (size_t)k, 0u);
    O = 0;
    size_t t0 = 0;
    for (auto &fb : frames) {
        const int F = fb.first, b = fb.second;
        for (int j = 0; j < F; j++) {
            const uint32_t *tp = x + (t0 + (size_t)j) * (size_t)k;
            for (int c = 0; c < k; c++) put_comp(a.data, k, c, O + (uint64_t)j * b, tp[c], b);
        }
        O += (uint64_t)F * b;
        t0 += (size_t)F;
    }
    a.data.resize((size_t)k * (size_t)((O + 31) / 32));
}

// ---- Group-PFD ----------------------------------------------------------
void enc_pfd(const uint32_t *x, size_t M, int k, int zn, int zd, int mode,
             const std::vector<uint8_t> &W, Areas &a) {
    const size_t nb = M / 32;
    const size_t BI = (size_t)32 * (size_t)k;
    BitWriter cw(a.ctrl);
    uint64_t dwords = 0;
    std::vector<uint32_t> slot(BI), pos, val;
    std::vector<uint8_t> isx(BI), tex(32);
    // first pass: widths, so the data area can be sized once
    std::vector<uint8_t> bsel(nb);
    for (size_t blk = 0; blk < nb; blk++) {
        // step 2: smallest b with (#tuples wider than b) / 32 < zeta
        int cnt[34] = {0};
        for (int t = 0; t < 32; t++) cnt[W[blk * 32 + (size_t)t]]++;
        int wider = 32 - cnt[0];   // tuples wider than b, for b = 0
        int b = 0;
        while ((long)wider * zd >= (long)zn * 32) {
            b++;
            wider -= cnt[b];
        }
        bsel[blk] = (uint8_t)b;
        dwords += (uint64_t)b;
    }
    a.data.assign((size_t)k * (size_t)dwords + (size_t)k, 0u);
    dwords = 0;
    for (size_t blk = 0; blk < nb; blk++) {
        const uint32_t *xb = x + blk * BI;
        const int b = bsel[blk];
        // step 3: exceptions are the wide integers of the wide tuples
        int maxw = 0;
        size_t nx = 0;
        for (int t = 0; t < 32; t++) {
            tex[t] = 0;
            const bool wide = W[blk * 32 + (size_t)t] > b;
            for (int c = 0; c < k; c++) {
                const size_t p = (size_t)t * (size_t)k + (size_t)c;
                const int w = width_of(xb[p]);
                isx[p] = (uint8_t)(wide && w > b);
                if (isx[p]) {
                    nx++;
                    tex[t] = 1;
                    maxw = std::max(maxw, w);
                }
            }
        }
        // step 4: 8, 16 or 32-bit exception values
        const int wcode = nx == 0 ? 0 : maxw <= 8 ? 1 : maxw <= 16 ? 2 : 3;
        const int ew = wcode ? (4 << wcode) : 0;
        pos.clear();
        val.clear();
        for (size_t p = 0; p < BI; p++) slot[p] = xb[p];
        uint32_t first = 0;
        if (mode == GC_PFD_LINKED) {
            const uint64_t lim = b >= 32 ? UINT64_MAX : ((1ull << b) - 1);
            long prev = -1;
            for (size_t p = 0; p < BI; p++) {
                if (!isx[p]) continue;
                if (prev >= 0)
                    while ((uint64_t)((long)p - prev - 1) > lim) {   // compulsory stop
                        const long cp = prev + (long)(1ull << b);
                        pos.push_back((uint32_t)cp);
                        val.push_back(xb[cp]);
                        prev = cp;
                    }
                pos.push_back((uint32_t)p);
                val.push_back(xb[p]);
                prev = (long)p;
            }
            for (size_t e = 0; e < pos.size(); e++)
                slot[pos[e]] = e + 1 < pos.size() ? pos[e + 1] - pos[e] - 1 : 0u;
            first = pos.empty() ? 0u : pos[0];
        } else {
            uint32_t nt = 0;
            for (size_t p = 0; p < BI; p++)
                if (isx[p]) {
                    pos.push_back((uint32_t)p);
                    val.push_back(xb[p]);
                    slot[p] = low_bits(xb[p], b);
                }
            for (int t = 0; t < 32; t++) nt += tex[t];
            first = nt;
        }
        const uint32_t nexc = (uint32_t)pos.size();
        cw.put((uint32_t)b | ((uint32_t)wcode << 6) | (first << 8) | (nexc << 20), 32);
        for (int t = 0; t < 32; t++)
            for (int c = 0; c < k; c++)
                put_comp(a.data, k, c, dwords * 32 + (uint64_t)t * (uint64_t)b,
                         slot[(size_t)t * (size_t)k + (size_t)c], b);
        dwords += (uint64_t)b;
        if (nexc == 0) continue;
        std::vector<uint32_t> blkx;
        BitWriter ewr(blkx);
        if (mode == GC_PFD_BITMAP) {
            uint32_t tm = 0;
            for (int t = 0; t < 32; t++) tm |= (uint32_t)tex[t] << t;
            ewr.put(tm, 32);
            for (int t = 0; t < 32; t++)
                if (tex[t])
                    for (int c = 0; c < k; c++) ewr.put(isx[(size_t)t * (size_t)k + (size_t)c], 1);
            ewr.pos = (ewr.pos + 31) / 32 * 32;
        }
        for (uint32_t e = 0; e < nexc; e++) ewr.put(val[e], ew);
        const size_t words = (size_t)((ewr.pos + 31) / 32);
        blkx.resize(words);
        a.exc.insert(a.exc.end(), blkx.begin(), blkx.end());
    }
    a.ctrl_bits = cw.pos;
    a.data.resize((size_t)k * (size_t)dwords);
}

}  // namespace

size_t bound_words(size_t n, int codec, int k) {
    const size_t T = (n + (size_t)k - 1) / (size_t)k + 32;
    size_t b = 8 + (size_t)k * (T + 2) + 2 * T + 8;
    if (codec == GC_PFD) b += (size_t)k * T + (T / 32 + 1) * (size_t)(k + 2) + 8;
    return b;
}

int check_params(int codec, const gc_params *p) {
    if (!p) return GC_EINVAL;
    if (codec < 0 || codec > 4) return GC_EINVAL;
    if (p->k < 4 || p->k > 64 || (p->k & (p->k - 1)) != 0) return GC_EINVAL;
    if (codec == GC_SCHEME) {
        if (p->cg != 1 && p->cg != 2 && p->cg != 4 && p->cg != 8) return GC_EINVAL;
        if (p->ld > 2 || (p->ld == GC_LD_IU && p->cg < 4)) return GC_EINVAL;
    }
    if (codec == GC_PFD) {
        if (p->zeta_num == 0 || p->zeta_den == 0 || p->zeta_num >= p->zeta_den) return GC_EINVAL;
        if (p->pfd_pos > 1) return GC_EINVAL;
    }
    if (p->flags & ~GC_DELTA) return GC_EINVAL;
    return GC_OK;
}

int encode_one(const uint32_t *in, size_t n, int codec, const gc_params *p, uint32_t *out,
               size_t cap, size_t *out_words) {
    int rc = check_params(codec, p);
    if (rc) return rc;
    if (n > 0xFFFFFFFFull) return GC_EINVAL;
    const int k = (int)p->k;
    const size_t T = (n + (size_t)k - 1) / (size_t)k;
    const size_t unit = codec == GC_AFOR || codec == GC_VSE ? 8 : codec == GC_PFD ? 32 : 1;
    const size_t M = (T + unit - 1) / unit * unit;
    std::vector<uint32_t> x(M * (size_t)k + 1, 0u);
    if (p->flags & GC_DELTA) {
        for (size_t i = 0; i < n; i++) x[i] = i ? in[i] - in[i - 1] : in[0];
    } else if (n) {
        std::memcpy(x.data(), in, n * 4);
    }
    std::vector<uint8_t> W(M);
    for (size_t t = 0; t < M; t++) {
        uint32_t o = 0;   // OR has the width of the max (Section 4.4)
        for (int c = 0; c < k; c++) o |= x[t * (size_t)k + (size_t)c];
        W[t] = (uint8_t)width_of(o);
    }
    Areas a;
    switch (codec) {
    case GC_SIMPLE: enc_simple(x.data(), T, k, W, a); break;
    case GC_SCHEME: enc_scheme(x.data(), T, k, p->cg, p->ld, W, a); break;
    case GC_AFOR: enc_afor(x.data(), M, k, W, a, false); break;
    case GC_VSE: enc_afor(x.data(), M, k, W, a, true); break;
    default: enc_pfd(x.data(), M, k, p->zeta_num, p->zeta_den, p->pfd_pos, W, a); break;
    }
    const size_t C = ((size_t)((a.ctrl_bits + 31) / 32) + 3) / 4 * 4;
    const size_t D = a.data.size();
    const size_t E4 = (a.exc.size() + 3) / 4 * 4;
    const size_t total = 4 + C + D + E4;
    if (total > cap) return GC_ENOSPC;
    std::memset(out, 0, total * 4);
    out[0] = header_word0(codec, k, codec == GC_SCHEME ? p->cg : 1, codec == GC_SCHEME ? p->ld : 0,
                          (p->flags & GC_DELTA) != 0, codec == GC_PFD ? p->pfd_pos : 0);
    out[1] = (uint32_t)n;
    out[2] = (uint32_t)C;
    out[3] = (uint32_t)D;
    a.ctrl.resize(std::max(a.ctrl.size(), C), 0u);
    std::memcpy(out + 4, a.ctrl.data(), C * 4);
    if (D) std::memcpy(out + 4 + C, a.data.data(), D * 4);
    if (!a.exc.empty()) std::memcpy(out + 4 + C + D, a.exc.data(), a.exc.size() * 4);
    *out_words = total;
    return GC_OK;
}

}  // namespace gcfmt

extern "C" {

size_t gc_encoded_bound_words(size_t n, gc_codec codec, const gc_params *p) {
    if (!p || p->k < 4 || p->k > 64) return 0;
    return gcfmt::bound_words(n, (int)codec, (int)p->k);
}

gc_status gc_encode(const uint32_t *h_in, size_t n, gc_codec codec, const gc_params *p,
                    uint32_t *h_out, size_t out_cap_words, size_t *out_words) {
    if ((!h_in && n) || !h_out || !out_words) return GC_EINVAL;
    try {
        return (gc_status)gcfmt::encode_one(h_in, n, (int)codec, p, h_out, out_cap_words,
                                            out_words);
    } catch (...) {
        return GC_ENOMEM;
    }
}

size_t gc_encoded_bound_words_lists(const uint64_t *in_offs, size_t nlists, const gc_codec *codecs,
                                    const gc_params *params, int one_param) {
    if (!in_offs || !codecs || !params) return 0;
    size_t total = 0;
    for (size_t i = 0; i < nlists; i++) {
        const gc_params *p = one_param ? params : params + i;
        if (in_offs[i + 1] < in_offs[i] || p->k < 4 || p->k > 64) return 0;
        total += gcfmt::bound_words(in_offs[i + 1] - in_offs[i], (int)codecs[i], (int)p->k);
    }
    return total;
}

gc_status gc_encode_lists(const uint32_t *h_in, const uint64_t *in_offs, size_t nlists,
                          const gc_codec *codecs, const gc_params *params, int one_param,
                          uint32_t *h_out, size_t out_cap_words, uint64_t *out_offs,
                          int nthreads) {
    if (!h_in || !in_offs || !codecs || !params || !h_out || !out_offs) return GC_EINVAL;
    // pass 1 (parallel): encode each list into its own bound-sized slot of a
    // scratch arena; pass 2: compact into h_out in list order
    std::vector<uint64_t> slot(nlists + 1, 0);
    for (size_t i = 0; i < nlists; i++) {
        const gc_params *p = one_param ? params : params + i;
        if (in_offs[i + 1] < in_offs[i] || p->k < 4 || p->k > 64) return GC_EINVAL;
        slot[i + 1] = slot[i] + gcfmt::bound_words(in_offs[i + 1] - in_offs[i], (int)codecs[i],
                                                   (int)p->k);
    }
    std::vector<uint32_t> arena;
    std::vector<uint64_t> len(nlists, 0);
    try {
        arena.resize(slot[nlists]);
    } catch (...) {
        return GC_ENOMEM;
    }
    int nt = nthreads > 0 ? nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
    std::atomic<size_t> next{0};
    std::atomic<int> err{0};
    auto work = [&]() {
        for (;;) {
            size_t i = next.fetch_add(1);
            if (i >= nlists) break;
            const gc_params *p = one_param ? params : params + i;
            size_t w = 0;
            int rc;
            try {
                rc = gcfmt::encode_one(h_in + in_offs[i], in_offs[i + 1] - in_offs[i],
                                       (int)codecs[i], p, arena.data() + slot[i],
                                       slot[i + 1] - slot[i], &w);
            } catch (...) {
                rc = GC_ENOMEM;
            }
            if (rc) {
                int z = 0;
                err.compare_exchange_strong(z, rc);
            }
            len[i] = w;
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; t++) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
    if (err.load()) return (gc_status)err.load();
    uint64_t off = 0;
    for (size_t i = 0; i < nlists; i++) {
        out_offs[i] = off;
        off += len[i];
    }
    out_offs[nlists] = off;
    if (off > out_cap_words) return GC_ENOSPC;
    for (size_t i = 0; i < nlists; i++)
        std::memcpy(h_out + out_offs[i], arena.data() + slot[i], len[i] * 4);
    return GC_OK;
}

}  // extern "C"
