// gc_format.h -- stream-format constants of libgc, shared by the host
// encoder, the host-side validation and the HIP kernels.
#pragma once
#include <stdint.h>

#define GC_FMT_VERSION 1u

#if defined(__HIPCC__)
#define GC_HD __host__ __device__
#else
#define GC_HD
#endif

// Header word 0: version:8 | codec:4 | log2(k):3 | log2(CG):2 | LD:2 |
// delta:1 | pfd_pos:1 | reserved:11.
GC_HD inline uint32_t header_word0(int codec, int k, int cg, int ld, int delta, int pfd_pos) {
    uint32_t lk = 0, lc = 0;
    while ((1 << lk) < k) lk++;
    while ((1 << lc) < cg) lc++;
    return GC_FMT_VERSION | ((uint32_t)codec << 8) | (lk << 12) | (lc << 15) | ((uint32_t)ld << 17) |
           ((uint32_t)(delta ? 1 : 0) << 19) | ((uint32_t)pfd_pos << 20);
}

struct HeaderFields {
    int codec, lk, k, lcg, cg, ld, delta, pfd_pos;
};

// Decodes word 0; returns false for a word no decoder accepts.
GC_HD inline bool header_fields(uint32_t w0, HeaderFields &h) {
    h.codec = (int)((w0 >> 8) & 15u);
    h.lk = (int)((w0 >> 12) & 7u);
    h.k = 1 << h.lk;
    h.lcg = (int)((w0 >> 15) & 3u);
    h.cg = 1 << h.lcg;
    h.ld = (int)((w0 >> 17) & 3u);
    h.delta = (int)((w0 >> 19) & 1u);
    h.pfd_pos = (int)((w0 >> 20) & 1u);
    if ((w0 & 0xFFu) != GC_FMT_VERSION || (w0 >> 21) != 0u) return false;
    if (h.codec > 4 || h.lk < 2 || h.lk > 6) return false;
    if (h.codec == 1) {
        if (h.ld > 2 || (h.ld == 2 && h.cg < 4)) return false;
    } else if (((w0 >> 15) & 15u) != 0u) {
        return false;
    }
    if (h.codec != 3 && h.pfd_pos != 0) return false;
    return true;
}

// Tuples of a Group-AFOR / Group-VSEncoding frame of class cls (bits 6..7 of
// its control byte): 8, 16, 32, and for Group-VSEncoding 12 (class 3, which
// Group-AFOR leaves unused).
GC_HD inline uint32_t frame_tuples(uint32_t cls) { return cls == 3u ? 12u : 8u << cls; }

#include <stddef.h>
namespace gcfmt {
size_t bound_words(size_t n, int codec, int k);
}
