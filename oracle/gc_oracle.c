/*
 * gc_oracle.c -- plain scalar CPU oracle for the Group integer codecs of
 * Zhao, Zhang, Lemire, Shan, Nie, Yan, Wen, "A General SIMD-based Approach to
 * Accelerating Compression Algorithms" (arXiv 1502.01916).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * Style: deliberately slow and obvious.  Every bitstream is written and read
 * one bit at a time; every selection rule is written in the order the paper
 * states it.  Where the paper leaves a byte-level detail open (its figures
 * are lost) this file follows one fixed reading; the readings are listed in
 * the design notes and pinned by the tests.
 *
 * Stream layout (one list):
 *   word 0   : version:8 | codec:4 | log2k:3 | cgcode:2 | ld:2 | delta:1 |
 *              pfd_pos:1 | reserved:11 (zero)
 *   word 1   : n, the number of integers in the list
 *   word 2   : C, control-area words (a multiple of 4)
 *   word 3   : D, data-area words (a multiple of k)
 *   then C control words, D data words, and (Group-PFD only) the exception
 *   area, padded with zero words to a multiple of 4.
 * The data area uses the k-way vertical layout (Section 2.1.2, Section 3.1):
 * word w of component c is data word k*w + c.  Each component is an LSB-first
 * bitstream; a value that crosses a word boundary keeps its low part in the
 * earlier word (the carry rule of Section 5.3.2, unary step 2).  The control
 * area is one LSB-first bitstream over little-endian words.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "gc_oracle.h"

/* ------------------------------------------------------------------------ */
/* Effective bit width (Section 2.1.2): the minimum number of bits that hold x
 * in binary; 0 for x = 0.  Equal to ceil(log2(x+1)) of eq. (1).           */
int or_bw(uint32_t x)
{
    int b = 0;
    while (x != 0) {
        b++;
        x >>= 1;
    }
    return b;
}

/* Quad max array (Section 4.2): quadmax[i] = max of the k integers of tuple i
 * (the paper's k is 4).  x holds T*k integers.                             */
void or_tuple_max(const uint32_t *x, size_t T, int k, uint32_t *qmax)
{
    for (size_t t = 0; t < T; t++) {
        uint32_t m = 0;
        for (int c = 0; c < k; c++)
            if (x[t * (size_t)k + c] > m)
                m = x[t * (size_t)k + c];
        qmax[t] = m;
    }
}

/* d-gaps (Section 2.1.1): g_1 = d_1, g_i = d_i - d_{i-1}; wrapping mod 2^32. */
void or_dgap(const uint32_t *d, size_t n, uint32_t *g)
{
    for (size_t i = 0; i < n; i++)
        g[i] = (i == 0) ? d[0] : (uint32_t)(d[i] - d[i - 1]);
}

/* Recovering docIDs from d-gaps: inclusive prefix sum, mod 2^32. */
void or_prefix_sum(const uint32_t *g, size_t n, uint32_t *d)
{
    uint32_t s = 0;
    for (size_t i = 0; i < n; i++) {
        s = (uint32_t)(s + g[i]);
        d[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Bit-at-a-time stream helpers.                                            */

typedef struct {
    uint32_t *w;       /* words (zero-initialised by the caller)          */
    size_t cap;        /* capacity in words                                */
    int stride;        /* 1 for the control stream, k for a component     */
    int comp;          /* component index for the data area               */
    uint64_t pos;      /* next bit position                                */
    int err;
} bitsink;

static void sink_bit(bitsink *s, int bit)
{
    uint64_t word = s->pos / 32;
    size_t idx = (size_t)word * (size_t)s->stride + (size_t)s->comp;
    if (idx >= s->cap) {
        s->err = 1;
    } else if (bit) {
        s->w[idx] |= (uint32_t)1u << (s->pos % 32);
    }
    s->pos++;
}

static void sink_value(bitsink *s, uint32_t v, int nbits)
{
    for (int i = 0; i < nbits; i++)
        sink_bit(s, (int)((v >> i) & 1u));
}

typedef struct {
    const uint32_t *w;
    size_t nwords;     /* words available to this reader (index bound)    */
    int stride;
    int comp;
    uint64_t pos;
    int err;
} bitsrc;

static int src_bit(bitsrc *s)
{
    uint64_t word = s->pos / 32;
    size_t idx = (size_t)word * (size_t)s->stride + (size_t)s->comp;
    s->pos++;
    if (idx >= s->nwords) {
        s->err = 1;
        return 0;
    }
    return (int)((s->w[idx] >> ((s->pos - 1) % 32)) & 1u);
}

static uint32_t src_value(bitsrc *s, int nbits)
{
    uint32_t v = 0;
    for (int i = 0; i < nbits; i++)
        v |= (uint32_t)src_bit(s) << i;
    return v;
}

static size_t round_up(size_t a, size_t m) { return (a + m - 1) / m * m; }
static size_t ceil_div(size_t a, size_t m) { return (a + m - 1) / m; }

/* ------------------------------------------------------------------------ */
/* Group-Simple, Table III.                                                 */
static const int GSIM_NUM[10] = {32, 16, 10, 8, 6, 5, 4, 3, 2, 1};
static const int GSIM_BW[10]  = { 1,  2,  3, 4, 5, 6, 8, 10, 16, 32};

void or_gsim_table(int *num, int *bw)
{
    for (int i = 0; i < 10; i++) {
        num[i] = GSIM_NUM[i];
        bw[i] = GSIM_BW[i];
    }
}

/* Algorithm 1 (Section 4.2): pattern selection on the quad max array.
 * MaxArr has L entries; returns TotalModeNum and fills ModeArr.            */
size_t or_gsim_select(const uint32_t *MaxArr, size_t L, uint8_t *ModeArr)
{
    size_t TotalModeNum = 0;
    size_t l = L;
    size_t j = 0, k = 0;
    while (l > 0) {
        int i;
        size_t pos = 0;
        for (i = 0; i <= 9; i++) {
            size_t n = (size_t)GSIM_NUM[i];
            int b = GSIM_BW[i];
            uint64_t mask = ((uint64_t)1 << b) - 1;   /* Power(2,b) - 1 */
            size_t lim = n < l ? n : l;
            pos = 0;
            while (pos < lim && (uint64_t)MaxArr[j + pos] <= mask)
                pos = pos + 1;
            if (pos == n || pos == l)
                break;
        }
        /* selector 9 (32 bits) always accepts one tuple, so i <= 9 here */
        l = l - pos;
        j = j + pos;
        ModeArr[k] = (uint8_t)i;
        k = k + 1;
        TotalModeNum = TotalModeNum + 1;
    }
    return TotalModeNum;
}

/* ------------------------------------------------------------------------ */
/* Parameters and header.                                                   */

static int log2_int(int v)
{
    int r = 0;
    while ((1 << r) < v)
        r++;
    return r;
}

static int params_ok(const or_params *p)
{
    if (p->codec < 0 || p->codec > 4)
        return 0;
    if (p->k < 4 || p->k > 64 || (p->k & (p->k - 1)) != 0)
        return 0;
    if (p->codec == OR_SCHEME) {
        if (p->cg != 1 && p->cg != 2 && p->cg != 4 && p->cg != 8)
            return 0;
        if (p->ld < 0 || p->ld > 2)
            return 0;
        /* incomplete unary only for 4- and 8-bit granularity (Section 5.2.1) */
        if (p->ld == OR_LD_IU && p->cg < 4)
            return 0;
    }
    if (p->codec == OR_PFD) {
        /* 0 < zeta < 1 (Section 6.2, step 2) */
        if (p->zeta_num <= 0 || p->zeta_den <= 0 || p->zeta_num >= p->zeta_den)
            return 0;
        if (p->pfd_pos < 0 || p->pfd_pos > 1)
            return 0;
    }
    return 1;
}

static uint32_t header_word0(const or_params *p)
{
    uint32_t cgcode = 0, ld = 0, pos = 0;
    if (p->codec == OR_SCHEME) {
        cgcode = (uint32_t)log2_int(p->cg);
        ld = (uint32_t)p->ld;
    }
    if (p->codec == OR_PFD)
        pos = (uint32_t)p->pfd_pos;
    return (uint32_t)OR_VERSION | ((uint32_t)p->codec << 8) |
           ((uint32_t)log2_int(p->k) << 12) | (cgcode << 15) | (ld << 17) |
           ((uint32_t)(p->delta ? 1 : 0) << 19) | (pos << 20);
}

/* Unpacks a header word into params; returns 0 if it is not a valid word. */
int or_parse_header(uint32_t w0, or_params *p)
{
    memset(p, 0, sizeof(*p));
    if ((w0 & 0xFFu) != OR_VERSION)
        return 0;
    if ((w0 >> 21) != 0)
        return 0;
    p->codec = (int)((w0 >> 8) & 0xFu);
    int lk = (int)((w0 >> 12) & 7u);
    p->k = 1 << lk;
    p->cg = 1 << ((w0 >> 15) & 3u);
    p->ld = (int)((w0 >> 17) & 3u);
    p->delta = (int)((w0 >> 19) & 1u);
    p->pfd_pos = (int)((w0 >> 20) & 1u);
    p->zeta_num = 1;
    p->zeta_den = 10;
    if (p->codec > 4 || lk < 2 || lk > 6)
        return 0;
    if (p->codec == OR_SCHEME) {
        if (p->ld > 2 || (p->ld == OR_LD_IU && p->cg < 4))
            return 0;
    } else if (((w0 >> 15) & 0xFu) != 0) {
        return 0;
    }
    if (p->codec != OR_PFD && p->pfd_pos != 0)
        return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Encoded areas, built before assembly into one stream.                    */
typedef struct {
    uint32_t *ctrl;   size_t ctrl_cap;  uint64_t ctrl_bits;  size_t C;
    uint32_t *data;   size_t data_cap;  size_t D;
    uint32_t *exc;    size_t exc_cap;   size_t E;
    int err;
} areas;

static void areas_free(areas *a)
{
    free(a->ctrl);
    free(a->data);
    free(a->exc);
}

static int areas_alloc(areas *a, size_t T, int k)
{
    memset(a, 0, sizeof(*a));
    /* generous bounds: <= 64 control bits per tuple, one extra word per
     * component for straddling values, exceptions <= every integer plus
     * per-block bookkeeping */
    a->ctrl_cap = 2 * T + 8;
    a->data_cap = (size_t)k * (T + 2);
    a->exc_cap = (size_t)k * T + (T / 32 + 1) * (size_t)(k + 2) + 8;
    a->ctrl = (uint32_t *)calloc(a->ctrl_cap, 4);
    a->data = (uint32_t *)calloc(a->data_cap, 4);
    a->exc = (uint32_t *)calloc(a->exc_cap, 4);
    return a->ctrl && a->data && a->exc;
}

/* ------------------------------------------------------------------------ */
/* Group-Simple encode (Section 4.2) on padded tuples.                      */
static void gsim_encode(const uint32_t *x, size_t T, int k, areas *a,
                        const uint8_t *forced_sel, size_t forced_S)
{
    uint32_t *qmax = (uint32_t *)calloc(T + 1, 4);
    uint8_t *sel = (uint8_t *)calloc(T + 1, 1);
    size_t S;
    or_tuple_max(x, T, k, qmax);
    if (forced_sel) {
        S = forced_S;
        memcpy(sel, forced_sel, S);
    } else {
        S = or_gsim_select(qmax, T, sel);
    }
    /* control area: selector s is the 4-bit snip s of the control stream */
    bitsink cs = {a->ctrl, a->ctrl_cap, 1, 0, 0, 0};
    for (size_t s = 0; s < S; s++)
        sink_value(&cs, sel[s], 4);
    a->ctrl_bits = cs.pos;
    a->C = round_up(ceil_div((size_t)cs.pos, 32), 4);
    /* data area: one vector (k words) per selector; tuple j of the vector
     * occupies bits [j*BW, (j+1)*BW) of every component                   */
    size_t t0 = 0;
    for (size_t s = 0; s < S; s++) {
        int i = sel[s];
        size_t num = (size_t)GSIM_NUM[i];
        int bw = GSIM_BW[i];
        if (t0 >= T) {
            a->err = 1;        /* a forced sequence longer than the list */
            break;
        }
        size_t cnt = (T - t0) < num ? (T - t0) : num;
        for (size_t j = 0; j < cnt; j++) {
            for (int c = 0; c < k; c++) {
                uint32_t v = x[(t0 + j) * (size_t)k + c];
                if (bw < 32 && (v >> bw) != 0)
                    a->err = 1;   /* a forced selector sequence that does not fit */
                bitsink ds = {a->data, a->data_cap, k, c, (uint64_t)s * 32 + j * (uint64_t)bw, 0};
                sink_value(&ds, v, bw);
                if (ds.err)
                    a->err = 1;
            }
        }
        t0 += cnt;
    }
    if (t0 != T)
        a->err = 1;
    a->D = (size_t)k * S;
    if (cs.err)
        a->err = 1;
    free(qmax);
    free(sel);
}

/* Group-Simple decode (Section 4.3).                                      */
static int gsim_decode(const uint32_t *ctrl, size_t C, const uint32_t *data, size_t D,
                       size_t T, int k, uint32_t *x)
{
    size_t S = D / (size_t)k;
    if (D % (size_t)k)
        return OR_ECORRUPT;
    if (S > C * 8)
        return OR_ECORRUPT;
    bitsrc cs = {ctrl, C, 1, 0, 0, 0};
    size_t done = 0;
    for (size_t s = 0; s < S; s++) {
        uint32_t sel = src_value(&cs, 4);        /* step 2: read four bits   */
        if (sel >= 10)
            return OR_ECORRUPT;
        if (done >= T)
            return OR_ECORRUPT;                  /* a selector with no tuple */
        size_t num = (size_t)GSIM_NUM[sel];
        int bw = GSIM_BW[sel];
        size_t cnt = (T - done) < num ? (T - done) : num;
        for (size_t j = 0; j < cnt; j++)          /* step 3: decode the vector */
            for (int c = 0; c < k; c++) {
                bitsrc ds = {data, D, k, c, (uint64_t)s * 32 + j * (uint64_t)bw, 0};
                x[(done + j) * (size_t)k + c] = src_value(&ds, bw);
            }
        done += cnt;                             /* step 4: advance          */
    }
    if (cs.err || done != T)
        return OR_ECORRUPT;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Group-Scheme (Section 5).                                                */

/* eq. (1) for the unary descriptor, floored at one unit: an all-zero tuple
 * still takes one unit of CG bits.                                         */
int or_gsc_units(uint32_t quadmax, int cg)
{
    int w = or_bw(quadmax);            /* ceil(log2(quadmax+1)) */
    int u = (w + cg - 1) / cg;
    return u < 1 ? 1 : u;
}

/* Binary length-descriptor packing unit (Section 5.2.1 b, footnote 2,
 * Section 7.2): fields per unit, unit size in bits, field width.           */
static void gsc_binary_unit(int cg, int *fields, int *unit_bits, int *field_bits)
{
    *field_bits = 5 - log2_int(cg);    /* Table IV: 5, 4, 3, 2 */
    switch (cg) {
    case 1: *fields = 3; *unit_bits = 16; break;   /* 16-bit pattern, 12 ints */
    case 2: *fields = 2; *unit_bits = 8; break;    /* 8-bit pattern, 8 ints   */
    case 4: *fields = 2; *unit_bits = 8; break;    /* 8-bit pattern, 8 ints   */
    default: *fields = 4; *unit_bits = 8; break;   /* 8-bit pattern, 16 ints  */
    }
}

static void gsc_encode(const uint32_t *x, size_t T, int k, int cg, int ld, areas *a)
{
    uint32_t *qmax = (uint32_t *)calloc(T + 1, 4);
    or_tuple_max(x, T, k, qmax);
    bitsink cs = {a->ctrl, a->ctrl_cap, 1, 0, 0, 0};
    uint64_t O = 0;                         /* shared component bit offset */
    int fields = 0, unit_bits = 0, field_bits = 0;
    if (ld == OR_LD_BINARY)
        gsc_binary_unit(cg, &fields, &unit_bits, &field_bits);
    for (size_t t = 0; t < T; t++) {
        int u = or_gsc_units(qmax[t], cg);
        int BW = cg * u;                     /* eq. (2) */
        if (ld == OR_LD_CU) {
            for (int i = 0; i < u - 1; i++)
                sink_bit(&cs, 1);
            sink_bit(&cs, 0);
        } else if (ld == OR_LD_IU) {
            int left = 8 - (int)(cs.pos % 8);
            if (u > left)                    /* no code crosses a byte: pad */
                for (int i = 0; i < left; i++)
                    sink_bit(&cs, 1);
            for (int i = 0; i < u - 1; i++)
                sink_bit(&cs, 1);
            sink_bit(&cs, 0);
        } else {
            uint64_t unit = t / (size_t)fields, f = t % (size_t)fields;
            cs.pos = unit * (uint64_t)unit_bits + f * (uint64_t)field_bits;
            sink_value(&cs, (uint32_t)(u - 1), field_bits);
            if (f == (uint64_t)fields - 1 || t == T - 1)
                cs.pos = (unit + 1) * (uint64_t)unit_bits;
        }
        for (int c = 0; c < k; c++) {
            bitsink ds = {a->data, a->data_cap, k, c, O, 0};
            sink_value(&ds, x[t * (size_t)k + c], BW);
            if (ds.err)
                a->err = 1;
        }
        O += (uint64_t)BW;
    }
    a->ctrl_bits = cs.pos;
    a->C = round_up(ceil_div((size_t)cs.pos, 32), 4);
    /* unary control areas are filled with 1 bits to the end of the area */
    if (ld != OR_LD_BINARY)
        while (cs.pos < (uint64_t)a->C * 32)
            sink_bit(&cs, 1);
    a->D = (size_t)k * ceil_div((size_t)O, 32);
    if (cs.err)
        a->err = 1;
    free(qmax);
}

static int gsc_decode(const uint32_t *ctrl, size_t C, const uint32_t *data, size_t D,
                      size_t T, int k, int cg, int ld, uint32_t *x)
{
    bitsrc cs = {ctrl, C, 1, 0, 0, 0};
    uint64_t O = 0;
    int umax = 32 / cg;
    int fields = 0, unit_bits = 0, field_bits = 0;
    if (ld == OR_LD_BINARY)
        gsc_binary_unit(cg, &fields, &unit_bits, &field_bits);
    for (size_t t = 0; t < T; t++) {
        int u;
        if (ld == OR_LD_CU) {
            int ones = 0;
            while (src_bit(&cs) == 1) {
                ones++;
                if (cs.err || ones >= umax)
                    return OR_ECORRUPT;
            }
            u = ones + 1;
        } else if (ld == OR_LD_IU) {
            int ones = 0;
            for (;;) {
                int bit = src_bit(&cs);
                if (cs.err)
                    return OR_ECORRUPT;
                if (bit == 0)
                    break;
                ones++;
                if (cs.pos % 8 == 0)
                    ones = 0;             /* a run of 1s up to a byte end is padding */
            }
            u = ones + 1;
            if (u > umax)
                return OR_ECORRUPT;
        } else {
            uint64_t unit = t / (size_t)fields, f = t % (size_t)fields;
            cs.pos = unit * (uint64_t)unit_bits + f * (uint64_t)field_bits;
            u = (int)src_value(&cs, field_bits) + 1;
        }
        if (cs.err)
            return OR_ECORRUPT;
        int BW = cg * u;                     /* eq. (2) */
        for (int c = 0; c < k; c++) {
            bitsrc ds = {data, D, k, c, O, 0};
            x[t * (size_t)k + c] = src_value(&ds, BW);
            if (ds.err)
                return OR_ECORRUPT;
        }
        O += (uint64_t)BW;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Group-AFOR (Section 6.1): frames of 8, 16 or 32 tuples (32/64/128 ints at
 * k = 4), optimal partition by dynamic programming.                        */

static int max_width(const uint32_t *qmax, size_t i, size_t F)
{
    int b = 0;
    for (size_t t = i; t < i + F; t++) {
        int w = or_bw(qmax[t]);
        if (w > b)
            b = w;
    }
    return b;
}

/* cost[i] = minimum bits to code tuples [i, M): each frame costs one
 * control byte plus k*F*b data bits.  Ties prefer the larger frame.
 * Fills frame sizes (in tuples) in order; returns the frame count.        */
size_t or_afor_partition(const uint32_t *qmax, size_t M, int k, uint8_t *Fout)
{
    static const int Fs[3] = {32, 16, 8};
    uint64_t *cost = (uint64_t *)calloc(M + 1, 8);
    uint8_t *choice = (uint8_t *)calloc(M + 1, 1);
    cost[M] = 0;
    for (size_t ii = M; ii-- > 0;) {
        if ((ii % 8) != 0)
            continue;
        uint64_t best = UINT64_MAX;
        int bestF = 0;
        for (int f = 0; f < 3; f++) {
            size_t F = (size_t)Fs[f];
            if (ii + F > M)
                continue;
            uint64_t c = 8 + (uint64_t)k * F * (uint64_t)max_width(qmax, ii, F) + cost[ii + F];
            if (c < best) {
                best = c;
                bestF = (int)F;
            }
        }
        cost[ii] = best;
        choice[ii] = (uint8_t)bestF;
    }
    size_t nf = 0;
    for (size_t i = 0; i < M; i += choice[i])
        Fout[nf++] = choice[i];
    free(cost);
    free(choice);
    return nf;
}

/* Group-VSEncoding: the same frames and control bytes, partitioned by the
 * dynamic programme of VSEncoding (Section 2.2 names its frame-length set
 * {1, 2, 4, 8, 12, 16, 32, 64}).  A group frame is a run of whole tuples
 * between 8 and 32 tuples long (the shortest and longest Group-AFOR frame),
 * so the lengths kept are 8, 12, 16 and 32 tuples; class 3 of the control
 * byte, unused by Group-AFOR, is the 12-tuple frame.  Frames start at
 * multiples of 4 tuples.  Same cost and tie rule as Group-AFOR.            */
size_t or_vse_partition(const uint32_t *qmax, size_t M, int k, uint8_t *Fout)
{
    static const int Fs[4] = {32, 16, 12, 8};
    uint64_t *cost = (uint64_t *)calloc(M + 1, 8);
    uint8_t *choice = (uint8_t *)calloc(M + 1, 1);
    cost[M] = 0;
    for (size_t ii = M; ii-- > 0;) {
        if ((ii % 4) != 0)
            continue;
        uint64_t best = UINT64_MAX;
        int bestF = 0;
        for (int f = 0; f < 4; f++) {
            size_t F = (size_t)Fs[f];
            if (ii + F > M || cost[ii + F] == UINT64_MAX)
                continue;
            uint64_t c = 8 + (uint64_t)k * F * (uint64_t)max_width(qmax, ii, F) + cost[ii + F];
            if (c < best) {
                best = c;
                bestF = (int)F;
            }
        }
        cost[ii] = best;
        choice[ii] = (uint8_t)bestF;
    }
    size_t nf = 0;
    for (size_t i = 0; i < M; i += choice[i])
        Fout[nf++] = choice[i];
    free(cost);
    free(choice);
    return nf;
}

static void afor_encode_frames(const uint32_t *x, size_t M, int k, const uint8_t *F,
                               size_t nf, areas *a)
{
    uint32_t *qmax = (uint32_t *)calloc(M + 1, 4);
    or_tuple_max(x, M, k, qmax);
    bitsink cs = {a->ctrl, a->ctrl_cap, 1, 0, 0, 0};
    uint64_t O = 0;
    size_t t0 = 0;
    for (size_t f = 0; f < nf; f++) {
        int cls = F[f] == 8 ? 0 : F[f] == 16 ? 1 : F[f] == 32 ? 2 : 3;   /* 3: 12 tuples */
        int b = max_width(qmax, t0, F[f]);
        sink_value(&cs, (uint32_t)b, 6);      /* control byte: b:6 | class:2 */
        sink_value(&cs, (uint32_t)cls, 2);
        for (size_t j = 0; j < F[f]; j++)
            for (int c = 0; c < k; c++) {
                bitsink ds = {a->data, a->data_cap, k, c, O + j * (uint64_t)b, 0};
                sink_value(&ds, x[(t0 + j) * (size_t)k + c], b);
                if (ds.err)
                    a->err = 1;
            }
        O += (uint64_t)F[f] * (uint64_t)b;
        t0 += F[f];
    }
    if (t0 != M)
        a->err = 1;
    a->ctrl_bits = cs.pos;
    a->C = round_up(ceil_div((size_t)cs.pos, 32), 4);
    a->D = (size_t)k * ceil_div((size_t)O, 32);
    if (cs.err)
        a->err = 1;
    free(qmax);
}

/* vse: class 3 is a 12-tuple frame (Group-VSEncoding); otherwise corrupt. */
static int afor_decode(const uint32_t *ctrl, size_t C, const uint32_t *data, size_t D,
                       size_t T, int k, int vse, uint32_t *x)
{
    bitsrc cs = {ctrl, C, 1, 0, 0, 0};
    uint64_t O = 0;
    size_t t0 = 0;
    while (t0 < T) {
        uint32_t b = src_value(&cs, 6);
        uint32_t cls = src_value(&cs, 2);
        if (cs.err || (cls == 3 && !vse) || b > 32)
            return OR_ECORRUPT;
        size_t F = cls == 3 ? 12 : (size_t)8 << cls;
        for (size_t j = 0; j < F; j++)
            for (int c = 0; c < k; c++) {
                bitsrc ds = {data, D, k, c, O + j * (uint64_t)b, 0};
                uint32_t v = src_value(&ds, (int)b);
                if (ds.err)
                    return OR_ECORRUPT;
                if (t0 + j < T)
                    x[(t0 + j) * (size_t)k + c] = v;
            }
        O += (uint64_t)F * b;
        t0 += F;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Group-PFD (Section 6.2): blocks of 32 tuples (128 ints at k = 4).        */

/* Step 2: the smallest b with an exception ratio, over the block's quad max
 * entries, strictly below zeta = num/den.                                  */
int or_pfd_width(const uint32_t *qmax, int ntuples, int num, int den)
{
    for (int b = 0; b <= 32; b++) {
        int E = 0;
        for (int t = 0; t < ntuples; t++)
            if (or_bw(qmax[t]) > b)
                E++;
        if ((long)E * den < (long)num * 32)
            return b;
    }
    return 32;
}

static int exc_wcode(int maxbw)
{
    /* Step 4: the most economical of 8, 16, 32 bits */
    if (maxbw <= 8)
        return 1;
    if (maxbw <= 16)
        return 2;
    return 3;
}

static void pfd_encode(const uint32_t *x, size_t T, int k, int num, int den, int mode,
                       areas *a)
{
    size_t nblocks = ceil_div(T, 32);
    size_t BI = (size_t)32 * (size_t)k;          /* ints per block */
    uint32_t *qmax = (uint32_t *)calloc(32, 4);
    uint32_t *slot = (uint32_t *)calloc(BI, 4);
    uint32_t *epos = (uint32_t *)calloc(BI, 4);
    uint32_t *eval = (uint32_t *)calloc(BI, 4);
    uint8_t *isx = (uint8_t *)calloc(BI, 1);
    bitsink cs = {a->ctrl, a->ctrl_cap, 1, 0, 0, 0};
    uint64_t dwords = 0;                          /* per-component words so far */
    size_t ew = 0;                                /* exception words so far     */
    for (size_t blk = 0; blk < nblocks; blk++) {
        const uint32_t *xb = x + blk * BI;       /* T is padded to whole blocks */
        /* Step 1: quad max array of the block */
        or_tuple_max(xb, 32, k, qmax);
        /* Step 2: bit width */
        int b = or_pfd_width(qmax, 32, num, den);
        /* Step 3: exceptional integers inside exceptional tuples */
        memset(isx, 0, BI);
        int maxbw = 0;
        size_t nX = 0;
        for (int t = 0; t < 32; t++) {
            if (or_bw(qmax[t]) <= b)
                continue;
            for (int c = 0; c < k; c++) {
                size_t p = (size_t)t * (size_t)k + (size_t)c;
                int w = or_bw(xb[p]);
                if (w > b) {
                    isx[p] = 1;
                    nX++;
                    if (w > maxbw)
                        maxbw = w;
                }
            }
        }
        int wcode = nX ? exc_wcode(maxbw) : 0;
        int w = wcode ? (4 << wcode) : 0;         /* 8, 16, 32 */
        size_t nexc = 0;
        uint32_t first = 0, nt = 0;
        for (size_t p = 0; p < BI; p++)
            slot[p] = xb[p];
        if (mode == OR_PFD_LINKED) {
            /* exception positions in order, with compulsory exceptions where a
             * gap does not fit in the b-bit slot of the previous exception */
            uint64_t lim = (b >= 32) ? UINT64_MAX : (((uint64_t)1 << b) - 1);
            long prev = -1;
            for (size_t p = 0; p < BI; p++) {
                if (!isx[p])
                    continue;
                if (prev >= 0) {
                    while ((uint64_t)((long)p - prev - 1) > lim) {
                        long cp = prev + (long)((uint64_t)1 << b);
                        epos[nexc] = (uint32_t)cp;
                        eval[nexc] = xb[cp];
                        nexc++;
                        prev = cp;
                    }
                }
                epos[nexc] = (uint32_t)p;
                eval[nexc] = xb[p];
                nexc++;
                prev = (long)p;
            }
            for (size_t e = 0; e < nexc; e++)
                slot[epos[e]] = (e + 1 < nexc) ? (epos[e + 1] - epos[e] - 1) : 0;
            first = nexc ? epos[0] : 0;
        } else {
            for (size_t p = 0; p < BI; p++)
                if (isx[p]) {
                    epos[nexc] = (uint32_t)p;
                    eval[nexc] = xb[p];
                    nexc++;
                    slot[p] = (b >= 32) ? xb[p] : (xb[p] & (((uint32_t)1 << b) - 1));
                }
            for (int t = 0; t < 32; t++) {
                int any = 0;
                for (int c = 0; c < k; c++)
                    any |= isx[(size_t)t * (size_t)k + (size_t)c];
                nt += (uint32_t)any;
            }
            first = nt;
        }
        /* descriptor: b:6 | wcode:2 | first (linked) or tuples (bitmap):12 | nexc:12 */
        sink_value(&cs, (uint32_t)b, 6);
        sink_value(&cs, (uint32_t)wcode, 2);
        sink_value(&cs, first, 12);
        sink_value(&cs, (uint32_t)nexc, 12);
        /* Step 4: normal array in the vertical layout, b words per component */
        for (int t = 0; t < 32; t++)
            for (int c = 0; c < k; c++) {
                bitsink ds = {a->data, a->data_cap, k, c, dwords * 32 + (uint64_t)t * (uint64_t)b, 0};
                sink_value(&ds, slot[(size_t)t * (size_t)k + (size_t)c], b);
                if (ds.err)
                    a->err = 1;
            }
        dwords += (uint64_t)b;
        /* exception area of the block, padded to 32 bits */
        if (nexc) {
            bitsink es = {a->exc + ew, a->exc_cap - ew, 1, 0, 0, 0};
            if (mode == OR_PFD_BITMAP) {
                for (int t = 0; t < 32; t++) {
                    int any = 0;
                    for (int c = 0; c < k; c++)
                        any |= isx[(size_t)t * (size_t)k + (size_t)c];
                    sink_bit(&es, any);
                }
                for (int t = 0; t < 32; t++) {
                    int any = 0;
                    for (int c = 0; c < k; c++)
                        any |= isx[(size_t)t * (size_t)k + (size_t)c];
                    if (any)
                        for (int c = 0; c < k; c++)
                            sink_bit(&es, isx[(size_t)t * (size_t)k + (size_t)c]);
                }
                es.pos = round_up((size_t)es.pos, 32);
            }
            for (size_t e = 0; e < nexc; e++)
                sink_value(&es, eval[e], w);
            if (es.err)
                a->err = 1;
            ew += ceil_div((size_t)es.pos, 32);
        }
    }
    a->ctrl_bits = cs.pos;
    a->C = round_up(ceil_div((size_t)cs.pos, 32), 4);
    a->D = (size_t)k * (size_t)dwords;
    a->E = ew;
    if (cs.err)
        a->err = 1;
    free(qmax);
    free(slot);
    free(epos);
    free(eval);
    free(isx);
}

static int pfd_decode(const uint32_t *ctrl, size_t C, const uint32_t *data, size_t D,
                      const uint32_t *exc, size_t Emax, size_t T, int k, int mode,
                      uint32_t *x)
{
    size_t nblocks = ceil_div(T, 32);
    size_t BI = (size_t)32 * (size_t)k;
    if (nblocks > C)
        return OR_ECORRUPT;
    uint32_t *slot = (uint32_t *)calloc(BI, 4);
    uint64_t dwords = 0;
    size_t ew = 0;
    int rc = OR_OK;
    bitsrc cs = {ctrl, C, 1, 0, 0, 0};
    for (size_t blk = 0; blk < nblocks && rc == OR_OK; blk++) {
        /* Step 1: bit width and first exception offset of the block */
        uint32_t b = src_value(&cs, 6);
        uint32_t wcode = src_value(&cs, 2);
        uint32_t first = src_value(&cs, 12);
        uint32_t nexc = src_value(&cs, 12);
        uint32_t w = wcode ? (4u << wcode) : 0;
        if (b > 32 || nexc > BI || (nexc && !wcode)) {
            rc = OR_ECORRUPT;
            break;
        }
        /* Step 2: the normal array */
        for (int t = 0; t < 32; t++)
            for (int c = 0; c < k; c++) {
                bitsrc ds = {data, D, k, c, dwords * 32 + (uint64_t)t * b, 0};
                slot[(size_t)t * (size_t)k + (size_t)c] = src_value(&ds, (int)b);
                if (ds.err)
                    rc = OR_ECORRUPT;
            }
        dwords += b;
        uint32_t *xb = x + blk * BI;
        for (size_t p = 0; p < BI; p++)
            xb[p] = slot[p];
        if (nexc == 0 || rc != OR_OK)
            continue;
        /* Step 3: exceptions replace the normal values at their positions */
        bitsrc es = {exc + ew, Emax > ew ? Emax - ew : 0, 1, 0, 0, 0};
        if (mode == OR_PFD_LINKED) {
            uint32_t p = first;
            for (uint32_t e = 0; e < nexc; e++) {
                if (p >= BI) {
                    rc = OR_ECORRUPT;
                    break;
                }
                uint32_t nxt = p + slot[p] + 1;
                xb[p] = src_value(&es, (int)w);
                p = nxt;
            }
        } else {
            uint32_t tmask = src_value(&es, 32);
            uint32_t nt = 0;
            for (int t = 0; t < 32; t++)
                nt += (tmask >> t) & 1u;
            if (nt != first) {
                rc = OR_ECORRUPT;
                break;
            }
            uint32_t *cm = (uint32_t *)calloc(32 * (size_t)k, 4);
            for (int t = 0; t < 32; t++)
                if ((tmask >> t) & 1u)
                    for (int c = 0; c < k; c++)
                        cm[(size_t)t * (size_t)k + (size_t)c] = (uint32_t)src_bit(&es);
            es.pos = round_up((size_t)es.pos, 32);
            uint32_t seen = 0;
            for (size_t p = 0; p < BI; p++)
                if (cm[p]) {
                    if (seen < nexc)
                        xb[p] = src_value(&es, (int)w);
                    seen++;
                }
            free(cm);
            if (seen != nexc)
                rc = OR_ECORRUPT;
        }
        if (es.err)
            rc = OR_ECORRUPT;
        ew += ceil_div((size_t)es.pos, 32);
    }
    free(slot);
    if (cs.err)
        rc = OR_ECORRUPT;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Whole-list encode / decode.                                              */

static long assemble(const or_params *p, size_t n, areas *a, uint32_t *out, size_t cap)
{
    size_t E4 = round_up(a->E, 4);
    size_t total = 4 + a->C + a->D + E4;
    if (a->err)
        return OR_EINVAL;
    if (total > cap)
        return OR_ENOSPC;
    memset(out, 0, total * 4);
    out[0] = header_word0(p);
    out[1] = (uint32_t)n;
    out[2] = (uint32_t)a->C;
    out[3] = (uint32_t)a->D;
    memcpy(out + 4, a->ctrl, a->C * 4);
    memcpy(out + 4 + a->C, a->data, a->D * 4);
    memcpy(out + 4 + a->C + a->D, a->exc, a->E * 4);
    return (long)total;
}

/* Shared front half of every encoder: d-gaps and zero padding to whole
 * codec units (k ints for Group-Simple/Scheme, 8 tuples for AFOR, 32 tuples
 * for PFD).  Returns the padded tuple array (caller frees).               */
static uint32_t *prepare(const uint32_t *in, size_t n, const or_params *p, size_t *T_out,
                         size_t *Tpad_out)
{
    size_t T = ceil_div(n, (size_t)p->k);
    size_t unit = p->codec == OR_AFOR || p->codec == OR_VSE ? 8 : p->codec == OR_PFD ? 32 : 1;
    size_t Tp = round_up(T, unit);
    uint32_t *x = (uint32_t *)calloc(Tp * (size_t)p->k + 1, 4);
    if (!x)
        return NULL;
    if (p->delta)
        or_dgap(in, n, x);
    else
        memcpy(x, in, n * 4);
    *T_out = T;
    *Tpad_out = Tp;
    return x;
}

long or_encode(const uint32_t *in, size_t n, const or_params *p, uint32_t *out, size_t cap)
{
    if (!params_ok(p) || n > 0xFFFFFFFFu)
        return OR_EINVAL;
    size_t T, Tp;
    uint32_t *x = prepare(in, n, p, &T, &Tp);
    if (!x)
        return OR_ENOMEM;
    areas a;
    if (!areas_alloc(&a, Tp, p->k)) {
        free(x);
        areas_free(&a);
        return OR_ENOMEM;
    }
    if (p->codec == OR_SIMPLE) {
        gsim_encode(x, T, p->k, &a, NULL, 0);
    } else if (p->codec == OR_SCHEME) {
        gsc_encode(x, T, p->k, p->cg, p->ld, &a);
    } else if (p->codec == OR_AFOR || p->codec == OR_VSE) {
        uint32_t *qmax = (uint32_t *)calloc(Tp + 1, 4);
        uint8_t *F = (uint8_t *)calloc(Tp / 8 + 1, 1);
        or_tuple_max(x, Tp, p->k, qmax);
        size_t nf = p->codec == OR_AFOR ? or_afor_partition(qmax, Tp, p->k, F)
                                        : or_vse_partition(qmax, Tp, p->k, F);
        afor_encode_frames(x, Tp, p->k, F, nf, &a);
        free(qmax);
        free(F);
    } else {
        pfd_encode(x, Tp, p->k, p->zeta_num, p->zeta_den, p->pfd_pos, &a);
    }
    long r = assemble(p, n, &a, out, cap);
    areas_free(&a);
    free(x);
    return r;
}

/* Group-Simple with a caller-chosen selector sequence (for hand-built
 * streams); fails with OR_EINVAL if a selector does not fit its tuples.   */
long or_gsim_encode_with(const uint32_t *in, size_t n, const or_params *p, const uint8_t *sel,
                         size_t S, uint32_t *out, size_t cap)
{
    if (!params_ok(p) || p->codec != OR_SIMPLE)
        return OR_EINVAL;
    for (size_t s = 0; s < S; s++)
        if (sel[s] > 9)
            return OR_EINVAL;
    size_t T, Tp;
    uint32_t *x = prepare(in, n, p, &T, &Tp);
    areas a;
    areas_alloc(&a, Tp + S, p->k);
    gsim_encode(x, T, p->k, &a, sel, S);
    /* every selector but the last must be full */
    size_t t0 = 0;
    for (size_t s = 0; s < S; s++) {
        size_t num = (size_t)GSIM_NUM[sel[s]];
        if (s + 1 < S && t0 + num > T)
            a.err = 1;
        t0 += num;
    }
    long r = assemble(p, n, &a, out, cap);
    areas_free(&a);
    free(x);
    return r;
}

/* Group-AFOR (or Group-VSEncoding) with a caller-chosen partition (frame
 * sizes in tuples; 12 only for Group-VSEncoding). */
long or_afor_encode_with(const uint32_t *in, size_t n, const or_params *p, const uint8_t *F,
                         size_t nf, uint32_t *out, size_t cap)
{
    if (!params_ok(p) || (p->codec != OR_AFOR && p->codec != OR_VSE))
        return OR_EINVAL;
    size_t T, Tp;
    uint32_t *x = prepare(in, n, p, &T, &Tp);
    areas a;
    areas_alloc(&a, Tp + 64, p->k);
    for (size_t f = 0; f < nf; f++)
        if (F[f] != 8 && F[f] != 16 && F[f] != 32 && !(F[f] == 12 && p->codec == OR_VSE))
            a.err = 1;
    afor_encode_frames(x, Tp, p->k, F, nf, &a);
    long r = assemble(p, n, &a, out, cap);
    areas_free(&a);
    free(x);
    return r;
}

long or_decode(const uint32_t *s, size_t words, uint32_t *out, size_t cap)
{
    or_params p;
    if (words < 4)
        return OR_ECORRUPT;
    if (!or_parse_header(s[0], &p))
        return OR_ECORRUPT;
    size_t n = s[1], C = s[2], D = s[3];
    if (C % 4 != 0 || D % (size_t)p.k != 0 || 4 + C + D > words)
        return OR_ECORRUPT;
    if (n > cap)
        return OR_ENOSPC;
    size_t T = ceil_div(n, (size_t)p.k);
    size_t unit = p.codec == OR_AFOR || p.codec == OR_VSE ? 8 : p.codec == OR_PFD ? 32 : 1;
    size_t Tp = round_up(T, unit);
    uint32_t *x = (uint32_t *)calloc(Tp * (size_t)p.k + 1, 4);
    if (!x)
        return OR_ENOMEM;
    const uint32_t *ctrl = s + 4, *data = s + 4 + C, *exc = s + 4 + C + D;
    size_t Emax = words - 4 - C - D;
    int rc;
    switch (p.codec) {
    case OR_SIMPLE: rc = gsim_decode(ctrl, C, data, D, T, p.k, x); break;
    case OR_SCHEME: rc = gsc_decode(ctrl, C, data, D, T, p.k, p.cg, p.ld, x); break;
    case OR_AFOR: rc = afor_decode(ctrl, C, data, D, T, p.k, 0, x); break;
    case OR_VSE: rc = afor_decode(ctrl, C, data, D, T, p.k, 1, x); break;
    default: rc = pfd_decode(ctrl, C, data, D, exc, Emax, Tp, p.k, p.pfd_pos, x); break;
    }
    if (rc == OR_OK) {
        if (p.delta)
            or_prefix_sum(x, n, out);
        else
            memcpy(out, x, n * 4);
    }
    free(x);
    return rc == OR_OK ? (long)n : rc;
}

/* ------------------------------------------------------------------------ */
/* Per-block container for the learned selector (not part of the paper):
 * every block of OR_BLOCK_INTS integers (32 tuples at k = 4) is coded on its
 * own with one of OR_NCLASS codec/parameter classes, by the rules above.
 * Container: header {version | codec 4 << 8 | log2k << 12, n, blocks,
 * payload words}, then one word per block -- class:5 | control words:9 |
 * data words:9 | exception words:9 -- then the block payloads back to back
 * (each: its control words unpadded, its data words, its exception words).
 * A block's size is 1 + its three word counts; the exhaustive choice is the
 * class of least size, the smaller class on ties.                          */

#define OR_BLOCK_INTS 128
#define OR_NCLASS 16
#define OR_CODEC_BLOCKMIX 4

static const int BLOCK_CLASS[OR_NCLASS][5] = {
    /* codec, cg, ld, zeta num, zeta den */
    {OR_SIMPLE, 1, 0, 1, 10},
    {OR_SCHEME, 1, OR_LD_BINARY, 1, 10}, {OR_SCHEME, 2, OR_LD_BINARY, 1, 10},
    {OR_SCHEME, 4, OR_LD_BINARY, 1, 10}, {OR_SCHEME, 8, OR_LD_BINARY, 1, 10},
    {OR_SCHEME, 1, OR_LD_CU, 1, 10}, {OR_SCHEME, 2, OR_LD_CU, 1, 10},
    {OR_SCHEME, 4, OR_LD_CU, 1, 10}, {OR_SCHEME, 8, OR_LD_CU, 1, 10},
    {OR_SCHEME, 4, OR_LD_IU, 1, 10}, {OR_SCHEME, 8, OR_LD_IU, 1, 10},
    {OR_AFOR, 1, 0, 1, 10},
    {OR_PFD, 1, 0, 1, 64}, {OR_PFD, 1, 0, 1, 10}, {OR_PFD, 1, 0, 2, 10}, {OR_PFD, 1, 0, 3, 10},
};

int or_block_class_params(int kappa, or_params *p)
{
    if (kappa < 0 || kappa >= OR_NCLASS)
        return 0;
    memset(p, 0, sizeof(*p));
    p->codec = BLOCK_CLASS[kappa][0];
    p->k = 4;
    p->cg = BLOCK_CLASS[kappa][1];
    p->ld = BLOCK_CLASS[kappa][2];
    p->delta = 0;
    p->pfd_pos = OR_PFD_LINKED;
    p->zeta_num = BLOCK_CLASS[kappa][3];
    p->zeta_den = BLOCK_CLASS[kappa][4];
    return 1;
}

/* Codes one block into its areas (32 tuples; no codec needs padding). */
static int block_areas(const uint32_t *x, int kappa, areas *a)
{
    or_params p;
    if (!or_block_class_params(kappa, &p))
        return 0;
    const size_t T = OR_BLOCK_INTS / 4;
    if (!areas_alloc(a, T, 4)) {
        areas_free(a);
        return 0;
    }
    if (p.codec == OR_SIMPLE) {
        gsim_encode(x, T, 4, a, NULL, 0);
    } else if (p.codec == OR_SCHEME) {
        gsc_encode(x, T, 4, p.cg, p.ld, a);
    } else if (p.codec == OR_AFOR) {
        uint32_t qmax[32];
        uint8_t F[4];
        or_tuple_max(x, T, 4, qmax);
        size_t nf = or_afor_partition(qmax, T, 4, F);
        afor_encode_frames(x, T, 4, F, nf, a);
    } else {
        pfd_encode(x, T, 4, p.zeta_num, p.zeta_den, p.pfd_pos, a);
    }
    if (a->err) {
        areas_free(a);
        return 0;
    }
    return 1;
}

/* Block word and payload of one block; returns the payload words written
 * (0 on error). */
long or_block_encode(const uint32_t *x, int kappa, uint32_t *payload, size_t cap, uint32_t *blockword)
{
    areas a;
    if (!block_areas(x, kappa, &a))
        return 0;
    size_t Cw = ceil_div((size_t)a.ctrl_bits, 32), Dw = a.D, Ew = a.E;
    long r = 0;
    if (Cw < 512 && Dw < 512 && Ew < 512 && Cw + Dw + Ew <= cap) {
        memcpy(payload, a.ctrl, Cw * 4);
        memcpy(payload + Cw, a.data, Dw * 4);
        memcpy(payload + Cw + Dw, a.exc, Ew * 4);
        *blockword = (uint32_t)kappa | (uint32_t)(Cw << 5) | (uint32_t)(Dw << 14) | (uint32_t)(Ew << 23);
        r = (long)(Cw + Dw + Ew);
    }
    areas_free(&a);
    return r;
}

/* Size of one block coded with class kappa, in words (block word included). */
long or_block_size(const uint32_t *x, int kappa)
{
    uint32_t buf[4 * OR_BLOCK_INTS + 64], bw;
    long w = or_block_encode(x, kappa, buf, sizeof(buf) / 4, &bw);
    return w > 0 ? 1 + w : OR_EINVAL;
}

/* Exhaustive selection: sizes of every class, the least one (smaller class
 * on ties). */
int or_block_best(const uint32_t *x, long *sizes)
{
    int best = -1;
    for (int kappa = 0; kappa < OR_NCLASS; kappa++) {
        sizes[kappa] = or_block_size(x, kappa);
        if (sizes[kappa] > 0 && (best < 0 || sizes[kappa] < sizes[best]))
            best = kappa;
    }
    return best;
}

/* Decodes one block payload by rebuilding the equivalent whole stream. */
int or_block_decode(uint32_t blockword, const uint32_t *payload, size_t words, uint32_t *x)
{
    int kappa = (int)(blockword & 31u);
    size_t Cw = (blockword >> 5) & 511u, Dw = (blockword >> 14) & 511u, Ew = (blockword >> 23) & 511u;
    or_params p;
    if (!or_block_class_params(kappa, &p) || Cw + Dw + Ew > words)
        return OR_ECORRUPT;
    size_t C = round_up(Cw, 4);
    size_t total = 4 + C + Dw + round_up(Ew, 4);
    uint32_t *s = (uint32_t *)calloc(total, 4);
    if (!s)
        return OR_ENOMEM;
    s[0] = header_word0(&p);
    s[1] = OR_BLOCK_INTS;
    s[2] = (uint32_t)C;
    s[3] = (uint32_t)Dw;
    memcpy(s + 4, payload, Cw * 4);
    /* padding control words read as 1 bits (unary codes end before them) */
    for (size_t i = Cw; i < C; i++)
        s[4 + i] = 0xFFFFFFFFu;
    memcpy(s + 4 + C, payload + Cw, Dw * 4);
    memcpy(s + 4 + C + Dw, payload + Cw + Dw, Ew * 4);
    long r = or_decode(s, total, x, OR_BLOCK_INTS);
    free(s);
    return r == OR_BLOCK_INTS ? OR_OK : OR_ECORRUPT;
}

/* The 40 block features (a reading of the selector's inputs): the maximum
 * bit width / 32; the histogram of the 32 tuple widths (a tuple's width is
 * its widest integer's), bins 0..32, each count / 32; the number of integers
 * wider than maxW - t, t = 1..6, / 128 (all of them when maxW - t < 0). */
void or_block_features(const uint32_t *x, double *f)
{
    /* the width of a tuple is the width of its widest integer (the width
     * every codec of the 4-way layout sizes a tuple by) */
    int hist[33] = {0}, maxw = 0;
    for (int t = 0; t < OR_BLOCK_INTS / 4; t++) {
        int w = 0;
        for (int c = 0; c < 4; c++)
            if (or_bw(x[4 * t + c]) > w)
                w = or_bw(x[4 * t + c]);
        hist[w]++;
        if (w > maxw)
            maxw = w;
    }
    f[0] = maxw / 32.0;
    for (int w = 0; w <= 32; w++)
        f[1 + w] = hist[w] / (double)(OR_BLOCK_INTS / 4);
    for (int t = 1; t <= 6; t++) {
        int b = maxw - t, cnt = 0;
        for (int i = 0; i < OR_BLOCK_INTS; i++)
            if (b < 0 || or_bw(x[i]) > b)
                cnt++;
        f[33 + t] = cnt / (double)OR_BLOCK_INTS;
    }
}

/* Codes n integers (zero-padded to whole blocks) block by block with the
 * given classes, or the exhaustive choice when kappas is NULL; the classes
 * used are written to kappa_out when it is not NULL.  Returns the words
 * written. */
long or_blockmix_encode(const uint32_t *in, size_t n, const uint8_t *kappas, uint32_t *out, size_t cap,
                        uint8_t *kappa_out)
{
    size_t nb = ceil_div(n, OR_BLOCK_INTS);
    if (n > 0xFFFFFFFFu || cap < 4 + nb)
        return cap < 4 + nb ? OR_ENOSPC : OR_EINVAL;
    size_t pos = 4 + nb;
    uint32_t x[OR_BLOCK_INTS];
    for (size_t b = 0; b < nb; b++) {
        size_t m = n - b * OR_BLOCK_INTS < OR_BLOCK_INTS ? n - b * OR_BLOCK_INTS : OR_BLOCK_INTS;
        memset(x, 0, sizeof(x));
        memcpy(x, in + b * OR_BLOCK_INTS, m * 4);
        int kappa;
        if (kappas) {
            kappa = kappas[b];
        } else {
            long sizes[OR_NCLASS];
            kappa = or_block_best(x, sizes);
        }
        if (kappa_out)
            kappa_out[b] = (uint8_t)kappa;
        uint32_t bw;
        long w = or_block_encode(x, kappa, out + pos, cap - pos, &bw);
        if (w <= 0)
            return cap - pos < 4 * OR_BLOCK_INTS + 64 ? OR_ENOSPC : OR_EINVAL;
        out[4 + b] = bw;
        pos += (size_t)w;
    }
    out[0] = (uint32_t)OR_VERSION | ((uint32_t)OR_CODEC_BLOCKMIX << 8) | (2u << 12);
    out[1] = (uint32_t)n;
    out[2] = (uint32_t)nb;
    out[3] = (uint32_t)(pos - 4 - nb);
    return (long)pos;
}

long or_blockmix_decode(const uint32_t *s, size_t words, uint32_t *out, size_t cap)
{
    if (words < 4 || s[0] != ((uint32_t)OR_VERSION | ((uint32_t)OR_CODEC_BLOCKMIX << 8) | (2u << 12)))
        return OR_ECORRUPT;
    size_t n = s[1], nb = s[2], pw = s[3];
    if (nb != ceil_div(n, OR_BLOCK_INTS) || 4 + nb + pw > words)
        return OR_ECORRUPT;
    if (n > cap)
        return OR_ENOSPC;
    size_t pos = 4 + nb, end = 4 + nb + pw;
    uint32_t x[OR_BLOCK_INTS];
    for (size_t b = 0; b < nb; b++) {
        uint32_t bw = s[4 + b];
        size_t len = ((bw >> 5) & 511u) + ((bw >> 14) & 511u) + ((bw >> 23) & 511u);
        if (pos + len > end || or_block_decode(bw, s + pos, len, x) != OR_OK)
            return OR_ECORRUPT;
        size_t m = n - b * OR_BLOCK_INTS < OR_BLOCK_INTS ? n - b * OR_BLOCK_INTS : OR_BLOCK_INTS;
        memcpy(out + b * OR_BLOCK_INTS, x, m * 4);
        pos += len;
    }
    return pos == end ? (long)n : OR_ECORRUPT;
}
