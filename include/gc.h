/*
 * gc.h -- C ABI of libgc: decoding of Group-codec posting lists on AMD
 * Instinct MI355X (gfx950).
 *
 * The codecs are those of Zhao et al., "A General SIMD-based Approach to
 * Accelerating Compression Algorithms" (arXiv 1502.01916): Group-Simple
 * (Section 4), Group-Scheme (Section 5), Group-AFOR (Section 6.1),
 * Group-PFD (Section 6.2) and a Group-VSEncoding (named in Section 6.1 without
 * a format; see GC_VSE), each storing its control patterns apart from the
 * packed data, which uses the k-way vertical layout (Section 3.1; the paper's
 * k is 4, wider k is a GPU-native option).  Decoding is followed by the
 * d-gap prefix sum that restores docIDs (Section 2.1.1).
 *
 * Conventions for every entry point:
 *   - Returns gc_status: GC_OK (0) or a negative error.  Never throws, never
 *     aborts, never prints.
 *   - The caller owns every buffer passed in, host or device; the library
 *     never frees or retains them past the call (a plan keeps the device
 *     pointers it captured until it is destroyed or re-executed with others).
 *   - "d_" pointers are device (HIP) pointers, "h_" pointers host pointers.
 *   - Decode calls are asynchronous on the given HIP stream (NULL = the null
 *     stream).  Stream corruption found on the device is not returned by the
 *     call; it is latched in the context and reported by gc_sync_status.
 *   - On any error the contents of the output range are unspecified, but the
 *     library never writes outside it.
 *
 * Stream format (little-endian uint32 words, self-describing):
 *   word 0  version:8 (=1) | codec:4 | log2(k):3 | log2(CG):2 | LD:2 |
 *           delta:1 | pfd_pos:1 | reserved:11 (zero)
 *   word 1  n, the number of integers
 *   word 2  C, control-area words (multiple of 4)
 *   word 3  D, data-area words (multiple of k)
 *   then the control area, the data area (word w of component c at k*w + c;
 *   each component an LSB-first bitstream, straddling values low part first)
 *   and, for Group-PFD, the exception area; total length a multiple of 4.
 */
#ifndef GC_H
#define GC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GC_OK = 0,
    GC_EINVAL = -1,       /* bad argument or unsupported parameter combination */
    GC_ENOSPC = -2,       /* output capacity too small                           */
    GC_ECORRUPT = -3,     /* malformed stream (host check or latched by device)  */
    GC_EDEVICE = -4,      /* a HIP runtime call failed                           */
    GC_EUNSUPPORTED = -5, /* valid stream the GPU path does not handle           */
    GC_ENOMEM = -6        /* host or device allocation failed                    */
} gc_status;

/* Codec identifiers (header word 0 bits 8..11). */
typedef enum {
    GC_SIMPLE = 0,  /* Group-Simple: 4-bit selectors of Table III, one vector each   */
    GC_SCHEME = 1,  /* Group-Scheme CG-LD: eq. (1)-(2), unary or binary descriptors   */
    GC_AFOR = 2,    /* Group-AFOR: frames of 8/16/32 tuples, DP partition            */
    GC_PFD = 3,     /* Group-PFD: 32-tuple blocks, exceptions in a separate area      */
    GC_VSE = 4      /* Group-VSEncoding (Section 6.1 names it; Section 2.2 gives
                     * VSEncoding's frame lengths): Group-AFOR's stream with frames
                     * of 8/12/16/32 tuples (class 3 = 12), DP partition.  Host
                     * encoder and GPU decoders only: gc_encode_lists_gpu returns
                     * GC_EINVAL for it.                                          */
} gc_codec;

/* Group-Scheme length descriptor (Section 5.2.1). */
enum { GC_LD_BINARY = 0, GC_LD_CU = 1, GC_LD_IU = 2 };
/* Group-PFD exception positions: a linked chain through the normal slots
 * (the paper's "first exception offset", Section 6.2) or a per-block bitmap. */
enum { GC_PFD_LINKED = 0, GC_PFD_BITMAP = 1 };

/* gc_params.flags */
#define GC_DELTA 1u   /* input is a docID list: code its d-gaps; decode prefix-sums */

typedef struct {
    uint32_t k;          /* layout width: 4 (the paper's) .. 64, a power of two      */
    uint8_t cg;          /* Group-Scheme compression granularity 1, 2, 4, 8 (Sec 5.1) */
    uint8_t ld;          /* Group-Scheme length descriptor GC_LD_*                    */
    uint8_t pfd_pos;     /* Group-PFD GC_PFD_LINKED or GC_PFD_BITMAP                  */
    uint8_t reserved;    /* zero                                                      */
    uint16_t zeta_num;   /* Group-PFD exception-ratio threshold zeta = num/den,       */
    uint16_t zeta_den;   /*   0 < zeta < 1 (Section 6.2, step 2); 1/10 in the paper   */
    uint32_t flags;      /* GC_DELTA                                                  */
} gc_params;

/* ---- host-side encoding (index build) --------------------------------- */

/* Upper bound, in words, of the stream gc_encode writes for n integers. */
size_t gc_encoded_bound_words(size_t n, gc_codec codec, const gc_params *p);

/* Encodes h_in[0..n) (host memory) into one stream at h_out (host memory,
 * capacity out_cap_words).  Group-Simple selection follows Algorithm 1
 * (Section 4.2), Group-AFOR the optimal DP partition (Section 6.1), Group-PFD
 * encoding steps 1-4 (Section 6.2).  *out_words receives the stream length.
 * GC_EINVAL for bad parameters, GC_ENOSPC if the capacity is too small.     */
gc_status gc_encode(const uint32_t *h_in, size_t n, gc_codec codec, const gc_params *p,
                    uint32_t *h_out, size_t out_cap_words, size_t *out_words);

/* Sum of gc_encoded_bound_words over the lists of a gc_encode_lists call
 * (same arguments); 0 on bad arguments.                                    */
size_t gc_encoded_bound_words_lists(const uint64_t *in_offs, size_t nlists, const gc_codec *codecs,
                                    const gc_params *params, int one_param);

/* Encodes many lists on all host cores.  List i is h_in[in_offs[i] ..
 * in_offs[i+1]), coded with codecs[i] / params[i] (params may hold a single
 * entry used for all lists when one_param != 0).  Streams are written back to
 * back into h_out; out_offs[i] receives stream i's word offset and
 * out_offs[nlists] the total.  nthreads = 0 uses every core.               */
gc_status gc_encode_lists(const uint32_t *h_in, const uint64_t *in_offs, size_t nlists,
                          const gc_codec *codecs, const gc_params *params, int one_param,
                          uint32_t *h_out, size_t out_cap_words, uint64_t *out_offs,
                          int nthreads);

/* Encodes nlists lists on the GPU, with one codec and parameter set for
 * all: list i is d_in[h_in_offs[i] .. h_in_offs[i+1]) (device memory; at
 * most 2^28 integers).  Writes exactly the streams gc_encode_lists writes
 * for the same lists (Algorithm 1 for Group-Simple, Section 4.2; eq. (1)-(2)
 * and the length descriptors of Section 5.2.1 for Group-Scheme; the optimal
 * frame partition of Section 6.1 for Group-AFOR; encoding steps 1-4 of
 * Section 6.2 for Group-PFD), back to back into d_out (device memory,
 * capacity out_cap_words); h_out_offs[i] (host memory, nlists + 1 entries)
 * receives stream i's word offset and h_out_offs[nlists] the total.
 * Index build, not the decode path: it reads the stream sizes back to the
 * host and returns once the streams are written (it synchronises
 * hip_stream).  Its device scratch (about 12 bytes per integer at most) and
 * pinned host staging are kept per device, for later calls, until the
 * process ends, and grow when a call needs more; calls on one device run
 * one at a time.  GC_EINVAL for bad parameters or GC_VSE (whose streams
 * come from gc_encode_lists), GC_ENOSPC if the streams do not fit (h_out_offs then holds their sizes), GC_ENOMEM if the scratch
 * does not fit.                                                            */
gc_status gc_encode_lists_gpu(const uint32_t *d_in, const uint64_t *h_in_offs, size_t nlists,
                              gc_codec codec, const gc_params *p, uint32_t *d_out,
                              size_t out_cap_words, uint64_t *h_out_offs, void *hip_stream);

/* ---- device context ---------------------------------------------------- */

typedef struct gc_ctx gc_ctx;     /* opaque, library-owned */
typedef struct gc_plan gc_plan;   /* opaque, library-owned */

/* Context options (zero-initialise for defaults). */
typedef struct {
    uint64_t max_list_ints;  /* longest list gc_decode decodes and gc_blockmix_encode /
                                gc_encode_blocks encode (at most 2^32 - 1); their
                                device tables are sized for it here; 0 = 2^24  */
    uint32_t reserved[2];    /* zero */
} gc_ctx_opts;

/* Creates a context on HIP device `device` (made current for the call).
 * Allocates the device status word and the tables of single-list decoding
 * and block encoding, sized for opts->max_list_ints (about 45 bytes per
 * 1024 integers for decoding, 170 bytes per 128 for block encoding; about
 * 24 MB at the default 2^24) -- the only allocations a context makes.
 * gc_ctx_create(device, ctx) is gc_ctx_create_opts(device, NULL, ctx).
 * GC_EINVAL for nonzero reserved words or a maximum above 2^32 - 1,
 * GC_ENOMEM if the tables do not fit, GC_EUNSUPPORTED on a device other
 * than gfx950.                                                             */
gc_status gc_ctx_create(int device, gc_ctx **ctx);
gc_status gc_ctx_create_opts(int device, const gc_ctx_opts *opts, gc_ctx **ctx);
gc_status gc_ctx_destroy(gc_ctx *ctx);

/* Decodes one stream (device memory, stream_words words) into d_out[0..n),
 * prefix-summing when the header's delta bit is set.  h_header is a host
 * copy of the stream's first 4 words (the index dictionary keeps each list's
 * length and codec, Section 2.1.1, so no device-to-host read is needed); n is
 * h_header[1].  The kernels re-check the device copy against it.
 * Asynchronous on hip_stream: it launches kernels only (the locate pass,
 * for a list of several tiles, and the decode pass, with a tile-sum pass and
 * carry scan for a long delta list); it allocates nothing and never
 * synchronises, so it may be captured in a hipGraph and replayed.  Calls on
 * one context must not overlap in time (they share its tables); use one
 * context per concurrent stream.  d_stream must be 16-byte aligned.
 * GC_ECORRUPT if h_header is malformed, GC_ENOSPC if the list is longer
 * than the context's max_list_ints (or its control area larger than such a
 * list's can be).                                                          */
gc_status gc_decode(gc_ctx *ctx, const uint32_t *d_stream, size_t stream_words,
                    const uint32_t *h_header, uint32_t *d_out, void *hip_stream);

/* gc_decode for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, output and errors as gc_decode, and the same kernels, but
 * the single-list tables (locate epochs, tile starts, tile carries,
 * look-back flags, locate chunk aggregates) live in one fixed device array
 * of about 434 KB that the library holds on each GPU it runs on until the
 * process ends; the array is found and cleared once per device when the
 * first context on it is created.  The call itself allocates nothing,
 * neither here nor in any library it calls, and never synchronises.
 * Lists of up to 2^22 integers (GC_ENOSPC above; a context's max_list_ints
 * does not apply).  Device errors go to ctx's status word (gc_sync_status).
 * Every call on one GPU shares that GPU's array, whatever the context:
 * calls that overlap in time on one GPU race and must be serialised by the
 * caller (one stream, or events between them).                            */
gc_status gc_decode_noalloc(gc_ctx *ctx, const uint32_t *d_stream, size_t stream_words,
                            const uint32_t *h_header, uint32_t *d_out, void *hip_stream);

/* One list of a batch: its stream at d_streams + stream_off_words (16-byte
 * aligned, stream_words long), its output at d_out + out_off (n words).    */
typedef struct {
    uint64_t stream_off_words;
    uint64_t stream_words;
    uint64_t out_off;
    uint32_t n;
    uint32_t reserved;
} gc_list_desc;

/* Plan options (zero-initialise for defaults). */
typedef struct {
    uint32_t tile_ints;      /* integers per wave tile (Group-Simple, -Scheme, -AFOR):
                                1024, 2048 or 4096, raised to 32*k for the widest
                                layout in the batch; 0 = autotuned / default       */
    uint32_t pfd_tile_ints;  /* integers per wave tile of Group-PFD (whole 32-tuple
                                blocks): 1024, 2048 or 4096, raised to 32*k for
                                the widest layout; 0 = autotuned / default      */
    uint32_t use_graph;      /* 1 = capture the launch sequence in a hipGraph       */
    uint32_t autotune;       /* 1 = time candidate tile sizes at creation           */
    uint32_t timing_slots;   /* > 0: time the kernels of each gc_decode_batch with
                                HIP events, in this many rotating slots (see
                                gc_plan_timings); the run is then not graphed  */
    uint32_t schedule;       /* 0: every kernel on the launch stream: one locate
                                pass over every class, then class by class the
                                other passes; 1: per-class locate kernels on a
                                second stream, ahead of the other kernels      */
    uint32_t class_tile_ints[5];  /* per codec class (see GC_CLASSES), nonzero
                                overrides tile_ints / pfd_tile_ints for that
                                class; the autotuner picks one size per class */
    uint32_t carry_pass;     /* how a tile of a delta list of several tiles gets
                                its carry (the sum of the list's d-gaps before
                                it): 1 in the decode pass itself, each tile
                                publishing its sum and reading those before
                                it (decoupled look-back); 2 a tile-sum pass
                                and a carry scan ahead of the decode pass;
                                3 look-back for lists of at most 64 tiles
                                (one window of flags), the tile-sum pass for
                                longer ones; 0 = default (3)                   */
    uint32_t pack_ints;      /* lists of at most this many integers (1 .. 4096)
                                are decoded many to a wave by the pack kernel
                                instead of by the class passes, when their
                                streams fit a pack (2 KB of stream for a
                                threshold up to 2048, else 4 KB); a pack holds
                                up to 32 lists of one stream format (codec,
                                k and codec parameters; docID and TF lists
                                mix); GC_PACK_OFF: none; 0 = autotuned (with
                                autotune) or the default, 2048               */
    uint32_t graph_serial;   /* 1 = a graph runs its kernels in one chain (the
                                pack kernel, the locate pass, then class after
                                class); 0 = branches: the pack kernel beside
                                the rest, and after the locate pass each
                                codec class's passes on a branch of their own
                                (with schedule 0)                            */
    uint32_t pack_groups;    /* workgroups (four waves) of the pack kernel per
                                CU, 1 .. 64: each wave then decodes packs in
                                turn, leaving room on every CU for the other
                                passes; GC_PACK_GROUPS_ALL: one wave per pack;
                                0 = autotuned (with autotune) or the default, 5 */
} gc_plan_opts;
#define GC_PACK_OFF 0x80000000u
#define GC_PACK_GROUPS_ALL 0x80000000u

/* Builds a batched decode plan for nlists lists.  h_headers holds the first
 * 4 words of every stream (4*nlists words, host memory).  The plan holds the
 * tile tables (tile -> list, the per-tile locate entries and carries) and
 * (optionally) an instantiated hipGraph; it allocates everything here, never
 * at execute.  With opts->autotune the plan times candidate tile sizes on the
 * device buffers given (d_streams, d_out) and keeps the fastest; results are
 * cached in a JSON file named by $GC_AUTOTUNE_CACHE when set.  For tests of
 * the look-back's bounded wait only, $GC_TEST_LOOKBACK_STALL = t (ticks of
 * the 100 MHz real-time counter) makes the plan's tiles withhold their
 * flags, so every look-back gives up after t ticks and reports GC_ECORRUPT
 * (detail 12) through gc_sync_status.  GC_EINVAL for
 * a tile size not listed above or nonzero reserved words.                  */
gc_status gc_plan_create(gc_ctx *ctx, const gc_list_desc *h_descs, size_t nlists,
                         const uint32_t *h_headers, const gc_plan_opts *opts,
                         const uint32_t *d_streams, uint32_t *d_out, gc_plan **plan);
gc_status gc_plan_destroy(gc_plan *plan);

/* Decodes every list of the plan: the pack kernels over the packed lists
 * (see opts->pack_ints), the locate pass, then per codec class the
 * tile-sum pass over its delta lists whose tiles take their carries from it
 * (see opts->carry_pass), the carry scan and the decode pass, replayed as one
 * hipGraph when the plan was created with use_graph.                       */
gc_status gc_decode_batch(gc_plan *plan, const uint32_t *d_streams, uint32_t *d_out,
                          void *hip_stream);

/* Decodes every list of the plan with one launch sequence per list (the
 * per-list baseline the batch is compared with).                          */
gc_status gc_decode_each(gc_plan *plan, const uint32_t *d_streams, uint32_t *d_out,
                         void *hip_stream);

/* Kernel durations of the last runs of a plan created with timing_slots > 0.
 * Such a plan launches its kernels directly (no graph), with HIP events
 * around each phase on the stream that runs it (the locate kernels on the
 * plan's second stream when opts->schedule is 1).  This synchronises those
 * events and writes, oldest run first, up to max_runs rows of
 * GC_TIMING_FIELDS floats (milliseconds) to ms:
 *   [0]                         the whole run, on the launch stream
 *   [1 + c]                     the locate kernels of codec class c (with
 *                               schedule 0 the one locate pass, in the column
 *                               of the first class the plan holds; 0 in the
 *                               others)
 *   [1 + GC_CLASSES + c]        its tile-sum pass and carry scan
 *   [1 + 2 * GC_CLASSES + c]    its decode pass
 *   [1 + 3 * GC_CLASSES]        the pack kernels
 * with classes c = 0 Group-Simple, 1 Group-Scheme with unary descriptors,
 * 2 Group-Scheme with binary descriptors, 3 Group-AFOR, 4 Group-PFD (0 for a
 * class the plan does not hold).  With schedule 1 locate kernels overlap the
 * other phases, so the phases need not add up to the whole run.  *nruns receives the rows
 * written.  GC_EINVAL if the plan records no events.                       */
#define GC_CLASSES 5
#define GC_TIMING_FIELDS (2 + 3 * GC_CLASSES)
gc_status gc_plan_timings(gc_plan *plan, uint32_t max_runs, float *ms, uint32_t *nruns);

/* Reports the chosen configuration of a plan: the tile size of its first
 * non-PFD codec class and of Group-PFD, the decode tiles of one run and, of
 * those, the tiles of its tile-sum pass.  Any pointer may be NULL.         */
gc_status gc_plan_config(const gc_plan *plan, uint32_t *tile_ints, uint32_t *pfd_tile_ints,
                         uint64_t *tiles, uint64_t *sum_tiles);

/* The packed-list threshold a plan uses (0: no packing), its packs (waves
 * of the pack kernels), the lists they hold and the pack kernel's
 * workgroups per CU (GC_PACK_GROUPS_ALL: one wave per pack).  Any pointer
 * may be NULL.                                                             */
gc_status gc_plan_pack_config(const gc_plan *plan, uint32_t *pack_ints, uint64_t *packs,
                              uint64_t *packed_lists, uint32_t *pack_groups);

/* Which lists of a plan the pack kernel decodes: h_packed[i] (host memory,
 * nlists bytes) = 1 for a packed list, 0 for one the class passes decode.  */
gc_status gc_plan_packed_lists(const gc_plan *plan, uint8_t *h_packed, size_t nlists);

/* The tile size (integers per wave tile) of every codec class of a plan,
 * GC_CLASSES entries in class order (sizes of classes the plan does not hold
 * are the defaults).                                                        */
gc_status gc_plan_class_tiles(const gc_plan *plan, uint32_t *tile_ints);

/* Synchronises hip_stream, then returns (and clears) the first device-side
 * error latched since the previous call: GC_OK or GC_ECORRUPT.  detail, if
 * not NULL, receives an implementation-specific code of the failed check.  */
gc_status gc_sync_status(gc_ctx *ctx, void *hip_stream, uint32_t *detail);

/* ---- query processing over decoded lists (Section 7.4) ----------------- */

/* Okapi BM25 parameters (the paper cites Robertson et al. and gives no
 * values; k1 = 1.2, b = 0.75 are the usual ones).                          */
typedef struct {
    float k1, b;
    float avgdl;          /* mean document length                                */
    uint32_t topk;        /* documents kept per query, 1 .. 64 (10 in the paper) */
    uint32_t ndocs;       /* N, documents in the collection (idf; doclen size)   */
    uint32_t reserved[2]; /* zero                                                */
} gc_bm25_params;

typedef struct gc_query_plan gc_query_plan;   /* opaque, library-owned */

/* A batch of AND queries over nterms terms: query q has the terms
 * h_query_terms[q*terms_per_query ..] (term indices, -1 = none; at most 8
 * per query); h_term_len[t] is the length of term t's posting list.  The
 * plan cuts every query's shortest list into work items of 8192 postings
 * and allocates their partial results (device memory, here only).
 * GC_EINVAL for a term index out of range or bad parameters.               */
gc_status gc_query_plan_create(const uint32_t *h_term_len, size_t nterms, const int32_t *h_query_terms,
                               uint32_t terms_per_query, uint32_t nq, const gc_bm25_params *p,
                               gc_query_plan **plan);
gc_status gc_query_plan_destroy(gc_query_plan *plan);

/* Runs the plan's queries over decoded lists in device memory: term t's
 * docIDs (ascending) at d_docs + d_term_off[t] and its TFs at the same
 * offset of d_tfs (as gc_decode_batch writes them), document lengths
 * d_doclen[0 .. ndocs).  Every query keeps the documents in all its terms'
 * lists, scores each by BM25 (the sum over its terms of
 * idf * tf * (k1 + 1) / (tf + k1 * (1 - b + b * dl / avgdl)), idf =
 * ln(1 + (N - df + 0.5) / (df + 0.5)), single precision) and writes its
 * topk best to d_top_doc / d_top_score[q*topk ..], higher score first, then
 * smaller docID; unused places get docID 0xFFFFFFFF and score 0.  Lookups
 * go through the lists' block heads every 512 postings (skip pointers,
 * Section 7.4).  Asynchronous on hip_stream; allocates nothing.             */
gc_status gc_query_run(gc_query_plan *plan, const uint32_t *d_docs, const uint32_t *d_tfs,
                       const uint64_t *d_term_off, const uint16_t *d_doclen, uint32_t *d_top_doc,
                       float *d_top_score, void *hip_stream);

/* ---- per-block container of the learned codec selector -----------------
 * Not part of the paper: a container in which every block of
 * GC_BLOCK_INTS integers (32 tuples of the 4-way layout) is coded on its own
 * with one of GC_BLOCK_CLASSES codec classes, each the whole-list rule of
 * its section applied to the block's 32 tuples:
 *   0 Group-Simple (Algorithm 1, Table III)
 *   1..4 Group-Scheme with binary descriptors, CG = 1, 2, 4, 8 (Section 5.2)
 *   5..8 Group-Scheme with complete unary descriptors, CG = 1, 2, 4, 8
 *   9, 10 Group-Scheme with incomplete unary descriptors, CG = 4, 8
 *   11 Group-AFOR (Section 6.1)
 *   12..15 Group-PFD with linked exceptions, zeta = 1/64, 1/10, 2/10, 3/10
 *        (Section 6.2; zeta below 1/32 is BP128, Section 6.3)
 * Layout: header {version 1 | codec 4 << 8 | log2 4 << 12, n, blocks,
 * payload words}; one word per block, class:5 | control words:9 | data
 * words:9 | exception words:9; then the block payloads back to back, each
 * its unpadded control words, its data words and its exception words.  A
 * block's size is 1 + its payload words.  Integers are coded as they are
 * (no d-gaps).                                                              */
#define GC_BLOCK_INTS 128
#define GC_BLOCK_CLASSES 16
#define GC_BLOCK_FEATURES 40

/* Device memory d_in holds nblocks * GC_BLOCK_INTS integers.  Writes the 40
 * features of every block to d_feat (nblocks x 40 floats, row-major): the
 * largest bit width / 32; the count of tuples (4 consecutive integers, the
 * width of the widest) of width 0..32 / 32; the count of integers wider
 * than (largest width - t), t = 1..6, / 128 (all integers when that is
 * negative).  Asynchronous on hip_stream.                                  */
gc_status gc_block_features(gc_ctx *ctx, const uint32_t *d_in, size_t nblocks, float *d_feat,
                            void *hip_stream);

/* The coded size in words (block word included) of every block in every
 * class to d_sizes (nblocks x GC_BLOCK_CLASSES, row-major), the least
 * one's class (the smaller class on ties: the exhaustive choice) to
 * d_best, and every class's relative excess (size - least) / least, in
 * fp32, to d_cost (nblocks x GC_BLOCK_CLASSES).  Any output may be NULL.
 * Asynchronous on hip_stream.                                               */
gc_status gc_block_sizes(gc_ctx *ctx, const uint32_t *d_in, size_t nblocks, uint32_t *d_sizes,
                         uint8_t *d_best, float *d_cost, void *hip_stream);

/* Words a container of n integers can take at most. */
size_t gc_blockmix_bound_words(size_t n);

/* Codes the n integers of d_in (device memory holding ceil(n/128) * 128
 * integers, the tail zero-padded) into a container at d_out, block b in
 * class d_class[b] (device memory, one byte per block).  *out_words
 * receives the container's length.  The sizing, offset and writing kernels
 * run on hip_stream back to back; the call returns once they have finished
 * and the total is read back.  GC_ENOSPC if out_cap_words is too small
 * or n exceeds the context's max_list_ints,
 * GC_EINVAL for a class >= GC_BLOCK_CLASSES or when
 * gc_blockmix_bound_words(n) exceeds 2^32 - 1; nothing is written past
 * out_cap_words, and after an error the contents of d_out are undefined.   */
gc_status gc_blockmix_encode(gc_ctx *ctx, const uint32_t *d_in, size_t n, const uint8_t *d_class,
                             uint32_t *d_out, size_t out_cap_words, size_t *out_words, void *hip_stream);

/* ---- learned codec selector -------------------------------------------------
 * Not part of the paper.  A network maps the 40 features of a block
 * (gc_block_features) to scores of the GC_BLOCK_CLASSES classes:
 * 40 -> 64 -> 64 -> 16, ReLU after the two hidden layers, softmax.  Matrix
 * products take bf16 operands (the weights and activations rounded to
 * nearest even) and accumulate in fp32 on the matrix cores; parameters and
 * Adam moments are fp32.  Parameters form one flat fp32 vector of
 * gc_mlp_param_count() values: W1[40][64], b1[64], W2[64][64], b2[64],
 * W3[64][16], b3[16], row-major, the first index the layer input.
 * Training minimises the mean over a batch of -log P[label] + lam *
 * sum_k P_k cost_k, where cost_k >= 0 is class k's relative size excess
 * over the block's least size (so the second term is the expected excess).
 * Calls on one model must not overlap.                                      */
typedef struct gc_mlp gc_mlp;

typedef struct {
    float lr, beta1, beta2, eps; /* Adam */
    float lam;                   /* weight of the expected-excess term */
    uint32_t batch;              /* samples per step, at most the model's max_batch */
    uint32_t reserved[2];
} gc_adam_opts;

size_t gc_mlp_param_count(void);

/* A model on ctx's device with zero parameters; max_batch bounds the batch
 * of gc_mlp_grad and gc_mlp_train.  Device memory is allocated here only. */
gc_status gc_mlp_create(gc_ctx *ctx, uint32_t max_batch, gc_mlp **out);
gc_status gc_mlp_destroy(gc_mlp *model);

/* Host parameter vector in/out (count must be gc_mlp_param_count()); set
 * also clears the Adam moments and step.  Both return when the copy is done. */
gc_status gc_mlp_set_params(gc_mlp *model, const float *h_params, size_t count, void *hip_stream);
gc_status gc_mlp_get_params(gc_mlp *model, float *h_params, size_t count, void *hip_stream);

/* The whole training state, for checkpoints: h_state holds 3 *
 * gc_mlp_param_count() floats -- the parameters, then Adam's first and
 * second moments, in the parameter layout -- and the Adam step count goes
 * with it.  set restores a state written by get (training then continues
 * exactly as it would have).  Both return when the copies are done.        */
gc_status gc_mlp_get_state(gc_mlp *model, float *h_state, size_t count, uint64_t *h_step, void *hip_stream);
gc_status gc_mlp_set_state(gc_mlp *model, const float *h_state, size_t count, uint64_t step, void *hip_stream);

/* Scores of n feature rows (device, n x 40): logits to d_logits (n x 16,
 * may be NULL) and the class of the largest logit (the smaller class on
 * ties) to d_class (may be NULL).  Asynchronous.                            */
gc_status gc_mlp_forward(gc_mlp *model, const float *d_feat, size_t n, float *d_logits, uint8_t *d_class,
                         void *hip_stream);

/* Gradient of the mean loss over `batch` samples: sample r is feature row
 * d_index[r] (row r when d_index is NULL) with label d_label[row] and costs
 * d_cost[row * 16 ..] (only read when lam != 0).  Writes the flat gradient
 * to d_grad and the mean loss to d_loss (either may be NULL).  Asynchronous. */
gc_status gc_mlp_grad(gc_mlp *model, const float *d_feat, const uint8_t *d_label, const float *d_cost,
                      const uint32_t *d_index, uint32_t batch, float lam, float *d_grad, float *d_loss,
                      void *hip_stream);

/* One pass of Adam steps over the samples d_index[0 .. nindex) (rows
 * 0 .. nindex when NULL), opt->batch at a time, the last batch possibly
 * smaller; the mean loss of step s goes to d_loss[s] (may be NULL).
 * Asynchronous.                                                              */
gc_status gc_mlp_train(gc_mlp *model, const float *d_feat, const uint8_t *d_label, const float *d_cost,
                       const uint32_t *d_index, size_t nindex, const gc_adam_opts *opt, float *d_loss,
                       void *hip_stream);

/* Block-container encoder with the class of every block chosen by
 *   GC_SELECT_EXHAUSTIVE  the least coded size (gc_block_sizes),
 *   GC_SELECT_LEARNED     the model's class for the block's features,
 *   GC_SELECT_FIXED       fixed_class for every block.
 * Same input, output and errors as gc_blockmix_encode; the classes also go
 * to d_class_out when it is not NULL (one byte per block).  Returns when
 * the container is written.                                                 */
#define GC_SELECT_EXHAUSTIVE 0
#define GC_SELECT_LEARNED 1
#define GC_SELECT_FIXED 2
gc_status gc_encode_blocks(gc_ctx *ctx, const uint32_t *d_in, size_t n, int mode, gc_mlp *model,
                           uint32_t fixed_class, uint32_t *d_out, size_t out_cap_words, size_t *out_words,
                           uint8_t *d_class_out, void *hip_stream);

/* Library version string. */
const char *gc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GC_H */
