// runtime.cpp -- host runtime of libgc: device contexts, single-list decode,
// batched decode plans (tile tables grouped by codec class, one hipGraph
// branch per class), per-run kernel timing and the autotuner that picks the
// tile sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "gc.h"
#include "gc_device.h"
#include "gc_format.h"
#include "gc_blocks.h"
#include "gc_mlp.h"

namespace gcdev {
int codec_class(uint32_t w0);
int launch_locate(const LocateArgs &a, int chunk_words, hipStream_t s);
int launch_carry_scan(const CarryArgs &a, hipStream_t s);
int launch_decode(int tile, int cls, int mode, const DecodeArgs &a, hipStream_t s);
int launch_pack(int pt, const PackArgs &a, hipStream_t s, uint32_t max_groups);
int noalloc_setup(int device, void **ptr);
void *noalloc_ptr(int device);
}  // namespace gcdev

using namespace gcdev;

namespace {

constexpr int kDefaultWaveTile = 2048;
constexpr int kDefaultPfdTile = 4096;
// Pack kernel workgroups per CU by default: five of the six its LDS allows.
constexpr uint32_t kDefaultPackGroups = 5u;
// Carries of delta lists: a list of at most lb_max tiles finds them in the
// decode pass by decoupled look-back (one window of flags covers a list of
// up to 64 tiles); longer lists take a tile-sum pass and a carry scan ahead
// of the decode pass.  0: every list takes the tile-sum pass.  The default
// mixes the two: on the mixed cfg2 batch it took 0.93 ms per step, against
// 0.98 ms with the tile-sum pass alone and 1.00 ms with look-back alone
// (thresholds of 16 to 128 tiles measured alike, 512 worse).
constexpr uint32_t kLookbackAll = 0xFFFFFFFFu;
constexpr uint32_t kLookbackHybrid = 64u;
constexpr uint32_t kDefaultLbMax = kLookbackHybrid;
// A list decoded alone (gc_decode) has no other lists' tiles in flight, so
// its look-back walks stay short for longer: a list of up to 2048 tiles
// finds its carries by look-back (2^20 to 2^22 integers: 2-4 us faster
// than the tile-sum pass and carry scan, equal at 2^23, slower at 2^24).
constexpr uint32_t kSingleLbMax = 2048u;
constexpr int kWaveTiles[3] = {1024, 2048, 4096};
// Longest list a context decodes alone (gc_decode) and encodes as a block
// container, unless gc_ctx_create_opts says otherwise.
constexpr uint64_t kDefaultMaxListInts = 1ull << 24;

constexpr int kClsPfd = 4;

bool valid_wave_tile(uint32_t t) { return t == 1024 || t == 2048 || t == 4096; }

#define HIP_OK(x)                         \
    do {                                  \
        if ((x) != hipSuccess) {          \
            (void)hipGetLastError();      \
            return GC_EDEVICE;            \
        }                                 \
    } while (0)

// Control words the locate pass scans (host mirror of the device rule).
uint32_t locate_words_host(const HeaderFields &h, uint32_t T, uint32_t C, uint32_t D) {
    switch (h.codec) {
    case 0: return std::min(C, ((D >> h.lk) + 7u) >> 3);
    case 1:
        if (h.ld == GC_LD_BINARY) {
            const uint32_t fpu = h.cg == 1 ? 3u : h.cg == 8 ? 4u : 2u;
            const uint32_t ub = h.cg == 1 ? 16u : 8u;
            const uint32_t fpw = fpu * (32u / ub);
            return std::min(C, (T + fpw - 1u) / fpw);
        }
        return C;
    case 2:
    case 4: return C;
    default: return std::min(C, (T + 31u) >> 5);
    }
}

template <typename T>
gc_status dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void **)p, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return GC_ENOMEM;
    }
    if (hipMemset(*p, 0, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(*p);
        *p = nullptr;
        return GC_EDEVICE;
    }
    return GC_OK;
}

// First locate epoch of codec class c (the device advances it by kClasses
// per run, so the epochs of different classes never coincide).
uint32_t first_epoch(int c) { return (uint32_t)c + 1u; }

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Device scratch of one launch sequence: the locate epoch of every codec
// class, the tile starts, the tile carries and the locate chunk aggregates
// and prefixes.
struct Scratch {
    RunState *state = nullptr;          // [class]
    TileInfo *tiles = nullptr;
    uint32_t *carry = nullptr;
    unsigned long long *flags = nullptr;   // single-pass carry flags, one per tile
    LocVal *agg = nullptr, *pre = nullptr;
    size_t tiles_cap = 0, chunks_cap = 0;

    gc_status init_state() {
        gc_status rc = dev_alloc(&state, kClasses);
        if (rc) return rc;
        std::vector<RunState> h(kClasses);
        for (int c = 0; c < kClasses; c++) h[c] = RunState{first_epoch(c), {0u, 0u, 0u}};
        HIP_OK(hipMemcpy(state, h.data(), h.size() * sizeof(RunState), hipMemcpyHostToDevice));
        return GC_OK;
    }
    // Grows the tables (plans and contexts call this only when they are
    // created, never on a decode).  On any failure every table is freed and
    // both capacities drop to zero, so a later call reallocates them all.
    gc_status reserve(size_t ntiles, size_t nchunks) {
        gc_status rc = GC_OK;
        if (ntiles > tiles_cap) {
            if (hipDeviceSynchronize() != hipSuccess) rc = GC_EDEVICE;
            dev_free(tiles);
            dev_free(carry);
            dev_free(flags);
            tiles_cap = 0;
            const size_t cap = ntiles;
            if (!rc) rc = dev_alloc(&tiles, cap);
            if (!rc) rc = dev_alloc(&carry, cap);
            // no flag may carry an epoch before it is written: zeroed once here
            if (!rc) rc = dev_alloc(&flags, cap);
            if (!rc) tiles_cap = cap;
        }
        if (!rc && nchunks > chunks_cap) {
            if (hipDeviceSynchronize() != hipSuccess) rc = GC_EDEVICE;
            dev_free(agg);
            dev_free(pre);
            chunks_cap = 0;
            const size_t cap = nchunks;
            if (!rc) rc = dev_alloc(&agg, cap);
            if (!rc) rc = dev_alloc(&pre, cap);
            if (!rc) chunks_cap = cap;
        }
        if (rc) {
            (void)hipGetLastError();
            dev_free(tiles);
            dev_free(carry);
            dev_free(flags);
            dev_free(agg);
            dev_free(pre);
            tiles_cap = chunks_cap = 0;
        }
        return rc;
    }
    void release() {
        dev_free(state);
        dev_free(tiles);
        dev_free(carry);
        dev_free(flags);
        dev_free(agg);
        dev_free(pre);
        tiles_cap = chunks_cap = 0;
    }
};

}  // namespace

// Device scratch of the block container encoder: per-block payload words
// and offsets, the scan's chunk sums, and {total words, bad class flag}.
struct BlockScratch {
    uint32_t *words = nullptr, *offs = nullptr, *csum = nullptr, *result = nullptr;
    float *feat = nullptr;   // features of every block (selector input)
    uint8_t *cls = nullptr;  // class of every block
    size_t cap = 0;
    // Called once, when the context is created; on failure nothing is kept.
    gc_status reserve(size_t nblocks) {
        release();
        const size_t c = std::max(nblocks, (size_t)1024);
        gc_status rc = dev_alloc(&words, c);
        if (!rc) rc = dev_alloc(&offs, c);
        if (!rc) rc = dev_alloc(&csum, gcblk::scan_chunks(c) + 1);
        if (!rc) rc = dev_alloc(&result, 2);
        if (!rc) rc = dev_alloc(&feat, c * gcblk::kFeatures);
        if (!rc) rc = dev_alloc(&cls, c);
        if (rc) release();
        else cap = c;
        return rc;
    }
    void release() {
        dev_free(words);
        dev_free(offs);
        dev_free(csum);
        dev_free(result);
        dev_free(feat);
        dev_free(cls);
        cap = 0;
    }
};

struct gc_ctx {
    int device = 0;
    int num_cus = 0;
    Status *status = nullptr;
    Scratch single;             // gc_decode's tables, sized for max_list_ints at creation
    BlockScratch blk;           // the block encoder's, likewise
    uint64_t max_list_ints = 0;
    std::string arch;           // the device's architecture name (autotune cache keys)
    int tile_w = kDefaultWaveTile, tile_p = kDefaultPfdTile;
    std::mutex mu;
};

// Tiles are numbered class by class; within a class the delta lists of more
// than one tile come first, so one launch range covers each pass.
struct ClassRange {
    uint32_t loc_lo = 0;    // first locate chunk item of the class
    uint32_t loc_count = 0; // its locate chunk items
    uint32_t lsc_lo = 0;    // first locate scan item (a list with chunks)
    uint32_t lsc_count = 0;
    uint32_t lo = 0;        // first tile of the class
    uint32_t count = 0;     // tiles of the class
    uint32_t sum = 0;       // leading tiles that need a tile sum
    uint32_t scan_lo = 0;   // first entry of the class in the scan list
    uint32_t scans = 0;     // lists to scan
};

// The packs of one pack kernel (capacity kPackInts[i]): descriptors in
// pack order, the list of each, and every pack's first descriptor.
struct PackSet {
    std::vector<PackDesc> h;       // pointers filled at upload
    std::vector<uint32_t> list;    // descriptor -> list
    std::vector<uint32_t> first;   // packs + 1 entries
    PackDesc *d = nullptr;
    uint32_t *d_first = nullptr;
    uint32_t packs() const { return first.empty() ? 0u : (uint32_t)first.size() - 1u; }
};

struct gc_plan {
    gc_ctx *ctx = nullptr;
    size_t nlists = 0;
    int tile[kClasses] = {kDefaultWaveTile, kDefaultWaveTile, kDefaultWaveTile, kDefaultWaveTile, kDefaultPfdTile};
    ClassRange cr[kClasses];
    uint32_t total_a = 0, total_s = 0, total_t = 0, total_scan = 0;
    bool use_graph = false;
    std::vector<ListDesc> h_lists;             // pointers filled at upload
    std::vector<int> cls;                      // codec class per list
    std::vector<uint64_t> stream_off, out_off;
    std::vector<uint32_t> item_a, item_s;      // locate: chunk -> list, scan -> list
    std::vector<uint32_t> tile_list, scan_list;
    ListDesc *d_lists = nullptr;
    uint32_t *d_item_a = nullptr, *d_item_s = nullptr, *d_scan_list = nullptr;
    Scratch sc;
    const uint32_t *bound_streams = nullptr;
    uint32_t *bound_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev;                // kEvPerSlot per timing slot
    hipStream_t aux = nullptr;                 // timing: the locate stream
    bool serial = true;                        // no locate stream
    uint32_t lb_max = kDefaultLbMax;           // lists of at most this many tiles: look-back carries
    uint32_t lb_stall = 0;                     // tests only: see GC_TEST_LOOKBACK_STALL
    uint32_t slots = 0;
    uint64_t runs = 0;
    // lists of at most pack_max integers whose streams fit a pack are
    // decoded by the pack kernel instead of the class passes; 0: none
    uint32_t pack_max = 0;
    bool pack_forced = false;                  // pack_max set by the plan options
    uint32_t pack_groups = kDefaultPackGroups; // pack workgroups per CU (GC_PACK_GROUPS_ALL: a wave per pack)
    bool groups_forced = false;                // pack_groups set by the plan options
    std::vector<uint8_t> packed;               // per list
    PackSet pk[2];                             // packs of the kernel of capacity kPackInts[0] / [1] (one is used)
    bool branches = true;                      // graph: the pack kernel and each class's passes on branches
    uint32_t total_chunks = 0;                 // locate chunks of every list (batch items first)
};

namespace {

// The pack kernels: integers of tuple space and staged stream words per
// pack; a plan uses the smaller one when its threshold allows.
constexpr uint32_t kPackInts[2] = {2048u, 4096u};
constexpr uint32_t kPackWords[2] = {512u, 1024u};
// Default pack_max: lists of up to 2048 integers.
constexpr uint32_t kDefaultPackMax = 2048u;
constexpr uint32_t kPackMaxLists = 32u;
int pack_cfg(uint32_t pack_max) { return pack_max <= kPackInts[0] ? 0 : 1; }

LocateArgs make_locate_args(const ListDesc *lists, const uint32_t *item_list, const uint32_t *scan_list,
                            const ListDesc &single, uint32_t total, uint32_t total_scan, int cls, Scratch &sc,
                            Status *st) {
    LocateArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lists = lists;
    a.item_list = item_list;
    a.scan_list = scan_list;
    a.single = single;
    a.total_items = total;
    a.total_scan = total_scan;
    a.tiles = sc.tiles;
    a.agg = sc.agg;
    a.pre = sc.pre;
    a.state = sc.state + cls;
    a.status = st;
    return a;
}

DecodeArgs make_decode_args(const ListDesc *lists, const ListDesc &single, uint32_t lo, uint32_t count, int cls,
                            Scratch &sc, Status *st) {
    DecodeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lists = lists;
    a.single = single;
    a.lo = lo;
    a.count = count;
    a.tiles = sc.tiles;
    a.carry = sc.carry;
    a.flags = sc.flags;
    a.loc_state = sc.state + cls;
    a.status = st;
    return a;
}

CarryArgs make_carry_args(const ListDesc *lists, const uint32_t *scan_list, const ListDesc &single, uint32_t count,
                          Scratch &sc) {
    CarryArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lists = lists;
    a.scan_list = scan_list;
    a.single = single;
    a.count = count;
    a.carry = sc.carry;
    return a;
}

uint32_t list_chunks(const HeaderFields &h, uint32_t n, uint32_t C, uint32_t D, uint32_t chunk_words) {
    const uint32_t T = (n + (uint32_t)h.k - 1u) >> h.lk;
    const uint32_t nw = locate_words_host(h, T, C, D);
    return std::max(1u, (nw + chunk_words - 1u) / chunk_words);
}

bool is_delta(uint32_t w0) {
    HeaderFields h;
    return header_fields(w0, h) && h.delta;
}

// A tile must hold at least 32 tuples: every control unit (selector,
// unary code word, frame, Group-PFD block) spans at most 32 tuples, so the
// locate pass meets at most one tile boundary per unit (and a Group-PFD
// tile holds whole blocks).
int min_class_tile(const gc_plan *p, int c) {
    int t = 1024;
    for (size_t i = 0; i < p->nlists; i++) {
        if (p->cls[i] != c) continue;
        HeaderFields h;
        header_fields(p->h_lists[i].w0, h);
        t = std::max(t, 32 << h.lk);
    }
    return t;
}

// Single-list view of list L for the per-list paths: its own tile range.
DecodeArgs single_args(const ListDesc &L, int cls, Scratch &sc, Status *st) {
    return make_decode_args(nullptr, L, L.tile_base, L.ntiles, cls, sc, st);
}

// Launches every pass of one list on stream s (the per-list paths).
// chunk_words: the control words per locate item that L.nchunks counts.
gc_status launch_one(const ListDesc &L, int cls, Scratch &sc, Status *st, hipStream_t s, uint32_t lb_max,
                     int chunk_words) {
    if (L.ntiles > 1) {
        LocateArgs a = make_locate_args(nullptr, nullptr, nullptr, L, L.nchunks, 1, cls, sc, st);
        if (launch_locate(a, chunk_words, s)) return GC_EDEVICE;
    }
    const int tile = (int)L.tile_ints;
    DecodeArgs d = single_args(L, cls, sc, st);
    d.lb_max_tiles = lb_max;
    const bool lookback = L.ntiles <= lb_max;
    if (!lookback && L.ntiles > 1 && is_delta(L.w0)) {
        if (launch_decode(tile, cls, 1, d, s)) return GC_EDEVICE;
        if (launch_carry_scan(make_carry_args(nullptr, nullptr, L, 1, sc), s)) return GC_EDEVICE;
    }
    if (launch_decode(tile, cls, lookback ? 2 : 0, d, s)) return GC_EDEVICE;
    return GC_OK;
}

// Tuples of list L in a pack's tuple space (its first at a multiple of
// 32 / k tuples, so every list starts at a 32-integer boundary).
uint32_t pack_tuples(const ListDesc &L, const HeaderFields &h) {
    const uint32_t T = (L.n + (uint32_t)h.k - 1u) >> h.lk;
    const uint32_t u = h.lk >= 5 ? 1u : 32u >> h.lk;
    return (T + u - 1u) & ~(u - 1u);
}

// Whether list L goes to the pack kernel of configuration cfg: 1 ..
// pack_max integers, its padded tuples and its stream within one pack.
bool pack_fits(const ListDesc &L, uint32_t pack_max, int cfg) {
    if (L.n == 0 || L.n > pack_max) return false;
    HeaderFields h;
    if (!header_fields(L.w0, h)) return false;
    if (L.stream_words > kPackWords[cfg] || (L.stream_words & 3u) || (L.C & 3u)) return false;
    return ((uint64_t)pack_tuples(L, h) << h.lk) <= kPackInts[cfg];
}

// Builds the tile tables of a plan for its tile sizes.
void build_tables(gc_plan *p) {
    for (int c = 0; c < kClasses; c++) p->tile[c] = std::max(p->tile[c], min_class_tile(p, c));
    p->item_a.clear();
    p->item_s.clear();
    p->tile_list.clear();
    p->scan_list.clear();
    p->packed.assign(p->nlists, 0);
    for (PackSet &ps : p->pk) {
        ps.h.clear();
        ps.list.clear();
        ps.first.clear();
    }
    for (size_t i = 0; i < p->nlists; i++) {
        ListDesc &L = p->h_lists[i];
        L.tile_ints = (uint32_t)p->tile[p->cls[i]];
        L.ntiles = (uint32_t)((L.n + (uint64_t)L.tile_ints - 1) / (uint64_t)L.tile_ints);
        L.nchunks = 0;
        if (L.ntiles > 1) {
            HeaderFields h;
            header_fields(L.w0, h);
            L.nchunks = list_chunks(h, L.n, L.C, L.D, kChunkWords);
        }
    }
    // Packs: lists of one stream format (header word 0 without its delta
    // bit), in list order, while they number at most 32 and their streams
    // and padded tuple spaces fit the kernel's buffers.
    if (p->pack_max) {
        const int cfg = pack_cfg(p->pack_max);
        PackSet &ps = p->pk[cfg];
        std::map<uint32_t, std::vector<uint32_t>> by_fmt;
        std::vector<uint32_t> order;   // formats in order of first appearance
        for (size_t i = 0; i < p->nlists; i++) {
            const ListDesc &L = p->h_lists[i];
            if (!pack_fits(L, p->pack_max, cfg)) continue;
            const uint32_t f = L.w0 & ~(1u << 19);
            auto &v = by_fmt[f];
            if (v.empty()) order.push_back(f);
            v.push_back((uint32_t)i);
        }
        for (uint32_t f : order) {
            uint32_t words = 0, ints = 0;
            bool fresh = true;   // the format's first list opens a pack
            for (uint32_t i : by_fmt[f]) {
                const ListDesc &L = p->h_lists[i];
                HeaderFields h;
                header_fields(L.w0, h);
                const uint32_t w = (uint32_t)L.stream_words, pi = pack_tuples(L, h) << h.lk;
                if (fresh || (uint32_t)ps.h.size() - ps.first.back() >= kPackMaxLists ||
                    words + w > kPackWords[cfg] || ints + pi > kPackInts[cfg]) {
                    fresh = false;
                    ps.first.push_back((uint32_t)ps.h.size());
                    words = ints = 0;
                }
                PackDesc d;
                std::memset(&d, 0, sizeof(d));
                d.n = L.n;
                d.w0 = L.w0;
                d.cd = L.C | (L.D << 16);
                d.words = w;
                ps.h.push_back(d);
                ps.list.push_back(i);
                words += w;
                ints += pi;
                p->packed[i] = 1;
            }
        }
        if (!ps.first.empty()) ps.first.push_back((uint32_t)ps.h.size());
    }
    // Locate items, tiles and carry scans are numbered class by class, so
    // each class's kernels cover one range of each table.  Within a class
    // the delta lists of more than one tile come first.  Packed lists come
    // after every class: the batch does not run them through these tables,
    // but one launch sequence per list (gc_decode_each) does.
    uint32_t cb = 0, tb = 0;
    for (int c = 0; c < kClasses; c++) {
        ClassRange &r = p->cr[c];
        r = ClassRange{};
        r.loc_lo = cb;
        r.lsc_lo = (uint32_t)p->item_s.size();
        for (size_t i = 0; i < p->nlists; i++) {
            ListDesc &L = p->h_lists[i];
            if (p->cls[i] != c || !L.nchunks || p->packed[i]) continue;
            L.chunk_base = cb;
            for (uint32_t k = 0; k < L.nchunks; k++) p->item_a.push_back((uint32_t)i);
            if (L.nchunks > 1) p->item_s.push_back((uint32_t)i);   // one chunk: no scan
            cb += L.nchunks;
        }
        r.loc_count = cb - r.loc_lo;
        r.lsc_count = (uint32_t)p->item_s.size() - r.lsc_lo;
        r.lo = tb;
        r.scan_lo = (uint32_t)p->scan_list.size();
        for (int pass = 0; pass < 2; pass++) {
            for (size_t i = 0; i < p->nlists; i++) {
                ListDesc &L = p->h_lists[i];
                if (p->cls[i] != c || L.ntiles == 0 || p->packed[i]) continue;
                const bool summed = L.ntiles > 1 && is_delta(L.w0) && L.ntiles > p->lb_max;
                if (summed != (pass == 0)) continue;
                L.tile_base = tb;
                for (uint32_t m = 0; m < L.ntiles; m++) p->tile_list.push_back((uint32_t)i);
                tb += L.ntiles;
                if (summed) {
                    r.sum += L.ntiles;
                    p->scan_list.push_back((uint32_t)i);
                }
            }
        }
        r.count = tb - r.lo;
        r.scans = (uint32_t)p->scan_list.size() - r.scan_lo;
    }
    p->total_a = (uint32_t)p->item_a.size();
    p->total_s = (uint32_t)p->item_s.size();
    p->total_scan = (uint32_t)p->scan_list.size();
    for (size_t i = 0; i < p->nlists; i++) {
        ListDesc &L = p->h_lists[i];
        if (!p->packed[i]) continue;
        L.chunk_base = cb;
        cb += L.nchunks;
        L.tile_base = tb;
        for (uint32_t m = 0; m < L.ntiles; m++) p->tile_list.push_back((uint32_t)i);
        tb += L.ntiles;
    }
    p->total_chunks = cb;
    p->total_t = tb;
}

void plan_free_graphs(gc_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec), p->exec = nullptr;
    if (p->graph) (void)hipGraphDestroy(p->graph), p->graph = nullptr;
}

void plan_free_device(gc_plan *p) {
    plan_free_graphs(p);
    dev_free(p->d_lists);
    dev_free(p->d_item_a);
    dev_free(p->d_item_s);
    dev_free(p->d_scan_list);
    for (PackSet &ps : p->pk) {
        dev_free(ps.d);
        dev_free(ps.d_first);
    }
    p->sc.release();
}

gc_status plan_upload(gc_plan *p, const uint32_t *d_streams, uint32_t *d_out) {
    std::vector<ListDesc> t(p->h_lists);
    for (size_t i = 0; i < p->nlists; i++) {
        t[i].stream = d_streams + p->stream_off[i];
        t[i].out = d_out + p->out_off[i];
    }
    HIP_OK(hipMemcpy(p->d_lists, t.data(), t.size() * sizeof(ListDesc), hipMemcpyHostToDevice));
    for (PackSet &ps : p->pk) {
        if (ps.h.empty()) continue;
        for (size_t j = 0; j < ps.h.size(); j++) {
            ps.h[j].stream = d_streams + p->stream_off[ps.list[j]];
            ps.h[j].out = d_out + p->out_off[ps.list[j]];
        }
        HIP_OK(hipMemcpy(ps.d, ps.h.data(), ps.h.size() * sizeof(PackDesc), hipMemcpyHostToDevice));
    }
    p->bound_streams = d_streams;
    p->bound_out = d_out;
    return GC_OK;
}

template <typename T>
gc_status upload_vec(T **d, const std::vector<T> &h) {
    dev_free(*d);
    gc_status rc = dev_alloc(d, h.size());
    if (rc) return rc;
    if (!h.empty()) HIP_OK(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return GC_OK;
}

// Allocates the device side of a plan for its current tile sizes.
gc_status plan_materialize(gc_plan *p) {
    plan_free_graphs(p);
    build_tables(p);
    gc_status rc = GC_OK;
    if (!p->d_lists) rc = dev_alloc(&p->d_lists, p->nlists);
    if (!rc && !p->sc.state) rc = p->sc.init_state();
    if (!rc) rc = upload_vec(&p->d_item_a, p->item_a);
    if (!rc) rc = upload_vec(&p->d_item_s, p->item_s);

    if (!rc) rc = upload_vec(&p->d_scan_list, p->scan_list);
    for (PackSet &ps : p->pk) {
        if (!rc) rc = upload_vec(&ps.d, ps.h);
        if (!rc) rc = upload_vec(&ps.d_first, ps.first);
    }
    if (!rc) rc = p->sc.reserve(p->total_t + 1, p->total_chunks);
    if (!rc && p->total_t) {
        // every tile names its list; the locate pass rewrites the entries of
        // tiles m >= 1 on each run, tile 0 of a list starts at zero
        std::vector<TileInfo> init(p->total_t);
        for (uint32_t t = 0; t < p->total_t; t++) {
            std::memset(&init[t], 0, sizeof(TileInfo));
            init[t].list = p->tile_list[t];
        }
        HIP_OK(hipMemcpy(p->sc.tiles, init.data(), init.size() * sizeof(TileInfo), hipMemcpyHostToDevice));
    }
    return rc;
}

// Launches the locate kernels of codec class c on stream s.
// Launches the locate kernels of every class at once on stream s, with the
// epoch of class 0 (the serial schedule: every class's passes follow it).
gc_status launch_all_locate(gc_plan *p, hipStream_t s) {
    if (!p->total_a) return GC_OK;
    ListDesc none;
    std::memset(&none, 0, sizeof(none));
    LocateArgs a = make_locate_args(p->d_lists, p->d_item_a, p->d_item_s, none, p->total_a, p->total_s, 0, p->sc,
                                    p->ctx->status);
    a.item_lo = 0;
    return launch_locate(a, kChunkWords, s) ? GC_EDEVICE : GC_OK;
}

// The class that reports the locate time: with the serial schedule the
// single locate pass is timed in the column of the first class with tiles.
int first_class(const gc_plan *p) {
    for (int c = 0; c < kClasses; c++)
        if (p->cr[c].count) return c;
    return 0;
}

gc_status launch_class_locate(gc_plan *p, int c, hipStream_t s) {
    const ClassRange &r = p->cr[c];
    if (!r.loc_count) return GC_OK;
    ListDesc none;
    std::memset(&none, 0, sizeof(none));
    LocateArgs a = make_locate_args(p->d_lists, p->d_item_a, p->d_item_s + r.lsc_lo, none, r.loc_count,
                                    r.lsc_count, c, p->sc, p->ctx->status);
    a.item_lo = r.loc_lo;
    return launch_locate(a, kChunkWords, s) ? GC_EDEVICE : GC_OK;
}

// Launches the tile sums and carry scan (delta lists of more than one tile)
// and the decode pass of codec class c on stream s; `mid`, if given, is
// recorded between the two.  per_class: the tile starts were written by the
// class's own locate kernels (tagged with its epoch), not by the one locate
// pass over every class (tagged with class 0's).
gc_status launch_class_work(gc_plan *p, int c, hipStream_t s, bool per_class, hipEvent_t mid = nullptr) {
    const ClassRange &r = p->cr[c];
    ListDesc none;
    std::memset(&none, 0, sizeof(none));
    const int tile = p->tile[c];
    const int epoch_cls = per_class ? c : 0;   // whose locate epoch tags the tile starts
    if (r.sum) {
        DecodeArgs d = make_decode_args(p->d_lists, none, r.lo, r.sum, epoch_cls, p->sc, p->ctx->status);
        if (launch_decode(tile, c, 1, d, s)) return GC_EDEVICE;
        CarryArgs ca = make_carry_args(p->d_lists, p->d_scan_list + r.scan_lo, none, r.scans, p->sc);
        if (launch_carry_scan(ca, s)) return GC_EDEVICE;
    }
    if (mid) HIP_OK(hipEventRecord(mid, s));
    DecodeArgs d = make_decode_args(p->d_lists, none, r.lo, r.count, epoch_cls, p->sc, p->ctx->status);
    d.lb_max_tiles = p->lb_max;
    d.lb_stall_ticks = p->lb_stall;
    return launch_decode(tile, c, p->lb_max ? 2 : 0, d, s) ? GC_EDEVICE : GC_OK;
}

// Launches a whole run on stream s: without an auxiliary stream, one locate
// pass over every class, then class after class the tile sums, carry scans
// and decode pass.  With an auxiliary stream `aux`, the locate kernels of
// every class run there in class order and the rest of class c waits only
// for its own locate, so the locate of the next class overlaps the passes of
// this one.  sync[c] signals the end
// of class c's locate; with `tev` (timing), class c records tev[5c .. 5c+4]:
// before and after its locate, before its tile sums, before and after its
// decode pass.
// Launches the pack kernels on stream s.
gc_status launch_packs(gc_plan *p, hipStream_t s) {
    for (int k = 0; k < 2; k++) {
        const PackSet &ps = p->pk[k];
        if (!ps.packs()) continue;
        PackArgs a;
        std::memset(&a, 0, sizeof(a));
        a.descs = ps.d;
        a.first = ps.d_first;
        a.npacks = ps.packs();
        a.status = p->ctx->status;
        const uint32_t cap = p->pack_groups == GC_PACK_GROUPS_ALL ? 0u : p->pack_groups * (uint32_t)p->ctx->num_cus;
        if (launch_pack((int)kPackInts[k], a, s, cap)) return GC_EDEVICE;
    }
    return GC_OK;
}

// The two events around the pack kernels, after the classes' five each
// (indices into the events plan_launch records).
constexpr int kTevPack = 5 * kClasses;

// With a pack stream `pks` (and its fork / join events), the pack kernel
// runs there, beside the locate pass and the class passes.  With class
// streams `cls` (one locate pass, no auxiliary stream), the passes of class
// c run on cls[c] once the locate pass is done (event loc_done), and s
// waits for all of them (events cjoin[c]).
gc_status plan_launch(gc_plan *p, hipStream_t s, hipStream_t aux = nullptr, hipEvent_t start = nullptr,
                      hipEvent_t *sync = nullptr, hipEvent_t *tev = nullptr, hipStream_t pks = nullptr,
                      hipEvent_t pk_fork = nullptr, hipEvent_t pk_join = nullptr, hipStream_t *cls = nullptr,
                      hipEvent_t loc_done = nullptr, hipEvent_t *cjoin = nullptr) {
    if (aux) {
        HIP_OK(hipEventRecord(start, s));
        HIP_OK(hipStreamWaitEvent(aux, start, 0));
    }
    // the packed lists depend on nothing the other passes compute
    const bool fork = pks && (p->pk[0].packs() || p->pk[1].packs());
    if (fork) {
        HIP_OK(hipEventRecord(pk_fork, s));
        HIP_OK(hipStreamWaitEvent(pks, pk_fork, 0));
    }
    const hipStream_t ps = fork ? pks : s;
    if (tev) HIP_OK(hipEventRecord(tev[kTevPack], ps));
    if (gc_status rc = launch_packs(p, ps)) return rc;
    if (tev) HIP_OK(hipEventRecord(tev[kTevPack + 1], ps));
    if (fork) HIP_OK(hipEventRecord(pk_join, ps));
    hipStream_t ls = aux ? aux : s;
    if (!aux) {
        const int c0 = first_class(p);
        if (tev) HIP_OK(hipEventRecord(tev[5 * c0], s));
        if (gc_status rc = launch_all_locate(p, s)) return rc;
        if (tev) HIP_OK(hipEventRecord(tev[5 * c0 + 1], s));
    }
    for (int c = 0; c < kClasses && aux; c++) {
        if (!p->cr[c].count) continue;
        if (tev) HIP_OK(hipEventRecord(tev[5 * c], ls));
        if (gc_status rc = launch_class_locate(p, c, ls)) return rc;
        HIP_OK(hipEventRecord(tev ? tev[5 * c + 1] : sync[c], ls));
    }
    const bool branch = cls && !aux && !tev;
    if (branch) HIP_OK(hipEventRecord(loc_done, s));
    for (int c = 0; c < kClasses; c++) {
        if (!p->cr[c].count) continue;
        const hipStream_t cs = branch ? cls[c] : s;
        if (branch) HIP_OK(hipStreamWaitEvent(cs, loc_done, 0));
        if (aux) HIP_OK(hipStreamWaitEvent(s, tev ? tev[5 * c + 1] : sync[c], 0));
        if (tev) HIP_OK(hipEventRecord(tev[5 * c + 2], s));
        if (gc_status rc = launch_class_work(p, c, cs, aux != nullptr, tev ? tev[5 * c + 3] : nullptr)) return rc;
        if (tev) HIP_OK(hipEventRecord(tev[5 * c + 4], s));
        if (branch) HIP_OK(hipEventRecord(cjoin[c], cs));
    }
    for (int c = 0; c < kClasses && branch; c++)
        if (p->cr[c].count) HIP_OK(hipStreamWaitEvent(s, cjoin[c], 0));
    if (fork) HIP_OK(hipStreamWaitEvent(s, pk_join, 0));
    return GC_OK;
}

gc_status capture_one(gc_plan *p, hipGraph_t *graph, hipGraphExec_t *exec) {
    hipStream_t s, aux, pks, cls[kClasses];
    hipEvent_t start, sync[kClasses], fork, join, loc_done, cjoin[kClasses];
    HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    HIP_OK(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
    HIP_OK(hipStreamCreateWithFlags(&pks, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&join, hipEventDisableTiming));
    HIP_OK(hipEventCreateWithFlags(&loc_done, hipEventDisableTiming));
    for (int c = 0; c < kClasses; c++) {
        HIP_OK(hipEventCreateWithFlags(&sync[c], hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&cjoin[c], hipEventDisableTiming));
        HIP_OK(hipStreamCreateWithFlags(&cls[c], hipStreamNonBlocking));
    }
    gc_status rc = GC_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = GC_EDEVICE;
    } else {
        // the graph's pack kernel is a branch of its own
        rc = plan_launch(p, s, p->serial ? nullptr : aux, start, sync, nullptr, p->branches ? pks : nullptr,
                         fork, join, p->branches ? cls : nullptr, loc_done, cjoin);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(s, &g) != hipSuccess || rc) {
            rc = GC_EDEVICE;
            if (g) (void)hipGraphDestroy(g);
        } else {
            *graph = g;
            if (hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) rc = GC_EDEVICE;
        }
    }
    for (int c = 0; c < kClasses; c++) {
        (void)hipEventDestroy(sync[c]);
        (void)hipEventDestroy(cjoin[c]);
        (void)hipStreamDestroy(cls[c]);
    }
    (void)hipEventDestroy(start);
    (void)hipEventDestroy(fork);
    (void)hipEventDestroy(join);
    (void)hipEventDestroy(loc_done);
    (void)hipStreamDestroy(pks);
    (void)hipStreamDestroy(aux);
    (void)hipStreamDestroy(s);
    (void)hipGetLastError();
    return rc;
}

gc_status plan_capture(gc_plan *p) {
    plan_free_graphs(p);
    return capture_one(p, &p->graph, &p->exec);
}

// Events of one timing slot: run start and end on the launch stream, five
// per class and two around the pack kernels (see plan_launch).
constexpr int kEvPerSlot = 4 + 5 * kClasses;

gc_status plan_run(gc_plan *p, hipStream_t s) {
    if (p->slots) {
        hipEvent_t *e = &p->ev[(size_t)(p->runs % p->slots) * kEvPerSlot];
        p->runs++;
        HIP_OK(hipEventRecord(e[0], s));
        if (gc_status rc = plan_launch(p, s, p->serial ? nullptr : p->aux, e[0], nullptr, e + 2)) return rc;
        HIP_OK(hipEventRecord(e[1], s));
        return GC_OK;
    }
    if (p->use_graph && p->exec) {
        HIP_OK(hipGraphLaunch(p->exec, s));
        return GC_OK;
    }
    return plan_launch(p, s);
}

// ---- autotune cache: one JSON object {key: [tile of each class, packed-list
// threshold, pack workgroups per CU], ...} ------------------------------------
std::string cache_path() {
    const char *e = std::getenv("GC_AUTOTUNE_CACHE");
    return e ? std::string(e) : std::string();
}

bool cache_lookup(const std::string &key, int *tiles, uint32_t *pack_max, uint32_t *pack_groups) {
    const std::string path = cache_path();
    if (path.empty()) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    const std::string pat = "\"" + key + "\": [";
    const size_t at = s.find(pat);
    if (at == std::string::npos) return false;
    int t[kClasses];
    unsigned pm = 0, pg = kDefaultPackGroups;
    static_assert(kClasses == 5, "five classes in the cache format");
    // [tiles of the five classes, packed-list threshold, pack workgroups per CU]
    if (std::sscanf(s.c_str() + at + pat.size(), "%d, %d, %d, %d, %d, %u, %u", &t[0], &t[1], &t[2], &t[3], &t[4],
                    &pm, &pg) != 7)
        return false;
    if (pg != GC_PACK_GROUPS_ALL && (pg == 0u || pg > 64u)) return false;
    for (int c = 0; c < kClasses; c++)   // an entry that fails validation falls back to the defaults
        if (!valid_wave_tile((uint32_t)t[c])) return false;
    if (pm > kPackInts[1]) return false;
    for (int c = 0; c < kClasses; c++) tiles[c] = t[c];
    *pack_max = pm;
    *pack_groups = pg;
    return true;
}

void cache_store(const std::string &key, const int *tiles, uint32_t pack_max, uint32_t pack_groups) {
    const std::string path = cache_path();
    if (path.empty()) return;
    std::string s;
    {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            s = ss.str();
        }
    }
    std::vector<std::string> entries;
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        const size_t e = s.find('"', pos + 1);
        if (e == std::string::npos) break;
        const std::string k = s.substr(pos + 1, e - pos - 1);
        const size_t lb = s.find('[', e), rb = s.find(']', e);
        if (lb == std::string::npos || rb == std::string::npos) break;
        if (k != key) entries.push_back("\"" + k + "\": " + s.substr(lb, rb - lb + 1));
        pos = rb + 1;
    }
    char buf[128];
    std::snprintf(buf, sizeof(buf), "[%d, %d, %d, %d, %d, %u, %u]", tiles[0], tiles[1], tiles[2], tiles[3],
                  tiles[4], pack_max, pack_groups);
    entries.push_back("\"" + key + "\": " + buf);
    std::ofstream f(path);
    f << "{\n";
    for (size_t i = 0; i < entries.size(); i++) f << "  " << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
    f << "}\n";
}

std::string plan_key(const gc_plan *p) {
    uint64_t total = 0, per_cls[kClasses] = {};
    int lk = 2;
    for (size_t i = 0; i < p->nlists; i++) {
        HeaderFields h;
        header_fields(p->h_lists[i].w0, h);
        per_cls[p->cls[i]] += p->h_lists[i].n;
        total += p->h_lists[i].n;
        lk = std::max(lk, h.lk);
    }
    int lg = 0;
    while ((1ull << lg) < total) lg++;
    const uint64_t mean = p->nlists ? total / p->nlists : 0;
    int lm = 0;
    while ((1ull << lm) < mean) lm++;
    // short lists decide the pack kernels' share: the fraction (in eighths)
    // of lists of at most 2048 integers
    uint64_t short_lists = 0;
    for (size_t i = 0; i < p->nlists; i++) short_lists += p->h_lists[i].n <= kPackInts[0];
    std::string key = p->ctx->arch + ":k" + std::to_string(1 << lk) + ":n2^" + std::to_string(lg) + ":mean2^" +
                      std::to_string(lm) + ":c" + std::to_string(p->lb_max) + ":s" +
                      std::to_string(p->nlists ? short_lists * 8 / p->nlists : 0) +
                      (p->pack_forced ? ":p" + std::to_string(p->pack_max) : std::string()) +
                      (p->groups_forced ? ":g" + std::to_string(p->pack_groups) : std::string()) + ":mix";
    for (int c = 0; c < kClasses; c++)
        key += (c ? "-" : "") + std::to_string(total ? per_cls[c] * 8 / total : 0);
    return key;
}

// Times the candidates and keeps the fastest: first, for every codec
// class, the tile size whose passes (tile sums, carry scan, decode) took
// least: one materialised plan per candidate, each class timed by HIP
// events around its own passes (a class's passes do not depend on the tile
// sizes of the others); then, at those tile sizes, the packed-list
// threshold (no packing, lists of up to 1024, 2048 or 4096 integers; unless
// the plan fixes it), by the whole run, replayed from a graph when the plan
// uses one.
gc_status autotune(gc_plan *p, const uint32_t *d_streams, uint32_t *d_out) {
    const std::string key = plan_key(p);
    int best_t[kClasses];
    for (int c = 0; c < kClasses; c++) best_t[c] = p->tile[c];
    uint32_t best_pm = p->pack_max, best_pg = p->pack_groups;
    if (cache_lookup(key, best_t, &best_pm, &best_pg)) {
        for (int c = 0; c < kClasses; c++) p->tile[c] = best_t[c];
        p->pack_max = best_pm;
        p->pack_groups = best_pg;
        return GC_OK;
    }
    bool present[kClasses] = {};
    for (size_t i = 0; i < p->nlists; i++) present[p->cls[i]] = true;
    std::vector<hipEvent_t> ev(kEvPerSlot);
    gc_status rc = GC_OK;
    for (hipEvent_t &e : ev)
        if (hipEventCreate(&e) != hipSuccess) rc = GC_EDEVICE;
    float best[kClasses];
    for (int c = 0; c < kClasses; c++) best[c] = 1e30f;
    for (int i = 0; i < 3 && !rc; i++) {
        for (int c = 0; c < kClasses; c++) p->tile[c] = kWaveTiles[i];
        rc = plan_materialize(p);   // raises a class's tile to its minimum
        if (!rc) rc = plan_upload(p, d_streams, d_out);
        for (int w = 0; w < 2 && !rc; w++) rc = plan_launch(p, nullptr);
        float acc[kClasses] = {};
        for (int r = 0; r < 5 && !rc; r++) {
            HIP_OK(hipEventRecord(ev[0], nullptr));
            rc = plan_launch(p, nullptr, nullptr, nullptr, nullptr, ev.data() + 2);
            HIP_OK(hipEventRecord(ev[1], nullptr));
            HIP_OK(hipEventSynchronize(ev[1]));
            for (int c = 0; c < kClasses && !rc; c++) {
                if (!present[c] || !p->cr[c].count) continue;
                const hipEvent_t *ce = ev.data() + 2 + 5 * c;
                float ms = 0;
                HIP_OK(hipEventElapsedTime(&ms, ce[2], ce[4]));
                acc[c] += ms;
            }
        }
        for (int c = 0; c < kClasses && !rc; c++) {
            if (present[c] && acc[c] < best[c]) {
                best[c] = acc[c];
                best_t[c] = p->tile[c];
            }
        }
    }
    for (int c = 0; c < kClasses; c++) p->tile[c] = best_t[c];
    if (!p->pack_forced || !p->groups_forced) {
        // the packed-list threshold and the pack kernel's workgroups per CU:
        // three sweeps over the candidates, each timing 8 runs queued back
        // to back (as a caller replays them, so that launching one overlaps
        // the previous), the best sweep kept: the candidates can differ by a
        // few per cent, and interleaving them spreads clock and cache drift
        std::vector<std::pair<uint32_t, uint32_t>> cand;
        const uint32_t pms[4] = {0u, 1024u, kPackInts[0], kPackInts[1]};
        const uint32_t gs[2] = {GC_PACK_GROUPS_ALL, kDefaultPackGroups};
        for (uint32_t pm : pms) {
            if (p->pack_forced && pm != p->pack_max) continue;
            for (uint32_t g : gs) {
                if (p->groups_forced && g != p->pack_groups) continue;
                if (pm == 0u && !cand.empty() && cand.back().first == 0u) continue;   // no packs: one candidate
                cand.emplace_back(pm, p->groups_forced ? p->pack_groups : g);
            }
        }
        if (cand.empty()) cand.emplace_back(p->pack_max, p->pack_groups);
        std::vector<float> best_ms(cand.size(), 1e30f);
        for (int sweep = 0; sweep < 3 && !rc && cand.size() > 1; sweep++) {
            for (size_t i = 0; i < cand.size() && !rc; i++) {
                p->pack_max = cand[i].first;
                p->pack_groups = cand[i].second;
                rc = plan_materialize(p);
                if (!rc) rc = plan_upload(p, d_streams, d_out);
                // a plan replayed from a graph is timed that way: its
                // branches overlap the pack kernel with the other passes
                const bool graph = p->use_graph && !rc;
                if (graph) rc = plan_capture(p);
                auto run = [&]() -> gc_status {
                    if (!graph) return plan_launch(p, nullptr);
                    return hipGraphLaunch(p->exec, nullptr) == hipSuccess ? GC_OK : GC_EDEVICE;
                };
                for (int w = 0; w < 2 && !rc; w++) rc = run();
                HIP_OK(hipEventRecord(ev[0], nullptr));
                for (int r = 0; r < 8 && !rc; r++) rc = run();
                HIP_OK(hipEventRecord(ev[1], nullptr));
                HIP_OK(hipEventSynchronize(ev[1]));
                if (rc) break;
                float ms = 0;
                HIP_OK(hipEventElapsedTime(&ms, ev[0], ev[1]));
                best_ms[i] = std::min(best_ms[i], ms);
            }
        }
        const size_t bi = std::min_element(best_ms.begin(), best_ms.end()) - best_ms.begin();
        best_pm = cand[bi].first;
        best_pg = cand[bi].second;
        plan_free_graphs(p);
        p->pack_max = best_pm;
        p->pack_groups = best_pg;
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    for (int c = 0; c < kClasses; c++) p->tile[c] = best_t[c];
    cache_store(key, best_t, p->pack_max, p->pack_groups);
    return GC_OK;
}

gc_status validate_header(const uint32_t *hd, uint64_t n, uint64_t stream_words) {
    HeaderFields h;
    if (stream_words < 4) return GC_EINVAL;
    if (!header_fields(hd[0], h)) return GC_ECORRUPT;
    if (hd[1] != n || (hd[2] & 3u) || (hd[3] & (uint32_t)(h.k - 1))) return GC_ECORRUPT;
    if (4ull + hd[2] + hd[3] > stream_words) return GC_ECORRUPT;
    // unary Group-Scheme control positions are 32-bit bit offsets
    if (h.codec == GC_SCHEME && h.ld != GC_LD_BINARY && hd[2] >= (1u << 27)) return GC_EUNSUPPORTED;
    return GC_OK;
}

// The descriptor of a list decoded alone, from the host copy of its header;
// *empty when it has no integers (nothing to launch).
gc_status single_list(const gc_ctx *ctx, const uint32_t *d_stream, size_t stream_words, const uint32_t *h_header,
                      uint32_t *d_out, ListDesc &L, int &cls, bool &empty) {
    empty = false;
    if (!d_stream || !h_header || stream_words < 4) return GC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_stream) & 15u) != 0u) return GC_EINVAL;
    const uint32_t n = h_header[1];
    if (gc_status rc = validate_header(h_header, n, stream_words)) return rc;
    if (n == 0) {
        empty = true;
        return GC_OK;
    }
    if (!d_out) return GC_EINVAL;
    cls = codec_class(h_header[0]);
    HeaderFields h;
    header_fields(h_header[0], h);
    const int tile = std::max(cls == kClsPfd ? ctx->tile_p : ctx->tile_w, 32 << h.lk);
    std::memset(&L, 0, sizeof(L));
    L.stream = d_stream;
    L.out = d_out;
    L.stream_words = stream_words;
    L.n = n;
    L.ntiles = (uint32_t)((n + (size_t)tile - 1) / (size_t)tile);
    L.nchunks = L.ntiles > 1 ? list_chunks(h, n, h_header[2], h_header[3], kChunkWordsSmall) : 0u;
    L.tile_ints = (uint32_t)tile;
    L.w0 = h_header[0];
    L.C = h_header[2];
    L.D = h_header[3];
    return GC_OK;
}

}  // namespace

extern "C" {

const char *gc_version(void) { return "libgc 0.3 (gfx950)"; }

gc_status gc_ctx_create(int device, gc_ctx **ctx) { return gc_ctx_create_opts(device, nullptr, ctx); }

gc_status gc_ctx_create_opts(int device, const gc_ctx_opts *opts, gc_ctx **ctx) {
    if (!ctx) return GC_EINVAL;
    *ctx = nullptr;
    uint64_t max_ints = kDefaultMaxListInts;
    if (opts) {
        if (opts->reserved[0] || opts->reserved[1]) return GC_EINVAL;
        if (opts->max_list_ints) max_ints = opts->max_list_ints;
    }
    if (max_ints > 0xFFFFFFFFull) return GC_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return GC_EDEVICE;
    }
    HIP_OK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GC_EUNSUPPORTED;
    gc_ctx *c = new (std::nothrow) gc_ctx();
    if (!c) return GC_ENOMEM;
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->max_list_ints = max_ints;
    c->arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
    gc_status rc = dev_alloc(&c->status, 1);
    if (!rc) rc = c->single.init_state();
    if (!rc) rc = c->single.reserve(single_tiles_cap(max_ints), single_chunks_cap(max_ints));
    if (!rc) rc = c->blk.reserve((size_t)((max_ints + gcblk::kBlockInts - 1) / gcblk::kBlockInts));
    // the fixed scratch of gc_decode_noalloc on this device (set up once)
    void *fixed = nullptr;
    if (!rc && noalloc_setup(device, &fixed)) rc = GC_EDEVICE;
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = GC_EDEVICE;
    if (rc) {
        (void)hipGetLastError();
        dev_free(c->status);
        c->single.release();
        c->blk.release();
        delete c;
        return rc;
    }
    *ctx = c;
    return GC_OK;
}

gc_status gc_ctx_destroy(gc_ctx *ctx) {
    if (!ctx) return GC_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    dev_free(ctx->status);
    ctx->single.release();
    ctx->blk.release();
    delete ctx;
    return GC_OK;
}

gc_status gc_decode(gc_ctx *ctx, const uint32_t *d_stream, size_t stream_words, const uint32_t *h_header,
                               uint32_t *d_out, void *hip_stream) {
    if (!ctx) return GC_EINVAL;
    ListDesc L;
    int cls = 0;
    bool empty = false;
    if (gc_status rc = single_list(ctx, d_stream, stream_words, h_header, d_out, L, cls, empty)) return rc;
    if (empty) return GC_OK;
    // the tables were sized when the context was created: nothing is
    // allocated here, and a list that needs more is refused
    if ((uint64_t)L.n > ctx->max_list_ints || L.ntiles + 1u > ctx->single.tiles_cap ||
        L.nchunks > ctx->single.chunks_cap)
        return GC_ENOSPC;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return launch_one(L, cls, ctx->single, ctx->status, (hipStream_t)hip_stream, kSingleLbMax, kChunkWordsSmall);
}

gc_status gc_decode_noalloc(gc_ctx *ctx, const uint32_t *d_stream, size_t stream_words, const uint32_t *h_header,
                            uint32_t *d_out, void *hip_stream) {
    if (!ctx) return GC_EINVAL;
    ListDesc L;
    int cls = 0;
    bool empty = false;
    if (gc_status rc = single_list(ctx, d_stream, stream_words, h_header, d_out, L, cls, empty)) return rc;
    if (empty) return GC_OK;
    constexpr NoallocLayout lay = noalloc_layout();
    if ((uint64_t)L.n > kNoallocMaxInts || L.ntiles + 1u > lay.tiles_cap || L.nchunks > lay.chunks_cap)
        return GC_ENOSPC;
    uint8_t *base = static_cast<uint8_t *>(noalloc_ptr(ctx->device));
    if (!base) return GC_EDEVICE;
    // a view of the fixed array, in the layout of the context's own tables
    // (nothing here owns or frees it)
    Scratch sc;
    sc.state = reinterpret_cast<RunState *>(base + lay.state);
    sc.tiles = reinterpret_cast<TileInfo *>(base + lay.tiles);
    sc.carry = reinterpret_cast<uint32_t *>(base + lay.carry);
    sc.flags = reinterpret_cast<unsigned long long *>(base + lay.flags);
    sc.agg = reinterpret_cast<LocVal *>(base + lay.agg);
    sc.pre = reinterpret_cast<LocVal *>(base + lay.pre);
    sc.tiles_cap = lay.tiles_cap;
    sc.chunks_cap = lay.chunks_cap;
    return launch_one(L, cls, sc, ctx->status, (hipStream_t)hip_stream, kSingleLbMax, kChunkWordsSmall);
}

gc_status gc_plan_create(gc_ctx *ctx, const gc_list_desc *h_descs, size_t nlists, const uint32_t *h_headers,
                         const gc_plan_opts *opts, const uint32_t *d_streams, uint32_t *d_out, gc_plan **plan) {
    if (!ctx || !plan || (nlists && (!h_descs || !h_headers))) return GC_EINVAL;
    *plan = nullptr;
    if (nlists > 0xFFFFFFFull) return GC_EINVAL;
    gc_plan_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.tile_ints && !valid_wave_tile(o.tile_ints)) return GC_EINVAL;
    if (o.pfd_tile_ints && !valid_wave_tile(o.pfd_tile_ints)) return GC_EINVAL;
    bool forced = o.tile_ints || o.pfd_tile_ints;
    for (int c = 0; c < kClasses; c++) {
        const uint32_t t = o.class_tile_ints[c];
        if (t && !valid_wave_tile(t)) return GC_EINVAL;
        forced = forced || t;
    }
    if (o.schedule > 1u || o.carry_pass > 3u) return GC_EINVAL;
    if (o.pack_ints && o.pack_ints != GC_PACK_OFF && o.pack_ints > kPackInts[1]) return GC_EINVAL;
    if (o.pack_groups && o.pack_groups != GC_PACK_GROUPS_ALL && o.pack_groups > 64u) return GC_EINVAL;
    if ((o.autotune || o.use_graph) && nlists && (!d_streams || !d_out)) return GC_EINVAL;
    gc_plan *p = new (std::nothrow) gc_plan();
    if (!p) return GC_ENOMEM;
    p->ctx = ctx;
    p->nlists = nlists;
    for (int c = 0; c < kClasses; c++) {
        const uint32_t group = c == kClsPfd ? o.pfd_tile_ints : o.tile_ints;
        const int dflt = c == kClsPfd ? kDefaultPfdTile : kDefaultWaveTile;
        p->tile[c] = o.class_tile_ints[c] ? (int)o.class_tile_ints[c] : group ? (int)group : dflt;
    }
    p->use_graph = o.use_graph != 0;
    p->serial = o.schedule == 0u;
    p->pack_forced = o.pack_ints != 0u;
    if (o.graph_serial > 1u) {
        delete p;
        return GC_EINVAL;
    }
    p->branches = o.graph_serial == 0u;
    p->pack_max = o.pack_ints == GC_PACK_OFF ? 0u : o.pack_ints ? o.pack_ints : kDefaultPackMax;
    p->groups_forced = o.pack_groups != 0u;
    if (o.pack_groups) p->pack_groups = o.pack_groups;
    p->lb_max = o.carry_pass == 1u ? kLookbackAll : o.carry_pass == 2u ? 0u
              : o.carry_pass == 3u ? kLookbackHybrid : kDefaultLbMax;
    // tests of the look-back's bounded wait: tiles stop publishing their
    // flags and a look-back gives up after this many 100 MHz ticks
    if (const char *e = std::getenv("GC_TEST_LOOKBACK_STALL")) p->lb_stall = (uint32_t)std::strtoul(e, nullptr, 10);
    p->slots = std::min<uint32_t>(o.timing_slots, 4096u);
    p->h_lists.resize(nlists);
    p->cls.resize(nlists);
    p->stream_off.resize(nlists);
    p->out_off.resize(nlists);
    uint64_t tiles_total = 0;
    for (size_t i = 0; i < nlists; i++) {
        const gc_list_desc &d = h_descs[i];
        gc_status rc = (d.stream_off_words & 3u) ? GC_EINVAL : validate_header(h_headers + 4 * i, d.n, d.stream_words);
        if (rc) {
            delete p;
            return rc;
        }
        ListDesc &L = p->h_lists[i];
        std::memset(&L, 0, sizeof(L));
        L.stream_words = d.stream_words;
        L.n = d.n;
        L.w0 = h_headers[4 * i];
        L.C = h_headers[4 * i + 2];
        L.D = h_headers[4 * i + 3];
        p->cls[i] = codec_class(L.w0);
        p->stream_off[i] = d.stream_off_words;
        p->out_off[i] = d.out_off;
        tiles_total += (d.n + 1023u) / 1024u;
    }
    if (tiles_total > 0xFFFFFFF0ull) {
        delete p;
        return GC_EINVAL;
    }
    (void)hipSetDevice(ctx->device);
    gc_status rc = GC_OK;
    if (o.autotune && nlists && !forced) rc = autotune(p, d_streams, d_out);
    for (uint32_t i = 0; i < (uint32_t)kEvPerSlot * p->slots && !rc; i++) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) rc = GC_EDEVICE;
        else p->ev.push_back(e);
    }
    if (p->slots && !rc && hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking) != hipSuccess) rc = GC_EDEVICE;
    if (!rc) rc = plan_materialize(p);
    if (!rc && d_streams && d_out) rc = plan_upload(p, d_streams, d_out);
    if (!rc && p->use_graph) rc = plan_capture(p);
    if (rc) {
        plan_free_device(p);
        for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
        if (p->aux) (void)hipStreamDestroy(p->aux);
        delete p;
        return rc;
    }
    *plan = p;
    return GC_OK;
}

gc_status gc_plan_destroy(gc_plan *plan) {
    if (!plan) return GC_EINVAL;
    (void)hipSetDevice(plan->ctx->device);
    (void)hipDeviceSynchronize();
    plan_free_device(plan);
    for (hipEvent_t e : plan->ev) (void)hipEventDestroy(e);
    if (plan->aux) (void)hipStreamDestroy(plan->aux);
    delete plan;
    return GC_OK;
}

gc_status gc_decode_batch(gc_plan *plan, const uint32_t *d_streams, uint32_t *d_out, void *hip_stream) {
    if (!plan) return GC_EINVAL;
    if (!plan->nlists) return GC_OK;
    if (!d_streams || !d_out || (reinterpret_cast<uintptr_t>(d_streams) & 15u)) return GC_EINVAL;
    if (d_streams != plan->bound_streams || d_out != plan->bound_out) {
        gc_status rc = plan_upload(plan, d_streams, d_out);
        if (rc) return rc;
    }
    return plan_run(plan, (hipStream_t)hip_stream);
}

gc_status gc_decode_each(gc_plan *plan, const uint32_t *d_streams, uint32_t *d_out, void *hip_stream) {
    if (!plan) return GC_EINVAL;
    if (!d_streams || !d_out || (reinterpret_cast<uintptr_t>(d_streams) & 15u)) return GC_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    for (size_t i = 0; i < plan->nlists; i++) {
        ListDesc L = plan->h_lists[i];
        if (L.n == 0) continue;
        L.stream = d_streams + plan->stream_off[i];
        L.out = d_out + plan->out_off[i];
        if (gc_status rc = launch_one(L, plan->cls[i], plan->sc, plan->ctx->status, s, plan->lb_max, kChunkWords))
            return rc;
    }
    return GC_OK;
}

gc_status gc_plan_timings(gc_plan *plan, uint32_t max_runs, float *ms, uint32_t *nruns) {
    if (!plan || !plan->slots || !ms || !nruns) return GC_EINVAL;
    const uint64_t avail = std::min<uint64_t>(plan->runs, plan->slots);
    const uint32_t n = (uint32_t)std::min<uint64_t>(avail, max_runs);
    for (uint32_t i = 0; i < n; i++) {
        const uint64_t run = plan->runs - n + i;
        hipEvent_t *e = &plan->ev[(size_t)(run % plan->slots) * kEvPerSlot];
        float *row = ms + (size_t)i * GC_TIMING_FIELDS;
        for (int f = 0; f < GC_TIMING_FIELDS; f++) row[f] = 0.0f;
        HIP_OK(hipEventSynchronize(e[1]));
        HIP_OK(hipEventElapsedTime(&row[0], e[0], e[1]));
        const int c0 = first_class(plan);
        for (int c = 0; c < kClasses; c++) {
            if (!plan->cr[c].count) continue;
            hipEvent_t *ce = e + 2 + 5 * c;
            if (!plan->serial || c == c0) HIP_OK(hipEventElapsedTime(&row[1 + c], ce[0], ce[1]));
            HIP_OK(hipEventElapsedTime(&row[1 + kClasses + c], ce[2], ce[3]));
            HIP_OK(hipEventElapsedTime(&row[1 + 2 * kClasses + c], ce[3], ce[4]));
        }
        HIP_OK(hipEventElapsedTime(&row[1 + 3 * kClasses], e[2 + kTevPack], e[2 + kTevPack + 1]));
    }
    *nruns = n;
    return GC_OK;
}

gc_status gc_plan_config(const gc_plan *plan, uint32_t *tile_ints, uint32_t *pfd_tile_ints, uint64_t *tiles,
                         uint64_t *sum_tiles) {
    if (!plan) return GC_EINVAL;
    uint64_t t = 0, st = 0;
    for (int c = 0; c < kClasses; c++) {
        t += plan->cr[c].count;
        st += plan->cr[c].sum;
    }
    int first_wave = 0;   // the first non-PFD class the plan holds
    for (int c = kClasses - 1; c >= 0; c--)
        if (c != kClsPfd && plan->cr[c].count) first_wave = c;
    if (tile_ints) *tile_ints = (uint32_t)plan->tile[first_wave];
    if (pfd_tile_ints) *pfd_tile_ints = (uint32_t)plan->tile[kClsPfd];
    if (tiles) *tiles = t;
    if (sum_tiles) *sum_tiles = st;
    return GC_OK;
}

gc_status gc_plan_pack_config(const gc_plan *plan, uint32_t *pack_ints, uint64_t *packs, uint64_t *packed_lists,
                              uint32_t *pack_groups) {
    if (!plan) return GC_EINVAL;
    uint64_t np = 0, nl = 0;
    for (const PackSet &ps : plan->pk) {
        np += ps.packs();
        nl += ps.h.size();
    }
    if (pack_ints) *pack_ints = plan->pack_max;
    if (packs) *packs = np;
    if (packed_lists) *packed_lists = nl;
    if (pack_groups) *pack_groups = plan->pack_groups;
    return GC_OK;
}

gc_status gc_plan_packed_lists(const gc_plan *plan, uint8_t *h_packed, size_t nlists) {
    if (!plan || !h_packed || nlists != plan->nlists) return GC_EINVAL;
    for (size_t i = 0; i < nlists; i++) h_packed[i] = i < plan->packed.size() ? plan->packed[i] : 0u;
    return GC_OK;
}

gc_status gc_plan_class_tiles(const gc_plan *plan, uint32_t *tile_ints) {
    if (!plan || !tile_ints) return GC_EINVAL;
    for (int c = 0; c < kClasses; c++) tile_ints[c] = (uint32_t)plan->tile[c];
    return GC_OK;
}

gc_status gc_block_features(gc_ctx *ctx, const uint32_t *d_in, size_t nblocks, float *d_feat, void *hip_stream) {
    if (!ctx || (nblocks && (!d_in || !d_feat))) return GC_EINVAL;
    if (nblocks > 0xFFFFFFFFull) return GC_EINVAL;
    (void)hipSetDevice(ctx->device);
    return gcblk::launch_block_features(d_in, nblocks, d_feat, (hipStream_t)hip_stream) ? GC_EDEVICE : GC_OK;
}

gc_status gc_block_sizes(gc_ctx *ctx, const uint32_t *d_in, size_t nblocks, uint32_t *d_sizes, uint8_t *d_best,
                         float *d_cost,
                         void *hip_stream) {
    if (!ctx || (nblocks && !d_in)) return GC_EINVAL;
    if (nblocks > 0xFFFFFFFFull) return GC_EINVAL;
    if (!d_sizes && !d_best && !d_cost) return GC_OK;
    (void)hipSetDevice(ctx->device);
    return gcblk::launch_block_sizes(d_in, nblocks, d_sizes, d_best, d_cost, (hipStream_t)hip_stream) ? GC_EDEVICE : GC_OK;
}

size_t gc_blockmix_bound_words(size_t n) {
    const size_t nb = (n + gcblk::kBlockInts - 1) / gcblk::kBlockInts;
    return 4 + nb * (1 + (size_t)gcblk::kMaxPayloadWords);
}

// The container of d_in with block b in class cls[b]; ctx->mu held.
static gc_status blockmix_encode_locked(gc_ctx *ctx, const uint32_t *d_in, size_t n, size_t nb, const uint8_t *cls,
                                        uint32_t *d_out, size_t out_cap_words, size_t *out_words, hipStream_t s) {
    // sizes, their scan, then the writes, with no host round trip between:
    // the emit pass writes the header and keeps within the capacity, and
    // the total and the class check come back at the end
    uint32_t res[2] = {0u, 0u};
    if (nb) {
        if (gcblk::launch_blockmix_plan(d_in, nb, cls, ctx->blk.words, ctx->blk.offs, ctx->blk.csum, ctx->blk.result,
                                        s))
            return GC_EDEVICE;
        if (gcblk::launch_blockmix_emit(d_in, nb, cls, ctx->blk.offs, d_out, out_cap_words, (uint32_t)n,
                                        ctx->blk.result, s))
            return GC_EDEVICE;
        HIP_OK(hipMemcpyAsync(res, ctx->blk.result, sizeof(res), hipMemcpyDeviceToHost, s));
    } else {
        const uint32_t hdr[4] = {GC_FMT_VERSION | (4u << 8) | (2u << 12), (uint32_t)n, 0u, 0u};
        HIP_OK(hipMemcpyAsync(d_out, hdr, sizeof(hdr), hipMemcpyHostToDevice, s));
    }
    HIP_OK(hipStreamSynchronize(s));
    if (res[1]) return GC_EINVAL;
    const size_t total = 4 + nb + (size_t)res[0];
    if (total > out_cap_words) return GC_ENOSPC;
    *out_words = total;
    return GC_OK;
}

gc_status gc_blockmix_encode(gc_ctx *ctx, const uint32_t *d_in, size_t n, const uint8_t *d_class, uint32_t *d_out,
                             size_t out_cap_words, size_t *out_words, void *hip_stream) {
    if (!ctx || !out_words || !d_out || (n && (!d_in || !d_class))) return GC_EINVAL;
    // offsets and the total are 32-bit words
    if (gc_blockmix_bound_words(n) > 0xFFFFFFFFull) return GC_EINVAL;
    const size_t nb = (n + gcblk::kBlockInts - 1) / gcblk::kBlockInts;
    if (out_cap_words < 4 + nb) return GC_ENOSPC;
    if (n > ctx->max_list_ints || nb > ctx->blk.cap) return GC_ENOSPC;   // sized when the context was created
    (void)hipSetDevice(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    return blockmix_encode_locked(ctx, d_in, n, nb, d_class, d_out, out_cap_words, out_words,
                                  (hipStream_t)hip_stream);
}

// ---- selector network ----------------------------------------------------------

struct gc_mlp {
    int device = 0;
    float *theta = nullptr, *m = nullptr, *v = nullptr, *partial = nullptr;
    uint16_t *wbuf = nullptr;
    gcmlp::Packed w{};
    uint32_t max_batch = 0;
    uint64_t step = 0;
    std::mutex mu;
};

static constexpr size_t kPackedHalves = 64 * 48 + 64 * 64 * 2 + 16 * 64 * 2;

gc_status gc_mlp_create(gc_ctx *ctx, uint32_t max_batch, gc_mlp **out) {
    if (!ctx || !out || !max_batch) return GC_EINVAL;
    *out = nullptr;
    (void)hipSetDevice(ctx->device);
    gc_mlp *m = new (std::nothrow) gc_mlp();
    if (!m) return GC_ENOMEM;
    m->device = ctx->device;
    m->max_batch = max_batch;
    const size_t groups = ((size_t)max_batch + gcmlp::kRows - 1) / gcmlp::kRows;
    gc_status rc = dev_alloc(&m->theta, gcmlp::kParams);
    if (!rc) rc = dev_alloc(&m->m, gcmlp::kParams);
    if (!rc) rc = dev_alloc(&m->v, gcmlp::kParams);
    if (!rc) rc = dev_alloc(&m->partial, groups * gcmlp::kPartialStride);
    if (!rc) rc = dev_alloc(&m->wbuf, kPackedHalves);
    if (!rc && (hipMemset(m->theta, 0, gcmlp::kParams * 4) != hipSuccess ||
                hipMemset(m->m, 0, gcmlp::kParams * 4) != hipSuccess ||
                hipMemset(m->v, 0, gcmlp::kParams * 4) != hipSuccess ||
                hipMemset(m->wbuf, 0, kPackedHalves * 2) != hipSuccess || hipDeviceSynchronize() != hipSuccess))
        rc = GC_EDEVICE;
    if (rc) {
        gc_mlp_destroy(m);
        return rc;
    }
    m->w.w1t = m->wbuf;
    m->w.w2t = m->w.w1t + 64 * 48;
    m->w.w2 = m->w.w2t + 64 * 64;
    m->w.w3t = m->w.w2 + 64 * 64;
    m->w.w3 = m->w.w3t + 16 * 64;
    *out = m;
    return GC_OK;
}

gc_status gc_mlp_destroy(gc_mlp *m) {
    if (!m) return GC_EINVAL;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    dev_free(m->theta);
    dev_free(m->m);
    dev_free(m->v);
    dev_free(m->partial);
    dev_free(m->wbuf);
    delete m;
    return GC_OK;
}

size_t gc_mlp_param_count(void) { return gcmlp::kParams; }

gc_status gc_mlp_set_params(gc_mlp *m, const float *h_theta, size_t count, void *hip_stream) {
    if (!m || !h_theta || count != (size_t)gcmlp::kParams) return GC_EINVAL;
    (void)hipSetDevice(m->device);
    std::lock_guard<std::mutex> lk(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_OK(hipMemcpyAsync(m->theta, h_theta, count * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemsetAsync(m->m, 0, count * 4, s));
    HIP_OK(hipMemsetAsync(m->v, 0, count * 4, s));
    if (gcmlp::launch_pack(m->theta, m->w, s)) return GC_EDEVICE;
    HIP_OK(hipStreamSynchronize(s));
    m->step = 0;
    return GC_OK;
}

gc_status gc_mlp_get_params(gc_mlp *m, float *h_theta, size_t count, void *hip_stream) {
    if (!m || !h_theta || count != (size_t)gcmlp::kParams) return GC_EINVAL;
    (void)hipSetDevice(m->device);
    std::lock_guard<std::mutex> lk(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_OK(hipMemcpyAsync(h_theta, m->theta, count * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return GC_OK;
}

gc_status gc_mlp_get_state(gc_mlp *m, float *h_state, size_t count, uint64_t *h_step, void *hip_stream) {
    const size_t P = gcmlp::kParams;
    if (!m || !h_state || !h_step || count != 3 * P) return GC_EINVAL;
    (void)hipSetDevice(m->device);
    std::lock_guard<std::mutex> lk(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_OK(hipMemcpyAsync(h_state, m->theta, P * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(h_state + P, m->m, P * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(h_state + 2 * P, m->v, P * 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *h_step = m->step;
    return GC_OK;
}

gc_status gc_mlp_set_state(gc_mlp *m, const float *h_state, size_t count, uint64_t step, void *hip_stream) {
    const size_t P = gcmlp::kParams;
    if (!m || !h_state || count != 3 * P) return GC_EINVAL;
    (void)hipSetDevice(m->device);
    std::lock_guard<std::mutex> lk(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_OK(hipMemcpyAsync(m->theta, h_state, P * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(m->m, h_state + P, P * 4, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(m->v, h_state + 2 * P, P * 4, hipMemcpyHostToDevice, s));
    if (gcmlp::launch_pack(m->theta, m->w, s)) return GC_EDEVICE;
    HIP_OK(hipStreamSynchronize(s));
    m->step = step;
    return GC_OK;
}

gc_status gc_mlp_forward(gc_mlp *m, const float *d_feat, size_t n, float *d_logits, uint8_t *d_class,
                         void *hip_stream) {
    if (!m || (n && !d_feat) || n > 0xFFFFFFFFull) return GC_EINVAL;
    (void)hipSetDevice(m->device);
    return gcmlp::launch_forward(d_feat, n, m->theta, m->w, d_logits, d_class, (hipStream_t)hip_stream) ? GC_EDEVICE
                                                                                                         : GC_OK;
}

gc_status gc_mlp_grad(gc_mlp *m, const float *d_feat, const uint8_t *d_label, const float *d_cost,
                      const uint32_t *d_index, uint32_t batch, float lam, float *d_grad, float *d_loss,
                      void *hip_stream) {
    if (!m || !batch || batch > m->max_batch || !d_feat || !d_label || (lam != 0.f && !d_cost)) return GC_EINVAL;
    (void)hipSetDevice(m->device);
    std::lock_guard<std::mutex> lk(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    const gcmlp::Batch b = {d_feat, d_index, d_label, lam != 0.f ? d_cost : nullptr, 0, batch, lam};
    const uint32_t parts = (batch + gcmlp::kRows - 1) / gcmlp::kRows;
    if (gcmlp::launch_grad_partials(b, m->theta, m->w, m->partial, s)) return GC_EDEVICE;
    if (gcmlp::launch_reduce_adam(m->partial, parts, d_grad, d_loss, m->theta, m->m, m->v, m->w, false, 0.f, 0.f,
                                  0.f, 0.f, 0.f, 0.f, s))
        return GC_EDEVICE;
    return GC_OK;
}

gc_status gc_mlp_train(gc_mlp *m, const float *d_feat, const uint8_t *d_label, const float *d_cost,
                       const uint32_t *d_index, size_t nindex, const gc_adam_opts *opt, float *d_loss,
                       void *hip_stream) {
    if (!m || !opt || !d_feat || !d_label || !opt->batch || opt->batch > m->max_batch) return GC_EINVAL;
    if (opt->lam != 0.f && !d_cost) return GC_EINVAL;
    if (!(opt->lr > 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) || !(opt->beta2 >= 0.f && opt->beta2 < 1.f) ||
        !(opt->eps > 0.f))
        return GC_EINVAL;
    (void)hipSetDevice(m->device);
    std::lock_guard<std::mutex> lk(m->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    size_t k = 0;
    for (size_t row0 = 0; row0 < nindex; row0 += opt->batch, k++) {
        const uint32_t count = (uint32_t)std::min<size_t>(opt->batch, nindex - row0);
        const gcmlp::Batch b = {d_feat, d_index, d_label, opt->lam != 0.f ? d_cost : nullptr, row0, count, opt->lam};
        const uint64_t t = ++m->step;
        const float c1 = (float)(1.0 / (1.0 - std::pow((double)opt->beta1, (double)t)));
        const float c2 = (float)(1.0 / (1.0 - std::pow((double)opt->beta2, (double)t)));
        if (gcmlp::launch_grad_partials(b, m->theta, m->w, m->partial, s)) return GC_EDEVICE;
        if (gcmlp::launch_reduce_adam(m->partial, (count + gcmlp::kRows - 1) / gcmlp::kRows, nullptr,
                                      d_loss ? d_loss + k : nullptr, m->theta, m->m, m->v, m->w, true, opt->lr,
                                      opt->beta1, opt->beta2, opt->eps, c1, c2, s))
            return GC_EDEVICE;
    }
    return GC_OK;
}

gc_status gc_encode_blocks(gc_ctx *ctx, const uint32_t *d_in, size_t n, int mode, gc_mlp *model,
                           uint32_t fixed_class, uint32_t *d_out, size_t out_cap_words, size_t *out_words,
                           uint8_t *d_class_out, void *hip_stream) {
    if (!ctx || !out_words || !d_out || (n && !d_in)) return GC_EINVAL;
    if (mode == GC_SELECT_LEARNED && (!model || model->device != ctx->device)) return GC_EINVAL;
    if (mode == GC_SELECT_FIXED && fixed_class >= (uint32_t)gcblk::kClasses) return GC_EINVAL;
    if (mode != GC_SELECT_EXHAUSTIVE && mode != GC_SELECT_LEARNED && mode != GC_SELECT_FIXED) return GC_EINVAL;
    if (gc_blockmix_bound_words(n) > 0xFFFFFFFFull) return GC_EINVAL;
    const size_t nb = (n + gcblk::kBlockInts - 1) / gcblk::kBlockInts;
    if (out_cap_words < 4 + nb) return GC_ENOSPC;
    if (n > ctx->max_list_ints || nb > ctx->blk.cap) return GC_ENOSPC;   // sized when the context was created
    (void)hipSetDevice(ctx->device);
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    uint8_t *cls = d_class_out;
    if (nb) {
        if (!cls) cls = ctx->blk.cls;
        int err = 0;
        if (mode == GC_SELECT_EXHAUSTIVE) {
            err = gcblk::launch_block_sizes(d_in, nb, nullptr, cls, nullptr, s);
        } else if (mode == GC_SELECT_LEARNED) {
            std::lock_guard<std::mutex> lm(model->mu);
            err = gcblk::launch_block_features(d_in, nb, ctx->blk.feat, s);
            if (!err) err = gcmlp::launch_forward(ctx->blk.feat, nb, model->theta, model->w, nullptr, cls, s);
        } else {
            err = hipMemsetAsync(cls, (int)fixed_class, nb, s) != hipSuccess;
        }
        if (err) return GC_EDEVICE;
    }
    return blockmix_encode_locked(ctx, d_in, n, nb, cls, d_out, out_cap_words, out_words, s);
}

gc_status gc_sync_status(gc_ctx *ctx, void *hip_stream, uint32_t *detail) {
    if (!ctx) return GC_EINVAL;
    HIP_OK(hipStreamSynchronize((hipStream_t)hip_stream));
    Status h = {0, 0};
    HIP_OK(hipMemcpy(&h, ctx->status, sizeof(h), hipMemcpyDeviceToHost));
    if (h.code) {
        Status z = {0, 0};
        HIP_OK(hipMemcpy(ctx->status, &z, sizeof(z), hipMemcpyHostToDevice));
    }
    if (detail) *detail = h.detail;
    return h.code ? (gc_status)(int32_t)h.code : GC_OK;
}

}  // extern "C"
