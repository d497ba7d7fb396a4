// runtime.cpp -- host runtime of libgc: device contexts, single-list decode,
// batched decode plans (work-item tables per codec class, persistent launches,
// hipGraph capture with one parallel branch per class), per-run kernel timing
// and the autotuner that picks the tile size and occupancy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "gc.h"
#include "gc_device.h"
#include "gc_format.h"

namespace gcdev {
int codec_class(uint32_t w0);
int launch_locate(const LocateArgs &a, uint32_t grid, hipStream_t s);
int launch_decode(int tile, int cls, const DecodeArgs &a, uint32_t grid, hipStream_t s);
int decode_occupancy(int tile, int cls, int *blocks_per_cu);
int locate_occupancy(int *blocks_per_cu);
}  // namespace gcdev

using namespace gcdev;

namespace {

constexpr int kDefaultTile = 2048;
constexpr int kTiles[3] = {2048, 4096, 8192};

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
    case 2: return C;
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
    if (hipMemset(*p, 0, count * sizeof(T)) != hipSuccess) return GC_EDEVICE;
    return GC_OK;
}

template <typename T>
void dev_free(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Look-back and queue state of one launch sequence.
struct Scratch {
    RunState *state = nullptr;          // [0] locate, [1 + class] decode
    TileInfo *tiles = nullptr;
    unsigned long long *tflags = nullptr;
    uint32_t *cflags = nullptr;
    LocVal *agg = nullptr, *incl = nullptr;
    size_t tiles_cap = 0, chunks_cap = 0;

    gc_status init_state() {
        gc_status rc = dev_alloc(&state, 1 + kClasses);
        if (rc) return rc;
        std::vector<RunState> h(1 + kClasses, RunState{0, 0, 1, 0});
        HIP_OK(hipMemcpy(state, h.data(), h.size() * sizeof(RunState), hipMemcpyHostToDevice));
        return GC_OK;
    }
    gc_status reserve(size_t ntiles, size_t nchunks) {
        if (ntiles > tiles_cap) {
            HIP_OK(hipDeviceSynchronize());
            dev_free(tiles);
            dev_free(tflags);
            const size_t cap = std::max(ntiles, tiles_cap * 2);
            gc_status rc = dev_alloc(&tiles, cap);
            if (!rc) rc = dev_alloc(&tflags, cap);
            if (rc) return rc;
            tiles_cap = cap;
        }
        if (nchunks > chunks_cap) {
            HIP_OK(hipDeviceSynchronize());
            dev_free(cflags);
            dev_free(agg);
            dev_free(incl);
            const size_t cap = std::max(nchunks, chunks_cap * 2);
            gc_status rc = dev_alloc(&cflags, cap);
            if (!rc) rc = dev_alloc(&agg, cap);
            if (!rc) rc = dev_alloc(&incl, cap);
            if (rc) return rc;
            chunks_cap = cap;
        }
        return GC_OK;
    }
    void release() {
        dev_free(state);
        dev_free(tiles);
        dev_free(tflags);
        dev_free(cflags);
        dev_free(agg);
        dev_free(incl);
        tiles_cap = chunks_cap = 0;
    }
};

}  // namespace

struct gc_ctx {
    int device = 0;
    int num_cus = 0;
    Status *status = nullptr;
    Scratch single;
    int tile = kDefaultTile;
    std::mutex mu;
};

struct gc_plan {
    gc_ctx *ctx = nullptr;
    size_t nlists = 0;
    int tile = kDefaultTile;
    uint32_t bpc = 0;                          // decode workgroups per CU (0 = max)
    uint32_t grid_a = 0, grid_b[kClasses] = {};
    uint32_t total_a = 0, total_b[kClasses] = {};
    bool use_graph = false;
    std::vector<ListDesc> h_lists;             // pointers filled at upload
    std::vector<int> cls;                      // codec class per list
    std::vector<uint64_t> stream_off, out_off;
    std::vector<uint32_t> item_a, item_b[kClasses];
    ListDesc *d_lists = nullptr;
    uint32_t *d_item_a = nullptr, *d_item_b[kClasses] = {};
    Scratch sc;
    const uint32_t *bound_streams = nullptr;
    uint32_t *bound_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_a = nullptr, graph_b = nullptr;    // timing: one graph per kernel group
    hipGraphExec_t exec_a = nullptr, exec_b = nullptr;
    std::vector<hipEvent_t> ev;                // 3 per timing slot
    uint32_t slots = 0;
    uint64_t runs = 0;
};

namespace {

int occupancy_decode(int tile, int cls) {
    int b = 0;
    if (decode_occupancy(tile, cls, &b) != 0 || b < 1) b = 1;
    return b;
}

int occupancy_locate() {
    int b = 0;
    if (locate_occupancy(&b) != 0 || b < 1) b = 1;
    return b;
}

LocateArgs make_locate_args(const ListDesc *lists, const uint32_t *item_list, const ListDesc &single,
                            uint32_t total, int tile, Scratch &sc, Status *st) {
    LocateArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lists = lists;
    a.item_list = item_list;
    a.single = single;
    a.total_items = total;
    a.tile_ints = (uint32_t)tile;
    a.tiles = sc.tiles;
    a.flags = sc.cflags;
    a.agg = sc.agg;
    a.incl = sc.incl;
    a.state = sc.state;
    a.status = st;
    return a;
}

DecodeArgs make_decode_args(const ListDesc *lists, const uint32_t *item_list, const ListDesc &single,
                            uint32_t total, int cls, Scratch &sc, Status *st) {
    DecodeArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lists = lists;
    a.item_list = item_list;
    a.single = single;
    a.total_items = total;
    a.tiles = sc.tiles;
    a.flags = sc.tflags;
    a.state = sc.state + 1 + cls;
    a.loc_state = sc.state;
    a.status = st;
    return a;
}

uint32_t list_chunks(const HeaderFields &h, uint32_t n, uint32_t C, uint32_t D) {
    const uint32_t T = (n + (uint32_t)h.k - 1u) >> h.lk;
    const uint32_t nw = locate_words_host(h, T, C, D);
    return std::max(1u, (nw + kChunkWords - 1u) / kChunkWords);
}

// Builds the per-list work tables of a plan for one tile size.
void build_tables(gc_plan *p, const uint32_t *h_headers) {
    p->item_a.clear();
    for (auto &v : p->item_b) v.clear();
    uint32_t tb = 0, cb = 0;
    for (size_t i = 0; i < p->nlists; i++) {
        ListDesc &L = p->h_lists[i];
        L.ntiles = (uint32_t)((L.n + (uint64_t)p->tile - 1) / (uint64_t)p->tile);
        L.tile_base = tb;
        L.chunk_base = cb;
        L.nchunks = 0;
        if (L.ntiles > 1) {
            HeaderFields h;
            header_fields(h_headers[4 * i], h);
            L.nchunks = list_chunks(h, L.n, h_headers[4 * i + 2], h_headers[4 * i + 3]);
        }
        L.cls_base = (uint32_t)p->item_b[p->cls[i]].size();
        for (uint32_t c = 0; c < L.nchunks; c++) p->item_a.push_back((uint32_t)i);
        for (uint32_t t = 0; t < L.ntiles; t++) p->item_b[p->cls[i]].push_back((uint32_t)i);
        tb += L.ntiles;
        cb += L.nchunks;
    }
    p->total_a = (uint32_t)p->item_a.size();
    for (int c = 0; c < kClasses; c++) p->total_b[c] = (uint32_t)p->item_b[c].size();
}

void plan_free_graphs(gc_plan *p) {
    for (hipGraphExec_t *e : {&p->exec, &p->exec_a, &p->exec_b})
        if (*e) (void)hipGraphExecDestroy(*e), *e = nullptr;
    for (hipGraph_t *g : {&p->graph, &p->graph_a, &p->graph_b})
        if (*g) (void)hipGraphDestroy(*g), *g = nullptr;
}

void plan_free_device(gc_plan *p) {
    plan_free_graphs(p);
    dev_free(p->d_lists);
    dev_free(p->d_item_a);
    for (auto &d : p->d_item_b) dev_free(d);
    p->sc.release();
}

gc_status plan_upload(gc_plan *p, const uint32_t *d_streams, uint32_t *d_out) {
    std::vector<ListDesc> t(p->h_lists);
    for (size_t i = 0; i < p->nlists; i++) {
        t[i].stream = d_streams + p->stream_off[i];
        t[i].out = d_out + p->out_off[i];
    }
    HIP_OK(hipMemcpy(p->d_lists, t.data(), t.size() * sizeof(ListDesc), hipMemcpyHostToDevice));
    p->bound_streams = d_streams;
    p->bound_out = d_out;
    return GC_OK;
}

// Allocates the device side of a plan for its current tile size.
gc_status plan_materialize(gc_plan *p, const uint32_t *h_headers) {
    plan_free_device(p);
    build_tables(p, h_headers);
    gc_status rc = dev_alloc(&p->d_lists, p->nlists);
    if (!rc) rc = dev_alloc(&p->d_item_a, p->total_a);
    for (int c = 0; c < kClasses && !rc; c++) rc = dev_alloc(&p->d_item_b[c], p->total_b[c]);
    if (!rc) rc = p->sc.init_state();
    uint32_t tiles = 0;
    for (int c = 0; c < kClasses; c++) tiles += p->total_b[c];
    if (!rc) rc = p->sc.reserve(tiles, p->total_a);
    if (rc) return rc;
    if (p->total_a)
        HIP_OK(hipMemcpy(p->d_item_a, p->item_a.data(), p->total_a * 4, hipMemcpyHostToDevice));
    const uint32_t cus = (uint32_t)p->ctx->num_cus;
    for (int c = 0; c < kClasses; c++) {
        if (p->total_b[c])
            HIP_OK(hipMemcpy(p->d_item_b[c], p->item_b[c].data(), p->total_b[c] * 4, hipMemcpyHostToDevice));
        const uint32_t occ = (uint32_t)occupancy_decode(p->tile, c);
        const uint32_t bpc = p->bpc ? std::min(p->bpc, occ) : occ;
        p->grid_b[c] = std::max(1u, std::min(p->total_b[c], bpc * cus));
    }
    p->grid_a = std::max(1u, std::min(p->total_a, (uint32_t)occupancy_locate() * cus));
    return GC_OK;
}

// Launches the locate kernel (which & 1) and the decode kernels (which & 2)
// on stream s; with `fork` streams the decode classes run as parallel
// branches that s waits for.
gc_status plan_launch(gc_plan *p, hipStream_t s, int which, hipStream_t *fork = nullptr,
                      hipEvent_t *fev = nullptr) {
    ListDesc none;
    std::memset(&none, 0, sizeof(none));
    if (p->total_a && (which & 1)) {
        LocateArgs a = make_locate_args(p->d_lists, p->d_item_a, none, p->total_a, p->tile, p->sc,
                                        p->ctx->status);
        if (launch_locate(a, p->grid_a, s)) return GC_EDEVICE;
    }
    if (!(which & 2)) return GC_OK;
    int nact = 0;
    for (int c = 0; c < kClasses; c++) nact += p->total_b[c] ? 1 : 0;
    const bool par = fork && nact > 1;
    if (par) HIP_OK(hipEventRecord(fev[kClasses], s));
    for (int c = 0; c < kClasses; c++) {
        if (!p->total_b[c]) continue;
        hipStream_t cs = s;
        if (par) {
            cs = fork[c];
            HIP_OK(hipStreamWaitEvent(cs, fev[kClasses], 0));
        }
        DecodeArgs d = make_decode_args(p->d_lists, p->d_item_b[c], none, p->total_b[c], c, p->sc,
                                        p->ctx->status);
        if (launch_decode(p->tile, c, d, p->grid_b[c], cs)) return GC_EDEVICE;
        if (par) {
            HIP_OK(hipEventRecord(fev[c], cs));
            HIP_OK(hipStreamWaitEvent(s, fev[c], 0));
        }
    }
    return GC_OK;
}

gc_status capture_one(gc_plan *p, int which, hipGraph_t *graph, hipGraphExec_t *exec) {
    hipStream_t s, fork[kClasses];
    hipEvent_t fev[kClasses + 1];
    HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    for (int c = 0; c < kClasses; c++) HIP_OK(hipStreamCreateWithFlags(&fork[c], hipStreamNonBlocking));
    for (int c = 0; c <= kClasses; c++) HIP_OK(hipEventCreateWithFlags(&fev[c], hipEventDisableTiming));
    gc_status rc = GC_OK;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = GC_EDEVICE;
    } else {
        rc = plan_launch(p, s, which, fork, fev);
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(s, &g) != hipSuccess || rc) {
            rc = GC_EDEVICE;
            if (g) (void)hipGraphDestroy(g);
        } else {
            *graph = g;
            if (hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) rc = GC_EDEVICE;
        }
    }
    for (int c = 0; c <= kClasses; c++) (void)hipEventDestroy(fev[c]);
    for (int c = 0; c < kClasses; c++) (void)hipStreamDestroy(fork[c]);
    (void)hipStreamDestroy(s);
    (void)hipGetLastError();
    return rc;
}

gc_status plan_capture(gc_plan *p) {
    plan_free_graphs(p);
    if (p->slots) {
        gc_status rc = capture_one(p, 1, &p->graph_a, &p->exec_a);
        return rc ? rc : capture_one(p, 2, &p->graph_b, &p->exec_b);
    }
    return capture_one(p, 3, &p->graph, &p->exec);
}

gc_status plan_run(gc_plan *p, hipStream_t s) {
    if (p->slots) {
        const size_t k = (size_t)(p->runs % p->slots) * 3;
        p->runs++;
        HIP_OK(hipEventRecord(p->ev[k], s));
        if (p->use_graph && p->exec_a) HIP_OK(hipGraphLaunch(p->exec_a, s));
        else if (gc_status rc = plan_launch(p, s, 1)) return rc;
        HIP_OK(hipEventRecord(p->ev[k + 1], s));
        if (p->use_graph && p->exec_b) HIP_OK(hipGraphLaunch(p->exec_b, s));
        else if (gc_status rc = plan_launch(p, s, 2)) return rc;
        HIP_OK(hipEventRecord(p->ev[k + 2], s));
        return GC_OK;
    }
    if (p->use_graph && p->exec) {
        HIP_OK(hipGraphLaunch(p->exec, s));
        return GC_OK;
    }
    return plan_launch(p, s, 3);
}

// ---- autotune cache: one JSON object {key: [tile, bpc], ...} -------------
std::string cache_path() {
    const char *e = std::getenv("GC_AUTOTUNE_CACHE");
    return e ? std::string(e) : std::string();
}

bool cache_lookup(const std::string &key, int &tile, uint32_t &bpc) {
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
    int t = 0, b = 0;
    if (std::sscanf(s.c_str() + at + pat.size(), "%d, %d", &t, &b) != 2) return false;
    if (t != 2048 && t != 4096 && t != 8192) return false;
    tile = t;
    bpc = (uint32_t)b;
    return true;
}

void cache_store(const std::string &key, int tile, uint32_t bpc) {
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
    char buf[64];
    std::snprintf(buf, sizeof(buf), "[%d, %u]", tile, bpc);
    entries.push_back("\"" + key + "\": " + buf);
    std::ofstream f(path);
    f << "{\n";
    for (size_t i = 0; i < entries.size(); i++) f << "  " << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
    f << "}\n";
}

std::string plan_key(const gc_plan *p, const uint32_t *h_headers) {
    uint64_t total = 0, per_cls[kClasses] = {};
    int lk = 2;
    for (size_t i = 0; i < p->nlists; i++) {
        HeaderFields h;
        header_fields(h_headers[4 * i], h);
        per_cls[p->cls[i]] += p->h_lists[i].n;
        total += p->h_lists[i].n;
        lk = std::max(lk, h.lk);
    }
    int lg = 0;
    while ((1ull << lg) < total) lg++;
    const uint64_t mean = p->nlists ? total / p->nlists : 0;
    int lm = 0;
    while ((1ull << lm) < mean) lm++;
    std::string key = "gfx950:k" + std::to_string(1 << lk) + ":n2^" + std::to_string(lg) + ":mean2^" +
                      std::to_string(lm) + ":mix";
    for (int c = 0; c < kClasses; c++)
        key += (c ? "-" : "") + std::to_string(total ? per_cls[c] * 8 / total : 0);
    return key;
}

gc_status autotune(gc_plan *p, const uint32_t *h_headers, const uint32_t *d_streams, uint32_t *d_out) {
    const std::string key = plan_key(p, h_headers);
    int best_tile = p->tile;
    uint32_t best_bpc = 0;
    if (cache_lookup(key, best_tile, best_bpc)) {
        p->tile = best_tile;
        p->bpc = best_bpc;
        return GC_OK;
    }
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    float best = 1e30f;
    gc_status rc = GC_OK;
    for (int tile : kTiles) {
        int occ = 1;
        for (int c = 0; c < kClasses; c++) occ = std::max(occ, occupancy_decode(tile, c));
        for (int bpc = occ; bpc >= 1 && !rc; bpc = bpc > 2 ? bpc - 2 : bpc - 1) {
            p->tile = tile;
            p->bpc = (uint32_t)bpc;
            rc = plan_materialize(p, h_headers);
            if (!rc) rc = plan_upload(p, d_streams, d_out);
            if (rc) break;
            for (int w = 0; w < 2 && !rc; w++) rc = plan_launch(p, nullptr, 3);
            if (rc) break;
            HIP_OK(hipEventRecord(e0, nullptr));
            for (int r = 0; r < 5 && !rc; r++) rc = plan_launch(p, nullptr, 3);
            HIP_OK(hipEventRecord(e1, nullptr));
            HIP_OK(hipEventSynchronize(e1));
            float ms = 0;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_tile = tile;
                best_bpc = (uint32_t)bpc;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    p->tile = best_tile;
    p->bpc = best_bpc;
    cache_store(key, best_tile, best_bpc);
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

}  // namespace

extern "C" {

const char *gc_version(void) { return "libgc 0.2 (gfx950)"; }

gc_status gc_ctx_create(int device, gc_ctx **ctx) {
    if (!ctx) return GC_EINVAL;
    *ctx = nullptr;
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
    gc_status rc = dev_alloc(&c->status, 1);
    if (!rc) rc = c->single.init_state();
    if (rc) {
        dev_free(c->status);
        c->single.release();
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
    delete ctx;
    return GC_OK;
}

gc_status gc_decode(gc_ctx *ctx, const uint32_t *d_stream, size_t stream_words, const uint32_t *h_header,
                    uint32_t *d_out, void *hip_stream) {
    if (!ctx || !d_stream || !h_header || stream_words < 4) return GC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(d_stream) & 15u) != 0u) return GC_EINVAL;
    const uint32_t n = h_header[1];
    if (gc_status rc = validate_header(h_header, n, stream_words)) return rc;
    if (n == 0) return GC_OK;
    if (!d_out) return GC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = (hipStream_t)hip_stream;
    const int tile = ctx->tile;
    const int cls = codec_class(h_header[0]);
    const uint32_t ntiles = (uint32_t)((n + (size_t)tile - 1) / (size_t)tile);
    HeaderFields h;
    header_fields(h_header[0], h);
    const uint32_t nchunks = ntiles > 1 ? list_chunks(h, n, h_header[2], h_header[3]) : 0u;
    gc_status rc = ctx->single.reserve(ntiles, nchunks);
    if (rc) return rc;
    ListDesc L;
    std::memset(&L, 0, sizeof(L));
    L.stream = d_stream;
    L.out = d_out;
    L.stream_words = stream_words;
    L.n = n;
    L.ntiles = ntiles;
    L.nchunks = nchunks;
    const uint32_t cus = (uint32_t)ctx->num_cus;
    if (ntiles > 1) {
        LocateArgs a = make_locate_args(nullptr, nullptr, L, 0, tile, ctx->single, ctx->status);
        if (launch_locate(a, std::max(1u, std::min(nchunks, (uint32_t)occupancy_locate() * cus)), s))
            return GC_EDEVICE;
    }
    DecodeArgs d = make_decode_args(nullptr, nullptr, L, 0, cls, ctx->single, ctx->status);
    const uint32_t g = std::max(1u, std::min(ntiles, (uint32_t)occupancy_decode(tile, cls) * cus));
    if (launch_decode(tile, cls, d, g, s)) return GC_EDEVICE;
    return GC_OK;
}

gc_status gc_plan_create(gc_ctx *ctx, const gc_list_desc *h_descs, size_t nlists, const uint32_t *h_headers,
                         const gc_plan_opts *opts, const uint32_t *d_streams, uint32_t *d_out, gc_plan **plan) {
    if (!ctx || !plan || (nlists && (!h_descs || !h_headers))) return GC_EINVAL;
    *plan = nullptr;
    if (nlists > 0xFFFFFFFull) return GC_EINVAL;
    gc_plan_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.tile_ints && o.tile_ints != 2048 && o.tile_ints != 4096 && o.tile_ints != 8192) return GC_EINVAL;
    if ((o.autotune || o.use_graph) && nlists && (!d_streams || !d_out)) return GC_EINVAL;
    gc_plan *p = new (std::nothrow) gc_plan();
    if (!p) return GC_ENOMEM;
    p->ctx = ctx;
    p->nlists = nlists;
    p->tile = o.tile_ints ? (int)o.tile_ints : kDefaultTile;
    p->bpc = o.blocks_per_cu;
    p->use_graph = o.use_graph != 0;
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
        p->cls[i] = codec_class(h_headers[4 * i]);
        p->stream_off[i] = d.stream_off_words;
        p->out_off[i] = d.out_off;
        tiles_total += (d.n + 2047u) / 2048u;
    }
    if (tiles_total > 0xFFFFFFF0ull) {
        delete p;
        return GC_EINVAL;
    }
    (void)hipSetDevice(ctx->device);
    gc_status rc = GC_OK;
    if (o.autotune && nlists && !o.tile_ints) rc = autotune(p, h_headers, d_streams, d_out);
    for (uint32_t i = 0; i < 3 * p->slots && !rc; i++) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) rc = GC_EDEVICE;
        else p->ev.push_back(e);
    }
    if (!rc) rc = plan_materialize(p, h_headers);
    if (!rc && d_streams && d_out) rc = plan_upload(p, d_streams, d_out);
    if (!rc && p->use_graph) rc = plan_capture(p);
    if (rc) {
        plan_free_device(p);
        for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
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
    const uint32_t cus = (uint32_t)plan->ctx->num_cus;
    const uint32_t occ_a = (uint32_t)occupancy_locate();
    uint32_t occ_b[kClasses];
    for (int c = 0; c < kClasses; c++) occ_b[c] = (uint32_t)occupancy_decode(plan->tile, c);
    for (size_t i = 0; i < plan->nlists; i++) {
        ListDesc L = plan->h_lists[i];
        if (L.n == 0) continue;
        L.stream = d_streams + plan->stream_off[i];
        L.out = d_out + plan->out_off[i];
        if (L.ntiles > 1) {
            LocateArgs a = make_locate_args(nullptr, nullptr, L, 0, plan->tile, plan->sc, plan->ctx->status);
            if (launch_locate(a, std::max(1u, std::min(L.nchunks, occ_a * cus)), s)) return GC_EDEVICE;
        }
        const int c = plan->cls[i];
        DecodeArgs d = make_decode_args(nullptr, nullptr, L, 0, c, plan->sc, plan->ctx->status);
        if (launch_decode(plan->tile, c, d, std::max(1u, std::min(L.ntiles, occ_b[c] * cus)), s))
            return GC_EDEVICE;
    }
    return GC_OK;
}

gc_status gc_plan_timings(gc_plan *plan, uint32_t max_runs, float *locate_ms, float *decode_ms,
                          uint32_t *nruns) {
    if (!plan || !plan->slots || !locate_ms || !decode_ms || !nruns) return GC_EINVAL;
    const uint64_t avail = std::min<uint64_t>(plan->runs, plan->slots);
    const uint32_t n = (uint32_t)std::min<uint64_t>(avail, max_runs);
    for (uint32_t i = 0; i < n; i++) {
        const uint64_t run = plan->runs - n + i;
        const size_t k = (size_t)(run % plan->slots) * 3;
        HIP_OK(hipEventSynchronize(plan->ev[k + 2]));
        HIP_OK(hipEventElapsedTime(&locate_ms[i], plan->ev[k], plan->ev[k + 1]));
        HIP_OK(hipEventElapsedTime(&decode_ms[i], plan->ev[k + 1], plan->ev[k + 2]));
    }
    *nruns = n;
    return GC_OK;
}

gc_status gc_plan_config(const gc_plan *plan, uint32_t *tile_ints, uint32_t *blocks_per_cu, uint32_t *grid_blocks) {
    if (!plan) return GC_EINVAL;
    uint32_t g = 0, b = 0;
    for (int c = 0; c < kClasses; c++) {
        if (!plan->total_b[c]) continue;
        g += plan->grid_b[c];
        b = std::max(b, plan->bpc ? std::min<uint32_t>(plan->bpc, (uint32_t)occupancy_decode(plan->tile, c))
                                  : (uint32_t)occupancy_decode(plan->tile, c));
    }
    if (tile_ints) *tile_ints = (uint32_t)plan->tile;
    if (blocks_per_cu) *blocks_per_cu = b;
    if (grid_blocks) *grid_blocks = g;
    return GC_OK;
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
