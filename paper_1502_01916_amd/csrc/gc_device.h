// gc_device.h -- device-side data structures shared by the libgc kernels and
// the host runtime that launches them.
#pragma once
#include <stdint.h>

namespace gcdev {

constexpr int kThreads = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kThreads / 64;
constexpr int kChunkWords = 256;       // control words per locate work item (one wave, 4 per lane)
constexpr int kChunkWordsSmall = 128;  // the same for a single list decoded alone (2 per lane)
constexpr int kClasses = 5;                 // decode kernel classes (codec families)

// Tables of a list decoded alone, for lists of up to max_ints integers: a
// tile holds at least 1024 integers (one spare entry follows the last), and
// a locate chunk 128 control words, of which a list has at most one per
// tuple of four integers (a unary Group-Scheme code is at most 32 bits) plus
// padding.
constexpr uint64_t single_tiles_cap(uint64_t max_ints) { return (max_ints + 1023u) / 1024u + 1u; }
constexpr uint64_t single_chunks_cap(uint64_t max_ints) { return ((max_ints + 3u) / 4u + 4u + 127u) / 128u + 1u; }

// The fixed device scratch of the allocation-free single-list decode: the
// same tables for lists of up to kNoallocMaxInts integers, at 256-byte
// aligned offsets (about 434 KB).
constexpr uint64_t kNoallocMaxInts = 1ull << 22;
constexpr uint64_t noalloc_round(uint64_t b) { return (b + 255u) & ~(uint64_t)255u; }
struct NoallocLayout {
    uint64_t state, tiles, carry, flags, agg, pre, bytes;
    uint64_t tiles_cap, chunks_cap;
};
constexpr NoallocLayout noalloc_layout();   // defined after the structures it sizes

// One list of a launch.  For a batch these live in a device table; for a
// single list the runtime passes one by value.  The header words come from
// the host's copy of the header; kernels check the stream against them.
struct ListDesc {
    const uint32_t *stream;   // 16-byte aligned; header at stream[0..3]
    uint32_t *out;            // n outputs
    uint64_t stream_words;
    uint32_t n;
    uint32_t ntiles;          // ceil(n / tile_ints)
    uint32_t tile_base;       // first entry of this list in the tile arrays
    uint32_t chunk_base;      // first entry in the locate arrays (ntiles > 1)
    uint32_t nchunks;         // locate work items (0 when ntiles <= 1)
    uint32_t tile_ints;       // integers per decode tile for this list's codec class
    uint32_t w0, C, D;        // header words 0, 2 and 3
    uint32_t pad;
};

// Where tile m of a list starts, written by the locate pass.
struct TileInfo {
    uint32_t unit;    // selector / control bit / frame / block where the tile starts
    uint32_t sub;     // tuples of that unit that belong to the previous tile
    uint32_t exc;     // Group-PFD: exception-area word offset of the unit
    uint32_t tag;     // epoch of the locate run that wrote this entry
    uint64_t data;    // component bit offset of the unit (Group-Scheme, Group-AFOR: of the tile's first tuple)
    uint32_t list;    // batch: the tile's list (tile 0 of a list: set by the host)
    uint32_t pad;
};

// Epoch of the locate pass: its first kernel advances it, its last tags
// every tile start with it, and the decode kernels accept only tile starts
// of the current epoch (a tile that the locate pass never reached is caught
// instead of decoded from a stale entry).  No counter needs resetting, so a
// run can be replayed from a captured graph without a memset.
struct RunState {
    uint32_t epoch;
    uint32_t pad[3];
};

// Device status: the first error latched, with a detail code.
struct Status {
    uint32_t code;     // 0 or (uint32_t)GC_ECORRUPT
    uint32_t detail;
};

// Locate-pass scan value of one control chunk.
struct LocVal {
    uint32_t tup;      // tuples
    uint32_t exc;      // exception words
    uint64_t data;     // component data bits
};

constexpr NoallocLayout noalloc_layout() {
    NoallocLayout l{};
    l.tiles_cap = single_tiles_cap(kNoallocMaxInts);
    l.chunks_cap = single_chunks_cap(kNoallocMaxInts);
    l.state = 0;
    l.tiles = noalloc_round(l.state + kClasses * sizeof(RunState));
    l.carry = noalloc_round(l.tiles + l.tiles_cap * sizeof(TileInfo));
    l.flags = noalloc_round(l.carry + l.tiles_cap * sizeof(uint32_t));
    l.agg = noalloc_round(l.flags + l.tiles_cap * sizeof(unsigned long long));
    l.pre = noalloc_round(l.agg + l.chunks_cap * sizeof(LocVal));
    l.bytes = noalloc_round(l.pre + l.chunks_cap * sizeof(LocVal));
    return l;
}
constexpr uint64_t kNoallocScratchBytes = noalloc_layout().bytes;
static_assert(kNoallocScratchBytes < (1u << 20), "the fixed scratch stays modest");

// Locate runs as three fence-free kernels: reduce (one aggregate per control
// chunk), scan (exclusive prefix of the aggregates within each list) and emit
// (tile starts from the prefixes).  Kernel boundaries order them.
struct LocateArgs {
    const ListDesc *lists;      // batch table, or nullptr for `single`
    const uint32_t *item_list;  // chunk work item -> list (batch)
    const uint32_t *scan_list;  // scan work item -> list (batch)
    ListDesc single;
    uint32_t total_items;       // chunk items of this launch (batch or single)
    uint32_t total_scan;        // lists with chunks (batch); 1 for single
    uint32_t item_lo;           // batch: first chunk item of this launch
    uint32_t pad;
    TileInfo *tiles;
    LocVal *agg;                // per chunk aggregate
    LocVal *pre;                // per chunk exclusive prefix within its list
    RunState *state;            // emit kernel: epoch that tags tile starts
    Status *status;
};

// One decode launch covers the tiles [lo, lo + count) of the tile arrays:
// a wave per tile.
struct DecodeArgs {
    const ListDesc *lists;      // batch table, or nullptr for `single`
    ListDesc single;
    uint32_t lo;
    uint32_t count;
    const TileInfo *tiles;
    uint32_t *carry;            // per tile: sum of its gaps (sum pass), then the
                                // exclusive prefix of those sums in its list
    unsigned long long *flags;  // single-pass carry: per tile epoch:30 | state:2 | value:32
    uint32_t lb_max_tiles;      // mode 2: lists of at most this many tiles take their
                                // carries by look-back, longer ones from carry[]
    uint32_t lb_stall_ticks;    // 0, or (tests of the bounded wait only): tiles do not
                                // publish their flags and a look-back gives up after
                                // this many ticks of the real-time counter
    const RunState *loc_state;
    Status *status;
};

// A list the pack kernel decodes: a short list whose whole stream fits a
// pack's staging buffer.  The lists of a pack are consecutive entries.
struct PackDesc {
    const uint32_t *stream;   // 16-byte aligned
    uint32_t *out;
    uint32_t n;
    uint32_t w0;              // header word 0 (host copy)
    uint32_t cd;              // header words 2 and 3 (host copy): C | D << 16, both < 2^16
    uint32_t words;           // stream words, a multiple of 4
};

// Pack kernel launch: a wave per pack; pack p holds the descriptors
// [first[p], first[p + 1]), at most 32 lists whose streams fit the
// kernel's staging buffer together.
struct PackArgs {
    const PackDesc *descs;
    const uint32_t *first;    // npacks + 1 entries
    uint32_t npacks;
    uint32_t pad;
    Status *status;
};

// Carry scan: one workgroup per delta list of more than one tile.
struct CarryArgs {
    const ListDesc *lists;      // batch table, or nullptr for `single`
    const uint32_t *scan_list;  // batch: work item -> list
    ListDesc single;
    uint32_t count;
    uint32_t pad;
    uint32_t *carry;
};

// Detail codes of device-side errors.
enum : uint32_t {
    kErrHeader = 1,
    kErrSelector = 2,
    kErrUnary = 3,
    kErrFrame = 4,
    kErrPfdDesc = 5,
    kErrPfdChain = 6,
    kErrRange = 7,
    kErrLocate = 8,
    kErrCount = 9,
    kErrBitmap = 11,
    kErrTimeout = 12,   // a carry look-back waited too long for an earlier tile
    kErrPack = 13,      // a pack's streams do not fit its staging buffer
};

}  // namespace gcdev
