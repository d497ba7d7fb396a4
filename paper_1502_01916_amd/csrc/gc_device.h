// gc_device.h -- device-side data structures shared by the libgc kernels and
// the host runtime that launches them.
#pragma once
#include <stdint.h>

namespace gcdev {

constexpr int kThreads = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kThreads / 64;
constexpr int kChunkWords = kThreads * 4;  // control words per locate work item
constexpr int kClasses = 5;                 // decode kernel classes (codec families)

// One list of a launch.  For a batch these live in a device table; for a
// single list the runtime passes one by value.
struct ListDesc {
    const uint32_t *stream;   // 16-byte aligned; header at stream[0..3]
    uint32_t *out;            // n outputs
    uint64_t stream_words;
    uint32_t n;
    uint32_t ntiles;          // ceil(n / tile_ints)
    uint32_t tile_base;       // first entry of this list in the tile arrays
    uint32_t chunk_base;      // first entry in the locate arrays (ntiles > 1)
    uint32_t nchunks;         // locate work items (0 when ntiles <= 1)
    uint32_t cls_base;        // first entry of this list in its decode class queue
};

// Where tile m of a list starts, written by the locate pass.
struct TileInfo {
    uint32_t unit;    // selector / control bit / frame / block where the tile starts
    uint32_t sub;     // tuples of that unit that belong to the previous tile
    uint32_t exc;     // Group-PFD: exception-area word offset of the unit
    uint32_t tag;     // epoch of the locate run that wrote this entry
    uint64_t data;    // component bit offset of the unit (Group-Scheme: of the tuple)
    uint64_t pad;
};

// Self-resetting state of one persistent kernel: work counter, finished
// workgroups, and the run epoch that tags look-back flags.  The last
// workgroup to finish clears the counters and advances the epoch, so a run
// needs no memset (and can sit in a captured graph).
struct RunState {
    uint32_t counter;
    uint32_t done;
    uint32_t epoch;
    uint32_t pad;
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

struct LocateArgs {
    const ListDesc *lists;      // batch table, or nullptr for `single`
    const uint32_t *item_list;  // work item -> list (batch)
    ListDesc single;
    uint32_t total_items;       // batch; single computes its own
    uint32_t tile_ints;
    TileInfo *tiles;
    uint32_t *flags;            // per chunk: epoch << 2 | state
    LocVal *agg;                // per chunk aggregate
    LocVal *incl;               // per chunk inclusive prefix
    RunState *state;
    Status *status;
};

struct DecodeArgs {
    const ListDesc *lists;
    const uint32_t *item_list;
    ListDesc single;
    uint32_t total_items;
    uint32_t pad;
    const TileInfo *tiles;
    unsigned long long *flags;  // per tile: epoch:30 | state:2 | sum:32
    RunState *state;
    const RunState *loc_state;  // the locate kernel's state (for the tile tags)
    Status *status;
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
    kErrTimeout = 10,
    kErrBitmap = 11,
};

}  // namespace gcdev
