// gc_blocks.h -- constants and launchers of the per-block container kernels
// (the encode side of the learned codec selector), shared by the kernels
// and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gcblk {

constexpr int kBlockInts = 128;    // integers per block (32 tuples at k = 4)
constexpr int kTuples = 32;
constexpr int kClasses = 16;       // codec classes of the container
constexpr int kFeatures = 40;      // selector inputs per block
constexpr int kMaxCtrlWords = 36;  // bounds of one block's payload areas
constexpr int kMaxDataWords = 132;
constexpr int kMaxExcWords = 132;
constexpr int kMaxPayloadWords = kMaxCtrlWords + kMaxDataWords + kMaxExcWords;

int launch_block_features(const uint32_t *in, size_t nblocks, float *feat, hipStream_t s);
int launch_block_sizes(const uint32_t *in, size_t nblocks, uint32_t *sizes, uint8_t *best, float *cost,
                       hipStream_t s);
size_t scan_chunks(size_t n);
int launch_blockmix_plan(const uint32_t *in, size_t nblocks, const uint8_t *cls, uint32_t *words, uint32_t *offs,
                         uint32_t *csum, uint32_t *result, hipStream_t s);
// Writes the container (header included) at out, no payload past cap_words;
// total: the payload words from the plan's scan (device memory).
int launch_blockmix_emit(const uint32_t *in, size_t nblocks, const uint8_t *cls, const uint32_t *offs,
                         uint32_t *out, size_t cap_words, uint32_t n, const uint32_t *total, hipStream_t s);

}  // namespace gcblk
