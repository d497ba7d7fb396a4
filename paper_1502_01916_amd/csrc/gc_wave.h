// gc_wave.h -- wave64 helpers shared by the libgc kernels: bit fields, DPP
// scans across a wave, and LDS ordering within a wave.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcdev {

__device__ __forceinline__ uint32_t mask_of(uint32_t b) { return b >= 32u ? 0xFFFFFFFFu : ((1u << b) - 1u); }

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh) {
    return __builtin_amdgcn_alignbit(hi, lo, sh);
}

template <int CTRL, int ROWS, bool BC>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, BC);
}

// Inclusive scan across a wave64 with DPP row shifts and row broadcasts.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += dpp<0x111, 0xF, true>(x);    // row_shr:1
    x += dpp<0x112, 0xF, true>(x);    // row_shr:2
    x += dpp<0x114, 0xF, true>(x);    // row_shr:4
    x += dpp<0x118, 0xF, true>(x);    // row_shr:8
    x += dpp<0x142, 0xA, false>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp<0x143, 0xC, false>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// Inclusive running maximum across a wave64 (same DPP pattern).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
    x = max(x, dpp<0x111, 0xF, true>(x));
    x = max(x, dpp<0x112, 0xF, true>(x));
    x = max(x, dpp<0x114, 0xF, true>(x));
    x = max(x, dpp<0x118, 0xF, true>(x));
    x = max(x, dpp<0x142, 0xA, false>(x));
    x = max(x, dpp<0x143, 0xC, false>(x));
    return x;
}

// The value of the previous lane (0 in lane 0): DPP wave_shr:1.
__device__ __forceinline__ uint32_t wave_shr1(uint32_t x) { return dpp<0x138, 0xF, true>(x); }

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(x), 63);
}

// 64-bit wave sum from 32-bit scans (16-bit halves of the low word cannot
// overflow across 64 lanes).
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    return (uint64_t)wave_sum(lo & 0xFFFFu) + ((uint64_t)wave_sum(lo >> 16) << 16) + ((uint64_t)wave_sum(hi) << 32);
}

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}


// Orders a wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_any(bool b) { return __ballot(b) != 0ull ? 1u : 0u; }

}  // namespace gcdev
