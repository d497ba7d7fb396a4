// noalloc.hip -- the fixed device scratch of gc_decode_noalloc.
//
// gc_decode_noalloc decodes one list with the tables of single-list
// decoding (epochs, tile starts, tile carries, look-back flags, locate chunk
// aggregates and prefixes) carved from one file-scope device array instead
// of the context's allocations.  Every GPU the library runs on holds its own
// copy of the array until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gc_device.h"

namespace gcdev {

static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

// Once per device, with that device current: resolves the array's device
// address and clears it, then sets the locate epoch of every codec class to
// its first value (class c starts at c + 1).  Later calls return the kept
// address.  Returns 0, or -1 when the device index is out of range or a HIP
// call fails.
int noalloc_setup(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) {
        *ptr = g_ptr[device];
        return 0;
    }
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return -1;
    }
    RunState st[kClasses];
    for (int c = 0; c < kClasses; c++) st[c] = RunState{(uint32_t)c + 1u, {0u, 0u, 0u}};
    if (hipMemset(p, 0, kNoallocScratchBytes) != hipSuccess ||
        hipMemcpy(static_cast<uint8_t *>(p) + noalloc_layout().state, st, sizeof(st), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    g_ptr[device] = p;
    *ptr = p;
    return 0;
}

// The kept address of device `device`'s array (nullptr before its set-up).
void *noalloc_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace gcdev
