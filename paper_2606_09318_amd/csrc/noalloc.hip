// lr_rank_noalloc: lr_rank with its workspace in a static device array, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The array lives in this file's code object, so a process that never calls
// lr_rank_noalloc never loads it. Every GPU the library runs this call on
// holds its own copy of the array until the process ends; its device address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is ever handed to kernels or copies: in host
// code the array's name is a host-side stand-in, not a device address.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "lr.h"

static_assert(LR_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size is a multiple of the workspace alignment");

// The workspace of every lr_rank_noalloc call on this device. lr_rank clears
// what it needs from it at the start of each call (its control block and
// counters are written by its first kernels), so stale contents from the
// previous call are harmless.
static __device__ __align__(256) unsigned char scratch[LR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};  // device address of `scratch`, per device ordinal

// The current device's address of `scratch`, looked up on its first use on
// that device. Returns nullptr when the lookup fails.
void* scratch_address(int dev) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_addr[dev] = p;
    }
    return g_addr[dev];
}

}  // namespace

extern "C" lr_status lr_rank_noalloc(const uint32_t* succ, uint32_t* rank, uint32_t* root, uint64_t n,
                                     const lr_opts* opts, void* stream) {
    if (n == 0) return LR_OK;
    if (!succ || !rank) return LR_ERR_INVALID_ARG;
    if (n >= (1ull << 31)) return LR_ERR_UNSUPPORTED;
    // LR_PROFILE creates timing events on first use; this entry point creates
    // nothing
    if (opts && (opts->flags & LR_PROFILE)) return LR_ERR_INVALID_ARG;
    const size_t need = lr_workspace_bytes(n, LR_W_NONE, opts);
    if (need == 0) return LR_ERR_INVALID_ARG;
    if (need > LR_NOALLOC_SCRATCH_BYTES) return LR_ERR_WORKSPACE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LR_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return LR_ERR_UNSUPPORTED;
    void* ws = scratch_address(dev);
    if (!ws) return LR_ERR_HIP;
    return lr_rank(succ, rank, root, n, ws, LR_NOALLOC_SCRATCH_BYTES, opts, stream);
}
