// Device calibration: the access rates the ranking kernels are bound by,
// measured on the caller's device (diagnostic; not part of any ranking call).
// Every kernel touches N = 2^28 elements at hashed positions over a buffer
// inside the caller's workspace, so the same pattern as the chase (4 B
// gathers over a 1 GiB successor array) and the random stores it replaced
// can be compared with a streaming copy.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lr.h"

namespace lr {

constexpr int CAL_TPB = 256;

__device__ __forceinline__ uint32_t cal_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

#define CAL_LOOP for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)

__global__ __launch_bounds__(CAL_TPB) void k_cal_init(uint32_t* a, uint64_t words) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        a[i] = cal_hash((uint32_t)i * 2654435761u + 1u);
}

__global__ __launch_bounds__(CAL_TPB) void k_cal_copy(const uint4* __restrict__ a, uint4* __restrict__ b, uint32_t n) {
    CAL_LOOP b[i] = a[i];
}

// 4 B gathers at hashed positions; the sum keeps the loads alive
__global__ __launch_bounds__(CAL_TPB) void k_cal_gather(const uint32_t* __restrict__ a, uint32_t mask, uint32_t n,
                                                        uint32_t* __restrict__ sink, uint32_t seed) {
    uint32_t acc = 0;
    CAL_LOOP acc += a[cal_hash(i ^ seed) & mask];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(CAL_TPB) void k_cal_store8(uint2* __restrict__ b, uint32_t mask, uint32_t n,
                                                        uint32_t seed) {
    CAL_LOOP {
        const uint32_t j = cal_hash(i ^ seed) & mask;
        b[j] = make_uint2(i, j);
    }
}

__global__ __launch_bounds__(CAL_TPB) void k_cal_store1(uint8_t* __restrict__ b, uint32_t mask, uint32_t n,
                                                        uint32_t seed) {
    CAL_LOOP b[cal_hash(i ^ seed) & mask] = 1;
}

__global__ __launch_bounds__(CAL_TPB) void k_cal_bitset(uint32_t* __restrict__ b, uint32_t mask, uint32_t n,
                                                        uint32_t seed) {
    CAL_LOOP {
        const uint32_t j = cal_hash(i ^ seed) & mask;
        atomicOr(&b[j >> 5], 1u << (j & 31));
    }
}

// Records (x, v) grouped by ranges of 2^s ids, x a bijection of its range
// (an odd multiple plus a per-range offset, modulo the range length)
__global__ __launch_bounds__(CAL_TPB) void k_cal_range_init(uint32_t* __restrict__ x, uint32_t* __restrict__ v,
                                                            uint32_t s, uint32_t n) {
    CAL_LOOP {
        const uint32_t c = i >> s, mask = (1u << s) - 1;
        x[i] = (c << s) | (((i & mask) * 0x9e3779b1u + cal_hash(c)) & mask);
        v[i] = i;
    }
}

// out[x] = v for every record, each range's records stored by the workgroups
// of one XCD (workgroup i runs on XCD i mod 8, and XCD x takes ranges x,
// x + 8, ... in order, tiles of CAL_RANGE_PER x CAL_TPB records): the access
// pattern of a placement pass that scattered each element range straight
// into the output through the owning XCD's L2
constexpr int CAL_RANGE_PER = 8;
__global__ __launch_bounds__(CAL_TPB) void k_cal_range4(const uint32_t* __restrict__ x, const uint32_t* __restrict__ v,
                                                        uint32_t* __restrict__ out, uint32_t s, uint32_t n) {
    constexpr uint32_t T = CAL_TPB * CAL_RANGE_PER;
    const uint32_t tiles = n / T, tpc = (1u << s) / T;
    const uint32_t lane8 = blockIdx.x % 8, step = gridDim.x / 8;
    for (uint32_t q = blockIdx.x / 8;; q += step) {
        const uint32_t c = lane8 + 8 * (q / tpc);
        if (c * tpc >= tiles) break;
        const uint32_t tile = c * tpc + q % tpc;
        uint32_t xs[CAL_RANGE_PER], vs[CAL_RANGE_PER];
#pragma unroll
        for (int j = 0; j < CAL_RANGE_PER; ++j) {
            const uint32_t i = tile * T + j * CAL_TPB + threadIdx.x;
            xs[j] = x[i];
            vs[j] = v[i];
        }
#pragma unroll
        for (int j = 0; j < CAL_RANGE_PER; ++j) out[xs[j]] = vs[j];
    }
}

}  // namespace lr

using namespace lr;

extern "C" size_t lr_calibrate_workspace_bytes(void) { return ((size_t)4 << 30) + 256; }

extern "C" int lr_calibrate(void* ws, size_t ws_bytes, double* out, int cap, void* stream) {
    const uint32_t N = 1u << 28;
    if (!ws || ws_bytes < lr_calibrate_workspace_bytes() || !out) return -(int)LR_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) / 256 * 256);
    const size_t sink_bytes = (size_t)64 << 20;
    uint32_t* a = reinterpret_cast<uint32_t*>(w);                   // [0, 1 GiB): gather source
    char* b = w + ((size_t)1 << 30);                                // [1 GiB, 3 GiB - 64 MiB): store targets
    uint32_t* sink = reinterpret_cast<uint32_t*>(w + ((size_t)3 << 30) - sink_bytes);
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint32_t nblocks = (uint32_t)std::min(cus, 2048) * 32;   // one sink word per lane: <= 64 MiB
    const dim3 G(nblocks), B(CAL_TPB);
    hipLaunchKernelGGL(k_cal_init, dim3(8192), B, 0, st, reinterpret_cast<uint32_t*>(w),
                       (((uint64_t)3 << 30) - sink_bytes) / 4);
    if (hipGetLastError() != hipSuccess) return -(int)LR_ERR_HIP;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -(int)LR_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -(int)LR_ERR_HIP; }
    int k = 0;
    bool fail = false;
    auto timed = [&](auto launch) -> double {
        launch();  // warm-up
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < 3; ++r) launch();
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) { fail = true; return 0; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms / 3;
    };
    const uint32_t m1g = (1u << 28) - 1;   // 2^28 words of 4 B
    const uint32_t m8g = (1u << 27) - 1;   // 2^27 records of 8 B: 1 GiB
    const uint32_t m8w = (1u << 25) - 1;   // 2^25 records of 8 B: 256 MiB
    const uint32_t m1b = (1u << 28) - 1;   // 2^28 bytes
    double v[7];
    // [0] streaming copy of 1 GiB, GB/s (read + write bytes)
    const double tc = timed([&] { hipLaunchKernelGGL(k_cal_copy, G, B, 0, st, reinterpret_cast<const uint4*>(a),
                                                     reinterpret_cast<uint4*>(b), N / 4); });
    v[0] = 2.0 * ((double)N * 4) / (tc * 1e-3) / 1e9;
    // [1] 4 B gathers over 1 GiB, G accesses/s
    const double tg = timed([&] { hipLaunchKernelGGL(k_cal_gather, G, B, 0, st, a, m1g, N, sink, 1u); });
    v[1] = N / (tg * 1e-3) / 1e9;
    // [2] 8 B stores over 1 GiB, G accesses/s
    const double ts = timed([&] { hipLaunchKernelGGL(k_cal_store8, G, B, 0, st, reinterpret_cast<uint2*>(b), m8g, N,
                                                     2u); });
    v[2] = N / (ts * 1e-3) / 1e9;
    // [3] 8 B stores over a 256 MiB window
    const double tw = timed([&] { hipLaunchKernelGGL(k_cal_store8, G, B, 0, st, reinterpret_cast<uint2*>(b), m8w, N,
                                                     3u); });
    v[3] = N / (tw * 1e-3) / 1e9;
    // [4] 1 B stores over 256 MiB
    const double t1 = timed([&] { hipLaunchKernelGGL(k_cal_store1, G, B, 0, st, reinterpret_cast<uint8_t*>(b),
                                                     m1b, N, 4u); });
    v[4] = N / (t1 * 1e-3) / 1e9;
    // [5] bit sets (atomicOr) over a 32 MiB bitmap
    const double tb = timed([&] { hipLaunchKernelGGL(k_cal_bitset, G, B, 0, st, reinterpret_cast<uint32_t*>(b), m1b,
                                                     N, 5u); });
    v[5] = N / (tb * 1e-3) / 1e9;
    // [6] 2^28 records (x, v) of two 1 GiB arrays streamed in, v stored at x,
    // x grouped in XCD-owned ranges of 2^15 ids (128 KiB of output each); the
    // records take the gather source and a third GiB past the store targets
    static_assert(((1u << 15) % (CAL_TPB * CAL_RANGE_PER)) == 0, "a range is whole tiles");
    uint32_t* rv = reinterpret_cast<uint32_t*>(w + ((size_t)3 << 30));
    hipLaunchKernelGGL(k_cal_range_init, dim3(8192), B, 0, st, a, rv, 15u, N);
    if (hipGetLastError() != hipSuccess) fail = true;
    const double tr = timed([&] { hipLaunchKernelGGL(k_cal_range4, dim3(nblocks / 8 * 8), B, 0, st, a, rv,
                                                     reinterpret_cast<uint32_t*>(b), 15u, N); });
    v[6] = N / (tr * 1e-3) / 1e9;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (fail) return -(int)LR_ERR_HIP;
    for (int i = 0; i < 7 && k < cap; ++i) out[k++] = v[i];
    return k;
}
