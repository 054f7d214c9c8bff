// Issue-rate probe for the 32-bit integer VALU roofline: long chains of one
// instruction kind at full occupancy, timed with HIP events.  The hashing
// kernels are built from these instructions (v_perm_b32 table addresses,
// v_bitop3_b32 three-input xors, v_alignbit rotations, v_add3_u32 in
// SHA-256, v_mad_u64_u32 in the field arithmetic), so their sustained rate
// on this chip is the practical ceiling a roofline fraction should be read
// against, beside the nominal 4-cycles-per-wave64-instruction figure.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/poslo.h"

namespace {

constexpr int kChains = 8;   // independent dependency chains per lane
constexpr int kUnroll = 16;  // instructions of each chain per loop trip

template <int OP>
__device__ __forceinline__ void step(uint32_t& a, uint32_t b, uint32_t c) {
    if constexpr (OP == POSLO_PROBE_XOR)
        asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a) : "v"(b));
    else if constexpr (OP == POSLO_PROBE_PERM)
        asm volatile("v_perm_b32 %0, %1, %0, %2" : "+v"(a) : "v"(b), "v"(c));
    else if constexpr (OP == POSLO_PROBE_BITOP3)
        asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a) : "v"(b), "v"(c));
    else if constexpr (OP == POSLO_PROBE_ADD3)
        asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    else if constexpr (OP == POSLO_PROBE_ALIGNBIT)
        asm volatile("v_alignbit_b32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
}

template <int OP>
__global__ __launch_bounds__(256) void k_probe(uint32_t iters, uint32_t seed, uint32_t* sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; k++) a[k] = seed ^ (tid * 0x9e3779b9u) ^ (uint32_t)k;
    const uint32_t b = seed * 3u + tid, c = 0x05040302u ^ (seed & 0x03030303u);
    if constexpr (OP == POSLO_PROBE_MAD64) {
        // 64-bit multiply-adds: acc = lo(acc) * b + acc, eight chains
        uint64_t acc[kChains];
#pragma unroll
        for (int k = 0; k < kChains; k++) acc[k] = a[k];
        for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
            for (int u = 0; u < kUnroll; u++)
#pragma unroll
                for (int k = 0; k < kChains; k++) acc[k] = (uint64_t)(uint32_t)acc[k] * b + acc[k];
        }
        uint32_t x = 0;
#pragma unroll
        for (int k = 0; k < kChains; k++) x ^= (uint32_t)acc[k] ^ (uint32_t)(acc[k] >> 32);
        if (x == 0x12345678u) sink[tid] = x;  // keeps the chains live
        return;
    }
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (int u = 0; u < kUnroll; u++)
#pragma unroll
            for (int k = 0; k < kChains; k++) step<OP>(a[k], b, c);
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kChains; k++) x ^= a[k];
    if (x == 0x12345678u) sink[tid] = x;  // keeps the chains live
}

}  // namespace

extern "C" int poslo_valu_probe(int device, int op, uint32_t waves_per_simd, uint32_t iters, double* lane_ops_per_s,
                                double* ms) {
    if (op < 0 || op > POSLO_PROBE_MAD64 || waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || !lane_ops_per_s)
        return POSLO_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return POSLO_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return POSLO_E_DEVICE;
    // four SIMDs per CU, 256-thread (4-wave) workgroups: waves_per_simd
    // workgroups per CU keep that many waves on every SIMD
    const uint32_t grid = (uint32_t)prop.multiProcessorCount * waves_per_simd;
    const uint32_t threads = grid * 256;
    uint32_t* sink = nullptr;
    if (hipMalloc((void**)&sink, (size_t)threads * 4) != hipSuccess) return POSLO_E_NOMEM;
    hipEvent_t e0, e1;
    int st = POSLO_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = POSLO_E_DEVICE;
    auto launch = [&](hipStream_t s) {
        switch (op) {
            case POSLO_PROBE_XOR: hipLaunchKernelGGL(k_probe<POSLO_PROBE_XOR>, grid, 256, 0, s, iters, 7u, sink); break;
            case POSLO_PROBE_PERM: hipLaunchKernelGGL(k_probe<POSLO_PROBE_PERM>, grid, 256, 0, s, iters, 7u, sink); break;
            case POSLO_PROBE_BITOP3:
                hipLaunchKernelGGL(k_probe<POSLO_PROBE_BITOP3>, grid, 256, 0, s, iters, 7u, sink);
                break;
            case POSLO_PROBE_ADD3: hipLaunchKernelGGL(k_probe<POSLO_PROBE_ADD3>, grid, 256, 0, s, iters, 7u, sink); break;
            case POSLO_PROBE_ALIGNBIT:
                hipLaunchKernelGGL(k_probe<POSLO_PROBE_ALIGNBIT>, grid, 256, 0, s, iters, 7u, sink);
                break;
            default: hipLaunchKernelGGL(k_probe<POSLO_PROBE_MAD64>, grid, 256, 0, s, iters, 7u, sink); break;
        }
    };
    float t = 0.f;
    if (!st) {
        launch(nullptr);  // warm-up: clocks and code object
        if (hipEventRecord(e0, nullptr) != hipSuccess) st = POSLO_E_DEVICE;
        launch(nullptr);
        if (!st && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess))
            st = POSLO_E_DEVICE;
    }
    if (!st) {
        const double ops = (double)threads * iters * kUnroll * kChains;
        *lane_ops_per_s = ops / (t / 1e3);
        if (ms) *ms = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    return st;
}
