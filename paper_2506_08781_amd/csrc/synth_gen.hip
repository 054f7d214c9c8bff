// Seeded synthetic log bytes generated on the device, for benchmarks and
// tests at sizes where host generation would dominate.
//
// Generator: xoshiro256** (Blackman and Vigna) seeded through splitmix64
// (Steele, Lea and Flood), written from their published definitions.  Stream
// (seed, sid) starts from splitmix64 state (seed << 32) | sid; entry t of a
// log with message seed s draws its bytes from stream (s, t): ceil(L/8)
// outputs, little-endian, truncated to L bytes.  This file holds no part of
// the signature scheme; the same convention is implemented independently by
// the host-side input generator of the test suite.
#include "../../include/poslo.h"
#include "common.h"

namespace poslo {

struct Xoshiro {
    uint64_t s0, s1, s2, s3;
};

__device__ __forceinline__ uint64_t splitmix_next(uint64_t& st) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

__device__ __forceinline__ Xoshiro stream_init(uint32_t seed, uint32_t sid) {
    uint64_t st = ((uint64_t)seed << 32) | sid;
    Xoshiro x;
    x.s0 = splitmix_next(st);
    x.s1 = splitmix_next(st);
    x.s2 = splitmix_next(st);
    x.s3 = splitmix_next(st);
    return x;
}

__device__ __forceinline__ uint64_t xoshiro_next(Xoshiro& x) {
    uint64_t r = rotl64(x.s1 * 5, 7) * 9;
    uint64_t t = x.s1 << 17;
    x.s2 ^= x.s0;
    x.s3 ^= x.s1;
    x.s1 ^= x.s2;
    x.s0 ^= x.s3;
    x.s2 ^= t;
    x.s3 = rotl64(x.s3, 45);
    return r;
}

// one entry per lane: entry p of the batch is stream (seed, t0 + p)
__global__ __launch_bounds__(256) void k_synth_messages(uint32_t seed, uint64_t t0, uint64_t n, const uint64_t* offsets,
                                                        uint64_t msg_len, uint8_t* out) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint64_t o = offsets ? offsets[p] : p * msg_len;
    uint64_t L = offsets ? offsets[p + 1] - offsets[p] : msg_len;
    Xoshiro x = stream_init(seed, (uint32_t)(t0 + p));
    uint8_t* dst = out + o;
    if ((o % 8) == 0 && (L % 8) == 0) {
        uint64_t* d64 = reinterpret_cast<uint64_t*>(dst);
        for (uint64_t w = 0; w < L / 8; w++) d64[w] = xoshiro_next(x);
        return;
    }
    for (uint64_t w = 0; w * 8 < L; w++) {
        uint64_t v = xoshiro_next(x);
        for (int b = 0; b < 8 && w * 8 + b < L; b++) dst[w * 8 + b] = (uint8_t)(v >> (8 * b));
    }
}

}  // namespace poslo

using namespace poslo;

extern "C" int poslo_synth_messages(uint32_t seed, const poslo_msgs* m, uint8_t* out, void* stream) {
    if (!m || (m->n && !out) || m->t0 + m->n > (1ull << 32)) return POSLO_E_INVAL;
    if (m->n == 0) return POSLO_OK;
    hipLaunchKernelGGL(k_synth_messages, dim3((uint32_t)((m->n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       seed, m->t0, m->n, m->offsets, m->msg_len, out);
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}
