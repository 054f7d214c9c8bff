// Device-side hashing of one log entry: the one-time seed
// x_t = PRF_0(x_0[i] || LE32(j)) and the digest H(m_t || x_t), for both
// instantiations, plus the per-epoch seed table (SR / SC of the seed tree).
//
// Per-epoch table entry (48 words):
//   words 0..43  AES instantiation: the 11 round keys of h1 = E_IV(x_0[i]) xor
//                x_0[i], the epoch-constant first MMO block of PRF_0, so that
//                each entry's PRF costs one AES with a precomputed schedule
//   words 44..47 x_0[i] as little-endian words
#pragma once

#include "aes128.h"
#include "sha256.h"

namespace poslo {

constexpr int kEpochWords = 48;

// constant tables for the device (built at compile time)
__constant__ const AesTables c_aes = make_aes_tables();
__constant__ const IvSchedules c_iv = make_iv_schedules();

// table reader over the constant table (small kernels)
struct ConstTables {
    __device__ __forceinline__ uint32_t t0(uint32_t x) const { return c_aes.te0[x]; }
    __device__ __forceinline__ uint32_t t1(uint32_t x) const { return rotl32(c_aes.te0[x], 8); }
    __device__ __forceinline__ uint32_t t2(uint32_t x) const { return rotl32(c_aes.te0[x], 16); }
    __device__ __forceinline__ uint32_t t3(uint32_t x) const { return rotl32(c_aes.te0[x], 24); }
};

// Table reader over bank-replicated copies in LDS.  NT = 4 keeps the four
// rotated tables, NT = 2 keeps te0 and te0 rotated by 16 (the other two are
// one rotation away), NT = 1 keeps te0 and rotates.  C copies are interleaved
// so that copy c of entry x sits at word x*C + c; a lane reads copy
// (lane mod C), which spreads a wave's random lookups over more banks.
template <int NT, int C>
struct LdsTables {
    const uint32_t* p;
    __device__ __forceinline__ uint32_t t0(uint32_t x) const { return p[x * C]; }
    __device__ __forceinline__ uint32_t t1(uint32_t x) const {
        if constexpr (NT == 4) return p[(256 + x) * C];
        else return rotl32(p[x * C], 8);
    }
    __device__ __forceinline__ uint32_t t2(uint32_t x) const {
        if constexpr (NT == 4) return p[(512 + x) * C];
        else if constexpr (NT == 2) return p[(256 + x) * C];
        else return rotl32(p[x * C], 16);
    }
    __device__ __forceinline__ uint32_t t3(uint32_t x) const {
        if constexpr (NT == 4) return p[(768 + x) * C];
        else if constexpr (NT == 2) return rotl32(p[(256 + x) * C], 8);
        else return rotl32(p[x * C], 24);
    }
};

template <int NT, int C>
__device__ __forceinline__ void lds_tables_fill(uint32_t* lds) {
    for (int k = threadIdx.x; k < NT * 256 * C; k += blockDim.x) {
        int e = k / C;
        int rot = NT == 2 ? 16 * (e >> 8) : 8 * (e >> 8);
        lds[k] = rotl32(c_aes.te0[e & 255], rot);
    }
}

// ---- PRF on device -------------------------------------------------------

// PRF_b(x) for a 16-byte x (the tree-node PRF, kappa = 128: 17-byte input)
template <class T>
__device__ __forceinline__ void prf_node_aes(const T& tb, const uint32_t x[4], uint32_t b, uint32_t out[4]) {
    uint32_t s[4] = {x[0], x[1], x[2], x[3]};
    aes128_encrypt_rk(tb, c_iv.a, s);
    uint32_t h1[4] = {s[0] ^ x[0], s[1] ^ x[1], s[2] ^ x[2], s[3] ^ x[3]};
    uint32_t blk[4] = {b, 0u, 0u, 0u};
    aes128_encrypt_otf(tb, h1, blk);
    out[0] = blk[0] ^ b;
    out[1] = blk[1];
    out[2] = blk[2];
    out[3] = blk[3];
}

// the tree PRF at kappa = 127: one MMO block x + b * 2^127 under the IV's
// schedule, reduced mod 2^127 (x has bit 127 clear)
template <class T>
__device__ __forceinline__ void prf_node_aes127(const T& tb, const uint32_t x[4], uint32_t b, uint32_t out[4]) {
    const uint32_t blk[4] = {x[0], x[1], x[2], x[3] | (b << 31)};
    uint32_t s[4] = {blk[0], blk[1], blk[2], blk[3]};
    aes128_encrypt_rk(tb, c_iv.a, s);
    out[0] = s[0] ^ blk[0];
    out[1] = s[1] ^ blk[1];
    out[2] = s[2] ^ blk[2];
    out[3] = (s[3] ^ blk[3]) & 0x7fffffffu;
}

__device__ __forceinline__ void prf_node_sha(const uint32_t x[4], uint32_t b, uint32_t out[4]) {
    uint32_t W[16] = {bswap32(x[0]), bswap32(x[1]), bswap32(x[2]), bswap32(x[3]),
                      (b << 24) | 0x00800000u, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 17u * 8u};
    uint32_t H[8];
    sha256_init(H);
    sha256_compress(H, W);
    out[0] = bswap32(H[0]);
    out[1] = bswap32(H[1]);
    out[2] = bswap32(H[2]);
    out[3] = bswap32(H[3]);
}

// ---- the disclosed seed stack, passed by value as a kernel argument ------

struct DsArg {
    uint32_t count;
    uint32_t depth[32];
    uint32_t index[32];
    uint32_t v[32][4];
};

// SR(ds, i'): covering node, or -1 ("bottom")
__device__ __forceinline__ int ds_cover(const DsArg& ds, uint64_t ip) {
    int k = (int)ds.count - 1;
    if (k < 0) return -1;
    if (ip >= (((uint64_t)ds.index[k] + 1) << ds.depth[k])) return -1;
    while (ip < ((uint64_t)ds.index[k] << ds.depth[k])) {
        if (--k < 0) return -1;
    }
    return k;
}

}  // namespace poslo
