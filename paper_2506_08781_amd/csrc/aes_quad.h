// AES-128 spread over the four lanes of a quad (lanes 4q..4q+3; lane c holds
// column c of the state), for chains of dependent encryptions such as the
// seed-tree walk, where latency rather than throughput decides.  Per round
// a lane does one column: three DPP moves fetch the other columns' words
// from its quad, then four lookups.  The key schedule runs redundantly in all
// four lanes, off the state's critical path.  Every lane of a quad must take
// part (the four lanes of a quad work on the same block).
#pragma once

#include "aes128.h"
#include "device_hash.h"

namespace poslo {

// the word of column (c + D) & 3 of this lane's quad
template <int D>
__device__ __forceinline__ uint32_t quad_rot(uint32_t v) {
    constexpr int ctrl = D == 1 ? 0x39 : D == 2 ? 0x4e : 0x93;  // quad_perm [c + D mod 4]
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t pick4(const uint32_t k[4], uint32_t c) {
    return c == 0 ? k[0] : c == 1 ? k[1] : c == 2 ? k[2] : k[3];
}

// all four columns, in order, in every lane of the quad
__device__ __forceinline__ void quad_gather(uint32_t v, uint32_t c, uint32_t w[4]) {
    const uint32_t r1 = quad_rot<1>(v), r2 = quad_rot<2>(v), r3 = quad_rot<3>(v);
#pragma unroll
    for (uint32_t j = 0; j < 4; j++) {
        const uint32_t d = (j - c) & 3u;  // column j is d columns to the right
        w[j] = d == 0 ? v : d == 1 ? r1 : d == 2 ? r2 : r3;
    }
}

template <class T>
__device__ __forceinline__ uint32_t quad_round(const T& tb, uint32_t s, uint32_t kc) {
    const uint32_t s1 = quad_rot<1>(s), s2 = quad_rot<2>(s), s3 = quad_rot<3>(s);
    return tb.t0(b0(s)) ^ tb.t1(b1(s1)) ^ tb.t2(b2(s2)) ^ tb.t3(b3(s3)) ^ kc;
}

template <class T>
__device__ __forceinline__ uint32_t quad_final_round(const T& tb, uint32_t s, uint32_t kc) {
    const uint32_t s1 = quad_rot<1>(s), s2 = quad_rot<2>(s), s3 = quad_rot<3>(s);
    return ((tb.t2(b0(s)) & 0x000000ffu) | (tb.t3(b1(s1)) & 0x0000ff00u) | (tb.t0(b2(s2)) & 0x00ff0000u) |
            (tb.t1(b3(s3)) & 0xff000000u)) ^
           kc;
}

// column c of E(s) under a precomputed schedule rk[44]
template <class T>
__device__ __forceinline__ uint32_t quad_encrypt_rk(const T& tb, const uint32_t* rk, uint32_t s, uint32_t c) {
    s ^= rk[c];
#pragma unroll
    for (int r = 1; r <= 9; r++) s = quad_round(tb, s, rk[4 * r + c]);
    return quad_final_round(tb, s, rk[40 + c]);
}

// column c of E_key(s), key (all four words) scheduled on the fly
template <class T>
__device__ __forceinline__ uint32_t quad_encrypt_otf(const T& tb, const uint32_t key[4], uint32_t s, uint32_t c) {
    uint32_t k[4] = {key[0], key[1], key[2], key[3]};
    s ^= pick4(k, c);
#pragma unroll
    for (int r = 1; r <= 9; r++) {
        aes_next_key(tb, k, aes_rcon(r));
        s = quad_round(tb, s, pick4(k, c));
    }
    aes_next_key(tb, k, aes_rcon(10));
    return quad_final_round(tb, s, pick4(k, c));
}

// column c of PRF_b(x) for a 16-byte tree node x (column c of x in xc):
// MMO over x || b, the first block under the IV's schedule, the second
// keyed by the chaining value
template <class T>
__device__ __forceinline__ uint32_t quad_prf_node(const T& tb, uint32_t xc, uint32_t b, uint32_t c) {
    const uint32_t h1c = quad_encrypt_rk(tb, c_iv.a, xc, c) ^ xc;
    uint32_t h1[4];
    quad_gather(h1c, c, h1);
    const uint32_t bc = c == 0 ? b : 0u;
    return quad_encrypt_otf(tb, h1, bc, c) ^ bc;
}

// the same at kappa = 127: PRF_b(x) is the one MMO block x + b * 2^127
// under the IV's schedule, reduced mod 2^127 (x has bit 127 clear)
template <class T>
__device__ __forceinline__ uint32_t quad_prf_node127(const T& tb, uint32_t xc, uint32_t b, uint32_t c) {
    const uint32_t blk = c == 3 ? xc | (b << 31) : xc;
    const uint32_t h = quad_encrypt_rk(tb, c_iv.a, blk, c) ^ blk;
    return c == 3 ? h & 0x7fffffffu : h;
}

// the AES epoch row of seed x_0[i] (column c in xc): words 4r + c of the
// schedule of the MMO chaining value after x_0[i]'s block, and word 44 + c
// = column c of x_0[i]
template <class T>
__device__ __forceinline__ void quad_epoch_row(const T& tb, uint32_t xc, uint32_t c, uint32_t* e) {
    const uint32_t h1c = quad_encrypt_rk(tb, c_iv.a, xc, c) ^ xc;
    uint32_t k[4];
    quad_gather(h1c, c, k);
    e[c] = pick4(k, c);
#pragma unroll
    for (int r = 1; r <= 10; r++) {
        aes_next_key(tb, k, aes_rcon(r));
        e[4 * r + c] = pick4(k, c);
    }
    e[44 + c] = xc;
}

}  // namespace poslo
