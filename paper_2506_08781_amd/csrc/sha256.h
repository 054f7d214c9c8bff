// SHA-256 compression (FIPS 180-4, section 6.2.2), host and device.
// Message words are big-endian; state is eight 32-bit words.
#pragma once

#include "common.h"

namespace poslo {

struct Sha256Consts {
    uint32_t k[64];
    uint32_t h0[8];
};

inline constexpr Sha256Consts kSha256 = {
    {0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u, 0xab1c5ed5u,
     0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu, 0x9bdc06a7u, 0xc19bf174u,
     0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, 0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau,
     0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, 0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u,
     0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, 0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u,
     0xa2bfe8a1u, 0xa81a664bu, 0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u,
     0x19a4c116u, 0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u,
     0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u},
    {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u, 0xa54ff53au, 0x510e527fu, 0x9b05688cu, 0x1f83d9abu, 0x5be0cd19u}};

// three-input xor and majority: one v_bitop3_b32 each on the device (both
// functions are symmetric in their inputs, so the truth table does not
// depend on operand order), plain C on the host
__device__ __forceinline__ uint32_t xor3_u32(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__host__ inline uint32_t xor3_u32(uint32_t a, uint32_t b, uint32_t c) { return a ^ b ^ c; }
__device__ __forceinline__ uint32_t maj3_u32(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xe8);
}
__host__ inline uint32_t maj3_u32(uint32_t a, uint32_t b, uint32_t c) { return (a & b) | (c & (a | b)); }

PD uint32_t sha_ch(uint32_t e, uint32_t f, uint32_t g) { return g ^ (e & (f ^ g)); }
PD uint32_t sha_maj(uint32_t a, uint32_t b, uint32_t c) { return maj3_u32(a, b, c); }
PD uint32_t sha_S0(uint32_t a) { return xor3_u32(rotr32(a, 2), rotr32(a, 13), rotr32(a, 22)); }
PD uint32_t sha_S1(uint32_t e) { return xor3_u32(rotr32(e, 6), rotr32(e, 11), rotr32(e, 25)); }
PD uint32_t sha_s0(uint32_t w) { return xor3_u32(rotr32(w, 7), rotr32(w, 18), w >> 3); }
PD uint32_t sha_s1(uint32_t w) { return xor3_u32(rotr32(w, 17), rotr32(w, 19), w >> 10); }

// H <- compress(H, W[0..15]); W is consumed as a 16-word rolling schedule
PD void sha256_compress(uint32_t H[8], uint32_t W[16]) {
    uint32_t a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7];
#pragma unroll
    for (int t = 0; t < 64; t++) {
        uint32_t w;
        if (t < 16) {
            w = W[t];
        } else {
            w = sha_s1(W[(t - 2) & 15]) + W[(t - 7) & 15] + sha_s0(W[(t - 15) & 15]) + W[t & 15];
            W[t & 15] = w;
        }
        uint32_t T1 = h + sha_S1(e) + sha_ch(e, f, g) + kSha256.k[t] + w;
        uint32_t T2 = sha_S0(a) + sha_maj(a, b, c);
        h = g;
        g = f;
        f = e;
        e = d + T1;
        d = c;
        c = b;
        b = a;
        a = T1 + T2;
    }
    H[0] += a;
    H[1] += b;
    H[2] += c;
    H[3] += d;
    H[4] += e;
    H[5] += f;
    H[6] += g;
    H[7] += h;
}

PD void sha256_init(uint32_t H[8]) {
#pragma unroll
    for (int i = 0; i < 8; i++) H[i] = kSha256.h0[i];
}

}  // namespace poslo
