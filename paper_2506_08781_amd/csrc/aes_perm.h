// AES-128 rounds for gfx950 with byte-addressed, bank-replicated T-tables in
// LDS (device only).
//
// Layout: 64 copies of each table, entry x of copy c at byte address
// (table << 16) | (x << 8) | (c << 2).  Lane l reads copy l mod 64, so a
// wave's 64 lookups fall in 64 distinct banks whatever the indices are, and
// the address of "byte k of w in table t" is one v_perm_b32 that drops byte
// k of w into bits 8..15 of a per-lane base word holding (t << 16) | (l << 2).
// Every address is below 2 * 64 KB by construction (byte 3 is forced to zero,
// byte 2 is the table bit).
//
// NT = 2 keeps te0 and te0 rotated by 16 (128 KB); the odd rotations are one
// v_alignbit away.  NT = 1 keeps te0 only (64 KB) and rotates for the rest.
//
// CP = 32 copies: entry x of copy c of table t at (t1 << 16) | (x << 8) |
// (t0 << 7) | (c << 2) with t = t0 + 2 t1, lane l reading copy l mod 32, so
// NT = 2 (te0, te0 rotated by 16) fits in 64 KB and NT = 4 (all four
// rotations, no rotate instructions) in 128 KB.  The two lanes of a
// wave that share a copy (l and l + 32) are served in different halves of
// the wave's LDS access when the LDS takes 32 lanes per cycle, which is what
// the PMC counters confirm (no bank conflicts on gfx950).
// S-box bytes for the key schedule and the final round come out of te0 (S
// sits in bytes 1 and 2) and are merged with v_perm_b32.  Three-input XORs
// use v_bitop3_b32.
#pragma once

#include "device_hash.h"

namespace poslo {

// v_perm_b32 selectors: byte0 <- base byte 0 (lane offset), byte1 <- byte k of
// w, byte2 <- base byte 2 (table bit), byte3 <- 0
__device__ __forceinline__ uint32_t perm_sel(int k) { return 0x0c020000u | ((uint32_t)(4 + k) << 8); }

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

template <int NT, int CP = 64>
struct PermTables {
    static_assert((CP == 64 && NT <= 2) || (CP == 32 && (NT == 1 || NT == 2 || NT == 4)),
                  "64 copies of one or two tables, or 32 copies of one, two or four");
    const uint8_t* lds;
    uint32_t base0;  // lane offset: te0
    uint32_t base1;  // te0 rotated by 8 (NT = 4)
    uint32_t base2;  // te0 rotated by 16 (NT >= 2)
    uint32_t base3;  // te0 rotated by 24 (NT = 4)

    __device__ __forceinline__ uint32_t ld(uint32_t addr) const {
        return *reinterpret_cast<const uint32_t*>(lds + addr);
    }
    // te0[byte k of w]
    __device__ __forceinline__ uint32_t T0(uint32_t w, int k) const {
        return ld(__builtin_amdgcn_perm(w, base0, perm_sel(k)));
    }
    // te0[byte k of w] rotated left by 8
    __device__ __forceinline__ uint32_t T1(uint32_t w, int k) const {
        if constexpr (NT == 4) return ld(__builtin_amdgcn_perm(w, base1, perm_sel(k)));
        else return rotl32(T0(w, k), 8);
    }
    // te0[byte k of w] rotated left by 16
    __device__ __forceinline__ uint32_t T2(uint32_t w, int k) const {
        if constexpr (NT >= 2) return ld(__builtin_amdgcn_perm(w, base2, perm_sel(k)));
        else return rotl32(T0(w, k), 16);
    }
    // te0[byte k of w] rotated left by 24
    __device__ __forceinline__ uint32_t T3(uint32_t w, int k) const {
        if constexpr (NT == 4) return ld(__builtin_amdgcn_perm(w, base3, perm_sel(k)));
        else return rotl32(T2(w, k), 8);
    }
};

// Word index (t << 14) | (x << 6) | c.  Lane l of each wave loads te0[4l..4l+3]
// once; then, per entry, the owning lane's word is read into a scalar
// register and the wave writes the entry's 64 copies (64 consecutive words,
// one store).  Needs a workgroup size that is a multiple of 64.
template <int NT, int CP = 64>
__device__ __forceinline__ void perm_tables_fill(uint32_t* lds) {
    if constexpr (CP == 32) {
        // word (t1 << 14) | (x << 6) | (t0 << 5) | c holds te0[x] rotated by
        // 16 t0 (NT = 2) or by 8 (t0 + 2 t1) (NT = 4)
        for (uint32_t w = threadIdx.x; w < NT * 256u * 32u; w += blockDim.x) {
            const uint32_t x = (w >> 6) & 255u, t0 = (w >> 5) & 1u, t1 = (w >> 14) & 1u;
            lds[w] = rotl32(c_aes.te0[x], NT == 4 ? 8 * (t0 + 2 * t1) : 16 * t0);
        }
        return;
    }
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const uint32_t v0 = c_aes.te0[4 * lane], v1 = c_aes.te0[4 * lane + 1], v2 = c_aes.te0[4 * lane + 2],
                   v3 = c_aes.te0[4 * lane + 3];
    for (uint32_t e = wave; e < NT * 256u; e += nwaves) {
        const uint32_t x = e & 255u, q = x & 3u;
        const uint32_t mine = q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3;
        const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)mine, (int)(x >> 2));
        lds[(e << 6) | lane] = rotl32(v, 16 * (e >> 8));
    }
}

template <int NT, int CP = 64>
__device__ __forceinline__ PermTables<NT, CP> perm_tables(const uint32_t* lds) {
    const uint32_t lane4 = (threadIdx.x & (CP - 1u)) << 2;
    const uint8_t* p = reinterpret_cast<const uint8_t*>(lds);
    if constexpr (CP == 64) return PermTables<NT, CP>{p, lane4, 0u, lane4 | (1u << 16), 0u};
    else if constexpr (NT == 4)
        return PermTables<NT, CP>{p, lane4, lane4 | 0x80u, lane4 | (1u << 16), lane4 | 0x80u | (1u << 16)};
    else return PermTables<NT, CP>{p, lane4, 0u, lane4 | 0x80u, 0u};
}

// full round: out_c = T0[s_c.b0] ^ T1[s_{c+1}.b1] ^ T2[s_{c+2}.b2] ^ T3[s_{c+3}.b3] ^ k_c
template <int NT, int CP>
__device__ __forceinline__ void pround(const PermTables<NT, CP>& tb, uint32_t s[4], const uint32_t k[4]) {
    uint32_t n[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        if constexpr (NT == 4) {
            n[c] = xor3(xor3(tb.T0(s[c], 0), tb.T1(s[(c + 1) & 3], 1), tb.T2(s[(c + 2) & 3], 2)),
                        tb.T3(s[(c + 3) & 3], 3), k[c]);
        } else if constexpr (NT == 2) {
            // T1[y] ^ T3[z] = rot8(T0[y] ^ T2[z]): one rotation, and the
            // xors (which issue faster than rotations) take the rest
            const uint32_t a = tb.T0(s[c], 0), d = tb.T2(s[(c + 2) & 3], 2);
            const uint32_t v = tb.T0(s[(c + 1) & 3], 1) ^ tb.T2(s[(c + 3) & 3], 3);
            n[c] = xor3(a, d, k[c]) ^ rotl32(v, 8);
        } else {
            uint32_t a = tb.T0(s[c], 0);
            uint32_t b = rotl32(tb.T0(s[(c + 1) & 3], 1), 8);
            uint32_t d = tb.T2(s[(c + 2) & 3], 2);
            uint32_t e = rotl32(tb.T2(s[(c + 3) & 3], 3), 8);
            n[c] = xor3(xor3(a, b, d), e, k[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; c++) s[c] = n[c];
}

// S-box bytes (S at byte 1 of te0 entries a, b, c, d) merged into
// S[a] | S[b] << 8 | S[c] << 16 | S[d] << 24
__device__ __forceinline__ uint32_t sbytes(uint32_t ta, uint32_t tb_, uint32_t tc, uint32_t td) {
    uint32_t lo = __builtin_amdgcn_perm(ta, tb_, 0x0c0c0105u);  // byte0 <- ta.1, byte1 <- tb.1
    uint32_t hi = __builtin_amdgcn_perm(tc, td, 0x01050c0cu);   // byte2 <- tc.1, byte3 <- td.1
    return lo | hi;
}

// final round: S bytes, ShiftRows, AddRoundKey
template <int NT, int CP>
__device__ __forceinline__ void pround_final(const PermTables<NT, CP>& tb, uint32_t s[4], const uint32_t k[4]) {
    uint32_t n[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        n[c] = sbytes(tb.T0(s[c], 0), tb.T0(s[(c + 1) & 3], 1), tb.T0(s[(c + 2) & 3], 2),
                      tb.T0(s[(c + 3) & 3], 3)) ^
               k[c];
    }
#pragma unroll
    for (int c = 0; c < 4; c++) s[c] = n[c];
}

// next round key: w0 ^= SubWord(RotWord(w3)) ^ rcon, then the chain
template <int NT, int CP>
__device__ __forceinline__ void pnext_key(const PermTables<NT, CP>& tb, uint32_t k[4], uint32_t rcon) {
    uint32_t w3 = k[3];
    uint32_t sub = sbytes(tb.T0(w3, 1), tb.T0(w3, 2), tb.T0(w3, 3), tb.T0(w3, 0));
    k[0] = xor3(k[0], sub, rcon);
    k[1] ^= k[0];
    k[2] ^= k[1];
    k[3] ^= k[2];
}

// the ten Rcon values of AES-128
__device__ __forceinline__ constexpr uint32_t prcon(int r) {
    return r == 1 ? 0x01u : r == 2 ? 0x02u : r == 3 ? 0x04u : r == 4 ? 0x08u : r == 5 ? 0x10u
         : r == 6 ? 0x20u : r == 7 ? 0x40u : r == 8 ? 0x80u : r == 9 ? 0x1bu : 0x36u;
}

// E_key(s) with the key schedule on the fly; two independent encryptions
// interleaved (the two MDC-2 lanes), rounds fully unrolled
template <int NT, int CP>
__device__ __forceinline__ void penc2_otf(const PermTables<NT, CP>& tb, const uint32_t keya[4], uint32_t sa[4],
                                          const uint32_t keyb[4], uint32_t sb[4]) {
    uint32_t ka[4] = {keya[0], keya[1], keya[2], keya[3]};
    uint32_t kb[4] = {keyb[0], keyb[1], keyb[2], keyb[3]};
#pragma unroll
    for (int c = 0; c < 4; c++) {
        sa[c] ^= ka[c];
        sb[c] ^= kb[c];
    }
#pragma unroll
    for (int r = 1; r <= 9; r++) {
        pnext_key(tb, ka, prcon(r));
        pnext_key(tb, kb, prcon(r));
        pround(tb, sa, ka);
        pround(tb, sb, kb);
    }
    pnext_key(tb, ka, prcon(10));
    pnext_key(tb, kb, prcon(10));
    pround_final(tb, sa, ka);
    pround_final(tb, sb, kb);
}

// E with a precomputed schedule rk[44]
template <int NT, int CP>
__device__ __forceinline__ void penc_rk(const PermTables<NT, CP>& tb, const uint32_t* rk, uint32_t s[4]) {
#pragma unroll
    for (int c = 0; c < 4; c++) s[c] ^= rk[c];
#pragma unroll
    for (int r = 1; r <= 9; r++) pround(tb, s, rk + 4 * r);
    pround_final(tb, s, rk + 40);
}

// two encryptions under two precomputed schedules, interleaved
template <int NT, int CP>
__device__ __forceinline__ void penc2_rk(const PermTables<NT, CP>& tb, const uint32_t* rka, uint32_t sa[4],
                                         const uint32_t* rkb, uint32_t sb[4]) {
#pragma unroll
    for (int c = 0; c < 4; c++) {
        sa[c] ^= rka[c];
        sb[c] ^= rkb[c];
    }
#pragma unroll
    for (int r = 1; r <= 9; r++) {
        pround(tb, sa, rka + 4 * r);
        pround(tb, sb, rkb + 4 * r);
    }
    pround_final(tb, sa, rka + 40);
    pround_final(tb, sb, rkb + 40);
}

}  // namespace poslo
