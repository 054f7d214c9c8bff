// AES-128 for the MMO and MDC-2 constructions (FIPS-197), host and device.
//
// MMO and MDC-2 re-key the cipher with a data-dependent chaining value for
// every 16-byte block (paper, Definitions "MMO" and "MDC-2"; the GPU section
// notes that key expansion therefore runs on the device for every block).
// The cipher here expands the key on the fly, one round key per round, and
// uses the 32-bit T-table formulation: one table lookup per state byte per
// round, four tables related by byte rotation.
//
// State convention: the 16-byte block is four little-endian 32-bit words,
// one per column; byte r of word c is state row r, column c.
#pragma once

#include "common.h"

namespace poslo {

// ---- table generation (compile time, from the S-box definition) ----------

PDC uint8_t gf_mul(uint8_t a, uint8_t b) {
    uint8_t r = 0;
    for (int i = 0; i < 8; i++) {
        if (b & 1) r ^= a;
        uint8_t hi = a & 0x80;
        a = (uint8_t)(a << 1);
        if (hi) a ^= 0x1b;
        b >>= 1;
    }
    return r;
}

PDC uint8_t gf_pow254(uint8_t a) {  // a^-1 in GF(2^8), with 0 -> 0
    uint8_t r = 1, base = a;
    int e = 254;
    while (e) {
        if (e & 1) r = gf_mul(r, base);
        base = gf_mul(base, base);
        e >>= 1;
    }
    return r;
}

PDC uint8_t rotl8(uint8_t x, int n) { return (uint8_t)((x << n) | (x >> (8 - n))); }

struct AesTables {
    uint8_t sbox[256];
    uint32_t te0[256];  // bytes (2S, S, S, 3S), little-endian
};

PDC AesTables make_aes_tables() {
    AesTables t{};
    for (int x = 0; x < 256; x++) {
        uint8_t b = gf_pow254((uint8_t)x);
        uint8_t s = (uint8_t)(b ^ rotl8(b, 1) ^ rotl8(b, 2) ^ rotl8(b, 3) ^ rotl8(b, 4) ^ 0x63);
        t.sbox[x] = s;
        uint32_t s2 = gf_mul(s, 2), s3 = gf_mul(s, 3);
        t.te0[x] = s2 | ((uint32_t)s << 8) | ((uint32_t)s << 16) | (s3 << 24);
    }
    return t;
}

// Rcon for rounds 1..10
PDC uint32_t aes_rcon(int i) {
    uint8_t r = 1;
    for (int k = 1; k < i; k++) r = gf_mul(r, 2);
    return r;
}

inline constexpr AesTables kAesTables = make_aes_tables();

// ---- round functions, generic over the table reader ---------------------
//
// A table reader T provides t0..t3(x) for a byte value x: te0[x] rotated
// left by 0, 8, 16, 24 bits.  The host reader uses the constant table; the
// device kernels read bank-replicated copies held in LDS.

struct HostTables {
    PD uint32_t t0(uint32_t x) const { return kAesTables.te0[x]; }
    PD uint32_t t1(uint32_t x) const { return rotl32(kAesTables.te0[x], 8); }
    PD uint32_t t2(uint32_t x) const { return rotl32(kAesTables.te0[x], 16); }
    PD uint32_t t3(uint32_t x) const { return rotl32(kAesTables.te0[x], 24); }
};

PD uint32_t b0(uint32_t w) { return w & 0xffu; }
PD uint32_t b1(uint32_t w) { return (w >> 8) & 0xffu; }
PD uint32_t b2(uint32_t w) { return (w >> 16) & 0xffu; }
PD uint32_t b3(uint32_t w) { return w >> 24; }

// next round key from the previous one (FIPS-197 5.2 for Nk = 4):
// w4 = w0 ^ SubWord(RotWord(w3)) ^ Rcon, then chained xors.  The S-box byte is
// taken from whichever rotated table holds plain S at that byte position.
template <class T>
PD void aes_next_key(const T& tb, uint32_t k[4], uint32_t rcon) {
    uint32_t w3 = k[3];
    uint32_t sub = (tb.t2(b1(w3)) & 0x000000ffu) | (tb.t3(b2(w3)) & 0x0000ff00u) |
                   (tb.t0(b3(w3)) & 0x00ff0000u) | (tb.t1(b0(w3)) & 0xff000000u);
    k[0] ^= sub ^ rcon;
    k[1] ^= k[0];
    k[2] ^= k[1];
    k[3] ^= k[2];
}

// one full round: SubBytes, ShiftRows, MixColumns via tables, then AddRoundKey
template <class T>
PD void aes_round(const T& tb, uint32_t s[4], const uint32_t k[4]) {
    uint32_t n0 = tb.t0(b0(s[0])) ^ tb.t1(b1(s[1])) ^ tb.t2(b2(s[2])) ^ tb.t3(b3(s[3])) ^ k[0];
    uint32_t n1 = tb.t0(b0(s[1])) ^ tb.t1(b1(s[2])) ^ tb.t2(b2(s[3])) ^ tb.t3(b3(s[0])) ^ k[1];
    uint32_t n2 = tb.t0(b0(s[2])) ^ tb.t1(b1(s[3])) ^ tb.t2(b2(s[0])) ^ tb.t3(b3(s[1])) ^ k[2];
    uint32_t n3 = tb.t0(b0(s[3])) ^ tb.t1(b1(s[0])) ^ tb.t2(b2(s[1])) ^ tb.t3(b3(s[2])) ^ k[3];
    s[0] = n0;
    s[1] = n1;
    s[2] = n2;
    s[3] = n3;
}

// final round: no MixColumns; S at byte r comes from the table whose byte r is S
template <class T>
PD void aes_final_round(const T& tb, uint32_t s[4], const uint32_t k[4]) {
    uint32_t n[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        n[c] = ((tb.t2(b0(s[c])) & 0x000000ffu) | (tb.t3(b1(s[(c + 1) & 3])) & 0x0000ff00u) |
                (tb.t0(b2(s[(c + 2) & 3])) & 0x00ff0000u) | (tb.t1(b3(s[(c + 3) & 3])) & 0xff000000u)) ^
               k[c];
    }
    s[0] = n[0];
    s[1] = n[1];
    s[2] = n[2];
    s[3] = n[3];
}

// E_key(s) in place with the key schedule computed round by round
template <class T>
PD void aes128_encrypt_otf(const T& tb, const uint32_t key[4], uint32_t s[4]) {
    uint32_t k[4] = {key[0], key[1], key[2], key[3]};
    s[0] ^= k[0];
    s[1] ^= k[1];
    s[2] ^= k[2];
    s[3] ^= k[3];
    for (int r = 1; r <= 9; r++) {
        aes_next_key(tb, k, aes_rcon(r));
        aes_round(tb, s, k);
    }
    aes_next_key(tb, k, aes_rcon(10));
    aes_final_round(tb, s, k);
}

// Two independent encryptions interleaved round by round (the two MDC-2
// lanes), which doubles the independent work in flight per lane.
template <class T>
PD void aes128_encrypt2_otf(const T& tb, const uint32_t keya[4], uint32_t sa[4],
                            const uint32_t keyb[4], uint32_t sb[4]) {
    uint32_t ka[4] = {keya[0], keya[1], keya[2], keya[3]};
    uint32_t kb[4] = {keyb[0], keyb[1], keyb[2], keyb[3]};
#pragma unroll
    for (int c = 0; c < 4; c++) {
        sa[c] ^= ka[c];
        sb[c] ^= kb[c];
    }
#pragma unroll 1
    for (int r = 1; r <= 9; r++) {
        uint32_t rc = aes_rcon(r);
        aes_next_key(tb, ka, rc);
        aes_next_key(tb, kb, rc);
        aes_round(tb, sa, ka);
        aes_round(tb, sb, kb);
    }
    aes_next_key(tb, ka, 0x36u);
    aes_next_key(tb, kb, 0x36u);
    aes_final_round(tb, sa, ka);
    aes_final_round(tb, sb, kb);
}

// E with a precomputed schedule rk[44] (11 round keys)
template <class T>
PD void aes128_encrypt_rk(const T& tb, const uint32_t* rk, uint32_t s[4]) {
    s[0] ^= rk[0];
    s[1] ^= rk[1];
    s[2] ^= rk[2];
    s[3] ^= rk[3];
    for (int r = 1; r <= 9; r++) aes_round(tb, s, rk + 4 * r);
    aes_final_round(tb, s, rk + 40);
}

template <class T>
PD void aes128_expand(const T& tb, const uint32_t key[4], uint32_t rk[44]) {
    uint32_t k[4] = {key[0], key[1], key[2], key[3]};
    for (int c = 0; c < 4; c++) rk[c] = k[c];
    for (int r = 1; r <= 10; r++) {
        aes_next_key(tb, k, aes_rcon(r));
        for (int c = 0; c < 4; c++) rk[4 * r + c] = k[c];
    }
}

// ---- MMO / MDC-2 initial values and their (constant) key schedules ------

PDC uint32_t kIvA = 0x52525252u;  // MMO and first MDC-2 lane: 0x52 x 16
PDC uint32_t kIvB = 0x25252525u;  // second MDC-2 lane: 0x25 x 16

struct IvSchedules {
    uint32_t a[44];
    uint32_t b[44];
};

struct ConstexprTables {
    PDC uint32_t t0(uint32_t x) const { return kAesTables.te0[x]; }
    PDC uint32_t t1(uint32_t x) const { return (kAesTables.te0[x] << 8) | (kAesTables.te0[x] >> 24); }
    PDC uint32_t t2(uint32_t x) const { return (kAesTables.te0[x] << 16) | (kAesTables.te0[x] >> 16); }
    PDC uint32_t t3(uint32_t x) const { return (kAesTables.te0[x] << 24) | (kAesTables.te0[x] >> 8); }
};

PDC IvSchedules make_iv_schedules() {
    IvSchedules s{};
    ConstexprTables tb{};
    uint32_t ka[4] = {kIvA, kIvA, kIvA, kIvA};
    uint32_t kb[4] = {kIvB, kIvB, kIvB, kIvB};
    for (int c = 0; c < 4; c++) {
        s.a[c] = ka[c];
        s.b[c] = kb[c];
    }
    for (int r = 1; r <= 10; r++) {
        uint32_t rc = aes_rcon(r);
        for (int lane = 0; lane < 2; lane++) {
            uint32_t* k = lane ? kb : ka;
            uint32_t w3 = k[3];
            uint32_t sub = (tb.t2((w3 >> 8) & 0xff) & 0xffu) | (tb.t3((w3 >> 16) & 0xff) & 0xff00u) |
                           (tb.t0(w3 >> 24) & 0xff0000u) | (tb.t1(w3 & 0xff) & 0xff000000u);
            k[0] ^= sub ^ rc;
            k[1] ^= k[0];
            k[2] ^= k[1];
            k[3] ^= k[2];
        }
        for (int c = 0; c < 4; c++) {
            s.a[4 * r + c] = ka[c];
            s.b[4 * r + c] = kb[c];
        }
    }
    return s;
}

inline constexpr IvSchedules kIvSchedules = make_iv_schedules();

}  // namespace poslo
