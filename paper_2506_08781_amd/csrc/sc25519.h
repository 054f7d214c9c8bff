// Scalars modulo the group order q = 2^252 + c, c = 27742317777372353535851937790883648493.
// Scalars and digests are little-endian arrays of 32-bit limbs.
//
// Reduction uses 2^252 = -c (mod q): a value X = hi * 2^252 + lo is congruent
// to lo - hi * c.  For X below 2^288, hi < 2^36 and hi * c < 2^161 < q, so one
// conditional addition of q yields the canonical residue.
#pragma once

#include "common.h"

namespace poslo {

#define POSLO_SC_Q {0x5cf5d3edu, 0x5812631au, 0xa2f79cd6u, 0x14def9deu, 0u, 0u, 0u, 0x10000000u}
#define POSLO_SC_C {0x5cf5d3edu, 0x5812631au, 0xa2f79cd6u, 0x14def9deu}

// r = X mod q for X < 2^288 given as nine limbs
PD void sc_reduce288(uint32_t r[8], const uint32_t x[9]) {
    const uint32_t q[8] = POSLO_SC_Q;
    const uint32_t c[4] = POSLO_SC_C;
    uint64_t hi = ((uint64_t)x[8] << 4) | (x[7] >> 28);
    uint32_t h0 = (uint32_t)hi, h1 = (uint32_t)(hi >> 32);
    // hc = hi * c, six limbs
    uint32_t hc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t cy = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        cy += (uint64_t)c[i] * h0;
        hc[i] = (uint32_t)cy;
        cy >>= 32;
    }
    hc[4] = (uint32_t)cy;
    cy = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        cy += (uint64_t)c[i] * h1 + hc[i + 1];
        hc[i + 1] = (uint32_t)cy;
        cy >>= 32;
    }
    hc[5] = (uint32_t)cy;
    // r = lo - hc (mod 2^256), lo = low 252 bits of X
    int64_t b = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        uint32_t lo = (i == 7) ? (x[7] & 0x0fffffffu) : x[i];
        b += (int64_t)lo - (int64_t)hc[i];
        r[i] = (uint32_t)b;
        b >>= 32;
    }
    if (b) {  // negative: add q
        uint64_t a = 0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            a += (uint64_t)r[i] + q[i];
            r[i] = (uint32_t)a;
            a >>= 32;
        }
    }
}

PD void sc_reduce256(uint32_t r[8], const uint32_t x[8]) {
    uint32_t y[9];
#pragma unroll
    for (int i = 0; i < 8; i++) y[i] = x[i];
    y[8] = 0;
    sc_reduce288(r, y);
}

// s < q (canonical scalar)
PD bool sc_is_canonical(const uint32_t s[8]) {
    const uint32_t q[8] = POSLO_SC_Q;
    for (int i = 7; i >= 0; i--) {
        if (s[i] < q[i]) return true;
        if (s[i] > q[i]) return false;
    }
    return false;  // equal to q
}

// acc (nine limbs) += x (eight limbs): the lazy sum of raw 256-bit digests
PD void acc288_add256(uint32_t acc[9], const uint32_t x[8]) {
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += (uint64_t)acc[i] + x[i];
        acc[i] = (uint32_t)c;
        c >>= 32;
    }
    acc[8] += (uint32_t)c;
}

PD void acc288_add(uint32_t acc[9], const uint32_t x[9]) {
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        c += (uint64_t)acc[i] + x[i];
        acc[i] = (uint32_t)c;
        c >>= 32;
    }
}

// (a + b) mod q for canonical a, b
PD void sc_add(uint32_t r[8], const uint32_t a[8], const uint32_t b[8]) {
    uint32_t t[9];
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += (uint64_t)a[i] + b[i];
        t[i] = (uint32_t)c;
        c >>= 32;
    }
    t[8] = (uint32_t)c;
    sc_reduce288(r, t);
}

}  // namespace poslo
