// Arithmetic in GF(p), p = 2^255 - 19, for the edwards25519 group that stands
// in for the paper's elliptic curve (the paper's curve constants are not
// given; the scheme only needs a prime-order group with a 256-bit-class q).
//
// Elements are eight 32-bit little-endian limbs holding a value below 2^256
// ("weakly reduced", congruent to the element); fe_freeze gives the
// canonical representative below p.  Reduction uses 2^256 = 38 (mod p).
#pragma once

#include "common.h"

namespace poslo {

struct fe {
    uint32_t v[8];
};

PD void fe_set(fe& r, uint32_t x) {
    r.v[0] = x;
#pragma unroll
    for (int i = 1; i < 8; i++) r.v[i] = 0;
}

PD void fe_copy(fe& r, const fe& a) {
#pragma unroll
    for (int i = 0; i < 8; i++) r.v[i] = a.v[i];
}

PD void fe_add(fe& r, const fe& a, const fe& b) {
    uint32_t t[8];
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += (uint64_t)a.v[i] + b.v[i];
        t[i] = (uint32_t)c;
        c >>= 32;
    }
    c *= 38;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += t[i];
        r.v[i] = (uint32_t)c;
        c >>= 32;
    }
    // a second wrap leaves r < 38, so adding 38 cannot carry
    r.v[0] += (uint32_t)c * 38u;
}

PD void fe_sub(fe& r, const fe& a, const fe& b) {
    uint32_t t[8];
    int64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += (int64_t)a.v[i] - (int64_t)b.v[i];
        t[i] = (uint32_t)c;
        c >>= 32;  // 0 or -1
    }
    // a borrow means the value is t - 2^256 = t - 38 (mod p)
    c *= 38;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += t[i];
        r.v[i] = (uint32_t)c;
        c >>= 32;
    }
    // a second borrow leaves r >= 2^256 - 38, so subtracting 38 cannot borrow
    r.v[0] -= (uint32_t)(-c) * 38u;
}

// a * k for a small constant k < 2^26 (2^256 = 38 mod p)
PD void fe_mul_small(fe& r, const fe& a, uint32_t k) {
    uint32_t t[8];
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += (uint64_t)a.v[i] * k;
        t[i] = (uint32_t)c;
        c >>= 32;
    }
    c *= 38;  // c < 2^26, so 38c < 2^32
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += t[i];
        r.v[i] = (uint32_t)c;
        c >>= 32;
    }
    // a second wrap leaves r < 2^32 - 38, so adding 38 cannot carry
    r.v[0] += (uint32_t)c * 38u;
}

// t_lo + 38 * t_hi for the 512-bit product t (2^256 = 38 mod p)
PD void fe_fold512(fe& r, const uint32_t t[16]) {
    uint32_t u[8];
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += (uint64_t)t[i + 8] * 38u + t[i];
        u[i] = (uint32_t)c;
        c >>= 32;
    }
    c *= 38;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        c += u[i];
        r.v[i] = (uint32_t)c;
        c >>= 32;
    }
    // after a second wrap r is below 38 * 38, so this cannot carry
    r.v[0] += (uint32_t)c * 38u;
}

#ifdef __HIP_DEVICE_COMPILE__
// (hi : acc) += a * b for a 96-bit column accumulator: one v_mad_u64_u32
// whose carry-out (in VCC) the following v_addc_co_u32 adds into hi.  The
// compiler does not use that carry-out by itself; this form takes about a
// third fewer instructions per limb product than 64-bit adds and shifts.
__device__ __forceinline__ void mad_acc96(uint64_t& acc, uint32_t& hi, uint32_t a, uint32_t b) {
    uint64_t r;
    uint32_t h;
    asm("v_mad_u64_u32 %0, vcc, %2, %3, %4\n\tv_addc_co_u32_e32 %1, vcc, 0, %5, vcc"
        : "=&v"(r), "=v"(h)
        : "v"(a), "v"(b), "v"(acc), "v"(hi)
        : "vcc");
    acc = r;
    hi = h;
}
#endif

PD void fe_mul(fe& r, const fe& a, const fe& b) {
    uint32_t t[16];
#ifdef __HIP_DEVICE_COMPILE__
    // product scanning: column k = sum of a_i * b_j over i + j = k
    uint64_t acc = 0;
    uint32_t hi = 0;
#pragma unroll
    for (int k = 0; k < 15; k++) {
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int j = k - i;
            if (j < 0 || j > 7) continue;
            mad_acc96(acc, hi, a.v[i], b.v[j]);
        }
        t[k] = (uint32_t)acc;
        acc = (acc >> 32) | ((uint64_t)hi << 32);
        hi = 0;
    }
    t[15] = (uint32_t)acc;
#else
#pragma unroll
    for (int i = 0; i < 16; i++) t[i] = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        uint64_t c = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            c += (uint64_t)a.v[i] * b.v[j] + t[i + j];
            t[i + j] = (uint32_t)c;
            c >>= 32;
        }
        t[i + 8] = (uint32_t)c;
    }
#endif
    fe_fold512(r, t);
}

// a^2 with 36 limb products: the 28 cross products once, doubled by a
// shift, plus the 8 squares
PD void fe_sq(fe& r, const fe& a) {
    uint32_t t[16];
#ifdef __HIP_DEVICE_COMPILE__
    uint64_t acc = 0;
    uint32_t hi = 0;
    t[0] = 0;
#pragma unroll
    for (int k = 1; k < 14; k++) {
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int j = k - i;
            if (j <= i || j > 7) continue;
            mad_acc96(acc, hi, a.v[i], a.v[j]);
        }
        t[k] = (uint32_t)acc;
        acc = (acc >> 32) | ((uint64_t)hi << 32);
        hi = 0;
    }
    t[14] = (uint32_t)acc;
    t[15] = (uint32_t)(acc >> 32);
#else
#pragma unroll
    for (int i = 0; i < 16; i++) t[i] = 0;
#pragma unroll
    for (int i = 0; i < 7; i++) {
        uint64_t c = 0;
#pragma unroll
        for (int j = i + 1; j < 8; j++) {
            c += (uint64_t)a.v[i] * a.v[j] + t[i + j];
            t[i + j] = (uint32_t)c;
            c >>= 32;
        }
        t[i + 8] = (uint32_t)c;
    }
#endif
    uint32_t top = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        uint32_t nt = (t[k] << 1) | top;
        top = t[k] >> 31;
        t[k] = nt;
    }
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        uint64_t sq = (uint64_t)a.v[i] * a.v[i];
        c += (uint64_t)t[2 * i] + (uint32_t)sq;
        t[2 * i] = (uint32_t)c;
        c >>= 32;
        c += (uint64_t)t[2 * i + 1] + (sq >> 32);
        t[2 * i + 1] = (uint32_t)c;
        c >>= 32;
    }
    fe_fold512(r, t);
}

PD void fe_sqn(fe& r, const fe& a, int n) {
    fe_sq(r, a);
    for (int i = 1; i < n; i++) fe_sq(r, r);
}

// canonical representative: a < 2^256 = 2p + 38, so at most two subtractions
PD void fe_freeze(fe& r, const fe& a) {
    fe x = a;
    const uint32_t p[8] = {0xffffffedu, 0xffffffffu, 0xffffffffu, 0xffffffffu,
                           0xffffffffu, 0xffffffffu, 0xffffffffu, 0x7fffffffu};
    for (int k = 0; k < 2; k++) {
        uint32_t t[8];
        int64_t c = 0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            c += (int64_t)x.v[i] - (int64_t)p[i];
            t[i] = (uint32_t)c;
            c >>= 32;
        }
        if (c == 0) {
#pragma unroll
            for (int i = 0; i < 8; i++) x.v[i] = t[i];
        }
    }
    r = x;
}

PD bool fe_iszero(const fe& a) {
    fe f;
    fe_freeze(f, a);
    uint32_t o = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) o |= f.v[i];
    return o == 0;
}

PD bool fe_equal(const fe& a, const fe& b) {
    fe d;
    fe_sub(d, a, b);
    return fe_iszero(d);
}

PD uint32_t fe_isodd(const fe& a) {
    fe f;
    fe_freeze(f, a);
    return f.v[0] & 1u;
}

PD void fe_neg(fe& r, const fe& a) {
    fe z;
    fe_set(z, 0);
    fe_sub(r, z, a);
}

// a^(p-2) = a^(2^255 - 21), the inverse (0 maps to 0)
PD void fe_inv(fe& r, const fe& z) {
    fe t0, t1, t2, t3;
    fe_sq(t0, z);             // 2
    fe_sqn(t1, t0, 2);        // 8
    fe_mul(t1, z, t1);        // 9
    fe_mul(t0, t0, t1);       // 11
    fe_sq(t2, t0);            // 22
    fe_mul(t1, t1, t2);       // 31 = 2^5 - 1
    fe_sqn(t2, t1, 5);
    fe_mul(t1, t2, t1);       // 2^10 - 1
    fe_sqn(t2, t1, 10);
    fe_mul(t2, t2, t1);       // 2^20 - 1
    fe_sqn(t3, t2, 20);
    fe_mul(t2, t3, t2);       // 2^40 - 1
    fe_sqn(t2, t2, 10);
    fe_mul(t1, t2, t1);       // 2^50 - 1
    fe_sqn(t2, t1, 50);
    fe_mul(t2, t2, t1);       // 2^100 - 1
    fe_sqn(t3, t2, 100);
    fe_mul(t2, t3, t2);       // 2^200 - 1
    fe_sqn(t2, t2, 50);
    fe_mul(t1, t2, t1);       // 2^250 - 1
    fe_sqn(t1, t1, 5);        // 2^255 - 32
    fe_mul(r, t1, t0);        // 2^255 - 21
}

// a^((p-5)/8) = a^(2^252 - 3), used for square roots
PD void fe_pow22523(fe& r, const fe& z) {
    fe t0, t1, t2;
    fe_sq(t0, z);             // 2
    fe_sqn(t1, t0, 2);        // 8
    fe_mul(t1, z, t1);        // 9
    fe_mul(t0, t0, t1);       // 11
    fe_sq(t0, t0);            // 22
    fe_mul(t0, t1, t0);       // 31 = 2^5 - 1
    fe_sqn(t1, t0, 5);
    fe_mul(t0, t1, t0);       // 2^10 - 1
    fe_sqn(t1, t0, 10);
    fe_mul(t1, t1, t0);       // 2^20 - 1
    fe_sqn(t2, t1, 20);
    fe_mul(t1, t2, t1);       // 2^40 - 1
    fe_sqn(t1, t1, 10);
    fe_mul(t0, t1, t0);       // 2^50 - 1
    fe_sqn(t1, t0, 50);
    fe_mul(t1, t1, t0);       // 2^100 - 1
    fe_sqn(t2, t1, 100);
    fe_mul(t1, t2, t1);       // 2^200 - 1
    fe_sqn(t1, t1, 50);
    fe_mul(t0, t1, t0);       // 2^250 - 1
    fe_sqn(t0, t0, 2);        // 2^252 - 4
    fe_mul(r, t0, z);         // 2^252 - 3
}

PD void fe_from_bytes(fe& r, const uint8_t b[32]) {
#pragma unroll
    for (int i = 0; i < 8; i++) r.v[i] = load_le32(b + 4 * i);
}

PD void fe_to_bytes(uint8_t b[32], const fe& a) {
    fe f;
    fe_freeze(f, a);
#pragma unroll
    for (int i = 0; i < 8; i++) store_le32(b + 4 * i, f.v[i]);
}

}  // namespace poslo
