// The edwards25519 group -x^2 + y^2 = 1 + d x^2 y^2 over GF(2^255 - 19), in
// extended coordinates (X : Y : Z : T) with x = X/Z, y = Y/Z, xy = T/Z.
// Encoding: 32 bytes, y little-endian with the parity of x in bit 255.
//
// The paper writes the verification equation multiplicatively (R = Y^e *
// alpha^s); on the curve it reads R = e*Y + s*G.
#pragma once

#include "fe25519.h"

namespace poslo {

struct ge {
    fe X, Y, Z, T;
};

// d = -121665/121666, 2d, sqrt(-1) = 2^((p-1)/4), and the base point
// G = (x, 4/5) with x even; limbs little-endian.
#define POSLO_FE_D {{0x135978a3u, 0x75eb4dcau, 0x4141d8abu, 0x00700a4du, 0x7779e898u, 0x8cc74079u, 0x2b6ffe73u, 0x52036ceeu}}
#define POSLO_FE_D2 {{0x26b2f159u, 0xebd69b94u, 0x8283b156u, 0x00e0149au, 0xeef3d130u, 0x198e80f2u, 0x56dffce7u, 0x2406d9dcu}}
#define POSLO_FE_SQRTM1 {{0x4a0ea0b0u, 0xc4ee1b27u, 0xad2fe478u, 0x2f431806u, 0x3dfbd7a7u, 0x2b4d0099u, 0x4fc1df0bu, 0x2b832480u}}
#define POSLO_FE_GX {{0x8f25d51au, 0xc9562d60u, 0x9525a7b2u, 0x692cc760u, 0xfdd6dc5cu, 0xc0a4e231u, 0xcd6e53feu, 0x216936d3u}}
#define POSLO_FE_GY {{0x66666658u, 0x66666666u, 0x66666666u, 0x66666666u, 0x66666666u, 0x66666666u, 0x66666666u, 0x66666666u}}
#define POSLO_FE_GT {{0xa5b7dda3u, 0x6dde8ab3u, 0x775152f5u, 0x20f09f80u, 0x64abe37du, 0x66ea4e8eu, 0xd78b7665u, 0x67875f0fu}}

PD void ge_identity(ge& r) {
    fe_set(r.X, 0);
    fe_set(r.Y, 1);
    fe_set(r.Z, 1);
    fe_set(r.T, 0);
}

PD void ge_base(ge& r) {
    const fe gx = POSLO_FE_GX, gy = POSLO_FE_GY, gt = POSLO_FE_GT;
    r.X = gx;
    r.Y = gy;
    fe_set(r.Z, 1);
    r.T = gt;
}

// complete addition (a = -1, k = 2d); valid for doubling and the identity
PD void ge_add(ge& r, const ge& p, const ge& q) {
    const fe d2 = POSLO_FE_D2;
    fe a, b, c, d, t;
    fe_sub(a, p.Y, p.X);
    fe_sub(t, q.Y, q.X);
    fe_mul(a, a, t);
    fe_add(b, p.Y, p.X);
    fe_add(t, q.Y, q.X);
    fe_mul(b, b, t);
    fe_mul(c, p.T, q.T);
    fe_mul(c, c, d2);
    fe_mul(d, p.Z, q.Z);
    fe_add(d, d, d);
    fe e, f, g, h;
    fe_sub(e, b, a);
    fe_sub(f, d, c);
    fe_add(g, d, c);
    fe_add(h, b, a);
    fe_mul(r.X, e, f);
    fe_mul(r.Y, g, h);
    fe_mul(r.T, e, h);
    fe_mul(r.Z, f, g);
}

// dedicated doubling (a = -1)
PD void ge_dbl(ge& r, const ge& p) {
    fe a, b, c, h, e, g, f, t;
    fe_sq(a, p.X);
    fe_sq(b, p.Y);
    fe_sq(c, p.Z);
    fe_add(c, c, c);
    fe_add(h, a, b);
    fe_add(t, p.X, p.Y);
    fe_sq(t, t);
    fe_sub(e, h, t);
    fe_sub(g, a, b);
    fe_add(f, c, g);
    fe_mul(r.X, e, f);
    fe_mul(r.Y, g, h);
    fe_mul(r.T, e, h);
    fe_mul(r.Z, f, g);
}

PD void ge_neg(ge& r, const ge& p) {
    fe_neg(r.X, p.X);
    r.Y = p.Y;
    r.Z = p.Z;
    fe_neg(r.T, p.T);
}

PD void ge_encode(uint8_t out[32], const ge& p) {
    fe zi, x, y;
    fe_inv(zi, p.Z);
    fe_mul(x, p.X, zi);
    fe_mul(y, p.Y, zi);
    fe_to_bytes(out, y);
    out[31] |= (uint8_t)(fe_isodd(x) << 7);
}

// y (or x) compared projectively: encode(p) == bytes of the point q
PD bool ge_equal(const ge& p, const ge& q) {
    fe a, b;
    fe_mul(a, p.X, q.Z);
    fe_mul(b, q.X, p.Z);
    if (!fe_equal(a, b)) return false;
    fe_mul(a, p.Y, q.Z);
    fe_mul(b, q.Y, p.Z);
    return fe_equal(a, b);
}

// RFC 8032 5.1.3: reject y >= p, non-squares, and x = 0 with the sign bit set
PD bool ge_decode(ge& r, const uint8_t in[32]) {
    const fe d = POSLO_FE_D, sqrtm1 = POSLO_FE_SQRTM1;
    fe y;
    fe_from_bytes(y, in);
    uint32_t sign = y.v[7] >> 31;
    y.v[7] &= 0x7fffffffu;
    // canonical: y < p
    {
        fe f;
        fe_freeze(f, y);
        for (int i = 0; i < 8; i++)
            if (f.v[i] != y.v[i]) return false;
    }
    fe one, u, v, v3, x, t;
    fe_set(one, 1);
    fe_sq(u, y);
    fe_mul(v, u, d);
    fe_sub(u, u, one);   // u = y^2 - 1
    fe_add(v, v, one);   // v = d y^2 + 1
    fe_sq(v3, v);
    fe_mul(v3, v3, v);   // v^3
    fe_sq(x, v3);
    fe_mul(x, x, v);
    fe_mul(x, x, u);     // u v^7
    fe_pow22523(x, x);   // (u v^7)^((p-5)/8)
    fe_mul(x, x, v3);
    fe_mul(x, x, u);     // u v^3 (u v^7)^((p-5)/8)
    fe_sq(t, x);
    fe_mul(t, t, v);     // v x^2
    if (!fe_equal(t, u)) {
        fe nu;
        fe_neg(nu, u);
        if (!fe_equal(t, nu)) return false;
        fe_mul(x, x, sqrtm1);
    }
    if (fe_iszero(x) && sign) return false;
    if (fe_isodd(x) != sign) fe_neg(x, x);
    fe_freeze(r.X, x);
    r.Y = y;
    fe_set(r.Z, 1);
    fe_mul(r.T, r.X, r.Y);
    return true;
}

PD uint32_t scalar_bit(const uint32_t s[8], int i) { return (s[i >> 5] >> (i & 31)) & 1u; }

// a*A + b*G by joint double-and-add over 253 bits (scalars below 2^253)
PD void ge_double_scalarmult(ge& r, const uint32_t a[8], const ge& A, const uint32_t b[8]) {
    ge Gp, AG;
    ge_base(Gp);
    ge_add(AG, A, Gp);
    ge R;
    ge_identity(R);
    for (int i = 252; i >= 0; i--) {
        ge_dbl(R, R);
        uint32_t ab = scalar_bit(a, i), bb = scalar_bit(b, i);
        if (ab && bb)
            ge_add(R, R, AG);
        else if (ab)
            ge_add(R, R, A);
        else if (bb)
            ge_add(R, R, Gp);
    }
    r = R;
}

// k*A by double-and-add (k below 2^256)
PD void ge_scalarmult(ge& r, const uint32_t k[8], const ge& A) {
    ge R;
    ge_identity(R);
    for (int i = 255; i >= 0; i--) {
        ge_dbl(R, R);
        if (scalar_bit(k, i)) ge_add(R, R, A);
    }
    r = R;
}

}  // namespace poslo
