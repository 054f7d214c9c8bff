// Device-side curve checks with fixed-base comb tables.
//
// A comb table of a point P holds, for 32 windows w and 128 magnitudes i, the
// affine point (i + 1) * 256^w * P in the form (y + x, y - x, 2d*x*y), 24
// words each.  A scalar k < 2^253 is recoded into 32 signed digits k_w in
// [-127, 128] with k = sum of k_w * 256^w; then
//   k * P = sum over w of sign(k_w) * t[w][|k_w| - 1],
// 32 mixed additions of 7 multiplications each and no doublings.  A negative
// digit swaps y + x with y - x and negates 2d*x*y; a zero digit adds the
// identity (1, 1, 0).
#pragma once

#include "comb.h"
#include "ge25519.h"
#include "sc25519.h"

namespace poslo {

__device__ __forceinline__ void load_point(ge& P, const uint32_t* p) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
        P.X.v[k] = p[k];
        P.Y.v[k] = p[8 + k];
        P.Z.v[k] = p[16 + k];
        P.T.v[k] = p[24 + k];
    }
}

__device__ __forceinline__ void store_point(uint32_t* p, const ge& P) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
        p[k] = P.X.v[k];
        p[8 + k] = P.Y.v[k];
        p[16 + k] = P.Z.v[k];
        p[24 + k] = P.T.v[k];
    }
}

__device__ __forceinline__ void shfl_down_point(ge& Q, const ge& P, int off) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
        Q.X.v[k] = __shfl_down(P.X.v[k], off);
        Q.Y.v[k] = __shfl_down(P.Y.v[k], off);
        Q.Z.v[k] = __shfl_down(P.Z.v[k], off);
        Q.T.v[k] = __shfl_down(P.T.v[k], off);
    }
}

// affine point in (y + x, y - x, 2d*x*y) form
struct gn {
    fe yp, ym, t2d;
};

// r = p + q for an affine q (a = -1, complete)
PD void ge_madd(ge& r, const ge& p, const gn& q) {
    fe a, b, c, d;
    fe_sub(a, p.Y, p.X);
    fe_mul(a, a, q.ym);
    fe_add(b, p.Y, p.X);
    fe_mul(b, b, q.yp);
    fe_mul(c, p.T, q.t2d);
    fe_add(d, p.Z, p.Z);
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

// signed radix-256 digit of window w; carry runs from window 0 upwards
PD int comb_digit(const uint32_t k[8], int w, uint32_t& carry) {
    const int v = (int)((k[w >> 2] >> (8 * (w & 3))) & 255u) + (int)carry;
    carry = v > 128 ? 1u : 0u;
    return v > 128 ? v - 256 : v;
}

// signed radix-65536 digit of window w (the wide generator table)
PD int wide_digit(const uint32_t k[8], int w, uint32_t& carry) {
    const int v = (int)((k[w >> 1] >> (16 * (w & 1))) & 0xffffu) + (int)carry;
    carry = v > 32768 ? 1u : 0u;
    return v > 32768 ? v - 65536 : v;
}

// t[w][|d| - 1] with the sign of d applied; the identity for d = 0
template <int PER = kCombPerWindow>
PD void comb_lookup(gn& q, const uint32_t* table, int w, int d) {
    const uint32_t m = (uint32_t)(d < 0 ? -d : d);
    const uint32_t* p = table + ((uint64_t)w * PER + (m ? m - 1 : 0)) * kCombEntryWords;
    fe a, b, t;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        a.v[k] = p[k];
        b.v[k] = p[8 + k];
        t.v[k] = p[16 + k];
    }
    if (m == 0) {
        fe_set(a, 1);
        fe_set(b, 1);
        fe_set(t, 0);
    }
    if (d < 0) {
        q.yp = b;
        q.ym = a;
        fe_neg(q.t2d, t);
    } else {
        q.yp = a;
        q.ym = b;
        q.t2d = t;
    }
}

// e*Y + s*G by one whole wave: lanes 0-31 take window w of e on Y's table,
// lanes 32-63 window w - 32 of s on G's table, then a six-level tree of
// additions; the result is valid in lane 0.  e < 2^253; s is any 256-bit
// value (reduced mod q here, exact since G has order q).  Every lane of the
// wave must call it.
__device__ __forceinline__ void wave_double_scalar(ge& P, const uint32_t* ty, const uint32_t* tg, const uint32_t e[8],
                                                   const uint32_t s[8]) {
    const int lane = threadIdx.x & 63;
    const int w = lane & 31;
    uint32_t sr[8];
    sc_reduce256(sr, s);
    const uint32_t* k = lane < 32 ? e : sr;
    uint32_t carry = 0;
    int d = 0;
    for (int i = 0; i < kCombWindows; i++) {
        const int di = comb_digit(k, i, carry);
        if (i == w) d = di;
    }
    gn q;
    comb_lookup(q, lane < 32 ? ty : tg, w, d);
    ge_identity(P);
    ge_madd(P, P, q);
    for (int off = 32; off > 0; off >>= 1) {
        ge Q;
        shfl_down_point(Q, P, off);
        ge_add(P, P, Q);
    }
}

// e*Y + s*G by one lane: 64 lookups and mixed additions; e, s < 2^253
__device__ __forceinline__ void lane_double_scalar(ge& P, const uint32_t* ty, const uint32_t* tg, const uint32_t e[8],
                                                   const uint32_t s[8]) {
    ge_identity(P);
    uint32_t ce = 0, cs = 0;
    for (int w = 0; w < kCombWindows; w++) {
        gn q;
        comb_lookup(q, ty, w, comb_digit(e, w, ce));
        ge_madd(P, P, q);
        comb_lookup(q, tg, w, comb_digit(s, w, cs));
        ge_madd(P, P, q);
    }
}

// e*Y + s*G by one lane with G's wide table: 32 + 16 lookups and mixed
// additions; e, s < 2^253
__device__ __forceinline__ void lane_double_scalar_wide(ge& P, const uint32_t* ty, const uint32_t* tg_wide,
                                                        const uint32_t e[8], const uint32_t s[8]) {
    ge_identity(P);
    uint32_t ce = 0, cs = 0;
    for (int w = 0; w < kWideWindows; w++) {
        gn q;
        comb_lookup(q, ty, 2 * w, comb_digit(e, 2 * w, ce));
        ge_madd(P, P, q);
        comb_lookup(q, ty, 2 * w + 1, comb_digit(e, 2 * w + 1, ce));
        ge_madd(P, P, q);
        comb_lookup<kWidePerWindow>(q, tg_wide, w, wide_digit(s, w, cs));
        ge_madd(P, P, q);
    }
}

// e*Y + s*G by one lane with both wide tables: 16 + 16 lookups and mixed
// additions; e, s < 2^253
__device__ __forceinline__ void lane_double_scalar_wide2(ge& P, const uint32_t* ty_wide, const uint32_t* tg_wide,
                                                         const uint32_t e[8], const uint32_t s[8]) {
    ge_identity(P);
    uint32_t ce = 0, cs = 0;
    for (int w = 0; w < kWideWindows; w++) {
        gn q;
        comb_lookup<kWidePerWindow>(q, ty_wide, w, wide_digit(e, w, ce));
        ge_madd(P, P, q);
        comb_lookup<kWidePerWindow>(q, tg_wide, w, wide_digit(s, w, cs));
        ge_madd(P, P, q);
    }
}

// k*P by one lane: 32 lookups and mixed additions; k < 2^253
__device__ __forceinline__ void lane_scalar(ge& P, const uint32_t* t, const uint32_t k[8]) {
    ge_identity(P);
    uint32_t c = 0;
    for (int w = 0; w < kCombWindows; w++) {
        gn q;
        comb_lookup(q, t, w, comb_digit(k, w, c));
        ge_madd(P, P, q);
    }
}

// encode(P) == bytes (32 bytes as eight little-endian words)
__device__ __forceinline__ bool ge_encodes_to(const ge& P, const uint32_t want[8]) {
    uint8_t enc[32];
    ge_encode(enc, P);
    uint32_t diff = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) diff |= load_le32(enc + 4 * k) ^ want[k];
    return diff == 0;
}

}  // namespace poslo
