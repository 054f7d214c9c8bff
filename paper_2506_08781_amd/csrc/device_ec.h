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

// the words of t[w][|d| - 1] (of t[w][0] for d = 0) and d, fetched ahead
// of their use so that the load overlaps other work
struct CombRaw {
    uint32_t v[kCombEntryWords];
    int d;
};

template <int PER = kCombPerWindow>
PD void comb_fetch(CombRaw& r, const uint32_t* table, int w, int d) {
    const uint32_t m = (uint32_t)(d < 0 ? -d : d);
    const uint32_t* p = table + ((uint64_t)w * PER + (m ? m - 1 : 0)) * kCombEntryWords;
#pragma unroll
    for (int k = 0; k < kCombEntryWords; k++) r.v[k] = p[k];
    r.d = d;
}

// the fetched entry with the sign of d applied; the identity for d = 0
PD void comb_apply(gn& q, const CombRaw& r) {
    const int d = r.d;
    fe a, b, t;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        a.v[k] = r.v[k];
        b.v[k] = r.v[8 + k];
        t.v[k] = r.v[16 + k];
    }
    if (d == 0) {
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
    // e's windows, then s's: only one scalar is live in each loop
    for (int w = 0; w < kCombWindows; w++) {
        gn q;
        comb_lookup(q, ty, w, comb_digit(e, w, ce));
        ge_madd(P, P, q);
    }
    for (int w = 0; w < kWideWindows; w++) {
        gn q;
        comb_lookup<kWidePerWindow>(q, tg_wide, w, wide_digit(s, w, cs));
        ge_madd(P, P, q);
    }
}

// e*Y + s*G by one lane with both wide tables: 16 + 16 lookups and mixed
// additions; e, s < 2^253.  Each table point is fetched one mixed addition
// ahead of its use (both tables are far larger than the L2).
__device__ __forceinline__ void lane_double_scalar_wide2(ge& P, const uint32_t* ty_wide, const uint32_t* tg_wide,
                                                         const uint32_t e[8], const uint32_t s[8]) {
    ge_identity(P);
    uint32_t ce = 0, cs = 0;
    // e's windows, then s's: only one scalar is live in each loop
    CombRaw r;
    comb_fetch<kWidePerWindow>(r, ty_wide, 0, wide_digit(e, 0, ce));
    for (int w = 0; w < kWideWindows; w++) {
        gn q;
        comb_apply(q, r);
        if (w + 1 < kWideWindows)
            comb_fetch<kWidePerWindow>(r, ty_wide, w + 1, wide_digit(e, w + 1, ce));
        else
            comb_fetch<kWidePerWindow>(r, tg_wide, 0, wide_digit(s, 0, cs));
        ge_madd(P, P, q);
    }
    for (int w = 0; w < kWideWindows; w++) {
        gn q;
        comb_apply(q, r);
        if (w + 1 < kWideWindows) comb_fetch<kWidePerWindow>(r, tg_wide, w + 1, wide_digit(s, w + 1, cs));
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

// word v of quad lane (c + D) & 3, for the lane c of this lane's quad
template <int D>
__device__ __forceinline__ uint32_t ec_quad_rot(uint32_t v) {
    constexpr int ctrl = D == 1 ? 0x39 : D == 2 ? 0x4e : 0x93;  // quad_perm [c + D mod 4]
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xf, 0xf, false);
}

__device__ __forceinline__ void lds_load_fe(fe& a, const uint32_t* p) {
#pragma unroll
    for (int k = 0; k < 8; k++) a.v[k] = p[k];
}

__device__ __forceinline__ void lds_store_fe(uint32_t* p, const fe& a) {
#pragma unroll
    for (int k = 0; k < 8; k++) p[k] = a.v[k];
}

constexpr int kQuadBlock = 256;               // threads of block_double_scalar_is
constexpr int kQuadLdsWords = 64 * 4 * 8;     // its LDS: 64 points of 4 coordinates

// e*Y + s*G by a whole 256-thread block, for a single sum where latency
// decides; the sum is left in LDS slot 0 (X, Y, Z, T at lds + 0, 8, 16, 24
// after the closing barrier).  The quad of lanes 4k..4k+3 owns point k of
// 64 (k < 32: window k of e on Y's comb table; k >= 32: window k - 32 of s on
// G's), lane c holding coordinate c in the order X, Y, Z, T.  A six-level
// tree of complete additions follows, each addition split over its quad:
// the four products A, B, C, D of the addition law go one per lane, then the
// four output products X3 = EF, Y3 = GH, Z3 = FG, T3 = EH go one per lane,
// so a level costs two multiplications of latency instead of nine.  The
// factor 2d = -2 * 121665 / 121666 of C is kept out of the chain by scaling
// A, B, C and D by 121666 (small-constant products): A and B by 121666, C by
// 2 * 121665 with its sign moved into F and G, D by 2 * 121666.  E, F, G and
// H then all carry the factor 121666, so the result is the same point with
// every coordinate scaled by 121666^2.  e, s < 2^253.
// lds holds kQuadLdsWords words; every thread of the block must call it.
__device__ __forceinline__ void block_double_scalar(uint32_t* lds, const uint32_t* ty, const uint32_t* tg,
                                                    const uint32_t e[8], const uint32_t s[8]) {
    const int k = (int)(threadIdx.x >> 2), c = (int)(threadIdx.x & 3);
    const uint32_t* sc = k < 32 ? e : s;
    const int w = k & 31;
    uint32_t carry = 0;
    int d = 0;
    for (int i = 0; i < kCombWindows; i++) {
        const int di = comb_digit(sc, i, carry);
        if (i == w) d = di;
    }
    gn q;
    comb_lookup(q, k < 32 ? ty : tg, w, d);
    // the affine point (x, y) as (4x : 4y : 4 : 4xy) from y + x and y - x
    fe a, b, m, v;
    fe_sub(a, q.yp, q.ym);
    fe_add(b, q.yp, q.ym);
    fe_mul(m, a, b);
    if (c == 0)
        fe_add(v, a, a);
    else if (c == 1)
        fe_add(v, b, b);
    else if (c == 2)
        fe_set(v, 4);
    else
        v = m;
    lds_store_fe(lds + (k * 4 + c) * 8, v);
    for (int o = 32; o >= 1; o >>= 1) {
        __syncthreads();
        if (k < o) {
            const uint32_t* p1 = lds + k * 32;
            const uint32_t* p2 = lds + (k + o) * 32;
            // lanes 0 and 1: 121666 (Y1 -+ X1)(Y2 -+ X2); lane 2: 243330 T1 T2
            // (= -121666 * 2d T1 T2); lane 3: 243332 Z1 Z2 (= 121666 * 2 Z1 Z2)
            const int co = c < 2 ? 0 : c == 2 ? 3 : 2;
            fe u1, u2, y1, y2;
            lds_load_fe(u1, p1 + co * 8);
            lds_load_fe(u2, p2 + co * 8);
            if (c < 2) {
                lds_load_fe(y1, p1 + 8);
                lds_load_fe(y2, p2 + 8);
                if (c == 0) {
                    fe_sub(u1, y1, u1);
                    fe_sub(u2, y2, u2);
                } else {
                    fe_add(u1, y1, u1);
                    fe_add(u2, y2, u2);
                }
            }
            fe_mul(m, u1, u2);
            fe_mul_small(m, m, c < 2 ? 121666u : c == 2 ? 243330u : 243332u);
            // every lane of the quad gets A, B, C, D
            fe A, B, C, D;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const uint32_t r0 = m.v[j], r1 = ec_quad_rot<1>(r0), r2 = ec_quad_rot<2>(r0),
                               r3 = ec_quad_rot<3>(r0);
                // the word of lane L sits (L - c) & 3 lanes to the right
                A.v[j] = c == 0 ? r0 : c == 1 ? r3 : c == 2 ? r2 : r1;
                B.v[j] = c == 1 ? r0 : c == 2 ? r3 : c == 3 ? r2 : r1;
                C.v[j] = c == 2 ? r0 : c == 3 ? r3 : c == 0 ? r2 : r1;
                D.v[j] = c == 3 ? r0 : c == 0 ? r3 : c == 1 ? r2 : r1;
            }
            // C holds minus the scaled 2d T1 T2: F = D + C, G = D - C
            fe E, F, G, H;
            fe_sub(E, B, A);
            fe_add(F, D, C);
            fe_sub(G, D, C);
            fe_add(H, B, A);
            // lane 0: X3 = EF, lane 1: Y3 = GH, lane 2: Z3 = FG, lane 3: T3 = EH
            const fe& l = c == 0 ? E : c == 1 ? G : c == 2 ? F : E;
            const fe& r = c == 0 ? F : c == 1 ? H : c == 2 ? G : H;
            fe_mul(v, l, r);
            lds_store_fe(lds + (k * 4 + c) * 8, v);
        }
    }
    __syncthreads();
}

// e*Y + s*G == R for R = (rx, ry) affine, compared in projective form
__device__ __forceinline__ bool block_double_scalar_is(uint32_t* lds, const uint32_t* ty, const uint32_t* tg,
                                                       const uint32_t e[8], const uint32_t s[8], const fe& rx,
                                                       const fe& ry) {
    block_double_scalar(lds, ty, tg, e, s);
    const int k = (int)(threadIdx.x >> 2), c = (int)(threadIdx.x & 3);
    // the sum sits in slot 0: X == x_R Z on lane 0 and Y == y_R Z on lane 1
    bool ok = true;
    if (k == 0 && c < 2) {
        fe Z, V, m;
        lds_load_fe(Z, lds + 2 * 8);
        lds_load_fe(V, lds + c * 8);
        fe_mul(m, c == 0 ? rx : ry, Z);
        ok = fe_equal(m, V);
    }
    const uint64_t bad = __ballot(!ok);
    return (bad & 3u) == 0;
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
