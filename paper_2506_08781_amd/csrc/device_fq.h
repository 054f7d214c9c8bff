// Per-entry checks on the FourQ group (fourq.h), the forms of device_ec.h
// and device_verify.h for it: lookups in FourQ comb tables (comb.h layout,
// GF(p^2) coordinates in the 24-word entries), e*Y + s*G on one lane and on
// one wave, and the comparison of a point with an encoding given 1/Z.  The
// check is the one of the paper's POSLO-F verification with FourQ as the
// group (section "Instantiations and Configurations"): s_t < N and the
// encoding of e_t*Y + s_t*G equals R_t.
#pragma once

#include "comb.h"
#include "device_ec.h"
#include "device_entry.h"
#include "fourq.h"

namespace poslo {

// t[w][|d| - 1] of a FourQ comb table (PER entries per window) with the
// sign of d applied; the identity for d = 0
template <int PER = kCombPerWindow>
PD void fq_comb_lookup(gnq& q, const uint32_t* table, int w, int d) {
    const uint32_t m = (uint32_t)(d < 0 ? -d : d);
    fq_load_entry(q, table + ((uint64_t)w * PER + (m ? m - 1 : 0)) * kCombEntryWords, d < 0);
    if (m == 0) {
        f2_one(q.yp);
        f2_one(q.ym);
        f2_zero(q.t2d);
    }
}

// e*Y + s*G by one lane with G's wide FourQ table (16 windows of 32,768
// points, comb.h layout): 32 + 16 lookups and mixed additions; e, s < N
__device__ __forceinline__ void lane_double_scalar_fq_wide(gq& P, const uint32_t* ty, const uint32_t* tg_wide,
                                                           const uint32_t e[8], const uint32_t s[8]) {
    gq_identity(P);
    uint32_t ce = 0, cs = 0;
    // e's windows, then s's: only one scalar is live in each loop
    for (int w = 0; w < kCombWindows; w++) {
        gnq q;
        fq_comb_lookup(q, ty, w, comb_digit(e, w, ce));
        gq_madd(P, P, q);
    }
    for (int w = 0; w < kWideWindows; w++) {
        gnq q;
        fq_comb_lookup<kWidePerWindow>(q, tg_wide, w, wide_digit(s, w, cs));
        gq_madd(P, P, q);
    }
}

__device__ __forceinline__ void shfl_down_point_fq(gq& Q, const gq& P, int off) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
        Q.X.a.v[k] = __shfl_down(P.X.a.v[k], off);
        Q.X.b.v[k] = __shfl_down(P.X.b.v[k], off);
        Q.Y.a.v[k] = __shfl_down(P.Y.a.v[k], off);
        Q.Y.b.v[k] = __shfl_down(P.Y.b.v[k], off);
        Q.Z.a.v[k] = __shfl_down(P.Z.a.v[k], off);
        Q.Z.b.v[k] = __shfl_down(P.Z.b.v[k], off);
        Q.T.a.v[k] = __shfl_down(P.T.a.v[k], off);
        Q.T.b.v[k] = __shfl_down(P.T.b.v[k], off);
    }
}

// e*Y + s*G by one whole wave: lanes 0-31 take window w of e on Y's table,
// lanes 32-63 window w - 32 of s on G's table, then a six-level tree of
// additions; the result is valid in lane 0.  e, s < N.  Every lane of the
// wave must call it.
__device__ __forceinline__ void wave_double_scalar_fq(gq& P, const uint32_t* ty, const uint32_t* tg,
                                                      const uint32_t e[8], const uint32_t s[8]) {
    const int lane = threadIdx.x & 63;
    const int w = lane & 31;
    const uint32_t* k = lane < 32 ? e : s;
    uint32_t carry = 0;
    int d = 0;
    for (int i = 0; i < kCombWindows; i++) {  // fixed trip count: the scalar stays in registers
        const int di = comb_digit(k, i, carry);
        if (i == w) d = di;
    }
    gnq q;
    fq_comb_lookup(q, lane < 32 ? ty : tg, w, d);
    gq_identity(P);
    gq_madd(P, P, q);
    for (int off = 32; off > 0; off >>= 1) {
        gq Q;
        shfl_down_point_fq(Q, P, off);
        gq_add(P, P, Q);
    }
}

// encode(P) == want (eight little-endian words: y0 || y1 with the sign of x
// in bit 255) given zi = 1 / Z
PD bool fq_encodes_zinv(const gq& P, const fp2& zi, const uint32_t want[8]) {
    fp2 x, y;
    f2_mul(x, P.X, zi);
    f2_mul(y, P.Y, zi);
    f2_freeze(x, x);
    f2_freeze(y, y);
    uint32_t diff = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) diff |= (y.a.v[k] ^ want[k]) | (y.b.v[k] ^ (k == 3 ? want[7] & 0x7fffffffu : want[4 + k]));
    diff |= (want[7] >> 31) ^ fq_sign(x);
    return diff == 0;
}

// the curve part of entry checks on FourQ, as verify_sig_batch (same stash
// layout: X, Y, Z and the running product before the entry, 32 words), with
// Y's 8-bit table and G's wide one.
// RAW: e points at the unreduced digest, reduced mod N here.
template <bool RAW>
__device__ __forceinline__ bool sig_point_fq(const uint8_t* sg, const uint32_t* e, bool go, const uint32_t* ty,
                                             const uint32_t* tg_wide, gq& P) {
    uint32_t ek[8], s[8];
    for (int w = 0; w < 8; w++) {
        s[w] = go ? gload_le32(sg + 4 * w) : 0u;
        ek[w] = go ? e[w] : 0u;
    }
    if constexpr (RAW) scN_reduce<8>(ek, ek);
    const bool c = go && scN_is_canonical(s);
    if (!c)
        for (int w = 0; w < 8; w++) s[w] = ek[w] = 0;  // the identity: Z stays nonzero
    lane_double_scalar_fq_wide(P, ty, tg_wide, ek, s);
    return c;
}

__device__ __forceinline__ bool sig_encodes_fq(const uint8_t* sg, bool c, const gq& P, const fp2& zi) {
    uint32_t r[8];
    for (int w = 0; w < 8; w++) r[w] = c ? gload_le32(sg + 32 + 4 * w) : 0u;
    return c && fq_encodes_zinv(P, zi, r);
}

__device__ __forceinline__ void stash_f2(uint32_t* o, uint32_t stride, const fp2& a) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
        o[k * stride] = a.a.v[k];
        o[(4 + k) * stride] = a.b.v[k];
    }
}

__device__ __forceinline__ void unstash_f2(fp2& a, const uint32_t* o, uint32_t stride) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
        a.a.v[k] = o[k * stride];
        a.b.v[k] = o[(4 + k) * stride];
    }
}

template <bool RAW = false, class ENT>
__device__ __forceinline__ uint32_t verify_sig_batch_fq(const ENT& ent, int ne, const uint32_t* ty,
                                                        const uint32_t* tg_wide, uint32_t* st, uint32_t stride) {
    if (ne <= 0) return 0;
    uint32_t okmask = 0;
    fp2 c, c_prev;
    f2_one(c_prev);
    gq P;
#pragma unroll 1
    for (int k = 0; k < ne; k++) {
        const uint8_t* sg;
        const uint32_t* e;
        bool go;
        ent(k, sg, e, go);
        if (sig_point_fq<RAW>(sg, e, go, ty, tg_wide, P)) okmask |= 1u << k;
        if (k == 0) {
            c = P.Z;
        } else {
            c_prev = c;
            f2_mul(c, c, P.Z);
        }
        if (k < ne - 1) {
            uint32_t* o = st + (uint64_t)32 * k * stride;
            stash_f2(o, stride, P.X);
            stash_f2(o + 8 * stride, stride, P.Y);
            stash_f2(o + 16 * stride, stride, P.Z);
            stash_f2(o + 24 * stride, stride, c_prev);
        }
    }
    fp2 inv, zi;
    f2_inv(inv, c);  // 1 / (Z_0 ... Z_{ne-1})
    {
        if (ne > 1) {
            f2_mul(zi, inv, c_prev);
            f2_mul(inv, inv, P.Z);
        } else {
            zi = inv;
        }
        const uint8_t* sg;
        const uint32_t* e;
        bool go;
        ent(ne - 1, sg, e, go);
        if (!sig_encodes_fq(sg, (okmask >> (ne - 1)) & 1u, P, zi)) okmask &= ~(1u << (ne - 1));
    }
#pragma unroll 1
    for (int k = ne - 2; k >= 0; k--) {
        const uint32_t* o = st + (uint64_t)32 * k * stride;
        fp2 z, ck;
        unstash_f2(P.X, o, stride);
        unstash_f2(P.Y, o + 8 * stride, stride);
        unstash_f2(z, o + 16 * stride, stride);
        unstash_f2(ck, o + 24 * stride, stride);
        if (k > 0) {
            f2_mul(zi, inv, ck);
            f2_mul(inv, inv, z);
        } else {
            zi = inv;
        }
        const uint8_t* sg;
        const uint32_t* e;
        bool go;
        ent(k, sg, e, go);
        if (!sig_encodes_fq(sg, (okmask >> k) & 1u, P, zi)) okmask &= ~(1u << k);
    }
    return okmask;
}

}  // namespace poslo
