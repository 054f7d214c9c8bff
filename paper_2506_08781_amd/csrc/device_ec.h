// Device-side curve checks with fixed-base comb tables.
//
// A comb table of a point P holds t[w][d] = d * 16^w * P for 64 windows w and
// digits d < 16, as 32-word extended points.  Then for a scalar k < 2^256
//   k * P = sum over w of t[w][k_w],  k_w = the w-th 4-bit digit of k,
// which replaces 253 dependent doublings by independent lookups and adds.
#pragma once

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

// ge_add with its multiplications kept apart by scheduling barriers: the
// same arithmetic with fewer values live at once, for kernels whose register
// budget is tight (the group checks)
__device__ __forceinline__ void ge_add_lean(ge& r, const ge& p, const ge& q) {
    const fe d2 = POSLO_FE_D2;
    fe a, b, c, d, t;
    fe_sub(a, p.Y, p.X);
    fe_sub(t, q.Y, q.X);
    fe_mul(a, a, t);
    __builtin_amdgcn_sched_barrier(0);
    fe_add(b, p.Y, p.X);
    fe_add(t, q.Y, q.X);
    fe_mul(b, b, t);
    __builtin_amdgcn_sched_barrier(0);
    fe_mul(c, p.T, q.T);
    __builtin_amdgcn_sched_barrier(0);
    fe_mul(c, c, d2);
    __builtin_amdgcn_sched_barrier(0);
    fe_mul(d, p.Z, q.Z);
    fe_add(d, d, d);
    __builtin_amdgcn_sched_barrier(0);
    fe e, f, g, h;
    fe_sub(e, b, a);
    fe_sub(f, d, c);
    fe_add(g, d, c);
    fe_add(h, b, a);
    fe_mul(r.X, e, f);
    __builtin_amdgcn_sched_barrier(0);
    fe_mul(r.Y, g, h);
    __builtin_amdgcn_sched_barrier(0);
    fe_mul(r.T, e, h);
    __builtin_amdgcn_sched_barrier(0);
    fe_mul(r.Z, f, g);
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ uint32_t digit4(const uint32_t k[8], int w) { return (k[w >> 3] >> (4 * (w & 7))) & 15u; }

__device__ __forceinline__ const uint32_t* comb_entry(const uint32_t* table, int w, uint32_t d) {
    return table + (uint64_t)(w * 16 + d) * 32;
}

// e*Y + s*G by one whole wave: lane w adds window w of both tables, then a
// six-level tree of additions; the result is valid in lane 0.  Every lane of
// the wave must call it.
__device__ __forceinline__ void wave_double_scalar(ge& P, const uint32_t* ty, const uint32_t* tg, const uint32_t e[8],
                                                   const uint32_t s[8]) {
    const int w = threadIdx.x & 63;
    ge Q;
    load_point(P, comb_entry(ty, w, digit4(e, w)));
    load_point(Q, comb_entry(tg, w, digit4(s, w)));
    ge_add(P, P, Q);
    for (int off = 32; off > 0; off >>= 1) {
        shfl_down_point(Q, P, off);
        ge_add(P, P, Q);
    }
}

// e*Y + s*G by one lane: 128 lookups and additions
__device__ __forceinline__ void lane_double_scalar(ge& P, const uint32_t* ty, const uint32_t* tg, const uint32_t e[8],
                                                   const uint32_t s[8]) {
    ge_identity(P);
    for (int w = 0; w < 64; w++) {
        ge Q;
        load_point(Q, comb_entry(ty, w, digit4(e, w)));
        ge_add(P, P, Q);
        load_point(Q, comb_entry(tg, w, digit4(s, w)));
        ge_add(P, P, Q);
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
