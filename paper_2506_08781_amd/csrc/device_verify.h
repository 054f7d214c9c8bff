// Per-entry work for variable-length, arbitrarily aligned messages, and the
// individual verification of one entry (the Distill / SeBVer check).
#pragma once

#include "aes_perm.h"
#include "device_ec.h"
#include "device_entry.h"

namespace poslo {

// Message bytes [o, o + 4*nw) of an entry as little-endian words (o + 4*nw
// <= L).  Aligned words are loaded directly; otherwise nw + 1 aligned words
// are funnel-shifted with v_alignbyte_b32.  `end` bounds the buffer, so no
// load reaches past it.
template <int NW>
__device__ __forceinline__ void load_msg_words(const uint8_t* m, uint64_t o, const uint8_t* end, uint32_t w[NW]) {
    const uint8_t* A = m + o;
    uintptr_t a = (uintptr_t)A;
    uint32_t sh = (uint32_t)(a & 3u);
    const uint32_t* base = reinterpret_cast<const uint32_t*>(a - sh);
    if (sh == 0) {
#pragma unroll
        for (int k = 0; k < NW; k++) w[k] = base[k];
    } else if (reinterpret_cast<const uint8_t*>(base + NW + 1) <= end) {
        uint32_t d[NW + 1];
#pragma unroll
        for (int k = 0; k <= NW; k++) d[k] = base[k];
#pragma unroll
        for (int k = 0; k < NW; k++) w[k] = __builtin_amdgcn_alignbyte(d[k + 1], d[k], sh);
    } else {
#pragma unroll
        for (int k = 0; k < NW; k++) w[k] = load_le32(A + 4 * k);
    }
}

// MDC-2 over m || x for any length and alignment, with a table reader T
template <class T, class AesBlock>
__device__ __forceinline__ void digest_mdc2_any(const T& tb, const EntryView& v, const uint8_t* end,
                                                const uint32_t x[4], uint32_t dig[8], AesBlock blockfn) {
    uint32_t h[4], hp[4];
    uint64_t nfull = v.L / 16, b = 0;
    for (; b < nfull; b++) {
        uint32_t m[4];
        load_msg_words<4>(v.m, 16 * b, end, m);
        blockfn(tb, h, hp, m, b == 0);
    }
    uint64_t nb = (v.L + 16 + 15) / 16;
    for (; b < nb; b++) {
        uint32_t m[4];
#pragma unroll
        for (int w = 0; w < 4; w++) {
            uint32_t word = 0;
#pragma unroll
            for (int k = 0; k < 4; k++) word |= stream_byte_aes(v, x, 16 * b + 4 * w + k) << (8 * k);
            m[w] = word;
        }
        blockfn(tb, h, hp, m, b == 0);
    }
#pragma unroll
    for (int w = 0; w < 4; w++) {
        dig[w] = h[w];
        dig[4 + w] = hp[w];
    }
}

// one MDC-2 block with the generic T-table reader
struct Mdc2BlockGeneric {
    template <class T>
    __device__ __forceinline__ void operator()(const T& tb, uint32_t h[4], uint32_t hp[4], const uint32_t m[4],
                                               bool first) const {
        uint32_t sa[4] = {m[0], m[1], m[2], m[3]}, sb[4] = {m[0], m[1], m[2], m[3]};
        if (first) {
            aes128_encrypt_rk(tb, c_iv.a, sa);
            aes128_encrypt_rk(tb, c_iv.b, sb);
        } else {
            aes128_encrypt2_otf(tb, h, sa, hp, sb);
        }
#pragma unroll
        for (int w = 0; w < 4; w++) {
            sa[w] ^= m[w];
            sb[w] ^= m[w];
        }
        h[0] = sa[0], h[1] = sa[1], h[2] = sb[2], h[3] = sb[3];
        hp[0] = sb[0], hp[1] = sb[1], hp[2] = sa[2], hp[3] = sa[3];
    }
};

// one MDC-2 block with the byte-addressed LDS tables
struct Mdc2BlockPerm {
    template <int NT>
    __device__ __forceinline__ void operator()(const PermTables<NT>& tb, uint32_t h[4], uint32_t hp[4],
                                               const uint32_t m[4], bool first) const {
        uint32_t sa[4] = {m[0], m[1], m[2], m[3]}, sb[4] = {m[0], m[1], m[2], m[3]};
        if (first)
            penc2_rk(tb, c_iv.a, sa, c_iv.b, sb);
        else
            penc2_otf(tb, h, sa, hp, sb);
#pragma unroll
        for (int w = 0; w < 4; w++) {
            sa[w] ^= m[w];
            sb[w] ^= m[w];
        }
        h[0] = sa[0], h[1] = sa[1], h[2] = sb[2], h[3] = sb[3];
        hp[0] = sb[0], hp[1] = sb[1], hp[2] = sa[2], hp[3] = sa[3];
    }
};

// SHA-256(m || x) for any length and alignment (xw: big-endian words of x_t)
__device__ __forceinline__ void digest_sha_any(const EntryView& v, const uint8_t* end, const uint32_t xw[4],
                                               uint32_t dig[8]) {
    uint64_t total = ((v.L + 16 + 9 + 63) / 64) * 64;
    uint32_t H[8];
    sha256_init(H);
    uint64_t off = 0;
    for (; off + 64 <= v.L; off += 64) {
        uint32_t W[16];
        load_msg_words<16>(v.m, off, end, W);
#pragma unroll
        for (int w = 0; w < 16; w++) W[w] = bswap32(W[w]);
        sha256_compress(H, W);
    }
    for (; off < total; off += 64) {
        uint32_t W[16];
#pragma unroll
        for (int w = 0; w < 16; w++) W[w] = sha_stream_word<false>(v, xw, off + 4 * w, total);
        sha256_compress(H, W);
    }
#pragma unroll
    for (int w = 0; w < 8; w++) dig[w] = bswap32(H[w]);
}

// Individual verification of the entry at batch position pos with signature
// bytes sg (80): x_t equals the re-derived one-time seed, s_t < q, and
// encode(e_t*Y + s_t*G) equals the R_t bytes.  On success e (mod q) and s are
// returned.
template <class T>
__device__ __forceinline__ bool verify_one(const T& tb, const BatchArgs& a, const uint8_t* end, uint32_t inst,
                                           uint64_t pos, const uint8_t* sg, const uint32_t* ty, const uint32_t* tg,
                                           uint32_t e[8], uint32_t s[8]) {
    uint32_t x[4], xs[4];
    for (int k = 0; k < 4; k++) xs[k] = load_le32(sg + 64 + 4 * k);
    EntryView ev = entry_view(a, pos);
    uint32_t dig[8];
    if (inst == INST_AES) {
        one_time_seed_aes(tb, a, pos, x);
        if ((x[0] ^ xs[0]) | (x[1] ^ xs[1]) | (x[2] ^ xs[2]) | (x[3] ^ xs[3])) return false;
        for (int k = 0; k < 8; k++) s[k] = load_le32(sg + 4 * k);
        if (!sc_is_canonical(s)) return false;
        digest_mdc2_any(tb, ev, end, x, dig, Mdc2BlockGeneric{});
    } else {
        one_time_seed_sha(a, pos, x);  // big-endian words of the bytes of x_t
        if ((bswap32(x[0]) ^ xs[0]) | (bswap32(x[1]) ^ xs[1]) | (bswap32(x[2]) ^ xs[2]) | (bswap32(x[3]) ^ xs[3]))
            return false;
        for (int k = 0; k < 8; k++) s[k] = load_le32(sg + 4 * k);
        if (!sc_is_canonical(s)) return false;
        digest_sha_any(ev, end, x, dig);
    }
    sc_reduce256(e, dig);
    ge P;
    lane_double_scalar(P, ty, tg, e, s);
    uint32_t r[8];
    for (int k = 0; k < 8; k++) r[k] = load_le32(sg + 32 + 4 * k);
    return ge_encodes_to(P, r);
}

// The signature part of the screen: s_t < q and the R_t bytes decode strictly.
__device__ __forceinline__ bool screen_sig(const uint8_t* sg, uint32_t s[8], ge& R) {
    for (int k = 0; k < 8; k++) s[k] = load_le32(sg + 4 * k);
    if (!sc_is_canonical(s)) return false;
    uint8_t rb[32];
    for (int k = 0; k < 8; k++) store_le32(rb + 4 * k, load_le32(sg + 32 + 4 * k));
    return ge_decode(R, rb);
}

// The per-entry part of a group check: x_t equals the re-derived one-time
// seed, s_t < q and the R_t bytes decode (strictly, so that a decoded R_t
// encodes back to the same bytes).  On success e_t (mod q), s_t and R_t are
// returned; the entry is then valid exactly when e_t*Y + s_t*G == R_t.
template <class T>
__device__ __forceinline__ bool screen_one(const T& tb, const BatchArgs& a, const uint8_t* end, uint32_t inst,
                                           uint64_t pos, const uint8_t* sg, uint32_t e[8], uint32_t s[8], ge& R) {
    uint32_t x[4], xs[4];
    for (int k = 0; k < 4; k++) xs[k] = load_le32(sg + 64 + 4 * k);
    EntryView ev = entry_view(a, pos);
    uint32_t dig[8];
    if (inst == INST_AES) {
        one_time_seed_aes(tb, a, pos, x);
        if ((x[0] ^ xs[0]) | (x[1] ^ xs[1]) | (x[2] ^ xs[2]) | (x[3] ^ xs[3])) return false;
    } else {
        one_time_seed_sha(a, pos, x);
        if ((bswap32(x[0]) ^ xs[0]) | (bswap32(x[1]) ^ xs[1]) | (bswap32(x[2]) ^ xs[2]) | (bswap32(x[3]) ^ xs[3]))
            return false;
    }
    for (int k = 0; k < 8; k++) s[k] = load_le32(sg + 4 * k);
    if (!sc_is_canonical(s)) return false;
    uint8_t rb[32];
    for (int k = 0; k < 8; k++) store_le32(rb + 4 * k, load_le32(sg + 32 + 4 * k));
    if (!ge_decode(R, rb)) return false;
    if (inst == INST_AES)
        digest_mdc2_any(tb, ev, end, x, dig, Mdc2BlockGeneric{});
    else
        digest_sha_any(ev, end, x, dig);
    sc_reduce256(e, dig);
    return true;
}

// ---- group checks -------------------------------------------------------------

__device__ __forceinline__ void shfl_xor_point(ge& Q, const ge& P, int m) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
        Q.X.v[k] = __shfl_xor(P.X.v[k], m);
        Q.Y.v[k] = __shfl_xor(P.Y.v[k], m);
        Q.Z.v[k] = __shfl_xor(P.Z.v[k], m);
        Q.T.v[k] = __shfl_xor(P.T.v[k], m);
    }
}

// append `value` for every lane with `flag` set: one atomic per wave (ballot,
// the lowest set lane adds the popcount, every set lane takes its rank among
// the set lanes below it)
__device__ __forceinline__ void wave_append(bool flag, uint64_t value, uint64_t* list, uint32_t* count) {
    const uint64_t mask = __ballot(flag);
    if (!mask) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
    base = __shfl(base, (int)leader);
    if (flag) list[base + (uint32_t)__popcll(mask & ((1ull << lane) - 1))] = value;
}

// e*Y + s*G by a group of 8 lanes that pass the same e and s: lane k of the
// group adds windows 8k..8k+7 of both tables, then three levels of
// additions; the result is valid in every lane of the group.
__device__ __forceinline__ void group8_double_scalar(ge& P, const uint32_t* ty, const uint32_t* tg, const uint32_t e[8],
                                                     const uint32_t s[8]) {
    const int sub = threadIdx.x & 7;
    ge_identity(P);
#pragma unroll 1
    for (int k = 0; k < 8; k++) {
        const int w = sub * 8 + k;
        ge Q;
        load_point(Q, comb_entry(ty, w, digit4(e, w)));
        ge_add_lean(P, P, Q);
        load_point(Q, comb_entry(tg, w, digit4(s, w)));
        ge_add_lean(P, P, Q);
    }
#pragma unroll 1
    for (int m = 1; m < 8; m <<= 1) {
        ge Q;
        shfl_xor_point(Q, P, m);
        ge_add_lean(P, P, Q);
    }
}

__device__ __forceinline__ bool same_point(const ge& P, const ge& R) {
    fe a1, b1, a2, b2;
    fe_mul(a1, P.X, R.Z);
    fe_mul(b1, R.X, P.Z);
    fe_mul(a2, P.Y, R.Z);
    fe_mul(b2, R.Y, P.Z);
    return fe_equal(a1, b1) && fe_equal(a2, b2);
}

// sums of (e, s, R) over the lanes that differ from this one only in the
// bits of `bits` (a butterfly over those bits)
__device__ __forceinline__ void lane_sums(uint32_t e[8], uint32_t s[8], ge& R, int first, int last) {
#pragma unroll 1
    for (int m = first; m <= last; m <<= 1) {
        uint32_t oe[8], os[8];
        for (int k = 0; k < 8; k++) {
            oe[k] = __shfl_xor(e[k], m);
            os[k] = __shfl_xor(s[k], m);
        }
        sc_add(e, e, oe);
        sc_add(s, s, os);
        ge Q;
        shfl_xor_point(Q, R, m);
        ge_add_lean(R, R, Q);
    }
}

__device__ __forceinline__ void store_sums(uint32_t* o, const uint32_t e[8], const uint32_t s[8], const ge& R) {
    for (int k = 0; k < 8; k++) {
        o[k] = e[k];
        o[8 + k] = s[k];
    }
    store_point(o + 16, R);
}

// The 8 groups' relations checked at once, 8 lanes per group (lanes 8g..8g+7
// check the sums in gs[g]); returns the mask of failing groups.
__device__ __forceinline__ uint32_t check_groups8(const uint32_t (*gs)[48], const uint32_t* ty, const uint32_t* tg) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t* g = gs[lane >> 3];
    uint32_t eg[8], sg[8];
    for (int k = 0; k < 8; k++) {
        eg[k] = g[k];
        sg[k] = g[8 + k];
    }
    ge Rg, P;
    load_point(Rg, g + 16);
    group8_double_scalar(P, ty, tg, eg, sg);
    const bool bad = (lane & 7) == 0 && !same_point(P, Rg);
    const uint64_t m = __ballot(bad);
    uint32_t fail = 0;
    for (int k = 0; k < 8; k++)
        if ((m >> (8 * k)) & 1ull) fail |= 1u << k;
    return fail;
}

// Group checks of (sum e)*Y + (sum s)*G == sum R over two partitions of the
// wave's 64 entries into 8 groups of 8: "rows" (lanes 8g..8g+7) and
// "columns" (lanes congruent to g mod 8).  A row and a column share exactly
// one lane, so errors of two invalid entries can cancel in at most one of
// the two groups that each of them belongs to; an entry needs an individual
// check when its row or its column fails.  (e, s, R) of each lane is (zero,
// zero, identity) for lanes that do not take part; gs is this wave's LDS
// area of 16 x 48 words.  Returns the wave-uniform masks: rows in bits 0-7,
// columns in bits 8-15.  e, s and R are overwritten; every lane of the wave
// must call it.  own is this wave's LDS area of 64 x 48 words: it keeps each
// lane's (e, s, R) (read back with load_own after the call).
__device__ __forceinline__ uint32_t wave_group_checks(uint32_t e[8], uint32_t s[8], ge& R, uint32_t (*gs)[48],
                                                      uint32_t (*own)[48], const uint32_t* ty, const uint32_t* tg) {
    const uint32_t lane = threadIdx.x & 63;
    store_sums(own[lane], e, s, R);
    lane_sums(e, s, R, 1, 4);  // rows
    if ((lane & 7) == 0) store_sums(gs[lane >> 3], e, s, R);
    for (int k = 0; k < 8; k++) {
        e[k] = own[lane][k];
        s[k] = own[lane][8 + k];
    }
    load_point(R, own[lane] + 16);
    lane_sums(e, s, R, 8, 32);  // columns
    if (lane < 8) store_sums(gs[8 + lane], e, s, R);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t rows = check_groups8(gs, ty, tg);
    const uint32_t cols = check_groups8(gs + 8, ty, tg);
    return rows | (cols << 8);
}

// an entry needs its individual check when its row or its column failed
__device__ __forceinline__ bool group_suspect(uint32_t masks) {
    const uint32_t lane = threadIdx.x & 63;
    return ((masks >> (lane >> 3)) & 1u) || ((masks >> (8 + (lane & 7))) & 1u);
}

}  // namespace poslo
