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
        for (int k = 0; k < NW; k++) w[k] = gload(base + k);
    } else if (reinterpret_cast<const uint8_t*>(base + NW + 1) <= end) {
        uint32_t d[NW + 1];
#pragma unroll
        for (int k = 0; k <= NW; k++) d[k] = gload(base + k);
#pragma unroll
        for (int k = 0; k < NW; k++) w[k] = __builtin_amdgcn_alignbyte(d[k + 1], d[k], sh);
    } else {
#pragma unroll
        for (int k = 0; k < NW; k++) w[k] = gload_le32(A + 4 * k);
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

// The same with x_t derived only for the final blocks: xf(x) writes it into
// x, which is returned; fewer values live across the message blocks
template <class T, class XF, class AesBlock>
__device__ __forceinline__ void digest_mdc2_any_late(const T& tb, const EntryView& v, const uint8_t* end, const XF& xf,
                                                     uint32_t x[4], uint32_t dig[8], AesBlock blockfn) {
    uint32_t h[4], hp[4];
    uint64_t nfull = v.L / 16, b = 0;
    for (; b < nfull; b++) {
        uint32_t m[4];
        load_msg_words<4>(v.m, 16 * b, end, m);
        blockfn(tb, h, hp, m, b == 0);
    }
    xf(x);
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
    template <int NT, int CP>
    __device__ __forceinline__ void operator()(const PermTables<NT, CP>& tb, uint32_t h[4], uint32_t hp[4],
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

// The curve part of an entry's check, given e_t (mod q): s_t < q and
// encode(e_t*Y + s_t*G) equals the R_t bytes of the signature sg (80 bytes:
// s_t, R_t, x_t).  s is returned.  ty: Y's table; tg_wide: G's wide table.
__device__ __forceinline__ bool verify_sig(const uint8_t* sg, const uint32_t e[8], const uint32_t* ty,
                                           const uint32_t* tg_wide, uint32_t s[8]) {
    for (int k = 0; k < 8; k++) s[k] = gload_le32(sg + 4 * k);
    if (!sc_is_canonical(s)) return false;
    ge P;
    lane_double_scalar_wide(P, ty, tg_wide, e, s);
    uint32_t r[8];
    for (int k = 0; k < 8; k++) r[k] = gload_le32(sg + 32 + 4 * k);
    return ge_encodes_to(P, r);
}

// encode(P) == bytes given 1/Z (eight little-endian words)
__device__ __forceinline__ bool encodes_to_zinv(const ge& P, const fe& zi, const uint32_t want[8]) {
    fe x, y;
    fe_mul(x, P.X, zi);
    fe_mul(y, P.Y, zi);
    uint8_t enc[32];
    fe_to_bytes(enc, y);
    enc[31] |= (uint8_t)(fe_isodd(x) << 7);
    uint32_t diff = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) diff |= load_le32(enc + 4 * k) ^ want[k];
    return diff == 0;
}

// WY: ty is Y's wide table (else its 8-bit table)
template <bool WY>
__device__ __forceinline__ bool sig_point(const uint8_t* sg, const uint32_t* e, bool go, const uint32_t* ty,
                                          const uint32_t* tg_wide, ge& P) {
    uint32_t ek[8], s[8];
    for (int w = 0; w < 8; w++) {
        s[w] = go ? gload_le32(sg + 4 * w) : 0u;
        ek[w] = go ? e[w] : 0u;
    }
    const bool c = go && sc_is_canonical(s);
    if (!c)
        for (int w = 0; w < 8; w++) s[w] = ek[w] = 0;  // the identity: Z stays nonzero
    if constexpr (WY)
        lane_double_scalar_wide2(P, ty, tg_wide, ek, s);
    else
        lane_double_scalar_wide(P, ty, tg_wide, ek, s);
    return c;
}

__device__ __forceinline__ bool sig_encodes(const uint8_t* sg, bool c, const ge& P, const fe& zi) {
    uint32_t r[8];
    for (int w = 0; w < 8; w++) r[w] = c ? gload_le32(sg + 32 + 4 * w) : 0u;
    return c && encodes_to_zinv(P, zi, r);
}

// The curve part of ne entries' checks per thread (1 <= ne <= 32, uniform
// across the wave) with one inversion for all of them (Montgomery's trick).
// Entries 0 .. ne-2 wait in global memory: entry k keeps X, Y, Z and
// c_{k-1} = Z_0 ... Z_{k-1} at st[(32 k + w) * stride], w < 32, where st is
// the thread's own base (only the thread itself reads its slots back); the
// last stays in registers.  With inv = 1 / c_{ne-1}, entry k takes
// 1/Z_k = inv * c_{k-1} and then inv *= Z_k, going down.  ent(k, sg, e, go)
// names entry k: signature, e_t in memory, and whether to check it
// (go = false reports it invalid; its pointers must still be readable).
// Bit k of the result is set when entry k is valid.
template <bool WY, class ENT>
__device__ __forceinline__ uint32_t verify_sig_batch(const ENT& ent, int ne, const uint32_t* ty,
                                                       const uint32_t* tg_wide, uint32_t* st, uint32_t stride) {
    if (ne <= 0) return 0;
    uint32_t okmask = 0;
    fe c, c_prev;
    fe_set(c_prev, 1);
    ge P;
#pragma unroll 1
    for (int k = 0; k < ne; k++) {
        const uint8_t* sg;
        const uint32_t* e;
        bool go;
        ent(k, sg, e, go);
        if (sig_point<WY>(sg, e, go, ty, tg_wide, P)) okmask |= 1u << k;
        if (k == 0) {
            c = P.Z;
        } else {
            c_prev = c;
            fe_mul(c, c, P.Z);
        }
        if (k < ne - 1) {
            uint32_t* o = st + (uint64_t)32 * k * stride;
#pragma unroll
            for (int w = 0; w < 8; w++) {
                o[w * stride] = P.X.v[w];
                o[(8 + w) * stride] = P.Y.v[w];
                o[(16 + w) * stride] = P.Z.v[w];
                o[(24 + w) * stride] = c_prev.v[w];
            }
        }
    }
    fe inv, zi;
    fe_inv(inv, c);  // 1 / (Z_0 ... Z_{ne-1})
    {
        // the last entry, from registers
        if (ne > 1) {
            fe_mul(zi, inv, c_prev);
            fe_mul(inv, inv, P.Z);
        } else {
            zi = inv;
        }
        const uint8_t* sg;
        const uint32_t* e;
        bool go;
        ent(ne - 1, sg, e, go);
        if (!sig_encodes(sg, (okmask >> (ne - 1)) & 1u, P, zi)) okmask &= ~(1u << (ne - 1));
    }
#pragma unroll 1
    for (int k = ne - 2; k >= 0; k--) {
        const uint32_t* o = st + (uint64_t)32 * k * stride;
        fe z, ck;
#pragma unroll
        for (int w = 0; w < 8; w++) {
            P.X.v[w] = o[w * stride];
            P.Y.v[w] = o[(8 + w) * stride];
            z.v[w] = o[(16 + w) * stride];
            ck.v[w] = o[(24 + w) * stride];
        }
        if (k > 0) {
            fe_mul(zi, inv, ck);
            fe_mul(inv, inv, z);
        } else {
            zi = inv;
        }
        const uint8_t* sg;
        const uint32_t* e;
        bool go;
        ent(k, sg, e, go);
        if (!sig_encodes(sg, (okmask >> k) & 1u, P, zi)) okmask &= ~(1u << k);
    }
    return okmask;
}

// Launch shape of the persistent check kernels: one wave per workgroup,
// two per SIMD (their register budget), each thread checking up to
// kVerifyNEMax entries of a tile with one shared inversion, the points
// waiting in kVerifyStashWords of global memory per wave.
constexpr int kVerifyNEMax = 16;
constexpr uint64_t kVerifyStashWords = (uint64_t)(kVerifyNEMax - 1) * 32 * 64;
constexpr int kVerifyWgPerCu = 8;

// entries per tile (a multiple of 64, at most 64 * kVerifyNEMax) for n
// entries: as many per thread as keeps every wave slot of the chip busy
inline uint32_t verify_tile_len(uint64_t n, int num_cu) {
    const uint64_t lanes = (uint64_t)num_cu * kVerifyWgPerCu * 64;
    const uint64_t per = (n + lanes - 1) / lanes;
    return 64u * (uint32_t)(per < 1 ? 1 : per > kVerifyNEMax ? kVerifyNEMax : per);
}

// The hashing part of the check of the entry at batch position pos with
// signature bytes sg (80): false when x_t differs from the re-derived
// one-time seed (or, POSLO++, when the message is longer than 31 bytes,
// which also sets a.bad); else dig = H(m_t || x_t) as eight little-endian
// words (POSLO++: Add_q(m_t, x_t), already below q).
template <class T>
__device__ __forceinline__ bool entry_digest(const T& tb, const BatchArgs& a, const uint8_t* end, uint32_t inst,
                                             uint64_t pos, const uint8_t* sg, uint32_t dig[8]) {
    uint32_t x[4], xs[4];
    for (int k = 0; k < 4; k++) xs[k] = gload_le32(sg + 64 + 4 * k);
    EntryView ev = entry_view(a, pos);
    if (inst_base(inst) == INST_AES_ADDQ) {
        if (ev.L > kAddqMaxLen) {
            if (a.bad) *a.bad = 1u;
            return false;
        }
        one_time_seed_aes(tb, a, pos, x);
        if ((x[0] ^ xs[0]) | (x[1] ^ xs[1]) | (x[2] ^ xs[2]) | (x[3] ^ xs[3])) return false;
        uint32_t mw[8];
        addq_message<0>(ev.m, (uint32_t)ev.L, mw);
        addq_digest(mw, x, dig);
        return true;
    }
    if (inst_base(inst) == INST_AES) {
        one_time_seed_aes(tb, a, pos, x);
        if ((x[0] ^ xs[0]) | (x[1] ^ xs[1]) | (x[2] ^ xs[2]) | (x[3] ^ xs[3])) return false;
        digest_mdc2_any(tb, ev, end, x, dig, Mdc2BlockGeneric{});
    } else {
        one_time_seed_sha(a, pos, x);  // big-endian words of the bytes of x_t
        if ((bswap32(x[0]) ^ xs[0]) | (bswap32(x[1]) ^ xs[1]) | (bswap32(x[2]) ^ xs[2]) | (bswap32(x[3]) ^ xs[3]))
            return false;
        digest_sha_any(ev, end, x, dig);
    }
    return true;
}

// Individual verification of the entry at batch position pos with signature
// bytes sg (80) on edwards25519: x_t equals the re-derived one-time seed,
// s_t < q, and encode(e_t*Y + s_t*G) equals the R_t bytes.  On success e
// (mod q) and s are returned.  inst: the instantiation word.  A POSLO++
// message longer than 31 bytes fails and sets a.bad.
template <class T>
__device__ __forceinline__ bool verify_one(const T& tb, const BatchArgs& a, const uint8_t* end, uint32_t inst,
                                           uint64_t pos, const uint8_t* sg, const uint32_t* ty, const uint32_t* tg_wide,
                                           uint32_t e[8], uint32_t s[8]) {
    uint32_t dig[8];
    if (!entry_digest(tb, a, end, inst, pos, sg, dig)) return false;
    if (inst_base(inst) == INST_AES_ADDQ)
        for (int k = 0; k < 8; k++) e[k] = dig[k];
    else
        sc_reduce256(e, dig);
    return verify_sig(sg, e, ty, tg_wide, s);
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

}  // namespace poslo
