// Host-side building blocks of the scheme: byte-level MMO / MDC-2 / SHA-256,
// the PRF and H of each instantiation, the seed tree functions SC / SSO / SR,
// scalar arithmetic mod q and fixed-base multiplication.  Used by the signer
// and by the verifier's host-side argument checks.
#pragma once

#include <string.h>

#include <vector>

#include "aes128.h"
#include "fourq.h"
#include "ge25519.h"
#include "sc25519.h"
#include "sha256.h"

namespace poslo {
namespace hostside {

// ---- MMO and MDC-2 over AES-128 (paper, Definitions "MMO" and "MDC-2") ----
// zero padding of the last block, max(1, ceil(len/16)) blocks, chaining
// value as the key; IVs 0x52.. and 0x25..

inline void block_at(const uint8_t* in, size_t len, size_t b, uint32_t m[4]) {
    uint8_t blk[16] = {0};
    size_t off = 16 * b;
    size_t take = len > off ? (len - off < 16 ? len - off : 16) : 0;
    if (take) memcpy(blk, in + off, take);
    for (int w = 0; w < 4; w++) m[w] = load_le32(blk + 4 * w);
}

inline void mmo(const uint8_t* in, size_t len, uint8_t out[16]) {
    HostTables tb;
    uint32_t h[4] = {kIvA, kIvA, kIvA, kIvA};
    size_t nb = len == 0 ? 1 : (len + 15) / 16;
    for (size_t b = 0; b < nb; b++) {
        uint32_t m[4], s[4];
        block_at(in, len, b, m);
        for (int w = 0; w < 4; w++) s[w] = m[w];
        aes128_encrypt_otf(tb, h, s);
        for (int w = 0; w < 4; w++) h[w] = s[w] ^ m[w];
    }
    for (int w = 0; w < 4; w++) store_le32(out + 4 * w, h[w]);
}

inline void mdc2(const uint8_t* in, size_t len, uint8_t out[32]) {
    HostTables tb;
    uint32_t h[4] = {kIvA, kIvA, kIvA, kIvA}, hp[4] = {kIvB, kIvB, kIvB, kIvB};
    size_t nb = len == 0 ? 1 : (len + 15) / 16;
    for (size_t b = 0; b < nb; b++) {
        uint32_t m[4], sa[4], sb[4];
        block_at(in, len, b, m);
        for (int w = 0; w < 4; w++) sa[w] = sb[w] = m[w];
        aes128_encrypt2_otf(tb, h, sa, hp, sb);
        for (int w = 0; w < 4; w++) {
            sa[w] ^= m[w];
            sb[w] ^= m[w];
        }
        // h = a^1 || b^2, h' = b^1 || a^2 (8-byte halves = word pairs)
        h[0] = sa[0], h[1] = sa[1], h[2] = sb[2], h[3] = sb[3];
        hp[0] = sb[0], hp[1] = sb[1], hp[2] = sa[2], hp[3] = sa[3];
    }
    for (int w = 0; w < 4; w++) {
        store_le32(out + 4 * w, h[w]);
        store_le32(out + 16 + 4 * w, hp[w]);
    }
}

inline void sha256(const uint8_t* in, size_t len, uint8_t out[32]) {
    uint32_t H[8];
    sha256_init(H);
    size_t total = ((len + 9 + 63) / 64) * 64;
    uint64_t bits = (uint64_t)len * 8u;
    for (size_t off = 0; off < total; off += 64) {
        uint8_t blk[64];
        for (size_t k = 0; k < 64; k++) {
            size_t pos = off + k;
            uint8_t v = 0;
            if (pos < len)
                v = in[pos];
            else if (pos == len)
                v = 0x80;
            else if (pos >= total - 8)
                v = (uint8_t)(bits >> (8 * (total - 1 - pos)));
            blk[k] = v;
        }
        uint32_t W[16];
        for (int w = 0; w < 16; w++) W[w] = bswap32(load_le32(blk + 4 * w));
        sha256_compress(H, W);
    }
    for (int w = 0; w < 8; w++) store_le32(out + 4 * w, bswap32(H[w]));
}

// F: MMO-AES-128 (POSLO+, POSLO++) or SHA-256 truncated to 16 bytes (POSLO);
// spec is the instantiation word (common.h)
inline void F(uint32_t spec, const uint8_t* in, size_t len, uint8_t out[16]) {
    if (prf_is_aes(spec)) {
        mmo(in, len, out);
    } else {
        uint8_t d[32];
        sha256(in, len, d);
        memcpy(out, d, 16);
    }
}

// H over a byte string: MDC-2-AES-128 or SHA-256 (Add_q takes the message
// and the seed apart: digest_e)
inline void H(uint32_t spec, const uint8_t* in, size_t len, uint8_t out[32]) {
    if (inst_base(spec) == INST_SHA256)
        sha256(in, len, out);
    else
        mdc2(in, len, out);
}

// PRF_b(z) = F(z || b), b one byte.  With kappa = 127 a 16-byte z is a seed
// and b its bit 127, one MMO block; every output is then taken mod 2^127.
inline void prf(uint32_t spec, uint32_t b, const uint8_t* in, size_t len, uint8_t out[16]) {
    if (kappa127(spec) && len == 16) {
        uint8_t blk[16];
        memcpy(blk, in, 16);
        blk[15] = (uint8_t)((blk[15] & 0x7f) | (b << 7));
        F(spec, blk, 16, out);
    } else {
        std::vector<uint8_t> z(len + 1);
        if (len) memcpy(z.data(), in, len);
        z[len] = (uint8_t)b;
        F(spec, z.data(), z.size(), out);
    }
    if (kappa127(spec)) out[15] &= 0x7f;
}

// ---- seed tree (section "POSLO Data Types and Seed Management") ---------

struct DsNode {
    uint32_t depth;
    uint32_t index;
    uint8_t v[16];
};

// SC: x_{d1}[i1] from x_{d0}[i0], PRF bit by bit of the path, MSB first
inline void seed_walk(uint32_t inst, const uint8_t x[16], uint32_t d0, uint64_t i1, uint32_t d1, uint8_t out[16]) {
    uint8_t cur[16];
    memcpy(cur, x, 16);
    for (int j = (int)d0 - (int)d1 - 1; j >= 0; j--) {
        uint8_t nxt[16];
        prf(inst, (uint32_t)((i1 >> j) & 1u), cur, 16, nxt);
        memcpy(cur, nxt, 16);
    }
    memcpy(out, cur, 16);
}

// SSO(ds_{i-1}, x_D[0], i) -> (ds_i, x_0[i])
inline void sso(uint32_t inst, std::vector<DsNode>& ds, const uint8_t root[16], uint32_t D, uint64_t i,
                uint8_t x0[16]) {
    uint32_t d1 = 0;
    uint64_t i1 = i;
    while (!ds.empty() && ds.back().depth == d1) {
        ds.pop_back();
        d1++;
        i1 >>= 1;
    }
    DsNode n;
    n.depth = d1;
    n.index = (uint32_t)i1;
    seed_walk(inst, root, D, i1, d1, n.v);
    ds.push_back(n);
    seed_walk(inst, n.v, d1, i, 0, x0);
}

// SR(ds, i'): index of the covering node in ds, or -1 for "bottom"
inline int sr_node(const DsNode* ds, int count, uint64_t ip) {
    if (count <= 0) return -1;
    int k = count - 1;
    if (ip >= ((uint64_t)ds[k].index + 1) << ds[k].depth) return -1;
    while (ip < ((uint64_t)ds[k].index << ds[k].depth)) {
        if (--k < 0) return -1;
    }
    return k;
}

// strict parse of the ds wire format into a fixed array of 32 nodes (no
// allocation); *count gets the number of nodes
inline bool ds_parse(const uint8_t* buf, size_t len, DsNode out[32], int* count) {
    *count = 0;
    if (!buf || len < 1) return false;
    uint32_t cnt = buf[0];
    if (cnt > 32 || len != 1 + 24 * (size_t)cnt) return false;
    for (uint32_t k = 0; k < cnt; k++) {
        const uint8_t* p = buf + 1 + 24 * k;
        DsNode& n = out[k];
        n.depth = p[0];
        if (p[1] | p[2] | p[3]) return false;
        n.index = load_le32(p + 4);
        if (n.depth > 32 || (n.depth > 0 && n.depth < 32 && (n.index >> (32 - n.depth)))) return false;
        memcpy(n.v, p + 8, 16);
    }
    *count = (int)cnt;
    return true;
}

inline bool ds_parse(const uint8_t* buf, size_t len, std::vector<DsNode>& out) {
    DsNode nodes[32];
    int cnt = 0;
    out.clear();
    if (!ds_parse(buf, len, nodes, &cnt)) return false;
    out.assign(nodes, nodes + cnt);
    return true;
}

inline void ds_serialize(const std::vector<DsNode>& ds, std::vector<uint8_t>& out) {
    out.assign(1 + 24 * ds.size(), 0);
    out[0] = (uint8_t)ds.size();
    for (size_t k = 0; k < ds.size(); k++) {
        uint8_t* p = out.data() + 1 + 24 * k;
        p[0] = (uint8_t)ds[k].depth;
        store_le32(p + 4, ds[k].index);
        memcpy(p + 8, ds[k].v, 16);
    }
}

// ---- scalars mod q ---------------------------------------------------------

inline void sc_from_bytes_reduce(uint32_t r[8], const uint8_t b[32]) {
    uint32_t x[8];
    for (int i = 0; i < 8; i++) x[i] = load_le32(b + 4 * i);
    sc_reduce256(r, x);
}

// e_t = H(m || x) mod q (mod N for FourQ) as eight LE words; POSLO++ takes Add_q(m, x) =
// LE(m) + LE(x), below q for |m| <= 31 bytes (false for longer messages)
inline bool digest_e(uint32_t spec, const uint8_t* m, size_t len, const uint8_t x[16], uint32_t e[8]) {
    if (inst_base(spec) == INST_AES_ADDQ) {
        if (len > kAddqMaxLen) return false;
        uint8_t mb[32] = {0};
        if (len) memcpy(mb, m, len);
        uint64_t c = 0;
        for (int w = 0; w < 8; w++) {
            c += (uint64_t)load_le32(mb + 4 * w) + (w < 4 ? load_le32(x + 4 * w) : 0u);
            e[w] = (uint32_t)c;
            c >>= 32;
        }
        return true;
    }
    std::vector<uint8_t> mx(len + 16);
    if (len) memcpy(mx.data(), m, len);
    memcpy(mx.data() + len, x, 16);
    uint8_t d[32];
    H(spec, mx.data(), mx.size(), d);
    if (spec & POSLO_GROUP_FOURQ) {  // LE256(H) mod N
        uint32_t w[8];
        for (int i = 0; i < 8; i++) w[i] = load_le32(d + 4 * i);
        scN_reduce<8>(e, w);
    } else {
        sc_from_bytes_reduce(e, d);
    }
    return true;
}

// LE256(b) reduced mod the group order of the instantiation word
inline void scalar_from_bytes(uint32_t spec, uint32_t r[8], const uint8_t b[32]) {
    if (spec & POSLO_GROUP_FOURQ) {
        uint32_t w[8];
        for (int i = 0; i < 8; i++) w[i] = load_le32(b + 4 * i);
        scN_reduce<8>(r, w);
    } else {
        sc_from_bytes_reduce(r, b);
    }
}

// (a * b) mod q: schoolbook product, then shift-and-subtract reduction
inline void sc_mul(uint32_t r[8], const uint32_t a[8], const uint32_t b[8]) {
    const uint32_t q[8] = POSLO_SC_Q;
    uint32_t t[16] = {0};
    for (int i = 0; i < 8; i++) {
        uint64_t c = 0;
        for (int j = 0; j < 8; j++) {
            c += (uint64_t)a[i] * b[j] + t[i + j];
            t[i + j] = (uint32_t)c;
            c >>= 32;
        }
        t[i + 8] = (uint32_t)c;
    }
    uint32_t acc[8] = {0};
    for (int bit = 511; bit >= 0; bit--) {
        uint32_t carry = (t[bit >> 5] >> (bit & 31)) & 1u;
        for (int i = 0; i < 8; i++) {
            uint32_t nc = acc[i] >> 31;
            acc[i] = (acc[i] << 1) | carry;
            carry = nc;
        }
        // acc < 2q < 2^254: subtract q if acc >= q
        uint32_t d[8];
        int64_t bw = 0;
        for (int i = 0; i < 8; i++) {
            bw += (int64_t)acc[i] - q[i];
            d[i] = (uint32_t)bw;
            bw >>= 32;
        }
        if (bw == 0)
            for (int i = 0; i < 8; i++) acc[i] = d[i];
    }
    for (int i = 0; i < 8; i++) r[i] = acc[i];
}

// (a - b) mod q for canonical a, b
inline void sc_sub(uint32_t r[8], const uint32_t a[8], const uint32_t b[8]) {
    const uint32_t q[8] = POSLO_SC_Q;
    int64_t bw = 0;
    for (int i = 0; i < 8; i++) {
        bw += (int64_t)a[i] - b[i];
        r[i] = (uint32_t)bw;
        bw >>= 32;
    }
    if (bw) {
        uint64_t c = 0;
        for (int i = 0; i < 8; i++) {
            c += (uint64_t)r[i] + q[i];
            r[i] = (uint32_t)c;
            c >>= 32;
        }
    }
}

// ---- fixed-base multiplication k*G with a 4-bit comb (64 windows) ---------

struct BaseTable {
    ge t[64][16];  // t[w][d] = d * 16^w * G
};

const BaseTable& base_table();  // built once per process

inline void ge_scalarmult_base(ge& r, const uint32_t k[8]) {
    const BaseTable& T = base_table();
    ge R;
    ge_identity(R);
    for (int w = 0; w < 64; w++) {
        uint32_t d = (k[w >> 3] >> (4 * (w & 7))) & 15u;
        if (d) ge_add(R, R, T.t[w][d]);
    }
    r = R;
}

// FourQ (fourq.h): the same fixed-base scheme over FourQ's generator
struct FqBaseTable {
    gq t[64][16];  // t[w][d] = d * 16^w * G
};

const FqBaseTable& fq_base_table();  // built once per process

inline void fq_scalarmult_base(gq& r, const uint32_t k[8]) {
    const FqBaseTable& T = fq_base_table();
    gq R;
    gq_identity(R);
    for (int w = 0; w < 64; w++) {
        uint32_t d = (k[w >> 3] >> (4 * (w & 7))) & 15u;
        if (d) gq_add(R, R, T.t[w][d]);
    }
    r = R;
}

// the instantiation word selects FourQ
inline bool group_fourq(uint32_t spec) { return (spec & POSLO_GROUP_FOURQ) != 0; }

}  // namespace hostside
}  // namespace poslo
