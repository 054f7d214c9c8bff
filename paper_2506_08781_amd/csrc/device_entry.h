// Per-entry device work shared by the verification kernels: the batch
// argument block, message views, the one-time seed x_t = PRF_0(x_0[i] || j)
// and the digest H(m_t || x_t) of both instantiations, and the 288-bit
// workgroup reduction.
#pragma once

#include "device_hash.h"
#include "sc25519.h"

namespace poslo {

struct BatchArgs {
    const uint8_t* data;
    const uint64_t* offsets;  // nullptr: fixed length
    uint64_t msg_len;
    uint64_t n;
    uint64_t t0;
    uint64_t epoch_first;
    uint32_t log2_n2;
    const uint32_t* tab;   // per-epoch table, kEpochWords each
    const uint32_t* skip;  // optional bitmap over batch positions
    const uint8_t* end;    // end of the data buffer, or nullptr when unknown
    // AES-based PRF: mask of x_t's top word (0x7fffffff at kappa = 127)
    uint32_t xmask = 0xffffffffu;
    // POSLO++: set to nonzero by any kernel that meets a (non-skipped) message
    // longer than 31 bytes; zeroed by the seed-table kernel
    uint32_t* bad = nullptr;
    // emitted e_t are reduced mod FourQ's N instead of q
    uint32_t emit_fq = 0;
};

struct EntryView {
    const uint8_t* m;
    uint64_t L;
};

// Loads through the global address space.  Pointers that kernels read out
// of job tables in memory are generic to the compiler, and generic (flat)
// loads also count against the LDS wait counter, which would tie every
// message load to the T-table lookups in flight.  Every pointer given to
// these is device memory.
template <class T>
__device__ __forceinline__ T gload(const T* p) {
    return *reinterpret_cast<const __attribute__((address_space(1))) T*>(reinterpret_cast<uintptr_t>(p));
}

// 16 bytes at a 16-byte-aligned address (a native vector type: HIP's uint4
// cannot be copied out of the global address space directly)
__device__ __forceinline__ uint4 gload(const uint4* p) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = *reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(reinterpret_cast<uintptr_t>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// little-endian 32-bit word at any byte address of device memory
__device__ __forceinline__ uint32_t gload_le32(const uint8_t* p) {
    return (uint32_t)gload(p) | ((uint32_t)gload(p + 1) << 8) | ((uint32_t)gload(p + 2) << 16) |
           ((uint32_t)gload(p + 3) << 24);
}

__device__ __forceinline__ EntryView entry_view(const BatchArgs& a, uint64_t pos) {
    EntryView v;
    if (a.offsets) {
        uint64_t o0 = gload(a.offsets + pos), o1 = gload(a.offsets + pos + 1);
        v.m = a.data + o0;
        v.L = o1 - o0;
    } else {
        v.m = a.data + pos * a.msg_len;
        v.L = a.msg_len;
    }
    return v;
}

__device__ __forceinline__ bool skipped(const BatchArgs& a, uint64_t pos) {
    return a.skip && ((a.skip[pos >> 5] >> (pos & 31)) & 1u);
}

// ---- POSLO+ (AES) ----------------------------------------------------------

// byte pos of the stream m || x || zero padding (x as four little-endian words)
__device__ __forceinline__ uint32_t stream_byte_aes(const EntryView& v, const uint32_t x[4], uint64_t pos) {
    if (pos < v.L) return gload(v.m + pos);
    uint64_t o = pos - v.L;
    if (o < 16) return (x[o >> 2] >> (8 * (o & 3))) & 0xffu;
    return 0;
}

// x_t: one AES under the epoch's precomputed schedule (the second MMO block
// of PRF_0(x_0[i] || LE32(j)); the first block is epoch-constant)
template <class T>
__device__ __forceinline__ void one_time_seed_aes(const T& tb, const BatchArgs& a, uint64_t pos, uint32_t x[4]) {
    uint64_t t = a.t0 + pos;
    uint64_t ep = (t >> a.log2_n2) - a.epoch_first;
    uint32_t j = (uint32_t)(t & ((1ull << a.log2_n2) - 1));
    const uint32_t* rk = a.tab + ep * kEpochWords;
    uint32_t s[4] = {j, 0u, 0u, 0u};
    aes128_encrypt_rk(tb, rk, s);
    x[0] = s[0] ^ j;
    x[1] = s[1];
    x[2] = s[2];
    x[3] = s[3] & a.xmask;
}

// MDC-2 over m || x; FAST: 16-byte aligned message of a length divisible by 16
template <bool FAST, class T>
__device__ __forceinline__ void digest_mdc2(const T& tb, const EntryView& v, const uint32_t x[4], uint32_t dig[8]) {
    uint64_t nb = (v.L + 16 + 15) / 16;
    uint32_t h[4], hp[4];
    for (uint64_t b = 0; b < nb; b++) {
        uint32_t m[4];
        if (FAST) {
            if (16 * b < v.L) {
                uint4 q = gload(reinterpret_cast<const uint4*>(v.m) + b);
                m[0] = q.x, m[1] = q.y, m[2] = q.z, m[3] = q.w;
            } else {
                m[0] = x[0], m[1] = x[1], m[2] = x[2], m[3] = x[3];
            }
        } else {
#pragma unroll
            for (int w = 0; w < 4; w++) {
                uint32_t word = 0;
#pragma unroll
                for (int k = 0; k < 4; k++) word |= stream_byte_aes(v, x, 16 * b + 4 * w + k) << (8 * k);
                m[w] = word;
            }
        }
        uint32_t sa[4] = {m[0], m[1], m[2], m[3]}, sb[4] = {m[0], m[1], m[2], m[3]};
        if (b == 0) {
            // the first block is keyed by the constant IVs: precomputed schedules
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
        // h = a^1 || b^2, h' = b^1 || a^2
        h[0] = sa[0], h[1] = sa[1], h[2] = sb[2], h[3] = sb[3];
        hp[0] = sb[0], hp[1] = sb[1], hp[2] = sa[2], hp[3] = sa[3];
    }
#pragma unroll
    for (int w = 0; w < 4; w++) {
        dig[w] = h[w];
        dig[4 + w] = hp[w];
    }
}

// ---- POSLO (SHA-256) -------------------------------------------------------

// x_t: one compression of x_0[i] || LE32(j) || 0x00; xw gets the first four
// state words (the bytes of x_t are their big-endian encodings)
__device__ __forceinline__ void one_time_seed_sha(const BatchArgs& a, uint64_t pos, uint32_t xw[4]) {
    uint64_t t = a.t0 + pos;
    uint64_t ep = (t >> a.log2_n2) - a.epoch_first;
    uint32_t j = (uint32_t)(t & ((1ull << a.log2_n2) - 1));
    const uint32_t* e = a.tab + ep * kEpochWords + 44;
    uint32_t W[16] = {bswap32(e[0]), bswap32(e[1]), bswap32(e[2]), bswap32(e[3]),
                      bswap32(j), 0x00800000u, 0, 0, 0, 0, 0, 0, 0, 0, 0, 21u * 8u};
    uint32_t H[8];
    sha256_init(H);
    sha256_compress(H, W);
    xw[0] = H[0], xw[1] = H[1], xw[2] = H[2], xw[3] = H[3];
}

// big-endian word at byte offset o of m || x || 0x80 || 0.. || BE64(bits)
template <bool FAST>
__device__ __forceinline__ uint32_t sha_stream_word(const EntryView& v, const uint32_t xw[4], uint64_t o,
                                                    uint64_t total) {
    uint64_t L = v.L;
    if (FAST) {
        if (o < L) return bswap32(gload(reinterpret_cast<const uint32_t*>(v.m + o)));
        if (o < L + 16) return xw[(o - L) >> 2];
        if (o == L + 16) return 0x80000000u;
        if (o == total - 8) return (uint32_t)((L + 16) >> 29);
        if (o == total - 4) return (uint32_t)((L + 16) << 3);
        return 0;
    }
    uint32_t word = 0;
    for (int k = 0; k < 4; k++) {
        uint64_t p = o + k;
        uint32_t byte;
        if (p < L)
            byte = gload(v.m + p);
        else if (p < L + 16)
            byte = (xw[(p - L) >> 2] >> (8 * (3 - ((p - L) & 3)))) & 0xffu;
        else if (p == L + 16)
            byte = 0x80;
        else if (p >= total - 8)
            byte = (uint32_t)(((L + 16) * 8) >> (8 * (total - 1 - p))) & 0xffu;
        else
            byte = 0;
        word |= byte << (8 * (3 - k));
    }
    return word;
}

// SHA-256(m || x) as eight little-endian limbs of the digest bytes.  FAST:
// 4-byte aligned message, length divisible by 4; VEC additionally 16-byte
// aligned with a length divisible by 16, so whole 64-byte message blocks
// come in as four 16-byte loads.
template <bool FAST, bool VEC = false>
__device__ __forceinline__ void digest_sha(const EntryView& v, const uint32_t xw[4], uint32_t dig[8]) {
    uint64_t total = ((v.L + 16 + 9 + 63) / 64) * 64;
    uint32_t H[8];
    sha256_init(H);
    uint64_t off = 0;
    if (VEC) {
        // whole 128-byte lines: one load burst, two compressions
        const uint4* p = reinterpret_cast<const uint4*>(v.m);
        for (; off + 128 <= v.L; off += 128) {
            uint4 q[8];
#pragma unroll
            for (int k = 0; k < 8; k++) q[k] = gload(p + off / 16 + k);
#pragma unroll
            for (int half = 0; half < 2; half++) {
                uint32_t W[16];
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    W[4 * k] = bswap32(q[4 * half + k].x);
                    W[4 * k + 1] = bswap32(q[4 * half + k].y);
                    W[4 * k + 2] = bswap32(q[4 * half + k].z);
                    W[4 * k + 3] = bswap32(q[4 * half + k].w);
                }
                sha256_compress(H, W);
            }
        }
    }
    for (; off < total; off += 64) {
        uint32_t W[16];
#pragma unroll
        for (int w = 0; w < 16; w++) W[w] = sha_stream_word<FAST>(v, xw, off + 4 * w, total);
        sha256_compress(H, W);
    }
#pragma unroll
    for (int w = 0; w < 8; w++) dig[w] = bswap32(H[w]);
}

// ---- POSLO++ (Add_q) ------------------------------------------------------

// m_t (L <= 31 bytes) as eight little-endian words, zero past the message.
// LAYOUT 2: L = 16 at a 16-byte aligned address (one 16-byte load);
// 1: a multiple of 4 at a 4-byte aligned address; 0: anything, read as the
// aligned words that hold a message byte (never a word past them, so no load
// leaves the pages the message lies in) and funnel-shifted.
template <int LAYOUT>
__device__ __forceinline__ void addq_message(const uint8_t* m, uint32_t L, uint32_t w[8]) {
    if constexpr (LAYOUT == 2) {
        const uint4 v = gload(reinterpret_cast<const uint4*>(m));
        w[0] = v.x, w[1] = v.y, w[2] = v.z, w[3] = v.w;
#pragma unroll
        for (int k = 4; k < 8; k++) w[k] = 0u;
    } else if constexpr (LAYOUT == 1) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(m);
#pragma unroll
        for (int k = 0; k < 8; k++) w[k] = 4u * k < L ? gload(p + k) : 0u;
    } else {
        const uintptr_t A = reinterpret_cast<uintptr_t>(m);
        const uint32_t sh = (uint32_t)(A & 3u);
        const uint32_t* base = reinterpret_cast<const uint32_t*>(A - sh);
        const uint32_t nw = L ? (sh + L + 3u) >> 2 : 0u;
        uint32_t d[9];
#pragma unroll
        for (int k = 0; k < 9; k++) d[k] = (uint32_t)k < nw ? gload(base + k) : 0u;
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint32_t v = __builtin_amdgcn_alignbyte(d[k + 1], d[k], sh);
            const int r = (int)L - 4 * k;  // message bytes in word k
            w[k] = r >= 4 ? v : r <= 0 ? 0u : v & ((1u << (8 * r)) - 1u);
        }
    }
}

// Add_q(m, x) = LE(m) + LE(x) as eight words (below 2^249 < q for |m| <= 31)
__device__ __forceinline__ void addq_digest(const uint32_t w[8], const uint32_t x[4], uint32_t e[8]) {
    uint64_t c = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
        c += (uint64_t)w[k] + (k < 4 ? x[k] : 0u);
        e[k] = (uint32_t)c;
        c >>= 32;
    }
}

// ---- reductions ------------------------------------------------------------

// 288-bit sums across a wave (butterfly of nine-limb adds)
__device__ __forceinline__ void wave_reduce288(uint32_t acc[9]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t o[9];
#pragma unroll
        for (int k = 0; k < 9; k++) o[k] = __shfl_xor(acc[k], off);
        acc288_add(acc, o);
    }
}

// workgroup sum; thread 0 writes the nine limbs to out
template <int BLOCK>
__device__ __forceinline__ void block_reduce288_store(uint32_t acc[9], uint32_t* out) {
    __shared__ uint32_t red[BLOCK / 64][9];
    wave_reduce288(acc);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int k = 0; k < 9; k++) red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s[9];
        for (int k = 0; k < 9; k++) s[k] = red[0][k];
        for (int w = 1; w < BLOCK / 64; w++) acc288_add(s, red[w]);
        for (int k = 0; k < 9; k++) out[k] = s[k];
    }
}

// workgroup sum through a caller-provided LDS scratch (BLOCK/64 * 9 words);
// the caller synchronizes before the call if the scratch was in use
template <int BLOCK>
__device__ __forceinline__ void block_reduce288_scratch(uint32_t acc[9], uint32_t* out, uint32_t* scratch) {
    wave_reduce288(acc);
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int k = 0; k < 9; k++) scratch[wave * 9 + k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s[9];
        for (int k = 0; k < 9; k++) s[k] = scratch[k];
        for (int w = 1; w < BLOCK / 64; w++) acc288_add(s, scratch + w * 9);
        for (int k = 0; k < 9; k++) out[k] = s[k];
    }
}

}  // namespace poslo
