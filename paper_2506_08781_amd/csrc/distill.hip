// POSLO-F distillation and selective batch verification on gfx950.
//
// Paper: section "POSLO-C Distillation and Selective Batch Verification"
// (figure "Distillation and selective batch verification"), applied entry by
// entry as the "Fine-grained public-key POSLO" text prescribes: every entry is
// verified individually; valid entries are aggregated into the overall tag
// CCD^v and into umbrella tags CCD^u; invalid entries are kept with their
// signatures in CCD^i.  SeBVer checks CCD^v (mode V), each umbrella (mode U)
// or each invalid entry (mode I).
//
// Entry validity: x_t equals the re-derived PRF_0(x_0[i] || j), s_t < q, and
// encode(e_t*Y + s_t*G) equals the R_t bytes.
//
// Aggregates: for a valid entry R_t = e_t*Y + s_t*G exactly, so the sum of the
// valid R_t of a range equals (sum e_t)*Y + (sum s_t)*G.  The kernels
// therefore sum e_t and s_t lazily over valid entries (as AVer does) and do
// one double-scalar multiplication per umbrella instead of one point addition
// per entry; the result is the same group element, hence the same bytes.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ccd.h"
#include "ctx.h"
#include "device_ec.h"
#include "device_entry.h"
#include "device_fq.h"
#include "device_verify.h"
#include "scheme_host.h"

namespace poslo {

constexpr int kTile = 256;  // entries per tile of SeBVer's e-key sums (one workgroup)
constexpr uint64_t kWideKeyMinEntries = 1u << 18;  // Distill batches that use Y's wide table

// tiles of `len` entries never straddle an umbrella: umbrella l covers
// [l*span, min(n, (l+1)*span))
struct TileGeom {
    uint64_t n;
    uint64_t span;
    uint32_t tiles_per_umb;
    uint32_t len;
};

__device__ __forceinline__ bool tile_range(const TileGeom& g, uint32_t tile, uint64_t& start, uint64_t& end) {
    uint64_t l = tile / g.tiles_per_umb, k = tile % g.tiles_per_umb;
    uint64_t u0 = l * g.span, u1 = u0 + g.span < g.n ? u0 + g.span : g.n;
    start = u0 + k * g.len;
    end = start + g.len < u1 ? start + g.len : u1;
    return start < end;
}

struct VerifyArgs {
    BatchArgs a;
    TileGeom g;
    uint32_t inst;
    const uint8_t* sigs;   // 80 bytes per entry (tile mode) or per list item (list mode)
    const uint64_t* list;  // list mode: batch positions
    uint64_t list_n;
    const uint32_t* ty;
    const uint32_t* tg;    // G's wide table (the per-entry checks)
    uint8_t* flags;        // 1 = invalid, per batch position (tile mode) or list item
    uint32_t* tile_part;   // 18 words per tile: lazy sums of e_t and s_t over valid entries
    uint32_t* stash;       // tile mode: kVerifyStashWords per wave
    uint32_t* next;        // tile mode: tile queue head (zero at launch)
    uint32_t n_tiles;
};

// individual verification of the entry at batch position pos (device_verify.h)
__device__ __forceinline__ bool verify_entry(const LdsTables<4, 1>& tb, const VerifyArgs& v, uint64_t pos,
                                             const uint8_t* sg, uint32_t e[8], uint32_t s[8]) {
    return verify_one(tb, v.a, v.a.end, v.inst, pos, sg, v.ty, v.tg, e, s);
}

// Per entry, ahead of the curve checks: e_t mod q and whether x_t differs
// from the signature's (AES with the byte-addressed bank-private LDS tables
// of the AVer hot kernel, 1,024 threads per workgroup)
// AES: one 64 KB table per workgroup and x_t derived only for the final
// blocks, so two 1,024-thread workgroups fit per CU (eight waves per SIMD)
// POSLO++ (INST_AES_ADDQ): e_t = Add_q(m_t, x_t); a message longer than 31
// bytes is marked bad (its x check fails) and sets a.bad.  FQ: the group is
// FourQ, e_t is reduced mod N.
template <int INST, int BLOCK, int WPE, bool FQ = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void k_distill_hash(
    BatchArgs a, const uint8_t* sigs, uint32_t* ekeys, uint8_t* xbad) {
    constexpr bool AESP = INST != INST_SHA256;  // AES-based PRF
    constexpr int TW = AESP ? 2 * 256 * 32 : 1;
    __shared__ uint32_t lds[TW];
    if constexpr (AESP) perm_tables_fill<2, 32>(lds);
    __syncthreads();
    const PermTables<2, 32> tb = perm_tables<2, 32>(lds);
    for (uint64_t p = (uint64_t)blockIdx.x * BLOCK + threadIdx.x; p < a.n; p += (uint64_t)gridDim.x * BLOCK) {
        EntryView ev = entry_view(a, p);
        uint32_t x[4], dig[8];
        if constexpr (AESP) {
            const uint64_t t = a.t0 + p;
            const uint32_t jj = (uint32_t)(t & ((1ull << a.log2_n2) - 1));
            const uint32_t* rk = a.tab + ((t >> a.log2_n2) - a.epoch_first) * kEpochWords;
            auto xf = [&](uint32_t y[4]) {
                y[0] = jj, y[1] = 0, y[2] = 0, y[3] = 0;
                penc_rk(tb, rk, y);
                y[0] ^= jj;
                y[3] &= a.xmask;
            };
            if constexpr (INST == INST_AES_ADDQ) {
                if (ev.L > kAddqMaxLen) {
                    *a.bad = 1u;
#pragma unroll
                    for (int w = 0; w < 8; w++) ekeys[p * 8 + w] = 0xffffffffu;
                    xbad[p] = 1;
                    continue;
                }
                xf(x);
                uint32_t mw[8];
                addq_message<0>(ev.m, (uint32_t)ev.L, mw);
                addq_digest(mw, x, dig);
            } else {
                digest_mdc2_any_late(tb, ev, a.end, xf, x, dig, Mdc2BlockPerm{});
            }
        } else {
            one_time_seed_sha(a, p, x);
            digest_sha_any(ev, a.end, x, dig);
#pragma unroll
            for (int w = 0; w < 4; w++) x[w] = bswap32(x[w]);
        }
        const uint8_t* sx = sigs + p * 80 + 64;
        uint32_t d = 0;
#pragma unroll
        for (int w = 0; w < 4; w++) d |= x[w] ^ gload_le32(sx + 4 * w);
        uint32_t e[8];
        if constexpr (FQ)
            scN_reduce<8>(e, dig);
        else if constexpr (INST == INST_AES_ADDQ)
            for (int w = 0; w < 8; w++) e[w] = dig[w];
        else
            sc_reduce256(e, dig);
#pragma unroll
        for (int w = 0; w < 8; w++) ekeys[p * 8 + w] = e[w];
        xbad[p] = d ? 1 : 0;
    }
}

// the curve part of every entry's check, with e_t and the x check from
// k_distill_hash; valid entries' (e_t, s_t) go into the tile's partials.
// Persistent, one wave per workgroup pulling tiles from a queue; thread i
// checks entries i + 64 k of its tile (k < ceil(len / 64)) with one shared
// inversion, the points waiting in the wave's slice of the stash.  ty_wide:
// v.ty is Y's wide table (else its 8-bit one).  FQ: the group is FourQ
// (Y's 8-bit table and G's wide one, scalars mod N).
template <bool FQ>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_verify_tiles(
    VerifyArgs v, const uint32_t* ekeys, const uint8_t* xbad, uint32_t ty_wide) {
    uint32_t* st = v.stash + (uint64_t)blockIdx.x * kVerifyStashWords + threadIdx.x;
#pragma unroll 1
    for (;;) {
        uint32_t tile = threadIdx.x == 0 ? atomicAdd(v.next, 1u) : 0u;
        tile = (uint32_t)__shfl((int)tile, 0);
        if (tile >= v.n_tiles) break;
        uint64_t start, end;
        const bool any = tile_range(v.g, tile, start, end);
        const int ne = any ? (int)((end - start + 63) / 64) : 0;
        auto ent = [&](int k, const uint8_t*& sg, const uint32_t*& e, bool& go) {
            const uint64_t pos = start + threadIdx.x + 64 * (uint64_t)k;
            go = any && pos < end && !xbad[pos];
            // skipped entries point at entry 0 (read by nothing that matters)
            sg = v.sigs + (go ? 80 * pos : 0);
            e = ekeys + (go ? pos * 8 : 0);
        };
        uint32_t okmask;
        if constexpr (FQ)
            okmask = verify_sig_batch_fq(ent, ne, v.ty, v.tg, st, 64);
        else
            okmask = ty_wide ? verify_sig_batch<true>(ent, ne, v.ty, v.tg, st, 64)
                             : verify_sig_batch<false>(ent, ne, v.ty, v.tg, st, 64);
        uint32_t ae[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, as[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
        for (int k = 0; k < ne; k++) {
            const uint64_t pos = start + threadIdx.x + 64 * (uint64_t)k;
            if (pos >= end) continue;
            const bool ok = (okmask >> k) & 1u;
            v.flags[pos] = ok ? 0 : 1;
            if (ok) {
                uint32_t w8[8];
                for (int w = 0; w < 8; w++) w8[w] = gload(ekeys + pos * 8 + w);
                acc288_add256(ae, w8);
                for (int w = 0; w < 8; w++) w8[w] = gload_le32(v.sigs + 80 * pos + 4 * w);
                acc288_add256(as, w8);
            }
        }
        uint32_t* out = v.tile_part + (uint64_t)tile * 18;
        block_reduce288_store<64>(ae, out);
        __syncthreads();
        block_reduce288_store<64>(as, out + 9);
        __syncthreads();
    }
}

__global__ void k_zero_word(uint32_t* p) { p[0] = 0; }

// list mode (SeBVer I): flags[i] = 1 when list item i is invalid.  FQ: the
// group is FourQ (v.tg is G's wide FourQ table, scalars mod N).
template <bool FQ>
__global__ __launch_bounds__(kTile) void k_verify_list(VerifyArgs v) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
    LdsTables<4, 1> tb{lds};
    uint64_t i = (uint64_t)blockIdx.x * kTile + threadIdx.x;
    if (i >= v.list_n) return;
    const uint8_t* sg = v.sigs + 80 * i;
    bool ok;
    if constexpr (FQ) {
        uint32_t dig[8], e[8], sc[8], r[8];
        ok = entry_digest(tb, v.a, v.a.end, v.inst, v.list[i], sg, dig);
        if (ok) {
            scN_reduce<8>(e, dig);
            for (int k = 0; k < 8; k++) sc[k] = gload_le32(sg + 4 * k);
            ok = scN_is_canonical(sc);
        }
        if (ok) {
            gq P;
            lane_double_scalar_fq_wide(P, v.ty, v.tg, e, sc);
            fp2 zi;
            f2_inv(zi, P.Z);
            for (int k = 0; k < 8; k++) r[k] = gload_le32(sg + 32 + 4 * k);
            ok = fq_encodes_zinv(P, zi, r);
        }
    } else {
        uint32_t e[8], sc[8];
        ok = verify_entry(tb, v, v.list[i], sg, e, sc);
    }
    v.flags[i] = ok ? 0 : 1;
}

// per-tile lazy sums of e_t over non-skipped entries (SeBVer U)
__global__ __launch_bounds__(kTile) void k_ekeys_tiles(BatchArgs a, TileGeom g, uint32_t inst, uint32_t* tile_part) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
    LdsTables<4, 1> tb{lds};
    uint64_t start, end;
    bool any = tile_range(g, blockIdx.x, start, end);
    uint64_t pos = start + threadIdx.x;
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (any && pos < end && !skipped(a, pos)) {
        uint32_t x[4], dig[8];
        EntryView ev = entry_view(a, pos);
        if (inst_base(inst) == INST_AES_ADDQ) {
            if (ev.L > kAddqMaxLen) {
                *a.bad = 1u;
            } else {
                one_time_seed_aes(tb, a, pos, x);
                uint32_t mw[8];
                addq_message<0>(ev.m, (uint32_t)ev.L, mw);
                addq_digest(mw, x, dig);
                acc288_add256(acc, dig);
            }
        } else if (inst_base(inst) == INST_AES) {
            one_time_seed_aes(tb, a, pos, x);
            digest_mdc2_any(tb, ev, a.end, x, dig, Mdc2BlockGeneric{});
            acc288_add256(acc, dig);
        } else {
            one_time_seed_sha(a, pos, x);
            digest_sha_any(ev, a.end, x, dig);
            acc288_add256(acc, dig);
        }
    }
    block_reduce288_store<kTile>(acc, tile_part + (uint64_t)blockIdx.x * 18);
}

// Per umbrella: fold the tiles' partials, reduce mod q, then
//   mode 0 (Distill): tag = LE32B(s) || enc(e*Y + s*G), and e, s mod q kept
//   mode 1 (SeBVer U): bit = [host checks ok] and e*Y + s*G == R of the tag
struct FoldArgs {
    const uint32_t* tile_part;
    uint32_t tiles_per_umb;
    uint32_t mode;
    const uint32_t* ty;
    const uint32_t* tg;
    const uint32_t* chk;  // mode 1: per umbrella 25 words: s[8], x_R[8], y_R[8], ok
    uint32_t* umb_es;     // mode 0: per umbrella e mod q [8], s mod q [8]
    uint8_t* umb_tags;    // mode 0: 64 bytes per umbrella
    uint32_t* umb_bits;   // mode 1: accept per umbrella
    uint32_t n_umb;       // mode 0 with valid_tag: block n_umb computes CCD^v
    uint8_t* valid_tag;   // mode 0: CCD^v (64 bytes), or nullptr
};

// Block n_umb (mode 0, valid_tag set) folds every tile instead: CCD^v, the
// aggregate of all valid entries, computed beside the umbrellas rather than
// after them (each block's curve work is one wave's latency).  FQ: the group
// is FourQ (scalars mod N; chk holds x_R, y_R as GF(p^2) words).
template <bool FQ>
__device__ __forceinline__ void fold_reduce(uint32_t r[8], const uint32_t t[9]) {
    if constexpr (FQ)
        scN_reduce<9>(r, t);
    else
        sc_reduce288(r, t);
}

// the edwards25519 outputs of a fold given the sum P = e*Y + s*G (any
// projective scaling): the tags (mode 0, CCD^v) or the umbrella's verdict
__device__ __forceinline__ void fold_point(const FoldArgs& f, uint32_t l, bool valid_block, const uint32_t e[8],
                                           const uint32_t s[8], const ge& P) {
    if (valid_block) {
        for (int k = 0; k < 8; k++) store_le32(f.valid_tag + 4 * k, s[k]);
        ge_encode(f.valid_tag + 32, P);
    } else if (f.mode == 0) {
        uint8_t* tag = f.umb_tags + (uint64_t)l * 64;
        for (int k = 0; k < 8; k++) {
            store_le32(tag + 4 * k, s[k]);
            f.umb_es[l * 16 + k] = e[k];
            f.umb_es[l * 16 + 8 + k] = s[k];
        }
        ge_encode(tag + 32, P);
    } else {
        const uint32_t* c = f.chk + l * 25;
        fe rx, ry, t0, t1;
        for (int k = 0; k < 8; k++) {
            rx.v[k] = c[8 + k];
            ry.v[k] = c[16 + k];
        }
        fe_mul(t0, rx, P.Z);
        fe_mul(t1, ry, P.Z);
        f.umb_bits[l] = (c[24] && fe_equal(t0, P.X) && fe_equal(t1, P.Y)) ? 1u : 0u;
    }
}

template <bool FQ>
__device__ __forceinline__ void fold_curve(const FoldArgs& f, uint32_t l, bool valid_block, const uint32_t e[8],
                                           const uint32_t s[8]) {
    if constexpr (FQ) {
        gq P;
        wave_double_scalar_fq(P, f.ty, f.tg, e, s);
        if (threadIdx.x != 0) return;
        if (valid_block) {
            for (int k = 0; k < 8; k++) store_le32(f.valid_tag + 4 * k, s[k]);
            fq_encode(f.valid_tag + 32, P);
        } else if (f.mode == 0) {
            uint8_t* tag = f.umb_tags + (uint64_t)l * 64;
            for (int k = 0; k < 8; k++) {
                store_le32(tag + 4 * k, s[k]);
                f.umb_es[l * 16 + k] = e[k];
                f.umb_es[l * 16 + 8 + k] = s[k];
            }
            fq_encode(tag + 32, P);
        } else {
            const uint32_t* c = f.chk + l * 25;
            fp2 rx, ry, t0, t1;
            for (int k = 0; k < 4; k++) {
                rx.a.v[k] = c[8 + k];
                rx.b.v[k] = c[12 + k];
                ry.a.v[k] = c[16 + k];
                ry.b.v[k] = c[20 + k];
            }
            f2_mul(t0, rx, P.Z);
            f2_mul(t1, ry, P.Z);
            f.umb_bits[l] = (c[24] && f2_eq(t0, P.X) && f2_eq(t1, P.Y)) ? 1u : 0u;
        }
    } else {
        ge P;
        wave_double_scalar(P, f.ty, f.tg, e, s);
        if (threadIdx.x != 0) return;
        fold_point(f, l, valid_block, e, s, P);
    }
}

template <bool FQ>
__global__ __launch_bounds__(kTile) void k_umbrella_fold(FoldArgs f) {
    __shared__ uint32_t tot_e[9], tot_s[9];
    __shared__ uint32_t sh[16];
    const uint32_t l = blockIdx.x;
    const bool valid_block = f.valid_tag && l == f.n_umb;
    uint32_t ae[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, as[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const uint64_t first = valid_block ? 0 : (uint64_t)l * f.tiles_per_umb;
    const uint64_t count = valid_block ? (uint64_t)f.n_umb * f.tiles_per_umb : f.tiles_per_umb;
    for (uint64_t k = threadIdx.x; k < count; k += kTile) {
        const uint32_t* tp = f.tile_part + (first + k) * 18;
        acc288_add(ae, tp);
        acc288_add(as, tp + 9);
    }
    block_reduce288_store<kTile>(ae, tot_e);
    __syncthreads();
    block_reduce288_store<kTile>(as, tot_s);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t e[8], s[8];
        fold_reduce<FQ>(e, tot_e);
        if (f.mode == 0) {
            fold_reduce<FQ>(s, tot_s);
        } else {
            for (int k = 0; k < 8; k++) s[k] = f.chk[l * 25 + k];
        }
        for (int k = 0; k < 8; k++) {
            sh[k] = e[k];
            sh[8 + k] = s[k];
        }
    }
    __syncthreads();
    uint32_t e[8], s[8];
    for (int k = 0; k < 8; k++) {
        e[k] = sh[k];
        s[k] = sh[8 + k];
    }
    if constexpr (FQ) {
        if (threadIdx.x < 64) fold_curve<FQ>(f, l, valid_block, e, s);
    } else {
        // the quad-split block sum (device_ec.h), every thread of the block
        static_assert(kTile == kQuadBlock, "the block sum takes the whole block");
        __shared__ uint32_t pts[kQuadLdsWords];
        uint32_t sr[8];
        sc_reduce256(sr, s);  // mode 1 may carry an s >= q (its check then fails on the host flag)
        block_double_scalar(pts, f.ty, f.tg, e, sr);
        if (threadIdx.x == 0) {
            ge P;
            lds_load_fe(P.X, pts);
            lds_load_fe(P.Y, pts + 8);
            lds_load_fe(P.Z, pts + 16);
            lds_load_fe(P.T, pts + 24);
            fold_point(f, l, valid_block, e, s, P);
        }
    }
}

// CCD^v: fold the umbrellas' (e, s) mod q (FQ: mod N) and encode e*Y + s*G
template <bool FQ>
__global__ __launch_bounds__(kTile) void k_valid_fold(const uint32_t* umb_es, uint32_t n_umb, const uint32_t* ty,
                                                      const uint32_t* tg, uint8_t* tag) {
    __shared__ uint32_t tot_e[9], tot_s[9];
    __shared__ uint32_t sh[16];
    uint32_t ae[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, as[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t l = threadIdx.x; l < n_umb; l += kTile) {
        acc288_add256(ae, umb_es + l * 16);
        acc288_add256(as, umb_es + l * 16 + 8);
    }
    block_reduce288_store<kTile>(ae, tot_e);
    __syncthreads();
    block_reduce288_store<kTile>(as, tot_s);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t e[8], s[8];
        fold_reduce<FQ>(e, tot_e);
        fold_reduce<FQ>(s, tot_s);
        for (int k = 0; k < 8; k++) {
            sh[k] = e[k];
            sh[8 + k] = s[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        uint32_t e[8], s[8];
        for (int k = 0; k < 8; k++) {
            e[k] = sh[k];
            s[k] = sh[8 + k];
        }
        FoldArgs f{};
        f.ty = ty;
        f.tg = tg;
        f.valid_tag = tag;
        fold_curve<FQ>(f, 0, true, e, s);
    }
}

// sorted list of invalid entries, in two passes over blocks of 4,096 flags:
// per-block counts, then each block adds the counts of the blocks before it,
// scans its threads' counts in LDS and writes its entries in order.  out_idx
// gets t0 + pos.
constexpr int kCmpThreads = 256, kCmpPer = 16, kCmpBlock = kCmpThreads * kCmpPer;

__device__ __forceinline__ uint32_t flags_of_thread(const uint8_t* flags, uint64_t n, uint64_t base) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kCmpPer; k++)
        if (base + k < n) c += flags[base + k];
    return c;
}

__global__ __launch_bounds__(kCmpThreads) void k_flag_count(const uint8_t* flags, uint64_t n, uint32_t* blk) {
    __shared__ uint32_t red[kCmpThreads / 64];
    uint64_t base = (uint64_t)blockIdx.x * kCmpBlock + (uint64_t)threadIdx.x * kCmpPer;
    uint32_t c = flags_of_thread(flags, n, base);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kCmpThreads / 64; w++) t += red[w];
        blk[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kCmpThreads) void k_flag_scatter(const uint8_t* flags, uint64_t n, uint64_t t0,
                                                              const uint32_t* blk, uint64_t* out_idx,
                                                              uint64_t* out_count) {
    __shared__ uint64_t red[kCmpThreads / 64];
    __shared__ uint32_t scan[kCmpThreads];
    // entries flagged in the blocks before this one
    uint64_t before = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kCmpThreads) before += blk[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) before += __shfl_xor(before, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = before;
    uint64_t base = (uint64_t)blockIdx.x * kCmpBlock + (uint64_t)threadIdx.x * kCmpPer;
    uint32_t c = flags_of_thread(flags, n, base);
    scan[threadIdx.x] = c;
    __syncthreads();
    uint64_t pre = 0;
    for (int w = 0; w < kCmpThreads / 64; w++) pre += red[w];
    // inclusive scan of the threads' counts
    for (int off = 1; off < kCmpThreads; off <<= 1) {
        uint32_t v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t o = pre + scan[threadIdx.x] - c;
    for (int k = 0; k < kCmpPer; k++)
        if (base + k < n && flags[base + k]) out_idx[o++] = t0 + base + k;
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kCmpThreads - 1) *out_count = pre + scan[kCmpThreads - 1];
}

__global__ void k_gather_sigs(const uint64_t* idx, uint64_t count, uint64_t t0, const uint8_t* sigs, uint8_t* out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count * 20) return;
    uint64_t k = i / 20, w = i % 20;
    const uint8_t* src = sigs + (idx[k] - t0) * 80 + 4 * w;
    uint8_t* dst = out + k * 80 + 4 * w;
    for (int b = 0; b < 4; b++) dst[b] = src[b];
}

}  // namespace poslo

// ===========================================================================
// host side
// ===========================================================================

using namespace poslo;

namespace {

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

int scratch(poslo_ctx* c, int slot, size_t bytes, void** out) { return ctx_scratch(c, slot, bytes, out); }

enum { S_FLAGS = 0, S_TILES, S_UMB_ES, S_UMB_TAGS, S_IDX, S_MISC, S_SIGS, S_AUX, S_EK = 16, S_XB, S_STASH };

int checked_sigs(const uint8_t* sigs, uint64_t n) {
    if (n && !sigs) return POSLO_E_INVAL;
    if ((uintptr_t)sigs % 4) return POSLO_E_INVAL;
    return POSLO_OK;
}

}  // namespace

extern "C" int poslo_distill(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m_in,
                             const uint8_t* sigs_in, const uint8_t* ds, size_t ds_len, uint32_t n_umbrella,
                             void* stream, poslo_ccd** out) {
    if (!out || !pk || !m_in || n_umbrella == 0) return POSLO_E_INVAL;
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (m_in->n && !sigs_in) return POSLO_E_INVAL;
    poslo_msgs dm;
    const uint8_t* sigs;
    int st = stage_msgs(c, m_in, s, dm, sigs_in, &sigs);
    if (st) return st;
    const poslo_msgs* m = &dm;
    BatchArgs a;
    DsArg dsa;
    uint32_t n_epochs;
    if ((st = prepare_batch(c, prm, m, ds, ds_len, a, dsa, n_epochs))) return st;
    if ((st = checked_sigs(sigs, m->n))) return st;
    HIP_TRY(hipSetDevice(c->device));
    const bool fq = (prm->inst & POSLO_GROUP_FOURQ) != 0;
    const KeyEntry* key = ctx_key_of(c, prm->inst, pk, &st);
    if (!key) return st;
    const uint32_t* gtab = fq ? ctx_gtable_fq(c) : c->d_gtable;
    if (!gtab) return POSLO_E_NOMEM;

    poslo_ccd* ccd = new (std::nothrow) poslo_ccd();
    if (!ccd) return POSLO_E_NOMEM;
    ccd->inst = prm->inst;
    ccd->log2_n1 = prm->log2_n1;
    ccd->log2_n2 = prm->log2_n2;
    ccd->t0 = m->t0;
    ccd->n = m->n;
    ccd->ds.assign(ds, ds + ds_len);
    uint64_t n = m->n;
    uint64_t span = std::max<uint64_t>(1, (n + n_umbrella - 1) / n_umbrella);
    uint64_t n_umb = n ? (n + span - 1) / span : 0;
    ccd->span = span;

    void *flags, *tiles, *umb_es, *umb_tags, *idx, *misc, *gsigs;
    const uint32_t vlen = verify_tile_len(n, c->num_cu);
    uint32_t tpu = (uint32_t)((span + vlen - 1) / vlen);
    uint64_t n_tiles = n_umb * tpu;
    if (n_tiles > 0x7fffffffull) {
        delete ccd;
        return POSLO_E_INVAL;
    }
    if ((st = scratch(c, S_FLAGS, std::max<uint64_t>(n, 1), &flags)) ||
        (st = scratch(c, S_TILES, std::max<uint64_t>(n_tiles, 1) * 72, &tiles)) ||
        (st = scratch(c, S_UMB_ES, std::max<uint64_t>(n_umb, 1) * 64, &umb_es)) ||
        (st = scratch(c, S_UMB_TAGS, std::max<uint64_t>(n_umb, 1) * 64, &umb_tags)) ||
        (st = scratch(c, S_IDX, std::max<uint64_t>(n, 1) * 8, &idx)) || (st = scratch(c, S_MISC, 256 + 4 * ((n + kCmpBlock - 1) / kCmpBlock), &misc))) {
        delete ccd;
        return st;
    }
    uint8_t* d_valid_tag = (uint8_t*)misc;
    uint64_t* d_count = (uint64_t*)((uint8_t*)misc + 128);
    auto fail = [&](int code) {
        delete ccd;
        return code;
    };
    if (n) {
        prof_begin(c, POSLO_KT_SEED, s);
        if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return fail(st);
        prof_end(c, POSLO_KT_SEED, s);
        // edwards25519: G's wide table, and Y's wide table if the key has a
        // resident one, else built for large batches (once per key, about
        // 0.3 ms) and kept in a small LRU set.  FourQ: the 8-bit tables.
        const uint32_t* gw = fq ? ctx_gtable_wide_fq(c) : ctx_gtable_wide(c);
        if (!gw) return fail(POSLO_E_NOMEM);
        const uint32_t* yw =
            fq ? nullptr : n >= kWideKeyMinEntries ? ctx_key_wide(c, pk) : ctx_key_wide_resident(c, pk);
        VerifyArgs v;
        v.a = a;
        v.g = TileGeom{n, span, tpu, vlen};
        v.inst = prm->inst;
        v.sigs = sigs;
        v.list = nullptr;
        v.list_n = 0;
        v.ty = yw ? yw : key->d_table;
        v.tg = gw;
        v.flags = (uint8_t*)flags;
        v.tile_part = (uint32_t*)tiles;
        const uint32_t vgrid = (uint32_t)std::min<uint64_t>(n_tiles, (uint64_t)c->num_cu * kVerifyWgPerCu);
        v.next = (uint32_t*)((uint8_t*)misc + 192);
        v.n_tiles = (uint32_t)n_tiles;
        prof_begin(c, POSLO_KT_VERIFY, s);
        void *ek, *xb, *stash;
        if ((st = scratch(c, S_EK, n * 32, &ek)) || (st = scratch(c, S_XB, n, &xb)) ||
            (st = scratch(c, S_STASH, (size_t)vgrid * kVerifyStashWords * 4, &stash)))
            return fail(st);
        v.stash = (uint32_t*)stash;
        hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(1), 0, s, v.next);
        if (inst_base(prm->inst) == INST_AES_ADDQ)
            hipLaunchKernelGGL((k_distill_hash<INST_AES_ADDQ, 1024, 8>), dim3(c->num_cu * 2), dim3(1024), 0, s, v.a,
                               sigs, (uint32_t*)ek, (uint8_t*)xb);
        else if (inst_base(prm->inst) == INST_AES && fq)
            hipLaunchKernelGGL((k_distill_hash<INST_AES, 1024, 8, true>), dim3(c->num_cu * 2), dim3(1024), 0, s, v.a,
                               sigs, (uint32_t*)ek, (uint8_t*)xb);
        else if (inst_base(prm->inst) == INST_AES)
            hipLaunchKernelGGL((k_distill_hash<INST_AES, 1024, 8>), dim3(c->num_cu * 2), dim3(1024), 0, s, v.a, sigs,
                               (uint32_t*)ek, (uint8_t*)xb);
        else if (fq)
            hipLaunchKernelGGL((k_distill_hash<INST_SHA256, 256, 4, true>), dim3(c->num_cu * 4), dim3(256), 0, s,
                               v.a, sigs, (uint32_t*)ek, (uint8_t*)xb);
        else
            hipLaunchKernelGGL((k_distill_hash<INST_SHA256, 256, 4>), dim3(c->num_cu * 4), dim3(256), 0, s, v.a,
                               sigs, (uint32_t*)ek, (uint8_t*)xb);
        if (fq)
            hipLaunchKernelGGL(k_verify_tiles<true>, dim3(vgrid), dim3(64), 0, s, v, (const uint32_t*)ek,
                               (const uint8_t*)xb, 0u);
        else
            hipLaunchKernelGGL(k_verify_tiles<false>, dim3(vgrid), dim3(64), 0, s, v, (const uint32_t*)ek,
                               (const uint8_t*)xb, yw ? 1u : 0u);
        if (hipGetLastError() != hipSuccess) return fail(POSLO_E_DEVICE);
        prof_end(c, POSLO_KT_VERIFY, s);
        FoldArgs f;
        f.tile_part = (uint32_t*)tiles;
        f.tiles_per_umb = tpu;
        f.mode = 0;
        f.ty = key->d_table;
        f.tg = gtab;
        f.chk = nullptr;
        f.umb_es = (uint32_t*)umb_es;
        f.umb_tags = (uint8_t*)umb_tags;
        f.umb_bits = nullptr;
        f.n_umb = (uint32_t)n_umb;
        f.valid_tag = d_valid_tag;
        prof_begin(c, POSLO_KT_COMPACT, s);
        if (fq)
            hipLaunchKernelGGL(k_umbrella_fold<true>, dim3((uint32_t)n_umb + 1), dim3(kTile), 0, s, f);
        else
            hipLaunchKernelGGL(k_umbrella_fold<false>, dim3((uint32_t)n_umb + 1), dim3(kTile), 0, s, f);
        const uint32_t nblk = (uint32_t)((n + kCmpBlock - 1) / kCmpBlock);
        uint32_t* blk = (uint32_t*)((uint8_t*)misc + 256);  // per-block counts after the tag and count
        hipLaunchKernelGGL(k_flag_count, dim3(nblk), dim3(kCmpThreads), 0, s, (const uint8_t*)flags, n, blk);
        hipLaunchKernelGGL(k_flag_scatter, dim3(nblk), dim3(kCmpThreads), 0, s, (const uint8_t*)flags, n, m->t0,
                           (const uint32_t*)blk, (uint64_t*)idx, d_count);
        if (hipGetLastError() != hipSuccess) return fail(POSLO_E_DEVICE);
    } else {
        prof_begin(c, POSLO_KT_COMPACT, s);
        if (fq)
            hipLaunchKernelGGL(k_valid_fold<true>, dim3(1), dim3(kTile), 0, s, (const uint32_t*)umb_es,
                               (uint32_t)n_umb, key->d_table, gtab, d_valid_tag);
        else
            hipLaunchKernelGGL(k_valid_fold<false>, dim3(1), dim3(kTile), 0, s, (const uint32_t*)umb_es,
                               (uint32_t)n_umb, key->d_table, gtab, d_valid_tag);
    }
    if (hipGetLastError() != hipSuccess) return fail(POSLO_E_DEVICE);
    prof_end(c, POSLO_KT_COMPACT, s);
    uint64_t count = 0;
    uint32_t bad = 0;  // POSLO++: a message longer than 31 bytes
    if ((n && hipMemcpyAsync(&count, d_count, 8, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        (n && hipMemcpyAsync(&bad, a.bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipMemcpyAsync(ccd->valid_tag, d_valid_tag, 64, hipMemcpyDeviceToHost, s) != hipSuccess)
        return fail(POSLO_E_DEVICE);
    ccd->umb_tags.resize(n_umb * 64);
    if (n_umb && hipMemcpyAsync(ccd->umb_tags.data(), umb_tags, n_umb * 64, hipMemcpyDeviceToHost, s) != hipSuccess)
        return fail(POSLO_E_DEVICE);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(POSLO_E_DEVICE);
    prof_collect(c);
    if (bad) return fail(POSLO_E_INVAL);
    ccd->invalid.resize(count);
    ccd->invalid_sigs.resize(count * 80);
    if (count) {
        if ((st = scratch(c, S_SIGS, count * 80, &gsigs))) return fail(st);
        uint64_t threads = count * 20;
        hipLaunchKernelGGL(k_gather_sigs, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s,
                           (const uint64_t*)idx, count, m->t0, sigs, (uint8_t*)gsigs);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(ccd->invalid.data(), idx, count * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(ccd->invalid_sigs.data(), gsigs, count * 80, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(POSLO_E_DEVICE);
    }
    *out = ccd;
    return POSLO_OK;
}

extern "C" void poslo_ccd_free(poslo_ccd* ccd) { delete ccd; }

extern "C" int poslo_ccd_invalid(const poslo_ccd* ccd, const uint64_t** idx, uint64_t* n) {
    if (!ccd || !idx || !n) return POSLO_E_INVAL;
    *idx = ccd->invalid.data();
    *n = ccd->invalid.size();
    return POSLO_OK;
}

extern "C" int poslo_ccd_invalid_sig(const poslo_ccd* ccd, uint64_t k, uint8_t sig[80]) {
    if (!ccd || !sig || k >= ccd->invalid.size()) return POSLO_E_INVAL;
    memcpy(sig, ccd->invalid_sigs.data() + 80 * k, 80);
    return POSLO_OK;
}

extern "C" int poslo_ccd_valid_tag(const poslo_ccd* ccd, uint8_t tag[64]) {
    if (!ccd || !tag) return POSLO_E_INVAL;
    memcpy(tag, ccd->valid_tag, 64);
    return POSLO_OK;
}

extern "C" int poslo_ccd_umbrellas(const poslo_ccd* ccd, uint8_t* tags, size_t cap, uint64_t* n_umb, uint64_t* span) {
    if (!ccd) return POSLO_E_INVAL;
    uint64_t k = ccd->umb_tags.size() / 64;
    if (n_umb) *n_umb = k;
    if (span) *span = ccd->span;
    if (tags) {
        if (cap < ccd->umb_tags.size()) return POSLO_E_INVAL;
        memcpy(tags, ccd->umb_tags.data(), ccd->umb_tags.size());
    }
    return POSLO_OK;
}

// Serialized CCD (for cold storage): magic "PCCD", u32 version 1, u32 inst,
// log2_n1, log2_n2, u64 t0, n, span, u32 ds_len, ds, valid tag (64), u64
// n_umb, tags (64 each), u64 n_inv, per invalid entry u64 t and sigma (80).
namespace {
void put32(std::vector<uint8_t>& o, uint32_t v) {
    uint8_t b[4];
    store_le32(b, v);
    o.insert(o.end(), b, b + 4);
}
void put64(std::vector<uint8_t>& o, uint64_t v) {
    put32(o, (uint32_t)v);
    put32(o, (uint32_t)(v >> 32));
}
struct Reader {
    const uint8_t* p;
    size_t left;
    bool ok = true;
    uint32_t u32() {
        if (left < 4) {
            ok = false;
            return 0;
        }
        uint32_t v = load_le32(p);
        p += 4;
        left -= 4;
        return v;
    }
    uint64_t u64() {
        uint64_t lo = u32();
        return lo | ((uint64_t)u32() << 32);
    }
    bool bytes(uint8_t* dst, size_t n) {
        if (left < n) return ok = false;
        memcpy(dst, p, n);
        p += n;
        left -= n;
        return true;
    }
};
}  // namespace

extern "C" int poslo_ccd_export(const poslo_ccd* ccd, uint8_t* buf, size_t cap, size_t* len) {
    if (!ccd || !len) return POSLO_E_INVAL;
    std::vector<uint8_t> o;
    o.insert(o.end(), {'P', 'C', 'C', 'D'});
    // version 1: POSLO-F; version 2: POSLO-C, with a granularity word
    put32(o, ccd->coarse ? 2 : 1);
    put32(o, ccd->inst);
    put32(o, ccd->log2_n1);
    put32(o, ccd->log2_n2);
    if (ccd->coarse) put32(o, 1);
    put64(o, ccd->t0);
    put64(o, ccd->n);
    put64(o, ccd->span);
    put32(o, (uint32_t)ccd->ds.size());
    o.insert(o.end(), ccd->ds.begin(), ccd->ds.end());
    o.insert(o.end(), ccd->valid_tag, ccd->valid_tag + 64);
    put64(o, ccd->umb_tags.size() / 64);
    o.insert(o.end(), ccd->umb_tags.begin(), ccd->umb_tags.end());
    put64(o, ccd->invalid.size());
    for (size_t k = 0; k < ccd->invalid.size(); k++) {
        put64(o, ccd->invalid[k]);
        o.insert(o.end(), ccd->invalid_sigs.begin() + 80 * k, ccd->invalid_sigs.begin() + 80 * (k + 1));
    }
    *len = o.size();
    if (!buf || cap < o.size()) return POSLO_E_INVAL;
    memcpy(buf, o.data(), o.size());
    return POSLO_OK;
}

extern "C" int poslo_ccd_import(const uint8_t* buf, size_t len, poslo_ccd** out) {
    if (!buf || !out) return POSLO_E_INVAL;
    *out = nullptr;
    Reader r{buf, len};
    uint8_t magic[4];
    if (!r.bytes(magic, 4) || memcmp(magic, "PCCD", 4) != 0) return POSLO_E_INVAL;
    const uint32_t version = r.u32();
    if (version != 1 && version != 2) return POSLO_E_INVAL;
    poslo_ccd* c = new (std::nothrow) poslo_ccd();
    if (!c) return POSLO_E_NOMEM;
    c->inst = r.u32();
    c->log2_n1 = r.u32();
    c->log2_n2 = r.u32();
    if (version == 2 && r.u32() != 1) r.ok = false;
    c->coarse = version == 2 ? 1 : 0;
    c->t0 = r.u64();
    c->n = r.u64();
    c->span = r.u64();
    uint32_t dl = r.u32();
    if (!r.ok || dl > 1 + 24 * 32) {
        delete c;
        return POSLO_E_INVAL;
    }
    c->ds.resize(dl);
    r.bytes(c->ds.data(), dl);
    r.bytes(c->valid_tag, 64);
    uint64_t nu = r.u64();
    if (!r.ok || nu > r.left / 64) {
        delete c;
        return POSLO_E_INVAL;
    }
    c->umb_tags.resize(nu * 64);
    r.bytes(c->umb_tags.data(), nu * 64);
    uint64_t ni = r.u64();
    if (!r.ok || ni > r.left / 88) {
        delete c;
        return POSLO_E_INVAL;
    }
    c->invalid.resize(ni);
    c->invalid_sigs.resize(ni * 80);
    for (uint64_t k = 0; k < ni; k++) {
        c->invalid[k] = r.u64();
        r.bytes(c->invalid_sigs.data() + 80 * k, 80);
    }
    if (!r.ok || r.left != 0) {
        delete c;
        return POSLO_E_INVAL;
    }
    *out = c;
    return POSLO_OK;
}

// skip bitmap of the CCD's invalid entries over batch positions (device);
// a coarse CCD's invalid epochs cover all their entries
static int upload_skip(poslo_ctx* c, const poslo_ccd* ccd, hipStream_t s, const uint32_t** out) {
    uint64_t words = (ccd->n + 31) / 32;
    std::vector<uint32_t> bm(std::max<uint64_t>(words, 1), 0);
    for (uint64_t t : ccd->invalid) {
        // items outside the batch make the CCD malformed
        const uint64_t unit = ccd->coarse ? ccd->log2_n2 : 0;
        if (t < (ccd->t0 >> unit) || t - (ccd->t0 >> unit) >= (ccd->n >> unit)) return POSLO_E_INVAL;
        const uint64_t first = t << unit, count = 1ull << unit;
        for (uint64_t p = first - ccd->t0; p < first - ccd->t0 + count; p++) bm[p >> 5] |= 1u << (p & 31);
    }
    void* d;
    int st = scratch(c, S_AUX, bm.size() * 4, &d);
    if (st) return st;
    if (hipMemcpyAsync(d, bm.data(), bm.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return POSLO_E_DEVICE;
    *out = (const uint32_t*)d;
    return POSLO_OK;
}

namespace poslo {
int aver_impl(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m, const uint8_t* ds,
              size_t ds_len, const uint8_t tag[64], void* stream, const uint32_t* skip, int* accept,
              uint8_t e_out[32]);
int sebver_impl(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m,
                const poslo_ccd* ccd, char mode, uint8_t* bits, size_t cap, size_t* n_bits, void* stream);
}

extern "C" int poslo_sebver(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m,
                            const poslo_ccd* ccd, char mode, uint8_t* bits, size_t cap, size_t* n_bits, void* stream) {
    if (!ccd || ccd->coarse) return POSLO_E_INVAL;
    return sebver_impl(c, prm, pk, m, ccd, mode, bits, cap, n_bits, stream);
}

// SeBVer over a CCD; a coarse (POSLO-C) CCD takes modes V and U only, with
// its invalid epochs left out entry by entry and umbrellas of span epochs
int poslo::sebver_impl(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m_in,
                       const poslo_ccd* ccd, char mode, uint8_t* bits, size_t cap, size_t* n_bits, void* stream) {
    if (!c || !prm || !pk || !m_in || !ccd || !n_bits) return POSLO_E_INVAL;
    const bool fq = (prm->inst & POSLO_GROUP_FOURQ) != 0;
    poslo_msgs dm;
    int st0 = stage_msgs(c, m_in, (hipStream_t)stream, dm, nullptr, nullptr);
    if (st0) return st0;
    const poslo_msgs* m = &dm;
    if (m->t0 != ccd->t0 || m->n != ccd->n || prm->inst != ccd->inst || prm->log2_n2 != ccd->log2_n2 ||
        prm->log2_n1 != ccd->log2_n1)
        return POSLO_E_INVAL;
    if (ccd->coarse && mode != 'V' && mode != 'U') return POSLO_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    int st;
    if (mode == 'V') {
        *n_bits = 1;
        if (!bits || cap < 1) return POSLO_E_INVAL;
        const uint32_t* skip = nullptr;
        if (!ccd->invalid.empty() && (st = upload_skip(c, ccd, s, &skip))) return st;
        int acc = 0;
        st = aver_impl(c, prm, pk, m, ccd->ds.data(), ccd->ds.size(), ccd->valid_tag, stream, skip, &acc, nullptr);
        if (st) return st;
        bits[0] = (uint8_t)acc;
        return POSLO_OK;
    }
    BatchArgs a;
    DsArg dsa;
    uint32_t n_epochs;
    if ((st = prepare_batch(c, prm, m, ccd->ds.data(), ccd->ds.size(), a, dsa, n_epochs))) return st;
    const KeyEntry* key = ctx_key_of(c, prm->inst, pk, &st);
    if (!key) return st;
    const uint32_t* gtab = fq ? ctx_gtable_fq(c) : c->d_gtable;
    if (!gtab) return POSLO_E_NOMEM;
    if (mode == 'U') {
        uint64_t n_umb = ccd->umb_tags.size() / 64;
        *n_bits = n_umb;
        if (!bits || cap < n_umb) return POSLO_E_INVAL;
        if (n_umb == 0) return POSLO_OK;
        uint64_t span = ccd->coarse ? ccd->span << ccd->log2_n2 : ccd->span;
        if (span == 0 || (m->n + span - 1) / span != n_umb) return POSLO_E_INVAL;
        const uint32_t* skip = nullptr;
        if (!ccd->invalid.empty() && (st = upload_skip(c, ccd, s, &skip))) return st;
        a.skip = skip;
        uint32_t tpu = (uint32_t)((span + kTile - 1) / kTile);
        uint64_t n_tiles = n_umb * tpu;
        // host checks of each umbrella tag: s below the group order and R
        // decodes (its affine x and y go to the device)
        std::vector<uint32_t> chk(n_umb * 25);
        for (uint64_t l = 0; l < n_umb; l++) {
            const uint8_t* tg = ccd->umb_tags.data() + 64 * l;
            uint32_t* ck = &chk[l * 25];
            for (int k = 0; k < 8; k++) ck[k] = load_le32(tg + 4 * k);
            bool ok;
            if (fq) {
                gq R;
                ok = scN_is_canonical(ck) && fq_decode(R, tg + 32);
                for (int k = 0; k < 4; k++) {
                    ck[8 + k] = ok ? R.X.a.v[k] : 0;
                    ck[12 + k] = ok ? R.X.b.v[k] : 0;
                    ck[16 + k] = ok ? R.Y.a.v[k] : 0;
                    ck[20 + k] = ok ? R.Y.b.v[k] : 0;
                }
            } else {
                ge R;
                ok = sc_is_canonical(ck) && ge_decode(R, tg + 32);
                for (int k = 0; k < 8; k++) {
                    ck[8 + k] = ok ? R.X.v[k] : 0;
                    ck[16 + k] = ok ? R.Y.v[k] : 0;
                }
            }
            ck[24] = ok ? 1 : 0;
        }
        void *tiles, *dchk, *dbits;
        if ((st = scratch(c, S_TILES, n_tiles * 72, &tiles)) || (st = scratch(c, S_UMB_ES, chk.size() * 4, &dchk)) ||
            (st = scratch(c, S_UMB_TAGS, n_umb * 4, &dbits)))
            return st;
        HIP_TRY(hipMemcpyAsync(dchk, chk.data(), chk.size() * 4, hipMemcpyHostToDevice, s));
        if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return st;
        hipLaunchKernelGGL(k_ekeys_tiles, dim3((uint32_t)n_tiles), dim3(kTile), 0, s, a, TileGeom{m->n, span, tpu, (uint32_t)kTile},
                           prm->inst, (uint32_t*)tiles);
        FoldArgs f;
        f.tile_part = (uint32_t*)tiles;
        f.tiles_per_umb = tpu;
        f.mode = 1;
        f.ty = key->d_table;
        f.tg = gtab;
        f.chk = (const uint32_t*)dchk;
        f.umb_es = nullptr;
        f.umb_tags = nullptr;
        f.umb_bits = (uint32_t*)dbits;
        f.n_umb = (uint32_t)n_umb;
        f.valid_tag = nullptr;
        if (fq)
            hipLaunchKernelGGL(k_umbrella_fold<true>, dim3((uint32_t)n_umb), dim3(kTile), 0, s, f);
        else
            hipLaunchKernelGGL(k_umbrella_fold<false>, dim3((uint32_t)n_umb), dim3(kTile), 0, s, f);
        HIP_TRY(hipGetLastError());
        std::vector<uint32_t> hb(n_umb);
        uint32_t bad = 0;
        HIP_TRY(hipMemcpyAsync(hb.data(), dbits, n_umb * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&bad, a.bad, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad) return POSLO_E_INVAL;
        for (uint64_t l = 0; l < n_umb; l++) bits[l] = (uint8_t)hb[l];
        return POSLO_OK;
    }
    if (mode == 'I') {
        uint64_t ni = ccd->invalid.size();
        *n_bits = ni;
        if (!bits || cap < ni) return POSLO_E_INVAL;
        if (ni == 0) return POSLO_OK;
        std::vector<uint64_t> pos(ni);
        for (uint64_t k = 0; k < ni; k++) {
            if (ccd->invalid[k] < m->t0 || ccd->invalid[k] - m->t0 >= m->n) return POSLO_E_INVAL;
            pos[k] = ccd->invalid[k] - m->t0;
        }
        const uint32_t* gw = fq ? ctx_gtable_wide_fq(c) : ctx_gtable_wide(c);
        if (!gw) return POSLO_E_NOMEM;
        void *dpos, *dsig, *dflags;
        if ((st = scratch(c, S_IDX, ni * 8, &dpos)) || (st = scratch(c, S_SIGS, ni * 80, &dsig)) ||
            (st = scratch(c, S_FLAGS, ni, &dflags)))
            return st;
        HIP_TRY(hipMemcpyAsync(dpos, pos.data(), ni * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(dsig, ccd->invalid_sigs.data(), ni * 80, hipMemcpyHostToDevice, s));
        if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return st;
        VerifyArgs v;
        v.a = a;
        v.g = TileGeom{m->n, 1, 1, (uint32_t)kTile};
        v.inst = prm->inst;
        v.sigs = (const uint8_t*)dsig;
        v.list = (const uint64_t*)dpos;
        v.list_n = ni;
        v.ty = key->d_table;
        v.tg = gw;
        v.flags = (uint8_t*)dflags;
        v.tile_part = nullptr;
        if (fq)
            hipLaunchKernelGGL(k_verify_list<true>, dim3((uint32_t)((ni + kTile - 1) / kTile)), dim3(kTile), 0, s, v);
        else
            hipLaunchKernelGGL(k_verify_list<false>, dim3((uint32_t)((ni + kTile - 1) / kTile)), dim3(kTile), 0, s, v);
        HIP_TRY(hipGetLastError());
        std::vector<uint8_t> hf(ni);
        uint32_t bad = 0;
        HIP_TRY(hipMemcpyAsync(hf.data(), dflags, ni, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&bad, a.bad, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad) return POSLO_E_INVAL;
        for (uint64_t k = 0; k < ni; k++) bits[k] = hf[k] ? 0 : 1;
        return POSLO_OK;
    }
    return POSLO_E_INVAL;
}
