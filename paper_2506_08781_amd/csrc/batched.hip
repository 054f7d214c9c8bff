// Batched verification of many signers' batches in one persistent launch.
//
// Each signer's batch is a job: its own key, entries, ds and tag (the paper
// verifies one batch per launch; section "POSLO Parallel Batch
// Verification").  Jobs are cut into work items of up to CHUNK entries that
// never straddle a job.  A persistent grid of workgroups pulls items from an
// atomic counter until the queue is empty; each item's entries are sorted
// inside the workgroup by MDC-2/SHA block count (a counting sort in LDS), so
// that the 64 lanes of a wave hash messages of similar length; digests are
// summed lazily into one 288-bit partial per item.  A second kernel folds
// each job's partials, reduces mod q and checks the job's tag with one wave
// (comb tables).  Entries of chosen jobs can then be verified individually
// (Distill's check); invalid ones are appended to a list with one atomic per
// wave (ballot + popcount) and sorted on the host.
//
// The kernel sequence can be captured in a hipGraph and replayed; an
// autotuner times the kernel variants on the caller's batch and caches the
// fastest per shape class.
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "aes_perm.h"
#include "aes_quad.h"
#include "batch_run.h"
#include "device_fq.h"
#include "device_verify.h"

namespace poslo {

__device__ __forceinline__ BatchArgs job_args(const BJob& J, uint32_t log2_n2, const uint32_t* tab) {
    BatchArgs a;
    a.data = J.data;
    a.offsets = J.offsets;
    a.msg_len = J.msg_len;
    a.n = J.n;
    a.t0 = J.t0;
    a.epoch_first = J.t0 >> log2_n2;
    a.log2_n2 = log2_n2;
    a.tab = tab + J.epoch_base * kEpochWords;
    a.skip = nullptr;
    a.end = J.end;
    return a;
}

// ---- seed rows: one lane per (job, epoch); row 0 resets the queue ---------
// Blocks past the rows decode each job's tag (one lane per job): s < q and
// R a point, with R's affine coordinates kept for the final check.

struct BSeeds {
    const BJob* jobs;
    const DsArg* ds;
    const uint32_t* job_of_row;
    uint64_t n_rows;
    uint32_t row_blocks;
    uint32_t njobs;
    uint32_t log2_n2;
    uint32_t inst;
    uint32_t* tab;
    uint32_t* counter;
    uint32_t* rdec;  // 17 words per job: ok, x[8], y[8] (FourQ: x and y as GF(p^2) words)
    uint32_t fq;     // the FourQ group
};

template <int INST>
__global__ __launch_bounds__(256) void k_batch_seeds(BSeeds S) {
    __shared__ uint32_t lds[INST == INST_AES ? 4 * 256 : 1];
    if (blockIdx.x >= S.row_blocks) {
        uint32_t j = (blockIdx.x - S.row_blocks) * blockDim.x + threadIdx.x;
        if (j >= S.njobs) return;
        const BJob& J = S.jobs[j];
        uint32_t sv[8];
        uint8_t rb[32];
        for (int k = 0; k < 8; k++) {
            sv[k] = J.tag[k];
            store_le32(rb + 4 * k, J.tag[8 + k]);
        }
        uint32_t* o = S.rdec + (uint64_t)j * 17;
        if (S.fq) {
            gq R;
            const bool ok = scN_is_canonical(sv) && fq_decode(R, rb);
            o[0] = ok ? 1u : 0u;
            for (int k = 0; k < 4; k++) {
                o[1 + k] = ok ? R.X.a.v[k] : 0u;
                o[5 + k] = ok ? R.X.b.v[k] : 0u;
                o[9 + k] = ok ? R.Y.a.v[k] : 0u;
                o[13 + k] = ok ? R.Y.b.v[k] : 0u;
            }
            return;
        }
        ge R;
        bool ok = sc_is_canonical(sv) && ge_decode(R, rb);
        o[0] = ok ? 1u : 0u;
        for (int k = 0; k < 8; k++) {
            o[1 + k] = ok ? R.X.v[k] : 0u;
            o[9 + k] = ok ? R.Y.v[k] : 0u;
        }
        return;
    }
    // AES: four lanes per row (aes_quad.h); SHA-256: one lane per row
    if constexpr (INST == INST_AES) lds_tables_fill<4, 1>(lds);
    __syncthreads();
    const LdsTables<4, 1> tb{lds};
    const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t row = INST == INST_AES ? g >> 2 : g;
    const uint32_t c = (uint32_t)g & 3u;
    if (g == 0) S.counter[0] = 0;
    if (row >= S.n_rows) return;  // whole quads leave together
    uint32_t j = S.job_of_row[row];
    const BJob& J = S.jobs[j];
    const DsArg& D = S.ds[j];
    uint64_t i = (J.t0 >> S.log2_n2) + (row - J.epoch_base);
    int k = ds_cover(D, i);
    if (k < 0) k = 0;  // coverage validated on the host
    uint32_t* e = S.tab + row * kEpochWords;
    if constexpr (INST == INST_AES) {
        uint32_t xc = D.v[k][c];
        for (int bt = (int)D.depth[k] - 1; bt >= 0; bt--) xc = quad_prf_node(tb, xc, (uint32_t)((i >> bt) & 1u), c);
        quad_epoch_row(tb, xc, c, e);
        return;
    }
    uint32_t x[4] = {D.v[k][0], D.v[k][1], D.v[k][2], D.v[k][3]};
    for (int bt = (int)D.depth[k] - 1; bt >= 0; bt--) {
        uint32_t nx[4];
        prf_node_sha(x, (uint32_t)((i >> bt) & 1u), nx);
        x[0] = nx[0], x[1] = nx[1], x[2] = nx[2], x[3] = nx[3];
    }
    for (int w = 0; w < 4; w++) e[44 + w] = x[w];
}

// ---- the persistent hashing kernel ------------------------------------------

// a record every lane of the wave loaded from the same address, word by word
// from the first lane, so that the compiler keeps it in scalar registers
template <class T>
__device__ __forceinline__ T wave_uniform(const T& v) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T out;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&v);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); k++) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
    return out;
}

struct BHot {
    const BJob* jobs;
    const BItem* items;
    uint32_t n_items;
    uint32_t log2_n2;
    const uint32_t* tab;
    uint32_t* counter;
    uint32_t* partials;  // 9 words per item
    uint32_t* e_out;     // optional: e_t mod q, 8 words per entry (job's ebase + offset)
    uint8_t* xbad;       // with e_out: 1 when x_t differs from the signature's
    uint32_t* pair_tmp;  // PAIR variants: 16 words per thread of the grid
    uint32_t emit_raw;   // e_out gets the unreduced digest (FourQ: reduced mod N by the checks)
};

// INST 1: MDC-2-AES over the byte-addressed tables (NT = 1 or 2);
// INST 0: SHA-256 (no tables).  CHUNK entries per item at most.
// PAIR (SORT, CHUNK == 2 * BLOCK): thread g takes the g-th shortest and the
// g-th longest entry of the sorted item, so every lane and wave gets about
// the same total length and waves do not idle at the item's closing barrier.
template <int INST, int NT, int BLOCK, int CHUNK, bool SORT, int WPE, bool EMIT, bool PAIR = false, int CP = 64>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void k_batch_hot(BHot A) {
    static_assert(!PAIR || (SORT && CHUNK == 2 * BLOCK), "pairing needs sorted items of two entries per thread");
    constexpr int TW = INST == INST_AES ? NT * 256 * CP : 0;  // table words
    constexpr int SW = 64 + 16 + CHUNK / 2 + CHUNK / 4;       // counts, misc, order (u16), keys (u8)
    __shared__ uint32_t lds[TW + SW + (BLOCK / 64) * 9];
    if constexpr (INST == INST_AES) {
        perm_tables_fill<NT, CP>(lds);
    }
    uint32_t* counts = lds + TW;                                // 64 bucket counters
    uint32_t* misc = counts + 64;                               // [0] item id
    uint16_t* order = reinterpret_cast<uint16_t*>(misc + 16);   // CHUNK slots
    uint8_t* keys = reinterpret_cast<uint8_t*>(order + CHUNK);  // CHUNK block counts
    uint32_t* red = lds + TW + SW;
    const PermTables<NT, CP> tb = perm_tables<NT, CP>(lds);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) misc[0] = atomicAdd(A.counter, 1u);
        if (SORT && threadIdx.x < 64) counts[threadIdx.x] = 0;
        __syncthreads();
        // uniform across the workgroup: keeps the item's job record in scalar registers
        const uint32_t item = __builtin_amdgcn_readfirstlane(misc[0]);
        if (item >= A.n_items) break;
        const BItem it = wave_uniform(A.items[item]);
        const BJob J = wave_uniform(A.jobs[it.job]);
        const BatchArgs a = job_args(J, A.log2_n2, A.tab);
        if (SORT) {
            // counting sort of the item's slots by block count
            for (uint32_t s = threadIdx.x; s < it.count; s += BLOCK) {
                uint64_t p = it.first + s;
                uint64_t L = a.offsets ? gload(a.offsets + p + 1) - gload(a.offsets + p) : a.msg_len;
                uint64_t nb = INST == INST_AES ? (L + 31) / 16 : (L + 25 + 63) / 64;
                uint32_t key = nb < 63 ? (uint32_t)nb : 63u;
                keys[s] = (uint8_t)key;
                atomicAdd(&counts[key], 1u);
            }
            __syncthreads();
            if (threadIdx.x < 64) {
                uint32_t v = counts[threadIdx.x], incl = v;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    uint32_t o = __shfl_up(incl, off);
                    if ((int)threadIdx.x >= off) incl += o;
                }
                counts[threadIdx.x] = incl - v;  // exclusive start of the bucket
            }
            __syncthreads();
            for (uint32_t s = threadIdx.x; s < it.count; s += BLOCK) {
                uint32_t pos = atomicAdd(&counts[keys[s]], 1u);
                order[pos] = (uint16_t)s;
            }
            __syncthreads();
        }
        // the digest of the entry in sorted slot s (EMIT: its e_t and x check
        // are stored as well)
        // batch position of the entry in sorted slot s (slots [BLOCK, count)
        // map to count - 1 - (s - BLOCK): the longest first)
        auto pos_of = [&](uint32_t s) -> uint64_t {
            const uint32_t slot = (PAIR && s >= BLOCK) ? it.count - 1 - (s - BLOCK) : s;
            return it.first + (SORT ? order[slot] : slot);
        };
        // the digest of the entry in sorted slot s = tid + h * BLOCK (EMIT:
        // its e_t and x check are stored as well).  The entry's position is
        // looked up again after the digest from an opaque copy of the thread
        // index, so that no per-entry address stays live across the digest.
        auto entry = [&](uint32_t tid, uint32_t h, uint32_t dig[8]) {
            const uint64_t p = pos_of(tid + h * BLOCK);
            EntryView ev = entry_view(a, p);
            uint32_t x[4];
            if constexpr (INST == INST_AES) {
                const uint64_t t = a.t0 + p;
                const uint32_t jj = (uint32_t)(t & ((1ull << a.log2_n2) - 1));
                const uint32_t* rk = a.tab + ((t >> a.log2_n2) - a.epoch_first) * kEpochWords;
                auto xf = [&](uint32_t y[4]) {
                    y[0] = jj, y[1] = 0, y[2] = 0, y[3] = 0;
                    penc_rk(tb, rk, y);
                    y[0] ^= jj;
                };
                digest_mdc2_any_late(tb, ev, a.end, xf, x, dig, Mdc2BlockPerm{});
            } else {
                one_time_seed_sha(a, p, x);
                digest_sha_any(ev, a.end, x, dig);
#pragma unroll
                for (int w = 0; w < 4; w++) x[w] = bswap32(x[w]);
            }
            if constexpr (EMIT) {
                uint32_t t2 = tid;
                asm volatile("" : "+v"(t2));
                const uint64_t p2 = pos_of(t2 + h * BLOCK);
                // x_t as little-endian words against the signature's x bytes
                const uint8_t* sg = J.sigs + p2 * 80 + 64;
                uint32_t d = 0;
#pragma unroll
                for (int w = 0; w < 4; w++) d |= x[w] ^ gload_le32(sg + 4 * w);
                uint32_t e[8];
                if (A.emit_raw)
#pragma unroll
                    for (int w = 0; w < 8; w++) e[w] = dig[w];
                else
                    sc_reduce256(e, dig);
                uint32_t* eo = A.e_out + (J.ebase + p2) * 8;
#pragma unroll
                for (int w = 0; w < 8; w++) eo[w] = e[w];
                A.xbad[J.ebase + p2] = d ? 1 : 0;
            }
        };
        uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (PAIR) {
            // two entries per thread, hashed by one loop over h; each digest
            // goes to the thread's slot h of pair_tmp and the sum is formed
            // after both, so that no accumulator stays live in registers
            // across a digest
#pragma unroll
            for (uint32_t h = 0; h < 2; h++) {
                if (threadIdx.x + h * BLOCK < it.count) {
                    uint32_t dig[8];
                    entry(threadIdx.x, h, dig);
                    uint32_t t2 = threadIdx.x;
                    asm volatile("" : "+v"(t2));
                    uint32_t* tmp = A.pair_tmp + (((uint64_t)blockIdx.x * BLOCK + t2) * 2 + h) * 8;
#pragma unroll
                    for (int w = 0; w < 8; w++) tmp[w] = dig[w];
                }
            }
#pragma unroll 1
            for (uint32_t h = 0; h < 2; h++) {
                if (threadIdx.x + h * BLOCK < it.count) {
                    const uint32_t* tmp = A.pair_tmp + (((uint64_t)blockIdx.x * BLOCK + threadIdx.x) * 2 + h) * 8;
                    uint32_t dig[8];
#pragma unroll
                    for (int w = 0; w < 8; w++) dig[w] = tmp[w];
                    acc288_add256(acc, dig);
                }
            }
        } else {
            // an item holds at most CHUNK entries: with CHUNK <= BLOCK a lane
            // has at most one, so nothing accumulates across the digest
            if constexpr (CHUNK <= BLOCK) {
                if (threadIdx.x < it.count) {
                    uint32_t dig[8];
                    entry(threadIdx.x, 0, dig);
                    acc288_add256(acc, dig);
                }
            } else {
                for (uint32_t h = 0; threadIdx.x + h * BLOCK < it.count; h++) {
                    uint32_t dig[8];
                    entry(threadIdx.x, h, dig);
                    acc288_add256(acc, dig);
                }
            }
        }
        block_reduce288_scratch<BLOCK>(acc, A.partials + (uint64_t)item * 9, red);
    }
}

// ---- per-job checks: one wave per job ----------------------------------------
// (many jobs at once: independent one-wave checks keep more of them resident
// than the quad-split block check, whose registers allow four blocks per CU)

// FQ: on FourQ (e mod N; rdec holds x and y as GF(p^2) words)
template <bool FQ>
__global__ __launch_bounds__(64) void k_batch_final(const BJob* jobs, const uint32_t* partials, const uint32_t* tg,
                                                    const uint32_t* rdec, uint32_t* result) {
    const BJob& J = jobs[blockIdx.x];
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t k = J.item_base + threadIdx.x; k < J.item_end; k += 64) acc288_add(acc, partials + k * 9);
    wave_reduce288(acc);  // every lane holds the sum
    uint32_t e[8], s[8];
    for (int k = 0; k < 8; k++) s[k] = J.tag[k];
    if constexpr (FQ) {
        scN_reduce<9>(e, acc);
        const uint32_t* r = rdec + (uint64_t)blockIdx.x * 17;
        if (!r[0])
            for (int k = 0; k < 8; k++) s[k] = 0;  // s >= N: any in-range digits, the result is 0
        gq P;
        wave_double_scalar_fq(P, J.ty, tg, e, s);
        if (threadIdx.x == 0) {
            fp2 rx, ry, t0, t1;
            unstash_f2(rx, r + 1, 1);
            unstash_f2(ry, r + 9, 1);
            f2_mul(t0, rx, P.Z);
            f2_mul(t1, ry, P.Z);
            result[blockIdx.x] = (r[0] && f2_eq(t0, P.X) && f2_eq(t1, P.Y)) ? 1u : 0u;
        }
        return;
    }
    sc_reduce288(e, acc);
    ge P;
    wave_double_scalar(P, J.ty, tg, e, s);
    if (threadIdx.x == 0) {
        const uint32_t* r = rdec + (uint64_t)blockIdx.x * 17;
        fe rx, ry, t0, t1;
        for (int k = 0; k < 8; k++) {
            rx.v[k] = r[1 + k];
            ry.v[k] = r[9 + k];
        }
        fe_mul(t0, rx, P.Z);
        fe_mul(t1, ry, P.Z);
        result[blockIdx.x] = (r[0] && fe_equal(t0, P.X) && fe_equal(t1, P.Y)) ? 1u : 0u;
    }
}

// ---- individual verification of the entries of chosen jobs ----------------

struct BVerify {
    const BJob* jobs;
    const BItem* tiles;  // up to 256 entries each
    const uint32_t* tg;  // G's wide table
    uint32_t inst;
    uint32_t log2_n2;
    const uint32_t* tab;
    const uint32_t* ekeys;  // PRE: e_t from the hashing kernel (job's ebase + offset)
    const uint8_t* xbad;    // PRE: x checks from the hashing kernel
    uint64_t* idx;    // appended slots (job's vbase + entry offset) of invalid entries
    uint32_t* count;  // number appended
    uint32_t* stash;  // PRE: kVerifyStashWords per workgroup
    uint32_t* next;   // PRE: tile queue head (zero at launch)
    uint32_t ntiles;
};

// The individual checks of the listed jobs' entries.
// With e_t and the x checks from the hashing kernel (launch with emit):
// k_batch_verify_pre, persistent, one wave per workgroup pulling tiles from
// a queue (largest first; every wave leaves once the queue is drained).  A
// tile holds up to verify_tile_len entries of one job; thread i checks
// entries i + 64 k, k < ne = ceil(count / 64), with one shared inversion,
// the points waiting in the workgroup's slice of the stash.  A
// key with a resident wide table (J.tyw) takes 16 + 16 mixed additions per
// entry instead of 32 + 16.
template <bool FQ>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_batch_verify_pre(BVerify V) {
    uint32_t* st = V.stash + (uint64_t)blockIdx.x * kVerifyStashWords + threadIdx.x;
#pragma unroll 1
    for (;;) {
        uint32_t t = threadIdx.x == 0 ? atomicAdd(V.next, 1u) : 0u;
        t = (uint32_t)__shfl((int)t, 0);
        if (t >= V.ntiles) break;
        const BItem it = wave_uniform(V.tiles[t]);
        const BJob J = wave_uniform(V.jobs[it.job]);
        const int ne = (int)((it.count + 63) / 64);
        auto ent = [&](int k, const uint8_t*& sg, const uint32_t*& e, bool& go) {
            const uint32_t idx = threadIdx.x + 64u * (uint32_t)k;
            const uint64_t p = it.first + (idx < it.count ? idx : 0);
            go = idx < it.count && !gload(V.xbad + J.ebase + p);
            // skipped entries point at the tile's first entry (in bounds)
            const uint64_t q = go ? p : it.first;
            sg = J.sigs + q * 80;
            e = V.ekeys + (J.ebase + q) * 8;
        };
        uint32_t okmask;
        if constexpr (FQ)
            okmask = verify_sig_batch_fq<true>(ent, ne, J.ty, V.tg, st, 64);
        else
            okmask = J.tyw ? verify_sig_batch<true>(ent, ne, J.tyw, V.tg, st, 64)
                           : verify_sig_batch<false>(ent, ne, J.ty, V.tg, st, 64);
#pragma unroll 1
        for (int k = 0; k < ne; k++) {
            const uint32_t idx = threadIdx.x + 64u * (uint32_t)k;
            wave_append(idx < it.count && !((okmask >> k) & 1u), J.vbase + it.first + idx, V.idx, V.count);
        }
    }
}

// Without them (tiles of 256): one entry per thread, hashing included.
__global__ __launch_bounds__(256) void k_batch_verify(BVerify V) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
    const BItem it = wave_uniform(V.tiles[blockIdx.x]);
    const BJob J = wave_uniform(V.jobs[it.job]);
    LdsTables<4, 1> tb{lds};
    bool bad = false;
    uint64_t slot = 0;
    if (threadIdx.x < it.count) {
        uint64_t p = it.first + threadIdx.x;
        uint32_t e[8], s[8];
        BatchArgs a = job_args(J, V.log2_n2, V.tab);
        bad = !verify_one(tb, a, a.end, V.inst, p, J.sigs + p * 80, J.ty, V.tg, e, s);
        slot = J.vbase + p;
    }
    wave_append(bad, slot, V.idx, V.count);
}

__global__ void k_zero_u32x2(uint32_t* p, uint32_t* q) {
    p[0] = 0;
    q[0] = 0;
}

// ---- tuning --------------------------------------------------------------------

static const HotVariant kHot[] = {
    {"aes_perm2_b1024_c1024_sorted", 1, 2, 1024, 1024, 1, 4}, {"aes_perm2_b1024_c2048_sorted", 1, 2, 1024, 2048, 1, 4},
    {"aes_perm2_b1024_c1024", 1, 2, 1024, 1024, 0, 4},        {"aes_perm1_b1024_c1024_sorted", 1, 1, 1024, 1024, 1, 4},
    {"aes_perm1_b512_c1024_sorted", 1, 1, 512, 1024, 1, 4},   {"sha_b256_c1024_sorted_w3", 0, 1, 256, 1024, 1, 3},
    {"sha_b256_c1024_sorted_w4", 0, 1, 256, 1024, 1, 4},      {"sha_b256_c256_sorted_w3", 0, 1, 256, 256, 1, 3},
    {"sha_b256_c1024_w3", 0, 1, 256, 1024, 0, 3},             {"sha_b512_c2048_sorted_w3", 0, 1, 512, 2048, 1, 3},
    {"aes_perm1_b1024_c1024_sorted_w8", 1, 1, 1024, 1024, 1, 8},
    {"aes_perm1_b1024_c2048_paired_w8", 1, 1, 1024, 2048, 1, 8, 1},
    {"aes_perm2_b1024_c2048_paired", 1, 2, 1024, 2048, 1, 4, 1},
    {"sha_b256_c512_paired_w3", 0, 1, 256, 512, 1, 3, 1},
    {"sha_b512_c1024_paired_w3", 0, 1, 512, 1024, 1, 3, 1},
    {"aes_p2x32_b1024_c1024_sorted_w8", 1, 2, 1024, 1024, 1, 8, 0, 32},
    {"aes_p2x32_b1024_c2048_paired_w8", 1, 2, 1024, 2048, 1, 8, 1, 32},
};
constexpr int kNumHot = sizeof kHot / sizeof kHot[0];

int batch_variant_count() { return kNumHot; }
const HotVariant& batch_variant(int v) { return kHot[v]; }
// AES: aes_p2x32_b1024_c2048_paired_w8, the autotuner's pick on the
// 4,096-signer log (1.52 G entries/s); SHA-256: sha_b256_c1024_sorted_w3
int batch_default_variant(uint32_t inst) { return inst_base(inst) == POSLO_INST_AES ? 16 : 5; }
bool batch_inst_ok(uint32_t inst) { return (inst & ~POSLO_GROUP_FOURQ) <= POSLO_INST_AES; }

size_t hot_lds_bytes(const HotVariant& v) {
    size_t tw = v.inst == 1 ? (size_t)v.nt * 256 * (v.copies ? v.copies : 64) : 0;
    return 4 * (tw + 64 + 16 + v.chunk / 2 + v.chunk / 4 + (v.block / 64) * 9);
}

static int launch_hot(int v, uint32_t grid, const BHot& A, hipStream_t s) {
#define HOT(I, NT, B, C, S, W)                                                                        \
    if (A.e_out)                                                                                      \
        hipLaunchKernelGGL((k_batch_hot<I, NT, B, C, S, W, true>), dim3(grid), dim3(B), 0, s, A);  \
    else                                                                                              \
        hipLaunchKernelGGL((k_batch_hot<I, NT, B, C, S, W, false>), dim3(grid), dim3(B), 0, s, A); \
    break
#define HOTP(I, NT, B, C, W)                                                                                 \
    if (A.e_out)                                                                                             \
        hipLaunchKernelGGL((k_batch_hot<I, NT, B, C, true, W, true, true>), dim3(grid), dim3(B), 0, s, A);  \
    else                                                                                                     \
        hipLaunchKernelGGL((k_batch_hot<I, NT, B, C, true, W, false, true>), dim3(grid), dim3(B), 0, s, A); \
    break
    switch (v) {
        case 0: HOT(1, 2, 1024, 1024, true, 4);
        case 1: HOT(1, 2, 1024, 2048, true, 4);
        case 2: HOT(1, 2, 1024, 1024, false, 4);
        case 3: HOT(1, 1, 1024, 1024, true, 4);
        case 4: HOT(1, 1, 512, 1024, true, 4);
        case 5: HOT(0, 1, 256, 1024, true, 3);
        case 6: HOT(0, 1, 256, 1024, true, 4);
        case 7: HOT(0, 1, 256, 256, true, 3);
        case 8: HOT(0, 1, 256, 1024, false, 3);
        case 9: HOT(0, 1, 512, 2048, true, 3);
        case 10: HOT(1, 1, 1024, 1024, true, 8);
        case 11: HOTP(1, 1, 1024, 2048, 8);
        case 12: HOTP(1, 2, 1024, 2048, 4);
        case 13: HOTP(0, 1, 256, 512, 3);
        case 14: HOTP(0, 1, 512, 1024, 3);
        case 15:
            if (A.e_out)
                hipLaunchKernelGGL((k_batch_hot<1, 2, 1024, 1024, true, 8, true, false, 32>), dim3(grid), dim3(1024),
                                   0, s, A);
            else
                hipLaunchKernelGGL((k_batch_hot<1, 2, 1024, 1024, true, 8, false, false, 32>), dim3(grid), dim3(1024),
                                   0, s, A);
            break;
        case 16:
            if (A.e_out)
                hipLaunchKernelGGL((k_batch_hot<1, 2, 1024, 2048, true, 8, true, true, 32>), dim3(grid), dim3(1024), 0,
                                   s, A);
            else
                hipLaunchKernelGGL((k_batch_hot<1, 2, 1024, 2048, true, 8, false, true, 32>), dim3(grid), dim3(1024),
                                   0, s, A);
            break;
        default: return POSLO_E_INVAL;
    }
#undef HOT
#undef HOTP
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

static uint32_t hot_wg_per_cu(const HotVariant& v, int override_wg) {
    if (override_wg > 0) return (uint32_t)override_wg;
    uint32_t by_lds = (uint32_t)((160 * 1024) / (hot_lds_bytes(v) + 512));
    uint32_t by_waves = 4 * v.waves_per_simd / (v.block / 64);
    return std::max<uint32_t>(1, std::min(by_lds, by_waves));
}

// ---- the runner ----------------------------------------------------------------

using namespace hostside;

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

BatchRunner::~BatchRunner() {
    forget_graphs();
    if (capture_) hipStreamDestroy(capture_);
    for (void* p : {d_jobs_, d_ds_, d_rows_, d_items_, d_tab_, d_part_, d_res_, d_misc_, d_rdec_, d_vtiles_, d_idx_,
                    d_ekeys_, d_xbad_, d_pair_, d_stash_})
        if (p) hipFree(p);
    if (h_res_) hipHostFree(h_res_);
    if (h_misc_) hipHostFree(h_misc_);
}

void BatchRunner::forget_graphs() {
    if (!graphs_.empty()) {
        hipDeviceSynchronize();
        for (auto& g : graphs_) hipGraphExecDestroy(g.second);
        graphs_.clear();
    }
}

int BatchRunner::grow(void** p, size_t* have, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (*have >= bytes) return POSLO_OK;
    // the old buffer may be read by queued work or baked into captured graphs
    forget_graphs();
    hipDeviceSynchronize();
    if (*p) hipFree(*p);
    *p = nullptr;
    *have = 0;
    size_t want = bytes + bytes / 4;
    if (hipMalloc(p, want) != hipSuccess) return POSLO_E_NOMEM;
    *have = want;
    return POSLO_OK;
}

int BatchRunner::grow_pinned(void** p, size_t* have, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (*have >= bytes) return POSLO_OK;
    forget_graphs();
    hipDeviceSynchronize();
    if (*p) hipHostFree(*p);
    *p = nullptr;
    *have = 0;
    size_t want = bytes + bytes / 4;
    if (hipHostMalloc(p, want, hipHostMallocDefault) != hipSuccess) return POSLO_E_NOMEM;
    *have = want;
    return POSLO_OK;
}

int BatchRunner::plan(const poslo_params* prm, const JobSpec* jobs, uint32_t njobs, const poslo_tuning& t,
                      int num_cu) {
    if (!params_ok(prm) || !batch_inst_ok(prm->inst) || (njobs && !jobs)) return POSLO_E_INVAL;
    if (t.variant < 0 || t.variant >= kNumHot || kHot[t.variant].inst != (int)inst_base(prm->inst) || t.wg_per_cu < 0 ||
        t.wg_per_cu > 64)
        return POSLO_E_INVAL;
    prm_ = *prm;
    tune_ = t;
    num_cu_ = num_cu;
    vtiles_.clear();
    vbase_.clear();
    const uint32_t chunk = (uint32_t)kHot[t.variant].chunk;
    jobs_.assign(njobs, BJob{});
    ds_.resize(njobs);
    job_of_row_.clear();
    items_.clear();
    uint64_t nmax = 1ull << (prm->log2_n1 + prm->log2_n2), total = 0;
    std::vector<DsNode> nodes;
    for (uint32_t j = 0; j < njobs; j++) {
        const JobSpec& in = jobs[j];
        if (!in.ty || !in.tag || in.t0 > nmax || in.n > nmax - in.t0 || (in.n && !in.data)) return POSLO_E_INVAL;
        total += in.n;
        if (total >= (1ull << 32)) return POSLO_E_INVAL;
        if (!ds_parse(in.ds, in.ds_len, nodes)) return POSLO_E_INVAL;
        DsArg& d = ds_[j];
        memset(&d, 0, sizeof d);
        d.count = (uint32_t)nodes.size();
        for (size_t k = 0; k < nodes.size(); k++) {
            d.depth[k] = nodes[k].depth;
            d.index[k] = nodes[k].index;
            for (int w = 0; w < 4; w++) d.v[k][w] = load_le32(nodes[k].v + 4 * w);
        }
        BJob& J = jobs_[j];
        J.ty = in.ty;
        J.tyw = in.tyw;
        J.data = in.data;
        J.offsets = in.offsets;
        J.msg_len = in.offsets ? 0 : in.msg_len;
        J.end = in.data_bytes ? in.data + in.data_bytes : (in.offsets ? nullptr : in.data + in.n * in.msg_len);
        J.sigs = in.sigs;
        J.t0 = in.t0;
        J.n = in.n;
        J.epoch_base = job_of_row_.size();
        J.item_base = items_.size();
        J.vbase = 0;
        J.ebase = total - in.n;
        for (int k = 0; k < 16; k++) J.tag[k] = load_le32(in.tag + 4 * k);
        if (in.n) {
            uint64_t e0 = in.t0 >> prm->log2_n2, e1 = (in.t0 + in.n - 1) >> prm->log2_n2;
            for (uint64_t e = e0; e <= e1; e++) {
                if (sr_node(nodes.data(), (int)nodes.size(), e) < 0) return POSLO_E_SEED;
                job_of_row_.push_back(j);
            }
            for (uint64_t f = 0; f < in.n; f += chunk)
                items_.push_back(BItem{j, (uint32_t)std::min<uint64_t>(chunk, in.n - f), f});
        }
        J.item_end = items_.size();
    }
    n_entries_ = total;
    emitted_ = false;
    return POSLO_OK;
}

template <class T>
static void key_bytes(std::string& k, const T& v) {
    k.append(reinterpret_cast<const char*>(&v), sizeof v);
}

int BatchRunner::launch(hipStream_t s, bool use_graph, poslo_ctx* prof, bool emit) {
    if (!prof || !prof->d_gtable) return POSLO_E_INVAL;
    const uint32_t njobs = (uint32_t)jobs_.size();
    const uint64_t rows = job_of_row_.size();
    int st;
    if (emit) {
        for (const BJob& J : jobs_)
            if (J.n && !J.sigs) return POSLO_E_INVAL;
        if ((st = grow(&d_ekeys_, &n_ekeys_b_, n_entries_ * 32)) || (st = grow(&d_xbad_, &n_xbad_b_, n_entries_)))
            return st;
    }
    emitted_ = emit;
    if ((st = grow(&d_jobs_, &n_jobs_b_, njobs * sizeof(BJob))) ||
        (st = grow(&d_ds_, &n_ds_b_, njobs * sizeof(DsArg))) || (st = grow(&d_rows_, &n_rows_b_, rows * 4)) ||
        (st = grow(&d_items_, &n_items_b_, items_.size() * sizeof(BItem))) ||
        (st = grow(&d_tab_, &n_tab_b_, rows * kEpochWords * 4)) ||
        (st = grow(&d_part_, &n_part_b_, items_.size() * 36)) || (st = grow(&d_res_, &n_res_b_, njobs * 4)) ||
        (st = grow(&d_misc_, &n_misc_b_, 256)) || (st = grow(&d_rdec_, &n_rdec_b_, njobs * 17 * 4)) ||
        (st = grow_pinned((void**)&h_res_, &h_res_b_, njobs * 4)))
        return st;
    if (njobs) {
        HIP_TRY(hipMemcpyAsync(d_jobs_, jobs_.data(), njobs * sizeof(BJob), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_ds_, ds_.data(), njobs * sizeof(DsArg), hipMemcpyHostToDevice, s));
    }
    if (rows) HIP_TRY(hipMemcpyAsync(d_rows_, job_of_row_.data(), rows * 4, hipMemcpyHostToDevice, s));
    if (!items_.empty())
        HIP_TRY(hipMemcpyAsync(d_items_, items_.data(), items_.size() * sizeof(BItem), hipMemcpyHostToDevice, s));
    const HotVariant& hv = kHot[tune_.variant];
    BSeeds S;
    memset(&S, 0, sizeof S);
    S.jobs = (const BJob*)d_jobs_;
    S.ds = (const DsArg*)d_ds_;
    S.job_of_row = (const uint32_t*)d_rows_;
    S.n_rows = rows;
    // AES rows take four lanes each
    const uint64_t row_lanes = rows * (inst_base(prm_.inst) == POSLO_INST_AES ? 4 : 1);
    S.row_blocks = (uint32_t)std::max<uint64_t>(1, (row_lanes + 255) / 256);
    S.njobs = njobs;
    S.log2_n2 = prm_.log2_n2;
    S.inst = prm_.inst;
    S.tab = (uint32_t*)d_tab_;
    S.counter = (uint32_t*)d_misc_;
    S.rdec = (uint32_t*)d_rdec_;
    const bool fq = (prm_.inst & POSLO_GROUP_FOURQ) != 0;
    S.fq = fq ? 1u : 0u;
    const uint32_t seed_grid = S.row_blocks + (njobs + 255) / 256;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(items_.size(), (uint64_t)num_cu_ * hot_wg_per_cu(hv, tune_.wg_per_cu)));
    BHot A;
    memset(&A, 0, sizeof A);
    A.jobs = (const BJob*)d_jobs_;
    A.items = (const BItem*)d_items_;
    A.n_items = (uint32_t)items_.size();
    A.log2_n2 = prm_.log2_n2;
    A.tab = (const uint32_t*)d_tab_;
    A.counter = (uint32_t*)d_misc_;
    A.partials = (uint32_t*)d_part_;
    A.e_out = emit ? (uint32_t*)d_ekeys_ : nullptr;
    A.xbad = emit ? (uint8_t*)d_xbad_ : nullptr;
    A.emit_raw = fq ? 1u : 0u;
    if (hv.pair) {
        if ((st = grow(&d_pair_, &n_pair_b_, (size_t)grid * hv.block * 64))) return st;
        A.pair_tmp = (uint32_t*)d_pair_;
    }
    const uint32_t* tg = fq ? ctx_gtable_fq(prof) : prof->d_gtable;
    if (!tg) return POSLO_E_NOMEM;
    auto launch_all = [&](hipStream_t q, bool timed) -> int {
        if (inst_base(prm_.inst) == POSLO_INST_AES)
            hipLaunchKernelGGL(k_batch_seeds<INST_AES>, dim3(seed_grid), dim3(256), 0, q, S);
        else
            hipLaunchKernelGGL(k_batch_seeds<INST_SHA256>, dim3(seed_grid), dim3(256), 0, q, S);
        if (timed) prof_begin(prof, POSLO_KT_BATCH_HOT, q);
        int r = launch_hot(tune_.variant, grid, A, q);
        if (timed) prof_end(prof, POSLO_KT_BATCH_HOT, q);
        if (r) return r;
        if (njobs && fq)
            hipLaunchKernelGGL(k_batch_final<true>, dim3(njobs), dim3(64), 0, q, (const BJob*)d_jobs_,
                               (const uint32_t*)d_part_, tg, (const uint32_t*)d_rdec_, (uint32_t*)d_res_);
        else if (njobs)
            hipLaunchKernelGGL(k_batch_final<false>, dim3(njobs), dim3(64), 0, q, (const BJob*)d_jobs_,
                               (const uint32_t*)d_part_, tg, (const uint32_t*)d_rdec_, (uint32_t*)d_res_);
        return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
    };
    prof_begin(prof, POSLO_KT_BATCH, s);
    if (use_graph) {
        std::string gk;
        key_bytes(gk, S);
        key_bytes(gk, A);
        key_bytes(gk, seed_grid);
        key_bytes(gk, grid);
        key_bytes(gk, tune_.variant);
        key_bytes(gk, tg);
        key_bytes(gk, d_res_);
        auto it = graphs_.find(gk);
        hipGraphExec_t exec = nullptr;
        if (it != graphs_.end()) {
            exec = it->second;
        } else {
            if (graphs_.size() >= 64) {
                HIP_TRY(hipStreamSynchronize(s));
                forget_graphs();
            }
            if (!capture_) HIP_TRY(hipStreamCreateWithFlags(&capture_, hipStreamNonBlocking));
            HIP_TRY(hipStreamBeginCapture(capture_, hipStreamCaptureModeThreadLocal));
            int r = launch_all(capture_, false);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(capture_, &g);
            if (r || ec != hipSuccess) {
                if (g) hipGraphDestroy(g);
                return r ? r : POSLO_E_DEVICE;
            }
            hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (ei != hipSuccess) return POSLO_E_DEVICE;
            graphs_[gk] = exec;
        }
        HIP_TRY(hipGraphLaunch(exec, s));
    } else {
        if ((st = launch_all(s, (prof->profile_mask >> POSLO_KT_BATCH_HOT) & 1u))) return st;
    }
    prof_end(prof, POSLO_KT_BATCH, s);
    if (njobs) HIP_TRY(hipMemcpyAsync(h_res_, d_res_, njobs * 4, hipMemcpyDeviceToHost, s));
    return POSLO_OK;
}

int BatchRunner::launch_verify(const std::vector<uint32_t>& which, hipStream_t s, poslo_ctx* prof) {
    if (!prof || !prof->d_gtable) return POSLO_E_INVAL;
    vtiles_.clear();
    vbase_.clear();
    n_checked_ = 0;
    uint64_t n_all = 0;
    for (uint32_t j : which) {
        if (j >= jobs_.size()) return POSLO_E_INVAL;
        n_all += jobs_[j].n;
    }
    const uint64_t tile = emitted_ ? verify_tile_len(n_all, prof->num_cu) : 256;
    for (uint32_t j : which) {
        BJob& J = jobs_[j];
        if (J.n && !J.sigs) return POSLO_E_INVAL;
        J.vbase = n_checked_;
        vbase_.push_back({n_checked_, j});
        for (uint64_t f = 0; f < J.n; f += tile)
            vtiles_.push_back(BItem{j, (uint32_t)std::min<uint64_t>(tile, J.n - f), f});
        n_checked_ += J.n;
    }
    if (n_checked_ >= (1ull << 32)) return POSLO_E_INVAL;
    // largest tiles first: the persistent waves then finish together
    if (emitted_)
        std::stable_sort(vtiles_.begin(), vtiles_.end(),
                         [](const BItem& x, const BItem& y) { return x.count > y.count; });
    const uint32_t grid = (uint32_t)std::min<size_t>(vtiles_.size(), (size_t)prof->num_cu * kVerifyWgPerCu);
    int st;
    if ((st = grow(&d_vtiles_, &n_vtiles_b_, vtiles_.size() * sizeof(BItem))) ||
        (st = grow(&d_idx_, &n_idx_b_, n_checked_ * 8)) || (st = grow_pinned((void**)&h_misc_, &h_misc_b_, 64)))
        return st;
    if (emitted_ && grid && (st = grow(&d_stash_, &n_stash_b_, (size_t)grid * kVerifyStashWords * 4))) return st;
    h_misc_[0] = 0;
    if (vtiles_.empty()) return POSLO_OK;
    HIP_TRY(hipMemcpyAsync(d_jobs_, jobs_.data(), jobs_.size() * sizeof(BJob), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_vtiles_, vtiles_.data(), vtiles_.size() * sizeof(BItem), hipMemcpyHostToDevice, s));
    uint32_t* cnt = (uint32_t*)d_misc_ + 4;
    uint32_t* next = (uint32_t*)d_misc_ + 8;
    hipLaunchKernelGGL(k_zero_u32x2, dim3(1), dim3(1), 0, s, cnt, next);
    BVerify V;
    V.jobs = (const BJob*)d_jobs_;
    V.tiles = (const BItem*)d_vtiles_;
    const bool fq = (prm_.inst & POSLO_GROUP_FOURQ) != 0;
    if (fq && !emitted_) return POSLO_E_INVAL;  // FourQ checks take the emitted digests
    V.tg = fq ? ctx_gtable_wide_fq(prof) : ctx_gtable_wide(prof);
    if (!V.tg) return POSLO_E_NOMEM;
    V.inst = prm_.inst;
    V.log2_n2 = prm_.log2_n2;
    V.tab = (const uint32_t*)d_tab_;
    V.ekeys = emitted_ ? (const uint32_t*)d_ekeys_ : nullptr;
    V.xbad = emitted_ ? (const uint8_t*)d_xbad_ : nullptr;
    V.idx = (uint64_t*)d_idx_;
    V.count = cnt;
    V.stash = emitted_ ? (uint32_t*)d_stash_ : nullptr;
    V.next = next;
    V.ntiles = (uint32_t)vtiles_.size();
    prof_begin(prof, POSLO_KT_VERIFY, s);
    if (emitted_ && fq)
        hipLaunchKernelGGL(k_batch_verify_pre<true>, dim3(grid), dim3(64), 0, s, V);
    else if (emitted_)
        hipLaunchKernelGGL(k_batch_verify_pre<false>, dim3(grid), dim3(64), 0, s, V);
    else
        hipLaunchKernelGGL(k_batch_verify, dim3((uint32_t)vtiles_.size()), dim3(256), 0, s, V);
    prof_end(prof, POSLO_KT_VERIFY, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h_misc_, cnt, 4, hipMemcpyDeviceToHost, s));
    return POSLO_OK;
}

int BatchRunner::invalid(std::vector<std::pair<uint32_t, uint64_t>>& out, hipStream_t s) {
    out.clear();
    if (vtiles_.empty()) return POSLO_OK;
    uint64_t count = (uint32_t)h_misc_[0];
    if (count > n_checked_) return POSLO_E_DEVICE;
    std::vector<uint64_t> slots(count);
    if (count) {
        HIP_TRY(hipMemcpyAsync(slots.data(), d_idx_, count * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    std::sort(slots.begin(), slots.end());
    out.reserve(count);
    for (uint64_t sl : slots) {
        auto it = std::upper_bound(vbase_.begin(), vbase_.end(), std::make_pair(sl, UINT32_MAX));
        uint32_t j = std::prev(it)->second;
        out.push_back({j, jobs_[j].t0 + (sl - jobs_[j].vbase)});
    }
    std::sort(out.begin(), out.end());
    return POSLO_OK;
}

}  // namespace poslo

// ===========================================================================
// synchronous entry points over a global entry layout
// ===========================================================================

using namespace poslo;

namespace {

struct BatchState {
    BatchRunner runner;
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, poslo_tuning> tuned;  // (inst, log2 mean L, log2 n)
};

std::map<poslo_ctx*, BatchState*>& states() {
    static std::map<poslo_ctx*, BatchState*> m;
    return m;
}

BatchState& state_of(poslo_ctx* c) {
    auto& m = states();
    auto it = m.find(c);
    if (it != m.end()) return *it->second;
    BatchState* s = new BatchState();
    m[c] = s;
    return *s;
}

uint32_t ilog2(uint64_t v) {
    uint32_t r = 0;
    while (v > 1) {
        v >>= 1;
        r++;
    }
    return r;
}

std::tuple<uint32_t, uint32_t, uint32_t> shape_class(const poslo_params* prm, uint64_t n_total, uint64_t bytes) {
    uint64_t mean = n_total ? bytes / n_total : 0;
    return {prm->inst, ilog2(mean + 1), ilog2(n_total + 1)};
}

// resolve keys and express the global layout as per-job views
int make_specs(poslo_ctx* c, bool fourq, const poslo_batch_job* jobs, uint32_t njobs, const uint8_t* data,
               const uint64_t* offsets, uint64_t data_bytes, const uint8_t* sigs, std::vector<JobSpec>& specs) {
    std::vector<uint8_t> pks((size_t)njobs * 32);
    for (uint32_t j = 0; j < njobs; j++) {
        if (!jobs[j].pk || !jobs[j].tag) return POSLO_E_INVAL;
        if (jobs[j].n && (!data || !offsets)) return POSLO_E_INVAL;
        if (jobs[j].entry_base > UINT64_MAX / 80 - jobs[j].n) return POSLO_E_INVAL;
        memcpy(&pks[(size_t)j * 32], jobs[j].pk, 32);
    }
    std::vector<const uint32_t*> tables;
    int st = ctx_keys_bulk(c, pks.data(), njobs, tables, nullptr, fourq);
    if (st) return st;
    specs.resize(njobs);
    for (uint32_t j = 0; j < njobs; j++) {
        const poslo_batch_job& in = jobs[j];
        JobSpec& sp = specs[j];
        sp.ty = tables[j];
        sp.tyw = fourq ? nullptr : ctx_key_wide_resident(c, jobs[j].pk);
        sp.data = data;
        sp.offsets = offsets ? offsets + in.entry_base : nullptr;
        sp.msg_len = 0;
        sp.data_bytes = data_bytes;
        sp.sigs = sigs ? sigs + 80 * in.entry_base : nullptr;
        sp.t0 = in.t0;
        sp.n = in.n;
        sp.ds = in.ds;
        sp.ds_len = in.ds_len;
        sp.tag = in.tag;
    }
    return POSLO_OK;
}

int run_sync(poslo_ctx* c, BatchRunner& R, const poslo_params* prm, const std::vector<JobSpec>& specs,
             const poslo_tuning& t, hipStream_t s, uint8_t* accept, bool emit = false) {
    int st = R.plan(prm, specs.data(), (uint32_t)specs.size(), t, c->num_cu);
    if (st) return st;
    if ((st = R.launch(s, t.use_graph != 0, c, emit))) return st;
    HIP_TRY(hipStreamSynchronize(s));
    prof_collect(c);
    for (uint32_t j = 0; j < R.njobs(); j++) accept[j] = (uint8_t)R.accept(j);
    return POSLO_OK;
}

}  // namespace

namespace poslo {

void batch_release(poslo_ctx* c) {
    auto& m = states();
    auto it = m.find(c);
    if (it == m.end()) return;
    hipDeviceSynchronize();
    delete it->second;
    m.erase(it);
}

}  // namespace poslo

extern "C" int poslo_batch_variant_count(void) { return kNumHot; }

extern "C" const char* poslo_batch_variant_name(int v) { return (v < 0 || v >= kNumHot) ? nullptr : kHot[v].name; }

extern "C" int poslo_verify_batch(poslo_ctx* c, const poslo_params* prm, const poslo_batch_job* jobs, uint32_t njobs,
                                  const uint8_t* data, const uint64_t* offsets, uint64_t data_bytes,
                                  const uint8_t* sigs, int distill, const poslo_tuning* tuning, void* stream,
                                  uint8_t* accept, uint64_t* invalid, size_t cap, size_t* n_invalid) {
    if (!c || !params_ok(prm) || !batch_inst_ok(prm->inst) || (njobs && (!jobs || !accept)) || distill < 0 ||
        distill > 2)
        return POSLO_E_INVAL;
    if (distill && (!sigs || !n_invalid || (cap && !invalid))) return POSLO_E_INVAL;
    if (n_invalid) *n_invalid = 0;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    // tuning: explicit, else the autotuner's cached choice, else the default
    poslo_tuning t;
    if (tuning) {
        t = *tuning;
    } else {
        t.variant = batch_default_variant(prm->inst);
        t.wg_per_cu = 0;
        t.use_graph = 0;
        t.reserved = 0;
        uint64_t n_total = 0;
        for (uint32_t j = 0; j < njobs; j++) n_total += jobs[j].n;
        auto& tuned = state_of(c).tuned;
        auto it = tuned.find(shape_class(prm, n_total, data_bytes));
        if (it != tuned.end()) t = it->second;
    }
    std::vector<JobSpec> specs;
    int st = make_specs(c, (prm->inst & POSLO_GROUP_FOURQ) != 0, jobs, njobs, data, offsets, data_bytes, sigs, specs);
    if (st) return st;
    BatchRunner& R = state_of(c).runner;
    if ((st = run_sync(c, R, prm, specs, t, s, accept, distill != 0))) return st;
    if (!distill) return POSLO_OK;
    std::vector<uint32_t> which;
    for (uint32_t j = 0; j < njobs; j++)
        if (!accept[j] || distill == 2) which.push_back(j);
    if ((st = R.launch_verify(which, s, c))) return st;
    HIP_TRY(hipStreamSynchronize(s));
    prof_collect(c);
    std::vector<std::pair<uint32_t, uint64_t>> out;
    if ((st = R.invalid(out, s))) return st;
    *n_invalid = out.size();
    if (out.size() > cap) return POSLO_OK;  // caller sees the count and may retry with room
    for (size_t k = 0; k < out.size(); k++) {
        invalid[2 * k] = out[k].first;
        invalid[2 * k + 1] = out[k].second;
    }
    return POSLO_OK;
}

extern "C" int poslo_autotune_batch(poslo_ctx* c, const poslo_params* prm, const poslo_batch_job* jobs, uint32_t njobs,
                                    const uint8_t* data, const uint64_t* offsets, uint64_t data_bytes, int reps,
                                    void* stream, poslo_tuning* best, double* best_ms) {
    if (!c || !params_ok(prm) || !batch_inst_ok(prm->inst) || !best || njobs == 0 || !jobs) return POSLO_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    if (reps < 1) reps = 3;
    std::vector<JobSpec> specs;
    int st = make_specs(c, (prm->inst & POSLO_GROUP_FOURQ) != 0, jobs, njobs, data, offsets, data_bytes, nullptr,
                        specs);
    if (st) return st;
    BatchRunner& R = state_of(c).runner;
    std::vector<uint8_t> acc_ref(njobs), acc(njobs);
    double best_t = 1e30;
    poslo_tuning bt{-1, 0, 0, 0};
    bool have_ref = false;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto done = [&](int code) {
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        return code;
    };
    for (int v = 0; v < kNumHot; v++) {
        if (kHot[v].inst != (int)inst_base(prm->inst)) continue;
        for (int wg : {0, 1, 2, 4}) {
            if (wg > 0 && wg * (kHot[v].block / 64) > 4 * kHot[v].waves_per_simd) continue;
            if (wg > 0 && (size_t)wg * (hot_lds_bytes(kHot[v]) + 512) > 160 * 1024) continue;
            poslo_tuning t{v, wg, 0, 0};
            if ((st = run_sync(c, R, prm, specs, t, s, acc.data()))) return done(st);
            // every candidate must agree on every job's verdict
            if (!have_ref) {
                acc_ref = acc;
                have_ref = true;
            } else if (acc != acc_ref) {
                return done(POSLO_E_DEVICE);
            }
            double total = 0;
            for (int r = 0; r < reps; r++) {
                hipEventRecord(e0, s);
                if ((st = run_sync(c, R, prm, specs, t, s, acc.data()))) return done(st);
                hipEventRecord(e1, s);
                hipEventSynchronize(e1);
                float ms = 0;
                hipEventElapsedTime(&ms, e0, e1);
                total += ms;
            }
            if (total / reps < best_t) {
                best_t = total / reps;
                bt = t;
            }
        }
    }
    done(0);
    uint64_t n_total = 0;
    for (uint32_t j = 0; j < njobs; j++) n_total += jobs[j].n;
    state_of(c).tuned[shape_class(prm, n_total, data_bytes)] = bt;
    *best = bt;
    if (best_ms) *best_ms = best_t;
    return POSLO_OK;
}

extern "C" int poslo_batch_forget(poslo_ctx* c) {
    if (!c) return POSLO_E_INVAL;
    batch_release(c);
    return POSLO_OK;
}
