// Batched verification of many signers' batches in one persistent launch.
//
// Each signer's batch is a job: its own key, entry range, ds and tag (the
// paper verifies one batch per launch; section "POSLO Parallel Batch
// Verification").  Jobs are cut into work items of up to CHUNK entries that
// never straddle a job.  A persistent grid of workgroups pulls items from an
// atomic counter until the queue is empty; each item's entries are sorted
// inside the workgroup by MDC-2/SHA block count (a counting sort in LDS), so
// that the 64 lanes of a wave hash messages of similar length; digests are
// summed lazily into one 288-bit partial per item.  A second kernel folds
// each job's partials, reduces mod q and checks the job's tag with one wave
// (comb tables).  Jobs that fail can be distilled: their entries are verified
// individually and the invalid ones reported as (job, t) pairs.
//
// The sequence (seed rows -> persistent hashing -> per-job checks -> result
// copy) can be captured in a hipGraph and replayed; an autotuner times the
// kernel variants on the caller's batch and caches the fastest per shape.
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "aes_perm.h"
#include "ctx.h"
#include "device_verify.h"
#include "scheme_host.h"

namespace poslo {

struct BJob {
    const uint32_t* ty;  // comb table of the job's key
    uint64_t t0, n;
    uint64_t entry_base;  // first entry in the global offsets array
    uint64_t epoch_base;  // first row of the epoch table
    uint64_t item_base, item_end;
    uint32_t tag[16];     // LE words: s[8] || R bytes[8]
};

struct BItem {
    uint32_t job;
    uint32_t count;
    uint64_t first;  // entry offset within the job
};

struct BHot {
    const BJob* jobs;
    const BItem* items;
    uint32_t n_items;
    uint32_t log2_n2;
    const uint8_t* data;
    const uint64_t* offsets;
    const uint8_t* end;
    const uint32_t* tab;
    uint32_t* counter;
    uint32_t* partials;  // 9 words per item
};

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
    uint32_t* rdec;  // 17 words per job: ok, x[8], y[8]
};

__global__ __launch_bounds__(256) void k_batch_seeds(BSeeds S) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
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
        ge R;
        bool ok = sc_is_canonical(sv) && ge_decode(R, rb);
        uint32_t* o = S.rdec + (uint64_t)j * 17;
        o[0] = ok ? 1u : 0u;
        for (int k = 0; k < 8; k++) {
            o[1 + k] = ok ? R.X.v[k] : 0u;
            o[9 + k] = ok ? R.Y.v[k] : 0u;
        }
        return;
    }
    LdsTables<4, 1> tb{lds};
    uint64_t row = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row == 0) S.counter[0] = 0;
    if (row >= S.n_rows) return;
    uint32_t j = S.job_of_row[row];
    const BJob& J = S.jobs[j];
    const DsArg& D = S.ds[j];
    uint64_t i = (J.t0 >> S.log2_n2) + (row - J.epoch_base);
    int k = ds_cover(D, i);
    if (k < 0) k = 0;  // coverage validated on the host
    uint32_t x[4] = {D.v[k][0], D.v[k][1], D.v[k][2], D.v[k][3]};
    for (int bt = (int)D.depth[k] - 1; bt >= 0; bt--) {
        uint32_t bit = (uint32_t)((i >> bt) & 1u), nx[4];
        if (S.inst == INST_AES)
            prf_node_aes(tb, x, bit, nx);
        else
            prf_node_sha(x, bit, nx);
        x[0] = nx[0], x[1] = nx[1], x[2] = nx[2], x[3] = nx[3];
    }
    uint32_t* e = S.tab + row * kEpochWords;
    if (S.inst == INST_AES) {
        uint32_t st[4] = {x[0], x[1], x[2], x[3]};
        aes128_encrypt_rk(tb, c_iv.a, st);
        uint32_t h1[4] = {st[0] ^ x[0], st[1] ^ x[1], st[2] ^ x[2], st[3] ^ x[3]};
        uint32_t rk[44];
        aes128_expand(tb, h1, rk);
        for (int w = 0; w < 44; w++) e[w] = rk[w];
    }
    for (int w = 0; w < 4; w++) e[44 + w] = x[w];
}

// ---- the persistent hashing kernel ------------------------------------------

__device__ __forceinline__ BatchArgs job_args(const BHot& A, const BJob& J) {
    BatchArgs a;
    a.data = A.data;
    a.offsets = A.offsets + J.entry_base;
    a.msg_len = 0;
    a.n = J.n;
    a.t0 = J.t0;
    a.epoch_first = J.t0 >> A.log2_n2;
    a.log2_n2 = A.log2_n2;
    a.tab = A.tab + J.epoch_base * kEpochWords;
    a.skip = nullptr;
    a.end = A.end;
    return a;
}

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

// INST 1: MDC-2-AES over the byte-addressed tables (NT = 1 or 2);
// INST 0: SHA-256 (no tables).  CHUNK entries per item at most.
template <int INST, int NT, int BLOCK, int CHUNK, bool SORT, int WPE>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void k_batch_hot(BHot A) {
    constexpr int TW = INST == INST_AES ? NT * 256 * 64 : 0;  // table words
    constexpr int SW = 64 + 16 + CHUNK / 2 + CHUNK / 4;       // counts, misc, order (u16), keys (u8)
    __shared__ uint32_t lds[TW + SW + (BLOCK / 64) * 9];
    if constexpr (INST == INST_AES) {
        perm_tables_fill<NT>(lds);
    }
    uint32_t* counts = lds + TW;                                   // 64 bucket counters
    uint32_t* misc = counts + 64;                                  // [0] item id
    uint16_t* order = reinterpret_cast<uint16_t*>(misc + 16);      // CHUNK slots
    uint8_t* keys = reinterpret_cast<uint8_t*>(order + CHUNK);     // CHUNK block counts
    uint32_t* red = lds + TW + SW;
    const PermTables<NT> tb = perm_tables<NT>(lds);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) misc[0] = atomicAdd(A.counter, 1u);
        if (SORT && threadIdx.x < 64) counts[threadIdx.x] = 0;
        __syncthreads();
        const uint32_t item = misc[0];
        if (item >= A.n_items) break;
        const BItem it = A.items[item];
        const BJob J = A.jobs[it.job];
        const BatchArgs a = job_args(A, J);
        if (SORT) {
            // counting sort of the item's slots by block count
            for (uint32_t s = threadIdx.x; s < it.count; s += BLOCK) {
                uint64_t p = it.first + s;
                uint64_t L = a.offsets[p + 1] - a.offsets[p];
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
        uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (uint32_t s = threadIdx.x; s < it.count; s += BLOCK) {
            uint64_t p = it.first + (SORT ? order[s] : s);
            EntryView ev = entry_view(a, p);
            uint32_t x[4], dig[8];
            if constexpr (INST == INST_AES) {
                uint64_t t = a.t0 + p;
                uint32_t jj = (uint32_t)(t & ((1ull << a.log2_n2) - 1));
                const uint32_t* rk = a.tab + ((t >> a.log2_n2) - a.epoch_first) * kEpochWords;
                x[0] = jj, x[1] = 0, x[2] = 0, x[3] = 0;
                penc_rk(tb, rk, x);
                x[0] ^= jj;
                digest_mdc2_any(tb, ev, a.end, x, dig, Mdc2BlockPerm{});
            } else {
                one_time_seed_sha(a, p, x);
                digest_sha_any(ev, a.end, x, dig);
            }
            acc288_add256(acc, dig);
        }
        block_reduce288_scratch<BLOCK>(acc, A.partials + (uint64_t)item * 9, red);
    }
}

// ---- per-job checks: one wave per job ----------------------------------------

__global__ __launch_bounds__(64) void k_batch_final(const BJob* jobs, const uint32_t* partials, const uint32_t* tg,
                                                    const uint32_t* rdec, uint32_t* result) {
    const BJob& J = jobs[blockIdx.x];
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t k = J.item_base + threadIdx.x; k < J.item_end; k += 64) acc288_add(acc, partials + k * 9);
    wave_reduce288(acc);  // every lane holds the sum
    uint32_t e[8], s[8];
    sc_reduce288(e, acc);
    for (int k = 0; k < 8; k++) s[k] = J.tag[k];
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

// ---- individual verification of the entries of failing jobs ----------------

struct BVerify {
    const BJob* jobs;
    const BItem* tiles;  // up to 256 entries each
    const uint8_t* sigs;  // 80 bytes per global entry
    const uint32_t* tg;
    uint32_t inst;
    uint32_t log2_n2;
    const uint8_t* data;
    const uint64_t* offsets;
    const uint8_t* end;
    const uint32_t* tab;
    uint8_t* flags;  // per global entry, 1 = invalid (entries of verified jobs only)
};

__global__ __launch_bounds__(256) void k_batch_verify(BVerify V) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
    LdsTables<4, 1> tb{lds};
    const BItem it = V.tiles[blockIdx.x];
    if (threadIdx.x >= it.count) return;
    const BJob J = V.jobs[it.job];
    BHot A;
    A.data = V.data;
    A.offsets = V.offsets;
    A.end = V.end;
    A.tab = V.tab;
    A.log2_n2 = V.log2_n2;
    BatchArgs a = job_args(A, J);
    uint64_t p = it.first + threadIdx.x;
    uint64_t g = J.entry_base + p;
    uint32_t e[8], s[8];
    bool ok = verify_one(tb, a, a.end, V.inst, p, V.sigs + g * 80, J.ty, V.tg, e, s);
    V.flags[g] = ok ? 0 : 1;
}

__global__ void k_fill_u8(uint8_t* p, uint64_t n) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// global entries flagged invalid, in order (per-thread counts, a scan, writes)
__global__ __launch_bounds__(1024) void k_batch_compact(const uint8_t* flags, uint64_t n, uint64_t* out_idx,
                                                        uint64_t* out_count) {
    __shared__ uint64_t scan[1024];
    uint64_t chunk = (n + 1023) / 1024;
    uint64_t a = (uint64_t)threadIdx.x * chunk, b = a + chunk < n ? a + chunk : n;
    uint64_t cnt = 0;
    for (uint64_t p = a; p < b; p++) cnt += flags[p];
    scan[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint64_t v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t o = scan[threadIdx.x] - cnt;
    for (uint64_t p = a; p < b; p++)
        if (flags[p]) out_idx[o++] = p;
    if (threadIdx.x == 1023) *out_count = scan[1023];
}

// ---- tuning --------------------------------------------------------------------

struct HotVariant {
    const char* name;
    int inst, nt, block, chunk, sort, waves_per_simd;
};

static const HotVariant kHot[] = {
    {"aes_perm2_b1024_c1024_sorted", 1, 2, 1024, 1024, 1, 4}, {"aes_perm2_b1024_c2048_sorted", 1, 2, 1024, 2048, 1, 4},
    {"aes_perm2_b1024_c1024", 1, 2, 1024, 1024, 0, 4},        {"aes_perm1_b1024_c1024_sorted", 1, 1, 1024, 1024, 1, 4},
    {"aes_perm1_b512_c1024_sorted", 1, 1, 512, 1024, 1, 4},   {"sha_b256_c1024_sorted_w3", 0, 1, 256, 1024, 1, 3},
    {"sha_b256_c1024_sorted_w4", 0, 1, 256, 1024, 1, 4},      {"sha_b256_c256_sorted_w3", 0, 1, 256, 256, 1, 3},
    {"sha_b256_c1024_w3", 0, 1, 256, 1024, 0, 3},             {"sha_b512_c2048_sorted_w3", 0, 1, 512, 2048, 1, 3},
};
constexpr int kNumHot = sizeof kHot / sizeof kHot[0];

static size_t hot_lds_bytes(const HotVariant& v) {
    size_t tw = v.inst == 1 ? (size_t)v.nt * 256 * 64 : 0;
    return 4 * (tw + 64 + 16 + v.chunk / 2 + v.chunk / 4 + (v.block / 64) * 9);
}

static int launch_hot(int v, uint32_t grid, const BHot& A, hipStream_t s) {
#define HOT(I, NT, B, C, S, W)                                                                  \
    hipLaunchKernelGGL((k_batch_hot<I, NT, B, C, S, W>), dim3(grid), dim3(B), 0, s, A); \
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
        default: return POSLO_E_INVAL;
    }
#undef HOT
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

static uint32_t hot_wg_per_cu(const HotVariant& v, int override_wg) {
    if (override_wg > 0) return (uint32_t)override_wg;
    uint32_t by_lds = (uint32_t)((160 * 1024) / (hot_lds_bytes(v) + 512));
    uint32_t by_waves = 4 * v.waves_per_simd / (v.block / 64);
    return std::max<uint32_t>(1, std::min(by_lds, by_waves));
}

}  // namespace poslo

// ===========================================================================
// host side
// ===========================================================================

using namespace poslo;
using namespace poslo::hostside;

namespace {

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

enum { X_JOBS = 16, X_DS, X_ROWS, X_ITEMS, X_TAB, X_PART, X_RESULT, X_TILES, X_FLAGS, X_IDX, X_MISC, X_RDEC };

struct Plan {
    std::vector<BJob> jobs;
    std::vector<DsArg> ds;
    std::vector<uint32_t> job_of_row;
    std::vector<BItem> items;
    uint64_t n_total = 0;
};

// job table, per-epoch rows and work items on the host
int make_plan(poslo_ctx* c, const poslo_params* prm, const poslo_batch_job* jobs, uint32_t njobs, uint32_t chunk,
              Plan& P) {
    P.jobs.resize(njobs);
    P.ds.resize(njobs);
    P.job_of_row.clear();
    P.items.clear();
    P.n_total = 0;
    uint64_t nmax = 1ull << (prm->log2_n1 + prm->log2_n2);
    std::vector<uint8_t> pks((size_t)njobs * 32);
    for (uint32_t j = 0; j < njobs; j++) {
        const poslo_batch_job& in = jobs[j];
        if (!in.pk || !in.tag || in.t0 > nmax || in.n > nmax - in.t0 || in.n >= (1ull << 32)) return POSLO_E_INVAL;
        if (in.entry_base > UINT64_MAX - in.n) return POSLO_E_INVAL;
        memcpy(&pks[(size_t)j * 32], in.pk, 32);
    }
    std::vector<const uint32_t*> tables;
    int st = ctx_keys_bulk(c, pks.data(), njobs, tables, nullptr);
    if (st) return st;
    std::vector<DsNode> nodes;
    for (uint32_t j = 0; j < njobs; j++) {
        const poslo_batch_job& in = jobs[j];
        if (!ds_parse(in.ds, in.ds_len, nodes)) return POSLO_E_INVAL;
        DsArg& d = P.ds[j];
        memset(&d, 0, sizeof d);
        d.count = (uint32_t)nodes.size();
        for (size_t k = 0; k < nodes.size(); k++) {
            d.depth[k] = nodes[k].depth;
            d.index[k] = nodes[k].index;
            for (int w = 0; w < 4; w++) d.v[k][w] = load_le32(nodes[k].v + 4 * w);
        }
        BJob& J = P.jobs[j];
        J.ty = tables[j];
        J.t0 = in.t0;
        J.n = in.n;
        J.entry_base = in.entry_base;
        J.epoch_base = P.job_of_row.size();
        J.item_base = P.items.size();
        for (int k = 0; k < 16; k++) J.tag[k] = load_le32(in.tag + 4 * k);
        if (in.n) {
            uint64_t e0 = in.t0 >> prm->log2_n2, e1 = (in.t0 + in.n - 1) >> prm->log2_n2;
            for (uint64_t e = e0; e <= e1; e++) {
                if (sr_node(nodes.data(), (int)nodes.size(), e) < 0) return POSLO_E_SEED;
                P.job_of_row.push_back(j);
            }
            for (uint64_t f = 0; f < in.n; f += chunk)
                P.items.push_back(BItem{j, (uint32_t)std::min<uint64_t>(chunk, in.n - f), f});
        }
        J.item_end = P.items.size();
        P.n_total = std::max(P.n_total, in.entry_base + in.n);
    }
    if (P.job_of_row.size() >= (1ull << 32) || P.items.size() >= (1ull << 32)) return POSLO_E_INVAL;
    return POSLO_OK;
}

template <class V>
int upload(poslo_ctx* c, int slot, const V& v, hipStream_t s, void** out) {
    size_t bytes = std::max<size_t>(v.size() * sizeof(v[0]), 16);
    int st = ctx_scratch(c, slot, bytes, out);
    if (st) return st;
    if (!v.empty() && hipMemcpyAsync(*out, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice, s) != hipSuccess)
        return POSLO_E_DEVICE;
    return POSLO_OK;
}

struct BatchState {
    // instantiated graphs keyed by the bytes of every launch argument
    std::map<std::string, hipGraphExec_t> graphs;
    hipStream_t capture = nullptr;  // private stream that graphs are captured on
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

template <class T>
void key_bytes(std::string& k, const T& v) {
    k.append(reinterpret_cast<const char*>(&v), sizeof v);
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

int default_variant(uint32_t inst) { return inst == POSLO_INST_AES ? 0 : 5; }

// the pipeline: seeds and tag decode -> persistent hashing -> per-job checks
int run_batch(poslo_ctx* c, const poslo_params* prm, const poslo_batch_job* jobs, uint32_t njobs, const uint8_t* data,
              const uint64_t* offsets, uint64_t data_bytes, const poslo_tuning& tune, hipStream_t s, uint8_t* accept,
              Plan& P, void** d_jobs_out, void** d_tab_out) {
    const HotVariant& hv = kHot[tune.variant];
    if ((uint32_t)hv.inst != prm->inst) return POSLO_E_INVAL;
    int st = make_plan(c, prm, jobs, njobs, (uint32_t)hv.chunk, P);
    if (st) return st;
    void *d_jobs, *d_ds, *d_rows, *d_items, *d_tab, *d_part, *d_res, *d_misc, *d_rdec;
    if ((st = upload(c, X_JOBS, P.jobs, s, &d_jobs)) || (st = upload(c, X_DS, P.ds, s, &d_ds)) ||
        (st = upload(c, X_ROWS, P.job_of_row, s, &d_rows)) || (st = upload(c, X_ITEMS, P.items, s, &d_items)) ||
        (st = ctx_scratch(c, X_TAB, std::max<size_t>(P.job_of_row.size(), 1) * kEpochWords * 4, &d_tab)) ||
        (st = ctx_scratch(c, X_PART, std::max<size_t>(P.items.size(), 1) * 36, &d_part)) ||
        (st = ctx_scratch(c, X_RESULT, std::max<size_t>(njobs, 1) * 4, &d_res)) ||
        (st = ctx_scratch(c, X_MISC, 256, &d_misc)) ||
        (st = ctx_scratch(c, X_RDEC, std::max<size_t>(njobs, 1) * 17 * 4, &d_rdec)))
        return st;
    *d_jobs_out = d_jobs;
    *d_tab_out = d_tab;
    BSeeds S;
    memset(&S, 0, sizeof S);
    S.jobs = (const BJob*)d_jobs;
    S.ds = (const DsArg*)d_ds;
    S.job_of_row = (const uint32_t*)d_rows;
    S.n_rows = P.job_of_row.size();
    S.row_blocks = (uint32_t)std::max<uint64_t>(1, (S.n_rows + 255) / 256);
    S.njobs = njobs;
    S.log2_n2 = prm->log2_n2;
    S.inst = prm->inst;
    S.tab = (uint32_t*)d_tab;
    S.counter = (uint32_t*)d_misc;
    S.rdec = (uint32_t*)d_rdec;
    uint32_t seed_grid = S.row_blocks + (njobs + 255) / 256;
    uint32_t grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(P.items.size(), (uint64_t)c->num_cu * hot_wg_per_cu(hv, tune.wg_per_cu)));
    BHot A;
    memset(&A, 0, sizeof A);
    A.jobs = (const BJob*)d_jobs;
    A.items = (const BItem*)d_items;
    A.n_items = (uint32_t)P.items.size();
    A.log2_n2 = prm->log2_n2;
    A.data = data;
    A.offsets = offsets;
    A.end = data_bytes ? data + data_bytes : nullptr;
    A.tab = (const uint32_t*)d_tab;
    A.counter = (uint32_t*)d_misc;
    A.partials = (uint32_t*)d_part;
    auto launch_all = [&](hipStream_t q, bool timed) -> int {
        hipLaunchKernelGGL(k_batch_seeds, dim3(seed_grid), dim3(256), 0, q, S);
        if (timed) prof_begin(c, POSLO_KT_BATCH_HOT, q);
        int r = launch_hot(tune.variant, grid, A, q);
        if (timed) prof_end(c, POSLO_KT_BATCH_HOT, q);
        if (r) return r;
        if (njobs)
            hipLaunchKernelGGL(k_batch_final, dim3(njobs), dim3(64), 0, q, (const BJob*)d_jobs,
                               (const uint32_t*)d_part, c->d_gtable, (const uint32_t*)d_rdec, (uint32_t*)d_res);
        return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
    };
    prof_begin(c, POSLO_KT_BATCH, s);
    if (tune.use_graph) {
        std::string gk;
        key_bytes(gk, S);
        key_bytes(gk, A);
        key_bytes(gk, seed_grid);
        key_bytes(gk, grid);
        key_bytes(gk, tune.variant);
        key_bytes(gk, c->d_gtable);
        key_bytes(gk, d_res);
        BatchState& bs = state_of(c);
        auto it = bs.graphs.find(gk);
        hipGraphExec_t exec = nullptr;
        if (it != bs.graphs.end()) {
            exec = it->second;
        } else {
            if (bs.graphs.size() >= 64) {
                HIP_TRY(hipStreamSynchronize(s));
                for (auto& g : bs.graphs) hipGraphExecDestroy(g.second);
                bs.graphs.clear();
            }
            if (!bs.capture) HIP_TRY(hipStreamCreateWithFlags(&bs.capture, hipStreamNonBlocking));
            HIP_TRY(hipStreamBeginCapture(bs.capture, hipStreamCaptureModeThreadLocal));
            int r = launch_all(bs.capture, false);
            hipGraph_t g = nullptr;
            hipError_t ec = hipStreamEndCapture(bs.capture, &g);
            if (r || ec != hipSuccess) {
                if (g) hipGraphDestroy(g);
                return r ? r : POSLO_E_DEVICE;
            }
            hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            hipGraphDestroy(g);
            if (ei != hipSuccess) return POSLO_E_DEVICE;
            bs.graphs[gk] = exec;
        }
        HIP_TRY(hipGraphLaunch(exec, s));
    } else {
        if ((st = launch_all(s, true))) return st;
    }
    prof_end(c, POSLO_KT_BATCH, s);
    std::vector<uint32_t> res(std::max<uint32_t>(njobs, 1));
    if (njobs) HIP_TRY(hipMemcpyAsync(res.data(), d_res, njobs * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    prof_collect(c);
    for (uint32_t j = 0; j < njobs; j++) accept[j] = (uint8_t)res[j];
    return POSLO_OK;
}

}  // namespace

extern "C" int poslo_batch_variant_count(void) { return kNumHot; }

extern "C" const char* poslo_batch_variant_name(int v) { return (v < 0 || v >= kNumHot) ? nullptr : kHot[v].name; }

extern "C" int poslo_verify_batch(poslo_ctx* c, const poslo_params* prm, const poslo_batch_job* jobs, uint32_t njobs,
                                  const uint8_t* data, const uint64_t* offsets, uint64_t data_bytes,
                                  const uint8_t* sigs, int distill, const poslo_tuning* tuning, void* stream,
                                  uint8_t* accept, uint64_t* invalid, size_t cap, size_t* n_invalid) {
    if (!c || !params_ok(prm) || (njobs && (!jobs || !accept)) || !offsets || distill < 0 || distill > 2)
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
        t.variant = default_variant(prm->inst);
        t.wg_per_cu = 0;
        t.use_graph = 0;
        uint64_t n_total = 0;
        for (uint32_t j = 0; j < njobs; j++) n_total += jobs[j].n;
        auto& tuned = state_of(c).tuned;
        auto it = tuned.find(shape_class(prm, n_total, data_bytes));
        if (it != tuned.end()) t = it->second;
    }
    if (t.variant < 0 || t.variant >= kNumHot || kHot[t.variant].inst != (int)prm->inst) return POSLO_E_INVAL;
    Plan P;
    void *d_jobs, *d_tab;
    int st = run_batch(c, prm, jobs, njobs, data, offsets, data_bytes, t, s, accept, P, &d_jobs, &d_tab);
    if (st) return st;
    if (!distill) return POSLO_OK;
    // individual verification of the entries of the rejected jobs (mode 1)
    // or of every job (mode 2)
    std::vector<BItem> tiles;
    for (uint32_t j = 0; j < njobs; j++) {
        if (accept[j] && distill == 1) continue;
        for (uint64_t f = 0; f < jobs[j].n; f += 256)
            tiles.push_back(BItem{j, (uint32_t)std::min<uint64_t>(256, jobs[j].n - f), f});
    }
    if (tiles.empty()) return POSLO_OK;
    void *d_tiles, *d_flags, *d_idx, *d_misc;
    uint64_t nt = P.n_total;
    if ((st = upload(c, X_TILES, tiles, s, &d_tiles)) || (st = ctx_scratch(c, X_FLAGS, std::max<uint64_t>(nt, 1), &d_flags)) ||
        (st = ctx_scratch(c, X_IDX, std::max<uint64_t>(nt, 1) * 8, &d_idx)) || (st = ctx_scratch(c, X_MISC, 256, &d_misc)))
        return st;
    hipLaunchKernelGGL(k_fill_u8, dim3((uint32_t)((nt + 255) / 256)), dim3(256), 0, s, (uint8_t*)d_flags, nt);
    BVerify V;
    V.jobs = (const BJob*)d_jobs;
    V.tiles = (const BItem*)d_tiles;
    V.sigs = sigs;
    V.tg = c->d_gtable;
    V.inst = prm->inst;
    V.log2_n2 = prm->log2_n2;
    V.data = data;
    V.offsets = offsets;
    V.end = data_bytes ? data + data_bytes : nullptr;
    V.tab = (const uint32_t*)d_tab;
    V.flags = (uint8_t*)d_flags;
    prof_begin(c, POSLO_KT_VERIFY, s);
    hipLaunchKernelGGL(k_batch_verify, dim3((uint32_t)tiles.size()), dim3(256), 0, s, V);
    hipLaunchKernelGGL(k_batch_compact, dim3(1), dim3(1024), 0, s, (const uint8_t*)d_flags, nt, (uint64_t*)d_idx,
                       (uint64_t*)d_misc + 8);
    HIP_TRY(hipGetLastError());
    prof_end(c, POSLO_KT_VERIFY, s);
    uint64_t count = 0;
    HIP_TRY(hipMemcpyAsync(&count, (uint64_t*)d_misc + 8, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    prof_collect(c);
    *n_invalid = count;
    if (count > cap) return POSLO_OK;  // caller sees the count and may retry with room
    std::vector<uint64_t> g(count);
    if (count) {
        HIP_TRY(hipMemcpyAsync(g.data(), d_idx, count * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    // global entry -> (job, t): jobs' entry ranges may come in any order
    std::vector<std::pair<uint64_t, uint32_t>> starts(njobs);
    for (uint32_t j = 0; j < njobs; j++) starts[j] = {jobs[j].entry_base, j};
    std::sort(starts.begin(), starts.end());
    std::vector<std::pair<uint32_t, uint64_t>> out;
    out.reserve(count);
    for (uint64_t gi : g) {
        auto it = std::upper_bound(starts.begin(), starts.end(), std::make_pair(gi, UINT32_MAX));
        uint32_t j = std::prev(it)->second;
        out.push_back({j, jobs[j].t0 + (gi - jobs[j].entry_base)});
    }
    std::sort(out.begin(), out.end());
    for (size_t k = 0; k < out.size(); k++) {
        invalid[2 * k] = out[k].first;
        invalid[2 * k + 1] = out[k].second;
    }
    return POSLO_OK;
}

extern "C" int poslo_autotune_batch(poslo_ctx* c, const poslo_params* prm, const poslo_batch_job* jobs, uint32_t njobs,
                                    const uint8_t* data, const uint64_t* offsets, uint64_t data_bytes, int reps,
                                    void* stream, poslo_tuning* best, double* best_ms) {
    if (!c || !params_ok(prm) || !best || njobs == 0) return POSLO_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    if (reps < 1) reps = 3;
    std::vector<uint8_t> acc_ref(njobs), acc(njobs);
    double best_t = 1e30;
    poslo_tuning bt{-1, 0, 0, 0};
    bool have_ref = false;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    for (int v = 0; v < kNumHot; v++) {
        if (kHot[v].inst != (int)prm->inst) continue;
        for (int wg : {0, 1, 2, 4}) {
            if (wg > 0 && wg * (kHot[v].block / 64) > 4 * kHot[v].waves_per_simd) continue;
            if (wg > 0 && (size_t)wg * (hot_lds_bytes(kHot[v]) + 512) > 160 * 1024) continue;
            poslo_tuning t{v, wg, 0, 0};
            Plan P;
            void *dj, *dt;
            int st = run_batch(c, prm, jobs, njobs, data, offsets, data_bytes, t, s, acc.data(), P, &dj, &dt);
            if (st) {
                hipEventDestroy(e0);
                hipEventDestroy(e1);
                return st;
            }
            // every candidate must agree on every job's verdict
            if (!have_ref) {
                acc_ref = acc;
                have_ref = true;
            } else if (acc != acc_ref) {
                hipEventDestroy(e0);
                hipEventDestroy(e1);
                return POSLO_E_DEVICE;
            }
            double total = 0;
            for (int r = 0; r < reps; r++) {
                hipEventRecord(e0, s);
                if ((st = run_batch(c, prm, jobs, njobs, data, offsets, data_bytes, t, s, acc.data(), P, &dj, &dt))) {
                    hipEventDestroy(e0);
                    hipEventDestroy(e1);
                    return st;
                }
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
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    uint64_t n_total = 0;
    for (uint32_t j = 0; j < njobs; j++) n_total += jobs[j].n;
    state_of(c).tuned[shape_class(prm, n_total, data_bytes)] = bt;
    *best = bt;
    if (best_ms) *best_ms = best_t;
    return POSLO_OK;
}

namespace poslo {

void batch_release(poslo_ctx* c) {
    auto& m = states();
    auto it = m.find(c);
    if (it == m.end()) return;
    hipDeviceSynchronize();
    for (auto& g : it->second->graphs) hipGraphExecDestroy(g.second);
    if (it->second->capture) hipStreamDestroy(it->second->capture);
    delete it->second;
    m.erase(it);
}

}  // namespace poslo

extern "C" int poslo_batch_forget(poslo_ctx* c) {
    if (!c) return POSLO_E_INVAL;
    batch_release(c);
    return POSLO_OK;
}
