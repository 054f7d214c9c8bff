// POSLO-F batch verification on gfx950: the seed table, the fused
// per-entry PRF + digest + lazy aggregate kernel, the final fold with the
// aggregate check, and the host entry points that launch them.
//
// Paper: section "POSLO Parallel Batch Verification" (figure "Parallel
// POSLO signature verification algorithm"): per entry SR, PRF_0, H mod q,
// a tree reduction to per-block sub-aggregates, a final sum and one check
// R = Y^e * alpha^s.  Differences from the paper's CUDA kernel: SR and the
// epoch-constant first MMO block of PRF_0 are hoisted into a per-epoch
// table instead of being recomputed by every thread; digests are summed
// lazily as raw 256-bit integers in a 288-bit accumulator and reduced mod q
// once (exact, since (sum H) mod q = (sum (H mod q)) mod q); the final fold
// and the curve check run on the GPU.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/poslo.h"
#include "device_hash.h"
#include "ge25519.h"
#include "scheme_host.h"

namespace poslo {

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------

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
};

struct Bytes32 {
    uint8_t b[32];
};
struct Bytes64 {
    uint8_t b[64];
};

// ---------------------------------------------------------------------------
// A1: per-epoch seeds x_0[i] = SR(ds, i), plus the hoisted MMO state
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_seed_table(DsArg ds, uint32_t inst, uint64_t epoch_first,
                                                   uint32_t n_epochs, uint32_t* tab) {
    uint32_t ep = blockIdx.x * blockDim.x + threadIdx.x;
    if (ep >= n_epochs) return;
    uint64_t i = epoch_first + ep;
    ConstTables tb;
    int k = ds_cover(ds, i);
    if (k < 0) k = 0;  // coverage is validated on the host before launch
    uint32_t x[4] = {ds.v[k][0], ds.v[k][1], ds.v[k][2], ds.v[k][3]};
    // SC: walk the bits of i below the node's depth, most significant first
    for (int j = (int)ds.depth[k] - 1; j >= 0; j--) {
        uint32_t b = (uint32_t)((i >> j) & 1u), nx[4];
        if (inst == INST_AES)
            prf_node_aes(tb, x, b, nx);
        else
            prf_node_sha(x, b, nx);
        x[0] = nx[0], x[1] = nx[1], x[2] = nx[2], x[3] = nx[3];
    }
    uint32_t* e = tab + (uint64_t)ep * kEpochWords;
    if (inst == INST_AES) {
        uint32_t s[4] = {x[0], x[1], x[2], x[3]};
        aes128_encrypt_rk(tb, c_iv.a, s);
        uint32_t h1[4] = {s[0] ^ x[0], s[1] ^ x[1], s[2] ^ x[2], s[3] ^ x[3]};
        uint32_t rk[44];
        aes128_expand(tb, h1, rk);
        for (int w = 0; w < 44; w++) e[w] = rk[w];
    }
    e[44] = x[0];
    e[45] = x[1];
    e[46] = x[2];
    e[47] = x[3];
}

// ---------------------------------------------------------------------------
// A2 + A3: one-time seed and digest of one entry
// ---------------------------------------------------------------------------

struct EntryView {
    const uint8_t* m;
    uint64_t L;
};

__device__ __forceinline__ EntryView entry_view(const BatchArgs& a, uint64_t pos) {
    EntryView v;
    if (a.offsets) {
        uint64_t o0 = a.offsets[pos], o1 = a.offsets[pos + 1];
        v.m = a.data + o0;
        v.L = o1 - o0;
    } else {
        v.m = a.data + pos * a.msg_len;
        v.L = a.msg_len;
    }
    return v;
}

// byte pos of the stream m || x || padding (x as four little-endian words)
__device__ __forceinline__ uint32_t stream_byte_aes(const EntryView& v, const uint32_t x[4], uint64_t pos) {
    if (pos < v.L) return v.m[pos];
    uint64_t o = pos - v.L;
    if (o < 16) return (x[o >> 2] >> (8 * (o & 3))) & 0xffu;
    return 0;  // zero padding of the last MMO block
}

// x_t for the AES instantiation: one AES under the epoch's precomputed schedule
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
    x[3] = s[3];
}

// MDC-2 over m || x; FAST: 16-byte aligned message whose length is a multiple of 16
template <bool FAST, class T>
__device__ __forceinline__ void digest_mdc2(const T& tb, const EntryView& v, const uint32_t x[4], uint32_t dig[8]) {
    uint64_t nb = (v.L + 16 + 15) / 16;
    uint32_t h[4], hp[4];
    for (uint64_t b = 0; b < nb; b++) {
        uint32_t m[4];
        if (FAST) {
            if (16 * b < v.L) {
                uint4 q = reinterpret_cast<const uint4*>(v.m)[b];
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
        h[0] = sa[0], h[1] = sa[1], h[2] = sb[2], h[3] = sb[3];
        hp[0] = sb[0], hp[1] = sb[1], hp[2] = sa[2], hp[3] = sa[3];
    }
#pragma unroll
    for (int w = 0; w < 4; w++) {
        dig[w] = h[w];
        dig[4 + w] = hp[w];
    }
}

// x_t for the SHA-256 instantiation: one compression of x_0[i] || LE32(j) || 0x00.
// xw holds the first four digest words (big-endian words of the bytes of x_t).
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
        if (o < L) return bswap32(*reinterpret_cast<const uint32_t*>(v.m + o));
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
            byte = v.m[p];
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

template <bool FAST>
__device__ __forceinline__ void digest_sha(const EntryView& v, const uint32_t xw[4], uint32_t dig[8]) {
    uint64_t total = ((v.L + 16 + 9 + 63) / 64) * 64;
    uint32_t H[8];
    sha256_init(H);
    for (uint64_t off = 0; off < total; off += 64) {
        uint32_t W[16];
#pragma unroll
        for (int w = 0; w < 16; w++) W[w] = sha_stream_word<FAST>(v, xw, off + 4 * w, total);
        sha256_compress(H, W);
    }
#pragma unroll
    for (int w = 0; w < 8; w++) dig[w] = bswap32(H[w]);  // digest bytes as LE limbs
}

// ---------------------------------------------------------------------------
// A2-A4 fused: per-entry digests summed into 288-bit lazy accumulators, then
// wave and workgroup reductions; one nine-word partial per workgroup
// ---------------------------------------------------------------------------

constexpr int kBlock = 256;

__device__ __forceinline__ void block_reduce288_store(uint32_t acc[9], uint32_t* out) {
    __shared__ uint32_t red[kBlock / 64][9];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        uint32_t o[9];
#pragma unroll
        for (int k = 0; k < 9; k++) o[k] = __shfl_xor(acc[k], off);
        acc288_add(acc, o);
    }
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int k = 0; k < 9; k++) red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s[9];
        for (int k = 0; k < 9; k++) s[k] = red[0][k];
        for (int w = 1; w < kBlock / 64; w++) acc288_add(s, red[w]);
        for (int k = 0; k < 9; k++) out[k] = s[k];
    }
}

__device__ __forceinline__ bool skipped(const BatchArgs& a, uint64_t pos) {
    return a.skip && ((a.skip[pos >> 5] >> (pos & 31)) & 1u);
}

template <int NT, int C, bool FAST>
__global__ __launch_bounds__(kBlock) void k_agg_ekeys_aes(BatchArgs a, uint32_t* partials) {
    __shared__ uint32_t lds[NT * 256 * C];
    lds_tables_fill<NT, C>(lds);
    __syncthreads();
    LdsTables<NT, C> tb{lds + (threadIdx.x % C)};
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t pos = (uint64_t)blockIdx.x * kBlock + threadIdx.x; pos < a.n; pos += (uint64_t)gridDim.x * kBlock) {
        if (skipped(a, pos)) continue;
        uint32_t x[4], dig[8];
        one_time_seed_aes(tb, a, pos, x);
        digest_mdc2<FAST>(tb, entry_view(a, pos), x, dig);
        acc288_add256(acc, dig);
    }
    block_reduce288_store(acc, partials + (uint64_t)blockIdx.x * 9);
}

template <bool FAST>
__global__ __launch_bounds__(kBlock) void k_agg_ekeys_sha(BatchArgs a, uint32_t* partials) {
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t pos = (uint64_t)blockIdx.x * kBlock + threadIdx.x; pos < a.n; pos += (uint64_t)gridDim.x * kBlock) {
        if (skipped(a, pos)) continue;
        uint32_t xw[4], dig[8];
        one_time_seed_sha(a, pos, xw);
        digest_sha<FAST>(entry_view(a, pos), xw, dig);
        acc288_add256(acc, dig);
    }
    block_reduce288_store(acc, partials + (uint64_t)blockIdx.x * 9);
}

// per-entry outputs: e_t mod q (eight LE words) and x_t bytes (four LE words)
template <bool FAST>
__global__ __launch_bounds__(kBlock) void k_ekeys(BatchArgs a, uint32_t inst, uint32_t* e_out, uint32_t* x_out) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
    LdsTables<4, 1> tb{lds};
    for (uint64_t pos = (uint64_t)blockIdx.x * kBlock + threadIdx.x; pos < a.n; pos += (uint64_t)gridDim.x * kBlock) {
        uint32_t x[4], dig[8], e[8];
        EntryView v = entry_view(a, pos);
        if (inst == INST_AES) {
            one_time_seed_aes(tb, a, pos, x);
            digest_mdc2<FAST>(tb, v, x, dig);
        } else {
            one_time_seed_sha(a, pos, x);
            digest_sha<FAST>(v, x, dig);
#pragma unroll
            for (int w = 0; w < 4; w++) x[w] = bswap32(x[w]);
        }
        sc_reduce256(e, dig);
#pragma unroll
        for (int w = 0; w < 8; w++) e_out[pos * 8 + w] = e[w];
        if (x_out)
#pragma unroll
            for (int w = 0; w < 4; w++) x_out[pos * 4 + w] = x[w];
    }
}

// ---------------------------------------------------------------------------
// A4 tail + A5: fold the partials, reduce mod q once, aggregate check
// result words: 0..7 e mod q, 8 accept, 9 status (1: pk not a point)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_finalize(const uint32_t* partials, uint32_t n_part, Bytes32 pk,
                                                     Bytes64 tag, uint32_t* result) {
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t p = threadIdx.x; p < n_part; p += kBlock) acc288_add(acc, partials + (uint64_t)p * 9);
    __shared__ uint32_t total[9];
    block_reduce288_store(acc, total);
    __syncthreads();
    if (threadIdx.x != 0) return;
    uint32_t e[8];
    sc_reduce288(e, total);
    for (int w = 0; w < 8; w++) result[w] = e[w];
    ge Y;
    if (!ge_decode(Y, pk.b)) {
        result[8] = 0;
        result[9] = 1;
        return;
    }
    result[9] = 0;
    uint32_t s[8];
    for (int w = 0; w < 8; w++) s[w] = load_le32(tag.b + 4 * w);
    if (!sc_is_canonical(s)) {
        result[8] = 0;
        return;
    }
    ge P;
    ge_double_scalarmult(P, e, Y, s);
    uint8_t enc[32];
    ge_encode(enc, P);
    uint32_t diff = 0;
    for (int k = 0; k < 32; k++) diff |= enc[k] ^ tag.b[32 + k];
    result[8] = diff == 0 ? 1u : 0u;
}

}  // namespace poslo

// ===========================================================================
// host side: context and entry points
// ===========================================================================

using namespace poslo;

enum { KT_SEED = 0, KT_AGG = 1, KT_FINAL = 2, KT_EKEYS = 3, KT_COUNT = 8 };

struct poslo_ctx {
    int device = 0;
    int num_cu = 256;
    // per-kernel timing with HIP events on the launch stream (opt-in)
    bool profile = false;
    hipEvent_t ev[KT_COUNT][2] = {};
    bool ev_pending[KT_COUNT] = {};
    double kt_ms[KT_COUNT] = {};
    uint64_t kt_launches[KT_COUNT] = {};
    uint32_t* d_tab = nullptr;
    size_t tab_words = 0;
    uint32_t* d_part = nullptr;
    size_t part_words = 0;
    uint32_t* d_result = nullptr;
    uint32_t* h_result = nullptr;  // pinned
};

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

static void prof_begin(poslo_ctx* c, int k, hipStream_t s) {
    if (!c->profile) return;
    if (!c->ev[k][0]) {
        hipEventCreate(&c->ev[k][0]);
        hipEventCreate(&c->ev[k][1]);
    }
    hipEventRecord(c->ev[k][0], s);
}

static void prof_end(poslo_ctx* c, int k, hipStream_t s) {
    if (!c->profile) return;
    hipEventRecord(c->ev[k][1], s);
    c->ev_pending[k] = true;
}

// after the stream is synchronized: fold pending event pairs into the totals
static void prof_collect(poslo_ctx* c) {
    for (int k = 0; k < KT_COUNT; k++) {
        if (!c->ev_pending[k]) continue;
        float ms = 0.f;
        if (hipEventSynchronize(c->ev[k][1]) == hipSuccess &&
            hipEventElapsedTime(&ms, c->ev[k][0], c->ev[k][1]) == hipSuccess) {
            c->kt_ms[k] += ms;
            c->kt_launches[k] += 1;
        }
        c->ev_pending[k] = false;
    }
}

static int ensure(uint32_t** buf, size_t* have, size_t words) {
    if (*have >= words) return POSLO_OK;
    if (*buf) hipFree(*buf);
    *buf = nullptr;
    *have = 0;
    size_t want = std::max(words, (size_t)1024);
    if (hipMalloc((void**)buf, want * sizeof(uint32_t)) != hipSuccess) return POSLO_E_NOMEM;
    *have = want;
    return POSLO_OK;
}

extern "C" int poslo_ctx_create(int device, poslo_ctx** out) {
    if (!out) return POSLO_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return POSLO_E_DEVICE;
    HIP_TRY(hipSetDevice(device));
    poslo_ctx* c = new poslo_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    if (hipMalloc((void**)&c->d_result, 64 * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_result, 64 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        poslo_ctx_destroy(c);
        return POSLO_E_NOMEM;
    }
    *out = c;
    return POSLO_OK;
}

extern "C" void poslo_ctx_destroy(poslo_ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    if (c->d_tab) hipFree(c->d_tab);
    if (c->d_part) hipFree(c->d_part);
    if (c->d_result) hipFree(c->d_result);
    if (c->h_result) hipHostFree(c->h_result);
    for (int k = 0; k < KT_COUNT; k++)
        for (int e = 0; e < 2; e++)
            if (c->ev[k][e]) hipEventDestroy(c->ev[k][e]);
    delete c;
}

static bool params_ok(const poslo_params* p) {
    return p && (p->inst == POSLO_INST_AES || p->inst == POSLO_INST_SHA256) && p->log2_n1 <= 31 &&
           p->log2_n2 <= 31 && p->log2_n1 + p->log2_n2 <= 40;
}

// host-side checks shared by the verifier entry points; fills the kernel
// argument block and the by-value ds
static int prepare_batch(poslo_ctx* c, const poslo_params* prm, const poslo_msgs* m, const uint8_t* ds,
                         size_t ds_len, BatchArgs& a, DsArg& dsa, uint32_t& n_epochs) {
    if (!c || !params_ok(prm) || !m) return POSLO_E_INVAL;
    if (m->n > 0 && !m->data) return POSLO_E_INVAL;
    uint64_t nmax = 1ull << (prm->log2_n1 + prm->log2_n2);
    if (m->t0 > nmax || m->n > nmax - m->t0) return POSLO_E_INVAL;
    if (m->n >= (1ull << 32)) return POSLO_E_INVAL;  // keeps the lazy sum below 2^288
    std::vector<hostside::DsNode> nodes;
    if (!hostside::ds_parse(ds, ds_len, nodes)) return POSLO_E_INVAL;
    memset(&dsa, 0, sizeof dsa);
    dsa.count = (uint32_t)nodes.size();
    for (size_t k = 0; k < nodes.size(); k++) {
        dsa.depth[k] = nodes[k].depth;
        dsa.index[k] = nodes[k].index;
        for (int w = 0; w < 4; w++) dsa.v[k][w] = load_le32(nodes[k].v + 4 * w);
    }
    a.data = m->data;
    a.offsets = m->offsets;
    a.msg_len = m->msg_len;
    a.n = m->n;
    a.t0 = m->t0;
    a.log2_n2 = prm->log2_n2;
    a.skip = nullptr;
    n_epochs = 0;
    a.epoch_first = m->t0 >> prm->log2_n2;
    if (m->n == 0) return POSLO_OK;
    uint64_t e_last = (m->t0 + m->n - 1) >> prm->log2_n2;
    uint64_t ne = e_last - a.epoch_first + 1;
    // SR must succeed for every epoch of the batch (bottom is an error)
    for (uint64_t i = a.epoch_first; i <= e_last; i++)
        if (hostside::sr_node(nodes.data(), (int)nodes.size(), i) < 0) return POSLO_E_SEED;
    n_epochs = (uint32_t)ne;
    int st = ensure(&c->d_tab, &c->tab_words, (size_t)ne * kEpochWords);
    if (st) return st;
    a.tab = c->d_tab;
    return POSLO_OK;
}

static bool fast_layout(const poslo_msgs* m, uint64_t align) {
    return !m->offsets && m->msg_len > 0 && m->msg_len % align == 0 && ((uintptr_t)m->data % align) == 0;
}

static int launch_seed_table(const DsArg& dsa, uint32_t inst, const BatchArgs& a, uint32_t n_epochs,
                             hipStream_t s) {
    if (n_epochs == 0) return POSLO_OK;
    hipLaunchKernelGGL(k_seed_table, dim3((n_epochs + 63) / 64), dim3(64), 0, s, dsa, inst, a.epoch_first,
                       n_epochs, const_cast<uint32_t*>(a.tab));
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

static uint32_t grid_for(const poslo_ctx* c, uint64_t n) {
    uint64_t want = (n + kBlock - 1) / kBlock;
    uint64_t cap = (uint64_t)c->num_cu * 8;
    return (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
}

extern "C" int poslo_aver(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m,
                          const uint8_t* ds, size_t ds_len, const uint8_t tag[64], void* stream, int* accept,
                          uint8_t e_out[32]) {
    if (!pk || !tag || !accept) return POSLO_E_INVAL;
    *accept = 0;
    BatchArgs a;
    DsArg dsa;
    uint32_t n_epochs;
    int st = prepare_batch(c, prm, m, ds, ds_len, a, dsa, n_epochs);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    uint32_t grid = m->n ? grid_for(c, m->n) : 0;
    if ((st = ensure(&c->d_part, &c->part_words, (size_t)std::max<uint32_t>(grid, 1) * 9))) return st;
    prof_begin(c, KT_SEED, s);
    if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return st;
    prof_end(c, KT_SEED, s);
    if (grid) {
        prof_begin(c, KT_AGG, s);
        if (prm->inst == POSLO_INST_AES) {
            if (fast_layout(m, 16))
                hipLaunchKernelGGL((k_agg_ekeys_aes<4, 1, true>), dim3(grid), dim3(kBlock), 0, s, a, c->d_part);
            else
                hipLaunchKernelGGL((k_agg_ekeys_aes<4, 1, false>), dim3(grid), dim3(kBlock), 0, s, a, c->d_part);
        } else {
            if (fast_layout(m, 4))
                hipLaunchKernelGGL((k_agg_ekeys_sha<true>), dim3(grid), dim3(kBlock), 0, s, a, c->d_part);
            else
                hipLaunchKernelGGL((k_agg_ekeys_sha<false>), dim3(grid), dim3(kBlock), 0, s, a, c->d_part);
        }
        HIP_TRY(hipGetLastError());
        prof_end(c, KT_AGG, s);
    }
    Bytes32 pkb;
    Bytes64 tagb;
    memcpy(pkb.b, pk, 32);
    memcpy(tagb.b, tag, 64);
    prof_begin(c, KT_FINAL, s);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, c->d_part, grid, pkb, tagb, c->d_result);
    HIP_TRY(hipGetLastError());
    prof_end(c, KT_FINAL, s);
    HIP_TRY(hipMemcpyAsync(c->h_result, c->d_result, 16 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    prof_collect(c);
    if (c->h_result[9] == 1) return POSLO_E_ENCODING;
    *accept = c->h_result[8] ? 1 : 0;
    if (e_out)
        for (int w = 0; w < 8; w++) store_le32(e_out + 4 * w, c->h_result[w]);
    return POSLO_OK;
}

extern "C" int poslo_ekeys(poslo_ctx* c, const poslo_params* prm, const poslo_msgs* m, const uint8_t* ds,
                           size_t ds_len, uint8_t* e_dev, uint8_t* x_dev, void* stream) {
    BatchArgs a;
    DsArg dsa;
    uint32_t n_epochs;
    int st = prepare_batch(c, prm, m, ds, ds_len, a, dsa, n_epochs);
    if (st) return st;
    if (m->n == 0) return POSLO_OK;
    if (!e_dev) return POSLO_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return st;
    uint32_t grid = grid_for(c, m->n);
    bool fast = fast_layout(m, prm->inst == POSLO_INST_AES ? 16 : 4);
    if (fast)
        hipLaunchKernelGGL(k_ekeys<true>, dim3(grid), dim3(kBlock), 0, s, a, prm->inst, (uint32_t*)e_dev,
                           (uint32_t*)x_dev);
    else
        hipLaunchKernelGGL(k_ekeys<false>, dim3(grid), dim3(kBlock), 0, s, a, prm->inst, (uint32_t*)e_dev,
                           (uint32_t*)x_dev);
    HIP_TRY(hipGetLastError());
    return POSLO_OK;
}

extern "C" int poslo_ctx_profile(poslo_ctx* c, int enable) {
    if (!c) return POSLO_E_INVAL;
    c->profile = enable != 0;
    return POSLO_OK;
}

extern "C" int poslo_ctx_kernel_time(poslo_ctx* c, int kernel, int reset, double* total_ms, uint64_t* launches) {
    if (!c || kernel < 0 || kernel >= KT_COUNT) return POSLO_E_INVAL;
    prof_collect(c);
    if (total_ms) *total_ms = c->kt_ms[kernel];
    if (launches) *launches = c->kt_launches[kernel];
    if (reset) {
        c->kt_ms[kernel] = 0;
        c->kt_launches[kernel] = 0;
    }
    return POSLO_OK;
}
