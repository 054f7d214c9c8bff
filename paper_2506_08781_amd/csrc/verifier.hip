// POSLO-F aggregate verification on gfx950: the per-epoch seed table,
// per-entry digests, the final fold with the curve check, and the context
// and AVer entry points.
//
// Paper: section "POSLO Parallel Batch Verification" (figure "Parallel
// POSLO signature verification algorithm"): per entry SR, PRF_0, H mod q, a
// tree reduction to per-block sub-aggregates, a final sum and one check
// R = Y^e * alpha^s.  Differences from the paper's CUDA design: SR and the
// epoch-constant first MMO block of PRF_0 are hoisted into a per-epoch
// table; digests are summed lazily as raw 256-bit integers in a 288-bit
// accumulator and reduced mod q once (exact, since (sum H) mod q =
// (sum (H mod q)) mod q); the final fold and the curve check run on the GPU
// with per-key fixed-base tables: 64 table lookups and a 6-level tree of
// point additions instead of a 253-step double-and-add chain.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "aes_quad.h"
#include "ctx.h"
#include "device_ec.h"
#include "device_entry.h"
#include "fourq.h"
#include "ge25519.h"
#include "scheme_host.h"

namespace poslo {

// ---------------------------------------------------------------------------
// A1: per-epoch seeds x_0[i] = SR(ds, i), plus the hoisted MMO state
// ---------------------------------------------------------------------------

// AES: four lanes per epoch (aes_quad.h), so each link of the walk's chain
// of dependent PRF calls costs about a third of a one-lane encryption;
// SHA-256: one lane per epoch.  K127: kappa = 127, one AES per tree level.
// The first thread also clears the flag word after the last row (tab.bad).
// SC from node value x (column c of it for AES, all four words for SHA-256)
// down the bits hi-1 .. lo of epoch index i
template <int INST, bool K127, class T>
__device__ __forceinline__ void seed_walk_dev(const T& tb, uint32_t x[4], uint32_t c, uint64_t i, int hi, int lo) {
    for (int j = hi - 1; j >= lo; j--) {
        const uint32_t b = (uint32_t)((i >> j) & 1u);
        if constexpr (INST == INST_AES) {
            x[0] = K127 ? quad_prf_node127(tb, x[0], b, c) : quad_prf_node(tb, x[0], b, c);
        } else {
            uint32_t nx[4];
            prf_node_sha(x, b, nx);
            x[0] = nx[0], x[1] = nx[1], x[2] = nx[2], x[3] = nx[3];
        }
    }
}

// Many epochs: the seeds of their subtrees of height h = kSeedMidHeight
// first (k_seed_mid), then each epoch walks the last h levels from its
// subtree's seed.  The work drops from depth to h tree PRFs per epoch (plus
// depth - h per 2^h epochs); the chain is as long as before.  mid holds 4
// words per subtree (i >> h) - (epoch_first >> h) whose covering ds node
// lies above height h.
constexpr int kMidHeight = kSeedMidHeight;
constexpr uint32_t kMidMinEpochs = 1u << 15;  // below this the one-pass walk is as fast

inline uint32_t seed_mid_count(uint64_t epoch_first, uint32_t n_epochs) {
    return n_epochs ? (uint32_t)(((epoch_first + n_epochs - 1) >> kMidHeight) - (epoch_first >> kMidHeight) + 1) : 0u;
}

template <int INST, bool K127>
__global__ __launch_bounds__(64) void k_seed_mid(DsArg ds, uint64_t epoch_first, uint32_t n_mid, uint32_t* mid) {
    __shared__ uint32_t lds[INST == INST_AES ? 4 * 256 : 1];
    if constexpr (INST == INST_AES) lds_tables_fill<4, 1>(lds);
    __syncthreads();
    const LdsTables<4, 1> tb{lds};
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t m = INST == INST_AES ? g >> 2 : g, c = g & 3u;
    if (m >= n_mid) return;  // whole quads leave together
    const uint64_t sub = (epoch_first >> kMidHeight) + m;
    const uint64_t i = (sub << kMidHeight) > epoch_first ? (sub << kMidHeight) : epoch_first;
    int k = ds_cover(ds, i);
    if (k < 0) k = 0;  // coverage is validated on the host before launch
    if ((int)ds.depth[k] <= kMidHeight) return;  // its epochs walk from the ds node
    uint32_t x[4] = {ds.v[k][0], ds.v[k][1], ds.v[k][2], ds.v[k][3]};
    if constexpr (INST == INST_AES) x[0] = ds.v[k][c];
    seed_walk_dev<INST, K127>(tb, x, c, i, (int)ds.depth[k], kMidHeight);
    uint32_t* o = mid + (uint64_t)m * 4;
    if constexpr (INST == INST_AES) o[c] = x[0];
    else o[0] = x[0], o[1] = x[1], o[2] = x[2], o[3] = x[3];
}

template <int INST, bool K127>
__global__ __launch_bounds__(64) void k_seed_table(DsArg ds, uint64_t epoch_first, uint32_t n_epochs, uint32_t* tab,
                                                   const uint32_t* mid) {
    __shared__ uint32_t lds[INST == INST_AES ? 4 * 256 : 1];
    if constexpr (INST == INST_AES) lds_tables_fill<4, 1>(lds);
    __syncthreads();
    const LdsTables<4, 1> tb{lds};
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) tab[(uint64_t)n_epochs * kEpochWords] = 0u;
    const uint32_t ep = INST == INST_AES ? g >> 2 : g, c = g & 3u;
    if (ep >= n_epochs) return;  // whole quads leave together
    uint64_t i = epoch_first + ep;
    int k = ds_cover(ds, i);
    if (k < 0) k = 0;  // coverage is validated on the host before launch
    uint32_t* e = tab + (uint64_t)ep * kEpochWords;
    // SC: walk the bits of i below the node's depth, most significant first
    // (from the subtree's seed when k_seed_mid has walked the upper levels)
    uint32_t x[4] = {ds.v[k][0], ds.v[k][1], ds.v[k][2], ds.v[k][3]};
    int hi = (int)ds.depth[k];
    if (mid && hi > kMidHeight) {
        const uint32_t* ms = mid + ((i >> kMidHeight) - (epoch_first >> kMidHeight)) * 4;
        x[0] = ms[0], x[1] = ms[1], x[2] = ms[2], x[3] = ms[3];
        hi = kMidHeight;
    }
    if constexpr (INST == INST_AES) {
        uint32_t xc[4] = {c == 0 ? x[0] : c == 1 ? x[1] : c == 2 ? x[2] : x[3], 0u, 0u, 0u};
        seed_walk_dev<INST, K127>(tb, xc, c, i, hi, 0);
        quad_epoch_row(tb, xc[0], c, e);
    } else {
        seed_walk_dev<INST, K127>(tb, x, c, i, hi, 0);
        e[44] = x[0];
        e[45] = x[1];
        e[46] = x[2];
        e[47] = x[3];
    }
}

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// A4 tail + A5: fold the partials, reduce mod q once, aggregate check
// e*Y + s*G = sum over 64 windows of T_Y[w][e_w] + T_G[w][s_w]: 128 lanes
// look up one point each, then pairs and a wave tree of point additions.
// result words: 0..7 e mod q, 8 accept, 9 status
// ---------------------------------------------------------------------------

struct FinalArgs {
    const uint32_t* partials;
    uint32_t n_part;
    uint32_t checks_ok;  // s < q and R decodes (host-side checks)
    const uint32_t* ty;  // comb table of Y
    const uint32_t* tg;  // comb table of G
    uint32_t s[8];
    uint32_t rx[8];      // decoded R (affine)
    uint32_t ry[8];
    uint32_t* result;
    const uint32_t* bad;  // POSLO++ long-message flag, or nullptr
};

static_assert(kBlock == kQuadBlock, "the aggregate check takes the whole block");

__global__ __launch_bounds__(kBlock) void k_finalize(FinalArgs f) {
    __shared__ uint32_t total[9];
    __shared__ uint32_t sh_es[16];
    __shared__ uint32_t pts[kQuadLdsWords];
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t p = threadIdx.x; p < f.n_part; p += kBlock) acc288_add(acc, f.partials + (uint64_t)p * 9);
    block_reduce288_store<kBlock>(acc, total);
    __syncthreads();
    // e mod q on the first wave and s mod q on the second, side by side
    if (threadIdx.x == 0) {
        uint32_t e[8];
        sc_reduce288(e, total);
        for (int k = 0; k < 8; k++) {
            sh_es[k] = e[k];
            f.result[k] = e[k];
        }
    } else if (threadIdx.x == 64) {
        uint32_t sr[8];
        sc_reduce256(sr, f.s);
        for (int k = 0; k < 8; k++) sh_es[8 + k] = sr[k];
    }
    __syncthreads();
    uint32_t e[8], sv[8];
    for (int k = 0; k < 8; k++) {
        e[k] = sh_es[k];
        sv[k] = sh_es[8 + k];
    }
    fe rx, ry;
    for (int k = 0; k < 8; k++) {
        rx.v[k] = f.rx[k];
        ry.v[k] = f.ry[k];
    }
    // e*Y + s*G == R, with R decoded on the host
    const bool eq = block_double_scalar_is(pts, f.ty, f.tg, e, sv, rx, ry);
    if (threadIdx.x == 0) {
        const uint32_t bad = f.bad ? *f.bad : 0u;
        f.result[8] = (f.checks_ok && eq && !bad) ? 1u : 0u;
        f.result[9] = bad ? 1u : 0u;
    }
}

// The same check on FourQ (fourq.h), with the quad-split tree of
// block_double_scalar_is: quad k of the block owns point k of 64 (k < 32:
// window k of e on Y's table, k >= 32: window k - 32 of s on G's), lane c
// coordinate c (X, Y, Z, T) as 8 words in LDS.  Per tree level lane 0 forms
// A = (Y1 - X1)(Y2 - X2), lane 1 B = (Y1 + X1)(Y2 + X2), lane 2
// C = 2d T1 T2 (one more product: 2d is a full GF(p^2) element here),
// lane 3 D = 2 Z1 Z2; the quad shares them by DPP moves, and lane c forms
// output coordinate c (X3 = EF, Y3 = GH, Z3 = FG, T3 = EH).  Then the sum
// is compared with the host-decoded R in projective form.
__device__ __forceinline__ void lds_load_f2(fp2& a, const uint32_t* p) {
#pragma unroll
    for (int k = 0; k < 4; k++) a.a.v[k] = p[k], a.b.v[k] = p[4 + k];
}

__device__ __forceinline__ void lds_store_f2(uint32_t* p, const fp2& a) {
#pragma unroll
    for (int k = 0; k < 4; k++) p[k] = a.a.v[k], p[4 + k] = a.b.v[k];
}

__device__ __forceinline__ bool block_double_scalar_is_fq(uint32_t* lds, const uint32_t* ty, const uint32_t* tg,
                                                          const uint32_t e[8], const uint32_t s[8], const fp2& rx,
                                                          const fp2& ry) {
    const int k = (int)(threadIdx.x >> 2), c = (int)(threadIdx.x & 3);
    const uint32_t* sc = k < 32 ? e : s;
    const int w = k & 31;
    uint32_t carry = 0;
    int d = 0;
    for (int i = 0; i < kCombWindows; i++) {  // fixed trip count: the scalar stays in registers
        const int di = comb_digit(sc, i, carry);
        if (i == w) d = di;
    }
    // the affine point (x, y) as (4x : 4y : 4 : 4xy) from y + x and y - x
    // (the identity (0 : 4 : 4 : 0) for a zero digit)
    fp2 a, b, m, v;
    if (d != 0) {
        const uint32_t mag = (uint32_t)(d < 0 ? -d : d);
        gnq q;
        fq_load_entry(q, (k < 32 ? ty : tg) + ((uint64_t)w * kCombPerWindow + mag - 1) * kCombEntryWords, d < 0);
        f2_sub(a, q.yp, q.ym);
        f2_add(b, q.yp, q.ym);
    } else {
        f2_zero(a);
        f2_one(b);
        f2_add(b, b, b);
    }
    f2_mul(m, a, b);
    if (c == 0) {
        f2_add(v, a, a);
    } else if (c == 1) {
        f2_add(v, b, b);
    } else if (c == 2) {
        f2_zero(v);
        v.a.v[0] = 4;
    } else {
        v = m;
    }
    lds_store_f2(lds + (k * 4 + c) * 8, v);
    const fp2 d2 = fq_d2();
    for (int o = 32; o >= 1; o >>= 1) {
        __syncthreads();
        if (k < o) {
            const uint32_t* p1 = lds + k * 32;
            const uint32_t* p2 = lds + (k + o) * 32;
            const int co = c < 2 ? 0 : c == 2 ? 3 : 2;
            fp2 u1, u2, y1, y2;
            lds_load_f2(u1, p1 + co * 8);
            lds_load_f2(u2, p2 + co * 8);
            if (c < 2) {
                lds_load_f2(y1, p1 + 8);
                lds_load_f2(y2, p2 + 8);
                if (c == 0) {
                    f2_sub(u1, y1, u1);
                    f2_sub(u2, y2, u2);
                } else {
                    f2_add(u1, y1, u1);
                    f2_add(u2, y2, u2);
                }
            }
            f2_mul(m, u1, u2);
            if (c == 2) f2_mul(m, m, d2);
            else if (c == 3) f2_add(m, m, m);
            // every lane of the quad gets A, B, C, D (the word of lane L
            // sits (L - c) & 3 lanes to the right)
            fp2 A, B, C, D;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const uint32_t r0 = j < 4 ? m.a.v[j & 3] : m.b.v[j & 3];
                const uint32_t r1 = ec_quad_rot<1>(r0), r2 = ec_quad_rot<2>(r0), r3 = ec_quad_rot<3>(r0);
                const uint32_t wa = c == 0 ? r0 : c == 1 ? r3 : c == 2 ? r2 : r1;
                const uint32_t wb = c == 1 ? r0 : c == 2 ? r3 : c == 3 ? r2 : r1;
                const uint32_t wc = c == 2 ? r0 : c == 3 ? r3 : c == 0 ? r2 : r1;
                const uint32_t wd = c == 3 ? r0 : c == 0 ? r3 : c == 1 ? r2 : r1;
                if (j < 4) {
                    A.a.v[j & 3] = wa, B.a.v[j & 3] = wb, C.a.v[j & 3] = wc, D.a.v[j & 3] = wd;
                } else {
                    A.b.v[j & 3] = wa, B.b.v[j & 3] = wb, C.b.v[j & 3] = wc, D.b.v[j & 3] = wd;
                }
            }
            fp2 E, F, G, H;
            f2_sub(E, B, A);
            f2_sub(F, D, C);
            f2_add(G, D, C);
            f2_add(H, B, A);
            // lane 0: X3 = EF, lane 1: Y3 = GH, lane 2: Z3 = FG, lane 3: T3 = EH
            fp2 l, r;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                l.a.v[j] = c == 1 ? G.a.v[j] : c == 2 ? F.a.v[j] : E.a.v[j];
                l.b.v[j] = c == 1 ? G.b.v[j] : c == 2 ? F.b.v[j] : E.b.v[j];
                r.a.v[j] = c == 0 ? F.a.v[j] : c == 2 ? G.a.v[j] : H.a.v[j];
                r.b.v[j] = c == 0 ? F.b.v[j] : c == 2 ? G.b.v[j] : H.b.v[j];
            }
            f2_mul(v, l, r);
            lds_store_f2(lds + (k * 4 + c) * 8, v);
        }
    }
    __syncthreads();
    bool ok = true;
    if (k == 0 && c < 2) {
        fp2 Z, V, R;
        lds_load_f2(Z, lds + 2 * 8);
        lds_load_f2(V, lds + c * 8);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            R.a.v[j] = c == 0 ? rx.a.v[j] : ry.a.v[j];
            R.b.v[j] = c == 0 ? rx.b.v[j] : ry.b.v[j];
        }
        f2_mul(m, R, Z);
        ok = f2_eq(m, V);
    }
    const uint64_t bad = __ballot(!ok);
    return (bad & 3u) == 0;
}

__global__ __launch_bounds__(kBlock) void k_finalize_fq(FinalArgs f) {
    __shared__ uint32_t total[9];
    __shared__ uint32_t sh_es[16];
    __shared__ uint32_t pts[kQuadLdsWords];
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t p = threadIdx.x; p < f.n_part; p += kBlock) acc288_add(acc, f.partials + (uint64_t)p * 9);
    block_reduce288_store<kBlock>(acc, total);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t[9], e[8];
        for (int k = 0; k < 9; k++) t[k] = total[k];
        scN_reduce<9>(e, t);
        for (int k = 0; k < 8; k++) {
            sh_es[k] = e[k];
            sh_es[8 + k] = f.s[k];  // s < N, checked on the host
            f.result[k] = e[k];
        }
    }
    __syncthreads();
    uint32_t e[8], sv[8];
    for (int k = 0; k < 8; k++) e[k] = sh_es[k], sv[k] = sh_es[8 + k];
    fp2 xr, yr;
    for (int i = 0; i < 4; i++) {
        xr.a.v[i] = f.rx[i], xr.b.v[i] = f.rx[4 + i];
        yr.a.v[i] = f.ry[i], yr.b.v[i] = f.ry[4 + i];
    }
    const bool eq = block_double_scalar_is_fq(pts, f.ty, f.tg, e, sv, xr, yr);
    if (threadIdx.x == 0) {
        const uint32_t bad = f.bad ? *f.bad : 0u;
        f.result[8] = (f.checks_ok && eq && !bad) ? 1u : 0u;
        f.result[9] = bad ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// context helpers
// ---------------------------------------------------------------------------

int ctx_ensure(uint32_t** buf, size_t* have, size_t words) {
    if (*have >= words) return POSLO_OK;
    if (*buf) hipFree(*buf);
    *buf = nullptr;
    *have = 0;
    size_t want = std::max(words, (size_t)1024);
    if (hipMalloc((void**)buf, want * sizeof(uint32_t)) != hipSuccess) return POSLO_E_NOMEM;
    *have = want;
    return POSLO_OK;
}

int ctx_scratch(poslo_ctx* c, int slot, size_t bytes, void** out) {
    if (slot < 0 || slot >= 32) return POSLO_E_INVAL;
    int st = ctx_ensure(&c->xbuf[slot], &c->xbuf_words[slot], (bytes + 3) / 4);
    if (st) return st;
    *out = c->xbuf[slot];
    return POSLO_OK;
}

void prof_begin(poslo_ctx* c, int k, hipStream_t s) {
    if (!((c->profile_mask >> k) & 1u)) return;
    if (!c->ev[k][0]) {
        hipEventCreate(&c->ev[k][0]);
        hipEventCreate(&c->ev[k][1]);
    }
    hipEventRecord(c->ev[k][0], s);
}

void prof_end(poslo_ctx* c, int k, hipStream_t s) {
    if (!((c->profile_mask >> k) & 1u)) return;
    hipEventRecord(c->ev[k][1], s);
    c->ev_pending[k] = true;
}

void prof_collect(poslo_ctx* c) {
    for (int k = 0; k < kKtCount; k++) {
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

const KeyEntry* ctx_key(poslo_ctx* c, const uint8_t pk[32], int* status) {
    std::vector<const uint32_t*> t;
    *status = ctx_keys_bulk(c, pk, 1, t, nullptr);
    if (*status) return nullptr;
    return &*c->key_index.at(std::string((const char*)pk, 32));
}

}  // namespace poslo

namespace poslo {

// ---------------------------------------------------------------------------
// fixed scratch of the allocation-free AVer entry point: per-epoch rows,
// per-workgroup partials and the result words, in one device array that
// every GPU the library runs on holds until the process ends
// ---------------------------------------------------------------------------

static_assert(kTabRowWords == (size_t)kEpochWords, "epoch row size");
constexpr uint64_t kFixedMaxEpochs = POSLO_AVER_FIXED_MAX_EPOCHS;
constexpr uint32_t kFixedMaxGrid = 4096;
constexpr size_t kFixedTabWords = epoch_tab_words(kFixedMaxEpochs);
constexpr size_t kFixedPartWords = (size_t)kFixedMaxGrid * 9;
constexpr size_t kFixedWords = kFixedTabWords + kFixedPartWords + 64;
static_assert(kFixedWords * 4 == (size_t)POSLO_AVER_FIXED_SCRATCH_BYTES, "scratch size in the header");

static __device__ __align__(256) uint32_t scratch[kFixedWords];

constexpr int kMaxDevices = 64;
static std::mutex g_fixed_mu;
static uint32_t* g_fixed[kMaxDevices];  // device address of `scratch` on each device

// the device address of this device's `scratch`, looked up once per device
// (the array's name is not a device address in host code); the device must
// be current
static int fixed_scratch_init(int device, uint32_t** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return POSLO_E_DEVICE;
    std::lock_guard<std::mutex> g(g_fixed_mu);
    if (!g_fixed[device]) {
        uint32_t* p = nullptr;
        if (hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return POSLO_E_DEVICE;
        g_fixed[device] = p;
    }
    *out = g_fixed[device];
    return POSLO_OK;
}

}  // namespace poslo

// ===========================================================================
// entry points
// ===========================================================================

using namespace poslo;

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

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
        hipHostMalloc((void**)&c->h_result, 64 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&c->d_gtable, (size_t)kCombWords * 4) != hipSuccess) {
        poslo_ctx_destroy(c);
        return POSLO_E_NOMEM;
    }
    ge G;
    ge_base(G);
    uint8_t genc[32];
    ge_encode(genc, G);
    std::vector<uint32_t> gok;
    if (build_comb_tables(genc, 1, c->d_gtable, gok) || !gok[0] || fixed_scratch_init(device, &c->d_fixed)) {
        poslo_ctx_destroy(c);
        return POSLO_E_DEVICE;
    }
    *out = c;
    return POSLO_OK;
}

extern "C" void poslo_ctx_destroy(poslo_ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    if (c->d_tab) hipFree(c->d_tab);
    if (c->d_part) hipFree(c->d_part);
    if (c->d_result) hipFree(c->d_result);
    if (c->h_result) hipHostFree(c->h_result);
    if (c->d_gtable) hipFree(c->d_gtable);
    if (c->d_gtable_wide) hipFree(c->d_gtable_wide);
    if (c->d_gtable_wide_fq) hipFree(c->d_gtable_wide_fq);
    if (c->d_gtable_fq) hipFree(c->d_gtable_fq);
    batch_release(c);
    c->key_index.clear();
    c->keys.clear();
    for (int k = 0; k < 32; k++)
        if (c->xbuf[k]) hipFree(c->xbuf[k]);
    for (int k = 0; k < kKtCount; k++)
        for (int e = 0; e < 2; e++)
            if (c->ev[k][e]) hipEventDestroy(c->ev[k][e]);
    delete c;
}

extern "C" int poslo_ctx_profile(poslo_ctx* c, int kernels) {
    if (!c || kernels < 0 || kernels > POSLO_PROFILE_ALL) return POSLO_E_INVAL;
    c->profile_mask = (uint32_t)kernels;
    return POSLO_OK;
}

extern "C" int poslo_ctx_kernel_time(poslo_ctx* c, int kernel, int reset, double* total_ms, uint64_t* launches) {
    if (!c || kernel < 0 || kernel >= kKtCount) return POSLO_E_INVAL;
    prof_collect(c);
    if (total_ms) *total_ms = c->kt_ms[kernel];
    if (launches) *launches = c->kt_launches[kernel];
    if (reset) {
        c->kt_ms[kernel] = 0;
        c->kt_launches[kernel] = 0;
    }
    return POSLO_OK;
}

extern "C" int poslo_agg_variant_count(void) { return agg_aes_variant_count(); }

extern "C" const char* poslo_agg_variant_name(int v) {
    if (v < 0 || v >= agg_aes_variant_count()) return nullptr;
    return agg_aes_variant(v).name;
}

extern "C" int poslo_ctx_set_tuning(poslo_ctx* c, int agg_variant, int wg_per_cu) {
    if (!c || agg_variant < -1 || agg_variant >= agg_aes_variant_count() || wg_per_cu < 0 || wg_per_cu > 64)
        return POSLO_E_INVAL;
    c->agg_variant = agg_variant;
    c->wg_per_cu = wg_per_cu;
    return POSLO_OK;
}

namespace poslo {

bool params_ok(const poslo_params* p) {
    return p && poslo_inst_valid(p->inst) && p->log2_n1 <= 31 &&
           p->log2_n2 <= 31 && p->log2_n1 + p->log2_n2 <= 40;
}

// host-side checks shared by the verifier entry points; fills the kernel
// argument block and the by-value ds.  The epoch table goes to the
// context's buffer (grown as needed), or to fixed_tab when it is set (no
// allocation; E_INVAL beyond fixed_epochs epochs; fixed_tab holds
// epoch_tab_words(fixed_epochs) words).  The word after the last epoch row
// is POSLO++'s long-message flag (a.bad).
int prepare_batch(poslo_ctx* c, const poslo_params* prm, const poslo_msgs* m, const uint8_t* ds, size_t ds_len,
                  BatchArgs& a, DsArg& dsa, uint32_t& n_epochs, uint32_t* fixed_tab, uint64_t fixed_epochs) {
    if (!c || !params_ok(prm) || !m) return POSLO_E_INVAL;
    // data may be null only for a fixed length of zero (nothing is read)
    if (m->n > 0 && !m->data && (m->offsets || m->msg_len)) return POSLO_E_INVAL;
    uint64_t nmax = 1ull << (prm->log2_n1 + prm->log2_n2);
    if (m->t0 > nmax || m->n > nmax - m->t0) return POSLO_E_INVAL;
    if (m->n >= (1ull << 32)) return POSLO_E_INVAL;  // keeps the lazy sum below 2^288
    hostside::DsNode nodes[32];
    int count = 0;
    if (!hostside::ds_parse(ds, ds_len, nodes, &count)) return POSLO_E_INVAL;
    memset(&dsa, 0, sizeof dsa);
    dsa.count = (uint32_t)count;
    for (int k = 0; k < count; k++) {
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
    a.tab = nullptr;
    a.bad = nullptr;
    a.xmask = kappa127(prm->inst) ? 0x7fffffffu : 0xffffffffu;
    a.emit_fq = (prm->inst & POSLO_GROUP_FOURQ) ? 1u : 0u;
    // POSLO++ on a fixed-length batch: the length is checked here, a
    // variable-length batch's lengths by the kernels (a.bad)
    if (inst_base(prm->inst) == INST_AES_ADDQ && !m->offsets && m->msg_len > kAddqMaxLen && m->n > 0)
        return POSLO_E_INVAL;
    if (m->data_bytes)
        a.end = m->data + m->data_bytes;
    else if (!m->offsets)
        a.end = m->data + m->n * m->msg_len;
    else
        a.end = nullptr;
    n_epochs = 0;
    a.epoch_first = m->t0 >> prm->log2_n2;
    if (m->n == 0) return POSLO_OK;
    uint64_t e_last = (m->t0 + m->n - 1) >> prm->log2_n2;
    uint64_t ne = e_last - a.epoch_first + 1;
    // SR must succeed for every epoch of the batch (bottom is an error); at
    // kappa = 127 a node that is walked must be a 127-bit seed
    for (uint64_t i = a.epoch_first; i <= e_last; i++) {
        const int k = hostside::sr_node(nodes, count, i);
        if (k < 0) return POSLO_E_SEED;
        if (kappa127(prm->inst) && nodes[k].depth > 0 && (nodes[k].v[15] & 0x80)) return POSLO_E_INVAL;
    }
    if (fixed_tab) {
        if (ne > fixed_epochs) return POSLO_E_INVAL;
        a.tab = fixed_tab;
    } else {
        int st = ctx_ensure(&c->d_tab, &c->tab_words, epoch_tab_words(ne));
        if (st) return st;
        a.tab = c->d_tab;
    }
    a.bad = const_cast<uint32_t*>(a.tab) + ne * kEpochWords;
    n_epochs = (uint32_t)ne;
    return POSLO_OK;
}

bool fast_layout(const poslo_msgs* m, uint64_t align) {
    return !m->offsets && m->msg_len > 0 && m->msg_len % align == 0 && ((uintptr_t)m->data % align) == 0;
}

template <int INST, bool K127>
static void launch_seeds(const DsArg& dsa, const BatchArgs& a, uint32_t n_epochs, uint32_t* tab, hipStream_t s) {
    const uint32_t per_block = INST == INST_AES ? 16 : 64;
    uint32_t* mid = nullptr;
    if (n_epochs >= kMidMinEpochs) {
        // the subtree seeds sit after the rows and the flag word (epoch_tab_words)
        mid = tab + (size_t)n_epochs * kEpochWords + 64;
        const uint32_t n_mid = seed_mid_count(a.epoch_first, n_epochs);
        hipLaunchKernelGGL((k_seed_mid<INST, K127>), dim3((n_mid + per_block - 1) / per_block), dim3(64), 0, s, dsa,
                           a.epoch_first, n_mid, mid);
    }
    hipLaunchKernelGGL((k_seed_table<INST, K127>), dim3((n_epochs + per_block - 1) / per_block), dim3(64), 0, s, dsa,
                       a.epoch_first, n_epochs, tab, (const uint32_t*)mid);
}

int launch_seed_table(const DsArg& dsa, uint32_t inst, const BatchArgs& a, uint32_t n_epochs, hipStream_t s) {
    if (n_epochs == 0) return POSLO_OK;
    uint32_t* tab = const_cast<uint32_t*>(a.tab);
    if (prf_is_aes(inst) && kappa127(inst)) launch_seeds<INST_AES, true>(dsa, a, n_epochs, tab, s);
    else if (prf_is_aes(inst)) launch_seeds<INST_AES, false>(dsa, a, n_epochs, tab, s);
    else launch_seeds<INST_SHA256, false>(dsa, a, n_epochs, tab, s);
    return hipGetLastError() == hipSuccess ? POSLO_OK : POSLO_E_DEVICE;
}

}  // namespace poslo

// workgroups resident per CU for an AES variant: bounded by LDS (160 KB per
// CU) and by 32 waves per CU
static uint32_t variant_wg_per_cu(const poslo_ctx* c, int v) {
    if (c->wg_per_cu > 0) return (uint32_t)c->wg_per_cu;
    const AggVariant& av = agg_aes_variant(v);
    size_t lds = agg_aes_lds_bytes(v) + 1024;
    uint32_t by_lds = (uint32_t)((160 * 1024) / lds);
    uint32_t by_waves = 32 / (av.block / 64);
    return std::max<uint32_t>(1, std::min(by_lds, by_waves));
}

namespace poslo {

AggShape agg_shape(const poslo_ctx* c, const poslo_params* prm, const poslo_msgs* m) {
    AggShape g{};
    const uint32_t base = inst_base(prm->inst);
    if (base == INST_AES_ADDQ) {
        g.addq_layout = (fast_layout(m, 16) && m->msg_len == 16) ? 2 : fast_layout(m, 4) ? 1 : 0;
        uint64_t want = (m->n + agg_addq_block() - 1) / agg_addq_block();
        // two 1,024-thread workgroups (64 KB of tables each) per CU
        uint64_t cap = (uint64_t)c->num_cu * (c->wg_per_cu > 0 ? c->wg_per_cu : 2);
        g.grid = (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
    } else if (base == INST_AES) {
        g.fast = fast_layout(m, 16);
        g.variant = g.fast ? (c->agg_variant >= 0 ? c->agg_variant : agg_aes_default_variant()) : -1;
        // the any-layout form shares the default variant's shape
        const int vs = g.fast ? g.variant : agg_aes_default_variant();
        uint32_t block = g.fast ? (uint32_t)agg_aes_variant(vs).block : (uint32_t)agg_aes_any_block();
        uint64_t want = (m->n + block - 1) / block;
        uint64_t cap = (uint64_t)c->num_cu * variant_wg_per_cu(c, vs);
        g.grid = (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
    } else {
        g.sha_layout = fast_layout(m, 16) ? 2 : fast_layout(m, 4) ? 1 : 0;
        uint64_t want = (m->n + kAggShaBlock - 1) / kAggShaBlock;
        // four resident workgroups per CU measured best for the SHA-256 kernel
        uint64_t cap = (uint64_t)c->num_cu * (c->wg_per_cu > 0 ? c->wg_per_cu : 4);
        g.grid = (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
    }
    return g;
}

int launch_agg(poslo_ctx* c, const poslo_params* prm, const AggShape& g, const BatchArgs& a, uint32_t* partials,
               uint32_t* e_out, uint32_t* x_out, hipStream_t s) {
    int st;
    prof_begin(c, POSLO_KT_AGG, s);
    if (inst_base(prm->inst) == INST_AES_ADDQ) {
        st = launch_agg_addq(g.addq_layout, g.grid, &a, partials, e_out, x_out, s);
    } else if (inst_base(prm->inst) == INST_AES) {
        if (e_out && g.fast && g.variant != agg_aes_default_variant()) return POSLO_E_INVAL;
        st = e_out ? launch_agg_aes_emit(g.fast, g.grid, &a, partials, e_out, x_out, s)
                   : launch_agg_aes(g.variant, g.fast, g.grid, &a, partials, s);
    } else {
        st = e_out ? launch_agg_sha_emit(g.sha_layout, g.grid, &a, partials, e_out, x_out, s)
                   : launch_agg_sha(g.sha_layout, g.grid, &a, partials, s);
    }
    if (st) return st;
    prof_end(c, POSLO_KT_AGG, s);
    return POSLO_OK;
}

}  // namespace poslo

// host-side tag checks: s < q and R decodes (done while the GPU hashes)
static void tag_checks(const uint8_t tag[64], FinalArgs& f) {
    for (int w = 0; w < 8; w++) f.s[w] = load_le32(tag + 4 * w);
    ge R;
    bool r_ok = ge_decode(R, tag + 32);
    f.checks_ok = (sc_is_canonical(f.s) && r_ok) ? 1u : 0u;
    if (r_ok) {
        for (int k = 0; k < 8; k++) {
            f.rx[k] = R.X.v[k];
            f.ry[k] = R.Y.v[k];
        }
    } else {
        memset(f.rx, 0, sizeof f.rx);
        memset(f.ry, 0, sizeof f.ry);
    }
}

// the same for FourQ: s < N, R decodes on FourQ (rx, ry: x and y as GF(p^2)
// words, real part first)
static void tag_checks_fq(const uint8_t tag[64], FinalArgs& f) {
    for (int w = 0; w < 8; w++) f.s[w] = load_le32(tag + 4 * w);
    gq R;
    const bool r_ok = fq_decode(R, tag + 32);
    f.checks_ok = (scN_is_canonical(f.s) && r_ok) ? 1u : 0u;
    for (int k = 0; k < 4; k++) {
        f.rx[k] = r_ok ? R.X.a.v[k] : 0u;
        f.rx[4 + k] = r_ok ? R.X.b.v[k] : 0u;
        f.ry[k] = r_ok ? R.Y.a.v[k] : 0u;
        f.ry[4 + k] = r_ok ? R.Y.b.v[k] : 0u;
    }
}

namespace poslo {

// AVer over a batch, optionally leaving out the entries set in a device
// bitmap over batch positions (SeBVer mode V)
// Host-resident batches: copy the messages (and offsets) into the
// context's staging buffers on the stream; dm then describes the device
// copy.  A device batch is passed through.  sigs (80 per entry, may be null)
// follow the batch's memory kind and are staged when sigs_out is given.
int stage_msgs(poslo_ctx* c, const poslo_msgs* m, hipStream_t s, poslo_msgs& dm, const uint8_t* sigs,
               const uint8_t** sigs_out) {
    if (!c || !m) return POSLO_E_INVAL;
    dm = *m;
    if (sigs_out) *sigs_out = sigs;
    if (!m->host) return POSLO_OK;
    dm.host = 0;
    if (m->n == 0) return POSLO_OK;
    if (!m->data) return POSLO_E_INVAL;
    uint64_t need;
    if (m->offsets) {
        need = m->offsets[m->n];
        if (m->offsets[0] > need) return POSLO_E_INVAL;
    } else {
        if (m->msg_len && m->n > UINT64_MAX / m->msg_len) return POSLO_E_INVAL;
        need = m->n * m->msg_len;
    }
    uint64_t bytes = m->data_bytes ? m->data_bytes : need;
    if (bytes < need) return POSLO_E_INVAL;
    int st;
    void* d;
    if (hipSetDevice(c->device) != hipSuccess) return POSLO_E_DEVICE;
    if ((st = ctx_scratch(c, kSlotStageData, std::max<uint64_t>(bytes, 1), &d))) return st;
    HIP_TRY(hipMemcpyAsync(d, m->data, bytes, hipMemcpyHostToDevice, s));
    dm.data = (const uint8_t*)d;
    dm.data_bytes = bytes;
    if (m->offsets) {
        void* o;
        if ((st = ctx_scratch(c, kSlotStageOffsets, (m->n + 1) * 8, &o))) return st;
        HIP_TRY(hipMemcpyAsync(o, m->offsets, (m->n + 1) * 8, hipMemcpyHostToDevice, s));
        dm.offsets = (const uint64_t*)o;
    }
    if (sigs_out && sigs) {
        void* g;
        if ((st = ctx_scratch(c, kSlotStageSigs, m->n * 80, &g))) return st;
        HIP_TRY(hipMemcpyAsync(g, sigs, m->n * 80, hipMemcpyHostToDevice, s));
        *sigs_out = (const uint8_t*)g;
    }
    return POSLO_OK;
}

// The final fold of n_part partials, mod q and the check R = e*Y + s*G
// against the tag, with accept and e mod q read back (synchronizes s).
// E_INVAL if the device flag bad (when given) is set: POSLO++ met a message
// longer than 31 bytes.
int final_check(poslo_ctx* c, const KeyEntry* key, const uint32_t* partials, uint32_t n_part,
                const uint8_t tag[64], hipStream_t s, int* accept, uint8_t e_out[32], const uint32_t* bad) {
    FinalArgs f;
    f.partials = partials;
    f.n_part = n_part;
    f.ty = key->d_table;
    f.tg = key->fourq ? ctx_gtable_fq(c) : c->d_gtable;
    if (!f.tg) return POSLO_E_NOMEM;
    f.result = c->d_result;
    f.bad = bad;
    if (key->fourq) tag_checks_fq(tag, f);
    else tag_checks(tag, f);
    prof_begin(c, POSLO_KT_FINAL, s);
    if (key->fourq) hipLaunchKernelGGL(k_finalize_fq, dim3(1), dim3(kBlock), 0, s, f);
    else hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, f);
    HIP_TRY(hipGetLastError());
    prof_end(c, POSLO_KT_FINAL, s);
    HIP_TRY(hipMemcpyAsync(c->h_result, c->d_result, 16 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    prof_collect(c);
    if (c->h_result[9]) return POSLO_E_INVAL;
    *accept = c->h_result[8] ? 1 : 0;
    if (e_out)
        for (int w = 0; w < 8; w++) store_le32(e_out + 4 * w, c->h_result[w]);
    return POSLO_OK;
}

int aver_impl(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m_in, const uint8_t* ds,
              size_t ds_len, const uint8_t tag[64], void* stream, const uint32_t* skip, int* accept,
              uint8_t e_out[32]) {
    if (!pk || !tag || !accept) return POSLO_E_INVAL;
    *accept = 0;
    hipStream_t s = (hipStream_t)stream;
    poslo_msgs dm;
    int st = stage_msgs(c, m_in, s, dm, nullptr, nullptr);
    if (st) return st;
    const poslo_msgs* m = &dm;
    BatchArgs a;
    DsArg dsa;
    uint32_t n_epochs;
    if ((st = prepare_batch(c, prm, m, ds, ds_len, a, dsa, n_epochs))) return st;
    a.skip = skip;
    HIP_TRY(hipSetDevice(c->device));
    const KeyEntry* key = ctx_key_of(c, prm->inst, pk, &st);
    if (!key) return st;
    prof_begin(c, POSLO_KT_SEED, s);
    if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return st;
    prof_end(c, POSLO_KT_SEED, s);
    uint32_t n_part = 0;
    if (m->n > 0) {
        const AggShape g = agg_shape(c, prm, m);
        if ((st = ctx_ensure(&c->d_part, &c->part_words, (size_t)g.grid * 9))) return st;
        if ((st = launch_agg(c, prm, g, a, c->d_part, nullptr, nullptr, s))) return st;
        n_part = g.grid;
    }
    return final_check(c, key, c->d_part, n_part, tag, s, accept, e_out, n_epochs ? a.bad : nullptr);
}

}  // namespace poslo

extern "C" int poslo_aver(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m,
                          const uint8_t* ds, size_t ds_len, const uint8_t tag[64], void* stream, int* accept,
                          uint8_t e_out[32]) {
    return aver_impl(c, prm, pk, m, ds, ds_len, tag, stream, nullptr, accept, e_out);
}

extern "C" int poslo_ekeys(poslo_ctx* c, const poslo_params* prm, const poslo_msgs* m_in, const uint8_t* ds,
                           size_t ds_len, uint8_t* e_dev, uint8_t* x_dev, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    poslo_msgs dm;
    int st = stage_msgs(c, m_in, s, dm, nullptr, nullptr);
    if (st) return st;
    const poslo_msgs* m = &dm;
    BatchArgs a;
    DsArg dsa;
    uint32_t n_epochs;
    if ((st = prepare_batch(c, prm, m, ds, ds_len, a, dsa, n_epochs))) return st;
    if (m->n == 0) return POSLO_OK;
    if (!e_dev) return POSLO_E_INVAL;
    HIP_TRY(hipSetDevice(c->device));
    if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return st;
    // the AVer hot kernel's default shape, in its emit form
    const int saved = c->agg_variant;
    c->agg_variant = -1;
    const AggShape g = agg_shape(c, prm, m);
    c->agg_variant = saved;
    if ((st = ctx_ensure(&c->d_part, &c->part_words, (size_t)g.grid * 9))) return st;
    return launch_agg(c, prm, g, a, c->d_part, (uint32_t*)e_dev, (uint32_t*)x_dev, s);
}

// AVer with no device allocation: the epoch rows, partials and result words
// live in this device's fixed scratch array, the key's table must already be
// resident, and the launch shape is the default one (grid capped at the
// array's partial slots).
extern "C" int poslo_aver_fixed(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m,
                                const uint8_t* ds, size_t ds_len, const uint8_t tag[64], void* stream, int* accept,
                                uint8_t e_out[32]) {
    if (!c || !pk || !tag || !accept || !m || m->host) return POSLO_E_INVAL;
    *accept = 0;
    if (!c->d_fixed) return POSLO_E_DEVICE;
    uint32_t* fx_tab = c->d_fixed;
    uint32_t* fx_part = c->d_fixed + kFixedTabWords;
    uint32_t* fx_result = fx_part + kFixedPartWords;
    BatchArgs a;
    DsArg dsa;
    uint32_t n_epochs;
    int st = prepare_batch(c, prm, m, ds, ds_len, a, dsa, n_epochs, fx_tab, kFixedMaxEpochs);
    if (st) return st;
    // the key's comb table must be resident (poslo_ctx_keys_load): a lookup
    // that neither builds nor reorders anything
    const bool fourq = (prm->inst & POSLO_GROUP_FOURQ) != 0;
    const std::string id = fourq ? fq_key_id(pk) : std::string((const char*)pk, 32);
    const KeyEntry* key = nullptr;
    for (const KeyEntry& k : c->keys)
        if (k.pk == id) {
            key = &k;
            break;
        }
    if (!key) return POSLO_E_INVAL;
    if (fourq && !c->d_gtable_fq) return POSLO_E_INVAL;  // built by a poslo_aver call on FourQ
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return st;
    uint32_t n_part = 0;
    if (m->n > 0) {
        AggShape g = agg_shape(c, prm, m);
        g.grid = std::min(g.grid, kFixedMaxGrid);
        const uint32_t base = inst_base(prm->inst);
        st = base == INST_AES        ? launch_agg_aes(g.variant, g.fast, g.grid, &a, fx_part, s)
             : base == INST_AES_ADDQ ? launch_agg_addq(g.addq_layout, g.grid, &a, fx_part, nullptr, nullptr, s)
                                     : launch_agg_sha(g.sha_layout, g.grid, &a, fx_part, s);
        if (st) return st;
        n_part = g.grid;
    }
    FinalArgs f;
    f.partials = fx_part;
    f.n_part = n_part;
    f.ty = key->d_table;
    f.tg = c->d_gtable;
    f.result = fx_result;
    f.bad = n_epochs ? a.bad : nullptr;
    if (fourq) {
        f.tg = c->d_gtable_fq;
        tag_checks_fq(tag, f);
        hipLaunchKernelGGL(k_finalize_fq, dim3(1), dim3(kBlock), 0, s, f);
    } else {
        tag_checks(tag, f);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, f);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(c->h_result, fx_result, 16 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->h_result[9]) return POSLO_E_INVAL;
    *accept = c->h_result[8] ? 1 : 0;
    if (e_out)
        for (int w = 0; w < 8; w++) store_le32(e_out + 4 * w, c->h_result[w]);
    return POSLO_OK;
}
