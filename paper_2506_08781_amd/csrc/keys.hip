// Device-resident public keys: fixed-base comb tables built on the device.
//
// The aggregate check e*Y + s*G (section "Fine-grained public-key POSLO",
// AVer; the paper's multiplicative Y^e * alpha^s read additively on
// edwards25519) and the individual checks read per-key tables of 32 windows
// of 128 affine points (comb.h).  One workgroup of 128 threads builds one
// table: thread i forms (i + 1) * Y by double-and-add, then walks the 32
// windows eight doublings apart, converting each point to affine form.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "comb.h"
#include "ctx.h"
#include "device_ec.h"
#include "device_fq.h"
#include "fourq.h"
#include "ge25519.h"

namespace poslo {

__global__ __launch_bounds__(kCombPerWindow) void k_comb_build(const uint8_t* pks, uint32_t* tables, uint32_t* ok) {
    const uint32_t key = blockIdx.x;
    uint8_t b[32];
    for (int k = 0; k < 32; k++) b[k] = pks[(uint64_t)key * 32 + k];
    ge Y;
    const bool good = ge_decode(Y, b);
    if (threadIdx.x == 0) ok[key] = good ? 1u : 0u;
    if (!good) return;
    const uint32_t m = threadIdx.x + 1;  // 1..128
    ge P;
    ge_identity(P);
    for (int bit = 7; bit >= 0; bit--) {
        ge_dbl(P, P);
        if ((m >> bit) & 1u) ge_add(P, P, Y);
    }
    uint32_t* dst = tables + (uint64_t)key * kCombWords + (uint64_t)threadIdx.x * kCombEntryWords;
    for (int w = 0; w < kCombWindows; w++) {
        uint32_t o[kCombEntryWords];
        comb_entry_of(o, P);
        uint4* q = reinterpret_cast<uint4*>(dst + (uint64_t)w * kCombPerWindow * kCombEntryWords);
#pragma unroll
        for (int k = 0; k < kCombEntryWords / 4; k++) q[k] = make_uint4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
        if (w + 1 < kCombWindows)
            for (int k = 0; k < 8; k++) ge_dbl(P, P);
    }
}

// The same table for a FourQ key (fourq.h: GF(p^2) coordinates in the same
// 24-word entries)
__global__ __launch_bounds__(kCombPerWindow) void k_comb_build_fq(const uint8_t* pks, uint32_t* tables, uint32_t* ok) {
    const uint32_t key = blockIdx.x;
    uint8_t b[32];
    for (int k = 0; k < 32; k++) b[k] = pks[(uint64_t)key * 32 + k];
    gq Y;
    const bool good = fq_decode(Y, b);
    if (threadIdx.x == 0) ok[key] = good ? 1u : 0u;
    if (!good) return;
    const uint32_t m = threadIdx.x + 1;  // 1..128
    gq P;
    gq_identity(P);
    for (int bit = 7; bit >= 0; bit--) {
        gq_dbl(P, P);
        if ((m >> bit) & 1u) gq_add(P, P, Y);
    }
    uint32_t* dst = tables + (uint64_t)key * kCombWords + (uint64_t)threadIdx.x * kCombEntryWords;
    for (int w = 0; w < kCombWindows; w++) {
        uint32_t o[kCombEntryWords];
        fq_comb_entry_of(o, P);
        uint4* q = reinterpret_cast<uint4*>(dst + (uint64_t)w * kCombPerWindow * kCombEntryWords);
#pragma unroll
        for (int k = 0; k < kCombEntryWords / 4; k++) q[k] = make_uint4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
        if (w + 1 < kCombWindows)
            for (int k = 0; k < 8; k++) gq_dbl(P, P);
    }
}

// Wide table of a point P from its 8-bit table t8.  Entry (w, m - 1) is
// m * 65536^w * P for m = 1 .. 32768; written m = 256 d1 + d0 with d0 in
// [-127, 128] and d1 in [0, 128], it is the sum of t8's entries (2w, d0) and
// (2w + 1, d1): two lookups and two mixed additions.  Each thread forms
// kWideBuildK consecutive entries of one window and converts them to affine
// form with one inversion (Montgomery's trick): the projective X, Y, Z wait
// in the entries' own table slots, the running products of the Z's in LDS.
constexpr int kWideBuildK = 8;
constexpr int kWideBuildBlock = 128;
static_assert(kWidePerWindow % kWideBuildK == 0, "a thread's entries share one window");

__global__ __launch_bounds__(kWideBuildBlock) void k_wide_build(const uint32_t* t8, uint32_t* wide) {
    __shared__ uint32_t cs[kWideBuildK * 8 * kWideBuildBlock];  // c_k = Z_0 ... Z_k, word j at (8k + j) * block
    uint32_t* my = cs + threadIdx.x;
    const uint32_t first = (blockIdx.x * kWideBuildBlock + threadIdx.x) * kWideBuildK;
    const int w = (int)(first / kWidePerWindow);
    fe c;
#pragma unroll 1
    for (int k = 0; k < kWideBuildK; k++) {
        const uint32_t m = first % kWidePerWindow + k + 1;
        int d0 = (int)(m & 255u), d1 = (int)(m >> 8);
        if (d0 > 128) {
            d0 -= 256;
            d1 += 1;
        }
        ge P;
        ge_identity(P);
        gn q;
        comb_lookup(q, t8, 2 * w, d0);
        ge_madd(P, P, q);
        comb_lookup(q, t8, 2 * w + 1, d1);
        ge_madd(P, P, q);
        uint4* o = reinterpret_cast<uint4*>(wide + (uint64_t)(first + k) * kCombEntryWords);
        o[0] = make_uint4(P.X.v[0], P.X.v[1], P.X.v[2], P.X.v[3]);
        o[1] = make_uint4(P.X.v[4], P.X.v[5], P.X.v[6], P.X.v[7]);
        o[2] = make_uint4(P.Y.v[0], P.Y.v[1], P.Y.v[2], P.Y.v[3]);
        o[3] = make_uint4(P.Y.v[4], P.Y.v[5], P.Y.v[6], P.Y.v[7]);
        o[4] = make_uint4(P.Z.v[0], P.Z.v[1], P.Z.v[2], P.Z.v[3]);
        o[5] = make_uint4(P.Z.v[4], P.Z.v[5], P.Z.v[6], P.Z.v[7]);
        if (k == 0)
            c = P.Z;
        else
            fe_mul(c, c, P.Z);
#pragma unroll
        for (int j = 0; j < 8; j++) my[(8 * k + j) * kWideBuildBlock] = c.v[j];
    }
    fe inv;
    fe_inv(inv, c);  // 1 / (Z_0 ... Z_{K-1})
#pragma unroll 1
    for (int k = kWideBuildK - 1; k >= 0; k--) {
        uint32_t* o = wide + (uint64_t)(first + k) * kCombEntryWords;
        fe X, Y, Z, zi;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            X.v[j] = o[j];
            Y.v[j] = o[8 + j];
            Z.v[j] = o[16 + j];
        }
        if (k > 0) {
            fe ck;
#pragma unroll
            for (int j = 0; j < 8; j++) ck.v[j] = my[(8 * (k - 1) + j) * kWideBuildBlock];
            fe_mul(zi, inv, ck);
            fe_mul(inv, inv, Z);
        } else {
            zi = inv;
        }
        uint32_t e[kCombEntryWords];
        comb_entry_zinv(e, X, Y, zi);
        uint4* q4 = reinterpret_cast<uint4*>(o);
#pragma unroll
        for (int t = 0; t < kCombEntryWords / 4; t++) q4[t] = make_uint4(e[4 * t], e[4 * t + 1], e[4 * t + 2], e[4 * t + 3]);
    }
}

// The same for FourQ (fourq.h): entries of FourQ's comb layout, GF(p^2)
// arithmetic, one GF(p^2) inversion per kWideBuildK entries
__global__ __launch_bounds__(kWideBuildBlock) void k_wide_build_fq(const uint32_t* t8, uint32_t* wide) {
    __shared__ uint32_t cs[kWideBuildK * 8 * kWideBuildBlock];
    uint32_t* my = cs + threadIdx.x;
    const uint32_t first = (blockIdx.x * kWideBuildBlock + threadIdx.x) * kWideBuildK;
    const int w = (int)(first / kWidePerWindow);
    fp2 c;
#pragma unroll 1
    for (int k = 0; k < kWideBuildK; k++) {
        const uint32_t m = first % kWidePerWindow + k + 1;
        int d0 = (int)(m & 255u), d1 = (int)(m >> 8);
        if (d0 > 128) {
            d0 -= 256;
            d1 += 1;
        }
        gq P;
        gq_identity(P);
        gnq q;
        fq_comb_lookup(q, t8, 2 * w, d0);
        gq_madd(P, P, q);
        fq_comb_lookup(q, t8, 2 * w + 1, d1);
        gq_madd(P, P, q);
        uint32_t* o = wide + (uint64_t)(first + k) * kCombEntryWords;
        stash_f2(o, 1, P.X);
        stash_f2(o + 8, 1, P.Y);
        stash_f2(o + 16, 1, P.Z);
        if (k == 0)
            c = P.Z;
        else
            f2_mul(c, c, P.Z);
        stash_f2(my + 8 * k * kWideBuildBlock, kWideBuildBlock, c);
    }
    fp2 inv;
    f2_inv(inv, c);
#pragma unroll 1
    for (int k = kWideBuildK - 1; k >= 0; k--) {
        uint32_t* o = wide + (uint64_t)(first + k) * kCombEntryWords;
        fp2 X, Y, Z, zi;
        unstash_f2(X, o, 1);
        unstash_f2(Y, o + 8, 1);
        unstash_f2(Z, o + 16, 1);
        if (k > 0) {
            fp2 ck;
            unstash_f2(ck, my + 8 * (k - 1) * kWideBuildBlock, kWideBuildBlock);
            f2_mul(zi, inv, ck);
            f2_mul(inv, inv, Z);
        } else {
            zi = inv;
        }
        uint32_t e[kCombEntryWords];
        fq_comb_entry_zinv(e, X, Y, zi);
        for (int t = 0; t < kCombEntryWords; t++) o[t] = e[t];
    }
}

static uint32_t* build_wide_fq(const uint32_t* t8) {
    uint32_t* d = nullptr;
    if (hipMalloc((void**)&d, kWideWords * 4) != hipSuccess) return nullptr;
    const uint32_t blocks = (uint32_t)(kWideWindows * kWidePerWindow / (kWideBuildK * kWideBuildBlock));
    hipLaunchKernelGGL(k_wide_build_fq, dim3(blocks), dim3(kWideBuildBlock), 0, 0, t8, d);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
        hipFree(d);
        return nullptr;
    }
    return d;
}

static uint32_t* build_wide(const uint32_t* t8) {
    uint32_t* d = nullptr;
    if (hipMalloc((void**)&d, kWideWords * 4) != hipSuccess) return nullptr;
    const uint32_t blocks = (uint32_t)(kWideWindows * kWidePerWindow / (kWideBuildK * kWideBuildBlock));
    hipLaunchKernelGGL(k_wide_build, dim3(blocks), dim3(kWideBuildBlock), 0, 0, t8, d);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
        hipFree(d);
        return nullptr;
    }
    return d;
}

const uint32_t* ctx_gtable_wide(poslo_ctx* c) {
    std::lock_guard<std::mutex> lk(c->wide_mu);
    if (!c->d_gtable_wide) c->d_gtable_wide = build_wide(c->d_gtable);
    return c->d_gtable_wide;
}

const uint32_t* ctx_gtable_wide_fq(poslo_ctx* c) {
    const uint32_t* t8 = ctx_gtable_fq(c);
    if (!t8) return nullptr;
    std::lock_guard<std::mutex> lk(c->wide_mu);
    if (!c->d_gtable_wide_fq) c->d_gtable_wide_fq = build_wide_fq(t8);
    return c->d_gtable_wide_fq;
}

const uint32_t* ctx_key_wide(poslo_ctx* c, const uint8_t pk[32]) {
    auto it = c->key_index.find(std::string((const char*)pk, 32));
    if (it == c->key_index.end()) return nullptr;
    KeyEntry& ke = *it->second;
    if (ke.wide) return (const uint32_t*)ke.wide.get();
    // keep at most kMaxWideKeys wide key tables built on demand: drop the
    // least recently used (widened keys keep theirs)
    size_t have = 0;
    for (const KeyEntry& k : c->keys) have += k.wide != nullptr && !k.wide_pinned;
    if (have >= kMaxWideKeys) {
        hipDeviceSynchronize();  // queued work may still read them
        for (auto r = c->keys.rbegin(); r != c->keys.rend() && have >= kMaxWideKeys; ++r)
            if (r->wide && !r->wide_pinned && &*r != &ke) {
                r->wide.reset();
                have--;
            }
    }
    uint32_t* d = build_wide(ke.d_table);
    if (!d) return nullptr;
    ke.wide = std::shared_ptr<void>(d, [](void* q) { hipFree(q); });
    return d;
}

const uint32_t* ctx_key_wide_resident(poslo_ctx* c, const uint8_t pk[32]) {
    auto it = c->key_index.find(std::string((const char*)pk, 32));
    return it == c->key_index.end() ? nullptr : (const uint32_t*)it->second->wide.get();
}

static int build_tables(bool fourq, const uint8_t* pks, size_t m, uint32_t* d_tab, std::vector<uint32_t>& ok) {
    ok.assign(m, 0);
    if (m == 0) return POSLO_OK;
    void *d_pks = nullptr, *d_ok = nullptr;
    if (hipMalloc(&d_pks, m * 32) != hipSuccess) return POSLO_E_NOMEM;
    if (hipMalloc(&d_ok, m * 4) != hipSuccess) {
        hipFree(d_pks);
        return POSLO_E_NOMEM;
    }
    bool fail = hipMemcpy(d_pks, pks, m * 32, hipMemcpyHostToDevice) != hipSuccess;
    if (!fail) {
        if (fourq)
            hipLaunchKernelGGL(k_comb_build_fq, dim3((uint32_t)m), dim3(kCombPerWindow), 0, 0, (const uint8_t*)d_pks,
                               d_tab, (uint32_t*)d_ok);
        else
            hipLaunchKernelGGL(k_comb_build, dim3((uint32_t)m), dim3(kCombPerWindow), 0, 0, (const uint8_t*)d_pks,
                               d_tab, (uint32_t*)d_ok);
        fail = hipGetLastError() != hipSuccess ||
               hipMemcpy(ok.data(), d_ok, m * 4, hipMemcpyDeviceToHost) != hipSuccess;
    }
    hipFree(d_pks);
    hipFree(d_ok);
    return fail ? POSLO_E_DEVICE : POSLO_OK;
}

const uint32_t* ctx_gtable_fq(poslo_ctx* c) {
    std::lock_guard<std::mutex> lk(c->wide_mu);
    if (c->d_gtable_fq) return c->d_gtable_fq;
    fp2 gx, gy;
    fq_gen_xy(gx, gy);
    gq G;
    gq_from_affine(G, gx, gy);
    uint8_t enc[32];
    fq_encode(enc, G);
    uint32_t* d = nullptr;
    if (hipMalloc((void**)&d, (size_t)kCombWords * 4) != hipSuccess) return nullptr;
    std::vector<uint32_t> ok;
    if (build_tables(true, enc, 1, d, ok) || !ok[0]) {
        hipFree(d);
        return nullptr;
    }
    c->d_gtable_fq = d;
    return d;
}

const KeyEntry* ctx_key_fq(poslo_ctx* c, const uint8_t pk[32], int* status) {
    const std::string id = fq_key_id(pk);
    auto it = c->key_index.find(id);
    if (it != c->key_index.end()) {
        c->keys.splice(c->keys.begin(), c->keys, it->second);
        *status = POSLO_OK;
        return &*it->second;
    }
    void* d_tab = nullptr;
    if (hipMalloc(&d_tab, (size_t)kCombWords * 4) != hipSuccess) {
        *status = POSLO_E_NOMEM;
        return nullptr;
    }
    std::shared_ptr<void> slab(d_tab, [](void* q) { hipFree(q); });
    std::vector<uint32_t> ok;
    if ((*status = build_tables(true, pk, 1, (uint32_t*)d_tab, ok))) return nullptr;
    if (!ok[0]) {
        *status = POSLO_E_ENCODING;
        return nullptr;
    }
    if (c->keys.size() + 1 > c->key_cap) {
        hipDeviceSynchronize();  // queued work may still read evicted tables
        while (c->keys.size() + 1 > c->key_cap && !c->keys.empty()) {
            c->key_index.erase(c->keys.back().pk);
            c->keys.pop_back();
        }
    }
    KeyEntry ke;
    ke.pk = id;
    ke.fourq = true;
    ke.d_table = (uint32_t*)d_tab;
    ke.slab = slab;
    c->keys.push_front(ke);
    c->key_index[id] = c->keys.begin();
    *status = POSLO_OK;
    return &c->keys.front();
}

const KeyEntry* ctx_key_of(poslo_ctx* c, uint32_t inst, const uint8_t pk[32], int* status) {
    return (inst & POSLO_GROUP_FOURQ) ? ctx_key_fq(c, pk, status) : ctx_key(c, pk, status);
}

int build_comb_tables(const uint8_t* pks, size_t m, uint32_t* d_tab, std::vector<uint32_t>& ok) {
    return build_tables(false, pks, m, d_tab, ok);
}

int ctx_keys_bulk(poslo_ctx* c, const uint8_t* pks, size_t n, std::vector<const uint32_t*>& tables, size_t* n_bad,
                  bool fourq) {
    auto id_of = [&](const uint8_t* pk) {
        return fourq ? fq_key_id(pk) : std::string((const char*)pk, 32);
    };
    tables.assign(n, nullptr);
    if (n_bad) *n_bad = 0;
    if (n == 0) return POSLO_OK;
    if (!pks) return POSLO_E_INVAL;
    // keys of this call stay resident for its duration
    if (c->key_cap < 2 * n) c->key_cap = 2 * n;
    std::vector<std::string> missing;
    std::unordered_map<std::string, size_t> slot;
    for (size_t k = 0; k < n; k++) {
        const std::string id = id_of(pks + 32 * k);
        auto it = c->key_index.find(id);
        if (it != c->key_index.end()) {
            c->keys.splice(c->keys.begin(), c->keys, it->second);
            tables[k] = it->second->d_table;
        } else if (slot.emplace(id, missing.size()).second) {
            missing.push_back(id);
        }
    }
    if (!missing.empty()) {
        size_t m = missing.size();
        std::vector<uint8_t> h_pks(m * 32);
        for (size_t k = 0; k < m; k++) memcpy(&h_pks[32 * k], missing[k].data(), 32);
        void* d_tab = nullptr;
        if (hipMalloc(&d_tab, m * (size_t)kCombWords * 4) != hipSuccess) return POSLO_E_NOMEM;
        std::shared_ptr<void> slab(d_tab, [](void* q) { hipFree(q); });
        std::vector<uint32_t> ok;
        int st = build_tables(fourq, h_pks.data(), m, (uint32_t*)d_tab, ok);
        if (st) return st;
        // make room: evict least recently used keys not touched by this call
        size_t good = 0;
        for (size_t k = 0; k < m; k++) good += ok[k] != 0;
        if (c->keys.size() + good > c->key_cap) {
            hipDeviceSynchronize();
            while (c->keys.size() + good > c->key_cap && !c->keys.empty()) {
                c->key_index.erase(c->keys.back().pk);
                c->keys.pop_back();
            }
        }
        std::vector<const uint32_t*> built(m, nullptr);
        for (size_t k = 0; k < m; k++) {
            if (!ok[k]) continue;
            KeyEntry ke;
            ke.pk = missing[k];
            ke.fourq = fourq;
            ke.d_table = (uint32_t*)d_tab + k * (size_t)kCombWords;
            ke.slab = slab;
            c->keys.push_front(ke);
            c->key_index[missing[k]] = c->keys.begin();
            built[k] = ke.d_table;
        }
        for (size_t k = 0; k < n; k++) {
            if (tables[k]) continue;
            tables[k] = built[slot[id_of(pks + 32 * k)]];
        }
    }
    // duplicates of a bad key count once per occurrence
    size_t bad_occ = 0;
    for (size_t k = 0; k < n; k++) bad_occ += tables[k] == nullptr;
    if (n_bad) *n_bad = bad_occ;
    return bad_occ ? POSLO_E_ENCODING : POSLO_OK;
}

}  // namespace poslo

using namespace poslo;

extern "C" int poslo_ctx_keys_load(poslo_ctx* c, const uint8_t* pks, size_t n, size_t* n_bad) {
    if (!c || (n && !pks)) return POSLO_E_INVAL;
    if (hipSetDevice(c->device) != hipSuccess) return POSLO_E_DEVICE;
    std::vector<const uint32_t*> t;
    return ctx_keys_bulk(c, pks, n, t, n_bad);
}

extern "C" int poslo_ctx_keys_widen(poslo_ctx* c, const uint8_t* pks, size_t n) {
    if (!c || (n && !pks)) return POSLO_E_INVAL;
    if (hipSetDevice(c->device) != hipSuccess) return POSLO_E_DEVICE;
    std::vector<const uint32_t*> t;
    size_t n_bad = 0;
    const int st = ctx_keys_bulk(c, pks, n, t, &n_bad);
    if (st != POSLO_OK && st != POSLO_E_ENCODING) return st;
    for (size_t k = 0; k < n; k++) {
        if (!t[k]) continue;  // not a point encoding
        auto it = c->key_index.find(std::string((const char*)pks + 32 * k, 32));
        if (it == c->key_index.end()) return POSLO_E_DEVICE;
        KeyEntry& ke = *it->second;
        if (!ke.wide) {
            uint32_t* d = build_wide(ke.d_table);
            if (!d) return POSLO_E_NOMEM;
            ke.wide = std::shared_ptr<void>(d, [](void* q) { hipFree(q); });
        }
        ke.wide_pinned = true;
    }
    return st;
}
