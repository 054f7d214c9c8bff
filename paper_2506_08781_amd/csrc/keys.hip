// Device-resident public keys: fixed-base comb tables built on the device.
//
// The aggregate check e*Y + s*G (section "Fine-grained public-key POSLO",
// AVer; the paper's multiplicative Y^e * alpha^s read additively on
// edwards25519) uses per-key tables t[w][d] = d * 16^w * Y, 64 windows of 16
// points.  Building one on the host costs about a thousand point additions;
// for thousands of resident keys the device builds them instead, one wave
// per key: lane 0 decodes the key and walks the 64 window bases (four
// doublings apart), then lane w fills window w with 15 additions.
#include <string.h>

#include <algorithm>
#include <vector>

#include "ctx.h"
#include "ge25519.h"

namespace poslo {

__global__ __launch_bounds__(64) void k_comb_build(const uint8_t* pks, uint32_t* tables, uint32_t* ok) {
    __shared__ uint32_t base[kCombWindows * 32];
    __shared__ uint32_t good;
    const uint32_t key = blockIdx.x;
    if (threadIdx.x == 0) {
        uint8_t b[32];
        for (int k = 0; k < 32; k++) b[k] = pks[(uint64_t)key * 32 + k];
        ge P;
        bool g = ge_decode(P, b);
        good = g ? 1u : 0u;
        ok[key] = good;
        if (g) {
            for (int w = 0; w < kCombWindows; w++) {
                uint32_t* o = base + w * 32;
                for (int k = 0; k < 8; k++) {
                    o[k] = P.X.v[k];
                    o[8 + k] = P.Y.v[k];
                    o[16 + k] = P.Z.v[k];
                    o[24 + k] = P.T.v[k];
                }
                ge_dbl(P, P);
                ge_dbl(P, P);
                ge_dbl(P, P);
                ge_dbl(P, P);
            }
        }
    }
    __syncthreads();
    if (!good) return;
    const int w = threadIdx.x;  // one window per lane (64 lanes, 64 windows)
    ge B, T;
    for (int k = 0; k < 8; k++) {
        B.X.v[k] = base[w * 32 + k];
        B.Y.v[k] = base[w * 32 + 8 + k];
        B.Z.v[k] = base[w * 32 + 16 + k];
        B.T.v[k] = base[w * 32 + 24 + k];
    }
    ge_identity(T);
    uint32_t* dst = tables + (uint64_t)key * kCombWords + (uint64_t)w * 16 * 32;
    for (int d = 0; d < 16; d++) {
        uint4* o = reinterpret_cast<uint4*>(dst + d * 32);
        o[0] = make_uint4(T.X.v[0], T.X.v[1], T.X.v[2], T.X.v[3]);
        o[1] = make_uint4(T.X.v[4], T.X.v[5], T.X.v[6], T.X.v[7]);
        o[2] = make_uint4(T.Y.v[0], T.Y.v[1], T.Y.v[2], T.Y.v[3]);
        o[3] = make_uint4(T.Y.v[4], T.Y.v[5], T.Y.v[6], T.Y.v[7]);
        o[4] = make_uint4(T.Z.v[0], T.Z.v[1], T.Z.v[2], T.Z.v[3]);
        o[5] = make_uint4(T.Z.v[4], T.Z.v[5], T.Z.v[6], T.Z.v[7]);
        o[6] = make_uint4(T.T.v[0], T.T.v[1], T.T.v[2], T.T.v[3]);
        o[7] = make_uint4(T.T.v[4], T.T.v[5], T.T.v[6], T.T.v[7]);
        if (d < 15) ge_add(T, T, B);
    }
}

int ctx_keys_bulk(poslo_ctx* c, const uint8_t* pks, size_t n, std::vector<const uint32_t*>& tables, size_t* n_bad) {
    tables.assign(n, nullptr);
    if (n_bad) *n_bad = 0;
    if (n == 0) return POSLO_OK;
    if (!pks) return POSLO_E_INVAL;
    // keys of this call stay resident for its duration
    if (c->key_cap < 2 * n) c->key_cap = 2 * n;
    std::vector<std::string> missing;
    std::unordered_map<std::string, size_t> slot;
    for (size_t k = 0; k < n; k++) {
        std::string id((const char*)pks + 32 * k, 32);
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
        void *d_pks = nullptr, *d_ok = nullptr, *d_tab = nullptr;
        if (hipMalloc(&d_pks, m * 32) != hipSuccess) return POSLO_E_NOMEM;
        if (hipMalloc(&d_ok, m * 4) != hipSuccess) {
            hipFree(d_pks);
            return POSLO_E_NOMEM;
        }
        if (hipMalloc(&d_tab, m * (size_t)kCombWords * 4) != hipSuccess) {
            hipFree(d_pks);
            hipFree(d_ok);
            return POSLO_E_NOMEM;
        }
        std::shared_ptr<void> slab(d_tab, [](void* q) { hipFree(q); });
        std::vector<uint32_t> ok(m, 0);
        bool fail = hipMemcpy(d_pks, h_pks.data(), m * 32, hipMemcpyHostToDevice) != hipSuccess;
        if (!fail) {
            hipLaunchKernelGGL(k_comb_build, dim3((uint32_t)m), dim3(64), 0, 0, (const uint8_t*)d_pks,
                               (uint32_t*)d_tab, (uint32_t*)d_ok);
            fail = hipGetLastError() != hipSuccess ||
                   hipMemcpy(ok.data(), d_ok, m * 4, hipMemcpyDeviceToHost) != hipSuccess;
        }
        hipFree(d_pks);
        hipFree(d_ok);
        if (fail) return POSLO_E_DEVICE;
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
            ke.d_table = (uint32_t*)d_tab + k * (size_t)kCombWords;
            ke.slab = slab;
            c->keys.push_front(ke);
            c->key_index[missing[k]] = c->keys.begin();
            built[k] = ke.d_table;
        }
        for (size_t k = 0; k < n; k++) {
            if (tables[k]) continue;
            tables[k] = built[slot[std::string((const char*)pks + 32 * k, 32)]];
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
