// POSLO-C on the verifier (paper figure "Coarse-grained signer-optimal
// POSLO": AVer, Distill, SeBVer), on the POSLO-F kernels.
//
// The public key holds Y and one aggregate commitment R~_i per epoch; an
// epoch's signature is s~_i.  AVer over whole epochs is the POSLO-F AVer
// with the tag (sum of s~, sum of the epochs' R~_i): the same seed rows,
// hot kernel and final check.  The key is loaded once: the R~_i are decoded
// on the host, kept as prefix sums (so the R~ of a range of epochs is one
// point subtraction) and as affine points on the device.  Distill checks
// every epoch on its own: the hot kernel's emit form writes every entry's
// e_t mod q, and one wave per epoch sums the epoch's e_t (the paper's
// per-block sub-aggregates e~_i) and checks e~_i*Y + s~_i*G = R~_i with the
// fixed-base tables.  SeBVer V and U are the POSLO-F ones over the entries
// of the valid epochs; I re-verifies each invalid epoch.  On the FourQ group
// (fourq.h) the same steps run with FourQ's points and scalars mod N.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ccd.h"
#include "ctx.h"
#include "device_ec.h"
#include "device_entry.h"
#include "device_fq.h"
#include "scheme_host.h"

namespace poslo {

// e~_i = sum of the epoch's e_t mod q, then e~_i*Y + s~_i*G = R~_i (R~_i
// affine, 16 words per epoch) and s~_i < q: one wave per epoch.  FQ: on
// FourQ (mod N; x and y of R~_i as GF(p^2) words)
template <bool FQ>
__global__ __launch_bounds__(64) void k_c_epoch_check(const uint32_t* ek, uint32_t log2_n2, const uint32_t* s_ep,
                                                      const uint32_t* r_aff, const uint32_t* ty, const uint32_t* tg,
                                                      uint32_t* res) {
    const uint64_t p = blockIdx.x;
    const uint64_t n2 = 1ull << log2_n2;
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t j = threadIdx.x; j < n2; j += 64) {
        uint32_t d[8];
#pragma unroll
        for (int k = 0; k < 8; k++) d[k] = ek[(p * n2 + j) * 8 + k];
        acc288_add256(acc, d);
    }
    wave_reduce288(acc);
    uint32_t e[8], s[8];
    for (int k = 0; k < 8; k++) s[k] = s_ep[p * 8 + k];
    if constexpr (FQ) {
        scN_reduce<9>(e, acc);
        const bool canon = scN_is_canonical(s);
        if (!canon)
            for (int k = 0; k < 8; k++) s[k] = 0;  // any in-range digits; the result is 0 anyway
        gq P;
        wave_double_scalar_fq(P, ty, tg, e, s);
        if (threadIdx.x == 0) {
            fp2 rx, ry, t0, t1;
            unstash_f2(rx, r_aff + p * 16, 1);
            unstash_f2(ry, r_aff + p * 16 + 8, 1);
            f2_mul(t0, rx, P.Z);
            f2_mul(t1, ry, P.Z);
            res[p] = (canon && f2_eq(t0, P.X) && f2_eq(t1, P.Y)) ? 1u : 0u;
        }
    } else {
        sc_reduce288(e, acc);
        ge P;
        wave_double_scalar(P, ty, tg, e, s);
        if (threadIdx.x == 0) {
            fe rx, ry, t0, t1;
            for (int k = 0; k < 8; k++) {
                rx.v[k] = r_aff[p * 16 + k];
                ry.v[k] = r_aff[p * 16 + 8 + k];
            }
            fe_mul(t0, rx, P.Z);
            fe_mul(t1, ry, P.Z);
            res[p] = (sc_is_canonical(s) && fe_equal(t0, P.X) && fe_equal(t1, P.Y)) ? 1u : 0u;
        }
    }
}

int aver_impl(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m, const uint8_t* ds,
              size_t ds_len, const uint8_t tag[64], void* stream, const uint32_t* skip, int* accept,
              uint8_t e_out[32]);
int sebver_impl(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const poslo_msgs* m,
                const poslo_ccd* ccd, char mode, uint8_t* bits, size_t cap, size_t* n_bits, void* stream);

}  // namespace poslo

using namespace poslo;

struct poslo_c_key {
    int device = 0;
    uint32_t log2_n1 = 0;
    bool fq = false;             // FourQ key: the gq vectors hold the points
    uint8_t y[32] = {};
    std::vector<uint8_t> r_enc;  // enc(R~_i), 32 bytes per epoch
    std::vector<ge> prefix;      // prefix[k] = R~_0 + ... + R~_{k-1}
    std::vector<ge> r;           // R~_i decoded (Z = 1)
    std::vector<gq> prefix_q;    // the same on FourQ
    std::vector<gq> r_q;
    uint32_t* d_r = nullptr;     // affine (x, y) of R~_i, 16 words per epoch
};

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

namespace {

// whole epochs of the key's tree: [i0, i0 + k)
int epoch_range(const poslo_params* prm, const poslo_c_key* key, const poslo_msgs* m, uint64_t& i0, uint64_t& k) {
    if (!prm || !key || !m || prm->log2_n1 != key->log2_n1) return POSLO_E_INVAL;
    const uint64_t n2 = 1ull << prm->log2_n2;
    if ((m->t0 & (n2 - 1)) || (m->n & (n2 - 1))) return POSLO_E_INVAL;  // AVer takes whole epochs
    i0 = m->t0 >> prm->log2_n2;
    k = m->n >> prm->log2_n2;
    if (i0 > (1ull << key->log2_n1) || k > (1ull << key->log2_n1) - i0) return POSLO_E_INVAL;
    return POSLO_OK;
}

// the group operations range_sum needs, on edwards25519 (ge) and FourQ (gq)
inline void pt_identity(ge& r) { ge_identity(r); }
inline void pt_identity(gq& r) { gq_identity(r); }
inline void pt_add(ge& r, const ge& p, const ge& q) { ge_add(r, p, q); }
inline void pt_add(gq& r, const gq& p, const gq& q) { gq_add(r, p, q); }
inline void pt_neg(ge& r, const ge& p) { ge_neg(r, p); }
inline void pt_neg(gq& r, const gq& p) {
    f2_neg(r.X, p.X);
    r.Y = p.Y;
    r.Z = p.Z;
    f2_neg(r.T, p.T);
}

// R~_i summed over the epochs [a, b) of the key that are not in `bad`
// (sorted absolute epoch indices): the prefix difference minus the bad ones,
// or the direct sum of the good ones, whichever takes fewer additions
template <class PT>
void range_sum_of(const std::vector<PT>& prefix, const std::vector<PT>& r, uint64_t a, uint64_t b,
                  const std::vector<uint64_t>& bad, PT& out) {
    auto lo = std::lower_bound(bad.begin(), bad.end(), a);
    auto hi = std::lower_bound(bad.begin(), bad.end(), b);
    const uint64_t nbad = (uint64_t)(hi - lo);
    if (nbad + 2 <= (b - a) - nbad) {
        PT neg;
        pt_neg(neg, prefix[a]);
        pt_add(out, prefix[b], neg);
        for (auto it = lo; it != hi; ++it) {
            pt_neg(neg, r[*it]);
            pt_add(out, out, neg);
        }
    } else {
        pt_identity(out);
        for (uint64_t i = a; i < b; i++) {
            if (lo != hi && *lo == i) {
                ++lo;
                continue;
            }
            pt_add(out, out, r[i]);
        }
    }
}

// enc of the sum of R~_i over [a, b) minus `bad`, on the key's group
void range_sum_enc(const poslo_c_key* key, uint64_t a, uint64_t b, const std::vector<uint64_t>& bad,
                   uint8_t out[32]) {
    if (key->fq) {
        gq R;
        range_sum_of(key->prefix_q, key->r_q, a, b, bad, R);
        fq_encode(out, R);
    } else {
        ge R;
        range_sum_of(key->prefix, key->r, a, b, bad, R);
        ge_encode(out, R);
    }
}

// sum of s~_i over the epochs [a, b) (positions in s_epochs) not in `bad`,
// mod q (mod N on FourQ)
void sum_s(const poslo_c_key* key, const uint8_t* s_epochs, uint64_t a, uint64_t b, const std::vector<uint64_t>& bad,
           uint64_t i0, uint8_t out[32]) {
    const uint32_t inst = key->fq ? POSLO_GROUP_FOURQ : 0u;
    uint32_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto lo = std::lower_bound(bad.begin(), bad.end(), i0 + a);
    for (uint64_t p = a; p < b; p++) {
        if (lo != bad.end() && *lo == i0 + p) {
            ++lo;
            continue;
        }
        uint32_t sp[8], tmp[8];
        hostside::scalar_from_bytes(inst, sp, s_epochs + 32 * p);
        if (key->fq)
            scN_add(tmp, acc, sp);
        else
            sc_add(tmp, acc, sp);
        memcpy(acc, tmp, sizeof acc);
    }
    for (int w = 0; w < 8; w++) store_le32(out + 4 * w, acc[w]);
}

}  // namespace

extern "C" int poslo_c_key_load(poslo_ctx* c, const poslo_params* prm, const uint8_t* pk, size_t pk_len,
                                poslo_c_key** out) {
    if (!c || !params_ok(prm) || !pk || !out || prm->log2_n1 > 20) return POSLO_E_INVAL;
    *out = nullptr;
    const uint64_t n1 = 1ull << prm->log2_n1;
    if (pk_len != 32 * (1 + n1)) return POSLO_E_INVAL;
    poslo_c_key* key = new (std::nothrow) poslo_c_key();
    if (!key) return POSLO_E_NOMEM;
    key->device = c->device;
    key->log2_n1 = prm->log2_n1;
    key->fq = (prm->inst & POSLO_GROUP_FOURQ) != 0;
    memcpy(key->y, pk, 32);
    key->r_enc.assign(pk + 32, pk + pk_len);
    std::vector<uint32_t> aff(16 * n1);
    bool ok;
    if (key->fq) {
        key->r_q.resize(n1);
        key->prefix_q.resize(n1 + 1);
        gq_identity(key->prefix_q[0]);
        gq Y;
        ok = fq_decode(Y, pk);
        for (uint64_t i = 0; ok && i < n1; i++) {
            ok = fq_decode(key->r_q[i], pk + 32 * (1 + i));
            if (!ok) break;
            gq_add(key->prefix_q[i + 1], key->prefix_q[i], key->r_q[i]);
            for (int w = 0; w < 4; w++) {
                aff[16 * i + w] = key->r_q[i].X.a.v[w];
                aff[16 * i + 4 + w] = key->r_q[i].X.b.v[w];
                aff[16 * i + 8 + w] = key->r_q[i].Y.a.v[w];
                aff[16 * i + 12 + w] = key->r_q[i].Y.b.v[w];
            }
        }
    } else {
        key->r.resize(n1);
        key->prefix.resize(n1 + 1);
        ge_identity(key->prefix[0]);
        ge Y;
        ok = ge_decode(Y, pk);
        for (uint64_t i = 0; ok && i < n1; i++) {
            ok = ge_decode(key->r[i], pk + 32 * (1 + i));
            if (!ok) break;
            ge_add(key->prefix[i + 1], key->prefix[i], key->r[i]);
            for (int w = 0; w < 8; w++) {
                aff[16 * i + w] = key->r[i].X.v[w];
                aff[16 * i + 8 + w] = key->r[i].Y.v[w];
            }
        }
    }
    int st = ok ? POSLO_OK : POSLO_E_ENCODING;
    if (!st && hipSetDevice(c->device) != hipSuccess) st = POSLO_E_DEVICE;
    if (!st && hipMalloc((void**)&key->d_r, aff.size() * 4) != hipSuccess) st = POSLO_E_NOMEM;
    if (!st && hipMemcpy(key->d_r, aff.data(), aff.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        st = POSLO_E_DEVICE;
    if (!st) ctx_key_of(c, prm->inst, key->y, &st);  // Y's comb table resident in the context
    if (!st && key->fq && !ctx_gtable_fq(c)) st = POSLO_E_NOMEM;
    if (st) {
        poslo_c_key_free(key);
        return st;
    }
    *out = key;
    return POSLO_OK;
}

extern "C" void poslo_c_key_free(poslo_c_key* key) {
    if (!key) return;
    if (key->d_r) {
        (void)hipSetDevice(key->device);
        (void)hipFree(key->d_r);
    }
    delete key;
}

extern "C" int poslo_c_aver(poslo_ctx* c, const poslo_params* prm, const poslo_c_key* key, const poslo_msgs* m,
                            const uint8_t* ds, size_t ds_len, const uint8_t s[32], void* stream, int* accept,
                            uint8_t e_out[32]) {
    if (!c || !s || !accept) return POSLO_E_INVAL;
    *accept = 0;
    uint64_t i0, k;
    int st = epoch_range(prm, key, m, i0, k);
    if (st) return st;
    if (((prm->inst & POSLO_GROUP_FOURQ) != 0) != key->fq) return POSLO_E_INVAL;
    // R~ = Agg of the epochs' commitments in pk
    uint8_t tag[64];
    memcpy(tag, s, 32);
    range_sum_enc(key, i0, i0 + k, {}, tag + 32);
    return aver_impl(c, prm, key->y, m, ds, ds_len, tag, stream, nullptr, accept, e_out);
}

extern "C" int poslo_c_distill(poslo_ctx* c, const poslo_params* prm, const poslo_c_key* key,
                               const poslo_msgs* m_in, const uint8_t* s_epochs, const uint8_t* ds, size_t ds_len,
                               uint32_t n_umbrella, void* stream, poslo_ccd** out) {
    if (!c || !out || n_umbrella < 1) return POSLO_E_INVAL;
    *out = nullptr;
    uint64_t i0, k;
    int st = epoch_range(prm, key, m_in, i0, k);
    if (st) return st;
    if (k && !s_epochs) return POSLO_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    poslo_msgs dm;
    if ((st = stage_msgs(c, m_in, s, dm, nullptr, nullptr))) return st;
    const poslo_msgs* m = &dm;
    BatchArgs a;
    DsArg dsa;
    uint32_t n_epochs;
    if ((st = prepare_batch(c, prm, m, ds, ds_len, a, dsa, n_epochs))) return st;
    HIP_TRY(hipSetDevice(c->device));
    if (((prm->inst & POSLO_GROUP_FOURQ) != 0) != key->fq) return POSLO_E_INVAL;
    const KeyEntry* ky = ctx_key_of(c, prm->inst, key->y, &st);
    if (!ky) return st;
    const uint32_t* gtab = key->fq ? ctx_gtable_fq(c) : c->d_gtable;
    if (!gtab) return POSLO_E_NOMEM;
    std::vector<uint32_t> bits(k, 0);
    if (k) {
        void *ek, *ds_s, *dres;
        if ((st = ctx_scratch(c, kSlotCEkeys, m->n * 32, &ek)) || (st = ctx_scratch(c, kSlotCSigs, k * 32, &ds_s)) ||
            (st = ctx_scratch(c, kSlotCBits, k * 4, &dres)))
            return st;
        std::vector<uint32_t> sw(8 * k);
        for (uint64_t p = 0; p < 8 * k; p++) sw[p] = load_le32(s_epochs + 4 * p);
        HIP_TRY(hipMemcpyAsync(ds_s, sw.data(), sw.size() * 4, hipMemcpyHostToDevice, s));
        if ((st = launch_seed_table(dsa, prm->inst, a, n_epochs, s))) return st;
        const int saved = c->agg_variant;
        c->agg_variant = -1;  // the emit form is the default variant's
        const AggShape g = agg_shape(c, prm, m);
        c->agg_variant = saved;
        if ((st = ctx_ensure(&c->d_part, &c->part_words, (size_t)g.grid * 9))) return st;
        prof_begin(c, POSLO_KT_VERIFY, s);
        if ((st = launch_agg(c, prm, g, a, c->d_part, (uint32_t*)ek, nullptr, s))) return st;
        if (key->fq)
            hipLaunchKernelGGL(k_c_epoch_check<true>, dim3((uint32_t)k), dim3(64), 0, s, (const uint32_t*)ek,
                               prm->log2_n2, (const uint32_t*)ds_s, key->d_r + 16 * i0, ky->d_table, gtab,
                               (uint32_t*)dres);
        else
            hipLaunchKernelGGL(k_c_epoch_check<false>, dim3((uint32_t)k), dim3(64), 0, s, (const uint32_t*)ek,
                               prm->log2_n2, (const uint32_t*)ds_s, key->d_r + 16 * i0, ky->d_table, gtab,
                               (uint32_t*)dres);
        HIP_TRY(hipGetLastError());
        prof_end(c, POSLO_KT_VERIFY, s);
        uint32_t bad = 0;  // POSLO++: a message longer than 31 bytes
        HIP_TRY(hipMemcpyAsync(bits.data(), dres, k * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&bad, a.bad, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        prof_collect(c);
        if (bad) return POSLO_E_INVAL;
    }
    poslo_ccd* ccd = new (std::nothrow) poslo_ccd();
    if (!ccd) return POSLO_E_NOMEM;
    ccd->inst = prm->inst;
    ccd->log2_n1 = prm->log2_n1;
    ccd->log2_n2 = prm->log2_n2;
    ccd->coarse = 1;
    ccd->t0 = m->t0;
    ccd->n = m->n;
    ccd->ds.assign(ds, ds + ds_len);
    for (uint64_t p = 0; p < k; p++) {
        if (bits[p]) continue;
        ccd->invalid.push_back(i0 + p);
        ccd->invalid_sigs.insert(ccd->invalid_sigs.end(), s_epochs + 32 * p, s_epochs + 32 * (p + 1));
        ccd->invalid_sigs.insert(ccd->invalid_sigs.end(), key->r_enc.begin() + 32 * (i0 + p),
                                 key->r_enc.begin() + 32 * (i0 + p + 1));
        ccd->invalid_sigs.insert(ccd->invalid_sigs.end(), 16, 0);
    }
    // valid aggregate and umbrellas of U = ceil(k / n_u) epochs
    const uint64_t span = std::max<uint64_t>(1, (k + n_umbrella - 1) / n_umbrella);
    ccd->span = span;
    range_sum_enc(key, i0, i0 + k, ccd->invalid, ccd->valid_tag + 32);
    sum_s(key, s_epochs, 0, k, ccd->invalid, i0, ccd->valid_tag);
    for (uint64_t a0 = 0; a0 < k; a0 += span) {
        const uint64_t b0 = std::min(k, a0 + span);
        uint8_t tg[64];
        range_sum_enc(key, i0 + a0, i0 + b0, ccd->invalid, tg + 32);
        sum_s(key, s_epochs, a0, b0, ccd->invalid, i0, tg);
        ccd->umb_tags.insert(ccd->umb_tags.end(), tg, tg + 64);
    }
    *out = ccd;
    return POSLO_OK;
}

extern "C" int poslo_c_sebver(poslo_ctx* c, const poslo_params* prm, const poslo_c_key* key, const poslo_msgs* m,
                              const poslo_ccd* ccd, char mode, uint8_t* bits, size_t cap, size_t* n_bits,
                              void* stream) {
    if (!c || !ccd || !n_bits || !ccd->coarse) return POSLO_E_INVAL;
    uint64_t i0, k;
    int st = epoch_range(prm, key, m, i0, k);
    if (st) return st;
    if (((prm->inst & POSLO_GROUP_FOURQ) != 0) != key->fq) return POSLO_E_INVAL;
    if (mode == 'V' || mode == 'U')
        return sebver_impl(c, prm, key->y, m, ccd, mode, bits, cap, n_bits, stream);
    if (mode != 'I') return POSLO_E_INVAL;
    if (m->t0 != ccd->t0 || m->n != ccd->n) return POSLO_E_INVAL;
    const uint64_t ni = ccd->invalid.size();
    *n_bits = ni;
    if (!bits || cap < ni) return POSLO_E_INVAL;
    // each invalid epoch against its own (s~_i, R~_i)
    const uint64_t n2 = 1ull << prm->log2_n2;
    for (uint64_t q = 0; q < ni; q++) {
        const uint64_t i = ccd->invalid[q];
        if (i < i0 || i >= i0 + k) return POSLO_E_INVAL;
        poslo_msgs em = *m;
        em.t0 = i * n2;
        em.n = n2;
        if (m->offsets)
            em.offsets = m->offsets + (i - i0) * n2;
        else
            em.data = m->data + (i - i0) * n2 * m->msg_len;
        if (m->data_bytes) em.data_bytes = m->data_bytes - (uint64_t)(em.data - m->data);
        int acc = 0;
        st = aver_impl(c, prm, key->y, &em, ccd->ds.data(), ccd->ds.size(), ccd->invalid_sigs.data() + 80 * q,
                       stream, nullptr, &acc, nullptr);
        if (st) return st;
        bits[q] = (uint8_t)acc;
    }
    return POSLO_OK;
}
