// Host-side POSLO-F signer and aggregation, used to produce verifier inputs:
// Kg, Sig (with SSO and BPV.Online) and Agg (paper, figure "Fine-grained
// public-key POSLO" and Definition "BPV"; Agg from figure "Digital signature
// algorithms").
//
// Randomness is derived deterministically from a 32-byte key seed with the
// instantiation's own PRF_0, so that keys and signatures are reproducible:
//   derive(label, c) = PRF_0(seed || label || LE32(2c)) || PRF_0(seed || label || LE32(2c+1))
//   y = LE256(derive("y", c)) mod q for the first c giving y != 0
//   x_D[0] = derive("x", 0)[0:16]
//   BPV table: r_k = LE256(derive("bpv", k)) mod q, R_k = r_k * G, k < v
//   subset S_t: the first k distinct (LE16 word mod v) of the stream
//               PRF_0(seed || "S" || LE32(t) || LE32(c)), c = 0, 1, ...
#include <string.h>

#include <algorithm>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/poslo.h"
#include "scheme_host.h"

using namespace poslo;
using namespace poslo::hostside;

struct poslo_signer {
    poslo_params prm;
    uint8_t seed[32];
    uint32_t y[8];
    uint8_t root[16];
    uint64_t t = 0;
    std::vector<DsNode> ds;
    uint8_t x0[16];
    std::vector<uint32_t> bpv_r;  // v scalars, 8 limbs each
    std::vector<ge> bpv_R;        // v points (edwards25519)
    std::vector<gq> bpv_Rq;       // v points (FourQ)
    bool fourq = false;
};

namespace {

int hw_threads(int want) {
    int hc = (int)std::thread::hardware_concurrency();
    if (hc <= 0) hc = 1;
    if (want <= 0 || want > hc) want = hc;
    return want;
}

template <class F>
void parallel_for(uint64_t n, int nthreads, F f) {
    nthreads = (int)std::min<uint64_t>((uint64_t)hw_threads(nthreads), std::max<uint64_t>(n, 1));
    if (nthreads <= 1) {
        for (uint64_t i = 0; i < n; i++) f(i);
        return;
    }
    std::vector<std::thread> th;
    uint64_t chunk = (n + nthreads - 1) / nthreads;
    for (int k = 0; k < nthreads; k++) {
        uint64_t a = k * chunk, b = std::min<uint64_t>(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([a, b, &f] {
            for (uint64_t i = a; i < b; i++) f(i);
        });
    }
    for (auto& t : th) t.join();
}

void derive(uint32_t inst, const uint8_t seed[32], const char* label, uint32_t c, uint8_t out[32]) {
    size_t ll = strlen(label);
    std::vector<uint8_t> z(32 + ll + 4);
    memcpy(z.data(), seed, 32);
    memcpy(z.data() + 32, label, ll);
    store_le32(z.data() + 32 + ll, 2 * c);
    prf(inst, 0, z.data(), z.size(), out);
    store_le32(z.data() + 32 + ll, 2 * c + 1);
    prf(inst, 0, z.data(), z.size(), out + 16);
}

bool params_valid(const poslo_params* p) {
    if (!p) return false;
    if (!poslo_inst_valid(p->inst)) return false;
    if (p->log2_n1 > 31 || p->log2_n2 > 31 || p->log2_n1 + p->log2_n2 > 32) return false;
    if (p->bpv_v == 0 || p->bpv_v > 65536 || (p->bpv_v & (p->bpv_v - 1))) return false;
    if (p->bpv_k == 0 || p->bpv_k > p->bpv_v) return false;
    return true;
}

void subset(const poslo_signer* sk, uint64_t t, std::vector<uint32_t>& out) {
    out.clear();
    uint8_t z[32 + 1 + 8];
    memcpy(z, sk->seed, 32);
    z[32] = 'S';
    store_le32(z + 33, (uint32_t)t);
    for (uint32_t c = 0; out.size() < sk->prm.bpv_k; c++) {
        store_le32(z + 37, c);
        uint8_t blk[16];
        prf(sk->prm.inst, 0, z, sizeof z, blk);
        for (int w = 0; w < 8 && out.size() < sk->prm.bpv_k; w++) {
            uint32_t val = ((uint32_t)blk[2 * w] | ((uint32_t)blk[2 * w + 1] << 8)) % sk->prm.bpv_v;
            if (std::find(out.begin(), out.end(), val) == out.end()) out.push_back(val);
        }
    }
}

// sigma_t for entry t with epoch seed x0 (read-only use of the signer)
void sign_entry(const poslo_signer* sk, uint64_t t, const uint8_t x0[16], const uint8_t* m, size_t len,
                uint8_t sig[80]) {
    const poslo_params& p = sk->prm;
    uint32_t j = (uint32_t)(t & ((1ull << p.log2_n2) - 1));
    // BPV.Online
    std::vector<uint32_t> S;
    subset(sk, t, S);
    uint32_t r[8] = {0};
    ge R;
    ge_identity(R);
    gq Rq;
    gq_identity(Rq);
    for (uint32_t k : S) {
        uint32_t tmp[8];
        if (sk->fourq) {
            scN_add(tmp, r, &sk->bpv_r[8 * k]);
            gq_add(Rq, Rq, sk->bpv_Rq[k]);
        } else {
            sc_add(tmp, r, &sk->bpv_r[8 * k]);
            ge_add(R, R, sk->bpv_R[k]);
        }
        memcpy(r, tmp, sizeof r);
    }
    // x_t = PRF_0(x_0[i] || LE32(j)); e_t = H(m || x_t) mod q
    uint8_t in20[20];
    memcpy(in20, x0, 16);
    store_le32(in20 + 16, j);
    uint8_t x[16];
    prf(p.inst, 0, in20, 20, x);
    uint32_t e[8], ey[8], s[8];
    digest_e(p.inst, m, len, x, e);  // message lengths are checked by the caller
    if (sk->fourq) {
        scN_mul(ey, e, sk->y);
        scN_sub(s, r, ey);
    } else {
        sc_mul(ey, e, sk->y);
        sc_sub(s, r, ey);
    }
    for (int w = 0; w < 8; w++) store_le32(sig + 4 * w, s[w]);
    if (sk->fourq) fq_encode(sig + 32, Rq);
    else ge_encode(sig + 32, R);
    memcpy(sig + 64, x, 16);
}

}  // namespace

const BaseTable& poslo::hostside::base_table() {
    static BaseTable* T = nullptr;
    static std::once_flag once;
    std::call_once(once, [] {
        T = new BaseTable();
        ge P;
        ge_base(P);
        for (int w = 0; w < 64; w++) {
            ge_identity(T->t[w][0]);
            T->t[w][1] = P;
            for (int d = 2; d < 16; d++) ge_add(T->t[w][d], T->t[w][d - 1], P);
            // P <- 16 P
            ge_dbl(P, P);
            ge_dbl(P, P);
            ge_dbl(P, P);
            ge_dbl(P, P);
        }
    });
    return *T;
}

const FqBaseTable& poslo::hostside::fq_base_table() {
    static FqBaseTable* T = nullptr;
    static std::once_flag once;
    std::call_once(once, [] {
        T = new FqBaseTable();
        fp2 gx, gy;
        fq_gen_xy(gx, gy);
        gq P;
        gq_from_affine(P, gx, gy);
        for (int w = 0; w < 64; w++) {
            gq_identity(T->t[w][0]);
            T->t[w][1] = P;
            for (int d = 2; d < 16; d++) gq_add(T->t[w][d], T->t[w][d - 1], P);
            for (int k = 0; k < 4; k++) gq_dbl(P, P);
        }
    });
    return *T;
}

extern "C" int poslo_inst_valid(uint32_t inst) {
    const uint32_t base = inst & 3u;
    return (inst & ~15u) == 0 && base <= 2u && !((inst & POSLO_KAPPA127) && base == 0u) &&
           !((inst & POSLO_GROUP_FOURQ) && base == 2u);
}

extern "C" const char* poslo_version(void) { return "poslo-mi355x 0.1"; }

extern "C" const char* poslo_strerror(int s) {
    switch (s) {
        case POSLO_OK: return "ok";
        case POSLO_E_INVAL: return "invalid argument";
        case POSLO_E_NOMEM: return "out of memory";
        case POSLO_E_DEVICE: return "device error";
        case POSLO_E_SEED: return "seed retrieval failed: ds does not cover an epoch";
        case POSLO_E_ENCODING: return "not a valid point encoding";
        case POSLO_E_EXHAUSTED: return "signer exhausted";
        case POSLO_E_BUSY: return "busy";
        default: return "unknown status";
    }
}

extern "C" int poslo_kg(const poslo_params* prm, const uint8_t seed[32], poslo_signer** out, uint8_t pk[32]) {
    if (!out || !seed || !pk || !params_valid(prm)) return POSLO_E_INVAL;
    *out = nullptr;
    poslo_signer* sk = new (std::nothrow) poslo_signer();
    if (!sk) return POSLO_E_NOMEM;
    sk->prm = *prm;
    sk->fourq = group_fourq(prm->inst);
    memcpy(sk->seed, seed, 32);
    for (uint32_t c = 0;; c++) {
        uint8_t d[32];
        derive(prm->inst, seed, "y", c, d);
        scalar_from_bytes(prm->inst, sk->y, d);
        uint32_t o = 0;
        for (int w = 0; w < 8; w++) o |= sk->y[w];
        if (o) break;
    }
    uint8_t xd[32];
    derive(prm->inst, seed, "x", 0, xd);
    memcpy(sk->root, xd, 16);
    uint32_t v = prm->bpv_v;
    sk->bpv_r.resize((size_t)v * 8);
    if (sk->fourq) {
        sk->bpv_Rq.resize(v);
        fq_base_table();
    } else {
        sk->bpv_R.resize(v);
        base_table();
    }
    parallel_for(v, 0, [&](uint64_t k) {
        uint8_t d[32];
        derive(prm->inst, seed, "bpv", (uint32_t)k, d);
        scalar_from_bytes(prm->inst, &sk->bpv_r[8 * k], d);
        if (sk->fourq) fq_scalarmult_base(sk->bpv_Rq[k], &sk->bpv_r[8 * k]);
        else ge_scalarmult_base(sk->bpv_R[k], &sk->bpv_r[8 * k]);
    });
    if (sk->fourq) {
        gq Y;
        fq_scalarmult_base(Y, sk->y);
        fq_encode(pk, Y);
    } else {
        ge Y;
        ge_scalarmult_base(Y, sk->y);
        ge_encode(pk, Y);
    }
    *out = sk;
    return POSLO_OK;
}

extern "C" void poslo_signer_free(poslo_signer* sk) { delete sk; }

extern "C" uint64_t poslo_signer_count(const poslo_signer* sk) { return sk ? sk->t : 0; }

// advance the state through entries t .. t+n-1: SSO at each epoch start;
// returns the epoch seeds of epochs first_epoch .. last_epoch
static void advance_epochs(poslo_signer* sk, uint64_t n, std::vector<uint8_t>& seeds, uint64_t& first_epoch) {
    const poslo_params& p = sk->prm;
    uint64_t t0 = sk->t;
    first_epoch = t0 >> p.log2_n2;
    uint64_t last_epoch = (t0 + n - 1) >> p.log2_n2;
    seeds.assign((last_epoch - first_epoch + 1) * 16, 0);
    uint64_t mask = (1ull << p.log2_n2) - 1;
    if (t0 & mask) memcpy(seeds.data(), sk->x0, 16);  // continuing the current epoch
    for (uint64_t i = first_epoch; i <= last_epoch; i++) {
        uint64_t start = i << p.log2_n2;
        if (start >= t0) {
            sso(p.inst, sk->ds, sk->root, p.log2_n1, i, sk->x0);
            memcpy(&seeds[(i - first_epoch) * 16], sk->x0, 16);
        }
    }
    sk->t = t0 + n;
}

extern "C" int poslo_sig(poslo_signer* sk, const uint8_t* m, size_t len, uint8_t sig[80]) {
    if (!sk || !sig || (len && !m)) return POSLO_E_INVAL;
    if (inst_base(sk->prm.inst) == INST_AES_ADDQ && len > kAddqMaxLen) return POSLO_E_INVAL;
    uint64_t n = 1ull << (sk->prm.log2_n1 + sk->prm.log2_n2);
    if (sk->t >= n) return POSLO_E_EXHAUSTED;
    uint64_t t = sk->t, first;
    std::vector<uint8_t> seeds;
    advance_epochs(sk, 1, seeds, first);
    sign_entry(sk, t, seeds.data(), m, len, sig);
    return POSLO_OK;
}

extern "C" int poslo_sig_batch(poslo_signer* sk, const uint8_t* msgs, const uint64_t* offsets, uint64_t msg_len,
                               uint64_t n, uint8_t* sigs, int nthreads) {
    if (!sk || (n && (!sigs || !msgs))) return POSLO_E_INVAL;
    if (n == 0) return POSLO_OK;
    uint64_t cap = 1ull << (sk->prm.log2_n1 + sk->prm.log2_n2);
    if (sk->t > cap || n > cap - sk->t) return POSLO_E_EXHAUSTED;
    if (inst_base(sk->prm.inst) == INST_AES_ADDQ)
        for (uint64_t p = 0; p < n; p++)
            if ((offsets ? offsets[p + 1] - offsets[p] : msg_len) > kAddqMaxLen) return POSLO_E_INVAL;
    uint64_t t0 = sk->t, first;
    std::vector<uint8_t> seeds;
    advance_epochs(sk, n, seeds, first);
    const poslo_signer* csk = sk;
    uint32_t l2 = sk->prm.log2_n2;
    parallel_for(n, nthreads, [&](uint64_t p) {
        uint64_t t = t0 + p;
        const uint8_t* m = offsets ? msgs + offsets[p] : msgs + p * msg_len;
        size_t len = offsets ? (size_t)(offsets[p + 1] - offsets[p]) : (size_t)msg_len;
        sign_entry(csk, t, &seeds[((t >> l2) - first) * 16], m, len, sigs + 80 * p);
    });
    return POSLO_OK;
}

extern "C" int poslo_ds_export(const poslo_signer* sk, uint8_t* buf, size_t cap, size_t* len) {
    if (!sk || !len) return POSLO_E_INVAL;
    std::vector<uint8_t> out;
    ds_serialize(sk->ds, out);
    *len = out.size();
    if (!buf || cap < out.size()) return POSLO_E_INVAL;
    memcpy(buf, out.data(), out.size());
    return POSLO_OK;
}

extern "C" int poslo_agg_inst(uint32_t inst, const uint8_t* sigs, size_t stride, uint64_t count, uint8_t tag[64]) {
    if (!poslo_inst_valid(inst)) return POSLO_E_INVAL;
    if (!group_fourq(inst)) return poslo_agg(sigs, stride, count, tag);
    if (!tag || stride < 80 || (count && !sigs)) return POSLO_E_INVAL;
    uint32_t s[8] = {0};
    gq R;
    gq_identity(R);
    for (uint64_t k = 0; k < count; k++) {
        const uint8_t* sg = sigs + k * stride;
        gq Rt;
        if (!fq_decode(Rt, sg + 32)) return POSLO_E_ENCODING;
        uint32_t st[8], w[8], tmp[8];
        for (int i = 0; i < 8; i++) w[i] = load_le32(sg + 4 * i);
        scN_reduce<8>(st, w);
        scN_add(tmp, s, st);
        memcpy(s, tmp, sizeof s);
        gq_add(R, R, Rt);
    }
    for (int w = 0; w < 8; w++) store_le32(tag + 4 * w, s[w]);
    fq_encode(tag + 32, R);
    return POSLO_OK;
}

extern "C" int poslo_agg(const uint8_t* sigs, size_t stride, uint64_t count, uint8_t tag[64]) {
    if (!tag || stride < 80 || (count && !sigs)) return POSLO_E_INVAL;
    uint32_t s[8] = {0};
    ge R;
    ge_identity(R);
    for (uint64_t k = 0; k < count; k++) {
        const uint8_t* sg = sigs + k * stride;
        ge Rt;
        if (!ge_decode(Rt, sg + 32)) return POSLO_E_ENCODING;
        uint32_t st[8], tmp[8];
        sc_from_bytes_reduce(st, sg);
        sc_add(tmp, s, st);
        memcpy(s, tmp, sizeof s);
        ge_add(R, R, Rt);
    }
    for (int w = 0; w < 8; w++) store_le32(tag + 4 * w, s[w]);
    ge_encode(tag + 32, R);
    return POSLO_OK;
}

extern "C" int poslo_prf_host(uint32_t inst, uint32_t b, const uint8_t* in, size_t len, uint8_t out16[16]) {
    if (!poslo_inst_valid(inst) || b > 1 || !out16 || (len && !in)) return POSLO_E_INVAL;
    if (kappa127(inst) && len == 16 && (in[15] & 0x80)) return POSLO_E_INVAL;
    prf(inst, b, in, len, out16);
    return POSLO_OK;
}

extern "C" int poslo_hash_host(uint32_t inst, const uint8_t* in, size_t len, uint8_t out32[32]) {
    if (!poslo_inst_valid(inst) || inst_base(inst) == INST_AES_ADDQ || !out32 || (len && !in)) return POSLO_E_INVAL;
    H(inst, in, len, out32);
    return POSLO_OK;
}
