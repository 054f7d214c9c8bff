// POSLO-F signing on the GPU for large synthetic workloads: the same bytes
// as the host signer (signer.hip), many keys and many batches per launch.
//
// Key material per key (figure "Fine-grained public-key POSLO", Kg; BPV
// Offline, Definition "BPV"): y, the seed-tree root x_D[0] and the public key
// are derived on the host; the BPV table {r_k, R_k = r_k * G} (v entries) is
// derived on the device, one lane per entry, with the fixed-base comb table of
// G.  Signing (Sig; BPV Online): per entry the subset S_t, r_t = sum r_k,
// R_t = sum R_k, x_t = PRF_0(x_0[i] || j), e_t = H(m_t || x_t) mod q and
// s_t = r_t - e_t * y mod q (Montgomery multiplication by y * 2^256 mod q).
// Per batch the aggregate tag is (sum s_t mod q, (sum r_t mod q) * G), which
// equals (sum s_t, sum R_t) since every R_t = r_t * G.  On the FourQ group
// (fourq.h) the same steps run with FourQ's points and scalars mod N.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ctx.h"
#include "device_ec.h"
#include "device_entry.h"
#include "device_fq.h"
#include "device_verify.h"
#include "scheme_host.h"

namespace poslo {

// ---- F over a short input given as little-endian words ----------------------
// z holds bytes 0..len-1 (len <= 44, bytes beyond len zero); returns F(z) as
// four little-endian words (MMO-AES-128, or SHA-256 truncated to 16 bytes),
// reduced mod 2^127 at kappa = 127 (inst: the instantiation word)
template <class T>
__device__ __forceinline__ void dev_F_words(const T& tb, uint32_t inst, const uint32_t z[12], int len,
                                            uint32_t out[4]) {
    if (prf_is_aes(inst)) {
        int nb = (len + 15) / 16;
        uint32_t h[4];
        for (int b = 0; b < nb; b++) {
            uint32_t m[4] = {z[4 * b], z[4 * b + 1], z[4 * b + 2], z[4 * b + 3]};
            uint32_t s[4] = {m[0], m[1], m[2], m[3]};
            if (b == 0)
                aes128_encrypt_rk(tb, c_iv.a, s);
            else
                aes128_encrypt_otf(tb, h, s);
            for (int w = 0; w < 4; w++) h[w] = s[w] ^ m[w];
        }
        for (int w = 0; w < 4; w++) out[w] = h[w];
        if (kappa127(inst)) out[3] &= 0x7fffffffu;
    } else {
        uint32_t W[16];
        for (int w = 0; w < 16; w++) W[w] = 0;
        for (int w = 0; w < 12; w++) W[w] = bswap32(z[w]);
        W[len >> 2] |= 0x80000000u >> (8 * (len & 3));
        W[15] = (uint32_t)len * 8u;
        uint32_t H[8];
        sha256_init(H);
        sha256_compress(H, W);
        for (int w = 0; w < 4; w++) out[w] = bswap32(H[w]);
    }
}

// ---- Montgomery multiplication modulo q (R = 2^256), CIOS ------------------

PDC uint32_t mont_qinv() {  // -q^{-1} mod 2^32 by Newton iteration
    uint32_t q0 = 0x5cf5d3edu, inv = 1;
    for (int i = 0; i < 6; i++) inv *= 2u - q0 * inv;
    return 0u - inv;
}

__device__ __forceinline__ void sc_mont_mul(uint32_t r[8], const uint32_t a[8], const uint32_t b[8]) {
    const uint32_t q[8] = POSLO_SC_Q;
    constexpr uint32_t qinv = mont_qinv();
    uint32_t t[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 8; i++) {
        uint64_t c = 0;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            c += (uint64_t)a[j] * b[i] + t[j];
            t[j] = (uint32_t)c;
            c >>= 32;
        }
        c += t[8];
        t[8] = (uint32_t)c;
        t[9] = (uint32_t)(c >> 32);
        uint32_t m = t[0] * qinv;
        c = ((uint64_t)m * q[0] + t[0]) >> 32;
#pragma unroll
        for (int j = 1; j < 8; j++) {
            c += (uint64_t)m * q[j] + t[j];
            t[j - 1] = (uint32_t)c;
            c >>= 32;
        }
        c += t[8];
        t[7] = (uint32_t)c;
        t[8] = t[9] + (uint32_t)(c >> 32);
    }
    // t < 2q: one conditional subtraction
    uint32_t d[8];
    int64_t bw = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        bw += (int64_t)t[j] - q[j];
        d[j] = (uint32_t)bw;
        bw >>= 32;
    }
    bool ge_q = t[8] || bw == 0;
#pragma unroll
    for (int j = 0; j < 8; j++) r[j] = ge_q ? d[j] : t[j];
}

__device__ __forceinline__ void sc_sub_dev(uint32_t r[8], const uint32_t a[8], const uint32_t b[8]) {
    const uint32_t q[8] = POSLO_SC_Q;
    int64_t bw = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) {
        bw += (int64_t)a[i] - b[i];
        r[i] = (uint32_t)bw;
        bw >>= 32;
    }
    if (bw) {
        uint64_t c = 0;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            c += (uint64_t)r[i] + q[i];
            r[i] = (uint32_t)c;
            c >>= 32;
        }
    }
}

// ---- device key material ---------------------------------------------------

struct DevKey {
    uint32_t seed[8];    // the 32-byte key seed as LE words
    uint32_t root[4];    // x_D[0]
    uint32_t y_mont[8];  // y * 2^256 mod q (edwards25519)
    uint32_t y_n[8];     // y (FourQ: below N)
};

// k*G on FourQ by one lane: 32 lookups and mixed additions; k < N
__device__ __forceinline__ void lane_scalar_fq(gq& P, const uint32_t* t, const uint32_t k[8]) {
    gq_identity(P);
    uint32_t c = 0;
    for (int w = 0; w < kCombWindows; w++) {
        gnq q;
        fq_comb_lookup(q, t, w, comb_digit(k, w, c));
        gq_madd(P, P, q);
    }
}

__device__ __forceinline__ void store_point_fq(uint32_t* p, const gq& P) {
    stash_f2(p, 1, P.X);
    stash_f2(p + 8, 1, P.Y);
    stash_f2(p + 16, 1, P.Z);
    stash_f2(p + 24, 1, P.T);
}

__device__ __forceinline__ void load_point_fq(gq& P, const uint32_t* p) {
    unstash_f2(P.X, p, 1);
    unstash_f2(P.Y, p + 8, 1);
    unstash_f2(P.Z, p + 16, 1);
    unstash_f2(P.T, p + 24, 1);
}

// BPV offline table: r_k = LE256(derive("bpv", k)) mod q, R_k = r_k * G, with
// derive(label, c) = PRF_0(seed || label || LE32(2c)) || PRF_0(... LE32(2c+1))
// (FQ: mod N on FourQ)
template <bool FQ>
__global__ __launch_bounds__(256) void k_bpv_table(const DevKey* keys, uint32_t nkeys, uint32_t v, uint32_t inst,
                                                   const uint32_t* tg, uint32_t* bpv_r, uint32_t* bpv_R) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
    LdsTables<4, 1> tb{lds};
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (uint64_t)nkeys * v) return;
    uint32_t key = (uint32_t)(g / v), k = (uint32_t)(g % v);
    const DevKey& K = keys[key];
    uint32_t d[8];
    for (int half = 0; half < 2; half++) {
        uint32_t c = 2 * k + half;
        uint32_t z[12] = {0};
        for (int w = 0; w < 8; w++) z[w] = K.seed[w];
        z[8] = 0x62u | (0x70u << 8) | (0x76u << 16) | ((c & 0xffu) << 24);  // "bpv", LE32(c) byte 0
        z[9] = c >> 8;                                                      // bytes 1..3, PRF bit 0
        dev_F_words(tb, inst, z, 40, d + 4 * half);
    }
    uint32_t r[8];
    if constexpr (FQ) {
        scN_reduce<8>(r, d);
        gq R;
        lane_scalar_fq(R, tg, r);
        store_point_fq(bpv_R + g * 32, R);
    } else {
        sc_reduce256(r, d);
        ge R;
        lane_scalar(R, tg, r);
        store_point(bpv_R + g * 32, R);
    }
    for (int w = 0; w < 8; w++) bpv_r[g * 8 + w] = r[w];
}

// per-(job, epoch) seed table for signing: x_0[i] = leaf i of the key's tree
struct SignJob {
    uint32_t key;
    uint32_t pad;
    uint64_t t0;         // first entry index
    uint64_t n;          // entries
    uint64_t entry_base; // index of the job's first entry in the global arrays
    uint64_t epoch_base; // first row of the job's epochs in the epoch table
    uint64_t tile_base;  // first tile of the job
};

__global__ __launch_bounds__(256) void k_sign_epochs(const SignJob* jobs, const uint32_t* job_of_epoch,
                                                     uint64_t n_rows, const DevKey* keys, uint32_t D, uint32_t log2_n2,
                                                     uint32_t inst, uint32_t* tab) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
    LdsTables<4, 1> tb{lds};
    uint64_t row = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row == 0) tab[n_rows * kEpochWords] = 0u;  // POSLO++'s long-message flag
    if (row >= n_rows) return;
    const SignJob& J = jobs[job_of_epoch[row]];
    uint64_t i = (J.t0 >> log2_n2) + (row - J.epoch_base);
    uint32_t x[4] = {keys[J.key].root[0], keys[J.key].root[1], keys[J.key].root[2], keys[J.key].root[3]};
    for (int j = (int)D - 1; j >= 0; j--) {
        uint32_t b = (uint32_t)((i >> j) & 1u), nx[4];
        if (prf_is_aes(inst) && kappa127(inst))
            prf_node_aes127(tb, x, b, nx);
        else if (prf_is_aes(inst))
            prf_node_aes(tb, x, b, nx);
        else
            prf_node_sha(x, b, nx);
        x[0] = nx[0], x[1] = nx[1], x[2] = nx[2], x[3] = nx[3];
    }
    uint32_t* e = tab + row * kEpochWords;
    if (prf_is_aes(inst)) {
        uint32_t s[4] = {x[0], x[1], x[2], x[3]};
        aes128_encrypt_rk(tb, c_iv.a, s);
        uint32_t h1[4] = {s[0] ^ x[0], s[1] ^ x[1], s[2] ^ x[2], s[3] ^ x[3]};
        uint32_t rk[44];
        aes128_expand(tb, h1, rk);
        for (int w = 0; w < 44; w++) e[w] = rk[w];
    }
    for (int w = 0; w < 4; w++) e[44 + w] = x[w];
}

// one tile = up to 256 consecutive entries of one job
struct SignTile {
    uint32_t job;
    uint32_t count;
    uint64_t first;  // entry offset within the job
};

struct SignArgs {
    const SignJob* jobs;
    const SignTile* tiles;
    const DevKey* keys;
    const uint32_t* bpv_r;
    const uint32_t* bpv_R;
    uint32_t v, k;
    uint32_t inst;
    uint32_t log2_n2;
    const uint8_t* data;
    const uint64_t* offsets;  // global entry offsets (n_total + 1)
    uint64_t n_total;
    const uint32_t* tab;      // epoch table rows
    uint8_t* sigs;            // 80 bytes per global entry
    uint32_t* tile_part;      // per tile: lazy sums of s_t [9] and r_t [9]
    uint32_t* bad;            // set when a POSLO++ message is longer than 31 bytes
};

template <bool FQ>
__global__ __launch_bounds__(256) void k_sign(SignArgs A) {
    __shared__ uint32_t lds[4 * 256];
    lds_tables_fill<4, 1>(lds);
    __syncthreads();
    LdsTables<4, 1> tb{lds};
    const SignTile T = A.tiles[blockIdx.x];
    const SignJob J = A.jobs[T.job];
    const DevKey& K = A.keys[J.key];
    uint32_t as_[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ar[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    bool live = threadIdx.x < T.count;
    if (live && inst_base(A.inst) == INST_AES_ADDQ) {
        const uint64_t g = J.entry_base + T.first + threadIdx.x;
        if (A.offsets[g + 1] - A.offsets[g] > kAddqMaxLen) {
            *A.bad = 1u;
            live = false;
        }
    }
    if (live) {
        uint64_t p = T.first + threadIdx.x;  // entry within the job
        uint64_t t = J.t0 + p;
        uint64_t gidx = J.entry_base + p;
        // BPV online: the first k distinct (LE16 word mod v) of the PRF_0 stream
        uint32_t chosen[16];
        uint32_t cnt = 0;
        uint32_t r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        ge R;
        ge_identity(R);
        gq Rq;
        gq_identity(Rq);
        for (uint32_t c = 0; cnt < A.k; c++) {
            uint32_t z[12] = {0};
            for (int w = 0; w < 8; w++) z[w] = K.seed[w];
            z[8] = 0x53u | (((uint32_t)t & 0xffffffu) << 8);
            z[9] = ((uint32_t)t >> 24) | ((c & 0xffffffu) << 8);
            z[10] = c >> 24;  // PRF bit 0 at byte 41
            uint32_t blk[4];
            dev_F_words(tb, A.inst, z, 42, blk);
            for (int h = 0; h < 8 && cnt < A.k; h++) {
                uint32_t val = ((blk[h >> 1] >> (16 * (h & 1))) & 0xffffu) & (A.v - 1);
                bool dup = false;
#pragma unroll
                for (int q = 0; q < 16; q++) dup |= (q < (int)cnt) && chosen[q] == val;
                if (dup) continue;
#pragma unroll
                for (int q = 0; q < 16; q++)
                    if (q == (int)cnt) chosen[q] = val;
                cnt++;
                const uint64_t bi = (uint64_t)J.key * A.v + val;
                uint32_t tmp[8];
                if constexpr (FQ) {
                    uint32_t rk[8];
                    for (int w = 0; w < 8; w++) rk[w] = A.bpv_r[bi * 8 + w];
                    scN_add(tmp, r, rk);
                    gq Q;
                    load_point_fq(Q, A.bpv_R + bi * 32);
                    gq_add(Rq, Rq, Q);
                } else {
                    sc_add(tmp, r, A.bpv_r + bi * 8);
                    ge Q;
                    load_point(Q, A.bpv_R + bi * 32);
                    ge_add(R, R, Q);
                }
                for (int w = 0; w < 8; w++) r[w] = tmp[w];
            }
        }
        // x_t and e_t
        BatchArgs ba;
        ba.data = A.data;
        ba.offsets = A.offsets + J.entry_base;
        ba.msg_len = 0;
        ba.n = J.n;
        ba.t0 = J.t0;
        ba.epoch_first = J.t0 >> A.log2_n2;
        ba.log2_n2 = A.log2_n2;
        ba.tab = A.tab + J.epoch_base * kEpochWords;
        ba.skip = nullptr;
        ba.end = A.data + A.offsets[A.n_total];
        ba.xmask = kappa127(A.inst) ? 0x7fffffffu : 0xffffffffu;
        EntryView ev = entry_view(ba, p);
        uint32_t x[4], dig[8];
        if (inst_base(A.inst) == INST_AES_ADDQ) {
            one_time_seed_aes(tb, ba, p, x);
            uint32_t mw[8];
            addq_message<0>(ev.m, (uint32_t)ev.L, mw);
            addq_digest(mw, x, dig);
        } else if (inst_base(A.inst) == INST_AES) {
            one_time_seed_aes(tb, ba, p, x);
            digest_mdc2_any(tb, ev, ba.end, x, dig, Mdc2BlockGeneric{});
        } else {
            one_time_seed_sha(ba, p, x);
            digest_sha_any(ev, ba.end, x, dig);
            for (int w = 0; w < 4; w++) x[w] = bswap32(x[w]);
        }
        uint32_t e[8], ey[8], s[8];
        uint8_t enc[32];
        if constexpr (FQ) {
            scN_reduce<8>(e, dig);
            uint32_t y[8];
            for (int w = 0; w < 8; w++) y[w] = K.y_n[w];
            scN_mul(ey, e, y);
            scN_sub(s, r, ey);
            fq_encode(enc, Rq);
        } else {
            sc_reduce256(e, dig);
            sc_mont_mul(ey, e, K.y_mont);
            sc_sub_dev(s, r, ey);
            ge_encode(enc, R);
        }
        uint8_t* out = A.sigs + gidx * 80;
        for (int w = 0; w < 8; w++) {
            store_le32(out + 4 * w, s[w]);
            store_le32(out + 32 + 4 * w, load_le32(enc + 4 * w));
        }
        for (int w = 0; w < 4; w++) store_le32(out + 64 + 4 * w, x[w]);
        acc288_add256(as_, s);
        acc288_add256(ar, r);
    }
    uint32_t* tp = A.tile_part + (uint64_t)blockIdx.x * 18;
    block_reduce288_store<256>(as_, tp);
    __syncthreads();
    block_reduce288_store<256>(ar, tp + 9);
}

// per job: tag = (sum s mod q, enc((sum r mod q) * G)) (FQ: mod N, on FourQ)
template <bool FQ>
__global__ __launch_bounds__(256) void k_sign_tags(const SignJob* jobs, const uint32_t* tile_part,
                                                   const uint64_t* tile_end, const uint32_t* tg, uint8_t* tags) {
    __shared__ uint32_t ts[9], tr[9];
    __shared__ uint32_t sh[16];
    const SignJob J = jobs[blockIdx.x];
    uint64_t a = J.tile_base, b = tile_end[blockIdx.x];
    uint32_t as_[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ar[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t k = a + threadIdx.x; k < b; k += 256) {
        acc288_add(as_, tile_part + k * 18);
        acc288_add(ar, tile_part + k * 18 + 9);
    }
    block_reduce288_store<256>(as_, ts);
    __syncthreads();
    block_reduce288_store<256>(ar, tr);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s[8], r[8];
        if constexpr (FQ) {
            scN_reduce<9>(s, ts);
            scN_reduce<9>(r, tr);
        } else {
            sc_reduce288(s, ts);
            sc_reduce288(r, tr);
        }
        for (int k = 0; k < 8; k++) {
            sh[k] = s[k];
            sh[8 + k] = r[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        uint32_t zero[8] = {0, 0, 0, 0, 0, 0, 0, 0}, r[8];
        for (int k = 0; k < 8; k++) r[k] = sh[8 + k];
        uint8_t* tag = tags + (uint64_t)blockIdx.x * 64;
        if constexpr (FQ) {
            gq P;
            wave_double_scalar_fq(P, tg, tg, zero, r);
            if (threadIdx.x == 0) fq_encode(tag + 32, P);
        } else {
            ge P;
            wave_double_scalar(P, tg, tg, zero, r);
            if (threadIdx.x == 0) ge_encode(tag + 32, P);
        }
        if (threadIdx.x == 0)
            for (int k = 0; k < 8; k++) store_le32(tag + 4 * k, sh[k]);
    }
}

}  // namespace poslo

// ===========================================================================
// host side
// ===========================================================================

using namespace poslo;
using namespace poslo::hostside;

struct poslo_gpu_keys {
    poslo_ctx* ctx = nullptr;
    poslo_params prm{};
    std::vector<DevKey> host;
    DevKey* d_keys = nullptr;
    uint32_t* d_bpv_r = nullptr;
    uint32_t* d_bpv_R = nullptr;
};

namespace {

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

void derive_host(uint32_t inst, const uint8_t seed[32], const char* label, uint32_t c, uint8_t out[32]) {
    size_t ll = strlen(label);
    std::vector<uint8_t> z(32 + ll + 4);
    memcpy(z.data(), seed, 32);
    memcpy(z.data() + 32, label, ll);
    store_le32(z.data() + 32 + ll, 2 * c);
    prf(inst, 0, z.data(), z.size(), out);
    store_le32(z.data() + 32 + ll, 2 * c + 1);
    prf(inst, 0, z.data(), z.size(), out + 16);
}

// y * 2^256 mod q by 256 modular doublings
void to_mont(uint32_t out[8], const uint32_t y[8]) {
    const uint32_t q[8] = POSLO_SC_Q;
    uint32_t a[8];
    memcpy(a, y, sizeof a);
    for (int i = 0; i < 256; i++) {
        uint32_t d[9];
        uint64_t c = 0;
        for (int w = 0; w < 8; w++) {
            c += (uint64_t)a[w] * 2;
            d[w] = (uint32_t)c;
            c >>= 32;
        }
        d[8] = (uint32_t)c;
        uint32_t s[8];
        int64_t bw = 0;
        for (int w = 0; w < 8; w++) {
            bw += (int64_t)d[w] - q[w];
            s[w] = (uint32_t)bw;
            bw >>= 32;
        }
        bool ge_q = d[8] || bw == 0;
        for (int w = 0; w < 8; w++) a[w] = ge_q ? s[w] : d[w];
    }
    memcpy(out, a, sizeof a);
}

}  // namespace

extern "C" int poslo_gpu_keys_create(poslo_ctx* c, const poslo_params* prm, const uint8_t* seeds, uint32_t nkeys,
                                     poslo_gpu_keys** out, uint8_t* pks) {
    if (!c || !prm || !out || (nkeys && (!seeds || !pks))) return POSLO_E_INVAL;
    if (!poslo_inst_valid(prm->inst) || prm->bpv_v == 0 || prm->bpv_v > 65536 || (prm->bpv_v & (prm->bpv_v - 1)) ||
        prm->bpv_k == 0 || prm->bpv_k > 16 || prm->bpv_k > prm->bpv_v || prm->log2_n1 + prm->log2_n2 > 32)
        return POSLO_E_INVAL;
    *out = nullptr;
    HIP_TRY(hipSetDevice(c->device));
    poslo_gpu_keys* K = new (std::nothrow) poslo_gpu_keys();
    if (!K) return POSLO_E_NOMEM;
    K->ctx = c;
    K->prm = *prm;
    K->host.resize(nkeys);
    const bool fq = group_fourq(prm->inst);
    const uint32_t* gtab = fq ? ctx_gtable_fq(c) : c->d_gtable;
    if (!gtab) {
        delete K;
        return POSLO_E_NOMEM;
    }
    if (fq)
        fq_base_table();
    else
        base_table();
    for (uint32_t k = 0; k < nkeys; k++) {
        const uint8_t* sd = seeds + 32 * (size_t)k;
        DevKey& dk = K->host[k];
        memset(&dk, 0, sizeof dk);
        for (int w = 0; w < 8; w++) dk.seed[w] = load_le32(sd + 4 * w);
        uint32_t y[8];
        for (uint32_t cc = 0;; cc++) {
            uint8_t d[32];
            derive_host(prm->inst, sd, "y", cc, d);
            scalar_from_bytes(prm->inst, y, d);
            uint32_t o = 0;
            for (int w = 0; w < 8; w++) o |= y[w];
            if (o) break;
        }
        uint8_t xd[32];
        derive_host(prm->inst, sd, "x", 0, xd);
        for (int w = 0; w < 4; w++) dk.root[w] = load_le32(xd + 4 * w);
        if (fq) {
            memcpy(dk.y_n, y, sizeof y);
            gq Y;
            fq_scalarmult_base(Y, y);
            fq_encode(pks + 32 * (size_t)k, Y);
        } else {
            to_mont(dk.y_mont, y);
            ge Y;
            ge_scalarmult_base(Y, y);
            ge_encode(pks + 32 * (size_t)k, Y);
        }
    }
    size_t v = prm->bpv_v;
    if (hipMalloc((void**)&K->d_keys, std::max<size_t>(nkeys, 1) * sizeof(DevKey)) != hipSuccess ||
        hipMalloc((void**)&K->d_bpv_r, std::max<size_t>(nkeys, 1) * v * 32) != hipSuccess ||
        hipMalloc((void**)&K->d_bpv_R, std::max<size_t>(nkeys, 1) * v * 128) != hipSuccess) {
        poslo_gpu_keys_free(K);
        return POSLO_E_NOMEM;
    }
    if (nkeys) {
        if (hipMemcpy(K->d_keys, K->host.data(), nkeys * sizeof(DevKey), hipMemcpyHostToDevice) != hipSuccess) {
            poslo_gpu_keys_free(K);
            return POSLO_E_DEVICE;
        }
        uint64_t lanes = (uint64_t)nkeys * v;
        if (fq)
            hipLaunchKernelGGL(k_bpv_table<true>, dim3((uint32_t)((lanes + 255) / 256)), dim3(256), 0, 0, K->d_keys,
                               nkeys, (uint32_t)v, prm->inst, gtab, K->d_bpv_r, K->d_bpv_R);
        else
            hipLaunchKernelGGL(k_bpv_table<false>, dim3((uint32_t)((lanes + 255) / 256)), dim3(256), 0, 0, K->d_keys,
                               nkeys, (uint32_t)v, prm->inst, gtab, K->d_bpv_r, K->d_bpv_R);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            poslo_gpu_keys_free(K);
            return POSLO_E_DEVICE;
        }
    }
    *out = K;
    return POSLO_OK;
}

extern "C" void poslo_gpu_keys_free(poslo_gpu_keys* K) {
    if (!K) return;
    if (K->d_keys) hipFree(K->d_keys);
    if (K->d_bpv_r) hipFree(K->d_bpv_r);
    if (K->d_bpv_R) hipFree(K->d_bpv_R);
    delete K;
}

// ds after the epochs 0..m-1 have begun: the maximal aligned blocks of the
// binary decomposition of m, largest first (what SSO leaves on its stack)
static void ds_for_epochs(uint32_t inst, const uint8_t root[16], uint32_t D, uint64_t m, std::vector<uint8_t>& out) {
    std::vector<DsNode> ds;
    uint64_t start = 0;
    for (int d = (int)D; d >= 0; d--) {
        if ((m >> d) & 1) {
            DsNode nd;
            nd.depth = (uint32_t)d;
            nd.index = (uint32_t)(start >> d);
            seed_walk(inst, root, D, nd.index, (uint32_t)d, nd.v);
            ds.push_back(nd);
            start += 1ull << d;
        }
    }
    ds_serialize(ds, out);
}

extern "C" int poslo_gpu_sign(poslo_gpu_keys* K, const poslo_sign_job* jobs, uint32_t njobs, const uint8_t* data,
                              const uint64_t* offsets, uint8_t* sigs, uint8_t* tags, uint8_t* ds_out, size_t ds_stride,
                              void* stream) {
    if (!K || (njobs && (!jobs || !data || !offsets || !sigs || !tags))) return POSLO_E_INVAL;
    if (ds_out && ds_stride < 1 + 24 * 32) return POSLO_E_INVAL;
    poslo_ctx* c = K->ctx;
    const poslo_params& p = K->prm;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    const bool fq = group_fourq(p.inst);
    const uint32_t* gtab = fq ? ctx_gtable_fq(c) : c->d_gtable;
    if (!gtab) return POSLO_E_NOMEM;
    uint64_t cap = 1ull << (p.log2_n1 + p.log2_n2);
    std::vector<SignJob> sj(njobs);
    std::vector<SignTile> tiles;
    std::vector<uint32_t> job_of_epoch;
    std::vector<uint64_t> tile_end(njobs);
    uint64_t rows = 0, n_total = 0;
    for (uint32_t j = 0; j < njobs; j++) {
        const poslo_sign_job& in = jobs[j];
        if (in.key >= K->host.size() || in.t0 > cap || in.n > cap - in.t0 || in.entry_base > UINT64_MAX - in.n)
            return POSLO_E_INVAL;
        n_total = std::max(n_total, in.entry_base + in.n);
        SignJob& o = sj[j];
        o.key = in.key;
        o.pad = 0;
        o.t0 = in.t0;
        o.n = in.n;
        o.entry_base = in.entry_base;
        o.epoch_base = rows;
        o.tile_base = tiles.size();
        if (in.n) {
            uint64_t e0 = in.t0 >> p.log2_n2, e1 = (in.t0 + in.n - 1) >> p.log2_n2;
            for (uint64_t e = e0; e <= e1; e++) job_of_epoch.push_back(j);
            rows += e1 - e0 + 1;
            for (uint64_t f = 0; f < in.n; f += 256)
                tiles.push_back(SignTile{j, (uint32_t)std::min<uint64_t>(256, in.n - f), f});
        }
        tile_end[j] = tiles.size();
    }
    void *d_jobs, *d_tiles, *d_joe, *d_tab, *d_part, *d_tend, *d_tags;
    int st;
    if ((st = ctx_scratch(c, 8, std::max<size_t>(njobs, 1) * sizeof(SignJob), &d_jobs)) ||
        (st = ctx_scratch(c, 9, std::max<size_t>(tiles.size(), 1) * sizeof(SignTile), &d_tiles)) ||
        (st = ctx_scratch(c, 10, std::max<size_t>(rows, 1) * 4, &d_joe)) ||
        (st = ctx_scratch(c, 11, epoch_tab_words(rows) * 4, &d_tab)) ||
        (st = ctx_scratch(c, 12, std::max<size_t>(tiles.size(), 1) * 72, &d_part)) ||
        (st = ctx_scratch(c, 13, std::max<size_t>(njobs, 1) * 8, &d_tend)) ||
        (st = ctx_scratch(c, 14, std::max<size_t>(njobs, 1) * 64, &d_tags)))
        return st;
    if (njobs == 0) return POSLO_OK;
    HIP_TRY(hipMemcpyAsync(d_jobs, sj.data(), njobs * sizeof(SignJob), hipMemcpyHostToDevice, s));
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(d_tiles, tiles.data(), tiles.size() * sizeof(SignTile), hipMemcpyHostToDevice, s));
    if (rows) HIP_TRY(hipMemcpyAsync(d_joe, job_of_epoch.data(), rows * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_tend, tile_end.data(), njobs * 8, hipMemcpyHostToDevice, s));
    if (rows)
        hipLaunchKernelGGL(k_sign_epochs, dim3((uint32_t)((rows + 255) / 256)), dim3(256), 0, s, (const SignJob*)d_jobs,
                           (const uint32_t*)d_joe, rows, K->d_keys, p.log2_n1, p.log2_n2, p.inst, (uint32_t*)d_tab);
    if (!tiles.empty()) {
        SignArgs A;
        A.jobs = (const SignJob*)d_jobs;
        A.tiles = (const SignTile*)d_tiles;
        A.keys = K->d_keys;
        A.bpv_r = K->d_bpv_r;
        A.bpv_R = K->d_bpv_R;
        A.v = p.bpv_v;
        A.k = p.bpv_k;
        A.inst = p.inst;
        A.log2_n2 = p.log2_n2;
        A.data = data;
        A.offsets = offsets;
        A.n_total = n_total;
        A.tab = (const uint32_t*)d_tab;
        A.sigs = sigs;
        A.tile_part = (uint32_t*)d_part;
        A.bad = (uint32_t*)d_tab + rows * kEpochWords;
        if (fq)
            hipLaunchKernelGGL(k_sign<true>, dim3((uint32_t)tiles.size()), dim3(256), 0, s, A);
        else
            hipLaunchKernelGGL(k_sign<false>, dim3((uint32_t)tiles.size()), dim3(256), 0, s, A);
    }
    if (fq)
        hipLaunchKernelGGL(k_sign_tags<true>, dim3(njobs), dim3(256), 0, s, (const SignJob*)d_jobs,
                           (const uint32_t*)d_part, (const uint64_t*)d_tend, gtab, (uint8_t*)d_tags);
    else
        hipLaunchKernelGGL(k_sign_tags<false>, dim3(njobs), dim3(256), 0, s, (const SignJob*)d_jobs,
                           (const uint32_t*)d_part, (const uint64_t*)d_tend, gtab, (uint8_t*)d_tags);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(tags, d_tags, (size_t)njobs * 64, hipMemcpyDeviceToHost, s));
    uint32_t bad = 0;
    if (rows) HIP_TRY(hipMemcpyAsync(&bad, (uint32_t*)d_tab + rows * kEpochWords, 4, hipMemcpyDeviceToHost, s));
    if (ds_out) {
        for (uint32_t j = 0; j < njobs; j++) {
            const DevKey& dk = K->host[jobs[j].key];
            uint8_t root[16];
            for (int w = 0; w < 4; w++) store_le32(root + 4 * w, dk.root[w]);
            uint64_t t_end = jobs[j].t0 + jobs[j].n;
            uint64_t m = t_end ? ((t_end - 1) >> p.log2_n2) + 1 : 0;
            std::vector<uint8_t> bytes;
            ds_for_epochs(p.inst, root, p.log2_n1, m, bytes);
            memset(ds_out + (size_t)j * ds_stride, 0, ds_stride);
            memcpy(ds_out + (size_t)j * ds_stride, bytes.data(), bytes.size());
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    return bad ? POSLO_E_INVAL : POSLO_OK;
}
