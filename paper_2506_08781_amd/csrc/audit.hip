// Streaming audit: AVer over a log too large to hold at once, fed in
// chunks (paper section "Experimental Evaluation on GPUs": the 1 TB audit
// is processed chunk by chunk; PAVer's sum e = sum of the per-block
// sub-aggregates is additive, so each chunk's e_t fold into a running
// e mod q, and the check R = e*Y + s*G runs once at the end).
//
// Each chunk runs the AVer kernels of a batch (seed rows for its epochs,
// the hot kernel) and one fold kernel that adds its partials to the running
// sum on the device.  Host-resident chunks are copied on a copy stream of
// the audit into one of two staging buffers, so that the copy of chunk
// k + 1 overlaps the hashing of chunk k; a staging buffer is reused only
// after the kernels that read it are done.  The running state (position,
// e mod q, key, ds) can be exported and resumed in another process.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ctx.h"
#include "device_entry.h"
#include "fourq.h"
#include "scheme_host.h"

namespace poslo {

// running e mod q (9 words, the top one zero) += the chunk's partials;
// run[9] keeps POSLO++'s long-message flag of every chunk (bad).  FQ: mod N
// (the FourQ group order) instead of q.
template <bool FQ>
__global__ __launch_bounds__(256) void k_audit_fold(const uint32_t* partials, uint32_t n_part, uint32_t* run,
                                                    const uint32_t* bad) {
    __shared__ uint32_t total[9];
    uint32_t acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t p = threadIdx.x; p < n_part; p += 256) acc288_add(acc, partials + (uint64_t)p * 9);
    block_reduce288_store<256>(acc, total);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t[9], e[8];
        for (int k = 0; k < 9; k++) t[k] = total[k];
        acc288_add(t, run);
        if (FQ) scN_reduce<9>(e, t);
        else sc_reduce288(e, t);
        for (int k = 0; k < 8; k++) run[k] = e[k];
        run[8] = 0;
        if (*bad) run[9] = 1u;
    }
}

}  // namespace poslo

using namespace poslo;

struct poslo_audit {
    poslo_ctx* c = nullptr;
    poslo_params prm{};
    uint8_t pk[32] = {};
    std::vector<uint8_t> ds;
    uint64_t t0 = 0, t_next = 0;
    uint32_t* d_run = nullptr;  // running e mod q, 9 words, then the long-message flag
    uint32_t* d_tab = nullptr;  // epoch rows of the chunk being hashed
    size_t tab_rows = 0;
    uint32_t* d_part = nullptr;
    size_t part_bytes = 0;
    // host chunks: two staging buffers, their copy and last-use events
    void* d_stage[2] = {nullptr, nullptr};
    size_t stage_cap[2] = {0, 0};
    void* d_soff[2] = {nullptr, nullptr};
    size_t soff_cap[2] = {0, 0};
    hipEvent_t ev_copied[2] = {nullptr, nullptr}, ev_used[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    int last_host = -1;  // staging buffer of the last host chunk, whose copy the next call waits for
    hipStream_t copy = nullptr;
    int buf = 0;
};

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

namespace {

int grow(void** p, size_t* have, size_t bytes) {
    if (*have >= bytes) return POSLO_OK;
    if (*p) {
        // the buffer may still be read by queued work
        if (hipDeviceSynchronize() != hipSuccess) return POSLO_E_DEVICE;
        (void)hipFree(*p);
    }
    *p = nullptr;
    *have = 0;
    size_t want = std::max<size_t>(bytes, 4096);
    if (hipMalloc(p, want) != hipSuccess) return POSLO_E_NOMEM;
    *have = want;
    return POSLO_OK;
}

// the copy of the previous host chunk is done: its host buffer is free
int release_host(poslo_audit* a) {
    if (a->last_host >= 0) {
        HIP_TRY(hipEventSynchronize(a->ev_copied[a->last_host]));
        a->last_host = -1;
    }
    return POSLO_OK;
}

int audit_new(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const uint8_t* ds, size_t ds_len,
              uint64_t t0, uint64_t t_next, const uint32_t e[8], poslo_audit** out) {
    if (!c || !params_ok(prm) || !pk || !ds || !out) return POSLO_E_INVAL;
    *out = nullptr;
    std::vector<hostside::DsNode> nodes;
    if (!hostside::ds_parse(ds, ds_len, nodes)) return POSLO_E_INVAL;
    const uint64_t nmax = 1ull << (prm->log2_n1 + prm->log2_n2);
    if (t0 > nmax || t_next < t0 || t_next > nmax) return POSLO_E_INVAL;
    int st;
    if (hipSetDevice(c->device) != hipSuccess) return POSLO_E_DEVICE;
    if (!ctx_key_of(c, prm->inst, pk, &st)) return st;  // E_ENCODING when pk is not a point
    poslo_audit* a = new (std::nothrow) poslo_audit();
    if (!a) return POSLO_E_NOMEM;
    a->c = c;
    a->prm = *prm;
    memcpy(a->pk, pk, 32);
    a->ds.assign(ds, ds + ds_len);
    a->t0 = t0;
    a->t_next = t_next;
    uint32_t run[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (e)
        for (int k = 0; k < 8; k++) run[k] = e[k];
    st = POSLO_OK;
    if (hipMalloc((void**)&a->d_run, 64) != hipSuccess) st = POSLO_E_NOMEM;
    if (!st && hipMemcpy(a->d_run, run, sizeof run, hipMemcpyHostToDevice) != hipSuccess) st = POSLO_E_DEVICE;
    for (int b = 0; b < 2 && !st; b++)
        if (hipEventCreateWithFlags(&a->ev_copied[b], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&a->ev_used[b], hipEventDisableTiming) != hipSuccess)
            st = POSLO_E_DEVICE;
    if (!st && hipStreamCreateWithFlags(&a->copy, hipStreamNonBlocking) != hipSuccess) st = POSLO_E_DEVICE;
    if (st) {
        poslo_audit_free(a);
        return st;
    }
    *out = a;
    return POSLO_OK;
}

}  // namespace

extern "C" int poslo_audit_begin(poslo_ctx* c, const poslo_params* prm, const uint8_t pk[32], const uint8_t* ds,
                                 size_t ds_len, uint64_t t0, poslo_audit** out) {
    return audit_new(c, prm, pk, ds, ds_len, t0, t0, nullptr, out);
}

extern "C" int poslo_audit_feed(poslo_audit* a, const poslo_msgs* m, void* stream) {
    if (!a || !m || m->t0 != a->t_next) return POSLO_E_INVAL;
    const uint64_t nmax = 1ull << (a->prm.log2_n1 + a->prm.log2_n2);
    if (m->n > nmax - a->t_next) return POSLO_E_INVAL;
    int st;
    if ((st = release_host(a))) return st;
    if (m->n == 0) return POSLO_OK;
    poslo_ctx* c = a->c;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(c->device));
    poslo_msgs dm = *m;
    int b = -1;
    if (m->host) {
        if (!m->data) return POSLO_E_INVAL;
        uint64_t need;
        if (m->offsets) {
            need = m->offsets[m->n];
            if (m->offsets[0] > need) return POSLO_E_INVAL;
        } else {
            if (m->msg_len && m->n > UINT64_MAX / m->msg_len) return POSLO_E_INVAL;
            need = m->n * m->msg_len;
        }
        const uint64_t bytes = m->data_bytes ? m->data_bytes : need;
        if (bytes < need) return POSLO_E_INVAL;
        b = a->buf;
        a->buf ^= 1;
        if ((st = grow(&a->d_stage[b], &a->stage_cap[b], bytes))) return st;
        if (m->offsets && (st = grow(&a->d_soff[b], &a->soff_cap[b], (m->n + 1) * 8))) return st;
        // the buffer's previous chunk must be hashed before it is overwritten
        if (a->used[b]) HIP_TRY(hipStreamWaitEvent(a->copy, a->ev_used[b], 0));
        HIP_TRY(hipMemcpyAsync(a->d_stage[b], m->data, bytes, hipMemcpyHostToDevice, a->copy));
        if (m->offsets)
            HIP_TRY(hipMemcpyAsync(a->d_soff[b], m->offsets, (m->n + 1) * 8, hipMemcpyHostToDevice, a->copy));
        HIP_TRY(hipEventRecord(a->ev_copied[b], a->copy));
        HIP_TRY(hipStreamWaitEvent(s, a->ev_copied[b], 0));
        dm.host = 0;
        dm.data = (const uint8_t*)a->d_stage[b];
        dm.offsets = m->offsets ? (const uint64_t*)a->d_soff[b] : nullptr;
        dm.data_bytes = bytes;
    }
    // the chunk's epoch rows in the audit's own table
    const uint64_t rows = ((m->t0 + m->n - 1) >> a->prm.log2_n2) - (m->t0 >> a->prm.log2_n2) + 1;
    if (a->tab_rows < rows) {
        size_t have = a->tab_rows ? epoch_tab_words(a->tab_rows) * 4 : 0;
        if ((st = grow((void**)&a->d_tab, &have, epoch_tab_words(rows) * 4))) return st;
        size_t r = (have / 4 - epoch_tab_words(0)) / kEpochWords;
        while (r > 0 && epoch_tab_words(r) * 4 > have) r--;
        a->tab_rows = r;
    }
    BatchArgs ba;
    DsArg dsa;
    uint32_t n_epochs;
    if ((st = prepare_batch(c, &a->prm, &dm, a->ds.data(), a->ds.size(), ba, dsa, n_epochs, a->d_tab,
                            a->tab_rows)))
        return st;
    if ((st = launch_seed_table(dsa, a->prm.inst, ba, n_epochs, s))) return st;
    const AggShape g = agg_shape(c, &a->prm, &dm);
    if ((st = grow((void**)&a->d_part, &a->part_bytes, (size_t)g.grid * 36))) return st;
    if ((st = launch_agg(c, &a->prm, g, ba, a->d_part, nullptr, nullptr, s))) return st;
    if (a->prm.inst & POSLO_GROUP_FOURQ)
        hipLaunchKernelGGL(k_audit_fold<true>, dim3(1), dim3(256), 0, s, (const uint32_t*)a->d_part, g.grid, a->d_run,
                           (const uint32_t*)ba.bad);
    else
        hipLaunchKernelGGL(k_audit_fold<false>, dim3(1), dim3(256), 0, s, (const uint32_t*)a->d_part, g.grid,
                           a->d_run, (const uint32_t*)ba.bad);
    HIP_TRY(hipGetLastError());
    if (b >= 0) {
        HIP_TRY(hipEventRecord(a->ev_used[b], s));
        a->used[b] = true;
        a->last_host = b;
    }
    a->t_next += m->n;
    return POSLO_OK;
}

extern "C" int poslo_audit_finish(poslo_audit* a, const uint8_t tag[64], void* stream, int* accept,
                                  uint8_t e_out[32]) {
    if (!a || !tag || !accept) return POSLO_E_INVAL;
    *accept = 0;
    int st;
    if ((st = release_host(a))) return st;
    poslo_ctx* c = a->c;
    HIP_TRY(hipSetDevice(c->device));
    const KeyEntry* key = ctx_key_of(c, a->prm.inst, a->pk, &st);
    if (!key) return st;
    return final_check(c, key, a->d_run, 1, tag, (hipStream_t)stream, accept, e_out, a->d_run + 9);
}

extern "C" int poslo_audit_position(const poslo_audit* a, uint64_t* t_next) {
    if (!a || !t_next) return POSLO_E_INVAL;
    *t_next = a->t_next;
    return POSLO_OK;
}

extern "C" int poslo_audit_export(poslo_audit* a, void* stream, uint8_t* buf, size_t cap, size_t* len) {
    if (!a || !len) return POSLO_E_INVAL;
    *len = 4 + 4 * 4 + 32 + 16 + 32 + 4 + a->ds.size();
    if (!buf || cap < *len) return POSLO_E_INVAL;
    int st;
    if ((st = release_host(a))) return st;
    HIP_TRY(hipSetDevice(a->c->device));
    uint32_t run[10];
    HIP_TRY(hipMemcpyAsync(run, a->d_run, sizeof run, hipMemcpyDeviceToHost, (hipStream_t)stream));
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    if (run[9]) return POSLO_E_INVAL;  // a POSLO++ message longer than 31 bytes was fed
    uint8_t* p = buf;
    memcpy(p, "PAUD", 4);
    p += 4;
    const uint32_t hdr[4] = {1, a->prm.inst, a->prm.log2_n1, a->prm.log2_n2};
    for (uint32_t v : hdr) {
        store_le32(p, v);
        p += 4;
    }
    memcpy(p, a->pk, 32);
    p += 32;
    store_le32(p, (uint32_t)a->t0);
    store_le32(p + 4, (uint32_t)(a->t0 >> 32));
    store_le32(p + 8, (uint32_t)a->t_next);
    store_le32(p + 12, (uint32_t)(a->t_next >> 32));
    p += 16;
    for (int k = 0; k < 8; k++) store_le32(p + 4 * k, run[k]);
    p += 32;
    store_le32(p, (uint32_t)a->ds.size());
    p += 4;
    memcpy(p, a->ds.data(), a->ds.size());
    return POSLO_OK;
}

extern "C" int poslo_audit_resume(poslo_ctx* c, const uint8_t* buf, size_t len, const poslo_params* prm,
                                  poslo_audit** out) {
    if (!c || !buf || !prm || !out) return POSLO_E_INVAL;
    *out = nullptr;
    const size_t fixed = 4 + 4 * 4 + 32 + 16 + 32 + 4;
    if (len < fixed || memcmp(buf, "PAUD", 4) != 0) return POSLO_E_INVAL;
    const uint8_t* p = buf + 4;
    if (load_le32(p) != 1 || load_le32(p + 4) != prm->inst || load_le32(p + 8) != prm->log2_n1 ||
        load_le32(p + 12) != prm->log2_n2)
        return POSLO_E_INVAL;
    p += 16;
    const uint8_t* pk = p;
    p += 32;
    const uint64_t t0 = load_le32(p) | ((uint64_t)load_le32(p + 4) << 32);
    const uint64_t tn = load_le32(p + 8) | ((uint64_t)load_le32(p + 12) << 32);
    p += 16;
    uint32_t e[8];
    for (int k = 0; k < 8; k++) e[k] = load_le32(p + 4 * k);
    if (!((prm->inst & POSLO_GROUP_FOURQ) ? scN_is_canonical(e) : sc_is_canonical(e))) return POSLO_E_INVAL;
    p += 32;
    const uint32_t dl = load_le32(p);
    p += 4;
    if (len != fixed + dl) return POSLO_E_INVAL;
    return audit_new(c, prm, pk, p, dl, t0, tn, e, out);
}

extern "C" void poslo_audit_free(poslo_audit* a) {
    if (!a) return;
    (void)hipSetDevice(a->c->device);
    if (a->copy) (void)hipStreamSynchronize(a->copy);
    (void)hipDeviceSynchronize();
    void* bufs[] = {a->d_run, a->d_tab, a->d_part, a->d_stage[0], a->d_stage[1], a->d_soff[0], a->d_soff[1]};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    for (int b = 0; b < 2; b++) {
        if (a->ev_copied[b]) (void)hipEventDestroy(a->ev_copied[b]);
        if (a->ev_used[b]) (void)hipEventDestroy(a->ev_used[b]);
    }
    if (a->copy) (void)hipStreamDestroy(a->copy);
    delete a;
}
