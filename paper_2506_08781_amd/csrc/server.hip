// The serving loop: continuous admission of verification requests into
// multi-signer launches kept in flight on several streams.
//
// Requests (one signer's batch each: key id, entries t0..t0+n-1, messages,
// signatures, ds, tag) are queued by submit from any thread.  A worker
// thread admits queued requests in arrival order while the device budget
// allows (staging copies of host buffers plus a per-request scratch
// estimate) and their key is not in flight, forms a group of admitted
// requests whenever a stream slot is free, and launches the group as one
// multi-signer verification (per-epoch seeds, persistent hashing, one
// aggregate check per request).  Completed groups release their memory, so
// requests that arrived meanwhile are admitted into the next groups while
// earlier ones still run.  After the checks, one lane folds each accepted
// request's tag into its key's device-resident aggregate state; rejected
// requests (or all, by configuration) then get their entries verified
// individually to name the invalid ones.  A request's verdict and invalid
// list depend only on its own inputs, not on its group.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_run.h"
#include "device_fq.h"
#include "ge25519.h"
#include "sc25519.h"

namespace poslo {

// per-key state words: s (8, reduced mod q), R = (X, Y, Z, T) (32), entries (2);
// on FourQ s is reduced mod N and the coordinates are GF(p^2) words
constexpr int kStateWords = 48;

__global__ __launch_bounds__(64) void k_key_state(const BJob* jobs, const uint32_t* accept, const uint32_t* rdec,
                            const uint32_t* slot_of_job, uint32_t njobs, uint32_t* state, uint32_t fq) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    // one lane in job order: a key's requests of one group are folded in turn
    for (uint32_t j = 0; j < njobs; j++) {
        if (!accept[j]) continue;
        uint32_t* st = state + (uint64_t)slot_of_job[j] * kStateWords;
        uint32_t s[8], t[8];
        for (int k = 0; k < 8; k++) {
            s[k] = st[k];
            t[k] = jobs[j].tag[k];
        }
        if (fq) {
            scN_add(s, s, t);
            gq A, R;
            unstash_f2(A.X, st + 8, 1);
            unstash_f2(A.Y, st + 16, 1);
            unstash_f2(A.Z, st + 24, 1);
            unstash_f2(A.T, st + 32, 1);
            const uint32_t* r = rdec + (uint64_t)j * 17;
            unstash_f2(R.X, r + 1, 1);
            unstash_f2(R.Y, r + 9, 1);
            f2_one(R.Z);
            f2_mul(R.T, R.X, R.Y);
            gq_add(A, A, R);
            for (int k = 0; k < 8; k++) st[k] = s[k];
            stash_f2(st + 8, 1, A.X);
            stash_f2(st + 16, 1, A.Y);
            stash_f2(st + 24, 1, A.Z);
            stash_f2(st + 32, 1, A.T);
            uint64_t e = ((uint64_t)st[41] << 32 | st[40]) + jobs[j].n;
            st[40] = (uint32_t)e;
            st[41] = (uint32_t)(e >> 32);
            continue;
        }
        sc_add(s, s, t);
        ge A, R;
        for (int k = 0; k < 8; k++) {
            A.X.v[k] = st[8 + k];
            A.Y.v[k] = st[16 + k];
            A.Z.v[k] = st[24 + k];
            A.T.v[k] = st[32 + k];
        }
        const uint32_t* r = rdec + (uint64_t)j * 17;
        for (int k = 0; k < 8; k++) {
            R.X.v[k] = r[1 + k];
            R.Y.v[k] = r[9 + k];
        }
        fe_set(R.Z, 1);
        fe_mul(R.T, R.X, R.Y);
        ge_add(A, A, R);
        for (int k = 0; k < 8; k++) {
            st[k] = s[k];
            st[8 + k] = A.X.v[k];
            st[16 + k] = A.Y.v[k];
            st[24 + k] = A.Z.v[k];
            st[32 + k] = A.T.v[k];
        }
        uint64_t e = ((uint64_t)st[41] << 32 | st[40]) + jobs[j].n;
        st[40] = (uint32_t)e;
        st[41] = (uint32_t)(e >> 32);
    }
}

}  // namespace poslo

using namespace poslo;

namespace {

using Clock = std::chrono::steady_clock;

#define HIP_TRY(x)                                     \
    do {                                               \
        if ((x) != hipSuccess) return POSLO_E_DEVICE;  \
    } while (0)

struct Req {
    uint64_t ticket = 0;
    poslo_request r{};
    std::vector<uint8_t> ds, tag;
    uint32_t key_slot = 0;
    const uint32_t* ty = nullptr;
    uint64_t data_bytes = 0;
    uint64_t need = 0;        // admission footprint
    uint64_t stage_off = 0;   // arena offset of the staging copy
    uint64_t stage_bytes = 0;
    double t_submit = 0, t_admit = 0, t_launch = 0;
    // device views used by the launch
    const uint8_t* d_data = nullptr;
    const uint64_t* d_offsets = nullptr;
    const uint8_t* d_sigs = nullptr;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    BatchRunner runner;
    std::vector<Req*> group;
    int phase = 0;  // 0 idle, 1 checks queued, 2 individual checks queued
    uint32_t* d_slot_of_job = nullptr;
    size_t slot_cap = 0;
    std::vector<uint32_t> slot_of_job;  // host source of the upload, kept until the next launch
};

// first-fit allocator over one device region
struct Arena {
    uint8_t* base = nullptr;
    uint64_t size = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
    void init(uint8_t* b, uint64_t n) {
        base = b;
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(uint64_t n, uint64_t* off) {
        n = (n + 255) & ~255ull;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                uint64_t rest = it->second - n, o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        n = (n + 255) & ~255ull;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct poslo_server {
    int device = 0;
    poslo_server_cfg cfg{};
    poslo_ctx* ctx = nullptr;  // comb table of G and the key tables (never evicted)
    Clock::time_point t0;
    std::mutex mu;
    std::mutex reg_mu;  // one key registration at a time
    std::condition_variable cv_work, cv_done;
    int launching = 0;  // a group taken from the admitted list is being launched
    std::thread worker;
    bool stop = false;
    // keys
    std::unordered_map<uint32_t, std::pair<uint32_t, const uint32_t*>> keys;  // id -> (state slot, table)
    std::vector<uint8_t> key_busy;                                           // by state slot
    uint32_t* d_state = nullptr;
    size_t state_cap = 0, n_slots = 0;
    // requests
    uint64_t next_ticket = 1;
    std::deque<Req*> pending;
    std::deque<Req*> admitted;
    std::vector<Slot*> slots;
    Arena arena;
    uint8_t* d_arena = nullptr;
    uint64_t in_use = 0, peak = 0;
    // results
    std::deque<poslo_result> results;
    std::unordered_map<uint64_t, std::vector<uint64_t>> invalid;
    std::vector<double> latencies;
    uint64_t submitted = 0, completed = 0, entries_completed = 0, groups = 0;

    double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
    void run();
    int launch_group(Slot& sl);
    void complete(Slot& sl);
    void finish_group(Slot& sl, const std::vector<std::vector<uint64_t>>* inv, int status);
};

namespace {

uint64_t footprint(const poslo_server_cfg& cfg, const Req& q) {
    uint64_t n = q.r.n;
    uint64_t epochs = n ? ((q.r.t0 + n - 1) >> cfg.params.log2_n2) - (q.r.t0 >> cfg.params.log2_n2) + 1 : 0;
    uint64_t scratch = epochs * (kEpochWords * 4 + 4) + (n / 256 + 1) * 52 + 1024 + (cfg.distill ? 8 * n : 0);
    return scratch + q.stage_bytes;
}

}  // namespace

int poslo_server::launch_group(Slot& sl) {
    hipStream_t s = sl.stream;
    std::vector<JobSpec> specs(sl.group.size());
    std::vector<uint32_t>& slot_of_job = sl.slot_of_job;
    slot_of_job.assign(sl.group.size(), 0);
    double t = now_ms();
    for (size_t k = 0; k < sl.group.size(); k++) {
        Req& q = *sl.group[k];
        q.t_launch = t;
        if (!q.r.on_device && q.stage_bytes) {
            // staging copy of host buffers into the arena
            uint8_t* p = d_arena + q.stage_off;
            uint64_t dbytes = q.data_bytes, obytes = q.r.offsets ? 8 * (q.r.n + 1) : 0;
            if (dbytes) HIP_TRY(hipMemcpyAsync(p, q.r.data, dbytes, hipMemcpyHostToDevice, s));
            q.d_data = p;
            uint64_t o = (dbytes + 255) & ~255ull;
            if (obytes) HIP_TRY(hipMemcpyAsync(p + o, q.r.offsets, obytes, hipMemcpyHostToDevice, s));
            q.d_offsets = obytes ? (const uint64_t*)(p + o) : nullptr;
            o += (obytes + 255) & ~255ull;
            if (q.r.sigs && cfg.distill) {
                HIP_TRY(hipMemcpyAsync(p + o, q.r.sigs, 80 * q.r.n, hipMemcpyHostToDevice, s));
                q.d_sigs = p + o;
            }
        }
        JobSpec& sp = specs[k];
        sp.ty = q.ty;
        sp.data = q.d_data;
        sp.offsets = q.d_offsets;
        sp.msg_len = q.r.msg_len;
        sp.data_bytes = q.data_bytes;
        sp.sigs = q.d_sigs;
        sp.t0 = q.r.t0;
        sp.n = q.r.n;
        sp.ds = q.ds.data();
        sp.ds_len = q.ds.size();
        sp.tag = q.tag.data();
        slot_of_job[k] = q.key_slot;
    }
    poslo_tuning tune{cfg.variant >= 0 ? cfg.variant : batch_default_variant(cfg.params.inst), 0, 0, 0};
    int st = sl.runner.plan(&cfg.params, specs.data(), (uint32_t)specs.size(), tune, ctx->num_cu);
    if (st) return st;
    if (sl.slot_cap < slot_of_job.size()) {
        if (sl.d_slot_of_job) hipFree(sl.d_slot_of_job);
        sl.d_slot_of_job = nullptr;
        sl.slot_cap = 0;
        size_t cap = std::max<size_t>(slot_of_job.size(), 1024);
        if (hipMalloc((void**)&sl.d_slot_of_job, cap * 4) != hipSuccess) return POSLO_E_NOMEM;
        sl.slot_cap = cap;
    }
    HIP_TRY(hipMemcpyAsync(sl.d_slot_of_job, slot_of_job.data(), slot_of_job.size() * 4, hipMemcpyHostToDevice, s));
    if ((st = sl.runner.launch(s, false, ctx, cfg.distill != 0))) return st;
    hipLaunchKernelGGL(k_key_state, dim3(1), dim3(64), 0, s, sl.runner.d_jobs(), sl.runner.d_accept(),
                       sl.runner.d_rdec(), (const uint32_t*)sl.d_slot_of_job, (uint32_t)specs.size(), d_state,
                       (cfg.params.inst & POSLO_GROUP_FOURQ) ? 1u : 0u);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(sl.ev, s));
    sl.phase = 1;
    return POSLO_OK;
}

void poslo_server::finish_group(Slot& sl, const std::vector<std::vector<uint64_t>>* inv, int status) {
    double t = now_ms();
    std::lock_guard<std::mutex> lk(mu);
    for (size_t k = 0; k < sl.group.size(); k++) {
        Req* q = sl.group[k];
        poslo_result res{};
        res.ticket = q->ticket;
        res.user = q->r.user;
        res.status = status;
        res.accept = status == POSLO_OK ? (int)sl.runner.accept((uint32_t)k) : 0;
        res.entries = q->r.n;
        res.t_submit_ms = q->t_submit;
        res.t_admit_ms = q->t_admit;
        res.t_launch_ms = q->t_launch;
        res.t_done_ms = t;
        if (inv && !(*inv)[k].empty()) {
            res.n_invalid = (*inv)[k].size();
            invalid[q->ticket] = (*inv)[k];
        }
        results.push_back(res);
        latencies.push_back(t - q->t_submit);
        completed++;
        entries_completed += q->r.n;
        in_use -= q->need;
        if (q->stage_bytes) arena.release(q->stage_off, q->stage_bytes);
        key_busy[q->key_slot] = 0;
        delete q;
    }
    sl.group.clear();
    sl.phase = 0;
    cv_done.notify_all();
}

void poslo_server::complete(Slot& sl) {
    if (sl.phase == 1) {
        const int mode = cfg.distill;
        std::vector<uint32_t> which;
        for (uint32_t k = 0; k < sl.group.size(); k++)
            if (mode == 2 || (mode == 1 && !sl.runner.accept(k))) which.push_back(k);
        if (!which.empty()) {
            int st = sl.runner.launch_verify(which, sl.stream, ctx);
            if (st == POSLO_OK && hipEventRecord(sl.ev, sl.stream) == hipSuccess) {
                sl.phase = 2;
                return;
            }
            finish_group(sl, nullptr, st ? st : POSLO_E_DEVICE);
            return;
        }
        finish_group(sl, nullptr, POSLO_OK);
        return;
    }
    std::vector<std::pair<uint32_t, uint64_t>> out;
    int st = sl.runner.invalid(out, sl.stream);
    std::vector<std::vector<uint64_t>> inv(sl.group.size());
    for (auto& p : out) inv[p.first].push_back(p.second);
    finish_group(sl, &inv, st);
}

void poslo_server::run() {
    hipSetDevice(device);
    for (;;) {
        bool progressed = false;
        // completions
        for (Slot* sl : slots) {
            if (!sl->phase) continue;
            hipError_t q = hipEventQuery(sl->ev);
            if (q == hipSuccess) {
                complete(*sl);
                progressed = true;
            } else if (q != hipErrorNotReady) {
                // the stream failed: report the group instead of waiting for it
                finish_group(*sl, nullptr, POSLO_E_DEVICE);
                progressed = true;
            }
        }
        // admission in arrival order, by device budget and key exclusivity
        std::vector<Req*> to_launch;
        Slot* free_slot = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            bool any_inflight = false;
            for (Slot* sl : slots) any_inflight |= sl->phase != 0;
            for (auto it = pending.begin(); it != pending.end();) {
                Req* q = *it;
                if (key_busy[q->key_slot]) {
                    ++it;
                    continue;
                }
                bool alone = in_use == 0 && admitted.empty() && !any_inflight;
                if (in_use + q->need > cfg.mem_bytes && !alone) break;  // keep arrival order
                if (q->stage_bytes && !arena.alloc(q->stage_bytes, &q->stage_off)) {
                    if (alone) {
                        // larger than the whole staging arena: fail it
                        poslo_result res{};
                        res.ticket = q->ticket;
                        res.user = q->r.user;
                        res.status = POSLO_E_NOMEM;
                        res.t_submit_ms = q->t_submit;
                        res.t_done_ms = now_ms();
                        results.push_back(res);
                        completed++;
                        delete q;
                        it = pending.erase(it);
                        cv_done.notify_all();
                        continue;
                    }
                    break;
                }
                q->t_admit = now_ms();
                in_use += q->need;
                peak = std::max(peak, in_use);
                key_busy[q->key_slot] = 1;
                admitted.push_back(q);
                it = pending.erase(it);
                progressed = true;
            }
            for (Slot* sl : slots)
                if (!sl->phase) {
                    free_slot = sl;
                    break;
                }
            if (free_slot && !admitted.empty()) {
                // up to max_group requests and max_group_entries entries (at least one)
                size_t take = 0;
                uint64_t ent = 0;
                while (take < admitted.size() && take < cfg.max_group) {
                    const uint64_t n = admitted[take]->r.n;
                    if (take > 0 && ent + n > cfg.max_group_entries) break;
                    ent += n;
                    take++;
                }
                to_launch.assign(admitted.begin(), admitted.begin() + take);
                admitted.erase(admitted.begin(), admitted.begin() + take);
                launching = 1;
                groups++;
            }
            if (stop && pending.empty() && admitted.empty() && to_launch.empty()) {
                bool busy = false;
                for (Slot* sl : slots) busy |= sl->phase != 0;
                if (!busy) return;
            }
        }
        if (!to_launch.empty()) {
            free_slot->group = to_launch;
            int st = launch_group(*free_slot);
            if (st) {
                // the group failed before its checks were queued: wait for what
                // was queued, report the error
                hipStreamSynchronize(free_slot->stream);
                finish_group(*free_slot, nullptr, st);
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                launching = 0;
            }
            progressed = true;
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

extern "C" int poslo_server_create(int device, const poslo_server_cfg* cfg, poslo_server** out) {
    if (!cfg || !out || !params_ok(&cfg->params) || !batch_inst_ok(cfg->params.inst)) return POSLO_E_INVAL;
    if (cfg->distill < 0 || cfg->distill > 2) return POSLO_E_INVAL;
    if (cfg->variant >= batch_variant_count() ||
        (cfg->variant >= 0 && batch_variant(cfg->variant).inst != (int)inst_base(cfg->params.inst)))
        return POSLO_E_INVAL;
    *out = nullptr;
    poslo_ctx* ctx = nullptr;
    int st = poslo_ctx_create(device, &ctx);
    if (st) return st;
    ctx->key_cap = SIZE_MAX / 4;  // registered keys are never evicted
    // the per-entry checks' generator table, built now rather than by the worker
    if (cfg->distill && !((cfg->params.inst & POSLO_GROUP_FOURQ) ? ctx_gtable_wide_fq(ctx) : ctx_gtable_wide(ctx))) {
        poslo_ctx_destroy(ctx);
        return POSLO_E_NOMEM;
    }
    poslo_server* S = new poslo_server();
    S->device = device;
    S->cfg = *cfg;
    if (!S->cfg.n_streams) S->cfg.n_streams = 4;
    if (!S->cfg.max_group) S->cfg.max_group = 256;
    if (!S->cfg.max_group_entries) S->cfg.max_group_entries = 1ull << 21;
    if (!S->cfg.mem_bytes) S->cfg.mem_bytes = 8ull << 30;
    if (S->cfg.variant < 0) S->cfg.variant = -1;
    S->ctx = ctx;
    S->t0 = Clock::now();
    for (uint32_t k = 0; k < S->cfg.n_streams; k++) {
        Slot* sl = new Slot();
        if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming) != hipSuccess) {
            delete sl;
            poslo_server_destroy(S);
            return POSLO_E_DEVICE;
        }
        S->slots.push_back(sl);
    }
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    return POSLO_OK;
}

extern "C" int poslo_server_register_keys(poslo_server* S, const uint32_t* ids, const uint8_t* pks, size_t n) {
    if (!S || (n && (!ids || !pks))) return POSLO_E_INVAL;
    if (hipSetDevice(S->device) != hipSuccess) return POSLO_E_DEVICE;
    std::lock_guard<std::mutex> reg(S->reg_mu);
    std::vector<const uint32_t*> tables;
    size_t bad = 0;
    int st = ctx_keys_bulk(S->ctx, pks, n, tables, &bad, (S->cfg.params.inst & POSLO_GROUP_FOURQ) != 0);
    if (st) return st;
    std::lock_guard<std::mutex> lk(S->mu);
    // an id registered again is replaced only while none of its requests is
    // queued, admitted or in flight: its key table and state slot are in use
    for (size_t k = 0; k < n; k++) {
        auto it = S->keys.find(ids[k]);
        if (it == S->keys.end()) continue;
        const uint32_t slot = it->second.first;
        if (S->launching || S->key_busy[slot]) return POSLO_E_BUSY;
        for (const Req* q : S->pending)
            if (q->key_slot == slot) return POSLO_E_BUSY;
        for (const Req* q : S->admitted)
            if (q->key_slot == slot) return POSLO_E_BUSY;
    }
    size_t need = S->n_slots;
    for (size_t k = 0; k < n; k++)
        if (!S->keys.count(ids[k])) need++;
    if (need > S->state_cap) {
        // growing the state array needs the device idle for this server
        for (Slot* sl : S->slots)
            if (sl->phase) return POSLO_E_BUSY;
        if (!S->pending.empty() || !S->admitted.empty() || S->launching) return POSLO_E_BUSY;
        size_t cap = std::max<size_t>(need, 2 * S->state_cap);
        uint32_t* d = nullptr;
        if (hipMalloc((void**)&d, cap * kStateWords * 4) != hipSuccess) return POSLO_E_NOMEM;
        if (S->d_state &&
            hipMemcpy(d, S->d_state, S->n_slots * kStateWords * 4, hipMemcpyDeviceToDevice) != hipSuccess) {
            hipFree(d);
            return POSLO_E_DEVICE;
        }
        if (S->d_state) hipFree(S->d_state);
        S->d_state = d;
        S->state_cap = cap;
        S->key_busy.resize(cap, 0);
    }
    // fresh state: s = 0, R = identity (0, 1, 1, 0), no entries
    std::vector<uint32_t> init(kStateWords, 0);
    init[16] = 1;
    init[24] = 1;
    for (size_t k = 0; k < n; k++) {
        auto it = S->keys.find(ids[k]);
        uint32_t slot;
        if (it != S->keys.end()) {
            slot = it->second.first;
            it->second.second = tables[k];
        } else {
            slot = (uint32_t)S->n_slots++;
            S->keys[ids[k]] = {slot, tables[k]};
        }
        if (hipMemcpy(S->d_state + (size_t)slot * kStateWords, init.data(), kStateWords * 4,
                      hipMemcpyHostToDevice) != hipSuccess)
            return POSLO_E_DEVICE;
    }
    return POSLO_OK;
}

extern "C" int poslo_server_submit(poslo_server* S, const poslo_request* r, uint64_t* ticket) {
    if (!S || !r || !ticket || !r->tag || !r->ds) return POSLO_E_INVAL;
    if (r->n && !r->data) return POSLO_E_INVAL;
    if (r->n && !r->offsets && !r->msg_len && r->data_bytes) return POSLO_E_INVAL;
    if (S->cfg.distill && r->n && !r->sigs) return POSLO_E_INVAL;
    // per-request checks here, so that a launch group never fails for one
    // request's inputs: entry range, ds format and SR coverage of its epochs
    {
        const poslo_params& pp = S->cfg.params;
        uint64_t nmax = 1ull << (pp.log2_n1 + pp.log2_n2);
        if (r->t0 > nmax || r->n > nmax - r->t0) return POSLO_E_INVAL;
        std::vector<hostside::DsNode> nodes;
        if (!hostside::ds_parse(r->ds, r->ds_len, nodes)) return POSLO_E_INVAL;
        if (r->n) {
            uint64_t e0 = r->t0 >> pp.log2_n2, e1 = (r->t0 + r->n - 1) >> pp.log2_n2;
            for (uint64_t e = e0; e <= e1; e++)
                if (hostside::sr_node(nodes.data(), (int)nodes.size(), e) < 0) return POSLO_E_SEED;
        }
    }
    Req* q = new Req();
    q->r = *r;
    q->ds.assign(r->ds, r->ds + r->ds_len);
    q->tag.assign(r->tag, r->tag + 64);
    q->r.ds = nullptr;
    q->r.tag = nullptr;
    // message bytes: given, else offsets[n] (host offsets only), else n * msg_len
    q->data_bytes = r->data_bytes;
    if (!q->data_bytes) {
        if (!r->offsets)
            q->data_bytes = r->n * r->msg_len;
        else if (!r->on_device)
            q->data_bytes = r->offsets[r->n];
    }
    if (r->on_device) {
        q->d_data = r->data;
        q->d_offsets = r->offsets;
        q->d_sigs = r->sigs;
    } else if (r->n) {
        uint64_t ob = r->offsets ? 8 * (r->n + 1) : 0;
        q->stage_bytes = ((q->data_bytes + 255) & ~255ull) + ((ob + 255) & ~255ull) + (S->cfg.distill ? 80 * r->n : 0);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->keys.find(r->key_id);
    if (it == S->keys.end()) {
        delete q;
        return POSLO_E_INVAL;
    }
    if (q->stage_bytes && !S->d_arena) {
        // the staging arena is taken from the budget on first use
        if (hipMalloc((void**)&S->d_arena, S->cfg.mem_bytes) != hipSuccess) {
            delete q;
            return POSLO_E_NOMEM;
        }
        S->arena.init(S->d_arena, S->cfg.mem_bytes);
    }
    q->key_slot = it->second.first;
    q->ty = it->second.second;
    q->need = footprint(S->cfg, *q);
    q->ticket = S->next_ticket++;
    q->t_submit = S->now_ms();
    S->pending.push_back(q);
    S->submitted++;
    *ticket = q->ticket;
    S->cv_work.notify_one();
    return POSLO_OK;
}

extern "C" int poslo_server_poll(poslo_server* S, poslo_result* out, size_t cap, size_t* n, double timeout_ms) {
    if (!S || !n || (cap && !out)) return POSLO_E_INVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->results.empty() && timeout_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms),
                            [S] { return !S->results.empty(); });
    size_t k = 0;
    while (k < cap && !S->results.empty()) {
        out[k++] = S->results.front();
        S->results.pop_front();
    }
    *n = k;
    return POSLO_OK;
}

extern "C" int poslo_server_take_invalid(poslo_server* S, uint64_t ticket, uint64_t* out, size_t cap, size_t* n) {
    if (!S || !n) return POSLO_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->invalid.find(ticket);
    if (it == S->invalid.end()) return POSLO_E_INVAL;
    *n = it->second.size();
    if (it->second.size() > cap) return POSLO_OK;  // call again with room; the list is kept
    if (!it->second.empty()) memcpy(out, it->second.data(), it->second.size() * 8);
    S->invalid.erase(it);
    return POSLO_OK;
}

extern "C" int poslo_server_key_state(poslo_server* S, uint32_t key_id, uint8_t tag[64], uint64_t* entries) {
    if (!S || !tag) return POSLO_E_INVAL;
    uint32_t slot;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->keys.find(key_id);
        if (it == S->keys.end()) return POSLO_E_INVAL;
        slot = it->second.first;
        if (S->key_busy[slot]) return POSLO_E_BUSY;
    }
    uint32_t w[kStateWords];
    if (hipSetDevice(S->device) != hipSuccess ||
        hipMemcpy(w, S->d_state + (size_t)slot * kStateWords, sizeof w, hipMemcpyDeviceToHost) != hipSuccess)
        return POSLO_E_DEVICE;
    for (int k = 0; k < 8; k++) store_le32(tag + 4 * k, w[k]);
    if (S->cfg.params.inst & POSLO_GROUP_FOURQ) {
        gq A;
        for (int k = 0; k < 4; k++) {
            A.X.a.v[k] = w[8 + k], A.X.b.v[k] = w[12 + k];
            A.Y.a.v[k] = w[16 + k], A.Y.b.v[k] = w[20 + k];
            A.Z.a.v[k] = w[24 + k], A.Z.b.v[k] = w[28 + k];
            A.T.a.v[k] = w[32 + k], A.T.b.v[k] = w[36 + k];
        }
        fq_encode(tag + 32, A);
    } else {
        ge A;
        for (int k = 0; k < 8; k++) {
            A.X.v[k] = w[8 + k];
            A.Y.v[k] = w[16 + k];
            A.Z.v[k] = w[24 + k];
            A.T.v[k] = w[32 + k];
        }
        ge_encode(tag + 32, A);
    }
    if (entries) *entries = (uint64_t)w[41] << 32 | w[40];
    return POSLO_OK;
}

extern "C" int poslo_server_stats_get(poslo_server* S, poslo_server_stats* o) {
    if (!S || !o) return POSLO_E_INVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    memset(o, 0, sizeof *o);
    o->submitted = S->submitted;
    o->completed = S->completed;
    o->queued = S->pending.size() + S->admitted.size();
    for (Slot* sl : S->slots) o->in_flight += sl->group.size();
    o->entries_completed = S->entries_completed;
    o->groups_launched = S->groups;
    o->bytes_in_use = S->in_use;
    o->bytes_peak = S->peak;
    if (!S->latencies.empty()) {
        std::vector<double> l = S->latencies;
        std::sort(l.begin(), l.end());
        o->latency_p50_ms = l[(size_t)(0.50 * (l.size() - 1) + 0.5)];
        o->latency_p99_ms = l[(size_t)(0.99 * (l.size() - 1) + 0.5)];
    }
    o->elapsed_ms = S->now_ms();
    return POSLO_OK;
}

extern "C" void poslo_server_destroy(poslo_server* S) {
    if (!S) return;
    if (S->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        S->worker.join();
    }
    hipSetDevice(S->device);
    hipDeviceSynchronize();
    for (Slot* sl : S->slots) {
        if (sl->d_slot_of_job) hipFree(sl->d_slot_of_job);
        if (sl->ev) hipEventDestroy(sl->ev);
        if (sl->stream) hipStreamDestroy(sl->stream);
        delete sl;
    }
    for (Req* q : S->pending) delete q;
    for (Req* q : S->admitted) delete q;
    if (S->d_state) hipFree(S->d_state);
    if (S->d_arena) hipFree(S->d_arena);
    if (S->ctx) poslo_ctx_destroy(S->ctx);
    delete S;
}
