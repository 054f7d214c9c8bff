// The multi-signer verification pipeline as a reusable, asynchronous unit:
// many signers' batches (jobs) verified by one persistent launch, with the
// device buffers and pinned staging of one in-flight launch.  Used by the
// synchronous batch entry points and by the serving loop, which keeps
// several runners in flight on separate streams.
#pragma once

#include <stdint.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "ctx.h"
#include "device_hash.h"
#include "scheme_host.h"

namespace poslo {

// device record of one job
struct BJob {
    const uint32_t* ty;       // comb table of the key
    const uint32_t* tyw;      // the key's wide table (comb.h), or nullptr
    const uint8_t* data;      // message bytes
    const uint64_t* offsets;  // job-local offsets (n + 1) into data, or nullptr: fixed msg_len
    uint64_t msg_len;
    const uint8_t* end;       // end of the readable message buffer, or nullptr
    const uint8_t* sigs;      // 80 bytes per entry (read by the individual checks only)
    uint64_t t0, n;
    uint64_t epoch_base;      // first row of the job in the epoch table
    uint64_t item_base, item_end;
    uint64_t vbase;           // first slot of the job in the individual-check numbering
    uint64_t ebase;           // first entry of the job in the launch's entry numbering
    uint32_t tag[16];         // LE words: s[8] || enc(R) bytes[8]
};

// work item: up to CHUNK (hashing) or 256 (individual checks) entries of one job
struct BItem {
    uint32_t job;
    uint32_t count;
    uint64_t first;  // entry offset within the job
};

// one job as the host hands it in
struct JobSpec {
    const uint32_t* ty;
    const uint32_t* tyw = nullptr;  // the key's resident wide table, if it has one
    const uint8_t* data;
    const uint64_t* offsets;
    uint64_t msg_len;
    uint64_t data_bytes;  // bytes readable from data, 0 if unknown
    const uint8_t* sigs;
    uint64_t t0, n;
    const uint8_t* ds;
    size_t ds_len;
    const uint8_t* tag;  // 64 bytes, host
};

struct HotVariant {
    const char* name;
    int inst, nt, block, chunk, sort, waves_per_simd;
    int pair;    // chunk = 2 * block: a lane takes the k-th shortest and the k-th longest entry
    int copies;  // AES table copies (0: 64; 32: two tables in 64 KB, aes_perm.h)
};
int batch_variant_count();
const HotVariant& batch_variant(int v);
int batch_default_variant(uint32_t inst);
// instantiations the multi-signer path takes: POSLO and POSLO+ at kappa = 128,
// on edwards25519 or FourQ
bool batch_inst_ok(uint32_t inst);
size_t hot_lds_bytes(const HotVariant& v);

class BatchRunner {
  public:
    BatchRunner() = default;
    BatchRunner(const BatchRunner&) = delete;
    BatchRunner& operator=(const BatchRunner&) = delete;
    ~BatchRunner();

    // host-side plan of a launch: checks every job (sizes, ds parse, SR
    // coverage of its epochs), builds the job, epoch-row and work-item
    // tables.  Keys must be resolved (JobSpec::ty).
    int plan(const poslo_params* prm, const JobSpec* jobs, uint32_t njobs, const poslo_tuning& t, int num_cu);
    // enqueue on s: table uploads, per-epoch seeds with the tags' decode,
    // the persistent hashing kernel, one aggregate check per job, and the
    // copy of the accept words to pinned memory.  With use_graph the kernel
    // sequence is captured once per argument set and replayed.
    // With emit, the hashing kernel also writes every entry's e_t mod q and
    // whether its x_t differs from the signature's (jobs need sigs), which
    // launch_verify then reads instead of hashing again.
    int launch(hipStream_t s, bool use_graph, poslo_ctx* prof, bool emit = false);
    // accept word of job j, valid once s has passed launch's work
    uint32_t accept(uint32_t j) const { return h_res_[j]; }
    // enqueue the individual checks of the listed jobs' entries; the invalid
    // ones are appended (in any order) to a device list whose count is
    // copied to pinned memory
    int launch_verify(const std::vector<uint32_t>& jobs, hipStream_t s, poslo_ctx* prof);
    // after s has passed launch_verify's work: the sorted (job, t) pairs
    int invalid(std::vector<std::pair<uint32_t, uint64_t>>& out, hipStream_t s);
    uint32_t njobs() const { return (uint32_t)jobs_.size(); }
    // device views for follow-up kernels on the same stream
    const BJob* d_jobs() const { return (const BJob*)d_jobs_; }
    const uint32_t* d_accept() const { return (const uint32_t*)d_res_; }
    const uint32_t* d_rdec() const { return (const uint32_t*)d_rdec_; }
    void forget_graphs();

  private:
    int grow(void** p, size_t* have, size_t bytes);
    int grow_pinned(void** p, size_t* have, size_t bytes);

    poslo_params prm_{};
    poslo_tuning tune_{};
    int num_cu_ = 256;
    std::vector<BJob> jobs_;
    std::vector<DsArg> ds_;
    std::vector<uint32_t> job_of_row_;
    std::vector<BItem> items_;
    std::vector<BItem> vtiles_;
    std::vector<std::pair<uint64_t, uint32_t>> vbase_;  // (slot base, job) of checked jobs
    uint64_t n_checked_ = 0;
    // device buffers (grown on demand, kept)
    void *d_jobs_ = nullptr, *d_ds_ = nullptr, *d_rows_ = nullptr, *d_items_ = nullptr, *d_tab_ = nullptr,
         *d_part_ = nullptr, *d_res_ = nullptr, *d_misc_ = nullptr, *d_rdec_ = nullptr, *d_vtiles_ = nullptr,
         *d_idx_ = nullptr, *d_ekeys_ = nullptr, *d_xbad_ = nullptr, *d_pair_ = nullptr, *d_stash_ = nullptr;
    size_t n_jobs_b_ = 0, n_ds_b_ = 0, n_rows_b_ = 0, n_items_b_ = 0, n_tab_b_ = 0, n_part_b_ = 0, n_res_b_ = 0,
           n_misc_b_ = 0, n_rdec_b_ = 0, n_vtiles_b_ = 0, n_idx_b_ = 0, n_ekeys_b_ = 0, n_xbad_b_ = 0,
           n_pair_b_ = 0, n_stash_b_ = 0;
    uint64_t n_entries_ = 0;
    bool emitted_ = false;  // the last launch wrote e_t and the x checks
    // pinned staging
    uint32_t* h_res_ = nullptr;
    size_t h_res_b_ = 0;
    uint64_t* h_misc_ = nullptr;
    size_t h_misc_b_ = 0;
    // captured graphs keyed by the bytes of every launch argument
    std::map<std::string, hipGraphExec_t> graphs_;
    hipStream_t capture_ = nullptr;
};

}  // namespace poslo
