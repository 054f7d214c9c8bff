// The verifier context shared by the library's translation units: device
// scratch buffers, cached per-key tables, tuning state and kernel timing.
#pragma once

#include <stdint.h>
#include <string.h>

#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/poslo.h"
#include "comb.h"
#include "common.h"
#include "ge25519.h"

namespace poslo {

constexpr int kKtCount = 8;

// AES hot-kernel variants (T-table layout x LDS replication x block size)
struct AggVariant {
    const char* name;
    int nt;      // distinct rotated tables held in LDS
    int copies;  // bank-replicated copies of each table
    int block;   // threads per workgroup
    int perm;    // byte-addressed layout (64 copies, v_perm_b32 addressing)
};
int agg_aes_variant_count();
const AggVariant& agg_aes_variant(int v);
int agg_aes_default_variant();
// launch variant v (fast layout) or the generic-layout kernel
int launch_agg_aes(int v, bool fast, uint32_t grid, const void* batch_args, uint32_t* partials, hipStream_t s);
// the default variant (fast layout) or the any-layout form, also storing
// every entry's e_t mod q (8 words) and x_t (4 words, x_out may be null)
int launch_agg_aes_emit(bool fast, uint32_t grid, const void* batch_args, uint32_t* partials, uint32_t* e_out,
                        uint32_t* x_out, hipStream_t s);
// threads per workgroup of the any-layout form (and of the emit launches)
int agg_aes_any_block();
size_t agg_aes_lds_bytes(int v);
// the POSLO++ hot kernel (agg_addq.hip): layout as AggShape::addq_layout;
// with e_out set also every entry's e_t and x_t.  a.bad must be set.
int launch_agg_addq(int layout, uint32_t grid, const void* batch_args, uint32_t* partials, uint32_t* e_out,
                    uint32_t* x_out, hipStream_t s);
int agg_addq_block();
// the POSLO hot kernel (agg_sha.hip): layout 2 = 16-byte aligned fixed
// length, 1 = 4-byte aligned fixed length, 0 = any
constexpr int kAggShaBlock = 256;
int launch_agg_sha(int layout, uint32_t grid, const void* batch_args, uint32_t* partials, hipStream_t s);
int launch_agg_sha_emit(int layout, uint32_t grid, const void* batch_args, uint32_t* partials, uint32_t* e_out,
                        uint32_t* x_out, hipStream_t s);

struct KeyEntry {
    std::string pk;               // cache id: the 32 key bytes (FourQ keys: plus one tag byte)
    bool fourq = false;           // a FourQ key (fourq.h) rather than an edwards25519 one
    uint32_t* d_table = nullptr;  // comb table of Y on the device
    std::shared_ptr<void> slab;   // allocation holding d_table (shared by a bulk load)
    std::shared_ptr<void> wide;   // Y's wide table (comb.h), built on demand
    bool wide_pinned = false;     // wide table asked for by poslo_ctx_keys_widen: kept with the key
};

constexpr size_t kMaxWideKeys = 8;  // wide key tables built on demand kept per context (48 MiB each)

}  // namespace poslo

struct poslo_ctx {
    int device = 0;
    int num_cu = 256;
    // tuning: AES kernel variant and workgroups per CU (0 = derived)
    int agg_variant = -1;
    int wg_per_cu = 0;
    // per-kernel timing with HIP events on the launch stream (opt-in)
    uint32_t profile_mask = 0;  // bit k: time kernel POSLO_KT_k
    hipEvent_t ev[poslo::kKtCount][2] = {};
    bool ev_pending[poslo::kKtCount] = {};
    double kt_ms[poslo::kKtCount] = {};
    uint64_t kt_launches[poslo::kKtCount] = {};
    // scratch
    uint32_t* d_tab = nullptr;
    size_t tab_words = 0;
    uint32_t* d_part = nullptr;
    size_t part_words = 0;
    uint32_t* d_result = nullptr;
    uint32_t* h_result = nullptr;  // pinned
    // this device's copy of the fixed scratch array of the allocation-free
    // AVer entry point (its device address; shared by every context on the
    // device, kept until the process ends)
    uint32_t* d_fixed = nullptr;
    // comb tables: G (static) and per-key Y, LRU-bounded
    uint32_t* d_gtable = nullptr;
    uint32_t* d_gtable_wide = nullptr;  // built on first use (ctx_gtable_wide)
    uint32_t* d_gtable_fq = nullptr;    // FourQ generator's comb table, built on first use
    uint32_t* d_gtable_wide_fq = nullptr;  // its wide table (ctx_gtable_wide_fq)
    std::mutex wide_mu;
    size_t key_cap = 4096;
    std::list<poslo::KeyEntry> keys;  // front = most recent
    std::unordered_map<std::string, std::list<poslo::KeyEntry>::iterator> key_index;
    // scratch slots of the Distill / SeBVer / batched entry points
    uint32_t* xbuf[32] = {};
    size_t xbuf_words[32] = {};
};

namespace poslo {

int ctx_ensure(uint32_t** buf, size_t* have, size_t words);
// device scratch slot of at least `bytes` bytes (grown on demand, kept until
// the context is destroyed)
int ctx_scratch(poslo_ctx* c, int slot, size_t bytes, void** out);
void prof_begin(poslo_ctx* c, int k, hipStream_t s);
void prof_end(poslo_ctx* c, int k, hipStream_t s);
void prof_collect(poslo_ctx* c);
// device comb table of the key (built on first use); nullptr and
// *status = POSLO_E_ENCODING if pk is not a point encoding
const KeyEntry* ctx_key(poslo_ctx* c, const uint8_t pk[32], int* status);
// FourQ keys (fourq.h): the key's comb table, built on first use and kept
// in the same cache; E_ENCODING when pk is not a FourQ point encoding
const KeyEntry* ctx_key_fq(poslo_ctx* c, const uint8_t pk[32], int* status);
// the key of an instantiation word's group
const KeyEntry* ctx_key_of(poslo_ctx* c, uint32_t inst, const uint8_t pk[32], int* status);
// FourQ generator's comb table (built on first use), or nullptr
const uint32_t* ctx_gtable_fq(poslo_ctx* c);
// the cache id of a FourQ key
inline std::string fq_key_id(const uint8_t pk[32]) { return std::string((const char*)pk, 32) + '\x01'; }
// device comb tables of many keys (built on the device for the missing
// ones); tables[k] is key k's table.  Keys that are not point encodings get
// nullptr and are counted in *n_bad (the call then returns E_ENCODING).
// Keys of one call are never evicted by that call.  fourq: FourQ keys.
int ctx_keys_bulk(poslo_ctx* c, const uint8_t* pks, size_t n, std::vector<const uint32_t*>& tables, size_t* n_bad,
                  bool fourq = false);
// G's wide table for the per-entry checks (comb.h), built on first use;
// nullptr if it cannot be allocated
const uint32_t* ctx_gtable_wide(poslo_ctx* c);
// FourQ generator's wide table for the per-entry checks, built on first use;
// nullptr if it cannot be allocated
const uint32_t* ctx_gtable_wide_fq(poslo_ctx* c);
// Y's wide table for a resident key (ctx_key first), built on first use
// and kept for the kMaxWideKeys most recently used keys (besides those
// widened by poslo_ctx_keys_widen); nullptr on failure
const uint32_t* ctx_key_wide(poslo_ctx* c, const uint8_t pk[32]);
// Y's wide table of a resident edwards25519 key if it has one, else nullptr
// (builds nothing)
const uint32_t* ctx_key_wide_resident(poslo_ctx* c, const uint8_t pk[32]);
// per-context state of the multi-signer path, released with the context
void batch_release(poslo_ctx* c);
// comb tables (comb.h layout) of the m encoded points pks (host, 32 bytes
// each) into d_tab (device, m * kCombWords words), built on the device;
// ok[k] = 0 where pks[k] is not a point encoding.  Synchronous.
int build_comb_tables(const uint8_t* pks, size_t m, uint32_t* d_tab, std::vector<uint32_t>& ok);

struct BatchArgs;
struct DsArg;
bool params_ok(const poslo_params* p);
// words of an epoch table of ne rows: the rows, then POSLO++'s long-message
// flag word (padded to keep allocations aligned), then the seeds of the
// rows' subtrees of height kSeedMidHeight (4 words each) that the seed walk
// of large batches passes through
constexpr size_t kTabRowWords = 48;  // one epoch row (kEpochWords)
constexpr int kSeedMidHeight = 4;
constexpr size_t epoch_tab_words(uint64_t ne) {
    return (size_t)ne * kTabRowWords + 64 + ((ne >> kSeedMidHeight) + 2) * 4;
}
// host-side checks of a batch (parameters, ds parse, SR coverage of every
// epoch); fills the kernel argument block and the by-value ds, sizes the
// epoch table (the context's, or fixed_tab of fixed_epochs rows when set)
int prepare_batch(poslo_ctx* c, const poslo_params* prm, const poslo_msgs* m, const uint8_t* ds, size_t ds_len,
                  BatchArgs& a, DsArg& dsa, uint32_t& n_epochs, uint32_t* fixed_tab = nullptr,
                  uint64_t fixed_epochs = 0);
bool fast_layout(const poslo_msgs* m, uint64_t align);
int launch_seed_table(const DsArg& dsa, uint32_t inst, const BatchArgs& a, uint32_t n_epochs, hipStream_t s);

// Launch shape of the fused per-entry kernel for a batch: the AES variant
// (the any-layout form for offsets or unaligned messages), the SHA-256
// layout, and the grid (the resident workgroups of every CU, fewer for small
// batches)
struct AggShape {
    bool fast;
    int variant;  // AES variant; -1 with fast = false: the any-layout form
    int sha_layout;
    int addq_layout;  // POSLO++: 2 = 16-byte messages 16-byte aligned, 1 = 4-byte aligned fixed length, 0 = any
    uint32_t grid;
};
AggShape agg_shape(const poslo_ctx* c, const poslo_params* prm, const poslo_msgs* m);
// launch the fused per-entry kernel (g.grid partials of 9 words into
// partials); with e_out set, the emit form that also stores every entry's
// e_t mod q and x_t (AES: the default variant's shape only)
int launch_agg(poslo_ctx* c, const poslo_params* prm, const AggShape& g, const BatchArgs& a, uint32_t* partials,
               uint32_t* e_out, uint32_t* x_out, hipStream_t s);

// context scratch slots (ctx_scratch) of the POSLO-C entry points and of
// the staging copies of host-resident batches
constexpr int kSlotCEkeys = 20, kSlotCSigs = 21, kSlotCBits = 22;
constexpr int kSlotStageData = 28, kSlotStageOffsets = 29, kSlotStageSigs = 30;

// a host-resident batch (m->host) copied into the staging slots on s, dm
// its device view; a device batch is passed through.  With sigs_out, the
// batch's signatures (80 per entry, same memory kind) are staged too.
int stage_msgs(poslo_ctx* c, const poslo_msgs* m, hipStream_t s, poslo_msgs& dm, const uint8_t* sigs,
               const uint8_t** sigs_out);
// the final fold of n_part partials (9 words each), mod q and the
// aggregate check against tag; synchronizes s and returns accept and e.
// E_INVAL when bad (a device word, optional) is set.
int final_check(poslo_ctx* c, const KeyEntry* key, const uint32_t* partials, uint32_t n_part,
                const uint8_t tag[64], hipStream_t s, int* accept, uint8_t e_out[32],
                const uint32_t* bad = nullptr);

}  // namespace poslo
