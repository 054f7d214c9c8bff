/*
 * poslo.h - C ABI of the POSLO-F verifier library for AMD Instinct MI355X
 * (gfx950).
 *
 * The library implements the verifier side of POSLO-F (Nouma and Yavuz,
 * "Lightweight and High-Throughput Secure Logging for Internet of Things and
 * Cold Cloud Continuum", arXiv 2506.08781): aggregate verification (AVer,
 * paper section "Fine-grained public-key POSLO", which reuses steps 2-8 of
 * POSLO-C.AVer), the GPU batch verifier of section "POSLO Parallel Batch
 * Verification" (figure "Parallel POSLO signature verification algorithm"),
 * and distillation / selective batch verification (Distill and SeBVer,
 * section "POSLO-C Distillation and Selective Batch Verification", applied
 * entry by entry as the POSLO-F text prescribes).  A host-side signer (Kg,
 * Sig, Agg) produces test data.
 *
 * Conventions
 *  - Every function returns 0 (POSLO_OK) or a negative POSLO_E_* code.
 *  - A verification reject is NOT an error: it is status 0 with *accept = 0,
 *    mirroring "return b = 0" in the paper.
 *  - Pointers documented as "device" point to GPU memory (hipMalloc or a
 *    torch CUDA tensor) on the context's device; "host" pointers point to
 *    CPU memory.  All buffers are owned by the caller unless a *_free call
 *    is named.
 *  - Work is issued on the caller's stream (a hipStream_t passed as void*;
 *    NULL means the default stream).  Calls that return a verdict
 *    synchronize that stream before returning.
 *  - A poslo_ctx is not thread-safe; use one per host thread.
 *
 * Byte formats (readings of the paper, which fixes no encodings)
 *  - entry index t is 0-based; epoch i = t >> log2_n2, j = t & (n2 - 1).
 *  - signature sigma_t: 80 bytes = LE32B(s_t) || enc(R_t) || x_t
 *    (|sigma| = 2|q| + kappa, paper table "Private/public key and signature
 *    sizes").
 *  - aggregate tag: 64 bytes = LE32B(s) || enc(R).
 *  - public key: 32 bytes = enc(Y).  enc() is the RFC 8032 point encoding
 *    of edwards25519 (y little-endian, parity of x in bit 255).
 *  - ds (disclosed seeds stack, section "POSLO Data Types and Seed
 *    Management"): 1 count byte, then per node {u8 depth; u8 pad[3] = 0;
 *    u32 LE index; u8 value[16]}, bottom of the stack first, at most 32
 *    nodes.
 */
#ifndef POSLO_H
#define POSLO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    POSLO_OK = 0,
    POSLO_E_INVAL = -1,     /* bad argument, size or parameter */
    POSLO_E_NOMEM = -2,     /* host or device allocation failed */
    POSLO_E_DEVICE = -3,    /* a HIP call failed */
    POSLO_E_SEED = -4,      /* SR returned bottom: ds does not cover an epoch */
    POSLO_E_ENCODING = -5,  /* a public key or commitment is not a point */
    POSLO_E_EXHAUSTED = -6, /* signer state reached t = n */
    POSLO_E_BUSY = -7       /* resource temporarily unavailable */
};

/* Instantiations (paper, table "Instantiations of POSLO schemes").
 * POSLO++ takes messages of at most 31 bytes: Add_q(m, x_t) = LE(m) + LE(x_t)
 * stays below q, so e_t needs no reduction; longer messages are E_INVAL. */
enum {
    POSLO_INST_SHA256 = 0,   /* POSLO: PRF and H from SHA-256 */
    POSLO_INST_AES = 1,      /* POSLO+: PRF from MMO-AES-128, H = MDC-2-AES-128 */
    POSLO_INST_AES_ADDQ = 2  /* POSLO++: PRF from MMO-AES-128, H = Add_q */
};

/* Flag on an AES-based instantiation: kappa = 127 (paper, the remark on
 * kappa = 127 under the instantiations).  Tree seeds are 127 bits (bit 127 of
 * their 16 bytes clear) and a tree PRF call PRF_b(x) is the one MMO block
 * x + b * 2^127; PRF inputs of any other length keep the byte suffix b.  Every
 * PRF output, x_t included, is taken mod 2^127.  Without the flag kappa = 128. */
#define POSLO_KAPPA127 4u

/* Flag: the FourQ group (the paper's curve) instead of edwards25519, with
 * POSLO or POSLO+.  FourQ is -x^2 + y^2 = 1 + d x^2 y^2 over GF(p^2),
 * p = 2^127 - 1, with FourQ's published d, subgroup order N (246 bits) and
 * generator; scalars (y, r_t, s_t, e_t = LE256(H) mod N) are taken mod N.
 * A point encodes as y0 || y1 (16-byte little-endian halves of
 * y = y0 + y1 i, each below p) with bit 255 holding the sign of x (x0 mod 2
 * if x0 != 0, else x1 mod 2).  Taken by the signer (poslo_kg, poslo_sig,
 * poslo_sig_batch, poslo_agg_inst), poslo_aver, poslo_aver_fixed, the
 * streaming audit, poslo_ekeys (e_t mod N), poslo_distill and poslo_sebver
 * (the individual checks with Y's 8-bit and G's wide FourQ tables),
 * POSLO-C (poslo_c_key_load with FourQ commitments, poslo_c_aver,
 * poslo_c_distill, poslo_c_sebver), the device signer
 * (poslo_gpu_keys_create, poslo_gpu_sign), the multi-signer batch
 * (poslo_verify_batch, poslo_autotune_batch) and the serving loop.
 * poslo_ctx_keys_load and poslo_ctx_keys_widen take edwards25519 keys only;
 * FourQ keys become resident on first use. */
#define POSLO_GROUP_FOURQ 8u

/* 1 if inst is an instantiation word (SHA256, AES or AES_ADDQ, the last two
 * optionally with POSLO_KAPPA127; SHA256 or AES optionally with
 * POSLO_GROUP_FOURQ), else 0 */
int poslo_inst_valid(uint32_t inst);

/* Public parameters I (paper, POSLO-F.Kg): instantiation word, n1 =
 * 2^log2_n1 epochs of n2 = 2^log2_n2 entries each.  BPV parameters (v, k)
 * are used by the signer only; v must be a power of two <= 65536.  The
 * multi-signer batch verifier and the serving loop take POSLO and POSLO+ at
 * kappa = 128 only (E_INVAL otherwise). */
typedef struct poslo_params {
    uint32_t inst;
    uint32_t log2_n1; /* 0..31 */
    uint32_t log2_n2; /* 0..31; log2_n1 + log2_n2 <= 40 */
    uint32_t bpv_v;   /* 1024 in the paper */
    uint32_t bpv_k;   /* 16 in the paper */
} poslo_params;

/* A batch of consecutive log entries t0 .. t0+n-1.  Fixed length:
 * offsets == NULL, entry p occupies data[p*msg_len .. (p+1)*msg_len).
 * Variable length: offsets (n+1 u64) gives entry p as
 * data[offsets[p] .. offsets[p+1]), msg_len is ignored.  data_bytes is the
 * size of the data buffer (0 = unknown); when known, unaligned messages are
 * read with aligned word loads that stay inside it.
 * host = 0: data and offsets are device pointers.  host = 1: they are host
 * pointers (pinned memory makes the copy asynchronous; pageable memory
 * works, with a synchronous copy), and the call copies the batch (and, for
 * Distill, the signatures, which are then host pointers too) into the
 * context's device staging buffers on its stream before hashing:
 * data_bytes (or n*msg_len, or offsets[n]) bytes, the offsets, 80*n
 * signature bytes.  The host buffers must stay unchanged until the call
 * returns.  poslo_aver_fixed takes device batches only. */
typedef struct poslo_msgs {
    const uint8_t* data;     /* device, or host when host = 1; may be NULL for a fixed length of 0 */
    const uint64_t* offsets; /* same memory as data, or NULL */
    uint64_t msg_len;
    uint64_t n;
    uint64_t t0;
    uint64_t data_bytes;
    uint32_t host;           /* 0: device pointers; 1: host pointers */
    uint32_t reserved;       /* 0 */
} poslo_msgs;

/* Library version string. */
const char* poslo_version(void);

/* Human-readable text for a status code. */
const char* poslo_strerror(int status);

/* ---------------------------------------------------------------- signer */

typedef struct poslo_signer poslo_signer;

/* POSLO-F.Kg (paper, figure "Fine-grained public-key POSLO"): y, root seed
 * x_D[0] and the BPV table derived deterministically from a 32-byte seed
 * with the scheme's PRF_0.  pk: host, 32 bytes out.  *sk is freed with
 * poslo_signer_free.  E_INVAL on bad params. */
int poslo_kg(const poslo_params* params, const uint8_t seed[32], poslo_signer** sk, uint8_t pk[32]);

void poslo_signer_free(poslo_signer* sk);

/* POSLO-F.Sig of the next entry t = St.t: sigma_t = (s_t, R_t, x_t) with
 * SSO at the first entry of each epoch and BPV.Online commitments.
 * m: host, len bytes.  sig: host, 80 bytes out.  E_EXHAUSTED at t = n. */
int poslo_sig(poslo_signer* sk, const uint8_t* m, size_t len, uint8_t sig[80]);

/* Sign n consecutive entries (host buffers; offsets has n+1 entries, or is
 * NULL for fixed msg_len) with up to nthreads host threads (0 = all cores).
 * Produces the same bytes as n calls of poslo_sig. sigs: host, 80*n out. */
int poslo_sig_batch(poslo_signer* sk, const uint8_t* msgs, const uint64_t* offsets, uint64_t msg_len,
                    uint64_t n, uint8_t* sigs, int nthreads);

/* Current state index t (number of entries signed). */
uint64_t poslo_signer_count(const poslo_signer* sk);

/* The signer's current disclosed-seed stack ds in the wire format above
 * (buf: host, cap bytes; *len gets the size).  E_INVAL if cap is too small. */
int poslo_ds_export(const poslo_signer* sk, uint8_t* buf, size_t cap, size_t* len);

/* POSLO-C.Agg as used by POSLO-F (paper, figure "Digital signature
 * algorithms"): s = sum s_t mod q, R = sum R_t.  sigs: host, count records
 * of stride bytes (>= 80).  tag: host, 64 bytes out.  E_ENCODING if an R_t
 * does not decode. */
int poslo_agg(const uint8_t* sigs, size_t stride, uint64_t count, uint8_t tag[64]);
/* The same in the group of an instantiation word (poslo_agg is edwards25519). */
int poslo_agg_inst(uint32_t inst, const uint8_t* sigs, size_t stride, uint64_t count, uint8_t tag[64]);

/* Host reference of the instantiated functions, for tooling and tests:
 * out16 = PRF_b(in) (b in {0,1}; with POSLO_KAPPA127 a 16-byte input is a
 * seed and must have bit 127 clear); out32 = H(in) (SHA-256 or MDC-2; E_INVAL
 * for POSLO++, whose Add_q is not a hash of one byte string). */
int poslo_prf_host(uint32_t inst, uint32_t b, const uint8_t* in, size_t len, uint8_t out16[16]);
int poslo_hash_host(uint32_t inst, const uint8_t* in, size_t len, uint8_t out32[32]);

/* ------------------------------------------------------------- verifier */

typedef struct poslo_ctx poslo_ctx;

/* A verifier context on one device: owns scratch buffers, cached key
 * tables and result staging.  E_DEVICE if the device cannot be used. */
int poslo_ctx_create(int device, poslo_ctx** ctx);
void poslo_ctx_destroy(poslo_ctx* ctx);

/* POSLO-F.AVer over a batch (the parallel verifier POSLO.PAVer: per entry
 * x_t = PRF_0(SR(ds, i) || j) and e_t = H(m_t || x_t), e = sum e_t mod q,
 * then the check R = e*Y + s*G).  pk, ds, tag: host.  *accept gets 1 or 0.
 * If e_out is not NULL it receives e mod q (32 bytes LE, host).
 * E_SEED if ds does not cover an epoch of the batch; E_ENCODING if pk is not
 * a point encoding; a non-canonical tag gives *accept = 0.  POSLO++: E_INVAL
 * if a message is longer than 31 bytes (found on the host for a fixed
 * length, by the kernels for an offsets batch).  kappa = 127: E_INVAL if a ds
 * node that the batch's epochs descend from has bit 127 set. */
int poslo_aver(poslo_ctx* ctx, const poslo_params* params, const uint8_t pk[32], const poslo_msgs* msgs,
               const uint8_t* ds, size_t ds_len, const uint8_t tag[64], void* stream, int* accept,
               uint8_t e_out[32]);

/* AVer that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as poslo_aver.
 * Its scratch (per-epoch seed rows, per-workgroup partial sums, result
 * words) is a fixed device array of POSLO_AVER_FIXED_SCRATCH_BYTES that each
 * GPU the library runs on holds until the process ends; the launch shape is
 * poslo_aver's default with the grid capped at 4096 workgroups.  Limits and
 * extra errors: E_INVAL when the batch spans more than
 * POSLO_AVER_FIXED_MAX_EPOCHS epochs, or when pk's table is not resident in
 * the context (load it first with poslo_ctx_keys_load; keys are evicted
 * only by later loads beyond the context's key capacity).  Every call on
 * one GPU uses the same array: calls that overlap in time on one GPU (any
 * context, any stream, any host thread) race and give wrong results; calls
 * that follow each other are independent (nothing in the array needs to
 * start at zero). */
#define POSLO_AVER_FIXED_MAX_EPOCHS 16384
#define POSLO_AVER_FIXED_SCRATCH_BYTES 3310112
int poslo_aver_fixed(poslo_ctx* ctx, const poslo_params* params, const uint8_t pk[32], const poslo_msgs* msgs,
                     const uint8_t* ds, size_t ds_len, const uint8_t tag[64], void* stream, int* accept,
                     uint8_t e_out[32]);

/* Kernel timing (opt-in): for each kernel whose bit (1 << POSLO_KT_*) is set
 * in the mask given to poslo_ctx_profile, the context records HIP events on
 * the launch stream around its launches and accumulates their elapsed time
 * (each event pair adds a few microseconds of stream gaps, so time only the
 * kernels you need; 0 turns timing off, POSLO_PROFILE_ALL times them all).
 * poslo_ctx_kernel_time returns the accumulated milliseconds and the number
 * of timed launches of one kernel (and clears them if reset != 0). */
enum {
    POSLO_KT_SEED = 0,   /* per-epoch seed table (SR / SC, hoisted PRF state) */
    POSLO_KT_AGG = 1,    /* fused PRF + digest + lazy aggregate (the hot loop) */
    POSLO_KT_FINAL = 2,  /* fold of partial sums, mod q, aggregate check */
    POSLO_KT_EKEYS = 3,  /* per-entry digests */
    POSLO_KT_VERIFY = 4, /* per-entry individual verification (Distill) */
    POSLO_KT_COMPACT = 5, /* invalid-index compaction and CCD aggregates */
    POSLO_KT_BATCH_HOT = 6, /* multi-signer persistent hashing kernel (eager launches only) */
    POSLO_KT_BATCH = 7      /* multi-signer pipeline: seeds, hashing, per-job checks */
};
#define POSLO_PROFILE_ALL 0xff
int poslo_ctx_profile(poslo_ctx* ctx, int kernels);
int poslo_ctx_kernel_time(poslo_ctx* ctx, int kernel, int reset, double* total_ms, uint64_t* launches);

/* Kernel tuning.  The POSLO+ hot kernel exists in several variants (number
 * of rotated T-tables held in LDS, bank-replicated copies of each, threads
 * per workgroup); poslo_agg_variant_name(v) describes variant v.
 * poslo_ctx_set_tuning selects a variant (-1: library default) and the
 * number of resident workgroups per compute unit (0: derived from the
 * variant's LDS footprint).  Results do not depend on the tuning. */
int poslo_agg_variant_count(void);
const char* poslo_agg_variant_name(int v);
int poslo_ctx_set_tuning(poslo_ctx* ctx, int agg_variant, int wg_per_cu);

/* Per-entry digests e_t mod q (mod N on FourQ; 32 bytes LE each) of a batch into e_dev
 * (device, 32*n bytes) and the one-time seeds x_t (16 bytes each) into
 * x_dev (device, 16*n bytes, may be NULL): the per-entry stage of AVer,
 * computed by poslo_aver's hot kernel (its default variant and launch
 * shape) in a form that also stores each entry's values.  Asynchronous on
 * stream, except for the seed-coverage check. */
int poslo_ekeys(poslo_ctx* ctx, const poslo_params* params, const poslo_msgs* msgs, const uint8_t* ds,
                size_t ds_len, uint8_t* e_dev, uint8_t* x_dev, void* stream);

/* ------------------------------------------------- distill and sebver */

/* Cold cryptographic data (paper, system model and section "POSLO-C
 * Distillation and Selective Batch Verification"): the valid aggregate
 * CCD^v, umbrella aggregates CCD^u over spans of U = ceil(n / n_umbrella)
 * entries, the invalid entries CCD^i with their signatures, and ds. */
typedef struct poslo_ccd poslo_ccd;

/* POSLO-F Distill over a batch: every entry is verified individually (x_t
 * equals PRF_0(x_0[i] || j), s_t below the group order (q; N on FourQ),
 * enc(e_t*Y + s_t*G) equals the R_t bytes); valid entries are aggregated
 * into CCD^v and their umbrella,
 * invalid ones are listed (sorted) with their signatures.  sigs: device,
 * 80*n bytes, 4-byte aligned, entry p at 80*p.  n_umbrella >= 1.  *out is
 * freed with poslo_ccd_free.  Errors as poslo_aver. */
int poslo_distill(poslo_ctx* ctx, const poslo_params* params, const uint8_t pk[32], const poslo_msgs* msgs,
                  const uint8_t* sigs, const uint8_t* ds, size_t ds_len, uint32_t n_umbrella, void* stream,
                  poslo_ccd** out);

/* CCD accessors (host memory owned by the CCD; valid until poslo_ccd_free). */
int poslo_ccd_invalid(const poslo_ccd* ccd, const uint64_t** idx, uint64_t* n);
int poslo_ccd_invalid_sig(const poslo_ccd* ccd, uint64_t k, uint8_t sig[80]);
int poslo_ccd_valid_tag(const poslo_ccd* ccd, uint8_t tag[64]);
/* umbrella tags (64 bytes each, in order) into tags (cap bytes, may be NULL
 * to query *n_umb and *span) */
int poslo_ccd_umbrellas(const poslo_ccd* ccd, uint8_t* tags, size_t cap, uint64_t* n_umb, uint64_t* span);
/* byte serialization for cold storage: *len gets the size; E_INVAL when cap
 * is too small or the input is malformed */
int poslo_ccd_export(const poslo_ccd* ccd, uint8_t* buf, size_t cap, size_t* len);
int poslo_ccd_import(const uint8_t* buf, size_t len, poslo_ccd** out);
void poslo_ccd_free(poslo_ccd* ccd);

/* SeBVer over distilled data (the same batch: msgs t0 and n must match the
 * CCD; a POSLO-C CCD is refused, see poslo_c_sebver).  mode 'V': one bit,
 * AVer of all entries not in CCD^i against CCD^v.
 * 'U': one bit per umbrella, AVer of its range minus CCD^i against its tag.
 * 'I': one bit per CCD^i entry, its individual verification (1 = valid).
 * bits: host, cap bytes; *n_bits gets the count. */
int poslo_sebver(poslo_ctx* ctx, const poslo_params* params, const uint8_t pk[32], const poslo_msgs* msgs,
                 const poslo_ccd* ccd, char mode, uint8_t* bits, size_t cap, size_t* n_bits, void* stream);

/* ------------------------------------------------------------- POSLO-C */

/* The coarse-grained variant POSLO-C (paper section "Coarse-grained
 * signer-optimal POSLO (POSLO-C)", figure "Coarse-grained signer-optimal
 * POSLO"): the public key holds Y and one aggregate commitment R~_i per
 * epoch, and a signature covers a whole epoch: s~_i = sum over the epoch's
 * entries of r_i^j - e_i^j * y.  Byte formats (readings; the paper fixes
 * none): pk = enc(Y) || enc(R~_0) || ... || enc(R~_{n1-1}), 32 * (1 + n1)
 * bytes; an epoch signature is LE32B(s~_i), with the signer's ds after the
 * epoch.  Batches are whole epochs (msgs->t0 and msgs->n multiples of n2;
 * E_INVAL otherwise, the paper's "return bottom"). */
typedef struct poslo_c_key poslo_c_key;

/* Load a POSLO-C public key (host, pk_len = 32 * (1 + 2^log2_n1) bytes,
 * log2_n1 <= 20) into the context's device: Y's fixed-base table, the epoch
 * commitments decoded once (kept as affine points on the device and as
 * prefix sums on the host).  E_ENCODING if Y or an R~_i is not a point
 * encoding.  Freed with poslo_c_key_free.  Synchronous. */
int poslo_c_key_load(poslo_ctx* ctx, const poslo_params* params, const uint8_t* pk, size_t pk_len,
                     poslo_c_key** out);
void poslo_c_key_free(poslo_c_key* key);

/* POSLO-C.AVer over the batch's epochs: e~ = sum over its entries of
 * H(m_i^j || PRF_0(SR(ds, i) || j)) mod q, R~ = Agg of the epochs' R~_i in
 * pk, accept iff s < q and R~ = e~*Y + s*G.  s: host, 32 bytes, the Agg
 * (sum mod q) of the epochs' signatures.  Same errors and e_out as
 * poslo_aver. */
int poslo_c_aver(poslo_ctx* ctx, const poslo_params* params, const poslo_c_key* key, const poslo_msgs* msgs,
                 const uint8_t* ds, size_t ds_len, const uint8_t s[32], void* stream, int* accept,
                 uint8_t e_out[32]);

/* POSLO-C.Distill: every epoch of the batch is verified on its own against
 * (s~_i, R~_i); valid epochs are aggregated into CCD^v and umbrellas of
 * U = ceil(k / n_umbrella) epochs (k epochs in the batch), invalid ones are
 * listed.  s_epochs: host, 32 bytes per epoch in order.  The CCD is
 * coarse: poslo_ccd_invalid gives sorted epoch indices i,
 * poslo_ccd_invalid_sig gives LE32B(s~_i) || enc(R~_i) || 16 zero bytes,
 * poslo_ccd_umbrellas' span counts epochs.  Errors as poslo_aver. */
int poslo_c_distill(poslo_ctx* ctx, const poslo_params* params, const poslo_c_key* key, const poslo_msgs* msgs,
                    const uint8_t* s_epochs, const uint8_t* ds, size_t ds_len, uint32_t n_umbrella, void* stream,
                    poslo_ccd** out);

/* POSLO-C.SeBVer over a coarse CCD of the same batch.  'V': AVer of every
 * epoch not in CCD^i against CCD^v; 'U': one bit per umbrella, AVer of its
 * epochs minus CCD^i against its tag; 'I': one bit per CCD^i epoch, AVer of
 * that epoch against its own (s~_i, R~_i).  bits: host, cap bytes. */
int poslo_c_sebver(poslo_ctx* ctx, const poslo_params* params, const poslo_c_key* key, const poslo_msgs* msgs,
                   const poslo_ccd* ccd, char mode, uint8_t* bits, size_t cap, size_t* n_bits, void* stream);

/* ------------------------------------------------------- streaming audit */

/* AVer over a log fed in chunks, for logs too large to hold on the device
 * at once (paper section "Experimental Evaluation on GPUs": a 1 TB log
 * audited in 1 GB chunks).  e = sum of H(m_t || x_t) mod q is additive, so
 * each chunk's digests fold into a running e mod q on the device and the
 * check R = e*Y + s*G runs once, at poslo_audit_finish.  The running state
 * (key, ds, first and next entry, e mod q) exports to bytes and resumes in
 * another process or on another device.
 * All calls on one audit use one stream (the chunks' kernels share the
 * audit's buffers in stream order) and one host thread. */
typedef struct poslo_audit poslo_audit;

/* Start an audit of entries t0, t0+1, ... of the signer with public key pk
 * (host, 32 bytes), whose ds (host) covers every epoch to be fed.  Errors:
 * E_INVAL, E_ENCODING (pk not a point). */
int poslo_audit_begin(poslo_ctx* ctx, const poslo_params* params, const uint8_t pk[32], const uint8_t* ds,
                      size_t ds_len, uint64_t t0, poslo_audit** out);
/* Add the next chunk: chunk->t0 must equal the audit's next entry.  Device
 * chunks are read by kernels queued on stream, so they must stay unchanged
 * until the stream has passed them.  Host chunks (chunk->host = 1; pinned
 * memory makes the copy asynchronous) are copied on the audit's own copy
 * stream into one of two staging buffers, so that a chunk's copy overlaps
 * the previous chunk's hashing; a host chunk must stay unchanged until the
 * next call on the audit returns.  Returns without waiting for the device.
 * E_SEED if the ds does not cover an epoch of the chunk.  POSLO++: a chunk
 * of fixed length above 31 bytes is E_INVAL here; a longer message in an
 * offsets chunk is found by the kernels and makes finish and export return
 * E_INVAL from then on. */
int poslo_audit_feed(poslo_audit* audit, const poslo_msgs* chunk, void* stream);
/* The next entry index (the first entry not yet fed). */
int poslo_audit_position(const poslo_audit* audit, uint64_t* t_next);
/* The check against the aggregate tag (host, 64 bytes) of entries t0 ..
 * t_next-1: *accept and, if e_out is set, e mod q (32 bytes).  Synchronous;
 * the audit stays usable (more chunks can follow for a later tag). */
int poslo_audit_finish(poslo_audit* audit, const uint8_t tag[64], void* stream, int* accept, uint8_t e_out[32]);
/* The running state as bytes: "PAUD", u32 version 1, u32 inst, log2_n1,
 * log2_n2, pk (32), u64 t0, u64 t_next, e mod q (32, LE), u32 ds length,
 * ds.  *len gets the size; E_INVAL when cap is too small.  Synchronizes
 * stream. */
int poslo_audit_export(poslo_audit* audit, void* stream, uint8_t* buf, size_t cap, size_t* len);
/* An audit continued from exported state; params must match it. */
int poslo_audit_resume(poslo_ctx* ctx, const uint8_t* state, size_t len, const poslo_params* params,
                       poslo_audit** out);
void poslo_audit_free(poslo_audit* audit);

/* ------------------------------------------------ measurement utilities */

/* Sustained issue rate of one 32-bit integer VALU instruction kind on the
 * device: waves_per_simd (1-8) waves of 64 lanes on every SIMD, each lane
 * running eight independent chains of iters * 16 instructions; the rate is
 * lane operations per second (a v_mad_u64_u32 counts as one).  This is the
 * measured ceiling beside the nominal 4 cycles per wave64 instruction that
 * roofline fractions are quoted against.  Synchronous. */
enum {
    POSLO_PROBE_XOR = 0,      /* v_xor_b32 */
    POSLO_PROBE_PERM = 1,     /* v_perm_b32 (T-table addresses, byte merges) */
    POSLO_PROBE_BITOP3 = 2,   /* v_bitop3_b32 (three-input xor) */
    POSLO_PROBE_ADD3 = 3,     /* v_add3_u32 (SHA-256 sums) */
    POSLO_PROBE_ALIGNBIT = 4, /* v_alignbit_b32 (rotations) */
    POSLO_PROBE_MAD64 = 5     /* v_mad_u64_u32 (field multiplication) */
};
int poslo_valu_probe(int device, int op, uint32_t waves_per_simd, uint32_t iters, double* lane_ops_per_s,
                     double* ms);

/* ------------------------------------------- synthetic data on the device */

/* Seeded message bytes generated on the device for benchmarks and tests:
 * entry p of the batch takes its bytes from xoshiro256** stream (seed, t0+p)
 * (splitmix64-seeded from (seed << 32) | (t0 + p)), little-endian, truncated
 * to its length; m->data is ignored, out (device) receives the bytes at the
 * layout m describes.  t0 + n must stay below 2^32. */
int poslo_synth_messages(uint32_t seed, const poslo_msgs* m, uint8_t* out, void* stream);

/* Keys held on the device for large-scale signing (test data): y, x_D[0]
 * and the public key derived on the host as poslo_kg does, the BPV table
 * derived on the device.  seeds: host, 32*nkeys; pks: host, 32*nkeys out.
 * bpv_k <= 16.  Freed with poslo_gpu_keys_free. */
typedef struct poslo_gpu_keys poslo_gpu_keys;
int poslo_gpu_keys_create(poslo_ctx* ctx, const poslo_params* params, const uint8_t* seeds, uint32_t nkeys,
                          poslo_gpu_keys** out, uint8_t* pks);
void poslo_gpu_keys_free(poslo_gpu_keys* keys);

/* One signing (or verification) job: entries t0 .. t0+n-1 of a signer whose
 * messages are entries entry_base .. entry_base+n-1 of a global batch. */
typedef struct poslo_sign_job {
    uint32_t key;
    uint32_t reserved;
    uint64_t t0;
    uint64_t n;
    uint64_t entry_base;
} poslo_sign_job;

/* Sign every job's entries as poslo_sig_batch would (same bytes).  With
 * n_total = max over jobs of entry_base + n: data (offsets[n_total] bytes),
 * offsets (n_total + 1 u64), sigs (80 per global entry): device.  tags
 * (64*njobs) and ds_out (ds_stride >= 769 bytes per job, may be NULL): host,
 * the aggregate tag of each job and the ds after its last entry.
 * Synchronous.  POSLO++: E_INVAL if a message is longer than 31 bytes (its
 * signature is left unwritten and the tags are not valid). */
int poslo_gpu_sign(poslo_gpu_keys* keys, const poslo_sign_job* jobs, uint32_t njobs, const uint8_t* data,
                   const uint64_t* offsets, uint8_t* sigs, uint8_t* tags, uint8_t* ds_out, size_t ds_stride,
                   void* stream);

/* ------------------------------------------------ many signers per launch */

/* Load public keys into the context's device-resident key cache (comb
 * tables built on the device, 384 KiB per key), so that later calls with
 * these keys start without a host-side table build.  pks: host, 32*n.
 * *n_bad (may be NULL) gets the number of keys that are not point
 * encodings; those are skipped and the call returns POSLO_E_ENCODING.
 * The cache holds at least the keys of the largest batch seen and evicts
 * the least recently used beyond that.  Synchronous. */
int poslo_ctx_keys_load(poslo_ctx* ctx, const uint8_t* pks, size_t n, size_t* n_bad);

/* Give resident edwards25519 keys a wide table as well: 16 windows of
 * 32,768 points m * 65536^w * Y (48 MiB per key, built on the device),
 * loading keys that are not yet in the cache.  The individual checks of a
 * key with a wide table (poslo_verify_batch with distill set, poslo_distill)
 * then add 16 points of it instead of 32 of its 8-bit table, besides 16 of
 * G's wide table; results do not change.  A widened key keeps its table
 * until the key leaves the cache or the context is destroyed.  pks: host,
 * 32*n.  E_ENCODING: some key is not a point encoding (the others are
 * widened); E_NOMEM: a table could not be allocated or built (the tables
 * built before it stay).  Synchronous. */
int poslo_ctx_keys_widen(poslo_ctx* ctx, const uint8_t* pks, size_t n);

/* One signer's batch inside a multi-signer verification: entries t0 ..
 * t0+n-1 of the signer with public key pk, whose messages are entries
 * entry_base .. entry_base+n-1 of the global (offsets) layout, with the
 * signer's ds after its last entry and its aggregate tag.  pk, ds and tag:
 * host.  Jobs may use the same key; their entry ranges must not overlap. */
typedef struct poslo_batch_job {
    const uint8_t* pk;
    const uint8_t* ds;
    size_t ds_len;
    const uint8_t* tag;
    uint64_t t0;
    uint64_t n;
    uint64_t entry_base;
} poslo_batch_job;

/* Launch parameters of the multi-signer path: variant (see
 * poslo_batch_variant_name: instantiation, LDS table copies, workgroup size,
 * entries per work item, length sort), workgroups per CU of the persistent
 * grid (0 = derived from LDS and wave budget), and whether to capture the
 * launch sequence in a hipGraph that is replayed for identical shapes. */
typedef struct poslo_tuning {
    int variant;
    int wg_per_cu;
    int use_graph;
    int reserved;
} poslo_tuning;

int poslo_batch_variant_count(void);
const char* poslo_batch_variant_name(int v);

/* AVer of every job in one persistent launch (section "POSLO Parallel Batch
 * Verification", extended to many signers: per-epoch seeds of all jobs, one
 * persistent hashing kernel that pulls fixed-size work items of any job from
 * a queue, then one aggregate check per job).  data (device, data_bytes
 * bytes or 0 if unknown) and offsets (device, u64, covering every job's
 * entries) hold the messages.  accept: host, njobs bytes.  tuning may be
 * NULL: the autotuner's choice for this shape class if one was made, else
 * the default.
 * distill: 0 = AVer only (sigs, invalid and n_invalid unused); 1 = the
 * entries of rejected jobs are verified individually (Distill's check);
 * 2 = the entries of every job are (AVer reads only messages, ds and tag,
 * so a corrupted signature in an accepted job is found by mode 2 only).
 * With distill set, the hashing kernel also keeps every entry's e_t and x
 * check for the individual checks, which then do only the curve part.
 * sigs: device, 80 bytes per global entry.  The invalid entries are
 * returned as sorted (job, t) pairs in invalid (host, 2*cap u64);
 * *n_invalid gets the count even when it exceeds cap (the pairs are then
 * not written).  Accept bits equal poslo_aver per job; the pairs of a job
 * equal poslo_distill's invalid list for it.  Errors: E_INVAL (bad job or
 * argument), E_SEED (a ds does not cover an epoch), E_ENCODING (a pk is not
 * a point).  Synchronous. */
int poslo_verify_batch(poslo_ctx* ctx, const poslo_params* params, const poslo_batch_job* jobs, uint32_t njobs,
                       const uint8_t* data, const uint64_t* offsets, uint64_t data_bytes, const uint8_t* sigs,
                       int distill, const poslo_tuning* tuning, void* stream, uint8_t* accept, uint64_t* invalid,
                       size_t cap, size_t* n_invalid);

/* Time every applicable variant and grid size on this batch (reps timed
 * runs each, after one untimed run whose verdicts must match the first
 * candidate's), cache the fastest for the batch's shape class (instantiation,
 * log2 mean message length, log2 entry count) and return it.  E_DEVICE if
 * two candidates disagree on a verdict. */
int poslo_autotune_batch(poslo_ctx* ctx, const poslo_params* params, const poslo_batch_job* jobs, uint32_t njobs,
                         const uint8_t* data, const uint64_t* offsets, uint64_t data_bytes, int reps, void* stream,
                         poslo_tuning* best, double* best_ms);

/* Drop the context's captured graphs and tuning cache. */
int poslo_batch_forget(poslo_ctx* ctx);

/* ------------------------------------------------------------ serving loop */

/* A verification server: requests (one signer's batch each) are submitted
 * from any thread as they arrive and verified by a worker thread that
 * admits them while device memory and launch slots allow, groups the
 * admitted requests into multi-signer launches and keeps several launches
 * in flight on separate streams (a request that arrives while others are on
 * the GPU joins the next group).  Public keys stay resident on the device
 * (comb tables) with a per-key aggregate state: the sum of the tags of the
 * key's accepted requests and the number of entries they covered.  A
 * request's result does not depend on what it was grouped with. */
typedef struct poslo_server poslo_server;

typedef struct poslo_server_cfg {
    poslo_params params;
    uint32_t n_streams;   /* launch groups in flight (0: 4) */
    uint32_t max_group;   /* requests per launch group (0: 256) */
    uint64_t mem_bytes;   /* device budget for admitted requests: staging copies of host
                             buffers and per-request scratch (0: 8 GiB) */
    int distill;          /* 0: accept bit only; 1: invalid entries of rejected requests;
                             2: invalid entries of every request */
    int variant;          /* hot-kernel variant (-1: the default of the instantiation) */
    uint64_t max_group_entries; /* entries per launch group (0: 2^21); a group always takes at
                                   least one request.  Smaller groups cut the time a request
                                   waits for its group's slowest member; larger ones batch more */
} poslo_server_cfg;

typedef struct poslo_request {
    uint32_t key_id;      /* a registered key */
    uint32_t on_device;   /* 1: data, offsets and sigs are device pointers; 0: host pointers,
                             copied to the device when the request is launched.  Either way
                             they stay valid and unchanged until the result is polled. */
    uint64_t t0, n;       /* entries t0 .. t0+n-1 */
    const uint8_t* data;
    const uint64_t* offsets;  /* n + 1 offsets into data, or NULL: fixed msg_len */
    uint64_t msg_len;
    uint64_t data_bytes;      /* bytes of data (0: offsets[n], or n * msg_len) */
    const uint8_t* sigs;      /* 80 per entry, or NULL when the server does not distill */
    const uint8_t* ds;        /* host, copied at submit */
    size_t ds_len;
    const uint8_t* tag;       /* host, 64 bytes, copied at submit */
    uint64_t user;            /* returned with the result */
} poslo_request;

typedef struct poslo_result {
    uint64_t ticket;
    uint64_t user;
    int status;           /* POSLO_OK, or the error this request failed with */
    int accept;
    uint64_t n_invalid;   /* invalid entries found (poslo_server_take_invalid) */
    uint64_t entries;
    double t_submit_ms;   /* times since the server was created */
    double t_admit_ms;
    double t_launch_ms;
    double t_done_ms;
} poslo_result;

typedef struct poslo_server_stats {
    uint64_t submitted, completed, queued, in_flight;
    uint64_t entries_completed, groups_launched;
    uint64_t bytes_in_use, bytes_peak;
    double latency_p50_ms, latency_p99_ms; /* submit to done, over completed requests */
    double elapsed_ms;                     /* since the server was created */
} poslo_server_stats;

/* device: HIP device index.  E_INVAL on a bad configuration. */
int poslo_server_create(int device, const poslo_server_cfg* cfg, poslo_server** out);
/* Register n keys (ids and 32-byte encodings, host).  E_ENCODING if one is
 * not a point (none is registered then).  An id registered again is
 * replaced, with a fresh aggregate state, but only while none of its
 * requests is queued or in flight (E_BUSY otherwise, and nothing is
 * registered).  Synchronous.  E_BUSY also when the key-state array must
 * grow while requests are queued or in flight: register keys before
 * serving. */
int poslo_server_register_keys(poslo_server* srv, const uint32_t* ids, const uint8_t* pks, size_t n);
/* Queue a request; never waits for the device.  *ticket identifies its
 * result.  The request's own inputs are checked here: E_INVAL for an
 * unknown key, inconsistent sizes or a malformed ds, E_SEED when the ds
 * does not cover one of its epochs. */
int poslo_server_submit(poslo_server* srv, const poslo_request* req, uint64_t* ticket);
/* Move up to cap finished results to out (in completion order); *n gets
 * the count.  timeout_ms > 0 waits that long for at least one. */
int poslo_server_poll(poslo_server* srv, poslo_result* out, size_t cap, size_t* n, double timeout_ms);
/* The sorted invalid entry indices t of a polled result; the list is
 * released by this call.  E_INVAL if the ticket has none pending. */
int poslo_server_take_invalid(poslo_server* srv, uint64_t ticket, uint64_t* out, size_t cap, size_t* n);
/* The key's device-resident aggregate state: the tag sum of its accepted
 * requests (64 bytes, the Agg format) and the entries they covered. */
int poslo_server_key_state(poslo_server* srv, uint32_t key_id, uint8_t tag[64], uint64_t* entries);
int poslo_server_stats_get(poslo_server* srv, poslo_server_stats* out);
/* Waits for every submitted request to finish, then frees the server. */
void poslo_server_destroy(poslo_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* POSLO_H */
