"""Oracle results over full-size batches, computed on the host cores.

Test infrastructure.  Everything here comes from ``oracle`` and ``synthlog``
alone: the messages are synthlog's, the keys, signatures, ds and tags are the
oracle signer's, and every expected value is an oracle function applied to
them.  Nothing is read back from the GPU library.

The batch is cut into umbrella-sized chunks (umbrella l covers batch
positions [l*U, min(N, (l+1)*U)), U = ceil(N / n_u)), and a process pool runs
the oracle on the chunks side by side.  Each chunk starts from the signer
state after the entries before it (``oracle.signer_at``), so the chunks'
signatures are the sequential signer's.  The per-batch results combine by
the plain sums that define them: e = (sum of the raw digests) mod q, and
Agg is a sum over its records, so the aggregate of a batch is Agg over the
aggregates of its parts.  ``test_oracle_fullsize.py`` checks the pooled
results against the sequential oracle (sign_batch, aver, distill) on a small
batch.

Per chunk the workers produce:
  * the honest signatures, per-entry raw digests H(m_t || x_t) reduced mod q
    and one-time seeds x_t (x_t re-derived from the final ds by SR, as AVer
    does);
  * after the corruption plan is applied (one flipped bit of m_t || sigma_t
    per planned entry): the individual verdict of every planned entry, the
    individual verdict of two unplanned entries (a sample: unplanned entries
    carry the honest signature, which the oracle's pins show valid), the
    umbrella's Agg over its valid entries, and the raw digest sum of the
    corrupted messages.
"""

from __future__ import annotations

import functools
import multiprocessing as mp
import os
import random
from dataclasses import dataclass, field

import numpy as np

import synthlog

# the box gives one GPU process a share of 16 host cores
MAX_WORKERS = 16


def workers() -> int:
    return max(1, min(MAX_WORKERS, os.cpu_count() or 1))


@dataclass
class FullCase:
    inst: int
    log2_n1: int
    log2_n2: int
    n: int
    L: int
    key_first: int
    msg_seed: int
    n_u: int
    pk: bytes
    ds: bytes
    tag: bytes                      # Agg over all honest signatures
    msgs: np.ndarray                # (n, L) honest messages
    sigs: np.ndarray                # (n, 80) honest signatures
    e_t: np.ndarray                 # (n, 32) H(m_t || x_t) mod q, little-endian
    x_t: np.ndarray                 # (n, 16)
    e: int                          # sum of e_t mod q (AVer's aggregate key)
    plan: list = field(default_factory=list)   # (entry, bit) flips
    cmsgs: np.ndarray | None = None            # corrupted copies
    csigs: np.ndarray | None = None
    invalid: list = field(default_factory=list)  # entries the oracle finds invalid
    span: int = 0
    umbrellas: list = field(default_factory=list)  # Agg over each umbrella's valid entries
    valid_tag: bytes = b""                         # Agg over all valid entries
    e_corrupt: int = 0                             # AVer's aggregate key of the corrupted batch
    aver_corrupt: bool = True                      # AVer of the corrupted batch under the honest tag
    aver_honest: bool = True                       # AVer of the honest batch



def _bpv_part(args):
    from oracle import oracle as O
    inst, log2_n1, log2_n2, seed, ks = args
    prm = O.Params(inst, log2_n1, log2_n2)
    signer, _ = O.kg(prm, seed)
    return {k: signer.bpv_pair(k) for k in ks}


def _chunk(args):
    from oracle import oracle as O
    (inst, log2_n1, log2_n2, seed, ds, msg_seed, L, a, b, plan, gamma) = args
    prm = O.Params(inst, log2_n1, log2_n2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, b - a, L, t0=a)]
    signer = O.signer_at(prm, seed, a)
    signer._gamma = gamma
    pk = O.encode(O.scalar_mult(signer.y, O.G))
    sigs = [O.sig(signer, m) for m in msgs]
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), a, b - a)
    e_t, x_t, raw = [], [], 0
    for p, m in enumerate(msgs):
        t = a + p
        x = O.one_time_seed(inst, seeds[t >> log2_n2], t & (prm.n2 - 1))
        d = O.digest_int(inst, m, x)
        raw += d
        e_t.append(O.to32(d % O.Q))
        x_t.append(x)
    # the corruption plan, then the verdicts the oracle gives on the result
    cm, cs = list(msgs), list(sigs)
    flipped = {}
    for e, bit in plan:
        p = e - a
        blob = bytearray(msgs[p] + sigs[p])
        blob[bit // 8] ^= 1 << (bit % 8)
        cm[p], cs[p] = bytes(blob[:L]), bytes(blob[L:])
        flipped[p] = True
    bad = []
    for p in sorted(flipped):
        t = a + p
        if not O.entry_valid(prm, pk, cm[p], t, cs[p], seeds[t >> log2_n2]):
            bad.append(t)
    rng = random.Random(a)
    unplanned = [p for p in range(b - a) if p not in flipped]
    sample_bad = []
    for p in rng.sample(unplanned, min(2, len(unplanned))):
        t = a + p
        if not O.entry_valid(prm, pk, cm[p], t, cs[p], seeds[t >> log2_n2]):
            sample_bad.append(t)
    bad_set = set(bad)
    valid_tag = O.agg([cs[p] for p in range(b - a) if a + p not in bad_set])
    raw_c = 0
    for p in flipped:
        t = a + p
        x = O.one_time_seed(inst, seeds[t >> log2_n2], t & (prm.n2 - 1))
        raw_c += O.digest_int(inst, cm[p], x) - O.digest_int(inst, msgs[p], x)
    return dict(a=a, b=b, sigs=b"".join(sigs), e_t=b"".join(e_t), x_t=b"".join(x_t), raw=raw,
                raw_c=raw + raw_c, bad=bad, sample_bad=sample_bad, valid_tag=valid_tag,
                bad_sigs=[sigs[t - a] for t in bad], cm={a + p: cm[p] for p in flipped},
                cs={a + p: cs[p] for p in flipped})


def _pool(n):
    return mp.get_context("spawn").Pool(n)


@functools.lru_cache(maxsize=None)
def full_case(inst: int, n: int, L: int, log2_n1: int, log2_n2: int, key_first: int, msg_seed: int,
              n_u: int, flip_seed: int, k_flips: int, nproc: int | None = None) -> FullCase:
    """Oracle-signed batch of n entries of L-byte messages (synthlog seed
    msg_seed, key seed bytes key_first..key_first+31) with its oracle
    results, and the same batch with k_flips entries corrupted
    (synthlog.corruption_plan with flip_seed over the 8 (L + 80) bits of
    m_t || sigma_t), distilled into n_u umbrellas."""
    from oracle import oracle as O
    prm = O.Params(inst, log2_n1, log2_n2)
    seed = synthlog.key_seed_bytes(key_first)
    signer = O.signer_at(prm, seed, n)
    ds = O.ds_encode(signer.ds)
    pk = O.encode(O.scalar_mult(signer.y, O.G))
    span = max(1, -(-n // n_u))
    plan = synthlog.corruption_plan(flip_seed, n, k_flips, 8 * (L + 80)) if k_flips else []
    nproc = nproc or workers()
    with _pool(nproc) as pool:
        ks = list(range(prm.v))
        parts = pool.map(_bpv_part, [(inst, log2_n1, log2_n2, seed, ks[i::nproc]) for i in range(nproc)])
        gamma = {}
        for p in parts:
            gamma.update(p)
        jobs = []
        for a in range(0, n, span):
            b = min(n, a + span)
            jobs.append((inst, log2_n1, log2_n2, seed, ds, msg_seed, L, a, b,
                         [(e, bit) for e, bit in plan if a <= e < b], gamma))
        res = pool.map(_chunk, jobs, chunksize=1)
    msgs = synthlog.messages_fixed(msg_seed, n, L)
    sigs = np.frombuffer(b"".join(r["sigs"] for r in res), dtype=np.uint8).reshape(n, 80)
    e_t = np.frombuffer(b"".join(r["e_t"] for r in res), dtype=np.uint8).reshape(n, 32)
    x_t = np.frombuffer(b"".join(r["x_t"] for r in res), dtype=np.uint8).reshape(n, 16)
    raw = sum(r["raw"] for r in res)
    raw_c = sum(r["raw_c"] for r in res)
    invalid = sorted(t for r in res for t in r["bad"])
    sample_bad = [t for r in res for t in r["sample_bad"]]
    if sample_bad:
        raise AssertionError(f"honest entries the oracle rejects: {sample_bad[:8]}")
    umbrellas = [r["valid_tag"] for r in res]
    # Agg over a batch is Agg over the aggregates of its parts
    valid_tag = O.agg(umbrellas)
    tag = O.agg(umbrellas + [s for r in res for s in r["bad_sigs"]])
    cmsgs, csigs = msgs.copy(), sigs.copy()
    for r in res:
        for t, m in r["cm"].items():
            cmsgs[t] = np.frombuffer(m, dtype=np.uint8)
        for t, s in r["cs"].items():
            csigs[t] = np.frombuffer(s, dtype=np.uint8)
    e = raw % O.Q
    e_c = raw_c % O.Q
    return FullCase(inst=inst, log2_n1=log2_n1, log2_n2=log2_n2, n=n, L=L, key_first=key_first,
                    msg_seed=msg_seed, n_u=n_u, pk=pk, ds=ds, tag=tag, msgs=msgs, sigs=sigs, e_t=e_t,
                    x_t=x_t, e=e, plan=plan, cmsgs=cmsgs, csigs=csigs, invalid=invalid, span=span,
                    umbrellas=umbrellas, valid_tag=valid_tag, e_corrupt=e_c,
                    aver_corrupt=O.aggregate_check(pk, e_c, tag), aver_honest=O.aggregate_check(pk, e, tag))


# ---------------------------------------------------------------------------
# one signer's job of a multi-signer log (variable-length messages)
# ---------------------------------------------------------------------------

@dataclass
class JobCase:
    n: int
    pk: bytes
    ds: bytes
    tag: bytes                      # Agg over the job's honest signatures
    sigs: bytes                     # honest signatures, 80 bytes each
    invalid: list                   # job-local t the oracle finds invalid after the plan
    aver_corrupt: bool              # AVer of the corrupted job under the honest tag


def _job_chunk(args):
    from oracle import oracle as O
    (inst, log2_n1, log2_n2, seed, ds, msg_seed, lens, base, a, b, plan, gamma) = args
    prm = O.Params(inst, log2_n1, log2_n2)
    data, off = synthlog.messages_var(msg_seed, np.asarray(lens[a:b], dtype=np.int64), t0=base + a)
    msgs = [bytes(data[int(off[i]):int(off[i + 1])]) for i in range(b - a)]
    signer = O.signer_at(prm, seed, a)
    signer._gamma = gamma
    pk = O.encode(O.scalar_mult(signer.y, O.G))
    sigs = [O.sig(signer, m) for m in msgs]
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), a, b - a)
    xs = [O.one_time_seed(inst, seeds[t >> log2_n2], t & (prm.n2 - 1)) for t in range(a, b)]
    raw = sum(O.digest_int(inst, m, x) for m, x in zip(msgs, xs))
    cm, cs = list(msgs), list(sigs)
    for t, bit in plan:
        p = t - a
        blob = bytearray(cm[p] + cs[p])
        blob[bit // 8] ^= 1 << (bit % 8)
        L = len(msgs[p])
        cm[p], cs[p] = bytes(blob[:L]), bytes(blob[L:])
    flipped = sorted({t - a for t, _ in plan})
    bad = [a + p for p in flipped
           if not O.entry_valid(prm, pk, cm[p], a + p, cs[p], seeds[(a + p) >> log2_n2])]
    raw_c = raw + sum(O.digest_int(inst, cm[p], xs[p]) - O.digest_int(inst, msgs[p], xs[p]) for p in flipped)
    rng = random.Random(base + a)
    fl = set(flipped)
    unplanned = [p for p in range(b - a) if p not in fl]
    sample_bad = [a + p for p in rng.sample(unplanned, min(2, len(unplanned)))
                  if not O.entry_valid(prm, pk, cm[p], a + p, cs[p], seeds[(a + p) >> log2_n2])]
    return dict(sigs=b"".join(sigs), tag=O.agg(sigs), raw=raw, raw_c=raw_c, bad=bad, sample_bad=sample_bad)


@functools.lru_cache(maxsize=None)
def job_case(inst: int, log2_n1: int, log2_n2: int, key_seed: bytes, msg_seed: int, lens: tuple, base: int,
             plan: tuple, nproc: int | None = None) -> JobCase:
    """A signer (key seed bytes key_seed) whose entries t = 0 .. n-1 are the
    multi-signer log's global entries base + t: messages of lens[t] bytes
    from synthlog stream msg_seed at sid base + t, signed by the oracle from
    t = 0.  plan: job-local (t, bit) flips of m_t || sigma_t.  Returns the
    honest signatures and tag and the oracle's results on the corrupted
    job."""
    from oracle import oracle as O
    prm = O.Params(inst, log2_n1, log2_n2)
    n = len(lens)
    signer = O.signer_at(prm, key_seed, n)
    ds = O.ds_encode(signer.ds)
    pk = O.encode(O.scalar_mult(signer.y, O.G))
    nproc = nproc or workers()
    span = max(1, -(-n // (2 * nproc)))
    with _pool(nproc) as pool:
        ks = list(range(prm.v))
        parts = pool.map(_bpv_part, [(inst, log2_n1, log2_n2, key_seed, ks[i::nproc]) for i in range(nproc)])
        gamma = {}
        for part in parts:
            gamma.update(part)
        jobs = [(inst, log2_n1, log2_n2, key_seed, ds, msg_seed, lens, base, a, min(n, a + span),
                 [(t, bit) for t, bit in plan if a <= t < min(n, a + span)], gamma) for a in range(0, n, span)]
        res = pool.map(_job_chunk, jobs, chunksize=1)
    sample_bad = [t for r in res for t in r["sample_bad"]]
    if sample_bad:
        raise AssertionError(f"honest entries the oracle rejects: {sample_bad[:8]}")
    tag = O.agg([r["tag"] for r in res]) if res else O.agg([])
    e_c = sum(r["raw_c"] for r in res) % O.Q
    return JobCase(n=n, pk=pk, ds=ds, tag=tag, sigs=b"".join(r["sigs"] for r in res),
                   invalid=sorted(t for r in res for t in r["bad"]),
                   aver_corrupt=O.aggregate_check(pk, e_c, tag))


# ---------------------------------------------------------------------------
# POSLO-C: one signature per epoch
# ---------------------------------------------------------------------------

@dataclass
class FullCaseC:
    inst: int
    log2_n1: int
    log2_n2: int
    n: int
    L: int
    n_u: int
    pk: bytes
    ds: bytes
    msgs: np.ndarray                # (n, L) honest messages
    s_epochs: bytes                 # 32 bytes per epoch, honest
    s_total: bytes                  # Agg of every epoch's signature
    e: int                          # e~ of the honest batch
    aver_honest: bool
    plan: list = field(default_factory=list)      # (epoch, bit) over m_i || s~_i
    cmsgs: np.ndarray | None = None
    cs_epochs: bytes = b""
    invalid: list = field(default_factory=list)   # epochs the oracle finds invalid
    span: int = 0
    umbrellas: list = field(default_factory=list)
    valid_tag: bytes = b""
    e_corrupt: int = 0
    aver_corrupt: bool = True


def _c_commitments(args):
    from oracle import oracle as O
    inst, log2_n1, log2_n2, r, epochs = args
    prm = O.Params(inst, log2_n1, log2_n2)
    return [O.posloc_commitment(prm, r, i) for i in epochs]


def _c_chunk(args):
    from oracle import oracle as O
    (inst, log2_n1, log2_n2, seed, pk, ds, msg_seed, L, a, b, plan) = args
    prm = O.Params(inst, log2_n1, log2_n2)
    n2 = prm.n2
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, (b - a) * n2, L, t0=a * n2)]
    signer = O.posloc_signer_at(prm, seed, a)
    s_list = [O.posloc_sig(signer, msgs[p * n2:(p + 1) * n2])[0] for p in range(b - a)]
    dsn = O.ds_decode(ds)
    raw = 0
    for p in range(b - a):
        x0 = O.SR(inst, dsn, a + p)
        for j in range(n2):
            raw += O.digest_int(inst, msgs[p * n2 + j], O.one_time_seed(inst, x0, j))
    cm, cs = list(msgs), list(s_list)
    raw_c = raw
    flipped_m = {}
    for i, bit in plan:
        p = i - a
        blob = bytearray(b"".join(msgs[p * n2:(p + 1) * n2]) + s_list[p])
        blob[bit // 8] ^= 1 << (bit % 8)
        x0 = O.SR(inst, dsn, i)
        for j in range(n2):
            m_new = bytes(blob[j * L:(j + 1) * L])
            if m_new != msgs[p * n2 + j]:
                x = O.one_time_seed(inst, x0, j)
                raw_c += O.digest_int(inst, m_new, x) - O.digest_int(inst, msgs[p * n2 + j], x)
                cm[p * n2 + j] = m_new
                flipped_m[a * n2 + p * n2 + j] = m_new
        cs[p] = bytes(blob[n2 * L:])
    ccd = O.posloc_distill(prm, pk, cm, cs, a, ds, 1)
    return dict(a=a, b=b, s=b"".join(s_list), cs=b"".join(cs), raw=raw, raw_c=raw_c,
                bad=[i for i, _ in ccd.invalid], umb=ccd.umbrellas[0][0], cm=flipped_m)


@functools.lru_cache(maxsize=None)
def full_case_c(inst: int, n: int, L: int, log2_n1: int, log2_n2: int, key_first: int, msg_seed: int,
                n_u: int, flip_seed: int, k_flips: int, nproc: int | None = None) -> FullCaseC:
    """Oracle-signed POSLO-C batch of n entries (whole epochs) with its
    oracle results, and the same batch with k_flips epochs corrupted by one
    flipped bit uniform over the epoch's message bytes and its signature
    (synthlog.corruption_plan over epochs), distilled into n_u umbrellas of
    epochs."""
    from oracle import oracle as O
    prm = O.Params(inst, log2_n1, log2_n2)
    seed = synthlog.key_seed_bytes(key_first)
    k = n // prm.n2
    if k * prm.n2 != n:
        raise ValueError("whole epochs only")
    st0 = O.posloc_signer_at(prm, seed, 0)
    Yb = O.encode(O.scalar_mult(st0.y, O.G))
    ds = O.ds_encode(O.posloc_signer_at(prm, seed, k).ds)
    span = max(1, -(-k // n_u))
    plan = synthlog.corruption_plan(flip_seed, k, k_flips, 8 * (prm.n2 * L + 32)) if k_flips else []
    nproc = nproc or workers()
    with _pool(nproc) as pool:
        eps = list(range(prm.n1))
        parts = pool.map(_c_commitments, [(inst, log2_n1, log2_n2, st0.r, eps[i::nproc]) for i in range(nproc)])
        com = [None] * prm.n1
        for i in range(nproc):
            for e, c in zip(eps[i::nproc], parts[i]):
                com[e] = c
        pk = Yb + b"".join(com)
        jobs = [(inst, log2_n1, log2_n2, seed, pk, ds, msg_seed, L, a, min(k, a + span),
                 [(e, bit) for e, bit in plan if a <= e < min(k, a + span)]) for a in range(0, k, span)]
        res = pool.map(_c_chunk, jobs, chunksize=1)
    msgs = synthlog.messages_fixed(msg_seed, n, L)
    s_epochs = b"".join(r["s"] for r in res)
    cs_epochs = b"".join(r["cs"] for r in res)
    cmsgs = msgs.copy()
    for r in res:
        for t, m in r["cm"].items():
            cmsgs[t] = np.frombuffer(m, dtype=np.uint8)
    e = sum(r["raw"] for r in res) % O.Q
    e_c = sum(r["raw_c"] for r in res) % O.Q
    s_total = O.posloc_agg_s([s_epochs[32 * i:32 * i + 32] for i in range(k)])
    R = O.IDENTITY
    for i in range(k):
        R = O.point_add(R, O.decode(com[i]))
    R_tag = O.encode(R)
    umbrellas = [r["umb"] for r in res]
    return FullCaseC(inst=inst, log2_n1=log2_n1, log2_n2=log2_n2, n=n, L=L, n_u=n_u, pk=pk, ds=ds, msgs=msgs,
                     s_epochs=s_epochs, s_total=s_total, e=e,
                     aver_honest=O.aggregate_check(Yb, e, s_total + R_tag), plan=plan, cmsgs=cmsgs,
                     cs_epochs=cs_epochs, invalid=sorted(i for r in res for i in r["bad"]), span=span,
                     umbrellas=umbrellas, valid_tag=O.agg(umbrellas), e_corrupt=e_c,
                     aver_corrupt=O.aggregate_check(
                         Yb, e_c, O.posloc_agg_s([cs_epochs[32 * i:32 * i + 32] for i in range(k)]) + R_tag))
