"""Seeded synthetic workloads built on the device through the C ABI.

Messages come from the device generator (same bytes as ``synthlog``),
signatures, tags and ds from the device signer (same bytes as the host
signer), corruption positions from ``synthlog``'s seeded plans.  Used by the
benchmark and the large GPU tests; nothing here verifies anything.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import synthlog

from . import BatchJobs, make_params, poslo_gpu_keys_create, poslo_gpu_sign, poslo_msgs, poslo_synth_messages


@dataclass
class MultiSignerLog:
    params: object
    counts: list[int]               # entries per signer
    lengths: np.ndarray             # message length per global entry
    offsets: np.ndarray             # uint64, total + 1
    data: object                    # CUDA uint8 tensor (message bytes)
    d_offsets: object               # CUDA int64 tensor
    sigs: object                    # CUDA uint8 tensor, 80 per entry
    pks: list[bytes]
    jobs: list[dict]                # pk, ds, tag, t0, n, entry_base, key
    plan: list[tuple[int, int]] = field(default_factory=list)  # (entry, bit) flips applied

    @property
    def total(self) -> int:
        return int(self.offsets.size - 1)

    def batch_jobs(self) -> BatchJobs:
        return BatchJobs(self.jobs)

    def job_of_entry(self, e: int) -> int:
        return int(np.searchsorted(self.bases, e, side="right") - 1)

    @property
    def bases(self) -> np.ndarray:
        return np.array([j["entry_base"] for j in self.jobs], dtype=np.int64)


def _flip(torch, log: MultiSignerLog, plan):
    """Flip one bit of m_t || sigma_t per planned entry, on the device."""
    if not plan:
        return
    msg_idx, msg_mask, sig_idx, sig_mask = [], [], [], []
    for e, bit in plan:
        L = int(log.lengths[e])
        if bit < 8 * L:
            msg_idx.append(int(log.offsets[e]) + bit // 8)
            msg_mask.append(1 << (bit % 8))
        else:
            b = bit - 8 * L
            sig_idx.append(80 * e + b // 8)
            sig_mask.append(1 << (b % 8))
    dev = log.data.device
    for buf, idx, mask in ((log.data, msg_idx, msg_mask), (log.sigs, sig_idx, sig_mask)):
        if idx:
            it = torch.tensor(idx, dtype=torch.int64, device=dev)
            mt = torch.tensor(mask, dtype=torch.uint8, device=dev)
            buf[it] = buf[it] ^ mt


def multi_signer(ctx, inst: int, n_signers: int, max_batch: int, len_lo: int, len_hi: int,
                 corrupt_frac: float, seed: int, log2_n1: int = 8, log2_n2: int = 8,
                 counts: list[int] | None = None) -> MultiSignerLog:
    """n_signers fresh signers, signer k with a log-uniform [1, max_batch]
    entry count (or counts[k]), messages of uniform [len_lo, len_hi] bytes,
    each signer's batch signed from t = 0 and aggregated into one tag; then
    round(corrupt_frac * total) distinct entries get one flipped bit,
    uniform over the 8 (L + 80) bits of m_t || sigma_t."""
    import torch

    params = make_params(inst, log2_n1, log2_n2)
    if counts is None:
        counts = synthlog.log_uniform_counts(seed, 0, n_signers, max_batch)
    counts = [int(c) for c in counts]
    total = sum(counts)
    lengths = synthlog.uniform_per_stream(seed + 1, np.arange(total), len_lo, len_hi)
    offsets = np.zeros(total + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    nbytes = int(offsets[-1])
    dev = torch.device("cuda", ctx.device)
    d_off = torch.from_numpy(offsets.view(np.int64)).to(dev)
    data = torch.empty(max(1, nbytes), dtype=torch.uint8, device=dev)
    poslo_synth_messages(seed + 2, poslo_msgs(data.data_ptr(), d_off.data_ptr(), 0, total, 0, nbytes), data)
    seeds = [synthlog.derived_key_seed(seed + 3, k) for k in range(n_signers)]
    keys = poslo_gpu_keys_create(ctx, params, seeds)
    bases = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64) if counts else np.zeros(0, np.int64)
    sjobs = [(k, 0, counts[k], int(bases[k])) for k in range(n_signers)]
    sigs = torch.empty(max(1, 80 * total), dtype=torch.uint8, device=dev)
    tags, ds = poslo_gpu_sign(keys, sjobs, data[:nbytes], d_off, sigs)
    jobs = [dict(key=k, pk=keys.pks[k], ds=ds[k], tag=tags[k], t0=0, n=counts[k], entry_base=int(bases[k]))
            for k in range(n_signers)]
    del keys
    log = MultiSignerLog(params=params, counts=counts, lengths=lengths, offsets=offsets, data=data[:nbytes],
                         d_offsets=d_off, sigs=sigs[:80 * total], pks=[j["pk"] for j in jobs], jobs=jobs)
    k = int(round(corrupt_frac * total))
    if k:
        bits = 8 * (lengths.astype(np.int64) + 80)
        log.plan = synthlog.corruption_plan_var(seed + 4, total, k, bits)
        _flip(torch, log, log.plan)
    torch.cuda.synchronize(dev)
    return log


@dataclass
class SingleSignerLog:
    params: object
    data: object        # CUDA uint8 tensor (n, L)
    sigs: object        # CUDA uint8 tensor (80 n)
    pk: bytes
    ds: bytes
    tag: bytes
    plan: list[tuple[int, int]] = field(default_factory=list)


def single_signer_fixed(ctx, inst: int, n: int, L: int, log2_n1: int, log2_n2: int, seed: int,
                        corrupt_frac: float = 0.0) -> SingleSignerLog:
    """One fresh signer, n entries of L-byte messages from stream seed, all
    signed from t = 0 into one tag; optionally round(corrupt_frac * n)
    entries with one flipped bit of m_t || sigma_t (the tag stays the honest
    one)."""
    import torch

    params = make_params(inst, log2_n1, log2_n2)
    dev = torch.device("cuda", ctx.device)
    data = torch.empty((n, L), dtype=torch.uint8, device=dev)
    poslo_synth_messages(seed, poslo_msgs(data.data_ptr(), None, L, n, 0, n * L), data)
    offs = torch.arange(0, (n + 1) * L, L, dtype=torch.int64, device=dev)
    keys = poslo_gpu_keys_create(ctx, params, [synthlog.derived_key_seed(seed + 3, 0)])
    sigs = torch.empty(80 * n, dtype=torch.uint8, device=dev)
    tags, ds = poslo_gpu_sign(keys, [(0, 0, n, 0)], data, offs, sigs)
    log = SingleSignerLog(params=params, data=data, sigs=sigs, pk=keys.pks[0], ds=ds[0], tag=tags[0])
    del keys
    k = int(round(corrupt_frac * n))
    if k:
        log.plan = synthlog.corruption_plan(seed + 4, n, k, 8 * (L + 80))
        flat = data.view(-1)
        view = MultiSignerLog(params=params, counts=[n], lengths=np.full(n, L), offsets=np.arange(n + 1) * L,
                              data=flat, d_offsets=offs, sigs=sigs, pks=[log.pk], jobs=[])
        _flip(torch, view, log.plan)
    torch.cuda.synchronize(dev)
    return log


@dataclass
class ServingLog:
    params: object
    L: int
    data: object          # CUDA uint8 tensor (total, L)
    sigs: object          # CUDA uint8 tensor (80 total)
    pks: list[bytes]      # by key id
    requests: list[dict]  # key, t0, n, base, ds, tag, flip: (entry in request, bit) or None

    def expected(self, r: int, distill: int):
        """(accept, invalid t list) the flips fix for request r."""
        q = self.requests[r]
        if q["flip"] is None:
            return True, []
        e, bit = q["flip"]
        msg = bit < 8 * self.L
        inv = [q["t0"] + e] if (distill == 2 or msg) else []
        return not msg, inv


def serving_requests(ctx, inst: int, n_keys: int, n_requests: int, max_batch: int, L: int, p_corrupt: float,
                     seed: int, log2_n1: int = 12, log2_n2: int = 8) -> ServingLog:
    """n_requests requests over n_keys signers: request r is for key
    uniform in [0, n_keys), with a log-uniform [1, max_batch] entry count,
    continuing that key's log (t0 = the entries its earlier requests
    covered); L-byte messages; with probability p_corrupt a request gets one
    flipped bit in one uniform entry, uniform over the 8 (L + 80) bits of
    m_t || sigma_t (its tag stays the honest one)."""
    import torch

    params = make_params(inst, log2_n1, log2_n2)
    keys_of = synthlog.uniform_ints(seed, 0, n_requests, 0, n_keys - 1)
    counts = synthlog.log_uniform_counts(seed, 1, n_requests, max_batch)
    g = synthlog.Xoshiro256ss(synthlog.stream_seed(seed, 2))
    next_t = [0] * n_keys
    reqs, base = [], 0
    cap = 1 << (log2_n1 + log2_n2)
    for r in range(n_requests):
        k, n = keys_of[r], counts[r]
        if next_t[k] + n > cap:
            raise ValueError("a key's log outgrew its parameter set")
        flip = None
        if g.uniform01() < p_corrupt:
            flip = (g.below(n), g.below(8 * (L + 80)))
        reqs.append(dict(key=k, t0=next_t[k], n=n, base=base, flip=flip))
        next_t[k] += n
        base += n
    total = base
    dev = torch.device("cuda", ctx.device)
    data = torch.empty((max(1, total), L), dtype=torch.uint8, device=dev)
    poslo_synth_messages(seed + 1, poslo_msgs(data.data_ptr(), None, L, total, 0, total * L), data)
    offs = torch.arange(0, (total + 1) * L, L, dtype=torch.int64, device=dev)
    keys = poslo_gpu_keys_create(ctx, params, [synthlog.derived_key_seed(seed + 3, k) for k in range(n_keys)])
    sigs = torch.empty(max(1, 80 * total), dtype=torch.uint8, device=dev)
    tags, ds = poslo_gpu_sign(keys, [(q["key"], q["t0"], q["n"], q["base"]) for q in reqs], data, offs, sigs)
    for q, t, d in zip(reqs, tags, ds):
        q["tag"], q["ds"] = t, d
    log = ServingLog(params=params, L=L, data=data[:total], sigs=sigs[:80 * total], pks=list(keys.pks),
                     requests=reqs)
    del keys
    plan = []
    for q in reqs:
        if q["flip"] is not None:
            plan.append((q["base"] + q["flip"][0], q["flip"][1]))
    if plan:
        view = MultiSignerLog(params=params, counts=[total], lengths=np.full(total, L),
                              offsets=np.arange(total + 1) * L, data=log.data.view(-1), d_offsets=offs,
                              sigs=log.sigs, pks=[], jobs=[])
        _flip(torch, view, sorted(plan))
    torch.cuda.synchronize(dev)
    return log
