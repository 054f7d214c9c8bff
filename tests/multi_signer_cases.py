"""Oracle-signed multi-signer cases shared by the batch and serving tests:
several signers with jobs of uneven sizes (including empty and single-entry
jobs, jobs starting mid-epoch and several jobs of one key at different t),
variable-length messages of 0 to 100 bytes, and a corrupted variant with
seeded single-bit flips and one tampered tag, with the oracle's expected
accept bits and invalid sets."""

import functools

import numpy as np

import synthlog

KEYS = 3
L1, L2 = 4, 3
# (key, t0, n); each key's jobs are consecutive in t
JOBS = [(0, 0, 37), (1, 0, 1), (2, 20, 50), (0, 37, 0), (0, 37, 26), (1, 1, 90)]


@functools.lru_cache(maxsize=None)
def oracle_jobs(inst):
    """Messages, keys and the oracle's signatures, tags and ds of JOBS."""
    from oracle import oracle as O
    # FourQ: a BPV table of 64 points and subsets of 8 keep the oracle's
    # scalar multiplications few (verification does not depend on them)
    prm = O.Params(inst, L1, L2, v=64, k=8) if inst & O.GROUP_FOURQ else O.Params(inst, L1, L2)
    total = sum(n for _, _, n in JOBS)
    lens = synthlog.uniform_per_stream(31, np.arange(total), 0, 100)
    data, off = synthlog.messages_var(32, lens)
    msgs = [bytes(data[off[e]:off[e + 1]]) for e in range(total)]
    seeds = [synthlog.derived_key_seed(50, k) for k in range(KEYS)]
    signers, pks = {}, {}
    for k in range(KEYS):
        signers[k], pks[k] = O.kg(prm, seeds[k])
    out, base = [], 0
    for key, t0, n in JOBS:
        s = signers[key]
        while s.t < t0:
            O.sig(s, b"")
        assert s.t == t0
        sg = [O.sig(s, msgs[base + p]) for p in range(n)]
        out.append(dict(key=key, t0=t0, n=n, entry_base=base, pk=pks[key], sigs=sg, tag=O.agg(sg, inst),
                        ds=O.ds_encode(s.ds)))
        base += n
    return prm, seeds, data, off, msgs, out


def corrupted_inputs(inst, n_flips=6, tamper_tag_of=4):
    """JOBS with seeded single-bit flips of m_t || sigma_t and one tampered
    tag; returns the oracle's expected accept bits and (job, t) pairs."""
    from oracle import oracle as O
    prm, seeds, data, off, msgs, jobs = oracle_jobs(inst)
    total = len(msgs)
    sigs = [sg for j in jobs for sg in j["sigs"]]
    lens = np.array([len(m) for m in msgs])
    plan = synthlog.corruption_plan_var(90 + inst, total, n_flips, 8 * (lens + 80))
    msgs, sigs = list(msgs), list(sigs)
    for e, bit in plan:
        blob = bytearray(msgs[e] + sigs[e])
        blob[bit // 8] ^= 1 << (bit % 8)
        msgs[e], sigs[e] = bytes(blob[:lens[e]]), bytes(blob[lens[e]:])
    jobs = [dict(j) for j in jobs]
    if tamper_tag_of is not None:
        t = bytearray(jobs[tamper_tag_of]["tag"])
        t[5] ^= 0x10
        jobs[tamper_tag_of]["tag"] = bytes(t)
    want_acc, want_inv, want_all = [], [], []
    for k, j in enumerate(jobs):
        b, n = j["entry_base"], j["n"]
        jm, js = msgs[b:b + n], sigs[b:b + n]
        ok = O.aver(prm, j["pk"], jm, j["t0"], j["ds"], j["tag"])
        want_acc.append(ok)
        bad = [(k, t) for t, _ in O.distill(prm, j["pk"], jm, js, j["t0"], j["ds"], 1).invalid]
        want_all += bad
        if not ok:
            want_inv += bad
    return jobs, b"".join(msgs), off, b"".join(sigs), want_acc, sorted(want_inv), sorted(want_all), plan


@functools.lru_cache(maxsize=None)
def corrupted_case(inst):
    return corrupted_inputs(inst)
