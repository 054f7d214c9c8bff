"""GPU parity of the multi-signer path (many signers' batches in one
persistent launch), the device signer and the device message generator,
through the C ABI.

Small cases: several signers with jobs of uneven sizes (including empty and
single-entry jobs, jobs starting mid-epoch and jobs of one key at different
t), variable-length messages (0 to 100 bytes, any alignment), signed by the
oracle, on edwards25519 and on FourQ.  The device signer must reproduce the oracle's signatures, tags and
ds byte for byte; the batch verifier's accept bits must equal the oracle's
AVer per job and its invalid (job, t) pairs the oracle's Distill on every
rejected job, for every kernel variant, with and without graph replay.
Large case: 4,096 signers with log-uniform [1, 65,536] entries of [64, 512]
bytes and 0.1% corrupted entries; accept bits and the invalid set must equal
what the injected corruption fixes, and sampled entries are re-verified one
by one by the oracle."""


import numpy as np
import pytest

import synthlog
from multi_signer_cases import L1, L2, corrupted_case, oracle_jobs

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def gpu(P):
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    ctx = P.poslo_ctx_create(0)
    yield torch, ctx
    ctx.close()


def to_dev(torch, data, off, sigs=b""):
    d = torch.from_numpy(np.frombuffer(bytes(data), dtype=np.uint8).copy()).cuda()
    o = torch.from_numpy(np.asarray(off, dtype=np.uint64).view(np.int64).copy()).cuda()
    s = torch.from_numpy(np.frombuffer(bytes(sigs), dtype=np.uint8).copy()).cuda() if sigs else None
    return d, o, s


def test_device_messages_equal_generator(P, gpu):
    torch, ctx = gpu
    rng = np.random.default_rng(3)
    lens = rng.integers(0, 300, 257)
    lens[5], lens[6], lens[7] = 0, 1, 8
    data, off = synthlog.messages_var(77, lens, t0=5)
    out = torch.zeros(data.size, dtype=torch.uint8, device="cuda")
    offs = torch.from_numpy(off.view(np.int64).copy()).cuda()
    print("device generator: variable layout", flush=True)
    P.poslo_synth_messages(77, P.poslo_msgs(None, offs.data_ptr(), 0, lens.size, 5, data.size), out)
    assert out.cpu().numpy().tobytes() == data.tobytes()
    want = synthlog.messages_fixed(78, 1000, 40, t0=3)
    out2 = torch.zeros((1000, 40), dtype=torch.uint8, device="cuda")
    print("device generator: fixed layout", flush=True)
    P.poslo_synth_messages(78, P.poslo_msgs(None, None, 40, 1000, 3, 40000), out2)
    assert np.array_equal(out2.cpu().numpy(), want)


@pytest.mark.parametrize("inst", [1, 0])
def test_gpu_signer_equals_oracle(P, gpu, inst):
    torch, ctx = gpu
    prm, seeds, data, off, msgs, jobs = oracle_jobs(inst)
    params = P.make_params(inst, L1, L2)
    print(f"inst {inst}: device keys", flush=True)
    keys = P.poslo_gpu_keys_create(ctx, params, seeds)
    for j in jobs:
        assert keys.pks[j["key"]] == j["pk"]
    d, o, _ = to_dev(torch, data, off)
    total = len(msgs)
    sigs = torch.zeros(80 * total, dtype=torch.uint8, device="cuda")
    print(f"inst {inst}: device signer over {len(jobs)} jobs", flush=True)
    tags, ds = P.poslo_gpu_sign(keys, [(j["key"], j["t0"], j["n"], j["entry_base"]) for j in jobs], d, o, sigs)
    hs = sigs.cpu().numpy().tobytes()
    for k, j in enumerate(jobs):
        b = j["entry_base"]
        got = [hs[80 * (b + p):80 * (b + p + 1)] for p in range(j["n"])]
        assert got == j["sigs"], f"job {k}"
        assert tags[k] == j["tag"], f"job {k}"
        assert ds[k] == j["ds"], f"job {k}"


def variants_of(P, inst):
    pre = "aes" if inst & 3 == 1 else "sha"
    return [v for v in range(P.poslo_batch_variant_count()) if P.poslo_batch_variant_name(v).startswith(pre)]


@pytest.mark.parametrize("inst", [1, 0, 1 | 8, 0 | 8])
def test_verify_batch_equals_oracle(P, gpu, inst):
    torch, ctx = gpu
    jobs, data, off, sigs, want_acc, want_inv, want_all, plan = corrupted_case(inst)
    # every flipped entry is invalid; only rejected jobs are distilled in mode 1
    assert {e for e, _ in plan} == {jobs[k]["entry_base"] + (t - jobs[k]["t0"]) for k, t in want_all}
    assert set(want_inv) <= set(want_all) and want_acc.count(False) >= 2
    params = P.make_params(inst, L1, L2)
    d, o, s = to_dev(torch, data, off, sigs)
    bj = P.BatchJobs(jobs)
    for v in variants_of(P, inst):
        for graph in (False, True):
            print(f"inst {inst}: variant {P.poslo_batch_variant_name(v)} graph {graph}", flush=True)
            acc, inv = P.poslo_verify_batch(ctx, params, bj, d, o, s, tuning=(v, 0, graph))
            assert acc == want_acc
            assert inv == want_inv
            acc2, inv2 = P.poslo_verify_batch(ctx, params, bj, d, o, None, tuning=(v, 0, graph))
            assert acc2 == want_acc and inv2 is None
            acc3, inv3 = P.poslo_verify_batch(ctx, params, bj, d, o, s, distill=2, tuning=(v, 0, graph))
            assert acc3 == want_acc and inv3 == want_all
    print(f"inst {inst}: default tuning", flush=True)
    assert P.poslo_verify_batch(ctx, params, bj, d, o, s) == (want_acc, want_inv)


@pytest.mark.parametrize("inst", [1, 0])
def test_verify_batch_wide_keys_equal_oracle(P, gpu, inst):
    """Keys given a wide table (poslo_ctx_keys_widen) are checked with it;
    the accept bits and invalid pairs stay the oracle's, with widened and
    plain keys mixed in one launch."""
    torch, _ = gpu
    jobs, data, off, sigs, want_acc, want_inv, want_all, plan = corrupted_case(inst)
    params = P.make_params(inst, L1, L2)
    d, o, s = to_dev(torch, data, off, sigs)
    bj = P.BatchJobs(jobs)
    ctx = P.poslo_ctx_create(0)
    try:
        pks = sorted({j["pk"] for j in jobs})
        print(f"inst {inst}: widening {len(pks) - 1} of {len(pks)} keys", flush=True)
        P.poslo_ctx_keys_widen(ctx, pks[:-1])
        for mode, want in ((1, want_inv), (2, want_all)):
            print(f"inst {inst}: distill {mode} with wide keys", flush=True)
            assert P.poslo_verify_batch(ctx, params, bj, d, o, s, distill=mode) == (want_acc, want)
        P.poslo_ctx_keys_widen(ctx, pks)
        assert P.poslo_verify_batch(ctx, params, bj, d, o, s, distill=2) == (want_acc, want_all)
        with pytest.raises(P.PosloError) as ei:
            P.poslo_ctx_keys_widen(ctx, [bytes([0xff] * 31 + [0x7f])])
        assert ei.value.status == P.POSLO_E_ENCODING
        P.poslo_ctx_keys_widen(ctx, [])
    finally:
        ctx.close()


@pytest.mark.parametrize("inst", [1, 0, 1 | 8])
def test_graph_replays_and_honest_jobs(P, gpu, inst):
    """Replays of one captured graph, with unrelated eager work and
    synchronizations between them, give the eager result every time; the
    honest jobs all accept."""
    torch, ctx = gpu
    prm, seeds, data, off, msgs, jobs = oracle_jobs(inst)
    sigs = b"".join(sg for j in jobs for sg in j["sigs"])
    params = P.make_params(inst, L1, L2)
    d, o, s = to_dev(torch, data, off, sigs)
    bj = P.BatchJobs(jobs)
    v = variants_of(P, inst)[0]
    eager = P.poslo_verify_batch(ctx, params, bj, d, o, s, tuning=(v, 0, False))
    assert eager == ([True] * len(jobs), [])
    x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
    for r in range(4):
        print(f"inst {inst}: graph replay {r}", flush=True)
        assert P.poslo_verify_batch(ctx, params, bj, d, o, s, tuning=(v, 0, True)) == eager
        x = (x * 1.0001).sin()
        torch.cuda.synchronize()
    # a tampered tag in a replayed shape flips only that job
    jobs2 = [dict(j) for j in jobs]
    t = bytearray(jobs2[2]["tag"])
    t[0] ^= 1
    jobs2[2]["tag"] = bytes(t)
    acc, inv = P.poslo_verify_batch(ctx, params, P.BatchJobs(jobs2), d, o, s, tuning=(v, 0, True))
    assert acc == [k != 2 for k in range(len(jobs))] and inv == []


def test_autotune_picks_a_parity_variant(P, gpu):
    torch, ctx = gpu
    for inst in (1, 0):
        jobs, data, off, sigs, want_acc, want_inv, _, _ = corrupted_case(inst)
        params = P.make_params(inst, L1, L2)
        d, o, s = to_dev(torch, data, off, sigs)
        bj = P.BatchJobs(jobs)
        print(f"inst {inst}: autotune", flush=True)
        best, ms = P.poslo_autotune_batch(ctx, params, bj, d, o, reps=2)
        assert best.variant in variants_of(P, inst) and ms > 0
        assert P.poslo_verify_batch(ctx, params, bj, d, o, s) == (want_acc, want_inv)
    P.poslo_batch_forget(ctx)


def test_verify_batch_errors(P, gpu):
    from oracle import oracle as O
    torch, ctx = gpu
    prm, seeds, data, off, msgs, jobs = oracle_jobs(1)
    params = P.make_params(1, L1, L2)
    d, o, s = to_dev(torch, data, off, b"".join(sg for j in jobs for sg in j["sigs"]))
    # a ds that does not cover the job's epochs
    bad = [dict(j) for j in jobs]
    bad[4]["ds"] = jobs[0]["ds"][:1 + 24 * 1]
    bad[4]["ds"] = bytes([1]) + bad[4]["ds"][1:]
    with pytest.raises(P.PosloError) as ei:
        P.poslo_verify_batch(ctx, params, P.BatchJobs(bad), d, o, s)
    assert ei.value.status == P.POSLO_E_SEED
    # a public key that is not a point
    y = 2
    while O.decode(y.to_bytes(32, "little")) is not None:
        y += 1
    bad = [dict(j) for j in jobs]
    bad[1]["pk"] = y.to_bytes(32, "little")
    with pytest.raises(P.PosloError) as ei:
        P.poslo_verify_batch(ctx, params, P.BatchJobs(bad), d, o, s)
    assert ei.value.status == P.POSLO_E_ENCODING
    assert P.poslo_ctx_keys_load(ctx, [jobs[0]["pk"], y.to_bytes(32, "little")]) == 1
    # no jobs at all
    assert P.poslo_verify_batch(ctx, params, P.BatchJobs([]), d, o, s) == ([], [])


@pytest.mark.parametrize("inst", [1, 0])
def test_full_size_multi_signer(P, gpu, inst):
    """4,096 signers, log-uniform [1, 65,536] entries each, messages of
    [64, 512] bytes, 0.1% of entries with one flipped bit."""
    from oracle import oracle as O
    from paper_2506_08781_amd import workloads
    torch, ctx = gpu
    print(f"inst {inst}: building the 4096-signer log on the device", flush=True)
    log = workloads.multi_signer(ctx, inst, 4096, 65536, 64, 512, 0.001, seed=7000 + inst)
    print(f"inst {inst}: {log.total} entries, {len(log.plan)} flips", flush=True)
    bases = log.bases
    flipped, msg_flipped = {}, set()
    for e, bit in log.plan:
        k = int(np.searchsorted(bases, e, side="right") - 1)
        flipped.setdefault(k, []).append(e - int(bases[k]))
        if bit < 8 * int(log.lengths[e]):
            msg_flipped.add(k)
    bj = log.batch_jobs()
    want = sorted((k, t) for k, ts in flipped.items() for t in ts)
    for mode in (1, 2):
        acc, inv = P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, log.sigs, distill=mode,
                                        cap=len(want) + 16)
        print(f"inst {inst}: verified (distill {mode}), {acc.count(False)} rejected, {len(inv)} invalid",
              flush=True)
        # AVer reads messages, ds and tags: a job is rejected iff a message bit flipped
        assert acc == [k not in msg_flipped for k in range(4096)]
        # mode 1 checks the entries of rejected jobs only
        assert inv == (want if mode == 2 else [p for p in want if p[0] in msg_flipped])
    # the same with the keys of jobs of 2^14 entries or more widened
    big = [k for k in range(4096) if log.counts[k] >= 1 << 14]
    print(f"inst {inst}: widening {len(big)} keys", flush=True)
    P.poslo_ctx_keys_widen(ctx, [log.jobs[k]["pk"] for k in big])
    results = {}
    for mode in (1, 2):
        results[mode] = P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, log.sigs,
                                             distill=mode, cap=len(want) + 16)
        print(f"inst {inst}: verified with wide keys (distill {mode})", flush=True)
        assert results[mode][0] == acc
        assert results[mode][1] == (want if mode == 2 else [p for p in want if p[0] in msg_flipped])
    # whole jobs against the oracle: the smallest, the largest, the one
    # whose last check tile is the most ragged, and a corrupted mid-size one;
    # the oracle signs each from synthlog's bytes and the plan is applied on
    # the host, so the GPU's inputs are checked byte for byte first
    import oracle_fullsize as F
    counts = log.counts
    nonempty = [k for k in range(4096) if counts[k]]
    pick = {min(nonempty, key=lambda k: counts[k]), max(nonempty, key=lambda k: counts[k]),
            min((k for k in nonempty if counts[k] > 1024 and counts[k] % 1024),
                key=lambda k: (counts[k] % 1024, counts[k]))}
    mid = [k for k in flipped if 1024 < counts[k] <= 8192]
    if mid:
        pick.add(mid[0])
    for k in sorted(pick):
        j = log.jobs[k]
        base, n = j["entry_base"], j["n"]
        lens = tuple(int(x) for x in log.lengths[base:base + n])
        plan = tuple((e - base, bit) for e, bit in log.plan if base <= e < base + n)
        print(f"inst {inst}: oracle over job {k} ({n} entries, {len(plan)} flips)", flush=True)
        case = F.job_case(inst, 8, 8, synthlog.derived_key_seed(7000 + inst + 3, k), 7000 + inst + 2, lens, base,
                          plan)
        assert (case.pk, case.ds, case.tag) == (j["pk"], j["ds"], j["tag"])
        msgs, _ = synthlog.messages_var(7000 + inst + 2, np.asarray(lens, dtype=np.int64), t0=base)
        blob_m = bytearray(msgs.tobytes())
        blob_s = bytearray(case.sigs)
        offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        for t, bit in plan:
            if bit < 8 * lens[t]:
                blob_m[offs[t] + bit // 8] ^= 1 << (bit % 8)
            else:
                b = bit - 8 * lens[t]
                blob_s[80 * t + b // 8] ^= 1 << (b % 8)
        o0, o1 = int(log.offsets[base]), int(log.offsets[base + n])
        assert log.data[o0:o1].cpu().numpy().tobytes() == bytes(blob_m)
        assert log.sigs[80 * base:80 * (base + n)].cpu().numpy().tobytes() == bytes(blob_s)
        assert acc[k] == case.aver_corrupt
        got = [t for kk, t in results[2][1] if kk == k]
        assert got == case.invalid
        assert [t for kk, t in results[1][1] if kk == k] == ([] if case.aver_corrupt else case.invalid)
    # sampled entries re-verified one by one by the oracle
    prm = O.Params(inst, 8, 8)
    hs_idx = [e for e, _ in log.plan[:3]] + [int(bases[k]) for k in (0, 1, 4095) if k not in flipped]
    for e in hs_idx:
        k = int(np.searchsorted(bases, e, side="right") - 1)
        j = log.jobs[k]
        t = e - j["entry_base"]
        L0, L1_ = int(log.offsets[e]), int(log.offsets[e + 1])
        m = log.data[L0:L1_].cpu().numpy().tobytes()
        sg = log.sigs[80 * e:80 * e + 80].cpu().numpy().tobytes()
        x0 = O.SR(inst, O.ds_decode(j["ds"]), t >> 8)
        assert O.entry_valid(prm, j["pk"], m, t, sg, x0) == (k not in flipped or t not in flipped[k])
