#!/usr/bin/env python3
"""Benchmark of POSLO-F verification on one MI355X.

A step of the headline workload is one aggregate verification (AVer) of a
device-resident batch: seed table (SR/SC and the hoisted PRF state), the
fused per-entry PRF + digest + lazy-sum kernel, and the final fold with the
curve check.  Headline workload: plain POSLO-F at the 128-bit parameter set,
one signer, 2^20 entries of 256-byte messages (seeded xoshiro256** bytes),
n2 = 256, n1 = 4096, POSLO+ instantiation (MMO-AES-128 PRF, MDC-2-AES-128
hash), one aggregate tag over honest signatures.

The same run also measures, each on its own synthetic log:
 - small: the 1,024 x 32-byte configuration (latency-bound): microseconds
   per AVer call, the kernels' durations and the launch overhead;
 - sha (or aes with --inst sha): the headline configuration under the other
   instantiation, with its own roofline;
 - host: inputs in pinned host memory with the copies included (the
   paper's convention): the headline batch per AVer call, the same batch
   streamed through the chunked audit, and a 2^25 x 32-byte log streamed in
   128 MiB chunks;
 - variants: POSLO++ (H = Add_q) at kappa = 127 and 128 and POSLO+ over 2^26
   entries of 16-byte messages, and POSLO+ at kappa = 127 and on the FourQ
   group on the headline batch;
 - distill: Distill of 2^20 x 256-byte entries with 1% of entries carrying
   one flipped bit of m_t || sigma_t (exact invalid set, CCD);
 - batched: 4,096 signers with log-uniform [1, 65,536] entries of uniform
   [64, 512]-byte messages, 0.1% flipped entries, verified in one persistent
   launch (autotuned) against the plain path (one AVer call per signer),
   plus the invalid set of every signer (AVer + individual checks);
 - serving: requests from 10,000 resident keys with log-uniform [1, 2^18]
   entries of 128-byte messages, 0.5% of requests with a flipped bit,
   submitted at Poisson arrival times of fixed rates and in one burst to the
   serving loop; p50/p99 submit-to-result latency and entries/s.  It runs in
   a process of its own (started before this one touches the GPU, released
   after the other sections), as a serving deployment would.
Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "verified log entries/sec on 1 MI355X + p99 verify latency, batched vs plain"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz of 32-bit integer VALU work
INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

CONFIGS = {
    "c1": dict(n=1024, L=32, log2_n1=2, log2_n2=8, seed=1,
               name="plain AVer, 1,024 entries x 32 B, n2=256, n1=4"),
    "c2": dict(n=1 << 20, L=256, log2_n1=12, log2_n2=8, seed=2,
               name="plain AVer, 2^20 entries x 256 B, n2=256, n1=4096"),
}
CLOCK_WARMUP_S = 0.3
DISTILL = dict(n=1 << 20, L=256, log2_n1=12, log2_n2=8, seed=3, frac=0.01, umbrellas=64)
BATCHED = dict(signers=4096, max_batch=65536, len_lo=64, len_hi=512, frac=0.001, seed=4, log2_n1=8, log2_n2=8)
VARIANT = dict(n=1 << 26, L=16, log2_n1=18, log2_n2=8, seed=6)
SERVING = dict(keys=10000, distinct=1500, max_batch=1 << 18, L=128, p_corrupt=0.005, seed=5, submissions=4000,
               qps=(2000, 10000, 40000))


# ---------------------------------------------------------------------------
# algorithmic work model: 32-bit integer VALU operations of the formulation
# the kernels implement on gfx950 (loads, loop control and address
# arithmetic for message pointers are not counted, so this is a lower bound
# of the executed instruction count; rocprof's SQ_INSTS_VALU cross-checks it)
# ---------------------------------------------------------------------------
# AES-128 over byte-addressed T-tables (te0 and te0 rotated by 16): a full
# round is 16 table-address v_perm, 4 rotations, 4 xors and 8 xor-type ops
# of three or two inputs (32); the
# final round is 16 address v_perm, 8 byte-merge v_perm, 4 ors, 4 xors (32);
# a key-schedule round is 4 address v_perm, 2 merge v_perm, 1 or, 1 xor3 and
# 3 xors (11); the initial key addition is 4.
AES_RK = 4 + 9 * 32 + 32          # encryption under a precomputed schedule
AES_OTF = AES_RK + 10 * 11        # with the schedule expanded on the fly
# SHA-256 compression: a round is 3+1 for each Sigma (rotations, xor3), 1 Ch,
# 1 Maj, 2 three-input adds for T1, 1 for a, 1 for e (14); a schedule word is
# 4 for each sigma and 2 adds (10); the feed-forward is 8 adds.
SHA_COMP = 64 * 14 + 48 * 10 + 8


# POSLO++ (H = Add_q): x_t by one AES under the epoch schedule, 1 xor of j,
# 1 and of the kappa mask; e_t = LE(m) + LE(x) as an eight-word carry chain
# (12); the 9-limb sum
ADDQ_OPS = AES_RK + 2 + 12 + 9


def ops_per_entry(inst: int, L):
    """Works on ints and numpy arrays of lengths."""
    if inst & 3 == 2:
        return ADDQ_OPS
    inst &= 3
    if inst == 1:
        B = (L + 16 + 15) // 16
        # PRF (one AES + 1 xor), MDC-2 block 0 under the constant IV schedules,
        # blocks 1.. with two on-the-fly schedules, 8 xors per block, 9-limb sum
        return (AES_RK + 1) + (2 * AES_RK + 8) + (B - 1) * (2 * AES_OTF + 8) + 9
    nb = (L + 16 + 9 + 63) // 64
    # PRF compression + message compressions, byte swaps of the message words
    # and of the digest, 9-limb sum
    return (1 + nb) * SHA_COMP + (L + 3) // 4 + 8 + 9


# The same operations split by measured issue class: poslo_valu_probe shows
# v_xor_b32 and v_bitop3_b32 (xor-class) issuing about 1.6 times faster than
# v_perm_b32, v_alignbit_b32, v_add3_u32 and v_mad_u64_u32 (perm-class) on
# MI355X.  AES (two tables, aes_perm.h): a full round is 20 perm-class (16
# addresses, 4 rotations) and 12 xor-class (T1[y] ^ T3[z] is taken as
# rot8(T0[y] ^ T2[z])); the final round 24 and 8; a key-schedule round 6
# and 5; the key addition 0 and 4.  SHA-256: a round is 10 perm-class (six
# rotations, four sums) and 4 xor-class (two three-input xors, Ch, Maj); a
# schedule word 8 and 2; shifts and or-merges are counted perm-class.
AES_RK_CLS = (9 * 20 + 24, 9 * 12 + 8 + 4)
AES_OTF_CLS = (AES_RK_CLS[0] + 10 * 6, AES_RK_CLS[1] + 10 * 5)
SHA_COMP_CLS = (64 * 10 + 48 * 8 + 8, 64 * 4 + 48 * 2)
ADDQ_CLS = (AES_RK_CLS[0] + 1 + 12 + 9, AES_RK_CLS[1] + 1)
assert sum(AES_RK_CLS) == AES_RK and sum(AES_OTF_CLS) == AES_OTF and sum(SHA_COMP_CLS) == SHA_COMP
assert sum(ADDQ_CLS) == ADDQ_OPS


def op_classes_per_entry(inst: int, L: int):
    """(perm-class, xor-class) split of ops_per_entry."""
    if inst & 3 == 2:
        return ADDQ_CLS
    inst &= 3
    if inst == 1:
        B = (L + 16 + 15) // 16
        slow = AES_RK_CLS[0] + 2 * AES_RK_CLS[0] + (B - 1) * 2 * AES_OTF_CLS[0] + 9
        fast = AES_RK_CLS[1] + 1 + 2 * AES_RK_CLS[1] + 8 + (B - 1) * (2 * AES_OTF_CLS[1] + 8)
    else:
        nb = (L + 16 + 9 + 63) // 64
        slow = (1 + nb) * SHA_COMP_CLS[0] + (L + 3) // 4 + 8 + 9
        fast = (1 + nb) * SHA_COMP_CLS[1]
    assert slow + fast == ops_per_entry(inst, L)
    return slow, fast


def probe_rates(P):
    """Sustained lane-ops/s of each probed instruction kind at 8 waves per
    SIMD (poslo_valu_probe), in T/s."""
    return {op: P.poslo_valu_probe(op, 8, 2048)[0] / 1e12 for op in P.PROBE_OPS}


def mix_peak(rates, inst: int, L: int):
    """Issue ceiling of the op model's mix: the operations of one entry at
    the measured rates of their class (perm-class at the mean of perm,
    alignbit, add3 and mad64; xor-class at the mean of xor and bitop3)."""
    slow, fast = op_classes_per_entry(inst, L)
    r_slow = sum(rates[k] for k in ("perm", "alignbit", "add3", "mad64")) / 4
    r_fast = (rates["xor"] + rates["bitop3"]) / 2
    return (slow + fast) / (slow / r_slow + fast / r_fast)


def hash_calls_per_entry(inst: int, L):
    """AES-128 block encryptions (POSLO+, POSLO++) or SHA-256 compressions (POSLO)."""
    if inst & 3 == 2:
        return 1
    inst &= 3
    if inst == 1:
        return 1 + 2 * ((L + 16 + 15) // 16)
    return 1 + (L + 16 + 9 + 63) // 64


# HBM traffic of the hot kernels from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, averaged) over the
# benchmark's plain and variants sections, each scaled by what the counter
# read for a plain 256 MiB device copy in the same runs (FETCH_SIZE
# 131,087 KiB -> x2.0, WRITE_SIZE 262,144 KiB -> x1.0).  Valid only for the
# kernel sources they were taken on: the sha256 prefix of those files must
# match, else traffic is null.
TRAFFIC = {
    "aes": {"fetch_kib": 190775.2, "write_kib": 32.0, "fetch_scale": 2.0, "write_scale": 1.0,
            "files": ["agg_aes.hip", "aes_perm.h", "aes128.h", "device_entry.h", "device_hash.h", "device_verify.h",
                      "common.h", "sc25519.h", "fourq.h"],
            "sha256": "a35867ececc68287", "profile": "profiles/pmc_aver_2p20x256.md"},
    "aes_2p26x16": {"fetch_kib": 556442.3, "write_kib": 32.0, "fetch_scale": 2.0, "write_scale": 1.0,
                    "files": ["agg_aes.hip", "aes_perm.h", "aes128.h", "device_entry.h", "device_hash.h",
                              "device_verify.h", "common.h", "sc25519.h", "fourq.h"],
                    "sha256": "a35867ececc68287", "profile": "profiles/pmc_aver_2p20x256.md"},
    "addq": {"fetch_kib": 573542.2, "write_kib": 32.0, "fetch_scale": 2.0, "write_scale": 1.0,
             "files": ["agg_addq.hip", "aes_perm.h", "aes128.h", "device_entry.h", "device_hash.h", "common.h",
                       "sc25519.h"],
             "sha256": "e6f91aa883f9a3fb", "profile": "profiles/pmc_aver_2p20x256.md"},
    "sha": {"fetch_kib": 133149.6, "write_kib": 1088.0, "fetch_scale": 2.0, "write_scale": 1.0,
            "files": ["agg_sha.hip", "sha256.h", "device_entry.h", "device_hash.h", "common.h", "sc25519.h", "fourq.h"],
            "sha256": "7f728dd1dd5128ba", "profile": "profiles/pmc_aver_2p20x256.md"},
}


def traffic_bytes(inst_name):
    """Measured HBM bytes per launch of the headline kernel, or None when its
    sources changed since the counters were taken."""
    import hashlib
    t = TRAFFIC[inst_name]
    h = hashlib.sha256()
    for f in t["files"]:
        with open(os.path.join(ROOT, "paper_2506_08781_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != t["sha256"]:
        return None
    return 1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def pct(xs, p):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(round(p / 100 * (len(xs) - 1))))]


def lat_summary(lat_s):
    ms = [1e3 * x for x in lat_s]
    return {"p50": pct(ms, 50), "p99": pct(ms, 99), "max": max(ms), "samples": len(ms)}


def kernel_ms(P, ctx, k):
    tot, n = P.poslo_ctx_kernel_time(ctx, k)
    return tot / max(n, 1)


def reset_times(P, ctx):
    for k in range(8):
        P.poslo_ctx_kernel_time(ctx, k, reset=True)


# ---------------------------------------------------------------------------


def cpu_baseline(cfg, inst, log, target_s: float):
    """The oracle's AVer timed on host cores over a bounded leading slice of
    the same batch (same key, messages, ds), single-threaded."""
    from oracle import oracle as O
    prm = O.Params(inst, cfg["log2_n1"], cfg["log2_n2"])
    cal = [bytes(r) for r in log.data[:64].cpu().numpy()]
    t = time.perf_counter()
    O.ekeys_sum(prm, cal, 0, log.ds)
    per = (time.perf_counter() - t) / 64
    ns = int(max(64, min(cfg["n"], target_s / max(per, 1e-9))))
    sample = [bytes(r) for r in log.data[:ns].cpu().numpy()]
    sg = log.sigs[:80 * ns].cpu().numpy().tobytes()
    tag = O.agg([sg[80 * k:80 * k + 80] for k in range(ns)])
    t = time.perf_counter()
    ok = O.aver(prm, log.pk, sample, 0, log.ds, tag)
    dt = time.perf_counter() - t
    return {"value": ns / dt, "unit": "entries/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle AVer over the first {ns} entries of the same batch ({dt:.1f} s, accept={ok})",
            "host": host_info()}


def host_info():
    """CPU model and core counts of the machine the oracle ran on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "cpu_count": os.cpu_count()}


def bench_plain(P, torch, ctx, cfg, inst, steps, warmup, calib_copy):
    from paper_2506_08781_amd import workloads
    t = time.perf_counter()
    log = workloads.single_signer_fixed(ctx, inst, cfg["n"], cfg["L"], cfg["log2_n1"], cfg["log2_n2"], cfg["seed"])
    print(f"# plain: inputs ready in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    msgs = P.make_msgs(log.data)
    stream = torch.cuda.current_stream()
    # untimed: the warmup steps, and more until the GPU has run this workload
    # for CLOCK_WARMUP_S (its clocks ramp up under sustained load)
    t_w, k = time.perf_counter(), 0
    while k < warmup or time.perf_counter() - t_w < CLOCK_WARMUP_S:
        ok, _ = P.poslo_aver(ctx, log.params, log.pk, msgs, log.ds, log.tag, stream)
        assert ok, "honest batch rejected"
        k += 1
    # timed: events around the hashing kernel only (the roofline's duration)
    P.poslo_ctx_profile(ctx, [P.POSLO_KT_AGG])
    reset_times(P, ctx)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s = time.perf_counter()
        ok, _ = P.poslo_aver(ctx, log.params, log.pk, msgs, log.ds, log.tag, stream)
        lat.append(time.perf_counter() - s)
        assert ok
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    P.poslo_ctx_profile(ctx, False)
    agg = kernel_ms(P, ctx, P.POSLO_KT_AGG)
    if calib_copy:
        log.data.clone()
        torch.cuda.synchronize()
    # untimed: the seed and final kernels' durations
    P.poslo_ctx_profile(ctx, [P.POSLO_KT_SEED, P.POSLO_KT_FINAL])
    reset_times(P, ctx)
    for _ in range(steps):
        P.poslo_aver(ctx, log.params, log.pk, msgs, log.ds, log.tag, stream)
    torch.cuda.synchronize()
    P.poslo_ctx_profile(ctx, False)
    kt = {"seed": kernel_ms(P, ctx, P.POSLO_KT_SEED), "agg": agg, "final": kernel_ms(P, ctx, P.POSLO_KT_FINAL)}
    return log, total, lat, kt


def bench_small(P, torch, ctx, inst, calls):
    """The 1,024 x 32-byte configuration: latency-bound, so the figures are
    microseconds per AVer call (host call to verdict), the kernels' own
    durations, and the launch overhead (call latency minus kernel time)."""
    from paper_2506_08781_amd import workloads
    cfg = CONFIGS["c1"]
    log = workloads.single_signer_fixed(ctx, inst, cfg["n"], cfg["L"], cfg["log2_n1"], cfg["log2_n2"], cfg["seed"])
    msgs = P.make_msgs(log.data)
    stream = torch.cuda.current_stream()
    for _ in range(20):
        assert P.poslo_aver(ctx, log.params, log.pk, msgs, log.ds, log.tag, stream)[0]
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        s = time.perf_counter()
        ok, _ = P.poslo_aver(ctx, log.params, log.pk, msgs, log.ds, log.tag, stream)
        lat.append(time.perf_counter() - s)
        assert ok
    total = time.perf_counter() - t0
    # untimed: each kernel's duration, one kernel timed per pass
    kt = {}
    for name, k in (("seed", P.POSLO_KT_SEED), ("agg", P.POSLO_KT_AGG), ("final", P.POSLO_KT_FINAL)):
        P.poslo_ctx_profile(ctx, [k])
        reset_times(P, ctx)
        for _ in range(50):
            P.poslo_aver(ctx, log.params, log.pk, msgs, log.ds, log.tag, stream)
        torch.cuda.synchronize()
        kt[name] = kernel_ms(P, ctx, k)
    P.poslo_ctx_profile(ctx, False)
    lat_us = {k: 1e3 * v for k, v in lat_summary(lat).items() if k != "samples"}
    kernels_us = 1e3 * sum(kt.values())
    return {"workload": cfg["name"] + (", POSLO+" if inst else ", POSLO"), "calls": calls,
            "entries_per_s": cfg["n"] * calls / total, "latency_us": lat_us,
            "kernel_us": {k: 1e3 * v for k, v in kt.items()},
            "launch_overhead_us": lat_us["p50"] - kernels_us}


def bench_plain_other(P, torch, ctx, inst, steps, warmup, rates):
    """The headline configuration under the other instantiation, with its own
    roofline (the same measurement as the headline)."""
    cfg = CONFIGS["c2"]
    log, total, lat, kt = bench_plain(P, torch, ctx, cfg, inst, steps, warmup, False)
    del log
    n = cfg["n"]
    ope = ops_per_entry(inst, cfg["L"])
    achieved = n * ope / (kt["agg"] / 1e3) / 1e12
    name = "aes" if inst else "sha"
    value = n / (total / steps)
    mp = mix_peak(rates, inst, cfg["L"])
    return {"workload": cfg["name"] + (", POSLO+ (MMO/MDC-2 over AES-128)" if inst else ", POSLO (SHA-256)"),
            "entries_per_s": value, "ms_per_step": 1e3 * total / steps, "latency_ms": lat_summary(lat),
            "hashes_per_s": value * hash_calls_per_entry(inst, cfg["L"]),
            "hash_unit": "AES-128 blocks/s" if inst else "SHA-256 compressions/s", "kernel_ms": kt,
            "roofline": {"bound": "alu", "kernel": "k_agg_ekeys_" + name, "achieved": achieved,
                         "peak": INT32_PEAK_TOPS, "unit": "Tops/s (int32)", "frac": achieved / INT32_PEAK_TOPS,
                         "ops_per_entry": ope, "traffic": traffic_bytes(name),
                         "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                         "algorithmic_bytes": n * cfg["L"], "hbm_GBs": n * cfg["L"] / (kt["agg"] / 1e3) / 1e9,
                         "peak_measured_mix": mp, "frac_measured_mix": achieved / mp}}


def bench_variants(P, torch, ctx, steps, warmup, rates):
    """The parameter variants: POSLO++ (H = Add_q) at kappa = 127 and 128 on
    2^26 entries of 16-byte messages (Add_q takes at most 31 bytes); on the
    headline configuration, POSLO+ at kappa = 127 (a seed walk of one AES per
    tree level instead of two) and POSLO+ on the FourQ group (the same
    hashing, the final check on FourQ)."""
    out = {}
    cfg = dict(VARIANT, name="plain AVer, 2^26 entries x 16 B, n2=256, n1=2^18")
    for inst, key in ((2 | 4, "poslopp_k127"), (2, "poslopp")):
        log, total, lat, kt = bench_plain(P, torch, ctx, cfg, inst, steps, warmup, False)
        del log
        torch.cuda.empty_cache()
        n = cfg["n"]
        ope = ops_per_entry(inst, cfg["L"])
        achieved = n * ope / (kt["agg"] / 1e3) / 1e12
        mp = mix_peak(rates, inst, cfg["L"])
        hbm = n * cfg["L"] / (kt["agg"] / 1e3) / 1e9
        out[key] = {
            "workload": cfg["name"] + ", POSLO++ (MMO-AES-128 PRF, H = Add_q), kappa = "
                        + ("127" if inst & 4 else "128"),
            "entries_per_s": n / (total / steps), "ms_per_step": 1e3 * total / steps,
            "latency_ms": lat_summary(lat), "kernel_ms": kt,
            "roofline": {"bound": "alu", "kernel": "k_agg_addq", "achieved": achieved, "peak": INT32_PEAK_TOPS,
                         "unit": "Tops/s (int32)", "frac": achieved / INT32_PEAK_TOPS, "ops_per_entry": ope,
                         "peak_measured_mix": mp, "frac_measured_mix": achieved / mp, "traffic": traffic_bytes("addq"),
                         "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                         "algorithmic_bytes": n * cfg["L"], "hbm_GBs": hbm, "hbm_frac": hbm / HBM_PEAK_GBS}}
    # POSLO+ on the same 2^26 x 16-byte log: the paper's small-message case
    log, total, lat, kt = bench_plain(P, torch, ctx, cfg, 1, steps, warmup, False)
    del log
    torch.cuda.empty_cache()
    n = cfg["n"]
    ope = ops_per_entry(1, cfg["L"])
    achieved = n * ope / (kt["agg"] / 1e3) / 1e12
    out["posloplus_2p26x16"] = {
        "workload": cfg["name"] + ", POSLO+ (MMO/MDC-2 over AES-128)",
        "entries_per_s": n / (total / steps), "ms_per_step": 1e3 * total / steps, "latency_ms": lat_summary(lat),
        "kernel_ms": kt, "hashes_per_s": n / (total / steps) * hash_calls_per_entry(1, cfg["L"]),
        "roofline": {"bound": "alu", "kernel": "k_agg_ekeys_aes", "achieved": achieved, "peak": INT32_PEAK_TOPS,
                     "unit": "Tops/s (int32)", "frac": achieved / INT32_PEAK_TOPS, "ops_per_entry": ope,
                     "traffic": traffic_bytes("aes_2p26x16"), "algorithmic_bytes": n * cfg["L"],
                     "hbm_GBs": n * cfg["L"] / (kt["agg"] / 1e3) / 1e9}}
    cfg2 = CONFIGS["c2"]
    log, total, lat, kt = bench_plain(P, torch, ctx, cfg2, 1 | 4, steps, warmup, False)
    del log
    torch.cuda.empty_cache()
    out["posloplus_k127"] = {"workload": cfg2["name"] + ", POSLO+ at kappa = 127",
                             "entries_per_s": cfg2["n"] / (total / steps), "ms_per_step": 1e3 * total / steps,
                             "latency_ms": lat_summary(lat), "kernel_ms": kt}
    log, total, lat, kt = bench_plain(P, torch, ctx, cfg2, 1 | P.GROUP_FOURQ, steps, warmup, False)
    del log
    torch.cuda.empty_cache()
    out["posloplus_fourq"] = {"workload": cfg2["name"] + ", POSLO+ on the FourQ group",
                              "entries_per_s": cfg2["n"] / (total / steps), "ms_per_step": 1e3 * total / steps,
                              "latency_ms": lat_summary(lat), "kernel_ms": kt}
    return out


def bench_host(P, torch, ctx, inst, steps):
    """Inputs resident in host memory, copies included (the paper's GPU
    timings include the host-to-device copies): the headline batch in pinned
    memory verified by one AVer call per step (copy, then hash); the same
    batch streamed through the audit in 8 chunks (a chunk's copy overlaps
    the previous chunk's hashing); and a 1 GiB log of 2^25 entries of 32
    bytes, the entry size of the paper's 1 TB audit, streamed in 8 chunks
    of 128 MiB."""
    from paper_2506_08781_amd import workloads
    out = {}
    cfg = CONFIGS["c2"]
    n, L = cfg["n"], cfg["L"]
    log = workloads.single_signer_fixed(ctx, inst, n, L, cfg["log2_n1"], cfg["log2_n2"], cfg["seed"])
    host = log.data.cpu().pin_memory()
    stream = torch.cuda.current_stream()
    hm = P.make_msgs(host)
    for _ in range(3):
        assert P.poslo_aver(ctx, log.params, log.pk, hm, log.ds, log.tag, stream)[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        assert P.poslo_aver(ctx, log.params, log.pk, hm, log.ds, log.tag, stream)[0]
    dt = (time.perf_counter() - t0) / steps
    out["aver_pinned_host"] = {"workload": cfg["name"] + ", messages in pinned host memory",
                               "entries_per_s": n / dt, "ms_per_step": 1e3 * dt, "GBs_from_host": n * L / dt / 1e9}

    def stream_run(lg, hbuf, chunks, reps):
        nn = hbuf.shape[0]
        step = nn // chunks
        best = None
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            au = P.poslo_audit_begin(ctx, lg.params, lg.pk, lg.ds, 0)
            for a in range(0, nn, step):
                au.feed(P.make_msgs(hbuf[a:a + step], t0=a), stream)
            ok, _ = au.finish(lg.tag, stream)
            dt_ = time.perf_counter() - t
            au.close()
            assert ok, "streamed audit rejected an honest log"
            if r and (best is None or dt_ < best):
                best = dt_
        return best

    dt = stream_run(log, host, 8, steps // 4 + 1)
    out["audit_stream_2p20x256"] = {"workload": cfg["name"] + ", streamed from pinned host memory in 8 chunks",
                                    "entries_per_s": n / dt, "ms": 1e3 * dt, "GBs_from_host": n * L / dt / 1e9}
    del log, host
    torch.cuda.empty_cache()
    n2, L2 = 1 << 25, 32
    log = workloads.single_signer_fixed(ctx, inst, n2, L2, 17, 8, 6)
    host = log.data.cpu().pin_memory()
    log.sigs = log.data = None  # the audit reads the host copy only
    torch.cuda.empty_cache()
    dt = stream_run(log, host, 8, 2)
    out["audit_stream_2p25x32"] = {"workload": "audit of 2^25 entries x 32 B (1 GiB), n2=256, n1=2^17, streamed "
                                               "from pinned host memory in 8 chunks of 128 MiB",
                                   "entries_per_s": n2 / dt, "ms": 1e3 * dt, "GBs_from_host": n2 * L2 / dt / 1e9}
    del log, host
    return out


def bench_distill(P, torch, ctx, inst, steps):
    from paper_2506_08781_amd import workloads
    c = DISTILL
    t = time.perf_counter()
    log = workloads.single_signer_fixed(ctx, inst, c["n"], c["L"], c["log2_n1"], c["log2_n2"], c["seed"],
                                        corrupt_frac=c["frac"])
    print(f"# distill: inputs ready in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    msgs = P.make_msgs(log.data)
    want = sorted(e for e, _ in log.plan)
    ccd = P.poslo_distill(ctx, log.params, log.pk, msgs, log.sigs, log.ds, c["umbrellas"])
    assert ccd.invalid() == want, "invalid set differs from the injected flips"
    del ccd
    n = c["n"]
    out = {
        "workload": f"Distill, 2^20 entries x 256 B, {int(c['frac'] * 100)}% entries with one flipped bit, "
                    f"{c['umbrellas']} umbrellas",
        "invalid": len(want),
    }
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s = time.perf_counter()
        ccd = P.poslo_distill(ctx, log.params, log.pk, msgs, log.sigs, log.ds, c["umbrellas"])
        lat.append(time.perf_counter() - s)
        del ccd
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    # untimed: kernel durations
    P.poslo_ctx_profile(ctx, True)
    reset_times(P, ctx)
    for _ in range(steps):
        ccd = P.poslo_distill(ctx, log.params, log.pk, msgs, log.sigs, log.ds, c["umbrellas"])
        del ccd
    torch.cuda.synchronize()
    P.poslo_ctx_profile(ctx, False)
    out.update({"entries_per_s": n * steps / total, "ms_per_step": 1e3 * total / steps,
                "latency_ms": lat_summary(lat),
                "kernel_ms": {"hash_and_checks": kernel_ms(P, ctx, P.POSLO_KT_VERIFY),
                              "fold_and_compact": kernel_ms(P, ctx, P.POSLO_KT_COMPACT)}})
    return out


def bench_batched(P, torch, ctx, inst, steps, rates):
    from paper_2506_08781_amd import workloads
    c = BATCHED
    t = time.perf_counter()
    log = workloads.multi_signer(ctx, inst, c["signers"], c["max_batch"], c["len_lo"], c["len_hi"], c["frac"],
                                 seed=c["seed"], log2_n1=c["log2_n1"], log2_n2=c["log2_n2"])
    print(f"# batched: {log.total} entries of {c['signers']} signers ready in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    total_entries = log.total
    bases = log.bases
    flipped, msg_flipped = {}, set()
    for e, bit in log.plan:
        k = int(np.searchsorted(bases, e, side="right") - 1)
        flipped.setdefault(k, []).append(e - int(bases[k]))
        if bit < 8 * int(log.lengths[e]):
            msg_flipped.add(k)
    want_acc = [k not in msg_flipped for k in range(c["signers"])]
    want_inv = sorted((k, t) for k, ts in flipped.items() for t in ts)
    bj = log.batch_jobs()
    P.poslo_ctx_keys_load(ctx, log.pks)  # keys resident before timing

    # autotune the persistent launch on this batch (AVer only)
    t = time.perf_counter()
    tuning, tuned_ms = P.poslo_autotune_batch(ctx, log.params, bj, log.data, log.d_offsets, reps=2)
    tune_s = time.perf_counter() - t
    tuned = (tuning.variant, tuning.wg_per_cu, False)
    acc, _ = P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, tuning=tuned)
    assert acc == want_acc, "batched accept bits differ from the injected flips"

    # batched AVer, eager launches, events around the hashing kernel only
    P.poslo_ctx_profile(ctx, [P.POSLO_KT_BATCH_HOT])
    reset_times(P, ctx)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s = time.perf_counter()
        P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, tuning=tuned)
        lat.append(time.perf_counter() - s)
    torch.cuda.synchronize()
    eager_total = time.perf_counter() - t0
    P.poslo_ctx_profile(ctx, False)
    hot_ms = kernel_ms(P, ctx, P.POSLO_KT_BATCH_HOT)
    # untimed: the whole launch sequence's duration
    P.poslo_ctx_profile(ctx, [P.POSLO_KT_BATCH])
    reset_times(P, ctx)
    for _ in range(3):
        P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, tuning=tuned)
    torch.cuda.synchronize()
    P.poslo_ctx_profile(ctx, False)
    pipe_ms = kernel_ms(P, ctx, P.POSLO_KT_BATCH)

    # the same with the launch sequence replayed from a captured graph
    graph = (tuning.variant, tuning.wg_per_cu, True)
    P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, tuning=graph)
    glat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s = time.perf_counter()
        acc, _ = P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, tuning=graph)
        glat.append(time.perf_counter() - s)
    torch.cuda.synchronize()
    graph_total = time.perf_counter() - t0
    assert acc == want_acc

    # AVer plus the exact invalid set of every signer (SeBVer's input): one
    # individual check per entry
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        acc, inv = P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, log.sigs, distill=2,
                                        tuning=graph, cap=len(want_inv) + 16)
    dt = (time.perf_counter() - t0) / reps
    assert acc == want_acc and inv == want_inv, "batched invalid set differs from the injected flips"
    # untimed: the check kernels' duration
    P.poslo_ctx_profile(ctx, [P.POSLO_KT_VERIFY])
    reset_times(P, ctx)
    P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, log.sigs, distill=2, tuning=graph,
                         cap=len(want_inv) + 16)
    torch.cuda.synchronize()
    P.poslo_ctx_profile(ctx, False)
    sets = {"entries_per_s": total_entries / dt, "ms": 1e3 * dt,
            "check_kernels_ms": kernel_ms(P, ctx, P.POSLO_KT_VERIFY),
            "rejected": acc.count(False), "invalid": len(inv)}

    # the same after giving the keys of jobs of 2^14 entries or more their
    # wide tables (resident key state, built before timing)
    big = [k for k in range(c["signers"]) if log.counts[k] >= 1 << 14]
    t = time.perf_counter()
    P.poslo_ctx_keys_widen(ctx, [log.jobs[k]["pk"] for k in big])
    widen_s = time.perf_counter() - t
    P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, log.sigs, distill=2, tuning=graph,
                         cap=len(want_inv) + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        acc, inv = P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, log.sigs, distill=2,
                                        tuning=graph, cap=len(want_inv) + 16)
    dt = (time.perf_counter() - t0) / reps
    assert acc == want_acc and inv == want_inv, "batched invalid set (wide keys) differs from the injected flips"
    P.poslo_ctx_profile(ctx, [P.POSLO_KT_VERIFY])
    reset_times(P, ctx)
    P.poslo_verify_batch(ctx, log.params, bj, log.data, log.d_offsets, log.sigs, distill=2, tuning=graph,
                         cap=len(want_inv) + 16)
    torch.cuda.synchronize()
    P.poslo_ctx_profile(ctx, False)
    sets_wide = {"entries_per_s": total_entries / dt, "ms": 1e3 * dt,
                 "check_kernels_ms": kernel_ms(P, ctx, P.POSLO_KT_VERIFY),
                 "widened_keys": len(big), "widened_entries": int(sum(log.counts[k] for k in big)),
                 "wide_table_bytes": len(big) * 48 * 2 ** 20, "widen_s": widen_s}

    # plain path: one AVer call per signer on the same device buffers
    plain_lat = []
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k, j in enumerate(log.jobs):
        m = P.poslo_msgs(log.data.data_ptr(), log.d_offsets.data_ptr() + 8 * j["entry_base"], 0, j["n"], j["t0"],
                         log.data.numel())
        s = time.perf_counter()
        ok, _ = P.poslo_aver(ctx, log.params, j["pk"], m, j["ds"], j["tag"], stream)
        plain_lat.append(time.perf_counter() - s)
        assert ok == want_acc[k]
    torch.cuda.synchronize()
    plain_total = time.perf_counter() - t0

    ops = int(np.sum(ops_per_entry(inst, log.lengths.astype(np.int64))))
    uniq, cnt = np.unique(log.lengths.astype(np.int64), return_counts=True)
    slow = sum(int(c) * op_classes_per_entry(inst, int(u))[0] for u, c in zip(uniq, cnt))
    r_slow = sum(rates[k] for k in ("perm", "alignbit", "add3", "mad64")) / 4
    r_fast = (rates["xor"] + rates["bitop3"]) / 2
    mp = ops / (slow / r_slow + (ops - slow) / r_fast)
    hashes = int(np.sum(hash_calls_per_entry(inst, log.lengths.astype(np.int64))))
    achieved = ops / (hot_ms / 1e3) / 1e12
    graph_eps = total_entries * steps / graph_total
    return {
        "workload": f"{c['signers']} signers, log-uniform [1, {c['max_batch']}] entries each "
                    f"({total_entries} total), messages uniform [{c['len_lo']}, {c['len_hi']}] B, "
                    f"{c['frac'] * 100:.1f}% entries with one flipped bit, n2={1 << c['log2_n2']}, "
                    f"n1={1 << c['log2_n1']}",
        "entries": total_entries,
        "msg_bytes": int(log.offsets[-1]),
        "tuning": {"variant": P.poslo_batch_variant_name(tuning.variant), "wg_per_cu": tuning.wg_per_cu,
                   "autotune_s": tune_s, "tuned_ms": tuned_ms},
        "batched": {"entries_per_s": graph_eps, "ms_per_step": 1e3 * graph_total / steps,
                    "latency_ms": lat_summary(glat), "launch": "hipGraph replay",
                    "eager_entries_per_s": total_entries * steps / eager_total,
                    "eager_latency_ms": lat_summary(lat),
                    "hashes_per_s": hashes * steps / graph_total},
        "batched_with_invalid_sets": sets,
        "batched_with_invalid_sets_wide_keys": sets_wide,
        "plain": {"entries_per_s": total_entries / plain_total, "ms_per_pass": 1e3 * plain_total,
                  "per_signer_latency_ms": lat_summary(plain_lat)},
        "speedup_vs_plain": graph_eps / (total_entries / plain_total),
        "kernel_ms": {"hot": hot_ms, "pipeline": pipe_ms},
        "roofline": {"bound": "alu", "kernel": "k_batch_hot", "achieved": achieved, "peak": INT32_PEAK_TOPS,
                     "unit": "Tops/s (int32)", "frac": achieved / INT32_PEAK_TOPS, "ops": ops, "traffic": None,
                     "hbm_GBs": int(log.offsets[-1]) / (hot_ms / 1e3) / 1e9,
                     "peak_measured_mix": mp, "frac_measured_mix": achieved / mp},
    }


def serve_run(P, srv, reqs, order, qps):
    """Submit reqs[order[k]] at Poisson times of rate qps (all at once when
    qps is 0) from this thread; returns the results and the wall time from
    the first submission to the last result."""
    import random
    rng = random.Random(11)
    results = {}
    t_first = time.perf_counter()
    t_next = t_first
    for k in order:
        if qps:
            t_next += rng.expovariate(qps)
            while time.perf_counter() < t_next:
                pass
        srv.submit(reqs[k])
        for r in srv.poll(256):
            results[r.ticket] = r
    while len(results) < len(order):
        for r in srv.poll(1024, timeout_ms=20):
            results[r.ticket] = r
    wall = time.perf_counter() - t_first
    return list(results.values()), wall


def bench_serving(P, torch, ctx, inst):
    from paper_2506_08781_amd import workloads
    c = SERVING
    t = time.perf_counter()
    log = workloads.serving_requests(ctx, inst, c["keys"], c["distinct"], c["max_batch"], c["L"], c["p_corrupt"],
                                     seed=c["seed"])
    n_entries = [q["n"] for q in log.requests]
    print(f"# serving: {len(log.requests)} distinct requests, {sum(n_entries)} entries, ready in "
          f"{time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    # the hashing variant: the autotuner's choice on a group shaped like the
    # groups the server launches (the pool's first requests, up to 256 and
    # 2^21 entries)
    jobs, ent = [], 0
    for q in log.requests:
        if len(jobs) == 256 or ent + q["n"] > (1 << 21):
            break
        jobs.append(dict(pk=log.pks[q["key"]], ds=q["ds"], tag=q["tag"], t0=q["t0"], n=q["n"],
                         entry_base=q["base"]))
        ent += q["n"]
    total = log.data.shape[0]
    offs = torch.arange(0, (total + 1) * log.L, log.L, dtype=torch.int64, device=log.data.device)
    P.poslo_ctx_keys_load(ctx, [j["pk"] for j in jobs])
    tuning, _ = P.poslo_autotune_batch(ctx, log.params, P.BatchJobs(jobs), log.data.reshape(-1), offs, reps=2)
    del offs
    srv = P.Server(0, log.params, n_streams=4, max_group=256, distill=1, variant=tuning.variant)
    srv.register_keys(list(range(c["keys"])), log.pks)
    L = log.L
    reqs = []
    for r, q in enumerate(log.requests):
        b, n = q["base"], q["n"]
        reqs.append(P.Request(q["key"], q["t0"], n, log.data[b:b + n], None, L, log.sigs[80 * b:80 * (b + n)],
                              q["ds"], q["tag"], user=r, data_bytes=n * L))
    import random
    rng = random.Random(3)
    # warm the streams' buffers with one pass over every distinct request
    res, _ = serve_run(P, srv, reqs, list(range(len(reqs))), 0)
    for r in res:
        acc, inv = log.expected(r.user, 1)
        assert r.status == P.POSLO_OK and bool(r.accept) == acc and r.n_invalid == len(inv), f"request {r.user}"
        if r.n_invalid:
            assert srv.take_invalid(r.ticket, r.n_invalid) == inv
    runs = []
    for qps in list(c["qps"]) + [0]:
        order = [rng.randrange(len(reqs)) for _ in range(c["submissions"])]
        res, wall = serve_run(P, srv, reqs, order, qps)
        ok = all(r.status == P.POSLO_OK and bool(r.accept) == log.expected(r.user, 1)[0] for r in res)
        for r in res:
            if r.n_invalid:
                srv.take_invalid(r.ticket, r.n_invalid)
        lat = [r.t_done_ms - r.t_submit_ms for r in res]
        ent = sum(r.entries for r in res)
        runs.append({"qps": qps if qps else "burst", "requests": len(res), "entries": ent,
                     "entries_per_s": ent / wall, "wall_s": wall, "correct": ok,
                     "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat)}})
        assert ok, "a served result differs from what its flips fix"
    st = srv.stats()
    srv.close()
    return {
        "workload": f"serving: Poisson arrivals from {c['keys']} resident keys, requests of log-uniform "
                    f"[1, 2^18] entries of {L}-byte messages, {c['p_corrupt'] * 100:.1f}% of requests with one "
                    f"flipped bit, {len(reqs)} distinct requests resubmitted, invalid entries of rejected "
                    f"requests reported",
        "runs": runs,
        "variant": P.poslo_batch_variant_name(tuning.variant),
        "groups_launched": st.groups_launched,
        "device_bytes_peak": st.bytes_peak,
    }


def start_serving_child(inst_name):
    """Start the process that will run the serving section.  It is started
    before this process touches the GPU and waits for a line "go" on its
    stdin before it does anything else (EOF makes it exit)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--serving-only", "--inst", inst_name]
    return subprocess.Popen(cmd, stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)


def finish_serving_child(child):
    """Let the serving process run now and return its JSON object."""
    out, _ = child.communicate("go\n", timeout=900)
    if child.returncode != 0:
        raise RuntimeError(f"serving section failed with status {child.returncode}")
    return json.loads(out.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--inst", default="aes", choices=["aes", "sha"])
    ap.add_argument("--sections", default="plain,small,other,host,variants,distill,batched,serving",
                    help="comma list of plain, small (the 1,024 x 32-byte configuration), other (the headline "
                         "configuration under the other instantiation), host (inputs in host memory, copies "
                         "included), variants (POSLO++ and kappa = 127), distill, batched, serving (plain "
                         "always runs)")
    ap.add_argument("--aes-variant", type=int, default=-1,
                    help="POSLO+ AVer hot-kernel variant for the plain section (poslo_ctx_set_tuning; -1: the "
                         "library's default)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving section and print its JSON object (used by the main run)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy the message buffer once (a plain copy of known size "
                         "that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    sections = set(args.sections.split(","))
    if args.serving_only:
        if sys.stdin.readline().strip() != "go":
            sys.exit(0)
    # the serving process, started while this one has not touched the GPU
    child = start_serving_child(args.inst) if ("serving" in sections and not args.serving_only) else None

    import torch
    import paper_2506_08781_amd as P
    P.lib()  # fails loudly if the native library is missing
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)

    cfg = CONFIGS[args.config]
    inst = 1 if args.inst == "aes" else 0
    ctx = P.poslo_ctx_create(0)
    if args.aes_variant >= 0:
        P.poslo_ctx_set_tuning(ctx, agg_variant=args.aes_variant)
    if args.serving_only:
        serving = bench_serving(P, torch, ctx, inst)
        ctx.close()
        print(json.dumps(serving), flush=True)
        return

    log, total, lat, kt = bench_plain(P, torch, ctx, cfg, inst, args.steps, args.warmup, args.calib_copy)
    n = cfg["n"]
    ms_step = 1e3 * total / args.steps
    value = n / (total / args.steps)
    agg_ms = kt["agg"]
    ope = ops_per_entry(inst, cfg["L"])
    achieved = n * ope / (agg_ms / 1e3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": cfg["name"] + (", POSLO+ (MMO/MDC-2 over AES-128)" if inst else ", POSLO (SHA-256)"),
                   "entries": n, "msg_bytes": cfg["L"], "n2": 1 << cfg["log2_n2"], "n1": 1 << cfg["log2_n1"],
                   "instantiation": args.inst, "path": "plain"},
        "latency_ms": lat_summary(lat),
        "hashes_per_s": value * hash_calls_per_entry(inst, cfg["L"]),
        "hash_unit": "AES-128 blocks/s" if inst else "SHA-256 compressions/s",
        "kernel_ms": kt,
        "roofline": {"bound": "alu", "kernel": "k_agg_ekeys_" + args.inst, "achieved": achieved,
                     "peak": INT32_PEAK_TOPS, "unit": "Tops/s (int32)", "frac": achieved / INT32_PEAK_TOPS,
                     "ops_per_entry": ope,
                     "traffic": traffic_bytes(args.inst) if args.config == "c2" else None,
                     "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "algorithmic_bytes": n * cfg["L"],
                     "hbm_GBs": n * cfg["L"] / (agg_ms / 1e3) / 1e9},
    }
    # the measured issue rates, and the ceiling of this kernel's op mix at them
    rates = probe_rates(P)
    mp = mix_peak(rates, inst, cfg["L"])
    out["roofline"].update({"peak_basis": "256 CUs x 64 lanes x 2.4 GHz (one wave64 VALU op per 4 cycles per SIMD)",
                            "probe_Tops": rates, "peak_measured_mix": mp, "frac_measured_mix": achieved / mp})
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, inst, log, args.cpu_seconds)
    del log
    torch.cuda.empty_cache()
    if "small" in sections:
        out["small"] = bench_small(P, torch, ctx, inst, 400)
    if "other" in sections:
        out["sha" if inst else "aes"] = bench_plain_other(P, torch, ctx, 1 - inst, args.steps, args.warmup, rates)
        torch.cuda.empty_cache()
    if "host" in sections:
        out["host"] = bench_host(P, torch, ctx, inst, max(4, args.steps // 2))
        torch.cuda.empty_cache()
    if "variants" in sections:
        out["variants"] = bench_variants(P, torch, ctx, args.steps, args.warmup, rates)
        torch.cuda.empty_cache()
    if "distill" in sections:
        out["distill"] = bench_distill(P, torch, ctx, inst, max(2, args.steps // 4))
        torch.cuda.empty_cache()
        # the same on the FourQ group (the paper's curve)
        out["distill"]["fourq"] = bench_distill(P, torch, ctx, inst | P.GROUP_FOURQ, max(2, args.steps // 4))
        torch.cuda.empty_cache()
    if "batched" in sections:
        out["multi_signer"] = bench_batched(P, torch, ctx, inst, max(3, args.steps // 2), rates)
        torch.cuda.empty_cache()
    ctx.close()
    # serving in a process of its own, as a serving deployment runs: its
    # request loop is host-bound Python, and in this process, after the
    # other sections, it measured slower (burst 1.10 vs 1.74 G entries/s),
    # while running it first slowed the invalid-set pass after it
    if child is not None:
        try:
            out["serving"] = finish_serving_child(child)
        except Exception as exc:  # the other sections' results still print
            child.kill()
            out["serving"] = {"error": f"{type(exc).__name__}: {exc}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
