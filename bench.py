#!/usr/bin/env python3
"""Benchmark of POSLO-F batch verification on one MI355X.

A step is one aggregate verification (AVer) of a device-resident batch:
seed table (SR/SC and the hoisted PRF state), the fused per-entry PRF +
digest + lazy-sum kernel, and the final fold with the curve check.

Default workload: plain POSLO-F at the 128-bit parameter set, one signer,
2^20 entries of 256-byte messages (seeded xoshiro256** bytes), n2 = 256,
n1 = 4096, POSLO+ instantiation (MMO-AES-128 PRF, MDC-2-AES-128 hash), one
aggregate tag over honest signatures.  Prints one JSON line.
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

import synthlog  # noqa: E402

METRIC = "verified log entries/sec on 1 MI355X + p99 verify latency, batched vs plain"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz of 32-bit integer VALU work
INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

CONFIGS = {
    "c1": dict(n=1024, L=32, log2_n1=2, log2_n2=8, key_first=0x00, msg_seed=1,
               name="plain AVer, 1,024 entries x 32 B, n2=256, n1=4"),
    "c2": dict(n=1 << 20, L=256, log2_n1=12, log2_n2=8, key_first=0x20, msg_seed=2,
               name="plain AVer, 2^20 entries x 256 B, n2=256, n1=4096"),
}


# ---------------------------------------------------------------------------
# algorithmic work model: 32-bit integer VALU operations of the formulation
# the kernels implement on gfx950 (loads, loop control and address
# arithmetic for message pointers are not counted, so this is a lower bound
# of the executed instruction count; rocprof's SQ_INSTS_VALU cross-checks it)
# ---------------------------------------------------------------------------
# AES-128 over byte-addressed T-tables: a full round is 16 table-address
# v_perm, 8 rotations of the odd tables and 8 three-input xors (32); the
# final round is 16 address v_perm, 8 byte-merge v_perm, 4 ors, 4 xors (32);
# a key-schedule round is 4 address v_perm, 2 merge v_perm, 1 or, 1 xor3 and
# 3 xors (11); the initial key addition is 4.
AES_RK = 4 + 9 * 32 + 32          # encryption under a precomputed schedule
AES_OTF = AES_RK + 10 * 11        # with the schedule expanded on the fly
# SHA-256 compression: a round is 3+1 for each Sigma (rotations, xor3), 1 Ch,
# 1 Maj, 2 three-input adds for T1, 1 for a, 1 for e (14); a schedule word is
# 4 for each sigma and 2 adds (10); the feed-forward is 8 adds.
SHA_COMP = 64 * 14 + 48 * 10 + 8


def ops_per_entry(inst: int, L: int) -> int:
    if inst == 1:
        B = (L + 16 + 15) // 16
        # PRF (one AES + 1 xor), MDC-2 block 0 under the constant IV schedules,
        # blocks 1.. with two on-the-fly schedules, 8 xors per block, 9-limb sum
        return (AES_RK + 1) + (2 * AES_RK + 8) + (B - 1) * (2 * AES_OTF + 8) + 9
    nb = (L + 16 + 9 + 63) // 64
    # PRF compression + message compressions, byte swaps of the message words
    # and of the digest, 9-limb sum
    return (1 + nb) * SHA_COMP + (L + 3) // 4 + 8 + 9


def hash_calls_per_entry(inst: int, L: int) -> int:
    """AES-128 block encryptions (POSLO+) or SHA-256 compressions (POSLO)."""
    if inst == 1:
        return 1 + 2 * ((L + 16 + 15) // 16)
    return 1 + (L + 16 + 9 + 63) // 64


# ---------------------------------------------------------------------------


def build_inputs(P, cfg, inst):
    arr = synthlog.messages_fixed(cfg["msg_seed"], cfg["n"], cfg["L"])
    params = P.make_params(inst, cfg["log2_n1"], cfg["log2_n2"])
    sk, pk = P.poslo_kg(params, synthlog.key_seed_bytes(cfg["key_first"]))
    sigs = P.poslo_sig_batch(sk, arr)
    ds = P.poslo_ds_export(sk)
    tag = P.poslo_agg(sigs)
    return arr, params, pk, sigs, ds, tag


def cpu_baseline(cfg, inst, arr, pk, sigs, ds, P, target_s: float):
    """The oracle's AVer timed on host cores over a bounded leading slice of
    the same batch (same key, messages, ds), single-threaded."""
    from oracle import oracle as O
    prm = O.Params(inst, cfg["log2_n1"], cfg["log2_n2"])
    # calibrate on 64 entries
    cal = [bytes(r) for r in arr[:64]]
    t = time.perf_counter()
    O.ekeys_sum(prm, cal, 0, ds)
    per = (time.perf_counter() - t) / 64
    ns = int(max(64, min(cfg["n"], target_s / max(per, 1e-9))))
    sample = [bytes(r) for r in arr[:ns]]
    tag = P.poslo_agg(sigs[:ns])
    t = time.perf_counter()
    ok = O.aver(prm, pk, sample, 0, ds, tag)
    dt = time.perf_counter() - t
    return {"value": ns / dt, "unit": "entries/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle AVer over the first {ns} entries of the same batch ({dt:.1f} s, accept={ok})"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--inst", default="aes", choices=["aes", "sha"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy the message buffer once (a plain copy of known size "
                         "that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2506_08781_amd as P
    P.lib()  # fails loudly if the native library is missing
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)

    cfg = CONFIGS[args.config]
    inst = 1 if args.inst == "aes" else 0
    t = time.perf_counter()
    arr, params, pk, sigs, ds, tag = build_inputs(P, cfg, inst)
    print(f"# inputs ready in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    d = torch.from_numpy(arr).cuda()
    msgs = P.make_msgs(d)
    ctx = P.poslo_ctx_create(0)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        ok, _ = P.poslo_aver(ctx, params, pk, msgs, ds, tag, stream)
        assert ok, "honest batch rejected"
    P.poslo_ctx_profile(ctx, True)
    for k in (P.POSLO_KT_SEED, P.POSLO_KT_AGG, P.POSLO_KT_FINAL):
        P.poslo_ctx_kernel_time(ctx, k, reset=True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = time.perf_counter()
        ok, _ = P.poslo_aver(ctx, params, pk, msgs, ds, tag, stream)
        lat.append(time.perf_counter() - s)
        assert ok
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    P.poslo_ctx_profile(ctx, False)
    if args.calib_copy:
        d.clone()
        torch.cuda.synchronize()
    kt = {name: P.poslo_ctx_kernel_time(ctx, k) for name, k in
          (("seed", P.POSLO_KT_SEED), ("agg", P.POSLO_KT_AGG), ("final", P.POSLO_KT_FINAL))}

    n = cfg["n"]
    ms_step = 1e3 * total / args.steps
    value = n / (total / args.steps)
    agg_ms = kt["agg"][0] / max(kt["agg"][1], 1)
    ope = ops_per_entry(inst, cfg["L"])
    achieved = n * ope / (agg_ms / 1e3) / 1e12
    lat_ms = sorted(1e3 * x for x in lat)

    def pct(p):
        return lat_ms[min(len(lat_ms) - 1, int(round(p / 100 * (len(lat_ms) - 1))))]

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
        "latency_ms": {"p50": pct(50), "p99": pct(99), "max": lat_ms[-1]},
        "hashes_per_s": value * hash_calls_per_entry(inst, cfg["L"]),
        "hash_unit": "AES-128 blocks/s" if inst else "SHA-256 compressions/s",
        "kernel_ms": {k: v[0] / max(v[1], 1) for k, v in kt.items()},
        "roofline": {"bound": "alu", "kernel": "k_agg_ekeys_" + args.inst, "achieved": achieved,
                     "peak": INT32_PEAK_TOPS, "unit": "Tops/s (int32)", "frac": achieved / INT32_PEAK_TOPS,
                     "ops_per_entry": ope, "traffic": None,
                     "hbm_GBs": n * cfg["L"] / (agg_ms / 1e3) / 1e9},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, inst, arr, pk, sigs, ds, P, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
