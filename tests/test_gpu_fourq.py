"""GPU parity of AVer over the FourQ group (the paper's curve) against the
oracle, through the C ABI: the aggregate check on the device (comb tables of
the key and of FourQ's generator built by the device, e folded mod N, the
64-point sum) under POSLO+ and POSLO at kappa = 128 and POSLO+ at kappa =
127; the allocation-free AVer, per-entry e_t mod N and x_t, and the
streaming audit on FourQ; the tag
checks (s >= N, R not a FourQ point); Distill and SeBVer V/U/I on FourQ
(invalid sets, invalid signatures, valid and umbrella tags); the device
signer on FourQ; and the refusal of POSLO++ on FourQ (POSLO-C, the
multi-signer path and the serving loop on FourQ are in test_gpu_posloc.py,
test_gpu_batch.py and test_gpu_server.py).  Keys, signatures, ds and tags come from the oracle's
FourQ signer."""

import functools

import numpy as np
import pytest

import synthlog

pytestmark = pytest.mark.gpu

FQ = 8
NAMES = {1 | FQ: "aes", 0 | FQ: "sha", 1 | 4 | FQ: "aes-k127"}


@pytest.fixture(scope="module")
def gpu(P):
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    ctx = P.poslo_ctx_create(0)
    yield torch, ctx
    ctx.close()


@functools.lru_cache(maxsize=None)
def signed(inst, n, L, log2_n1, log2_n2, key_first, msg_seed):
    """A FourQ batch signed by the oracle (a BPV table of 64 points, subsets
    of 8, to keep its scalar multiplications few)."""
    from oracle import oracle as O
    prm = O.Params(inst, log2_n1, log2_n2, v=64, k=8)
    arr = synthlog.messages_fixed(msg_seed, n, L)
    msgs = [bytes(r) for r in arr]
    pk, sigs, ds, tag, _ = O.sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    sig_arr = np.frombuffer(b"".join(sigs), dtype=np.uint8).reshape(n, 80).copy()
    return prm, arr, msgs, pk, sig_arr, ds, tag


CASES = [
    # inst, n, L, log2_n1, log2_n2
    (1 | FQ, 777, 48, 4, 6),
    (0 | FQ, 300, 37, 4, 5),
    (1 | 4 | FQ, 1024, 32, 2, 8),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{NAMES[c[0]]}-n{c[1]}-L{c[2]}")
def test_fourq_aver_parity(P, O, gpu, case):
    torch, ctx = gpu
    inst, n, L, l1, l2 = case
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, n, L, l1, l2, 0x61, 4)
    params = P.make_params(inst, l1, l2)
    d = torch.from_numpy(arr.copy()).cuda()
    m = P.make_msgs(d)
    print(f"case {case}: aver", flush=True)
    acc, e = P.poslo_aver(ctx, params, pk, m, ds, tag)
    want = O.ekeys_sum(prm, msgs, 0, ds)
    assert want < O.FQ_N
    assert acc and int.from_bytes(e, "little") == want
    assert O.aggregate_check(pk, want, tag, inst)
    # the allocation-free entry point, now that the key and G tables are resident
    assert P.poslo_aver_fixed(ctx, params, pk, m, ds, tag) == (True, e)
    # per-entry e_t mod N and x_t
    eg, xg = P.poslo_ekeys(ctx, params, m, ds)
    eg, xg = eg.cpu().numpy(), xg.cpu().numpy()
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, n)
    for t in range(n):
        x = O.one_time_seed(inst, seeds[t >> l2], t & (prm.n2 - 1))
        assert bytes(xg[t]) == x
        assert int.from_bytes(bytes(eg[t]), "little") == O.digest_int(inst, msgs[t], x) % O.FQ_N
    # a flipped tag bit, a flipped message bit, s + N (same residue, not
    # canonical), and an R that is not a FourQ point are rejected
    bad = bytearray(tag)
    bad[40] ^= 0x10
    assert not P.poslo_aver(ctx, params, pk, m, ds, bytes(bad))[0]
    assert not O.aggregate_check(pk, want, bytes(bad), inst)
    s = int.from_bytes(tag[:32], "little")
    big = (s + O.FQ_N).to_bytes(32, "little") + tag[32:]
    assert not P.poslo_aver(ctx, params, pk, m, ds, big)[0]
    assert not O.aggregate_check(pk, want, big, inst)
    notpt = tag[:32] + (2 ** 127 - 1).to_bytes(16, "little") + tag[48:]
    assert not P.poslo_aver(ctx, params, pk, m, ds, notpt)[0]
    d2 = d.clone()
    d2[n // 2, 0] ^= 1
    assert not P.poslo_aver(ctx, params, pk, P.make_msgs(d2), ds, tag)[0]
    # a slice starting mid-epoch against its own aggregate
    a, b = 37, n - 5
    sub_tag = O.agg([bytes(r) for r in sigs[a:b]], inst)
    acc, e2 = P.poslo_aver(ctx, params, pk, P.make_msgs(d[a:b], t0=a), ds, sub_tag)
    assert acc and int.from_bytes(e2, "little") == O.ekeys_sum(prm, msgs[a:b], a, ds)


def test_fourq_empty_batch_and_key_errors(P, O, gpu):
    torch, ctx = gpu
    inst = 1 | FQ
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, 777, 48, 4, 6, 0x61, 4)
    params = P.make_params(inst, 4, 6)
    empty = torch.zeros((0, 48), dtype=torch.uint8, device="cuda")
    acc, e = P.poslo_aver(ctx, params, pk, P.make_msgs(empty), ds, O.agg([], inst))
    assert acc and e == bytes(32)
    d = torch.from_numpy(arr.copy()).cuda()
    badpk = (2 ** 127 - 1).to_bytes(16, "little") + pk[16:]
    with pytest.raises(P.PosloError) as ei:
        P.poslo_aver(ctx, params, badpk, P.make_msgs(d), ds, tag)
    assert ei.value.status == P.POSLO_E_ENCODING
    # the edwards25519 key cache and the FourQ one do not mix: the same 32
    # bytes verified under edwards25519 are another key (or no point at all)
    try:
        ok, _ = P.poslo_aver(ctx, P.make_params(1, 4, 6), pk, P.make_msgs(d), ds, tag)
    except P.PosloError as err:
        assert err.status == P.POSLO_E_ENCODING
    else:
        assert not ok


def test_fourq_audit(P, O, gpu):
    torch, ctx = gpu
    inst = 1 | FQ
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, 777, 48, 4, 6, 0x61, 4)
    params = P.make_params(inst, 4, 6)
    d = torch.from_numpy(arr.copy()).cuda()
    host = torch.from_numpy(arr.copy()).pin_memory()
    au = P.poslo_audit_begin(ctx, params, pk, ds, 0)
    cuts = [0, 100, 101, 500, 777]
    for k, (a, b) in enumerate(zip(cuts, cuts[1:])):
        src = host if k % 2 else d
        au.feed(P.make_msgs(src[a:b], t0=a))
    acc, e = au.finish(tag)
    assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)
    state = au.export()
    au.close()
    au2 = P.poslo_audit_resume(ctx, state, params)
    assert au2.finish(tag) == (True, e)
    au2.close()


def corrupt(msgs, sigs, plan):
    msgs, sigs = list(msgs), list(sigs)
    for e, bit in plan:
        L = len(msgs[e])
        blob = bytearray(msgs[e] + sigs[e])
        blob[bit // 8] ^= 1 << (bit % 8)
        msgs[e], sigs[e] = bytes(blob[:L]), bytes(blob[L:])
    return msgs, sigs


DISTILL_CASES = [
    # inst, n, L, log2_n1, log2_n2, corrupted entries, umbrellas
    (1 | FQ, 200, 48, 4, 4, 7, 5),
    (0 | FQ, 130, 37, 3, 5, 4, 3),
    (1 | 4 | FQ, 256, 32, 2, 8, 5, 4),
    (1 | FQ, 65, 16, 3, 4, 65, 1),   # every entry corrupted, one umbrella
]


@pytest.mark.parametrize("case", DISTILL_CASES, ids=lambda c: f"{NAMES[c[0]]}-n{c[1]}-k{c[5]}-u{c[6]}")
def test_fourq_distill_sebver(P, O, gpu, case):
    """Distill on FourQ (per-entry checks with FourQ's comb tables, scalars
    mod N, umbrella and valid tags as FourQ aggregates) and SeBVer V/U/I
    equal the oracle's."""
    torch, ctx = gpu
    inst, n, L, l1, l2, k, nu = case
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, n, L, l1, l2, 0x62, 5)
    plan = synthlog.corruption_plan(60 + k, n, k, 8 * (L + 80))
    cm, cs = corrupt(msgs, [bytes(r) for r in sigs], plan)
    params = P.make_params(inst, l1, l2)
    dm = torch.from_numpy(np.frombuffer(b"".join(cm), dtype=np.uint8).reshape(n, L).copy()).cuda()
    dsig = torch.from_numpy(np.frombuffer(b"".join(cs), dtype=np.uint8).copy()).cuda()
    print(f"case {case}: distill", flush=True)
    ccd = P.poslo_distill(ctx, params, pk, P.make_msgs(dm), dsig, ds, nu)
    want = O.distill(prm, pk, cm, cs, 0, ds, nu)
    got = ccd.invalid()
    assert got == [t for t, _ in want.invalid]
    assert got == sorted(e for e, _ in plan)
    for i, (t, sg) in enumerate(want.invalid):
        assert ccd.invalid_sig(i) == sg
    assert ccd.valid_tag() == want.valid_tag
    tags, span = ccd.umbrellas()
    assert span == want.span and tags == [t for t, _ in want.umbrellas]
    m = P.make_msgs(dm)
    for mode in "VUI":
        print(f"case {case}: sebver {mode}", flush=True)
        assert P.poslo_sebver(ctx, params, pk, m, ccd, mode) == O.sebver(prm, pk, cm, want, mode), mode
    # a tampered umbrella tag fails that umbrella only
    blob = bytearray(ccd.export())
    hdr = 4 + 4 + 4 * 3 + 8 * 3
    ds_len = int.from_bytes(blob[hdr:hdr + 4], "little")
    umb0 = hdr + 4 + ds_len + 64 + 8
    blob[umb0 + 3] ^= 1
    bits = P.poslo_sebver(ctx, params, pk, m, P.poslo_ccd_import(bytes(blob)), "U")
    assert bits[0] is False and all(bits[1:])


def test_fourq_distill_empty_batch(P, O, gpu):
    torch, ctx = gpu
    inst = 1 | FQ
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, 200, 48, 4, 4, 0x62, 5)
    params = P.make_params(inst, 4, 4)
    empty = torch.zeros((0, 48), dtype=torch.uint8, device="cuda")
    nosig = torch.zeros(0, dtype=torch.uint8, device="cuda")
    ccd = P.poslo_distill(ctx, params, pk, P.make_msgs(empty), nosig, ds, 3)
    assert ccd.invalid() == [] and ccd.valid_tag() == O.agg([], inst)


@pytest.mark.parametrize("inst", [1 | FQ, 0 | FQ, 1 | 4 | FQ], ids=lambda i: NAMES[i])
def test_fourq_device_signer_equals_oracle(P, O, gpu, inst):
    """The device signer on FourQ (BPV table R_k = r_k * G with FourQ's comb
    table, s_t = r_t - e_t * y mod N, tags from the sums) gives the oracle
    signer's keys, signatures, tags and ds byte for byte, for jobs of two
    keys starting at t = 0 and mid-epoch, over messages of 0 to 70 bytes."""
    torch, ctx = gpu
    l1, l2 = 3, 4
    prm = O.Params(inst, l1, l2, v=64, k=8)
    params = P.make_params(inst, l1, l2, 64, 8)
    seeds = [synthlog.derived_key_seed(81, k) for k in range(2)]
    jobs = [(0, 0, 40), (1, 5, 33), (0, 40, 1)]
    total = sum(n for _, _, n in jobs)
    lens = synthlog.uniform_per_stream(82, np.arange(total), 0, 70)
    data, off = synthlog.messages_var(83, lens)
    msgs = [bytes(data[off[e]:off[e + 1]]) for e in range(total)]
    print(f"inst {inst}: device keys and signer", flush=True)
    keys = P.poslo_gpu_keys_create(ctx, params, seeds)
    d = torch.from_numpy(data.copy()).cuda()
    o = torch.from_numpy(off.view(np.int64).copy()).cuda()
    sigs = torch.zeros(80 * total, dtype=torch.uint8, device="cuda")
    sj, base = [], 0
    for key, t0, n in jobs:
        sj.append((key, t0, n, base))
        base += n
    tags, ds = P.poslo_gpu_sign(keys, sj, d, o, sigs)
    hs = sigs.cpu().numpy().tobytes()
    for key in range(2):
        assert keys.pks[key] == O.kg(prm, seeds[key])[1]
    for k, (key, t0, n, b) in enumerate(sj):
        signer = O.signer_at(prm, seeds[key], t0)
        want = [O.sig(signer, msgs[b + p]) for p in range(n)]
        assert [hs[80 * (b + p):80 * (b + p + 1)] for p in range(n)] == want, f"job {k}"
        assert tags[k] == O.agg(want, inst), f"job {k}"
        assert ds[k] == O.ds_encode(signer.ds), f"job {k}"


def test_fourq_refuses_poslopp(P, gpu):
    """POSLO++ (H = Add_q) is not defined on FourQ: every entry point that
    takes the instantiation word refuses 2 | GROUP_FOURQ."""
    torch, ctx = gpu
    inst = 1 | FQ
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, 777, 48, 4, 6, 0x61, 4)
    d = torch.from_numpy(arr.copy()).cuda()
    bad = P.make_params(2 | FQ, 4, 6)
    assert P.lib().poslo_inst_valid(2 | FQ) == 0
    for name, call in {
        "aver": lambda: P.poslo_aver(ctx, bad, pk, P.make_msgs(d), ds, tag),
        "ekeys": lambda: P.poslo_ekeys(ctx, bad, P.make_msgs(d), ds),
        "server": lambda: P.Server(0, bad),
    }.items():
        with pytest.raises(P.PosloError) as ei:
            call()
        assert ei.value.status == P.POSLO_E_INVAL, name
