"""GPU parity of AVer over the FourQ group (the paper's curve) against the
oracle, through the C ABI: the aggregate check on the device (comb tables of
the key and of FourQ's generator built by the device, e folded mod N, the
64-point sum) under POSLO+ and POSLO at kappa = 128 and POSLO+ at kappa =
127; the allocation-free AVer and the streaming audit on FourQ; the tag
checks (s >= N, R not a FourQ point); and the entry points that take
edwards25519 only.  Keys, signatures, ds and tags come from the oracle's
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


def test_fourq_refused_where_not_built(P, gpu):
    torch, ctx = gpu
    inst = 1 | FQ
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, 777, 48, 4, 6, 0x61, 4)
    params = P.make_params(inst, 4, 6)
    d = torch.from_numpy(arr.copy()).cuda()
    dsig = torch.from_numpy(sigs.reshape(-1).copy()).cuda()
    calls = {
        "ekeys": lambda: P.poslo_ekeys(ctx, params, P.make_msgs(d), ds),
        "distill": lambda: P.poslo_distill(ctx, params, pk, P.make_msgs(d), dsig, ds, 4),
        "c_key_load": lambda: P.poslo_c_key_load(ctx, P.make_params(inst, 2, 4), bytes(32 * 5)),
        "gpu_keys": lambda: P.poslo_gpu_keys_create(ctx, params, [bytes(32)]),
        "server": lambda: P.Server(0, params),
    }
    for name, call in calls.items():
        with pytest.raises(P.PosloError) as ei:
            call()
        assert ei.value.status == P.POSLO_E_INVAL, name
