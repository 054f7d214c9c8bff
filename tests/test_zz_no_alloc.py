"""The allocation-free AVer entry point (poslo_aver_fixed) gives the same
accept bit and e mod q as poslo_aver, through the C ABI, on two calls in a
row (the second on a smaller batch, so that stale scratch contents from the
first would show), for both instantiations and for a fixed-length and an
offset-indexed layout; oversized batches and non-resident keys are refused
on the host."""

import numpy as np
import pytest

import synthlog

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu(P):
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    ctx = P.poslo_ctx_create(0)
    yield torch, ctx
    ctx.close()


def signed(O, inst, n, L, log2_n1, log2_n2, key_first, msg_seed):
    prm = O.Params(inst, log2_n1, log2_n2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, n, L)]
    pk, sigs, ds, tag, _ = O.sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    return prm, msgs, pk, sigs, ds, tag


@pytest.mark.parametrize("inst", [1, 0])
def test_fixed_scratch_aver_equals_aver(P, O, gpu, inst):
    torch, ctx = gpu
    big = signed(O, inst, 3000, 48, 6, 6, 0x41, 21)
    small = signed(O, inst, 129, 40, 3, 5, 0x42, 22)
    params = {id(big): P.make_params(inst, 6, 6), id(small): P.make_params(inst, 3, 5)}
    for case in (big, small):
        P.poslo_ctx_keys_load(ctx, [case[2]])
    for case in (big, small):
        prm, msgs, pk, sigs, ds, tag = case
        arr = np.frombuffer(b"".join(msgs), dtype=np.uint8).reshape(len(msgs), -1)
        d = torch.from_numpy(arr.copy()).cuda()
        off = torch.from_numpy(np.arange(0, arr.size + 1, arr.shape[1], dtype=np.int64)).cuda()
        for m in (P.make_msgs(d), P.make_msgs(d.reshape(-1), off)):
            print(f"inst {inst} n {len(msgs)} offsets {m.offsets is not None}", flush=True)
            want = P.poslo_aver(ctx, params[id(case)], pk, m, ds, tag)
            got = P.poslo_aver_fixed(ctx, params[id(case)], pk, m, ds, tag)
            assert got == want
            assert got[0] is True and int.from_bytes(got[1], "little") == O.ekeys_sum(prm, msgs, 0, ds)
            bad = bytearray(tag)
            bad[33] ^= 2
            assert P.poslo_aver_fixed(ctx, params[id(case)], pk, m, ds, bytes(bad)) == \
                P.poslo_aver(ctx, params[id(case)], pk, m, ds, bytes(bad))


def test_fixed_scratch_limits(P, O, gpu):
    torch, ctx = gpu
    prm, msgs, pk, sigs, ds, tag = signed(O, 1, 16, 32, 2, 2, 0x43, 23)
    params = P.make_params(1, 2, 2)
    arr = np.frombuffer(b"".join(msgs), dtype=np.uint8).reshape(16, 32)
    d = torch.from_numpy(arr.copy()).cuda()
    # a key that was never loaded is refused before anything runs
    with pytest.raises(P.PosloError) as ei:
        P.poslo_aver_fixed(ctx, params, pk, P.make_msgs(d), ds, tag)
    assert ei.value.status == P.POSLO_E_INVAL
    P.poslo_ctx_keys_load(ctx, [pk])
    assert P.poslo_aver_fixed(ctx, params, pk, P.make_msgs(d), ds, tag)[0] is True
    # a batch spanning more epochs than the scratch holds is refused on the
    # host: n2 = 1, a ds made of the root node (covering every epoch), and
    # one entry more than the epoch limit
    wide = P.make_params(1, 15, 0)
    root_ds = bytes([1]) + bytes([15, 0, 0, 0]) + (0).to_bytes(4, "little") + bytes(16)
    n = P.POSLO_AVER_FIXED_MAX_EPOCHS + 1
    dz = torch.zeros((n, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(P.PosloError) as ei:
        P.poslo_aver_fixed(ctx, wide, pk, P.make_msgs(dz), root_ds, tag)
    assert ei.value.status == P.POSLO_E_INVAL
