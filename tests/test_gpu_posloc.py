"""GPU parity of POSLO-C (coarse-grained: one signature per epoch) against
the oracle, through the C ABI: AVer over whole epochs, Distill's invalid
epochs, valid tag and umbrella tags, SeBVer V/U/I, the coarse CCD's byte
export, and the argument errors, on edwards25519 and on FourQ.  Keys,
signatures and ds come from the oracle's POSLO-C signer."""

import functools

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


@functools.lru_cache(maxsize=None)
def signed_c(inst, k, L, log2_n1, log2_n2, key_first, msg_seed):
    from oracle import oracle as O
    prm = O.Params(inst, log2_n1, log2_n2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, k * prm.n2, L)]
    pk, s_list, ds, _ = O.posloc_sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    return prm, msgs, pk, s_list, ds


def upload(torch, msgs, fixed=True):
    L = len(msgs[0])
    arr = np.frombuffer(b"".join(msgs), dtype=np.uint8).reshape(len(msgs), L)
    d = torch.from_numpy(arr.copy()).cuda()
    if fixed:
        return d, None
    off = torch.from_numpy(np.arange(0, arr.size + 1, L, dtype=np.int64)).cuda()
    return d.reshape(-1), off


CASES = [
    # inst, epochs, L, log2_n1, log2_n2: fast layout, any layout, one entry per epoch
    (1, 6, 48, 3, 4),
    (0, 6, 48, 3, 4),
    (1, 5, 37, 3, 3),
    (0, 5, 37, 3, 3),
    (1, 4, 64, 2, 0),
    (1 | 8, 6, 48, 3, 4),   # the FourQ group
    (0 | 8, 5, 37, 3, 3),
]


def _ep(prm, msgs, i):
    return (i, msgs[i * prm.n2:(i + 1) * prm.n2])


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"inst{c[0]}-k{c[1]}-L{c[2]}-n1_{c[3]}-n2_{c[4]}")
def test_c_aver_distill_sebver_equal_oracle(P, gpu, case):
    from oracle import oracle as O
    torch, ctx = gpu
    inst, k, L, l1, l2 = case
    prm, msgs, pk, s_list, ds = signed_c(inst, k, L, l1, l2, 0x61, 41)
    params = P.make_params(inst, l1, l2)
    key = P.poslo_c_key_load(ctx, params, pk)
    n2 = prm.n2
    for fixed in (True, False):
        d, off = upload(torch, msgs, fixed)
        m = P.make_msgs(d, off)
        print(f"case {case} fixed {fixed}: aver", flush=True)
        acc, e = P.poslo_c_aver(ctx, params, key, m, ds, O.posloc_agg_s(s_list, inst))
        assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)
        # a range of epochs against its own aggregate; a wrong aggregate
        a, b = 1, k - 1
        sub = msgs[a * n2:b * n2]
        ds_, off_ = upload(torch, sub, fixed)
        ms = P.make_msgs(ds_, off_, t0=a * n2)
        assert P.poslo_c_aver(ctx, params, key, ms, ds, O.posloc_agg_s(s_list[a:b], inst))[0]
        assert not P.poslo_c_aver(ctx, params, key, ms, ds, O.posloc_agg_s(s_list[a:b + 1], inst))[0]
    # Distill with a flipped message bit in epoch 1 and a flipped s bit in epoch k-2
    cm, cs = list(msgs), list(s_list)
    mm = bytearray(cm[n2 + n2 // 2])
    mm[3] ^= 0x08
    cm[n2 + n2 // 2] = bytes(mm)
    sv = bytearray(cs[k - 2])
    sv[17] ^= 0x40
    cs[k - 2] = bytes(sv)
    want = O.posloc_distill(prm, pk, cm, cs, 0, ds, 2)
    assert [i for i, _ in want.invalid] == [1, k - 2]
    for fixed in (True, False):
        d, off = upload(torch, cm, fixed)
        m = P.make_msgs(d, off)
        ccd = P.poslo_c_distill(ctx, params, key, m, b"".join(cs), ds, 2)
        assert ccd.invalid() == [1, k - 2]
        assert [ccd.invalid_sig(q) for q in range(2)] == [sg + bytes(16) for _, sg in want.invalid]
        assert ccd.valid_tag() == want.valid_tag
        umb, span = ccd.umbrellas()
        assert span == want.span and umb == [t for t, _ in want.umbrellas]
        for mode in "VUI":
            assert P.poslo_c_sebver(ctx, params, key, m, ccd, mode) == O.posloc_sebver(prm, pk, cm, want, mode)
        # the coarse CCD survives its byte export; the POSLO-F SeBVer refuses it
        back = P.poslo_ccd_import(ccd.export())
        assert back.invalid() == ccd.invalid() and back.valid_tag() == ccd.valid_tag()
        assert P.poslo_c_sebver(ctx, params, key, m, back, "U") == O.posloc_sebver(prm, pk, cm, want, "U")
        with pytest.raises(P.PosloError):
            P.poslo_sebver(ctx, params, pk[:32], m, back, "V")


def test_c_errors(P, gpu):
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, pk, s_list, ds = signed_c(1, 6, 48, 3, 4, 0x61, 41)
    params = P.make_params(1, 3, 4)
    key = P.poslo_c_key_load(ctx, params, pk)
    d, _ = upload(torch, msgs)
    # not whole epochs: a batch that ends mid-epoch, and one that starts mid-epoch
    with pytest.raises(P.PosloError) as ei:
        P.poslo_c_aver(ctx, params, key, P.make_msgs(d[:20]), ds, s_list[0])
    assert ei.value.status == P.POSLO_E_INVAL
    with pytest.raises(P.PosloError) as ei:
        P.poslo_c_aver(ctx, params, key, P.make_msgs(d[:16], t0=3), ds, s_list[0])
    assert ei.value.status == P.POSLO_E_INVAL
    # a key of the wrong size, and a commitment that is not a point
    with pytest.raises(P.PosloError) as ei:
        P.poslo_c_key_load(ctx, params, pk[:-32])
    assert ei.value.status == P.POSLO_E_INVAL
    bad = bytearray(pk)
    bad[32 * 3:32 * 4] = (2 ** 255 - 19 + 3).to_bytes(32, "little")
    with pytest.raises(P.PosloError) as ei:
        P.poslo_c_key_load(ctx, params, bytes(bad))
    assert ei.value.status == P.POSLO_E_ENCODING
    # the empty batch accepts the zero aggregate only
    z = torch.zeros((0, 48), dtype=torch.uint8, device="cuda")
    assert P.poslo_c_aver(ctx, params, key, P.make_msgs(z), ds, bytes(32)) == (True, bytes(32))
    assert not P.poslo_c_aver(ctx, params, key, P.make_msgs(z), ds, O.to32(1))[0]
