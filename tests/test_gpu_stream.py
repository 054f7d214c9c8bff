"""Host-resident batches and the streaming audit, through the C ABI.

* Host batches (pinned and pageable CPU tensors): AVer, per-entry digests,
  Distill (with host signatures) and POSLO-C AVer give the oracle's results,
  the same as the device batches.
* The streaming audit: an oracle-signed log fed in chunks of uneven sizes,
  starting mid-epoch, from host and device memory, gives the oracle's e and
  verdict; its state exported after some chunks and resumed gives the same;
  misuse is refused.  At the full 2^20 x 256-byte size the log streamed
  from pinned host memory in eight chunks gives the oracle's e over the
  whole batch.
"""

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
def signed(inst, n, L, log2_n1, log2_n2, key_first, msg_seed):
    from oracle import oracle as O
    prm = O.Params(inst, log2_n1, log2_n2)
    arr = synthlog.messages_fixed(msg_seed, n, L)
    msgs = [bytes(r) for r in arr]
    pk, sigs, ds, tag, _ = O.sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    return prm, arr, msgs, pk, sigs, ds, tag


@pytest.mark.parametrize("inst", [1, 0])
def test_host_batches_equal_device_and_oracle(P, O, gpu, inst):
    torch, ctx = gpu
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, 700, 48, 4, 6, 0x71, 51)
    params = P.make_params(inst, 4, 6)
    want_e = O.ekeys_sum(prm, msgs, 0, ds)
    dev = torch.from_numpy(arr.copy()).cuda()
    for pin in (True, False):
        h = torch.from_numpy(arr.copy())
        if pin:
            h = h.pin_memory()
        print(f"inst {inst} pinned {pin}", flush=True)
        got = P.poslo_aver(ctx, params, pk, P.make_msgs(h), ds, tag)
        assert got == P.poslo_aver(ctx, params, pk, P.make_msgs(dev), ds, tag)
        assert got[0] and int.from_bytes(got[1], "little") == want_e
        # offsets in host memory too
        hf = h.reshape(-1)
        ho = torch.from_numpy(np.arange(0, arr.size + 1, 48, dtype=np.int64))
        assert P.poslo_aver(ctx, params, pk, P.make_msgs(hf, ho), ds, tag) == got
        eg, xg = P.poslo_ekeys(ctx, params, P.make_msgs(h), ds)
        ed, xd = P.poslo_ekeys(ctx, params, P.make_msgs(dev), ds)
        assert torch.equal(eg, ed) and torch.equal(xg, xd)
    # Distill of a host batch with host signatures
    plan = synthlog.corruption_plan(52, 700, 5, 8 * (48 + 80))
    cm, cs = list(msgs), list(sigs)
    for e, bit in plan:
        blob = bytearray(cm[e] + cs[e])
        blob[bit // 8] ^= 1 << (bit % 8)
        cm[e], cs[e] = bytes(blob[:48]), bytes(blob[48:])
    want = O.distill(prm, pk, cm, cs, 0, ds, 3)
    hm = torch.from_numpy(np.frombuffer(b"".join(cm), dtype=np.uint8).reshape(700, 48).copy()).pin_memory()
    hs = torch.from_numpy(np.frombuffer(b"".join(cs), dtype=np.uint8).copy()).pin_memory()
    ccd = P.poslo_distill(ctx, params, pk, P.make_msgs(hm), hs, ds, 3)
    assert ccd.invalid() == [t for t, _ in want.invalid]
    assert ccd.valid_tag() == want.valid_tag
    assert ccd.umbrellas()[0] == [u for u, _ in want.umbrellas]
    for mode in "VUI":
        assert P.poslo_sebver(ctx, params, pk, P.make_msgs(hm), ccd, mode) == O.sebver(prm, pk, cm, want, mode)


def test_host_posloc_aver(P, O, gpu):
    torch, ctx = gpu
    prm = O.Params(1, 3, 4)
    msgs = [bytes(r) for r in synthlog.messages_fixed(53, 5 * 16, 40)]
    pk, s_list, ds, _ = O.posloc_sign_batch(prm, synthlog.key_seed_bytes(0x72), msgs)
    params = P.make_params(1, 3, 4)
    key = P.poslo_c_key_load(ctx, params, pk)
    h = torch.from_numpy(np.frombuffer(b"".join(msgs), dtype=np.uint8).reshape(80, 40).copy()).pin_memory()
    acc, e = P.poslo_c_aver(ctx, params, key, P.make_msgs(h), ds, O.posloc_agg_s(s_list))
    assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)


@pytest.mark.parametrize("inst", [1, 0])
def test_audit_chunks_resume_and_errors(P, O, gpu, inst):
    torch, ctx = gpu
    n, L = 3000, 48
    prm, arr, msgs, pk, sigs, ds, tag = signed(inst, n, L, 6, 6, 0x73, 54)
    params = P.make_params(inst, 6, 6)
    dev = torch.from_numpy(arr.copy()).cuda()
    host = torch.from_numpy(arr.copy()).pin_memory()
    # uneven chunks, the first starting at entry 100 (mid-epoch), host and
    # device chunks alternating
    cuts = [100, 101, 230, 1024, 1025, 1900, 2999, 3000]
    t0 = cuts[0]
    sub_tag = O.agg(sigs[t0:])
    want_e = O.ekeys_sum(prm, msgs[t0:], t0, ds)
    au = P.poslo_audit_begin(ctx, params, pk, ds, t0)
    state = None
    for k, (a, b) in enumerate(zip(cuts, cuts[1:])):
        src = host if k % 2 == 0 else dev
        au.feed(P.make_msgs(src[a:b], t0=a))
        assert au.position() == b
        if b == 1024:
            state = au.export()
    acc, e = au.finish(sub_tag)
    assert acc and int.from_bytes(e, "little") == want_e
    # a tampered tag is rejected; the audit can go on after a finish
    bad = bytearray(sub_tag)
    bad[5] ^= 1
    assert not au.finish(bytes(bad))[0]
    au.close()
    # resume from the state after entry 1023 and feed the rest in one chunk
    au2 = P.poslo_audit_resume(ctx, state, params)
    assert au2.position() == 1024
    au2.feed(P.make_msgs(host[1024:], t0=1024))
    assert au2.finish(sub_tag) == (True, e)
    # misuse: a chunk that does not continue the log, a state for other
    # parameters, a ds that does not cover the chunk
    with pytest.raises(P.PosloError) as ei:
        au2.feed(P.make_msgs(dev[:10], t0=5))
    assert ei.value.status == P.POSLO_E_INVAL
    with pytest.raises(P.PosloError):
        P.poslo_audit_resume(ctx, state, P.make_params(inst, 6, 5))
    with pytest.raises(P.PosloError):
        P.poslo_audit_resume(ctx, state[:-1], params)
    short_ds = O.ds_encode(O.signer_at(prm, synthlog.key_seed_bytes(0x73), 64).ds)
    au3 = P.poslo_audit_begin(ctx, params, pk, short_ds, 0)
    with pytest.raises(P.PosloError) as ei:
        au3.feed(P.make_msgs(dev[:200]))
    assert ei.value.status == P.POSLO_E_SEED


@pytest.mark.parametrize("inst", [1, 0])
def test_full_size_audit_from_pinned_host(P, gpu, inst):
    import oracle_fullsize as F
    from test_gpu_fullsize import FLIP_SEED, K_FLIPS, KEY_FIRST, L, LOG2_N1, LOG2_N2, MSG_SEED, N, N_U
    torch, ctx = gpu
    c = F.full_case(inst, N, L, LOG2_N1, LOG2_N2, KEY_FIRST, MSG_SEED, N_U, FLIP_SEED, K_FLIPS)
    params = P.make_params(inst, LOG2_N1, LOG2_N2)
    host = torch.from_numpy(c.msgs).pin_memory()
    au = P.poslo_audit_begin(ctx, params, c.pk, c.ds, 0)
    step = N // 8
    for a in range(0, N, step):
        au.feed(P.make_msgs(host[a:a + step], t0=a))
    acc, e = au.finish(c.tag)
    assert acc is True and int.from_bytes(e, "little") == c.e
