"""GPU parity of the parameter variants against the oracle, through the C
ABI: kappa = 127 (tree PRF in one AES block, every PRF output mod 2^127)
under POSLO+ and POSLO++, and POSLO++ (H = Add_q, messages of at most 31
bytes) at kappa = 128.

Covered: AVer and the allocation-free AVer, per-entry e_t and x_t, every
POSLO++ message layout of the hot kernel (16-byte aligned, 4-byte aligned,
any; n2 >= 64 with scalar round keys and smaller epochs), batches starting
mid-epoch and mid-wave-unit, Distill and SeBVer V/U/I, POSLO-C, the
streaming audit, the device signer, and the errors the variants add
(longer messages, a kappa = 127 ds node with bit 127 set, the multi-signer
paths that take kappa = 128 POSLO and POSLO+ only).  Keys, signatures, ds
and tags come from the oracle's signer."""

import functools

import numpy as np
import pytest

import synthlog

pytestmark = pytest.mark.gpu

AES127, ADDQ, ADDQ127 = 1 | 4, 2, 2 | 4
NAMES = {AES127: "aes-k127", ADDQ: "addq", ADDQ127: "addq-k127"}


@pytest.fixture(scope="module")
def gpu(P):
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    ctx = P.poslo_ctx_create(0)
    yield torch, ctx
    ctx.close()


@functools.lru_cache(maxsize=None)
def signed(inst, lens, log2_n1, log2_n2, key_first, msg_seed, n=None):
    """Oracle-signed batch.  lens: an int (fixed length, n entries) or a
    tuple of lengths."""
    from oracle import oracle as O
    prm = O.Params(inst, log2_n1, log2_n2)
    if isinstance(lens, int):
        msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, n, lens)]
    else:
        data, off = synthlog.messages_var(msg_seed, np.array(lens))
        msgs = [bytes(data[off[k]:off[k + 1]]) for k in range(len(lens))]
    pk, sigs, ds, tag, _ = O.sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    return prm, msgs, pk, sigs, ds, tag


def upload(torch, msgs, fixed, pad_front=0):
    """Messages as a CUDA tensor (fixed: (n, L)); pad_front shifts the data
    off 16-byte alignment."""
    flat = np.frombuffer(b"".join(msgs), dtype=np.uint8) if msgs else np.zeros(0, np.uint8)
    if fixed:
        L = len(msgs[0]) if msgs else 0
        if pad_front:
            buf = torch.zeros(pad_front + flat.size, dtype=torch.uint8, device="cuda")
            buf[pad_front:] = torch.from_numpy(flat.copy()).cuda()
            return buf[pad_front:].view(len(msgs), L), None
        return torch.from_numpy(flat.copy().reshape(len(msgs), L)).cuda(), None
    off = np.zeros(len(msgs) + 1, dtype=np.int64)
    np.cumsum([len(m) for m in msgs], out=off[1:])
    return torch.from_numpy(flat.copy()).cuda(), torch.from_numpy(off).cuda()


CASES = [
    # inst, n, L, log2_n1, log2_n2, pad
    (AES127, 777, 48, 4, 6, 0),   # fast AES path, ragged tail, multi-node ds
    (AES127, 300, 37, 4, 5, 0),   # any-layout AES path
    (ADDQ, 1100, 16, 3, 8, 0),    # 16-byte aligned messages, scalar round keys
    (ADDQ127, 1100, 16, 3, 8, 0),
    (ADDQ, 777, 31, 4, 6, 0),     # any layout, n2 = 64 (one epoch per unit)
    (ADDQ127, 500, 12, 5, 4, 0),  # 4-byte aligned, n2 = 16 (per-lane keys)
    (ADDQ, 300, 16, 4, 5, 3),     # 16-byte messages off alignment: any layout
    (ADDQ, 300, 0, 4, 5, 0),      # empty messages: e_t = x_t
    (ADDQ127, 64, 31, 1, 5, 0),   # n2 = 32
    (ADDQ127, 7, 20, 3, 0, 0),    # n2 = 1
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{NAMES[c[0]]}-n{c[1]}-L{c[2]}-n1_{c[3]}-n2_{c[4]}-p{c[5]}")
def test_aver_and_ekeys_parity(P, gpu, case):
    from oracle import oracle as O
    torch, ctx = gpu
    inst, n, L, l1, l2, pad = case
    prm, msgs, pk, sigs, ds, tag = signed(inst, L, l1, l2, 0x31, 2, n)
    params = P.make_params(inst, l1, l2)
    d, _ = upload(torch, msgs, True, pad)
    m = P.make_msgs(d)
    print(f"case {case}: aver", flush=True)
    acc, e = P.poslo_aver(ctx, params, pk, m, ds, tag)
    want_e = O.ekeys_sum(prm, msgs, 0, ds)
    assert acc and int.from_bytes(e, "little") == want_e
    P.poslo_ctx_keys_load(ctx, [pk])
    assert P.poslo_aver_fixed(ctx, params, pk, m, ds, tag) == (True, e)
    eg, xg = P.poslo_ekeys(ctx, params, m, ds)
    eg, xg = eg.cpu().numpy(), xg.cpu().numpy()
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, n)
    for t in range(n):
        x = O.one_time_seed(inst, seeds[t >> l2], t & ((1 << l2) - 1))
        assert bytes(xg[t]) == x == sigs[t][64:80], t
        assert int.from_bytes(bytes(eg[t]), "little") == O.digest_int(inst, msgs[t], x) % O.Q, t
    bad = bytearray(tag)
    bad[40] ^= 0x10
    assert not P.poslo_aver(ctx, params, pk, m, ds, bytes(bad))[0]
    if L:
        mm = list(msgs)
        k = n // 2
        mm[k] = mm[k][:-1] + bytes([mm[k][-1] ^ 0x80])  # the message's top bit
        d2, _ = upload(torch, mm, True, pad)
        assert not P.poslo_aver(ctx, params, pk, P.make_msgs(d2), ds, tag)[0]


@pytest.mark.parametrize("inst", [AES127, ADDQ, ADDQ127], ids=lambda i: NAMES[i])
def test_variable_length_and_slices(P, gpu, inst):
    from oracle import oracle as O
    torch, ctx = gpu
    hi = 90 if inst == AES127 else 31
    lens = tuple(synthlog.uniform_ints(33, 0, 700, 0, hi))
    prm, msgs, pk, sigs, ds, tag = signed(inst, lens, 4, 6, 0x32, 6)
    params = P.make_params(inst, 4, 6)
    d, off = upload(torch, msgs, False)
    acc, e = P.poslo_aver(ctx, params, pk, P.make_msgs(d, off), ds, tag)
    assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)
    # slices starting mid-epoch and mid-unit of 64 positions, and one that
    # starts at a unit boundary inside an epoch
    for a, b in ((37, 600), (128, 193), (1, 2)):
        sub = msgs[a:b]
        d3, off3 = upload(torch, sub, False)
        acc, e = P.poslo_aver(ctx, params, pk, P.make_msgs(d3, off3, t0=a), ds, O.agg(sigs[a:b]))
        assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, sub, a, ds), (a, b)
        eg, _ = P.poslo_ekeys(ctx, params, P.make_msgs(d3, off3, t0=a), ds)
        eg = eg.cpu().numpy()
        seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, b)
        for k, t in enumerate(range(a, b)):
            x = O.one_time_seed(inst, seeds[t >> 6], t & 63)
            assert int.from_bytes(bytes(eg[k]), "little") == O.digest_int(inst, msgs[t], x) % O.Q, t


def test_addq_long_messages_are_errors(P, gpu):
    from oracle import oracle as O
    torch, ctx = gpu
    lens = tuple(synthlog.uniform_ints(34, 0, 300, 0, 31))
    prm, msgs, pk, sigs, ds, tag = signed(ADDQ, lens, 4, 5, 0x33, 7)
    params = P.make_params(ADDQ, 4, 5)
    # one message of 32 bytes in an offsets batch: found by the kernels
    long = list(msgs)
    long[150] = bytes(range(32))
    d, off = upload(torch, long, False)
    m = P.make_msgs(d, off)
    dsig = torch.from_numpy(np.frombuffer(b"".join(sigs), np.uint8).copy()).cuda()
    P.poslo_ctx_keys_load(ctx, [pk])
    calls = {
        "aver": lambda: P.poslo_aver(ctx, params, pk, m, ds, tag),
        "aver_fixed": lambda: P.poslo_aver_fixed(ctx, params, pk, m, ds, tag),
        "distill": lambda: P.poslo_distill(ctx, params, pk, m, dsig, ds, 4),
    }
    for name, call in calls.items():
        with pytest.raises(P.PosloError) as ei:
            call()
        assert ei.value.status == P.POSLO_E_INVAL, name
    eg, _ = P.poslo_ekeys(ctx, params, m, ds)
    assert bytes(eg[150].cpu().numpy()) == b"\xff" * 32
    # the flag does not outlive the call: the honest batch verifies again
    d, off = upload(torch, msgs, False)
    acc, e = P.poslo_aver(ctx, params, pk, P.make_msgs(d, off), ds, tag)
    assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)
    # a fixed length above 31 bytes is refused on the host
    d32 = torch.zeros((64, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(P.PosloError) as ei:
        P.poslo_aver(ctx, params, pk, P.make_msgs(d32), ds, tag)
    assert ei.value.status == P.POSLO_E_INVAL


@pytest.mark.parametrize("inst", [AES127, ADDQ127], ids=lambda i: NAMES[i])
def test_kappa127_ds_node_with_bit_127_is_an_error(P, gpu, inst):
    from oracle import oracle as O
    torch, ctx = gpu
    L = 48 if inst == AES127 else 24
    prm, msgs, pk, sigs, ds, tag = signed(inst, L, 4, 6, 0x31, 2, 777)
    params = P.make_params(inst, 4, 6)
    nodes = O.ds_decode(ds)
    k = next(i for i, nd in enumerate(nodes) if nd.depth > 0)
    raw = bytearray(ds)
    raw[1 + 24 * k + 8 + 15] |= 0x80
    # a batch of the first epoch below node k (messages unsigned: the ds is
    # refused before any hashing; with the honest ds it is a plain reject)
    first = nodes[k].index << nodes[k].depth
    d = torch.zeros((64, L), dtype=torch.uint8, device="cuda")
    m = P.make_msgs(d, t0=first * 64)
    assert not P.poslo_aver(ctx, params, pk, m, ds, tag)[0]
    with pytest.raises(P.PosloError) as ei:
        P.poslo_aver(ctx, params, pk, m, bytes(raw), tag)
    assert ei.value.status == P.POSLO_E_INVAL
    # a node at depth 0 is the epoch seed itself, used without a tree PRF call
    k0 = next((i for i, nd in enumerate(nodes) if nd.depth == 0), None)
    if k0 is not None:
        raw0 = bytearray(ds)
        raw0[1 + 24 * k0 + 8 + 15] |= 0x80
        m0 = P.make_msgs(torch.zeros((64, L), dtype=torch.uint8, device="cuda"), t0=nodes[k0].index * 64)
        assert not P.poslo_aver(ctx, params, pk, m0, bytes(raw0), tag)[0]


def corrupt(msgs, sigs, plan):
    cm, cs = list(msgs), list(sigs)
    for t, bit in plan:
        L = len(cm[t])
        if bit < 8 * L:
            b = bytearray(cm[t])
            b[bit // 8] ^= 1 << (bit % 8)
            cm[t] = bytes(b)
        else:
            b = bytearray(cs[t])
            bb = bit - 8 * L
            b[bb // 8] ^= 1 << (bb % 8)
            cs[t] = bytes(b)
    return cm, cs


DISTILL_CASES = [
    # inst, n, L, log2_n1, log2_n2, corrupted, umbrellas
    (AES127, 200, 40, 4, 4, 7, 5),
    (ADDQ, 200, 20, 4, 4, 7, 5),
    (ADDQ127, 129, 31, 4, 4, 9, 3),
    (ADDQ, 64, 16, 3, 3, 11, 64),
]


@pytest.mark.parametrize("case", DISTILL_CASES, ids=lambda c: f"{NAMES[c[0]]}-n{c[1]}-L{c[2]}-k{c[5]}-u{c[6]}")
def test_distill_and_sebver_match_oracle(P, gpu, case):
    from oracle import oracle as O
    torch, ctx = gpu
    inst, n, L, l1, l2, k, nu = case
    prm, msgs, pk, sigs, ds, tag = signed(inst, L, l1, l2, 0x34, 8, n)
    plan = synthlog.corruption_plan(60 + k, n, k, 8 * (L + 80))
    cm, cs = corrupt(msgs, sigs, plan)
    params = P.make_params(inst, l1, l2)
    dm, _ = upload(torch, cm, True)
    dsig = torch.from_numpy(np.frombuffer(b"".join(cs), dtype=np.uint8).copy()).cuda()
    print(f"case {case}: distill", flush=True)
    ccd = P.poslo_distill(ctx, params, pk, P.make_msgs(dm), dsig, ds, nu)
    want = O.distill(prm, pk, cm, cs, 0, ds, nu)
    assert ccd.invalid() == [t for t, _ in want.invalid] == sorted(e for e, _ in plan)
    assert ccd.valid_tag() == want.valid_tag
    tags, span = ccd.umbrellas()
    assert span == want.span and tags == [t for t, _ in want.umbrellas]
    m = P.make_msgs(dm)
    for mode in "VUI":
        assert P.poslo_sebver(ctx, params, pk, m, ccd, mode) == O.sebver(prm, pk, cm, want, mode), mode


C_CASES = [
    # inst, epochs, L, log2_n1, log2_n2
    (AES127, 6, 48, 3, 4),
    (ADDQ, 6, 24, 3, 4),
    (ADDQ127, 5, 31, 3, 3),
    (ADDQ, 4, 16, 3, 6),
]


@pytest.mark.parametrize("case", C_CASES, ids=lambda c: f"{NAMES[c[0]]}-k{c[1]}-L{c[2]}-n2_{c[4]}")
def test_posloc_matches_oracle(P, gpu, case):
    from oracle import oracle as O
    torch, ctx = gpu
    inst, k, L, l1, l2 = case
    prm = O.Params(inst, l1, l2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(43, k * prm.n2, L)]
    pk, s_list, ds, _ = O.posloc_sign_batch(prm, synthlog.key_seed_bytes(0x35), msgs)
    params = P.make_params(inst, l1, l2)
    key = P.poslo_c_key_load(ctx, params, pk)
    for fixed in (True, False):
        d, off = upload(torch, msgs, fixed)
        m = P.make_msgs(d, off)
        acc, e = P.poslo_c_aver(ctx, params, key, m, ds, O.posloc_agg_s(s_list))
        assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)
    n2 = prm.n2
    cm, cs = list(msgs), list(s_list)
    mm = bytearray(cm[n2 + n2 // 2])
    mm[0] ^= 0x08
    cm[n2 + n2 // 2] = bytes(mm)
    want = O.posloc_distill(prm, pk, cm, cs, 0, ds, 2)
    assert [i for i, _ in want.invalid] == [1]
    d, off = upload(torch, cm, False)
    m = P.make_msgs(d, off)
    ccd = P.poslo_c_distill(ctx, params, key, m, b"".join(cs), ds, 2)
    assert ccd.invalid() == [1] and ccd.valid_tag() == want.valid_tag
    for mode in "VUI":
        assert P.poslo_c_sebver(ctx, params, key, m, ccd, mode) == O.posloc_sebver(prm, pk, cm, want, mode)


@pytest.mark.parametrize("inst", [ADDQ, ADDQ127], ids=lambda i: NAMES[i])
def test_audit_chunks(P, O, gpu, inst):
    torch, ctx = gpu
    lens = tuple(synthlog.uniform_ints(35, 0, 1500, 0, 31))
    prm, msgs, pk, sigs, ds, tag = signed(inst, lens, 5, 6, 0x36, 9)
    params = P.make_params(inst, 5, 6)
    cuts = [0, 100, 101, 640, 1499, 1500]
    au = P.poslo_audit_begin(ctx, params, pk, ds, 0)
    for a, b in zip(cuts, cuts[1:]):
        d, off = upload(torch, msgs[a:b], False)
        au.feed(P.make_msgs(d, off, t0=a))
    acc, e = au.finish(tag)
    assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)
    # a chunk with a 32-byte message poisons the audit: finish and export fail
    d, off = upload(torch, [bytes(32)], False)
    au.close()
    au2 = P.poslo_audit_begin(ctx, params, pk, ds, 0)
    d0, off0 = upload(torch, msgs[:100], False)
    au2.feed(P.make_msgs(d0, off0))
    au2.feed(P.make_msgs(d, off, t0=100))
    with pytest.raises(P.PosloError) as ei:
        au2.finish(tag)
    assert ei.value.status == P.POSLO_E_INVAL
    with pytest.raises(P.PosloError):
        au2.export()
    au2.close()


@pytest.mark.parametrize("inst", [AES127, ADDQ, ADDQ127], ids=lambda i: NAMES[i])
def test_device_signer_matches_host_signer(P, gpu, inst):
    torch, ctx = gpu
    params = P.make_params(inst, 4, 5)
    seeds = [synthlog.key_seed_bytes(0x37 + k) for k in range(2)]
    keys = P.poslo_gpu_keys_create(ctx, params, seeds)
    hi = 70 if inst == AES127 else 31
    lens = synthlog.uniform_ints(36, 0, 300, 0, hi)
    data, off = synthlog.messages_var(11, np.array(lens))
    d = torch.from_numpy(data.copy()).cuda()
    o = torch.from_numpy(off.astype(np.int64)).cuda()
    sigs = torch.zeros(300 * 80, dtype=torch.uint8, device="cuda")
    jobs = [(0, 0, 180, 0), (1, 33, 120, 180)]
    tags, dss = P.poslo_gpu_sign(keys, jobs, d, o, sigs)
    got = sigs.cpu().numpy().reshape(300, 80)
    for k, (key, t0, n, base) in enumerate(jobs):
        sk, pk = P.poslo_kg(params, seeds[key])
        assert pk == keys.pks[key]
        if t0:
            P.poslo_sig_batch(sk, np.zeros((t0, 1), np.uint8))  # advance to t0
        want = P.poslo_sig_batch(sk, data[off[base]:off[base + n]], offsets=off[base:base + n + 1] - off[base])
        assert got[base:base + n].tobytes() == want.tobytes(), k
        assert tags[k] == P.poslo_agg(want.tobytes())
        assert dss[k] == P.poslo_ds_export(sk)
    if inst & 3 == 2:
        lens2 = list(lens)
        lens2[7] = 32
        data2, off2 = synthlog.messages_var(12, np.array(lens2))
        with pytest.raises(P.PosloError) as ei:
            P.poslo_gpu_sign(keys, [(0, 0, 300, 0)], torch.from_numpy(data2.copy()).cuda(),
                             torch.from_numpy(off2.astype(np.int64)).cuda(), sigs)
        assert ei.value.status == P.POSLO_E_INVAL


@pytest.mark.parametrize("inst", [AES127, ADDQ], ids=lambda i: NAMES[i])
def test_multi_signer_paths_refuse_variants(P, gpu, inst):
    torch, ctx = gpu
    params = P.make_params(inst, 2, 4)
    prm, msgs, pk, sigs, ds, tag = signed(inst, 16, 2, 4, 0x38, 3, 20)
    d, off = upload(torch, msgs, False)
    jobs = P.BatchJobs([dict(pk=pk, ds=ds, tag=tag, t0=0, n=20, entry_base=0)])
    with pytest.raises(P.PosloError) as ei:
        P.poslo_verify_batch(ctx, params, jobs, d, off)
    assert ei.value.status == P.POSLO_E_INVAL
    with pytest.raises(P.PosloError) as ei:
        P.Server(0, params)
    assert ei.value.status == P.POSLO_E_INVAL
