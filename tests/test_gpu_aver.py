"""GPU parity of aggregate verification (AVer) and per-entry digests against
the oracle, through the C ABI.

Inputs are seeded synthetic messages; keys, signatures, ds and tags for the
small cases come from the oracle's own signer.  The full 2^20 x 256-byte
configuration is compared with the oracle over the whole batch in
test_gpu_fullsize.py."""

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
def oracle_case(inst, n, lens, log2_n1, log2_n2, key_first, msg_seed):
    """Oracle-signed batch.  lens: an int (fixed) or a tuple (variable)."""
    from oracle import oracle as O
    prm = O.Params(inst, log2_n1, log2_n2)
    if isinstance(lens, int):
        arr = synthlog.messages_fixed(msg_seed, n, lens)
        msgs = [bytes(r) for r in arr]
    else:
        data, off = synthlog.messages_var(msg_seed, np.array(lens))
        msgs = [bytes(data[off[k]:off[k + 1]]) for k in range(n)]
    pk, sigs, ds, tag, _ = O.sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    return prm, msgs, pk, sigs, ds, tag


def upload(torch, msgs, fixed):
    if fixed:
        L = len(msgs[0]) if msgs else 0
        arr = np.frombuffer(b"".join(msgs), dtype=np.uint8).reshape(len(msgs), L)
        return torch.from_numpy(arr.copy()).cuda(), None
    flat = np.frombuffer(b"".join(msgs), dtype=np.uint8) if msgs else np.zeros(0, np.uint8)
    off = np.zeros(len(msgs) + 1, dtype=np.int64)
    np.cumsum([len(m) for m in msgs], out=off[1:])
    return torch.from_numpy(flat.copy()).cuda(), torch.from_numpy(off).cuda()


CASES = [
    # inst, n, lens, log2_n1, log2_n2 : the first two are the 1,024 x 32-byte
    # configuration at n2 = 256 (both instantiations)
    (1, 1024, 32, 2, 8),
    (0, 1024, 32, 2, 8),
    (1, 777, 48, 4, 6),    # ragged tail, multi-node ds, fast AES path
    (1, 300, 37, 4, 5),    # length not a multiple of 16: generic path
    (0, 300, 37, 4, 5),    # length not a multiple of 4: generic SHA path
    (0, 519, 64, 6, 4),    # SHA fast path, several SHA blocks
    (1, 1, 256, 1, 0),     # single entry, n2 = 1
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"inst{c[0]}-n{c[1]}-L{c[2]}-n1_{c[3]}-n2_{c[4]}")
def test_aver_and_ekeys_parity(P, gpu, case):
    from oracle import oracle as O
    torch, ctx = gpu
    inst, n, L, l1, l2 = case
    prm, msgs, pk, sigs, ds, tag = oracle_case(inst, n, L, l1, l2, 0, 1)
    params = P.make_params(inst, l1, l2)
    d, off = upload(torch, msgs, True)
    m = P.make_msgs(d)
    print(f"case {case}: aver", flush=True)
    acc, e = P.poslo_aver(ctx, params, pk, m, ds, tag)
    assert acc
    assert int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)
    # per-entry digests and one-time seeds
    eg, xg = P.poslo_ekeys(ctx, params, m, ds)
    eg, xg = eg.cpu().numpy(), xg.cpu().numpy()
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, n)
    for t in range(n):
        x = O.one_time_seed(inst, seeds[t >> l2], t & ((1 << l2) - 1))
        assert bytes(xg[t]) == x == sigs[t][64:80], t
        assert int.from_bytes(bytes(eg[t]), "little") == O.digest_int(inst, msgs[t], x) % O.Q, t
    # a flipped tag bit and a flipped message bit are rejected
    bad = bytearray(tag)
    bad[40] ^= 0x10
    assert not P.poslo_aver(ctx, params, pk, m, ds, bytes(bad))[0]
    mm = list(msgs)
    k = n // 2
    mm[k] = bytes([mm[k][0] ^ 1]) + mm[k][1:]
    d2, _ = upload(torch, mm, True)
    assert not P.poslo_aver(ctx, params, pk, P.make_msgs(d2), ds, tag)[0]


@pytest.mark.parametrize("inst", [0, 1])
def test_variable_length_and_slices(P, gpu, inst):
    from oracle import oracle as O
    torch, ctx = gpu
    lens = tuple(synthlog.uniform_ints(31, 0, 203, 0, 90))
    prm, msgs, pk, sigs, ds, tag = oracle_case(inst, 203, lens, 4, 4, 3, 5)
    params = P.make_params(inst, 4, 4)
    d, off = upload(torch, msgs, False)
    acc, e = P.poslo_aver(ctx, params, pk, P.make_msgs(d, off), ds, tag)
    assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, 0, ds)
    # a slice starting mid-epoch verifies against its own aggregate
    a, b = 37, 160
    sub = msgs[a:b]
    d3, off3 = upload(torch, sub, False)
    acc, e = P.poslo_aver(ctx, params, pk, P.make_msgs(d3, off3, t0=a), ds, O.agg(sigs[a:b]))
    assert acc and int.from_bytes(e, "little") == O.ekeys_sum(prm, sub, a, ds)


def test_empty_batch_and_errors(P, gpu):
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, pk, sigs, ds, tag = oracle_case(1, 777, 48, 4, 6, 0, 1)
    params = P.make_params(1, 4, 6)
    empty = torch.zeros((0, 48), dtype=torch.uint8, device="cuda")
    acc, e = P.poslo_aver(ctx, params, pk, P.make_msgs(empty), ds, O.agg([]))
    assert acc and e == bytes(32)
    # ds after entry 776 covers epochs 0..12; entries of epoch 13 are not covered
    d, _ = upload(torch, msgs[:64], True)
    with pytest.raises(P.PosloError) as ei:
        P.poslo_aver(ctx, params, pk, P.make_msgs(d, t0=13 * 64), ds, tag)
    assert ei.value.status == P.POSLO_E_SEED
    # a public key that is not a point encoding is an error, not a reject
    badpk = (2 ** 255 - 19 + 3).to_bytes(32, "little")
    d, _ = upload(torch, msgs, True)
    with pytest.raises(P.PosloError) as ei:
        P.poslo_aver(ctx, params, badpk, P.make_msgs(d), ds, tag)
    assert ei.value.status == P.POSLO_E_ENCODING
    # a malformed ds is an invalid argument
    with pytest.raises(P.PosloError):
        P.poslo_aver(ctx, params, pk, P.make_msgs(d), ds + b"\0", tag)


def test_every_tuning_variant_agrees(P, gpu):
    """Every hot-kernel variant and grid shape gives the same aggregate."""
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, pk, sigs, ds, tag = oracle_case(1, 777, 48, 4, 6, 0, 1)
    params = P.make_params(1, 4, 6)
    d, _ = upload(torch, msgs, True)
    want = O.ekeys_sum(prm, msgs, 0, ds)
    try:
        for v in range(P.poslo_agg_variant_count()):
            for wg in (0, 1):
                print(f"variant {P.poslo_agg_variant_name(v)} wg {wg}", flush=True)
                P.poslo_ctx_set_tuning(ctx, v, wg)
                acc, e = P.poslo_aver(ctx, params, pk, P.make_msgs(d), ds, tag)
                assert acc and int.from_bytes(e, "little") == want, P.poslo_agg_variant_name(v)
    finally:
        P.poslo_ctx_set_tuning(ctx, -1, 0)


def test_kernel_timing_mask(P, gpu):
    """Only the kernels named in the profile mask are timed."""
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, pk, sigs, ds, tag = oracle_case(1, 777, 48, 4, 6, 0, 1)
    params = P.make_params(1, 4, 6)
    d, _ = upload(torch, msgs, True)
    for k in range(8):
        P.poslo_ctx_kernel_time(ctx, k, reset=True)
    P.poslo_ctx_profile(ctx, [P.POSLO_KT_AGG])
    try:
        for _ in range(3):
            acc, _ = P.poslo_aver(ctx, params, pk, P.make_msgs(d), ds, tag)
            assert acc
    finally:
        P.poslo_ctx_profile(ctx, False)
    ms, n = P.poslo_ctx_kernel_time(ctx, P.POSLO_KT_AGG, reset=True)
    assert n == 3 and ms > 0
    for k in (P.POSLO_KT_SEED, P.POSLO_KT_FINAL):
        assert P.poslo_ctx_kernel_time(ctx, k, reset=True) == (0.0, 0)
    P.poslo_ctx_profile(ctx, True)
    try:
        P.poslo_aver(ctx, params, pk, P.make_msgs(d), ds, tag)
    finally:
        P.poslo_ctx_profile(ctx, False)
    for k in (P.POSLO_KT_SEED, P.POSLO_KT_AGG, P.POSLO_KT_FINAL):
        assert P.poslo_ctx_kernel_time(ctx, k, reset=True)[1] == 1
    with pytest.raises(P.PosloError):
        P.poslo_ctx_profile(ctx, [9])


def test_aggregate_check_scalar_extremes(P, gpu):
    """Tags whose s sits at the edges of the signed comb digits (0, digits of
    128 / 129, q - 1, 2^252, ...), with R = e*Y + s*G computed by the oracle
    for the batch's own e: the single-batch check (the block-wide quad tree)
    and the per-job check of the multi-signer path must accept exactly where
    the oracle does, and reject R + G and s >= q."""
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, pk, sigs, ds, tag = oracle_case(1, 777, 48, 4, 6, 0, 1)
    params = P.make_params(1, 4, 6)
    d, _ = upload(torch, msgs, True)
    q = O.Q
    e = O.ekeys_sum(prm, msgs, 0, ds) % q
    Y = O.decode(pk)
    eY = O.scalar_mult(e, Y)
    rep8 = sum(0x80 << (8 * k) for k in range(31))
    special = [0, 1, 127, 128, 129, 255, 256, q - 1, q - 2, q - 128, 2 ** 252, 2 ** 252 - 1, rep8, rep8 + 1,
               (rep8 ^ (rep8 >> 1)) % q]
    tags, want = [], []
    for s in special:
        R = O.point_add(eY, O.scalar_mult(s, O.G))
        tags.append(O.to32(s) + O.encode(R))
        tags.append(O.to32(s) + O.encode(O.point_add(R, O.G)))
    # s = q: R equals e*Y + s*G on the curve, but s is not canonical
    tags.append(O.to32(q) + O.encode(eY))
    want = [O.aggregate_check(pk, e, t) for t in tags]
    assert want == [True, False] * len(special) + [False]
    got = [P.poslo_aver(ctx, params, pk, P.make_msgs(d), ds, t)[0] for t in tags]
    assert got == want
    n = len(msgs)
    bj = P.BatchJobs([dict(pk=pk, ds=ds, tag=t, t0=0, n=n, entry_base=k * n) for k, t in enumerate(tags)])
    base = np.frombuffer(b"".join(msgs), dtype=np.uint8)
    flat = torch.from_numpy(np.tile(base, len(tags))).cuda()
    L = len(msgs[0])
    # job k reads its own copy of the messages, entries k * n .. k * n + n - 1
    off = torch.arange(0, len(tags) * n * L + 1, L, dtype=torch.int64, device="cuda")
    acc, _ = P.poslo_verify_batch(ctx, params, bj, flat, off)
    assert acc == want


def test_aggregate_check_doubling_and_cancelling(P, gpu):
    """With Y = G, s = e makes every first-level addition of the check's tree
    a doubling (window w of e on Y's table meets window w of s on G's), and
    s = q - e makes every one cancel to the identity; the complete addition
    law (and its quad-split, scaled form) must handle both.  R comes from the
    oracle; R + G must be rejected."""
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, _, _, ds, _ = oracle_case(1, 777, 48, 4, 6, 0, 1)
    params = P.make_params(1, 4, 6)
    d, _ = upload(torch, msgs, True)
    q = O.Q
    e = O.ekeys_sum(prm, msgs, 0, ds) % q
    pk = O.encode(O.G)
    tags = []
    for s in (e, (q - e) % q, 0):
        R = O.scalar_mult((e + s) % q, O.G)
        tags.append(O.to32(s) + O.encode(R))
        tags.append(O.to32(s) + O.encode(O.point_add(R, O.G)))
    want = [O.aggregate_check(pk, e, t) for t in tags]
    assert want == [True, False] * 3
    assert tags[2][32:] == (1).to_bytes(32, "little")  # s = q - e: R is the identity
    got = [P.poslo_aver(ctx, params, pk, P.make_msgs(d), ds, t)[0] for t in tags]
    assert got == want
    n, L = len(msgs), len(msgs[0])
    bj = P.BatchJobs([dict(pk=pk, ds=ds, tag=t, t0=0, n=n, entry_base=k * n) for k, t in enumerate(tags)])
    flat = torch.from_numpy(np.tile(np.frombuffer(b"".join(msgs), dtype=np.uint8), len(tags))).cuda()
    off = torch.arange(0, len(tags) * n * L + 1, L, dtype=torch.int64, device="cuda")
    acc, _ = P.poslo_verify_batch(ctx, params, bj, flat, off)
    assert acc == want


@pytest.mark.parametrize("inst", [1, 0, 1 | 4])
def test_many_epochs_two_level_seed_walk(P, gpu, inst):
    """Batches of at least 2^15 epochs derive the seeds of their height-4
    subtrees first and walk the last 4 levels per epoch.  n2 = 1 and 40,000
    epochs from epoch 5, with the signer's ds after epoch 40,004: nodes of
    depth 15, 12, 11, 10 and 6 (walked through subtree seeds) and 2 and 0
    (walked directly).  e and sampled x_t equal the oracle's."""
    from oracle import oracle as O
    torch, ctx = gpu
    prm = O.Params(inst, 17, 0)
    t0, n = 5, 40000
    ds = O.ds_encode(O.signer_at(prm, synthlog.key_seed_bytes(0x77), t0 + n).ds)
    depths = sorted(nd.depth for nd in O.ds_decode(ds))
    assert depths[0] <= 4 < depths[-1]
    arr = synthlog.messages_fixed(77, n, 16)
    msgs = [bytes(r) for r in arr]
    params = P.make_params(inst, 17, 0)
    d = torch.from_numpy(arr.copy()).cuda()
    m = P.make_msgs(d, t0=t0)
    pk = O.encode(O.scalar_mult(12345, O.G))  # any key: only e is compared
    print(f"inst {inst}: aver over {n} epochs", flush=True)
    _, e = P.poslo_aver(ctx, params, pk, m, ds, bytes(64))
    assert int.from_bytes(e, "little") == O.ekeys_sum(prm, msgs, t0, ds)
    _, xg = P.poslo_ekeys(ctx, params, m, ds)
    xg = xg.cpu().numpy()
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), t0, n)
    for p in list(range(0, n, 997)) + [n - 1]:
        assert bytes(xg[p]) == O.one_time_seed(inst, seeds[t0 + p], 0), p
