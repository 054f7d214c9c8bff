"""GPU parity of Distill and SeBVer against the oracle, through the C ABI.

Small batches are signed by the oracle and corrupted at seeded single-bit
positions of m_t || sigma_t; the GPU's CCD (sorted invalid set, invalid
signatures, valid tag, umbrella tags) must equal the oracle's byte for byte,
and SeBVer's bits must equal the oracle's.  The full 2^20 x 256-byte
configuration with 1% corruption is compared with the oracle in
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


def corrupt(msgs, sigs, plan):
    msgs, sigs = list(msgs), list(sigs)
    for e, bit in plan:
        L = len(msgs[e])
        blob = bytearray(msgs[e] + sigs[e])
        blob[bit // 8] ^= 1 << (bit % 8)
        msgs[e], sigs[e] = bytes(blob[:L]), bytes(blob[L:])
    return msgs, sigs


@functools.lru_cache(maxsize=None)
def signed(inst, n, L, l1, l2, key_first, msg_seed):
    from oracle import oracle as O
    prm = O.Params(inst, l1, l2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, n, L)]
    pk, sigs, ds, tag, _ = O.sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    return prm, msgs, pk, sigs, ds, tag


def to_dev(torch, msgs, sigs):
    L = len(msgs[0])
    m = torch.from_numpy(np.frombuffer(b"".join(msgs), dtype=np.uint8).reshape(len(msgs), L).copy()).cuda()
    s = torch.from_numpy(np.frombuffer(b"".join(sigs), dtype=np.uint8).copy()).cuda()
    return m, s


CASES = [
    # inst, n, L, log2_n1, log2_n2, corrupted, umbrellas
    (1, 200, 40, 4, 4, 7, 5),
    (0, 200, 40, 4, 4, 7, 5),
    (1, 300, 32, 5, 4, 0, 3),     # nothing to find
    (0, 64, 16, 3, 3, 11, 64),    # one entry per umbrella
    (1, 129, 48, 4, 4, 129, 1),   # every entry corrupted, one umbrella
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"inst{c[0]}-n{c[1]}-L{c[2]}-k{c[5]}-u{c[6]}")
def test_distill_and_sebver_match_oracle(P, gpu, case):
    from oracle import oracle as O
    torch, ctx = gpu
    inst, n, L, l1, l2, k, nu = case
    prm, msgs, pk, sigs, ds, tag = signed(inst, n, L, l1, l2, 0x11, 8)
    plan = synthlog.corruption_plan(40 + k, n, k, 8 * (L + 80))
    cm, cs = corrupt(msgs, sigs, plan)
    params = P.make_params(inst, l1, l2)
    dm, dsig = to_dev(torch, cm, cs)
    print(f"case {case}: distill", flush=True)
    ccd = P.poslo_distill(ctx, params, pk, P.make_msgs(dm), dsig, ds, nu)
    want = O.distill(prm, pk, cm, cs, 0, ds, nu)
    got_inv = ccd.invalid()
    assert got_inv == [t for t, _ in want.invalid]
    assert got_inv == sorted(e for e, _ in plan)
    for i, (t, sg) in enumerate(want.invalid):
        assert ccd.invalid_sig(i) == sg
    assert ccd.valid_tag() == want.valid_tag
    tags, span = ccd.umbrellas()
    assert span == want.span and tags == [t for t, _ in want.umbrellas]
    m = P.make_msgs(dm)
    for mode in "VUI":
        assert P.poslo_sebver(ctx, params, pk, m, ccd, mode) == O.sebver(prm, pk, cm, want, mode), mode
    # the serialized CCD verifies the same way after a round trip
    ccd2 = P.poslo_ccd_import(ccd.export())
    assert ccd2.invalid() == got_inv and ccd2.valid_tag() == ccd.valid_tag()
    assert P.poslo_sebver(ctx, params, pk, m, ccd2, "V") == [True]


def test_sebver_detects_tampered_ccd(P, gpu):
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, pk, sigs, ds, tag = signed(1, 200, 40, 4, 4, 0x11, 8)
    params = P.make_params(1, 4, 4)
    plan = synthlog.corruption_plan(47, 200, 7, 8 * 120)
    cm, cs = corrupt(msgs, sigs, plan)
    dm, dsig = to_dev(torch, cm, cs)
    ccd = P.poslo_distill(ctx, params, pk, P.make_msgs(dm), dsig, ds, 5)
    blob = bytearray(ccd.export())
    # flip a bit of the first umbrella tag's R: that umbrella must fail
    hdr = 4 + 4 + 4 * 3 + 8 * 3
    ds_len = int.from_bytes(blob[hdr:hdr + 4], "little")
    umb0 = hdr + 4 + ds_len + 64 + 8
    blob[umb0 + 40] ^= 1
    bad = P.poslo_ccd_import(bytes(blob))
    bits = P.poslo_sebver(ctx, params, pk, P.make_msgs(dm), bad, "U")
    assert bits[0] is False and all(bits[1:])


def _flip_s_bit(sig, b):
    s = bytearray(sig)
    s[b // 8] ^= 1 << (b % 8)
    return bytes(s)


@pytest.mark.parametrize("inst", [1, 0])
def test_distill_finds_errors_that_cancel_in_sums(P, gpu, inst):
    """Tampering that keeps sums of s unchanged: a pair with the same bit of
    s flipped in opposite directions, and four entries at the corners of a
    rectangle of an 8 x 8 arrangement of 64 consecutive entries (+2^b, -2^b
    on one row, -2^b, +2^b on another), which leaves every row sum and every
    column sum of s as it was.  Each entry is checked on its own, so all of
    them must be named, exactly as the oracle's Distill names them."""
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, pk, sigs, ds, tag = signed(inst, 200, 40, 4, 4, 0x11, 8)
    sigs = list(sigs)

    def s_int(k):
        return int.from_bytes(sigs[k][:32], "little")

    def bit(k, b):
        return (s_int(k) >> b) & 1

    i, j = 16, 19
    b = next(b for b in range(8, 240) if bit(i, b) and not bit(j, b))
    before = s_int(i) + s_int(j)
    sigs[i], sigs[j] = _flip_s_bit(sigs[i], b), _flip_s_bit(sigs[j], b)
    assert s_int(i) + s_int(j) == before
    plus, minus = (74, 102), (78, 98)  # rows 1 and 4, columns 2 and 6 of entries 64..127
    b = next(b for b in range(8, 240) if all(not bit(k, b) for k in plus) and all(bit(k, b) for k in minus))
    before = [s_int(k) for k in plus + minus]
    for k in plus + minus:
        sigs[k] = _flip_s_bit(sigs[k], b)
    after = [s_int(k) for k in plus + minus]
    assert after[0] - before[0] == after[1] - before[1] == before[2] - after[2] == before[3] - after[3] == 1 << b
    want = O.distill(prm, pk, msgs, sigs, 0, ds, 1)
    expect = [16, 19, 74, 78, 98, 102]
    assert [t for t, _ in want.invalid] == expect
    params = P.make_params(inst, 4, 4)
    dm, dsig = to_dev(torch, msgs, sigs)
    ccd = P.poslo_distill(ctx, params, pk, P.make_msgs(dm), dsig, ds, 1)
    assert ccd.invalid() == expect
    assert ccd.valid_tag() == want.valid_tag
    # the multi-signer path (the tag is the honest one, so AVer accepts)
    bj = P.BatchJobs([dict(pk=pk, ds=ds, tag=tag, t0=0, n=200, entry_base=0)])
    off = torch.arange(0, 201 * 40, 40, dtype=torch.int64, device="cuda")
    acc, inv = P.poslo_verify_batch(ctx, params, bj, dm.reshape(-1), off, dsig, distill=2)
    assert acc == [True] and inv == [(0, t) for t in expect]


@pytest.mark.parametrize("inst", [1, 0])
def test_table_digit_extremes(P, gpu, inst):
    """Entries re-signed with scalars at the edges of the fixed-base tables'
    signed digits (0, digits of 128 / 129 / 32768 / 32769, q - 1, 2^252,
    ...): R_t = e_t*Y + s_t*G is computed by the oracle, so these entries
    are valid; s_t = q and s_t = 2^256 - 1 are not.  Distill and the
    multi-signer checks must agree with the oracle entry by entry."""
    from oracle import oracle as O
    torch, ctx = gpu
    prm, msgs, pk, sigs, ds, tag = signed(inst, 64, 40, 4, 4, 0x11, 8)
    sigs = list(sigs)
    q = O.Q
    rep8 = sum(0x80 << (8 * k) for k in range(31))
    rep16 = sum(0x8000 << (16 * k) for k in range(15))
    special = [0, 1, 2, 127, 128, 129, 255, 256, 32767, 32768, 32769, 65535, 65536, q - 1, q - 2, q - 32768,
               q - 128, 2 ** 252, 2 ** 252 - 1, rep8, rep8 + 1, rep16, rep16 + 0x10001, (rep8 ^ (rep8 >> 1)) % q]
    assert all(0 <= s < q for s in special)
    Y = O.decode(pk)
    for t, s in enumerate(special):
        x = sigs[t][64:80]
        e = O.digest_int(prm.inst, msgs[t], x) % q
        R = O.point_add(O.scalar_mult(e, Y), O.scalar_mult(s, O.G))
        sigs[t] = O.to32(s) + O.encode(R) + x
    bad = {40: q, 41: 2 ** 256 - 1}
    for t, s in bad.items():
        sigs[t] = s.to_bytes(32, "little") + sigs[t][32:]
    want = O.distill(prm, pk, msgs, sigs, 0, ds, 1)
    assert [t for t, _ in want.invalid] == sorted(bad)
    params = P.make_params(inst, 4, 4)
    dm, dsig = to_dev(torch, msgs, sigs)
    ccd = P.poslo_distill(ctx, params, pk, P.make_msgs(dm), dsig, ds, 1)
    assert ccd.invalid() == sorted(bad)
    assert ccd.valid_tag() == want.valid_tag
    bj = P.BatchJobs([dict(pk=pk, ds=ds, tag=tag, t0=0, n=64, entry_base=0)])
    off = torch.arange(0, 65 * 40, 40, dtype=torch.int64, device="cuda")
    acc, inv = P.poslo_verify_batch(ctx, params, bj, dm.reshape(-1), off, dsig, distill=2)
    assert acc == [True] and inv == [(0, t) for t in sorted(bad)]
    # the same with the key's wide table (16 + 16 additions per entry)
    ctx2 = P.poslo_ctx_create(0)
    try:
        P.poslo_ctx_keys_widen(ctx2, [pk])
        print(f"inst {inst}: digit extremes with a wide key table", flush=True)
        ccd2 = P.poslo_distill(ctx2, params, pk, P.make_msgs(dm), dsig, ds, 1)
        assert ccd2.invalid() == sorted(bad) and ccd2.valid_tag() == want.valid_tag
        acc, inv = P.poslo_verify_batch(ctx2, params, bj, dm.reshape(-1), off, dsig, distill=2)
        assert acc == [True] and inv == [(0, t) for t in sorted(bad)]
    finally:
        ctx2.close()
