"""Pins of the oracle's POSLO-C (coarse-grained, one signature per epoch):
honest epochs verify alone and in any combination, the verification
equation holds in closed form against the POSLO-F per-entry hash sums,
every single flipped bit of a message, an epoch signature or the ds is
rejected, and Distill's invalid epochs equal brute-force per-epoch AVer and
the injected corruption, with umbrellas that sum to the valid tag."""

import functools

import pytest

import synthlog


def _epochs(O, inst, k, L, log2_n1, log2_n2, seed_first=0x50, msg_seed=31):
    prm = O.Params(inst, log2_n1, log2_n2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, k * prm.n2, L)]
    pk, s_list, ds, signer = O.posloc_sign_batch(prm, synthlog.key_seed_bytes(seed_first), msgs)
    return prm, msgs, pk, s_list, ds, signer


def _ep(prm, msgs, i):
    return (i, msgs[i * prm.n2:(i + 1) * prm.n2])


@pytest.fixture
def memo_scalar_mult(O, monkeypatch):
    monkeypatch.setattr(O, "scalar_mult", functools.lru_cache(maxsize=None)(O.scalar_mult))


@pytest.mark.parametrize("inst", [0, 1])
def test_honest_epochs_accept(O, inst):
    prm, msgs, pk, s_list, ds, signer = _epochs(O, inst, 3, 20, 2, 2)
    # ds after epoch 2 of n1 = 4: the node covering epochs 0-1, then x_0[2]
    assert [(n.depth, n.index) for n in O.ds_decode(ds)] == [(1, 0), (0, 2)]
    for i in range(3):
        assert O.posloc_aver(prm, pk, [_ep(prm, msgs, i)], ds, s_list[i])
    assert O.posloc_aver(prm, pk, [_ep(prm, msgs, i) for i in range(3)], ds, O.posloc_agg_s(s_list))
    assert O.posloc_aver(prm, pk, [_ep(prm, msgs, 0), _ep(prm, msgs, 2)], ds,
                         O.posloc_agg_s([s_list[0], s_list[2]]))
    # a signature of one epoch does not verify another
    assert not O.posloc_aver(prm, pk, [_ep(prm, msgs, 1)], ds, s_list[0])
    # AVer takes whole epochs only
    with pytest.raises(ValueError):
        O.posloc_aver(prm, pk, [(0, msgs[:3])], ds, s_list[0])


def test_closed_form_against_per_entry_sums(O):
    # R~_i = r~_i * G and s~_i = r~_i - y * e~_i give e~_i * Y + s~_i * G = R~_i,
    # with e~_i the POSLO-F aggregate key of the epoch's entries
    prm, msgs, pk, s_list, ds, signer = _epochs(O, 1, 2, 24, 1, 3)
    Yb, Rs = O.posloc_pk_parts(prm, pk)
    assert O.points_equal(O.decode(Yb), O.scalar_mult(signer.y, O.G))
    for i in range(2):
        e_i = O.ekeys_sum(prm, msgs[i * prm.n2:(i + 1) * prm.n2], i * prm.n2, ds)
        assert e_i == O.posloc_epoch_e(prm, msgs[i * prm.n2:(i + 1) * prm.n2], i, O.ds_decode(ds))
        r_i = (O.le256(s_list[i]) + signer.y * e_i) % O.Q
        assert O.encode(O.scalar_mult(r_i, O.G)) == Rs[i]
        # r~_i is the sum of the epoch's per-entry commitments
        assert r_i == sum(O.posloc_r(1, signer.r, i, j) for j in range(prm.n2)) % O.Q


@pytest.mark.parametrize("inst", [0, 1])
def test_every_single_bit_flip_rejected(O, inst, memo_scalar_mult):
    prm, msgs, pk, s_list, ds, signer = _epochs(O, inst, 2, 6, 1, 1)
    eps = [_ep(prm, msgs, i) for i in range(2)]
    s = O.posloc_agg_s(s_list)

    def rejects(e, d, sv):
        try:
            return not O.posloc_aver(prm, pk, e, d, sv)
        except (LookupError, ValueError):
            return True

    assert not rejects(eps, ds, s)
    for i in range(2):
        for j in range(prm.n2):
            for bit in range(8 * len(msgs[2 * i + j])):
                m = bytearray(msgs[2 * i + j])
                m[bit // 8] ^= 1 << (bit % 8)
                em = list(eps[i][1])
                em[j] = bytes(m)
                e2 = list(eps)
                e2[i] = (i, em)
                assert rejects(e2, ds, s), (i, j, bit)
    for bit in range(256):
        sv = bytearray(s)
        sv[bit // 8] ^= 1 << (bit % 8)
        assert rejects(eps, ds, bytes(sv)), bit
    for bit in range(8 * len(ds)):
        d = bytearray(ds)
        d[bit // 8] ^= 1 << (bit % 8)
        assert rejects(eps, bytes(d), s), bit


@pytest.mark.parametrize("inst", [0, 1])
def test_distill_invalid_epochs_exact(O, inst):
    prm, msgs, pk, s_list, ds, signer = _epochs(O, inst, 6, 12, 3, 2)
    cm, cs = list(msgs), list(s_list)
    m = bytearray(cm[1 * prm.n2 + 2])
    m[5] ^= 0x20
    cm[1 * prm.n2 + 2] = bytes(m)   # a message of epoch 1
    s = bytearray(cs[4])
    s[9] ^= 1
    cs[4] = bytes(s)                # the signature of epoch 4
    ccd = O.posloc_distill(prm, pk, cm, cs, 0, ds, 3)
    assert [i for i, _ in ccd.invalid] == [1, 4]
    brute = [i for i in range(6) if not O.posloc_aver(prm, pk, [_ep(prm, cm, i)], ds, cs[i])]
    assert brute == [1, 4]
    _, Rs = O.posloc_pk_parts(prm, pk)
    assert ccd.invalid[1][1] == cs[4] + Rs[4]
    assert ccd.span == 2 and [l for _, l in ccd.umbrellas] == [0, 1, 2]
    s_sum, R = 0, O.IDENTITY
    for tag, _ in ccd.umbrellas:
        s_sum = (s_sum + O.le256(tag[:32])) % O.Q
        R = O.point_add(R, O.decode(tag[32:]))
    assert O.to32(s_sum) + O.encode(R) == ccd.valid_tag
    assert O.posloc_sebver(prm, pk, cm, ccd, "V") == [True]
    assert O.posloc_sebver(prm, pk, cm, ccd, "U") == [True] * 3
    assert O.posloc_sebver(prm, pk, cm, ccd, "I") == [False, False]
    # an honest batch distills into no invalid epochs and the full aggregate
    ccd = O.posloc_distill(prm, pk, msgs, s_list, 0, ds, 1)
    assert ccd.invalid == [] and ccd.valid_tag[:32] == O.posloc_agg_s(s_list)


def test_signer_limits(O):
    prm, msgs, pk, s_list, ds, signer = _epochs(O, 0, 2, 8, 1, 1)
    with pytest.raises(RuntimeError):
        O.posloc_sig(signer, msgs[:2])       # both epochs are signed
    prm2 = O.Params(0, 1, 1)
    signer2, _ = O.posloc_kg(prm2, synthlog.key_seed_bytes(1))
    with pytest.raises(ValueError):
        O.posloc_sig(signer2, msgs[:1])      # not a whole epoch


def test_signer_at_and_commitments_continue_kg_and_sig(O):
    prm, msgs, pk, s_list, ds, signer = _epochs(O, 1, 4, 16, 2, 2)
    seed = synthlog.key_seed_bytes(0x50)
    Yb, Rs = O.posloc_pk_parts(prm, pk)
    st = O.posloc_signer_at(prm, seed, 0)
    assert [O.posloc_commitment(prm, st.r, i) for i in range(prm.n1)] == Rs
    for i in (0, 1, 3):
        st = O.posloc_signer_at(prm, seed, i)
        got = [O.posloc_sig(st, msgs[e * prm.n2:(e + 1) * prm.n2]) for e in range(i, 4)]
        assert [g[0] for g in got] == s_list[i:], i
        assert got[-1][1] == ds
