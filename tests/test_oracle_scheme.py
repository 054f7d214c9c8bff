"""Scheme-level pins of the oracle: honest signatures verify, every single
flipped bit is rejected, Distill's invalid set equals brute-force individual
verification and the injected corruption, and the SeBVer modes agree."""

import functools

import pytest

import synthlog


def _batch(O, inst, n, L, log2_n1=2, log2_n2=2, seed_first=0, msg_seed=1):
    prm = O.Params(inst=inst, log2_n1=log2_n1, log2_n2=log2_n2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, n, L)]
    pk, sigs, ds, tag, signer = O.sign_batch(prm, synthlog.key_seed_bytes(seed_first), msgs)
    return prm, msgs, pk, sigs, ds, tag, signer


@pytest.fixture
def memo_scalar_mult(O, monkeypatch):
    """Memoise the (pure) scalar multiplication so that brute-force flip
    loops do not recompute identical products."""
    monkeypatch.setattr(O, "scalar_mult", functools.lru_cache(maxsize=None)(O.scalar_mult))


@pytest.mark.parametrize("inst", [0, 1])
def test_honest_batch_accepts(O, inst):
    # 11 entries with n2 = 4: epochs 0, 1 full, epoch 2 partial -> ds has 2 nodes
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, inst, 11, 24)
    assert [(n.depth, n.index) for n in O.ds_decode(ds)] == [(1, 0), (0, 2)]
    assert O.aver(prm, pk, msgs, 0, ds, tag)
    # a slice in the middle verifies against its own aggregate
    assert O.aver(prm, pk, msgs[3:9], 3, ds, O.agg(sigs[3:9]))
    # every signature satisfies R_t = e_t*Y + s_t*G on its own
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, 11)
    for t, sg in enumerate(sigs):
        assert O.entry_valid(prm, pk, msgs[t], t, sg, seeds[t >> prm.log2_n2])
    # the empty batch verifies against the empty aggregate
    assert O.aver(prm, pk, [], 0, ds, O.agg([]))


def test_verification_equation_closed_form(O):
    # R = alpha^r and s = r - e*y give Y^e * alpha^s = alpha^(ye + r - ey) = R
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, 1, 4, 16)
    Y = O.decode(pk)
    assert O.points_equal(Y, O.scalar_mult(signer.y, O.G))
    s_sum, e_sum = 0, 0
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, 4)
    for t, sg in enumerate(sigs):
        x = O.one_time_seed(prm.inst, seeds[t >> prm.log2_n2], t & (prm.n2 - 1))
        assert x == sg[64:80]
        e = O.digest_int(prm.inst, msgs[t], x) % O.Q
        r, R = O.bpv_online(signer, t)
        assert O.encode(R) == sg[32:64]
        assert O.le256(sg[0:32]) == (r - e * signer.y) % O.Q
        s_sum, e_sum = (s_sum + O.le256(sg[0:32])) % O.Q, (e_sum + e) % O.Q
    assert O.le256(tag[0:32]) == s_sum
    assert e_sum == O.ekeys_sum(prm, msgs, 0, ds)


def test_partition_invariance_of_ekeys(O):
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, 0, 10, 40)
    whole = O.ekeys_sum(prm, msgs, 0, ds)
    for cut in (0, 3, 7, 10):
        a = O.ekeys_sum(prm, msgs[:cut], 0, ds)
        b = O.ekeys_sum(prm, msgs[cut:], cut, ds)
        assert (a + b) % O.Q == whole
    # the lazy form: sum of raw digests, reduced once
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, 10)
    raw = sum(O.digest_int(prm.inst, m, O.one_time_seed(prm.inst, seeds[t >> prm.log2_n2],
                                                       t & (prm.n2 - 1)))
              for t, m in enumerate(msgs))
    assert raw % O.Q == whole


@pytest.mark.parametrize("inst", [0, 1])
def test_every_single_bit_flip_rejected_by_aver(O, inst, memo_scalar_mult):
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, inst, 3, 8, log2_n1=2, log2_n2=1)

    def rejects(m, d, tg):
        try:
            return not O.aver(prm, pk, m, 0, d, tg)
        except (LookupError, ValueError):
            return True

    assert not rejects(msgs, ds, tag)
    for pos in range(len(msgs)):
        for bit in range(8 * len(msgs[pos])):
            mm = bytearray(msgs[pos])
            mm[bit // 8] ^= 1 << (bit % 8)
            assert rejects(msgs[:pos] + [bytes(mm)] + msgs[pos + 1:], ds, tag), (pos, bit)
    for bit in range(8 * len(tag)):
        tg = bytearray(tag)
        tg[bit // 8] ^= 1 << (bit % 8)
        assert rejects(msgs, ds, bytes(tg)), bit
    for bit in range(8 * len(ds)):
        d = bytearray(ds)
        d[bit // 8] ^= 1 << (bit % 8)
        assert rejects(msgs, bytes(d), tag), bit


@pytest.mark.parametrize("inst", [0, 1])
def test_every_single_bit_flip_rejected_individually(O, inst, memo_scalar_mult):
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, inst, 2, 8, log2_n1=1, log2_n2=1)
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, 2)
    for t in range(2):
        x0 = seeds[t >> prm.log2_n2]
        assert O.entry_valid(prm, pk, msgs[t], t, sigs[t], x0)
        blob = msgs[t] + sigs[t]
        for bit in range(8 * len(blob)):
            b = bytearray(blob)
            b[bit // 8] ^= 1 << (bit % 8)
            m, sg = bytes(b[:len(msgs[t])]), bytes(b[len(msgs[t]):])
            assert not O.entry_valid(prm, pk, m, t, sg, x0), (t, bit)


def _corrupt(msgs, sigs, plan):
    msgs, sigs = list(msgs), list(sigs)
    for e, bit in plan:
        blob = bytearray(msgs[e] + sigs[e])
        blob[bit // 8] ^= 1 << (bit % 8)
        L = len(msgs[e])
        msgs[e], sigs[e] = bytes(blob[:L]), bytes(blob[L:])
    return msgs, sigs


@pytest.mark.parametrize("inst", [0, 1])
def test_distill_invalid_set_is_exact(O, inst):
    n, L = 24, 16
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, inst, n, L, log2_n1=3, log2_n2=2)
    plan = synthlog.corruption_plan(21, n, 5, 8 * (L + 80))
    cm, cs = _corrupt(msgs, sigs, plan)
    ccd = O.distill(prm, pk, cm, cs, 0, ds, 4)
    got = [t for t, _ in ccd.invalid]
    assert got == sorted(e for e, _ in plan)
    # brute force: individual verification of every entry
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, n)
    brute = [t for t in range(n)
             if not O.entry_valid(prm, pk, cm[t], t, cs[t], seeds[t >> prm.log2_n2])]
    assert brute == got
    # umbrellas partition the valid aggregate
    assert len(ccd.umbrellas) == 4 and ccd.span == 6
    s, R = 0, O.IDENTITY
    for utag, _ in ccd.umbrellas:
        s = (s + O.le256(utag[:32])) % O.Q
        R = O.point_add(R, O.decode(utag[32:]))
    assert O.to32(s) + O.encode(R) == ccd.valid_tag
    # AVer reads messages and the tag, not the signatures: it fails exactly
    # when a flip landed in a message; SeBVer over distilled data succeeds
    msg_flipped = any(bit < 8 * L for _, bit in plan)
    assert O.aver(prm, pk, cm, 0, ds, tag) == (not msg_flipped)
    assert O.sebver(prm, pk, cm, ccd, "V") == [True]
    assert O.sebver(prm, pk, cm, ccd, "U") == [True] * 4
    assert O.sebver(prm, pk, cm, ccd, "I") == [False] * 5


def test_distill_ragged_umbrellas(O):
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, 1, 10, 8, log2_n1=2, log2_n2=2)
    ccd = O.distill(prm, pk, msgs, sigs, 0, ds, 4)
    # span ceil(10/4) = 3: umbrellas [0,3) [3,6) [6,9) [9,10)
    assert ccd.span == 3 and [l for _, l in ccd.umbrellas] == [0, 1, 2, 3]
    assert ccd.invalid == [] and ccd.valid_tag == tag
    assert O.sebver(prm, pk, msgs, ccd, "U") == [True] * 4


def test_seed_retrieval_failure_and_exhaustion(O):
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, 0, 5, 8, log2_n1=2, log2_n2=1)
    # ds after entry 4 covers epochs 0..2 only; entry 6 lives in epoch 3
    with pytest.raises(LookupError):
        O.aver(prm, pk, msgs + [b"x" * 8, b"y" * 8], 0, ds, tag)
    for k in range(3):
        O.sig(signer, bytes(8))
    with pytest.raises(RuntimeError):
        O.sig(signer, bytes(8))  # t = n1 * n2 = 8


@pytest.mark.parametrize("inst", [0, 1])
def test_signer_at_continues_the_sequential_signer(O, inst):
    # the state after t entries, reached by SSO calls alone, signs the rest
    # of the batch exactly as the signer that signed entries 0 .. t-1
    prm, msgs, pk, sigs, ds, tag, signer = _batch(O, inst, 19, 12, log2_n1=3, log2_n2=2)
    seed = synthlog.key_seed_bytes(0)
    for t in (0, 1, 3, 4, 5, 8, 16, 19):
        st = O.signer_at(prm, seed, t)
        assert [O.sig(st, m) for m in msgs[t:]] == sigs[t:], t
        assert O.ds_encode(st.ds) == ds
    with pytest.raises(ValueError):
        O.signer_at(prm, seed, prm.n1 * prm.n2 + 1)
