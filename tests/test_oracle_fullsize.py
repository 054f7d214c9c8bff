"""The pooled full-size oracle results (tests/oracle_fullsize.py) equal the
sequential oracle on a small batch: the chunked signer continues the
sequential signer exactly, and the combined sums (e, Agg, umbrellas, the
invalid set) equal sign_batch, aver and distill run in order."""

import numpy as np

import synthlog


def _corrupt(msgs, sigs, plan):
    msgs, sigs = list(msgs), list(sigs)
    for e, bit in plan:
        blob = bytearray(msgs[e] + sigs[e])
        blob[bit // 8] ^= 1 << (bit % 8)
        L = len(msgs[e])
        msgs[e], sigs[e] = bytes(blob[:L]), bytes(blob[L:])
    return msgs, sigs


def test_pooled_case_equals_sequential_oracle(O):
    import oracle_fullsize as F
    inst, n, L, l1, l2, key_first, msg_seed, n_u, flip_seed, k = 1, 150, 40, 4, 4, 9, 11, 4, 12, 6
    case = F.full_case(inst, n, L, l1, l2, key_first, msg_seed, n_u, flip_seed, k, nproc=3)
    prm = O.Params(inst, l1, l2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, n, L)]
    pk, sigs, ds, tag, _ = O.sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    assert case.pk == pk and case.ds == ds and case.tag == tag
    assert [bytes(r) for r in case.msgs] == msgs
    assert [bytes(r) for r in case.sigs] == sigs
    assert case.e == O.ekeys_sum(prm, msgs, 0, ds)
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, n)
    for t in range(n):
        x = O.one_time_seed(inst, seeds[t >> l2], t & (prm.n2 - 1))
        assert bytes(case.x_t[t]) == x
        assert int.from_bytes(bytes(case.e_t[t]), "little") == O.digest_int(inst, msgs[t], x) % O.Q
    assert case.aver_honest
    plan = synthlog.corruption_plan(flip_seed, n, k, 8 * (L + 80))
    assert case.plan == plan
    cm, cs = _corrupt(msgs, sigs, plan)
    assert [bytes(r) for r in case.cmsgs] == cm and [bytes(r) for r in case.csigs] == cs
    ccd = O.distill(prm, pk, cm, cs, 0, ds, n_u)
    assert case.invalid == [t for t, _ in ccd.invalid] == sorted(e for e, _ in plan)
    assert case.span == ccd.span
    assert case.umbrellas == [u for u, _ in ccd.umbrellas]
    assert case.valid_tag == ccd.valid_tag
    assert case.e_corrupt == O.ekeys_sum(prm, cm, 0, ds)
    assert case.aver_corrupt == O.aver(prm, pk, cm, 0, ds, tag)
    assert isinstance(case.msgs, np.ndarray)


def test_pooled_posloc_case_equals_sequential_oracle(O):
    import oracle_fullsize as F
    inst, l1, l2, L, key_first, msg_seed, n_u, flip_seed, kf = 0, 3, 2, 20, 0x33, 12, 3, 13, 2
    k = 7
    n = k * 4
    c = F.full_case_c(inst, n, L, l1, l2, key_first, msg_seed, n_u, flip_seed, kf, nproc=3)
    prm = O.Params(inst, l1, l2)
    msgs = [bytes(r) for r in synthlog.messages_fixed(msg_seed, n, L)]
    pk, s_list, ds, _ = O.posloc_sign_batch(prm, synthlog.key_seed_bytes(key_first), msgs)
    assert c.pk[:32 + 32 * prm.n1] == pk and c.ds == ds and c.s_epochs == b"".join(s_list)
    eps = [(i, msgs[i * 4:(i + 1) * 4]) for i in range(k)]
    assert c.e == O.ekeys_sum(prm, msgs, 0, ds)
    assert c.aver_honest == O.posloc_aver(prm, pk, eps, ds, c.s_total) is True
    # the corruption: one bit of each planned epoch's messages || signature
    plan = synthlog.corruption_plan(flip_seed, k, kf, 8 * (4 * L + 32))
    assert c.plan == plan
    cm, cs = list(msgs), list(s_list)
    for i, bit in plan:
        blob = bytearray(b"".join(cm[i * 4:(i + 1) * 4]) + cs[i])
        blob[bit // 8] ^= 1 << (bit % 8)
        cm[i * 4:(i + 1) * 4] = [bytes(blob[j * L:(j + 1) * L]) for j in range(4)]
        cs[i] = bytes(blob[4 * L:])
    assert [bytes(r) for r in c.cmsgs] == cm and c.cs_epochs == b"".join(cs)
    ccd = O.posloc_distill(prm, pk, cm, cs, 0, ds, n_u)
    assert c.invalid == [i for i, _ in ccd.invalid] == sorted(i for i, _ in plan)
    assert c.span == ccd.span and c.umbrellas == [u for u, _ in ccd.umbrellas]
    assert c.valid_tag == ccd.valid_tag
    assert c.e_corrupt == O.ekeys_sum(prm, cm, 0, ds)
    cep = [(i, cm[i * 4:(i + 1) * 4]) for i in range(k)]
    assert c.aver_corrupt == O.posloc_aver(prm, pk, cep, ds, O.posloc_agg_s(cs))


def test_pooled_job_case_equals_sequential_oracle(O):
    """One signer's job of a multi-signer log: messages of varying length
    at global stream ids base + t, signed from t = 0; the pooled results
    equal sign_batch, aver and distill run in order."""
    import oracle_fullsize as F
    inst, l1, l2, n, base, msg_seed = 1, 4, 3, 97, 1234, 21
    key_seed = synthlog.derived_key_seed(22, 5)
    lens = synthlog.uniform_per_stream(23, np.arange(base, base + n), 0, 70)
    flips = synthlog.corruption_plan_var(24, n, 5, 8 * (lens.astype(np.int64) + 80))
    case = F.job_case(inst, l1, l2, key_seed, msg_seed, tuple(int(x) for x in lens), base, tuple(flips), nproc=3)
    prm = O.Params(inst, l1, l2)
    data, off = synthlog.messages_var(msg_seed, lens, t0=base)
    msgs = [bytes(data[off[t]:off[t + 1]]) for t in range(n)]
    pk, sigs, ds, tag, _ = O.sign_batch(prm, key_seed, msgs)
    assert (case.pk, case.ds, case.tag, case.sigs) == (pk, ds, tag, b"".join(sigs))
    cm, cs = _corrupt(msgs, sigs, flips)
    assert case.aver_corrupt == O.aver(prm, pk, cm, 0, ds, tag)
    ccd = O.distill(prm, pk, cm, cs, 0, ds, 1)
    assert case.invalid == [t for t, _ in ccd.invalid] == sorted(t for t, _ in flips)
