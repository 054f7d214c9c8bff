"""The seeded input generator: the vectorised path equals the scalar
definition, and the splitmix64 seeding matches its published first output."""

import numpy as np

import synthlog


def test_splitmix64_seed0_first_output():
    # splitmix64 from state 0: first output 0xe220a8397b1dcdaf
    assert synthlog.splitmix64_next(0)[1] == 0xE220A8397B1DCDAF


def test_vector_stream_equals_scalar():
    sids = np.array([0, 1, 2, 1000, 123456], dtype=np.uint64)
    words = synthlog.stream_words(7, sids, 5)
    for r, sid in enumerate(sids):
        g = synthlog.Xoshiro256ss(synthlog.stream_seed(7, int(sid)))
        assert [int(w) for w in words[r]] == [g.next() for _ in range(5)]


def test_messages_fixed_and_var():
    m = synthlog.messages_fixed(3, 10, 13, t0=5)
    for k in range(10):
        assert bytes(m[k]) == synthlog.stream_bytes(3, 5 + k, 13)
    lens = np.array([4, 0, 9, 4, 17])
    data, off = synthlog.messages_var(3, lens, t0=2)
    assert list(off) == [0, 4, 4, 13, 17, 34]
    for k in range(5):
        assert bytes(data[off[k]:off[k + 1]]) == synthlog.stream_bytes(3, 2 + k, int(lens[k]))


def test_sampling_helpers():
    s = synthlog.sample_distinct(1, 0, 100, 100)
    assert sorted(s) == list(range(100))
    plan = synthlog.corruption_plan(4, 1000, 10, 64)
    assert len({e for e, _ in plan}) == 10 and all(0 <= b < 64 for _, b in plan)
    c = synthlog.log_uniform_counts(5, 0, 1000, 65536)
    assert min(c) >= 1 and max(c) <= 65536
    u = synthlog.uniform_ints(6, 0, 500, 64, 512)
    assert min(u) >= 64 and max(u) <= 512


def test_uniform_per_stream():
    v = synthlog.uniform_per_stream(9, np.arange(20000), 64, 512)
    assert v.min() >= 64 and v.max() <= 512 and abs(v.mean() - 288) < 3
    g = synthlog.Xoshiro256ss(synthlog.stream_seed(9, 17))
    u = (g.next() >> 11) * (1.0 / (1 << 53))
    assert v[17] == 64 + int(u * 449)


def test_corruption_plan_var():
    bits = np.array([8 * (L + 80) for L in range(1, 501)])
    plan = synthlog.corruption_plan_var(12, 500, 40, bits)
    assert len({e for e, _ in plan}) == 40
    assert all(0 <= b < bits[e] for e, b in plan)
    assert plan == sorted(plan)
    # fixed bit counts reduce to the fixed-length plan
    assert synthlog.corruption_plan_var(4, 1000, 10, np.full(1000, 64)) == synthlog.corruption_plan(4, 1000, 10, 64)
