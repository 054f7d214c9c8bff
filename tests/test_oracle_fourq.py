"""Pins of the oracle's FourQ group (reading R12), by computation rather than
by restating its formulas:

* the field: p = 2^127 - 1 is prime, GF(p^2) products equal the product of
  the Gaussian integers reduced mod p, square roots square back, and the
  Euler criterion separates squares from non-squares;
* the curve: d is not a square in GF(p^2), so the twisted Edwards addition
  law is complete; random points land on the curve, and
  [392 N] P = O with [392] P != O for random P while N is prime and 392 N
  lies in the Hasse interval, which fixes #E = 392 N;
* the generator: G is on the curve, G != O and [N] G = O;
* the group law: identity, inverse (-x, y), commutativity, associativity,
  and [a] P + [b] P = [a + b] P; a point doubled through the general law
  equals the affine doubling formula;
* the encoding: round trips, the sign bit, and the rejection of halves
  >= p, of bit 127, of a y with no x, of x = 0 with the sign set;
* the scheme over FourQ: honest batches accept, every single-bit flip of a
  message is rejected, Distill equals brute force, POSLO-C accepts.
"""

import functools
import random

import pytest

import synthlog

P127 = 2 ** 127 - 1


def miller_rabin(n, rounds=32, seed=3):
    if n < 2:
        return False
    for sp in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % sp == 0:
            return n == sp
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    rng = random.Random(seed)
    for _ in range(rounds):
        x = pow(rng.randrange(2, n - 1), d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def gauss_mul(a, b):
    """(a0 + a1 i)(b0 + b1 i) as Python complex-free integers, then mod p."""
    re = a[0] * b[0] - a[1] * b[1]
    im = a[0] * b[1] + a[1] * b[0]
    return (re % P127, im % P127)


def f2_pow(O, a, e):
    r = (1, 0)
    while e:
        if e & 1:
            r = O.f2_mul(r, a)
        a = O.f2_mul(a, a)
        e >>= 1
    return r


def random_point(O, rng):
    """A point of E (any order): a random y with a square x^2."""
    while True:
        y = (rng.randrange(P127), rng.randrange(P127))
        y2 = O.f2_mul(y, y)
        x2 = O.f2_mul(O.f2_sub(y2, O.FQ_ONE), O.f2_inv(O.f2_add(O.f2_mul(O.FQ_D, y2), O.FQ_ONE)))
        x = O.f2_sqrt(x2)
        if x is not None:
            assert O.fq_on_curve(x, y)
            return (x, y, O.FQ_ONE, O.f2_mul(x, y))


def eq(O, A, B):
    return O.fq_affine(A) == O.fq_affine(B)


def test_field(O):
    assert O.FQ_P == P127 and miller_rabin(P127)
    rng = random.Random(11)
    for _ in range(200):
        a = (rng.randrange(P127), rng.randrange(P127))
        b = (rng.randrange(P127), rng.randrange(P127))
        assert O.f2_mul(a, b) == gauss_mul(a, b)
        if a != (0, 0):
            assert O.f2_mul(a, O.f2_inv(a)) == (1, 0)
        sq = O.f2_mul(a, a)
        r = O.f2_sqrt(sq)
        assert r is not None and O.f2_mul(r, r) == sq
    # Euler's criterion in GF(p^2): exactly the squares have a root
    half = (P127 * P127 - 1) // 2
    for _ in range(20):
        a = (rng.randrange(P127), rng.randrange(P127))
        is_sq = f2_pow(O, a, half) == (1, 0)
        assert (O.f2_sqrt(a) is not None) == is_sq
    # i is a square root of -1, and GF(p) elements are squares in GF(p^2)
    assert O.f2_mul((0, 1), (0, 1)) == (P127 - 1, 0)
    assert O.f2_sqrt((5, 0)) is not None and O.f2_sqrt((P127 - 5, 0)) is not None


def test_curve_order_and_generator(O):
    N = O.FQ_N
    assert miller_rabin(N) and N.bit_length() == 246
    # d is not a square: the addition law has no exceptional cases
    assert f2_pow(O, O.FQ_D, (P127 * P127 - 1) // 2) == (P127 - 1, 0)
    # #E = 392 N: every sampled point is killed by 392 N; the N-part of its
    # order is N, and 392 N is the only multiple of N in the Hasse interval
    lo, hi = P127 ** 2 + 1 - 2 * P127, P127 ** 2 + 1 + 2 * P127
    assert lo <= O.FQ_COFACTOR * N <= hi
    assert sum(1 for k in range(lo // N, hi // N + 2) if lo <= k * N <= hi) == 1
    rng = random.Random(12)
    for _ in range(3):
        Pt = random_point(O, rng)
        assert eq(O, O.fq_scalar_mult(O.FQ_COFACTOR * N, Pt), O.FQ_IDENTITY)
        C = O.fq_scalar_mult(O.FQ_COFACTOR, Pt)
        assert not eq(O, C, O.FQ_IDENTITY)
        assert eq(O, O.fq_scalar_mult(N, C), O.FQ_IDENTITY)
    G = O.FQ_GEN
    assert O.fq_on_curve(*O.fq_affine(G))
    assert not eq(O, G, O.FQ_IDENTITY)
    assert eq(O, O.fq_scalar_mult(N, G), O.FQ_IDENTITY)


def test_group_law(O):
    rng = random.Random(13)
    A, B, C = (random_point(O, rng) for _ in range(3))
    add = O.fq_point_add
    assert eq(O, add(A, O.FQ_IDENTITY), A)
    negA = (O.f2_sub(O.FQ_ZERO, A[0]), A[1], A[2], O.f2_sub(O.FQ_ZERO, A[3]))
    assert eq(O, add(A, negA), O.FQ_IDENTITY)
    assert eq(O, add(A, B), add(B, A))
    assert eq(O, add(add(A, B), C), add(A, add(B, C)))
    a, b = rng.randrange(O.FQ_N), rng.randrange(O.FQ_N)
    G = O.FQ_GEN
    assert eq(O, add(O.fq_scalar_mult(a, G), O.fq_scalar_mult(b, G)), O.fq_scalar_mult((a + b) % O.FQ_N, G))
    # doubling through the unified law equals the affine doubling formula of
    # -x^2 + y^2 = 1 + d x^2 y^2: x' = 2xy / (y^2 - x^2), y' = (y^2 + x^2) / (2 - y^2 + x^2)
    x, y = O.fq_affine(A)
    x2, y2, xy = O.f2_mul(x, x), O.f2_mul(y, y), O.f2_mul(x, y)
    xd = O.f2_mul(O.f2_add(xy, xy), O.f2_inv(O.f2_sub(y2, x2)))
    yd = O.f2_mul(O.f2_add(y2, x2), O.f2_inv(O.f2_add(O.f2_sub((2, 0), y2), x2)))
    assert O.fq_affine(add(A, A)) == (xd, yd)


def test_encoding(O):
    rng = random.Random(14)
    for _ in range(10):
        A = O.fq_scalar_mult(rng.randrange(1, O.FQ_N), O.FQ_GEN)
        b = O.fq_encode(A)
        assert len(b) == 32 and b[15] >> 7 == 0
        D = O.fq_decode(b)
        assert D is not None and eq(O, D, A)
        # the other sign decodes to -A (x -> -x)
        b2 = bytearray(b)
        b2[31] ^= 0x80
        D2 = O.fq_decode(bytes(b2))
        assert D2 is not None and O.fq_affine(D2)[0] == O.f2_sub(O.FQ_ZERO, O.fq_affine(A)[0])
    assert O.fq_encode(O.FQ_IDENTITY) == (1).to_bytes(16, "little") + bytes(16)
    assert eq(O, O.fq_decode((1).to_bytes(16, "little") + bytes(16)), O.FQ_IDENTITY)
    # x = 0 with the sign bit set, halves >= p, bit 127 set
    assert O.fq_decode((1).to_bytes(16, "little") + bytes(15) + b"\x80") is None
    good = O.fq_encode(O.FQ_GEN)
    assert O.fq_decode(P127.to_bytes(16, "little") + good[16:]) is None
    assert O.fq_decode(good[:16] + (P127 | (good[31] >> 7 << 127)).to_bytes(16, "little")) is None
    assert O.fq_decode(good[:15] + bytes([good[15] | 0x80]) + good[16:]) is None
    # some y have no x: about half of random encodings fail
    fails = sum(O.fq_decode(bytes(rng.randrange(256) for _ in range(15)) + b"\x00" +
                            bytes(rng.randrange(256) for _ in range(15)) + b"\x00") is None for _ in range(40))
    assert 8 <= fails <= 32


@pytest.fixture
def memo_fq(O, monkeypatch):
    monkeypatch.setattr(O, "fq_scalar_mult", functools.lru_cache(maxsize=None)(O.fq_scalar_mult))
    g = O.FOURQ
    monkeypatch.setattr(O, "FOURQ", O.Group(g.name, g.q, g.G, g.O, g.add, O.fq_scalar_mult, g.enc, g.dec))


@pytest.mark.parametrize("inst", [1, 0, 1 | 4])
def test_scheme_over_fourq(O, inst, memo_fq):
    fq = inst | O.GROUP_FOURQ
    assert O.group_of(fq).name == "FourQ"
    prm = O.Params(fq, 2, 1, v=64, k=8)
    msgs = [bytes(r) for r in synthlog.messages_fixed(71, 3, 8)]
    pk, sigs, ds, tag, signer = O.sign_batch(prm, synthlog.key_seed_bytes(0x51), msgs)
    # the key is a FourQ point, y*G, and the signature's R_t decode on FourQ
    assert eq(O, O.fq_decode(pk), O.fq_scalar_mult(signer.y, O.FQ_GEN))
    assert all(O.fq_decode(sg[32:64]) is not None for sg in sigs)
    assert O.aver(prm, pk, msgs, 0, ds, tag)
    for pos in range(3):
        for bit in range(0, 64, 5):
            mm = bytearray(msgs[pos])
            mm[bit // 8] ^= 1 << (bit % 8)
            assert not O.aver(prm, pk, msgs[:pos] + [bytes(mm)] + msgs[pos + 1:], 0, ds, tag)
    # the same inputs under edwards25519 do not verify (or pk is no point there)
    try:
        ok = O.aver(O.Params(inst, 2, 1), pk, msgs, 0, ds, tag)
    except ValueError:
        ok = False
    assert not ok
    cm, cs = list(msgs), list(sigs)
    cs[1] = cs[1][:5] + bytes([cs[1][5] ^ 2]) + cs[1][6:]
    ccd = O.distill(prm, pk, cm, cs, 0, ds, 2)
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, 3)
    brute = [t for t in range(3) if not O.entry_valid(prm, pk, cm[t], t, cs[t], seeds[t >> prm.log2_n2])]
    assert [t for t, _ in ccd.invalid] == brute == [1]
    assert O.sebver(prm, pk, cm, ccd, "V") == [True]
    # POSLO-C over FourQ: whole epochs accept against their aggregate
    cmsgs = [bytes(r) for r in synthlog.messages_fixed(72, 4, 8)]
    pkc, s_list, dsc, _ = O.posloc_sign_batch(prm, synthlog.key_seed_bytes(0x52), cmsgs)
    eps = [(i, cmsgs[2 * i:2 * i + 2]) for i in range(2)]
    assert O.posloc_aver(prm, pkc, eps, dsc, O.posloc_agg_s(s_list, fq))
    assert not O.posloc_aver(prm, pkc, eps, dsc, O.posloc_agg_s(s_list[:1] + s_list[:1], fq))


def test_fourq_rules(O):
    with pytest.raises(ValueError):
        O.group_of(2 | 8)   # POSLO++ is not defined on FourQ
    with pytest.raises(ValueError):
        O.group_of(16)
