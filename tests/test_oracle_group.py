"""Pins of the oracle's group arithmetic (edwards25519 prime-order subgroup):
RFC 8032 public-key vectors, closed-form identities and encoding rules."""

import hashlib
import random

from conftest import golden_lines


def test_base_point_and_order(O):
    assert O.encode(O.G).hex() == "58" + "66" * 31
    # on the curve: -x^2 + y^2 = 1 + d x^2 y^2
    x, y = O.G[0], O.G[1]
    assert (-x * x + y * y - 1 - O.D_CURVE * x * x * y * y) % O.P == 0
    assert O.points_equal(O.scalar_mult(O.Q, O.G), O.IDENTITY)
    assert not O.points_equal(O.scalar_mult(O.Q - 1, O.G), O.IDENTITY)
    # q is the RFC 8032 group order L
    assert O.Q == 2 ** 252 + 27742317777372353535851937790883648493


def test_rfc8032_public_keys(O):
    rows = list(golden_lines("ed25519_rfc8032.txt"))
    assert len(rows) == 3
    for sk, pk in rows:
        h = hashlib.sha512(bytes.fromhex(sk)).digest()
        a = int.from_bytes(h[:32], "little")
        a &= (1 << 254) - 8
        a |= 1 << 254
        assert O.encode(O.scalar_mult(a, O.G)).hex() == pk


def test_group_law(O):
    rng = random.Random(5)
    for _ in range(3):
        a, b = rng.randrange(O.Q), rng.randrange(O.Q)
        lhs = O.scalar_mult((a + b) % O.Q, O.G)
        rhs = O.point_add(O.scalar_mult(a, O.G), O.scalar_mult(b, O.G))
        assert O.points_equal(lhs, rhs)
        # doubling through the addition law
        A = O.scalar_mult(a, O.G)
        assert O.points_equal(O.point_add(A, A), O.scalar_mult(2 * a % O.Q, O.G))
        # additive inverse
        assert O.points_equal(O.point_add(A, O.scalar_mult(O.Q - a, O.G)), O.IDENTITY)


def test_encoding_rules(O):
    rng = random.Random(9)
    A = O.scalar_mult(rng.randrange(1, O.Q), O.G)
    enc = O.encode(A)
    assert O.points_equal(O.decode(enc), A)
    # identity encodes as y = 1
    assert O.encode(O.IDENTITY) == (1).to_bytes(32, "little")
    # y >= p is not canonical
    assert O.decode((O.P + 1).to_bytes(32, "little")) is None
    # x = 0 with the sign bit set is not canonical
    assert O.decode(((1 << 255) | 1).to_bytes(32, "little")) is None
    # a y with no matching x: y = 2 gives x^2 = 3/(4d+1); check that decode
    # and the curve equation agree on every small y
    for y in range(2, 40):
        pt = O.decode(y.to_bytes(32, "little"))
        if pt is not None:
            x = pt[0]
            assert (-x * x + y * y - 1 - O.D_CURVE * x * x * y * y) % O.P == 0
