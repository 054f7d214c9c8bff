"""Pins of the oracle's byte-level primitives against published vectors and
independent library routines (hashlib; the openssl command-line AES)."""

import hashlib
import random
import shutil
import subprocess

import pytest

from conftest import golden_lines

HAVE_OPENSSL = shutil.which("openssl") is not None


def openssl_aes128(key: bytes, block: bytes) -> bytes:
    """AES-128-ECB of one block by the openssl command-line tool."""
    out = subprocess.run(
        ["openssl", "enc", "-aes-128-ecb", "-nopad", "-K", key.hex()],
        input=block, capture_output=True, check=True).stdout
    assert len(out) == 16
    return out


def test_aes128_fips197(O):
    rows = list(golden_lines("aes128_fips197.txt"))
    assert len(rows) == 2
    for key, pt, ct in rows:
        assert O.aes128(bytes.fromhex(key), bytes.fromhex(pt)).hex() == ct


@pytest.mark.skipif(not HAVE_OPENSSL, reason="openssl command not available")
def test_aes128_random_vs_openssl(O):
    rng = random.Random(7)
    for _ in range(24):
        key = bytes(rng.randrange(256) for _ in range(16))
        pt = bytes(rng.randrange(256) for _ in range(16))
        assert O.aes128(key, pt) == openssl_aes128(key, pt)


def test_sha256_fips180(O):
    rows = list(golden_lines("sha256_fips180.txt"))
    assert len(rows) == 2
    for msg, dg in rows:
        assert O.sha256(msg.encode()).hex() == dg


def test_sha256_every_padding_boundary(O):
    rng = random.Random(11)
    for n in list(range(0, 200)) + [447, 448, 511, 512, 1000]:
        data = bytes(rng.randrange(256) for _ in range(n))
        assert O.sha256(data) == hashlib.sha256(data).digest(), n


def _xor(a, b):
    return bytes(x ^ y for x, y in zip(a, b))


@pytest.mark.skipif(not HAVE_OPENSSL, reason="openssl command not available")
def test_mmo_one_block_and_chain(O):
    # one block: E_IV(z) xor z with IV = 0x52 * 16 (the MMO definition)
    iv = bytes([0x52]) * 16
    z = bytes(range(16))
    assert O.mmo(z) == _xor(openssl_aes128(iv, z), z)
    # empty input is one zero block
    zero = bytes(16)
    assert O.mmo(b"") == _xor(openssl_aes128(iv, zero), zero)
    # three blocks with a ragged tail: chaining value is the next key
    data = bytes((7 * k + 3) & 0xFF for k in range(37))
    blocks = [data[0:16], data[16:32], data[32:37] + bytes(11)]
    h = iv
    for m in blocks:
        h = _xor(openssl_aes128(h, m), m)
    assert O.mmo(data) == h


@pytest.mark.skipif(not HAVE_OPENSSL, reason="openssl command not available")
def test_mdc2_one_block_and_chain(O):
    A, B = bytes([0x52]) * 16, bytes([0x25]) * 16
    z = bytes(range(100, 116))
    a = _xor(openssl_aes128(A, z), z)
    b = _xor(openssl_aes128(B, z), z)
    # the 128-bit input case: two MMO iterations with the halves swapped
    assert O.mdc2(z) == a[:8] + b[8:] + b[:8] + a[8:]
    data = bytes((11 * k + 5) & 0xFF for k in range(40))
    blocks = [data[0:16], data[16:32], data[32:40] + bytes(8)]
    h, hp = A, B
    for m in blocks:
        a = _xor(openssl_aes128(h, m), m)
        b = _xor(openssl_aes128(hp, m), m)
        h, hp = a[:8] + b[8:], b[:8] + a[8:]
    assert O.mdc2(data) == h + hp


def test_mdc2_halves_are_not_plain_mmo(O):
    # a dropped half-swap would make the first half equal to plain MMO over
    # two or more blocks; the swap must make them differ
    data = bytes(range(48))
    assert O.mdc2(data)[:16] != O.mmo(data)


def test_prf_sha_is_truncated_sha256(O):
    z = bytes(range(16)) + (5).to_bytes(4, "little")
    for b in (0, 1):
        assert O.prf(O.INST_SHA256, b, z) == hashlib.sha256(z + bytes([b])).digest()[:16]
    assert O.H(O.INST_SHA256, z) == hashlib.sha256(z).digest()


@pytest.mark.skipif(not HAVE_OPENSSL, reason="openssl command not available")
def test_prf_aes_is_two_block_mmo(O):
    # kappa = 128: x || b is 17 bytes, so PRF costs two block cipher calls
    x = bytes(range(16))
    iv = bytes([0x52]) * 16
    for b in (0, 1):
        h1 = _xor(openssl_aes128(iv, x), x)
        m2 = bytes([b]) + bytes(15)
        assert O.prf(O.INST_AES, b, x) == _xor(openssl_aes128(h1, m2), m2)
    assert O.prf(O.INST_AES, 0, x) != O.prf(O.INST_AES, 1, x)
    with pytest.raises(ValueError):
        O.prf(O.INST_AES, 2, x)
