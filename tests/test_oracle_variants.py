"""Pins of the oracle's parameter variants: kappa = 127 (the tree PRF in one
AES block) and POSLO++ (H = Add_q for messages below 32 bytes).

* The kappa = 127 tree PRF equals one block of the openssl AES under the MMO
  IV, xored with the block and reduced mod 2^127; other PRF inputs are the
  kappa = 128 PRF reduced mod 2^127; every seed of the tree has bit 127
  clear; SR equals the recursive tree equation and the paper's worked
  example keeps its shape.
* Add_q is additive in the message and the seed and refuses 32-byte
  messages; its digest changes by exactly the change of the message.
* Both variants: honest batches accept (POSLO-F and POSLO-C), every
  single-bit flip of a message is rejected, Distill's invalid set equals
  brute force and the injected corruption.
"""

import functools
import random
import shutil
import subprocess

import pytest

import synthlog

HAVE_OPENSSL = shutil.which("openssl") is not None


def openssl_aes128(key: bytes, block: bytes) -> bytes:
    out = subprocess.run(["openssl", "enc", "-aes-128-ecb", "-nopad", "-K", key.hex()],
                         input=block, capture_output=True, check=True).stdout
    assert len(out) == 16
    return out


@pytest.fixture
def memo_scalar_mult(O, monkeypatch):
    monkeypatch.setattr(O, "scalar_mult", functools.lru_cache(maxsize=None)(O.scalar_mult))


def variants(O):
    return [O.INST_AES | O.KAPPA127, O.INST_AES_ADDQ, O.INST_AES_ADDQ | O.KAPPA127]


@pytest.mark.skipif(not HAVE_OPENSSL, reason="openssl command not available")
def test_kappa127_tree_prf_is_one_block(O):
    rng = random.Random(71)
    iv = bytes([0x52] * 16)
    for inst in (O.INST_AES | O.KAPPA127, O.INST_AES_ADDQ | O.KAPPA127):
        for _ in range(6):
            x = rng.getrandbits(127)
            for b in (0, 1):
                blk = (x | (b << 127)).to_bytes(16, "little")
                h = bytes(u ^ v for u, v in zip(openssl_aes128(iv, blk), blk))
                want = (int.from_bytes(h, "little") & ((1 << 127) - 1)).to_bytes(16, "little")
                assert O.prf(inst, b, x.to_bytes(16, "little")) == want
        # a one-time seed's input is longer: the kappa = 128 PRF, reduced
        z = bytes(rng.randrange(256) for _ in range(20))
        full = int.from_bytes(O.prf(O.INST_AES, 0, z), "little")
        assert O.prf(inst, 0, z) == (full & ((1 << 127) - 1)).to_bytes(16, "little")
        with pytest.raises(ValueError):
            O.prf(inst, 0, (1 << 127).to_bytes(16, "little"))


def test_kappa127_seed_tree(O):
    inst = O.INST_AES | O.KAPPA127
    prm = O.Params(inst, 3, 0)
    signer, _ = O.kg(prm, synthlog.key_seed_bytes(5))
    root = signer.root
    assert int.from_bytes(root, "little") >> 127 == 0
    dss = []
    for i in range(prm.n1):
        signer.ds, x0 = O.SSO(inst, signer.ds, root, prm.log2_n1, i)
        assert x0 == O.tree_node(inst, root, prm.log2_n1, 0, i)
        assert int.from_bytes(x0, "little") >> 127 == 0
        dss.append(list(signer.ds))
        for ip in range(i + 1):
            assert O.SR(inst, signer.ds, ip) == O.tree_node(inst, root, prm.log2_n1, 0, ip)
    # the paper's worked example keeps its shape: ds_5 = {x_2[0], x_1[2]}
    assert [(n.depth, n.index) for n in dss[5]] == [(2, 0), (1, 2)]
    # kappa changes the seeds
    assert O.tree_node(O.INST_AES, root, 3, 0, 5) != O.tree_node(inst, root, 3, 0, 5)


def test_addq_digest(O):
    inst = O.INST_AES_ADDQ
    x = bytes(range(16))
    m = bytes(range(100, 131))  # 31 bytes
    e = O.digest_int(inst, m, x)
    assert O.digest_int(inst, b"", bytes(16)) == 0
    # additive in the message and in the seed
    m2 = bytearray(m)
    m2[3] ^= 0x10
    d = int.from_bytes(bytes(m2), "little") - int.from_bytes(m, "little")
    assert (O.digest_int(inst, bytes(m2), x) - e) % O.Q == d % O.Q
    x2 = bytearray(x)
    x2[15] ^= 0x80
    assert (O.digest_int(inst, m, bytes(x2)) - e) % O.Q == (1 << 127) % O.Q or \
        (e - O.digest_int(inst, m, bytes(x2))) % O.Q == (1 << 127) % O.Q
    # the largest message is still below q
    assert O.digest_int(inst, b"\xff" * 31, bytes(16)) == (1 << 248) - 1
    with pytest.raises(ValueError):
        O.digest_int(inst, bytes(32), x)


@pytest.mark.parametrize("which", [0, 1, 2])
def test_variant_schemes_accept_and_reject(O, which, memo_scalar_mult):
    inst = variants(O)[which]
    prm = O.Params(inst, 2, 1)
    msgs = [bytes(r) for r in synthlog.messages_fixed(61, 3, 8)]
    pk, sigs, ds, tag, signer = O.sign_batch(prm, synthlog.key_seed_bytes(0x22), msgs)
    assert O.aver(prm, pk, msgs, 0, ds, tag)
    seeds = O.epoch_seeds(prm, O.ds_decode(ds), 0, 3)
    for t, sg in enumerate(sigs):
        assert O.entry_valid(prm, pk, msgs[t], t, sg, seeds[t >> prm.log2_n2])
        if O.kappa_of(inst) == 127:
            assert sg[79] >> 7 == 0
    for pos in range(3):
        for bit in range(64):
            mm = bytearray(msgs[pos])
            mm[bit // 8] ^= 1 << (bit % 8)
            assert not O.aver(prm, pk, msgs[:pos] + [bytes(mm)] + msgs[pos + 1:], 0, ds, tag), (pos, bit)
    # Distill: one flipped message bit and one flipped x bit
    cm, cs = list(msgs), list(sigs)
    cm[1] = bytes([cm[1][0] ^ 4]) + cm[1][1:]
    cs[2] = cs[2][:70] + bytes([cs[2][70] ^ 1]) + cs[2][71:]
    ccd = O.distill(prm, pk, cm, cs, 0, ds, 2)
    brute = [t for t in range(3) if not O.entry_valid(prm, pk, cm[t], t, cs[t], seeds[t >> prm.log2_n2])]
    assert [t for t, _ in ccd.invalid] == brute == [1, 2]
    # POSLO-C under the same instantiation
    prmc = O.Params(inst, 2, 1)
    cmsgs = [bytes(r) for r in synthlog.messages_fixed(62, 6, 12)]
    pkc, s_list, dsc, _ = O.posloc_sign_batch(prmc, synthlog.key_seed_bytes(0x23), cmsgs)
    eps = [(i, cmsgs[2 * i:2 * i + 2]) for i in range(3)]
    assert O.posloc_aver(prmc, pkc, eps, dsc, O.posloc_agg_s(s_list))
    assert not O.posloc_aver(prmc, pkc, eps, dsc, O.posloc_agg_s(s_list[:2] + [s_list[1]]))


def test_variant_rules(O):
    with pytest.raises(ValueError):
        O.inst_base(O.INST_SHA256 | O.KAPPA127)  # kappa = 127 needs the AES-based PRF
    with pytest.raises(ValueError):
        O.inst_base(3)
    prm = O.Params(O.INST_AES_ADDQ, 1, 1)
    with pytest.raises(ValueError):
        O.sign_batch(prm, synthlog.key_seed_bytes(1), [bytes(32)])
