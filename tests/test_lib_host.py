"""The native library without a GPU: it loads, exports every symbol its
header declares, and its host-side signer and hash functions produce the
oracle's bytes."""

import ctypes
import os
import random

import numpy as np
import pytest

import synthlog


def test_exports_every_declared_symbol(P):
    names = P.exported_symbols()
    assert len(names) >= 15
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_errors_and_version(P):
    assert P.poslo_version().startswith("poslo")
    assert "seed" in P._strerror(P.POSLO_E_SEED)


@pytest.mark.parametrize("inst", [0, 1])
def test_host_prf_and_hash_match_oracle(P, O, inst):
    rng = random.Random(inst)
    for n in list(range(0, 70)) + [100, 255, 256, 257, 300, 528]:
        d = bytes(rng.randrange(256) for _ in range(n))
        assert P.poslo_hash_host(inst, d) == O.H(inst, d), n
        for b in (0, 1):
            assert P.poslo_prf_host(inst, b, d) == O.prf(inst, b, d), (n, b)


@pytest.mark.parametrize("inst", [0, 1])
def test_host_signer_matches_oracle(P, O, inst):
    seed = synthlog.key_seed_bytes(0x40)
    prm = P.make_params(inst, 3, 2)
    sk, pk = P.poslo_kg(prm, seed)
    osk, opk = O.kg(O.Params(inst, 3, 2), seed)
    assert pk == opk
    lens = [0, 5, 16, 17, 31, 32, 48, 64, 3, 100, 7, 12, 9]
    data, off = synthlog.messages_var(9, np.array(lens))
    msgs = [bytes(data[off[k]:off[k + 1]]) for k in range(len(lens))]
    sigs = [P.poslo_sig(sk, m) for m in msgs]
    for k, m in enumerate(msgs):
        assert sigs[k] == O.sig(osk, m), k
    assert P.poslo_ds_export(sk) == O.ds_encode(osk.ds)
    assert P.poslo_agg(b"".join(sigs)) == O.agg(sigs)
    # the threaded batch signer gives the same bytes, variable or fixed length
    sk2, _ = P.poslo_kg(prm, seed)
    batch = P.poslo_sig_batch(sk2, data, offsets=off, nthreads=4)
    assert batch.tobytes() == b"".join(sigs)
    assert P.poslo_signer_count(sk2) == len(lens)


VARIANTS = [1 | 4, 2, 2 | 4]  # POSLO+ at kappa = 127, POSLO++ at 128 and 127


@pytest.mark.parametrize("inst", VARIANTS)
def test_host_prf_of_variants_matches_oracle(P, O, inst):
    rng = random.Random(inst + 7)
    for n in list(range(0, 40)) + [41, 42, 64]:
        d = bytearray(rng.randrange(256) for _ in range(n))
        if n == 16:
            d[15] &= 0x7F  # a 127-bit seed
        for b in (0, 1):
            assert P.poslo_prf_host(inst, b, bytes(d)) == O.prf(inst, b, bytes(d)), (n, b)
    if inst & 4:
        with pytest.raises(P.PosloError):
            P.poslo_prf_host(inst, 0, bytes(15) + b"\x80")
    if inst & 3 == 2:
        with pytest.raises(P.PosloError):
            P.poslo_hash_host(inst, b"abc")
    else:
        assert P.poslo_hash_host(inst, b"abc") == O.H(inst, b"abc")


@pytest.mark.parametrize("inst", VARIANTS)
def test_host_signer_of_variants_matches_oracle(P, O, inst):
    seed = synthlog.key_seed_bytes(0x41)
    prm = P.make_params(inst, 3, 2)
    sk, pk = P.poslo_kg(prm, seed)
    osk, opk = O.kg(O.Params(inst, 3, 2), seed)
    assert pk == opk
    lens = [0, 5, 16, 17, 31, 30, 1, 3, 12, 9, 31]
    data, off = synthlog.messages_var(10, np.array(lens))
    msgs = [bytes(data[off[k]:off[k + 1]]) for k in range(len(lens))]
    sigs = [P.poslo_sig(sk, m) for m in msgs]
    for k, m in enumerate(msgs):
        assert sigs[k] == O.sig(osk, m), k
    assert P.poslo_ds_export(sk) == O.ds_encode(osk.ds)
    sk2, _ = P.poslo_kg(prm, seed)
    assert P.poslo_sig_batch(sk2, data, offsets=off, nthreads=3).tobytes() == b"".join(sigs)
    if inst & 3 == 2:
        # Add_q takes at most 31 bytes; the refused call leaves the state alone
        with pytest.raises(P.PosloError) as ei:
            P.poslo_sig(sk, bytes(32))
        assert ei.value.status == P.POSLO_E_INVAL
        assert P.poslo_signer_count(sk) == len(lens)
        with pytest.raises(P.PosloError):
            P.poslo_sig_batch(sk2, np.zeros((2, 32), np.uint8))
        assert P.poslo_signer_count(sk2) == len(lens)


@pytest.mark.parametrize("inst", [1 | 8, 0 | 8, 1 | 4 | 8])
def test_host_signer_fourq_matches_oracle(P, O, inst):
    """The host signer over FourQ gives the oracle's key, signatures, ds and
    aggregate tag byte for byte."""
    seed = synthlog.key_seed_bytes(0x42)
    prm = P.make_params(inst, 3, 2, bpv_v=64, bpv_k=8)
    sk, pk = P.poslo_kg(prm, seed)
    osk, opk = O.kg(O.Params(inst, 3, 2, v=64, k=8), seed)
    assert pk == opk
    lens = [0, 5, 16, 17, 31, 48, 3, 100, 9]
    data, off = synthlog.messages_var(13, np.array(lens))
    msgs = [bytes(data[off[k]:off[k + 1]]) for k in range(len(lens))]
    sigs = [P.poslo_sig(sk, m) for m in msgs]
    for k, m in enumerate(msgs):
        assert sigs[k] == O.sig(osk, m), k
    assert P.poslo_ds_export(sk) == O.ds_encode(osk.ds)
    assert P.poslo_agg(b"".join(sigs), inst) == O.agg(sigs, inst)
    sk2, _ = P.poslo_kg(prm, seed)
    assert P.poslo_sig_batch(sk2, data, offsets=off, nthreads=3).tobytes() == b"".join(sigs)
    # a commitment that is not a FourQ point
    bad = bytearray(sigs[0])
    bad[32:48] = (2 ** 127 - 1).to_bytes(16, "little")
    with pytest.raises(P.PosloError) as ei:
        P.poslo_agg(bytes(bad), inst)
    assert ei.value.status == P.POSLO_E_ENCODING


def test_instantiation_words(P):
    for inst in (0, 1, 2, 5, 6, 8, 9, 13):
        assert P.lib().poslo_inst_valid(inst) == 1
        P.poslo_kg(P.make_params(inst, 1, 1, bpv_v=16, bpv_k=4), bytes(32))
    for inst in (3, 4, 7, 10, 12, 14, 16, 0x101):
        assert P.lib().poslo_inst_valid(inst) == 0
        with pytest.raises(P.PosloError):
            P.poslo_kg(P.make_params(inst, 1, 1), bytes(32))


def test_signer_exhaustion_and_bad_params(P):
    prm = P.make_params(1, 1, 1)
    sk, pk = P.poslo_kg(prm, bytes(32))
    for _ in range(4):
        P.poslo_sig(sk, b"m")
    with pytest.raises(P.PosloError) as ei:
        P.poslo_sig(sk, b"m")
    assert ei.value.status == -6
    with pytest.raises(P.PosloError):
        P.poslo_kg(P.make_params(7, 1, 1), bytes(32))
    with pytest.raises(P.PosloError):
        P.poslo_kg(P.make_params(1, 1, 1, bpv_v=1000), bytes(32))


def test_agg_rejects_undecodable_commitment(P):
    bad = bytearray(80)
    bad[32:64] = (2 ** 255 - 19 + 1).to_bytes(32, "little")  # y >= p
    with pytest.raises(P.PosloError) as ei:
        P.poslo_agg(bytes(bad))
    assert ei.value.status == -5


def _ccd_blob(ds=b"\x00", n_umb=2, invalid=((5, b"\x07" * 80),)):
    out = bytearray(b"PCCD") + (1).to_bytes(4, "little")
    for v in (1, 3, 4):
        out += v.to_bytes(4, "little")
    for v in (0, 100, 50):
        out += v.to_bytes(8, "little")
    out += len(ds).to_bytes(4, "little") + ds + b"\x01" * 64
    out += n_umb.to_bytes(8, "little") + b"\x02" * (64 * n_umb)
    out += len(invalid).to_bytes(8, "little")
    for t, sg in invalid:
        out += t.to_bytes(8, "little") + sg
    return bytes(out)


def test_ccd_serialization_roundtrip_and_strictness(P):
    blob = _ccd_blob()
    ccd = P.poslo_ccd_import(blob)
    assert ccd.invalid() == [5] and ccd.invalid_sig(0) == b"\x07" * 80
    assert ccd.valid_tag() == b"\x01" * 64
    tags, span = ccd.umbrellas()
    assert span == 50 and tags == [b"\x02" * 64] * 2
    assert ccd.export() == blob
    for bad in (blob[:-1], blob + b"\0", b"XCCD" + blob[4:]):
        with pytest.raises(P.PosloError):
            P.poslo_ccd_import(bad)


def test_request_keeps_device_buffers_alive(P):
    """A queued request's device buffers must outlive the caller's
    references: the server reads them when the request is launched."""
    import gc
    import weakref

    class DeviceBuffer:  # stands in for a CUDA tensor (data_ptr, numel)
        def __init__(self, n):
            self.n = n

        def data_ptr(self):
            return 0x10000

        def numel(self):
            return self.n

    bufs = [DeviceBuffer(16), DeviceBuffer(2), DeviceBuffer(80)]
    refs = [weakref.ref(b) for b in bufs]
    q = P.Request(0, 0, 1, bufs[0], bufs[1], 0, bufs[2], b"\x00", bytes(64))
    assert q.req.on_device == 1 and q.req.data_bytes == 16
    del bufs
    gc.collect()
    assert all(r() is not None for r in refs)
    del q
    gc.collect()
    assert all(r() is None for r in refs)
