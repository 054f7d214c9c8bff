"""Python binding of libposlo, the POSLO-F verifier library for MI355X.

Argument marshalling only: every step of signing and verification runs in
the native library (HIP kernels on the GPU, C++ on the host).  Functions keep
the C ABI's names (include/poslo.h).  Device buffers are torch CUDA tensors;
streams are torch streams.  The library must be built (``_build.build()``);
importing the functions without it raises, there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libposlo.so")

INST_SHA256 = 0
INST_AES = 1
INST_AES_ADDQ = 2  # POSLO++ (H = Add_q, messages of at most 31 bytes)
KAPPA127 = 4       # flag on an AES-based instantiation: kappa = 127
GROUP_FOURQ = 8    # flag: the FourQ group (POSLO and POSLO+)

POSLO_OK = 0
POSLO_E_INVAL = -1
POSLO_E_NOMEM = -2
POSLO_E_DEVICE = -3
POSLO_E_SEED = -4
POSLO_E_ENCODING = -5
POSLO_E_EXHAUSTED = -6
POSLO_E_BUSY = -7
# limit of the allocation-free AVer entry point (include/poslo.h)
POSLO_AVER_FIXED_MAX_EPOCHS = 16384


class PosloError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_strerror(status)} ({status})")


class poslo_params(ctypes.Structure):
    _fields_ = [("inst", ctypes.c_uint32), ("log2_n1", ctypes.c_uint32), ("log2_n2", ctypes.c_uint32),
                ("bpv_v", ctypes.c_uint32), ("bpv_k", ctypes.c_uint32)]


class poslo_msgs(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("msg_len", ctypes.c_uint64),
                ("n", ctypes.c_uint64), ("t0", ctypes.c_uint64), ("data_bytes", ctypes.c_uint64),
                ("host", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class poslo_sign_job(ctypes.Structure):
    _fields_ = [("key", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("t0", ctypes.c_uint64),
                ("n", ctypes.c_uint64), ("entry_base", ctypes.c_uint64)]


class poslo_batch_job(ctypes.Structure):
    _fields_ = [("pk", ctypes.c_void_p), ("ds", ctypes.c_void_p), ("ds_len", ctypes.c_size_t),
                ("tag", ctypes.c_void_p), ("t0", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("entry_base", ctypes.c_uint64)]


class poslo_tuning(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("wg_per_cu", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("reserved", ctypes.c_int)]


class poslo_server_cfg(ctypes.Structure):
    _fields_ = [("params", poslo_params), ("n_streams", ctypes.c_uint32), ("max_group", ctypes.c_uint32),
                ("mem_bytes", ctypes.c_uint64), ("distill", ctypes.c_int), ("variant", ctypes.c_int),
                ("max_group_entries", ctypes.c_uint64)]


class poslo_request(ctypes.Structure):
    _fields_ = [("key_id", ctypes.c_uint32), ("on_device", ctypes.c_uint32), ("t0", ctypes.c_uint64),
                ("n", ctypes.c_uint64), ("data", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("msg_len", ctypes.c_uint64), ("data_bytes", ctypes.c_uint64), ("sigs", ctypes.c_void_p),
                ("ds", ctypes.c_void_p), ("ds_len", ctypes.c_size_t), ("tag", ctypes.c_void_p),
                ("user", ctypes.c_uint64)]


class poslo_result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("user", ctypes.c_uint64), ("status", ctypes.c_int),
                ("accept", ctypes.c_int), ("n_invalid", ctypes.c_uint64), ("entries", ctypes.c_uint64),
                ("t_submit_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double),
                ("t_launch_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


class poslo_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("in_flight", ctypes.c_uint64), ("entries_completed", ctypes.c_uint64),
                ("groups_launched", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64),
                ("bytes_peak", ctypes.c_uint64), ("latency_p50_ms", ctypes.c_double),
                ("latency_p99_ms", ctypes.c_double), ("elapsed_ms", ctypes.c_double)]


def make_params(inst: int, log2_n1: int, log2_n2: int, bpv_v: int = 1024, bpv_k: int = 16) -> poslo_params:
    return poslo_params(inst, log2_n1, log2_n2, bpv_v, bpv_k)


_lib = None
_VP = ctypes.c_void_p
_U8P = ctypes.c_char_p
_SZ = ctypes.c_size_t
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32
_I = ctypes.c_int


def lib():
    """The loaded native library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libposlo.so is not built at {LIB_PATH}; run paper_2506_08781_amd._build.build()")
        # torch ships its own HIP runtime and asks for it by an unversioned
        # name; loading torch first lets this library bind to that same
        # runtime (same soname) instead of bringing up a second one.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        sigs = {
            "poslo_version": ([], ctypes.c_char_p),
            "poslo_strerror": ([_I], ctypes.c_char_p),
            "poslo_kg": ([P(poslo_params), _U8P, P(_VP), _VP], _I),
            "poslo_signer_free": ([_VP], None),
            "poslo_sig": ([_VP, _U8P, _SZ, _VP], _I),
            "poslo_sig_batch": ([_VP, _VP, _VP, _U64, _U64, _VP, _I], _I),
            "poslo_signer_count": ([_VP], _U64),
            "poslo_ds_export": ([_VP, _VP, _SZ, P(_SZ)], _I),
            "poslo_agg": ([_VP, _SZ, _U64, _VP], _I),
            "poslo_agg_inst": ([_U32, _VP, _SZ, _U64, _VP], _I),
            "poslo_inst_valid": ([_U32], _I),
            "poslo_prf_host": ([_U32, _U32, _U8P, _SZ, _VP], _I),
            "poslo_hash_host": ([_U32, _U8P, _SZ, _VP], _I),
            "poslo_ctx_create": ([_I, P(_VP)], _I),
            "poslo_ctx_destroy": ([_VP], None),
            "poslo_aver": ([_VP, P(poslo_params), _U8P, P(poslo_msgs), _U8P, _SZ, _U8P, _VP, P(_I), _VP], _I),
            "poslo_aver_fixed": ([_VP, P(poslo_params), _U8P, P(poslo_msgs), _U8P, _SZ, _U8P, _VP, P(_I), _VP],
                                 _I),
            "poslo_ekeys": ([_VP, P(poslo_params), P(poslo_msgs), _U8P, _SZ, _VP, _VP, _VP], _I),
            "poslo_ctx_profile": ([_VP, _I], _I),
            "poslo_ctx_kernel_time": ([_VP, _I, _I, P(ctypes.c_double), P(_U64)], _I),
            "poslo_agg_variant_count": ([], _I),
            "poslo_agg_variant_name": ([_I], ctypes.c_char_p),
            "poslo_ctx_set_tuning": ([_VP, _I, _I], _I),
            "poslo_distill": ([_VP, P(poslo_params), _U8P, P(poslo_msgs), _VP, _U8P, _SZ, _U32, _VP, P(_VP)], _I),
            "poslo_ccd_invalid": ([_VP, P(P(_U64)), P(_U64)], _I),
            "poslo_ccd_invalid_sig": ([_VP, _U64, _VP], _I),
            "poslo_ccd_valid_tag": ([_VP, _VP], _I),
            "poslo_ccd_umbrellas": ([_VP, _VP, _SZ, P(_U64), P(_U64)], _I),
            "poslo_ccd_export": ([_VP, _VP, _SZ, P(_SZ)], _I),
            "poslo_ccd_import": ([_U8P, _SZ, P(_VP)], _I),
            "poslo_ccd_free": ([_VP], None),
            "poslo_sebver": ([_VP, P(poslo_params), _U8P, P(poslo_msgs), _VP, ctypes.c_char, _VP, _SZ, P(_SZ),
                              _VP], _I),
            "poslo_c_key_load": ([_VP, P(poslo_params), _U8P, _SZ, P(_VP)], _I),
            "poslo_c_key_free": ([_VP], None),
            "poslo_c_aver": ([_VP, P(poslo_params), _VP, P(poslo_msgs), _U8P, _SZ, _U8P, _VP, P(_I), _VP], _I),
            "poslo_c_distill": ([_VP, P(poslo_params), _VP, P(poslo_msgs), _U8P, _U8P, _SZ, _U32, _VP, P(_VP)],
                                _I),
            "poslo_c_sebver": ([_VP, P(poslo_params), _VP, P(poslo_msgs), _VP, ctypes.c_char, _VP, _SZ, P(_SZ),
                                _VP], _I),
            "poslo_audit_begin": ([_VP, P(poslo_params), _U8P, _U8P, _SZ, _U64, P(_VP)], _I),
            "poslo_audit_feed": ([_VP, P(poslo_msgs), _VP], _I),
            "poslo_audit_position": ([_VP, P(_U64)], _I),
            "poslo_audit_finish": ([_VP, _U8P, _VP, P(_I), _VP], _I),
            "poslo_audit_export": ([_VP, _VP, _VP, _SZ, P(_SZ)], _I),
            "poslo_audit_resume": ([_VP, _U8P, _SZ, P(poslo_params), P(_VP)], _I),
            "poslo_audit_free": ([_VP], None),
            "poslo_valu_probe": ([_I, _I, _U32, _U32, P(ctypes.c_double), P(ctypes.c_double)], _I),
            "poslo_synth_messages": ([_U32, P(poslo_msgs), _VP, _VP], _I),
            "poslo_gpu_keys_create": ([_VP, P(poslo_params), _U8P, _U32, P(_VP), _VP], _I),
            "poslo_gpu_keys_free": ([_VP], None),
            "poslo_gpu_sign": ([_VP, P(poslo_sign_job), _U32, _VP, _VP, _VP, _VP, _VP, _SZ, _VP], _I),
            "poslo_ctx_keys_load": ([_VP, _U8P, _SZ, P(_SZ)], _I),
            "poslo_ctx_keys_widen": ([_VP, _U8P, _SZ], _I),
            "poslo_batch_variant_count": ([], _I),
            "poslo_batch_variant_name": ([_I], ctypes.c_char_p),
            "poslo_verify_batch": ([_VP, P(poslo_params), P(poslo_batch_job), _U32, _VP, _VP, _U64, _VP, _I,
                                    P(poslo_tuning), _VP, _VP, _VP, _SZ, P(_SZ)], _I),
            "poslo_autotune_batch": ([_VP, P(poslo_params), P(poslo_batch_job), _U32, _VP, _VP, _U64, _I, _VP,
                                      P(poslo_tuning), P(ctypes.c_double)], _I),
            "poslo_batch_forget": ([_VP], _I),
            "poslo_server_create": ([_I, P(poslo_server_cfg), P(_VP)], _I),
            "poslo_server_register_keys": ([_VP, _VP, _U8P, _SZ], _I),
            "poslo_server_submit": ([_VP, P(poslo_request), P(_U64)], _I),
            "poslo_server_poll": ([_VP, P(poslo_result), _SZ, P(_SZ), ctypes.c_double], _I),
            "poslo_server_take_invalid": ([_VP, _U64, _VP, _SZ, P(_SZ)], _I),
            "poslo_server_key_state": ([_VP, _U32, _VP, P(_U64)], _I),
            "poslo_server_stats_get": ([_VP, P(poslo_server_stats)], _I),
            "poslo_server_destroy": ([_VP], None),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    """Names of the C ABI functions declared in include/poslo.h."""
    import re
    hdr = os.path.join(os.path.dirname(HERE), "include", "poslo.h")
    with open(hdr) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(poslo_[a-z0-9_]+)\s*\(", text)))


def _strerror(status: int) -> str:
    try:
        return lib().poslo_strerror(status).decode()
    except Exception:
        return "error"


def _check(status: int, where: str):
    if status != POSLO_OK:
        raise PosloError(status, where)


def poslo_version() -> str:
    return lib().poslo_version().decode()


# ----------------------------------------------------------------- signer

class Signer:
    """Owns a poslo_signer*."""

    def __init__(self, handle: int, params: poslo_params):
        self.handle = ctypes.c_void_p(handle)
        self.params = params

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and h.value and _lib is not None:
            _lib.poslo_signer_free(h)
            self.handle = None


def poslo_kg(params: poslo_params, seed: bytes):
    if len(seed) != 32:
        raise ValueError("seed must be 32 bytes")
    h = ctypes.c_void_p()
    pk = ctypes.create_string_buffer(32)
    _check(lib().poslo_kg(ctypes.byref(params), seed, ctypes.byref(h), pk), "poslo_kg")
    return Signer(h.value, params), pk.raw


def poslo_sig(sk: Signer, m: bytes) -> bytes:
    out = ctypes.create_string_buffer(80)
    _check(lib().poslo_sig(sk.handle, bytes(m), len(m), out), "poslo_sig")
    return out.raw


def poslo_sig_batch(sk: Signer, msgs: np.ndarray, offsets: np.ndarray | None = None, nthreads: int = 0) -> np.ndarray:
    """Sign consecutive entries.  msgs: uint8 (n, L) array, or a flat uint8
    array with offsets (n+1 uint64).  Returns a uint8 (n, 80) array."""
    if offsets is None:
        msgs = np.ascontiguousarray(msgs, dtype=np.uint8)
        n, L = msgs.shape
        off_ptr = None
    else:
        msgs = np.ascontiguousarray(msgs, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        n, L = offsets.size - 1, 0
        off_ptr = offsets.ctypes.data
    sigs = np.empty((n, 80), dtype=np.uint8)
    _check(lib().poslo_sig_batch(sk.handle, msgs.ctypes.data if msgs.size else None, off_ptr, L, n,
                                 sigs.ctypes.data if n else None, nthreads), "poslo_sig_batch")
    return sigs


def poslo_signer_count(sk: Signer) -> int:
    return lib().poslo_signer_count(sk.handle)


def poslo_ds_export(sk: Signer) -> bytes:
    buf = ctypes.create_string_buffer(1 + 24 * 32)
    ln = ctypes.c_size_t()
    _check(lib().poslo_ds_export(sk.handle, buf, len(buf), ctypes.byref(ln)), "poslo_ds_export")
    return buf.raw[:ln.value]


def poslo_agg(sigs, inst: int | None = None) -> bytes:
    """The aggregate tag; inst (an instantiation word) selects the group,
    edwards25519 when absent."""
    arr = np.ascontiguousarray(np.frombuffer(bytes(sigs), dtype=np.uint8) if isinstance(sigs, (bytes, bytearray))
                               else sigs, dtype=np.uint8).reshape(-1, 80)
    tag = ctypes.create_string_buffer(64)
    ptr = arr.ctypes.data if arr.size else None
    if inst is None:
        _check(lib().poslo_agg(ptr, 80, arr.shape[0], tag), "poslo_agg")
    else:
        _check(lib().poslo_agg_inst(inst, ptr, 80, arr.shape[0], tag), "poslo_agg_inst")
    return tag.raw


def poslo_prf_host(inst: int, b: int, data: bytes) -> bytes:
    out = ctypes.create_string_buffer(16)
    _check(lib().poslo_prf_host(inst, b, bytes(data), len(data), out), "poslo_prf_host")
    return out.raw


def poslo_hash_host(inst: int, data: bytes) -> bytes:
    out = ctypes.create_string_buffer(32)
    _check(lib().poslo_hash_host(inst, bytes(data), len(data), out), "poslo_hash_host")
    return out.raw


# --------------------------------------------------------------- verifier

class Ctx:
    """Owns a poslo_ctx* on one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().poslo_ctx_create(device, ctypes.byref(h)), "poslo_ctx_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle and self.handle.value:
            lib().poslo_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def poslo_ctx_create(device: int = 0) -> Ctx:
    return Ctx(device)


(POSLO_KT_SEED, POSLO_KT_AGG, POSLO_KT_FINAL, POSLO_KT_EKEYS, POSLO_KT_VERIFY, POSLO_KT_COMPACT,
 POSLO_KT_BATCH_HOT, POSLO_KT_BATCH) = range(8)
POSLO_PROFILE_ALL = 0xFF


def poslo_agg_variant_count() -> int:
    return lib().poslo_agg_variant_count()


def poslo_agg_variant_name(v: int) -> str:
    r = lib().poslo_agg_variant_name(v)
    if r is None:
        raise IndexError(v)
    return r.decode()


def poslo_ctx_set_tuning(ctx: Ctx, agg_variant: int = -1, wg_per_cu: int = 0) -> None:
    _check(lib().poslo_ctx_set_tuning(ctx.handle, agg_variant, wg_per_cu), "poslo_ctx_set_tuning")


def poslo_ctx_profile(ctx: Ctx, kernels) -> None:
    """Time the kernels whose POSLO_KT_* ids are given (an iterable of ids;
    True: all of them; False or empty: none)."""
    if kernels is True:
        mask = POSLO_PROFILE_ALL
    elif kernels is False or kernels is None:
        mask = 0
    else:
        mask = 0
        for k in kernels:
            mask |= 1 << int(k)
    _check(lib().poslo_ctx_profile(ctx.handle, mask), "poslo_ctx_profile")


def poslo_ctx_kernel_time(ctx: Ctx, kernel: int, reset: bool = False) -> tuple[float, int]:
    """(accumulated milliseconds, timed launches) of one kernel."""
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    _check(lib().poslo_ctx_kernel_time(ctx.handle, kernel, 1 if reset else 0, ctypes.byref(ms), ctypes.byref(n)),
           "poslo_ctx_kernel_time")
    return ms.value, n.value


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def make_msgs(data, offsets=None, msg_len: int = 0, n: int | None = None, t0: int = 0) -> poslo_msgs:
    """Batch descriptor over torch tensors: data uint8 (n, L) or flat,
    offsets uint64 (int64) (n+1) or None.  CUDA tensors give a device batch;
    CPU tensors (pinned for an asynchronous copy) a host batch, which the
    library copies to the device itself."""
    host = 0 if data.is_cuda else 1
    if offsets is not None and offsets.is_cuda != data.is_cuda:
        raise ValueError("data and offsets must be in the same memory")
    if offsets is None:
        if data.dim() == 2:
            n_, L = data.shape
        else:
            if n is None:
                raise ValueError("n is required for a flat fixed-length buffer")
            n_, L = n, msg_len
        return poslo_msgs(data.data_ptr() if data.numel() else None, None, L, n_, t0, data.numel(), host)
    n_ = offsets.numel() - 1
    return poslo_msgs(data.data_ptr() if data.numel() else None, offsets.data_ptr(), 0, n_, t0, data.numel(),
                      host)


def poslo_aver(ctx: Ctx, params: poslo_params, pk: bytes, msgs: poslo_msgs, ds: bytes, tag: bytes,
               stream=None) -> tuple[bool, bytes]:
    """Aggregate verification of a device-resident batch.
    Returns (accept, e mod q as 32 LE bytes)."""
    acc = ctypes.c_int()
    e = ctypes.create_string_buffer(32)
    st = lib().poslo_aver(ctx.handle, ctypes.byref(params), bytes(pk), ctypes.byref(msgs), bytes(ds), len(ds),
                          bytes(tag), _stream_ptr(stream), ctypes.byref(acc), e)
    _check(st, "poslo_aver")
    return bool(acc.value), e.raw


def poslo_aver_fixed(ctx: Ctx, params: poslo_params, pk: bytes, msgs: poslo_msgs, ds: bytes, tag: bytes,
                     stream=None) -> tuple[bool, bytes]:
    """poslo_aver without device allocation (fixed per-device scratch; pk
    must be resident, see poslo_ctx_keys_load).  Returns (accept, e mod q)."""
    acc = ctypes.c_int()
    e = ctypes.create_string_buffer(32)
    st = lib().poslo_aver_fixed(ctx.handle, ctypes.byref(params), bytes(pk), ctypes.byref(msgs), bytes(ds),
                                len(ds), bytes(tag), _stream_ptr(stream), ctypes.byref(acc), e)
    _check(st, "poslo_aver_fixed")
    return bool(acc.value), e.raw


def poslo_ekeys(ctx: Ctx, params: poslo_params, msgs: poslo_msgs, ds: bytes, stream=None):
    """Per-entry e_t mod q (uint8 (n, 32)) and x_t (uint8 (n, 16)) as CUDA tensors."""
    import torch
    n = msgs.n
    dev = torch.device("cuda", ctx.device)
    e = torch.empty((max(n, 1), 32), dtype=torch.uint8, device=dev)
    x = torch.empty((max(n, 1), 16), dtype=torch.uint8, device=dev)
    st = lib().poslo_ekeys(ctx.handle, ctypes.byref(params), ctypes.byref(msgs), bytes(ds), len(ds),
                           e.data_ptr(), x.data_ptr(), _stream_ptr(stream))
    _check(st, "poslo_ekeys")
    return e[:n], x[:n]


# ------------------------------------------------------ distill / sebver

class CCD:
    """Owns a poslo_ccd* (cold cryptographic data of a distilled batch)."""

    def __init__(self, handle):
        self.handle = ctypes.c_void_p(handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and h.value and _lib is not None:
            _lib.poslo_ccd_free(h)
            self.handle = None

    def invalid(self) -> list[int]:
        p = ctypes.POINTER(ctypes.c_uint64)()
        n = ctypes.c_uint64()
        _check(lib().poslo_ccd_invalid(self.handle, ctypes.byref(p), ctypes.byref(n)), "poslo_ccd_invalid")
        return [p[k] for k in range(n.value)]

    def invalid_sig(self, k: int) -> bytes:
        out = ctypes.create_string_buffer(80)
        _check(lib().poslo_ccd_invalid_sig(self.handle, k, out), "poslo_ccd_invalid_sig")
        return out.raw

    def valid_tag(self) -> bytes:
        out = ctypes.create_string_buffer(64)
        _check(lib().poslo_ccd_valid_tag(self.handle, out), "poslo_ccd_valid_tag")
        return out.raw

    def umbrellas(self) -> tuple[list[bytes], int]:
        n = ctypes.c_uint64()
        span = ctypes.c_uint64()
        _check(lib().poslo_ccd_umbrellas(self.handle, None, 0, ctypes.byref(n), ctypes.byref(span)),
               "poslo_ccd_umbrellas")
        buf = ctypes.create_string_buffer(max(1, 64 * n.value))
        _check(lib().poslo_ccd_umbrellas(self.handle, buf, len(buf), ctypes.byref(n), ctypes.byref(span)),
               "poslo_ccd_umbrellas")
        return [buf.raw[64 * k:64 * k + 64] for k in range(n.value)], span.value

    def export(self) -> bytes:
        ln = ctypes.c_size_t()
        lib().poslo_ccd_export(self.handle, None, 0, ctypes.byref(ln))
        buf = ctypes.create_string_buffer(ln.value)
        _check(lib().poslo_ccd_export(self.handle, buf, len(buf), ctypes.byref(ln)), "poslo_ccd_export")
        return buf.raw[:ln.value]


def poslo_ccd_import(data: bytes) -> CCD:
    h = ctypes.c_void_p()
    _check(lib().poslo_ccd_import(bytes(data), len(data), ctypes.byref(h)), "poslo_ccd_import")
    return CCD(h.value)


def poslo_distill(ctx: Ctx, params: poslo_params, pk: bytes, msgs: poslo_msgs, sigs, ds: bytes,
                  n_umbrella: int, stream=None) -> CCD:
    """Distill a batch; sigs is a uint8 tensor of 80*n bytes in the batch's
    memory (CUDA for a device batch, CPU for a host batch)."""
    h = ctypes.c_void_p()
    st = lib().poslo_distill(ctx.handle, ctypes.byref(params), bytes(pk), ctypes.byref(msgs),
                             sigs.data_ptr() if sigs.numel() else None, bytes(ds), len(ds), n_umbrella,
                             _stream_ptr(stream), ctypes.byref(h))
    _check(st, "poslo_distill")
    return CCD(h.value)


def poslo_sebver(ctx: Ctx, params: poslo_params, pk: bytes, msgs: poslo_msgs, ccd: CCD, mode: str,
                 stream=None) -> list[bool]:
    cap = max(1, len(ccd.invalid()), len(ccd.umbrellas()[0]))
    bits = ctypes.create_string_buffer(cap)
    nb = ctypes.c_size_t()
    st = lib().poslo_sebver(ctx.handle, ctypes.byref(params), bytes(pk), ctypes.byref(msgs), ccd.handle,
                            mode.encode(), bits, cap, ctypes.byref(nb), _stream_ptr(stream))
    _check(st, "poslo_sebver")
    return [bool(b) for b in bits.raw[:nb.value]]


# ------------------------------------------------------------- POSLO-C

class CKey:
    """Owns a poslo_c_key* (a POSLO-C public key loaded on a device)."""

    def __init__(self, handle):
        self.handle = ctypes.c_void_p(handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and h.value and _lib is not None:
            _lib.poslo_c_key_free(h)
            self.handle = None


def poslo_c_key_load(ctx: Ctx, params: poslo_params, pk: bytes) -> CKey:
    h = ctypes.c_void_p()
    _check(lib().poslo_c_key_load(ctx.handle, ctypes.byref(params), bytes(pk), len(pk), ctypes.byref(h)),
           "poslo_c_key_load")
    return CKey(h.value)


def poslo_c_aver(ctx: Ctx, params: poslo_params, key: CKey, msgs: poslo_msgs, ds: bytes, s: bytes,
                 stream=None) -> tuple[bool, bytes]:
    """POSLO-C aggregate verification of whole epochs against the aggregate
    s (32 bytes).  Returns (accept, e mod q)."""
    acc = ctypes.c_int()
    e = ctypes.create_string_buffer(32)
    st = lib().poslo_c_aver(ctx.handle, ctypes.byref(params), key.handle, ctypes.byref(msgs), bytes(ds), len(ds),
                            bytes(s), _stream_ptr(stream), ctypes.byref(acc), e)
    _check(st, "poslo_c_aver")
    return bool(acc.value), e.raw


def poslo_c_distill(ctx: Ctx, params: poslo_params, key: CKey, msgs: poslo_msgs, s_epochs: bytes, ds: bytes,
                    n_umbrella: int, stream=None) -> CCD:
    """POSLO-C Distill; s_epochs holds 32 bytes per epoch of the batch."""
    h = ctypes.c_void_p()
    st = lib().poslo_c_distill(ctx.handle, ctypes.byref(params), key.handle, ctypes.byref(msgs), bytes(s_epochs),
                               bytes(ds), len(ds), n_umbrella, _stream_ptr(stream), ctypes.byref(h))
    _check(st, "poslo_c_distill")
    return CCD(h.value)


def poslo_c_sebver(ctx: Ctx, params: poslo_params, key: CKey, msgs: poslo_msgs, ccd: CCD, mode: str,
                   stream=None) -> list[bool]:
    cap = max(1, len(ccd.invalid()), len(ccd.umbrellas()[0]))
    bits = ctypes.create_string_buffer(cap)
    nb = ctypes.c_size_t()
    st = lib().poslo_c_sebver(ctx.handle, ctypes.byref(params), key.handle, ctypes.byref(msgs), ccd.handle,
                              mode.encode(), bits, cap, ctypes.byref(nb), _stream_ptr(stream))
    _check(st, "poslo_c_sebver")
    return [bool(b) for b in bits.raw[:nb.value]]


# ------------------------------------------------------- streaming audit

class Audit:
    """Owns a poslo_audit* (AVer over a log fed in chunks)."""

    def __init__(self, handle):
        self.handle = ctypes.c_void_p(handle)

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "handle", None)
        if h and h.value and _lib is not None:
            _lib.poslo_audit_free(h)
            self.handle = None

    def feed(self, msgs: poslo_msgs, stream=None) -> None:
        _check(lib().poslo_audit_feed(self.handle, ctypes.byref(msgs), _stream_ptr(stream)), "poslo_audit_feed")

    def position(self) -> int:
        t = ctypes.c_uint64()
        _check(lib().poslo_audit_position(self.handle, ctypes.byref(t)), "poslo_audit_position")
        return t.value

    def finish(self, tag: bytes, stream=None) -> tuple[bool, bytes]:
        acc = ctypes.c_int()
        e = ctypes.create_string_buffer(32)
        _check(lib().poslo_audit_finish(self.handle, bytes(tag), _stream_ptr(stream), ctypes.byref(acc), e),
               "poslo_audit_finish")
        return bool(acc.value), e.raw

    def export(self, stream=None) -> bytes:
        ln = ctypes.c_size_t()
        lib().poslo_audit_export(self.handle, _stream_ptr(stream), None, 0, ctypes.byref(ln))
        buf = ctypes.create_string_buffer(ln.value)
        _check(lib().poslo_audit_export(self.handle, _stream_ptr(stream), buf, len(buf), ctypes.byref(ln)),
               "poslo_audit_export")
        return buf.raw[:ln.value]


def poslo_audit_begin(ctx: Ctx, params: poslo_params, pk: bytes, ds: bytes, t0: int = 0) -> Audit:
    h = ctypes.c_void_p()
    _check(lib().poslo_audit_begin(ctx.handle, ctypes.byref(params), bytes(pk), bytes(ds), len(ds), t0,
                                   ctypes.byref(h)), "poslo_audit_begin")
    return Audit(h.value)


def poslo_audit_resume(ctx: Ctx, state: bytes, params: poslo_params) -> Audit:
    h = ctypes.c_void_p()
    _check(lib().poslo_audit_resume(ctx.handle, bytes(state), len(state), ctypes.byref(params), ctypes.byref(h)),
           "poslo_audit_resume")
    return Audit(h.value)


# ------------------------------------------------- measurement utilities

PROBE_OPS = {"xor": 0, "perm": 1, "bitop3": 2, "add3": 3, "alignbit": 4, "mad64": 5}


def poslo_valu_probe(op: str, waves_per_simd: int = 8, iters: int = 4096, device: int = 0) -> tuple[float, float]:
    """Sustained lane operations per second of one VALU instruction kind at
    the given occupancy, and the timed launch's milliseconds."""
    rate = ctypes.c_double()
    ms = ctypes.c_double()
    _check(lib().poslo_valu_probe(device, PROBE_OPS[op], waves_per_simd, iters, ctypes.byref(rate),
                                  ctypes.byref(ms)), "poslo_valu_probe")
    return rate.value, ms.value


# --------------------------------------------------- device-side test data

def poslo_synth_messages(seed: int, msgs: poslo_msgs, out, stream=None) -> None:
    """Fill out (CUDA uint8 tensor at the layout msgs describes) with the
    seeded message bytes of entries t0 .. t0+n-1."""
    _check(lib().poslo_synth_messages(seed, ctypes.byref(msgs), out.data_ptr() if out.numel() else None,
                                      _stream_ptr(stream)), "poslo_synth_messages")


class GpuKeys:
    """Owns a poslo_gpu_keys* (signing keys held on the device)."""

    def __init__(self, handle, pks: list[bytes]):
        self.handle = ctypes.c_void_p(handle)
        self.pks = pks

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.poslo_gpu_keys_free(self.handle)
            self.handle = ctypes.c_void_p()


def poslo_gpu_keys_create(ctx: Ctx, params: poslo_params, seeds: list[bytes]) -> GpuKeys:
    n = len(seeds)
    blob = b"".join(bytes(s) for s in seeds)
    if len(blob) != 32 * n:
        raise ValueError("seeds must be 32 bytes each")
    pks = ctypes.create_string_buffer(max(1, 32 * n))
    h = ctypes.c_void_p()
    _check(lib().poslo_gpu_keys_create(ctx.handle, ctypes.byref(params), blob, n, ctypes.byref(h), pks),
           "poslo_gpu_keys_create")
    return GpuKeys(h.value, [pks.raw[32 * k:32 * k + 32] for k in range(n)])


DS_STRIDE = 1 + 32 * 24


def poslo_gpu_sign(keys: GpuKeys, jobs: list[tuple[int, int, int, int]], data, offsets, sigs,
                   want_ds: bool = True, stream=None):
    """Sign jobs (key, t0, n, entry_base) on the device.  data/offsets/sigs:
    CUDA tensors (sigs: uint8, 80 per global entry).  Returns (tags, ds)
    lists of bytes, one per job."""
    nj = len(jobs)
    arr = (poslo_sign_job * max(1, nj))()
    for k, (key, t0, n, base) in enumerate(jobs):
        arr[k] = poslo_sign_job(key, 0, t0, n, base)
    tags = ctypes.create_string_buffer(max(1, 64 * nj))
    ds = ctypes.create_string_buffer(max(1, DS_STRIDE * nj)) if want_ds else None
    st = lib().poslo_gpu_sign(keys.handle, arr, nj, data.data_ptr() if data.numel() else None,
                              offsets.data_ptr(), sigs.data_ptr() if sigs.numel() else None, tags, ds,
                              DS_STRIDE, _stream_ptr(stream))
    _check(st, "poslo_gpu_sign")
    out_tags = [tags.raw[64 * k:64 * k + 64] for k in range(nj)]
    out_ds = None
    if want_ds:
        raw = ds.raw
        out_ds = []
        for k in range(nj):
            rec = raw[DS_STRIDE * k:DS_STRIDE * (k + 1)]
            out_ds.append(rec[:1 + 24 * rec[0]])
    return out_tags, out_ds


# --------------------------------------------------- many signers per launch

def poslo_ctx_keys_load(ctx: Ctx, pks: list[bytes]) -> int:
    """Make the keys device-resident; returns the number of non-point keys."""
    blob = b"".join(bytes(p) for p in pks)
    bad = ctypes.c_size_t()
    st = lib().poslo_ctx_keys_load(ctx.handle, blob, len(pks), ctypes.byref(bad))
    if st not in (POSLO_OK, POSLO_E_ENCODING):
        _check(st, "poslo_ctx_keys_load")
    return bad.value


def poslo_ctx_keys_widen(ctx: Ctx, pks: list[bytes]) -> None:
    """Give resident keys their wide table (48 MiB each) for the individual
    checks; raises on a non-point key or when device memory runs out."""
    blob = b"".join(bytes(p) for p in pks)
    _check(lib().poslo_ctx_keys_widen(ctx.handle, blob, len(pks)), "poslo_ctx_keys_widen")


def poslo_batch_variant_count() -> int:
    return lib().poslo_batch_variant_count()


def poslo_batch_variant_name(v: int) -> str:
    r = lib().poslo_batch_variant_name(v)
    if r is None:
        raise ValueError(f"no batch variant {v}")
    return r.decode()


class BatchJobs:
    """A ctypes job table plus the host buffers it points into."""

    def __init__(self, jobs: list[dict]):
        self._keep = []
        self.n = len(jobs)
        self.arr = (poslo_batch_job * max(1, self.n))()
        for k, j in enumerate(jobs):
            pk = ctypes.create_string_buffer(bytes(j["pk"]), 32)
            tag = ctypes.create_string_buffer(bytes(j["tag"]), 64)
            dsb = bytes(j["ds"])
            ds = ctypes.create_string_buffer(dsb, max(1, len(dsb)))
            self._keep += [pk, tag, ds]
            self.arr[k] = poslo_batch_job(ctypes.addressof(pk), ctypes.addressof(ds), len(dsb),
                                          ctypes.addressof(tag), j["t0"], j["n"], j["entry_base"])


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, poslo_tuning):
        return ctypes.byref(t)
    variant, wg, graph = t
    return ctypes.byref(poslo_tuning(variant, wg, 1 if graph else 0, 0))


def poslo_verify_batch(ctx: Ctx, params: poslo_params, jobs: BatchJobs, data, offsets, sigs=None,
                       distill: int = 1, tuning=None, stream=None, cap: int | None = None):
    """AVer of every job in one launch.  With sigs, distill = 1 verifies the
    entries of rejected jobs individually, 2 those of every job.  Returns
    (accept list, sorted invalid (job, t) list, or None without sigs)."""
    acc = ctypes.create_string_buffer(max(1, jobs.n))
    n_inv = ctypes.c_size_t()
    mode = distill if sigs is not None else 0
    cap = (4096 if cap is None else cap) if mode else 0
    inv = (ctypes.c_uint64 * max(2, 2 * cap))()
    st = lib().poslo_verify_batch(ctx.handle, ctypes.byref(params), jobs.arr, jobs.n,
                                  data.data_ptr() if data.numel() else None, offsets.data_ptr(), data.numel(),
                                  sigs.data_ptr() if mode and sigs.numel() else None, mode,
                                  _tuning(tuning), _stream_ptr(stream), acc, inv, cap,
                                  ctypes.byref(n_inv) if mode else None)
    _check(st, "poslo_verify_batch")
    accept = [bool(b) for b in acc.raw[:jobs.n]]
    if not mode:
        return accept, None
    if n_inv.value > cap:
        return poslo_verify_batch(ctx, params, jobs, data, offsets, sigs, distill, tuning, stream, cap=n_inv.value)
    return accept, [(int(inv[2 * k]), int(inv[2 * k + 1])) for k in range(n_inv.value)]


def poslo_autotune_batch(ctx: Ctx, params: poslo_params, jobs: BatchJobs, data, offsets, reps: int = 3,
                         stream=None) -> tuple[poslo_tuning, float]:
    best = poslo_tuning()
    ms = ctypes.c_double()
    st = lib().poslo_autotune_batch(ctx.handle, ctypes.byref(params), jobs.arr, jobs.n,
                                    data.data_ptr() if data.numel() else None, offsets.data_ptr(), data.numel(),
                                    reps, _stream_ptr(stream), ctypes.byref(best), ctypes.byref(ms))
    _check(st, "poslo_autotune_batch")
    return best, ms.value


def poslo_batch_forget(ctx: Ctx) -> None:
    _check(lib().poslo_batch_forget(ctx.handle), "poslo_batch_forget")


# ------------------------------------------------------------- serving loop

class Request:
    """A poslo_request plus the host buffers it points into (ds, tag, and
    host message buffers when on_device is 0)."""

    def __init__(self, key_id: int, t0: int, n: int, data, offsets, msg_len: int, sigs, ds: bytes, tag: bytes,
                 user: int = 0, data_bytes: int | None = None):
        self._ds = ctypes.create_string_buffer(bytes(ds), max(1, len(ds)))
        self._tag = ctypes.create_string_buffer(bytes(tag), 64)
        self._keep = []

        def ptr(x):
            if x is None:
                return None, True
            if hasattr(x, "data_ptr"):  # CUDA tensor, kept alive with the request
                self._keep.append(x)
                return (x.data_ptr() if x.numel() else None), True
            arr = np.ascontiguousarray(x)
            self._keep.append(arr)
            return (arr.ctypes.data if arr.size else None), False

        dp, dev = ptr(data)
        op, _ = ptr(offsets)
        sp, _ = ptr(sigs)
        if data_bytes is None:
            data_bytes = 0 if data is None else (data.numel() if hasattr(data, "numel") else np.asarray(data).nbytes)
        self.req = poslo_request(key_id, 1 if dev else 0, t0, n, dp, op, msg_len, data_bytes, sp,
                                 ctypes.addressof(self._ds), len(ds), ctypes.addressof(self._tag), user)


class Server:
    """Owns a poslo_server*."""

    def __init__(self, device: int, params: poslo_params, n_streams: int = 4, max_group: int = 256,
                 mem_bytes: int = 0, distill: int = 1, variant: int = -1, max_group_entries: int = 0):
        cfg = poslo_server_cfg(params, n_streams, max_group, mem_bytes, distill, variant, max_group_entries)
        h = ctypes.c_void_p()
        _check(lib().poslo_server_create(device, ctypes.byref(cfg), ctypes.byref(h)), "poslo_server_create")
        self.handle = h
        self._live = {}

    def register_keys(self, ids: list[int], pks: list[bytes]) -> None:
        arr = (ctypes.c_uint32 * max(1, len(ids)))(*ids)
        _check(lib().poslo_server_register_keys(self.handle, arr, b"".join(bytes(p) for p in pks), len(ids)),
               "poslo_server_register_keys")

    def submit(self, req: Request) -> int:
        t = ctypes.c_uint64()
        _check(lib().poslo_server_submit(self.handle, ctypes.byref(req.req), ctypes.byref(t)), "poslo_server_submit")
        self._live[t.value] = req  # keep its buffers alive until polled
        return t.value

    def poll(self, cap: int = 1024, timeout_ms: float = 0.0) -> list[poslo_result]:
        buf = (poslo_result * cap)()
        n = ctypes.c_size_t()
        _check(lib().poslo_server_poll(self.handle, buf, cap, ctypes.byref(n), timeout_ms), "poslo_server_poll")
        out = [buf[k] for k in range(n.value)]
        for r in out:
            self._live.pop(r.ticket, None)
        return out

    def take_invalid(self, ticket: int, n: int) -> list[int]:
        arr = (ctypes.c_uint64 * max(1, n))()
        got = ctypes.c_size_t()
        _check(lib().poslo_server_take_invalid(self.handle, ticket, arr, n, ctypes.byref(got)),
               "poslo_server_take_invalid")
        return [int(arr[k]) for k in range(got.value)]

    def key_state(self, key_id: int) -> tuple[bytes, int]:
        tag = ctypes.create_string_buffer(64)
        e = ctypes.c_uint64()
        _check(lib().poslo_server_key_state(self.handle, key_id, tag, ctypes.byref(e)), "poslo_server_key_state")
        return tag.raw, e.value

    def stats(self) -> poslo_server_stats:
        st = poslo_server_stats()
        _check(lib().poslo_server_stats_get(self.handle, ctypes.byref(st)), "poslo_server_stats_get")
        return st

    def close(self) -> None:
        if getattr(self, "handle", None) and self.handle.value:
            lib().poslo_server_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        if _lib is not None:
            self.close()
