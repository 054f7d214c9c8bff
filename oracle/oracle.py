"""POSLO-F oracle: plain, slow, single-threaded reference of the verifier path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library in ``paper_2506_08781_amd`` and is never called by it.

Byte-level primitives (AES-128, SHA-256, MMO, MDC-2, F, H) come from the
plain C file ``poslo_oracle.c`` next to this module; everything else (the
seed tree, arithmetic modulo q, the group, and the scheme) is written here
with Python integers, step by step in the paper's order and notation.

Paper passages followed (sections, figures, definitions of the paper):
  * seed tree and SC / SSO / SR ..... "POSLO Data Types and Seed Management",
                                      the tree equation and figure "Seed
                                      Management Functions"
  * Agg, C-AVer steps 2-8 ........... "POSLO-C", figure "Digital signature
                                      algorithms"
  * Kg, Sig, AVer of POSLO-F ........ "POSLO-F", figure "Fine-grained
                                      public-key POSLO"
  * BPV ............................. Preliminaries, Definition "BPV"
  * Distill / SeBVer ................ "POSLO-C Distillation and Selective
                                      Batch Verification" (figure
                                      "Distillation and selective batch
                                      verification"), applied entry by entry
                                      as the POSLO-F text prescribes
  * PRF_j(x) = F(x || j) ............ "Instantiations of PRF"

Readings where the paper is silent, garbled or inconsistent (each also listed
in the design notes of the repository):
  R1  indices are 0-based: entry t is entry j = t mod n2 of epoch i = t div n2
      (the POSLO-F Sig writes "j <- i mod n2", "if j = 1", "if j = n2").
  R2  the epoch seed is x_0[i] = SR(ds, i); the one-time seed is
      x_t = PRF_0(x_0[i] || LE32(j)) with j as 4 little-endian bytes.
  R3  e_t = LE256(H(m_t || x_t)) mod q: the digest read as a little-endian
      256-bit integer.
  R4  the group is the prime-order subgroup of edwards25519 (RFC 8032
      encoding) instead of FourQ, whose constants the paper does not give;
      the multiplicative notation Y^e * alpha^s is read additively.
  R5  an entry is valid iff x_t equals the re-derived one-time seed, s_t < q,
      and encode(e_t*Y + s_t*G) equals the R_t bytes.
  R6  SSO at epoch i is called as SSO(ds_{i-1}, x_D[0], i) (the figure drops
      the index argument and once writes x_D[i]); it runs when entry j = 0 of
      epoch i is signed, so a batch's ds after its last entry covers a
      partial final epoch.
  R7  signer randomness is derived deterministically from a 32-byte seed with
      the scheme's own PRF_0 (see ``derive``), and the BPV subset S_t from a
      PRF_0 stream, so that keys and signatures are reproducible.
  R8  umbrella span U = ceil(N / n_u) entries; umbrella l covers batch
      positions [l*U, min(N, (l+1)*U)).
  R9  signature bytes: LE32B(s_t) || encode(R_t) || x_t (80 bytes); aggregate
      tag: LE32B(s) || encode(R) (64 bytes); ds wire format: one count byte,
      then per node {u8 depth, 3 zero bytes, u32 LE index, 16-byte value},
      bottom of the stack first.
  R10 kappa = 127 (AES-based PRF only): a seed is a 127-bit value held in 16
      bytes with bit 127 clear; the tree PRF of a seed x is one MMO block,
      PRF_b(x) = (E_IV(x + b*2^127) xor (x + b*2^127)) mod 2^127 (the
      paper's "x || j is exactly 128 bits"); every other PRF input (one-time
      seeds, key derivation) appends b as a byte, as for kappa = 128, and
      every PRF output is taken mod 2^127.
  R11 POSLO++: H = Add_q, e_t = (LE(m_t) + LE(x_t)) mod q with the message
      read as a little-endian integer; Add_q takes messages of at most 31
      bytes (below 2^248 < q, "|m| < |q|"); the signing equation stays
      s_t = r_t - e_t * y.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "poslo_oracle.c")

INST_SHA256 = 0    # POSLO: PRF and H from SHA-256
INST_AES = 1       # POSLO+: PRF from MMO-AES-128, H = MDC-2-AES-128
INST_AES_ADDQ = 2  # POSLO++: PRF from MMO-AES-128, H = Add_q (messages below 32 bytes)
KAPPA127 = 4       # flag on an AES-based instantiation: kappa = 127 (reading R10)


def inst_base(inst: int) -> int:
    """The instantiation without the kappa flag."""
    if inst & ~7 or (inst & 3) > 2 or (inst & KAPPA127 and (inst & 3) == INST_SHA256):
        raise ValueError("unknown instantiation")
    return inst & 3


def kappa_of(inst: int) -> int:
    inst_base(inst)
    return 127 if inst & KAPPA127 else 128


def build(force: bool = False) -> str:
    """Compile the C primitives with gcc (plain -O2, no intrinsics)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                        "-o", tmp, _SRC_PATH, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _c():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        u8p = ctypes.c_char_p
        _lib.oracle_aes128_encrypt.argtypes = [u8p, u8p, ctypes.c_void_p]
        _lib.oracle_sha256.argtypes = [u8p, ctypes.c_size_t, ctypes.c_void_p]
        _lib.oracle_mmo.argtypes = [u8p, ctypes.c_size_t, ctypes.c_void_p]
        _lib.oracle_mdc2.argtypes = [u8p, ctypes.c_size_t, ctypes.c_void_p]
        _lib.oracle_F.argtypes = [ctypes.c_int, u8p, ctypes.c_size_t, ctypes.c_void_p]
        _lib.oracle_H.argtypes = [ctypes.c_int, u8p, ctypes.c_size_t, ctypes.c_void_p]
    return _lib


# ---------------------------------------------------------------------------
# Byte-level primitives (C)
# ---------------------------------------------------------------------------

def aes128(key: bytes, block: bytes) -> bytes:
    out = ctypes.create_string_buffer(16)
    _c().oracle_aes128_encrypt(bytes(key), bytes(block), out)
    return out.raw


def sha256(data: bytes) -> bytes:
    out = ctypes.create_string_buffer(32)
    _c().oracle_sha256(bytes(data), len(data), out)
    return out.raw


def mmo(data: bytes) -> bytes:
    out = ctypes.create_string_buffer(16)
    _c().oracle_mmo(bytes(data), len(data), out)
    return out.raw


def mdc2(data: bytes) -> bytes:
    out = ctypes.create_string_buffer(32)
    _c().oracle_mdc2(bytes(data), len(data), out)
    return out.raw


def F(inst: int, z: bytes) -> bytes:
    """The PRF's underlying function (MMO-AES-128, or SHA-256 truncated)."""
    out = ctypes.create_string_buffer(16)
    if _c().oracle_F(0 if inst_base(inst) == INST_SHA256 else 1, bytes(z), len(z), out) != 0:
        raise ValueError("unknown instantiation")
    return out.raw


def H(inst: int, z: bytes) -> bytes:
    """The message hash (MDC-2-AES-128, or SHA-256); 32 bytes.  (Add_q
    takes the message and the seed apart: see digest_int.)"""
    base = inst_base(inst)
    if base == INST_AES_ADDQ:
        raise ValueError("Add_q is not a hash of a byte string")
    out = ctypes.create_string_buffer(32)
    if _c().oracle_H(base, bytes(z), len(z), out) != 0:
        raise ValueError("unknown instantiation")
    return out.raw


MASK127 = (1 << 127) - 1


def prf(inst: int, b: int, z: bytes) -> bytes:
    """PRF_b(z) = F(z || b) with b in {0, 1} appended as one byte; for
    kappa = 127 (reading R10) a 16-byte z is a seed and b its 128th bit, and
    the output is taken mod 2^127."""
    if b not in (0, 1):
        raise ValueError("PRF index must be 0 or 1")
    if kappa_of(inst) == 127:
        if len(z) == 16:
            v = int.from_bytes(z, "little")
            if v >> 127:
                raise ValueError("a 127-bit seed has bit 127 clear")
            out = F(inst, (v | (b << 127)).to_bytes(16, "little"))
        else:
            out = F(inst, bytes(z) + bytes([b]))
        return (int.from_bytes(out, "little") & MASK127).to_bytes(16, "little")
    return F(inst, bytes(z) + bytes([b]))


def le32(v: int) -> bytes:
    return int(v).to_bytes(4, "little")


# ---------------------------------------------------------------------------
# Seed tree (POSLOT) and the seed management functions SC, SSO, SR
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Node:
    depth: int      # d: the node is x_d[index]
    index: int
    value: bytes    # kappa = 128 bits


def tree_node(inst: int, root: bytes, D: int, d: int, i: int) -> bytes:
    """x_d[i] by the tree equation, recursing from x_D[0]:
    x_d[i] = PRF_{i mod 2}(x_{d+1}[i div 2])."""
    if d == D:
        if i != 0:
            raise ValueError("the root level has a single node")
        return root
    return prf(inst, i % 2, tree_node(inst, root, D, d + 1, i // 2))


def SC(inst: int, x: bytes, d0: int, i0: int, d1: int, i1: int) -> bytes:
    """Seed computation: x_{d1}[i1] from its ancestor x_{d0}[i0] by walking the
    bits of i = i1 - i0 * 2^(d0-d1), most significant first, applying
    PRF_0 for a 0 bit and PRF_1 for a 1 bit."""
    if not d1 <= d0:
        raise ValueError("target must not be above the source")
    if i1 >> (d0 - d1) != i0:
        raise ValueError("target is not a descendant of the source")
    xp = x
    i = i1 - i0 * (1 << (d0 - d1))
    for j in range(d0 - d1 - 1, -1, -1):
        xp = prf(inst, (i >> j) % 2, xp)
    return xp


def SSO(inst: int, ds: list[Node], root: bytes, D: int, i: int):
    """Seed storage optimizer: from ds_{i-1} returns (ds_i, x_0[i]).
    Pops every top node that is a complete sibling subtree at the current
    depth, moving one level up each time, then pushes the covering node."""
    if not 0 <= i < (1 << D):
        raise ValueError("epoch index out of range")
    d1, i1 = 0, i
    ds = list(ds)
    while ds and ds[-1].depth == d1:
        ds.pop()
        d1 += 1
        i1 //= 2
    node = Node(d1, i1, SC(inst, root, D, 0, d1, i1))
    ds.append(node)
    return ds, SC(inst, node.value, d1, i1, 0, i)


def SR(inst: int, ds: list[Node], ip: int):
    """Seed retrieval: x_0[ip] from the disclosed stack, or None for "bottom"
    when no disclosed node covers leaf ip.  The stack is read from its top
    without modifying the caller's copy."""
    stack = list(ds)
    if not stack:
        return None
    node = stack.pop()
    if ip >= (node.index + 1) * (1 << node.depth):
        return None
    while ip < node.index * (1 << node.depth):
        if not stack:
            return None
        node = stack.pop()
    return SC(inst, node.value, node.depth, node.index, 0, ip)


def ds_encode(ds: list[Node]) -> bytes:
    out = bytearray([len(ds)])
    for n in ds:
        out += bytes([n.depth, 0, 0, 0]) + le32(n.index) + n.value
    return bytes(out)


def ds_decode(buf: bytes) -> list[Node]:
    """Strict parse of the wire format: exact length, zero pad bytes,
    depth <= 32 and index < 2^(32 - depth); anything else is malformed."""
    if len(buf) < 1:
        raise ValueError("empty ds buffer")
    cnt = buf[0]
    if cnt > 32 or len(buf) != 1 + 24 * cnt:
        raise ValueError("malformed ds buffer length")
    nodes = []
    for k in range(cnt):
        o = 1 + 24 * k
        depth, pad = buf[o], bytes(buf[o + 1:o + 4])
        index = int.from_bytes(buf[o + 4:o + 8], "little")
        if pad != b"\0\0\0" or depth > 32 or (depth > 0 and index >> (32 - depth)):
            raise ValueError("malformed ds node")
        nodes.append(Node(depth, index, bytes(buf[o + 8:o + 24])))
    return nodes


# ---------------------------------------------------------------------------
# The group: prime-order subgroup of edwards25519 (RFC 8032, section 5.1)
# ---------------------------------------------------------------------------

P = 2 ** 255 - 19
Q = 2 ** 252 + 27742317777372353535851937790883648493   # group order q
D_CURVE = (-121665 * pow(121666, P - 2, P)) % P          # d = -121665/121666
SQRT_M1 = pow(2, (P - 1) // 4, P)
IDENTITY = (0, 1, 1, 0)  # extended coordinates (X, Y, Z, T), x = X/Z, y = Y/Z, xy = T/Z


def fe_inv(x: int) -> int:
    return pow(x, P - 2, P)


def recover_x(y: int, sign: int):
    """x from y on -x^2 + y^2 = 1 + d x^2 y^2 with the given parity, or None."""
    if y >= P:
        return None
    x2 = (y * y - 1) * fe_inv(D_CURVE * y * y + 1) % P
    if x2 == 0:
        return None if sign else 0
    x = pow(x2, (P + 3) // 8, P)
    if (x * x - x2) % P != 0:
        x = x * SQRT_M1 % P
    if (x * x - x2) % P != 0:
        return None
    if x % 2 != sign:
        x = P - x
    return x


_GY = 4 * fe_inv(5) % P
_GX = recover_x(_GY, 0)
G = (_GX, _GY, 1, _GX * _GY % P)


def point_add(A, B):
    """Complete addition law in extended coordinates for a = -1 (RFC 8032
    section 5.1.4); also used for doubling."""
    X1, Y1, Z1, T1 = A
    X2, Y2, Z2, T2 = B
    a = (Y1 - X1) * (Y2 - X2) % P
    b = (Y1 + X1) * (Y2 + X2) % P
    c = T1 * 2 * D_CURVE * T2 % P
    d = Z1 * 2 * Z2 % P
    e, f, g, h = b - a, d - c, d + c, b + a
    return (e * f % P, g * h % P, f * g % P, e * h % P)


def scalar_mult(k: int, A):
    """k*A by double-and-add over the bits of k, most significant first."""
    R = IDENTITY
    for bit in bin(k)[2:] if k > 0 else "":
        R = point_add(R, R)
        if bit == "1":
            R = point_add(R, A)
    return R


def encode(A) -> bytes:
    X, Y, Z, _ = A
    zi = fe_inv(Z)
    x, y = X * zi % P, Y * zi % P
    return (y | ((x & 1) << 255)).to_bytes(32, "little")


def decode(b: bytes):
    """Point from its 32-byte encoding, or None if it is not a canonical
    encoding of a curve point."""
    if len(b) != 32:
        return None
    v = int.from_bytes(b, "little")
    y, sign = v & ((1 << 255) - 1), v >> 255
    x = recover_x(y, sign)
    if x is None:
        return None
    return (x, y, 1, x * y % P)


def points_equal(A, B) -> bool:
    return (A[0] * B[2] - B[0] * A[2]) % P == 0 and (A[1] * B[2] - B[1] * A[2]) % P == 0


def le256(b: bytes) -> int:
    return int.from_bytes(b, "little")


def to32(v: int) -> bytes:
    return int(v).to_bytes(32, "little")


# ---------------------------------------------------------------------------
# POSLO-F: Kg, Sig, Agg, AVer (figure "Fine-grained public-key POSLO")
# ---------------------------------------------------------------------------

def derive(inst: int, seed: bytes, label: bytes, c: int) -> bytes:
    """Reading R7: 32 pseudo-random bytes
    PRF_0(seed || label || LE32(2c)) || PRF_0(seed || label || LE32(2c+1))."""
    return (prf(inst, 0, seed + label + le32(2 * c)) +
            prf(inst, 0, seed + label + le32(2 * c + 1)))


@dataclass
class Params:
    inst: int
    log2_n1: int          # D: n1 = 2^D epochs
    log2_n2: int          # n2 = 2^log2_n2 entries per epoch
    v: int = 1024         # BPV table size
    k: int = 16           # BPV subset size

    @property
    def n1(self) -> int:
        return 1 << self.log2_n1

    @property
    def n2(self) -> int:
        return 1 << self.log2_n2


@dataclass
class Signer:
    params: Params
    seed: bytes
    y: int
    root: bytes                   # x_D[0]
    t: int = 0                    # state St = (t, ds)
    ds: list = field(default_factory=list)
    x0: bytes = b""               # x_0[i] of the current epoch
    _gamma: dict = field(default_factory=dict)   # BPV table, filled on use

    def bpv_pair(self, k: int):
        """Gamma entry (r_k, R_k = r_k * G) of the BPV offline table."""
        if k not in self._gamma:
            r = le256(derive(self.params.inst, self.seed, b"bpv", k)) % Q
            self._gamma[k] = (r, scalar_mult(r, G))
        return self._gamma[k]


def kg(params: Params, seed: bytes):
    """POSLO-F.Kg: y in Z_q^*, Y = y*G, root x_D[0], BPV table; St = (0, empty)."""
    if len(seed) != 32:
        raise ValueError("key seed must be 32 bytes")
    if params.v & (params.v - 1) or not 0 < params.v <= 1 << 16 or not 0 < params.k <= params.v:
        raise ValueError("BPV parameters need v a power of two <= 2^16 and k <= v")
    c = 0
    while True:
        y = le256(derive(params.inst, seed, b"y", c)) % Q
        if y != 0:
            break
        c += 1
    root = derive(params.inst, seed, b"x", 0)[:16]
    if kappa_of(params.inst) == 127:
        root = (int.from_bytes(root, "little") & MASK127).to_bytes(16, "little")
    signer = Signer(params=params, seed=seed, y=y, root=root)
    pk = encode(scalar_mult(y, G))
    return signer, pk


def bpv_subset(signer: Signer, t: int) -> list[int]:
    """Reading R7: the first k distinct values (LE16 word mod v) of the stream
    PRF_0(seed || "S" || LE32(t) || LE32(c)), c = 0, 1, ..."""
    prm = signer.params
    chosen: list[int] = []
    c = 0
    while len(chosen) < prm.k:
        blk = prf(prm.inst, 0, signer.seed + b"S" + le32(t) + le32(c))
        for w in range(8):
            val = int.from_bytes(blk[2 * w:2 * w + 2], "little") % prm.v
            if val not in chosen and len(chosen) < prm.k:
                chosen.append(val)
        c += 1
    return chosen


def bpv_online(signer: Signer, t: int):
    """BPV.Online: r = sum of r_k mod q, R = sum of R_k over the subset S_t."""
    r, R = 0, IDENTITY
    for k in bpv_subset(signer, t):
        rk, Rk = signer.bpv_pair(k)
        r = (r + rk) % Q
        R = point_add(R, Rk)
    return r, R


def one_time_seed(inst: int, x0_i: bytes, j: int) -> bytes:
    """x_t = PRF_0(x_0[i] || j) (reading R2)."""
    return prf(inst, 0, x0_i + le32(j))


def digest_int(inst: int, m: bytes, x: bytes) -> int:
    """H(m || x) as a little-endian integer, not yet reduced mod q; for
    POSLO++ (reading R11) Add_q(m, x) = (LE(m) + LE(x)) mod q."""
    if inst_base(inst) == INST_AES_ADDQ:
        if len(m) > 31:
            raise ValueError("Add_q takes messages of at most 31 bytes")
        return (int.from_bytes(bytes(m), "little") + int.from_bytes(bytes(x), "little")) % Q
    return le256(H(inst, bytes(m) + bytes(x)))


def sig(signer: Signer, m: bytes) -> bytes:
    """POSLO-F.Sig for entry t = St.t: returns sigma_t = (s_t, R_t, x_t)."""
    prm = signer.params
    t = signer.t
    if t >= prm.n1 * prm.n2:
        raise RuntimeError("signer exhausted: t = n")
    i, j = t >> prm.log2_n2, t & (prm.n2 - 1)
    if j == 0:
        signer.ds, signer.x0 = SSO(prm.inst, signer.ds, signer.root, prm.log2_n1, i)
    r, R = bpv_online(signer, t)
    x = one_time_seed(prm.inst, signer.x0, j)
    e = digest_int(prm.inst, m, x) % Q
    s = (r - e * signer.y) % Q
    signer.t = t + 1
    return to32(s) + encode(R) + x


def agg(sigs: list[bytes]) -> bytes:
    """Agg: s = sum s_t mod q (additive part), R = sum R_t (multiplicative
    part, a point sum); returns the 64-byte tag."""
    s, R = 0, IDENTITY
    for sg in sigs:
        Rt = decode(sg[32:64])
        if Rt is None:
            raise ValueError("undecodable commitment in a signature")
        s = (s + le256(sg[0:32])) % Q
        R = point_add(R, Rt)
    return to32(s) + encode(R)


def epoch_seeds(prm: Params, ds: list[Node], t0: int, n: int) -> dict[int, bytes]:
    """x_0[i] = SR(ds, i) for every epoch touched by entries t0..t0+n-1."""
    seeds = {}
    if n == 0:
        return seeds
    for i in range(t0 >> prm.log2_n2, ((t0 + n - 1) >> prm.log2_n2) + 1):
        x = SR(prm.inst, ds, i)
        if x is None:
            raise LookupError(f"SR returned bottom for epoch {i}")
        seeds[i] = x
    return seeds


def aggregate_check(pk: bytes, e: int, tag: bytes) -> bool:
    """accept iff s < q and R = e*Y + s*G, compared by encoding."""
    Y = decode(pk)
    if Y is None:
        raise ValueError("public key is not a point encoding")
    s = le256(tag[0:32])
    if s >= Q:
        return False
    return encode(point_add(scalar_mult(e % Q, Y), scalar_mult(s, G))) == bytes(tag[32:64])


def aver(prm: Params, pk: bytes, msgs: list[bytes], t0: int, ds_bytes: bytes,
         tag: bytes, skip: set | None = None) -> bool:
    """POSLO-F.AVer over a batch (the POSLO-C.AVer steps 2-8, then the check):
    e = sum over entries of H(m_t || PRF_0(SR(ds, i) || j)) mod q.
    Entries whose batch position is in ``skip`` are left out."""
    ds = ds_decode(ds_bytes)
    seeds = epoch_seeds(prm, ds, t0, len(msgs))
    e = 0
    for pos, m in enumerate(msgs):
        if skip and pos in skip:
            continue
        t = t0 + pos
        i, j = t >> prm.log2_n2, t & (prm.n2 - 1)
        x = one_time_seed(prm.inst, seeds[i], j)
        e = (e + digest_int(prm.inst, m, x)) % Q
    return aggregate_check(pk, e, tag)


def ekeys_sum(prm: Params, msgs: list[bytes], t0: int, ds_bytes: bytes) -> int:
    """The aggregate ephemeral key e (mod q) of a batch, as AVer computes it."""
    ds = ds_decode(ds_bytes)
    seeds = epoch_seeds(prm, ds, t0, len(msgs))
    e = 0
    for pos, m in enumerate(msgs):
        t = t0 + pos
        i, j = t >> prm.log2_n2, t & (prm.n2 - 1)
        e = (e + digest_int(prm.inst, m, one_time_seed(prm.inst, seeds[i], j))) % Q
    return e


def entry_valid(prm: Params, pk: bytes, m: bytes, t: int, sg: bytes, x0_i: bytes) -> bool:
    """Individual verification of entry t (reading R5)."""
    if len(sg) != 80:
        return False
    j = t & (prm.n2 - 1)
    x = bytes(sg[64:80])
    if x != one_time_seed(prm.inst, x0_i, j):
        return False
    s = le256(sg[0:32])
    if s >= Q:
        return False
    Y = decode(pk)
    if Y is None:
        raise ValueError("public key is not a point encoding")
    e = digest_int(prm.inst, m, x) % Q
    return encode(point_add(scalar_mult(e, Y), scalar_mult(s, G))) == bytes(sg[32:64])


# ---------------------------------------------------------------------------
# Distill and SeBVer, entry-granular as POSLO-F prescribes
# ---------------------------------------------------------------------------

@dataclass
class CCD:
    valid_tag: bytes                                  # CCD^v
    umbrellas: list = field(default_factory=list)     # CCD^u: (tag, l)
    invalid: list = field(default_factory=list)       # CCD^i: (t, sigma_t)
    ds: bytes = b""
    t0: int = 0
    n: int = 0
    span: int = 0                                     # umbrella span U


def distill(prm: Params, pk: bytes, msgs: list[bytes], sigs: list[bytes], t0: int,
            ds_bytes: bytes, n_u: int) -> CCD:
    """Verify every entry individually; aggregate the valid ones into the
    overall tag and into umbrella tags of span U; keep invalid entries with
    their signatures."""
    if len(msgs) != len(sigs):
        raise ValueError("one signature per message")
    if n_u < 1:
        raise ValueError("at least one umbrella")
    n = len(msgs)
    ds = ds_decode(ds_bytes)
    seeds = epoch_seeds(prm, ds, t0, n)
    span = max(1, -(-n // n_u))
    sv, Rv = 0, IDENTITY
    su, Ru = 0, IDENTITY
    ccd = CCD(valid_tag=b"", ds=bytes(ds_bytes), t0=t0, n=n, span=span)
    for pos in range(n):
        t = t0 + pos
        sg = sigs[pos]
        if entry_valid(prm, pk, msgs[pos], t, sg, seeds[t >> prm.log2_n2]):
            s, R = le256(sg[0:32]), decode(sg[32:64])
            sv, Rv = (sv + s) % Q, point_add(Rv, R)
            su, Ru = (su + s) % Q, point_add(Ru, R)
        else:
            ccd.invalid.append((t, bytes(sg)))
        if (pos + 1) % span == 0 or pos == n - 1:
            ccd.umbrellas.append((to32(su) + encode(Ru), pos // span))
            su, Ru = 0, IDENTITY
    ccd.valid_tag = to32(sv) + encode(Rv)
    return ccd


def sebver(prm: Params, pk: bytes, msgs: list[bytes], ccd: CCD, mode: str) -> list[bool]:
    """Selective batch verification over distilled data.
    V: AVer of all entries not in CCD^i against CCD^v.
    U: per umbrella, AVer of its range minus CCD^i against its tag.
    I: individual verification of each CCD^i entry."""
    bad = {t - ccd.t0 for t, _ in ccd.invalid}
    if mode == "V":
        return [aver(prm, pk, msgs, ccd.t0, ccd.ds, ccd.valid_tag, skip=bad)]
    if mode == "U":
        out = []
        for tag, l in ccd.umbrellas:
            a, b = l * ccd.span, min(ccd.n, (l + 1) * ccd.span)
            t_first = ccd.t0 + a
            sub_skip = {p - a for p in bad if a <= p < b}
            out.append(aver(prm, pk, msgs[a:b], t_first, ccd.ds, tag, skip=sub_skip))
        return out
    if mode == "I":
        ds = ds_decode(ccd.ds)
        out = []
        for t, sg in ccd.invalid:
            x0 = SR(prm.inst, ds, t >> prm.log2_n2)
            if x0 is None:
                raise LookupError("SR returned bottom")
            out.append(entry_valid(prm, pk, msgs[t - ccd.t0], t, sg, x0))
        return out
    raise ValueError("mode must be V, U or I")


def sign_batch(prm: Params, seed: bytes, msgs: list[bytes]):
    """Key generation, then signing every message in order, then the ds after
    the last entry and the aggregate tag: the honest inputs of an AVer."""
    signer, pk = kg(prm, seed)
    sigs = [sig(signer, m) for m in msgs]
    return pk, sigs, ds_encode(signer.ds), agg(sigs), signer


def signer_at(prm: Params, seed: bytes, t: int) -> Signer:
    """The signer's state St after entries 0 .. t-1 have been signed, reached
    through POSLO-F.Sig's state transitions alone: Sig changes (ds, x_0)
    only at the first entry of an epoch (the SSO call) and otherwise only
    advances the counter, so St after t entries is SSO applied for epochs
    0 .. ceil(t / n2) - 1 with the counter at t.  Signing from this state
    gives the same signatures as signing every earlier entry first."""
    if not 0 <= t <= prm.n1 * prm.n2:
        raise ValueError("state index out of range")
    signer, _ = kg(prm, seed)
    for i in range(-(-t // prm.n2)):
        signer.ds, signer.x0 = SSO(prm.inst, signer.ds, signer.root, prm.log2_n1, i)
    signer.t = t
    return signer


# ---------------------------------------------------------------------------
# POSLO-C: coarse-grained, one aggregate signature per epoch (figure
# "Coarse-grained signer-optimal POSLO": Kg, Agg, Sig, AVer, Distill,
# SeBVer).  Readings beyond R1-R9:
#   C1  r_i^j = PRF_0(r || LE32(i) || LE32(j)) read as a little-endian
#       128-bit integer (below q, so its "mod q" leaves it unchanged); r is
#       the first 16 bytes of derive(seed, "r", 0).
#   C2  Sig's one-time seed is x_i^j = PRF_0(x_0[i] || LE32(j)) with
#       (ds_i, x_0[i]) = SSO(ds_{i-1}, x_D[0], i) (the figure writes x_D[i]
#       in both places; AVer re-derives x_0[i] by SR, so the two must agree).
#   C3  byte formats: pk = enc(Y) || enc(R~_0) || ... || enc(R~_{n1-1});
#       an epoch signature is LE32B(s~_i) with ds_i after epoch i; a
#       verifier's aggregate tag over a set of epochs is LE32B(s~) || enc(R~).
#   C4  the umbrella span is U = ceil(k / n_u) epochs of a k-epoch batch
#       (Distill's "i = 0 mod floor(n1/n^u)" for 0-based epochs, with the
#       batch's k in place of n1, as R8 reads it for entries).
# ---------------------------------------------------------------------------

@dataclass
class CSigner:
    params: Params
    seed: bytes
    y: int
    root: bytes          # x_D[0]
    r: bytes             # seed of the per-entry commitments r_i^j
    i: int = 0           # next epoch (state St = (i, ds))
    ds: list = field(default_factory=list)


def posloc_r(inst: int, r: bytes, i: int, j: int) -> int:
    """r_i^j = PRF_0(r || i || j) mod q (reading C1)."""
    return le256(prf(inst, 0, r + le32(i) + le32(j))) % Q


def posloc_kg(params: Params, seed: bytes):
    """POSLO-C.Kg: y and Y = y*G as in POSLO-F.Kg, the root x_D[0], the
    commitment seed r, and per epoch i the aggregate commitment
    R~_i = (sum over j of r_i^j mod q) * G.  Returns (signer, pk bytes)."""
    signer_f, pk_y = kg(params, seed)
    r = derive(params.inst, seed, b"r", 0)[:16]
    out = bytearray(pk_y)
    for i in range(params.n1):
        out += posloc_commitment(params, r, i)
    return CSigner(params=params, seed=seed, y=signer_f.y, root=signer_f.root, r=r), bytes(out)


def posloc_commitment(params: Params, r: bytes, i: int) -> bytes:
    """enc(R~_i) with R~_i = (sum over j of r_i^j mod q) * G (Kg's loop body)."""
    ri = 0
    for j in range(params.n2):
        ri = (ri + posloc_r(params.inst, r, i, j)) % Q
    return encode(scalar_mult(ri, G))


def posloc_signer_at(params: Params, seed: bytes, i: int) -> CSigner:
    """The POSLO-C signer's state after epochs 0 .. i-1 are signed, through
    Sig's state transitions alone (SSO for each of those epochs, the epoch
    counter at i); signing from it continues the sequence exactly.  The
    public key is not built (its commitments do not enter Sig)."""
    if not 0 <= i <= params.n1:
        raise ValueError("epoch index out of range")
    signer_f, _ = kg(params, seed)
    cs = CSigner(params=params, seed=seed, y=signer_f.y, root=signer_f.root,
                 r=derive(params.inst, seed, b"r", 0)[:16])
    for e in range(i):
        cs.ds, _ = SSO(params.inst, cs.ds, cs.root, params.log2_n1, e)
    cs.i = i
    return cs


def posloc_pk_parts(params: Params, pk: bytes):
    """(Y bytes, [R~_i bytes]) of a POSLO-C public key."""
    if len(pk) != 32 * (1 + params.n1):
        raise ValueError("POSLO-C public key holds Y and one commitment per epoch")
    return pk[:32], [pk[32 * (1 + i):32 * (2 + i)] for i in range(params.n1)]


def posloc_sig(signer: CSigner, msgs: list[bytes]) -> tuple[bytes, bytes]:
    """POSLO-C.Sig of epoch i = St.i over its n2 messages: s~_i = sum over j
    of (r_i^j - e_i^j * y) mod q; returns (LE32B(s~_i), ds_i)."""
    prm = signer.params
    i = signer.i
    if i >= prm.n1:
        raise RuntimeError("signer exhausted: every epoch is signed")
    if len(msgs) != prm.n2:
        raise ValueError("an epoch signature covers exactly n2 messages")
    signer.ds, x0 = SSO(prm.inst, signer.ds, signer.root, prm.log2_n1, i)
    s = 0
    for j, m in enumerate(msgs):
        x = one_time_seed(prm.inst, x0, j)
        e = digest_int(prm.inst, m, x) % Q
        s = (s + posloc_r(prm.inst, signer.r, i, j) - e * signer.y) % Q
    signer.i = i + 1
    return to32(s), ds_encode(signer.ds)


def posloc_epoch_e(prm: Params, msgs: list[bytes], i: int, ds: list[Node]) -> int:
    """AVer's inner loops for one epoch: sum over j of H(m_i^j || x_i^j) mod q
    with x_0[i] = SR(ds, i)."""
    x0 = SR(prm.inst, ds, i)
    if x0 is None:
        raise LookupError(f"SR returned bottom for epoch {i}")
    e = 0
    for j, m in enumerate(msgs):
        e = (e + digest_int(prm.inst, m, one_time_seed(prm.inst, x0, j))) % Q
    return e


def posloc_aver(prm: Params, pk: bytes, epochs: list, ds_bytes: bytes, s_tag: bytes,
                R_tag: bytes | None = None) -> bool:
    """POSLO-C.AVer over the epochs [(i, [n2 messages]), ...] against the
    aggregate s~ (32 bytes).  R~ is the Agg of the epochs' R~_i in pk unless
    the signature carries one (R_tag).  accept iff every epoch is whole,
    s~ < q and R~ = e~*Y + s~*G with e~ the sum of the epochs' hashes."""
    Yb, Rs = posloc_pk_parts(prm, pk)
    for i, msgs in epochs:
        if len(msgs) != prm.n2 or not 0 <= i < prm.n1:
            raise ValueError("AVer takes whole epochs")
    if R_tag is None:
        R = IDENTITY
        for i, _ in epochs:
            Ri = decode(Rs[i])
            if Ri is None:
                raise ValueError("undecodable epoch commitment in pk")
            R = point_add(R, Ri)
        R_tag = encode(R)
    ds = ds_decode(ds_bytes)
    e = 0
    for i, msgs in epochs:
        e = (e + posloc_epoch_e(prm, msgs, i, ds)) % Q
    return aggregate_check(Yb, e, bytes(s_tag) + bytes(R_tag))


def posloc_agg_s(s_list: list[bytes]) -> bytes:
    """POSLO-C.Agg of the additive parts: sum mod q."""
    s = 0
    for b in s_list:
        s = (s + le256(b)) % Q
    return to32(s)


@dataclass
class CCDC:
    valid_tag: bytes                                  # CCD^v: LE32B(s~) || enc(R~)
    umbrellas: list = field(default_factory=list)     # CCD^u: (tag, l)
    invalid: list = field(default_factory=list)       # CCD^i: (i, LE32B(s~_i) || enc(R~_i))
    ds: bytes = b""
    i0: int = 0
    k: int = 0
    span: int = 0


def posloc_distill(prm: Params, pk: bytes, msgs: list[bytes], s_epochs: list[bytes], i0: int,
                   ds_bytes: bytes, n_u: int) -> CCDC:
    """POSLO-C.Distill over k consecutive epochs i0 .. i0+k-1 (msgs holds
    their k*n2 messages in order, s_epochs their signatures s~_i): each
    epoch is checked by AVer against (s~_i, R~_i from pk); valid epochs go
    into CCD^v and the current umbrella, invalid ones into CCD^i with
    (s~_i, R~_i)."""
    if len(msgs) != len(s_epochs) * prm.n2:
        raise ValueError("n2 messages per epoch signature")
    if n_u < 1:
        raise ValueError("at least one umbrella")
    k = len(s_epochs)
    _, Rs = posloc_pk_parts(prm, pk)
    span = max(1, -(-k // n_u))
    sv, Rv, su, Ru = 0, IDENTITY, 0, IDENTITY
    ccd = CCDC(valid_tag=b"", ds=bytes(ds_bytes), i0=i0, k=k, span=span)
    for p in range(k):
        i = i0 + p
        em = msgs[p * prm.n2:(p + 1) * prm.n2]
        if posloc_aver(prm, pk, [(i, em)], ds_bytes, s_epochs[p]):
            s, R = le256(s_epochs[p]), decode(Rs[i])
            sv, Rv = (sv + s) % Q, point_add(Rv, R)
            su, Ru = (su + s) % Q, point_add(Ru, R)
        else:
            ccd.invalid.append((i, bytes(s_epochs[p]) + Rs[i]))
        if (p + 1) % span == 0 or p == k - 1:
            ccd.umbrellas.append((to32(su) + encode(Ru), p // span))
            su, Ru = 0, IDENTITY
    ccd.valid_tag = to32(sv) + encode(Rv)
    return ccd


def posloc_sebver(prm: Params, pk: bytes, msgs: list[bytes], ccd: CCDC, mode: str) -> list[bool]:
    """POSLO-C.SeBVer.  V: AVer of every epoch not in CCD^i against CCD^v.
    U: per umbrella, AVer of its epochs minus CCD^i against its tag.
    I: AVer of each CCD^i epoch against its own (s~_i, R~_i)."""
    bad = {i for i, _ in ccd.invalid}

    def ep(p):
        return (ccd.i0 + p, msgs[p * prm.n2:(p + 1) * prm.n2])

    if mode == "V":
        eps = [ep(p) for p in range(ccd.k) if ccd.i0 + p not in bad]
        return [posloc_aver(prm, pk, eps, ccd.ds, ccd.valid_tag[:32], ccd.valid_tag[32:])]
    if mode == "U":
        out = []
        for tag, l in ccd.umbrellas:
            a, b = l * ccd.span, min(ccd.k, (l + 1) * ccd.span)
            eps = [ep(p) for p in range(a, b) if ccd.i0 + p not in bad]
            out.append(posloc_aver(prm, pk, eps, ccd.ds, tag[:32], tag[32:]))
        return out
    if mode == "I":
        return [posloc_aver(prm, pk, [ep(i - ccd.i0)], ccd.ds, sg[:32], sg[32:]) for i, sg in ccd.invalid]
    raise ValueError("mode must be V, U or I")


def posloc_sign_batch(prm: Params, seed: bytes, msgs: list[bytes]):
    """POSLO-C key generation and signing of len(msgs) / n2 whole epochs in
    order: (pk, [s~_i], ds after the last epoch, signer)."""
    if len(msgs) % prm.n2:
        raise ValueError("whole epochs only")
    signer, pk = posloc_kg(prm, seed)
    s_list, ds = [], ds_encode([])
    for p in range(len(msgs) // prm.n2):
        s, ds = posloc_sig(signer, msgs[p * prm.n2:(p + 1) * prm.n2])
        s_list.append(s)
    return pk, s_list, ds, signer
