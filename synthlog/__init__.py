"""Seeded synthetic log generator shared by the tests, the benchmark and the
oracle's test drivers.

This module draws random bytes and random indices only: it holds none of the
signature scheme's arithmetic (no hashing, no PRF, no group law), so that the
oracle and the GPU path can both consume its outputs without sharing any of
the method's code.

Generator: xoshiro256** (Blackman and Vigna, "Scrambled linear pseudorandom
number generators", 2018/2021), seeded through splitmix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", 2014), both written
from their published definitions.

Stream convention (a convention of this project; the paper does not fix one):
the xoshiro256** state of stream ``(seed, sid)`` is four consecutive
splitmix64 outputs starting from the 64-bit state ``(seed << 32) | sid``, with
``seed`` and ``sid`` both below 2**32.  Entry ``t`` of a log with message seed
``s`` draws its message bytes from stream ``(s, t)``: ceil(L/8) outputs,
little-endian, truncated to L bytes.
"""

from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


# ---------------------------------------------------------------------------
# Scalar definitions (plain Python integers)
# ---------------------------------------------------------------------------

def splitmix64_next(state: int) -> tuple[int, int]:
    """One splitmix64 step: returns (new_state, output)."""
    state = (state + _GOLDEN) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def _rotl(x: int, k: int) -> int:
    return ((x << k) | (x >> (64 - k))) & MASK64


class Xoshiro256ss:
    """xoshiro256** with a splitmix64-expanded 64-bit seed."""

    def __init__(self, seed64: int):
        st = seed64 & MASK64
        s = []
        for _ in range(4):
            st, out = splitmix64_next(st)
            s.append(out)
        self.s = s

    def next(self) -> int:
        s = self.s
        result = (_rotl((s[1] * 5) & MASK64, 7) * 9) & MASK64
        t = (s[1] << 17) & MASK64
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = _rotl(s[3], 45)
        return result

    def below(self, bound: int) -> int:
        """Uniform integer in [0, bound) by rejection (bound < 2**64)."""
        if bound <= 0:
            raise ValueError("bound must be positive")
        lim = (1 << 64) - ((1 << 64) % bound)
        while True:
            v = self.next()
            if v < lim:
                return v % bound

    def uniform01(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def stream_seed(seed: int, sid: int) -> int:
    if not (0 <= seed < (1 << 32) and 0 <= sid < (1 << 32)):
        raise ValueError("seed and stream id must be below 2**32")
    return (seed << 32) | sid


def stream_bytes(seed: int, sid: int, nbytes: int) -> bytes:
    """Bytes of stream (seed, sid): scalar reference for the vector path."""
    g = Xoshiro256ss(stream_seed(seed, sid))
    out = bytearray()
    while len(out) < nbytes:
        out += g.next().to_bytes(8, "little")
    return bytes(out[:nbytes])


# ---------------------------------------------------------------------------
# Vectorised form (numpy, one xoshiro state per stream)
# ---------------------------------------------------------------------------

def _np_splitmix(state: np.ndarray):
    state = state + np.uint64(_GOLDEN)
    z = state.copy()
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return state, z ^ (z >> np.uint64(31))


def _np_rotl(x: np.ndarray, k: int) -> np.ndarray:
    return (x << np.uint64(k)) | (x >> np.uint64(64 - k))


def stream_words(seed: int, sids: np.ndarray, nwords: int) -> np.ndarray:
    """First ``nwords`` xoshiro256** outputs of every stream in ``sids``.

    Returns a uint64 array of shape (len(sids), nwords)."""
    sids = np.asarray(sids, dtype=np.uint64)
    if sids.size and int(sids.max()) >= (1 << 32):
        raise ValueError("stream id must be below 2**32")
    if not (0 <= seed < (1 << 32)):
        raise ValueError("seed must be below 2**32")
    with np.errstate(over="ignore"):
        st = (np.uint64(seed) << np.uint64(32)) | sids
        s = []
        for _ in range(4):
            st, out = _np_splitmix(st)
            s.append(out)
        s0, s1, s2, s3 = s
        out = np.empty((sids.size, nwords), dtype=np.uint64)
        for w in range(nwords):
            out[:, w] = _np_rotl(s1 * np.uint64(5), 7) * np.uint64(9)
            t = s1 << np.uint64(17)
            s2 = s2 ^ s0
            s3 = s3 ^ s1
            s1 = s1 ^ s2
            s0 = s0 ^ s3
            s2 = s2 ^ t
            s3 = _np_rotl(s3, 45)
    return out


def messages_fixed(seed: int, n: int, length: int, t0: int = 0,
                   chunk: int = 1 << 18) -> np.ndarray:
    """n messages of ``length`` bytes for entries t0..t0+n-1, shape (n, length)."""
    out = np.empty((n, length), dtype=np.uint8)
    nw = (length + 7) // 8
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        sids = np.arange(t0 + a, t0 + b, dtype=np.uint64)
        words = stream_words(seed, sids, nw)
        out[a:b] = words.view(np.uint8).reshape(b - a, nw * 8)[:, :length]
    return out


def messages_var(seed: int, lengths: np.ndarray, t0: int = 0):
    """Variable-length messages: returns (concatenated uint8, offsets[n+1])."""
    lengths = np.asarray(lengths, dtype=np.int64)
    n = lengths.size
    offsets = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lengths, out=offsets[1:])
    data = np.empty(int(offsets[-1]), dtype=np.uint8)
    if n == 0:
        return data, offsets
    order = np.argsort(lengths, kind="stable")
    # group by length so each group is one vector draw
    uniq, starts = np.unique(lengths[order], return_index=True)
    bounds = list(starts) + [n]
    for gi, L in enumerate(uniq):
        idx = order[bounds[gi]:bounds[gi + 1]]
        L = int(L)
        if L == 0:
            continue
        nw = (L + 7) // 8
        for a in range(0, idx.size, 1 << 16):
            sub = idx[a:a + (1 << 16)]
            words = stream_words(seed, (sub + t0).astype(np.uint64), nw)
            rows = words.view(np.uint8).reshape(sub.size, nw * 8)[:, :L]
            for r, e in enumerate(sub):
                o = int(offsets[e])
                data[o:o + L] = rows[r]
    return data, offsets


def uniform_per_stream(seed: int, sids: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """One integer in [lo, hi] per stream: lo + floor(u * (hi - lo + 1)) with
    u = (first output >> 11) * 2^-53 of stream (seed, sid).  Vectorised; each
    value depends only on its own stream, so any entry's value can be drawn
    independently (the device generator computes the same values)."""
    w = stream_words(seed, np.asarray(sids, dtype=np.uint64), 1)[:, 0]
    u = (w >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    return (lo + np.floor(u * (hi - lo + 1))).astype(np.int64)


def uniform_ints(seed: int, sid: int, n: int, lo: int, hi: int) -> list[int]:
    """n uniform integers in [lo, hi] from stream (seed, sid)."""
    g = Xoshiro256ss(stream_seed(seed, sid))
    return [lo + g.below(hi - lo + 1) for _ in range(n)]


def log_uniform_counts(seed: int, sid: int, n: int, hi: int) -> list[int]:
    """n integers floor(exp(u * ln(hi + 1))) with u uniform in [0, 1): values
    in [1, hi]."""
    import math
    g = Xoshiro256ss(stream_seed(seed, sid))
    out = []
    for _ in range(n):
        v = int(math.floor(math.exp(g.uniform01() * math.log(hi + 1))))
        out.append(min(max(v, 1), hi))
    return out


def sample_distinct(seed: int, sid: int, population: int, k: int) -> list[int]:
    """k distinct indices from range(population) by a partial Fisher-Yates
    shuffle (first k positions), returned in draw order."""
    if k > population:
        raise ValueError("k exceeds population")
    g = Xoshiro256ss(stream_seed(seed, sid))
    swapped: dict[int, int] = {}
    out = []
    for a in range(k):
        b = a + g.below(population - a)
        va = swapped.get(a, a)
        vb = swapped.get(b, b)
        swapped[a], swapped[b] = vb, va
        out.append(vb)
    return out


def corruption_plan(seed: int, n: int, k: int, bits_per_entry: int):
    """k distinct entries of n and, for each, one bit position uniform over
    ``bits_per_entry`` bits.  Returns a list of (entry, bit) sorted by entry."""
    entries = sample_distinct(seed, 0, n, k)
    g = Xoshiro256ss(stream_seed(seed, 1))
    plan = [(e, g.below(bits_per_entry)) for e in entries]
    plan.sort()
    return plan


def corruption_plan_var(seed: int, n: int, k: int, bits) -> list[tuple[int, int]]:
    """As corruption_plan, with entry e's bit drawn uniform over bits[e] bits
    (entries of different lengths)."""
    entries = sample_distinct(seed, 0, n, k)
    g = Xoshiro256ss(stream_seed(seed, 1))
    plan = [(e, g.below(int(bits[e]))) for e in entries]
    plan.sort()
    return plan


def key_seed_bytes(first: int) -> bytes:
    """32-byte key seed made of consecutive byte values first..first+31."""
    return bytes((first + i) & 0xFF for i in range(32))


def derived_key_seed(master: int, k: int) -> bytes:
    """32-byte key seed for signer k drawn from stream (master, k)."""
    return stream_bytes(master, k, 32)
