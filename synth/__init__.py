"""Seeded synthetic inputs for the network-coding workloads.

This module only draws random numbers and lays them out; it contains no
finite-field arithmetic.  Both the CPU oracle tests and the GPU path take
their inputs from here, so a given (seed, shape) always yields the same bytes.

Randomness is SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter mode: the i-th
64-bit word of the stream with seed ``s`` is ``mix(s + (i + 1) * GAMMA)``.
Sub-streams are keyed by hashing a tuple of integers into a seed.

Workload shapes follow the paper's setting (Sec. II: a generation is N source
packets of M words; Sec. V-A: random linear combinations of N = 16 packets of
uniformly random payload), widened to the batch, decode and serving workloads
this library measures.  Payloads are uniform random bytes; coefficients are
uniform over the field (Sec. II, coefficients drawn i.i.d. from F_q) unless a
workload says "nonzero".
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

#: base seed of each workload family; workload ``i`` uses ``BASE_SEED + i``
BASE_SEED = 190902871

#: field name -> bits per word n
FIELDS = {"GF2": 1, "GF4": 2, "GF16": 4, "GF256": 8}


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _mix_int(z: int) -> int:
    m = (1 << 64) - 1
    z &= m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def key(*parts: int) -> int:
    """Hash a tuple of non-negative integers into a 64-bit stream seed."""
    h = 0x6A09E667F3BCC908
    for p in parts:
        h = _mix_int(h ^ _mix_int((int(p) + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)))
    return h


def words(seed: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` 64-bit words of the counter-mode SplitMix64 stream ``seed``."""
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & ((1 << 64) - 1)) + idx * GAMMA
    return _mix(state)


def random_bytes(seed: int, nbytes: int) -> np.ndarray:
    """``nbytes`` uniform random bytes (little-endian bytes of the word stream)."""
    nw = (nbytes + 7) // 8
    return words(seed, nw).view(np.uint8)[:nbytes].copy()


def uniform_field(seed: int, count: int, n: int) -> np.ndarray:
    """``count`` elements uniform over GF(2^n): the low n bits of uniform bytes."""
    b = random_bytes(seed, count)
    return (b & np.uint8((1 << n) - 1)).astype(np.uint8)


def uniform_nonzero(seed: int, count: int, n: int) -> np.ndarray:
    """``count`` elements uniform over GF(2^n) minus {0}, by rejection."""
    out = np.empty(0, dtype=np.uint8)
    chunk = 0
    while out.size < count:
        b = random_bytes(key(seed, chunk), 2 * count + 64) & np.uint8((1 << n) - 1)
        out = np.concatenate([out, b[b != 0]])
        chunk += 1
    return out[:count].copy()


def uniform_ints(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """``count`` integers uniform in [lo, hi] (inclusive)."""
    w = words(seed, count)
    return (np.uint64(lo) + w % np.uint64(hi - lo + 1)).astype(np.int64)


def unit_floats(seed: int, count: int) -> np.ndarray:
    """``count`` doubles uniform in [0, 1) (53 high bits of each word)."""
    return (words(seed, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def log_uniform_ints(seed: int, count: int, lo: int, hi: int) -> np.ndarray:
    """``count`` integers floor(lo * (hi/lo)^u), u ~ U[0,1), clipped to [lo, hi]."""
    u = unit_floats(seed, count)
    v = np.floor(lo * np.exp(u * math.log(hi / lo))).astype(np.int64)
    return np.clip(v, lo, hi)


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------

@dataclass
class Generation:
    """One generation: K x N coefficients C, N source packets S of ``length`` bytes."""
    n: int            # bits per field word
    N: int            # generation size (source packets)
    K: int            # coded packets to produce
    length: int       # packet length in bytes
    C: np.ndarray     # uint8[K, N]
    S: np.ndarray     # uint8[N, length]


def generation(seed: int, n: int, N: int, K: int, length: int,
               nonzero: bool = False) -> Generation:
    """A generation with uniform random payload and uniform (or nonzero) coefficients."""
    S = random_bytes(key(seed, 1), N * length).reshape(N, length)
    if nonzero:
        C = uniform_nonzero(key(seed, 2), K * N, n).reshape(K, N)
    else:
        C = uniform_field(key(seed, 2), K * N, n).reshape(K, N)
    return Generation(n, N, K, length, C, S)


def single_generation() -> Generation:
    """GF(256), N = K = 16 packets of 1500 B, coefficients uniform nonzero."""
    return generation(key(BASE_SEED + 0, 0), 8, 16, 16, 1500, nonzero=True)


def sweep_generation(n: int, length: int, index: int, N: int = 64, K: int = 64) -> Generation:
    """Generation ``index`` of the plain sweep: N = K = 64, one field and packet size."""
    return generation(key(BASE_SEED + 1, n, length, index), n, N, K, length)


def uneven_shapes(count: int, n: int, seed_off: int = 0):
    """(N, length) of ``count`` uneven generations: N ~ U{8..256}, length log-U[64, 9000]."""
    base = key(BASE_SEED + 2, n, seed_off)
    Ns = uniform_ints(key(base, 1), count, 8, 256)
    Ls = log_uniform_ints(key(base, 2), count, 64, 9000)
    return Ns, Ls


def uneven_generation(n: int, index: int, N: int, length: int, seed_off: int = 0) -> Generation:
    """Generation ``index`` of the uneven batch (K = N)."""
    return generation(key(BASE_SEED + 2, n, seed_off, 100 + index), n, N, N, length)


def decode_shapes(count: int, seed_off: int = 0) -> np.ndarray:
    """N of each decode system: uniform over {32, 64, 128}."""
    pick = uniform_ints(key(BASE_SEED + 3, seed_off, 1), count, 0, 2)
    return np.array([32, 64, 128], dtype=np.int64)[pick]


def decode_candidate(index: int, attempt: int, N: int, n: int = 8, seed_off: int = 0) -> np.ndarray:
    """Candidate coefficient matrix ``attempt`` of decode system ``index``.

    The workload keeps the first candidate that is invertible; deciding that
    needs field arithmetic and is left to the caller.
    """
    return uniform_field(key(BASE_SEED + 3, seed_off, 2, index, attempt), N * N, n).reshape(N, N)


def decode_sources(index: int, N: int, length: int, seed_off: int = 0) -> np.ndarray:
    return random_bytes(key(BASE_SEED + 3, seed_off, 3, index), N * length).reshape(N, length)


@dataclass
class Request:
    rid: int
    arrival_s: float
    kind: str          # "encode" or "decode"
    N: int
    length: int
    seed: int


def serving_stream(count: int, rate_per_s: float, seed_off: int = 0,
                   decode_frac: float = 0.3) -> List[Request]:
    """Poisson arrivals of mixed encode/decode requests over GF(256)."""
    base = key(BASE_SEED + 4, seed_off)
    gaps = -np.log1p(-unit_floats(key(base, 1), count)) / rate_per_s
    t = np.cumsum(gaps)
    kinds = unit_floats(key(base, 2), count) < decode_frac
    Ns = uniform_ints(key(base, 3), count, 8, 256)
    Ls = log_uniform_ints(key(base, 4), count, 64, 9000)
    return [Request(i, float(t[i]), "decode" if kinds[i] else "encode", int(Ns[i]), int(Ls[i]),
                    key(base, 5, i)) for i in range(count)]


def coded_arrivals(seed: int, N: int, loss: float = 0.1, max_packets: Optional[int] = None):
    """Rateless sender: an endless list of (coefficient seed, dropped?) per emitted packet.

    Each emitted coded packet carries fresh uniform coefficients; it is lost
    i.i.d. with probability ``loss``.  Returns a generator of (packet_index, lost).
    """
    i = 0
    while max_packets is None or i < max_packets:
        lost = bool(unit_floats(key(seed, 7, i), 1)[0] < loss)
        yield i, lost
        i += 1


# --------------------------------------------------------------------------
# Batched layouts: every generation's rows padded to a multiple of 16 bytes,
# generations packed back to back in one payload blob and one coefficient blob.
# --------------------------------------------------------------------------

ROW_ALIGN = 16


def padded(length: int, align: int = ROW_ALIGN) -> int:
    return (int(length) + align - 1) // align * align


@dataclass
class Batch:
    n: int
    Ns: np.ndarray          # generation sizes
    Ks: np.ndarray          # coded rows per generation
    Ls: np.ndarray          # packet lengths (bytes)
    lds: np.ndarray         # row pitch (bytes)
    s_off: np.ndarray       # byte offset of each generation's first source row in the payload blob
    y_off: np.ndarray       # byte offset of each generation's first coded row in the output blob
    c_off: np.ndarray       # byte offset of each generation's coefficients in the coefficient blob
    s_bytes: int
    y_bytes: int
    c_bytes: int
    seed: int

    def source_blob(self) -> np.ndarray:
        return random_bytes(key(self.seed, 11), self.s_bytes)

    def coef_blob(self) -> np.ndarray:
        return uniform_field(key(self.seed, 12), self.c_bytes, self.n)

    def generation(self, i: int, S_blob: np.ndarray, C_blob: np.ndarray):
        """(C[K, N], S[N, L]) views of generation i."""
        N, K, L, ld = int(self.Ns[i]), int(self.Ks[i]), int(self.Ls[i]), int(self.lds[i])
        S = S_blob[self.s_off[i]:self.s_off[i] + N * ld].reshape(N, ld)[:, :L]
        C = C_blob[self.c_off[i]:self.c_off[i] + K * N].reshape(K, N)
        return C, S

    @property
    def source_bytes(self) -> int:
        """Useful source payload (sum of N * L)."""
        return int((self.Ns * self.Ls).sum())

    @property
    def byte_madds(self) -> int:
        return int((self.Ks * self.Ns * self.Ls).sum())


def _layout(n: int, Ns, Ks, Ls, seed: int) -> Batch:
    Ns = np.asarray(Ns, dtype=np.int64)
    Ks = np.asarray(Ks, dtype=np.int64)
    Ls = np.asarray(Ls, dtype=np.int64)
    lds = (Ls + ROW_ALIGN - 1) // ROW_ALIGN * ROW_ALIGN
    s_sz = Ns * lds
    y_sz = Ks * lds
    c_sz = (Ks * Ns + ROW_ALIGN - 1) // ROW_ALIGN * ROW_ALIGN
    s_off = np.concatenate([[0], np.cumsum(s_sz)[:-1]]) if len(Ns) else np.zeros(0, np.int64)
    y_off = np.concatenate([[0], np.cumsum(y_sz)[:-1]]) if len(Ns) else np.zeros(0, np.int64)
    c_off = np.concatenate([[0], np.cumsum(c_sz)[:-1]]) if len(Ns) else np.zeros(0, np.int64)
    return Batch(n, Ns, Ks, Ls, lds, s_off, y_off, c_off, int(s_sz.sum()), int(y_sz.sum()),
                 int(c_sz.sum()), seed)


def uneven_batch(n: int, count: int = 10000, seed_off: int = 0) -> Batch:
    """The uneven batch: N ~ U{8..256}, L log-uniform in [64, 9000] B, K = N."""
    Ns, Ls = uneven_shapes(count, n, seed_off)
    return _layout(n, Ns, Ns, Ls, key(BASE_SEED + 2, n, seed_off, 7))


def sweep_batch(n: int, length: int, count: int = 4096, N: int = 64, K: int = 64) -> Batch:
    """The plain sweep: ``count`` generations of N = K = 64 packets of ``length`` bytes."""
    return _layout(n, np.full(count, N), np.full(count, K), np.full(count, length),
                   key(BASE_SEED + 1, n, length, 7))


def decode_batch(count: int = 2048, length: int = 1500, seed_off: int = 0) -> Batch:
    """The decode batch over GF(256): N uniform over {32, 64, 128}, L = 1500 B.

    ``coef_blob`` holds first candidates only; invertibility is decided by the
    caller with ``decode_candidate`` redraws.
    """
    Ns = decode_shapes(count, seed_off)
    return _layout(8, Ns, Ns, np.full(count, length), key(BASE_SEED + 3, seed_off, 7))
