"""Python access to the plain C oracle (``gforacle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously correct CPU
reference the GPU library is checked against.  Only the tests, the package
smoke check and the benchmark's CPU-baseline leg may import this module.

The shared object is compiled with the system C compiler on first use (or by
``build()``); it is never linked with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gforacle.c")
_HDR = os.path.join(_HERE, "gforacle.h")
_LIB = os.path.join(_HERE, "libgforacle.so")
_lib = None

_u8p = C.POINTER(C.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle into ``libgforacle.so`` (plain C, -O2, no intrinsics)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= max(
            os.path.getmtime(_SRC), os.path.getmtime(_HDR)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Werror", "-fopenmp", "-shared", "-fPIC",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GFO_LIB")   # a separately built copy (e.g. with host sanitizers)
        if not path:
            build(force=False)
            path = _LIB
        L = C.CDLL(path)
        sig = {
            "gfo_valid_field": (C.c_int, [C.c_int]),
            "gfo_poly": (C.c_int, [C.c_int]),
            "gfo_mul": (C.c_int, [C.c_int, C.c_int, C.c_int]),
            "gfo_mul_peasant": (C.c_int, [C.c_int, C.c_int, C.c_int]),
            "gfo_inv": (C.c_int, [C.c_int, C.c_int]),
            "gfo_pow": (C.c_int, [C.c_int, C.c_int, C.c_int]),
            "gfo_mulbyte": (C.c_int, [C.c_int, C.c_int, C.c_int]),
            "gfo_shuffle_tables": (None, [C.c_int, C.c_int, _u8p, _u8p]),
            "gfo_shuffle_byte": (C.c_int, [C.c_int, C.c_int, C.c_int]),
            "gfo_imul_powers": (None, [C.c_int, C.c_int, C.POINTER(C.c_int)]),
            "gfo_imul_word": (C.c_uint32, [C.c_int, C.c_int, C.c_uint32]),
            "gfo_region_madd": (C.c_int, [C.c_int, _u8p, _u8p, C.c_int, C.c_size_t]),
            "gfo_region_mul": (C.c_int, [C.c_int, _u8p, _u8p, C.c_int, C.c_size_t]),
            "gfo_encode": (C.c_int, [C.c_int, _u8p, C.c_int, C.c_int, _u8p, C.c_size_t,
                                     _u8p, C.c_size_t, C.c_size_t]),
            "gfo_encode_batch": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int64), _u8p, _u8p, _u8p, C.c_int]),
            "gfo_matmul": (C.c_int, [C.c_int, _u8p, _u8p, _u8p, C.c_int, C.c_int, C.c_int]),
            "gfo_recode": (C.c_int, [C.c_int, _u8p, C.c_int, C.c_int, C.c_int, _u8p, _u8p, C.c_size_t,
                                     _u8p, _u8p, C.c_size_t, C.c_size_t]),
            "gfo_rank": (C.c_int, [C.c_int, _u8p, C.c_int, C.c_int]),
            "gfo_invert": (C.c_int, [C.c_int, _u8p, C.c_int, _u8p]),
            "gfo_decode": (C.c_int, [C.c_int, _u8p, _u8p, C.c_size_t, C.c_int, _u8p,
                                     C.c_size_t, C.c_size_t]),
            "gfo_count_invertible": (C.c_longlong, [C.c_int, C.c_int]),
            "gfo_prog_new": (C.c_void_p, [C.c_int, C.c_int, C.c_size_t]),
            "gfo_prog_free": (None, [C.c_void_p]),
            "gfo_prog_rank": (C.c_int, [C.c_void_p]),
            "gfo_prog_add": (C.c_int, [C.c_void_p, _u8p, _u8p]),
            "gfo_prog_solve": (C.c_int, [C.c_void_p, _u8p, C.c_size_t]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(_u8p)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint8))


# ---------------------------------------------------------------- scalars

def mul(n: int, a: int, b: int) -> int:
    return lib().gfo_mul(n, a, b)


def mul_peasant(n: int, a: int, b: int) -> int:
    return lib().gfo_mul_peasant(n, a, b)


def inv(n: int, a: int) -> int:
    return lib().gfo_inv(n, a)


def pow_(n: int, a: int, e: int) -> int:
    return lib().gfo_pow(n, a, e)


def mulbyte(n: int, c: int, b: int) -> int:
    return lib().gfo_mulbyte(n, c, b)


def mul_table(n: int) -> np.ndarray:
    """q x q table of field products (for tests)."""
    q = 1 << n
    return np.array([[mul(n, a, b) for b in range(q)] for a in range(q)], dtype=np.int64)


def mulbyte_table(n: int) -> np.ndarray:
    """256 x 256 table T[c][b] = c * b word-wise; rows c >= q are unused (zero)."""
    q = 1 << n
    t = np.zeros((256, 256), dtype=np.uint8)
    for c in range(q):
        for b in range(256):
            t[c, b] = mulbyte(n, c, b)
    return t


def shuffle_tables(n: int, c: int):
    tl = np.zeros(16, np.uint8)
    th = np.zeros(16, np.uint8)
    lib().gfo_shuffle_tables(n, c, _p(tl), _p(th))
    return tl, th


def shuffle_byte(n: int, c: int, a: int) -> int:
    return lib().gfo_shuffle_byte(n, c, a)


def imul_powers(n: int, c: int):
    p = (C.c_int * 8)()
    lib().gfo_imul_powers(n, c, p)
    return [p[i] for i in range(n)]


def imul_word(n: int, c: int, v: int) -> int:
    return lib().gfo_imul_word(n, c, v)


# ---------------------------------------------------------------- regions

def region_madd(n: int, y: np.ndarray, x: np.ndarray, c: int) -> np.ndarray:
    """Return y + c*x (does not modify the argument)."""
    y = _u8(y).copy()
    x = _u8(x)
    assert y.size == x.size
    rc = lib().gfo_region_madd(n, _p(y), _p(x), c, y.size)
    if rc != 0:
        raise ValueError("gfo_region_madd: invalid field or coefficient")
    return y


def region_mul(n: int, x: np.ndarray, c: int) -> np.ndarray:
    x = _u8(x)
    y = np.empty_like(x)
    rc = lib().gfo_region_mul(n, _p(y), _p(x), c, x.size)
    if rc != 0:
        raise ValueError("gfo_region_mul: invalid field or coefficient")
    return y


def encode(n: int, Cm: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Y[K, len] = C[K, N] * S[N, len] over GF(2^n)."""
    Cm = _u8(Cm)
    S = _u8(S)
    K, N = Cm.shape
    assert S.shape[0] == N
    length = S.shape[1]
    Y = np.zeros((K, length), np.uint8)
    rc = lib().gfo_encode(n, _p(Cm), K, N, _p(S), length, _p(Y), length, length)
    assert rc == 0
    return Y


def encode_batch(n: int, desc: np.ndarray, C_blob: np.ndarray, S_blob: np.ndarray, Y_blob: np.ndarray,
                 threads: int = 1) -> int:
    """Eq. (1) for every generation of a batch, written into Y_blob in place.

    desc: int64[count, 8] rows {C offset, S offset, Y offset, ld_s, ld_y, len, K, N}
    (byte offsets into the blobs).  Generations are shared among ``threads``
    OpenMP threads.  Returns the number of threads that ran."""
    desc = np.ascontiguousarray(desc, dtype=np.int64)
    assert desc.ndim == 2 and desc.shape[1] == 8
    for b in (C_blob, S_blob, Y_blob):
        assert b.dtype == np.uint8 and b.flags.c_contiguous
    used = lib().gfo_encode_batch(n, desc.shape[0], desc.ctypes.data_as(C.POINTER(C.c_int64)), _p(C_blob),
                                  _p(S_blob), _p(Y_blob), threads)
    if used < 0:
        raise ValueError("gfo_encode_batch: bad argument")
    return used


def matmul(n: int, P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    P = _u8(P)
    Q = _u8(Q)
    a, b = P.shape
    b2, c = Q.shape
    assert b == b2
    R = np.zeros((a, c), np.uint8)
    lib().gfo_matmul(n, _p(P), _p(Q), _p(R), a, b, c)
    return R


def recode(n: int, R: np.ndarray, Cin: np.ndarray, Bin: np.ndarray):
    """(Cout, Yout) = (R * Cin, R * Bin): recoding M received coded packets with a
    Kout x M matrix R (Sec. I)."""
    R = _u8(R)
    Cin = _u8(Cin)
    Bin = _u8(Bin)
    Kout, M = R.shape
    assert Cin.shape[0] == M and Bin.shape[0] == M
    N = Cin.shape[1]
    length = Bin.shape[1]
    Cout = np.zeros((Kout, N), np.uint8)
    Yout = np.zeros((Kout, length), np.uint8)
    rc = lib().gfo_recode(n, _p(R), Kout, M, N, _p(Cin), _p(Bin), length, _p(Cout), _p(Yout), length, length)
    assert rc == 0
    return Cout, Yout


def rank(n: int, M: np.ndarray) -> int:
    M = _u8(M)
    return lib().gfo_rank(n, _p(M), M.shape[0], M.shape[1])


def invert(n: int, Cm: np.ndarray) -> Optional[np.ndarray]:
    Cm = _u8(Cm)
    N = Cm.shape[0]
    out = np.zeros((N, N), np.uint8)
    r = lib().gfo_invert(n, _p(Cm), N, _p(out))
    return out if r == N else None


def decode(n: int, Cm: np.ndarray, B: np.ndarray):
    """(rank, S) with S = C^-1 B when C is invertible, else (rank, None)."""
    Cm = _u8(Cm)
    B = _u8(B)
    N = Cm.shape[0]
    length = B.shape[1]
    S = np.zeros((N, length), np.uint8)
    r = lib().gfo_decode(n, _p(Cm), _p(B), length, N, _p(S), length, length)
    return r, (S if r == N else None)


def count_invertible(n: int, N: int) -> int:
    return int(lib().gfo_count_invertible(n, N))


class Progressive:
    """Progressive (packet-at-a-time) Gauss-Jordan decoder of one generation."""

    def __init__(self, n: int, N: int, length: int):
        self.n, self.N, self.length = n, N, length
        self._h = lib().gfo_prog_new(n, N, length)
        if not self._h:
            raise ValueError("bad progressive decoder arguments")

    def add(self, c: np.ndarray, b: np.ndarray) -> bool:
        c = _u8(c)
        b = _u8(b)
        assert c.size == self.N and b.size == self.length
        r = lib().gfo_prog_add(self._h, _p(c), _p(b))
        if r < 0:
            raise MemoryError
        return bool(r)

    @property
    def rank(self) -> int:
        return lib().gfo_prog_rank(self._h)

    def solve(self) -> Optional[np.ndarray]:
        S = np.zeros((self.N, self.length), np.uint8)
        r = lib().gfo_prog_solve(self._h, _p(S), self.length)
        return S if r == self.N else None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().gfo_prog_free(h)
            self._h = None
