"""The table form (Alg. 1's per-coefficient product tables, re-cut for an
8-entry byte select), checked on the CPU against the oracle.

The product by c is GF(2)-linear in the byte's bits, so
c * b = c * (b & 0x07) ^ c * (b & 0x38) ^ c * (b & 0xC0); each part takes at
most 8 values, and a byte-permute instruction looks 4 of them up at once in an
8-byte table held in two registers.  These tests emulate the byte permute
(V_PERM_B32: selector values 0-7 pick a byte of the 64-bit pair, bytes 0-3
from the second operand) and the table layout, and compare every product with
the oracle's.
"""
import numpy as np
import pytest

import oracle


def perm(s0: int, s1: int, sel: int) -> int:
    """V_PERM_B32 for selector bytes 0..7: byte k of {s0:s1} (s1 holds bytes 0-3)."""
    pair = ((s0 & 0xFFFFFFFF) << 32) | (s1 & 0xFFFFFFFF)
    out = 0
    for i in range(4):
        k = (sel >> (8 * i)) & 0xFF
        assert k < 8
        out |= ((pair >> (8 * k)) & 0xFF) << (8 * i)
    return out


def tables(n: int, c: int):
    """Five dwords: c times v (bits 0-2) for v = 0..7, c times v << 3 for v = 0..7, c times v << 6 for v = 0..3."""
    pb = lambda b: oracle.mulbyte(n, c, b)   # noqa: E731
    t = [0] * 5
    for v in range(8):
        t[v >> 2] |= pb(v) << (8 * (v & 3))
        t[2 + (v >> 2)] |= pb(v << 3) << (8 * (v & 3))
    for v in range(4):
        t[4] |= pb(v << 6) << (8 * v)
    return t


def prod4(t, x: int) -> int:
    a, b, c = x & 0x07070707, (x >> 3) & 0x07070707, (x >> 6) & 0x03030303
    return perm(t[1], t[0], a) ^ perm(t[3], t[2], b) ^ perm(t[4], t[4], c)


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_byte_select_product_equals_the_oracle(n):
    T = oracle.mulbyte_table(n)
    rng = np.random.default_rng(n)
    for c in range(1 << n):
        t = tables(n, c)
        # every byte value in every byte position of a dword
        for base in range(0, 256, 4):
            x = base | ((base + 1) << 8) | ((base + 2) << 16) | ((base + 3) << 24)
            got = prod4(t, x)
            for i in range(4):
                assert (got >> (8 * i)) & 0xFF == T[c, (x >> (8 * i)) & 0xFF]
        x = int(rng.integers(0, 1 << 32))
        got = prod4(t, x)
        assert all((got >> (8 * i)) & 0xFF == T[c, (x >> (8 * i)) & 0xFF] for i in range(4))
