"""The bit-plane form (the bit decomposition of Sec. IV-B with the roles of
data and coefficient swapped), checked on the CPU against the oracle.

With c = sum_b c_b x^b, c * a = XOR over b of c_b * (x^b * a): the kernels
build the planes x^b * a word-wise with a few shifts and masks per dword and
add each one under an all-ones or all-zero mask with a single 3-input bit
operation.  These tests emulate those word-wise formulas and the bit
operation's truth tables and compare with the oracle's product for every
coefficient and byte.
"""
import numpy as np
import pytest

import oracle


def times_x(n: int, v: np.ndarray) -> np.ndarray:
    """x times every n-bit word of a 32-bit value, as the bit-plane kernels compute it."""
    v = v.astype(np.uint64) & 0xFFFFFFFF
    if n == 2:      # x^2 = x + 1: (h, l) -> (h ^ l, h)
        return ((v >> 1) & 0x55555555) | ((v ^ (v << 1)) & 0xAAAAAAAA)
    if n == 4:      # x^4 = x + 1: shift up in the nibble; the top bit folds into bits 0 and 1
        t = v & 0x88888888
        return ((v << 1) & 0xEEEEEEEE) ^ (t >> 3) ^ (t >> 2)
    raise ValueError(n)


def bitop3(a: int, b: int, c: int, table: int) -> int:
    """V_BITOP3_B32: bit i of the result is bit (a_i << 2 | b_i << 1 | c_i) of `table`."""
    out = 0
    for i in range(32):
        idx = (((a >> i) & 1) << 2) | (((b >> i) & 1) << 1) | ((c >> i) & 1)
        out |= ((table >> idx) & 1) << i
    return out


@pytest.mark.parametrize("n", [2, 4])
def test_times_x_is_the_fields_product_by_x(n):
    words = np.arange(256, dtype=np.uint64)
    # four bytes of a dword: every byte value in every position
    dw = words | (np.roll(words, 1) << 8) | (np.roll(words, 2) << 16) | (np.roll(words, 3) << 24)
    got = times_x(n, dw)
    for pos in range(4):
        byte = (dw >> (8 * pos)) & 0xFF
        want = np.array([oracle.mulbyte(n, 2, int(b)) for b in byte], dtype=np.uint64)
        assert np.array_equal((got >> (8 * pos)) & 0xFF, want)


@pytest.mark.parametrize("n", [1, 2, 4])
def test_planes_under_coefficient_bits_give_the_product(n):
    q = 1 << n
    a = np.arange(256, dtype=np.uint64)
    planes = [a]
    for _ in range(1, n):
        planes.append(times_x(n, planes[-1]))
    T = oracle.mulbyte_table(n)
    for c in range(q):
        acc = np.zeros(256, dtype=np.uint64)
        for b in range(n):
            mask = np.uint64(0xFFFFFFFF) if (c >> b) & 1 else np.uint64(0)
            acc ^= planes[b] & mask
        assert np.array_equal(acc & 0xFF, T[c].astype(np.uint64)), c


def test_bit_operation_truth_tables():
    rng = np.random.default_rng(3)
    for a, b, c in rng.integers(0, 1 << 32, size=(200, 3), dtype=np.uint64):
        a, b, c = int(a), int(b), int(c)
        assert bitop3(a, b, c, 0x78) == a ^ (b & c)       # bit-plane form: acc ^ (plane & mask)
        assert bitop3(a, b, c, 0x96) == a ^ b ^ c         # table form: three-way XOR
