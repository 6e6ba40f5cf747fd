"""The bit-matrix product on FP4 matrix cores, checked on the CPU against the oracle.

Multiplication by a constant c acts on a byte's 8 bits as a GF(2)-linear map
(Sec. II: addition is XOR, and the word-wise product distributes over it), so
output bit b of c * a is the parity of (row b of the map) AND a.  The matrix
cores sum such products as FP4 (E2M1) values from FP32 accumulators that start
at 2^23.  These tests emulate, in numpy, the operand encoding the encode
kernels use (masks of the packed bits, the coefficient rows stored with bits 0
and 2 and bits 4 and 6 exchanged, bits 3 and 7 shifted down) and check, for
every field, coefficient and byte, that each FP4 product is 0 or 1, that their
sum counts the common set bits, and that its parity is the oracle's product.
The GPU tests check the kernels themselves; these pin the method they rely on.
"""
import numpy as np
import pytest

import oracle

FIELDS = [1, 2, 4, 8]


def _e2m1(nibble: np.ndarray) -> np.ndarray:
    """FP4 E2M1 value of each nibble: sign, 2 exponent bits (bias 1), 1 mantissa bit."""
    s = (nibble >> 3) & 1
    e = (nibble >> 1) & 3
    m = nibble & 1
    mag = np.where(e == 0, 0.5 * m, np.exp2(e.astype(np.float64) - 1.0) * (1.0 + 0.5 * m))
    return np.where(s == 1, -mag, mag)


def _source_regs(a: np.ndarray):
    """The four operand registers made from source bytes (one byte per element)."""
    return [a & 0x11, a & 0x22, a & 0x44, (a >> 2) & 0x22]


def _coef_regs(r: np.ndarray):
    return [r & 0x44, r & 0x22, r & 0x11, (r >> 2) & 0x22]


def _swap_0_2(r: np.ndarray) -> np.ndarray:
    """Bits 0 <-> 2 and 4 <-> 6 of each byte exchanged."""
    return (r & 0xAA) | ((r & 0x11) << 2) | ((r & 0x44) >> 2)


def _fp4_dot(a: np.ndarray, r_swapped: np.ndarray) -> np.ndarray:
    """Sum over the 4 registers and both nibbles of FP4(source) * FP4(coefficient)."""
    total = np.zeros(np.broadcast(a, r_swapped).shape, dtype=np.float64)
    for sa, cr in zip(_source_regs(a), _coef_regs(r_swapped)):
        for shift in (0, 4):
            total += _e2m1((sa >> shift) & 0xF) * _e2m1((cr >> shift) & 0xF)
    return total


def _bit_rows(n: int) -> np.ndarray:
    """rows[c, b]: byte whose bit j is bit b of c * (1 << j), from the oracle's word-wise product."""
    T = oracle.mulbyte_table(n).astype(np.int64)          # T[c, x] = c * x word-wise
    q = 1 << n
    rows = np.zeros((q, 8), dtype=np.int64)
    for b in range(8):
        for j in range(8):
            rows[:, b] |= ((T[:q, 1 << j] >> b) & 1) << j
    return rows


@pytest.mark.parametrize("n", FIELDS)
def test_fp4_products_count_common_bits_and_give_the_field_product(n):
    q = 1 << n
    T = oracle.mulbyte_table(n).astype(np.int64)
    rows = _bit_rows(n)                                   # (q, 8)
    a = np.arange(256, dtype=np.int64)[None, None, :]     # every source byte
    r = rows[:, :, None]                                  # every coefficient and output bit
    s = _fp4_dot(a, _swap_0_2(r))
    # every product is 0 or 1, so the sum is the count of common set bits
    common = np.vectorize(lambda v: bin(int(v)).count("1"))(r & a)
    assert np.array_equal(s, common.astype(np.float64))
    # its parity is bit b of the oracle's product c * a
    parity = (s.astype(np.int64) & 1)
    want = (T[:q, :][:, None, :] >> np.arange(8)[None, :, None]) & 1
    assert np.array_equal(parity, want)


def test_each_register_pair_multiplies_to_exactly_one():
    """Single set input bits: the source and coefficient nibbles of the same bit
    multiply to 1, of different bits to 0 (no cross terms)."""
    for i in range(8):
        for j in range(8):
            s = _fp4_dot(np.array([1 << i]), _swap_0_2(np.array([1 << j])))
            assert s[0] == (1.0 if i == j else 0.0), (i, j)


def test_operands_never_use_the_sign_bit():
    a = np.arange(256, dtype=np.int64)
    for reg in _source_regs(a) + _coef_regs(a):
        assert not np.any(reg & 0x88)


def test_biased_fp32_counts_are_exact_and_keep_their_parity():
    """Accumulators start at 2^23; a tile adds at most 2048 per strip for at most
    2048 strips before restarting, so every partial sum stays below 2^23 + 2^22.
    Below 2^24 every integer is exact in FP32 and the count's parity is bit 0."""
    counts = np.arange(0, (1 << 22) + 1, dtype=np.int64)
    f = np.float32(1 << 23) + counts.astype(np.float32)
    assert np.array_equal(f.astype(np.int64) - (1 << 23), counts)
    assert np.array_equal(f.view(np.uint32) & 1, (counts & 1).astype(np.uint32))
    # running sums of per-instruction increments (each at most 64) in FP32
    rng = np.random.default_rng(190902871)
    inc = rng.integers(0, 65, size=200_000).astype(np.float32)
    acc = np.float32(1 << 23)
    ref = 1 << 23
    for v in inc[:20_000]:
        acc = np.float32(acc + v)
        ref += int(v)
    assert int(acc) == ref and (int(np.float32(acc).view(np.uint32)) & 1) == (ref & 1)


def test_strip_parity_from_running_totals():
    """A strip's output bit is the parity of the running total XOR that of the
    previous total: the parity of the strip's own count."""
    rng = np.random.default_rng(2)
    per_strip = rng.integers(0, 2049, size=1000)
    totals = np.cumsum(per_strip)
    prev = np.concatenate([[0], totals[:-1]])
    assert np.array_equal((totals & 1) ^ (prev & 1), per_strip & 1)
