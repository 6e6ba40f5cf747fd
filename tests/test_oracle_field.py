"""Pins of the oracle's field arithmetic against facts that do not depend on it.

Paper Sec. II defines the fields: words of n bits, q = 2^n, addition by XOR,
multiplication by reduction with a field polynomial.  Sec. IV-A (Algorithm 1,
split-nibble tables) and Sec. IV-B (Algorithm 2, multiplication by the
products of c with the basis elements) are two further ways to compute the
same word-wise product; emulating them must reproduce the oracle exactly.
"""
import os

import numpy as np
import pytest

import oracle

FIELDS = [1, 2, 4, 8]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table(n):
    return oracle.mul_table(n)


@pytest.mark.parametrize("n", FIELDS)
def test_axioms_exhaustive(n):
    """Commutativity, identities, distributivity and associativity over all elements."""
    q = 1 << n
    T = _table(n)
    a = np.arange(q)
    assert (T == T.T).all()
    assert (T[0] == 0).all() and (T[1] == a).all()
    assert T.min() >= 0 and T.max() < q
    # distributivity a(b+c) = ab + ac, with + = XOR, for all triples
    A, B, Cc = np.meshgrid(a, a, a, indexing="ij")
    assert (T[A, B ^ Cc] == (T[A, B] ^ T[A, Cc])).all()
    # associativity (ab)c = a(bc) for all q^3 triples
    assert (T[T[A, B], Cc] == T[A, T[B, Cc]]).all()


@pytest.mark.parametrize("n", FIELDS)
def test_no_zero_divisors_and_latin_rows(n):
    """Each nonzero row of the product table is a permutation of the nonzero elements."""
    q = 1 << n
    T = _table(n)
    for a in range(1, q):
        assert sorted(T[a, 1:].tolist()) == list(range(1, q))


@pytest.mark.parametrize("n", FIELDS)
def test_two_multipliers_agree(n):
    """Full carry-less product then reduction == shift-and-reduce-each-step."""
    q = 1 << n
    for a in range(q):
        for b in range(q):
            assert oracle.mul(n, a, b) == oracle.mul_peasant(n, a, b)


@pytest.mark.parametrize("n", FIELDS)
def test_inverse(n):
    q = 1 << n
    for a in range(1, q):
        assert oracle.mul(n, a, oracle.inv(n, a)) == 1
        # Lagrange: a^(q-1) = 1, so a^(q-2) is the inverse
        assert oracle.pow_(n, a, q - 2) == oracle.inv(n, a) or q == 2


@pytest.mark.parametrize("n", [2, 4, 8])
def test_x_is_primitive(n):
    """x (= 2) has order q-1: the polynomials named for each field are primitive."""
    q = 1 << n
    seen = set()
    e = 1
    for i in range(q - 1):
        seen.add(e)
        e = oracle.mul(n, e, 2)
    assert e == 1 and len(seen) == q - 1


@pytest.mark.parametrize("n", [2, 4, 8])
def test_log_exp_multiplier(n):
    """mul(a, b) = x^(log a + log b), with logs read off the powers of x."""
    q = 1 << n
    exp = [1]
    for _ in range(q - 2):
        exp.append(oracle.mul(n, exp[-1], 2))
    log = {v: i for i, v in enumerate(exp)}
    for a in range(1, q):
        for b in range(1, q):
            assert oracle.mul(n, a, b) == exp[(log[a] + log[b]) % (q - 1)]


def test_golden_values():
    path = os.path.join(GOLDEN, "field_values.txt")
    count = 0
    with open(path) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            kind, n, a, b, want = line.split()
            n, a, b, want = int(n), int(a), int(b), int(want)
            if kind == "mul":
                got = oracle.mul(n, a, b)
            elif kind == "mulbyte":
                got = oracle.mulbyte(n, a, b)
            elif kind == "inv":
                got = oracle.inv(n, a)
            elif kind == "pow":
                got = oracle.pow_(n, a, b)
            else:
                raise AssertionError(kind)
            assert got == want, line
            count += 1
    assert count >= 20


def test_golden_powers():
    with open(os.path.join(GOLDEN, "powers_of_x.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            n, vals = line.split(":")
            n = int(n)
            vals = [int(v) for v in vals.split()]
            assert len(set(vals)) == (1 << n) - 1
            for i, v in enumerate(vals):
                assert oracle.pow_(n, 2, i) == v


@pytest.mark.parametrize("n", FIELDS)
def test_mulbyte_is_wordwise(n):
    """Byte-wise product == product of each unpacked word, repacked (LSB-first words)."""
    T = _table(n)
    mask = (1 << n) - 1
    for c in range(1 << n):
        for b in range(256):
            want = 0
            for k in range(8 // n):
                want |= int(T[c, (b >> (n * k)) & mask]) << (n * k)
            assert oracle.mulbyte(n, c, b) == want


@pytest.mark.parametrize("n", FIELDS)
def test_paper_shuffle_algorithm(n):
    """Sec. IV-A: XOR of the low- and high-nibble table lookups equals the product."""
    for c in range(1 << n):
        tl, th = oracle.shuffle_tables(n, c)
        # the tables hold the products of c with the 16 possible nibbles
        for x in range(16):
            assert tl[x] == oracle.mulbyte(n, c, x)
            assert th[x] == oracle.mulbyte(n, c, x << 4)
        for a in range(256):
            assert oracle.shuffle_byte(n, c, a) == oracle.mulbyte(n, c, a)


@pytest.mark.parametrize("n", FIELDS)
def test_paper_imul_algorithm(n):
    """Sec. IV-B: masked bit planes times c*x^i, XORed, equals the product on 32-bit lanes."""
    rng = np.random.default_rng(7)
    vals = [0, 0xFFFFFFFF, 0x55555555, 0xAAAAAAAA, 0x12345678] + \
        rng.integers(0, 1 << 32, 200, dtype=np.uint64).tolist()
    for c in range(1 << n):
        p = oracle.imul_powers(n, c)
        # p[i] is c times the i-th basis element
        for i in range(n):
            assert p[i] == oracle.mul(n, c, 1 << i)
        for v in vals:
            want = 0
            for t in range(4):
                want |= oracle.mulbyte(n, c, (int(v) >> (8 * t)) & 0xFF) << (8 * t)
            assert oracle.imul_word(n, c, int(v)) == want


def test_gf4_powers_example_from_paper_masks():
    """GF(4), c = 2: the products with the basis are [2, 3] (the pow table of Algorithm 2)."""
    assert oracle.imul_powers(2, 2) == [2, 3]
    assert oracle.imul_powers(2, 3) == [3, 1]


def test_invalid_arguments_rejected():
    assert oracle.mul(8, 256, 1) == -1
    assert oracle.mul(4, 16, 1) == -1
    assert oracle.mul(1, 2, 1) == -1
    with pytest.raises(ValueError):
        oracle.region_madd(4, np.zeros(4, np.uint8), np.zeros(4, np.uint8), 16)
    with pytest.raises(ValueError):
        oracle.region_madd(1, np.zeros(4, np.uint8), np.zeros(4, np.uint8), 2)
