"""The serving runtime's progressive decode, checked on the CPU against the oracle.

The device state of a decode request keeps R, the reduced row echelon form of
the innovative coefficient vectors received so far, the transform T with
R = T * Csel (Csel: the accepted packets' raw coefficient rows, in order of
acceptance), and each accepted packet's payload.  A packet's vector is
reduced against all rows of R in one pass (R is reduced, so no row
reintroduces a pivot another row cleared), and its transform row is the same
combination of T's rows plus its own unit weight; a zero vector means the
packet is not innovative and is dropped.  Otherwise both are scaled so the
vector's lowest nonzero column holds 1, that column is cleared from the other
rows of R (T's rows take the same updates), and the payload is kept.  At rank
N, R is the identity with its rows in pivot order, so row pivot(j) of
Csel^-1 is row j of T, and the sources are Csel^-1 * Bsel with no inversion.
These tests emulate that scheme and compare the innovative decisions, the
rank and the decoded sources with the oracle's progressive decoder (which
eliminates over [coefficients | payload] instead), and the inverse with the
oracle's inverse of Csel.
"""
import numpy as np
import pytest

import oracle
import synth


class Absorb:
    def __init__(self, n: int, N: int):
        self.n, self.N = n, N
        self.M = oracle.mul_table(n)
        self.R = []            # (pivot column, row of R, row of T), reduced
        self.Csel, self.Bsel = [], []

    def add(self, c: np.ndarray, b: np.ndarray) -> bool:
        M, N = self.M, self.N
        v = c.astype(np.int64).copy()
        f = [int(v[p]) for p, _, _ in self.R]   # factors from the vector as received
        for (p, row, trow), fr in zip(self.R, f):
            v ^= M[fr][row]
        nz = np.nonzero(v)[0]
        if len(nz) == 0:
            return False
        t = np.zeros(N, dtype=np.int64)
        t[len(self.R)] = 1                      # the new packet's own weight (innovative: rank < N)
        for (p, row, trow), fr in zip(self.R, f):
            t ^= M[fr][trow]
        p = int(nz[0])
        iv = oracle.inv(self.n, int(v[p]))
        v, t = M[iv][v], M[iv][t]
        for i, (q, row, trow) in enumerate(self.R):
            g = int(row[p])
            self.R[i] = (q, row ^ M[g][v], trow ^ M[g][t])
        self.R.append((p, v, t))
        self.Csel.append(c.copy())
        self.Bsel.append(b.copy())
        return True

    @property
    def rank(self) -> int:
        return len(self.R)

    def inverse(self):
        """Csel^-1 read off T: row pivot(j) is row j of T."""
        Cinv = np.zeros((self.N, self.N), dtype=np.uint8)
        for p, _, trow in self.R:
            Cinv[p] = trow
        return Cinv

    def solve(self):
        if self.rank < self.N:
            return None
        return oracle.encode(self.n, self.inverse(), np.array(self.Bsel, dtype=np.uint8))


@pytest.mark.parametrize("n", [1, 2, 4, 8])
@pytest.mark.parametrize("N", [1, 3, 8, 24])
def test_absorb_matches_the_oracle_progressive_decoder(n, N):
    L = 37
    S = synth.random_bytes(synth.key(80, n, N), N * L).reshape(N, L)
    a, o = Absorb(n, N), oracle.Progressive(n, N, L)
    for i in range(3 * N + 4):
        c = synth.uniform_field(synth.key(81, n, N, i), N, n)
        if i % 5 == 4 and a.Csel:
            c = a.Csel[0].copy()                           # a repeated packet
        if i % 7 == 6 and len(a.Csel) >= 2:                # a combination of two kept packets
            c = (a.Csel[0] ^ a.Csel[1]).astype(np.uint8)
        b = oracle.encode(n, c.reshape(1, N), S)[0]
        assert a.add(c, b) == o.add(c, b), i
        assert a.rank == o.rank
        R = np.zeros((len(a.R), N), dtype=np.int64)
        for j, (p, row, trow) in enumerate(sorted(a.R, key=lambda t: t[0])):
            R[j] = row
            assert row[p] == 1 and all(other[p] == 0 for q, other, _ in a.R if q != p)
            # R = T * Csel holds row by row
            C = np.array(a.Csel, dtype=np.uint8)
            assert np.array_equal(oracle.matmul(n, trow[:len(a.Csel)].astype(np.uint8).reshape(1, -1), C)[0], row)
    got, want = a.solve(), o.solve()
    if want is None:
        assert got is None
    else:
        assert np.array_equal(got, want) and np.array_equal(got, S)
        assert np.array_equal(a.inverse(), oracle.invert(n, np.array(a.Csel, dtype=np.uint8)))


def test_dependent_packets_never_raise_the_rank():
    n, N = 8, 6
    a = Absorb(n, N)
    base = [synth.uniform_field(synth.key(82, i), N, n) for i in range(3)]
    for c in base:
        a.add(c, np.zeros(4, np.uint8))
    r = a.rank
    M = oracle.mul_table(n)
    for k in range(20):
        coeffs = synth.uniform_field(synth.key(83, k), 3, n)
        c = np.zeros(N, dtype=np.int64)
        for f, v in zip(coeffs, base):
            c ^= M[int(f)][v.astype(np.int64)]
        assert not a.add(c.astype(np.uint8), np.zeros(4, np.uint8))
    assert a.rank == r
