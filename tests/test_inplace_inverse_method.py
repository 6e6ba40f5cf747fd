"""The in-place Gauss-Jordan inversion the decode kernels use, checked on the
CPU against the oracle's elimination on [C | I].

In place: for each pivot column k, the lowest row at or below k with a nonzero
entry in column k is swapped into row k; the pivot entry is replaced by 1 and
the row scaled by the pivot's inverse, so that column k of the row ends up
holding the inverse's entry; every other row i then has its column-k entry
replaced by 0 and the pivot row times that entry added to it.  After the last
pivot the matrix holds the inverse with its columns permuted by the row swaps,
which are undone as column swaps in reverse order.  A column without a pivot
means rank < N.
"""
import numpy as np
import pytest

import oracle
import synth


def inplace_inverse(n: int, C: np.ndarray):
    M = oracle.mul_table(n)
    A = C.astype(np.int64).copy()
    N = A.shape[0]
    swaps = []
    for k in range(N):
        rows = [r for r in range(k, N) if A[r, k] != 0]
        if not rows:
            return None
        p = rows[0]
        if p != k:
            A[[k, p]] = A[[p, k]]
        swaps.append(p)
        inv = oracle.inv(n, int(A[k, k]))
        A[k, k] = 1
        A[k] = M[inv][A[k]]
        for i in range(N):
            if i != k and A[i, k] != 0:
                f = int(A[i, k])
                A[i, k] = 0
                A[i] ^= M[f][A[k]]
    for k in reversed(range(N)):
        p = swaps[k]
        if p != k:
            A[:, [k, p]] = A[:, [p, k]]
    return A


@pytest.mark.parametrize("n", [1, 2, 4, 8])
@pytest.mark.parametrize("N", [1, 2, 5, 16, 33])
def test_inplace_inverse_equals_the_oracle(n, N):
    for t in range(6):
        C = synth.uniform_field(synth.key(70, n, N, t), N * N, n).reshape(N, N)
        if t == 5 and N > 1:
            C[N - 1] = C[0]            # a repeated row: singular
        want = oracle.invert(n, C)
        got = inplace_inverse(n, C)
        if want is None:
            assert got is None and oracle.rank(n, C) < N
        else:
            assert got is not None and np.array_equal(got, want.astype(np.int64))


def test_pivots_need_row_swaps():
    """A matrix whose leading entries are zero exercises the swap and its undoing."""
    n, N = 8, 4
    C = np.array([[0, 1, 0, 0], [0, 0, 3, 0], [5, 0, 0, 0], [0, 0, 0, 7]], dtype=np.uint8)
    assert np.array_equal(inplace_inverse(n, C), oracle.invert(n, C).astype(np.int64))
