"""Pins of the oracle's region, encode and decode operations.

Paper Sec. II: a coded packet is b = A c, the sum of c_i times source packet
a_i (Eq. 1); madd is y := y + c x.  Decoding (implied in Sec. I) inverts the
coefficient matrix.  The checks below use properties fixed by linear algebra
over a field: linearity, composition of encodings, identity and zero matrices,
brute-force counts of invertible matrices, order-independence of progressive
decoding.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth

FIELDS = [1, 2, 4, 8]


def _words(n, a):
    """Unpack bytes into n-bit words, LSB-first (independent of the oracle)."""
    a = np.asarray(a, dtype=np.int64)
    per = 8 // n
    mask = (1 << n) - 1
    return np.stack([(a >> (n * k)) & mask for k in range(per)], axis=-1)


def _pack(n, w):
    per = 8 // n
    out = np.zeros(w.shape[:-1], dtype=np.int64)
    for k in range(per):
        out |= w[..., k] << (n * k)
    return out.astype(np.uint8)


@pytest.mark.parametrize("n", FIELDS)
def test_region_madd_matches_wordwise_definition(n):
    T = oracle.mul_table(n)
    x = synth.random_bytes(11, 777)
    y = synth.random_bytes(12, 777)
    for c in range(1 << n):
        got = oracle.region_madd(n, y, x, c)
        want = _pack(n, _words(n, y) ^ T[c][_words(n, x)])
        assert (got == want).all()
        assert (oracle.region_mul(n, x, c) == _pack(n, T[c][_words(n, x)])).all()


@pytest.mark.parametrize("n", FIELDS)
def test_region_trivial_coefficients(n):
    """c = 0 leaves y unchanged; c = 1 is a plain XOR (Sec. IV, trivial cases)."""
    x = synth.random_bytes(1, 1000)
    y = synth.random_bytes(2, 1000)
    assert (oracle.region_madd(n, y, x, 0) == y).all()
    assert (oracle.region_madd(n, y, x, 1) == (y ^ x)).all()


@pytest.mark.parametrize("n", FIELDS)
def test_encode_linearity_and_identity(n):
    g = synth.generation(5, n, 9, 7, 301)
    Y = oracle.encode(n, g.C, g.S)
    # identity and zero coefficient matrices
    assert (oracle.encode(n, np.eye(9, dtype=np.uint8), g.S) == g.S).all()
    assert (oracle.encode(n, np.zeros((3, 9), np.uint8), g.S) == 0).all()
    # linear in S: encode(S1 ^ S2) = encode(S1) ^ encode(S2)
    S2 = synth.random_bytes(99, g.S.size).reshape(g.S.shape)
    assert (oracle.encode(n, g.C, g.S ^ S2) == (Y ^ oracle.encode(n, g.C, S2))).all()
    # linear in C
    C2 = synth.uniform_field(98, g.C.size, n).reshape(g.C.shape)
    assert (oracle.encode(n, g.C ^ C2, g.S) == (Y ^ oracle.encode(n, C2, g.S))).all()
    # each coded row equals the madd chain of Eq. (1)
    for k in range(g.K):
        acc = np.zeros(g.length, np.uint8)
        for i in range(g.N):
            acc = oracle.region_madd(n, acc, g.S[i], int(g.C[k, i]))
        assert (acc == Y[k]).all()


@pytest.mark.parametrize("n", FIELDS)
def test_encode_composition(n):
    """encode(C1, encode(C2, S)) == encode(C1 C2, S): catches transposed operands."""
    S = synth.random_bytes(3, 6 * 50).reshape(6, 50)
    C2 = synth.uniform_field(4, 5 * 6, n).reshape(5, 6)
    C1 = synth.uniform_field(5, 4 * 5, n).reshape(4, 5)
    lhs = oracle.encode(n, C1, oracle.encode(n, C2, S))
    rhs = oracle.encode(n, oracle.matmul(n, C1, C2), S)
    assert (lhs == rhs).all()


def test_gf2_encode_is_xor_of_rows():
    g = synth.generation(6, 1, 12, 10, 128)
    Y = oracle.encode(1, g.C, g.S)
    for k in range(10):
        acc = np.zeros(128, np.uint8)
        for i in range(12):
            if g.C[k, i]:
                acc ^= g.S[i]
        assert (acc == Y[k]).all()


@pytest.mark.parametrize("n", FIELDS)
def test_decode_inverts_encode(n):
    N, L = 10, 123
    S = synth.random_bytes(21, N * L).reshape(N, L)
    attempt = 0
    while True:
        Cm = synth.uniform_field(synth.key(22, attempt), N * N, n).reshape(N, N)
        if oracle.rank(n, Cm) == N:
            break
        attempt += 1
    B = oracle.encode(n, Cm, S)
    r, got = oracle.decode(n, Cm, B)
    assert r == N and (got == S).all()
    Ci = oracle.invert(n, Cm)
    assert (oracle.matmul(n, Ci, Cm) == np.eye(N, dtype=np.uint8)).all()
    assert (oracle.matmul(n, Cm, Ci) == np.eye(N, dtype=np.uint8)).all()
    assert (oracle.encode(n, Ci, B) == S).all()


@pytest.mark.parametrize("n", FIELDS)
def test_decode_singular_reports_rank(n):
    N = 6
    Cm = synth.uniform_field(31, N * N, n).reshape(N, N)
    Cm[4] = Cm[1]                 # duplicate row -> rank <= N-1
    r, S = oracle.decode(n, Cm, np.zeros((N, 10), np.uint8))
    assert r < N and S is None


@pytest.mark.parametrize("n,N,expected", [(1, 2, 6), (1, 3, 168), (2, 2, 180), (2, 3, 181440)])
def test_gl_counts(n, N, expected):
    """|GL(N, q)| = prod_{i<N} (q^N - q^i), counted by enumerating every matrix."""
    q = 1 << n
    assert math.prod(q ** N - q ** i for i in range(N)) == expected
    assert oracle.count_invertible(n, N) == expected


@pytest.mark.parametrize("n,N", [(1, 2), (1, 3), (2, 2)])
def test_inverse_brute_force(n, N):
    """Every invertible matrix's inverse equals the unique X with M X = I found by search."""
    q = 1 << n
    T = oracle.mul_table(n)
    eye = np.eye(N, dtype=np.int64)
    mats = [np.array(v, dtype=np.int64).reshape(N, N)
            for v in itertools.product(range(q), repeat=N * N)]

    def prod(A, B):
        R = np.zeros((N, N), dtype=np.int64)
        for i in range(N):
            for j in range(N):
                acc = 0
                for t in range(N):
                    acc ^= int(T[A[i, t], B[t, j]])
                R[i, j] = acc
        return R

    for M in mats:
        inv = oracle.invert(n, M.astype(np.uint8))
        found = [X for X in mats if (prod(M, X) == eye).all()]
        if inv is None:
            assert not found
        else:
            assert len(found) == 1 and (found[0] == inv).all()


@pytest.mark.parametrize("n,expect", [(1, 0.2888), (2, 0.6885), (4, 0.9336)])
def test_invertible_fraction(n, expect):
    """Fraction of uniform random 16x16 matrices that are invertible ~ prod(1 - q^-i)."""
    trials = 600
    hits = sum(oracle.rank(n, synth.uniform_field(synth.key(40, n, t), 256, n).reshape(16, 16)) == 16
               for t in range(trials))
    p = math.prod(1 - (1 << n) ** -i for i in range(1, 17))
    assert abs(p - expect) < 1e-3
    sd = math.sqrt(p * (1 - p) / trials)
    assert abs(hits / trials - p) < 5 * sd + 1e-9


@pytest.mark.parametrize("n", FIELDS)
def test_progressive_decode_order_invariant(n):
    N, L = 8, 57
    S = synth.random_bytes(50, N * L).reshape(N, L)
    Cm = synth.uniform_field(51, 3 * N * N, n).reshape(3 * N, N)   # 3N coded packets
    B = oracle.encode(n, Cm, S)
    results = []
    for perm_seed in range(4):
        order = np.argsort(synth.words(synth.key(52, perm_seed), 3 * N))
        dec = oracle.Progressive(n, N, L)
        innov = 0
        for idx in order:
            innov += dec.add(Cm[idx], B[idx])
            # a packet identical to one already received is never innovative
            assert not dec.add(Cm[idx], B[idx])
        assert innov == dec.rank == oracle.rank(n, Cm)
        results.append(dec.solve())
    if oracle.rank(n, Cm) == N:
        for r in results:
            assert (r == S).all()


@pytest.mark.parametrize("n", FIELDS)
def test_progressive_equals_batch_decode(n):
    N, L = 12, 40
    S = synth.random_bytes(60, N * L).reshape(N, L)
    attempt = 0
    while True:
        Cm = synth.uniform_field(synth.key(61, attempt), N * N, n).reshape(N, N)
        if oracle.rank(n, Cm) == N:
            break
        attempt += 1
    B = oracle.encode(n, Cm, S)
    dec = oracle.Progressive(n, N, L)
    for i in range(N):
        assert dec.add(Cm[i], B[i])
    assert (dec.solve() == oracle.decode(n, Cm, B)[1]).all()


def _full_rank(n, seed, rows, cols):
    attempt = 0
    while True:
        Cm = synth.uniform_field(synth.key(seed, attempt), rows * cols, n).reshape(rows, cols)
        if oracle.rank(n, Cm) == min(rows, cols):
            return Cm
        attempt += 1


@pytest.mark.parametrize("n", FIELDS)
def test_recode_decodes_to_source(n):
    """Sec. I: a node forwards combinations of packets it received.  Recoded
    packets carry the combined coefficient vectors, so any N of them with an
    invertible header decode to the generation's sources."""
    N, M, Kout, L = 7, 10, 12, 97
    S = synth.random_bytes(31, N * L).reshape(N, L)
    Cin = _full_rank(n, 32, M, N)
    Bin = oracle.encode(n, Cin, S)
    R = synth.uniform_field(33, Kout * M, n).reshape(Kout, M)
    Cout, Yout = oracle.recode(n, R, Cin, Bin)
    assert Cout.shape == (Kout, N) and Yout.shape == (Kout, L)
    # pick N recoded packets whose headers are independent, greedily
    rows = []
    for k in range(Kout):
        if oracle.rank(n, Cout[rows + [k]]) == len(rows) + 1:
            rows.append(k)
        if len(rows) == N:
            break
    if len(rows) < N:   # R could lose rank; over GF(2) with these seeds it does not
        pytest.skip("recoded headers not of full rank for this draw")
    r, got = oracle.decode(n, Cout[rows], Yout[rows])
    assert r == N and (got == S).all()


def test_recode_gf2_is_xor_of_received_packets():
    """Over GF(2) every recoded packet, header and payload, is the XOR of the
    received packets its row of R selects."""
    M, N, Kout, L = 9, 6, 8, 64
    R = synth.uniform_field(41, Kout * M, 1).reshape(Kout, M)
    Cin = synth.uniform_field(42, M * N, 1).reshape(M, N)
    Bin = synth.random_bytes(43, M * L).reshape(M, L)
    Cout, Yout = oracle.recode(1, R, Cin, Bin)
    for k in range(Kout):
        hc = np.zeros(N, np.uint8)
        hy = np.zeros(L, np.uint8)
        for m in range(M):
            if R[k, m]:
                hc ^= Cin[m]
                hy ^= Bin[m]
        assert (hc == Cout[k]).all() and (hy == Yout[k]).all()


@pytest.mark.parametrize("n", FIELDS)
def test_recode_identity_and_two_hops(n):
    """R = I forwards the packets unchanged; recoding twice equals recoding
    once with the product of the two local matrices."""
    M, N, L = 8, 5, 45
    Cin = synth.uniform_field(51, M * N, n).reshape(M, N)
    Bin = synth.random_bytes(52, M * L).reshape(M, L)
    Cout, Yout = oracle.recode(n, np.eye(M, dtype=np.uint8), Cin, Bin)
    assert (Cout == Cin).all() and (Yout == Bin).all()
    R1 = synth.uniform_field(53, 6 * M, n).reshape(6, M)
    R2 = synth.uniform_field(54, 4 * 6, n).reshape(4, 6)
    C1, Y1 = oracle.recode(n, R1, Cin, Bin)
    C2, Y2 = oracle.recode(n, R2, C1, Y1)
    C3, Y3 = oracle.recode(n, oracle.matmul(n, R2, R1), Cin, Bin)
    assert (C2 == C3).all() and (Y2 == Y3).all()


@pytest.mark.parametrize("n", FIELDS)
def test_recode_header_consistent_with_payload(n):
    """The header product is on whole field elements and the payload product
    word by word; on bytes holding one element (< q) the two agree, so a
    recoded header equals the word-wise encode of the received headers."""
    M, N = 6, 11
    R = synth.uniform_field(61, 5 * M, n).reshape(5, M)
    Cin = synth.uniform_field(62, M * N, n).reshape(M, N)
    Cout, _ = oracle.recode(n, R, Cin, np.zeros((M, 0), np.uint8))
    assert (Cout == oracle.encode(n, R, Cin)).all()


def test_encode_batch_is_the_per_generation_encode():
    """The OpenMP batch entry computes each generation exactly as the single
    encode does (generations are independent), with any thread count, and
    leaves the row padding alone."""
    b = synth.uniform_batch(8, 5, 3, 37, 4, synth.key(4242))
    b2 = synth._layout(4, [3, 9, 1, 4], [2, 5, 3, 1], [17, 40, 1, 64], synth.key(4243))
    for bt in (b, b2):
        S_blob, C_blob = bt.source_blob(), bt.coef_blob()
        desc = np.stack([bt.c_off, bt.s_off, bt.y_off, bt.lds, bt.lds, bt.Ls, bt.Ks, bt.Ns], axis=1)
        for threads in (1, 3):
            Y = np.full(bt.y_bytes, 0xA5, np.uint8)
            assert oracle.encode_batch(bt.n, desc, C_blob, S_blob, Y, threads) >= 1
            for i in range(len(bt.Ns)):
                Cm, S = bt.generation(i, S_blob, C_blob)
                K, L, ld = int(bt.Ks[i]), int(bt.Ls[i]), int(bt.lds[i])
                got = Y[bt.y_off[i]:bt.y_off[i] + K * ld].reshape(K, ld)
                assert (got[:, :L] == oracle.encode(bt.n, Cm, S)).all()
                assert (got[:, L:] == 0xA5).all()
