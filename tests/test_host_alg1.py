"""The host AVX-512BW shuffle madd (Sec. IV-A) that bench.py times as CPU
context: it must give the oracle's bytes before its timings mean anything."""
import numpy as np
import pytest

import bench
import oracle
import synth


@pytest.fixture(scope="module")
def alg1():
    L = bench.alg1_lib()
    if not L.alg1_supported():
        pytest.skip("host CPU has no AVX-512BW")
    return L


@pytest.mark.parametrize("n", [1, 2, 4, 8])
@pytest.mark.parametrize("length", [0, 1, 63, 64, 65, 1500, 4099])
def test_region_madd_matches_oracle(alg1, n, length):
    x = synth.random_bytes(synth.key(90, n, length), length)
    y0 = synth.random_bytes(synth.key(91, n, length), length)
    for c in sorted({0, 1, (1 << n) - 1, 2 % (1 << n), 0x53 % (1 << n)}):
        y = y0.copy()
        assert alg1.alg1_region_madd(n, y.ctypes.data, x.ctypes.data, c, length) == 0
        assert (y == oracle.region_madd(n, y0, x, c)).all(), c


def test_region_madd_rejects_bad_arguments(alg1):
    y = np.zeros(8, np.uint8)
    assert alg1.alg1_region_madd(3, y.ctypes.data, y.ctypes.data, 1, 8) == -1
    assert alg1.alg1_region_madd(4, y.ctypes.data, y.ctypes.data, 16, 8) == -1
    assert alg1.alg1_region_madd(1, y.ctypes.data, y.ctypes.data, 2, 8) == -1


@pytest.mark.parametrize("n", [2, 4, 8])
def test_encode_matches_oracle(alg1, n):
    g = synth.generation(synth.key(92, n), n, 16, 16, 777)
    S = np.ascontiguousarray(g.S)
    Cm = np.ascontiguousarray(g.C)
    Y = np.full((16, 777), 0xAB, np.uint8)
    t = alg1.alg1_encode_seconds(n, Cm.ctypes.data, 16, 16, S.ctypes.data, 777, Y.ctypes.data, 777, 777, 3)
    assert t > 0
    assert (Y == oracle.encode(n, Cm, S)).all()
