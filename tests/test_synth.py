"""The seeded input generators: determinism and the workload distributions."""
import numpy as np

import synth


def test_splitmix64_reference_values():
    # First outputs of SplitMix64 seeded with 0 (published reference sequence
    # of the generator: state advances by the golden gamma before mixing).
    w = synth.words(0, 3)
    assert [int(v) for v in w] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_deterministic_and_offsettable():
    a = synth.words(123, 100)
    b = synth.words(123, 60, start=40)
    assert (a[40:] == b).all()
    assert (synth.random_bytes(5, 33) == synth.random_bytes(5, 33)).all()
    assert not (synth.random_bytes(5, 33) == synth.random_bytes(6, 33)).all()


def test_distributions():
    b = synth.random_bytes(1, 1 << 16)
    counts = np.bincount(b, minlength=256)
    assert counts.min() > 150 and counts.max() < 370
    nz = synth.uniform_nonzero(2, 5000, 8)
    assert nz.min() >= 1 and nz.size == 5000
    f4 = synth.uniform_field(3, 4000, 2)
    assert set(np.unique(f4).tolist()) == {0, 1, 2, 3}
    Ns, Ls = synth.uneven_shapes(10000, 8)
    assert Ns.min() >= 8 and Ns.max() <= 256 and abs(Ns.mean() - 132) < 3
    assert Ls.min() >= 64 and Ls.max() <= 9000
    # log-uniform: mean (hi-lo)/ln(hi/lo) ~ 1807
    assert abs(Ls.mean() - 1807) < 60
    dN = synth.decode_shapes(3000)
    assert set(np.unique(dN).tolist()) == {32, 64, 128}


def test_single_generation_shape():
    g = synth.single_generation()
    assert g.C.shape == (16, 16) and g.S.shape == (16, 1500)
    assert g.C.min() >= 1


def test_serving_stream():
    reqs = synth.serving_stream(2000, 1000.0)
    t = np.array([r.arrival_s for r in reqs])
    assert (np.diff(t) >= 0).all()
    assert abs(t[-1] - 2.0) < 0.3
    frac = np.mean([r.kind == "decode" for r in reqs])
    assert abs(frac - 0.3) < 0.05


def test_stream_slices_equal_the_whole_stream():
    whole = synth.random_bytes(77, 1000)
    for off, n in [(0, 1000), (1, 7), (8, 16), (13, 500), (999, 1), (500, 0)]:
        assert (synth.random_bytes_at(77, off, n) == whole[off:off + n]).all(), (off, n)
    b = synth.sweep_batch(4, 1500, count=6)
    S_blob, C_blob = b.source_blob(), b.coef_blob()
    for i in (0, 3, 5):
        C, S = b.generation(i, S_blob, C_blob)
        assert (b.source_rows(i) == S).all() and (b.coef_rows(i) == C).all()


def test_device_generator_equals_host_stream():
    """The torch generator (int64 arithmetic, run here on the CPU) yields the host stream's bytes."""
    import torch
    for seed in (0, 5, synth.key(1, 2, 3), (1 << 64) - 1):
        for n in (0, 1, 7, 8, 9, 1001):
            want = synth.random_bytes(seed, n)
            got = synth.device_random_bytes(torch, seed, n, device="cpu", chunk_words=3).numpy()
            assert (got == want).all(), (seed, n)
    b = synth.uniform_batch(2, 5, 7, 100, 3, synth.key(9))
    S, Cb = b.device_blobs(torch, device="cpu")
    assert (S.numpy() == b.source_blob()).all() and (Cb.numpy() == b.coef_blob()).all()
