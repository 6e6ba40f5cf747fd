"""GPU results against the CPU oracle, byte for byte (integer work: bit-exact).

Region madd (paper Sec. II and Sec. IV), encoding (Sec. II, Eq. 1 for K
coding vectors) and Gauss-Jordan decoding, over GF(2), GF(4), GF(16) and
GF(256), through the C ABI.  Inputs come from the seeded generators; sizes
span several tiles and ragged tails; unaligned rows and offsets take the
byte path and are covered too.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, padded_rows, torch_cuda

pytestmark = pytest.mark.gpu

FIELDS = [1, 2, 4, 8]


@pytest.fixture(scope="module")
def gf():
    torch_cuda()
    import paper_1909_02871_amd as g
    g.gf_init()
    return g


def _coefs(n):
    q = 1 << n
    return sorted({0, 1, q - 1, min(2, q - 1), (0x53 % q)})


# ------------------------------------------------------------------ region

@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("length", [0, 1, 15, 16, 17, 1000, 4109, 70001])
def test_region_madd_mul(gf, n, length):
    torch = torch_cuda()
    x = synth.random_bytes(synth.key(1, n, length), length)
    y = synth.random_bytes(synth.key(2, n, length), length)
    for c in _coefs(n):
        print("region", n, length, c, flush=True)
        yd = dev(y) if length else torch.zeros(0, dtype=torch.uint8, device="cuda")
        xd = dev(x) if length else torch.zeros(0, dtype=torch.uint8, device="cuda")
        gf.gf_region_madd(n, yd, xd, c)
        assert (host(yd) == oracle.region_madd(n, y, x, c)).all()
        gf.gf_region_mul(n, yd, xd, c)
        assert (host(yd) == oracle.region_mul(n, x, c)).all()


@pytest.mark.parametrize("n,c", [(8, 0x53), (1, 1)])
@pytest.mark.parametrize("offset", [0, 5])
def test_region_madd_large(gf, n, c, offset):
    """A region past 32 MiB (a launch of 5,121 workgroups of 8 KiB, where the grid
    was once capped and looped), with a 13-byte tail, and one off the 16-byte grid
    (the byte path): every byte equals the oracle's, the bytes around untouched."""
    torch = torch_cuda()
    L = (40 << 20) + 13
    x = synth.random_bytes(synth.key(64, n, offset), L)
    y = synth.random_bytes(synth.key(65, n, offset), L)
    xb = torch.zeros(L + 32, dtype=torch.uint8, device="cuda")
    yb = torch.full((L + 32,), 0x2D, dtype=torch.uint8, device="cuda")
    xb[offset:offset + L] = dev(x)
    yb[offset:offset + L] = dev(y)
    gf.gf_region_madd(n, yb[offset:offset + L], xb[offset:offset + L], c)
    out = host(yb)
    assert (out[offset:offset + L] == oracle.region_madd(n, y, x, c)).all()
    assert (out[:offset] == 0x2D).all() and (out[offset + L:] == 0x2D).all()


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("xo,yo", [(1, 1), (3, 0), (0, 5), (7, 9)])
def test_region_unaligned(gf, n, xo, yo):
    torch = torch_cuda()
    L = 3001
    x = synth.random_bytes(synth.key(3, n, xo), L)
    y = synth.random_bytes(synth.key(4, n, yo), L)
    c = (1 << n) - 1
    xb = torch.zeros(L + 32, dtype=torch.uint8, device="cuda")
    yb = torch.zeros(L + 32, dtype=torch.uint8, device="cuda")
    xb[xo:xo + L] = dev(x)
    yb[yo:yo + L] = dev(y)
    gf.gf_region_madd(n, yb[yo:yo + L], xb[xo:xo + L], c)
    out = host(yb)
    assert (out[yo:yo + L] == oracle.region_madd(n, y, x, c)).all()
    assert (out[:yo] == 0).all() and (out[yo + L:] == 0).all()


@pytest.mark.parametrize("n", FIELDS)
def test_region_alias(gf, n):
    x = synth.random_bytes(5, 5000)
    for c in _coefs(n):
        xd = dev(x)
        gf.gf_region_madd(n, xd, xd, c)   # y == x: (1 + c) x
        assert (host(xd) == oracle.region_madd(n, x, x, c)).all()


@pytest.mark.parametrize("n", FIELDS)
def test_region_batched(gf, n):
    torch = torch_cuda()
    cnt = 300
    Ls = synth.log_uniform_ints(synth.key(6, n), cnt, 1, 20000)
    cs = synth.uniform_field(synth.key(7, n), cnt, n)
    xs = [synth.random_bytes(synth.key(8, n, i), int(L)) for i, L in enumerate(Ls)]
    ys = [synth.random_bytes(synth.key(9, n, i), int(L)) for i, L in enumerate(Ls)]
    xd = [dev(a) for a in xs]
    yd = [dev(a) for a in ys]
    regs = gf.make_regions([(yd[i].data_ptr(), xd[i].data_ptr(), int(Ls[i]), int(cs[i])) for i in range(cnt)])
    gf.gf_region_madd_batched(n, regs, cnt, int(Ls.max()))
    torch.cuda.synchronize()
    for i in range(cnt):
        assert (host(yd[i]) == oracle.region_madd(n, ys[i], xs[i], int(cs[i]))).all(), i


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("max_len", [16, 600, 1500, 2048, 3000])
def test_region_batched_short(gf, n, max_len):
    """Short regions (the kernels that give a region half a wave or a wave):
    lengths from 0 to max_len, zero coefficients, an odd count, and every
    seventh region off the 16-byte grid (its pair then goes piece by piece);
    bytes around every region untouched."""
    torch = torch_cuda()
    cnt = 301
    Ls = synth.uniform_ints(synth.key(60, n, max_len), cnt, 0, max_len)
    Ls[:4] = [0, 1, max_len, max_len - 1]
    cs = synth.uniform_field(synth.key(61, n, max_len), cnt, n)
    cs[5::9] = 0
    xs = [synth.random_bytes(synth.key(62, n, i), int(L)) for i, L in enumerate(Ls)]
    ys = [synth.random_bytes(synth.key(63, n, i), int(L)) for i, L in enumerate(Ls)]
    bufs, regs = [], []
    for i, L in enumerate(Ls):
        off = 3 if i % 7 == 6 else 0
        xb = torch.full((int(L) + 48,), 0x77, dtype=torch.uint8, device="cuda")
        yb = torch.full((int(L) + 48,), 0x66, dtype=torch.uint8, device="cuda")
        if L:
            xb[off:off + L] = dev(xs[i])
            yb[off:off + L] = dev(ys[i])
        bufs.append((xb, yb, off))
        regs.append((yb.data_ptr() + off, xb.data_ptr() + off, int(L), int(cs[i])))
    gf.gf_region_madd_batched(n, gf.make_regions(regs), cnt, int(Ls.max()))
    torch.cuda.synchronize()
    for i, (xb, yb, off) in enumerate(bufs):
        L = int(Ls[i])
        out = host(yb)
        assert (out[off:off + L] == oracle.region_madd(n, ys[i], xs[i], int(cs[i]))).all(), (i, L)
        assert (out[:off] == 0x66).all() and (out[off + L:] == 0x66).all(), i


# ------------------------------------------------------------------ encode

SHAPES = [(1, 1, 1), (3, 7, 33), (16, 16, 1500), (64, 64, 1500), (40, 200, 513), (255, 256, 77),
          (8, 256, 9000), (33, 5, 4096 + 5), (2, 3, 20000)]


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("K,N,L", SHAPES)
def test_encode(gf, n, K, N, L):
    torch = torch_cuda()
    print("encode", n, K, N, L, flush=True)
    g = synth.generation(synth.key(10, n, K, N, L), n, N, K, L)
    want = oracle.encode(n, g.C, g.S)
    Cd = dev(g.C)
    for ld_pad, off in [(0, 0), (16, 0), (3, 1)]:
        ld = synth.padded(L) + ld_pad if ld_pad != 3 else L + 3
        _, Sd = padded_rows(g.S, ld, off)
        yb, Yd = padded_rows(np.zeros((K, L), np.uint8), ld, off, fill=0x5A)
        gf.gf_encode(n, Cd, Sd, Yd)
        got = host(Yd)
        assert (got == want).all(), (ld_pad, off)
        # bytes between rows and around the output are untouched
        raw = host(yb)
        mask = np.ones(raw.size, bool)
        for k in range(K):
            mask[off + k * ld: off + k * ld + L] = False
        assert (raw[mask] == 0x5A).all()


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("form,bpl", [(1, 0), (1, 4), (1, 8), (1, 16), (2, 0), (3, 0), (3, 4), (3, 8), (3, 16)])
@pytest.mark.parametrize("grid", [0, 1, 7, -1])
def test_encode_every_variant(gf, n, form, bpl, grid):
    """Every schedule of every kernel form gives the same bytes (batched path, 30
    generations; N up to 80 spans several mask stages of the bit-plane form);
    grid -1 is the non-persistent dispatch of the vector-ALU forms (a workgroup
    per four wave tiles), which the bit-matrix form refuses."""
    torch = torch_cuda()
    if form == 3 and n == 8:
        C1, S1, Y1 = dev(np.ones((2, 2), np.uint8)), dev(np.ones((2, 8), np.uint8)), dev(np.zeros((2, 8), np.uint8))
        with pytest.raises(gf.GFError):      # the bit-plane form covers n <= 4 only
            gf.gf_plan_encode(n, [(C1, S1, Y1)], tune={"form": 3})
        return
    gens, keep, wants = [], [], []
    for i in range(30):
        N = int(synth.uniform_ints(synth.key(11, i), 1, 1, 80)[0])
        K = int(synth.uniform_ints(synth.key(12, i), 1, 1, 70)[0])
        L = int(synth.uniform_ints(synth.key(13, i), 1, 1, 5000)[0])
        g = synth.generation(synth.key(14, n, i), n, N, K, L)
        wants.append(oracle.encode(n, g.C, g.S))
        Cd = dev(g.C)
        _, Sd = padded_rows(g.S, synth.padded(L))
        _, Yd = padded_rows(np.zeros((K, L), np.uint8), synth.padded(L))
        keep.append((Cd, Sd, Yd))
    if grid == -1 and form == 2:
        with pytest.raises(gf.GFError):
            gf.gf_plan_encode(n, keep, tune={"form": form, "bytes_per_lane": bpl, "grid_blocks": grid})
        return
    plan = gf.gf_plan_encode(n, keep, tune={"form": form, "bytes_per_lane": bpl, "grid_blocks": grid})
    assert plan.tuning()["bytes_per_lane"] == bpl and plan.tuning()["form"] == form
    assert grid == 0 or plan.tuning()["grid_blocks"] == (grid if grid > 0 else plan.tuning()["grid_blocks"])
    assert plan.tuning()["grid_blocks"] > 0
    for rep in range(2):      # the work counter resets itself between launches
        for _, _, Yd in keep:
            Yd.zero_()
        gf.gf_plan_launch(plan)
        torch.cuda.synchronize()
        for (Cd, Sd, Yd), w in zip(keep, wants):
            assert (host(Yd) == w).all()
    # per-generation launches with the same schedule
    for _, _, Yd in keep:
        Yd.zero_()
    gf.gf_encode_each(n, keep, tune={"bytes_per_lane": bpl})
    torch.cuda.synchronize()
    for (Cd, Sd, Yd), w in zip(keep, wants):
        assert (host(Yd) == w).all()


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("form", [0, 2, 3])
@pytest.mark.parametrize("pitch,off", [(3, 1), (4, 4)])
def test_batched_encode_odd_rows(gf, n, form, pitch, off):
    """Row pitch and offset off the 16-byte grid: odd (byte paths of every form)
    and word-aligned (word copies of the bit-matrix form); the autotuned plan."""
    torch = torch_cuda()
    if form == 3 and n == 8:
        pytest.skip("the bit-plane form covers n <= 4")
    items, wants = [], []
    for i in range(12):
        N = [1, 7, 8, 9, 16, 17, 33, 100, 255, 256, 40, 3][i]
        K = [1, 9, 16, 17, 31, 64, 5, 100, 3, 256, 48, 2][i]
        L = [1, 2, 3, 255, 256, 257, 511, 1000, 77, 300, 2049, 4096][i]
        g = synth.generation(synth.key(15, n, i), n, N, K, L)
        wants.append(oracle.encode(n, g.C, g.S))
        _, Sd = padded_rows(g.S, (L + 3) // 4 * 4 + pitch, off)
        yb, Yd = padded_rows(np.zeros((K, L), np.uint8), L + 5, 3, fill=0x5A)
        items.append((dev(g.C), Sd, Yd, yb, K, L))
    plan = gf.gf_plan_encode(n, [(C, S, Y) for C, S, Y, _, _, _ in items], tune={"form": form})
    assert plan.tuning()["form"] == form if form else plan.tuning()["form"] in ((1, 2, 3) if n <= 4 else (1, 2))
    for _, _, Yd, _, _, _ in items:
        Yd.zero_()
    gf.gf_plan_launch(plan)
    torch.cuda.synchronize()
    for (C, S, Yd, yb, K, L), w in zip(items, wants):
        assert (host(Yd) == w).all()
        raw = host(yb)
        mask = np.ones(raw.size, bool)
        for k in range(K):
            mask[3 + k * (L + 5): 3 + k * (L + 5) + L] = False
        assert (raw[mask] == 0x5A).all()


@pytest.mark.parametrize("form", [1, 2])
def test_encode_long_packet(gf, form):
    """Packets longer than 2048 strips of 256 bytes: the bit-matrix kernel's running
    accumulators restart on the way (GF(256), 20 x 9, ragged length)."""
    torch = torch_cuda()
    L = 2048 * 256 + 777
    g = synth.generation(synth.key(16, 8, 1), 8, 9, 20, L)
    want = oracle.encode(8, g.C, g.S)
    Cd, Sd = dev(g.C), dev(g.S)
    Yd = torch.zeros((20, L), dtype=torch.uint8, device="cuda")
    plan = gf.gf_plan_encode(8, [(Cd, Sd, Yd)], tune={"form": form})
    gf.gf_plan_launch(plan)
    torch.cuda.synchronize()
    got = host(Yd)
    bad = np.argwhere(got != want)
    assert bad.size == 0, bad[:5]


def test_encode_single_generation_workload(gf):
    """GF(256), 16 packets of 1500 B, 16 x 16 nonzero coefficients; then decode back."""
    torch = torch_cuda()
    g = synth.single_generation()
    want = oracle.encode(8, g.C, g.S)
    Cd, Sd = dev(g.C), dev(g.S)
    Yd = torch.zeros((16, 1500), dtype=torch.uint8, device="cuda")
    gf.gf_encode(8, Cd, Sd, Yd)
    assert (host(Yd) == want).all()
    r, S_or = oracle.decode(8, g.C, want)
    out = torch.zeros((16, 1500), dtype=torch.uint8, device="cuda")
    rank = torch.zeros(1, dtype=torch.int32, device="cuda")
    gf.gf_decode(8, Cd, Yd, out, d_rank=rank)
    assert int(rank.item()) == r
    if r == 16:
        assert (host(out) == S_or).all() and (host(out) == g.S).all()


# ------------------------------------------------------------------ decode

def _invertible(n, N, seed):
    a = 0
    while True:
        Cm = synth.uniform_field(synth.key(seed, a), N * N, n).reshape(N, N)
        if oracle.rank(n, Cm) == N:
            return Cm
        a += 1


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("N", [1, 2, 3, 7, 16, 33, 64, 100, 128, 200, 256])
def test_invert(gf, n, N):
    torch = torch_cuda()
    print("invert", n, N, flush=True)
    Cm = _invertible(n, N, synth.key(20, n, N))
    Ci = torch.zeros((N, N), dtype=torch.uint8, device="cuda")
    rank = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    gf.gf_invert(n, dev(Cm), Ci, rank)
    torch.cuda.synchronize()
    assert int(rank.item()) == N
    assert (host(Ci) == oracle.invert(n, Cm)).all()


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("N,L", [(1, 10), (5, 1000), (32, 1500), (64, 1500), (128, 1500), (256, 300)])
def test_decode(gf, n, N, L):
    torch = torch_cuda()
    print("decode", n, N, L, flush=True)
    Cm = _invertible(n, N, synth.key(21, n, N))
    S = synth.random_bytes(synth.key(22, n, N), N * L).reshape(N, L)
    B = oracle.encode(n, Cm, S)
    out = torch.zeros((N, L), dtype=torch.uint8, device="cuda")
    rank = torch.zeros(1, dtype=torch.int32, device="cuda")
    gf.gf_decode(n, dev(Cm), dev(B), out, d_rank=rank)
    torch.cuda.synchronize()
    assert int(rank.item()) == N
    assert (host(out) == S).all()


@pytest.mark.parametrize("n", FIELDS)
def test_decode_small_every_N(gf, n):
    """The one-launch decode for N = 1 .. 17 (N <= 16 inverts in one wave's
    registers, 17 in LDS): matrices with a zero leading entry (so a lower pivot
    row is swapped up, and the inverse's columns swapped back) decode to the
    sources; singular ones leave the output untouched and report the oracle's
    rank."""
    torch = torch_cuda()
    for N in range(1, 18):
        L = 4 * (50 + N)   # rows 4-byte aligned: the one-launch path
        S = synth.random_bytes(synth.key(71, n, N), N * L).reshape(N, L)
        cases = []
        if N > 1:
            for t in range(50):   # a zero in the top-left corner, still invertible
                Cm = synth.uniform_field(synth.key(72, n, N, t), N * N, n).reshape(N, N)
                Cm[0, 0] = 0
                if oracle.rank(n, Cm) == N:
                    cases.append(Cm)
                    break
        Cs = synth.uniform_field(synth.key(73, n, N), N * N, n).reshape(N, N)
        if N > 1:
            Cs[N - 1] = Cs[0]
        else:
            Cs[0, 0] = 0
        cases.append(Cs)
        for Cm in cases:
            r = oracle.rank(n, Cm)
            B = oracle.encode(n, Cm, S)
            out = torch.full((N, L), 0x77, dtype=torch.uint8, device="cuda")
            rank = torch.zeros(1, dtype=torch.int32, device="cuda")
            gf.gf_decode(n, dev(Cm), dev(B), out, d_rank=rank)
            torch.cuda.synchronize()
            assert int(rank.item()) == r, (N, r)
            if r == N:
                assert (host(out) == S).all(), N
            else:
                assert (host(out) == 0x77).all(), N


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("N", [2, 9, 64, 130])
def test_decode_singular(gf, n, N):
    torch = torch_cuda()
    Cm = synth.uniform_field(synth.key(23, n, N), N * N, n).reshape(N, N)
    Cm[N - 1] = Cm[0]
    if N > 8:
        Cm[3] = 0
        Cm[5] = Cm[1] ^ Cm[2] if n == 1 else Cm[5]
    want_rank = oracle.rank(n, Cm)
    assert want_rank < N
    L = 100
    out = torch.full((N, L), 0x77, dtype=torch.uint8, device="cuda")
    rank = torch.zeros(1, dtype=torch.int32, device="cuda")
    gf.gf_decode(n, dev(Cm), dev(synth.random_bytes(1, N * L).reshape(N, L)), out, d_rank=rank)
    Ci = torch.full((N, N), 0x33, dtype=torch.uint8, device="cuda")
    rank2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    gf.gf_invert(n, dev(Cm), Ci, rank2)
    torch.cuda.synchronize()
    assert int(rank.item()) == want_rank == int(rank2.item())
    assert (host(out) == 0x77).all() and (host(Ci) == 0x33).all()


# ------------------------------------------------------------------ batched

def _uneven(n, count, seed, maxN=256, maxL=9000):
    torch = torch_cuda()
    items = []
    for i in range(count):
        N = int(synth.uniform_ints(synth.key(seed, 1, i), 1, 1, maxN)[0])
        L = int(synth.log_uniform_ints(synth.key(seed, 2, i), 1, 1, maxL)[0])
        g = synth.generation(synth.key(seed, 3, i), n, N, N, L)
        _, Sd = padded_rows(g.S, synth.padded(L))
        _, Yd = padded_rows(np.zeros((N, L), np.uint8), synth.padded(L))
        items.append((g, dev(g.C), Sd, Yd))
    return items


@pytest.mark.parametrize("n", FIELDS)
def test_batched_encode_and_graph(gf, n):
    torch = torch_cuda()
    items = _uneven(n, 60, synth.key(30, n), maxN=96, maxL=3000)
    wants = [oracle.encode(n, g.C, g.S) for g, _, _, _ in items]
    plan = gf.gf_plan_encode(n, [(C, S, Y) for _, C, S, Y in items])
    gf.gf_plan_launch(plan)
    torch.cuda.synchronize()
    for (g, _, _, Yd), w in zip(items, wants):
        assert (host(Yd) == w).all()
    # graph replays, with eager work and synchronisation in between
    for rep in range(3):
        for _, _, _, Yd in items:
            Yd.fill_(rep + 1)
        torch.cuda.synchronize()
        gf.gf_plan_launch_graph(plan)
        torch.cuda.synchronize()
        for (g, _, _, Yd), w in zip(items, wants):
            assert (host(Yd) == w).all(), rep


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("layout", ["packed", "padded"])
def test_batched_decode(gf, n, layout):
    """Packed rows (any alignment: table-form apply) and 16-byte row pitch
    (the bit-matrix apply that decode plans pick by default)."""
    torch = torch_cuda()
    count = 40
    systems, wants, ranks_or = [], [], []
    for i in range(count):
        N = [1, 17, 32, 33, 64, 65, 128, 129, 200, 256][i % 10]
        L = int(synth.uniform_ints(synth.key(31, n, i), 1, 1, 2000)[0])
        if i % 7 == 3:
            Cm = synth.uniform_field(synth.key(32, n, i), N * N, n).reshape(N, N)
            Cm[N - 1] = 0
        else:
            Cm = _invertible(n, N, synth.key(33, n, i))
        S = synth.random_bytes(synth.key(34, n, i), N * L).reshape(N, L)
        B = oracle.encode(n, Cm, S)
        r = oracle.rank(n, Cm)
        ranks_or.append(r)
        wants.append(S if r == N else None)
        if layout == "packed":
            out = torch.full((N, L), 0x3C, dtype=torch.uint8, device="cuda")
            Bd = dev(B)
        else:
            _, out = padded_rows(np.full((N, L), 0x3C, np.uint8), synth.padded(L))
            _, Bd = padded_rows(B, synth.padded(L))
        systems.append((dev(Cm), Bd, out))
    plan = gf.gf_plan_decode(n, systems)
    assert plan.tuning()["form"] == (2 if layout == "padded" else 1)
    rank = torch.full((count,), -1, dtype=torch.int32, device="cuda")
    for mode in ("eager", "graph", "graph"):
        for _, _, out in systems:
            out.fill_(0x3C)
        torch.cuda.synchronize()
        if mode == "eager":
            gf.gf_plan_launch(plan, rank)
        else:
            gf.gf_plan_launch_graph(plan, rank)
        torch.cuda.synchronize()
        assert host(rank).tolist() == ranks_or
        for (Cd, Bd, out), w in zip(systems, wants):
            if w is None:
                assert (host(out) == 0x3C).all()
            else:
                assert (host(out) == w).all()


# ------------------------------------------------------------------ recoding

def _relay(n, seed, Kout, M, N, L):
    """Inputs of one recoding: R (Kout x M), received headers Cin (M x N) and
    payloads Bin (M x L).  Recoding is linear in Bin, so random bytes serve."""
    R = synth.uniform_field(synth.key(seed, 1), Kout * M, n).reshape(Kout, M)
    Cin = synth.uniform_field(synth.key(seed, 2), M * N, n).reshape(M, N)
    Bin = synth.random_bytes(synth.key(seed, 3), M * L).reshape(M, L)
    return R, Cin, Bin


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("Kout,M,N,L", [(1, 1, 1, 1), (5, 9, 7, 1000), (24, 64, 33, 1501), (40, 256, 256, 4099),
                                       (3, 17, 200, 0), (0, 4, 4, 10)])
def test_recode(gf, n, Kout, M, N, L):
    torch = torch_cuda()
    R, Cin, Bin = _relay(n, synth.key(70, n, Kout, M, N, L), Kout, M, N, L)
    wantC, wantY = oracle.recode(n, R, Cin, Bin)
    Cout = torch.full((Kout, N), 0x5A, dtype=torch.uint8, device="cuda")
    Yout = torch.full((Kout, L), 0x5A, dtype=torch.uint8, device="cuda")
    gf.gf_recode(n, dev(R), dev(Cin), dev(Bin), Cout, Yout)
    torch.cuda.synchronize()
    assert (host(Cout) == wantC).all()
    assert (host(Yout) == wantY).all()


@pytest.mark.parametrize("n", [1, 8])
def test_recoded_packets_decode_on_gpu(gf, n):
    """Encode, recode at a relay, decode at the receiver -- all on the GPU --
    gives back the sources (Sec. I)."""
    torch = torch_cuda()
    N, M, L = 48, 60, 2000
    S = synth.random_bytes(synth.key(71, n), N * L).reshape(N, L)
    Cin = _invertible(n, N, synth.key(72, n))
    Cin = np.concatenate([Cin, synth.uniform_field(synth.key(73, n), (M - N) * N, n).reshape(M - N, N)])
    Bd = torch.empty((M, L), dtype=torch.uint8, device="cuda")
    gf.gf_encode(n, dev(Cin), dev(S), Bd)
    attempt = 0
    while True:   # a relay matrix whose recoded headers have full rank
        R = synth.uniform_field(synth.key(74, n, attempt), N * M, n).reshape(N, M)
        if oracle.rank(n, oracle.matmul(n, R, Cin)) == N:
            break
        attempt += 1
    Cout = torch.empty((N, N), dtype=torch.uint8, device="cuda")
    Yout = torch.empty((N, L), dtype=torch.uint8, device="cuda")
    gf.gf_recode(n, dev(R), dev(Cin), Bd, Cout, Yout)
    out = torch.zeros((N, L), dtype=torch.uint8, device="cuda")
    rank = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    gf.gf_decode(n, Cout, Yout, out, d_rank=rank)
    torch.cuda.synchronize()
    assert int(host(rank)[0]) == N
    assert (host(out) == S).all()


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("form", [0, 1, 2])
def test_batched_recode_and_graph(gf, n, form):
    torch = torch_cuda()
    items, wants = [], []
    for i in range(50):
        M = int(synth.uniform_ints(synth.key(75, n, i), 1, 1, 130)[0])
        N = int(synth.uniform_ints(synth.key(76, n, i), 1, 1, 130)[0])
        Kout = int(synth.uniform_ints(synth.key(77, n, i), 1, 0, 70)[0])
        L = int(synth.log_uniform_ints(synth.key(78, n, i), 1, 1, 3000)[0])
        R, Cin, Bin = _relay(n, synth.key(79, n, i), Kout, M, N, L)
        wants.append(oracle.recode(n, R, Cin, Bin))
        _, Bd = padded_rows(Bin, synth.padded(L))
        _, Yd = padded_rows(np.zeros((Kout, L), np.uint8), synth.padded(L))
        Cd = torch.zeros((Kout, N), dtype=torch.uint8, device="cuda")
        items.append((dev(R), dev(Cin), Bd, Cd, Yd))
    plan = gf.gf_plan_recode(n, items, {"form": form})
    if form:
        assert plan.tuning()["form"] == form
    for mode in ("eager", "graph", "graph"):
        for it in items:
            it[3].fill_(0xC3)
            it[4].fill_(0xC3)
        torch.cuda.synchronize()
        if mode == "eager":
            gf.gf_plan_launch(plan)
        else:
            gf.gf_plan_launch_graph(plan)
        torch.cuda.synchronize()
        for it, (wc, wy) in zip(items, wants):
            assert (host(it[3]) == wc).all(), mode
            assert (host(it[4]) == wy).all(), mode


def _packet_rows(Cm, B, ld, fill=0x77):
    """Device buffer of packets stored as rows [coefficients | payload], `ld` bytes apart.
    Returns (coefficient view, payload view)."""
    torch = torch_cuda()
    rows, N = Cm.shape
    L = B.shape[1]
    buf = torch.full((max(rows, 1) * ld,), fill, dtype=torch.uint8, device="cuda")
    v = buf[:rows * ld].view(rows, ld)
    if rows:
        v[:, :N].copy_(torch.from_numpy(np.ascontiguousarray(Cm)).to("cuda"))
        v[:, N:N + L].copy_(torch.from_numpy(np.ascontiguousarray(B)).to("cuda"))
    return v[:, :N], v[:, N:N + L]


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("Kout,M,N,L,ld", [(5, 9, 7, 1000, 1008), (33, 64, 64, 1500, 1568), (16, 200, 131, 777, 910),
                                          (40, 256, 256, 4099, 4368)])
def test_recode_packet_rows(gf, n, Kout, M, N, L, ld):
    """Packets stored as one row each, coefficients in front of the payload
    (header and payload become one product over N + len bytes)."""
    torch = torch_cuda()
    R, Cin, Bin = _relay(n, synth.key(80, n, Kout, M, N), Kout, M, N, L)
    wantC, wantY = oracle.recode(n, R, Cin, Bin)
    Ci, Bi = _packet_rows(Cin, Bin, ld)
    Co, Yo = _packet_rows(np.zeros((Kout, N), np.uint8), np.zeros((Kout, L), np.uint8), ld, fill=0x11)
    gf.gf_recode(n, dev(R), Ci, Bi, Co, Yo)
    torch.cuda.synchronize()
    assert (host(Co) == wantC).all()
    assert (host(Yo) == wantY).all()
    # the pitch padding after each output packet is left alone
    full = host(Co.as_strided((Kout, ld), (ld, 1)))
    assert (full[:, N + L:] == 0x11).all()


@pytest.mark.parametrize("n", [2, 8])
@pytest.mark.parametrize("form", [0, 2])
def test_batched_recode_mixed_layouts(gf, n, form):
    """A plan over relays of both layouts: packet rows (one fused product) and
    separate header and payload buffers (header launch, then payload launch)."""
    torch = torch_cuda()
    items, wants = [], []
    for i in range(40):
        M = int(synth.uniform_ints(synth.key(81, n, i), 1, 1, 256)[0])
        N = int(synth.uniform_ints(synth.key(82, n, i), 1, 1, 256)[0])
        Kout = int(synth.uniform_ints(synth.key(83, n, i), 1, 0, 80)[0])
        L = int(synth.log_uniform_ints(synth.key(84, n, i), 1, 64, 9000)[0])
        R, Cin, Bin = _relay(n, synth.key(85, n, i), Kout, M, N, L)
        wants.append(oracle.recode(n, R, Cin, Bin))
        if i % 2 == 0:
            ld = synth.padded(N + L)
            Ci, Bi = _packet_rows(Cin, Bin, ld)
            Co, Yo = _packet_rows(np.zeros((Kout, N), np.uint8), np.zeros((Kout, L), np.uint8), ld)
        else:
            Ci = dev(Cin)
            _, Bi = padded_rows(Bin, synth.padded(L))
            Co = torch.zeros((Kout, N), dtype=torch.uint8, device="cuda")
            _, Yo = padded_rows(np.zeros((Kout, L), np.uint8), synth.padded(L))
        items.append((dev(R), Ci, Bi, Co, Yo))
    plan = gf.gf_plan_recode(n, items, {"form": form})
    for mode in ("eager", "graph", "graph"):
        for it in items:
            it[3].fill_(0xE7)
            it[4].fill_(0xE7)
        torch.cuda.synchronize()
        if mode == "eager":
            gf.gf_plan_launch(plan)
        else:
            gf.gf_plan_launch_graph(plan)
        torch.cuda.synchronize()
        for i, (it, (wc, wy)) in enumerate(zip(items, wants)):
            assert (host(it[3]) == wc).all(), (mode, i)
            assert (host(it[4]) == wy).all(), (mode, i)


# ------------------------------------------------------------------ binding checks

def test_binding_rejects_host_and_short_buffers(gf):
    """Arguments that would hand a kernel a host pointer, or a rank or output
    buffer shorter than the call writes, raise in the binding before any launch."""
    torch = torch_cuda()
    print("binding checks", flush=True)
    N = 8
    Cm = dev(_invertible(8, N, synth.key(2024)))
    Cinv_host = torch.empty((N, N), dtype=torch.uint8)
    with pytest.raises(TypeError):
        gf.gf_invert(8, Cm, Cinv_host)
    with pytest.raises(TypeError):   # rank must be int32 on the device
        gf.gf_invert(8, Cm, torch.empty((N, N), dtype=torch.uint8, device="cuda"),
                     d_rank=torch.zeros(1, dtype=torch.int64, device="cuda"))
    B = dev(synth.random_bytes(synth.key(2025), N * 64).reshape(N, 64))
    S = torch.empty((N, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(TypeError):   # workspace on the host
        gf.gf_decode(8, Cm, B, S, ws=torch.empty(gf.gf_decode_workspace(8, N), dtype=torch.uint8))
    plan = gf.gf_plan_decode(8, [(Cm, B, S), (Cm, B, torch.empty_like(S))])
    with pytest.raises(ValueError):  # one rank slot for two systems
        gf.gf_plan_launch(plan, d_rank=torch.zeros(1, dtype=torch.int32, device="cuda"))
    rank = torch.zeros(2, dtype=torch.int32, device="cuda")
    gf.gf_plan_launch(plan, d_rank=rank)
    torch.cuda.synchronize()
    assert host(rank).tolist() == [N, N]
    plan.destroy()

    srv = gf.Server(field=8, budget_bytes=1 << 24)
    with pytest.raises(TypeError):   # encode inputs on the host
        srv.submit_encode(1, torch.zeros((4, N), dtype=torch.uint8), S, 4, N, 64, 64, 0.0)
    Ce = synth.uniform_field(synth.key(2026), 4 * N, 8).reshape(4, N)
    srv.submit_encode(1, dev(Ce), S, 4, N, 64, 64, 0.0)
    srv.step(0.0)
    srv.drain(0.0)
    (d,) = srv.poll()
    with pytest.raises(ValueError):  # three rows for a four-row output
        srv.copy_out(1, torch.empty((3, 64), dtype=torch.uint8, device="cuda"))
    out = torch.empty((4, 64), dtype=torch.uint8, device="cuda")
    srv.copy_out(1, out)
    torch.cuda.synchronize()
    assert (host(out) == oracle.encode(8, Ce, host(S))).all()
    srv.release(1)
    srv.close()


@pytest.mark.parametrize("n", FIELDS)
@pytest.mark.parametrize("smax", [1, 2, 3, 8])
@pytest.mark.parametrize("aligned", [True, False])
@pytest.mark.parametrize("form", [4, 5])
def test_stream_form_small_generations(gf, n, smax, aligned, form):
    """Forms 4 and 5 (small generations streamed in bursts of strips, from work
    queues or one burst per wave; the kernel instance follows the batch's
    largest K or N): every byte equals the oracle's, on generations of one to
    many 1 KiB strips, tiles of 64 strips, runs split evenly and ragged ends
    (whose last 16-byte block is read whole and written only up to the row's
    end); padding untouched.  Rows that are not 16-byte aligned are refused by
    both, and the autotuned plan over them (another form) matches as well."""
    torch = torch_cuda()
    items, wants = [], []
    for i in range(40):
        N = int(synth.uniform_ints(synth.key(17, smax, i), 1, 1, smax)[0])
        K = int(synth.uniform_ints(synth.key(18, smax, i), 1, 1, smax)[0])
        L = [1, 15, 1023, 1024, 1025, 3000, 9000, 65536, 70001, 2049][i % 10]
        g = synth.generation(synth.key(19, n, smax, i), n, N, K, L)
        wants.append(oracle.encode(n, g.C, g.S))
        ld = synth.padded(L) if aligned else L + 3
        _, Sd = padded_rows(g.S, ld, 0 if aligned else 1)
        yb, Yd = padded_rows(np.zeros((K, L), np.uint8), ld, fill=0x5A)
        items.append((dev(g.C), Sd, Yd, yb, K, L, ld))
    gens = [(C, S, Y) for C, S, Y, _, _, _, _ in items]
    if aligned:
        plan = gf.gf_plan_encode(n, gens, tune={"form": form})
        assert plan.tuning()["form"] == form
    else:
        with pytest.raises(gf.GFError):      # forms 4 and 5 read whole 16-byte blocks
            gf.gf_plan_encode(n, gens, tune={"form": form})
        plan = gf.gf_plan_encode(n, gens)
        assert plan.tuning()["form"] not in (4, 5)
    for rep in range(2):
        for _, _, Yd, _, _, _, _ in items:
            Yd.fill_(0x5A)
        if rep == 0:
            gf.gf_plan_launch(plan)
        else:
            gf.gf_plan_launch_graph(plan)
        torch.cuda.synchronize()
        for (C, S, Yd, yb, K, L, ld), w in zip(items, wants):
            assert (host(Yd) == w).all(), (K, L)
            raw = host(yb)[:K * ld].reshape(K, ld)
            assert (raw[:, L:] == 0x5A).all()
    plan.destroy()
    big = [(dev(np.ones((9, 2), np.uint8)), dev(np.ones((2, 8), np.uint8)), dev(np.zeros((9, 8), np.uint8)))]
    with pytest.raises(gf.GFError):      # K = 9: not a small generation
        gf.gf_plan_encode(n, big, tune={"form": form})
