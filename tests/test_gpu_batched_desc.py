"""The batched calls that read their descriptors from device memory at launch
(gf_encode_batched with a plan of shapes; gf_decode_batched with a workspace
and no plan), through the C ABI, against the oracle byte for byte (encode:
Sec. II, Eq. (1); decode: Gauss-Jordan, the sources themselves).

One plan serves two different device descriptor arrays (new buffers, the
same shapes); a descriptor whose shape differs from the plan's is skipped and
counted; both calls replay from a captured HIP graph with eager work between
the replays."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, padded_rows, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gf():
    torch_cuda()
    import paper_1909_02871_amd as g
    g.gf_init()
    return g


def _shapes(n, count, seed):
    out = []
    for i in range(count):
        N = [1, 7, 8, 16, 33, 64, 100, 255, 256, 40][i % 10]
        K = [1, 16, 5, 17, 33, 64, 2, 100, 256, 48][i % 10]
        L = int(synth.uniform_ints(synth.key(seed, i), 1, 1, 3000)[0])
        out.append((K, N, L))
    return out


def _buffers(gf, torch, n, shapes, seed):
    """One set of device buffers (rows padded to 16 bytes, the output filled
    with 0x5A), its device descriptor array, and the oracle's outputs."""
    keep, descs, wants = [], (gf.gf_gen * len(shapes))(), []
    for i, (K, N, L) in enumerate(shapes):
        g = synth.generation(synth.key(seed, n, i), n, N, K, L)
        wants.append(oracle.encode(n, g.C, g.S))
        ld = synth.padded(L)
        Cd = dev(g.C)
        _, Sd = padded_rows(g.S, ld)
        yb, Yd = padded_rows(np.zeros((K, L), np.uint8), ld, fill=0x5A)
        Yd.fill_(0x5A)
        keep.append((Cd, Sd, Yd, yb))
        descs[i] = gf.gf_gen(Cd.data_ptr(), Sd.data_ptr(), Yd.data_ptr(), K, N, L, ld, ld)
    return keep, gf.make_gens(descs), wants


def _check(keep, wants):
    for (Cd, Sd, Yd, yb), w in zip(keep, wants):
        assert (host(Yd) == w).all()
        K, L = w.shape
        ld = synth.padded(L)
        raw = host(yb)[:K * ld].reshape(K, ld)
        assert (raw[:, L:] == 0x5A).all()


@pytest.mark.parametrize("n", [8, 4, 1])
@pytest.mark.parametrize("form", [0, 1, 2])
def test_one_plan_two_descriptor_arrays(gf, n, form):
    torch = torch_cuda()
    shapes = _shapes(n, 30, 40 + n)
    ld = [synth.padded(L) for _, _, L in shapes]
    plan_descs = (gf.gf_gen * len(shapes))(*[gf.gf_gen(None, None, None, K, N, L, l, l)
                                              for (K, N, L), l in zip(shapes, ld)])
    plan = gf.gf_plan_encode_desc(n, plan_descs, len(shapes), tune={"form": form})
    assert plan.tuning()["form"] == form if form else plan.tuning()["form"] in ((1, 2, 3) if n <= 4 else (1, 2))
    with pytest.raises(gf.GFError):          # a plan of shapes has no buffers of its own to run on
        gf.gf_plan_launch(plan)
    for seed in (41, 42):
        keep, d_gens, wants = _buffers(gf, torch, n, shapes, seed)
        torch.cuda.synchronize()
        gf.gf_encode_batched(n, d_gens, len(shapes), plan)
        torch.cuda.synchronize()
        _check(keep, wants)
        assert plan.errors() == 0
    with pytest.raises(gf.GFError):          # field and count must be the plan's
        gf.gf_encode_batched(4 if n != 4 else 8, d_gens, len(shapes), plan)
    with pytest.raises(gf.GFError):
        gf.gf_encode_batched(n, d_gens, len(shapes) - 1, plan)
    plan.destroy()


def test_plan_with_pointers_runs_other_descriptors_and_skips_mismatches(gf):
    torch = torch_cuda()
    n = 8
    shapes = _shapes(n, 20, 50)
    keep0, d0, wants0 = _buffers(gf, torch, n, shapes, 51)
    plan = gf.gf_plan_encode(n, [(C, S, Y) for C, S, Y, _ in keep0], tune={"form": 0})
    keep1, d1, wants1 = _buffers(gf, torch, n, shapes, 52)
    for _, _, Y, _ in keep0:
        Y.fill_(0x5A)
    torch.cuda.synchronize()
    gf.gf_encode_batched(n, d1, len(shapes), plan)     # the other buffers: the plan's own stay as they were
    gf.gf_encode_batched(n, None, len(shapes), plan)   # then the plan's own descriptors
    torch.cuda.synchronize()
    _check(keep1, wants1)
    _check(keep0, wants0)
    # a descriptor array whose generation 3 has another K: that one is skipped and counted
    bad = (gf.gf_gen * len(shapes)).from_buffer_copy(bytes(host(d1)))
    bad[3].K = bad[3].K + 1
    d_bad = gf.make_gens(bad)
    for _, _, Y, _ in keep1:
        Y.fill_(0x5A)
    torch.cuda.synchronize()
    gf.gf_encode_batched(n, d_bad, len(shapes), plan)
    torch.cuda.synchronize()
    assert plan.errors() == 1 and plan.errors() == 0
    for i, ((C, S, Y, yb), w) in enumerate(zip(keep1, wants1)):
        if i == 3:
            assert (host(Y) == 0x5A).all()
        else:
            assert (host(Y) == w).all()
    plan.destroy()


@pytest.mark.parametrize("n", [8, 1])
@pytest.mark.parametrize("form", [4, 5])
def test_streaming_forms_over_descriptors(gf, n, form):
    """The two small-generation streaming forms (K, N <= 8) on a plan of shapes: two
    descriptor arrays give the oracle's bytes, and a descriptor whose K differs from
    the plan's is skipped (its output untouched) and counted."""
    torch = torch_cuda()
    shapes = []
    for i in range(24):
        K = [1, 8, 3, 5, 2, 7, 4, 6][i % 8]
        N = [8, 1, 5, 2, 7, 3, 6, 4][i % 8]
        L = [1, 15, 16, 1023, 1025, 9000, 8192, 20000][(3 * i) % 8]
        shapes.append((K, N, L))
    ld = [synth.padded(L) for _, _, L in shapes]
    plan_descs = (gf.gf_gen * len(shapes))(*[gf.gf_gen(None, None, None, K, N, L, l, l)
                                              for (K, N, L), l in zip(shapes, ld)])
    plan = gf.gf_plan_encode_desc(n, plan_descs, len(shapes), tune={"form": form})
    assert plan.tuning()["form"] == form
    for seed in (71, 72):
        keep, d_gens, wants = _buffers(gf, torch, n, shapes, seed)
        torch.cuda.synchronize()
        gf.gf_encode_batched(n, d_gens, len(shapes), plan)
        torch.cuda.synchronize()
        _check(keep, wants)
        assert plan.errors() == 0
    bad = (gf.gf_gen * len(shapes)).from_buffer_copy(bytes(host(d_gens)))
    bad[5].K = bad[5].K - 1
    for _, _, Y, _ in keep:
        Y.fill_(0x5A)
    torch.cuda.synchronize()
    gf.gf_encode_batched(n, gf.make_gens(bad), len(shapes), plan)
    torch.cuda.synchronize()
    assert plan.errors() == 1
    for i, ((C, S, Y, yb), w) in enumerate(zip(keep, wants)):
        if i == 5:
            assert (host(Y) == 0x5A).all()
        else:
            assert (host(Y) == w).all(), i
    plan.destroy()


def test_encode_batched_in_a_captured_graph(gf):
    """gf_encode_batched allocates nothing, so it can be captured; replays with
    other work between them give the oracle's bytes every time."""
    torch = torch_cuda()
    n = 8
    shapes = _shapes(n, 12, 60)
    keep, d_gens, wants = _buffers(gf, torch, n, shapes, 61)
    ld = [synth.padded(L) for _, _, L in shapes]
    plan = gf.gf_plan_encode_desc(n, (gf.gf_gen * len(shapes))(
        *[gf.gf_gen(None, None, None, K, N, L, l, l) for (K, N, L), l in zip(shapes, ld)]), len(shapes))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gf.gf_encode_batched(n, d_gens, len(shapes), plan, stream=s)    # warm-up outside the graph
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gf.gf_encode_batched(n, d_gens, len(shapes), plan, stream=s)
    junk = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    for rep in range(3):
        for _, _, Y, _ in keep:
            Y.fill_(0x5A)
        junk.add_(1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check(keep, wants)
    plan.destroy()


def _invertible(n, N, seed):
    for attempt in range(64):
        Cm = synth.uniform_field(synth.key(seed, attempt), N * N, n).reshape(N, N)
        if oracle.rank(n, Cm) == N:
            return Cm
    raise AssertionError("no invertible draw")


def _systems(gf, torch, n, seed, count=36):
    """Systems of every size class, 16-byte and odd row pitches, a singular one
    every 7th, and the oracle's rank and sources."""
    items, descs = [], (gf.gf_sys * count)()
    for i in range(count):
        N = [1, 5, 32, 33, 64, 65, 100, 128, 129, 200, 256, 17][i % 12]
        L = int(synth.uniform_ints(synth.key(seed, 1, i), 1, 1, 1600)[0])
        if i % 7 == 3:
            Cm = synth.uniform_field(synth.key(seed, 2, i), N * N, n).reshape(N, N)
            Cm[N - 1] = 0
        else:
            Cm = _invertible(n, N, synth.key(seed, 3, i))
        S = synth.random_bytes(synth.key(seed, 4, i), N * L).reshape(N, L)
        B = oracle.encode(n, Cm, S)
        r = oracle.rank(n, Cm)
        ld = synth.padded(L) if i % 2 == 0 else L + 3
        _, Bd = padded_rows(B, ld, 0 if i % 2 == 0 else 1)
        ob, out = padded_rows(np.full((N, L), 0x3C, np.uint8), ld)
        Cd = dev(Cm)
        items.append((Cd, Bd, out, ob, r, S))
        descs[i] = gf.gf_sys(Cd.data_ptr(), Bd.data_ptr(), out.data_ptr(), N, 0, L, ld, ld)
    return items, gf.make_systems(descs)


@pytest.mark.parametrize("n", [8, 4, 1])
def test_decode_batched_two_descriptor_arrays(gf, n):
    torch = torch_cuda()
    count = 36
    ws = torch.empty(gf.gf_decode_workspace(n, 256, count), dtype=torch.uint8, device="cuda")
    for seed in (70, 71):
        items, d_sys = _systems(gf, torch, n, synth.key(seed, n), count)
        rank = torch.full((count,), -5, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        gf.gf_decode_batched(n, d_sys, count, rank, ws)
        torch.cuda.synchronize()
        assert host(rank).tolist() == [it[4] for it in items]
        for Cd, Bd, out, ob, r, S in items:
            N = S.shape[0]
            if r == N:
                assert (host(out) == S).all()
            else:
                assert (host(out) == 0x3C).all()


def test_decode_batched_rejects_what_the_workspace_cannot_hold(gf):
    """A workspace sized for N <= 64: a system of N = 100 gets rank -1 and no
    output, the others decode; a system with N = 0 likewise; ranks kept in the
    workspace when no rank array is given."""
    torch = torch_cuda()
    n, count = 8, 4
    shapes = [(20, 300), (100, 200), (64, 1000), (0, 10)]
    items, descs = [], (gf.gf_sys * count)()
    for i, (N, L) in enumerate(shapes):
        Nm = max(N, 1)
        Cm = _invertible(n, Nm, synth.key(75, i))
        S = synth.random_bytes(synth.key(76, i), Nm * L).reshape(Nm, L)
        Bd = dev(oracle.encode(n, Cm, S))
        out = torch.full((Nm, L), 0x3C, dtype=torch.uint8, device="cuda")
        Cd = dev(Cm)
        items.append((Cd, Bd, out, S))
        descs[i] = gf.gf_sys(Cd.data_ptr(), Bd.data_ptr(), out.data_ptr(), N, 0, L, L, L)
    d_sys = gf.make_systems(descs)
    ws = torch.empty(gf.gf_decode_workspace(n, 64, count), dtype=torch.uint8, device="cuda")
    rank = torch.full((count,), -5, dtype=torch.int32, device="cuda")
    gf.gf_decode_batched(n, d_sys, count, rank, ws)
    gf.gf_decode_batched(n, d_sys, count, None, ws)      # ranks inside the workspace
    torch.cuda.synchronize()
    assert host(rank).tolist() == [20, -1, 64, -1]
    for i, (Cd, Bd, out, S) in enumerate(items):
        assert (host(out) == S).all() if i in (0, 2) else (host(out) == 0x3C).all()


def test_decode_batched_in_a_captured_graph(gf):
    torch = torch_cuda()
    n, count = 8, 24
    items, d_sys = _systems(gf, torch, n, synth.key(77), count)
    ws = torch.empty(gf.gf_decode_workspace(n, 256, count), dtype=torch.uint8, device="cuda")
    rank = torch.full((count,), -5, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gf.gf_decode_batched(n, d_sys, count, rank, ws, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gf.gf_decode_batched(n, d_sys, count, rank, ws, stream=s)
    for rep in range(3):
        for _, _, out, _, _, _ in items:
            out.fill_(0x3C)
        rank.fill_(-5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert host(rank).tolist() == [it[4] for it in items]
        for Cd, Bd, out, ob, r, S in items:
            assert (host(out) == S).all() if r == S.shape[0] else (host(out) == 0x3C).all()


def test_autotuner_trials_leave_outputs_and_repeat_through_the_cache(gf):
    """Creating an autotuned plan runs its trials on scratch memory (the
    caller's outputs keep their bytes), the choice is written to the tuning
    cache, and a second plan of the same batch takes the same schedule."""
    import json
    import os
    torch = torch_cuda()
    n = 8
    shapes = _shapes(n, 24, 90)
    keep, d_gens, wants = _buffers(gf, torch, n, shapes, 91)
    items = [(C, S, Y) for C, S, Y, _ in keep]
    torch.cuda.synchronize()
    p1 = gf.gf_plan_encode(n, items, tune={"form": 0})
    torch.cuda.synchronize()
    for _, _, Y, _ in keep:
        assert (host(Y) == 0x5A).all()          # the trials wrote elsewhere
    p2 = gf.gf_plan_encode(n, items, tune={"form": 0})
    assert p1.tuning() == p2.tuning()
    path = os.environ.get("GFNC_TUNE_CACHE") or os.path.join(os.path.dirname(gf.LIB_PATH), "gfnc_tune.json")
    entries = json.load(open(path))["entries"]
    assert any(e["key"].split("|")[1] == "f8" and e["form"] == p1.tuning()["form"] for e in entries)
    for p in (p1, p2):
        for _, _, Y, _ in keep:
            Y.fill_(0x5A)
        torch.cuda.synchronize()
        gf.gf_plan_launch(p)
        torch.cuda.synchronize()
        _check(keep, wants)
    p1.destroy()
    p2.destroy()


@pytest.mark.parametrize("what", [0, 4])
@pytest.mark.parametrize("nbytes", [64, 32 * 1000 + 48, 1 << 22])
def test_ceiling_copies(gf, what, nbytes):
    """The two copy microbenchmarks that the roofline report times (grid-stride and one
    workgroup per 16 KiB) move the first bytes // 32 words of 16 bytes to just after them,
    whole and in place, ragged counts of words included; the tail is untouched."""
    torch = torch_cuda()
    src = synth.random_bytes(synth.key(90, what, nbytes), nbytes)
    buf = dev(src)
    gf.gf_ceiling(what, buf, 3, 0)
    torch.cuda.synchronize()
    half = nbytes // 32 * 16
    got = host(buf)
    assert (got[half:2 * half] == src[:half]).all()
    assert (got[:half] == src[:half]).all() and (got[2 * half:] == src[2 * half:]).all()
    with pytest.raises(gf.GFError):
        gf.gf_ceiling(5, buf, 3, 0)
