"""The decode that allocates nothing (gf_decode_noalloc: the inverse goes to the
library's fixed per-device scratch array) against gf_decode with a caller
workspace, byte for byte, through the C ABI, on calls in a row whose sizes
shrink (the scratch keeps the previous call's bytes), and against the sources
(Gauss-Jordan decoding recovers them; Sec. I, Sec. II Eq. (1)).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev, host, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gf():
    torch_cuda()
    import paper_1909_02871_amd as g
    g.gf_init()
    return g


def _invertible(n, N, seed):
    for attempt in range(64):
        Cm = synth.uniform_field(synth.key(seed, attempt), N * N, n).reshape(N, N)
        if oracle.rank(n, Cm) == N:
            return Cm
    raise AssertionError("no invertible draw")


def _both(gf, torch, n, Cm, B, L, d_rank):
    N = Cm.shape[0]
    Cd, Bd = dev(Cm), dev(B)
    out_ws = torch.full((N, L), 0x5A, dtype=torch.uint8, device="cuda")
    out_na = torch.full((N, L), 0xA5, dtype=torch.uint8, device="cuda")
    r_ws = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    r_na = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    gf.gf_decode(n, Cd, Bd, out_ws, d_rank=r_ws)
    gf.gf_decode_noalloc(n, Cd, Bd, out_na, d_rank=r_na if d_rank else None)
    torch.cuda.synchronize()
    return out_ws, out_na, int(r_ws.item()), (int(r_na.item()) if d_rank else None)


@pytest.mark.parametrize("n", [8, 4, 1])
def test_noalloc_decode_equals_workspace_decode(gf, n):
    """Calls in a row, each smaller than the one before: N = 200 (the inverse
    fills most of the scratch), then 40, then one generation small enough for
    the one-launch path, then a rank kept in the scratch (d_rank NULL)."""
    torch = torch_cuda()
    for N, L, with_rank in [(200, 3001, True), (40, 777, True), (16, 1500, True), (12, 333, False)]:
        print("noalloc decode", n, N, L, with_rank, flush=True)
        Cm = _invertible(n, N, synth.key(80, n, N))
        S = synth.random_bytes(synth.key(81, n, N), N * L).reshape(N, L)
        B = oracle.encode(n, Cm, S)
        out_ws, out_na, r_ws, r_na = _both(gf, torch, n, Cm, B, L, with_rank)
        assert r_ws == N
        if with_rank:
            assert r_na == N
        assert torch.equal(out_na, out_ws), (n, N, L)
        assert (host(out_na) == S).all(), (n, N, L)


@pytest.mark.parametrize("n", [8, 2])
def test_noalloc_decode_singular_leaves_output(gf, n):
    """A singular matrix after an invertible one: the rank is the oracle's and
    the output keeps its bytes, as with gf_decode."""
    torch = torch_cuda()
    N, L = 90, 500
    Cm = _invertible(n, N, synth.key(82, n))
    S = synth.random_bytes(synth.key(83, n), N * L).reshape(N, L)
    _, out_na, _, r_na = _both(gf, torch, n, Cm, oracle.encode(n, Cm, S), L, True)
    assert r_na == N and (host(out_na) == S).all()
    Cs = Cm.copy()
    Cs[N - 1] = Cs[0]
    Cs[7] = 0
    want = oracle.rank(n, Cs)
    assert want < N
    out_ws, out_na, r_ws, r_na = _both(gf, torch, n, Cs, S[:N], L, True)
    assert r_ws == r_na == want
    assert (host(out_na) == 0xA5).all() and (host(out_ws) == 0x5A).all()


def test_noalloc_decode_rejects_sizes_past_the_scratch(gf):
    torch = torch_cuda()
    N = 257
    Cd = torch.zeros((N, N), dtype=torch.uint8, device="cuda")
    Bd = torch.zeros((N, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(gf.GFError) as e:
        gf.gf_decode_noalloc(8, Cd, Bd, torch.zeros_like(Bd))
    assert e.value.code == gf.GF_ERANGE
