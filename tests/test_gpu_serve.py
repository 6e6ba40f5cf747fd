"""Serving on the GPU: encode and progressive-decode requests give the same
bytes alone and in a continuously batched mix, and those bytes are the
oracle's (encode: Sec. II, Eq. 1; decode: the source generation itself).

Decode requests receive coded packets with uniform coefficient vectors, in a
random order, 10% lost, plus one repeated packet that must be recognised as
not innovative; packets are released over time, so the echelon state lives on
the device across several steps."""
import math
import time

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


class Workload:
    def __init__(self, n, count, seed, maxN=48, maxL=1200):
        from paper_1909_02871_amd.serving import TraceRequest
        torch = torch_cuda()
        self.keep, self.reqs, self.want = [], [], {}
        for i in range(count):
            N = int(synth.uniform_ints(synth.key(seed, 1, i), 1, 2, maxN)[0])
            L = int(synth.log_uniform_ints(synth.key(seed, 2, i), 1, 16, maxL)[0])
            kind = "decode" if i % 3 == 1 else "encode"
            if kind == "encode":
                g = synth.generation(synth.key(seed, 3, i), n, N, N, L)
                Cd, Sd = dev(g.C), dev(g.S)
                self.keep += [Cd, Sd]
                self.want[i] = oracle.encode(n, g.C, g.S)
                self.reqs.append(TraceRequest(i, 0.0, "encode", N, L, C=Cd.data_ptr(), S=Sd.data_ptr(), K=N,
                                              ld_s=L))
            else:
                S = synth.random_bytes(synth.key(seed, 4, i), N * L).reshape(N, L)
                P = int(math.ceil(1.5 * N)) + 4
                coef = synth.uniform_field(synth.key(seed, 5, i), P * N, n).reshape(P, N)
                lost = synth.unit_floats(synth.key(seed, 6, i), P) < 0.1
                order = np.argsort(synth.words(synth.key(seed, 7, i), P))
                delivered = [j for j in order if not lost[j]]
                # rateless sender: emit more packets until the receiver can decode
                extra = 0
                while oracle.rank(n, coef[delivered]) < N:
                    more = synth.uniform_field(synth.key(seed, 8, i, extra), N, n).reshape(1, N)
                    coef = np.vstack([coef, more])
                    delivered.append(coef.shape[0] - 1)
                    extra += 1
                B = oracle.encode(n, coef, S)
                Cd, Bd = dev(coef), dev(B)
                self.keep += [Cd, Bd]
                pk = []
                for t, j in enumerate(delivered):
                    pk.append((Cd[j].data_ptr(), Bd[j].data_ptr(), 2e-4 * t))
                # a repeat of the first delivered packet: never innovative
                j0 = delivered[0]
                pk.insert(min(3, len(pk)), (Cd[j0].data_ptr(), Bd[j0].data_ptr(), 2e-4 * min(3, len(pk))))
                self.want[i] = S
                self.reqs.append(TraceRequest(i, 0.0, "decode", N, L, packets=pk))
        torch.cuda.synchronize()


def _run(gf, n, reqs, budget, burst, max_slots=0):
    torch = torch_cuda()
    from paper_1909_02871_amd.serving import replay
    srv = gf.Server(field=n, budget_bytes=budget, burst=burst, max_slots=max_slots)
    outs = {}

    def on_done(d):
        rows = d["rank"]
        r = next(x for x in reqs if x.rid == d["id"])
        t = torch.zeros((rows, r.length), dtype=torch.uint8, device="cuda")
        srv.copy_out(d["id"], t)
        outs[d["id"]] = (host(t), d)

    done = replay(srv, reqs, on_done=on_done, timeout_s=120)
    st = srv.stats()
    srv.close()
    assert len(done) == len(reqs)
    return outs, st


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_alone_equals_mix_equals_oracle(gf, n):
    from paper_1909_02871_amd.serving import TraceRequest
    w = Workload(n, 18, synth.key(70, n))
    # each request alone
    alone = {}
    for r in w.reqs:
        o, _ = _run(gf, n, [r], budget=64 << 20, burst=8)
        alone[r.rid] = o[r.rid][0]
        assert (alone[r.rid] == w.want[r.rid]).all(), (r.rid, r.kind)
    # all of them, arriving over ~5 ms, through a small arena and few slots
    arrivals = np.cumsum(-np.log1p(-synth.unit_floats(synth.key(71, n), len(w.reqs))) * 3e-4)
    mix = [TraceRequest(r.rid, float(a), r.kind, r.N, r.length, r.C, r.S, r.K, r.ld_s, r.packets)
           for r, a in zip(w.reqs, arrivals)]
    outs, st = _run(gf, n, mix, budget=1 << 20, burst=5, max_slots=6)
    assert st["arena_peak"] <= 1 << 20
    for r in w.reqs:
        got, d = outs[r.rid]
        assert (got == alone[r.rid]).all(), r.rid
        assert (got == w.want[r.rid]).all(), r.rid
        if r.kind == "decode":
            assert d["rank"] == r.N
            assert d["packets_dropped"] >= 1 or d["packets_seen"] < len(r.packets)


def test_copy_out_then_release_keeps_the_bytes_until_the_copy_ran(gf):
    """copy_out on a busy side stream, release at once, then a new request that
    would take the same arena memory: the copy still reads the first request's
    bytes (the memory is reused only after the copy has run)."""
    torch = torch_cuda()
    N, L = 32, 4000
    gA = synth.generation(synth.key(95, 1), 8, N, N, L)
    gB = synth.generation(synth.key(95, 2), 8, N, N, L)
    want = oracle.encode(8, gA.C, gA.S)
    keep = [dev(gA.C), dev(gA.S), dev(gB.C), dev(gB.S)]
    ld = (L + 15) // 16 * 16
    srv = gf.Server(field=8, budget_bytes=N * ld + 256)      # room for one request only
    srv.submit_encode(1, keep[0], keep[1], N, N, L, L, 0.0)
    t = 0.0
    done = []
    while not done:
        t += 0.001
        srv.step(t)
        done = srv.poll()
    side = torch.cuda.Stream()
    dst = torch.full((N, L), 0x11, dtype=torch.uint8, device="cuda")
    a = torch.randn((4096, 4096), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for _ in range(40):                # keeps the side stream busy before the copy (tens of ms)
            a = torch.tanh(a @ a)
    srv.copy_out(1, dst, stream=side)
    srv.release(1)
    srv.submit_encode(2, keep[2], keep[3], N, N, L, L, t)
    out2 = None
    t_end = time.perf_counter() + 20.0
    while time.perf_counter() < t_end:
        t += 0.001
        srv.step(t)
        got = srv.poll()
        if got:
            out2 = got[0]
            break
    assert out2 is not None and out2["id"] == 2
    side.synchronize()
    torch.cuda.synchronize()
    assert (host(dst) == want).all()
    o2 = torch.empty((N, L), dtype=torch.uint8, device="cuda")
    srv.copy_out(2, o2)
    torch.cuda.synchronize()
    assert (host(o2) == oracle.encode(8, gB.C, gB.S)).all()
    srv.release(2)
    srv.close()
