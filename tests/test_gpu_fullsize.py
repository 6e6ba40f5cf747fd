"""The workloads at their full sizes, in the launch configuration bench.py
times (autotuned plan, one graph-replayed persistent launch), checked against
the oracle on sampled outputs (each sampled byte is Eq. (1) over the
generation's whole column) or, for decoding, by the output equalling the
sources everywhere.

Workloads: the uneven batch (10,000 generations, N ~ U{8..256}, packets
log-uniform in [64, 9000] B, K = N) over GF(16) and GF(256); the plain sweep
(4096 generations, N = K = 64, 1500 / 9000 / 65536 B) over all four fields;
the batched decode (2,048 systems, N in {32, 64, 128}, 1500 B) over GF(256);
recoding at 10,000 relays; the 4000-request serving stream.
"""
import numpy as np
import pytest

import bench
import oracle
import synth
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gf():
    torch_cuda()
    import paper_1909_02871_amd as g
    g.gf_init()
    return g


def _sample_cols(rng, L, extra=3):
    return sorted({0, L - 1, *(int(x) for x in rng.integers(0, L, extra))})


def _sample_rows(rng, K):
    return sorted({0, K - 1, int(rng.integers(0, K))})


@pytest.mark.parametrize("n", [8, 4])
def test_uneven_batch_full_size(gf, n):
    torch = torch_cuda()
    count = 10000
    b = synth.uneven_batch(n, count)
    S_host, C_host = b.source_blob(), b.coef_blob()
    S_dev = torch.from_numpy(S_host).to("cuda")
    C_dev = torch.from_numpy(C_host).to("cuda")
    Y_dev = torch.full((b.y_bytes,), 0xA5, dtype=torch.uint8, device="cuda")
    descs = (gf.gf_gen * count)()
    s0, c0, y0 = S_dev.data_ptr(), C_dev.data_ptr(), Y_dev.data_ptr()
    for i in range(count):
        descs[i] = gf.gf_gen(c0 + int(b.c_off[i]), s0 + int(b.s_off[i]), y0 + int(b.y_off[i]), int(b.Ks[i]),
                             int(b.Ns[i]), int(b.Ls[i]), int(b.lds[i]), int(b.lds[i]))
    plan = gf.gf_plan_encode_desc(n, descs, count, tune={"form": 0}, keep=(S_dev, C_dev, Y_dev))
    Y_dev.fill_(0xA5)
    torch.cuda.synchronize()
    for _ in range(2):
        gf.gf_plan_launch_graph(plan)
    torch.cuda.synchronize()
    Y_host = Y_dev.cpu().numpy()
    rng = np.random.default_rng(synth.key(60, n))
    for g in sorted({0, count - 1, *(int(x) for x in rng.integers(0, count, 46))}):
        Cm, S = b.generation(g, S_host, C_host)
        K, L, ld = int(b.Ks[g]), int(b.Ls[g]), int(b.lds[g])
        rows, cols = _sample_rows(rng, K), _sample_cols(rng, L)
        want = oracle.encode(n, Cm[rows], np.ascontiguousarray(S[:, cols]))
        Y = Y_host[b.y_off[g]:b.y_off[g] + K * ld].reshape(K, ld)
        assert (Y[np.ix_(rows, cols)] == want).all(), (g, rows, cols)
    plan.destroy()


@pytest.mark.parametrize("n", [1, 2, 4, 8])
@pytest.mark.parametrize("L", [1500, 9000, 65536])
def test_sweep_full_size(gf, n, L):
    torch = torch_cuda()
    count, N = 4096, 64
    plan, S, Cm, Y, ld = bench.uniform_plan(gf, torch, n, N, N, L, count, synth.BASE_SEED + 1 + 100 * n + L)
    Y.fill_(0xA5)
    torch.cuda.synchronize()
    gf.gf_plan_launch_graph(plan)
    torch.cuda.synchronize()
    S3 = S.view(count, N, ld)
    C3 = Cm.view(count, N, N)
    Y3 = Y.view(count, N, ld)
    rng = np.random.default_rng(synth.key(61, n, L))
    for g in sorted({0, count - 1, *(int(x) for x in rng.integers(0, count, 14))}):
        rows, cols = _sample_rows(rng, N), _sample_cols(rng, L)
        cidx = torch.tensor(cols, device="cuda")
        Sg = S3[g].index_select(1, cidx).cpu().numpy()
        want = oracle.encode(n, C3[g].cpu().numpy()[rows], Sg)
        got = Y3[g].index_select(1, cidx).cpu().numpy()[rows]
        assert (got == want).all(), (g, rows, cols)
    plan.destroy()
    del plan, S, Cm, Y
    torch.cuda.empty_cache()


def test_decode_batch_full_size(gf):
    """2,048 systems; singular draws are redrawn (as the bench does, by the
    device's own rank); every decoded byte equals its source."""
    torch = torch_cuda()
    db = synth.decode_batch(2048, 1500)
    count = len(db.Ns)
    S_dev = torch.from_numpy(db.source_blob()).to("cuda")
    B_dev = torch.empty_like(S_dev)
    R_dev = torch.empty_like(S_dev)
    attempt = np.zeros(count, dtype=np.int64)
    C_host = np.zeros(db.c_bytes, dtype=np.uint8)

    def fill(i):
        Nn = int(db.Ns[i])
        C_host[db.c_off[i]:db.c_off[i] + Nn * Nn] = synth.decode_candidate(i, int(attempt[i]), Nn).reshape(-1)

    for i in range(count):
        fill(i)
    rank = torch.zeros(count, dtype=torch.int32, device="cuda")
    for _ in range(8):
        C_dev = torch.from_numpy(C_host).to("cuda")
        sysd = (gf.gf_sys * count)()
        encd = (gf.gf_gen * count)()
        for i in range(count):
            Nn, L, ld = int(db.Ns[i]), int(db.Ls[i]), int(db.lds[i])
            cp = C_dev.data_ptr() + int(db.c_off[i])
            sp, bp, rp = (t.data_ptr() + int(db.s_off[i]) for t in (S_dev, B_dev, R_dev))
            encd[i] = gf.gf_gen(cp, sp, bp, Nn, Nn, L, ld, ld)
            sysd[i] = gf.gf_sys(cp, bp, rp, Nn, 0, L, ld, ld)
        eplan = gf.gf_plan_encode_desc(8, encd, count, keep=(C_dev, S_dev, B_dev))
        gf.gf_encode_batched(eplan)
        dplan = gf.gf_plan_decode_desc(8, sysd, count, keep=(C_dev, B_dev, R_dev))
        R_dev.fill_(0x3C)
        torch.cuda.synchronize()
        gf.gf_plan_launch_graph(dplan, rank)
        torch.cuda.synchronize()
        ranks = rank.cpu().numpy()
        bad = np.nonzero(ranks != db.Ns)[0]
        if len(bad) == 0:
            break
        for i in bad:
            attempt[i] += 1
            fill(int(i))
        eplan.destroy()
        dplan.destroy()
    else:
        pytest.fail("singular systems left after 8 redraws")
    # the coded rows are the oracle's encode of the sources (sampled), and the decode returns the sources
    rng = np.random.default_rng(synth.key(62))
    S_host = S_dev.cpu().numpy()
    B_host = B_dev.cpu().numpy()
    for i in sorted({0, count - 1, *(int(x) for x in rng.integers(0, count, 10))}):
        Nn, L, ld, so = int(db.Ns[i]), int(db.Ls[i]), int(db.lds[i]), int(db.s_off[i])
        Cm = C_host[db.c_off[i]:db.c_off[i] + Nn * Nn].reshape(Nn, Nn)
        S = S_host[so:so + Nn * ld].reshape(Nn, ld)[:, :L]
        want = oracle.encode(8, Cm, np.ascontiguousarray(S))
        assert (B_host[so:so + Nn * ld].reshape(Nn, ld)[:, :L] == want).all(), i
    valid = torch.zeros_like(S_dev, dtype=torch.bool)
    for i in range(count):
        Nn, L, ld, so = int(db.Ns[i]), int(db.Ls[i]), int(db.lds[i]), int(db.s_off[i])
        valid[so:so + Nn * ld].view(Nn, ld)[:, :L] = True
    assert torch.equal(R_dev[valid], S_dev[valid])
    eplan.destroy()
    dplan.destroy()


def test_recode_relay_full_size(gf):
    """10,000 relays (the uneven GF(256) shapes, M = N received packets stored as rows
    [coefficients | payload], Kout = N): sampled header and payload bytes of the
    recoded packets against the oracle's recode; the row padding stays untouched."""
    torch = torch_cuda()
    rb = bench.relay_batch(gf, torch, 10000, keep_host=True)
    b, Ns, Ls, lds, offs = rb["batch"], rb["Ns"], rb["Ls"], rb["lds"], rb["offs"]
    rb["Out"].fill_(0xA5)
    torch.cuda.synchronize()
    gf.gf_plan_launch_graph(rb["plan"])
    torch.cuda.synchronize()
    Out = rb["Out"].cpu().numpy()
    In, Rh = rb["In_host"], rb["R_host"]
    rng = np.random.default_rng(synth.key(63))
    for g in sorted({0, 9999, *(int(x) for x in rng.integers(0, 10000, 30))}):
        N, L, ld, off = int(Ns[g]), int(Ls[g]), int(lds[g]), int(offs[g])
        rows_in = In[off:off + N * ld].reshape(N, ld)
        R = Rh[b.c_off[g]:b.c_off[g] + N * N].reshape(N, N)
        rows, hcols, pcols = _sample_rows(rng, N), _sample_cols(rng, N), _sample_cols(rng, L)
        wantC, wantY = oracle.recode(8, R[rows], np.ascontiguousarray(rows_in[:, hcols]),
                                     np.ascontiguousarray(rows_in[:, [N + c for c in pcols]]))
        got = Out[off:off + N * ld].reshape(N, ld)[rows]
        assert (got[:, hcols] == wantC).all(), g
        assert (got[:, [N + c for c in pcols]] == wantY).all(), g
        assert (got[:, N + L:] == 0xA5).all(), g
    rb["plan"].destroy()


def test_serving_full_size(gf):
    """The serving workload (4000 requests, 70% encode / 30% decode, GF(256), 10%
    loss, random order) all arriving at once through a 4 GiB arena: every encode's
    sampled bytes are the oracle's and every decode returns its sources exactly."""
    from paper_1909_02871_amd.serving import replay
    torch = torch_cuda()
    st = bench.serving_trace(gf, torch, 4000)
    where, S_host, C_host, S_dev = st["where"], st["S_host"], st["C_host"], st["S_dev"]
    rng = np.random.default_rng(synth.key(64))
    srv = gf.Server(field=8, budget_bytes=4 << 30)
    bad = []

    def check(d):
        w = where[d["id"]]
        N, L, ld, so = w["N"], w["length"], w["ld"], w["s_off"]
        out = torch.empty((N, L), dtype=torch.uint8, device="cuda")
        srv.copy_out(d["id"], out)
        torch.cuda.synchronize()
        if w["kind"] == "decode":
            if d["rank"] != N or not torch.equal(out, S_dev[so:so + N * ld].view(N, ld)[:, :L]):
                bad.append(d["id"])
            return
        rows, cols = _sample_rows(rng, N), _sample_cols(rng, L)
        Cm = C_host[w["c_off"]:w["c_off"] + N * N].reshape(N, N)
        S = S_host[so:so + N * ld].reshape(N, ld)
        want = oracle.encode(8, Cm[rows], np.ascontiguousarray(S[:, cols]))
        got = out.cpu().numpy()[np.ix_(rows, cols)]
        if not (got == want).all():
            bad.append(d["id"])

    done = replay(srv, st["trace"], on_done=check, timeout_s=300)
    srv.close()
    assert len(done) == 4000
    assert not bad, bad[:10]


@pytest.mark.parametrize("n,form", [(8, 1), (8, 2), (4, 3), (8, "single")])
def test_generation_past_2_gib(gf, n, form):
    """One generation whose sources span more than 2^31 bytes (16 rows of 128 MiB +
    12,345 B): the kernels' 64-bit offset paths, checked on sampled columns near the
    start, across the 2^31 boundary of the row offsets and at the ragged end."""
    torch = torch_cuda()
    N, K, L = 16, 4, (1 << 27) + 12345
    ld = L + 3          # odd pitch: rows are not word aligned past the first
    if form in (2,):
        ld = (L + 15) // 16 * 16   # the bit-matrix form's DMA path needs word-aligned rows
    S = bench.device_bytes(torch, N * ld, synth.key(65, n))
    Cm = bench.device_bytes(torch, K * N, synth.key(66, n), 1 << n).view(K, N)
    Y = torch.full((K * ld,), 0xA5, dtype=torch.uint8, device="cuda")
    S2, Y2 = S.view(N, ld)[:, :L], Y.view(K, ld)[:, :L]
    if form == "single":
        gf.gf_encode(n, Cm, S2, Y2)
    else:
        plan = gf.gf_plan_encode(n, [(Cm, S2, Y2)], tune={"form": form})
        assert plan.tuning()["form"] == form
        gf.gf_plan_launch_graph(plan)
    torch.cuda.synchronize()
    rng = np.random.default_rng(synth.key(67, n))
    cols = sorted({0, 1, 255, 256, L - 1, L - 2, L - 300, (1 << 27) - 1, 1 << 27,
                   *(int(x) for x in rng.integers(0, L, 8))})
    cidx = torch.tensor(cols, device="cuda")
    want = oracle.encode(n, Cm.cpu().numpy(), S2.index_select(1, cidx).cpu().numpy())
    got = Y2.index_select(1, cidx).cpu().numpy()
    assert (got == want).all(), cols
    if form != "single":
        plan.destroy()
