"""Write the oracle's per-generation output digests for the full-size workloads.

Calls only ``oracle`` (the plain CPU reference) and ``synth`` (the seeded
inputs); nothing here touches the GPU library.  Each output is Eq. (1) of the
paper (Sec. II) for every coded packet of every generation: the uneven batches
over GF(256) and GF(16), the plain sweep over every field at 1500 and 9000 B
(every generation) and at 64 KiB (one generation from each block of 64), and
the relays' recoding (Sec. I; header R * Cin and payload R * Bin of each
output packet row).  For the decode batch it stores which coefficient draw of
each system the oracle finds invertible, and the oracle's rank of every draw
it rejects.

Usage: python tests/golden/make_digests.py [workload ...] [--threads T]
(no workload: all of them; several hours of CPU on 8 cores).
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)

import digests  # noqa: E402
import oracle  # noqa: E402
import synth  # noqa: E402

FIELD_NAME = {1: "gf2", 2: "gf4", 4: "gf16", 8: "gf256"}
SAMPLE_BLOCK = 64          # 64 KiB sweep: one generation from each block of 64


def sample_indices(count: int, n: int) -> list:
    """One generation per block of SAMPLE_BLOCK, at a seeded position inside it."""
    pos = synth.uniform_ints(synth.key(90, n), count // SAMPLE_BLOCK, 0, SAMPLE_BLOCK - 1)
    return [SAMPLE_BLOCK * b + int(p) for b, p in enumerate(pos)]


def _batch_digests(b: synth.Batch, threads: int) -> list:
    S_blob, C_blob = b.source_blob(), b.coef_blob()
    Y = np.zeros(b.y_bytes, np.uint8)
    desc = np.stack([b.c_off, b.s_off, b.y_off, b.lds, b.lds, b.Ls, b.Ks, b.Ns], axis=1)
    oracle.encode_batch(b.n, desc, C_blob, S_blob, Y, threads)
    out = []
    for i in range(len(b.Ns)):
        K, L, ld = int(b.Ks[i]), int(b.Ls[i]), int(b.lds[i])
        out.append((i, digests.digest_rows(Y[b.y_off[i]:b.y_off[i] + K * ld].reshape(K, ld)[:, :L])))
    return out


def _sample_digests(b: synth.Batch, idx: list, threads: int) -> list:
    """Only the listed generations, each drawn from its place in the streams."""
    Cs = [b.coef_rows(i) for i in idx]
    Ss = [b.source_rows(i) for i in idx]
    L = int(b.Ls[0])
    K, N = int(b.Ks[0]), int(b.Ns[0])
    C_blob = np.ascontiguousarray(np.concatenate([c.reshape(-1) for c in Cs]))
    S_blob = np.ascontiguousarray(np.concatenate([s.reshape(-1) for s in Ss]))
    Y = np.zeros(len(idx) * K * L, np.uint8)
    desc = np.array([[j * K * N, j * N * L, j * K * L, L, L, L, K, N] for j in range(len(idx))], np.int64)
    oracle.encode_batch(b.n, desc, C_blob, S_blob, Y, threads)
    return [(i, digests.digest_rows(Y[j * K * L:(j + 1) * K * L].reshape(K, L))) for j, i in enumerate(idx)]


_RELAY = {}


def _relay_one(i: int):
    rl = _RELAY["rl"]
    In, Rb = _RELAY["in"], _RELAY["R"]
    b = rl.batch
    N, L, ld, off = int(b.Ns[i]), int(b.Ls[i]), int(rl.lds[i]), int(rl.offs[i])
    rows = In[off:off + N * ld].reshape(N, ld)
    R = Rb[b.c_off[i]:b.c_off[i] + N * N].reshape(N, N)
    Cout, Yout = oracle.recode(8, R, np.ascontiguousarray(rows[:, :N]), np.ascontiguousarray(rows[:, N:N + L]))
    return i, digests.digest_rows(np.concatenate([Cout, Yout], axis=1))


def relay_digests(count: int, threads: int) -> list:
    rl = synth.relay_batch(count)
    _RELAY.update(rl=rl, **{"in": rl.in_blob(), "R": rl.R_blob()})
    order = np.argsort(-(rl.batch.Ns.astype(np.int64) ** 2 * (rl.batch.Ns + rl.batch.Ls)))
    with mp.get_context("fork").Pool(threads) as pool:
        out = pool.map(_relay_one, [int(i) for i in order], chunksize=4)
    return sorted(out)


def decode_draws(count: int = 2048) -> list:
    """Per system: the index of the first coefficient draw the oracle finds
    invertible, then 'attempt:rank' of each draw before it."""
    db = synth.decode_batch(count, 1500)
    out = []
    for i in range(count):
        N = int(db.Ns[i])
        rejected = []
        attempt = 0
        while True:
            r = oracle.rank(8, synth.decode_candidate(i, attempt, N))
            if r == N:
                break
            rejected.append("%d:%d" % (attempt, r))
            attempt += 1
        out.append((i, attempt, rejected))
    return out


def workloads() -> dict:
    w = {"uneven_gf256": None, "uneven_gf16": None, "relay_gf256": None, "decode_2048": None}
    for L in (1500, 9000):
        for n in (8, 4, 2, 1):
            w["sweep_%s_%d" % (FIELD_NAME[n], L)] = None
    for n in (8, 4, 2, 1):
        w["sweep_%s_65536_sample" % FIELD_NAME[n]] = None
    return w


def make(name: str, threads: int) -> None:
    cmd = "python tests/golden/make_digests.py %s" % name
    t0 = time.time()
    if name.startswith("uneven_"):
        n = 8 if name.endswith("gf256") else 4
        b = synth.uneven_batch(n, 10000)
        items = _batch_digests(b, threads)
        header = ["uneven batch over %s: 10,000 generations, N ~ U{8..256}, L log-uniform in [64, 9000] B, "
                  "K = N (synth.uneven_batch(%d, 10000))" % (name[7:].upper(), n)]
    elif name.startswith("sweep_") and name.endswith("_sample"):
        n = {v: k for k, v in FIELD_NAME.items()}[name.split("_")[1]]
        b = synth.sweep_batch(n, 65536)
        items = _sample_digests(b, sample_indices(4096, n), threads)
        header = ["plain sweep over %s at 65536 B, N = K = 64: generation 64 b + p of each block b of 64 "
                  "(p seeded), synth.sweep_batch(%d, 65536)" % (name.split("_")[1].upper(), n)]
    elif name.startswith("sweep_"):
        _, f, L = name.split("_")
        n = {v: k for k, v in FIELD_NAME.items()}[f]
        b = synth.sweep_batch(n, int(L))
        items = _batch_digests(b, threads)
        header = ["plain sweep over %s at %s B, N = K = 64, 4096 generations (synth.sweep_batch(%d, %s))"
                  % (f.upper(), L, n, L)]
    elif name == "relay_gf256":
        items = relay_digests(10000, threads)
        header = ["recoding at 10,000 relays over GF(256) (synth.relay_batch(10000)): digest of each relay's "
                  "N output packet rows, [R * Cin | R * Bin], N + L bytes each"]
    elif name == "decode_2048":
        rows = decode_draws()
        with open(digests.path(name), "w") as fo:
            fo.write("# decode batch, 2,048 systems over GF(256), N in {32, 64, 128} (synth.decode_batch): per\n")
            fo.write("# system the first draw (synth.decode_candidate) the oracle finds invertible, then\n")
            fo.write("# 'attempt:rank' of each earlier draw it rejects.  Written by: %s\n" % cmd)
            fo.write("# index attempt rejected...\n")
            for i, a, rej in rows:
                fo.write("%d %d %s\n" % (i, a, " ".join(rej)))
        print(name, "%.0f s" % (time.time() - t0), flush=True)
        return
    else:
        raise SystemExit("unknown workload " + name)
    header = ["SHA-256 (first 16 hex digits) of each generation's output rows, row after row, useful bytes only,",
              "computed by the oracle (Eq. (1), Sec. II) on the seeded inputs of the"] + header + [
              "written by: " + cmd, "index digest"]
    digests.write(name, header, items)
    print(name, len(items), "generations, %.0f s" % (time.time() - t0), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--threads", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    a = ap.parse_args()
    for name in a.names or list(workloads()):
        make(name, a.threads)


if __name__ == "__main__":
    main()
