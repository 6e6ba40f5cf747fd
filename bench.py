#!/usr/bin/env python3
"""Throughput benchmark of the batched GF(256) encode on one MI355X.

Workload: 10,000 uneven generations over GF(256) (x^8+x^4+x^3+x^2+1): N
uniform in {8..256} source packets, packet length log-uniform in [64, 9000]
bytes, K = N coded packets per generation (the coefficient-matrix product of
the paper's Sec. II, Eq. 1, for K coding vectors), uniform random payload and
coefficients from the seeded generators.  All inputs are resident in HBM
before timing starts.

One step = one launch of the whole batch (a single persistent kernel replayed
from a HIP graph).  The same work as one launch per generation ("plain") is
timed beside it.  `value` is GB/s of source payload, sum(N * L) / step time.

Also reported: the roofline of the encode kernel (measured with HIP events
on the launch stream), the fraction of the HBM roofline, and the CPU oracle
timed on a bounded sample of the same generations (whose outputs are checked
byte for byte against the GPU's).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "GF(256) encode GB/s (batched vs plain, 1 GPU, bit-exact); serve p50/p99 ms"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock at 2.4 GHz = 39.3 T 32-bit lane-ops/s.
VALU_LANE_OPS = 256 * 64 * 2.4e9
# The table form spends 3 byte-selects + 1.5 three-input XORs per dword of 4 byte-madds.
TABLE_OPS_PER_MADD = 4.5 / 4.0
HBM_PEAK_GBS = 8000.0
MFMA_FP4_TFLOPS = 10100.0

# Sources each persistent encode kernel is built from: its counters below stay valid while they are unchanged.
KERNEL_SOURCES = {2: ("gf_mfma.hip", "gf_queue.h", "gf_types.h"),
                  1: ("gf_kernels.hip", "gf_queue.h", "gf_types.h", "gf_internal.h"),
                  3: ("gf_kernels.hip", "gf_queue.h", "gf_types.h", "gf_internal.h")}

# HBM bytes per launch of the batched encode kernel of each form, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB, averages over the profiled launches), scaled by what the same counters read for a
# 1 GiB device copy (fetch x 2.000, write x 1.000); keyed by the sha256 of the kernel's sources, so a
# changed kernel reports null until it is measured again.
MEASURED_TRAFFIC = {
    ("0595e90e7ffdd4b1850a77f56b39c8190ea78b594436014ba6ebcbee44393cc0", 2): 1481220 * 1024 * 2.0 + 2512510 * 1024,
}


def kernel_source_hash(form: int) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES.get(form, ()):
        with open(os.path.join(ROOT, "paper_1909_02871_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


ALG1_SRC = os.path.join(ROOT, "bench_alg1.c")
ALG1_LIB = os.path.join(ROOT, "libbench_alg1.so")


def alg1_build() -> str:
    """Compile the host AVX-512BW region madd (Sec. IV-A) used as CPU context."""
    import subprocess
    tmp = ALG1_LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Werror", "-shared", "-fPIC", "-o", tmp, ALG1_SRC])
    os.replace(tmp, ALG1_LIB)
    return ALG1_LIB


def alg1_lib():
    import ctypes as C
    if not os.path.exists(ALG1_LIB) or os.path.getmtime(ALG1_LIB) < os.path.getmtime(ALG1_SRC):
        alg1_build()
    L = C.CDLL(ALG1_LIB)
    L.alg1_supported.restype = C.c_int
    L.alg1_region_madd.restype = C.c_int
    L.alg1_region_madd.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_size_t]
    L.alg1_encode_seconds.restype = C.c_double
    L.alg1_encode_seconds.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p,
                                      C.c_size_t, C.c_size_t, C.c_int]
    return L


def host_alg1_sweep() -> dict:
    """One host core running the paper's split-nibble shuffle madd (AVX-512BW): encode of one
    generation, N = K = 16, over packet lengths from 128 B to 64 KiB (the shape of the paper's
    single-core measurements), per field.  Context for the GPU figures, not a target."""
    L = alg1_lib()
    if not L.alg1_supported():
        return {"supported": False}
    out = {"supported": True, "cores": 1, "N": 16, "K": 16, "points": []}
    for n in (2, 4, 8):
        for P in (128, 512, 1500, 8192, 65536):
            g = synth.generation(synth.key(synth.BASE_SEED + 9, n, P), n, 16, 16, P)
            S = np.ascontiguousarray(g.S)
            Cm = np.ascontiguousarray(g.C)
            Y = np.zeros((16, P), np.uint8)
            reps = 21 if P <= 8192 else 7
            t = L.alg1_encode_seconds(n, Cm.ctypes.data, 16, 16, S.ctypes.data, P, Y.ctypes.data, P, P, reps)
            out["points"].append({"field": "GF(2^%d)" % n, "packet_bytes": P, "encode_us": round(t * 1e6, 3),
                                  "gbs": round(16 * P / t / 1e9, 3),
                                  "coded_gbit_s": round(16 * P * 8 / t / 1e9, 2)})
    return out


def make_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--count", type=int, default=10000, help="generations in the batch")
    ap.add_argument("--field", type=int, default=8)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=30.0, help="target CPU-oracle sample time (estimate)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--bytes-per-lane", type=int, default=0)
    ap.add_argument("--form", type=int, default=0, help="0 autotune, 1 table, 2 bit-matrix MFMA")
    ap.add_argument("--serve-requests", type=int, default=20000, help="requests per serving run (0: skip)")
    ap.add_argument("--serve-budget-gib", type=float, default=4.0)
    ap.add_argument("--serve-burst", type=int, default=0,
                    help="packets a decode request absorbs per step (0: the library default)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (single generation, field/length sweep, GF(16) batch, "
                         "batched decode, K sweep)")
    ap.add_argument("--only", default=None,
                    choices=[name for name, _ in EXTRA_PARTS] + ["serve"],
                    help="run just this one of the other workloads (or the serving runs), print its JSON "
                         "and exit (for profiling one workload's kernels)")
    ap.add_argument("--sweep-fields", default="1,2,4,8",
                    help="word widths n of the field/length sweep (comma-separated; for profiling one point)")
    ap.add_argument("--sweep-lengths", default="1500,9000,65536",
                    help="packet lengths of the field/length sweep (comma-separated)")
    ap.add_argument("--k-list", default="1,2,4,8,16,32,64,128,256",
                    help="K = N values of the K sweep (comma-separated)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (to calibrate HBM counters) and exit")
    return ap


def main():
    args = make_parser().parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the generations are independent, so several GPUs would each "
              "run their own share with no communication; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1909_02871_amd as gf

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nb}))
        return
    gf.gf_init()
    if args.only:
        res = serve_bench(gf, torch, args) if args.only == "serve" else extra_workloads(gf, torch, args, args.only)
        print(json.dumps({"only": args.only, "result": res}), flush=True)
        return
    n = args.field

    # ------------------------------------------------------------ inputs
    t0 = time.time()
    b = synth.uneven_batch(n, args.count)
    S_host = b.source_blob()
    C_host = b.coef_blob()
    log("generated %.2f GB of payload in %.1f s" % (b.s_bytes / 1e9, time.time() - t0))
    S_dev = torch.from_numpy(S_host).to("cuda")
    C_dev = torch.from_numpy(C_host).to("cuda")
    Y_dev = torch.empty(b.y_bytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    import ctypes
    descs = (gf.gf_gen * args.count)()
    s0, c0, y0 = S_dev.data_ptr(), C_dev.data_ptr(), Y_dev.data_ptr()
    for i in range(args.count):
        descs[i] = gf.gf_gen(c0 + int(b.c_off[i]), s0 + int(b.s_off[i]), y0 + int(b.y_off[i]), int(b.Ks[i]),
                             int(b.Ns[i]), int(b.Ls[i]), int(b.lds[i]), int(b.lds[i]))
    tune = {"form": args.form}
    if args.bytes_per_lane:
        tune["bytes_per_lane"] = args.bytes_per_lane
    t0 = time.time()
    plan = gf.gf_plan_encode_desc(n, descs, args.count, tune=tune, keep=(S_dev, C_dev, Y_dev))
    tuning = plan.tuning()
    log("plan built in %.2f s: %s" % (time.time() - t0, tuning))
    stream = torch.cuda.current_stream()

    # each kernel form on its own, graph-replayed (the autotuned plan keeps the faster)
    forms = {}
    for f in (1, 2):
        pf = gf.gf_plan_encode_desc(n, descs, args.count, tune={"form": f}, keep=(S_dev, C_dev, Y_dev))
        for _ in range(2):
            gf.gf_plan_launch_graph(pf)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            gf.gf_plan_launch_graph(pf)
        e1.record(stream)
        torch.cuda.synchronize()
        fms = e0.elapsed_time(e1) / 5
        forms["table" if f == 1 else "bitmatrix_mfma"] = {"ms": round(fms, 4),
                                                          "gbs": round(b.source_bytes / (fms * 1e-3) / 1e9, 3)}
        pf.destroy()
    log("forms: %s" % forms)

    launch = (lambda: gf.gf_plan_launch(plan)) if args.no_graph else (lambda: gf.gf_plan_launch_graph(plan))

    # ------------------------------------------------------------ batched
    for _ in range(args.warmup):
        launch()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_all0.record(stream)
    for i in range(args.steps):
        starts[i].record(stream)
        launch()
        ends[i].record(stream)
    t_all1.record(stream)
    torch.cuda.synchronize()
    total_ms = t_all0.elapsed_time(t_all1)
    per_launch = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_step = total_ms / args.steps
    kern_ms = float(np.mean(per_launch))
    value = b.source_bytes / (ms_step * 1e-3) / 1e9
    log("batched: %.3f ms/step, %.1f GB/s of source" % (ms_step, value))

    # ------------------------------------------------------------ plain
    plain = None
    if args.plain_steps > 0:
        gf.gf_encode_each(n, descs, args.count, tune=tune)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.plain_steps):
            gf.gf_encode_each(n, descs, args.count, tune=tune)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / args.plain_steps
        plain = {"value": round(b.source_bytes / (pms * 1e-3) / 1e9, 3), "ms_per_step": round(pms, 4),
                 "launches_per_step": int((b.Ks > 0).sum())}
        log("plain: %.3f ms/step, %.1f GB/s" % (pms, plain["value"]))
        # the plain pass rewrote Y; run the batched plan once more so the check below sees its output
        launch()
        torch.cuda.synchronize()

    # ------------------------------------------------------------ roofline
    madds = b.byte_madds
    hbm_bytes = b.source_bytes + int((b.Ks * b.Ls).sum()) + int((b.Ks * b.Ns).sum())
    hbm_roof_src = HBM_PEAK_GBS * b.source_bytes / hbm_bytes
    traffic = MEASURED_TRAFFIC.get((kernel_source_hash(tuning["form"]), tuning["form"])) if n == 8 and args.count == 10000 \
        else None
    kernel = {1: "k_encode_waves", 2: "k_encode_mfma_dma", 3: "k_encode_planes"}[tuning["form"]]
    # the HBM roofline: algorithmic bytes of one launch (sources, coefficients and coded rows, each
    # moved once) over the kernel's measured time, against the 8 TB/s peak
    achieved = hbm_bytes / (kern_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None if traffic is None else int(traffic),
                "kernel": kernel, "kernel_ms": round(kern_ms, 4), "algorithmic_bytes": hbm_bytes,
                "byte_madds_per_s": round(madds / (kern_ms * 1e-3), 1)}
    # what actually bounds it: the kernel's own compute roofline
    if tuning["form"] == 2:
        # the bit-matrix product: 8K x 8N x L bit multiply-adds = 64 per byte-madd, 2 flops each,
        # against the dense FP4 matrix-core peak; at 100% of it this batch would run at
        # 78.9 T byte-madd/s / (byte-weighted mean K) of source
        tflops = 128.0 * madds / (kern_ms * 1e-3) / 1e12
        cap_src = MFMA_FP4_TFLOPS * 1e12 / 128.0 * b.source_bytes / madds / 1e9
        roofline["compute"] = {"bound": "mfma", "achieved": round(tflops, 2), "peak": MFMA_FP4_TFLOPS,
                               "unit": "TFLOP/s", "frac": round(tflops / MFMA_FP4_TFLOPS, 4),
                               "source_gbs_at_peak": round(cap_src, 1),
                               "hbm_frac_at_peak": round(cap_src / hbm_roof_src, 4)}
    else:
        peak = VALU_LANE_OPS / TABLE_OPS_PER_MADD / 1e12
        got = madds / (kern_ms * 1e-3) / 1e12
        roofline["compute"] = {"bound": "alu", "achieved": round(got, 3), "peak": round(peak, 3),
                               "unit": "T byte-madd/s", "frac": round(got / peak, 4)}
    ceil = measure_ceilings(gf, torch)
    ceil["torch_copy_gbs"] = round(stream_copy_gbs(torch), 1)
    roofline["measured_ceilings"] = ceil
    roofline["frac_of_measured_copy"] = round(achieved / max(ceil["copy_gbs"], ceil["copy_chunks_gbs"]), 4)
    if tuning["form"] == 2:
        roofline["compute"]["frac_of_measured_fp4"] = round(roofline["compute"]["achieved"] / ceil["fp4_mfma_tflops"], 4)
    log("roofline: %.1f GB/s of algorithmic HBM bytes = %.3f of 8 TB/s; measured ceilings %s"
        % (achieved, achieved / HBM_PEAK_GBS, ceil))

    # ------------------------------------------------------------ CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cpu = cpu_oracle_baseline(oracle, b, S_host, C_host, Y_dev.cpu().numpy(), args)
        cpu["single_generation"] = single_generation_oracle(gf, torch, oracle)

    del S_dev, C_dev, Y_dev, plan
    torch.cuda.empty_cache()
    extra = None
    if not args.no_extra:
        extra = extra_workloads(gf, torch, args)

    serve = None
    if args.serve_requests > 0:
        serve = serve_bench(gf, torch, args)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "uneven_encode_gf256", "field": "GF(2^%d)" % n, "generations": args.count,
                   "N": "U{8..256}", "K": "N", "packet_bytes": "log-U[64, 9000]",
                   "source_bytes": b.source_bytes, "byte_madds": madds, "launch": "hip graph, 1 persistent kernel"
                   if not args.no_graph else "1 persistent kernel"},
        "plain": plain,
        "speedup_vs_plain": round(value / plain["value"], 3) if plain else None,
        "hbm_roofline_gbs": round(hbm_roof_src, 1), "hbm_roofline_frac": round(value / hbm_roof_src, 4),
        "roofline": roofline, "forms": forms, "cpu_baseline": cpu, "tuning": tuning, "serve": serve,
        "other_workloads": extra,
    }
    print(json.dumps(out), flush=True)


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_ms(torch, fn, reps=5, warm=2) -> float:
    """Mean milliseconds of fn() on torch's current stream (after warm-up calls)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def device_bytes(torch, nbytes: int, seed: int, hi: int = 256):
    """Seeded uniform bytes in [0, hi) (hi a power of two), drawn on the device from the
    seeded stream ``synth.random_bytes(seed, nbytes)`` (large inputs stay off the host)."""
    t = synth.device_random_bytes(torch, seed, nbytes)
    if hi < 256:
        t &= hi - 1
    return t


def uniform_plan(gf, torch, b, tune=None):
    """The generations of a same-shape batch (``synth.uniform_batch`` / ``synth.sweep_batch``
    layout) back to back on the device, inputs drawn there from the batch's seeded streams;
    returns an autotuned plan, the source, coefficient and output blobs and the row pitch."""
    S, Cm = b.device_blobs(torch)
    Y = torch.empty(b.y_bytes, dtype=torch.uint8, device="cuda")
    count = len(b.Ns)
    K, N, L, ld = int(b.Ks[0]), int(b.Ns[0]), int(b.Ls[0]), int(b.lds[0])
    descs = (gf.gf_gen * count)()
    s0, c0, y0 = S.data_ptr(), Cm.data_ptr(), Y.data_ptr()
    for i in range(count):
        descs[i] = gf.gf_gen(c0 + int(b.c_off[i]), s0 + int(b.s_off[i]), y0 + int(b.y_off[i]), K, N, L, ld, ld)
    plan = gf.gf_plan_encode_desc(b.n, descs, count, tune=tune if tune is not None else {"form": 0},
                                  keep=(S, Cm, Y))
    return plan, S, Cm, Y, ld


def relay_batch(gf, torch, count: int, keep_host: bool = False) -> dict:
    """The relay workload: the uneven GF(256) shapes, each relay holding M = N received packets and
    sending Kout = N recoded ones, packets stored as rows [N coefficients | payload] at a 16-byte
    pitch; returns the recode plan (autotuned), the device buffers and the layout."""
    rl = synth.relay_batch(count)
    b, lds, offs = rl.batch, rl.lds, rl.offs
    Ns, Ls = b.Ns.astype(np.int64), b.Ls.astype(np.int64)
    In_host = rl.in_blob()
    R_host = rl.R_blob()
    In_dev = torch.from_numpy(In_host).to("cuda")
    Out_dev = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")
    R_dev = torch.from_numpy(R_host).to("cuda")
    descs = (gf.gf_recode_desc * count)()
    i0, o0, r0 = In_dev.data_ptr(), Out_dev.data_ptr(), R_dev.data_ptr()
    for i in range(count):
        N, L, ld, off = int(Ns[i]), int(Ls[i]), int(lds[i]), int(offs[i])
        descs[i] = gf.gf_recode_desc(r0 + int(b.c_off[i]), i0 + off, i0 + off + N, o0 + off, o0 + off + N,
                                     N, N, N, 0, L, ld, ld, ld, ld)
    plan = gf.gf_plan_recode_desc(8, descs, count, keep=(In_dev, Out_dev, R_dev))
    out = {"batch": b, "Ns": Ns, "Ls": Ls, "lds": lds, "offs": offs, "plan": plan, "In": In_dev, "Out": Out_dev,
           "R": R_dev}
    if keep_host:
        out.update(In_host=In_host, R_host=R_host)
    return out


def extra_workloads(gf, torch, args, only=None) -> dict:
    """The other measured workloads: one generation (latency), the plain field/length sweep,
    the uneven batch over GF(16), recoding at a relay, the batched decode, a K sweep at fixed
    packet length and the paper's CPU method on the host.  `only`: run just that one."""
    out = {}
    for name, fn in EXTRA_PARTS:
        if only is None or only == name:
            out.update(fn(gf, torch, args))
    return out


def part_region(gf, torch, args) -> dict:
    """The paper's primitive on its own: one gf_region_madd call y ^= c x over a region of 1500 B
    to 1 GiB, GF(256) with c = 0x53 and GF(2) with c = 1, back to back through the C ABI; GB/s of
    x and the share of the HBM roofline (3 bytes of traffic per byte of x; the 64 MiB point's x
    and y fit the 256 MB last-level cache, so its repeated calls read partly from there).  Checked by a property that holds at any size
    (the parity tests compare the bytes with the oracle): two calls give y back, since the
    field's addition is XOR."""
    out = []
    lib = gf.lib()
    st = torch.cuda.current_stream().cuda_stream
    for L in (1500, 65536, 1 << 20, 64 << 20, 1 << 30):
        x = device_bytes(torch, L, synth.key(synth.BASE_SEED + 7, L, 1))
        y = device_bytes(torch, L, synth.key(synth.BASE_SEED + 7, L, 2))
        for n, c in ((8, 0x53), (1, 1)):
            y0 = y.clone()
            gf.gf_region_madd(n, y, x, c)
            changed = not torch.equal(y, y0)
            gf.gf_region_madd(n, y, x, c)
            ok = changed and torch.equal(y, y0)
            del y0
            reps = 20 if L >= (64 << 20) else 200
            # C-ABI calls, arguments marshalled once (the binding's checks are not the library's latency)
            yp, xp = y.data_ptr(), x.data_ptr()
            ms = time_ms(torch, lambda: lib.gf_region_madd(n, yp, xp, c, L, st), reps=reps, warm=3)
            out.append({"field": "GF(2^%d)" % n, "c": c, "bytes": L, "gbs": round(L / ms / 1e6, 2),
                        "us": round(ms * 1e3, 2), "hbm_frac": round(3 * L / ms / 1e6 / HBM_PEAK_GBS, 4),
                        "twice_is_identity": ok})
            log("region madd GF(2^%d) %d B: %.1f GB/s of x (%.0f%% of HBM roofline), %.2f us"
                % (n, L, L / ms / 1e6, 100 * 3 * L / ms / 1e6 / HBM_PEAK_GBS, ms * 1e3))
        del x, y
        torch.cuda.empty_cache()
    return {"region_madd_single": out}


def part_single_generation(gf, torch, args) -> dict:
    out = {}
    # ---- one generation: GF(256), 16 x 16 x 1500 B, encode and decode back (latency, one launch each)
    g = synth.single_generation()
    Cd = torch.from_numpy(g.C).to("cuda")
    Sd = torch.from_numpy(g.S).to("cuda")
    Yd = torch.empty_like(Sd)
    Rd = torch.empty_like(Sd)
    ws = torch.empty(gf.gf_decode_workspace(8, 16), dtype=torch.uint8, device="cuda")
    rank = torch.zeros(1, dtype=torch.int32, device="cuda")
    # the C-ABI calls with their arguments marshalled once (the Python binding's own checks cost
    # several microseconds per call and are not the library's latency)
    L = gf.lib()
    st = torch.cuda.current_stream().cuda_stream
    cp, sp, yp, rp, wp, kp = Cd.data_ptr(), Sd.data_ptr(), Yd.data_ptr(), Rd.data_ptr(), ws.data_ptr(), rank.data_ptr()
    nws = ws.numel()
    enc = lambda: L.gf_encode(8, cp, 16, 16, sp, 1500, yp, 1500, 1500, st)   # noqa: E731
    dec = lambda: L.gf_decode(8, cp, yp, 1500, 16, rp, 1500, 1500, wp, nws, kp, st)   # noqa: E731
    enc_ms = time_ms(torch, enc, reps=500, warm=20)
    dec_ms = time_ms(torch, dec, reps=500, warm=20)

    def one_launch_us(fn, reps=200):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3)
        return float(np.median(ts))

    enc_one, dec_one = one_launch_us(enc), one_launch_us(dec)
    torch.cuda.synchronize()
    out["single_generation"] = {"field": "GF(2^8)", "N": 16, "K": 16, "packet_bytes": 1500,
                                "encode_us": round(enc_ms * 1e3, 2), "decode_us": round(dec_ms * 1e3, 2),
                                "encode_one_launch_us": round(enc_one, 2), "decode_one_launch_us": round(dec_one, 2),
                                "decoded_equals_source": bool(torch.equal(Rd, Sd)) and int(rank.item()) == 16,
                                "timing": "encode_us/decode_us: mean per call of 500 back-to-back C-ABI calls; "
                                          "*_one_launch_us: median HIP-event time around one call on an idle "
                                          "stream; inputs in HBM"}
    log("single generation: encode %.1f us, decode %.1f us per call (one isolated call: %.1f / %.1f us)"
        % (enc_ms * 1e3, dec_ms * 1e3, enc_one, dec_one))
    del Cd, Sd, Yd, Rd, ws
    return out


def part_sweep(gf, torch, args) -> dict:
    out = {}
    # ---- plain sweep: 4096 generations, N = K = 64, every field and packet length
    sweep = []
    count = 4096
    for n in [int(v) for v in args.sweep_fields.split(",")]:
        for L in [int(v) for v in args.sweep_lengths.split(",")]:
            plan, S, Cm, Y, ld = uniform_plan(gf, torch, synth.sweep_batch(n, L, count))
            ms = time_ms(torch, lambda: gf.gf_plan_launch_graph(plan), reps=3, warm=1)
            src = count * 64 * L
            t = plan.tuning()
            # region madd: one madd per (generation, source) into its own destination row
            R = torch.empty_like(S)
            nreg = count * 64
            dt = np.dtype([("y", "<u8"), ("x", "<u8"), ("len", "<u8"), ("c", "<u4"), ("r", "<u4")])
            regs = np.zeros(nreg, dtype=dt)
            idx = np.arange(nreg, dtype=np.uint64)
            regs["y"] = np.uint64(R.data_ptr()) + idx * np.uint64(ld)
            regs["x"] = np.uint64(S.data_ptr()) + idx * np.uint64(ld)
            regs["len"] = L
            regs["c"] = (np.arange(nreg) % ((1 << n) - 1)) + 1
            d_regs = torch.from_numpy(regs.view(np.uint8).copy()).to("cuda")
            mms = time_ms(torch, lambda: gf.gf_region_madd_batched(n, d_regs, nreg, L), reps=3, warm=1)
            hbm_enc = HBM_PEAK_GBS * (64 * L) / (64 * L + 64 * L + 64 * 64)
            sweep.append({"field": "GF(2^%d)" % n, "packet_bytes": L, "generations": count,
                          "encode_gbs": round(src / ms / 1e6, 2), "encode_ms": round(ms, 3),
                          "encode_hbm_frac": round(src / ms / 1e6 / hbm_enc, 4), "form": t["form"],
                          "grid_blocks": t["grid_blocks"],
                          "madd_gbs": round(src / mms / 1e6, 2), "madd_ms": round(mms, 3),
                          "madd_hbm_frac": round(3 * src / mms / 1e6 / HBM_PEAK_GBS, 4)})
            log("sweep GF(2^%d) L=%d: encode %.1f GB/s (form %d, %d workgroups), region madd %.1f GB/s"
                % (n, L, src / ms / 1e6, t["form"], t["grid_blocks"], src / mms / 1e6))
            plan.destroy()
            del plan, S, Cm, Y, R, d_regs
            torch.cuda.empty_cache()
    out["sweep"] = sweep
    return out


def part_uneven_gf16(gf, torch, args) -> dict:
    out = {}
    # ---- the uneven batch over GF(16)
    b = synth.uneven_batch(4, args.count)
    S_dev = torch.from_numpy(b.source_blob()).to("cuda")
    C_dev = torch.from_numpy(b.coef_blob()).to("cuda")
    Y_dev = torch.empty(b.y_bytes, dtype=torch.uint8, device="cuda")
    descs = (gf.gf_gen * args.count)()
    s0, c0, y0 = S_dev.data_ptr(), C_dev.data_ptr(), Y_dev.data_ptr()
    for i in range(args.count):
        descs[i] = gf.gf_gen(c0 + int(b.c_off[i]), s0 + int(b.s_off[i]), y0 + int(b.y_off[i]), int(b.Ks[i]),
                             int(b.Ns[i]), int(b.Ls[i]), int(b.lds[i]), int(b.lds[i]))
    plan = gf.gf_plan_encode_desc(4, descs, args.count, tune={"form": 0}, keep=(S_dev, C_dev, Y_dev))
    ms = time_ms(torch, lambda: gf.gf_plan_launch_graph(plan), reps=5, warm=2)
    out["uneven_gf16"] = {"generations": args.count, "source_bytes": b.source_bytes,
                          "gbs": round(b.source_bytes / ms / 1e6, 2), "ms": round(ms, 3),
                          "form": plan.tuning()["form"]}
    log("uneven GF(16): %.1f GB/s" % (b.source_bytes / ms / 1e6))
    plan.destroy()
    del plan, S_dev, C_dev, Y_dev
    torch.cuda.empty_cache()
    return out


def part_recode(gf, torch, args) -> dict:
    out = {}
    # ---- recoding at a relay: the uneven GF(256) shapes; each relay holds M = N received packets
    # and sends Kout = N recoded ones.  Packets are rows [N coefficients | payload], 16-byte pitch.
    rb = relay_batch(gf, torch, args.count)
    b, Ns, plan = rb["batch"], rb["Ns"], rb["plan"]
    ms = time_ms(torch, lambda: gf.gf_plan_launch_graph(plan), reps=5, warm=2)
    out["recode_uneven_gf256"] = {"relays": args.count, "received_payload_bytes": b.source_bytes,
                                  "header_bytes": int((Ns * Ns).sum()), "layout": "packet rows [coefficients | payload]",
                                  "gbs": round(b.source_bytes / ms / 1e6, 2), "ms": round(ms, 3),
                                  "form": plan.tuning()["form"],
                                  "launch": "hip graph, 1 persistent kernel (header and payload in one product)"}
    log("recode, uneven GF(256): %.1f GB/s of received payload, %.3f ms" % (b.source_bytes / ms / 1e6, ms))
    plan.destroy()
    del plan, rb
    torch.cuda.empty_cache()
    return out


def part_decode(gf, torch, args) -> dict:
    out = {}
    # ---- batched decode: 2048 systems, N in {32, 64, 128}, 1500 B, GF(256)
    db = synth.decode_batch(2048, 1500)
    count = len(db.Ns)
    S_dev = torch.from_numpy(db.source_blob()).to("cuda")
    B_dev = torch.empty_like(S_dev)
    R_dev = torch.empty_like(S_dev)
    attempt = np.zeros(count, dtype=np.int64)
    C_host = np.zeros(db.c_bytes, dtype=np.uint8)

    def fill(i):
        N = int(db.Ns[i])
        C_host[db.c_off[i]:db.c_off[i] + N * N] = synth.decode_candidate(i, int(attempt[i]), N).reshape(-1)

    for i in range(count):
        fill(i)
    rank = torch.zeros(count, dtype=torch.int32, device="cuda")
    eplan = dplan = None
    for _ in range(8):    # redraw singular candidates (the device reports each system's rank)
        if eplan is not None:
            eplan.destroy()
            dplan.destroy()
        C_dev = torch.from_numpy(C_host).to("cuda")
        sysd = (gf.gf_sys * count)()
        encd = (gf.gf_gen * count)()
        for i in range(count):
            N, L, ld = int(db.Ns[i]), int(db.Ls[i]), int(db.lds[i])
            cp = C_dev.data_ptr() + int(db.c_off[i])
            sp = S_dev.data_ptr() + int(db.s_off[i])
            bp = B_dev.data_ptr() + int(db.s_off[i])
            rp = R_dev.data_ptr() + int(db.s_off[i])
            encd[i] = gf.gf_gen(cp, sp, bp, N, N, L, ld, ld)
            sysd[i] = gf.gf_sys(cp, bp, rp, N, 0, L, ld, ld)
        eplan = gf.gf_plan_encode_desc(8, encd, count, tune={"form": 1}, keep=(C_dev, S_dev, B_dev))
        gf.gf_plan_launch(eplan)
        dplan = gf.gf_plan_decode_desc(8, sysd, count, keep=(C_dev, B_dev, R_dev))
        gf.gf_plan_launch(dplan, rank)
        torch.cuda.synchronize()
        ranks = rank.cpu().numpy()
        bad = np.nonzero(ranks != db.Ns)[0]
        if len(bad) == 0:
            break
        for i in bad:
            attempt[i] += 1
            fill(int(i))
    else:
        raise RuntimeError("decode batch: singular systems left after 8 redraws")
    ms = time_ms(torch, lambda: gf.gf_plan_launch_graph(dplan, rank), reps=5, warm=2)
    src = int((db.Ns * db.Ls).sum())
    out["decode_batched"] = {"systems": count, "N": "U{32,64,128}", "packet_bytes": 1500,
                             "source_bytes": src, "gbs": round(src / ms / 1e6, 2), "ms": round(ms, 3),
                             "redrawn": int((attempt > 0).sum()),
                             "decoded_equals_source": bool(torch.equal(R_dev.view(-1, 1504)[:, :1500],
                                                                       S_dev.view(-1, 1504)[:, :1500]))}
    log("batched decode: %.1f GB/s, bit-exact %s" % (src / ms / 1e6, out["decode_batched"]["decoded_equals_source"]))
    eplan.destroy()
    dplan.destroy()
    del S_dev, B_dev, R_dev, C_dev
    torch.cuda.empty_cache()
    return out


def part_k_sweep(gf, torch, args) -> dict:
    out = {}
    # ---- K sweep at 9000 B: where encode meets the HBM roofline
    ks = []
    for K in [int(v) for v in args.k_list.split(",")]:
        count = int(np.ceil(1e9 / (K * 9000)))
        plan, S, Cm, Y, ld = uniform_plan(gf, torch, synth.uniform_batch(8, K, K, 9000, count,
                                                                     synth.key(synth.BASE_SEED + 5, K)))
        ms = time_ms(torch, lambda: gf.gf_plan_launch_graph(plan), reps=3, warm=1)
        src = count * K * 9000
        hbm = HBM_PEAK_GBS * (K * 9000) / (2 * K * 9000 + K * K)
        ks.append({"K": K, "N": K, "generations": count, "gbs": round(src / ms / 1e6, 2),
                   "hbm_roofline_gbs": round(hbm, 1), "hbm_frac": round(src / ms / 1e6 / hbm, 4),
                   "byte_madds_per_s": round(K * src / ms * 1e3, 1), "form": plan.tuning()["form"],
                   "grid_blocks": plan.tuning()["grid_blocks"]})
        log("K sweep K=%d: %.1f GB/s (%.0f%% of HBM roofline, form %d)"
            % (K, src / ms / 1e6, 100 * src / ms / 1e6 / hbm, plan.tuning()["form"]))
        plan.destroy()
        del plan, S, Cm, Y
        torch.cuda.empty_cache()
    out["k_sweep_gf256_9000B"] = ks
    return out


def part_host_alg1(gf, torch, args) -> dict:
    out = {}
    # ---- the paper's own CPU method on this host, one core (context)
    out["host_alg1_avx512"] = host_alg1_sweep()
    for pt in out["host_alg1_avx512"].get("points", []):
        if pt["packet_bytes"] in (1500, 65536):
            log("host Alg. 1 %s %d B: %.2f GB/s (%.1f us per 16 x 16 encode)"
                % (pt["field"], pt["packet_bytes"], pt["gbs"], pt["encode_us"]))
    return out


EXTRA_PARTS = (("single_generation", part_single_generation), ("region", part_region), ("sweep", part_sweep),
               ("uneven_gf16", part_uneven_gf16), ("recode", part_recode), ("decode", part_decode),
               ("k_sweep", part_k_sweep), ("host_alg1", part_host_alg1))


def stream_copy_gbs(torch, nbytes: int = 4 << 30, reps: int = 5) -> float:
    """HBM bandwidth a plain device-to-device copy reaches (bytes read + written per second)."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(reps):
        e0, e1 = _events(torch)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


def measure_ceilings(gf, torch) -> dict:
    """What the chip delivers for each kernel form's instruction mix, by the library's
    microbenchmarks (gf_ceiling): device copy bandwidth, byte-madds/s of the table form's
    lookup step, dense FP4 MFMA TFLOP/s, and 3-input bit operations/s of the bit-plane step."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}

    def timed(what, buf, blocks, iters):
        gf.gf_ceiling(what, buf, blocks, max(1, iters // 10))        # warm-up
        e0, e1 = _events(torch)
        e0.record()
        gf.gf_ceiling(what, buf, blocks, iters)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    buf = torch.empty(4 << 30, dtype=torch.uint8, device="cuda")
    t = min(timed(0, buf, cus * 32, 0) for _ in range(3))
    out["copy_gbs"] = round(buf.numel() / t / 1e9, 1)                  # half read + half written
    t = min(timed(4, buf, 1, 0) for _ in range(3))
    out["copy_chunks_gbs"] = round(buf.numel() / t / 1e9, 1)           # the same, a workgroup per 16 KiB
    small = torch.empty(cus * 64 * 1024, dtype=torch.uint8, device="cuda")
    blocks, iters = cus * 8, 4000
    t = timed(1, small, blocks, iters)
    out["table_byte_madds_per_s"] = round(blocks * 256 * iters * 64 / t, 1)
    blocks_m, iters_m = cus * 2, 4000
    t = timed(2, small, blocks_m, iters_m)
    out["fp4_mfma_tflops"] = round(blocks_m * 4 * iters_m * 8 * 2 * 32 * 32 * 64 / t / 1e12, 1)
    t = timed(3, small, blocks, iters)
    out["bitplane_ops_per_s"] = round(blocks * 256 * iters * 64 / t, 1)
    del buf, small
    torch.cuda.empty_cache()
    return out


def host_cpu() -> dict:
    """Host cores and CPU model, for the CPU baseline."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model,
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_oracle_baseline(oracle, b, S_host, C_host, Y_host, args) -> dict:
    """The plain oracle on a bounded sample of the batch: all host cores (OpenMP over generations,
    the thread count of OMP_NUM_THREADS or the usable cores, at most 16) and one core (the paper's
    protocol); the GPU's bytes are checked against the oracle's on the sample."""
    hc = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS") or 0) or hc["affinity"] or hc["nproc"] or 1
    threads = max(1, min(threads, 16))
    order = np.argsort(synth.words(synth.key(synth.BASE_SEED + 2, 99), len(b.Ns)))

    def pick(budget):
        picked, acc = [], 0
        for i in order:
            w = int(b.Ks[i] * b.Ns[i] * b.Ls[i])
            if acc + w > budget and picked:
                continue
            picked.append(int(i))
            acc += w
            if acc >= budget:
                break
        return picked, acc

    def run(picked, nthreads):
        Cs = [b.generation(i, S_host, C_host) for i in picked]
        desc, c_parts, s_parts, co, so, yo = [], [], [], 0, 0, 0
        for i, (Cm, S) in zip(picked, Cs):
            K, N, L = int(b.Ks[i]), int(b.Ns[i]), int(b.Ls[i])
            desc.append([co, so, yo, L, L, L, K, N])
            c_parts.append(np.ascontiguousarray(Cm).reshape(-1))
            s_parts.append(np.ascontiguousarray(S).reshape(-1))
            co, so, yo = co + K * N, so + N * L, yo + K * L
        Cb, Sb = np.concatenate(c_parts), np.concatenate(s_parts)
        Yb = np.zeros(yo, np.uint8)
        t0 = time.perf_counter()
        used = oracle.encode_batch(b.n, np.array(desc, np.int64), Cb, Sb, Yb, nthreads)
        dt = time.perf_counter() - t0
        ok = True
        for (i, d) in zip(picked, desc):
            K, L, ld = int(b.Ks[i]), int(b.Ls[i]), int(b.lds[i])
            got = Y_host[b.y_off[i]:b.y_off[i] + K * ld].reshape(K, ld)[:, :L]
            ok = ok and bool((got == Yb[d[2]:d[2] + K * L].reshape(K, L)).all())
        return used, dt, so, ok

    # about 4e7 byte-madds per second per core for the plain oracle
    picked, acc = pick(args.cpu_seconds * 4e7 * threads)
    used, dt, src, ok = run(picked, threads)
    p1, acc1 = pick(max(2.0, args.cpu_seconds / 3) * 4e7)
    _, dt1, src1, ok1 = run(p1, 1)
    out = {"value": round(src / dt / 1e9, 6), "unit": "GB/s", "cores": used, "kind": "oracle",
           "sample": "%d of %d generations (%.3g byte-madds, %.1f MB of source), plain C oracle, OpenMP over "
                     "generations on %d threads" % (len(picked), len(b.Ns), acc, src / 1e6, used),
           "seconds": round(dt, 2), "gpu_output_bit_exact_on_sample": ok and ok1, **hc,
           "one_core": {"value": round(src1 / dt1 / 1e9, 6), "unit": "GB/s", "cores": 1,
                        "sample": "%d generations (%.3g byte-madds)" % (len(p1), acc1), "seconds": round(dt1, 2)}}
    log("cpu oracle: %.4f GB/s on %d threads (%s), %.4f GB/s on one; GPU bit-exact on sample: %s"
        % (out["value"], used, hc["cpu_model"], out["one_core"]["value"], ok and ok1))
    return out


def single_generation_oracle(gf, torch, oracle) -> dict:
    """The oracle's CPU seconds for the one-generation encode and decode (GF(256), 16 x 16 x 1500 B),
    checked against the GPU's bytes."""
    g = synth.single_generation()
    t0 = time.perf_counter()
    Y = oracle.encode(8, g.C, g.S)
    t1 = time.perf_counter()
    r, R = oracle.decode(8, g.C, Y)
    t2 = time.perf_counter()
    Cd = torch.from_numpy(g.C).to("cuda")
    Sd = torch.from_numpy(g.S).to("cuda")
    Yd = torch.empty_like(Sd)
    gf.gf_encode(8, Cd, Sd, Yd)
    torch.cuda.synchronize()
    return {"encode_s": round(t1 - t0, 6), "decode_s": round(t2 - t1, 6),
            "gpu_encode_bit_exact": bool((Yd.cpu().numpy() == Y).all()),
            "decode_equals_source": bool(r == 16 and R is not None and (R == g.S).all())}


SENDER_POOL = 3          # a decode's sender can emit up to 3 N coded packets


def serving_trace(gf, torch, count: int, n: int = 8) -> dict:
    """The serving workload's requests: 70% encode / 30% decode over GF(2^n), N uniform in
    {8..256}, packet length log-uniform in [64, 9000] B.  A decode request's sender is rateless:
    it emits coded packets with fresh uniform coefficient vectors, one every microsecond from the
    request's arrival, in a random order of its pool of 3 N, each lost i.i.d. with probability
    0.1, until the server reports the generation decoded (the replay stops it there).  Sources
    and coefficients are drawn on the device from the seeded streams.  Arrival times are left at
    0 (the caller scales `unit_gaps`).  Also returns, per request, where its coefficients and
    sources sit in the device blobs."""
    from paper_1909_02871_amd.serving import TraceRequest

    reqs = synth.serving_stream(count, 1.0)          # shapes and kinds; arrival times are rescaled later
    unit_gaps = np.array([r.arrival_s for r in reqs])
    enc = [r for r in reqs if r.kind == "encode"]
    dec = [r for r in reqs if r.kind == "decode"]
    pool = {r.rid: SENDER_POOL * r.N for r in dec}
    s_need = sum(r.N * synth.padded(r.length) for r in reqs)
    c_need = sum(r.N * r.N for r in enc) + sum(pool[r.rid] * r.N for r in dec)
    base = synth.key(synth.BASE_SEED + 4, 99)
    S_dev = synth.device_random_bytes(torch, synth.key(base, 1), s_need)
    C_dev = device_bytes(torch, c_need, synth.key(base, 2), 1 << n)
    b_need = sum(pool[r.rid] * synth.padded(r.length) for r in dec)
    B_dev = torch.empty(max(b_need, 16), dtype=torch.uint8, device="cuda")
    s_off = c_off = b_off = 0
    trace, where = [], {}
    src_bytes = 0
    for r in reqs:
        ld = synth.padded(r.length)
        S = S_dev[s_off:s_off + r.N * ld].view(r.N, ld)
        where[r.rid] = {"kind": r.kind, "N": r.N, "length": r.length, "ld": ld, "s_off": s_off, "c_off": c_off}
        s_off += r.N * ld
        src_bytes += r.N * r.length
        if r.kind == "encode":
            Cm = C_dev[c_off:c_off + r.N * r.N].view(r.N, r.N)
            c_off += r.N * r.N
            trace.append(TraceRequest(r.rid, 0.0, "encode", r.N, r.length, C=Cm.data_ptr(), S=S.data_ptr(), K=r.N,
                                      ld_s=ld))
        else:
            P = pool[r.rid]
            Cp = C_dev[c_off:c_off + P * r.N].view(P, r.N)
            c_off += P * r.N
            Bp = B_dev[b_off:b_off + P * ld].view(P, ld)
            b_off += P * ld
            gf.gf_encode(n, Cp, S[:, :r.length], Bp[:, :r.length])     # the sender's coded packets
            lost = synth.unit_floats(synth.key(r.seed, 1), P) < 0.1
            order = np.argsort(synth.words(synth.key(r.seed, 2), P))
            pk = [(Cp[j].data_ptr(), Bp[j].data_ptr(), 1e-6 * t) for t, j in enumerate(order) if not lost[j]]
            trace.append(TraceRequest(r.rid, 0.0, "decode", r.N, r.length, packets=pk))
    torch.cuda.synchronize()
    return {"trace": trace, "unit_gaps": unit_gaps, "src_bytes": src_bytes, "enc": enc, "where": where,
            "S_dev": S_dev, "C_dev": C_dev, "B_dev": B_dev}


def serve_bench(gf, torch, args) -> dict:
    """Serving: Poisson arrivals of 70% encode / 30% decode requests over GF(256).

    N uniform in {8..256}, packet length log-uniform in [64, 9000] B; a decode
    request is fed by a rateless sender (see serving_trace) that stops once the
    server reports the generation decoded.  The server admits requests by an HBM
    budget.  For each budget (4 GiB and a tight 512 MiB) a run with every request
    arriving at once gives the saturation throughput, then runs at 50%, 80% and
    95% of it give the latency percentiles.
    """
    from paper_1909_02871_amd.serving import percentile, replay

    n = 8
    count = args.serve_requests
    t0 = time.perf_counter()
    st_ = serving_trace(gf, torch, count)
    trace, unit_gaps, src_bytes, enc = st_["trace"], st_["unit_gaps"], st_["src_bytes"], st_["enc"]
    log("serving trace of %d requests built in %.1f s" % (count, time.perf_counter() - t0))
    sum_N_dec = sum(tr.N for tr in trace if tr.kind == "decode")

    def run(rate, budget):
        for tr, g in zip(trace, unit_gaps):
            tr.arrival = 0.0 if rate is None else float(g) / rate
        srv = gf.Server(field=n, budget_bytes=budget, burst=args.serve_burst)
        t0 = time.perf_counter()
        done = replay(srv, trace, timeout_s=300)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        ok = [d for d in done if d["status"] == 0]
        lat = [d["latency"] * 1e3 for d in ok]
        lat_e = [d["latency"] * 1e3 for d in ok if d["kind"] == "encode"]
        lat_d = [d["latency"] * 1e3 for d in ok if d["kind"] == "decode"]
        sent = sum(d["packets_sent"] for d in done if d["kind"] == "decode")
        return {"offered_rps": None if rate is None else round(rate, 1), "completed": len(ok),
                "cancelled": len(done) - len(ok),
                "decodes_complete": all(d["rank"] == d_N for d, d_N in
                                        ((d, where_N[d["id"]]) for d in done if d["kind"] == "decode")),
                "wall_s": round(wall, 3), "throughput_rps": round(len(ok) / wall, 1),
                "source_gbs": round(src_bytes / wall / 1e9, 3),
                "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
                "encode_p50_ms": round(percentile(lat_e, 50), 3), "encode_p99_ms": round(percentile(lat_e, 99), 3),
                "decode_p50_ms": round(percentile(lat_d, 50), 3), "decode_p99_ms": round(percentile(lat_d, 99), 3),
                "steps": st["steps"], "arena_peak_gib": round(st["arena_peak"] / (1 << 30), 3),
                "packets_sent_per_N": round(sent / max(1, sum_N_dec), 3),
                "packets_absorbed": st["packets_absorbed"]}

    where_N = {rid: w["N"] for rid, w in st_["where"].items()}
    budgets = [4.0, 0.5] if args.serve_budget_gib == 4.0 else [args.serve_budget_gib]
    runs = []
    for gib in budgets:
        budget = int(gib * (1 << 30))
        sat = run(None, budget)
        sat.update(budget_gib=gib, load_fraction=None)
        log("serve %.1f GiB saturation: %s" % (gib, sat))
        runs.append(sat)
        cap = sat["throughput_rps"]
        for frac in (0.5, 0.8, 0.95):
            res = run(cap * frac, budget)
            res.update(budget_gib=gib, load_fraction=frac)
            runs.append(res)
            log("serve %.1f GiB at %.0f%%: %s" % (gib, 100 * frac, res))
    head = next(r for r in runs if r["budget_gib"] == budgets[0] and r["load_fraction"] == 0.8)
    return {"workload": "mixed_serving_gf256", "requests": count, "encode_fraction": round(len(enc) / count, 3),
            "N": "U{8..256}", "packet_bytes": "log-U[64, 9000]", "loss": 0.1, "packet_gap_us": 1.0,
            "sender": "rateless: up to %d N packets, stops when the server reports rank N" % SENDER_POOL,
            "runs": runs, "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
            "p50_p99_at": "%.1f GiB budget, 80%% of saturation" % budgets[0]}


if __name__ == "__main__":
    main()
