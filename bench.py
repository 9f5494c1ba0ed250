#!/usr/bin/env python3
"""Benchmark of the base64 hot path on one MI355X.

Default (one JSON line): the single-buffer 1 GiB workload (n = 1,073,741,823
uniform random bytes, standard alphabet).  One step = encode the buffer
(b64_encode) and decode the result back (b64_decode_async, validation
included), inputs resident in HBM.  Throughput counts base64 characters, as the
paper does (Section "Experiments"): value = 2 * N / step time, N = 4*ceil(n/3).

Also reported in the same line: each direction against a same-size
device-to-device hipMemcpyAsync (the paper's memcpy yardstick), the roofline of
the slower kernel (algorithmic bytes / average duration from HIP events on the
launch stream, against the 8 TB/s HBM peak), the oracle's CPU throughput on a
bounded sample, and the metric's other two parts: `batch` (the 100,000-buffer
ragged workload, one graph-captured batched launch per direction against one
launch per buffer) and `serve` (p50 / p99 latency of the continuous-batching
server at 10^4 and 3 x 10^5 requests per second).

Other modes (--mode): ceiling (streaming kernels with the codec's access
patterns and grids but no arithmetic, and a same-size copy: the attainable
bandwidth), sweep (size sweep 2^k + r), batch (100,000 ragged
buffers, batched launch vs one launch per buffer), serve (continuous batching
loop), small (the 3 MiB workload), validate (read-only validation of the
1 GiB encoding), host (the 1 GiB workload in host memory through the chunked
host-device pipeline, PCIe included), variants (the 1 GiB payload unpadded,
and as MIME text: 76-character lines with CR LF, wrapped encode and
whitespace-skipping decode / validate), fused (rows of base64 float32 decoded
straight into bfloat16, against decode + a separate conversion).  Each prints
its own JSON lines.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "encode/decode GB/s as % of D2D memcpy; batched vs per-buffer GB/s; p99"
# sources of the single-buffer kernels; a change to them voids the recorded HBM traffic
KERNEL_SRCS = [os.path.join(ROOT, "paper_1910_05109_amd", "csrc", f)
               for f in ("b64_device.h", "b64_single.hip")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, n_launch_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(kernel)
    if not ent or ent.get("kernel_src_sha256_16") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def events_ms(pairs):
    return [a.elapsed_time(b) for a, b in pairs]


def time_memcpy(torch, nbytes: int, reps: int = 20):
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    pairs = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        b.copy_(a)
        e.record()
        pairs.append((s, e))
    torch.cuda.synchronize()
    ms = events_ms(pairs)
    del a, b
    return statistics.median(ms)


def cpu_baseline(x: np.ndarray, sample_bytes: int, reps: int):
    """The oracle as it stands on the first `sample_bytes` bytes: encode then
    decode, median of `reps`; GB/s of base64 characters over both directions,
    like the GPU value.  Timed on every host core (the oracle's C functions
    called on chunks cut at 3-byte / 4-character boundaries from one thread
    per core; ctypes releases the GIL during the calls) and on one thread."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    xs = np.ascontiguousarray(x[:sample_bytes])
    nchar = 4 * ((sample_bytes + 2) // 3)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()

    def one_thread():
        text = oracle.encode(xs)
        dec, bad = oracle.decode(text)
        assert bad is None and dec.size == xs.size

    def all_cores(pool):
        step = -(-sample_bytes // (3 * cores)) * 3              # a multiple of 3 bytes
        parts = [xs[i:i + step] for i in range(0, sample_bytes, step)]
        texts = list(pool.map(oracle.encode, parts))
        decs = list(pool.map(oracle.decode, texts))
        assert all(b is None for _, b in decs) and sum(d.size for d, _ in decs) == xs.size

    def med(fn):
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            times.append(time.perf_counter() - t0)
        return statistics.median(times)

    with ThreadPoolExecutor(max_workers=cores) as pool:
        t_all = med(lambda: all_cores(pool))
    t_one = med(one_thread)
    return {"value": round(2 * nchar / t_all / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "single_thread": {"value": round(2 * nchar / t_one / 1e9, 4), "cores": 1},
            "sample": f"first {sample_bytes} bytes of the 1 GiB input, encode+decode, median of "
                      f"{reps}; value on {cores} threads (one per available host core, chunks "
                      f"of 3-byte / 4-character multiples), single_thread on one"}


YARD_KINDS = {"read_only": 0, "write_only": 1, "encode_pattern": 2, "decode_pattern": 3,
              "copy_same_grid": 4}


def ceiling_measure(torch, n: int, N: int, reps: int = 20) -> dict:
    """Attainable bandwidth with the codec kernels' access patterns and grids
    and none of their arithmetic (b64_yardstick), for the byte counts of an
    n-byte encode / N-character decode: median ms, bytes moved and GB/s of
    each pattern, and a hipMemcpyAsync of N bytes."""
    import ctypes
    from paper_1910_05109_amd import _lib
    from paper_1910_05109_amd import stream_ptr
    L = _lib.load()
    a = torch.empty(N, dtype=torch.uint8, device="cuda").fill_(0x41)
    b = torch.empty(N, dtype=torch.uint8, device="cuda")
    st = stream_ptr()
    cases = {  # kind: (lane chunks, bytes read per chunk, bytes written per chunk)
        "encode_pattern": (n // 12, 12, 16), "decode_pattern": (N // 16, 16, 12),
        "read_only": (N // 16, 16, 0), "write_only": (N // 16, 0, 16),
        "copy_same_grid": (N // 16, 16, 16)}
    out = {}
    for name, (nch, rin, wout) in cases.items():
        kind = YARD_KINDS[name]
        fn = lambda: L.b64_yardstick(kind, a.data_ptr(), b.data_ptr(), nch, st)
        for _ in range(3):
            assert fn() == 0, name
        t = _events_time(torch, fn, reps)["median"]
        moved = nch * (rin + wout)
        out[name] = {"ms": round(t, 4), "bytes": moved, "gbps": round(moved / t / 1e6, 1),
                     "frac_of_peak": round(moved / t / 1e6 / HBM_PEAK_GBS, 4)}
    t = _events_time(torch, lambda: b.copy_(a), reps)["median"]
    out["memcpy_N"] = {"ms": round(t, 4), "bytes": 2 * N, "gbps": round(2 * N / t / 1e6, 1),
                       "frac_of_peak": round(2 * N / t / 1e6 / HBM_PEAK_GBS, 4)}
    del a, b
    torch.cuda.empty_cache()
    return out


def run_ceiling(args, torch, b64):
    """The attainable-bandwidth ceiling at the 1 GiB workload's sizes."""
    n = workloads.SINGLE_1GIB[0]
    N = 4 * ((n + 2) // 3)
    res = {"workload": "bandwidth ceiling at the 1 GiB workload's sizes", "n_bytes": n,
           "n_chars": N, **ceiling_measure(torch, n, N, args.steps)}
    print(json.dumps(res), flush=True)


def run_single(args, torch, b64):
    n = workloads.SINGLE_1GIB[0]
    N = 4 * ((n + 2) // 3)
    log("generate", n, "bytes")
    x = workloads.random_bytes(workloads.SEED_BASE + 2, n)
    dx = torch.from_numpy(x).cuda()
    dtext = torch.empty(N, dtype=torch.uint8, device="cuda")
    ddec = torch.empty(3 * (N // 4), dtype=torch.uint8, device="cuda")
    status = torch.empty(2, dtype=torch.int64, device="cuda")

    def step(rec=None):
        if rec is not None:
            rec[0].record()
        b64.encode(dx, out=dtext)
        if rec is not None:
            rec[1].record()
        b64.decode_async(dtext, out=ddec, status=status)
        if rec is not None:
            rec[2].record()

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = status.cpu().tolist()
    assert st == [n, -1], st
    assert torch.equal(ddec[:n], dx), "round trip mismatch"

    recs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(recs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    enc_ms = [r[0].elapsed_time(r[1]) for r in recs]
    dec_ms = [r[1].elapsed_time(r[2]) for r in recs]
    assert status.cpu().tolist() == [n, -1]

    ms_step = wall * 1e3 / args.steps
    value = 2 * N / (ms_step * 1e-3) / 1e9
    enc_avg, dec_avg = statistics.mean(enc_ms), statistics.mean(dec_ms)
    log("memcpy yardstick")
    mc_N = time_memcpy(torch, N)
    mc_n = time_memcpy(torch, n)
    alg = n + N                                  # bytes each direction reads + writes
    if enc_avg >= dec_avg:
        kname, kms = "k_encode", enc_avg
    else:
        kname, kms = "k_decode", dec_avg
    achieved = alg / (kms * 1e-3) / 1e9
    log("bandwidth ceiling (codec access patterns, no arithmetic)")
    ceil = ceiling_measure(torch, n, N)
    pat = ceil["encode_pattern" if kname == "k_encode" else "decode_pattern"]
    rec = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "single 1 GiB buffer: encode + decode with validation, "
                               "standard alphabet", "n_bytes": n, "n_chars": N},
        "encode": {"ms": round(enc_avg, 4), "gbps_b64": round(N / enc_avg / 1e6, 1),
                   "pct_memcpy_N": round(100 * mc_N / enc_avg, 1),
                   "pct_memcpy_n": round(100 * mc_n / enc_avg, 1)},
        "decode": {"ms": round(dec_avg, 4), "gbps_b64": round(N / dec_avg / 1e6, 1),
                   "pct_memcpy_N": round(100 * mc_N / dec_avg, 1),
                   "pct_memcpy_n": round(100 * mc_n / dec_avg, 1)},
        "memcpy": {"ms_N": round(mc_N, 4), "ms_n": round(mc_n, 4),
                   "gbps_N": round(2 * N / mc_N / 1e6, 1)},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(kname, alg),
                     "ceiling": pat["gbps"], "frac_of_ceiling": round(achieved / pat["gbps"], 4)},
        "ceiling": {k: {"ms": v["ms"], "gbps": v["gbps"]} for k, v in ceil.items()},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(x, args.cpu_sample, args.cpu_reps)
    del dx, dtext, ddec
    torch.cuda.empty_cache()
    if not args.no_extras:
        # the other two parts of the metric: batched vs per-buffer GB/s on the
        # ragged-batch workload, and serving latency at two arrival rates
        log("batch part of the metric")
        bm = batch_measure(torch, b64, args.nbuf, 5, same_bytes=False)
        rec["batch"] = {"workload": bm["workload"], "buffers": bm["buffers"], "chars": bm["chars"],
                        **{k: {kk: bm[k][kk] for kk in ("batched_ms", "batched_gbps_b64",
                                                        "per_buffer_gbps_b64", "speedup")}
                           for k in ("encode", "decode")}}
        log("serving part of the metric")
        from paper_1910_05109_amd import serve
        count = 20_000
        kinds, payload, off, sizes, spoil = serve_requests(torch, b64, count)
        keys = ("rate", "requests", "p50_us", "p99_us", "gbps_b64", "mean_batch", "max_concurrent",
                "zero_copy_launches")

        def serve_rows(zero_copy_max):
            rows = []
            with serve.Server(budget_bytes=32 << 30, nstreams=args.serve_streams,
                              depth=args.serve_depth, zero_copy_max=zero_copy_max,
                              staging=args.serve_staging) as srv:
                # untimed warm-up traffic at both rates: in a server's first
                # runs the HIP runtime's DMA copies now and then block the
                # scheduler thread for 5-8 ms (seen inside hipMemcpyAsync, most
                # often in the first run and the first run at a high rate),
                # which would decide the p99 of a 67 ms window by itself
                for rate in (1e4, 3e5):
                    serve_rate(srv, torch, b64, kinds, payload, off, sizes, spoil, rate, count)
                for rate in (1e4, 3e5):
                    r = serve_rate(srv, torch, b64, kinds, payload, off, sizes, spoil, rate, count)
                    rows.append({k: (round(v, 2) if isinstance(v, float) else v)
                                 for k, v in r.items() if k in keys})
            return rows

        rec["serve"] = {"workload": "Poisson arrivals, log-normal sizes (median 8 KiB, sigma 1.5), "
                                    "payloads from pinned host memory, staged in device memory "
                                    "under the HBM budget", "rows": serve_rows(args.serve_zero_copy_max)}
        if args.serve_zero_copy_max is None:
            # the same requests with every launch zero-copy: the kernels work on
            # the pinned host pools over PCIe, nothing staged in device memory
            rec["serve_zero_copy"] = {"workload": "the same, every launch zero-copy (no DMA, no arena)",
                                      "rows": serve_rows(64 << 20)}
    print(json.dumps(rec), flush=True)


def _events_time(torch, fn, reps, before=None):
    """Median / min / p90 ms of `fn` over `reps` runs, HIP events on the
    launch stream; `before` (untimed) runs ahead of each timed call."""
    pairs = []
    for _ in range(reps):
        if before is not None:
            before()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        pairs.append((a, b))
    torch.cuda.synchronize()
    ms = sorted(x.elapsed_time(y) for x, y in pairs)
    return {"median": ms[len(ms) // 2], "min": ms[0], "p90": ms[min(len(ms) - 1, int(0.9 * len(ms)))]}


def _graph_time(torch, fn, reps):
    """Median ms per replay of `fn` captured in a HIP graph (launch overhead
    amortised the way a captured serving loop would see it)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(10):
            fn()
    g.replay()
    torch.cuda.synchronize()
    r = _events_time(torch, g.replay, reps)
    return {k: v / 10 for k, v in r.items()}


def run_small(args, torch, b64):
    """The 3 MiB workload: launch-latency regime, warm in L2 / MALL."""
    n = workloads.SINGLE_3MIB
    x = torch.from_numpy(workloads.random_bytes(workloads.SEED_BASE + 1, n)).cuda()
    N = 4 * ((n + 2) // 3)
    text = torch.empty(N, dtype=torch.uint8, device="cuda")
    dec = torch.empty(n, dtype=torch.uint8, device="cuda")
    st = torch.empty(2, dtype=torch.int64, device="cuda")
    enc = lambda: b64.encode(x, out=text)
    dcd = lambda: b64.decode_async(text, out=dec, status=st)
    for _ in range(5):
        enc(); dcd()
    mc = lambda: dec.copy_(x)
    res = {"workload": "single 3 MiB buffer", "n_bytes": n, "n_chars": N,
           "encode_ms": _events_time(torch, enc, 50), "decode_ms": _events_time(torch, dcd, 50),
           "encode_graph_ms": _graph_time(torch, enc, 20), "decode_graph_ms": _graph_time(torch, dcd, 20),
           "memcpy_n_ms": _events_time(torch, mc, 50)}
    t0 = time.perf_counter()
    for _ in range(200):
        r = b64.decode(text, out=dec)
    res["decode_blocking_us"] = (time.perf_counter() - t0) / 200 * 1e6
    assert r[1] is None
    # Bursts of 200 back-to-back calls at 16 KiB, 256 KiB and 3 MiB of raw
    # bytes -- encode, decode, torch's device copy of the text and the
    # decode-pattern yardstick (decode's access pattern and grid, no
    # arithmetic) -- whose kernel durations a kernel trace of this run gives.
    import ctypes
    from paper_1910_05109_amd import _lib, stream_ptr
    L = _lib.load()
    sp = stream_ptr()
    bursts = {}
    for m in (16 << 10, 256 << 10, n):
        Nm = 4 * ((m + 2) // 3)
        xm, tm = x[:m], text[:Nm]
        cp = torch.empty(Nm, dtype=torch.uint8, device="cuda")
        fns = {"encode": lambda: b64.encode(xm, out=tm),
               "decode": lambda: b64.decode_async(tm, out=dec, status=st),
               "copy": lambda: cp.copy_(tm),
               "yardstick_decode_pattern": lambda: L.b64_yardstick(
                   YARD_KINDS["decode_pattern"], tm.data_ptr(), cp.data_ptr(), Nm // 16, sp)}
        row = {}
        for name, fn in fns.items():
            fn()                                  # a kernel's first launch loads its code
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(200):
                fn()
            b.record()
            torch.cuda.synchronize()
            row[name + "_us_per_call"] = a.elapsed_time(b) * 1e3 / 200
        b64.encode(xm, out=tm)
        bursts[str(m)] = row
    res["bursts"] = bursts
    # Host time per call with the GPU idle between groups: 1,000 calls on 48
    # bytes back to back, best of 5 (the device finishes a call sooner than
    # the host issues the next, so this is the host's cost).
    m = 48
    xm, tm = x[:m], text[:64]
    b64.encode(xm, out=tm)
    a_std = b64._alpha(b64.STD)
    tp, dp, stp = tm.data_ptr(), dec.data_ptr(), st.data_ptr()
    cp = torch.empty(64, dtype=torch.uint8, device="cuda")
    calls = {"decode_async": lambda: b64.decode_async(tm, out=dec, status=st),
             "encode": lambda: b64.encode(xm, out=tm),
             "validate_async": lambda: b64.validate_async(tm, status=st),
             "copy_": lambda: cp.copy_(tm),
             "raw_decode_async": lambda: L.b64_decode_async(tp, 64, dp, stp, stp + 8, a_std, sp)}
    if _lib.fast is not None:
        calls["fast_decode_async"] = lambda: _lib.fast.decode_async(
            tp, 64, dp, stp, stp + 8, ctypes.addressof(a_std), sp)
    host = {}
    for name, fn in calls.items():
        for _ in range(500):
            fn()
        torch.cuda.synchronize()
        best = []
        for _ in range(5):
            t0 = time.perf_counter()
            for _ in range(1000):
                fn()
            best.append((time.perf_counter() - t0) / 1000 * 1e6)
            torch.cuda.synchronize()
        host[name] = min(best)
    res["host_us_per_call"] = host
    assert b64.decode(text, out=dec)[1] is None
    print(json.dumps(res), flush=True)


def run_sweep(args, torch, b64):
    """Size sweep 2^k + r (k = 10..26, r = 0..2) plus the paper's four file
    sizes as lengths of random data; warm (back-to-back) and cold (the 256 MiB
    last-level cache flushed by a 512 MiB write before each run)."""
    lengths = workloads.sweep_lengths() + list(workloads.TABLE_PERF_LENGTHS)
    big = max(lengths)
    x = torch.from_numpy(workloads.random_bytes(workloads.SEED_BASE + 3, big)).cuda()
    text = torch.empty(4 * ((big + 2) // 3), dtype=torch.uint8, device="cuda")
    dec = torch.empty(big + 3, dtype=torch.uint8, device="cuda")
    mc_dst = torch.empty(4 * ((big + 2) // 3), dtype=torch.uint8, device="cuda")
    st = torch.empty(2, dtype=torch.int64, device="cuda")
    scratch = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    flush = lambda: scratch.fill_(1)
    rows = []
    for n in sorted(lengths):
        N = 4 * ((n + 2) // 3)
        xs, ts = x[:n], text[:N]
        enc = lambda: b64.encode(xs, out=ts)
        dcd = lambda: b64.decode_async(ts, out=dec, status=st)
        mcN = lambda: mc_dst[:N].copy_(ts)
        for _ in range(3):
            enc(); dcd(); mcN()
        row = {"n": n, "N": N}
        for name, fn in (("encode", enc), ("decode", dcd), ("memcpy_N", mcN)):
            w = _events_time(torch, fn, 20)
            c = _events_time(torch, fn, 10, before=flush)
            row[name] = {"warm_ms": w["median"], "cold_ms": c["median"]}
        for name in ("encode", "decode"):
            for reg in ("warm", "cold"):
                t = row[name][f"{reg}_ms"]
                row[name][f"{reg}_gbps_b64"] = N / t / 1e6
                row[name][f"{reg}_pct_memcpy_N"] = 100 * row["memcpy_N"][f"{reg}_ms"] / t
        if n <= (1 << 20) + 2:
            row["encode"]["graph_ms"] = _graph_time(torch, enc, 10)["median"]
            row["decode"]["graph_ms"] = _graph_time(torch, dcd, 10)["median"]
        working = n + 2 * N
        row["regime"] = ("latency" if N < (1 << 20) else
                         "on-chip" if working <= (256 << 20) else "hbm")
        assert st.cpu().tolist() == [n, -1]
        rows.append(row)
        log("sweep", n, row["regime"], f"enc {row['encode']['warm_gbps_b64']:.0f} GB/s",
            f"dec {row['decode']['warm_gbps_b64']:.0f} GB/s")
    print(json.dumps({"workload": "size sweep", "rows": rows}), flush=True)


def batch_measure(torch, b64, nbuf: int, steps: int, same_bytes: bool = True) -> dict:
    """The ragged-batch workload: `nbuf` buffers with log-uniform lengths in
    [16 B, 1 MiB) (uniform random bytes made on the device), one
    graph-captured batched launch per direction against one launch per
    buffer on one stream (no graph); every length and status is checked."""
    import ctypes
    from paper_1910_05109_amd import _lib
    from paper_1910_05109_amd.batch import GraphBatch
    seed = workloads.SEED_BASE + 4
    lens = workloads.batch_lengths(seed, nbuf)
    in_off = workloads.offsets(lens)
    total = int(in_off[-1])
    log("batch: generate", total, "bytes in", lens.size, "buffers")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    src = torch.randint(0, 256, (total,), dtype=torch.uint8, device="cuda", generator=gen)
    genc = GraphBatch("encode", lens.size, total)
    genc.load(lens, src)
    genc.replay()
    torch.cuda.synchronize()
    enc_dst, enc_off, enc_len, _ = genc.results()
    tlens = 4 * ((lens + 2) // 3)
    assert np.array_equal(enc_len.cpu().numpy(), tlens)
    ntext = int(tlens.sum())
    gdec = GraphBatch("decode", lens.size, ntext)
    gdec.load(tlens, enc_dst[:ntext])
    gdec.replay()
    torch.cuda.synchronize()
    _, _, dlen, dbad = gdec.results()
    assert np.array_equal(dlen.cpu().numpy(), lens) and (dbad.cpu().numpy() == -1).all()
    t_enc = _events_time(torch, genc.replay, steps)
    t_dec = _events_time(torch, gdec.replay, steps)
    # one launch per buffer, same stream, no graph
    L = _lib.load()
    alpha = ctypes.create_string_buffer(b64.STD, 64)
    stream = b64.stream_ptr()
    sp, dp = src.data_ptr(), enc_dst.data_ptr()
    per_dst = torch.empty(int(gdec.host_out_off[-1]) + 1, dtype=torch.uint8, device="cuda")
    stat = torch.empty(2 * lens.size, dtype=torch.int64, device="cuda")
    pp, stp = per_dst.data_ptr(), stat.data_ptr()
    ioff = in_off.tolist(); eol = genc.host_out_off.tolist(); dol = gdec.host_out_off.tolist()
    ll = lens.tolist(); tl = tlens.tolist()

    def per_enc():
        for b in range(len(ll)):
            L.b64_encode(sp + ioff[b], ll[b], dp + eol[b], alpha, stream)

    def per_dec():
        for b in range(len(ll)):
            L.b64_decode_async(dp + eol[b], tl[b], pp + dol[b], stp + 16 * b, stp + 16 * b + 8,
                               alpha, stream)

    res = {"workload": "ragged batch: log-uniform 16 B .. 1 MiB", "buffers": int(lens.size),
           "bytes": total, "chars": ntext}
    for name, fn, tb in (("encode", per_enc, t_enc), ("decode", per_dec, t_dec)):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = a.elapsed_time(b)
        res[name] = {"batched_ms": round(tb["median"], 4),
                     "batched_gbps_b64": round(ntext / tb["median"] / 1e6, 1),
                     "batched_hbm_gbps": round((total + ntext) / tb["median"] / 1e6, 1),
                     "per_buffer_ms": round(gpu_ms, 3), "per_buffer_wall_ms": round(wall * 1e3, 3),
                     "per_buffer_gbps_b64": round(ntext / gpu_ms / 1e6, 2),
                     "speedup": round(gpu_ms / tb["median"], 1)}
        log("batch", name, json.dumps(res[name]))
    st = stat.view(-1, 2).cpu().numpy()
    assert np.array_equal(st[:, 0], lens) and (st[:, 1] == -1).all()
    del per_dst, stat
    if same_bytes:
        # yardstick: the packed input as ONE buffer, the same bytes to move, so
        # that the batched rates can be told apart from the cost of the footprint
        text1 = b64.encode(src)
        out1, st1 = b64.decode_async(text1)
        torch.cuda.synchronize()
        assert st1.cpu().tolist() == [total, -1]
        t1e = _events_time(torch, lambda: b64.encode(src, out=text1), steps)
        t1d = _events_time(torch, lambda: b64.decode_async(text1, out=out1, status=st1), steps)
        n1 = int(text1.numel())
        res["one_buffer_same_bytes"] = {
            "chars": n1, "encode_ms": t1e["median"], "decode_ms": t1d["median"],
            "encode_hbm_gbps": (total + n1) / t1e["median"] / 1e6,
            "decode_hbm_gbps": (total + n1) / t1d["median"] / 1e6}
        log("batch one buffer", json.dumps(res["one_buffer_same_bytes"]))
    del genc, gdec, src
    torch.cuda.empty_cache()
    return res


def run_batch(args, torch, b64):
    """100,000 ragged buffers (log-uniform 16 B .. 1 MiB): one graph-captured
    batched launch per direction vs one launch per buffer on one stream."""
    print(json.dumps(batch_measure(torch, b64, args.nbuf, args.steps)), flush=True)


def serve_requests(torch, b64, count: int):
    """The serving workload's requests (without arrival times): sizes
    log-normal (median 8 KiB, sigma 1.5) clipped to [1 B, 16 MiB], 50/50
    encode / decode, 1% of decodes spoiled by one byte outside the alphabet.
    Decode payloads are encodings of random bytes (made on the GPU with the
    batched encode).  Returns kinds, packed host payloads, their offsets, the
    raw lengths and the indices of the spoiled requests."""
    seed = workloads.SEED_BASE + 5
    sizes = workloads.serve_sizes(seed, count)
    is_dec, is_bad = workloads.serve_kinds(seed + 1, count)
    raw = workloads.random_bytes(seed + 3, int(sizes.sum()))
    roff = workloads.offsets(sizes)
    dec_idx = np.nonzero(is_dec)[0]
    # encodings of the decode requests' bytes, one batched launch
    draw = np.concatenate([raw[roff[i]:roff[i + 1]] for i in dec_idx]) if dec_idx.size else raw[:0]
    d_in = torch.from_numpy(draw if draw.size else np.zeros(1, np.uint8)).cuda()
    dtext, doff, _ = b64.encode_batch(d_in, torch.from_numpy(workloads.offsets(sizes[dec_idx])).cuda())
    dtext = dtext.cpu().numpy()
    doff = doff.cpu().numpy()
    lens = sizes.copy()
    lens[dec_idx] = np.diff(doff)
    off = workloads.offsets(lens)
    payload = np.empty(int(off[-1]), dtype=np.uint8)
    enc_idx = np.nonzero(~is_dec)[0]
    for i in enc_idx:
        payload[off[i]:off[i + 1]] = raw[roff[i]:roff[i + 1]]
    for k, i in enumerate(dec_idx):
        payload[off[i]:off[i + 1]] = dtext[doff[k]:doff[k + 1]]
    g = workloads.rng(seed + 4)
    bad_bytes = workloads.non_alphabet_bytes(b64.STD)
    spoil = np.nonzero(is_bad)[0]
    for i in spoil:
        if off[i + 1] > off[i]:
            payload[off[i] + int(g.integers(0, off[i + 1] - off[i]))] = bad_bytes[g.integers(0, bad_bytes.size)]
    return is_dec.astype(np.int32), payload, off, sizes, spoil


def serve_rate(srv, torch, b64, kinds, payload, off, sizes, spoil, rate, count):
    """Serve the first `count` requests at Poisson rate `rate`; check every
    status; return the run's summary."""
    seed = workloads.SEED_BASE + 5
    arrival = workloads.serve_arrivals(seed + 2, count, rate)
    arrival -= arrival[0]
    res = srv.run(kinds[:count], arrival, payload, off[:count + 1])
    enc = kinds[:count] == 0
    sp = spoil[spoil < count]
    ok = np.ones(count, dtype=bool)
    ok[sp] = False
    want_len = np.where(enc, 4 * ((sizes[:count] + 2) // 3), sizes[:count])
    assert np.array_equal(res.out_len[ok], want_len[ok]) and (res.first_bad[ok] == -1).all()
    assert (res.first_bad[sp] >= 0).all() and (res.out_len[sp] == -1).all()
    summ = {"rate": rate, **res.summary(), "invalid": int(sp.size)}
    return summ


def run_serve(args, torch, b64):
    """Poisson arrivals of mixed encode/decode requests through the native
    continuous-batching server at swept rates (at least 100,000 requests or
    10 s of arrivals per rate), payloads starting in pinned host memory."""
    from paper_1910_05109_amd import serve
    count_max = args.requests
    log("serve: making", count_max, "requests")
    kinds, payload, off, sizes, spoil = serve_requests(torch, b64, count_max)
    out = []
    with serve.Server(budget_bytes=32 << 30, nstreams=args.serve_streams,
                      depth=args.serve_depth, zero_copy_max=args.serve_zero_copy_max,
                      staging=args.serve_staging) as srv:
        for rate in args.rates:
            count = int(min(count_max, max(2000, rate * args.seconds)))
            summ = serve_rate(srv, torch, b64, kinds, payload, off, sizes, spoil, rate, count)
            log("serve", json.dumps(summ))
            out.append(summ)
    print(json.dumps({"workload": "serving", "sigma": workloads.SERVE_SIGMA,
                      "streams": args.serve_streams, "depth": args.serve_depth,
                      "zero_copy_max": args.serve_zero_copy_max, "staging": args.serve_staging,
                      "rows": out}),
          flush=True)


def run_validate(args, torch, b64):
    """Read-only validation of the 1 GiB workload's encoding, against decode."""
    n = workloads.SINGLE_1GIB[0]
    N = 4 * ((n + 2) // 3)
    x = torch.from_numpy(workloads.random_bytes(workloads.SEED_BASE + 2, n)).cuda()
    text = b64.encode(x)
    dec = torch.empty(n + 3, dtype=torch.uint8, device="cuda")
    st = torch.empty(2, dtype=torch.int64, device="cuda")
    val = lambda: b64.validate_async(text, status=st)
    dcd = lambda: b64.decode_async(text, out=dec, status=st)
    for _ in range(3):
        val(); dcd()
    tv = _events_time(torch, val, args.steps)
    td = _events_time(torch, dcd, args.steps)
    assert st.cpu().tolist() == [n, -1]
    res = {"workload": "validate 1 GiB encoding", "n_chars": N,
           "validate_ms": tv["median"], "validate_gbps_b64": N / tv["median"] / 1e6,
           "validate_hbm_frac": N / tv["median"] / 1e6 / HBM_PEAK_GBS,
           "decode_ms": td["median"], "decode_gbps_b64": N / td["median"] / 1e6}
    print(json.dumps(res), flush=True)


def run_host(args, torch, b64):
    """The 1 GiB workload starting and ending in host memory, through the
    chunked host -> device -> host pipeline; PCIe included."""
    from paper_1910_05109_amd.pipeline import HostPipeline
    n = workloads.SINGLE_1GIB[0]
    N = 4 * ((n + 2) // 3)
    x = workloads.random_bytes(workloads.SEED_BASE + 2, n)
    text = np.empty(N, dtype=np.uint8)
    dec = np.empty(n + 3, dtype=np.uint8)
    res = {"workload": "1 GiB in host memory, pipelined through the GPU", "n_bytes": n, "n_chars": N}
    with HostPipeline(chunk_bytes=args.chunk_mib << 20, depth=args.host_depth, host_threads=8) as p:
        p.encode(x[: 64 << 20], out=text)            # warm-up
        te = []
        td = []
        for _ in range(3):
            t0 = time.perf_counter()
            p.encode(x, out=text)
            te.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            out, bad = p.decode(text, out=dec)
            td.append(time.perf_counter() - t0)
            assert bad is None and out.size == n
        # the same calls with source and destination in pinned host memory:
        # the pipeline then copies straight between them and the device
        px = torch.empty(n, dtype=torch.uint8, pin_memory=True).numpy()
        ptext = torch.empty(N, dtype=torch.uint8, pin_memory=True).numpy()
        pdec = torch.empty(n + 3, dtype=torch.uint8, pin_memory=True).numpy()
        px[:] = x
        tpe = []
        tpd = []
        for _ in range(3):
            t0 = time.perf_counter()
            p.encode(px, out=ptext)
            tpe.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            out, bad = p.decode(ptext, out=pdec)
            tpd.append(time.perf_counter() - t0)
            assert bad is None and out.size == n
        assert np.array_equal(ptext, text) and np.array_equal(pdec[:n], x)
        del px, ptext, pdec, out
    # reference: the same bytes over PCIe with pinned torch copies (no codec)
    h_in = torch.empty(n, dtype=torch.uint8).pin_memory()
    h_out = torch.empty(N, dtype=torch.uint8).pin_memory()
    d_in = torch.empty(n, dtype=torch.uint8, device="cuda")
    d_out = torch.empty(N, dtype=torch.uint8, device="cuda")
    t0 = time.perf_counter()
    d_in.copy_(h_in, non_blocking=True)
    torch.cuda.synchronize()
    t_h2d = time.perf_counter() - t0
    t0 = time.perf_counter()
    h_out.copy_(d_out, non_blocking=True)
    torch.cuda.synchronize()
    t_d2h = time.perf_counter() - t0
    # both at once on two streams: the floor for a 1 GiB encode host -> host
    # (a decode moves the same bytes the other way)
    s_in, s_out = torch.cuda.Stream(), torch.cuda.Stream()
    t_both = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s_in):
            d_in.copy_(h_in, non_blocking=True)
        with torch.cuda.stream(s_out):
            h_out.copy_(d_out, non_blocking=True)
        torch.cuda.synchronize()
        t_both.append(time.perf_counter() - t0)
    res.update({"encode_s": min(te), "encode_gbps_b64": N / min(te) / 1e9,
                "decode_s": min(td), "decode_gbps_b64": N / min(td) / 1e9,
                "pinned_encode_s": min(tpe), "pinned_encode_gbps_b64": N / min(tpe) / 1e9,
                "pinned_decode_s": min(tpd), "pinned_decode_gbps_b64": N / min(tpd) / 1e9,
                "pcie_h2d_gbps": n / t_h2d / 1e9, "pcie_d2h_gbps": N / t_d2h / 1e9,
                "pcie_both_s": min(t_both), "pcie_both_gbps_b64": N / min(t_both) / 1e9,
                "pinned_encode_frac_of_both": min(t_both) / min(tpe),
                "chunk_mib": args.chunk_mib, "depth": args.host_depth})
    print(json.dumps(res), flush=True)


def run_variants(args, torch, b64):
    """The 1 GiB payload through the variants: unpadded encode / decode, and
    MIME text (lines of 76 characters, CR LF) through the line-wrapped encode
    and the whitespace-skipping decode and validate.  Algorithmic bytes are
    what any codec must move (input + output).  Regular lines take the checked
    decode (one read of the text); the same text with one space inserted near
    its start takes the counted path, which reads the text twice by design
    (count pass, then decode pass)."""
    n = args.variants_bytes or workloads.SINGLE_1GIB[0]
    L = workloads.MIME_LINE
    x = torch.from_numpy(workloads.random_bytes(workloads.SEED_BASE + 2, n)).cuda()
    size = "1 GiB payload" if n == workloads.SINGLE_1GIB[0] else f"{n}-byte payload"
    res = {"workload": f"{size}: unpadded; MIME text (76-char lines, CR LF)", "n_bytes": n}
    # unpadded
    Nn = b64.encoded_len(n, b64.NOPAD)
    tn = torch.empty(Nn, dtype=torch.uint8, device="cuda")
    dn = torch.empty(n + 3, dtype=torch.uint8, device="cuda")
    st = torch.empty(2, dtype=torch.int64, device="cuda")
    enc = lambda: b64.encode(x, out=tn, flags=b64.NOPAD)
    dec = lambda: b64.decode_async(tn, out=dn, status=st, flags=b64.NOPAD)
    for _ in range(3):
        enc(); dec()
    te, td = _events_time(torch, enc, args.steps), _events_time(torch, dec, args.steps)
    assert st.cpu().tolist() == [n, -1] and torch.equal(dn[:n], x)
    res["nopad"] = {"n_chars": Nn, "encode_ms": te["median"], "decode_ms": td["median"],
                    "encode_hbm_frac": (n + Nn) / te["median"] / 1e6 / HBM_PEAK_GBS,
                    "decode_hbm_frac": (n + Nn) / td["median"] / 1e6 / HBM_PEAK_GBS}
    del tn, dn
    # MIME
    M = b64.encoded_len(n, 0, L)
    tm = torch.empty(M, dtype=torch.uint8, device="cuda")
    dm = torch.empty(b64.decoded_max_len(M, b64.SKIP_WS), dtype=torch.uint8, device="cuda")
    ws = torch.empty(b64.workspace_size(M, b64.SKIP_WS), dtype=torch.uint8, device="cuda")
    wenc = lambda: b64.encode(x, out=tm, line_len=L)
    wdec = lambda: b64.decode_async(tm, out=dm, status=st, flags=b64.SKIP_WS, workspace=ws)
    wval = lambda: b64.validate_async(tm, status=st, flags=b64.SKIP_WS, workspace=ws)
    for _ in range(3):
        wenc(); wdec()
    tw = _events_time(torch, wenc, args.steps)
    tdw = _events_time(torch, wdec, args.steps)
    assert st.cpu().tolist() == [n, -1] and torch.equal(dm[:n], x)
    tv = _events_time(torch, wval, args.steps)
    assert st.cpu().tolist() == [n, -1]
    # the counted path: one extra space near the start breaks the regular layout
    tm2 = torch.cat([tm[:1000], torch.full((1,), ord(" "), dtype=torch.uint8, device="cuda"), tm[1000:]])
    ws2 = torch.empty(b64.workspace_size(M + 1, b64.SKIP_WS), dtype=torch.uint8, device="cuda")
    dm2 = torch.empty(b64.decoded_max_len(M + 1, b64.SKIP_WS), dtype=torch.uint8, device="cuda")
    wdec2 = lambda: b64.decode_async(tm2, out=dm2, status=st, flags=b64.SKIP_WS, workspace=ws2)
    wdec2()
    tdc = _events_time(torch, wdec2, args.steps)
    assert st.cpu().tolist() == [n, -1] and torch.equal(dm2[:n], x)
    del tm2, dm2, ws2
    res["mime"] = {"n_chars": M, "line_len": L,
                   "wrap_encode_ms": tw["median"], "wrap_encode_gbps_b64": M / tw["median"] / 1e6,
                   "wrap_encode_hbm_frac": (n + M) / tw["median"] / 1e6 / HBM_PEAK_GBS,
                   "ws_decode_ms": tdw["median"], "ws_decode_gbps_b64": M / tdw["median"] / 1e6,
                   "ws_decode_hbm_frac_alg": (M + n) / tdw["median"] / 1e6 / HBM_PEAK_GBS,
                   "ws_decode_counted_ms": tdc["median"],
                   "ws_decode_counted_hbm_frac_alg": (M + n) / tdc["median"] / 1e6 / HBM_PEAK_GBS,
                   "ws_decode_counted_hbm_frac_design": (2 * M + n) / tdc["median"] / 1e6 / HBM_PEAK_GBS,
                   "ws_validate_ms": tv["median"], "ws_validate_gbps_b64": M / tv["median"] / 1e6}
    print(json.dumps(res), flush=True)


def run_fused(args, torch, b64):
    """Decode fused into its consumer: 65,536 rows of base64 float32 (1,536
    per row, the size of a common text-embedding vector) straight into a
    bfloat16 tensor, against decoding the rows to bytes (one batched launch)
    and converting them with torch in a second pass."""
    dim, nrows = 1536, 65536
    raw = torch.from_numpy(workloads.random_bytes(workloads.SEED_BASE + 250, 4 * dim * nrows)).cuda()
    in_off = torch.from_numpy(workloads.offsets(np.full(nrows, 4 * dim, dtype=np.int64))).cuda()
    text, t_off, _ = b64.encode_batch(raw, in_off)            # the rows' base64 text
    t_off = t_off.clone()
    N = int(t_off[-1].item())
    text = text[:N]
    out = torch.empty((nrows, dim), dtype=torch.bfloat16, device="cuda")
    st = torch.empty(nrows, dtype=torch.int64, device="cuda")
    fused = lambda: b64.decode_f32_bf16(text, t_off, dim, dst=out, status=st, validate=False)
    dbytes = torch.empty(nrows * 4 * dim + 16, dtype=torch.uint8, device="cuda")
    d_off = torch.arange(nrows + 1, dtype=torch.int64, device="cuda") * (4 * dim)
    dlen = torch.empty(nrows, dtype=torch.int64, device="cuda")
    dbad = torch.empty(nrows, dtype=torch.int64, device="cuda")
    out2 = torch.empty((nrows, dim), dtype=torch.bfloat16, device="cuda")

    def unfused():
        b64.decode_batch(text, t_off, dst=dbytes, out_off=d_off, out_len=dlen, first_bad=dbad,
                         validate=False)
        out2.copy_(dbytes[: nrows * 4 * dim].view(torch.float32).view(nrows, dim))

    for _ in range(3):
        fused(); unfused()
    for _ in range(10):
        fused()
    tf = _events_time(torch, fused, args.steps)
    for _ in range(5):
        unfused()
    tu = _events_time(torch, unfused, args.steps)
    assert bool((st == -1).all()) and bool((dbad == -1).all())
    keep = ~torch.isnan(out2)                                # NaN encodings differ by convention
    assert torch.equal(out.view(torch.int16)[keep], out2.view(torch.int16)[keep])
    fb = N + 2 * nrows * dim                                 # algorithmic bytes of the fused kernel
    ub = N + 2 * 4 * nrows * dim + 2 * nrows * dim           # decode to bytes, then convert
    res = {"workload": f"{nrows} rows of base64 float32 x {dim} -> bfloat16", "n_chars": N,
           "fused_ms": tf["median"], "fused_min_ms": tf["min"], "fused_gbps_b64": N / tf["median"] / 1e6,
           "fused_hbm_frac": fb / tf["median"] / 1e6 / HBM_PEAK_GBS,
           "unfused_ms": tu["median"], "unfused_gbps_b64": N / tu["median"] / 1e6,
           "speedup": tu["median"] / tf["median"], "bytes_fused": fb, "bytes_unfused": ub}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="single",
                    choices=["single", "ceiling", "small", "sweep", "batch", "serve", "validate",
                             "host", "variants", "fused"])
    ap.add_argument("--chunk-mib", type=int, default=64)
    ap.add_argument("--variants-bytes", type=int, default=0,
                    help="variants: payload bytes (default: the 1 GiB workload)")
    ap.add_argument("--host-depth", type=int, default=3, help="host pipeline: chunks in flight")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="default line without its batch and serve objects")
    ap.add_argument("--cpu-sample", type=int, default=512 << 20)
    ap.add_argument("--cpu-reps", type=int, default=5)
    ap.add_argument("--nbuf", type=int, default=workloads.BATCH_BUFFERS)
    ap.add_argument("--rates", type=float, nargs="+",
                    default=[1e3, 3e3, 1e4, 3e4, 1e5, 2e5, 3e5, 5e5, 1e6, 2e6])
    ap.add_argument("--requests", type=int, default=100_000)
    ap.add_argument("--seconds", type=float, default=10.0)
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-depth", type=int, default=2, help="launches in flight at most")
    ap.add_argument("--serve-staging", choices=["auto", "kernels", "dma"], default=None,
                    help="staged launches: copy kernels up to 1 MiB then DMA (auto, the default), "
                         "copy kernels or DMA")
    ap.add_argument("--serve-zero-copy-max", type=int, default=None,
                    help="payload bytes of a launch at most for zero-copy (0: off; default: the library's)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1910_05109_amd as b64
    b64.load()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    {"single": run_single, "ceiling": run_ceiling, "small": run_small, "sweep": run_sweep,
     "batch": run_batch,
     "serve": run_serve, "validate": run_validate, "host": run_host,
     "variants": run_variants, "fused": run_fused}[args.mode](args, torch, b64)


if __name__ == "__main__":
    main()
