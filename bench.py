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
launch stream, against the 8 TB/s HBM peak), and the oracle's CPU throughput
on a bounded sample.

Other modes (--mode): sweep (size sweep 2^k + r), batch (100,000 ragged
buffers, batched launch vs one launch per buffer), serve (continuous batching
loop), small (the 3 MiB workload).  Each prints its own JSON lines.
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
KERNEL_SRC = os.path.join(ROOT, "paper_1910_05109_amd", "csrc", "b64hip.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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
    """The oracle (single thread, as it stands) on the first `sample_bytes`
    bytes: encode then decode, median of `reps`; GB/s of base64 characters
    over both directions, like the GPU value."""
    import oracle
    xs = np.ascontiguousarray(x[:sample_bytes])
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        text = oracle.encode(xs)
        dec, bad = oracle.decode(text)
        times.append(time.perf_counter() - t0)
        assert bad is None and dec.size == xs.size
    t = statistics.median(times)
    nchar = 4 * ((sample_bytes + 2) // 3)
    return {"value": round(2 * nchar / t / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample_bytes} bytes of the 1 GiB input, encode+decode, "
                      f"median of {reps}, 1 thread ({os.cpu_count()} host cpus visible)"}


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
                     "traffic": measured_traffic(kname, alg)},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(x, args.cpu_sample, args.cpu_reps)
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="single", choices=["single"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-sample", type=int, default=512 << 20)
    ap.add_argument("--cpu-reps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this codec shards without exchanging payload "
              "(see the design notes); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1910_05109_amd as b64
    b64.load()
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.mode == "single":
        run_single(args, torch, b64)


if __name__ == "__main__":
    main()
