"""Self-written autotuner for the launch shape of each operation.

The shape of a launch is (unroll, blocks_per_cu, nontemporal): `unroll` lane chunks in
flight per lane (a lane chunk is 12 bytes -> 16 characters for encode and
16 characters -> 12 bytes for decode, so unroll 4 is the paper's 48 -> 64
block) and `blocks_per_cu` workgroups of 256 threads per compute unit (the
grid-stride and persistent kernels loop over the rest).  The tuner times every
shape of a grid with HIP events on the launch stream (median of `reps`
launches after warm-up), keeps the fastest, applies it with b64_tune_set and
stores it in a JSON cache keyed by device name and operation.

  python -m paper_1910_05109_amd.tune [--ops encode decode ...] [--mib 256]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics

import numpy as np

from . import (OPS, SKIP_WS, STD, decode_async, decode_batch, encode, encode_batch, tune_get,
               tune_set, validate_async, workspace_size)

UNROLLS = (1, 2, 4, 8)
BLOCKS_PER_CU = (1, 2, 4, 8, 16, 32)
NONTEMPORAL = (0, 1)
CACHE = os.environ.get("B64HIP_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "b64hip", "tune.json"))


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|cu{p.multi_processor_count}"


def _time(torch, fn, reps):
    for _ in range(3):
        fn()
    pairs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        pairs.append((a, b))
    torch.cuda.synchronize()
    return statistics.median(x.elapsed_time(y) for x, y in pairs)


def _workload(torch, op, nbytes, seed=191005109):
    """A launch closure for `op` over about `nbytes` input bytes."""
    g = np.random.Generator(np.random.PCG64(seed))
    x = torch.from_numpy(g.integers(0, 256, size=nbytes, dtype=np.uint8)).cuda()
    text = encode(x, STD)
    torch.cuda.synchronize()
    if op == "encode":
        out = torch.empty_like(text)
        return lambda: encode(x, STD, out=out)
    if op == "decode":
        out = torch.empty(3 * (text.numel() // 4), dtype=torch.uint8, device="cuda")
        st = torch.empty(2, dtype=torch.int64, device="cuda")
        return lambda: decode_async(text, STD, out=out, status=st)
    if op == "validate":
        st = torch.empty(2, dtype=torch.int64, device="cuda")
        return lambda: validate_async(text, STD, status=st)
    if op in ("encode_wrap", "decode_ws"):
        # MIME text: lines of 76 characters separated by CR LF
        mime = encode(x, STD, line_len=76)
        if op == "encode_wrap":
            out = torch.empty_like(mime)
            return lambda: encode(x, STD, out=out, line_len=76)
        out = torch.empty(3 * (mime.numel() // 4), dtype=torch.uint8, device="cuda")
        st = torch.empty(2, dtype=torch.int64, device="cuda")
        ws = torch.empty(workspace_size(mime.numel(), SKIP_WS), dtype=torch.uint8, device="cuda")
        return lambda: decode_async(mime, STD, out=out, status=st, flags=SKIP_WS, workspace=ws)
    # ragged batches: log-uniform lengths in [16, 1 MiB) up to nbytes in total
    lens = []
    total = 0
    while total < nbytes:
        n = int(16 * (65536 ** g.random()))
        lens.append(n)
        total += n
    lens = np.array(lens, dtype=np.int64)
    off = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    src = torch.from_numpy(g.integers(0, 256, size=int(off[-1]), dtype=np.uint8)).cuda()
    d_off = torch.from_numpy(off).cuda()
    dst, out_off, out_len = encode_batch(src, d_off, STD)
    if op == "encode_batch":
        return lambda: encode_batch(src, d_off, STD, dst=dst, out_off=out_off, out_len=out_len)
    ddst, dout_off, dlen, dbad = decode_batch(dst, out_off, STD)
    return lambda: decode_batch(dst, out_off, STD, dst=ddst, out_off=dout_off, out_len=dlen,
                                first_bad=dbad)


# the whitespace-skipping decode keeps 1, 2 or 4 rounds of loads in flight per
# wave; 64 VGPRs and 8.5 KiB of LDS per workgroup fit 8 workgroups per CU
GRIDS = {"decode_ws": {"unrolls": (1, 2, 4), "bpcs": (2, 4, 6, 8, 12, 16)}}


def tune_op(op: str, nbytes: int, reps: int = 10, unrolls=UNROLLS, bpcs=BLOCKS_PER_CU,
            nts=NONTEMPORAL, verbose: bool = True):
    import torch
    unrolls = GRIDS.get(op, {}).get("unrolls", unrolls)
    bpcs = GRIDS.get(op, {}).get("bpcs", bpcs)
    fn = _workload(torch, op, nbytes)
    old = tune_get(op)
    results = []
    for nt in nts:
        for u in unrolls:
            for b in bpcs:
                tune_set(op, u, b, nt)
                ms = _time(torch, fn, reps)
                results.append((ms, u, b, nt))
                if verbose:
                    print(f"[tune] {op:13s} unroll={u} blocks/cu={b:2d} nt={nt}: {ms:.4f} ms",
                          flush=True)
    results.sort()
    ms, u, b, nt = results[0]
    tune_set(op, u, b, nt)
    return {"unroll": u, "blocks_per_cu": b, "nontemporal": nt, "ms": ms, "bytes": nbytes,
            "previous": list(old), "grid": [[r[1], r[2], r[3], r[0]] for r in results]}


def save(entries: dict, path: str = CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data.setdefault(device_key(), {}).update(entries)
    with open(path, "w") as f:
        json.dump(data, f, indent=1)


def apply_cached(path: str = CACHE) -> dict:
    """Apply cached shapes for the current device, if any; returns them."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    ent = data.get(device_key(), {})
    for op, v in ent.items():
        if op in OPS:
            tune_set(op, int(v["unroll"]), int(v["blocks_per_cu"]), int(v.get("nontemporal", 1)))
    return ent


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ops", nargs="+", default=list(OPS))
    ap.add_argument("--mib", type=int, default=256, help="input MiB per timed launch")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--json", default=None, help="also write the full sweep here")
    args = ap.parse_args()
    found = {}
    for op in args.ops:
        found[op] = tune_op(op, args.mib << 20, args.reps)
        print(f"[tune] best {op}: unroll={found[op]['unroll']} "
              f"blocks/cu={found[op]['blocks_per_cu']} nt={found[op]['nontemporal']} "
              f"{found[op]['ms']:.4f} ms", flush=True)
    keys = ("unroll", "blocks_per_cu", "nontemporal", "ms", "bytes")
    save({k: {kk: v[kk] for kk in keys} for k, v in found.items()}, args.out)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(found, f, indent=1)


if __name__ == "__main__":
    main()
