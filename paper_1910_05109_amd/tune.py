"""Self-written autotuner for the launch shape of each operation and size.

The shape of a launch is (unroll, blocks_per_cu, nontemporal): `unroll` lane
chunks in flight per lane (a lane chunk is 12 bytes -> 16 characters for
encode and 16 characters -> 12 bytes for decode, so unroll 4 is the paper's
48 -> 64 block) and `blocks_per_cu` workgroups of 256 threads per compute
unit (an input that fewer workgroups cover in one round gets just those; the
grid-stride and persistent kernels loop over the rest).  The library keeps one
shape per operation and size bucket of the input (below 64 KiB, below 1 MiB,
below 16 MiB, below 128 MiB, larger); the batched and fused operations use
the last bucket only.

The tuner times every shape of a grid with HIP events on the launch stream
on three input sizes spread over each bucket (one for the last) -- below
16 MiB per call replayed from a HIP graph (the device time, which the host's
launch cost would otherwise hide), above it per call in groups of
back-to-back calls.  A bucket spans up to 16x in size and the best shape
moves within it (more workgroups pay off at its small end, fewer at its
large end), so each shape is scored by its time relative to the fastest
shape at each size, averaged over the sizes, and the lowest score is kept.
It is applied with b64_tune_set_bucket and stored in a JSON cache keyed by
device, operation and bucket.  The package applies
the cache of the current device when it loads the library (load()), from
$B64HIP_TUNE_CACHE or ~/.cache/b64hip/tune.json; B64HIP_TUNE_CACHE=off
skips it.  Every shape the grid holds is covered by the launch-shape parity
tests, so a cached choice cannot change results.

  python -m paper_1910_05109_amd.tune [--ops encode decode ...] [--buckets 0 1 2 3]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics

import numpy as np

from . import (BUCKETS, OPS, SKIP_WS, STD, decode_async, decode_batch, decode_f32_bf16, encode,
               encode_batch, tune_get, tune_set, tune_ws_guess_min, tune_ws_small_max,
               validate_async, workspace_size)

UNROLLS = (1, 2, 4, 8)
BLOCKS_PER_CU = (1, 2, 4, 8, 16, 32, 64)
NONTEMPORAL = (0, 1)
# input sizes timed per bucket (bytes of the operation's input), spread over
# the bucket's range: < 64 KiB, < 1 MiB, < 16 MiB, < 128 MiB, larger
BUCKET_SIZES = ((4 << 10, 16 << 10, 48 << 10), (96 << 10, 256 << 10, 768 << 10),
                (2 << 20, 4 << 20, 12 << 20), (24 << 20, 48 << 20, 96 << 20), (1 << 30,))
# operations whose total size is known only on the device: last bucket only
LAST_BUCKET_ONLY = ("encode_batch", "decode_batch", "decode_f32_bf16")
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "b64hip", "tune.json")
# the whitespace-skipping decode keeps 1, 2 or 4 rounds of loads in flight per
# wave; 64 VGPRs and 8.5 KiB of LDS per workgroup fit 8 workgroups per CU
GRIDS = {"decode_ws": {"unrolls": (1, 2, 4), "bpcs": (2, 4, 6, 8, 12, 16)}}


def cache_path() -> str | None:
    p = os.environ.get("B64HIP_TUNE_CACHE", DEFAULT_CACHE)
    return None if p.lower() in ("", "off", "none", "0") else p


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|cu{p.multi_processor_count}"


def _graph_time(torch, fn, reps, inner=20):
    """Milliseconds per call of `fn` replayed from a HIP graph of `inner`
    calls (median of `reps` replays): the device time of a call without the
    host's launch cost, which would hide the kernels of small calls."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(inner):
            fn()
    g.replay()
    torch.cuda.synchronize()
    pairs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        pairs.append((a, b))
    torch.cuda.synchronize()
    del g
    return statistics.median(x.elapsed_time(y) for x, y in pairs) / inner


def _time(torch, fn, reps, inner=None):
    """Milliseconds per call of `fn` in a stream of back-to-back calls: the
    median over `reps` groups of `inner` calls between two HIP events (more
    calls per group for short calls, so that event and launch noise average
    out)."""
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    if inner is None:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        inner = max(1, min(50, int(1.0 / max(a.elapsed_time(b), 1e-3))))
    pairs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(inner):
            fn()
        b.record()
        pairs.append((a, b))
    torch.cuda.synchronize()
    return statistics.median(x.elapsed_time(y) for x, y in pairs) / inner


def _workload(torch, op, nbytes, seed=191005109):
    """A launch closure for `op` over `nbytes` input bytes (text bytes for the
    decoding operations), uniform random data made on the device."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)

    def rand(n):
        return torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=gen)

    if op in ("encode", "encode_wrap"):
        x = rand(nbytes)
        line = 76 if op == "encode_wrap" else 0
        out = encode(x, STD, line_len=line)
        return lambda: encode(x, STD, out=out, line_len=line)
    if op in ("decode", "validate"):
        text = encode(rand(nbytes * 3 // 4))
        st = torch.empty(2, dtype=torch.int64, device="cuda")
        if op == "validate":
            return lambda: validate_async(text, STD, status=st)
        out = torch.empty(max(3 * (text.numel() // 4), 1), dtype=torch.uint8, device="cuda")
        return lambda: decode_async(text, STD, out=out, status=st)
    if op == "decode_ws":
        # MIME text: lines of 76 characters separated by CR LF
        mime = encode(rand(nbytes * 3 * 76 // (4 * 78)), STD, line_len=76)
        out = torch.empty(max(3 * (mime.numel() // 4), 1), dtype=torch.uint8, device="cuda")
        st = torch.empty(2, dtype=torch.int64, device="cuda")
        ws = torch.empty(max(workspace_size(mime.numel(), SKIP_WS), 1), dtype=torch.uint8,
                         device="cuda")
        return lambda: decode_async(mime, STD, out=out, status=st, flags=SKIP_WS, workspace=ws)
    if op == "decode_f32_bf16":
        dim = 1536
        nrows = max(1, nbytes // (4 * dim * 4 // 3))
        raw = rand(4 * dim * nrows)
        r_off = torch.arange(nrows + 1, dtype=torch.int64, device="cuda") * (4 * dim)
        text, t_off, _ = encode_batch(raw, r_off, STD)
        t_off = t_off.clone()
        dst = torch.empty((nrows, dim), dtype=torch.bfloat16, device="cuda")
        st = torch.empty(nrows, dtype=torch.int64, device="cuda")
        return lambda: decode_f32_bf16(text, t_off, dim, STD, dst=dst, status=st, validate=False)
    # ragged batches: log-uniform lengths in [16, 1 MiB) up to nbytes in total
    g = np.random.Generator(np.random.PCG64(seed))
    lens, total = [], 0
    while total < nbytes:
        n = int(16 * (65536 ** g.random()))
        lens.append(n)
        total += n
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(np.array(lens, dtype=np.int64), out=off[1:])
    src = rand(int(off[-1]))
    d_off = torch.from_numpy(off).cuda()
    dst, out_off, out_len = encode_batch(src, d_off, STD)
    if op == "encode_batch":
        return lambda: encode_batch(src, d_off, STD, dst=dst, out_off=out_off, out_len=out_len,
                                    validate=False)
    ddst, dout_off, dlen, dbad = decode_batch(dst, out_off, STD)
    return lambda: decode_batch(dst, out_off, STD, dst=ddst, out_off=dout_off, out_len=dlen,
                                first_bad=dbad, validate=False)


def buckets_of(op: str) -> tuple[int, ...]:
    return (BUCKETS - 1,) if op in LAST_BUCKET_ONLY else tuple(range(BUCKETS))


def tune_op(op: str, bucket: int, nbytes: int | None = None, reps: int = 10, unrolls=UNROLLS,
            bpcs=BLOCKS_PER_CU, nts=NONTEMPORAL, verbose: bool = True) -> dict:
    """Time every shape of the grid for `op` in size `bucket` (on inputs of
    the bucket's sizes, or of `nbytes` alone), apply the shape with the lowest
    mean time relative to the fastest shape at each size, and return it with
    the whole grid."""
    import torch
    unrolls = GRIDS.get(op, {}).get("unrolls", unrolls)
    bpcs = GRIDS.get(op, {}).get("bpcs", bpcs)
    sizes = BUCKET_SIZES[bucket] if nbytes is None else (nbytes,)
    old = tune_get(op, bucket)
    times = {}                                   # shape -> ms per size
    # the whitespace-skipping decode's shape is the multi-launch path's: small
    # texts would otherwise take the one-workgroup path, which has no shape
    small_old = tune_ws_small_max(0) if op == "decode_ws" else None
    try:
        for size in sizes:
            fn = _workload(torch, op, size)
            try:
                _sweep(torch, op, bucket, fn, reps, unrolls, bpcs, nts, size, times, verbose)
            finally:
                del fn
                torch.cuda.empty_cache()
    finally:
        if small_old is not None:
            tune_ws_small_max(small_old)
    scored, best_at = rank_shapes(times)
    score, (u, b, nt), ms = scored[0]
    tune_set(op, u, b, nt, bucket=bucket)
    return {"unroll": u, "blocks_per_cu": b, "nontemporal": nt, "ms": list(ms),
            "bytes": list(sizes), "score": score, "best_ms": best_at, "previous": list(old),
            "previous_ms": list(times.get(tuple(old), [])),
            "grid": [[sh[0], sh[1], sh[2], sc] + list(t) for sc, sh, t in scored]}


def rank_shapes(times: dict) -> tuple[list, list]:
    """Shapes ranked by their mean time relative to the fastest shape at each
    size: `times` maps a shape to its times at the same sizes, in order.
    Returns ([(score, shape, times)], fastest time at each size), best first;
    ties go to the smaller shape tuple."""
    nsizes = len(next(iter(times.values())))
    if any(len(ms) != nsizes for ms in times.values()):
        raise ValueError("every shape needs a time at every size")
    best_at = [min(ms[i] for ms in times.values()) for i in range(nsizes)]
    scored = sorted((statistics.fmean(t / b for t, b in zip(ms, best_at)), sh, list(ms))
                    for sh, ms in times.items())
    return scored, best_at


def _sweep(torch, op, bucket, fn, reps, unrolls, bpcs, nts, nbytes, times, verbose):
    for nt in nts:
        for u in unrolls:
            for b in bpcs:
                tune_set(op, u, b, nt, bucket=bucket)
                # small calls: device time from graph replays; large ones: stream timing
                ms = _graph_time(torch, fn, reps) if nbytes < (16 << 20) else _time(torch, fn, reps)
                times.setdefault((u, b, nt), []).append(ms)
                if verbose:
                    print(f"[tune] {op:15s} bucket={bucket} bytes={nbytes} unroll={u} "
                          f"blocks/cu={b:2d} nt={nt}: {ms * 1e3:9.2f} us", flush=True)


# MIME text sizes at which the whitespace-skipping decode's two paths are
# compared (payload bytes; the text is about 4/3 of that with line breaks)
GUESS_SIZES = (1 << 20, 2 << 20, 4 << 20, 6 << 20, 8 << 20, 12 << 20, 16 << 20, 24 << 20,
               32 << 20)


def tune_ws_guess(reps: int = 10, sizes=GUESS_SIZES, verbose: bool = True) -> dict:
    """The whitespace-skipping decode of text in regular lines either guesses
    the line layout (a few more launches, one read of the text) or counts the
    significant characters first (fewer launches, two reads).  Time both on
    MIME text of each size and return the smallest text size from which the
    guess is faster at that size and every larger one (applied with
    b64_tune_ws_guess_min)."""
    import torch
    old = tune_ws_guess_min(-1)
    rows = []
    try:
        for nbytes in sizes:
            gen = torch.Generator(device="cuda")
            gen.manual_seed(nbytes)
            x = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=gen)
            mime = encode(x, STD, line_len=76)
            out = torch.empty(3 * (mime.numel() // 4), dtype=torch.uint8, device="cuda")
            st = torch.empty(2, dtype=torch.int64, device="cuda")
            ws = torch.empty(workspace_size(mime.numel(), SKIP_WS), dtype=torch.uint8, device="cuda")
            fn = lambda: decode_async(mime, STD, out=out, status=st, flags=SKIP_WS, workspace=ws)
            tune_ws_guess_min(0)
            t_guess = _time(torch, fn, reps)
            tune_ws_guess_min(1 << 62)
            t_count = _time(torch, fn, reps)
            rows.append((int(mime.numel()), t_guess, t_count))
            if verbose:
                print(f"[tune] decode_ws text {mime.numel():>10d} B: guess {t_guess * 1e3:8.2f} us, "
                      f"counted {t_count * 1e3:8.2f} us", flush=True)
    finally:
        tune_ws_guess_min(old)
    chosen = rows[-1][0] + 1 if rows else old
    for n, tg, tc in reversed(rows):
        if tg < tc:
            chosen = n
        else:
            break
    tune_ws_guess_min(chosen)
    return {"min_chars": chosen, "previous": old,
            "grid": [[n, tg, tc] for n, tg, tc in rows]}


def save(entries: dict, path: str | None = None):
    """Merge {op: {bucket: shape}} (and "ws_guess_min": {"min_chars": n})
    into the cache under the current device."""
    path = path or cache_path()
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    dev = data.setdefault(device_key(), {})
    for op, per_bucket in entries.items():
        dev.setdefault(op, {}).update({str(k): v for k, v in per_bucket.items()})
    with open(path, "w") as f:
        json.dump(data, f, indent=1)


def apply_cached(path: str | None = None) -> dict:
    """Apply the cached shapes of the current device, if any; returns them
    as {op: {bucket: shape}}.  A malformed entry raises ValueError."""
    path = path or cache_path()
    if not path or not os.path.exists(path):
        return {}
    import torch
    if not torch.cuda.is_available():
        return {}
    with open(path) as f:
        data = json.load(f)
    ent = data.get(device_key(), {})
    for op, per_bucket in ent.items():
        if op == "ws_guess_min":
            n = int(per_bucket["min_chars"])
            if n < 0:
                raise ValueError(f"tune cache {path}: negative ws_guess_min")
            tune_ws_guess_min(n)
            continue
        if op not in OPS:
            raise ValueError(f"tune cache {path}: unknown operation {op!r}")
        for bucket, v in per_bucket.items():
            b = int(bucket)
            if not 0 <= b < BUCKETS:
                raise ValueError(f"tune cache {path}: bad bucket {bucket!r} for {op}")
            tune_set(op, int(v["unroll"]), int(v["blocks_per_cu"]), int(v.get("nontemporal", 1)),
                     bucket=b)
    return ent


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ops", nargs="+", default=list(OPS))
    ap.add_argument("--buckets", nargs="+", type=int, default=list(range(BUCKETS)))
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default=None, help="cache file (default: the package's cache)")
    ap.add_argument("--json", default=None, help="also write the full sweep here")
    ap.add_argument("--no-ws-guess", action="store_true",
                    help="skip timing the whitespace decode's guess against its counted path")
    args = ap.parse_args()
    found = {}
    for op in args.ops:
        for bucket in buckets_of(op):
            if bucket not in args.buckets:
                continue
            r = tune_op(op, bucket, reps=args.reps)
            found.setdefault(op, {})[bucket] = r
            us = " / ".join(f"{m * 1e3:.2f}" for m in r["ms"])
            print(f"[tune] best {op} bucket {bucket}: unroll={r['unroll']} "
                  f"blocks/cu={r['blocks_per_cu']} nt={r['nontemporal']} {us} us "
                  f"(x{r['score']:.3f} of the best per size)", flush=True)
    keys = ("unroll", "blocks_per_cu", "nontemporal", "ms", "bytes", "score")
    entries = {op: {b: {k: r[k] for k in keys} for b, r in per.items()}
               for op, per in found.items()}
    if not args.no_ws_guess and "decode_ws" in args.ops:
        g = tune_ws_guess(args.reps)
        print(f"[tune] best ws_guess_min: {g['min_chars']} (was {g['previous']})", flush=True)
        found["ws_guess_min"] = g
        entries["ws_guess_min"] = {"min_chars": g["min_chars"]}
    save(entries, args.out)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(found, f, indent=1)


if __name__ == "__main__":
    main()
