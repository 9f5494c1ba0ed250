"""Continuous-batching request server: the binding of b64_server_* in the C ABI.

The server itself is native (csrc/b64_serve.hip): one scheduler thread
admits requests as they arrive, coalesces the queued requests of one kind
into ONE batched launch while the device arena (the HBM budget) has room for
their payloads and outputs, and enqueues each launch on the next of several
HIP streams, so that launches run at the same time on the device; a launch's
requests are done when its results are in pinned host memory.  Optionally,
launches run zero-copy: the kernels work on the pinned host pools directly,
with no DMA and no arena space.  This module only marshals arrays: a schedule (kind, arrival time,
payload of each request, in host memory) goes in; outputs, lengths, first
invalid offsets, completion times and the run's counters come out.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import STD, _lib
from ._lib import B64Error, load
from .batch import decoded_capacity, encoded_lengths

ENC, DEC = 0, 1
STATS = ("launches", "wall_ns", "peak_arena_bytes", "max_inflight", "max_concurrent",
         "overlapped_launches", "arena_bytes", "zero_copy_launches")
STAT_COUNT = 8


def out_layout(kinds: np.ndarray, lens: np.ndarray) -> np.ndarray:
    """Host output offsets (nreq + 1) for requests of these kinds and payload
    lengths: each request gets the capacity of its kind."""
    kinds = np.asarray(kinds)
    lens = np.asarray(lens, dtype=np.int64)
    cap = np.where(kinds == ENC, encoded_lengths(lens), decoded_capacity(lens))
    off = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(cap, out=off[1:])
    return off


@dataclass
class Result:
    """Per request i: out[out_off[i] : out_off[i] + out_len[i]], out_len[i]
    (-1 for an invalid decode), first_bad[i] (-1 or the first invalid
    offset), latency[i] seconds (results in host memory minus arrival)."""
    out: np.ndarray
    out_off: np.ndarray
    out_len: np.ndarray
    first_bad: np.ndarray
    latency: np.ndarray
    stats: dict
    chars: int = 0
    extra: dict = field(default_factory=dict)

    def output(self, i: int) -> np.ndarray:
        n = int(self.out_len[i])
        return self.out[self.out_off[i]: self.out_off[i] + max(n, 0)]

    def summary(self) -> dict:
        lat = self.latency * 1e6
        wall = self.stats["wall_ns"] * 1e-9
        return {"requests": int(lat.size), "p50_us": float(np.percentile(lat, 50)),
                "p99_us": float(np.percentile(lat, 99)), "max_us": float(lat.max()),
                "launches": self.stats["launches"],
                "mean_batch": lat.size / max(self.stats["launches"], 1),
                "wall_s": wall, "gbps_b64": self.chars / wall / 1e9 if wall > 0 else 0.0,
                "max_inflight": self.stats["max_inflight"],
                "max_concurrent": self.stats["max_concurrent"],
                "overlapped_launches": self.stats["overlapped_launches"],
                "peak_arena_bytes": self.stats["peak_arena_bytes"],
                "arena_bytes": self.stats["arena_bytes"],
                "zero_copy_launches": self.stats["zero_copy_launches"], **self.extra}


class Server:
    """A native continuous-batching server on the current device.

    budget_bytes: the device arena for the payloads and outputs in flight (HBM budget);
    nstreams: HIP streams the launches go to in turn; depth: launches in
    flight at most; max_batch / max_batch_bytes: requests / payload bytes per
    launch at most; zero_copy_max: launches with at most this many payload
    bytes run zero-copy (the kernel works on the pinned host pools, no DMA
    and no arena space; 0 turns it off, None keeps the library's default);
    staging: how staged launches move bytes between the host pools and the
    arena: "auto" (the default: copy kernels on the mapped pools for
    launches up to 1 MiB of payload, DMA above), "kernels" or "dma"
    (hipMemcpyAsync).
    The defaults (two streams, one launch in flight on each) gave the lowest
    p99 on MI355X: a device has four hardware queues, and more streams than
    the queues left beside the default stream stall now and then for
    milliseconds."""

    def __init__(self, budget_bytes: int = 32 << 30, nstreams: int = 2, depth: int = 2,
                 max_batch: int = 8192, max_batch_bytes: int = 64 << 20,
                 zero_copy_max: int | None = None, staging: str | None = None):
        L = load()
        self._h = L.b64_server_create(int(budget_bytes), int(nstreams), int(depth), int(max_batch),
                                      int(max_batch_bytes))
        if not self._h:
            raise B64Error("b64_server_create: " + (L.b64_server_last_error() or b"").decode())
        if zero_copy_max is not None:
            if zero_copy_max < 0 or L.b64_server_set_zero_copy_max(self._h, int(zero_copy_max)) < 0:
                self.close()
                raise ValueError("zero_copy_max must be >= 0")
        if staging is not None:
            modes = {"kernels": 0, "dma": 1, "auto": 2}
            if staging not in modes:
                self.close()
                raise ValueError("staging must be 'auto', 'kernels' or 'dma'")
            L.b64_server_set_staging(self._h, modes[staging])

    def close(self):
        if self._h:
            load().b64_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, kinds, arrival_s, payload, in_off, alphabet=STD) -> Result:
        """Serve requests i = 0..n-1: kinds[i] (ENC / DEC), arrival_s[i]
        seconds after the start (non-decreasing), payload[in_off[i] :
        in_off[i+1]] (host uint8)."""
        kinds = np.ascontiguousarray(kinds, dtype=np.int32)
        n = kinds.size
        arrival = np.ascontiguousarray(np.round(np.asarray(arrival_s, dtype=np.float64) * 1e9),
                                       dtype=np.int64)
        payload = np.ascontiguousarray(payload, dtype=np.uint8)
        in_off = np.ascontiguousarray(in_off, dtype=np.int64)
        if arrival.size != n or in_off.size != n + 1:
            raise ValueError("kinds, arrival_s and in_off must describe the same requests")
        if n and (in_off[0] < 0 or in_off[-1] > payload.size):
            raise ValueError("in_off must lie within the payload")
        lens = np.diff(in_off)
        out_off = out_layout(kinds, lens)
        out = np.empty(max(int(out_off[-1]), 1), dtype=np.uint8)
        out_len = np.empty(max(n, 1), dtype=np.int64)
        first_bad = np.empty(max(n, 1), dtype=np.int64)
        done = np.empty(max(n, 1), dtype=np.int64)
        stats = np.zeros(STAT_COUNT, dtype=np.int64)
        alpha = ctypes.create_string_buffer(bytes(alphabet), 64)
        p = lambda a: a.ctypes.data
        r = load().b64_server_run(self._h, n, p(kinds), p(arrival), p(payload), p(in_off), p(out),
                                  p(out_off), p(out_len), p(first_bad), p(done), alpha, p(stats))
        if r in (_lib.EARG, _lib.EHIP):
            raise B64Error("b64_server_run: " + (load().b64_server_last_error() or b"").decode())
        enc = kinds == ENC
        chars = int(encoded_lengths(lens[enc]).sum() + lens[~enc].sum())
        return Result(out=out, out_off=out_off, out_len=out_len[:n], first_bad=first_bad[:n],
                      latency=(done[:n] - arrival) * 1e-9,
                      stats={k: int(stats[i]) for i, k in enumerate(STATS)}, chars=chars)
