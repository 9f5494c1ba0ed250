"""Continuous-batching request loop over the batched HIP codec.

Requests (encode or decode) arrive over time; their payloads are already
resident in device memory, packed per kind in arrival order (a "pool"), and
their results stay in device memory.  The loop

  1. retires finished launches in order (a HIP event per launch): the
     per-request output lengths / first invalid offsets have been copied to
     pinned host memory, so the results are visible to the host; the
     request's latency is retirement time minus its scheduled arrival;
  2. admits every request that has arrived, in order;
  3. while fewer than `max_inflight` launches are outstanding, coalesces the
     admitted requests of one kind (consecutive in its pool, so the batch's
     input offsets are a slice of the pool's offset array and need no copy)
     into ONE b64_encode_batch / b64_decode_batch launch, as long as their
     outputs fit in the output arena (the HBM budget): requests that do not
     fit wait until earlier launches retire and free their space.

Requests arriving while others are on the GPU join the next launch, and up to
`max_inflight` launches overlap on the device.  The output arena is a ring:
launches retire in order, so space is freed in order.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import STD, _lib
from .batch import decoded_capacity, encoded_lengths

ENC, DEC = 0, 1


def _prefix(lens):
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


@dataclass
class Pool:
    """Payloads of one kind, packed in arrival order, resident on the device."""
    kind: int
    data: object                 # uint8 CUDA tensor
    in_off: np.ndarray           # host, nreq+1
    out_rel: np.ndarray          # host, nreq+1: prefix sum of output capacities
    d_in_off: object = None
    d_out_rel: object = None
    d_len: object = None         # per-request out_len (device)
    d_bad: object = None         # per-request first_bad (device)
    h_len: object = None         # pinned host copies
    h_bad: object = None

    def __post_init__(self):
        import torch
        n = self.in_off.size - 1
        self.d_in_off = torch.from_numpy(self.in_off).cuda()
        self.d_out_rel = torch.from_numpy(self.out_rel).cuda()
        self.d_len = torch.zeros(max(n, 1), dtype=torch.int64, device="cuda")
        self.d_bad = torch.full((max(n, 1),), -1, dtype=torch.int64, device="cuda")
        self.h_len = torch.zeros(max(n, 1), dtype=torch.int64).pin_memory()
        self.h_bad = torch.full((max(n, 1),), -1, dtype=torch.int64).pin_memory()


def make_pool(kind: int, data, lens: np.ndarray) -> Pool:
    lens = np.asarray(lens, dtype=np.int64)
    cap = encoded_lengths(lens) if kind == ENC else decoded_capacity(lens)
    return Pool(kind, data, _prefix(lens), _prefix(cap))


class OutputRing:
    """Ring allocator for the output arena.  Allocations are released in the
    order they were made (launches retire in order), so the live region is
    one contiguous (possibly wrapped) span; an allocation that does not fit
    before the end of the arena skips the tail, which stays held until the
    allocation retires."""

    def __init__(self, size: int):
        self.size = int(size)
        self.head = 0            # next free byte
        self.used = 0            # bytes held, including skipped tails
        self.live = 0            # allocations not yet released

    def alloc(self, n: int):
        """Returns (start, held) or None if `n` bytes do not fit now."""
        if n > self.size:
            raise ValueError("a single request's output exceeds the HBM budget")
        free_tail = self.size - self.head
        if n <= free_tail:
            if self.used + n > self.size:
                return None
            start, waste = self.head, 0
        else:
            waste = free_tail
            if self.used + waste + n > self.size:
                return None
            start = 0
        self.head = start + n
        self.used += waste + n
        self.live += 1
        return start, waste + n

    def release(self, held: int):
        self.used -= held
        self.live -= 1
        if self.live == 0:
            self.head, self.used = 0, 0


@dataclass
class Launch:
    kind: int
    first: int
    count: int
    start: int          # arena offset of the outputs
    size: int
    event: object
    t_launch: float


@dataclass
class Stats:
    latency: np.ndarray
    done_at: np.ndarray
    launches: int
    mean_batch: float
    wall: float
    chars: int
    extra: dict = field(default_factory=dict)

    def summary(self) -> dict:
        lat = self.latency * 1e3
        return {"requests": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
                "launches": self.launches, "mean_batch": self.mean_batch,
                "wall_s": self.wall, "gbps_b64": self.chars / self.wall / 1e9, **self.extra}


class Server:
    """Run a request schedule through the batched codec.

    kinds[i] (ENC/DEC) and arrival[i] (seconds) describe request i; request i
    is entry pos[i] of the pool of its kind (requests of one kind appear in
    their pool in arrival order).  `budget_bytes` bounds the output arena."""

    def __init__(self, enc_pool: Pool, dec_pool: Pool, budget_bytes: int, alphabet=STD,
                 max_inflight: int = 4, max_batch: int = 8192, on_retire=None):
        import torch
        self.pools = (enc_pool, dec_pool)
        self.alphabet = bytes(alphabet)
        self._alpha = ctypes.create_string_buffer(self.alphabet, 64)
        need = max(int(enc_pool.out_rel[-1]), int(dec_pool.out_rel[-1]), 1)
        self.arena_bytes = int(min(budget_bytes, max(need * 2, 1 << 20)))
        self.arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device="cuda")
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.on_retire = on_retire
        self.stream = torch.cuda.current_stream()
        self.lib = _lib.load()
        self.ring = OutputRing(self.arena_bytes)
        self.inflight: deque[Launch] = deque()
        self.peak_used = 0

    def _launch(self, kind: int, first: int, count: int):
        import torch
        kind, first, count = int(kind), int(first), int(count)
        pool = self.pools[kind]
        size = int(pool.out_rel[first + count] - pool.out_rel[first])
        if size > self.ring.size:
            if count == 1:
                raise ValueError("a single request's output exceeds the HBM budget")
            return None          # the caller retries with fewer requests
        got = self.ring.alloc(size)
        if got is None:
            return None
        start, held = got
        self.peak_used = max(self.peak_used, self.ring.used)
        base = self.arena.data_ptr() + start - int(pool.out_rel[first])
        s = self.stream.cuda_stream
        in_off = pool.d_in_off.data_ptr() + 8 * first
        out_off = pool.d_out_rel.data_ptr() + 8 * first
        olen = pool.d_len.data_ptr() + 8 * first
        if kind == ENC:
            r = self.lib.b64_encode_batch(pool.data.data_ptr(), in_off, count, base, out_off, olen,
                                          self._alpha, s)
        else:
            bad = pool.d_bad.data_ptr() + 8 * first
            r = self.lib.b64_decode_batch(pool.data.data_ptr(), in_off, count, base, out_off, olen,
                                          bad, self._alpha, s)
            pool.h_bad[first:first + count].copy_(pool.d_bad[first:first + count], non_blocking=True)
        _lib.check(r, "batch launch")
        pool.h_len[first:first + count].copy_(pool.d_len[first:first + count], non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(self.stream)
        return Launch(kind, first, count, start, held, ev, time.perf_counter())

    def run(self, kinds: np.ndarray, arrival: np.ndarray, pos: np.ndarray) -> Stats:
        nreq = kinds.size
        order = np.argsort(arrival, kind="stable")
        # request id by (kind, pool position), to map retired pool ranges back
        req_of = [np.full(self.pools[k].in_off.size - 1, -1, dtype=np.int64) for k in (ENC, DEC)]
        for i in range(nreq):
            req_of[kinds[i]][pos[i]] = i
        done_at = np.full(nreq, np.nan)
        ready_hi = [0, 0]        # admitted pool prefix per kind
        next_first = [0, 0]      # first pool entry not yet launched per kind
        launches, batched = 0, 0
        nxt = 0                  # next arrival in `order`
        t0 = time.perf_counter()
        retired = 0
        turn = 0
        while retired < nreq:
            now = time.perf_counter() - t0
            # 1. retire in order
            while self.inflight and self.inflight[0].event.query():
                L = self.inflight.popleft()
                tnow = time.perf_counter() - t0
                ids = req_of[L.kind][L.first:L.first + L.count]
                done_at[ids] = tnow
                retired += L.count
                if self.on_retire is not None:
                    self.on_retire(L, self)
                self.ring.release(L.size)
            # 2. admit arrivals
            while nxt < nreq and arrival[order[nxt]] <= now:
                i = order[nxt]
                ready_hi[int(kinds[i])] = max(ready_hi[int(kinds[i])], int(pos[i]) + 1)
                nxt += 1
            # 3. launch coalesced batches while slots are free
            launched = False
            for k in (turn, 1 - turn):
                if len(self.inflight) >= self.max_inflight:
                    break
                first = next_first[k]
                count = min(ready_hi[k] - first, self.max_batch)
                if count <= 0:
                    continue
                L = None
                while count > 0:
                    L = self._launch(k, first, count)
                    if L is not None:
                        break
                    count //= 2        # shrink to what the free space allows
                if L is None:
                    continue
                self.inflight.append(L)
                next_first[k] += count
                launches += 1
                batched += count
                launched = True
            turn ^= 1
            if not launched and not (self.inflight and self.inflight[0].event.query()):
                # idle: wait a little for the next arrival or completion
                if nxt < nreq and not self.inflight:
                    wait = arrival[order[nxt]] - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
        wall = time.perf_counter() - t0
        lat = done_at - arrival
        chars = int(self.pools[ENC].out_rel[-1] + self.pools[DEC].in_off[-1])
        return Stats(latency=lat, done_at=done_at, launches=launches,
                     mean_batch=batched / max(launches, 1), wall=wall, chars=chars,
                     extra={"arena_bytes": self.arena_bytes, "peak_arena_used": self.peak_used})

    def results(self, kind: int):
        """Per pool entry: (out_len, first_bad) as host arrays after run()."""
        p = self.pools[kind]
        n = p.in_off.size - 1
        return p.h_len[:n].numpy(), p.h_bad[:n].numpy()
