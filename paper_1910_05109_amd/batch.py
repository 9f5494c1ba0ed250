"""Graph-captured batched encode / decode over fixed-capacity device buffers.

A GraphBatch owns device buffers sized for at most `max_buffers` buffers and
`max_bytes` input bytes, captures one b64_encode_batch or b64_decode_batch
launch (with its status kernels) in a HIP graph through torch.cuda.CUDAGraph,
and replays it for each new batch.  The graph reads its offset arrays from
fixed device addresses, so a replay needs no node update: a batch with fewer
buffers is padded with empty buffers (repeated end offset), which the kernels
skip at no cost beyond one offset read.

Host-side work per batch is argument marshalling only: copying the packed
input and the offsets into the fixed buffers (when they come from the host)
and the prefix sum of output capacities.
"""
from __future__ import annotations

import numpy as np

from . import STD, decode_batch, encode_batch


def encoded_lengths(lens: np.ndarray) -> np.ndarray:
    return 4 * ((lens + 2) // 3)


def decoded_capacity(lens: np.ndarray) -> np.ndarray:
    return 3 * (lens // 4)


def prefix(lens: np.ndarray) -> np.ndarray:
    off = np.zeros(lens.size + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


class GraphBatch:
    """op: "encode" or "decode"."""

    def __init__(self, op: str, max_buffers: int, max_bytes: int, alphabet=STD, device="cuda"):
        import torch
        if op not in ("encode", "decode"):
            raise ValueError(op)
        self.op = op
        self.alphabet = bytes(alphabet)
        self.max_buffers = int(max_buffers)
        self.max_bytes = int(max_bytes)
        out_cap = (4 * ((self.max_bytes + 2) // 3) + 4 * self.max_buffers if op == "encode"
                   else 3 * (self.max_bytes // 4))
        self.src = torch.zeros(max(self.max_bytes, 1), dtype=torch.uint8, device=device)
        self.in_off = torch.zeros(self.max_buffers + 1, dtype=torch.int64, device=device)
        self.dst = torch.zeros(max(out_cap, 1), dtype=torch.uint8, device=device)
        self.out_off = torch.zeros(self.max_buffers + 1, dtype=torch.int64, device=device)
        self.out_len = torch.zeros(self.max_buffers, dtype=torch.int64, device=device)
        self.first_bad = torch.zeros(self.max_buffers, dtype=torch.int64, device=device)
        self.nbuf = 0
        self.graph = None
        self._capture(torch)

    def _launch(self):
        if self.op == "encode":
            encode_batch(self.src, self.in_off, self.alphabet, dst=self.dst, out_off=self.out_off,
                         out_len=self.out_len, validate=False)
        else:
            decode_batch(self.src, self.in_off, self.alphabet, dst=self.dst, out_off=self.out_off,
                         out_len=self.out_len, first_bad=self.first_bad, validate=False)

    def _capture(self, torch):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._launch()          # warm-up outside the graph (module load, first launch)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._launch()
        torch.cuda.synchronize()

    def load(self, lens: np.ndarray, src=None, out_off: np.ndarray | None = None):
        """Set the batch layout (host lengths) and, optionally, its packed input
        (a host numpy array or a device uint8 tensor of sum(lens) bytes)."""
        import torch
        lens = np.asarray(lens, dtype=np.int64)
        nbuf = lens.size
        if nbuf > self.max_buffers:
            raise ValueError("too many buffers for this graph")
        in_off = prefix(lens)
        if in_off[-1] > self.max_bytes:
            raise ValueError("batch larger than the graph's input capacity")
        pad_in = np.full(self.max_buffers + 1, in_off[-1], dtype=np.int64)
        pad_in[: nbuf + 1] = in_off
        if (lens < 0).any():
            raise ValueError("negative buffer length")
        cap = encoded_lengths(lens) if self.op == "encode" else decoded_capacity(lens)
        if out_off is None:
            out_off = prefix(cap)
        out_off = np.asarray(out_off, dtype=np.int64)
        if nbuf and ((out_off[:nbuf] < 0).any() or (out_off[:nbuf] + cap).max() > self.dst.numel()):
            raise ValueError("batch outputs exceed the graph's output capacity")
        pad_out = np.full(self.max_buffers + 1, out_off[-1], dtype=np.int64)
        pad_out[: nbuf + 1] = out_off
        self.in_off.copy_(torch.from_numpy(pad_in), non_blocking=False)
        self.out_off.copy_(torch.from_numpy(pad_out), non_blocking=False)
        if src is not None:
            n = int(in_off[-1])
            if isinstance(src, np.ndarray):
                self.src[:n].copy_(torch.from_numpy(np.ascontiguousarray(src[:n])))
            else:
                self.src[:n].copy_(src[:n])
        self.nbuf = nbuf
        self.host_in_off = in_off
        self.host_out_off = np.asarray(out_off, dtype=np.int64)

    def replay(self):
        self.graph.replay()

    def results(self):
        """(dst, out_off, out_len, first_bad) views for the loaded batch."""
        n = self.nbuf
        return self.dst, self.out_off[: n + 1], self.out_len[:n], self.first_bad[:n]
