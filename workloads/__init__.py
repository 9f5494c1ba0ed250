"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no codec arithmetic: it only draws random bytes, lengths,
positions and arrival times.  Both the HIP path and the oracle are fed from
here, and neither is imported by it.

The paper measures on random binary data and notes that content does not
change the speed of a vectorized codec (Section "Experiments"), so every
payload is uniform random bytes from numpy's PCG64, seeded per workload.

Workloads (sizes as named in the design notes):
  single 3 MiB   : 3,145,728 bytes -> 4,194,304 characters, plus a decode copy
                   with one byte outside the alphabet and not '=' at a seeded
                   uniform position.
  single 1 GiB   : n = 1,073,741,823 (n mod 3 = 0) and n = 2^30 (n mod 3 = 1).
  size sweep     : n = 2^k + r, k = 10..26, r = 0,1,2, plus the byte counts of
                   the paper's four decode test files (Table tab:perf) used as
                   lengths of random data, since the files themselves are not
                   available.
  ragged batch   : 100,000 buffers, lengths floor(16 * 2^(16u)), u ~ U[0,1)
                   (log-uniform over [16 B, 1 MiB]); 0.5% of decode buffers get
                   one invalid byte.
  serving        : Poisson arrivals, sizes log-normal (median 8 KiB, sigma 1.5)
                   clipped to [1 B, 16 MiB], 50/50 encode/decode, 1% of decode
                   requests carry one invalid byte.
  MIME text      : the encoding in lines of 76 characters separated by CR LF
                   (the MIME line length), optionally with extra whitespace
                   runs inserted at seeded positions (sprinkle_ws).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 191005109

SINGLE_3MIB = 3_145_728
SINGLE_1GIB = (1_073_741_823, 1_073_741_824)
TABLE_PERF_LENGTHS = (2_357, 141_020, 247_222, 34_904_444)
BATCH_BUFFERS = 100_000
BATCH_MIN, BATCH_MAX = 16, 1 << 20
SERVE_MEDIAN, SERVE_SIGMA = 8192, 1.5
SERVE_MIN, SERVE_MAX = 1, 16 << 20
PAD = ord("=")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_bytes(seed: int, n: int) -> np.ndarray:
    """n uniform random bytes (uint8), deterministic in (seed, n)."""
    words = rng(seed).integers(0, 2 ** 64 - 1, size=(n + 7) // 8, dtype=np.uint64,
                               endpoint=True)
    return words.view(np.uint8)[:n]


def sweep_lengths() -> list[int]:
    """2^k + r for k = 10..26, r = 0, 1, 2 (all residues mod 3)."""
    return [(1 << k) + r for k in range(10, 27) for r in range(3)]


def non_alphabet_bytes(alpha: bytes) -> np.ndarray:
    """Byte values that are neither in the alphabet nor '=' (191 of them for
    a 64-byte alphabet)."""
    bad = np.ones(256, dtype=bool)
    bad[np.frombuffer(bytes(alpha), dtype=np.uint8)] = False
    bad[PAD] = False
    return np.nonzero(bad)[0].astype(np.uint8)


def plant_invalid(text: np.ndarray, seed: int, alpha: bytes, lo: int = 0, hi: int | None = None):
    """Copy `text` and overwrite one seeded uniform position in [lo, hi) with a
    seeded byte that is neither an alphabet character nor '='.
    Returns (copy, position)."""
    g = rng(seed)
    hi = text.size if hi is None else hi
    pos = int(g.integers(lo, hi))
    bad = non_alphabet_bytes(alpha)
    out = text.copy()
    out[pos] = bad[int(g.integers(0, bad.size))]
    return out, pos


def batch_lengths(seed: int, nbuf: int = BATCH_BUFFERS, lo: int = BATCH_MIN,
                  hi: int = BATCH_MAX) -> np.ndarray:
    """Log-uniform lengths in [lo, hi): floor(lo * (hi/lo)^u), u ~ U[0,1)."""
    u = rng(seed).random(nbuf)
    lens = np.floor(lo * np.power(hi / lo, u)).astype(np.int64)
    return np.clip(lens, lo, hi - 1)


def offsets(lengths: np.ndarray) -> np.ndarray:
    """Exclusive prefix sum with a trailing total: nbuf + 1 int64 entries."""
    off = np.zeros(lengths.size + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off


def pick_buffers(seed: int, nbuf: int, frac: float) -> np.ndarray:
    """A seeded sorted sample of round(frac * nbuf) distinct buffer indices."""
    k = int(round(frac * nbuf))
    return np.sort(rng(seed).choice(nbuf, size=k, replace=False))


def serve_sizes(seed: int, count: int, median: int = SERVE_MEDIAN,
                sigma: float = SERVE_SIGMA) -> np.ndarray:
    s = rng(seed).lognormal(mean=np.log(median), sigma=sigma, size=count)
    return np.clip(np.floor(s), SERVE_MIN, SERVE_MAX).astype(np.int64)


def serve_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times in seconds of a Poisson process of the given rate."""
    gaps = rng(seed).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)


def serve_kinds(seed: int, count: int, invalid_frac: float = 0.01):
    """Per request: is_decode (50/50) and, for decodes, is_invalid (1%)."""
    g = rng(seed)
    is_dec = g.random(count) < 0.5
    is_bad = is_dec & (g.random(count) < invalid_frac)
    return is_dec, is_bad


WHITESPACE = np.frombuffer(b" \t\r\n", dtype=np.uint8)
MIME_LINE = 76


def sprinkle_ws(text: np.ndarray, seed: int, runs: int, max_run: int = 5,
                long_runs: int = 0, long_len: int = 1 << 17) -> np.ndarray:
    """Insert `runs` runs of 1..max_run whitespace bytes (space, tab, CR, LF)
    and `long_runs` runs of long_len spaces at seeded positions."""
    g = rng(seed)
    pos = np.sort(g.integers(0, text.size + 1, size=runs + long_runs))
    lens = np.concatenate([g.integers(1, max_run + 1, size=runs),
                           np.full(long_runs, long_len, dtype=np.int64)])
    g.shuffle(lens)
    parts, prev = [], 0
    for p, k in zip(pos.tolist(), lens.tolist()):
        parts.append(text[prev:p])
        parts.append(WHITESPACE[g.integers(0, 4, size=k)] if k <= max_run
                     else np.full(k, ord(" "), dtype=np.uint8))
        prev = p
    parts.append(text[prev:])
    return np.concatenate(parts).astype(np.uint8) if parts else text.copy()
