"""Independent references built only from Python's standard-library base64
codec (a library routine, not shared code), used to pin the oracle.

- encode_ref(x, alpha): base64.b64encode, then a byte translation from the
  standard alphabet to `alpha` (any 64-byte mapping, Section "Encoding" step 2).
- PrefixRule: the first invalid offset defined as the length of the longest
  prefix of the input that is still a prefix of some valid padded encoding.
  The valid 4-character quanta are taken as images of the standard-library
  encoder: every 3-byte group (data quanta), every 2-byte and 1-byte input
  (the final quanta "xyz=" and "xy==").  A valid encoding is any number of
  data quanta optionally ending with one final quantum.
"""
from __future__ import annotations

import base64
import itertools

import numpy as np

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
WS = b" \t\r\n"


def translator(alpha: bytes) -> bytes:
    return bytes.maketrans(STD, bytes(alpha))


def encode_ref(x: bytes, alpha: bytes = STD) -> bytes:
    return base64.b64encode(bytes(x)).translate(translator(alpha))


class PrefixRule:
    """Longest-extendable-prefix rule over the images of the stdlib encoder."""

    def __init__(self, alpha: bytes = STD):
        tr = translator(alpha)
        self.alpha = bytes(alpha)
        self.chars = set(self.alpha)
        # final quanta: images of every 1-byte and 2-byte input
        self.final = set()
        for a in range(256):
            self.final.add(base64.b64encode(bytes([a])).translate(tr))
        for a, b in itertools.product(range(256), repeat=2):
            self.final.add(base64.b64encode(bytes([a, b])).translate(tr))
        # data quanta: images of 3-byte groups.  Their set is every 4-tuple of
        # alphabet characters; confirmed from the encoder on all 2^24 groups
        # by the exhaustive encode test, so here membership is "4 alphabet chars".
        self.final_prefix = {q[:r] for q in self.final for r in range(1, 4)}

    def is_data(self, q: bytes) -> bool:
        return len(q) == 4 and all(c in self.chars for c in q)

    def is_quantum_prefix(self, p: bytes) -> bool:
        if all(c in self.chars for c in p):
            return True  # prefix of some data quantum
        return p in self.final_prefix

    def result(self, s: bytes) -> int:
        """Decoded length if s is a valid encoding, else ~first_invalid_offset.

        Walks whole quanta while they are data quanta; at the first quantum
        that is not, the longest extendable prefix ends inside or right after
        it: after a final quantum nothing may follow, otherwise it ends after
        the longest leading part that is still a prefix of some quantum."""
        s = bytes(s)
        n = len(s)
        k = 0
        while k + 4 <= n and self.is_data(s[k:k + 4]):
            k += 4
        if k == n:
            return 3 * (n // 4)
        blk = s[k:k + 4]
        if len(blk) == 4 and blk in self.final:
            if k + 4 == n:
                return 3 * (n // 4) - blk.count(b"=")
            return ~(k + 4)
        r = 0
        while r < min(len(blk), 3) and self.is_quantum_prefix(blk[:r + 1]):
            r += 1
        if k + r == n:
            return ~n  # every character fits, but the input stops mid-quantum
        return ~(k + r)


def brute_force_results(symbols: list[int], length: int, alpha: bytes = STD):
    """All len(symbols)^length strings over `symbols` (as a 2-D uint8 array) and
    their expected results under PrefixRule, computed with numpy over quanta."""
    rule = PrefixRule(alpha)
    k = len(symbols)
    sym = np.array(symbols, dtype=np.uint8)
    nrows = k ** length
    digits = np.indices((k,) * length).reshape(length, -1).T if length else np.zeros((1, 0), dtype=np.int64)
    rows = sym[digits].astype(np.uint8) if length else np.zeros((1, 0), dtype=np.uint8)
    assert rows.shape == (nrows, length)

    # tables over single quanta / partial quanta of the symbol set
    def code(block):
        c = 0
        for d in block:
            c = c * k + d
        return c

    is_data = np.zeros(k ** 4, dtype=bool)
    is_final = np.zeros(k ** 4, dtype=bool)
    for block in itertools.product(range(k), repeat=4):
        q = bytes(sym[list(block)])
        is_data[code(block)] = rule.is_data(q)
        is_final[code(block)] = q in rule.final
    is_prefix = {}
    for r in range(1, 4):
        t = np.zeros(k ** r, dtype=bool)
        for block in itertools.product(range(k), repeat=r):
            t[code(block)] = rule.is_quantum_prefix(bytes(sym[list(block)]))
        is_prefix[r] = t

    # ext[:, l] == prefix of length l extendable
    ext = np.zeros((nrows, length + 1), dtype=bool)
    ext[:, 0] = True
    all_data_before = np.ones(nrows, dtype=bool)  # blocks 0..q-1 all data
    for l in range(1, length + 1):
        q, r = divmod(l, 4)
        if r == 0:
            blk = np.zeros(nrows, dtype=np.int64)
            for j in range(4):
                blk = blk * k + digits[:, 4 * (q - 1) + j]
            ext[:, l] = all_data_before & (is_data[blk] | is_final[blk])
            all_data_before = all_data_before & is_data[blk]
        else:
            blk = np.zeros(nrows, dtype=np.int64)
            for j in range(r):
                blk = blk * k + digits[:, 4 * q + j]
            ext[:, l] = all_data_before & is_prefix[r][blk]
    # a prefix of an extendable prefix is extendable: the table must be monotone
    assert not (ext[:, 1:] & ~ext[:, :-1]).any()
    lo = ext.sum(axis=1) - 1
    expected = np.where(lo < length, ~lo, 0).astype(np.int64)
    full = lo == length
    if length % 4 != 0:
        expected[full] = ~np.int64(length)
    else:
        pads = (rows[:, -2:] == ord("=")).sum(axis=1) if length else np.zeros(nrows, dtype=np.int64)
        expected[full] = 3 * (length // 4) - pads[full]
    return rows, expected


# ------------------------------------------------------------- variants --
# References for the unpadded, line-wrapped and whitespace-skipping forms,
# built from the standard-library codec and the prefix rule above.

def ref_nopad(x: bytes, alpha: bytes) -> bytes:
    return base64.b64encode(x).rstrip(b"=").translate(translator(alpha))


def ref_wrap(text: bytes, line_len: int) -> bytes:
    return b"\r\n".join(text[i:i + line_len] for i in range(0, len(text), line_len))


def nopad_reference(s: bytes, alpha: bytes) -> int:
    """Decoded length, or ~first_invalid_offset, from the standard library."""
    chars = set(alpha)
    for i, c in enumerate(s):
        if c not in chars:
            return ~i
    n = len(s)
    if n % 4 == 1:
        return ~n
    std = s.translate(bytes.maketrans(alpha, STD))
    d = base64.b64decode(std + b"=" * ((4 - n % 4) % 4), validate=True)
    if base64.b64encode(d).rstrip(b"=") != std:
        return ~n          # non-canonical trailing bits: could still be completed
    return len(d)


def compacted(s: bytes):
    keep = [i for i, c in enumerate(s) if c not in WS]
    return bytes(s[i] for i in keep), keep


_RULES = {}


def skip_ws_reference(s: bytes, alpha: bytes, nopad: bool) -> int:
    c, keep = compacted(s)
    if not nopad and alpha not in _RULES:
        _RULES[alpha] = PrefixRule(alpha)
    r = nopad_reference(c, alpha) if nopad else _RULES[alpha].result(c)
    if r >= 0:
        return r
    off = ~r
    return ~(keep[off] if off < len(c) else len(s))
