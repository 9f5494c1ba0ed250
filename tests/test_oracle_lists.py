"""Pins for the oracle's packed-buffer helpers (CPU only): b64o_encode_list,
b64o_decode_list, b64o_encode_mode_list and b64o_decode_mode_list.

The paper defines the codec one buffer at a time (Section "Base64"), so a
list of buffers has one correct result per buffer.  Each helper is checked
buffer by buffer against references built from the standard-library codec
(stdlib_refs): the encoding (translated to the alphabet, '=' stripped for the
unpadded form, cut into CR LF lines for a line length), the decoded bytes,
and the first invalid offset of the prefix rule (the longest prefix that is
still a prefix of some valid encoding).  The layouts hold empty, 1-byte and
truncated buffers, bytes outside the alphabet, misplaced '=' and whitespace;
the outputs are placed at gapped offsets, and the bytes in the gaps must be
left alone.
"""
import base64

import numpy as np
import pytest

import workloads
from stdlib_refs import (STD, WS, PrefixRule, encode_ref, nopad_reference, ref_nopad, ref_wrap,
                         skip_ws_reference)

URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"
SENTINEL = 0xA5


def _ptr(a):
    return a.ctypes.data


def _lengths(seed, nbuf, maxlen):
    g = workloads.rng(seed)
    lens = g.integers(0, maxlen + 1, size=nbuf).astype(np.int64)
    lens[g.random(nbuf) < 0.1] = 0
    lens[:10] = np.arange(10)          # empty, 1-byte and every residue
    return lens


def _gapped(caps, seed):
    """Output offsets with a random gap of 0..7 bytes after every buffer."""
    g = workloads.rng(seed)
    gaps = g.integers(0, 8, size=caps.size).astype(np.int64)
    out_off = np.zeros(caps.size + 1, dtype=np.int64)
    np.cumsum(caps + gaps, out=out_off[1:])
    return out_off


def _buffers(src, in_off):
    return [bytes(src[in_off[b]:in_off[b + 1]]) for b in range(in_off.size - 1)]


def _spoil(texts, seed, alpha, skip_ws=False):
    """Mutate about a third of the buffers: a byte outside the alphabet, a
    misplaced '=', a truncation by 1..3 characters, or (skip_ws) inserted
    whitespace, which is not an error there."""
    g = workloads.rng(seed)
    outside = workloads.non_alphabet_bytes(alpha)
    if skip_ws:
        outside = np.array([c for c in outside if c not in WS], dtype=np.uint8)
    out = []
    for t in texts:
        t = bytearray(t)
        kind = int(g.integers(0, 6))
        if t and kind == 0:
            t[int(g.integers(0, len(t)))] = int(outside[g.integers(0, outside.size)])
        elif t and kind == 1:
            t[int(g.integers(0, len(t)))] = ord("=")
        elif t and kind == 2:
            del t[len(t) - int(g.integers(1, min(3, len(t)) + 1)):]
        elif skip_ws and kind == 3:
            for _ in range(int(g.integers(1, 4))):
                p = int(g.integers(0, len(t) + 1))
                t[p:p] = bytes(g.choice(np.frombuffer(WS, dtype=np.uint8), 2).tolist())
        out.append(bytes(t))
    return out


def _pack(bufs):
    lens = np.array([len(b) for b in bufs], dtype=np.int64)
    in_off = workloads.offsets(lens)
    src = np.frombuffer(b"".join(bufs) + b"\0", dtype=np.uint8)[: int(in_off[-1])].copy()
    return src, in_off, lens


def _run_encode_list(oracle, src, in_off, alpha, flags=None, line_len=0, seed=0):
    nbuf = in_off.size - 1
    lens = np.diff(in_off)
    if flags is None:
        olen = 4 * ((lens + 2) // 3)
    else:
        olen = np.array([oracle.encoded_len_mode(int(k), flags, line_len) for k in lens],
                        dtype=np.int64)
    out_off = _gapped(olen, seed)
    dst = np.full(int(out_off[-1]) + 1, SENTINEL, dtype=np.uint8)
    out_len = np.full(nbuf + 1, -7, dtype=np.int64)
    a = np.frombuffer(alpha, dtype=np.uint8).copy()
    L = oracle.lib()
    if flags is None:
        L.b64o_encode_list(_ptr(src), _ptr(in_off), nbuf, _ptr(dst), _ptr(out_off), _ptr(out_len),
                           _ptr(a))
    else:
        L.b64o_encode_mode_list(_ptr(src), _ptr(in_off), nbuf, _ptr(dst), _ptr(out_off),
                                _ptr(out_len), _ptr(a), flags, line_len)
    assert out_len[nbuf] == -7, "wrote past out_len[nbuf-1]"
    return dst, out_off, out_len[:nbuf], olen


def _run_decode_list(oracle, src, in_off, alpha, flags=None, seed=0):
    nbuf = in_off.size - 1
    lens = np.diff(in_off)
    cap = 3 * (lens // 4)
    if flags is not None and flags & oracle.NOPAD:
        cap = cap + np.maximum(lens % 4 - 1, 0)
    out_off = _gapped(cap, seed)
    dst = np.full(int(out_off[-1]) + 1, SENTINEL, dtype=np.uint8)
    res = np.full(nbuf + 1, -7, dtype=np.int64)
    a = np.frombuffer(alpha, dtype=np.uint8).copy()
    L = oracle.lib()
    if flags is None:
        L.b64o_decode_list(_ptr(src), _ptr(in_off), nbuf, _ptr(dst), _ptr(out_off), _ptr(res),
                           _ptr(a))
    else:
        L.b64o_decode_mode_list(_ptr(src), _ptr(in_off), nbuf, _ptr(dst), _ptr(out_off), _ptr(res),
                                _ptr(a), flags)
    assert res[nbuf] == -7, "wrote past result[nbuf-1]"
    return dst, out_off, res[:nbuf], cap


def _check_gaps(dst, out_off, used):
    """Every byte outside [out_off[b], out_off[b] + used[b]) keeps the sentinel."""
    mask = np.ones(dst.size, dtype=bool)
    for b in range(used.size):
        mask[out_off[b]: out_off[b] + max(int(used[b]), 0)] = False
    assert (dst[mask] == SENTINEL).all(), "a helper wrote outside its buffer's output"


@pytest.mark.parametrize("alpha", [STD, URL], ids=["std", "url"])
def test_encode_list_matches_stdlib_per_buffer(oracle, alpha):
    lens = _lengths(workloads.SEED_BASE + 400, 600, 700)
    in_off = workloads.offsets(lens)
    src = workloads.random_bytes(workloads.SEED_BASE + 401, int(in_off[-1]))
    dst, out_off, out_len, olen = _run_encode_list(oracle, src, in_off, alpha, seed=402)
    assert np.array_equal(out_len, olen)
    for b, x in enumerate(_buffers(src, in_off)):
        got = bytes(dst[out_off[b]: out_off[b] + out_len[b]])
        assert got == encode_ref(x, alpha), b
    _check_gaps(dst, out_off, out_len)
    # the Python wrapper: packed outputs, the same bytes
    wdst, woff, wlen = oracle.encode_list(src, in_off, alpha)
    assert np.array_equal(wlen, olen) and np.array_equal(np.diff(woff), olen)
    assert bytes(wdst) == b"".join(encode_ref(x, alpha) for x in _buffers(src, in_off))


@pytest.mark.parametrize("alpha", [STD, URL], ids=["std", "url"])
def test_decode_list_matches_prefix_rule_per_buffer(oracle, alpha):
    lens = _lengths(workloads.SEED_BASE + 403, 600, 500)
    raw = workloads.random_bytes(workloads.SEED_BASE + 404, int(lens.sum()))
    payloads = _buffers(raw, workloads.offsets(lens))
    texts = [encode_ref(x, alpha) for x in payloads]
    texts = _spoil(texts, workloads.SEED_BASE + 405, alpha)
    # a few buffers of raw bytes and of '=' runs
    texts[10:14] = [b"=", b"A===", bytes(raw[:9]), b"QR=="]
    src, in_off, tl = _pack(texts)
    dst, out_off, res, cap = _run_decode_list(oracle, src, in_off, alpha, seed=406)
    rule = PrefixRule(alpha)
    nvalid = 0
    std_text = bytes.maketrans(alpha, STD)
    for b, t in enumerate(texts):
        exp = rule.result(t)
        assert res[b] == exp, (b, t[:40], res[b], exp)
        if exp >= 0:
            nvalid += 1
            ref = base64.b64decode(t.translate(std_text), validate=True)
            assert bytes(dst[out_off[b]: out_off[b] + exp]) == ref, b
    assert 100 < nvalid < len(texts) - 100
    _check_gaps(dst, out_off, np.where(res >= 0, res, 0))
    # the Python wrapper gives the same per-buffer results
    _, _, wres = oracle.decode_list(src, in_off, alpha)
    assert np.array_equal(wres, res)


@pytest.mark.parametrize("line_len", [0, 4, 76])
def test_encode_mode_list_matches_stdlib_per_buffer(oracle, line_len):
    lens = _lengths(workloads.SEED_BASE + 407, 400, 600)
    in_off = workloads.offsets(lens)
    src = workloads.random_bytes(workloads.SEED_BASE + 408, int(in_off[-1]))
    for flags in (0, oracle.NOPAD):
        for alpha in (STD, URL):
            dst, out_off, out_len, olen = _run_encode_list(oracle, src, in_off, alpha, flags,
                                                           line_len, seed=409 + flags)
            assert np.array_equal(out_len, olen)
            for b, x in enumerate(_buffers(src, in_off)):
                text = ref_nopad(x, alpha) if flags else encode_ref(x, alpha)
                exp = ref_wrap(text, line_len) if line_len else text
                got = bytes(dst[out_off[b]: out_off[b] + out_len[b]])
                assert got == exp, (b, flags, line_len)
            _check_gaps(dst, out_off, out_len)
    if line_len == 0:
        wdst, woff, wlen = oracle.encode_mode_list(src, in_off, STD, oracle.NOPAD)
        assert bytes(wdst) == b"".join(ref_nopad(x, STD) for x in _buffers(src, in_off))


def test_decode_mode_list_nopad_matches_stdlib_per_buffer(oracle):
    lens = _lengths(workloads.SEED_BASE + 411, 500, 400)
    raw = workloads.random_bytes(workloads.SEED_BASE + 412, int(lens.sum()))
    payloads = _buffers(raw, workloads.offsets(lens))
    for alpha in (STD, URL):
        texts = _spoil([ref_nopad(x, alpha) for x in payloads], workloads.SEED_BASE + 413, alpha)
        texts[10:13] = [b"A", b"QR", b"QRS="]
        src, in_off, _ = _pack(texts)
        dst, out_off, res, cap = _run_decode_list(oracle, src, in_off, alpha, oracle.NOPAD, seed=414)
        std_text = bytes.maketrans(alpha, STD)
        for b, t in enumerate(texts):
            exp = nopad_reference(t, alpha)
            assert res[b] == exp, (b, t[:40], res[b], exp)
            if exp >= 0:
                pad = b"=" * ((4 - len(t) % 4) % 4)
                ref = base64.b64decode(t.translate(std_text) + pad, validate=True)
                assert bytes(dst[out_off[b]: out_off[b] + exp]) == ref, b
        assert (res >= 0).sum() > 100
        _check_gaps(dst, out_off, np.where(res >= 0, res, 0))
        _, _, wres = oracle.decode_mode_list(src, in_off, alpha, oracle.NOPAD)
        assert np.array_equal(wres, res)


@pytest.mark.parametrize("nopad", [0, 1])
def test_decode_mode_list_skip_ws_matches_reference_per_buffer(oracle, nopad):
    flags = oracle.SKIP_WS | (oracle.NOPAD if nopad else 0)
    lens = _lengths(workloads.SEED_BASE + 415, 300, 300)
    raw = workloads.random_bytes(workloads.SEED_BASE + 416, int(lens.sum()))
    payloads = _buffers(raw, workloads.offsets(lens))
    texts = []
    for x in payloads:
        t = ref_nopad(x, STD) if nopad else encode_ref(x, STD)
        texts.append(ref_wrap(t, 8))          # CR LF every 8 characters
    texts = _spoil(texts, workloads.SEED_BASE + 417, STD, skip_ws=True)
    texts[10:13] = [b"\r\n", b" \t", b"QR==\n"]
    src, in_off, _ = _pack(texts)
    dst, out_off, res, cap = _run_decode_list(oracle, src, in_off, STD, flags, seed=418)
    for b, t in enumerate(texts):
        exp = skip_ws_reference(t, STD, bool(nopad))
        assert res[b] == exp, (b, t[:40], res[b], exp)
        if exp >= 0:
            c = bytes(ch for ch in t if ch not in WS)
            pad = b"=" * ((4 - len(c) % 4) % 4) if nopad else b""
            ref = base64.b64decode(c + pad, validate=True)
            assert bytes(dst[out_off[b]: out_off[b] + exp]) == ref, b
    assert (res >= 0).sum() > 50
    _check_gaps(dst, out_off, np.where(res >= 0, res, 0))
