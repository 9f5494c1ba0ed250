"""Pins for the oracle's decoder (CPU only).

  - Figure fig:decoding1's worked example (golden fixture): 'd' -> 0x1d,
    '6' -> 0x3a, 0xff and 0xc3 invalid (0xc3 although its low 7 bits are 'C').
  - Exhaustive round trip over all 2^24 groups (every one of the 64^4 valid
    data quanta) and agreement with the standard-library decoder on them.
  - Round trips for every length 0..4096 with the standard and URL alphabets,
    and with two custom alphabets (one of them with bytes >= 0x80).
  - The first invalid offset against an independent definition (longest
    prefix still extendable to a valid encoding, built from the images of the
    standard-library encoder): every non-alphabet byte value at every position
    of first, middle and last quanta, and brute force over all strings of
    length <= 8 drawn from small symbol sets chosen to exercise the '=' rules
    and the canonical-bits checks.
"""
import base64
import os

import numpy as np
import pytest

import workloads
from stdlib_refs import STD, PrefixRule, brute_force_results, encode_ref, translator

URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"


def _all_groups() -> np.ndarray:
    g = np.arange(1 << 24, dtype=np.uint32)
    out = np.empty((1 << 24, 3), dtype=np.uint8)
    out[:, 0] = g >> 16
    out[:, 1] = (g >> 8) & 0xFF
    out[:, 2] = g & 0xFF
    return out.reshape(-1)


def test_figure_decoding1_worked_example(oracle, golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "fig_decoding1.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            pos, inp, out = line.split()
            rows.append((int(pos), int(inp, 16), out))
    assert len(rows) == 4
    for pos, c, out in rows:
        if out == "invalid":
            # the byte alone, placed at each position of an otherwise valid quantum
            for p in range(4):
                q = bytearray(b"AAAA")
                q[p] = c
                assert oracle.decode_raw(bytes(q)) == ~p
        else:
            v = int(out, 16)
            # value v as the first character: first byte = v*4 + 0
            dec, bad = oracle.decode(bytes([c]) + b"AAA")
            assert bad is None and dec[0] == (v * 4) & 0xFF
            # value v as the last character: third byte = 0 + v
            dec, bad = oracle.decode(b"AAA" + bytes([c]))
            assert bad is None and dec[2] == v
    # the whole example quantum: first error at byte 2 (0xff)
    assert oracle.decode_raw(bytes([0x64, 0x36, 0xFF, 0xC3])) == ~2


def test_closed_form_4_to_3_on_all_quanta(oracle):
    """All 2^24 groups encode to all 64^4 data quanta; decoding must invert
    exactly, and agree with the standard library."""
    x = _all_groups()
    text = np.frombuffer(base64.b64encode(x.tobytes()), dtype=np.uint8)
    dec, bad = oracle.decode(text)
    assert bad is None
    assert np.array_equal(dec, x)


@pytest.mark.parametrize("alpha", [STD, URL], ids=["std", "url"])
def test_round_trip_lengths_0_4096(oracle, alpha):
    data = workloads.random_bytes(workloads.SEED_BASE + 110, 4096 * 2)
    for n in range(0, 4097):
        x = data[n: 2 * n]
        text = encode_ref(x.tobytes(), alpha)
        dec, bad = oracle.decode(text, alpha)
        assert bad is None, n
        assert dec.tobytes() == x.tobytes(), n
        # standard library on the same canonical text
        std_text = text.translate(bytes.maketrans(alpha, STD))
        assert base64.b64decode(std_text, validate=True) == x.tobytes()


def test_custom_alphabets_round_trip(oracle):
    g = workloads.rng(workloads.SEED_BASE + 111)
    printable = np.array([c for c in range(0x21, 0x7F) if c != ord("=")], dtype=np.uint8)
    ascii_perm = bytes(g.permutation(printable)[:64])
    high = bytes(g.choice(np.array([c for c in range(256) if c != ord("=")], dtype=np.uint8),
                          size=64, replace=False))
    x = workloads.random_bytes(workloads.SEED_BASE + 112, 5000)
    for alpha in (ascii_perm, high):
        rule = PrefixRule(alpha)
        for n in (0, 1, 2, 3, 4, 5, 63, 64, 65, 4999, 5000):
            text = encode_ref(x[:n].tobytes(), alpha)
            dec, bad = oracle.decode(text, alpha)
            assert bad is None and dec.tobytes() == x[:n].tobytes()
            assert rule.result(text) == len(dec)
        # a standard character that is not in this alphabet is invalid
        missing = [c for c in STD if c not in alpha]
        if missing:
            s = bytearray(encode_ref(x[:30].tobytes(), alpha))
            s[13] = missing[0]
            assert oracle.decode_raw(bytes(s), alpha) == ~13 == rule.result(bytes(s))


def test_encode_decode_encode_is_identity_on_valid_text(oracle):
    """Non-canonical trailing bits are rejected, so every accepted text is the
    encoding of its decoding."""
    data = workloads.random_bytes(workloads.SEED_BASE + 113, 300)
    for n in range(0, 300):
        text = oracle.encode(data[:n])
        dec, bad = oracle.decode(text)
        assert bad is None
        assert oracle.encode(dec).tobytes() == text.tobytes()


def test_non_canonical_padding_rejected(oracle):
    """'QR==' carries a nonzero low nibble before '=='; the standard library
    (Python 3.10) accepts it, this decoder rejects it at the first '='."""
    assert base64.b64decode(b"QR==", validate=True) == b"A"
    assert oracle.decode_raw(b"QR==") == ~2
    assert oracle.decode_raw(b"QUF=") == ~3          # 'F' = 5: low two bits nonzero
    assert oracle.decode_raw(b"QUE=") == 2           # 'E' = 4: canonical
    assert oracle.decode_raw(b"QQ==") == 1


@pytest.mark.parametrize("where", ["first", "middle", "last"])
def test_every_invalid_byte_at_every_position(oracle, where):
    """Each of the 192 byte values outside the alphabet (including '=' where it
    is misplaced, and whitespace) at every position of a quantum."""
    rule = PrefixRule(STD)
    x = workloads.random_bytes(workloads.SEED_BASE + 114, 30)
    base = bytearray(encode_ref(x.tobytes()))       # 40 chars, 10 quanta, no pad
    qstart = {"first": 0, "middle": 20, "last": 36}[where]
    outside = [c for c in range(256) if c not in STD]
    assert len(outside) == 192
    for c in outside:
        for p in range(4):
            s = bytearray(base)
            s[qstart + p] = c
            got = oracle.decode_raw(bytes(s))
            assert got == rule.result(bytes(s)), (c, p)
            if c != ord("="):
                assert got == ~(qstart + p)


def test_whitespace_is_invalid(oracle):
    for ws in b" \t\r\n":
        assert oracle.decode_raw(b"QUFB" + bytes([ws]) + b"QUFB") == ~4


def test_truncated_lengths(oracle):
    text = encode_ref(b"0123456789")                 # 16 chars
    for n in range(0, 16):
        got = oracle.decode_raw(text[:n])
        if n % 4 == 0:
            assert got == 3 * (n // 4)
        else:
            assert got == ~n


@pytest.mark.parametrize("symbols,maxlen", [
    # values 0, 1, 16, 48 (exercise the canonical-bit checks), '=', '!', 0xC3
    ([ord("A"), ord("B"), ord("Q"), ord("w"), ord("="), ord("!"), 0xC3], 8),
    # values 0, 1, 4, 16: separates the two-bit (xyz=) and four-bit (xy==) checks
    ([ord("A"), ord("B"), ord("E"), ord("Q"), ord("="), ord("\n")], 8),
], ids=["set7", "set6"])
def test_brute_force_first_invalid_offset(oracle, symbols, maxlen):
    total = 0
    for length in range(0, maxlen + 1):
        rows, expected = brute_force_results(symbols, length)
        got = oracle.decode_rows(rows) if length else np.array([oracle.decode_raw(b"")])
        bad = np.nonzero(got != expected)[0]
        assert bad.size == 0, (length, rows[bad[:5]], got[bad[:5]], expected[bad[:5]])
        total += rows.shape[0]
    assert total == sum(len(symbols) ** l for l in range(maxlen + 1))


def test_prefix_rule_and_brute_force_agree(oracle):
    """The two independent formulations of the prefix rule agree with each other."""
    rule = PrefixRule(STD)
    syms = [ord("A"), ord("B"), ord("Q"), ord("="), ord("!")]
    for length in range(0, 7):
        rows, expected = brute_force_results(syms, length)
        for k in range(0, rows.shape[0], 7):
            assert rule.result(rows[k].tobytes()) == expected[k]


def test_bad_arguments(oracle):
    assert oracle.decode_raw(b"QUFB", STD[:63] + b"=") == oracle.EARG
    assert oracle.decode_raw(b"QUFB", STD[:62] + b"AA") == oracle.EARG
