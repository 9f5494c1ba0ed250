"""Pins for the oracle's encoder (CPU only).

Each test checks the oracle against something other than itself:
  - Table tab:base64table (golden fixture transcribed from the paper),
  - the paper's own encoding identities of Section "Encoding" (byte gather
    s1,s2,s3 -> s2,s1,s3,s2 and the multishift amounts 10,4,22,16),
  - Python's standard-library encoder on all 2^24 three-byte groups and on
    random inputs of every length 0..4096 (all n mod 3 cases),
  - the padding/length rule of Section "Base64".
"""
import base64
import os

import numpy as np
import pytest

import workloads
from stdlib_refs import STD, encode_ref

URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"


def _table(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "table_base64.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v, h, c = line.split()
            rows.append((int(v), int(h, 16), c))
    return rows


def _all_groups() -> np.ndarray:
    """All 2^24 three-byte groups, big-endian counter order, 48 MiB."""
    g = np.arange(1 << 24, dtype=np.uint32)
    out = np.empty((1 << 24, 3), dtype=np.uint8)
    out[:, 0] = g >> 16
    out[:, 1] = (g >> 8) & 0xFF
    out[:, 2] = g & 0xFF
    return out.reshape(-1)


def test_table_rows_give_characters(oracle, golden_dir):
    """Group (4v, 0, v): its first index is 4v div 4 = v and its last is v mod 64
    = v; both characters must be the table's character for v."""
    rows = _table(golden_dir)
    assert len(rows) == 64
    for v, hexval, ch in rows:
        assert ord(ch) == hexval
        out = oracle.encode(bytes([4 * v, 0, v]))
        assert out[0] == hexval, v
        assert out[3] == hexval, v


def test_url_alphabet_substitution(oracle):
    """base64url differs from the standard alphabet only in values 62 and 63."""
    assert sum(a != b for a, b in zip(STD, URL)) == 2
    assert oracle.encode(bytes([0xFB, 0xFF, 0xFF]), URL).tobytes() == b"-___"
    assert oracle.encode(bytes([0xFB, 0xFF, 0xFF]), STD).tobytes() == b"+///"


def test_padding_and_length(oracle):
    """4*ceil(n/3) characters; zero, two or one '=' for n mod 3 = 0, 1, 2."""
    for n in range(0, 4097):
        assert oracle.encoded_len(n) == 4 * -(-n // 3)
    for n in range(0, 200):
        out = oracle.encode(np.full(n, 0xA5, dtype=np.uint8)).tobytes()
        assert len(out) == 4 * -(-n // 3)
        assert out.count(b"=") == {0: 0, 1: 2, 2: 1}[n % 3]
        if n:
            assert out.endswith({0: b"", 1: b"==", 2: b"="}[n % 3])


def test_all_groups_match_stdlib(oracle):
    """Exhaustive: all 2^24 groups, compared with the standard library."""
    x = _all_groups()
    got = oracle.encode(x)
    ref = np.frombuffer(base64.b64encode(x.tobytes()), dtype=np.uint8)
    assert got.size == ref.size == 4 << 24
    assert np.array_equal(got, ref)


def test_all_groups_are_a_bijection_onto_alphabet_quads(oracle):
    """Section "Base64": the map from three bytes to four 6-bit values is
    bijective, so the 2^24 images are exactly the 64^4 quads of characters."""
    got = oracle.encode(_all_groups()).view(np.uint32)
    assert np.unique(got).size == 1 << 24
    assert np.isin(got.view(np.uint8), np.frombuffer(STD, dtype=np.uint8)).all()


def test_paper_gather_and_multishift_identity(oracle, golden_dir):
    """Section "Encoding": gather (s1,s2,s3) -> (s2,s1,s3,s2), then take the low
    six bits of the 32-bit word shifted right by 10, 4, 22, 16.  On every group
    the resulting indices must address the oracle's characters."""
    gather = np.loadtxt(os.path.join(golden_dir, "fig_encoding_gather.txt"),
                        comments="#", dtype=np.int64).reshape(-1)
    shifts = np.loadtxt(os.path.join(golden_dir, "encoding_shifts.txt"),
                        comments="#", dtype=np.int64).reshape(-1)
    # the printed example: input bytes 0..47, group j = (3j, 3j+1, 3j+2),
    # becomes (3j+1, 3j, 3j+2, 3j+1), i.e. (s2, s1, s3, s2)
    j = np.arange(16)
    assert np.array_equal(gather.reshape(16, 4),
                          np.stack([3 * j + 1, 3 * j, 3 * j + 2, 3 * j + 1], axis=1))
    groups = _all_groups().reshape(-1, 3).astype(np.uint64)
    s1, s2, s3 = groups[:, 0], groups[:, 1], groups[:, 2]
    # bytes laid out little-endian in one word: s2 | s1<<8 | s3<<16 | s2<<24
    w = s2 | (s1 << 8) | (s3 << 16) | (s2 << 24)
    idx = np.stack([(w >> np.uint64(s)) & np.uint64(63) for s in shifts[:4]], axis=1)
    # the upper four shifts address the next 32-bit word of the 64-bit lane
    assert list(shifts[4:] - 32) == list(shifts[:4])
    chars = np.frombuffer(STD, dtype=np.uint8)[idx.astype(np.int64)]
    got = oracle.encode(_all_groups()).reshape(-1, 4)
    assert np.array_equal(got, chars)


@pytest.mark.parametrize("alpha", [STD, URL], ids=["std", "url"])
def test_random_lengths_0_4096_match_stdlib(oracle, alpha):
    data = workloads.random_bytes(workloads.SEED_BASE + 100, 4096 * 2)
    for n in range(0, 4097):
        x = data[n: 2 * n]
        assert oracle.encode(x, alpha).tobytes() == encode_ref(x.tobytes(), alpha), n


def test_one_mib_matches_stdlib(oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 101, (1 << 20) + 1)
    assert oracle.encode(x).tobytes() == base64.b64encode(x.tobytes())
    assert oracle.encode(x, URL).tobytes() == base64.urlsafe_b64encode(x.tobytes())


def test_custom_alphabets_match_translated_stdlib(oracle):
    g = workloads.rng(workloads.SEED_BASE + 102)
    printable = np.array([c for c in range(0x21, 0x7F) if c != ord("=")], dtype=np.uint8)
    ascii_perm = bytes(g.permutation(printable)[:64])
    high = bytes(g.choice(np.array([c for c in range(256) if c != ord("=")], dtype=np.uint8),
                          size=64, replace=False))
    x = workloads.random_bytes(workloads.SEED_BASE + 103, 10000)
    for alpha in (ascii_perm, high):
        assert oracle.alphabet_ok(alpha)
        for n in (0, 1, 2, 3, 47, 48, 49, 9999, 10000):
            assert oracle.encode(x[:n], alpha).tobytes() == encode_ref(x[:n].tobytes(), alpha)


def test_bad_alphabets_rejected(oracle):
    assert not oracle.alphabet_ok(STD[:63] + b"A")       # duplicate
    assert not oracle.alphabet_ok(STD[:63] + b"=")       # contains the pad
    assert oracle.alphabet_ok(STD) and oracle.alphabet_ok(URL)
    with pytest.raises(ValueError):
        oracle.encode(b"abc", STD[:63] + b"=")
