"""GPU parity of the single-buffer entry points (b64_encode, b64_decode,
b64_decode_async) against the oracle, bit-exact.

Covers: the 3 MiB workload with its invalid copy, all 2^24 groups, every
length 0..4096 with both alphabets, custom alphabets (one with bytes >= 0x80),
misaligned source and destination pointers, every non-alphabet byte at every
quantum position in first / body / last quanta, '=' misuse at chunk
boundaries, the size sweep 2^k + r (k = 10..26) plus the paper's four file
sizes, and the 1 GiB workload (n mod 3 = 0 and 1) with both alphabets.
"""
import numpy as np
import pytest

import workloads
from gpu_util import first_mismatch, say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


def _check_encode(b64, oracle, x, alpha=STD, label=""):
    say("encode", label, "n =", x.size)
    got = to_host(b64.encode(to_dev(x), alpha)) if x.size else np.zeros(0, np.uint8)
    ref = oracle.encode(x, alpha)
    assert first_mismatch(got, ref) is None, (label, first_mismatch(got, ref))
    return ref


def _check_decode(b64, oracle, text, alpha=STD, label=""):
    say("decode", label, "n =", text.size)
    import torch
    dtext = to_dev(text) if text.size else torch.empty(0, dtype=torch.uint8, device="cuda")
    dec, bad = b64.decode(dtext, alpha)
    ref, ref_bad = oracle.decode(text, alpha)
    assert bad == ref_bad, (label, bad, ref_bad)
    if ref_bad is None:
        got = to_host(dec)
        assert first_mismatch(got, ref) is None, (label, first_mismatch(got, ref))
    return bad


def test_single_3mib_workload(b64, oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 1, workloads.SINGLE_3MIB)
    text = _check_encode(b64, oracle, x, label="3MiB")
    assert text.size == 4_194_304
    _check_decode(b64, oracle, text, label="3MiB")
    bad_text, pos = workloads.plant_invalid(text, workloads.SEED_BASE + 1, STD)
    assert _check_decode(b64, oracle, bad_text, label="3MiB invalid") == pos
    # the asynchronous form reports the same through device memory
    out, status = b64.decode_async(to_dev(bad_text))
    assert to_host(status).tolist() == [-1, pos]
    out, status = b64.decode_async(to_dev(text))
    assert to_host(status).tolist() == [x.size, -1]
    assert first_mismatch(to_host(out)[: x.size], x) is None


def test_all_groups(b64, oracle):
    g = np.arange(1 << 24, dtype=np.uint32)
    x = np.stack([(g >> 16).astype(np.uint8), ((g >> 8) & 0xFF).astype(np.uint8),
                  (g & 0xFF).astype(np.uint8)], axis=1).reshape(-1)
    text = _check_encode(b64, oracle, x, label="all groups")
    _check_decode(b64, oracle, text, label="all quanta")


@pytest.mark.parametrize("alpha", [STD, URL], ids=["std", "url"])
def test_every_length_0_4096(b64, oracle, alpha):
    data = workloads.random_bytes(workloads.SEED_BASE + 120, 8192)
    say("lengths 0..4096", alpha[-2:])
    for n in range(0, 4097):
        x = data[n: 2 * n]
        text = _check_encode(b64, oracle, x, alpha, label=f"len {n}") if n else oracle.encode(x, alpha)
        _check_decode(b64, oracle, text, alpha, label=f"len {n}")


def test_custom_alphabets(b64, oracle):
    g = workloads.rng(workloads.SEED_BASE + 121)
    printable = np.array([c for c in range(0x21, 0x7F) if c != ord("=")], dtype=np.uint8)
    ascii_perm = bytes(g.permutation(printable)[:64])
    high = bytes(g.choice(np.array([c for c in range(256) if c != ord("=")], dtype=np.uint8),
                          size=64, replace=False))
    x = workloads.random_bytes(workloads.SEED_BASE + 122, 300_001)
    for alpha in (ascii_perm, high):
        for n in (1, 2, 3, 11, 12, 13, 767, 768, 769, 300_000, 300_001):
            text = _check_encode(b64, oracle, x[:n], alpha, label=f"custom {n}")
            _check_decode(b64, oracle, text, alpha, label=f"custom {n}")
        bad, pos = workloads.plant_invalid(oracle.encode(x, alpha), workloads.SEED_BASE + 123, alpha)
        assert _check_decode(b64, oracle, bad, alpha, label="custom invalid") == pos


def test_misaligned_pointers(b64, oracle):
    """Source and destination at every byte offset mod 16."""
    import torch
    xb = workloads.random_bytes(workloads.SEED_BASE + 124, 40_064)
    dxb = to_dev(xb)
    out = torch.empty(60_000, dtype=torch.uint8, device="cuda")
    x = xb[:27_000]
    t = oracle.encode(x)                                 # 36,000 characters
    for so in range(16):
        hb = np.concatenate([np.zeros(so, np.uint8), t, np.zeros(16, np.uint8)])
        dt = to_dev(hb)[so: so + t.size]
        for do in (0, 1, 2, 3, 5, 8, 13, 15):
            n = 37_000 + 7 * so + do
            say("misaligned encode", so, do, n)
            r = b64.encode(dxb[so: so + n], out=out[do:])
            assert first_mismatch(to_host(r), oracle.encode(xb[so: so + n])) is None, (so, do)
            say("misaligned decode", so, do)
            dec, bad = b64.decode(dt, out=out[do:])
            assert bad is None
            assert first_mismatch(to_host(dec), x) is None, (so, do)


def test_encode_to_unaligned_destinations(b64, oracle):
    """Destinations 1-3 bytes past a 4-byte boundary (no head groups, every
    chunk store unaligned): every length up to 300, lengths around rounds,
    and 64 MiB + 1 (many pipelined rounds), padded and unpadded; the bytes
    around the output stay untouched."""
    import torch
    x = workloads.random_bytes(workloads.SEED_BASE + 126, (64 << 20) + 1)
    dx = to_dev(x)
    lengths = list(range(0, 300)) + [1000, 4095, 4096, 4097, 12_345, 100_003, (3 << 20) + 1]
    for flags in (0, 1):
        for n in lengths + ([(64 << 20) + 1] if flags == 0 else []):
            ref = oracle.encode_mode(x[:n], STD, flags)
            for do in (1, 2, 3):
                if n > 5000 and do != 2 and n != (64 << 20) + 1:
                    continue
                say("unaligned destination", n, "offset", do, "flags", flags)
                buf = torch.full((ref.size + do + 64,), 0xA5, dtype=torch.uint8, device="cuda")
                b64.encode(dx[:n], STD, out=buf[do:], flags=flags)
                got = to_host(buf)
                assert first_mismatch(got[do: do + ref.size], ref) is None, (n, do, flags)
                assert (got[:do] == 0xA5).all() and (got[do + ref.size:] == 0xA5).all(), (n, do)


@pytest.mark.parametrize("where", ["first", "chunk_edge", "body", "last_body", "final"])
def test_every_invalid_byte_at_every_position(b64, oracle, where):
    x = workloads.random_bytes(workloads.SEED_BASE + 125, 3 * 1500)
    text = oracle.encode(x)                              # 6000 characters
    q = {"first": 0, "chunk_edge": 4 * 3, "body": 4 * 777, "last_body": 5992, "final": 5996}[where]
    outside = [c for c in range(256) if c not in STD]
    for c in outside:
        for p in range(4):
            s = text.copy()
            s[q + p] = c
            _check_decode(b64, oracle, s, label=f"{where} byte {c} pos {p}")


@pytest.mark.parametrize("pattern", [b"AA==", b"AAA=", b"A===", b"AB==", b"AAB=", b"=AAA", b"A=AA",
                                     b"AA=A", b"AA==AAAA", b"AAA=AAAA", b"QQ==", b"AA=!", b"AA\n="])
def test_pad_misuse_across_chunks(b64, oracle, pattern):
    """'=' rules inside the body (where lanes rescan their chunk) and at the end."""
    x = workloads.random_bytes(workloads.SEED_BASE + 126, 3 * 600)
    text = oracle.encode(x)                              # 2400 characters
    qmax = (text.size - len(pattern)) // 4
    for q in (0, 1, 3, 4, 15, 16, 63, 64, 255, 256, 592, qmax - 1, qmax):
        s = text.copy()
        at = 4 * q
        s[at: at + len(pattern)] = np.frombuffer(pattern, dtype=np.uint8)
        _check_decode(b64, oracle, s, label=f"{pattern!r} at quantum {q}")
        # the same with the text cut right after the pattern
        _check_decode(b64, oracle, s[: at + len(pattern)], label=f"{pattern!r} final at {q}")


def test_truncations(b64, oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 127, 3000)
    text = oracle.encode(x)
    for n in list(range(0, 80)) + list(range(3900, 4000)):
        _check_decode(b64, oracle, text[:n], label=f"truncated {n}")


def test_size_sweep(b64, oracle):
    lengths = workloads.sweep_lengths() + list(workloads.TABLE_PERF_LENGTHS)
    x = workloads.random_bytes(workloads.SEED_BASE + 3, max(lengths))
    for n in lengths:
        text = _check_encode(b64, oracle, x[:n], label=f"sweep {n}")
        _check_decode(b64, oracle, text, label=f"sweep {n}")


@pytest.mark.parametrize("n", workloads.SINGLE_1GIB, ids=["n_mod3_0", "n_mod3_1"])
def test_1gib_workload(b64, oracle, n):
    import torch
    say("1GiB generate", n)
    x = workloads.random_bytes(workloads.SEED_BASE + 2, n)
    dx = to_dev(x)
    for alpha in (STD, URL):
        say("1GiB encode", n, alpha[-2:])
        dtext = b64.encode(dx, alpha)
        ref = oracle.encode(x, alpha)
        got = to_host(dtext)
        assert first_mismatch(got, ref) is None
        del got
        say("1GiB decode", n, alpha[-2:])
        dec, bad = b64.decode(dtext, alpha)
        assert bad is None
        assert dec.numel() == n and torch.equal(dec, dx)
        del dec
    # one invalid byte: the reported offset is exactly where it was planted
    say("1GiB invalid")
    bad_text, pos = workloads.plant_invalid(ref, workloads.SEED_BASE + 2, URL)
    dec, bad = b64.decode(to_dev(bad_text), URL)
    assert bad == pos
    assert oracle.decode_raw(bad_text, URL) == ~pos
