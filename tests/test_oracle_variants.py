"""Pins for the oracle's variants (CPU only): unpadded output, CR LF line
wrapping and whitespace-skipping decode (Section "Base64": padding is
optional; Section "Introduction": base64 carried in MIME email).

Each pin reduces the variant to something fixed outside the oracle:
  - unpadded encode == the standard-library encoding with its '=' removed;
  - wrapped encode at 76 characters == the standard library's MIME encoder
    (base64.encodebytes) with LF turned into CR LF and the final line break
    dropped; other line lengths == the standard-library encoding cut into
    lines;
  - unpadded decode, brute force: valid exactly when every character is in the
    alphabet, the length is not 1 mod 4 and re-encoding the standard library's
    decoding gives the input back; else the first non-alphabet character, or
    the end of the input;
  - whitespace-skipping decode == the pinned padded (or unpadded) decode of the
    input with the whitespace removed, its first invalid offset mapped back to
    the input's own offsets;
  - flags 0 of the variant decoder == the base decoder (two formulations).
"""
import base64

import numpy as np
import pytest

import workloads
from stdlib_refs import (STD, WS, brute_force_results, nopad_reference, ref_nopad, ref_wrap,
                         skip_ws_reference)

URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"


def _alphabets():
    rng = np.random.default_rng(workloads.SEED_BASE + 71)
    perm = bytes(rng.permutation(np.frombuffer(STD, dtype=np.uint8)).tolist())
    hi = bytes(sorted(rng.choice(np.array([c for c in range(256) if c != ord("=") and c not in WS]),
                                 64, replace=False).tolist()))
    return [STD, URL, perm, hi]


# ---------------------------------------------------------------- encode --

def test_nopad_encode_matches_stdlib_all_lengths(oracle):
    for alpha in _alphabets():
        x = workloads.random_bytes(5, 700).tobytes()
        for n in range(0, 700, 1 if alpha == STD else 7):
            got = bytes(oracle.encode_mode(x[:n], alpha, oracle.NOPAD))
            assert got == ref_nopad(x[:n], alpha), (alpha[:4], n)
            assert oracle.encoded_len_mode(n, oracle.NOPAD) == len(got)


def test_wrap76_matches_stdlib_mime_encoder(oracle):
    x = workloads.random_bytes(6, 3000).tobytes()
    for n in list(range(0, 400)) + [2999, 3000]:
        mime = base64.encodebytes(x[:n]).replace(b"\n", b"\r\n")
        if mime.endswith(b"\r\n"):
            mime = mime[:-2]
        got = bytes(oracle.encode_mode(x[:n], STD, 0, 76))
        assert got == mime, n
        assert oracle.encoded_len_mode(n, 0, 76) == len(got)


@pytest.mark.parametrize("line_len", [4, 8, 64, 72, 76, 1000])
@pytest.mark.parametrize("flags", [0, 1])
def test_wrap_matches_cut_stdlib_encoding(oracle, line_len, flags):
    x = workloads.random_bytes(7, 1500).tobytes()
    for n in range(0, 1500, 13):
        text = base64.b64encode(x[:n])
        if flags:
            text = text.rstrip(b"=")
        got = bytes(oracle.encode_mode(x[:n], STD, flags, line_len))
        assert got == ref_wrap(text, line_len), (n, line_len, flags)
        assert oracle.encoded_len_mode(n, flags, line_len) == len(got)
        # no line is longer than line_len, and only the last may be shorter
        lines = got.split(b"\r\n")
        assert all(len(s) == line_len for s in lines[:-1])
        assert len(lines[-1]) <= line_len


def test_encoded_len_mode_closed_form(oracle):
    for n in range(0, 2000):
        padded = 4 * ((n + 2) // 3)
        nopad = (4 * n + 2) // 3
        assert oracle.encoded_len_mode(n, 0, 0) == padded
        assert oracle.encoded_len_mode(n, oracle.NOPAD, 0) == nopad
        for L in (4, 76):
            m = padded
            assert oracle.encoded_len_mode(n, 0, L) == m + 2 * max(0, (m - 1) // L)


# ---------------------------------------------------------------- decode --

@pytest.mark.parametrize("length", range(0, 8))
def test_nopad_decode_brute_force(oracle, length):
    # 'Q' has value 16 (low four bits zero), 'R' 17, 'E' 4 (low two bits zero)
    symbols = [ord(ch) for ch in "AQRE=*"]
    rows, _ = brute_force_results(symbols, length)
    got = oracle.decode_mode_rows(rows, STD, oracle.NOPAD)
    for row, g in zip(rows, got):
        assert g == nopad_reference(bytes(row), STD), (bytes(row), g)


@pytest.mark.parametrize("flags", [2, 3])
@pytest.mark.parametrize("length", range(0, 8))
def test_skip_ws_decode_brute_force(oracle, flags, length):
    symbols = [ord(ch) for ch in "AQR=\n "]
    rows, _ = brute_force_results(symbols, length)
    got = oracle.decode_mode_rows(rows, STD, flags)
    for row, g in zip(rows, got):
        assert g == skip_ws_reference(bytes(row), STD, flags & 1), (bytes(row), flags, g)


def test_flags0_agrees_with_base_decoder(oracle):
    for length in range(0, 9):
        rows, expected = brute_force_results([ord(ch) for ch in "AQR=*"], length)
        assert (oracle.decode_mode_rows(rows, STD, 0) == expected).all()
        assert (oracle.decode_rows(rows, STD) == expected).all()
    x = workloads.random_bytes(8, 5000).tobytes()
    for alpha in _alphabets():
        enc = bytes(oracle.encode(x, alpha))
        assert oracle.decode_mode_raw(enc, alpha, 0) == oracle.decode_raw(enc, alpha) == 5000


def test_nopad_round_trip_and_invalid(oracle):
    x = workloads.random_bytes(9, 3000).tobytes()
    for alpha in _alphabets():
        for n in range(0, 300):
            enc = bytes(oracle.encode_mode(x[:n], alpha, oracle.NOPAD))
            dec, bad = oracle.decode_mode(enc, alpha, oracle.NOPAD)
            assert bad is None and bytes(dec) == x[:n]
            # the padded form is not an unpadded encoding: '=' is invalid
            padded = bytes(oracle.encode(x[:n], alpha))
            if n % 3:
                assert oracle.decode_mode(padded, alpha, oracle.NOPAD) == (None, len(enc))


def test_skip_ws_decodes_stdlib_mime_output(oracle):
    x = workloads.random_bytes(10, 20000).tobytes()
    rng = np.random.default_rng(workloads.SEED_BASE + 72)
    for n in list(range(0, 200)) + [19999, 20000]:
        mime = base64.encodebytes(x[:n])                     # 76 chars + LF lines
        dec, bad = oracle.decode_mode(mime, STD, oracle.SKIP_WS)
        assert bad is None and bytes(dec) == x[:n], n
        crlf = mime.replace(b"\n", b"\r\n")
        dec, bad = oracle.decode_mode(crlf, STD, oracle.SKIP_WS)
        assert bad is None and bytes(dec) == x[:n], n
    # whitespace sprinkled anywhere, in runs of any length
    for trial in range(200):
        n = int(rng.integers(0, 300))
        text = bytearray(base64.b64encode(x[:n]))
        for _ in range(int(rng.integers(0, 20))):
            pos = int(rng.integers(0, len(text) + 1))
            run = bytes(rng.choice(np.frombuffer(WS, dtype=np.uint8), int(rng.integers(1, 6))).tolist())
            text[pos:pos] = run
        dec, bad = oracle.decode_mode(bytes(text), STD, oracle.SKIP_WS)
        assert bad is None and bytes(dec) == x[:n], trial
        # without skipping, the first whitespace byte is the first invalid offset
        first_ws = min([i for i, c in enumerate(text) if c in WS], default=None)
        if first_ws is not None:
            assert oracle.decode(bytes(text))[1] == first_ws


def test_skip_ws_invalid_offsets_random(oracle):
    rng = np.random.default_rng(workloads.SEED_BASE + 73)
    x = workloads.random_bytes(11, 400).tobytes()
    for trial in range(400):
        n = int(rng.integers(0, 120))
        flags = int(rng.integers(2, 4))
        text = bytearray(bytes(oracle.encode_mode(x[:n], STD, flags & 1, 8)))
        for _ in range(int(rng.integers(1, 4))):           # mutations
            pos = int(rng.integers(0, len(text) + 1))
            kind = int(rng.integers(0, 3))
            if kind == 0:
                text[pos:pos] = b"\t "
            elif kind == 1 and pos < len(text):
                text[pos] = int(rng.choice([ord("*"), ord("="), 0x80, ord("A")]))
            elif pos < len(text):
                del text[pos]
        s = bytes(text)
        assert oracle.decode_mode_raw(s, STD, flags) == skip_ws_reference(s, STD, flags & 1), (s, flags)


def test_variant_argument_errors(oracle):
    EARG = oracle.EARG
    L = oracle.lib()
    a = np.frombuffer(STD, dtype=np.uint8).copy()
    src = np.zeros(8, dtype=np.uint8)
    dst = np.zeros(64, dtype=np.uint8)
    assert L.b64o_encode_mode(src.ctypes.data, 8, dst.ctypes.data, a.ctypes.data, 2, 0) == EARG
    assert L.b64o_encode_mode(src.ctypes.data, 8, dst.ctypes.data, a.ctypes.data, 0, -1) == EARG
    assert L.b64o_decode_mode(src.ctypes.data, 8, dst.ctypes.data, a.ctypes.data, 4) == EARG
    assert oracle.encoded_len_mode(-1) == EARG
    # whitespace skipping is undefined for an alphabet that holds whitespace
    with_space = bytearray(STD)
    with_space[62] = ord(" ")
    ws = np.frombuffer(bytes(with_space), dtype=np.uint8).copy()
    assert L.b64o_decode_mode(src.ctypes.data, 8, dst.ctypes.data, ws.ctypes.data, 2) == EARG
    assert L.b64o_decode_mode(src.ctypes.data, 8, dst.ctypes.data, ws.ctypes.data, 1) != EARG
