"""The oracle: a plain scalar CPU base64 codec, written in C (b64_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product
library never loads it and shares no code with it; the two meet only through
the seeded input generators in ``workloads``.

Functions follow Section "Base64" of Mula & Lemire (the closed forms, Table
tab:base64table, '=' padding, base64url) and Section "Encoding" step 2 (any
64-byte alphabet).  See b64_oracle.c for the readings taken where the paper is
silent.

Python API (numpy uint8 arrays in, numpy arrays out):
  encode(x, alpha=STD) -> uint8 array of 4*ceil(n/3) characters
  decode(s, alpha=STD) -> (uint8 array, None) if valid, (None, first_bad) if not
  decode_raw(s, alpha) -> the C return value (length, or ~first_bad)
  decode_rows(rows2d, alpha) -> int64 array of C return values, one per row
  encode_list / decode_list -> per-buffer results over packed buffers
  encode_mode / decode_mode / decode_mode_raw / decode_mode_rows /
  encoded_len_mode / encode_mode_list / decode_mode_list -> the variants:
  flags NOPAD (no '=') and SKIP_WS (decode ignores space, tab, CR, LF), and
  line_len > 0 (encode breaks lines with CR LF)
  f32_to_bf16 / decode_f32_bf16_rows -> the fused consumer: rows of base64
  float32 decoded into bfloat16 (round to nearest, ties to even)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "b64_oracle.c")
_LIB = os.path.join(_HERE, "libb64oracle.so")

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"
EARG = -(2 ** 63)
NOPAD = 1
SKIP_WS = 2


def build(force: bool = True) -> str:
    """Compile b64_oracle.c with gcc -O2 into oracle/libb64oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC",
                               "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        p, i64, vp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
        L.b64o_encoded_len.argtypes = [i64]
        L.b64o_encoded_len.restype = i64
        L.b64o_alphabet_ok.argtypes = [p]
        L.b64o_alphabet_ok.restype = ctypes.c_int
        for fn in (L.b64o_encode, L.b64o_decode):
            fn.argtypes = [p, i64, p, p]
            fn.restype = i64
        L.b64o_decode_rows.argtypes = [p, i64, i64, p, p]
        L.b64o_decode_rows.restype = None
        for fn in (L.b64o_encode_list, L.b64o_decode_list):
            fn.argtypes = [p, p, i64, p, p, p, p]
            fn.restype = None
        u32 = ctypes.c_uint
        L.b64o_encoded_len_mode.argtypes = [i64, u32, i64]
        L.b64o_encoded_len_mode.restype = i64
        L.b64o_encode_mode.argtypes = [p, i64, p, p, u32, i64]
        L.b64o_encode_mode.restype = i64
        L.b64o_decode_mode.argtypes = [p, i64, p, p, u32]
        L.b64o_decode_mode.restype = i64
        L.b64o_decode_mode_rows.argtypes = [p, i64, i64, p, u32, p]
        L.b64o_decode_mode_rows.restype = None
        L.b64o_encode_mode_list.argtypes = [p, p, i64, p, p, p, p, u32, i64]
        L.b64o_encode_mode_list.restype = None
        L.b64o_decode_mode_list.argtypes = [p, p, i64, p, p, p, p, u32]
        L.b64o_decode_mode_list.restype = None
        L.b64o_f32_to_bf16.argtypes = [ctypes.c_uint32]
        L.b64o_f32_to_bf16.restype = ctypes.c_uint16
        L.b64o_decode_f32_bf16_rows.argtypes = [p, p, i64, i64, p, p, p, u32]
        L.b64o_decode_f32_bf16_rows.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _alpha(alpha) -> np.ndarray:
    a = np.frombuffer(bytes(alpha), dtype=np.uint8)
    if a.size != 64:
        raise ValueError("alphabet must have 64 bytes")
    return np.ascontiguousarray(a)


def _u8(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(x), dtype=np.uint8)
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint8).reshape(-1))


def encoded_len(n: int) -> int:
    return int(lib().b64o_encoded_len(n))


def alphabet_ok(alpha) -> bool:
    return bool(lib().b64o_alphabet_ok(_ptr(_alpha(alpha))))


def encode(x, alpha=STD) -> np.ndarray:
    x = _u8(x)
    a = _alpha(alpha)
    out = np.empty(max(4 * ((x.size + 2) // 3), 1), dtype=np.uint8)
    r = lib().b64o_encode(_ptr(x), x.size, _ptr(out), _ptr(a))
    if r < 0:
        raise ValueError("bad argument")
    return out[:r]


def decode_raw(s, alpha=STD) -> int:
    s = _u8(s)
    a = _alpha(alpha)
    out = np.empty(max(3 * (s.size // 4) + 3, 1), dtype=np.uint8)
    return int(lib().b64o_decode(_ptr(s), s.size, _ptr(out), _ptr(a)))


def decode(s, alpha=STD):
    """(bytes, None) for valid input, (None, first_invalid_offset) otherwise."""
    s = _u8(s)
    a = _alpha(alpha)
    out = np.empty(max(3 * (s.size // 4) + 3, 1), dtype=np.uint8)
    r = int(lib().b64o_decode(_ptr(s), s.size, _ptr(out), _ptr(a)))
    if r == EARG:
        raise ValueError("bad argument")
    if r < 0:
        return None, ~r
    return out[:r], None


def decode_rows(rows: np.ndarray, alpha=STD) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.uint8)
    nrows, length = rows.shape
    a = _alpha(alpha)
    res = np.empty(nrows, dtype=np.int64)
    lib().b64o_decode_rows(_ptr(rows), nrows, length, _ptr(a), _ptr(res))
    return res


def encode_list(src: np.ndarray, in_off: np.ndarray, alpha=STD):
    """Encode packed buffers; returns (dst, out_off, out_len)."""
    src = _u8(src)
    in_off = np.ascontiguousarray(in_off, dtype=np.int64)
    nbuf = in_off.size - 1
    lens = np.diff(in_off)
    olen = 4 * ((lens + 2) // 3)
    out_off = np.zeros(nbuf + 1, dtype=np.int64)
    np.cumsum(olen, out=out_off[1:])
    dst = np.empty(max(int(out_off[-1]), 1), dtype=np.uint8)
    out_len = np.empty(max(nbuf, 1), dtype=np.int64)
    a = _alpha(alpha)
    lib().b64o_encode_list(_ptr(src), _ptr(in_off), nbuf, _ptr(dst), _ptr(out_off),
                           _ptr(out_len), _ptr(a))
    return dst[: int(out_off[-1])], out_off, out_len[:nbuf]


def decode_list(src: np.ndarray, in_off: np.ndarray, alpha=STD):
    """Decode packed buffers; returns (dst, out_off, result) where result[b] is
    the decoded length or ~first_invalid_offset, and out_off[b] is the start of
    buffer b's output (capacity 3*(len//4) each)."""
    src = _u8(src)
    in_off = np.ascontiguousarray(in_off, dtype=np.int64)
    nbuf = in_off.size - 1
    lens = np.diff(in_off)
    cap = 3 * (lens // 4) + 3
    out_off = np.zeros(nbuf + 1, dtype=np.int64)
    np.cumsum(cap, out=out_off[1:])
    dst = np.empty(max(int(out_off[-1]), 1), dtype=np.uint8)
    res = np.empty(max(nbuf, 1), dtype=np.int64)
    a = _alpha(alpha)
    lib().b64o_decode_list(_ptr(src), _ptr(in_off), nbuf, _ptr(dst), _ptr(out_off),
                           _ptr(res), _ptr(a))
    return dst, out_off, res[:nbuf]


# ------------------------------------------------------------- variants --

def encoded_len_mode(n: int, flags: int = 0, line_len: int = 0) -> int:
    return int(lib().b64o_encoded_len_mode(n, flags, line_len))


def encode_mode(x, alpha=STD, flags: int = 0, line_len: int = 0) -> np.ndarray:
    x = _u8(x)
    a = _alpha(alpha)
    m = encoded_len_mode(x.size, flags, line_len)
    if m < 0:
        raise ValueError("bad argument")
    out = np.empty(max(m, 1), dtype=np.uint8)
    r = lib().b64o_encode_mode(_ptr(x), x.size, _ptr(out), _ptr(a), flags, line_len)
    if r < 0:
        raise ValueError("bad argument")
    assert r == m
    return out[:r]


def decode_mode_raw(s, alpha=STD, flags: int = 0) -> int:
    s = _u8(s)
    a = _alpha(alpha)
    out = np.empty(max(3 * (s.size // 4) + 3, 1), dtype=np.uint8)
    return int(lib().b64o_decode_mode(_ptr(s), s.size, _ptr(out), _ptr(a), flags))


def decode_mode(s, alpha=STD, flags: int = 0):
    """(bytes, None) for valid input, (None, first_invalid_offset) otherwise."""
    s = _u8(s)
    a = _alpha(alpha)
    out = np.empty(max(3 * (s.size // 4) + 3, 1), dtype=np.uint8)
    r = int(lib().b64o_decode_mode(_ptr(s), s.size, _ptr(out), _ptr(a), flags))
    if r == EARG:
        raise ValueError("bad argument")
    if r < 0:
        return None, ~r
    return out[:r], None


def decode_mode_rows(rows: np.ndarray, alpha=STD, flags: int = 0) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.uint8)
    nrows, length = rows.shape
    a = _alpha(alpha)
    res = np.empty(nrows, dtype=np.int64)
    lib().b64o_decode_mode_rows(_ptr(rows), nrows, length, _ptr(a), flags, _ptr(res))
    return res


def encode_mode_list(src: np.ndarray, in_off: np.ndarray, alpha=STD, flags: int = 0,
                     line_len: int = 0):
    """Encode packed buffers with a variant; returns (dst, out_off, out_len)."""
    src = _u8(src)
    in_off = np.ascontiguousarray(in_off, dtype=np.int64)
    nbuf = in_off.size - 1
    olen = np.array([encoded_len_mode(int(k), flags, line_len) for k in np.diff(in_off)],
                    dtype=np.int64)
    out_off = np.zeros(nbuf + 1, dtype=np.int64)
    np.cumsum(olen, out=out_off[1:])
    dst = np.empty(max(int(out_off[-1]), 1), dtype=np.uint8)
    out_len = np.empty(max(nbuf, 1), dtype=np.int64)
    a = _alpha(alpha)
    lib().b64o_encode_mode_list(_ptr(src), _ptr(in_off), nbuf, _ptr(dst), _ptr(out_off),
                                _ptr(out_len), _ptr(a), flags, line_len)
    return dst[: int(out_off[-1])], out_off, out_len[:nbuf]


def decode_mode_list(src: np.ndarray, in_off: np.ndarray, alpha=STD, flags: int = 0):
    """Decode packed buffers with a variant; as decode_list."""
    src = _u8(src)
    in_off = np.ascontiguousarray(in_off, dtype=np.int64)
    nbuf = in_off.size - 1
    lens = np.diff(in_off)
    cap = 3 * (lens // 4) + 3
    out_off = np.zeros(nbuf + 1, dtype=np.int64)
    np.cumsum(cap, out=out_off[1:])
    dst = np.empty(max(int(out_off[-1]), 1), dtype=np.uint8)
    res = np.empty(max(nbuf, 1), dtype=np.int64)
    a = _alpha(alpha)
    lib().b64o_decode_mode_list(_ptr(src), _ptr(in_off), nbuf, _ptr(dst), _ptr(out_off),
                                _ptr(res), _ptr(a), flags)
    return dst, out_off, res[:nbuf]


# --------------------------------------------------------- fused consumer --

def f32_to_bf16(bits) -> np.ndarray:
    """bfloat16 bits of float32 bit patterns (uint32 array), one C call each."""
    bits = np.ascontiguousarray(np.asarray(bits, dtype=np.uint32).reshape(-1))
    L = lib()
    return np.array([L.b64o_f32_to_bf16(int(u)) for u in bits], dtype=np.uint16)


def decode_f32_bf16_rows(src, in_off, dim: int, alpha=STD, flags: int = 0):
    """(dst uint16 [nrows, dim], status int64 [nrows])."""
    src = _u8(src)
    in_off = np.ascontiguousarray(in_off, dtype=np.int64)
    nrows = in_off.size - 1
    dst = np.zeros((max(nrows, 1), max(dim, 1)), dtype=np.uint16)
    status = np.empty(max(nrows, 1), dtype=np.int64)
    a = _alpha(alpha)
    lib().b64o_decode_f32_bf16_rows(_ptr(src), _ptr(in_off), nrows, dim, _ptr(dst), _ptr(status),
                                    _ptr(a), flags)
    return dst[:nrows, :dim], status[:nrows]
