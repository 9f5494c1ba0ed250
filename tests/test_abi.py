"""The C-ABI library loads and exports every symbol that include/b64hip.h
declares; host-side argument checks work without a GPU (CPU only: nothing
here launches a kernel)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "b64hip.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    funcs = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(b64_\w+)\s*\(", text, flags=re.M)
    data = re.findall(r"extern\s+const\s+char\s+(b64_\w+)\s*\[", text)
    return funcs, data


@pytest.fixture(scope="module")
def lib():
    from paper_1910_05109_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libb64hip.so not built")
    return _lib.load()


def test_header_declares_the_boundary():
    funcs, data = _declared()
    assert set(funcs) == {
        "b64_encoded_len", "b64_decoded_max_len", "b64_encode", "b64_decode", "b64_decode_async",
        "b64_validate", "b64_validate_async", "b64_encode_batch", "b64_decode_batch",
        "b64_encoded_len_mode", "b64_decoded_max_len_mode", "b64_decode_workspace_size",
        "b64_encode_mode", "b64_decode_mode", "b64_decode_mode_async", "b64_validate_mode",
        "b64_validate_mode_async", "b64_encode_batch_mode", "b64_decode_batch_mode",
        "b64_decode_ws_async_noalloc", "b64_decode_f32_bf16",
        "b64_pipeline_create", "b64_pipeline_destroy", "b64_pipeline_encode",
        "b64_pipeline_decode", "b64_pipeline_last_error",
        "b64_server_create", "b64_server_destroy", "b64_server_last_error", "b64_server_run",
        "b64_server_set_zero_copy_max", "b64_server_set_staging",
        "b64_tune_set_bucket", "b64_tune_set", "b64_tune_get_bucket", "b64_tune_get",
        "b64_tune_bucket", "b64_tune_ws_guess_min", "b64_tune_ws_small_max", "b64_yardstick",
        "b64_last_error"}
    assert set(data) == {"b64_alphabet_std", "b64_alphabet_url"}


def test_library_exports_every_declared_symbol(lib):
    from paper_1910_05109_amd import _lib
    funcs, data = _declared()
    for name in funcs + data:
        assert hasattr(lib, name), name
    assert set(funcs) == set(_lib.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in funcs + data:
        assert name in exported, name


def test_alphabet_constants(lib, golden_dir):
    from paper_1910_05109_amd import _lib, STD, URL
    rows = [l.split() for l in open(os.path.join(golden_dir, "table_base64.txt"))
            if not l.startswith("#")]
    table = bytes(int(h, 16) for _, h, _ in rows)
    assert _lib.alphabet_bytes("std") == table == STD
    assert _lib.alphabet_bytes("url") == table[:62] + b"-_" == URL


def test_length_helpers(lib):
    for n in range(0, 100):
        assert lib.b64_encoded_len(n) == 4 * ((n + 2) // 3)
        assert lib.b64_decoded_max_len(n) == 3 * (n // 4)
    assert lib.b64_encoded_len(-1) == -(2 ** 63)
    assert lib.b64_decoded_max_len(-5) == -(2 ** 63)
    big = (1 << 40) + 1
    assert lib.b64_encoded_len(big) == 4 * ((big + 2) // 3)


def test_variant_length_helpers_match_oracle(lib, oracle):
    """Output lengths and capacities of the variants, against the oracle's
    own encoder (lengths) and decoder (largest valid output)."""
    EARG = -(2 ** 63)
    for n in range(0, 200):
        for flags in (0, 1):
            for L in (0, 4, 8, 76, 1000):
                assert lib.b64_encoded_len_mode(n, flags, L) == oracle.encoded_len_mode(n, flags, L)
        r = n % 4
        assert lib.b64_decoded_max_len_mode(n, 0) == 3 * (n // 4)
        assert lib.b64_decoded_max_len_mode(n, 2) == 3 * (n // 4)
        assert lib.b64_decoded_max_len_mode(n, 1) == 3 * (n // 4) + max(0, r - 1)
        assert lib.b64_decoded_max_len_mode(n, 3) == 3 * (n // 4) + max(0, r - 1)
        assert lib.b64_decode_workspace_size(n, 0) == 0
        assert lib.b64_decode_workspace_size(n, 1) == 0
        assert lib.b64_decode_workspace_size(n, 2) >= 16
    # the largest unpadded decoded length fits the capacity
    for n in range(0, 64):
        m = oracle.encoded_len_mode(n, 1)
        assert lib.b64_decoded_max_len_mode(m, 1) >= n
    assert lib.b64_encoded_len_mode(5, 2, 0) == EARG        # SKIP_WS is a decode flag
    assert lib.b64_encoded_len_mode(5, 0, 6) == EARG        # line length not a multiple of 4
    assert lib.b64_encoded_len_mode(5, 0, -4) == EARG
    assert lib.b64_decoded_max_len_mode(5, 4) == EARG
    assert lib.b64_decode_workspace_size(-1, 2) == EARG
    # workspace: 8 bytes per tile (4 KiB .. 32 KiB) plus 24
    big = 1 << 30
    ws = lib.b64_decode_workspace_size(big, 2)
    assert 24 + 8 * (big // 32768) <= ws <= 24 + 8 * (big // 4096 + 1)


def test_argument_errors_without_gpu(lib):
    """Bad arguments are rejected on the host, before any HIP call."""
    EARG = -(2 ** 63)
    std = ctypes.create_string_buffer(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/", 64)
    dup = ctypes.create_string_buffer(b"A" * 64, 64)
    with_pad = ctypes.create_string_buffer(b"=" + std.raw[1:], 64)
    fake = ctypes.c_void_p(0x1000)
    assert lib.b64_encode(fake, -1, fake, std, None) == EARG
    assert lib.b64_encode(None, 10, fake, std, None) == EARG
    assert lib.b64_encode(fake, 10, fake, dup, None) == EARG
    assert lib.b64_encode(fake, 10, fake, with_pad, None) == EARG
    assert lib.b64_encode(fake, 10, fake, None, None) == EARG
    assert lib.b64_decode(fake, 10, fake, with_pad, None) == EARG
    assert lib.b64_decode(fake, -3, fake, std, None) == EARG
    assert lib.b64_decode_async(fake, 10, fake, None, fake, std, None) == EARG
    assert lib.b64_validate(None, 10, std, None) == EARG
    assert lib.b64_validate(fake, 10, dup, None) == EARG
    assert lib.b64_validate_async(fake, 10, fake, None, std, None) == EARG
    # the allocation-free whitespace decode: B64_SKIP_WS required, length capped
    assert lib.b64_decode_ws_async_noalloc(fake, 10, fake, fake, fake, std, 0, None) == EARG
    assert lib.b64_decode_ws_async_noalloc(fake, 10, fake, fake, fake, std, 1, None) == EARG
    assert lib.b64_decode_ws_async_noalloc(fake, 4294868993, fake, fake, fake, std, 2, None) == EARG
    assert b"B64_NOALLOC_MAX_CHARS" in lib.b64_last_error()
    assert lib.b64_decode_ws_async_noalloc(fake, -1, fake, fake, fake, std, 2, None) == EARG
    assert lib.b64_decode_ws_async_noalloc(fake, 10, fake, None, fake, std, 2, None) == EARG
    assert lib.b64_decode_ws_async_noalloc(fake, 10, fake, fake, fake, dup, 2, None) == EARG
    # the cap matches the workspace the whitespace decode needs
    assert lib.b64_decode_workspace_size(4294868992, 2) == 1 << 20
    assert lib.b64_decode_workspace_size(4294868993, 2) > 1 << 20
    assert lib.b64_encode_batch(fake, fake, -1, fake, fake, fake, std, None) == EARG
    assert lib.b64_encode_batch(fake, None, 3, fake, fake, fake, std, None) == EARG
    assert lib.b64_decode_batch(fake, fake, 3, fake, fake, fake, None, std, None) == EARG
    assert lib.b64_decode_batch(fake, fake, 3, fake, fake, fake, fake, dup, None) == EARG
    assert b"alphabet" in lib.b64_last_error()
    assert lib.b64_pipeline_create(10, 2, 1) is None             # chunk too small
    assert lib.b64_pipeline_create(1 << 20, 0, 1) is None        # no slots
    assert b"chunk_bytes" in lib.b64_pipeline_last_error()
    assert lib.b64_pipeline_encode(None, fake, 10, fake, std) == EARG
    assert lib.b64_pipeline_decode(None, fake, 10, fake, std) == EARG
    lib.b64_pipeline_destroy(None)
    # server: limits checked before any device call
    assert lib.b64_server_create(1 << 19, 1, 2, 64, 1 << 20) is None    # budget below 1 MiB
    assert b"budget_bytes" in lib.b64_server_last_error()
    assert lib.b64_server_create(1 << 20, 0, 2, 64, 1 << 20) is None    # no stream
    assert lib.b64_server_create(1 << 20, 17, 17, 64, 1 << 20) is None  # more than 16 streams
    assert b"nstreams" in lib.b64_server_last_error()
    assert lib.b64_server_create(1 << 20, 2, 1, 64, 1 << 20) is None    # depth below nstreams
    assert lib.b64_server_create(1 << 20, 2, 65, 64, 1 << 20) is None   # depth above 64
    assert b"depth" in lib.b64_server_last_error()
    assert lib.b64_server_create(1 << 20, 2, 2, 0, 1 << 20) is None
    assert lib.b64_server_create(1 << 20, 2, 2, 64, 0) is None
    assert b"batch limits" in lib.b64_server_last_error()
    assert lib.b64_server_set_zero_copy_max(None, 0) == EARG
    assert lib.b64_server_set_staging(None, 0) == EARG
    stats = (ctypes.c_int64 * 8)()
    assert lib.b64_server_run(None, 0, None, None, None, None, None, None, None, None, None,
                              std, stats) == EARG
    assert b"null server" in lib.b64_server_last_error()
    lib.b64_server_destroy(None)
    # variants
    with_space = ctypes.create_string_buffer(b" " + std.raw[1:], 64)
    assert lib.b64_encode_mode(fake, 10, fake, std, 2, 0, None) == EARG          # SKIP_WS
    assert lib.b64_encode_mode(fake, 10, fake, std, 0, 2, None) == EARG          # line_len 2
    assert lib.b64_encode_mode(fake, 10, fake, dup, 1, 0, None) == EARG
    assert lib.b64_decode_mode(fake, 10, fake, std, 8, None) == EARG             # unknown flag
    assert lib.b64_decode_mode(fake, 10, fake, with_space, 2, None) == EARG
    assert b"SKIP_WS" in lib.b64_last_error()
    assert lib.b64_validate_mode(fake, 10, with_space, 3, None) == EARG
    assert lib.b64_decode_mode_async(fake, 10, fake, fake, fake, std, 2, None, 0, None) == EARG
    assert lib.b64_decode_mode_async(fake, 1 << 20, fake, fake, fake, std, 2, fake, 8, None) == EARG
    assert b"workspace" in lib.b64_last_error()
    assert lib.b64_validate_mode_async(fake, 10, fake, fake, std, 2, None, 0, None) == EARG
    assert lib.b64_encode_batch_mode(fake, fake, 3, fake, fake, fake, std, 2, None) == EARG
    assert lib.b64_decode_batch_mode(fake, fake, 3, fake, fake, fake, fake, std, 2, None) == EARG
    # fused decode
    assert lib.b64_decode_f32_bf16(fake, fake, -1, 4, fake, fake, std, 0, None) == EARG
    assert lib.b64_decode_f32_bf16(fake, fake, 3, -4, fake, fake, std, 0, None) == EARG
    assert lib.b64_decode_f32_bf16(fake, fake, 3, 4, fake, fake, std, 2, None) == EARG
    assert lib.b64_decode_f32_bf16(fake, None, 3, 4, fake, fake, std, 0, None) == EARG
    assert lib.b64_decode_f32_bf16(fake, fake, 3, 4, fake, None, std, 0, None) == EARG
    assert lib.b64_decode_f32_bf16(fake, fake, 3, 4, fake, fake, dup, 1, None) == EARG
    assert lib.b64_decode_f32_bf16(None, None, 0, 4, None, None, std, 0, None) == 0
    # zero-size work needs no device
    assert lib.b64_encode(None, 0, None, std, None) == 0
    assert lib.b64_encode_mode(None, 0, None, std, 1, 76, None) == 0
    assert lib.b64_encode_batch(None, None, 0, None, None, None, std, None) == 0
    assert lib.b64_encode_batch_mode(None, None, 0, None, None, None, std, 1, None) == 0


def test_tuning_interface(lib):
    EARG = -(2 ** 63)
    old = [lib.b64_tune_get_bucket(0, b) for b in range(5)]
    assert lib.b64_tune_get(0) == old[4]
    assert lib.b64_tune_set(0, 3, 8, 0) == EARG
    assert lib.b64_tune_set(0, 4, 0, 0) == EARG
    assert lib.b64_tune_set(8, 4, 8, 0) == EARG
    assert lib.b64_tune_set(5, 3, 8, 0) == EARG
    assert lib.b64_tune_get(4) > 0
    assert lib.b64_tune_get(6) > 0
    assert lib.b64_tune_get(7) > 0
    assert lib.b64_tune_get(8) == EARG
    assert lib.b64_tune_set(0, 4, 8, 2) == EARG
    assert lib.b64_tune_set(0, 8, 16, 1) == 0
    assert [lib.b64_tune_get_bucket(0, b) for b in range(5)] == [10816] * 5
    # one bucket at a time
    assert lib.b64_tune_set_bucket(0, 2, 2, 3, 0) == 0
    assert [lib.b64_tune_get_bucket(0, b) for b in range(5)] == [10816, 10816, 203, 10816, 10816]
    assert lib.b64_tune_set_bucket(0, 5, 2, 3, 0) == EARG
    assert lib.b64_tune_set_bucket(0, -2, 2, 3, 0) == EARG
    assert lib.b64_tune_get_bucket(0, 5) == EARG
    assert lib.b64_tune_get_bucket(0, -1) == EARG
    for b, v in enumerate(old):
        assert lib.b64_tune_set_bucket(0, b, (v // 100) % 100, v % 100, v // 10000) == 0
    assert [lib.b64_tune_get_bucket(0, b) for b in range(5)] == old
    # size buckets: < 64 KiB, < 1 MiB, < 16 MiB, < 128 MiB, larger
    for n, b in ((0, 0), ((64 << 10) - 1, 0), (64 << 10, 1), ((1 << 20) - 1, 1), (1 << 20, 2),
                 ((16 << 20) - 1, 2), (16 << 20, 3), ((128 << 20) - 1, 3), (128 << 20, 4),
                 (1 << 40, 4)):
        assert lib.b64_tune_bucket(n) == b, n
    assert lib.b64_tune_bucket(-1) == EARG
    # the whitespace decode's guess threshold: default, set, read, restore
    assert lib.b64_tune_ws_guess_min(-1) == 14 << 20
    assert lib.b64_tune_ws_guess_min(0) == 14 << 20
    assert lib.b64_tune_ws_guess_min(-5) == 0
    assert lib.b64_tune_ws_guess_min(14 << 20) == 0
    assert lib.b64_tune_ws_guess_min(-1) == 14 << 20


def test_binding_size_copies_match_the_library(lib):
    """The Python side computes output sizes itself on hot paths (no library
    round trip per call); every such copy must equal the library's helpers."""
    import torch

    import paper_1910_05109_amd as b64
    from paper_1910_05109_amd import batch
    ns = list(range(0, 3000)) + [2 ** k + r for k in range(12, 41) for r in (-2, -1, 0, 1, 2)]
    arr = np.array(ns, dtype=np.int64)
    t = torch.from_numpy(arr)
    enc = np.array([lib.b64_encoded_len(n) for n in ns])
    dec = np.array([lib.b64_decoded_max_len(n) for n in ns])
    enc_np = np.array([lib.b64_encoded_len_mode(n, 1, 0) for n in ns])
    dec_np = np.array([lib.b64_decoded_max_len_mode(n, 1) for n in ns])
    assert [b64._plain_enc_len(n) for n in ns] == enc.tolist()
    assert [b64._plain_dec_cap(n) for n in ns] == dec.tolist()
    assert np.array_equal(batch.encoded_lengths(arr), enc)
    assert np.array_equal(batch.decoded_capacity(arr), dec)
    assert np.array_equal(b64._enc_cap(t).numpy(), enc)
    assert np.array_equal(b64._dec_cap(t).numpy(), dec)
    assert np.array_equal(b64._enc_cap_nopad(t).numpy(), enc_np)
    assert np.array_equal(b64._dec_cap_nopad(t).numpy(), dec_np)


def test_fast_binding_reaches_the_same_library(lib):
    """The fast-call binding (_b64fast) calls the entry points of the loaded
    library: the same host-side argument errors as through ctypes, the error
    message left in that library's b64_last_error, argument-count and type
    errors raised in Python, and zero-size work done without a device."""
    from paper_1910_05109_amd import _lib
    F = _lib.fast
    assert F is not None
    EARG = -(2 ** 63)
    std = ctypes.create_string_buffer(b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/", 64)
    dup = ctypes.create_string_buffer(b"A" * 64, 64)
    a_std, a_dup = ctypes.addressof(std), ctypes.addressof(dup)
    fake = 0x1000
    assert F.encode(fake, -1, fake, a_std, 0) == EARG
    assert b"negative" in lib.b64_last_error()
    assert F.encode(fake, 10, fake, a_dup, 0) == EARG
    assert b"alphabet" in lib.b64_last_error()
    assert F.encode(0, 10, fake, a_std, 0) == EARG
    assert F.encode_mode(fake, 10, fake, a_std, 2, 0, 0) == EARG           # SKIP_WS
    assert F.encode_mode(fake, 10, fake, a_std, 0, 2, 0) == EARG           # line_len 2
    assert F.decode(fake, -3, fake, a_std, 0) == EARG
    assert F.decode(fake, 10, fake, a_dup, 0) == EARG
    assert F.decode_async(fake, 10, fake, 0, fake, a_std, 0) == EARG
    assert F.validate(0, 10, a_std, 0) == EARG
    assert F.validate_async(fake, 10, fake, 0, a_std, 0) == EARG
    assert F.encode(0, 0, 0, a_std, 0) == 0
    assert F.encode_mode(0, 0, 0, a_std, 1, 76, 0) == 0
    with pytest.raises(TypeError):
        F.encode(fake, 10, fake, a_std)
    with pytest.raises(TypeError):
        F.decode_async(fake, "10", fake, fake, fake, a_std, 0)
    with pytest.raises(OverflowError):
        F.validate(fake, 1 << 70, a_std, 0)
    with pytest.raises(ValueError):
        F.bind(0, 0, 0, 0, 0, 0)
    # the binding's alphabet addresses point at the 64 bytes themselves
    import paper_1910_05109_amd as b64
    for alpha in (b64.STD, b64.URL, bytes(bytearray(b64.URL)[::-1])):
        assert ctypes.string_at(b64._alpha_addr(alpha), 64) == alpha


def test_ws_small_max_knob(lib):
    """The one-workgroup limit of the whitespace-skipping decode: read,
    set, restored; above 65,536 rejected (no device needed)."""
    EARG = -(2 ** 63)
    old = lib.b64_tune_ws_small_max(-1)
    assert old == 65536
    assert lib.b64_tune_ws_small_max(65537) == EARG
    assert lib.b64_tune_ws_small_max(1000) == old
    assert lib.b64_tune_ws_small_max(-1) == 1000
    assert lib.b64_tune_ws_small_max(old) == 1000
    assert lib.b64_tune_ws_small_max(-1) == old
