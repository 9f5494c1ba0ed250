"""GPU test of the allocation-free entry point b64_decode_ws_async_noalloc.

Called through the C ABI, it must give what b64_decode_mode_async (the same
whitespace-skipping decode with a workspace the caller allocates) gives, bit
for bit, and what the oracle gives: first on a larger MIME text, then on a
smaller one right after it (the library's scratch array keeps the first
call's contents), then on spoiled and unpadded texts and on the regular-line
path, with valid and invalid inputs in turn.
"""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
NOPAD, SKIP_WS = 1, 2


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_05109_amd import _lib
    return _lib.load()


def _mime(oracle, x, flags=0):
    return oracle.encode_mode(x, STD, flags & NOPAD, workloads.MIME_LINE)


def _both(lib, text, flags):
    """(status, bytes) of the allocation-free call and of the workspace call."""
    import torch
    from paper_1910_05109_amd import stream_ptr
    n = text.size
    s = to_dev(text) if n else torch.zeros(1, dtype=torch.uint8, device="cuda")
    cap = max(int(lib.b64_decoded_max_len_mode(n, flags)), 1)
    alpha = ctypes.create_string_buffer(STD, 64)
    stream = stream_ptr()
    out_a = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    st_a = torch.full((2,), 99, dtype=torch.int64, device="cuda")
    r = lib.b64_decode_ws_async_noalloc(s.data_ptr(), n, out_a.data_ptr(), st_a.data_ptr(),
                                        st_a.data_ptr() + 8, alpha, flags, stream)
    assert r == 0, lib.b64_last_error()
    wsb = int(lib.b64_decode_workspace_size(n, flags))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    out_b = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    st_b = torch.full((2,), 77, dtype=torch.int64, device="cuda")
    r = lib.b64_decode_mode_async(s.data_ptr(), n, out_b.data_ptr(), st_b.data_ptr(),
                                  st_b.data_ptr() + 8, alpha, flags, ws.data_ptr(), wsb, stream)
    assert r == 0, lib.b64_last_error()
    torch.cuda.synchronize()
    return to_host(st_a).tolist(), to_host(out_a), to_host(st_b).tolist(), to_host(out_b)


def _check(lib, oracle, text, flags, label):
    say("noalloc", label, "n", text.size, "flags", flags)
    st_a, out_a, st_b, out_b = _both(lib, text, flags)
    ref, bad = oracle.decode_mode(text, STD, flags)
    want = [ref.size, -1] if bad is None else [-1, bad]
    assert st_a == st_b == want, (label, st_a, st_b, want)
    if bad is None:
        assert np.array_equal(out_a[: ref.size], out_b[: ref.size]), label
        assert np.array_equal(out_a[: ref.size], ref), label


def test_two_calls_second_smaller(lib, oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 370, 6 << 20)
    big = workloads.sprinkle_ws(_mime(oracle, x), workloads.SEED_BASE + 371, 3000, 5, 1, 1 << 15)
    small = _mime(oracle, x[:100_003])
    _check(lib, oracle, big, SKIP_WS, "first, larger")
    _check(lib, oracle, small, SKIP_WS, "second, smaller")


def test_more_calls_in_a_row(lib, oracle):
    """Spoiled, unpadded, empty and regular-line texts one after another."""
    import paper_1910_05109_amd as b64
    x = workloads.random_bytes(workloads.SEED_BASE + 372, 3 << 20)
    regular = _mime(oracle, x)
    spoiled = regular.copy()
    spoiled[regular.size // 3] = ord("*")
    unpadded = _mime(oracle, x[: (1 << 20) + 1], NOPAD)
    old = b64.tune_ws_guess_min(-1)
    try:
        for guess_min in (old, 0):           # counted path, then the regular-line guess
            b64.tune_ws_guess_min(guess_min)
            _check(lib, oracle, regular, SKIP_WS, f"regular {guess_min}")
            _check(lib, oracle, spoiled, SKIP_WS, f"spoiled {guess_min}")
            _check(lib, oracle, unpadded, SKIP_WS | NOPAD, f"unpadded {guess_min}")
            _check(lib, oracle, regular[:4001], SKIP_WS, f"cut {guess_min}")
            _check(lib, oracle, np.zeros(0, np.uint8), SKIP_WS, f"empty {guess_min}")
    finally:
        b64.tune_ws_guess_min(old)


def test_length_cap(lib):
    """Inputs past the scratch array's capacity are refused before any launch."""
    fake = ctypes.c_void_p(0x1000)
    alpha = ctypes.create_string_buffer(STD, 64)
    assert lib.b64_decode_ws_async_noalloc(fake, 4294868993, fake, fake, fake, alpha, SKIP_WS,
                                           None) == -(2 ** 63)
