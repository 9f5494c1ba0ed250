"""GPU parity past 32-bit sizes: one buffer of 2^32 + 1000 bytes (5.7 G
characters) and a ragged batch of the same bytes whose buffers start past
2^31 and 2^32.  Every index and offset in the kernels is 64-bit; these cases
make a 32-bit slip show.

The input is a seeded block of a prime length (49,999,991 bytes) repeated, so
that the host can rebuild any slice for the oracle.  Windows at the start,
around 2^31 and 2^32 and at the end (with the padding) are compared with the
oracle's encoding; the decode round trip is compared on the device; an
invalid byte planted past 2^32 must come back as the first invalid offset.
"""
import numpy as np
import pytest

import workloads
from gpu_util import first_mismatch, say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
PERIOD = 49_999_991
N_BYTES = (1 << 32) + 1000                 # n mod 3 = 2: the last group is padded


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


@pytest.fixture(scope="module")
def big():
    """(host block, device input of N_BYTES bytes)."""
    import torch
    block = workloads.random_bytes(workloads.SEED_BASE + 260, PERIOD)
    say("large: build input", N_BYTES)
    reps = -(-N_BYTES // PERIOD)
    x = to_dev(block).repeat(reps)[:N_BYTES]
    assert x.is_contiguous() and x.numel() == N_BYTES
    yield block, x
    del x
    torch.cuda.empty_cache()


def _host(block, a, b):
    return np.take(block, np.arange(a, b, dtype=np.int64) % PERIOD)


def _windows(n):
    """Group-aligned input windows [a, b) to compare with the oracle: the
    start, input offset 2^31, output offset 2^32 (input 3 * 2^30), and the
    tail with the padding (input offset 2^32)."""
    w = 3 * 4000
    starts = [0, 3 * ((1 << 31) // 3) - w // 2, 3 * (1 << 30) - w // 2]
    out = [(a, a + w) for a in starts]
    out.append((3 * ((n - w) // 3), n))
    assert all(b <= n for _, b in out) and out[-1][0] < (1 << 32) < n
    return out


def test_single_buffer_past_4g(b64, oracle, big):
    import torch
    block, x = big
    n = N_BYTES
    say("large: encode", n)
    text = b64.encode(x)
    N = 4 * ((n + 2) // 3)
    assert text.numel() == N
    for a, b in _windows(n):
        say("large: encode window", a, b)
        ref = oracle.encode(_host(block, a, b))
        got = to_host(text[4 * a // 3: 4 * a // 3 + ref.size])
        assert first_mismatch(got, ref) is None, (a, first_mismatch(got, ref))
    say("large: decode", N)
    out, bad = b64.decode(text)
    assert bad is None and out.numel() == n
    assert torch.equal(out, x)
    del out
    say("large: validate", N)
    assert b64.validate(text) == (n, None)
    # one invalid byte past 2^32 characters, then one before it too
    p = (1 << 32) + 12_345
    keep = int(text[p])
    text[p] = ord("*")
    say("large: invalid at", p)
    assert b64.decode(text)[1] == p
    _, st = b64.decode_async(text)
    assert to_host(st).tolist() == [-1, p]
    q = (1 << 31) + 5                      # second character of a quantum
    keep_q = int(text[q])
    text[q] = ord("=")
    assert ~oracle.decode_raw(to_host(text[q - 9: q + 7])) == 9
    assert b64.decode(text)[1] == q
    text[q] = keep_q
    text[p] = keep
    assert b64.validate(text) == (n, None)
    del text
    torch.cuda.empty_cache()


def test_batch_offsets_past_4g(b64, oracle, big):
    import torch
    block, x = big
    n = N_BYTES
    in_off = np.array([0, (1 << 31) + 5, (1 << 32) + 3, n - 17, n], dtype=np.int64)
    lens = np.diff(in_off)
    say("large: encode_batch", lens.tolist())
    dst, out_off, out_len = b64.encode_batch(x, to_dev(in_off))
    tl = 4 * ((lens + 2) // 3)
    assert (to_host(out_len) == tl).all()
    o_off = to_host(out_off)
    assert (np.diff(o_off) == tl).all()
    for b in range(lens.size):
        s, e = int(in_off[b]), int(in_off[b + 1])
        head = min(3000, 3 * ((e - s) // 3))
        tail0 = s + 3 * max(0, (e - s - 3000) // 3)
        for a, z in ((s, s + head), (tail0, e)):
            say("large: batch window", b, a, z)
            ref = oracle.encode(_host(block, a, z))
            at = int(o_off[b]) + 4 * (a - s) // 3
            got = to_host(dst[at: at + ref.size])
            assert first_mismatch(got, ref) is None, (b, a, first_mismatch(got, ref))
    say("large: decode_batch")
    dec, dout_off, dlen, dbad = b64.decode_batch(dst, out_off)
    assert (to_host(dbad) == -1).all() and (to_host(dlen) == lens).all()
    d_off = to_host(dout_off)
    for b in range(lens.size):
        s, e = int(in_off[b]), int(in_off[b + 1])
        assert torch.equal(dec[int(d_off[b]): int(d_off[b]) + (e - s)], x[s:e]), b
    # an invalid character in the buffer that starts past 2^32 bytes
    p = int(o_off[2]) + 4 * 11
    keep = int(dst[p])
    dst[p] = ord("!")
    say("large: decode_batch invalid at", p)
    _, _, dlen, dbad = b64.decode_batch(dst, out_off, dst=dec, out_off=dout_off)
    want = np.full(lens.size, -1)
    want[2] = 4 * 11
    assert to_host(dbad).tolist() == want.tolist()
    dst[p] = keep
    del dst, dec
    torch.cuda.empty_cache()


def test_mime_past_4g(b64, oracle, big):
    """CR LF line-wrapped encode of the same input (5.8 G characters, over
    177,000 whitespace-decode tiles, so the tile scan takes four passes) and
    its whitespace-skipping decode and validation."""
    import torch
    block, x = big
    n, L = N_BYTES, workloads.MIME_LINE
    per_line = L // 4 * 3                  # input bytes per full line
    say("large: wrapped encode", n)
    text = b64.encode(x, line_len=L)
    N = 4 * ((n + 2) // 3)
    assert text.numel() == N + 2 * ((N + L - 1) // L - 1)
    for k in (0, (1 << 31) // per_line - 40, (3 << 30) // per_line - 40, (n - 9000) // per_line):
        a = k * per_line
        z = min(n, a + 80 * per_line)
        say("large: wrapped window", a, z)
        ref = oracle.encode_mode(_host(block, a, z), STD, 0, L)
        got = to_host(text[(L + 2) * k: (L + 2) * k + ref.size])
        assert first_mismatch(got, ref) is None, (a, first_mismatch(got, ref))
    say("large: whitespace-skipping decode", text.numel())
    out, bad = b64.decode(text, flags=2)
    assert bad is None and out.numel() == n
    assert torch.equal(out, x)
    del out
    assert b64.validate(text, flags=2) == (n, None)
    del text
    torch.cuda.empty_cache()


def test_fused_rows_past_4g(b64, oracle):
    """The fused consumer with 1,400,000 rows of 1,536 float32: 2.15 G
    bfloat16 values (4.3 GB of output, element indices past 2^31, byte
    offsets past 2^32) from 11.5 GB of base64.  Every row is compared on the
    device with PyTorch's float32 -> bfloat16 conversion (NaN lanes aside,
    whose rule the oracle pins); rows around the 2^31-element and 2^32-byte
    marks and the last rows are compared with the oracle."""
    import torch
    dim, nrows = 1536, 1_400_000
    say("large: fused input", nrows, dim)
    nraw = nrows * dim * 4
    block = to_dev(workloads.random_bytes(workloads.SEED_BASE + 280, PERIOD))
    raw = block.repeat(-(-nraw // PERIOD))[:nraw]
    del block
    in_off = torch.arange(0, nrows + 1, dtype=torch.int64, device="cuda") * (4 * dim)
    text, t_off, _ = b64.encode_batch(raw, in_off)
    del in_off
    say("large: fused decode")
    out, st = b64.decode_f32_bf16(text, t_off, dim)
    assert (st == -1).all().item()
    f = raw.view(torch.float32).view(nrows, dim)
    for r0 in range(0, nrows, 100_000):
        blk = f[r0: r0 + 100_000]
        ref = blk.to(torch.bfloat16).view(torch.int16)
        got = out[r0: r0 + 100_000].view(torch.int16)
        ok = (got == ref) | torch.isnan(blk)
        assert ok.all().item(), r0
    tt = to_host(t_off)
    for b in ((1 << 31) // dim, (1 << 32) // (2 * dim), (1 << 32) // (2 * dim) + 1, nrows - 1):
        row = to_host(text[int(tt[b]): int(tt[b + 1])])
        ref, rst = oracle.decode_f32_bf16_rows(row, np.array([0, row.size], dtype=np.int64), dim)
        assert rst.tolist() == [-1]
        got = to_host(out[b].view(torch.int16)).view(np.uint16)
        assert (got == ref.reshape(-1)).all(), b
    del raw, text, out, f
    torch.cuda.empty_cache()
