"""GPU parity of the batched entry points (b64_encode_batch, b64_decode_batch)
against the oracle, bit-exact, buffer by buffer.

Covers: small ragged batches with empty buffers, invalid bytes and '=' misuse;
every string of length 0..8 over a 7-symbol set (each string one buffer);
input offsets at every alignment and outputs with gaps; HIP-graph capture and
replay; and the 100,000-buffer log-uniform workload at full size (every
buffer against the oracle).
"""
import numpy as np
import pytest

import workloads
from gpu_util import first_mismatch, say, to_dev, to_host
from stdlib_refs import brute_force_results

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


def _ragged_lengths(seed, nbuf, maxlen):
    g = workloads.rng(seed)
    lens = g.integers(0, maxlen + 1, size=nbuf).astype(np.int64)
    lens[g.random(nbuf) < 0.05] = 0
    lens[:12] = np.arange(12)          # every tiny length, incl. all residues
    return lens


def _check_decode_results(oracle, text, in_off, out_len, first_bad, dst, out_off, alpha, label):
    ref_dst, ref_off, ref_res = oracle.decode_list(text, in_off, alpha)
    nbuf = in_off.size - 1
    exp_len = np.where(ref_res >= 0, ref_res, -1)
    exp_bad = np.where(ref_res >= 0, -1, ~ref_res)
    bad = np.nonzero((out_len != exp_len) | (first_bad != exp_bad))[0]
    assert bad.size == 0, (label, bad[:5], out_len[bad[:5]], first_bad[bad[:5]], ref_res[bad[:5]])
    for b in range(nbuf):
        if ref_res[b] > 0:
            got = dst[out_off[b]: out_off[b] + ref_res[b]]
            ref = ref_dst[ref_off[b]: ref_off[b] + ref_res[b]]
            assert first_mismatch(got, ref) is None, (label, b)


@pytest.mark.parametrize("alpha", [STD, URL], ids=["std", "url"])
def test_small_ragged_batch(b64, oracle, alpha):
    lens = _ragged_lengths(workloads.SEED_BASE + 130, 3000, 4000)
    in_off = workloads.offsets(lens)
    src = workloads.random_bytes(workloads.SEED_BASE + 131, int(in_off[-1]))
    say("encode_batch small", alpha[-2:])
    dst, out_off, out_len = b64.encode_batch(to_dev(src), to_dev(in_off), alpha)
    ref_dst, ref_off, ref_len = oracle.encode_list(src, in_off, alpha)
    assert np.array_equal(to_host(out_off), ref_off)
    assert np.array_equal(to_host(out_len), ref_len)
    assert first_mismatch(to_host(dst)[: ref_dst.size], ref_dst) is None

    # decode: the encodings with some buffers spoiled
    text = ref_dst.copy()
    g = workloads.rng(workloads.SEED_BASE + 132)
    outside = workloads.non_alphabet_bytes(alpha)
    spoiled = g.choice(3000, size=150, replace=False)
    for b in spoiled:
        n = int(ref_off[b + 1] - ref_off[b])
        if n == 0:
            continue
        kind = g.integers(0, 3)
        p = int(ref_off[b] + g.integers(0, n))
        if kind == 0:
            text[p] = outside[g.integers(0, outside.size)]
        elif kind == 1:
            text[p] = ord("=")
        else:
            text[p] = alpha[0] if text[p] != alpha[0] else alpha[1]   # may break canonical pad bits
    tin = ref_off.copy()
    # a few truncated buffers: shorten by moving boundaries (keeps packing)
    say("decode_batch small", alpha[-2:])
    d_dst, d_off, d_len, d_bad = b64.decode_batch(to_dev(text), to_dev(tin), alpha)
    _check_decode_results(oracle, text, tin, to_host(d_len), to_host(d_bad), to_host(d_dst),
                          to_host(d_off), alpha, "small")


def test_truncated_and_odd_lengths_in_batch(b64, oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 133, 3000)
    base = oracle.encode(x)                   # 4000 chars
    lens = np.array([0, 1, 2, 3, 4, 5, 6, 7, 8, 63, 64, 65, 66, 67, 68, 1023, 1024, 1025, 3999, 4000],
                    dtype=np.int64)
    text = np.concatenate([base[:n] for n in lens])
    in_off = workloads.offsets(lens)
    say("decode_batch truncations")
    d_dst, d_off, d_len, d_bad = b64.decode_batch(to_dev(text), to_dev(in_off))
    _check_decode_results(oracle, text, in_off, to_host(d_len), to_host(d_bad), to_host(d_dst),
                          to_host(d_off), STD, "truncations")


def test_brute_force_strings_as_buffers(b64, oracle):
    """Every string of length 0..8 over values 0,1,16,48 and '=', '!', 0xC3,
    each one buffer; expected results from the prefix rule and the oracle."""
    symbols = [ord("A"), ord("B"), ord("Q"), ord("w"), ord("="), ord("!"), 0xC3]
    for length in range(0, 9):
        rows, expected = brute_force_results(symbols, length)
        nrows = rows.shape[0]
        in_off = np.arange(nrows + 1, dtype=np.int64) * length
        say("decode_batch brute force length", length, "rows", nrows)
        src = to_dev(rows.reshape(-1)) if length else to_dev(np.zeros(1, np.uint8))
        d_dst, d_off, d_len, d_bad = b64.decode_batch(src, to_dev(in_off))
        got = np.where(to_host(d_bad) >= 0, ~to_host(d_bad), to_host(d_len))
        assert np.array_equal(got, expected), length
        if length:
            assert np.array_equal(got, oracle.decode_rows(rows)), length


def test_misaligned_offsets_and_gapped_outputs(b64, oracle):
    import torch
    lens = _ragged_lengths(workloads.SEED_BASE + 134, 500, 3000)
    for base in (1, 2, 3, 5, 7, 11, 13, 15):
        in_off = workloads.offsets(lens) + base
        src = workloads.random_bytes(workloads.SEED_BASE + 135 + base, int(in_off[-1]))
        enc_len = 4 * ((lens + 2) // 3)
        out_off = np.zeros(lens.size + 1, dtype=np.int64)
        np.cumsum(enc_len + (np.arange(lens.size) % 7), out=out_off[1:])   # gaps of 0..6 bytes
        out_off += 3
        say("encode_batch misaligned", base)
        dst = torch.zeros(int(out_off[-1]) + 8, dtype=torch.uint8, device="cuda")
        b64.encode_batch(to_dev(src), to_dev(in_off), dst=dst, out_off=to_dev(out_off))
        got = to_host(dst)
        for b in range(lens.size):
            ref = oracle.encode(src[in_off[b]: in_off[b + 1]])
            assert first_mismatch(got[out_off[b]: out_off[b] + ref.size], ref) is None, (base, b)
        # gaps are untouched
        mask = np.ones(got.size, dtype=bool)
        for b in range(lens.size):
            mask[out_off[b]: out_off[b] + enc_len[b]] = False
        assert not got[mask].any()
        # decode those texts placed at misaligned offsets with gapped outputs
        texts = [oracle.encode(src[in_off[b]: in_off[b + 1]]) for b in range(lens.size)]
        t_off = workloads.offsets(np.array([t.size for t in texts], dtype=np.int64)) + base
        text = np.concatenate([np.zeros(base, np.uint8)] + texts)
        dec_cap = 3 * (np.diff(t_off) // 4)
        d_out_off = np.zeros(lens.size + 1, dtype=np.int64)
        np.cumsum(dec_cap + (np.arange(lens.size) % 5), out=d_out_off[1:])
        d_out_off += base
        say("decode_batch misaligned", base)
        ddst = torch.zeros(int(d_out_off[-1]) + 8, dtype=torch.uint8, device="cuda")
        _, _, d_len, d_bad = b64.decode_batch(to_dev(text), to_dev(t_off), dst=ddst,
                                              out_off=to_dev(d_out_off))
        assert np.array_equal(to_host(d_len), lens) and (to_host(d_bad) == -1).all()
        dg = to_host(ddst)
        for b in range(lens.size):
            assert first_mismatch(dg[d_out_off[b]: d_out_off[b] + lens[b]],
                                  src[in_off[b]: in_off[b + 1]]) is None, (base, b)


def test_graph_capture_and_replay(b64, oracle):
    """Encode + decode batches captured once in a HIP graph, replayed with new
    contents in the same buffers; every replay checked against the oracle."""
    import torch
    lens = _ragged_lengths(workloads.SEED_BASE + 136, 700, 5000)
    in_off = workloads.offsets(lens)
    total = int(in_off[-1])
    enc_off = workloads.offsets(4 * ((lens + 2) // 3))
    dec_off = workloads.offsets(3 * (np.diff(enc_off) // 4))
    d_src = torch.zeros(total, dtype=torch.uint8, device="cuda")
    d_in = to_dev(in_off)
    d_enc = torch.zeros(int(enc_off[-1]), dtype=torch.uint8, device="cuda")
    d_enc_off = to_dev(enc_off)
    d_enc_len = torch.zeros(lens.size, dtype=torch.int64, device="cuda")
    d_dec = torch.zeros(int(dec_off[-1]), dtype=torch.uint8, device="cuda")
    d_dec_off = to_dev(dec_off)
    d_dec_len = torch.zeros(lens.size, dtype=torch.int64, device="cuda")
    d_bad = torch.zeros(lens.size, dtype=torch.int64, device="cuda")

    def step():
        b64.encode_batch(d_src, d_in, dst=d_enc, out_off=d_enc_off, out_len=d_enc_len)
        b64.decode_batch(d_enc, d_enc_off, dst=d_dec, out_off=d_dec_off, out_len=d_dec_len,
                         first_bad=d_bad)

    say("graph warmup")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("graph capture")
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        src = workloads.random_bytes(workloads.SEED_BASE + 137 + rep, total)
        d_src.copy_(to_dev(src))
        d_dec.zero_()
        torch.cuda.synchronize()
        say("graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        ref_enc, _, ref_len = oracle.encode_list(src, in_off)
        assert first_mismatch(to_host(d_enc), ref_enc) is None, rep
        assert np.array_equal(to_host(d_enc_len), ref_len)
        assert np.array_equal(to_host(d_dec_len), lens) and (to_host(d_bad) == -1).all()
        dd = to_host(d_dec)
        for b in range(0, lens.size, 7):
            assert first_mismatch(dd[dec_off[b]: dec_off[b] + lens[b]], src[in_off[b]: in_off[b + 1]]) is None


def _slices(nbuf, per=2000):
    return [(b0, min(b0 + per, nbuf)) for b0 in range(0, nbuf, per)]


def _pool():
    import os
    from concurrent.futures import ThreadPoolExecutor
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return ThreadPoolExecutor(max_workers=max(1, min(16, n)))


def test_batch_workload_full_size(b64, oracle):
    """100,000 buffers, log-uniform lengths in [16 B, 1 MiB]: one encode launch
    and one decode launch; 0.5% of the decode buffers carry one invalid byte.
    Every buffer's encoding and every valid buffer's decoded bytes are compared
    with the oracle's (the oracle runs on slices of 2,000 buffers in parallel
    host threads), and every length and first invalid offset too."""
    import torch
    seed = workloads.SEED_BASE + 4
    lens = workloads.batch_lengths(seed)
    in_off = workloads.offsets(lens)
    total = int(in_off[-1])
    say("batch full: generate", total, "bytes")
    src = workloads.random_bytes(seed, total)
    d_src = to_dev(src)
    say("batch full: encode_batch")
    d_enc, d_enc_off, d_enc_len = b64.encode_batch(d_src, to_dev(in_off))
    enc_off = to_host(d_enc_off)
    assert np.array_equal(to_host(d_enc_len), 4 * ((lens + 2) // 3))
    assert np.array_equal(enc_off, workloads.offsets(4 * ((lens + 2) // 3)))
    h_enc = to_host(d_enc[: int(enc_off[-1])])
    del d_src
    say("batch full: oracle encode of every buffer")

    def enc_slice(bounds):
        b0, b1 = bounds
        ref, ref_off, ref_len = oracle.encode_list(src[in_off[b0]: in_off[b1]],
                                                   in_off[b0: b1 + 1] - in_off[b0])
        assert np.array_equal(ref_off + enc_off[b0], enc_off[b0: b1 + 1]), (b0, b1)
        return first_mismatch(h_enc[enc_off[b0]: enc_off[b1]], ref), b0

    with _pool() as pool:
        for mism, b0 in pool.map(enc_slice, _slices(lens.size)):
            assert mism is None, (b0, mism)
    # plant one invalid byte in 0.5% of the buffers
    bad_bufs = workloads.pick_buffers(seed + 2, lens.size, 0.005)
    g = workloads.rng(seed + 3)
    outside = workloads.non_alphabet_bytes(STD)
    nchar = np.diff(enc_off)
    pos = np.array([g.integers(0, nchar[b]) for b in bad_bufs], dtype=np.int64)
    vals = outside[g.integers(0, outside.size, size=bad_bufs.size)]
    d_enc[to_dev(enc_off[bad_bufs] + pos)] = to_dev(vals)
    h_enc[enc_off[bad_bufs] + pos] = vals
    say("batch full: decode_batch")
    d_dec, d_dec_off, d_len, d_bad = b64.decode_batch(d_enc, d_enc_off)
    dec_off = to_host(d_dec_off)
    got_len, got_bad = to_host(d_len), to_host(d_bad)
    h_dec = to_host(d_dec)
    del d_enc, d_dec
    torch.cuda.empty_cache()
    exp_bad = np.full(lens.size, -1, dtype=np.int64)
    exp_bad[bad_bufs] = pos
    exp_len = lens.copy()
    exp_len[bad_bufs] = -1
    assert np.array_equal(got_bad, exp_bad)
    assert np.array_equal(got_len, exp_len)
    say("batch full: oracle decode of every buffer")

    def dec_slice(bounds):
        b0, b1 = bounds
        ref, ref_off, res = oracle.decode_list(h_enc[enc_off[b0]: enc_off[b1]],
                                               enc_off[b0: b1 + 1] - enc_off[b0])
        wrong = []
        for k in range(b1 - b0):
            b = b0 + k
            r = int(res[k])
            if (r >= 0) != (got_len[b] >= 0) or (r >= 0 and r != got_len[b]) or \
                    (r < 0 and ~r != got_bad[b]):
                wrong.append(("status", b))
            elif r >= 0 and not np.array_equal(h_dec[dec_off[b]: dec_off[b] + r],
                                               ref[ref_off[k]: ref_off[k] + r]):
                wrong.append(("bytes", b))
        return wrong

    with _pool() as pool:
        for wrong in pool.map(dec_slice, _slices(lens.size)):
            assert not wrong, wrong[:5]


def test_layout_validation_rejects_out_of_bounds(b64):
    """The binding checks a batch layout against the tensor sizes on the host
    and raises before any launch."""
    import torch
    src = torch.zeros(1000, dtype=torch.uint8, device="cuda")
    too_long = to_dev(np.array([0, 600, 1200], dtype=np.int64))
    with pytest.raises(ValueError):
        b64.encode_batch(src, too_long)
    with pytest.raises(ValueError):
        b64.decode_batch(src, too_long)
    decreasing = to_dev(np.array([0, 600, 500], dtype=np.int64))
    with pytest.raises(ValueError):
        b64.encode_batch(src, decreasing)
    ok = to_dev(np.array([0, 600, 1000], dtype=np.int64))
    small_dst = torch.zeros(100, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        b64.encode_batch(src, ok, dst=small_dst)
    torch.cuda.synchronize()
