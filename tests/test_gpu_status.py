"""GPU tests of how single-buffer decodes and validations report their status.

Outside graph capture a decode or validation is one launch: the kernel's last
workgroup writes the public status, and the stream's status slot in library
memory is back to zero for the next call.  These tests run many such calls
back to back without synchronizing, with valid inputs and inputs spoiled in
the first, a middle and the last workgroup's share, on one stream, on several
streams at once, and on hipStreamPerThread from several host threads, and
check every status (and every decoded byte of the valid inputs) against the
oracle.
"""
import ctypes
import threading

import pytest

import workloads
from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
PER_THREAD_STREAM = 2          # hipStreamPerThread


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


@pytest.fixture(scope="module")
def cases(oracle):
    """(text, expected [length, first_bad], decoded bytes or None) for
    encodings of several sizes (one workgroup to the streaming grid), valid and
    spoiled at seeded positions near the start, the middle and the end."""
    g = workloads.rng(workloads.SEED_BASE + 350)
    x = workloads.random_bytes(workloads.SEED_BASE + 351, 40 << 20)
    out = []
    for n in (0, 1, 5, 700, 3001, 100_000, 1_000_003, (12 << 20) + 1, 40 << 20):
        text = oracle.encode(x[:n])
        out.append((text, [n, -1], x[:n]))
        if text.size < 8:
            continue
        for lo, hi in ((0, text.size // 16), (text.size // 3, 2 * text.size // 3),
                       (text.size - 8, text.size)):
            s, _ = workloads.plant_invalid(text, int(g.integers(1 << 30)), STD, lo, max(hi, lo + 1))
            out.append((s, [-1, ~oracle.decode_raw(s)], None))
    return [(to_dev(t), st, None if r is None else to_dev(r)) for t, st, r in out]


def _run(b64, cases, order, stream=None):
    import torch
    st = torch.full((len(order), 2), 7, dtype=torch.int64, device="cuda")
    vt = torch.full((len(order), 2), 7, dtype=torch.int64, device="cuda")
    outs = []
    for k, i in enumerate(order):
        t, _, _ = cases[i]
        out, _ = b64.decode_async(t, status=st[k], stream=stream)
        b64.validate_async(t, status=vt[k], stream=stream)
        outs.append(out)
    return st, vt, outs


def _check(cases, order, st, vt, outs, label):
    import torch
    st, vt = to_host(st), to_host(vt)
    for k, i in enumerate(order):
        _, want, ref = cases[i]
        assert st[k].tolist() == want, (label, k, i, st[k], want)
        assert vt[k].tolist() == want, (label, k, i, vt[k], want)
        if ref is not None:
            assert torch.equal(outs[k][: ref.numel()], ref), (label, k, i)


def test_back_to_back_one_stream(b64, cases):
    import torch
    g = workloads.rng(workloads.SEED_BASE + 352)
    order = [int(v) for v in g.integers(0, len(cases), size=300)]
    say("status back to back", len(order))
    st, vt, outs = _run(b64, cases, order)
    torch.cuda.synchronize()
    _check(cases, order, st, vt, outs, "one stream")


def test_blocking_between_async(b64, cases):
    """Blocking decodes and validations between asynchronous ones."""
    import torch
    st = torch.empty(2, dtype=torch.int64, device="cuda")
    for rep in range(3):
        for i, (t, want, ref) in enumerate(cases):
            say("status blocking", rep, i)
            b64.decode_async(t, status=st)
            out, bad = b64.decode(t)
            if want[1] == -1:
                assert bad is None and torch.equal(out, ref), (rep, i)
            else:
                assert out is None and bad == want[1], (rep, i, bad)
            assert b64.validate(t) == ((want[0], None) if want[1] == -1 else (None, want[1]))
            assert to_host(st).tolist() == want, (rep, i)


def test_four_streams_at_once(b64, cases):
    import torch
    streams = [torch.cuda.Stream() for _ in range(4)]
    g = workloads.rng(workloads.SEED_BASE + 353)
    orders = [[int(v) for v in g.integers(0, len(cases), size=80)] for _ in streams]
    torch.cuda.synchronize()
    say("status four streams")
    results = [_run(b64, cases, o, s) for o, s in zip(orders, streams)]
    torch.cuda.synchronize()
    for k, (o, r) in enumerate(zip(orders, results)):
        _check(cases, o, *r, f"stream {k}")


def test_per_thread_stream_from_four_threads(b64, cases):
    """b64_decode and b64_validate on hipStreamPerThread, four host threads
    at once: each thread has its own stream and its own status slot."""
    import torch
    from paper_1910_05109_amd import _lib
    L = _lib.load()
    alpha = ctypes.create_string_buffer(STD, 64)
    outs = [[torch.zeros(max(3 * (t.numel() // 4), 1), dtype=torch.uint8, device="cuda")
             for t, _, _ in cases] for _ in range(4)]
    torch.cuda.synchronize()
    errors = []

    def worker(tid):
        try:
            for rep in range(20):
                for i in ((tid + rep) % len(cases), (3 * tid + 5 * rep) % len(cases)):
                    t, want, _ = cases[i]
                    exp = want[0] if want[1] == -1 else ~want[1]
                    r = L.b64_validate(t.data_ptr(), t.numel(), alpha, PER_THREAD_STREAM)
                    if r != exp:
                        errors.append(("validate", tid, rep, i, r, exp))
                    r = L.b64_decode(t.data_ptr(), t.numel(), outs[tid][i].data_ptr(), alpha,
                                     PER_THREAD_STREAM)
                    if r != exp:
                        errors.append(("decode", tid, rep, i, r, exp))
        except Exception as e:       # noqa: BLE001 -- reported below
            errors.append(("exception", tid, repr(e)))

    say("status per-thread stream, 4 threads")
    threads = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors[:5]
    torch.cuda.synchronize()
    for tid in range(4):
        for rep in range(20):
            for i in ((tid + rep) % len(cases), (3 * tid + 5 * rep) % len(cases)):
                _, want, ref = cases[i]
                if want[1] == -1:
                    assert torch.equal(outs[tid][i][: ref.numel()], ref), (tid, i)


def test_graph_replays_back_to_back(b64, cases):
    """A captured decode and validation own a status slot: replays queued
    back to back, each after new input contents are copied in and followed by
    a copy of its status words, all give the oracle's statuses."""
    import torch
    picks = [i for i, (t, _, _) in enumerate(cases) if 0 < t.numel() <= 4 << 20]
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for i in picks:
        t, want, ref = cases[i]
        n = t.numel()
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        out = torch.empty(max(3 * (n // 4), 1), dtype=torch.uint8, device="cuda")
        st = torch.empty(2, dtype=torch.int64, device="cuda")
        vt = torch.empty(2, dtype=torch.int64, device="cuda")
        with torch.cuda.stream(stream):
            src.copy_(t)
            b64.decode_async(src, out=out, status=st)          # warm-up outside the capture
            b64.validate_async(src, status=vt)
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            b64.decode_async(src, out=out, status=st)
            b64.validate_async(src, status=vt)
        # replays alternate this input with a spoiled copy, all queued at once
        bad = t.clone()
        bad[n // 2] = ord("*")
        bad_first = min(want[1], n // 2) if want[1] >= 0 else n // 2
        hist = torch.empty((12, 4), dtype=torch.int64, device="cuda")
        with torch.cuda.stream(stream):
            for rep in range(12):
                src.copy_(bad if rep % 2 else t)
                st.fill_(-7)
                vt.fill_(-7)
                g.replay()
                hist[rep, :2].copy_(st)
                hist[rep, 2:].copy_(vt)
        stream.synchronize()
        say("status graph replays", i, "n", n)
        h = to_host(hist)
        for rep in range(12):
            exp = [-1, bad_first] if rep % 2 else want
            assert h[rep, :2].tolist() == exp and h[rep, 2:].tolist() == exp, (i, rep, h[rep], exp)
        if ref is not None:
            # the last replay decoded the spoiled copy; one more of the input itself
            with torch.cuda.stream(stream):
                src.copy_(t)
                g.replay()
            stream.synchronize()
            assert to_host(st).tolist() == want and torch.equal(out[: ref.numel()], ref), i
