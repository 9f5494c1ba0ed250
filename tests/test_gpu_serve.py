"""The native serving loop (b64_server_run): every request's result in the
coalesced, overlapping mix equals its result alone (the single-buffer entry
points) and the oracle's, bit-exact; launches run at the same time on the
device; the device arena (the HBM budget) bounds what is in flight, and
requests wait when it is full.

Requests follow the serving workload's law -- sizes log-normal with median
8 KiB and sigma 1.5 clipped to [1 B, 16 MiB], 50/50 encode and decode, some
decodes spoiled by one invalid byte -- and a second case adds requests of
several MiB up to 16 MiB under a budget small enough that the arena wraps and
admission waits.  Each case runs with every launch staged through the arena
(copies by kernels up to 1 MiB and by DMA above, the default; all by
kernels; all by DMA), with launches of up to 1 MiB zero-copy (the kernel
works on the pinned host pools), and with every launch zero-copy.
"""
import numpy as np
import pytest

import workloads
from gpu_util import first_mismatch, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


def _schedule(oracle, seed, sizes, rate, invalid_frac):
    """kinds, arrivals, packed host payloads and offsets; decode requests
    carry the oracle's encoding of their bytes, some spoiled by one byte
    outside the alphabet."""
    count = sizes.size
    is_dec, is_bad = workloads.serve_kinds(seed + 1, count, invalid_frac=invalid_frac)
    arrival = workloads.serve_arrivals(seed + 2, count, rate)
    raw = workloads.random_bytes(seed + 3, int(sizes.sum()))
    roff = workloads.offsets(sizes)
    g = workloads.rng(seed + 4)
    bad_bytes = workloads.non_alphabet_bytes(oracle.STD)
    parts = []
    for i in range(count):
        x = raw[roff[i]:roff[i + 1]]
        if is_dec[i]:
            x = oracle.encode(x)
            if is_bad[i] and x.size:
                x = x.copy()
                x[int(g.integers(0, x.size))] = bad_bytes[int(g.integers(0, bad_bytes.size))]
        parts.append(x)
    payload = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    in_off = workloads.offsets(np.array([p.size for p in parts], dtype=np.int64))
    return is_dec.astype(np.int32), arrival, payload, in_off, parts


def _check_mix_alone_oracle(b64, oracle, res, kinds, parts, label):
    import torch
    for i, x in enumerate(parts):
        if kinds[i] == 0:
            ref = oracle.encode(x)
            alone = to_host(b64.encode(to_dev(x))) if x.size else np.zeros(0, np.uint8)
            assert res.out_len[i] == ref.size and res.first_bad[i] == -1, (label, i)
            assert first_mismatch(res.output(i), ref) is None, (label, i)
            assert first_mismatch(alone, ref) is None, (label, i)
        else:
            ref, ref_bad = oracle.decode(x)
            dx = to_dev(x) if x.size else torch.empty(0, dtype=torch.uint8, device="cuda")
            alone, alone_bad = b64.decode(dx)
            assert alone_bad == ref_bad, (label, i)
            if ref_bad is None:
                assert res.first_bad[i] == -1 and res.out_len[i] == ref.size, (label, i)
                assert first_mismatch(res.output(i), ref) is None, (label, i)
                assert first_mismatch(to_host(alone), ref) is None, (label, i)
            else:
                assert res.first_bad[i] == ref_bad and res.out_len[i] == -1, (label, i)


ZERO_COPY = pytest.mark.parametrize(
    "zc,staging", [(None, None), (None, "kernels"), (None, "dma"), (1 << 20, None), (64 << 20, None)],
    ids=["staged", "staged-kernels", "staged-dma", "mixed", "zero-copy"])


@ZERO_COPY
def test_mix_equals_alone_serving_law(b64, oracle, zc, staging):
    """3,000 requests of the serving law at 200,000 per second: coalesced,
    with launches overlapping on the device."""
    from paper_1910_05109_amd import serve
    seed = workloads.SEED_BASE + 140
    sizes = workloads.serve_sizes(seed, 3000)
    kinds, arrival, payload, in_off, parts = _schedule(oracle, seed, sizes, 2e5, 0.02)
    say("serve law", sizes.size, int(sizes.sum()), "zero-copy max", zc)
    with serve.Server(budget_bytes=32 << 30, nstreams=4, depth=8, zero_copy_max=zc,
                      staging=staging) as srv:
        res = srv.run(kinds, arrival, payload, in_off)
    summ = res.summary()
    say("serve summary", summ)
    if zc is None:                                   # the default: every launch staged
        assert summ["zero_copy_launches"] == 0
    else:
        assert summ["zero_copy_launches"] > 0
    assert np.isfinite(res.latency).all() and (res.latency > 0).all()
    assert summ["launches"] < sizes.size and summ["mean_batch"] > 1.0     # coalescing happened
    assert summ["max_concurrent"] >= 2 and summ["overlapped_launches"] >= 2, summ
    assert summ["peak_arena_bytes"] <= summ["arena_bytes"]
    _check_mix_alone_oracle(b64, oracle, res, kinds, parts, "law")


@ZERO_COPY
def test_large_requests_under_a_tight_budget(b64, oracle, zc, staging):
    """Requests of 1..16 MiB among small ones, a 40 MiB arena: the ring wraps
    and requests wait for space; every result still equals the oracle's.
    With zero-copy, launches of at most 1 MiB skip the arena and the larger
    ones still go through it."""
    from paper_1910_05109_amd import serve
    seed = workloads.SEED_BASE + 145
    sizes = workloads.serve_sizes(seed, 400)
    big = workloads.rng(seed + 9).choice(sizes.size, size=12, replace=False)
    sizes[big] = np.array([1 << 20, 3 << 20, (5 << 20) + 1, 7 << 20, (9 << 20) + 2, 11 << 20,
                           12 << 20, (13 << 20) + 1, 14 << 20, 15 << 20, 16 << 20,
                           (16 << 20) - 1])[: big.size]
    kinds, arrival, payload, in_off, parts = _schedule(oracle, seed, sizes, 5e4, 0.05)
    budget = 40 << 20
    say("serve tight", sizes.size, int(sizes.sum()), "budget", budget, "zero-copy max", zc)
    with serve.Server(budget_bytes=budget, nstreams=3, depth=6, max_batch=64,
                      max_batch_bytes=4 << 20, zero_copy_max=zc, staging=staging) as srv:
        res = srv.run(kinds, arrival, payload, in_off)
    summ = res.summary()
    say("serve summary", summ)
    assert summ["arena_bytes"] == budget and summ["peak_arena_bytes"] <= budget
    if zc is None or zc < (5 << 20):
        assert summ["peak_arena_bytes"] > budget // 2      # the budget was the limit
    else:
        assert summ["peak_arena_bytes"] == 0 and summ["zero_copy_launches"] == summ["launches"]
    _check_mix_alone_oracle(b64, oracle, res, kinds, parts, "tight")


def test_server_argument_errors(b64):
    from paper_1910_05109_amd import serve
    from paper_1910_05109_amd._lib import B64Error
    with pytest.raises(B64Error):
        serve.Server(budget_bytes=1 << 10)
    with pytest.raises(B64Error):
        serve.Server(budget_bytes=1 << 20, nstreams=0)
    with pytest.raises(ValueError):
        serve.Server(budget_bytes=1 << 20, zero_copy_max=-2)
    with pytest.raises(ValueError):
        serve.Server(budget_bytes=1 << 20, staging="pigeon")
    with serve.Server(budget_bytes=1 << 20, nstreams=1, depth=1, zero_copy_max=0) as srv:
        payload = np.zeros(4 << 20, dtype=np.uint8)
        with pytest.raises(B64Error):          # one request larger than the budget
            srv.run(np.zeros(1, np.int32), np.zeros(1), payload, np.array([0, payload.size]))
        with pytest.raises(B64Error):          # arrivals out of order
            srv.run(np.zeros(2, np.int32), np.array([1e-3, 0.0]), payload[:8],
                    np.array([0, 4, 8]))
        res = srv.run(np.zeros(0, np.int32), np.zeros(0), payload[:0], np.zeros(1, np.int64))
        assert res.out_len.size == 0
    with serve.Server(budget_bytes=1 << 20, nstreams=1, depth=1, zero_copy_max=4 << 20) as srv:
        # the same request zero-copy: no arena space needed
        payload = workloads.random_bytes(workloads.SEED_BASE + 146, 4 << 20)
        res = srv.run(np.zeros(1, np.int32), np.zeros(1), payload, np.array([0, payload.size]))
        assert res.summary()["zero_copy_launches"] == 1
        import base64
        assert res.output(0).tobytes() == base64.b64encode(payload.tobytes())
