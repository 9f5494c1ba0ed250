"""Host logic of the serving loop and the batch planner (CPU only)."""
import numpy as np
import pytest

import workloads
from paper_1910_05109_amd.batch import decoded_capacity, encoded_lengths, prefix
from paper_1910_05109_amd.serve import OutputRing


def _overlaps(a, b):
    return a[0] < b[1] and b[0] < a[1]


@pytest.mark.parametrize("seed", range(6))
def test_ring_never_overlaps_and_frees_in_order(seed):
    g = workloads.rng(seed)
    size = int(g.integers(100, 5000))
    ring = OutputRing(size)
    live = []            # (start, end, held)
    for _ in range(3000):
        if live and (g.random() < 0.45 or len(live) > 20):
            s, e, held = live.pop(0)           # retire in order
            ring.release(held)
            continue
        n = int(g.integers(1, size // 3 + 2))
        got = ring.alloc(n)
        if got is None:
            # must not fit: the contiguous free space is smaller than n
            assert live, "an empty ring must accept any size up to its capacity"
            continue
        start, held = got
        iv = (start, start + n)
        assert 0 <= iv[0] and iv[1] <= size
        for s, e, _ in live:
            assert not _overlaps(iv, (s, e)), (iv, (s, e))
        live.append((iv[0], iv[1], held))
        assert ring.used <= size


def test_ring_rejects_oversized_and_accepts_full_capacity():
    ring = OutputRing(1000)
    with pytest.raises(ValueError):
        ring.alloc(1001)
    start, held = ring.alloc(1000)
    assert (start, held) == (0, 1000)
    assert ring.alloc(1) is None
    ring.release(held)
    assert ring.alloc(1) == (0, 1)


def test_layout_helpers():
    lens = np.array([0, 1, 2, 3, 4, 5, 100], dtype=np.int64)
    assert encoded_lengths(lens).tolist() == [0, 4, 4, 4, 8, 8, 136]
    assert decoded_capacity(lens).tolist() == [0, 0, 0, 0, 3, 3, 75]
    assert prefix(lens).tolist() == [0, 0, 1, 3, 6, 10, 15, 115]


def test_workload_recipes():
    lens = workloads.batch_lengths(workloads.SEED_BASE + 4)
    assert lens.size == 100_000 and lens.min() >= 16 and lens.max() < (1 << 20)
    # log-uniform over [16, 2^20): mean (2^20 - 16) / ln(2^16) ~ 94.5 KB
    assert 85_000 < lens.mean() < 105_000
    sizes = workloads.serve_sizes(1, 50_000)
    assert sizes.min() >= 1 and sizes.max() <= 16 << 20
    assert 7000 < np.median(sizes) < 9500
    arr = workloads.serve_arrivals(2, 20_000, 1e4)
    assert np.all(np.diff(arr) > 0) and 1.8 < arr[-1] < 2.2
    is_dec, is_bad = workloads.serve_kinds(3, 100_000)
    assert 0.48 < is_dec.mean() < 0.52 and not (is_bad & ~is_dec).any()
    assert 0.008 < is_bad[is_dec].mean() < 0.012
    assert workloads.non_alphabet_bytes(
        b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/").size == 191
    assert len(workloads.sweep_lengths()) == 51


def test_pipeline_output_buffer_checks():
    """The host pipeline writes through a raw pointer, so a short or unusable
    caller buffer must be refused before the call."""
    from paper_1910_05109_amd.pipeline import check_out
    assert check_out(None, 10, "t").size == 10
    ok = np.zeros(16, dtype=np.uint8)
    assert check_out(ok, 16, "t") is ok
    with pytest.raises(ValueError):
        check_out(np.zeros(15, dtype=np.uint8), 16, "t")
    with pytest.raises(ValueError):
        check_out(np.zeros(16, dtype=np.int32), 16, "t")
    with pytest.raises(ValueError):
        check_out(np.zeros((4, 4), dtype=np.uint8), 16, "t")
    with pytest.raises(ValueError):
        check_out(np.zeros(32, dtype=np.uint8)[::2], 16, "t")
    ro = np.zeros(16, dtype=np.uint8)
    ro.setflags(write=False)
    with pytest.raises(ValueError):
        check_out(ro, 16, "t")
    with pytest.raises(ValueError):
        check_out(bytearray(16), 16, "t")
