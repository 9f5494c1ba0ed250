"""Host logic of the serving binding, the batch planner, the workload
recipes and the host pipeline's buffer checks (CPU only)."""
import numpy as np
import pytest

import workloads
from paper_1910_05109_amd.batch import decoded_capacity, encoded_lengths, prefix
from paper_1910_05109_amd.serve import DEC, ENC, out_layout


def test_layout_helpers():
    lens = np.array([0, 1, 2, 3, 4, 5, 100], dtype=np.int64)
    assert encoded_lengths(lens).tolist() == [0, 4, 4, 4, 8, 8, 136]
    assert decoded_capacity(lens).tolist() == [0, 0, 0, 0, 3, 3, 75]
    assert prefix(lens).tolist() == [0, 0, 1, 3, 6, 10, 15, 115]


def test_server_output_layout():
    """Each request gets the output capacity of its kind, packed in order."""
    kinds = np.array([ENC, DEC, ENC, DEC, DEC], dtype=np.int32)
    lens = np.array([5, 9, 0, 4, 3], dtype=np.int64)
    assert out_layout(kinds, lens).tolist() == [0, 8, 14, 14, 17, 17]


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
