"""Host logic of the autotuner (CPU only): how it ranks launch shapes timed
on several sizes of one size bucket, and that the sizes it times lie in the
bucket the library files them under."""
import os

import pytest

from paper_1910_05109_amd import BUCKETS
from paper_1910_05109_amd.tune import BUCKET_SIZES, rank_shapes


def test_a_shape_close_to_the_best_everywhere_wins():
    # one shape fastest at the small end and slow at the large end, one the
    # reverse, one 10% behind the best at both
    times = {(1, 64, 0): [1.0, 4.0], (4, 1, 0): [2.0, 2.0], (2, 8, 0): [1.1, 2.2]}
    scored, best = rank_shapes(times)
    assert best == [1.0, 2.0]
    assert [sh for _, sh, _ in scored] == [(2, 8, 0), (1, 64, 0), (4, 1, 0)]   # the tie: smaller first
    assert scored[0][0] == pytest.approx(1.1)
    assert scored[1][0] == pytest.approx(1.5) and scored[2][0] == pytest.approx(1.5)


def test_relative_not_absolute_time_decides():
    # (2, 2, 1) saves more microseconds in total (at the large size) but is
    # twice as slow at the small one
    times = {(1, 4, 0): [1.0, 100.0], (2, 2, 1): [2.0, 98.0]}
    scored, _ = rank_shapes(times)
    assert scored[0][1] == (1, 4, 0)
    assert scored[0][0] == pytest.approx((1.0 + 100.0 / 98.0) / 2)


def test_one_size_picks_the_fastest():
    scored, best = rank_shapes({(8, 1, 1): [3.0], (2, 2, 1): [2.5], (1, 1, 0): [2.75]})
    assert scored[0][1] == (2, 2, 1) and scored[0][0] == 1.0 and best == [2.5]


def test_missing_times_are_refused():
    with pytest.raises(ValueError):
        rank_shapes({(1, 1, 0): [1.0, 2.0], (2, 1, 0): [1.0]})


def test_bucket_sizes_lie_in_their_buckets():
    from paper_1910_05109_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libb64hip.so not built")
    lib = _lib.load()
    assert len(BUCKET_SIZES) == BUCKETS
    for bucket, sizes in enumerate(BUCKET_SIZES):
        assert list(sizes) == sorted(sizes)
        for n in sizes:
            assert lib.b64_tune_bucket(n) == bucket, (bucket, n)
