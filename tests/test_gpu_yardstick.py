"""GPU check of the bandwidth yardstick kernels (b64_yardstick): they move
exactly the bytes their access pattern names and nothing past them, so the
ceiling they measure is the ceiling of the codec's own loads and stores."""
import ctypes

import numpy as np
import pytest

import workloads
from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_05109_amd import _lib
    return _lib.load()


@pytest.mark.parametrize("nch", [1, 7, 1000, 123_457, 3_000_001])
def test_patterns_move_the_named_bytes(lib, nch):
    import torch
    from paper_1910_05109_amd import stream_ptr
    x = workloads.random_bytes(workloads.SEED_BASE + 380, 16 * nch + 64)
    src = to_dev(x)
    w = x[: 16 * nch].view(np.uint32).reshape(-1, 4)
    for kind, rin, wout in ((2, 12, 16), (3, 16, 12), (4, 16, 16), (1, 0, 16)):
        say("yardstick", kind, nch)
        dst = torch.full((16 * nch + 256,), 0xA5, dtype=torch.uint8, device="cuda")
        assert lib.b64_yardstick(kind, src.data_ptr(), dst.data_ptr(), nch, stream_ptr()) == 0
        got = to_host(dst)
        assert (got[wout * nch:] == 0xA5).all(), (kind, nch)       # nothing past the end
        if kind == 2:
            i = x[: 12 * nch].view(np.uint32).reshape(-1, 3)
            exp = np.stack([i[:, 0], i[:, 1], i[:, 2], i[:, 0] ^ i[:, 2]], axis=1)
            assert np.array_equal(got[: 16 * nch].view(np.uint32).reshape(-1, 4), exp)
        elif kind == 3:
            exp = np.stack([w[:, 0] ^ w[:, 3], w[:, 1], w[:, 2]], axis=1)
            assert np.array_equal(got[: 12 * nch].view(np.uint32).reshape(-1, 3), exp)
        elif kind == 4:
            assert np.array_equal(got[: 16 * nch], x[: 16 * nch])
        else:
            words = got[: 16 * nch].view(np.uint32).reshape(-1, 4)
            assert (words[:, 3] == 0x3D3D3D3D).all()                  # every chunk written
            assert np.array_equal(words[:, 0], (np.arange(nch) & 0xFFFFFFFF).astype(np.uint32))
    # read only: one word per workgroup, nothing past 64 KiB
    dst = torch.full((1 << 17,), 0xA5, dtype=torch.uint8, device="cuda")
    assert lib.b64_yardstick(0, src.data_ptr(), dst.data_ptr(), nch, stream_ptr()) == 0
    assert (to_host(dst)[1 << 16:] == 0xA5).all()


def test_bad_arguments(lib):
    fake = ctypes.c_void_p(0x1000)
    EARG = -(2 ** 63)
    assert lib.b64_yardstick(5, fake, fake, 10, None) == EARG
    assert lib.b64_yardstick(2, fake, fake, -1, None) == EARG
    assert lib.b64_yardstick(2, None, fake, 10, None) == EARG
    assert lib.b64_yardstick(2, fake, fake, 0, None) == 0
