"""Host-memory encode / decode through the library's chunked pipeline
(b64_pipeline_* in the C ABI): chunks of the host input stream through pinned
staging, host-to-device copies, the HIP kernels and device-to-host copies,
one stream per stage, up to three chunks in flight.  Arrays in pinned host
memory (torch's pin_memory tensors, viewed with .numpy()) are copied to and
from the device directly, without the staging copies.  The Python side only
passes numpy buffers."""
from __future__ import annotations

import ctypes

import numpy as np

from . import STD, _lib
from ._lib import B64Error, check, load


def check_out(out, need: int, what: str) -> np.ndarray:
    """A host output buffer of at least `need` bytes for the C pipeline, which
    writes `need` bytes through a raw pointer: a new one when `out` is None,
    else `out` itself if it is a writable, contiguous, one-dimensional uint8
    numpy array that large (anything else raises ValueError)."""
    if out is None:
        return np.empty(max(need, 1), dtype=np.uint8)
    if (not isinstance(out, np.ndarray) or out.dtype != np.uint8 or out.ndim != 1
            or not out.flags.c_contiguous or not out.flags.writeable):
        raise ValueError(f"{what}: out must be a writable, contiguous 1-D uint8 numpy array")
    if out.size < need:
        raise ValueError(f"{what}: out holds {out.size} bytes, {need} are needed")
    return out


class HostPipeline:
    """Owns the pipeline's streams and staging buffers until close()."""

    def __init__(self, chunk_bytes: int = 64 << 20, depth: int = 3, host_threads: int = 8):
        L = load()
        self._h = L.b64_pipeline_create(int(chunk_bytes), int(depth), int(host_threads))
        if not self._h:
            raise B64Error("b64_pipeline_create: " + (L.b64_pipeline_last_error() or b"").decode())

    def close(self):
        if self._h:
            load().b64_pipeline_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _u8(x) -> np.ndarray:
        if isinstance(x, (bytes, bytearray, memoryview)):
            return np.frombuffer(bytes(x), dtype=np.uint8)
        return np.ascontiguousarray(np.asarray(x, dtype=np.uint8).reshape(-1))

    def _check(self, r, what):
        if r in (_lib.EARG, _lib.EHIP):
            msg = load().b64_pipeline_last_error() or load().b64_last_error() or b""
            raise B64Error(f"{what}: {msg.decode(errors='replace')}")
        return r

    def encode(self, x, alphabet=STD, out: np.ndarray | None = None) -> np.ndarray:
        x = self._u8(x)
        out = check_out(out, check(load().b64_encoded_len(x.size), "b64_encoded_len"),
                        "HostPipeline.encode")
        a = ctypes.create_string_buffer(bytes(alphabet), 64)
        r = self._check(load().b64_pipeline_encode(self._h, x.ctypes.data, x.size,
                                                   out.ctypes.data, a), "b64_pipeline_encode")
        return out[:r]

    def decode(self, s, alphabet=STD, out: np.ndarray | None = None):
        """(bytes, None) if valid, (None, first_invalid_offset) if not."""
        s = self._u8(s)
        out = check_out(out, check(load().b64_decoded_max_len(s.size), "b64_decoded_max_len"),
                        "HostPipeline.decode")
        a = ctypes.create_string_buffer(bytes(alphabet), 64)
        r = self._check(load().b64_pipeline_decode(self._h, s.ctypes.data, s.size,
                                                   out.ctypes.data, a), "b64_pipeline_decode")
        return (out[:r], None) if r >= 0 else (None, ~r)
