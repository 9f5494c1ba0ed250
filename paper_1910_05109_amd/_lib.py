"""ctypes binding of libb64hip.so (C ABI declared in include/b64hip.h).

Argument marshalling only: pointers, sizes and the HIP stream go across; every
step of encoding, decoding and validation runs in the library's HIP kernels.
The single-buffer entry points are also reached through `fast`, a CPython
fast-call module (csrc/b64_pyfast.c) that load() binds to the same loaded
library: it marshals the same integers without ctypes' per-argument cost.
The library must have been built (python -m paper_1910_05109_amd.build); if it
is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libb64hip.so")

EARG = -(2 ** 63)
EHIP = -(2 ** 63) + 1

# entry points and their signatures, in the order of include/b64hip.h
_P, _I64, _INT, _U32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32
SIGNATURES = {
    "b64_encoded_len": ([_I64], _I64),
    "b64_decoded_max_len": ([_I64], _I64),
    "b64_encode": ([_P, _I64, _P, _P, _P], _I64),
    "b64_decode": ([_P, _I64, _P, _P, _P], _I64),
    "b64_decode_async": ([_P, _I64, _P, _P, _P, _P, _P], _I64),
    "b64_validate": ([_P, _I64, _P, _P], _I64),
    "b64_validate_async": ([_P, _I64, _P, _P, _P, _P], _I64),
    "b64_encode_batch": ([_P, _P, _I64, _P, _P, _P, _P, _P], _I64),
    "b64_decode_batch": ([_P, _P, _I64, _P, _P, _P, _P, _P, _P], _I64),
    "b64_encoded_len_mode": ([_I64, _U32, _I64], _I64),
    "b64_decoded_max_len_mode": ([_I64, _U32], _I64),
    "b64_decode_workspace_size": ([_I64, _U32], _I64),
    "b64_encode_mode": ([_P, _I64, _P, _P, _U32, _I64, _P], _I64),
    "b64_decode_mode": ([_P, _I64, _P, _P, _U32, _P], _I64),
    "b64_decode_mode_async": ([_P, _I64, _P, _P, _P, _P, _U32, _P, _I64, _P], _I64),
    "b64_decode_ws_async_noalloc": ([_P, _I64, _P, _P, _P, _P, _U32, _P], _I64),
    "b64_validate_mode": ([_P, _I64, _P, _U32, _P], _I64),
    "b64_validate_mode_async": ([_P, _I64, _P, _P, _P, _U32, _P, _I64, _P], _I64),
    "b64_encode_batch_mode": ([_P, _P, _I64, _P, _P, _P, _P, _U32, _P], _I64),
    "b64_decode_batch_mode": ([_P, _P, _I64, _P, _P, _P, _P, _P, _U32, _P], _I64),
    "b64_decode_f32_bf16": ([_P, _P, _I64, _I64, _P, _P, _P, _U32, _P], _I64),
    "b64_pipeline_create": ([_I64, _INT, _INT], _P),
    "b64_pipeline_destroy": ([_P], None),
    "b64_pipeline_encode": ([_P, _P, _I64, _P, _P], _I64),
    "b64_pipeline_decode": ([_P, _P, _I64, _P, _P], _I64),
    "b64_pipeline_last_error": ([], ctypes.c_char_p),
    "b64_server_create": ([_I64, _INT, _INT, _I64, _I64], _P),
    "b64_server_destroy": ([_P], None),
    "b64_server_set_zero_copy_max": ([_P, _I64], _I64),
    "b64_server_set_staging": ([_P, _INT], _I64),
    "b64_server_last_error": ([], ctypes.c_char_p),
    "b64_server_run": ([_P, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I64),
    "b64_tune_set_bucket": ([_INT, _INT, _INT, _INT, _INT], _I64),
    "b64_tune_set": ([_INT, _INT, _INT, _INT], _I64),
    "b64_tune_get_bucket": ([_INT, _INT], _I64),
    "b64_tune_get": ([_INT], _I64),
    "b64_tune_bucket": ([_I64], _I64),
    "b64_tune_ws_guess_min": ([_I64], _I64),
    "b64_tune_ws_small_max": ([_I64], _I64),
    "b64_yardstick": ([_INT, _P, _P, _I64, _P], _I64),
    "b64_last_error": ([], ctypes.c_char_p),
}
DATA_SYMBOLS = ("b64_alphabet_std", "b64_alphabet_url")

_lib = None


class B64Error(RuntimeError):
    """Raised when the library returns B64_EARG or B64_EHIP."""


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_1910_05109_amd.build` "
                "(there is no fallback codec)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _bind_fast(L)
        _lib = L
        _apply_tune_cache()
    return _lib


fast = None
FAST_ENTRY_POINTS = ("b64_encode", "b64_encode_mode", "b64_decode", "b64_decode_async",
                     "b64_validate", "b64_validate_async")


def _bind_fast(L: ctypes.CDLL) -> None:
    """Hand the fast-call binding (_b64fast, built beside the library) the
    addresses of its entry points in this loaded copy of the library."""
    global fast
    try:
        from . import _b64fast
    except ImportError as e:
        raise ImportError("the fast-call binding _b64fast is not built; run "
                          "`python -m paper_1910_05109_amd.build`") from e
    _b64fast.bind(*(ctypes.cast(getattr(L, name), ctypes.c_void_p).value
                    for name in FAST_ENTRY_POINTS))
    fast = _b64fast


def _apply_tune_cache() -> None:
    """Apply the autotuner's cached launch shapes of the current device, when
    a cache exists ($B64HIP_TUNE_CACHE, else ~/.cache/b64hip/tune.json;
    B64HIP_TUNE_CACHE=off skips it)."""
    from . import tune
    path = tune.cache_path()
    if path and os.path.exists(path):
        tune.apply_cached(path)


def last_error() -> str:
    msg = load().b64_last_error()
    return msg.decode(errors="replace") if msg else ""


def check(ret: int, what: str) -> int:
    if ret in (EARG, EHIP):
        kind = "bad argument" if ret == EARG else "HIP error"
        raise B64Error(f"{what}: {kind}: {last_error()}")
    return ret


def alphabet_bytes(name: str) -> bytes:
    """The library's own 64-byte alphabet constant ('std' or 'url')."""
    sym = {"std": "b64_alphabet_std", "url": "b64_alphabet_url"}[name]
    arr = (ctypes.c_char * 64).in_dll(load(), sym)
    return bytes(arr.raw)
