"""Base64 codec for AMD MI355X (gfx950): HIP kernels behind a C ABI.

After W. Mula and D. Lemire, "Base64 encoding and decoding at almost the
speed of a memory copy".  PyTorch is used only for device memory and streams;
every step of the codec runs in libb64hip.so.

  encode(x)                -> uint8 CUDA tensor of 4*ceil(n/3) characters
  decode(s)                -> (uint8 tensor, None) or (None, first_invalid_offset)
  decode_async(s)          -> (out, status) with status = int64[2] on the device:
                              [decoded length or -1, -1 or first invalid offset]
  validate(s)              -> (decoded length, None) or (None, first_invalid_offset),
                              reading s only (no output is written)
  encode_batch(src, in_off)-> (dst, out_off, out_len)
  decode_batch(src, in_off)-> (dst, out_off, out_len, first_bad)

Variants (keyword arguments; the paper makes '=' optional and names MIME):
  flags=NOPAD     no '=' (encode), '=' invalid and a final quantum of 2-3
                  characters allowed (decode / validate; also in batches)
  flags=SKIP_WS   decode / validate ignore space, tab, CR, LF
  line_len=L      encode breaks lines of L characters (a multiple of 4) with CR LF

Fused consumer:
  decode_f32_bf16(src, in_off, dim) -> (bf16 tensor [nrows, dim], status [nrows]):
                  rows of base64 float32 decoded straight into bfloat16

Tensors are torch.uint8 (data) / torch.int64 (offsets) on the current CUDA
(HIP) device; work is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import B64Error, check, load

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"

OPS = {"encode": 0, "decode": 1, "encode_batch": 2, "decode_batch": 3, "validate": 4,
       "encode_wrap": 5, "decode_ws": 6, "decode_f32_bf16": 7}
NOPAD = 1
SKIP_WS = 2

__all__ = ["STD", "URL", "NOPAD", "SKIP_WS", "B64Error", "load", "encoded_len", "decoded_max_len",
           "workspace_size", "encode",
           "decode", "decode_async", "validate", "validate_async", "encode_batch", "decode_batch",
           "decode_f32_bf16", "tune_set", "tune_get", "tune_shapes", "tune_restore", "tune_bucket",
           "tune_ws_guess_min", "tune_ws_small_max", "stream_ptr", "BUCKETS"]


# The wrappers below sit on the launch path of every call, so they keep their
# own host work small: at a few MiB a call costs about as much on the host as
# on the GPU.  torch's types and stream accessors are looked up once, and the
# single-buffer entry points go through the fast-call binding (_lib.fast).
_torch_mod = None
_Tensor = _U8 = _I64 = None
_raw_stream = _cur_device = None


def _torch():
    global _torch_mod, _Tensor, _U8, _I64, _raw_stream, _cur_device
    if _torch_mod is None:
        import torch
        _Tensor, _U8, _I64 = torch.Tensor, torch.uint8, torch.int64
        c = torch._C
        if hasattr(c, "_cuda_getCurrentRawStream"):
            _raw_stream, _cur_device = c._cuda_getCurrentRawStream, c._cuda_getDevice
        _torch_mod = torch
    return _torch_mod


def _fast():
    if _lib.fast is None:
        load()
    return _lib.fast


def stream_ptr(stream=None) -> int:
    """Raw HIP stream of `stream`, or of torch's current stream."""
    if stream is not None:
        return int(stream.cuda_stream)
    if _raw_stream is not None:
        # the raw accessor skips building a torch Stream object (about 3 us)
        return _raw_stream(_cur_device())
    return int(_torch().cuda.current_stream().cuda_stream)


_alpha_cache: dict = {}


def _alpha(alphabet) -> ctypes.Array:
    """The 64 alphabet bytes as a C buffer (the library copies them by value
    at each call); kept per alphabet."""
    buf = _alpha_cache.get(alphabet) if isinstance(alphabet, bytes) else None
    if buf is None:
        a = bytes(alphabet)
        if len(a) != 64:
            raise ValueError("alphabet must have 64 bytes")
        buf = ctypes.create_string_buffer(a, 64)
        if isinstance(alphabet, bytes) and len(_alpha_cache) < 256:
            _alpha_cache[alphabet] = buf
    return buf


_alpha_addrs: dict = {}


def _alpha_addr(alphabet) -> int:
    """Address of _alpha(alphabet)'s buffer, for the fast-call binding; the
    buffer stays alive in _alpha_cache (or in `_alpha_addrs`' own entry for
    alphabets that are not cached there)."""
    hit = _alpha_addrs.get(alphabet) if isinstance(alphabet, bytes) else None
    if hit is not None:
        return hit[0]
    buf = _alpha(alphabet)
    addr = ctypes.addressof(buf)
    if isinstance(alphabet, bytes) and len(_alpha_addrs) < 256:
        _alpha_addrs[alphabet] = (addr, buf)
    else:
        _alpha_keep.append(buf)
        del _alpha_keep[:-8]
    return addr


_alpha_keep: list = []


def _check_u8(t, what):
    if _Tensor is None:
        _torch()
    if not isinstance(t, _Tensor) or t.dtype is not _U8 or not t.is_cuda:
        raise TypeError(f"{what} must be a torch.uint8 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def _check_i64(t, what):
    if _Tensor is None:
        _torch()
    if not isinstance(t, _Tensor) or t.dtype is not _I64 or not t.is_cuda:
        raise TypeError(f"{what} must be a torch.int64 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


# The plain sizes 4*ceil(n/3) and 3*floor(n/4) (b64_encoded_len and
# b64_decoded_max_len) computed here, without a library round trip on every
# call; tests/test_abi.py pins these copies to the library's helpers.
def _plain_enc_len(n: int) -> int:
    return 4 * ((n + 2) // 3)


def _plain_dec_cap(n: int) -> int:
    return 3 * (n // 4)


def encoded_len(n: int, flags: int = 0, line_len: int = 0) -> int:
    if flags == 0 and line_len == 0:
        return check(load().b64_encoded_len(n), "encoded_len")
    return check(load().b64_encoded_len_mode(n, flags, line_len), "encoded_len_mode")


def decoded_max_len(n: int, flags: int = 0) -> int:
    if flags == 0:
        return check(load().b64_decoded_max_len(n), "decoded_max_len")
    return check(load().b64_decoded_max_len_mode(n, flags), "decoded_max_len_mode")


def workspace_size(n: int, flags: int = 0) -> int:
    """Device workspace bytes of an asynchronous decode / validate."""
    return check(load().b64_decode_workspace_size(n, flags), "decode_workspace_size")


def _workspace(n, flags, workspace, device):
    need = workspace_size(n, flags)
    if need == 0:
        return 0, 0
    if workspace is None:
        workspace = _torch().empty(need, dtype=_torch().uint8, device=device)
    _check_u8(workspace, "workspace")
    return workspace.data_ptr(), workspace.numel()


def encode(x, alphabet=STD, out=None, stream=None, flags: int = 0, line_len: int = 0):
    """Encode a uint8 CUDA tensor; returns out[:encoded length] (asynchronous)."""
    F = _lib.fast or _fast()
    _check_u8(x, "x")
    n = x.numel()
    plain = flags == 0 and line_len == 0
    m = _plain_enc_len(n) if plain else encoded_len(n, flags, line_len)
    if out is None:
        out = _torch_mod.empty(max(m, 1), dtype=_U8, device=x.device)
    else:
        _check_u8(out, "out")
        if out.numel() < m:
            raise ValueError("out too small")
    hit = _alpha_addrs.get(alphabet) if alphabet.__class__ is bytes else None
    a = hit[0] if hit is not None else _alpha_addr(alphabet)
    st = _raw_stream(_cur_device()) if stream is None and _raw_stream is not None else stream_ptr(stream)
    if plain:
        r = F.encode(x.data_ptr(), n, out.data_ptr(), a, st)
    else:
        r = F.encode_mode(x.data_ptr(), n, out.data_ptr(), a, flags, line_len, st)
    if r < 0:
        check(r, "b64_encode" if plain else "b64_encode_mode")
    return out if out.numel() == r else out[:r]


def decode(s, alphabet=STD, out=None, stream=None, flags: int = 0):
    """Blocking decode: (bytes_tensor, None) if valid, (None, first_bad) if not."""
    F = _fast()
    _check_u8(s, "s")
    n = s.numel()
    cap = _plain_dec_cap(n) if flags == 0 else decoded_max_len(n, flags)
    if out is None:
        out = _torch().empty(max(cap, 1), dtype=_U8, device=s.device)
    else:
        _check_u8(out, "out")
        if out.numel() < cap:
            raise ValueError("out too small")
    if flags == 0:
        r = check(F.decode(s.data_ptr(), n, out.data_ptr(), _alpha_addr(alphabet),
                           stream_ptr(stream)), "b64_decode")
    else:
        r = check(load().b64_decode_mode(s.data_ptr(), n, out.data_ptr(), _alpha(alphabet), flags,
                                         stream_ptr(stream)), "b64_decode_mode")
    if r < 0:
        return None, ~r
    return out[:r], None


def decode_async(s, alphabet=STD, out=None, status=None, stream=None, flags: int = 0,
                 workspace=None):
    """Asynchronous decode.  Returns (out, status), status = int64[2] on the
    device: [decoded length or -1, -1 or first invalid offset].  With SKIP_WS a
    device workspace of workspace_size(n, flags) bytes is used (allocated here
    unless given)."""
    F = _lib.fast or _fast()
    _check_u8(s, "s")
    n = s.numel()
    cap = _plain_dec_cap(n) if flags == 0 else decoded_max_len(n, flags)
    if out is None:
        out = _torch_mod.empty(max(cap, 1), dtype=_U8, device=s.device)
    else:
        _check_u8(out, "out")
    if status is None:
        status = _torch_mod.empty(2, dtype=_I64, device=s.device)
    else:
        _check_i64(status, "status")
    if out.numel() < cap or status.numel() < 2:
        raise ValueError("out or status too small")
    sp = status.data_ptr()
    st = _raw_stream(_cur_device()) if stream is None and _raw_stream is not None else stream_ptr(stream)
    if flags == 0:
        hit = _alpha_addrs.get(alphabet) if alphabet.__class__ is bytes else None
        a = hit[0] if hit is not None else _alpha_addr(alphabet)
        r = F.decode_async(s.data_ptr(), n, out.data_ptr(), sp, sp + 8, a, st)
        if r < 0:
            check(r, "b64_decode_async")
    else:
        wp, wn = _workspace(n, flags, workspace, s.device)
        check(load().b64_decode_mode_async(s.data_ptr(), n, out.data_ptr(), sp, sp + 8,
                                           _alpha(alphabet), flags, wp, wn, st),
              "b64_decode_mode_async")
    return out, status


def validate(s, alphabet=STD, stream=None, flags: int = 0):
    """Blocking, read-only: (decoded length, None) if s is a valid encoding,
    (None, first_invalid_offset) if not."""
    F = _fast()
    _check_u8(s, "s")
    if flags == 0:
        r = check(F.validate(s.data_ptr(), s.numel(), _alpha_addr(alphabet), stream_ptr(stream)),
                  "b64_validate")
    else:
        r = check(load().b64_validate_mode(s.data_ptr(), s.numel(), _alpha(alphabet), flags,
                                           stream_ptr(stream)), "b64_validate_mode")
    return (r, None) if r >= 0 else (None, ~r)


def validate_async(s, alphabet=STD, status=None, stream=None, flags: int = 0, workspace=None):
    """Asynchronous validation; status = int64[2] on the device:
    [decoded length or -1, -1 or first invalid offset]."""
    F = _lib.fast or _fast()
    _check_u8(s, "s")
    if status is None:
        status = _torch_mod.empty(2, dtype=_I64, device=s.device)
    else:
        _check_i64(status, "status")
    if status.numel() < 2:
        raise ValueError("status too small")
    sp = status.data_ptr()
    st = _raw_stream(_cur_device()) if stream is None and _raw_stream is not None else stream_ptr(stream)
    if flags == 0:
        hit = _alpha_addrs.get(alphabet) if alphabet.__class__ is bytes else None
        a = hit[0] if hit is not None else _alpha_addr(alphabet)
        r = F.validate_async(s.data_ptr(), s.numel(), sp, sp + 8, a, st)
        if r < 0:
            check(r, "b64_validate_async")
    else:
        wp, wn = _workspace(s.numel(), flags, workspace, s.device)
        check(load().b64_validate_mode_async(s.data_ptr(), s.numel(), sp, sp + 8, _alpha(alphabet),
                                             flags, wp, wn, st),
              "b64_validate_mode_async")
    return status


def _validate_layout(src, in_off, dst, out_off, cap_of, what):
    """Host-side bounds check of a batch layout before launching: offsets
    non-decreasing and inside `src`, every output region inside `dst`.  The
    kernels trust the offsets, so a bad layout must be stopped here."""
    torch = _torch()
    nbuf = in_off.numel() - 1
    if nbuf <= 0:
        return
    if torch.cuda.is_current_stream_capturing():
        return  # no host sync inside a capture; graph users check layouts when loading them
    if out_off.numel() < nbuf:
        raise ValueError(f"{what}: out_off needs {nbuf} entries")
    lens = in_off[1:] - in_off[:-1]
    ends = out_off[:nbuf] + cap_of(lens)
    stats = torch.stack([in_off[0], in_off[-1], lens.min(), out_off[:nbuf].min(), ends.max()]).cpu()
    first, last, min_len, min_out, max_end = (int(v) for v in stats)
    if first < 0 or min_len < 0 or last > src.numel():
        raise ValueError(f"{what}: in_off must be non-decreasing within src "
                         f"(first {first}, last {last}, src has {src.numel()} bytes)")
    if min_out < 0 or max_end > dst.numel():
        raise ValueError(f"{what}: outputs end at {max_end}, dst has {dst.numel()} bytes")


def _enc_cap(L):
    return 4 * _torch().div(L + 2, 3, rounding_mode="floor")


def _dec_cap(L):
    return 3 * _torch().div(L, 4, rounding_mode="floor")


def _enc_cap_nopad(L):
    return _torch().div(4 * L + 2, 3, rounding_mode="floor")


def _dec_cap_nopad(L):
    r = L % 4
    return 3 * _torch().div(L, 4, rounding_mode="floor") + (r - 1).clamp(min=0)


def _batch_layout(in_off, per_len):
    torch = _torch()
    lens = in_off[1:] - in_off[:-1]
    out_off = torch.zeros_like(in_off)
    torch.cumsum(per_len(lens), 0, out=out_off[1:])
    return out_off


def encode_batch(src, in_off, alphabet=STD, dst=None, out_off=None, out_len=None, stream=None,
                 validate=True, flags: int = 0):
    """Encode nbuf = len(in_off)-1 packed buffers in one launch (asynchronous
    unless `validate`, which checks the layout on the host first).
    Returns (dst, out_off, out_len); out_off has nbuf+1 entries."""
    torch = _torch()
    _check_u8(src, "src")
    _check_i64(in_off, "in_off")
    nbuf = in_off.numel() - 1
    cap = _enc_cap_nopad if flags & NOPAD else _enc_cap
    if out_off is None:
        out_off = _batch_layout(in_off, cap)
    _check_i64(out_off, "out_off")
    if dst is None:
        dst = torch.empty(max(int(out_off[-1].item()), 1), dtype=torch.uint8, device=src.device)
    if out_len is None:
        out_len = torch.empty(max(nbuf, 1), dtype=torch.int64, device=src.device)
    _check_u8(dst, "dst")
    _check_i64(out_len, "out_len")
    if out_len.numel() < nbuf:
        raise ValueError("out_len too small")
    if validate:
        _validate_layout(src, in_off, dst, out_off, cap, "encode_batch")
    if flags == 0:
        check(load().b64_encode_batch(src.data_ptr(), in_off.data_ptr(), nbuf, dst.data_ptr(),
                                      out_off.data_ptr(), out_len.data_ptr(), _alpha(alphabet),
                                      stream_ptr(stream)), "b64_encode_batch")
    else:
        check(load().b64_encode_batch_mode(src.data_ptr(), in_off.data_ptr(), nbuf, dst.data_ptr(),
                                           out_off.data_ptr(), out_len.data_ptr(), _alpha(alphabet),
                                           flags, stream_ptr(stream)), "b64_encode_batch_mode")
    return dst, out_off, out_len[:nbuf]


def decode_batch(src, in_off, alphabet=STD, dst=None, out_off=None, out_len=None,
                 first_bad=None, stream=None, validate=True, flags: int = 0):
    """Decode nbuf packed buffers in one launch (asynchronous).  Returns
    (dst, out_off, out_len, first_bad): out_len[b] = length or -1,
    first_bad[b] = -1 or the first invalid offset within buffer b."""
    torch = _torch()
    _check_u8(src, "src")
    _check_i64(in_off, "in_off")
    nbuf = in_off.numel() - 1
    cap = _dec_cap_nopad if flags & NOPAD else _dec_cap
    if out_off is None:
        out_off = _batch_layout(in_off, cap)
    _check_i64(out_off, "out_off")
    if dst is None:
        dst = torch.empty(max(int(out_off[-1].item()), 1), dtype=torch.uint8, device=src.device)
    if out_len is None:
        out_len = torch.empty(max(nbuf, 1), dtype=torch.int64, device=src.device)
    if first_bad is None:
        first_bad = torch.empty(max(nbuf, 1), dtype=torch.int64, device=src.device)
    _check_u8(dst, "dst")
    _check_i64(out_len, "out_len")
    _check_i64(first_bad, "first_bad")
    if out_len.numel() < nbuf or first_bad.numel() < nbuf:
        raise ValueError("out_len / first_bad too small")
    if validate:
        _validate_layout(src, in_off, dst, out_off, cap, "decode_batch")
    if flags == 0:
        check(load().b64_decode_batch(src.data_ptr(), in_off.data_ptr(), nbuf, dst.data_ptr(),
                                      out_off.data_ptr(), out_len.data_ptr(), first_bad.data_ptr(),
                                      _alpha(alphabet), stream_ptr(stream)), "b64_decode_batch")
    else:
        check(load().b64_decode_batch_mode(src.data_ptr(), in_off.data_ptr(), nbuf, dst.data_ptr(),
                                           out_off.data_ptr(), out_len.data_ptr(),
                                           first_bad.data_ptr(), _alpha(alphabet), flags,
                                           stream_ptr(stream)), "b64_decode_batch_mode")
    return dst, out_off, out_len[:nbuf], first_bad[:nbuf]


def decode_f32_bf16(src, in_off, dim: int, alphabet=STD, dst=None, status=None, stream=None,
                    validate=True, flags: int = 0):
    """Decode nrows = len(in_off)-1 packed rows, each the base64 encoding of
    `dim` float32 values, straight into a [nrows, dim] bfloat16 tensor
    (asynchronous).  Returns (dst, status): status[b] = -1 (good), the first
    invalid offset, or -2 (valid base64 of the wrong length)."""
    torch = _torch()
    _check_u8(src, "src")
    _check_i64(in_off, "in_off")
    nrows = in_off.numel() - 1
    if dim < 0 or nrows < 0:
        raise ValueError("dim and the row count must be >= 0")
    if dst is None:
        dst = torch.empty((max(nrows, 1), max(dim, 1)), dtype=torch.bfloat16, device=src.device)
    if status is None:
        status = torch.empty(max(nrows, 1), dtype=torch.int64, device=src.device)
    if dst.dtype != torch.bfloat16 or not dst.is_cuda or not dst.is_contiguous():
        raise TypeError("dst must be a contiguous torch.bfloat16 CUDA tensor")
    _check_i64(status, "status")
    if dst.numel() < nrows * dim or status.numel() < nrows:
        raise ValueError("dst or status too small")
    if validate and nrows > 0 and not torch.cuda.is_current_stream_capturing():
        lens = in_off[1:] - in_off[:-1]
        first, last, min_len = (int(v) for v in torch.stack([in_off[0], in_off[-1], lens.min()]).cpu())
        if first < 0 or min_len < 0 or last > src.numel():
            raise ValueError("decode_f32_bf16: in_off must be non-decreasing within src")
    check(load().b64_decode_f32_bf16(src.data_ptr(), in_off.data_ptr(), nrows, dim,
                                     dst.data_ptr(), status.data_ptr(), _alpha(alphabet), flags,
                                     stream_ptr(stream)), "b64_decode_f32_bf16")
    return dst.reshape(-1)[: nrows * dim].view(nrows, dim), status[:nrows]


BUCKETS = 5   # size buckets of the launch shapes: < 64 KiB, < 1 MiB, < 16 MiB, < 128 MiB, larger


def tune_set(op: str, unroll: int, blocks_per_cu: int, nontemporal: int = 1,
             bucket: int = -1) -> None:
    """Launch shape of `op` for inputs in size `bucket` (-1: every bucket)."""
    check(load().b64_tune_set_bucket(OPS[op], bucket, unroll, blocks_per_cu, int(nontemporal)),
          "b64_tune_set_bucket")


def tune_bucket(n: int) -> int:
    """Size bucket of an input of n bytes."""
    return check(load().b64_tune_bucket(n), "b64_tune_bucket")


def tune_ws_guess_min(min_chars: int = -1) -> int:
    """Size in bytes from which the whitespace-skipping decode tries the
    regular-line guess; sets it when min_chars >= 0.  Returns the previous
    size."""
    return int(load().b64_tune_ws_guess_min(int(min_chars)))


def tune_ws_small_max(max_chars: int = -1) -> int:
    """Size in bytes up to which the whitespace-skipping decode runs in one
    launch of one workgroup (at most 65,536); sets it when max_chars >= 0.
    Returns the previous size."""
    return check(load().b64_tune_ws_small_max(int(max_chars)), "b64_tune_ws_small_max")


def tune_get(op: str, bucket: int = BUCKETS - 1) -> tuple[int, int, int]:
    """(unroll, blocks_per_cu, nontemporal) of `op` in size `bucket`."""
    v = check(load().b64_tune_get_bucket(OPS[op], bucket), "b64_tune_get_bucket")
    return (v // 100) % 100, v % 100, v // 10000


def tune_shapes(op: str) -> list[tuple[int, int, int]]:
    """The shapes of `op` in every size bucket."""
    return [tune_get(op, b) for b in range(BUCKETS)]


def tune_restore(op: str, shapes) -> None:
    """Set the shapes of `op` in every bucket (as tune_shapes returns them)."""
    for b, sh in enumerate(shapes):
        tune_set(op, *sh, bucket=b)
