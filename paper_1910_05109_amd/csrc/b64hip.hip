// b64hip.hip -- base64 encode / decode kernels for gfx950 and the C ABI of
// libb64hip.so (declared in include/b64hip.h).
//
// Method: W. Mula and D. Lemire, "Base64 encoding and decoding at almost the
// speed of a memory copy".  The paper's AVX-512 kernels process 48 input
// bytes (encode) or 64 characters (decode) per register; here every lane of a
// 64-wide wavefront processes a 12-byte -> 16-character (encode) or
// 16-character -> 12-byte (decode) chunk, and consecutive lanes own
// consecutive chunks, so that every wave-wide load and store is one contiguous
// 768- or 1024-byte span.
//
// Encode (Section "Encoding"): the byte gather (s1,s2,s3) -> (s2,s1,s3,s2) is
// one v_perm_b32 per group; the four 6-bit indices are the low six bits of
// that word shifted right by 10, 4, 22 and 16 (the paper's multishift
// amounts), and each index selects its character from the runtime alphabet
// staged in LDS (the paper's second vpermb).
//
// Decode (Section "Decoding"): each character goes through a 256-entry map in
// LDS holding its 6-bit value or 0xFF (the paper's 0x80 "invalid" value; the
// 256-entry map also covers bytes >= 0x80 directly).  The map values are ORed
// into a per-lane error word that is tested once, after the lane's whole
// share of the input (the paper's deferred vpternlogd/vpmovb2m check); a
// wave-wide ballot skips the slow path when every lane is clean.  A lane that
// saw an invalid character (or a '=') rescans its chunks to find the first
// invalid offset and publishes it with an atomic minimum.  Four 6-bit values
// are packed as a<<18 | b<<12 | c<<6 | d (the paper's two multiply-adds) and
// the three bytes of four quanta are packed into three dwords by v_perm_b32
// (the paper's final vpermb).  The last quantum, with its '=' rules, goes
// through a separate single-lane path (the paper's "conventional code path").
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "b64hip.h"

extern "C" {
const char b64_alphabet_std[64] = {
    'A', 'B', 'C', 'D', 'E', 'F', 'G', 'H', 'I', 'J', 'K', 'L', 'M', 'N', 'O', 'P',
    'Q', 'R', 'S', 'T', 'U', 'V', 'W', 'X', 'Y', 'Z', 'a', 'b', 'c', 'd', 'e', 'f',
    'g', 'h', 'i', 'j', 'k', 'l', 'm', 'n', 'o', 'p', 'q', 'r', 's', 't', 'u', 'v',
    'w', 'x', 'y', 'z', '0', '1', '2', '3', '4', '5', '6', '7', '8', '9', '+', '/'};
const char b64_alphabet_url[64] = {
    'A', 'B', 'C', 'D', 'E', 'F', 'G', 'H', 'I', 'J', 'K', 'L', 'M', 'N', 'O', 'P',
    'Q', 'R', 'S', 'T', 'U', 'V', 'W', 'X', 'Y', 'Z', 'a', 'b', 'c', 'd', 'e', 'f',
    'g', 'h', 'i', 'j', 'k', 'l', 'm', 'n', 'o', 'p', 'q', 'r', 's', 't', 'u', 'v',
    'w', 'x', 'y', 'z', '0', '1', '2', '3', '4', '5', '6', '7', '8', '9', '-', '_'};
}

namespace {

constexpr int kThreads = 256;          // 4 waves of 64 lanes per workgroup
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kPad = '=';
constexpr uint32_t kBad = 0xFF;        // decode-map value of a non-alphabet byte
constexpr int64_t kNoError = INT64_MAX;
constexpr int kXcds = 8;               // MI355X: 8 accelerator dies, each with its own L2
constexpr int kLine = 128;             // L2 cache line, bytes

// Runtime alphabet, passed by value as a kernel argument.
struct EncTab { uint32_t w[16]; };     // byte v = character of value v
struct DecMap { uint32_t w[64]; };     // byte c = value of character c, or kBad

// Byte-aligned vector types: the amdhsa ABI runs with unaligned global access
// enabled, so these compile to single dwordx3 / dwordx4 accesses whatever the
// address; packed ragged buffers start at arbitrary byte offsets.
typedef uint32_t u32x3 __attribute__((ext_vector_type(3), aligned(1)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4), aligned(1)));
typedef uint32_t u32a1 __attribute__((aligned(1)));

// Streaming loads and stores of 12 or 16 bytes at any byte address; NT marks
// them nontemporal (each byte is touched once, so nothing is worth keeping in
// the caches).  The pointer types carry the byte alignment explicitly.
template <bool NT>
__device__ __forceinline__ u32x3 load12(const uint8_t *p)
{
    if constexpr (NT) return __builtin_nontemporal_load((const u32x3 *)p);
    else return *(const u32x3 *)p;
}
template <bool NT>
__device__ __forceinline__ u32x4 load16(const uint8_t *p)
{
    if constexpr (NT) return __builtin_nontemporal_load((const u32x4 *)p);
    else return *(const u32x4 *)p;
}
template <bool NT>
__device__ __forceinline__ void store12(uint8_t *p, u32x3 v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, (u32x3 *)p);
    else *(u32x3 *)p = v;
}
template <bool NT>
__device__ __forceinline__ void store16(uint8_t *p, u32x4 v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, (u32x4 *)p);
    else *(u32x4 *)p = v;
}

// ---------------------------------------------------------------- encode --

// Four characters of one group.  g holds the gathered bytes
// s2 | s1<<8 | s3<<16 | s2<<24; shifting right by 10, 4, 22, 16 and keeping
// six bits gives s1 div 4, (s2 div 16)+(s1*16 mod 64), (s2*4 mod 64)+(s3 div 64)
// and s3 mod 64 (Section "Encoding", step 1; Section "Base64" closed form).
__device__ __forceinline__ uint32_t enc_group(uint32_t g, const uint8_t *tab)
{
    uint32_t c0 = tab[(g >> 10) & 63];
    uint32_t c1 = tab[(g >> 4) & 63];
    uint32_t c2 = tab[(g >> 22) & 63];
    uint32_t c3 = tab[(g >> 16) & 63];
    return c0 | (c1 << 8) | (c2 << 16) | (c3 << 24);
}

// 12 input bytes b0..b11 (little-endian in three dwords) -> 16 characters.
// v_perm_b32(hi, lo, sel) picks bytes of the 8-byte value hi:lo.
__device__ __forceinline__ u32x4 enc_chunk(u32x3 in, const uint8_t *tab)
{
    u32x4 o;
    o.x = enc_group(__builtin_amdgcn_perm(in.x, in.x, 0x01020001u), tab);  // b1 b0 b2 b1
    o.y = enc_group(__builtin_amdgcn_perm(in.y, in.x, 0x04050304u), tab);  // b4 b3 b5 b4
    o.z = enc_group(__builtin_amdgcn_perm(in.z, in.y, 0x03040203u), tab);  // b7 b6 b8 b7
    o.w = enc_group(__builtin_amdgcn_perm(in.z, in.z, 0x02030102u), tab);  // b10 b9 b11 b10
    return o;
}

// Scalar path for 0..r bytes: whole groups, then a last group of one or two
// bytes zero-filled and padded with '=' (Section "Base64").
__device__ void enc_scalar(const uint8_t *p, int64_t r, uint8_t *o, const uint8_t *tab)
{
    int64_t i = 0;
    for (; i + 3 <= r; i += 3, o += 4) {
        uint32_t s1 = p[i], s2 = p[i + 1], s3 = p[i + 2];
        *(u32a1 *)o = enc_group(s2 | (s1 << 8) | (s3 << 16) | (s2 << 24), tab);
    }
    if (r - i == 1) {
        uint32_t q = enc_group((uint32_t)p[i] << 8, tab);
        *(u32a1 *)o = (q & 0xFFFFu) | (kPad << 16) | (kPad << 24);
    } else if (r - i == 2) {
        uint32_t s1 = p[i], s2 = p[i + 1];
        uint32_t q = enc_group(s2 | (s1 << 8) | (s2 << 24), tab);
        *(u32a1 *)o = (q & 0xFFFFFFu) | (kPad << 24);
    }
}

__device__ __forceinline__ void stage_enc_table(uint32_t *s_tab, const EncTab &tab)
{
    if (threadIdx.x < 16) s_tab[threadIdx.x] = tab.w[threadIdx.x];
    __syncthreads();
}

// Workgroups are dealt round-robin over the XCDs.  Renumber them so that
// consecutive logical blocks, which write adjacent output spans, run on the
// same XCD: a cache line shared by two spans is then completed in one L2
// instead of being written back in two partial halves from two L2s.
__device__ __forceinline__ int64_t logical_block()
{
    const int64_t G = gridDim.x, b = blockIdx.x;
    if (G % kXcds != 0) return b;
    return (b % kXcds) * (G / kXcds) + b / kXcds;
}

// Single buffer.  `head` whole groups are set aside so that the chunk outputs
// start on a 128-byte line (when dst is 4-byte aligned); then lane chunk c
// covers input [3*head + 12c, +12) and output [4*head + 16c, +16), grid-stride
// with U chunks in flight per lane.  Threads t < head encode one head group
// each; the last thread encodes the at most three whole groups and the
// partial group left after the chunks.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_encode(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, EncTab tab)
{
    __shared__ uint32_t s_tab[16];
    stage_enc_table(s_tab, tab);
    const uint8_t *a = (const uint8_t *)s_tab;

    const int64_t ng = n / 3;
    const uint64_t da = (uint64_t)(uintptr_t)dst;
    int64_t head = (da & 3) ? 0 : (int64_t)((((uint64_t)kLine - (da & (kLine - 1))) & (kLine - 1)) >> 2);
    if (head > ng) head = ng;
    const int64_t nch = (ng - head) >> 2;
    const uint8_t *s0 = src + 3 * head;
    uint8_t *d0 = dst + 4 * head;
    const int64_t T = (int64_t)gridDim.x * kThreads;
    const int64_t t = logical_block() * kThreads + threadIdx.x;
    for (int64_t c0 = t; c0 < nch; c0 += U * T) {
        u32x3 in[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t c = c0 + j * T;
            if (c < nch) in[j] = load12<NT>(s0 + 12 * c);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t c = c0 + j * T;
            if (c < nch) store16<NT>(d0 + 16 * c, enc_chunk(in[j], a));
        }
    }
    if (t < head) enc_scalar(src + 3 * t, 3, dst + 4 * t, a);
    if (t == kThreads - 1) {
        const int64_t g = head + 4 * nch;
        enc_scalar(src + 3 * g, n - 3 * g, dst + 4 * g, a);
    }
}

// ---------------------------------------------------------------- decode --

// Values of four characters (one quantum, little-endian in q) packed as
// a<<18 | b<<12 | c<<6 | d; their map entries are ORed into err.
__device__ __forceinline__ uint32_t dec_quantum(uint32_t q, const uint8_t *map, uint32_t &err)
{
    uint32_t m0 = map[q & 0xFF];
    uint32_t m1 = map[(q >> 8) & 0xFF];
    uint32_t m2 = map[(q >> 16) & 0xFF];
    uint32_t m3 = map[q >> 24];
    err |= m0 | m1 | m2 | m3;
    return (m0 << 18) | (m1 << 12) | (m2 << 6) | m3;
}

// 16 characters -> 12 bytes.  Quantum value v holds its three output bytes
// as v.b2 v.b1 v.b0; v_perm_b32 lays four quanta out as 12 consecutive bytes.
__device__ __forceinline__ u32x3 dec_chunk(u32x4 in, const uint8_t *map, uint32_t &err)
{
    uint32_t v0 = dec_quantum(in.x, map, err);
    uint32_t v1 = dec_quantum(in.y, map, err);
    uint32_t v2 = dec_quantum(in.z, map, err);
    uint32_t v3 = dec_quantum(in.w, map, err);
    u32x3 o;
    o.x = __builtin_amdgcn_perm(v1, v0, 0x06000102u);   // v0.b2 v0.b1 v0.b0 v1.b2
    o.y = __builtin_amdgcn_perm(v2, v1, 0x05060001u);   // v1.b1 v1.b0 v2.b2 v2.b1
    o.z = __builtin_amdgcn_perm(v3, v2, 0x04050600u);   // v2.b0 v3.b2 v3.b1 v3.b0
    return o;
}

enum { kData = 0, kPad1 = 1, kDone = 2 };

// Validate characters p[0..len) that start at a quantum boundary in the data
// state.  Returns the offset (relative to p) of the first character that
// cannot extend a valid encoding, or -1; *state gets the state after p[len-1]:
// kPad1 after a '=' at quantum position 2, kDone after the final '='.
// Rules: a non-alphabet character is invalid; '=' may stand only at quantum
// positions 2 and 3; before "==" the last value needs four zero low bits,
// before a single '=' two; nothing may follow the padded quantum.
__device__ int64_t dec_validate(const uint8_t *p, int64_t len, const uint8_t *map, int *state)
{
    int st = kData;
    for (int64_t i = 0; i < len; ++i) {
        const uint32_t c = p[i];
        const int pos = (int)(i & 3);
        if (st == kDone) return i;
        if (c != kPad) {
            if (map[c] == kBad || st == kPad1) return i;
            continue;
        }
        if (pos < 2) return i;
        if (pos == 2) {
            if (map[p[i - 1]] & 15) return i;
            st = kPad1;
        } else {
            if (st != kPad1 && (map[p[i - 1]] & 3)) return i;
            st = kDone;
        }
    }
    *state = st;
    return -1;
}

// First invalid offset (relative to p) inside a run of whole quanta that is
// known to be followed by at least one more character, or -1 if the run is
// clean.  A run ending with its padded quantum makes the next character the
// first invalid one.
__device__ __forceinline__ int64_t dec_check_inner(const uint8_t *p, int64_t len, const uint8_t *map)
{
    int st = kData;
    int64_t bad = dec_validate(p, len, map, &st);
    if (bad >= 0) return bad;
    return st == kDone ? len : -1;
}

// The last (up to 19) characters of a buffer: validate as the end of the
// input and, when valid, decode them.  Returns -1 and sets *out_len (the
// buffer's whole decoded length) when valid, else the first invalid offset
// relative to p.  `n_total` is the buffer length, p starts at a quantum
// boundary.
__device__ int64_t dec_tail(const uint8_t *p, int64_t len, int64_t n_total, uint8_t *o,
                            const uint8_t *map, int64_t *out_len)
{
    int st = kData;
    int64_t bad = dec_validate(p, len, map, &st);
    if (bad >= 0) return bad;
    if (st == kPad1 || ((n_total & 3) != 0 && st != kDone)) return len;
    int npad = 0;
    for (int64_t q = 0; q < len; q += 4) {
        const uint32_t a = map[p[q]], b = map[p[q + 1]];
        const bool pc = p[q + 2] == kPad, pd = p[q + 3] == kPad;
        const uint32_t c = pc ? 0u : map[p[q + 2]], d = pd ? 0u : map[p[q + 3]];
        const uint32_t v = (a << 18) | (b << 12) | (c << 6) | d;
        *o++ = (uint8_t)(v >> 16);
        if (!pc) *o++ = (uint8_t)(v >> 8);
        if (!pd) *o++ = (uint8_t)v;
        npad = (int)pc + (int)pd;
    }
    *out_len = 3 * (n_total >> 2) - npad;
    return -1;
}

__device__ __forceinline__ void stage_dec_map(uint32_t *s_map, const DecMap &map)
{
    if (threadIdx.x < 64) s_map[threadIdx.x] = map.w[threadIdx.x];
    __syncthreads();
}

__device__ __forceinline__ void atomic_min_i64(int64_t *p, int64_t v)
{
    atomicMin((unsigned long long *)p, (unsigned long long)v);
}

// Single buffer.  The body is every quantum but the last (nbq quanta).
// `head` body quanta are set aside so that the chunk outputs start on a
// 128-byte line (3*head = -dst mod 128; 43 is the inverse of 3 mod 128); then
// lane chunk c covers characters [4*head + 16c, +16) and bytes
// [3*head + 12c, +12).  Threads t < head decode one head quantum each; the
// last thread runs dec_tail over the (at most three) body quanta left after
// the chunks and the last quantum.  first_bad must hold kNoError before the
// launch; out_len is written only when the tail is valid.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_decode(const uint8_t *__restrict__ src, int64_t n,
                                                     uint8_t *__restrict__ dst, DecMap map,
                                                     int64_t *__restrict__ out_len,
                                                     int64_t *__restrict__ first_bad)
{
    __shared__ uint32_t s_map[64];
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;

    const int64_t nbq = n >= 1 ? (n - 1) >> 2 : 0;
    const uint64_t da = (uint64_t)(uintptr_t)dst;
    int64_t head = (int64_t)(((0 - da) * 43u) & (uint64_t)(kLine - 1));
    if (head > nbq) head = nbq;
    const int64_t nch = (nbq - head) >> 2;
    const uint8_t *s0 = src + 4 * head;
    uint8_t *d0 = dst + 3 * head;
    const int64_t T = (int64_t)gridDim.x * kThreads;
    const int64_t t = logical_block() * kThreads + threadIdx.x;
    uint32_t err = 0;
    for (int64_t c0 = t; c0 < nch; c0 += U * T) {
        u32x4 in[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t c = c0 + j * T;
            if (c < nch) in[j] = load16<NT>(s0 + 16 * c);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t c = c0 + j * T;
            if (c < nch) store12<NT>(d0 + 12 * c, dec_chunk(in[j], m, err));
        }
    }
    // One test per lane for its whole share (bit 7 is set only by kBad).
    if (__ballot(err & 0x80)) {
        if (err & 0x80) {
            for (int64_t c = t; c < nch; c += T) {
                const int64_t bad = dec_check_inner(s0 + 16 * c, 16, m);
                if (bad >= 0) {
                    atomic_min_i64(first_bad, 4 * head + 16 * c + bad);
                    break;   // later chunks of this lane have larger offsets
                }
            }
        }
    }
    if (t < head) {
        uint32_t qerr = 0;
        const uint32_t v = dec_quantum(*(const u32a1 *)(src + 4 * t), m, qerr);
        dst[3 * t] = (uint8_t)(v >> 16);
        dst[3 * t + 1] = (uint8_t)(v >> 8);
        dst[3 * t + 2] = (uint8_t)v;
        if (qerr & 0x80) {
            const int64_t bad = dec_check_inner(src + 4 * t, 4, m);
            if (bad >= 0) atomic_min_i64(first_bad, 4 * t + bad);
        }
    }
    if (t == kThreads - 1) {
        const int64_t q = head + 4 * nch;
        const int64_t bad = dec_tail(src + 4 * q, n - 4 * q, n, dst + 3 * q, m, out_len);
        if (bad >= 0) atomic_min_i64(first_bad, 4 * q + bad);
    }
}

__global__ void k_fill_i64(int64_t *p, int64_t count, int64_t value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

// After a decode: first_bad == kNoError becomes -1 (valid); otherwise the
// buffer is invalid and its out_len becomes -1.
__global__ void k_finish_status(int64_t *out_len, int64_t *first_bad, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        if (first_bad[i] == kNoError) first_bad[i] = -1;
        else out_len[i] = -1;
    }
}

// ----------------------------------------------------------------- batch --
//
// Buffers are packed back to back: buffer b is src[in_off[b] .. in_off[b+1]).
// The packed input [in_off[0], in_off[nbuf]) is cut into one contiguous span
// per wave (a multiple of 768 bytes); a wave processes the groups (encode) or
// quanta (decode) whose first byte lies in its span, buffer after buffer, with
// consecutive lanes on consecutive chunks.  No work queue and no atomics:
// balance comes from equal spans.  The wave that owns a buffer's first byte
// writes its out_len (encode); the wave that owns a buffer's last quantum runs
// the tail path (decode).

struct WaveSpan {
    int64_t lo, hi;   // owned packed-input byte range [lo, hi)
    int64_t b0;       // first buffer that may intersect it
    bool last;        // last wave: also owns empty buffers at the very end
};

__device__ WaveSpan wave_span(const int64_t *__restrict__ in_off, int64_t nbuf, int64_t quantum)
{
    WaveSpan s;
    const int64_t nwaves = (int64_t)gridDim.x * kWaves;
    // the wave index is uniform across the wave; say so, so that the span and
    // the per-buffer offsets live in scalar registers
    const int64_t w = logical_block() * kWaves +
                      __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t base = in_off[0], end = in_off[nbuf];
    const int64_t per = (end - base + nwaves - 1) / nwaves;
    const int64_t span = (per + quantum - 1) / quantum * quantum;
    s.last = (w == nwaves - 1);
    s.lo = base + w * span;
    if (s.lo > end) s.lo = end;
    s.hi = s.last ? end : (s.lo + span < end ? s.lo + span : end);
    // first b with in_off[b+1] >= lo (buffers ending before lo are not ours)
    int64_t l = 0, r = nbuf;
    while (l < r) {
        const int64_t mid = (l + r) >> 1;
        if (in_off[mid + 1] < s.lo) l = mid + 1;
        else r = mid;
    }
    s.b0 = l;
    return s;
}

template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_encode_batch(
    const uint8_t *__restrict__ src, const int64_t *__restrict__ in_off, int64_t nbuf,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off, int64_t *__restrict__ out_len,
    EncTab tab)
{
    __shared__ uint32_t s_tab[16];
    stage_enc_table(s_tab, tab);
    const uint8_t *a = (const uint8_t *)s_tab;
    const int lane = threadIdx.x & 63;
    const WaveSpan ws = wave_span(in_off, nbuf, 768);
    if (ws.lo >= ws.hi && !ws.last) return;

    for (int64_t b = ws.b0; b < nbuf; ++b) {
        const int64_t s = in_off[b], e = in_off[b + 1];
        if (s >= ws.hi && !(ws.last && s == ws.hi)) break;
        const int64_t len = e - s;
        const int64_t ngroups = (len + 2) / 3, nfull = len / 3;
        if (s >= ws.lo && lane == 0) out_len[b] = 4 * ngroups;
        // groups g whose first byte s + 3g lies in [lo, hi)
        const int64_t g_lo = s >= ws.lo ? 0 : (ws.lo - s + 2) / 3;
        int64_t g_hi = ws.hi <= s ? 0 : (ws.hi - s + 2) / 3;
        if (g_hi > ngroups) g_hi = ngroups;
        if (g_lo >= g_hi) continue;
        const int64_t g_full = g_hi < nfull ? g_hi : nfull;
        const int64_t nchunk = g_full > g_lo ? (g_full - g_lo) >> 2 : 0;
        const uint8_t *sp = src + s + 3 * g_lo;
        uint8_t *dp = dst + out_off[b] + 4 * g_lo;
        for (int64_t k0 = 0; k0 < nchunk; k0 += 64 * U) {
            u32x3 in[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t k = k0 + j * 64 + lane;
                if (k < nchunk) in[j] = load12<NT>(sp + 12 * k);
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t k = k0 + j * 64 + lane;
                if (k < nchunk) store16<NT>(dp + 16 * k, enc_chunk(in[j], a));
            }
        }
        // at most three whole groups and the buffer's partial last group
        const int64_t g = g_lo + 4 * nchunk + lane;
        if (lane < 4 && g < g_hi) {
            const int64_t rem = len - 3 * g;
            enc_scalar(src + s + 3 * g, rem < 3 ? rem : 3, dst + out_off[b] + 4 * g, a);
        }
    }
}

// Decode: the body of buffer b is its quanta but the last; chunks of four
// body quanta go to lanes, then lanes 0..3 take up to three leftover body
// quanta and the last quantum (lane 3 at most, via dec_tail).
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_decode_batch(
    const uint8_t *__restrict__ src, const int64_t *__restrict__ in_off, int64_t nbuf,
    uint8_t *__restrict__ dst, const int64_t *__restrict__ out_off, int64_t *__restrict__ out_len,
    int64_t *__restrict__ first_bad, DecMap map)
{
    __shared__ uint32_t s_map[64];
    stage_dec_map(s_map, map);
    const uint8_t *m = (const uint8_t *)s_map;
    const int lane = threadIdx.x & 63;
    const WaveSpan ws = wave_span(in_off, nbuf, 1024);
    if (ws.lo >= ws.hi && !ws.last) return;

    for (int64_t b = ws.b0; b < nbuf; ++b) {
        const int64_t s = in_off[b], e = in_off[b + 1];
        if (s >= ws.hi && !(ws.last && s == ws.hi)) break;
        const int64_t len = e - s;
        if (len == 0) {
            if (s >= ws.lo && lane == 0) out_len[b] = 0;
            continue;
        }
        const int64_t nq = (len + 3) >> 2;           // quanta, the last maybe partial
        const int64_t nbody = (len - 1) >> 2;        // all quanta but the last
        const int64_t q_lo = s >= ws.lo ? 0 : (ws.lo - s + 3) >> 2;
        int64_t q_hi = ws.hi <= s ? 0 : (ws.hi - s + 3) >> 2;
        if (q_hi > nq) q_hi = nq;
        if (q_lo >= q_hi) continue;
        const int64_t q_body = q_hi < nbody ? q_hi : nbody;
        const int64_t nchunk = q_body > q_lo ? (q_body - q_lo) >> 2 : 0;
        const uint8_t *sp = src + s + 4 * q_lo;
        uint8_t *dp = dst + out_off[b] + 3 * q_lo;
        uint32_t err = 0;
        for (int64_t k0 = 0; k0 < nchunk; k0 += 64 * U) {
            u32x4 in[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t k = k0 + j * 64 + lane;
                if (k < nchunk) in[j] = load16<NT>(sp + 16 * k);
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t k = k0 + j * 64 + lane;
                if (k < nchunk) store12<NT>(dp + 12 * k, dec_chunk(in[j], m, err));
            }
        }
        if (__ballot(err & 0x80)) {
            if (err & 0x80) {
                for (int64_t k = lane; k < nchunk; k += 64) {
                    const int64_t bad = dec_check_inner(sp + 16 * k, 16, m);
                    if (bad >= 0) {
                        atomic_min_i64(first_bad + b, 4 * q_lo + 16 * k + bad);
                        break;
                    }
                }
            }
        }
        const int64_t q = q_lo + 4 * nchunk + lane;
        if (lane < 4 && q < q_hi) {
            const uint8_t *qp = src + s + 4 * q;
            uint8_t *qo = dst + out_off[b] + 3 * q;
            if (q < nbody) {
                uint32_t qerr = 0;
                const uint32_t v = dec_quantum(*(const u32a1 *)qp, m, qerr);
                qo[0] = (uint8_t)(v >> 16);
                qo[1] = (uint8_t)(v >> 8);
                qo[2] = (uint8_t)v;
                if (qerr & 0x80) {
                    const int64_t bad = dec_check_inner(qp, 4, m);
                    if (bad >= 0) atomic_min_i64(first_bad + b, 4 * q + bad);
                }
            } else {
                int64_t ol = 0;
                const int64_t bad = dec_tail(qp, len - 4 * q, len, qo, m, &ol);
                if (bad >= 0) atomic_min_i64(first_bad + b, 4 * q + bad);
                else out_len[b] = ol;
            }
        }
    }
}

// ------------------------------------------------------------------ host --

thread_local char g_err[256];

int64_t fail(int64_t code, const char *fmt, const char *detail)
{
    snprintf(g_err, sizeof g_err, fmt, detail);
    return code;
}

int64_t hip_fail(hipError_t e, const char *where)
{
    snprintf(g_err, sizeof g_err, "%s: %s", where, hipGetErrorString(e));
    return B64_EHIP;
}

bool alphabet_ok(const char *alphabet)
{
    if (!alphabet) return false;
    bool seen[256] = {false};
    for (int v = 0; v < 64; ++v) {
        const uint8_t c = (uint8_t)alphabet[v];
        if (c == kPad || seen[c]) return false;
        seen[c] = true;
    }
    return true;
}

EncTab make_enc(const char *alphabet)
{
    EncTab t;
    memcpy(t.w, alphabet, 64);
    return t;
}

DecMap make_dec(const char *alphabet)
{
    DecMap d;
    uint8_t *b = (uint8_t *)d.w;
    memset(b, (int)kBad, 256);
    for (int v = 0; v < 64; ++v) b[(uint8_t)alphabet[v]] = (uint8_t)v;
    return d;
}

// Launch shapes per operation: {unroll, blocks per CU, nontemporal}; the
// defaults are the autotuner's choices on MI355X (1 GiB single buffers, 2 GiB
// log-uniform ragged batches).
struct Shape { int unroll, bpc, nt; };
Shape g_shape[4] = {{4, 2, 1}, {4, 2, 1}, {2, 4, 0}, {4, 32, 1}};
std::mutex g_mu;

constexpr int kMaxDevices = 64;
int g_cus[kMaxDevices];

hipError_t cu_count(int *cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_cus[dev] == 0) {
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        g_cus[dev] = v > 0 ? v : 1;
    }
    *cus = g_cus[dev];
    return hipSuccess;
}

Shape shape_of(int op)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_shape[op];
}

// Blocks for a grid-stride launch over `nch` lane chunks.
int64_t grid_for(int64_t nch, Shape sh, int cus)
{
    const int64_t per_block = (int64_t)kThreads * sh.unroll;
    int64_t need = (nch + per_block - 1) / per_block;
    const int64_t cap = (int64_t)cus * sh.bpc;
    if (need > cap) need = cap;
    if (need >= kXcds) need -= need % kXcds;   // a whole number of blocks per XCD
    return need < 1 ? 1 : need;
}

#define B64_LAUNCH(KERNEL, U_, NT_, GRID, STREAM, ...) \
    hipLaunchKernelGGL((KERNEL<U_, NT_>), dim3(GRID), dim3(kThreads), 0, STREAM, __VA_ARGS__)
#define B64_DISPATCH_NT(KERNEL, U_, SH, GRID, STREAM, ...)                 \
    do {                                                                  \
        if ((SH).nt) B64_LAUNCH(KERNEL, U_, true, GRID, STREAM, __VA_ARGS__);  \
        else B64_LAUNCH(KERNEL, U_, false, GRID, STREAM, __VA_ARGS__);         \
    } while (0)
// Instantiates KERNEL for every (unroll, nontemporal) shape and launches the
// one `SH` selects.
#define B64_DISPATCH(KERNEL, SH, GRID, STREAM, ...)                                  \
    do {                                                                            \
        switch ((SH).unroll) {                                                      \
        case 1: B64_DISPATCH_NT(KERNEL, 1, SH, GRID, STREAM, __VA_ARGS__); break;   \
        case 2: B64_DISPATCH_NT(KERNEL, 2, SH, GRID, STREAM, __VA_ARGS__); break;   \
        case 8: B64_DISPATCH_NT(KERNEL, 8, SH, GRID, STREAM, __VA_ARGS__); break;   \
        default: B64_DISPATCH_NT(KERNEL, 4, SH, GRID, STREAM, __VA_ARGS__); break;  \
        }                                                                           \
    } while (0)

int64_t launch_fill(int64_t *p, int64_t count, int64_t value, hipStream_t stream)
{
    const int64_t blocks = (count + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_fill_i64, dim3(blocks), dim3(kThreads), 0, stream, p, count, value);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : hip_fail(e, "fill launch");
}

int64_t launch_finish(int64_t *out_len, int64_t *first_bad, int64_t count, hipStream_t stream)
{
    const int64_t blocks = (count + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_finish_status, dim3(blocks), dim3(kThreads), 0, stream, out_len, first_bad,
                       count);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : hip_fail(e, "status launch");
}

// Per thread and device: 2 int64 of device memory and of pinned host memory
// for the blocking b64_decode (held until the process ends).
struct StatusSlot { int dev = -1; int64_t *d = nullptr; int64_t *h = nullptr; };
thread_local StatusSlot g_slot[kMaxDevices];

hipError_t status_slot(StatusSlot **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    StatusSlot &s = g_slot[dev];
    if (!s.d) {
        e = hipMalloc((void **)&s.d, 2 * sizeof(int64_t));
        if (e != hipSuccess) return e;
        e = hipHostMalloc((void **)&s.h, 2 * sizeof(int64_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            (void)hipFree(s.d);
            s.d = nullptr;
            return e;
        }
        s.dev = dev;
    }
    *out = &s;
    return hipSuccess;
}

// Enqueue one single-buffer decode: reset first_bad, run k_decode, and (with
// `finish`) turn the raw status into the public form.
int64_t decode_launch(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *out_len,
                      int64_t *first_bad, const char *alphabet, hipStream_t stream, bool finish)
{
    if (n < 0) return fail(B64_EARG, "negative length%s", "");
    if (!alphabet_ok(alphabet))
        return fail(B64_EARG, "alphabet must be 64 distinct bytes without '='%s", "");
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    int64_t r = launch_fill(first_bad, 1, kNoError, stream);
    if (r) return r;
    const Shape sh = shape_of(1);
    const int64_t nbq = n >= 1 ? (n - 1) >> 2 : 0;
    const int64_t grid = grid_for(nbq >> 2, sh, cus);
    B64_DISPATCH(k_decode, sh, grid, stream, src, n, dst, make_dec(alphabet), out_len, first_bad);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return finish ? launch_finish(out_len, first_bad, 1, stream) : 0;
}

}  // namespace

extern "C" {

int64_t b64_encoded_len(int64_t n)
{
    if (n < 0) return fail(B64_EARG, "negative length%s", "");
    return 4 * ((n + 2) / 3);
}

int64_t b64_decoded_max_len(int64_t n)
{
    if (n < 0) return fail(B64_EARG, "negative length%s", "");
    return 3 * (n / 4);
}

const char *b64_last_error(void) { return g_err; }

int64_t b64_tune_set(int op, int unroll, int blocks_per_cu, int nontemporal)
{
    if (op < 0 || op > 3) return fail(B64_EARG, "bad op%s", "");
    if (!(unroll == 1 || unroll == 2 || unroll == 4 || unroll == 8))
        return fail(B64_EARG, "unroll must be 1, 2, 4 or 8%s", "");
    if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(B64_EARG, "blocks_per_cu out of range%s", "");
    if (nontemporal != 0 && nontemporal != 1) return fail(B64_EARG, "nontemporal must be 0 or 1%s", "");
    std::lock_guard<std::mutex> lk(g_mu);
    g_shape[op] = Shape{unroll, blocks_per_cu, nontemporal};
    return 0;
}

int64_t b64_tune_get(int op)
{
    if (op < 0 || op > 3) return fail(B64_EARG, "bad op%s", "");
    Shape s = shape_of(op);
    return (int64_t)s.nt * 10000 + (int64_t)s.unroll * 100 + s.bpc;
}

int64_t b64_encode(const uint8_t *src, int64_t n, uint8_t *dst, const char *alphabet,
                   hipStream_t stream)
{
    if (n < 0) return fail(B64_EARG, "negative length%s", "");
    if (n > 0 && (!src || !dst)) return fail(B64_EARG, "null buffer%s", "");
    if (!alphabet_ok(alphabet))
        return fail(B64_EARG, "alphabet must be 64 distinct bytes without '='%s", "");
    if (n == 0) return 0;
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    const Shape sh = shape_of(0);
    const int64_t grid = grid_for(n / 12, sh, cus);
    B64_DISPATCH(k_encode, sh, grid, stream, src, n, dst, make_enc(alphabet));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "encode launch");
    return 4 * ((n + 2) / 3);
}

int64_t b64_decode_async(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *out_len,
                         int64_t *first_bad, const char *alphabet, hipStream_t stream)
{
    if ((n > 0 && (!src || !dst)) || !out_len || !first_bad)
        return fail(B64_EARG, "null pointer%s", "");
    return decode_launch(src, n, dst, out_len, first_bad, alphabet, stream, true);
}

int64_t b64_decode(const uint8_t *src, int64_t n, uint8_t *dst, const char *alphabet,
                   hipStream_t stream)
{
    StatusSlot *slot = nullptr;
    if (n > 0 && (!src || !dst)) return fail(B64_EARG, "null buffer%s", "");
    if (n < 0) return fail(B64_EARG, "negative length%s", "");
    if (!alphabet_ok(alphabet))
        return fail(B64_EARG, "alphabet must be 64 distinct bytes without '='%s", "");
    hipError_t e = status_slot(&slot);
    if (e != hipSuccess) return hip_fail(e, "status slot");
    // raw status: slot->d[0] = length if the tail is valid, slot->d[1] = the
    // smallest invalid offset or kNoError; read back and combined here.
    int64_t r = decode_launch(src, n, dst, slot->d, slot->d + 1, alphabet, stream, false);
    if (r) return r;
    e = hipMemcpyAsync(slot->h, slot->d, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, stream);
    if (e != hipSuccess) return hip_fail(e, "status copy");
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    const int64_t len = slot->h[0], bad = slot->h[1];
    return bad == kNoError ? len : ~bad;
}

int64_t b64_encode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf, uint8_t *dst,
                         const int64_t *out_off, int64_t *out_len, const char *alphabet,
                         hipStream_t stream)
{
    if (nbuf < 0) return fail(B64_EARG, "negative buffer count%s", "");
    if (nbuf == 0) return 0;
    if (!src || !in_off || !dst || !out_off || !out_len) return fail(B64_EARG, "null pointer%s", "");
    if (!alphabet_ok(alphabet))
        return fail(B64_EARG, "alphabet must be 64 distinct bytes without '='%s", "");
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    const Shape sh = shape_of(2);
    const int64_t grid = (int64_t)cus * sh.bpc;
    B64_DISPATCH(k_encode_batch, sh, grid, stream, src, in_off, nbuf, dst, out_off, out_len,
                   make_enc(alphabet));
    e = hipGetLastError();
    return e == hipSuccess ? 0 : hip_fail(e, "encode_batch launch");
}

int64_t b64_decode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf, uint8_t *dst,
                         const int64_t *out_off, int64_t *out_len, int64_t *first_bad,
                         const char *alphabet, hipStream_t stream)
{
    if (nbuf < 0) return fail(B64_EARG, "negative buffer count%s", "");
    if (nbuf == 0) return 0;
    if (!src || !in_off || !dst || !out_off || !out_len || !first_bad)
        return fail(B64_EARG, "null pointer%s", "");
    if (!alphabet_ok(alphabet))
        return fail(B64_EARG, "alphabet must be 64 distinct bytes without '='%s", "");
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    int64_t r = launch_fill(first_bad, nbuf, kNoError, stream);
    if (r) return r;
    const Shape sh = shape_of(3);
    const int64_t grid = (int64_t)cus * sh.bpc;
    B64_DISPATCH(k_decode_batch, sh, grid, stream, src, in_off, nbuf, dst, out_off, out_len,
                   first_bad, make_dec(alphabet));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "decode_batch launch");
    return launch_finish(out_len, first_bad, nbuf, stream);
}

}  // extern "C"
