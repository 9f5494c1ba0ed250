// b64_device.h -- device-side building blocks of the base64 kernels (gfx950).
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
// into a per-lane error word that is tested once, after the lane's share of
// the input (the paper's deferred vpternlogd/vpmovb2m check); a wave-wide
// ballot skips the slow path when every lane is clean.  A lane that saw an
// invalid character (or a '=') rescans its chunks to find the first invalid
// offset and publishes it with an atomic minimum.  Four 6-bit values are
// packed as a<<18 | b<<12 | c<<6 | d (the paper's two multiply-adds) and the
// three bytes of four quanta are packed into three dwords by v_perm_b32 (the
// paper's final vpermb).  The last quanta, with the '=' rules, go through a
// separate single-lane path (the paper's "conventional code path"),
// dec_tail_fast, which loads them all at once and checks them on registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace b64hip {

constexpr int kThreads = 256;          // 4 waves of 64 lanes per workgroup
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kPad = '=';
constexpr uint32_t kBad = 0xFF;        // decode-map value of a non-alphabet byte
constexpr int64_t kNoError = INT64_MAX;
constexpr int kXcds = 8;               // MI355X: 8 accelerator dies, each with its own L2
constexpr int kLine = 128;             // L2 cache line, bytes

// Variant flags (the values of B64_NOPAD and B64_SKIP_WS in b64hip.h).
constexpr uint32_t kFlagNoPad = 1;     // no '=': final quantum of 2 or 3 characters
constexpr uint32_t kFlagSkipWs = 2;    // decode ignores space, tab, CR and LF

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
// bytes zero-filled and either padded with '=' (Section "Base64") or, when
// `pad` is false, cut to the 2 or 3 characters that carry input bits.
__device__ inline void enc_scalar(const uint8_t *p, int64_t r, uint8_t *o, const uint8_t *tab,
                                  bool pad = true)
{
    int64_t i = 0;
    for (; i + 3 <= r; i += 3, o += 4) {
        uint32_t s1 = p[i], s2 = p[i + 1], s3 = p[i + 2];
        *(u32a1 *)o = enc_group(s2 | (s1 << 8) | (s3 << 16) | (s2 << 24), tab);
    }
    const int64_t k = r - i;
    if (k == 0) return;
    uint32_t q = k == 1 ? enc_group((uint32_t)p[i] << 8, tab)
                        : enc_group(p[i + 1] | ((uint32_t)p[i] << 8) | ((uint32_t)p[i + 1] << 24), tab);
    if (pad) {
        q = k == 1 ? (q & 0xFFFFu) | (kPad << 16) | (kPad << 24) : (q & 0xFFFFFFu) | (kPad << 24);
        *(u32a1 *)o = q;
    } else {
        o[0] = (uint8_t)q;
        o[1] = (uint8_t)(q >> 8);
        if (k == 2) o[2] = (uint8_t)(q >> 16);
    }
}

// The r <= 11 bytes left after an encode's chunks (at most three whole groups
// and a partial group), or one head group (r = 3), fetched early and encoded
// later: a kernel issues the loads before it stages its table and encodes
// from registers afterwards.  The loads are whole dwords of a 12-byte window
// of the input that holds the bytes (starting at them, or else ending where
// they end) and nothing is extracted from them here, so no instruction waits
// for a load; inputs too short for either window load bytes.
struct EncTailIn {
    uint32_t w[3];
    int off;          // window offset of the first byte
};

// p = input + before, in an input of n bytes.
__device__ __forceinline__ EncTailIn enc_tail_load(const uint8_t *p, int r, int64_t before,
                                                   int64_t n)
{
    EncTailIn ti = {{0u, 0u, 0u}, 0};
    if (r <= 0) return ti;
    if (before + 12 <= n) {                 // the window [p, p + 12)
        ti.w[0] = *(const u32a1 *)p;
        ti.w[1] = *(const u32a1 *)(p + 4);
        ti.w[2] = *(const u32a1 *)(p + 8);
    } else if (before + r >= 12) {          // the window [p + r - 12, p + r)
        const uint8_t *wp = p + r - 12;
        ti.w[0] = *(const u32a1 *)wp;
        ti.w[1] = *(const u32a1 *)(wp + 4);
        ti.w[2] = *(const u32a1 *)(wp + 8);
        ti.off = 12 - r;
    } else {
#pragma unroll
        for (int i = 0; i < 11; ++i)
            if (i < r) ti.w[i >> 2] |= (uint32_t)p[i] << (8 * (i & 3));
    }
    return ti;
}

// enc_scalar on bytes fetched by enc_tail_load (r <= 11).
__device__ __forceinline__ void enc_tail_regs(const EncTailIn &ti, int r, uint8_t *o,
                                              const uint8_t *tab, bool pad = true)
{
    // shift the window right by off bytes: t0..t2 hold the r bytes in order
    const int q = ti.off >> 2;
    const uint32_t k = (uint32_t)(ti.off & 3);
    const uint32_t x0 = __builtin_amdgcn_alignbyte(ti.w[1], ti.w[0], k);
    const uint32_t x1 = __builtin_amdgcn_alignbyte(ti.w[2], ti.w[1], k);
    const uint32_t x2 = __builtin_amdgcn_alignbyte(0u, ti.w[2], k);
    const uint32_t t0 = q == 0 ? x0 : q == 1 ? x1 : q == 2 ? x2 : 0u;
    const uint32_t t1 = q == 0 ? x1 : q == 1 ? x2 : 0u;
    const uint32_t t2 = q == 0 ? x2 : 0u;
    const uint32_t t[3] = {t0, t1, t2};
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int i = 3 * g;
        const uint32_t s1 = (t[i >> 2] >> (8 * (i & 3))) & 0xFF;
        const uint32_t s2 = i + 1 < 12 ? (t[(i + 1) >> 2] >> (8 * ((i + 1) & 3))) & 0xFF : 0u;
        const uint32_t s3 = i + 2 < 12 ? (t[(i + 2) >> 2] >> (8 * ((i + 2) & 3))) & 0xFF : 0u;
        if (i + 3 <= r) {
            *(u32a1 *)(o + 4 * g) = enc_group(s2 | (s1 << 8) | (s3 << 16) | (s2 << 24), tab);
        } else if (i < r) {
            const int kk = r - i;
            uint32_t v = kk == 1 ? enc_group(s1 << 8, tab) : enc_group(s2 | (s1 << 8) | (s2 << 24), tab);
            if (pad) {
                v = kk == 1 ? (v & 0xFFFFu) | (kPad << 16) | (kPad << 24) : (v & 0xFFFFFFu) | (kPad << 24);
                *(u32a1 *)(o + 4 * g) = v;
            } else {
                o[4 * g] = (uint8_t)v;
                o[4 * g + 1] = (uint8_t)(v >> 8);
                if (kk == 2) o[4 * g + 2] = (uint8_t)(v >> 16);
            }
        }
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

// Complete rounds of `rstep` lane chunks in `nch` chunks.  Both fit 32 bits
// for every input below 64 GiB, and a 32-bit quotient is a short instruction
// sequence where a 64-bit one is over a hundred scalar instructions.
__device__ __forceinline__ int64_t full_rounds(int64_t nch, int64_t rstep)
{
    if ((uint64_t)nch <= 0xFFFFFFFFull && (uint64_t)rstep <= 0xFFFFFFFFull)
        return (int64_t)((uint32_t)nch / (uint32_t)rstep);
    return nch / rstep;
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
// before a single '=' two; nothing may follow the padded quantum.  With
// `nopad`, '=' is an ordinary non-alphabet character.
__device__ inline int64_t dec_validate(const uint8_t *p, int64_t len, const uint8_t *map, int *state,
                                       bool nopad = false)
{
    int st = kData;
    for (int64_t i = 0; i < len; ++i) {
        const uint32_t c = p[i];
        const int pos = (int)(i & 3);
        if (st == kDone) return i;
        if (c != kPad || nopad) {
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
__device__ __forceinline__ int64_t dec_check_inner(const uint8_t *p, int64_t len, const uint8_t *map,
                                                   bool nopad = false)
{
    int st = kData;
    int64_t bad = dec_validate(p, len, map, &st, nopad);
    if (bad >= 0) return bad;
    return st == kDone ? len : -1;
}

// The final quantum of an input: its r (1..4) characters in bytes 0..r-1 of
// c.  The rules of dec_validate, and the end-of-input rules (padded: the
// input ends in the data state with a length that is a multiple of four, or
// right after the padded quantum; unpadded: a last quantum of 2 or 3
// characters with zero trailing bits, or of 4), for one quantum, unrolled on
// registers.  Returns -1 for a valid end (*nd = its data characters, *val =
// their values packed as a<<18 | b<<12 | c<<6 | d, absent ones 0), else the
// offset in the quantum of the first invalid character, r when the input ends
// too early.
__device__ __forceinline__ int final_quantum(uint32_t c, int r, const uint8_t *map, bool nopad,
                                             int *nd, uint32_t *val)
{
    int st = kData, ndata = 0;
    uint32_t v = 0, prev = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < r) {
            const uint32_t ch = (c >> (8 * i)) & 0xFF;
            if (st == kDone) return i;
            if (ch != kPad || nopad) {
                const uint32_t x = map[ch];
                if (x == kBad || st == kPad1) return i;
                v |= x << (18 - 6 * i);
                prev = x;
                ++ndata;
            } else if (i < 2) {
                return i;
            } else if (i == 2) {
                if (prev & 15) return i;
                st = kPad1;
            } else {
                if (st != kPad1 && (prev & 3)) return i;
                st = kDone;
            }
        }
    }
    if (nopad) {
        if (r == 1) return r;
        if (r < 4 && (prev & (r == 2 ? 15u : 3u))) return r;
    } else if (r != 4 || st == kPad1) {
        return r;
    }
    *nd = ndata;
    *val = v;
    return -1;
}

// The last characters of an input, p[0..len) from a quantum boundary to the
// end (len <= 16: up to three body quanta and the final quantum), loaded into
// registers: the body quanta in q[0..nb) and the final quantum's r
// characters in bytes 0..r-1 of fq.  Every load is issued at once, so the
// tail costs one memory round trip; a kernel may issue them early and use
// them later.
struct TailIn {
    uint32_t q[3];
    uint32_t fq;
};

// Every value is kept as loaded (the shift that aligns the final quantum is
// applied by dec_tail_regs), so no instruction here waits for a load.
__device__ __forceinline__ TailIn tail_load(const uint8_t *p, int64_t len)
{
    TailIn ti = {{0u, 0u, 0u}, 0u};
    if (len <= 0) return ti;
    if (len >= 4) {
        const int nb = (int)((len - 1) >> 2);              // body quanta, 0..3
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (i < nb) ti.q[i] = *(const u32a1 *)(p + 4 * i);
        ti.fq = *(const u32a1 *)(p + len - 4);             // the last four characters
    } else {
        // no body quantum: q[i] holds character i of the final quantum
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (i < len) ti.q[i] = p[i];
    }
    return ti;
}

// The tail p[0..len) of an input of n_total characters, loaded by tail_load,
// validated as the end of the input and, when valid, decoded to o (o ==
// nullptr: validate only); the rules run on registers.  Returns -1 and sets
// *out_len (the whole input's decoded length) when valid, else the first
// invalid offset relative to p.
__device__ inline int64_t dec_tail_regs(const TailIn &ti, const uint8_t *p, int64_t len,
                                        int64_t n_total, uint8_t *o, const uint8_t *map,
                                        int64_t *out_len, bool nopad)
{
    if (len <= 0) {
        *out_len = 0;
        return -1;
    }
    const int nb = (int)((len - 1) >> 2);
    const int r = (int)(len - 4 * nb);
    uint32_t v[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (i < nb) {
            uint32_t qerr = 0;
            v[i] = dec_quantum(ti.q[i], map, qerr);
            if (qerr & 0x80) {
                const int64_t bad = dec_check_inner(p + 4 * i, 4, map, nopad);
                if (bad >= 0) return 4 * i + bad;
            }
        }
    }
    int nd = 0;
    uint32_t fv = 0;
    // the final quantum's r characters in bytes 0..r-1
    const uint32_t fq = len >= 4 ? ti.fq >> (8 * (4 - r)) : ti.q[0] | (ti.q[1] << 8) | (ti.q[2] << 16);
    const int fbad = final_quantum(fq, r, map, nopad, &nd, &fv);
    if (fbad >= 0) return 4 * nb + fbad;
    if (o) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (i < nb) {
                o[3 * i] = (uint8_t)(v[i] >> 16);
                o[3 * i + 1] = (uint8_t)(v[i] >> 8);
                o[3 * i + 2] = (uint8_t)v[i];
            }
        }
        uint8_t *of = o + 3 * nb;
        if (nd >= 2) of[0] = (uint8_t)(fv >> 16);
        if (nd >= 3) of[1] = (uint8_t)(fv >> 8);
        if (nd >= 4) of[2] = (uint8_t)fv;
    }
    *out_len = 3 * ((n_total - r) >> 2) + nd - 1;
    return -1;
}

// tail_load and dec_tail_regs in one step.
__device__ inline int64_t dec_tail_fast(const uint8_t *p, int64_t len, int64_t n_total, uint8_t *o,
                                        const uint8_t *map, int64_t *out_len, bool nopad)
{
    return dec_tail_regs(tail_load(p, len), p, len, n_total, o, map, out_len, nopad);
}

__device__ __forceinline__ void stage_dec_map(uint32_t *s_map, const DecMap &map)
{
    if (threadIdx.x < 64) s_map[threadIdx.x] = map.w[threadIdx.x];
    __syncthreads();
}

// The same map built in LDS from the alphabet (a 64-byte kernel argument in
// place of the 256-byte map): every entry kBad, then entry alphabet[v] = v;
// the host has checked that the 64 bytes are distinct.  The first barrier
// passes while the caller's earlier loads are still in flight; only the
// scatter and the second barrier wait for them.
__device__ __forceinline__ void stage_dec_map_alpha(uint32_t *s_map, const EncTab &alpha)
{
    uint32_t w = 0;
    if (threadIdx.x < 64) {
        s_map[threadIdx.x] = kBad * 0x01010101u;
        w = alpha.w[threadIdx.x >> 2];
    }
    __syncthreads();
    if (threadIdx.x < 64)
        ((uint8_t *)s_map)[(w >> (8 * (threadIdx.x & 3))) & 0xFF] = (uint8_t)threadIdx.x;
    __syncthreads();
}

__device__ __forceinline__ void atomic_min_i64(int64_t *p, int64_t v)
{
    atomicMin((unsigned long long *)p, (unsigned long long)v);
}

// Keeps `v` alive in a register: the wave waits here until an atomic's
// returned value has arrived, i.e. until the atomic has been performed.
__device__ __forceinline__ void consume(int64_t v) { asm volatile("" ::"v"(v)); }

// Where a single-buffer decode or validation leaves its result.
//
// Raw form (slot == nullptr): *first_bad holds kNoError before the launch and
// receives the smallest invalid offset by atomic minimum; *out_len receives
// the decoded length when the end of the input is valid.  Two more launches
// (reset before, k_finish_status after) give the public form.
//
// Slot form: slot points at kSlotWords int64 words of library memory that are
// zero between calls, and the kernel itself leaves the public form in
// *out_len / *first_bad (the length and -1 for a valid input, -1 and the first
// invalid offset otherwise).  slot[0] collects kNoError - offset of every
// invalid character found, by atomic maximum (the largest key is the smallest
// offset).  Every workgroup, when done, makes one atomic add of a count word:
// finished workgroups in bits 32..63, workgroups that found an invalid
// character in bits 0..23, and the number of data characters of the valid
// final quantum in bits 24..31 (from the workgroup of the tail lane; with the
// input length it gives the decoded length).  Atomics on one word are
// performed one at a time, about 10 ns each on MI355X, so a grid of more than
// 8 * kSinkGroups workgroups counts in two levels: workgroup b adds to the
// word of group b mod kSinkGroups (each on its own 128-byte line), and the
// last workgroup of each group adds the group's sum to the total at slot[1];
// smaller grids add to slot[1] directly.  The workgroup whose add completes
// the total writes the public form; only when some workgroup found an invalid
// character does it read slot[0] (one more atomic).  Each completing
// workgroup puts the word it completed back to zero, and the reader of
// slot[0] clears it.  Every report to slot[0] is an atomic whose returned
// value the lane waits for, so it has been performed before the lane reaches
// the workgroup's final barrier, and the workgroup's add is issued after that
// barrier; each add that completes a count is issued after the adds it
// counts were performed, so the last one sees every report.  Only atomics at
// device scope touch the slot, so no cache writeback is needed.  A grid of one
// workgroup skips the count.  Calls that may run at the same time must use
// different slots.
constexpr int kSinkGroups = 32;
constexpr int kSlotWords = 16 * (kSinkGroups + 1);   // line 0: key, total; then one line per group
struct DecSink {
    int64_t *out_len, *first_bad, *slot;
};

// Per-lane record of what the lane reported in the slot form.
struct SinkLane {
    int bad = 0;   // reported an invalid offset
    int nd = 0;    // tail lane with a valid end: data characters of the final quantum
};

__device__ __forceinline__ void sink_bad(const DecSink &s, SinkLane &l, int64_t off)
{
    if (s.slot) {
        consume(__hip_atomic_fetch_max(s.slot, kNoError - off, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT));
        l.bad = 1;
    } else {
        atomic_min_i64(s.first_bad, off);
    }
}

// Length of a valid input of n >= 1 characters whose final quantum (the
// last ((n - 1) mod 4) + 1 characters) holds nd data characters.
__device__ __forceinline__ int64_t sink_length(int64_t n, int nd)
{
    const int64_t r = ((n - 1) & 3) + 1;
    return 3 * ((n - r) >> 2) + nd - 1;
}

// The tail lane's valid end: decoded length len of the whole input of n
// characters.
__device__ __forceinline__ void sink_len(const DecSink &s, SinkLane &l, int64_t len, int64_t n)
{
    if (s.slot)
        l.nd = n > 0 ? (int)(len - sink_length(n, 1) + 1) : 1;
    else
        *s.out_len = len;
}

// Called by every thread of every workgroup after its last report; `tail` is
// whether this workgroup holds the tail lane (thread kThreads - 1).
__device__ __forceinline__ void sink_finish(const DecSink &s, const SinkLane &l, bool tail,
                                            int64_t n)
{
    if (!s.slot) return;
    // Whether any lane of the workgroup reported: a ballot per wave, one LDS
    // word per wave, one barrier.  (__syncthreads_or reads the workgroup size
    // from the dispatch packet and then waits for every memory operation the
    // wave has issued, the output stores included: a full store round trip
    // before the count.)
    __shared__ uint32_t s_bad[kWaves];
    const uint32_t wave_bad = __ballot(l.bad) != 0 ? 1u : 0u;
    if ((threadIdx.x & 63) == 0) s_bad[threadIdx.x >> 6] = wave_bad;
    __syncthreads();
    if ((int)threadIdx.x != (tail ? kThreads - 1 : 0)) return;
    uint32_t any_bad = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) any_bad |= s_bad[w];
    constexpr int64_t kOne = (int64_t)1 << 32;
    int64_t v = kOne | ((int64_t)l.nd << 24) | (any_bad ? 1 : 0);
    const int64_t G = gridDim.x;
    if (G > 1) {
        int64_t expect = G;
        if (G > 8 * kSinkGroups) {
            const int g = (int)(blockIdx.x % kSinkGroups);
            int64_t *cnt = s.slot + 16 * (g + 1);
            const int64_t members = (G - 1 - g) / kSinkGroups + 1;
            const int64_t old =
                __hip_atomic_fetch_add(cnt, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((old >> 32) + 1 != members) return;
            __hip_atomic_store(cnt, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            v = kOne | ((old + v) & 0xFFFFFFFF);        // the group counts as one
            expect = kSinkGroups;
        }
        const int64_t old =
            __hip_atomic_fetch_add(s.slot + 1, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((old >> 32) + 1 != expect) return;
        v += old;
        __hip_atomic_store(s.slot + 1, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if ((v & 0xFFFFFF) == 0) {
        *s.first_bad = -1;
        *s.out_len = n > 0 ? sink_length(n, (int)((v >> 24) & 0xFF)) : 0;
    } else {
        const int64_t key =
            __hip_atomic_exchange(s.slot, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s.first_bad = kNoError - key;
        *s.out_len = -1;
    }
}

// `nrounds` complete rounds of lane chunks: round r holds chunks
// c0 + r*rstep + j*stride, j < U, all in range.  Software-pipelined: the loads
// of round r+1 are issued before round r is computed and stored.  On gfx9 the
// vector-memory counter covers loads and stores alike, so waiting for a load
// also waits for every store issued before it; issuing the next loads first
// keeps them ahead of the stores, and no load ever waits for a store.  The
// straight-line rounds (no per-chunk guards) let the compiler wait for each
// chunk's own load only.
template <int U, bool NT>
__device__ __forceinline__ void enc_load(u32x3 (&v)[U], const uint8_t *s0, int64_t c, int64_t stride)
{
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = load12<NT>(s0 + 12 * (c + j * stride));
}
template <int U, bool NT>
__device__ __forceinline__ void enc_store(const u32x3 (&v)[U], uint8_t *d0, int64_t c, int64_t stride,
                                          const uint8_t *tab)
{
#pragma unroll
    for (int j = 0; j < U; ++j) store16<NT>(d0 + 16 * (c + j * stride), enc_chunk(v[j], tab));
}

template <int U, bool NT>
__device__ __forceinline__ void enc_stream(const uint8_t *s0, uint8_t *d0, int64_t c0, int64_t stride,
                                           int64_t rstep, int64_t nrounds, const uint8_t *tab)
{
    if (nrounds <= 0) return;
    u32x3 A[U], B[U];                 // rounds alternate between two register sets
    enc_load<U, NT>(A, s0, c0, stride);
    int64_t r = 0;
    for (; r + 2 < nrounds; r += 2) {
        enc_load<U, NT>(B, s0, c0 + rstep, stride);
        enc_store<U, NT>(A, d0, c0, stride, tab);
        enc_load<U, NT>(A, s0, c0 + 2 * rstep, stride);
        enc_store<U, NT>(B, d0, c0 + rstep, stride, tab);
        c0 += 2 * rstep;
    }
    if (r + 1 < nrounds) {
        enc_load<U, NT>(B, s0, c0 + rstep, stride);
        enc_store<U, NT>(A, d0, c0, stride, tab);
        enc_store<U, NT>(B, d0, c0 + rstep, stride, tab);
    } else {
        enc_store<U, NT>(A, d0, c0, stride, tab);
    }
}

// The last, partial round: only chunks below nch are stored.  Lanes past the
// end load the round's last in-range chunk again instead of skipping the load,
// so the loads stay outside any branch and the compiler waits for each load
// alone rather than for every earlier store.
template <int U, bool NT>
__device__ __forceinline__ void enc_round_load(u32x3 (&in)[U], const uint8_t *s0, int64_t c0,
                                               int64_t stride, int64_t nch)
{
    if (nch <= 0) return;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int64_t c = c0 + j * stride;
        in[j] = load12<NT>(s0 + 12 * (c < nch ? c : nch - 1));
    }
}
template <int U, bool NT>
__device__ __forceinline__ void enc_round_store(const u32x3 (&in)[U], uint8_t *d0, int64_t c0,
                                                int64_t stride, const uint8_t *tab, int64_t nch)
{
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int64_t c = c0 + j * stride;
        if (c < nch) store16<NT>(d0 + 16 * c, enc_chunk(in[j], tab));
    }
}
template <int U, bool NT>
__device__ __forceinline__ void enc_round_tail(const uint8_t *s0, uint8_t *d0, int64_t c0,
                                               int64_t stride, const uint8_t *tab, int64_t nch)
{
    u32x3 in[U];
    enc_round_load<U, NT>(in, s0, c0, stride, nch);
    enc_round_store<U, NT>(in, d0, c0, stride, tab, nch);
}

template <int U, bool NT>
__device__ __forceinline__ void dec_load(u32x4 (&v)[U], const uint8_t *s0, int64_t c, int64_t stride)
{
#pragma unroll
    for (int j = 0; j < U; ++j) v[j] = load16<NT>(s0 + 16 * (c + j * stride));
}
template <int U, bool NT>
__device__ __forceinline__ void dec_store(const u32x4 (&v)[U], uint8_t *d0, int64_t c, int64_t stride,
                                          const uint8_t *map, uint32_t &err)
{
#pragma unroll
    for (int j = 0; j < U; ++j) store12<NT>(d0 + 12 * (c + j * stride), dec_chunk(v[j], map, err));
}

template <int U, bool NT>
__device__ __forceinline__ void dec_stream(const uint8_t *s0, uint8_t *d0, int64_t c0, int64_t stride,
                                           int64_t rstep, int64_t nrounds, const uint8_t *map,
                                           uint32_t &err)
{
    if (nrounds <= 0) return;
    u32x4 A[U], B[U];                 // rounds alternate between two register sets
    dec_load<U, NT>(A, s0, c0, stride);
    int64_t r = 0;
    for (; r + 2 < nrounds; r += 2) {
        dec_load<U, NT>(B, s0, c0 + rstep, stride);
        dec_store<U, NT>(A, d0, c0, stride, map, err);
        dec_load<U, NT>(A, s0, c0 + 2 * rstep, stride);
        dec_store<U, NT>(B, d0, c0 + rstep, stride, map, err);
        c0 += 2 * rstep;
    }
    if (r + 1 < nrounds) {
        dec_load<U, NT>(B, s0, c0 + rstep, stride);
        dec_store<U, NT>(A, d0, c0, stride, map, err);
        dec_store<U, NT>(B, d0, c0 + rstep, stride, map, err);
    } else {
        dec_store<U, NT>(A, d0, c0, stride, map, err);
    }
}

// The last, partial round in two steps, so that a kernel can issue its loads
// early: the loads (lanes past the end load the last in-range chunk again),
// then the decodes and stores of the chunks below nch.
template <int U, bool NT>
__device__ __forceinline__ void dec_round_load(u32x4 (&in)[U], const uint8_t *s0, int64_t c0,
                                               int64_t stride, int64_t nch)
{
    if (nch <= 0) return;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int64_t c = c0 + j * stride;
        in[j] = load16<NT>(s0 + 16 * (c < nch ? c : nch - 1));
    }
}
template <int U, bool NT>
__device__ __forceinline__ void dec_round_store(const u32x4 (&in)[U], uint8_t *d0, int64_t c0,
                                                int64_t stride, const uint8_t *map, uint32_t &err,
                                                int64_t nch)
{
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int64_t c = c0 + j * stride;
        if (c < nch) store12<NT>(d0 + 12 * c, dec_chunk(in[j], map, err));
    }
}
template <int U, bool NT>
__device__ __forceinline__ void dec_round_tail(const uint8_t *s0, uint8_t *d0, int64_t c0,
                                               int64_t stride, const uint8_t *map, uint32_t &err,
                                               int64_t nch)
{
    u32x4 in[U];
    dec_round_load<U, NT>(in, s0, c0, stride, nch);
    dec_round_store<U, NT>(in, d0, c0, stride, map, err, nch);
}

}  // namespace b64hip
