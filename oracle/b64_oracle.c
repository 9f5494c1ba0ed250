/*
 * b64_oracle.c -- plain, slow, obviously correct scalar base64 codec.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP codec is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the product library: its alphabet table, decode map and
 * arithmetic are written out here independently.
 *
 * What it follows (Mula & Lemire, "Base64 encoding and decoding at almost the
 * speed of a memory copy"):
 *   - Section "Base64": the alphabet of Table tab:base64table, the 3-byte ->
 *     four 6-bit values closed form, '=' padding to a multiple of four
 *     characters, the base64url substitution of the last two characters, and
 *     the 4 values -> 3 bytes closed form used by the look-up-table decoder
 *     (with a special value marking characters outside the alphabet).
 *   - Section "Encoding" (step 2): any 64-byte mapping may serve as alphabet.
 * Readings where the paper is silent (in the base functions padding is always
 * emitted; the tail zero-fills the missing bytes; '=' is legal only as the
 * last one or two characters of the final quantum; non-canonical trailing bits
 * are rejected; any non-alphabet byte including whitespace is invalid; a
 * length that is not a multiple of four is invalid at offset n) are stated in
 * the design notes and implemented in b64o_decode below.  The variants
 * (b64o_*_mode: unpadded output, CR LF line wrapping, whitespace skipping)
 * follow the paper's remarks that padding is optional and that base64 is
 * carried in MIME email; their readings are stated where they are defined.
 *
 * Every function is a direct transcription of the definition: ÷, × and mod
 * exactly as the closed forms print them, one group / one character at a time,
 * no blocking, no lookahead beyond what the definition needs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define B64O_INVALID 0xFFu          /* "special value" of the decode map       */
#define B64O_PAD     ((uint8_t)'=') /* padding character, fixed                */
#define B64O_EARG    INT64_MIN      /* bad argument (NULL, n < 0, bad alphabet) */

/* Variants (Section "Base64": padding "may" be appended; Section
 * "Introduction": base64 inside MIME email, whose lines are wrapped). */
#define B64O_NOPAD   1u  /* encode: no '='; decode: '=' is invalid, the final
                            quantum may be 2 or 3 characters                */
#define B64O_SKIP_WS 2u  /* decode: space, tab, CR and LF are ignored        */

/* Table tab:base64table: value v -> ASCII.  Written out row by row. */
const char b64o_alphabet_std[65] =
    "ABCDEFGHIJKLMNOPQRSTUVWXYZ"   /* values  0..25 */
    "abcdefghijklmnopqrstuvwxyz"   /* values 26..51 */
    "0123456789"                   /* values 52..61 */
    "+/";                          /* values 62, 63 */

/* Section "Base64": base64url replaces '+' by '-' and '/' by '_'. */
const char b64o_alphabet_url[65] =
    "ABCDEFGHIJKLMNOPQRSTUVWXYZ"
    "abcdefghijklmnopqrstuvwxyz"
    "0123456789"
    "-_";

/* Length of the padded encoding: groups of three bytes become four
 * characters and a partial last group is padded to four (Section "Base64"). */
int64_t b64o_encoded_len(int64_t n)
{
    if (n < 0) return B64O_EARG;
    return 4 * ((n + 2) / 3);
}

/* An alphabet must be invertible (Section "Base64": the map is invertible),
 * so its 64 bytes are distinct, and none of them may be the pad character. */
int b64o_alphabet_ok(const uint8_t *alpha)
{
    int seen[256];
    int v;
    if (!alpha) return 0;
    memset(seen, 0, sizeof seen);
    for (v = 0; v < 64; v++) {
        if (alpha[v] == B64O_PAD || seen[alpha[v]]) return 0;
        seen[alpha[v]] = 1;
    }
    return 1;
}

/* Encode n bytes to 4*ceil(n/3) characters with alphabet `alpha`.
 * Section "Base64": three bytes s1,s2,s3 map to the four 6-bit values
 *   s1 div 4,  (s2 div 16) + (s1*16 mod 64),  (s2*4 mod 64) + (s3 div 64),  s3 mod 64,
 * each then replaced by its character (Table tab:base64table, or the runtime
 * alphabet of Section "Encoding").  A last group of one or two bytes is
 * completed with zero bytes, only the characters that carry input bits are
 * kept, and '=' fills the quantum to four characters.
 * Returns the number of characters written, or B64O_EARG. */
int64_t b64o_encode(const uint8_t *src, int64_t n, uint8_t *dst, const uint8_t *alpha)
{
    int64_t i, o = 0;
    if (n < 0 || (n > 0 && (!src || !dst)) || !b64o_alphabet_ok(alpha)) return B64O_EARG;
    for (i = 0; i + 3 <= n; i += 3) {
        unsigned s1 = src[i], s2 = src[i + 1], s3 = src[i + 2];
        dst[o++] = alpha[s1 / 4];
        dst[o++] = alpha[(s2 / 16) + (s1 * 16) % 64];
        dst[o++] = alpha[(s2 * 4) % 64 + (s3 / 64)];
        dst[o++] = alpha[s3 % 64];
    }
    if (n - i == 1) {                  /* one leftover byte: s2 = s3 = 0 */
        unsigned s1 = src[i];
        dst[o++] = alpha[s1 / 4];
        dst[o++] = alpha[(s1 * 16) % 64];
        dst[o++] = B64O_PAD;
        dst[o++] = B64O_PAD;
    } else if (n - i == 2) {           /* two leftover bytes: s3 = 0 */
        unsigned s1 = src[i], s2 = src[i + 1];
        dst[o++] = alpha[s1 / 4];
        dst[o++] = alpha[(s2 / 16) + (s1 * 16) % 64];
        dst[o++] = alpha[(s2 * 4) % 64];
        dst[o++] = B64O_PAD;
    }
    return o;
}

/* The decode map of Section "Base64" (the look-up-table decoder): every byte
 * value maps to the special invalid value except the 64 alphabet characters,
 * which map to their 6-bit value. */
static void b64o_build_map(const uint8_t *alpha, uint8_t map[256])
{
    int c, v;
    for (c = 0; c < 256; c++) map[c] = B64O_INVALID;
    for (v = 0; v < 64; v++) map[alpha[v]] = (uint8_t)v;
}

/* Decode n characters.  Returns the decoded length r >= 0 when the input is a
 * valid padded encoding, ~off (= -off-1) when it is not, where off in [0, n]
 * is the first invalid offset: the length of the longest prefix of the input
 * that is still a prefix of some valid encoding (off == n: truncated input),
 * or B64O_EARG.  On invalid input the contents of dst are unspecified.
 *
 * Validation walks the characters in order with three states:
 *   DATA  -- inside the data quanta,
 *   PAD1  -- one '=' seen at position 2 of the final quantum,
 *   DONE  -- the final padded quantum is complete; nothing may follow.
 * A character outside the alphabet is invalid (Section "Base64": the special
 * value of the look-up table).  '=' may only stand at position 2 or 3 of a
 * quantum; at position 2 the previous value must have its low four bits zero,
 * at position 3 after a data character the previous value must have its low
 * two bits zero (a canonical encoding of one or two bytes).
 * Each full quantum a,b,c,d becomes
 *   (a*4) + (b div 16),  (b*16 mod 256) + (c div 4),  (c*64 mod 256) + d
 * (Section "Base64"); a final "xx==" yields the first byte, "xxx=" the first two. */
int64_t b64o_decode(const uint8_t *src, int64_t n, uint8_t *dst, const uint8_t *alpha)
{
    enum { DATA, PAD1, DONE } state = DATA;
    uint8_t map[256];
    int64_t i, q, o = 0;
    if (n < 0 || (n > 0 && (!src || !dst)) || !b64o_alphabet_ok(alpha)) return B64O_EARG;
    b64o_build_map(alpha, map);

    /* pass 1: validation, first invalid offset */
    for (i = 0; i < n; i++) {
        uint8_t c = src[i];
        int64_t p = i % 4;
        if (state == DONE) return ~i;
        if (c != B64O_PAD) {
            if (map[c] == B64O_INVALID) return ~i;
            if (state == PAD1) return ~i;
            continue;
        }
        if (p == 0 || p == 1) return ~i;
        if (p == 2) {
            if (map[src[i - 1]] % 16 != 0) return ~i;
            state = PAD1;
        } else { /* p == 3 */
            if (state == PAD1) {
                state = DONE;
            } else {
                if (map[src[i - 1]] % 4 != 0) return ~i;
                state = DONE;
            }
        }
    }
    if (state == PAD1 || (n % 4 != 0 && state != DONE)) return ~n;

    /* pass 2: every quantum a,b,c,d -> three bytes; a padded final quantum
     * keeps only the bytes its data characters carry. */
    for (q = 0; q < n; q += 4) {
        unsigned a = map[src[q]], b = map[src[q + 1]];
        unsigned c = src[q + 2] == B64O_PAD ? 0 : map[src[q + 2]];
        unsigned d = src[q + 3] == B64O_PAD ? 0 : map[src[q + 3]];
        int npad = (src[q + 2] == B64O_PAD) + (src[q + 3] == B64O_PAD);
        dst[o++] = (uint8_t)((a * 4) + (b / 16));
        if (npad < 2) dst[o++] = (uint8_t)((b * 16) % 256 + (c / 4));
        if (npad < 1) dst[o++] = (uint8_t)((c * 64) % 256 + d);
    }
    return o;
}

/* Decode `nrows` strings of the same length `len`, stored back to back in
 * `rows`, writing each call's return value to result[k].  A convenience loop
 * over b64o_decode for the brute-force tests (no other logic). */
void b64o_decode_rows(const uint8_t *rows, int64_t nrows, int64_t len,
                      const uint8_t *alpha, int64_t *result)
{
    uint8_t out[64];
    int64_t k;
    for (k = 0; k < nrows; k++) {
        if (len > 80) { result[k] = B64O_EARG; continue; }
        result[k] = b64o_decode(rows + k * len, len, out, alpha);
    }
}

/* Encode / decode a list of buffers packed back to back: buffer b is
 * src[in_off[b] .. in_off[b+1]) and its output starts at dst + out_off[b].
 * out_len[b] receives b64o_encode's / b64o_decode's return value.  Plain loop
 * over the single-buffer functions (the batch result is defined buffer by
 * buffer). */
void b64o_encode_list(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                      uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                      const uint8_t *alpha)
{
    int64_t b;
    for (b = 0; b < nbuf; b++)
        out_len[b] = b64o_encode(src + in_off[b], in_off[b + 1] - in_off[b],
                                 dst + out_off[b], alpha);
}

void b64o_decode_list(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                      uint8_t *dst, const int64_t *out_off, int64_t *result,
                      const uint8_t *alpha)
{
    int64_t b;
    for (b = 0; b < nbuf; b++)
        result[b] = b64o_decode(src + in_off[b], in_off[b + 1] - in_off[b],
                                dst + out_off[b], alpha);
}

/* ------------------------------------------------------------ variants -- */

/* The four bytes B64O_SKIP_WS ignores: space, tab, carriage return, line feed. */
static int b64o_is_ws(uint8_t c)
{
    return c == ' ' || c == '\t' || c == '\r' || c == '\n';
}

/* Characters of the unwrapped encoding: 4 per whole group and, for a last
 * group of r = 1 or 2 bytes, 4 when padded or r + 1 (the characters that carry
 * input bits) without padding. */
static int64_t b64o_chars(int64_t n, unsigned flags)
{
    int64_t r = n % 3;
    if (r == 0 || !(flags & B64O_NOPAD)) return 4 * ((n + 2) / 3);
    return 4 * (n / 3) + r + 1;
}

/* Length of the encoding with `flags` (B64O_NOPAD or 0) and, when line_len > 0,
 * a CR LF pair between consecutive lines of line_len characters. */
int64_t b64o_encoded_len_mode(int64_t n, unsigned flags, int64_t line_len)
{
    int64_t m;
    if (n < 0 || line_len < 0 || (flags & ~B64O_NOPAD)) return B64O_EARG;
    m = b64o_chars(n, flags);
    if (line_len > 0 && m > 0) m += 2 * ((m - 1) / line_len);
    return m;
}

/* Encode with padding (flags 0) or without (B64O_NOPAD), then, when
 * line_len > 0, break the character stream into lines of line_len
 * characters separated by CR LF; no line break follows the last line.
 * The characters themselves are b64o_encode's; without padding the trailing
 * '=' characters are simply not emitted.  Returns the length written or
 * B64O_EARG. */
int64_t b64o_encode_mode(const uint8_t *src, int64_t n, uint8_t *dst, const uint8_t *alpha,
                         unsigned flags, int64_t line_len)
{
    uint8_t quantum[4];
    int64_t g, o = 0, col = 0;
    int k, m;
    if (n < 0 || (n > 0 && (!src || !dst)) || !b64o_alphabet_ok(alpha) || line_len < 0 ||
        (flags & ~B64O_NOPAD))
        return B64O_EARG;
    for (g = 0; g < n; g += 3) {
        int64_t r = n - g < 3 ? n - g : 3;
        /* one group through the padded encoder: four characters */
        b64o_encode(src + g, r, quantum, alpha);
        m = 4;
        if (flags & B64O_NOPAD) while (m > 0 && quantum[m - 1] == B64O_PAD) m--;
        for (k = 0; k < m; k++) {
            if (line_len > 0 && col == line_len) {
                dst[o++] = '\r';
                dst[o++] = '\n';
                col = 0;
            }
            dst[o++] = quantum[k];
            col++;
        }
    }
    return o;
}

/* Decode with `flags`.  The significant characters are all characters, or,
 * with B64O_SKIP_WS, those that are not space, tab, CR or LF; the rules below
 * apply to the sequence of significant characters, and offsets count every
 * character of the input.  Returns the decoded length, ~off with off the first
 * invalid offset (n when the input ends too early), or B64O_EARG (also for
 * B64O_SKIP_WS with an alphabet that contains one of the four ignored bytes).
 *
 * Padded (no B64O_NOPAD): the rules of b64o_decode.
 * Unpadded (B64O_NOPAD): every significant character must be in the alphabet
 * ('=' is not); the count k of significant characters may not be 1 mod 4; a
 * final quantum of 2 (3) characters is canonical only when its last value has
 * its low 4 (2) bits zero, otherwise the input ends too early (it could still
 * be completed to a valid encoding).  A final quantum of 2 characters yields
 * one byte, of 3 characters two bytes, by the same closed form. */
int64_t b64o_decode_mode(const uint8_t *src, int64_t n, uint8_t *dst, const uint8_t *alpha,
                         unsigned flags)
{
    enum { DATA, PAD1, DONE } state = DATA;
    const int nopad = (flags & B64O_NOPAD) != 0, skip = (flags & B64O_SKIP_WS) != 0;
    uint8_t map[256], prev = 0;
    unsigned val[4];
    int64_t i, k = 0, o = 0;
    int m = 0;
    if (n < 0 || (n > 0 && (!src || !dst)) || !b64o_alphabet_ok(alpha) ||
        (flags & ~(B64O_NOPAD | B64O_SKIP_WS)))
        return B64O_EARG;
    if (skip)
        for (i = 0; i < 64; i++)
            if (b64o_is_ws(alpha[i])) return B64O_EARG;
    b64o_build_map(alpha, map);

    /* pass 1: validation over the significant characters */
    for (i = 0; i < n; i++) {
        uint8_t c = src[i];
        int64_t p = k % 4;
        if (skip && b64o_is_ws(c)) continue;
        if (state == DONE) return ~i;
        if (c != B64O_PAD || nopad) {
            if (map[c] == B64O_INVALID) return ~i;
            if (state == PAD1) return ~i;
        } else if (p == 0 || p == 1) {
            return ~i;
        } else if (p == 2) {
            if (map[prev] % 16 != 0) return ~i;
            state = PAD1;
        } else if (state == PAD1) {
            state = DONE;
        } else {
            if (map[prev] % 4 != 0) return ~i;
            state = DONE;
        }
        prev = c;
        k++;
    }
    if (nopad) {
        if (k % 4 == 1) return ~n;
        if (k % 4 == 2 && map[prev] % 16 != 0) return ~n;
        if (k % 4 == 3 && map[prev] % 4 != 0) return ~n;
    } else if (state == PAD1 || (k % 4 != 0 && state != DONE)) {
        return ~n;
    }

    /* pass 2: the data values, four at a time, through the closed form
     * (a*4) + (b div 16), (b*16 mod 256) + (c div 4), (c*64 mod 256) + d;
     * a last group of 2 or 3 values keeps the bytes they carry. */
    for (i = 0; i < n; i++) {
        uint8_t c = src[i];
        if (skip && b64o_is_ws(c)) continue;
        if (c == B64O_PAD) break;      /* only reached in padded mode */
        val[m++] = map[c];
        if (m == 4) {
            dst[o++] = (uint8_t)((val[0] * 4) + (val[1] / 16));
            dst[o++] = (uint8_t)((val[1] * 16) % 256 + (val[2] / 4));
            dst[o++] = (uint8_t)((val[2] * 64) % 256 + val[3]);
            m = 0;
        }
    }
    if (m >= 2) dst[o++] = (uint8_t)((val[0] * 4) + (val[1] / 16));
    if (m == 3) dst[o++] = (uint8_t)((val[1] * 16) % 256 + (val[2] / 4));
    return o;
}

/* b64o_decode_mode over `nrows` strings of length `len` (brute-force tests). */
void b64o_decode_mode_rows(const uint8_t *rows, int64_t nrows, int64_t len, const uint8_t *alpha,
                           unsigned flags, int64_t *result)
{
    uint8_t out[64];
    int64_t k;
    for (k = 0; k < nrows; k++) {
        if (len > 80) { result[k] = B64O_EARG; continue; }
        result[k] = b64o_decode_mode(rows + k * len, len, out, alpha, flags);
    }
}

/* Packed-buffer loops over the variant functions, as b64o_encode_list /
 * b64o_decode_list. */
void b64o_encode_mode_list(const uint8_t *src, const int64_t *in_off, int64_t nbuf, uint8_t *dst,
                           const int64_t *out_off, int64_t *out_len, const uint8_t *alpha,
                           unsigned flags, int64_t line_len)
{
    int64_t b;
    for (b = 0; b < nbuf; b++)
        out_len[b] = b64o_encode_mode(src + in_off[b], in_off[b + 1] - in_off[b], dst + out_off[b],
                                      alpha, flags, line_len);
}

void b64o_decode_mode_list(const uint8_t *src, const int64_t *in_off, int64_t nbuf, uint8_t *dst,
                           const int64_t *out_off, int64_t *result, const uint8_t *alpha,
                           unsigned flags)
{
    int64_t b;
    for (b = 0; b < nbuf; b++)
        result[b] = b64o_decode_mode(src + in_off[b], in_off[b + 1] - in_off[b], dst + out_off[b],
                                     alpha, flags);
}

/* ------------------------------------------------------ fused consumer -- */

/* float32 bits -> bfloat16 bits, rounding to nearest with ties to even; every
 * NaN becomes the quiet NaN 0x7FC0.  Written from the definition: the upper
 * 16 bits of the float, plus one unit in the last place when the dropped
 * 16 bits exceed half a unit, or equal it and the kept part is odd. */
uint16_t b64o_f32_to_bf16(uint32_t u)
{
    uint32_t keep = u >> 16, drop = u & 0xFFFFu;
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0) return 0x7FC0;
    if (drop > 0x8000u || (drop == 0x8000u && (keep & 1u))) keep += 1;
    return (uint16_t)keep;
}

/* Decode `nrows` rows packed back to back (row b is src[in_off[b] ..
 * in_off[b+1])), each the base64 encoding (b64o_decode_mode with `flags`) of
 * `dim` little-endian float32 values, into dst[b*dim .. (b+1)*dim) as
 * bfloat16.  status[b] = -1 for a good row, the first invalid offset for an
 * invalid encoding, -2 for a valid encoding whose length is not 4*dim bytes
 * (its dst row is then unspecified).  A plain loop: decode the row, then
 * convert each float (the consumer). */
void b64o_decode_f32_bf16_rows(const uint8_t *src, const int64_t *in_off, int64_t nrows, int64_t dim,
                               uint16_t *dst, int64_t *status, const uint8_t *alpha, unsigned flags)
{
    int64_t b, k, cap = 0;
    uint8_t *tmp = 0;
    for (b = 0; b < nrows; b++) {
        int64_t len = in_off[b + 1] - in_off[b], need = 3 * (len / 4) + 3, r;
        if (need > cap) {
            uint8_t *t = (uint8_t *)realloc(tmp, (size_t)need);
            if (!t) { status[b] = B64O_EARG; continue; }
            tmp = t;
            cap = need;
        }
        r = b64o_decode_mode(src + in_off[b], len, tmp, alpha, flags);
        if (r < 0) { status[b] = r == B64O_EARG ? B64O_EARG : ~r; continue; }
        if (r != 4 * dim) { status[b] = -2; continue; }
        for (k = 0; k < dim; k++) {
            uint32_t u = (uint32_t)tmp[4 * k] | ((uint32_t)tmp[4 * k + 1] << 8) |
                         ((uint32_t)tmp[4 * k + 2] << 16) | ((uint32_t)tmp[4 * k + 3] << 24);
            dst[b * dim + k] = b64o_f32_to_bf16(u);
        }
        status[b] = -1;
    }
    free(tmp);
}
