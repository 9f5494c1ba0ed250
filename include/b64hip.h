/*
 * b64hip.h -- C ABI of libb64hip.so, a base64 codec for AMD Instinct MI355X
 * (gfx950), after W. Mula and D. Lemire, "Base64 encoding and decoding at
 * almost the speed of a memory copy".
 *
 * Conventions for every entry point
 *   - Data pointers (src, dst, in_off, out_off, out_len, first_bad, status
 *     words) are DEVICE pointers on the current HIP device, owned by the
 *     caller.  The library never frees them and keeps no reference to them
 *     once the enqueued work has completed.  No alignment is required.
 *   - `alphabet` is a HOST pointer to 64 bytes, copied by value into the
 *     kernel arguments of the launch (Section "Encoding", step 2: any 64-byte
 *     mapping may be used, even one chosen at run time).  It must hold 64
 *     distinct bytes, none equal to '='; bytes >= 0x80 are allowed.
 *   - Work is enqueued on the caller's `stream` (a hipStream_t; 0 means the
 *     null stream).  Functions marked "asynchronous" return as soon as the
 *     work is enqueued; functions marked "blocking" synchronize `stream`.
 *   - Errors never abort or throw.  Bad arguments return B64_EARG; a failing
 *     HIP call returns B64_EHIP.  b64_last_error() then gives a message.
 *     Invalid base64 CONTENT is not an API error: it is reported as a first
 *     invalid offset (below).
 *   - Lengths, offsets and counts are int64 bytes.
 *
 * Output format (Section "Base64"): groups of three bytes s1,s2,s3 become the
 * characters of the four 6-bit values s1 div 4, (s2 div 16) + (s1*16 mod 64),
 * (s2*4 mod 64) + (s3 div 64), s3 mod 64; a last group of one or two bytes is
 * zero-filled and padded with '=' to four characters.  Decoding inverts this
 * with the 4 -> 3 byte closed form of the same section.
 *
 * First invalid offset.  Decoding validates its input (Section "Decoding":
 * characters outside the alphabet are detected).  For an input that is not a
 * valid padded encoding, the reported offset `off` in [0, n] is the length of
 * the longest prefix of the input that is still a prefix of some valid
 * encoding: the position of the first character outside the alphabet, of a
 * misplaced '=', of a '=' after a value with nonzero trailing bits, of any
 * character after the final padded quantum; off == n means the input is
 * truncated (n not a multiple of 4).  Whitespace is invalid.  The output
 * bytes written for an invalid input are unspecified.
 */
#ifndef B64HIP_H
#define B64HIP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define B64_EARG INT64_MIN         /* bad argument                              */
#define B64_EHIP (INT64_MIN + 1)   /* a HIP runtime call failed                 */

/* Table tab:base64table: A-Z a-z 0-9 + /  (64 bytes, not NUL-terminated use). */
extern const char b64_alphabet_std[64];
/* base64url (Section "Base64"): '+' -> '-', '/' -> '_'.                       */
extern const char b64_alphabet_url[64];

/* 4*ceil(n/3): characters produced by encoding n bytes; B64_EARG if n < 0.    */
int64_t b64_encoded_len(int64_t n);
/* 3*(n/4): capacity to allocate for decoding n characters; B64_EARG if n < 0. */
int64_t b64_decoded_max_len(int64_t n);

/* Encode src[0..n) to dst[0..4*ceil(n/3)).  Asynchronous.
 * Returns the encoded length (known on the host) or B64_EARG / B64_EHIP.
 * dst must hold b64_encoded_len(n) bytes; src and dst must not overlap.
 * Encoding cannot fail on content.  (Section "Encoding".) */
int64_t b64_encode(const uint8_t *src, int64_t n, uint8_t *dst,
                   const char *alphabet, hipStream_t stream);

/* Decode src[0..n) into dst (capacity b64_decoded_max_len(n)).  Blocking.
 * Returns the decoded length r >= 0 for a valid input, ~off (= -off-1) for an
 * invalid one (off as defined above), or B64_EARG / B64_EHIP (both below
 * -2^62).  One kernel launch, whose last workgroup writes the status into
 * pinned host memory of the calling thread; then `stream` is synchronized.
 * (Section "Decoding".) */
int64_t b64_decode(const uint8_t *src, int64_t n, uint8_t *dst,
                   const char *alphabet, hipStream_t stream);

/* Decode, asynchronous form.  Results land in device memory once `stream`
 * reaches them: *out_len = decoded length (or -1 if invalid), *first_bad = -1
 * if valid (else the first invalid offset); their previous contents do not
 * matter.  Returns 0 or B64_EARG / B64_EHIP.  One kernel launch, whose last
 * workgroup writes the status: the library keeps a 2 KiB status slot in
 * device memory per stream handle (hipStreamPerThread gets one per host
 * thread), which is back to zero after every call.  Safe to capture in a HIP
 * graph: the launches captured from one stream in one capture share a slot
 * of their own (they run in order within a replay, and launches of one graph
 * run one after another).  Once the 1024 slots of a device are taken, calls
 * on new streams and in new captures take three launches (reset, decode,
 * finish) with the status in *out_len / *first_bad alone.
 * (Section "Decoding".) */
int64_t b64_decode_async(const uint8_t *src, int64_t n, uint8_t *dst,
                         int64_t *out_len, int64_t *first_bad,
                         const char *alphabet, hipStream_t stream);

/* Validate src[0..n) as a padded base64 encoding without decoding it: the
 * characters are read and nothing is written.  Blocking.  Returns what
 * b64_decode would return -- the decoded length r >= 0 for a valid input,
 * ~off for an invalid one, or B64_EARG / B64_EHIP -- at about 4/7 of the
 * memory traffic.  (Section "Decoding": the look-up-table validation.) */
int64_t b64_validate(const uint8_t *src, int64_t n, const char *alphabet, hipStream_t stream);

/* Validate, asynchronous form; results in device memory, launches and
 * status slots as for b64_decode_async.  Returns 0 or B64_EARG / B64_EHIP.
 * (Section "Decoding".) */
int64_t b64_validate_async(const uint8_t *src, int64_t n, int64_t *out_len, int64_t *first_bad,
                           const char *alphabet, hipStream_t stream);

/* Batched encode of nbuf ragged buffers packed back to back.  Asynchronous.
 * Buffer b is src[in_off[b] .. in_off[b+1]); in_off has nbuf+1 non-decreasing
 * entries.  Output b is written at dst + out_off[b] (capacity
 * b64_encoded_len(length_b); out_off has nbuf entries; outputs must not
 * overlap each other or the input).  out_len[b] receives 4*ceil(length_b/3).
 * Returns 0 or B64_EARG / B64_EHIP.  One launch covers every buffer.
 * Safe to capture in a HIP graph.  (Section "Encoding", applied per buffer.) */
int64_t b64_encode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                         uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                         const char *alphabet, hipStream_t stream);

/* Batched decode, asynchronous; layout as b64_encode_batch (output capacity
 * b64_decoded_max_len(length_b)).  Per buffer: first_bad[b] = -1 and
 * out_len[b] = decoded length if valid, else first_bad[b] = the first invalid
 * offset within buffer b and out_len[b] = -1.  Returns 0 or B64_EARG /
 * B64_EHIP.  Safe to capture in a HIP graph.  (Section "Decoding", per buffer.) */
int64_t b64_decode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                         uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                         int64_t *first_bad, const char *alphabet, hipStream_t stream);

/* ---------------------------------------------------------------- variants --
 * Section "Base64" makes the '=' padding optional ("may be appended") and
 * names base64url; Section "Introduction" names MIME email, which carries
 * base64 in lines.  The _mode entry points take `flags`:
 *   B64_NOPAD    encode: no '=' -- a last group of 1 or 2 bytes gives 2 or 3
 *                characters.  decode: '=' is invalid everywhere; the final
 *                quantum may have 2 or 3 characters (1 or 2 bytes); a final
 *                quantum of 1 character, or of 2 (3) characters whose last
 *                value has nonzero low 4 (2) bits, makes the input end too
 *                early (first invalid offset n).
 *   B64_SKIP_WS  decode / validate: space, tab, CR and LF are ignored; every
 *                rule applies to the remaining characters, and offsets count
 *                every byte of the input.  The alphabet may not contain any
 *                of those four bytes.  The decode may leave any bytes in dst
 *                past the decoded length (within the output capacity): text
 *                in regular lines is first decoded with guessed line
 *                positions, and decoded again if the guess fails.
 * and encode takes `line_len`: 0 for one line, else a multiple of 4; CR LF
 * then separates consecutive lines of line_len characters (no CR LF after
 * the last line).  flags = 0 and line_len = 0 give the plain entry points. */
#define B64_NOPAD   1u
#define B64_SKIP_WS 2u

/* Characters produced by b64_encode_mode(n, flags, line_len), line breaks
 * included; B64_EARG for n < 0, a bad line_len or a flag other than B64_NOPAD. */
int64_t b64_encoded_len_mode(int64_t n, uint32_t flags, int64_t line_len);
/* Output capacity for decoding n characters with `flags`: 3*(n/4), plus
 * max(0, n%4 - 1) under B64_NOPAD; B64_EARG for n < 0 or unknown flags. */
int64_t b64_decoded_max_len_mode(int64_t n, uint32_t flags);
/* Device workspace, in bytes, that the asynchronous B64_SKIP_WS decode and
 * validate need for n characters (0 without B64_SKIP_WS): 8 bytes per tile of
 * 4-32 KiB of input plus 24.  B64_EARG for n < 0 or unknown flags. */
int64_t b64_decode_workspace_size(int64_t n, uint32_t flags);

/* Encode with variants.  Asynchronous; returns b64_encoded_len_mode(n, flags,
 * line_len) or B64_EARG / B64_EHIP; dst holds that many bytes. */
int64_t b64_encode_mode(const uint8_t *src, int64_t n, uint8_t *dst, const char *alphabet,
                        uint32_t flags, int64_t line_len, hipStream_t stream);
/* Decode with variants.  Blocking; returns as b64_decode.  dst holds
 * b64_decoded_max_len_mode(n, flags) bytes.  With B64_SKIP_WS the library
 * uses a device workspace of its own, per thread and device, grown with
 * hipMalloc as inputs grow and kept until the process ends. */
int64_t b64_decode_mode(const uint8_t *src, int64_t n, uint8_t *dst, const char *alphabet,
                        uint32_t flags, hipStream_t stream);
/* Decode with variants, asynchronous; status as b64_decode_async.
 * `workspace` is a device buffer of workspace_bytes >=
 * b64_decode_workspace_size(n, flags) bytes (may be NULL when that is 0),
 * owned by the caller and busy until the stream has run the decode.  Safe to
 * capture in a HIP graph. */
int64_t b64_decode_mode_async(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *out_len,
                              int64_t *first_bad, const char *alphabet, uint32_t flags,
                              void *workspace, int64_t workspace_bytes, hipStream_t stream);
/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * whitespace-skipping decode of b64_decode_mode_async (flags = B64_SKIP_WS,
 * optionally | B64_NOPAD; results in *out_len / *first_bad as there) whose
 * workspace is a fixed 1 MiB array of device memory inside the library
 * instead of a caller's buffer.  The library holds one such array per
 * device until the process ends; the call allocates nothing.  Every call on
 * one device uses that device's array, so calls that overlap on one device
 * (on different streams, or from different threads) race and must not be
 * made; calls one after another on one stream are fine (each starts by
 * resetting what must start at zero).  Inputs longer than
 * B64_NOALLOC_MAX_CHARS bytes, or flags without B64_SKIP_WS, return
 * B64_EARG.  Asynchronous; returns 0 or B64_EARG / B64_EHIP. */
#define B64_NOALLOC_MAX_CHARS INT64_C(4294868992)   /* 131,069 tiles of 32 KiB */
int64_t b64_decode_ws_async_noalloc(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *out_len,
                                    int64_t *first_bad, const char *alphabet, uint32_t flags,
                                    hipStream_t stream);
/* Validate with variants.  Blocking; returns what b64_decode_mode would
 * return; writes no output. */
int64_t b64_validate_mode(const uint8_t *src, int64_t n, const char *alphabet, uint32_t flags,
                          hipStream_t stream);
/* Validate with variants, asynchronous; status and workspace as
 * b64_decode_mode_async. */
int64_t b64_validate_mode_async(const uint8_t *src, int64_t n, int64_t *out_len, int64_t *first_bad,
                                const char *alphabet, uint32_t flags, void *workspace,
                                int64_t workspace_bytes, hipStream_t stream);
/* Batched encode / decode with variants: as b64_encode_batch /
 * b64_decode_batch, `flags` 0 or B64_NOPAD (out_len[b] of an unpadded encode
 * is ceil(4*length_b/3); decode capacity per buffer is
 * b64_decoded_max_len_mode(length_b, flags)). */
int64_t b64_encode_batch_mode(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                              uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                              const char *alphabet, uint32_t flags, hipStream_t stream);
int64_t b64_decode_batch_mode(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                              uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                              int64_t *first_bad, const char *alphabet, uint32_t flags,
                              hipStream_t stream);

/* ----------------------------------------------------------- fused decode --
 * Decode fused into its consumer (Section "Conclusion": run the decoder inside
 * the code that uses the data).  Each of `nrows` rows packed back to back
 * (row b is src[in_off[b] .. in_off[b+1]), in_off has nrows+1 non-decreasing
 * entries) is the base64 encoding (padded, or unpadded with B64_NOPAD) of
 * `dim` little-endian IEEE-754 float32 values; they are decoded and rounded
 * to bfloat16 (nearest, ties to even; every NaN becomes 0x7FC0) in registers
 * and written to dst[b*dim .. (b+1)*dim) (row-major [nrows, dim] bfloat16,
 * device memory, 2*nrows*dim bytes).  The decoded bytes are never stored.
 * status[b] (device, nrows entries) = -1 for a good row, the first invalid
 * offset within the row for an invalid encoding, or -2 for a valid encoding
 * whose decoded length is not 4*dim bytes; dst rows of bad rows are
 * unspecified (but nothing outside them is written).  Asynchronous; returns 0
 * or B64_EARG / B64_EHIP.  Safe to capture in a HIP graph. */
int64_t b64_decode_f32_bf16(const uint8_t *src, const int64_t *in_off, int64_t nrows, int64_t dim,
                            uint16_t *dst, int64_t *status, const char *alphabet, uint32_t flags,
                            hipStream_t stream);

/* Host-memory pipeline (an opaque handle).  Encodes or decodes data that
 * lives in ordinary host memory by cutting it into chunks that stream through
 * pinned staging, host-to-device copies, the kernels and device-to-host
 * copies, with up to `depth` chunks in flight (one stream per stage).  The
 * handle owns, until b64_pipeline_destroy, slots x 2 pinned host buffers and
 * slots x 2 device buffers of 4/3 x chunk_bytes each (chunk_bytes is rounded
 * up to a multiple of 1536; slots = min(depth, 3)), and is bound to the HIP
 * device current at creation.  One handle serves one calling thread at a
 * time.  (Section "Experiments": large inputs are best processed in parts.)
 * b64_pipeline_create: chunk_bytes >= 48, 1 <= depth <= 16 (values above 3
 * act as 3: on MI355X, copies queued further ahead run slower),
 * 1 <= host_threads <= 64 (threads for the host-side copies); returns NULL on
 * error (message: b64_pipeline_last_error()). */
typedef struct b64_pipeline b64_pipeline;
b64_pipeline *b64_pipeline_create(int64_t chunk_bytes, int depth, int host_threads);
void b64_pipeline_destroy(b64_pipeline *p);
/* Blocking.  src / dst are HOST pointers (any memory).  Returns
 * 4*ceil(n/3), or B64_EARG / B64_EHIP.  dst holds b64_encoded_len(n) bytes.
 * A src or dst in pinned host memory (hipHostMalloc, or registered) is copied
 * to or from the device directly, with no staging copy on that side; this
 * applies to decode as well.                                                */
int64_t b64_pipeline_encode(b64_pipeline *p, const uint8_t *src, int64_t n, uint8_t *dst,
                            const char *alphabet);
/* Blocking.  src / dst are HOST pointers; dst holds b64_decoded_max_len(n)
 * bytes.  Returns the decoded length, ~off (the first invalid offset of the
 * whole input, as b64_decode defines it), or B64_EARG / B64_EHIP.  With a
 * pinned dst, dst may also receive bytes past the decoded length (up to
 * b64_decoded_max_len(n)), and, for an invalid input, bytes of chunks after
 * the first invalid one. */
int64_t b64_pipeline_decode(b64_pipeline *p, const uint8_t *src, int64_t n, uint8_t *dst,
                            const char *alphabet);
const char *b64_pipeline_last_error(void);

/* ------------------------------------------------------------- serving --
 * A continuous-batching request server over the batched codec (the growth
 * path that serves many small requests: requests that arrive while others
 * are on the GPU join the next launch, and launches on different streams run
 * at the same time).  b64_server_create allocates the device arena of
 * `budget_bytes` (the HBM budget: every staged launch's payloads and outputs
 * are allocated in it, and requests wait while it is full),
 * `nstreams` HIP streams (1..16, default priority, launches go round robin)
 * and events for up to `depth` launches in flight (nstreams..64); a launch
 * coalesces up to `max_batch` queued requests of one kind and up to
 * `max_batch_bytes` payload bytes (a single larger request still goes
 * alone).  Launches can skip the arena (b64_server_set_zero_copy_max).  The
 * server is bound to the device current at creation.  Returns NULL on error
 * (message: b64_server_last_error()). */
typedef struct b64_server b64_server;
b64_server *b64_server_create(int64_t budget_bytes, int nstreams, int depth, int64_t max_batch,
                              int64_t max_batch_bytes);
void b64_server_destroy(b64_server *s);
/* Launches whose payload is at most `bytes` run zero-copy: their kernel reads
 * the payloads from, and writes the outputs to, the pinned host pools (mapped
 * into the device's address space) over PCIe, with no DMA copy and no arena
 * space; larger launches stage through the arena.  0 (the default) turns
 * zero-copy off: buffers then stay in device memory under the HBM budget.  Returns the previous value (bytes = -1 only reads
 * it), or B64_EARG. */
int64_t b64_server_set_zero_copy_max(b64_server *s, int64_t bytes);
/* How staged launches move payloads into the arena and outputs out of it:
 * B64_STAGE_KERNELS -- copy kernels that read or write the pinned host
 * pools, mapped into the device's address space; B64_STAGE_DMA --
 * hipMemcpyAsync; B64_STAGE_AUTO (the default) -- kernels for launches of
 * at most 1 MiB of payload, DMA for larger ones.  Returns the previous mode
 * (mode = -1 only reads it), or B64_EARG. */
#define B64_STAGE_KERNELS 0
#define B64_STAGE_DMA 1
#define B64_STAGE_AUTO 2
int64_t b64_server_set_staging(b64_server *s, int mode);
const char *b64_server_last_error(void);
#define B64_SERVE_ENCODE 0
#define B64_SERVE_DECODE 1
/* stats[] entries written by b64_server_run                                  */
#define B64_STAT_LAUNCHES 0        /* batched launches                          */
#define B64_STAT_WALL_NS 1         /* first arrival window to last result, ns   */
#define B64_STAT_PEAK_ARENA 2      /* most arena bytes held at once             */
#define B64_STAT_MAX_INFLIGHT 3    /* most launches enqueued and not finished   */
#define B64_STAT_MAX_CONCURRENT 4  /* most launches running on the device at once
                                      (from device timestamps of their first and
                                      last operation)                           */
#define B64_STAT_OVERLAPPED 5      /* launches that ran at the same time as another */
#define B64_STAT_ARENA 6           /* arena bytes                               */
#define B64_STAT_ZERO_COPY 7       /* launches that ran zero-copy               */
#define B64_STAT_COUNT 8
/* Blocking.  Serves `nreq` requests on the calling thread and returns when
 * all are done.  Request i (kind[i] = B64_SERVE_ENCODE or B64_SERVE_DECODE)
 * arrives arrival_ns[i] nanoseconds after the call starts serving
 * (non-decreasing); its payload is src[in_off[i] .. in_off[i+1]) in HOST
 * memory (in_off: nreq+1 non-decreasing entries).  Before serving, the
 * payloads are copied into pinned host pools (as a network stack would have
 * left them); each request's bytes go to the device only when its launch is
 * enqueued (or are read there by the kernel, for a zero-copy launch).  Results, in HOST memory: dst + out_off[i] receives the output
 * (capacity b64_encoded_len / b64_decoded_max_len of the payload length),
 * out_len[i] the output length (-1 for an invalid decode), first_bad[i] -1
 * or the first invalid offset (decodes), done_ns[i] the time the request's
 * results were in host memory (same clock as arrival_ns).  stats must hold
 * B64_STAT_COUNT entries.  Returns 0, or B64_EARG / B64_EHIP (message:
 * b64_server_last_error()).  One call at a time per server.
 * (Section "Encoding" and Section "Decoding", per request.) */
int64_t b64_server_run(b64_server *s, int64_t nreq, const int32_t *kind, const int64_t *arrival_ns,
                       const uint8_t *src, const int64_t *in_off, uint8_t *dst,
                       const int64_t *out_off, int64_t *out_len, int64_t *first_bad,
                       int64_t *done_ns, const char *alphabet, int64_t *stats);

/* Launch shape used by the kernels of operation `op` (0 encode, 1 decode,
 * 2 encode_batch, 3 decode_batch, 4 validate, 5 line-wrapped encode,
 * 6 whitespace-skipping decode / validate, 7 fused float32 -> bfloat16
 * decode) for inputs in size bucket `bucket`: `unroll` lane chunks in flight
 * per lane (1, 2, 4 or 8; a lane chunk is 12 bytes -> 16 characters or back;
 * for op 6 the rounds of 1024 characters a decoding wave has in flight: 1, 2
 * or 4, and 8 runs as 2), `blocks_per_cu` workgroups of 256 threads per
 * compute unit (1..64; an input that fewer workgroups cover in one round gets
 * just those), and `nontemporal` (0 or 1) for streaming loads and stores.
 * Size buckets of the input length n in bytes: 0 for n < 64 KiB, 1 for
 * n < 1 MiB, 2 for n < 16 MiB, 3 for n < 128 MiB, 4 from 128 MiB; ops 2, 3
 * and 7 always use bucket 4 (their total size lives in device memory);
 * bucket -1 sets every bucket.  Process-wide; meant for the autotuner.  Does not change results
 * (every unroll x nontemporal pair is tested against the oracle at 1, 3, 8
 * and 64 workgroups per CU).  Returns 0 or B64_EARG. */
int64_t b64_tune_set_bucket(int op, int bucket, int unroll, int blocks_per_cu, int nontemporal);
/* b64_tune_set_bucket(op, -1, ...): the same shape for every size.           */
int64_t b64_tune_set(int op, int unroll, int blocks_per_cu, int nontemporal);
/* Shape of `op` in `bucket` packed as nontemporal*10000 + unroll*100 +
 * blocks_per_cu, or B64_EARG.                                                */
int64_t b64_tune_get_bucket(int op, int bucket);
/* b64_tune_get_bucket(op, 4): the shape of the largest inputs.              */
int64_t b64_tune_get(int op);
/* Size bucket (0..4) of an input of n bytes, or B64_EARG for n < 0.          */
int64_t b64_tune_bucket(int64_t n);
/* Whitespace-skipping decode (B64_SKIP_WS): texts of at least `min_chars`
 * bytes first try decoding as regular lines (the guess), shorter ones count
 * their whitespace straight away.  min_chars >= 0 sets the size, a negative
 * value only reads it; returns the size in force before the call (default
 * 14 MiB, where the two paths cost the same on MI355X).  Process-wide, for the
 * autotuner and for tests that want either path on small texts.  Does not
 * change results.  Not a paper operation: a launch-policy knob.              */
int64_t b64_tune_ws_guess_min(int64_t min_chars);
/* Whitespace-skipping decode and validation (B64_SKIP_WS): texts of at most
 * `max_chars` bytes (0 .. 65,536; default 65,536) run in one launch of one
 * workgroup, which compacts the significant characters in LDS; longer texts
 * take the multi-launch paths above.  max_chars >= 0 sets the size, a
 * negative value only reads it; returns the size in force before the call,
 * or B64_EARG above 65,536.  Process-wide, for tests that want the
 * multi-launch paths on small texts.  Does not change results.  Not a paper
 * operation: a launch-policy knob.                                           */
int64_t b64_tune_ws_small_max(int64_t max_chars);

/* Bandwidth yardstick (not a codec operation; Section "Experiments" measures
 * the codec against a memory copy): streaming kernels with the codec kernels'
 * access pattern and grid and none of their arithmetic, over nch lane
 * chunks.  kind 0: reads 16*nch bytes of src (dst receives one word per
 * workgroup: it must hold 65,536 bytes); 1: writes 16*nch bytes of dst; 2:
 * encode's pattern, reads 12*nch and writes 16*nch; 3: decode's pattern,
 * reads 16*nch and writes 12*nch; 4: copies 16*nch bytes.  Device pointers,
 * caller-owned, sized as stated.  Asynchronous; returns 0, B64_EARG or
 * B64_EHIP. */
int64_t b64_yardstick(int kind, const uint8_t *src, uint8_t *dst, int64_t nch, hipStream_t stream);

/* Message for the last B64_EARG / B64_EHIP returned on this thread.          */
const char *b64_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* B64HIP_H */
