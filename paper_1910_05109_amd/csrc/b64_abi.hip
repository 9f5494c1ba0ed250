// b64_abi.hip -- the C ABI of libb64hip.so (declared in include/b64hip.h):
// argument checks, the alphabet tables passed to the kernels, launch shapes,
// per-device queries and the blocking decode's status slot.
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <unordered_map>

#include "b64_launch.h"
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

using namespace b64hip;

// Device scratch of b64_decode_ws_async_noalloc: the workspace of the
// whitespace-skipping decode as a fixed array of device memory, one copy per
// device, held until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: its address on each device comes
// from hipGetSymbolAddress (scratch_ptr below), and only that address is
// passed to kernels.
constexpr int64_t kScratchBytes = 1 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

thread_local char g_err[256];

int64_t fail(int64_t code, const char *msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

int64_t hip_fail(hipError_t e, const char *where)
{
    snprintf(g_err, sizeof g_err, "%s: %s", where, hipGetErrorString(e));
    return B64_EHIP;
}

bool is_ws(uint8_t c) { return c == ' ' || c == '\t' || c == '\r' || c == '\n'; }

// Codes of the whitespace-skipping kernels: alphabet values, 0x40 for the four
// ignored bytes, 0x81 for '=' (padded mode), 0x80 for every other byte.
DecMap make_dec_ws(const char *alphabet, bool nopad)
{
    DecMap d;
    uint8_t *b = (uint8_t *)d.w;
    memset(b, 0x80, 256);
    b[' '] = b['\t'] = b['\r'] = b['\n'] = 0x40;
    if (!nopad) b[kPad] = 0x81;
    for (int v = 0; v < 64; ++v) b[(uint8_t)alphabet[v]] = (uint8_t)v;
    return d;
}

// Launch shapes per operation (encode, decode, encode_batch, decode_batch,
// validate, line-wrapped encode, whitespace-skipping decode, fused float32 ->
// bfloat16 decode) and size bucket of the operation's input: below 64 KiB
// and below 1 MiB (launch-latency bound; the smallest inputs can take a grid
// of one workgroup, which skips the decode status count), below 16 MiB and
// below 128 MiB (resident in the L2 and last-level caches), and from 128 MiB
// (HBM streaming).  The batched
// and fused operations find their total size only on the device and always
// take the last bucket's shape.  The defaults are the autotuner's choices on
// MI355X (python -m paper_1910_05109_amd.tune: each shape timed on three
// sizes spread over each of the first four buckets -- 4 / 16 / 48 KiB,
// 96 / 256 / 768 KiB, 2 / 4 / 12 MiB, 24 / 48 / 96 MiB -- and on 1 GiB for
// the last; the lowest mean time relative to the fastest shape at each size,
// averaged over two sweeps where the code was the same in both).
constexpr int kOps = 8;
constexpr int kBuckets = 5;
constexpr int64_t kBucketLimit[kBuckets - 1] = {64 << 10, 1 << 20, 16 << 20, 128 << 20};
Shape g_shape[kOps][kBuckets] = {
    {{1, 4, 0}, {1, 4, 0}, {2, 4, 0}, {1, 8, 0}, {8, 1, 1}},      // encode
    {{1, 2, 1}, {1, 32, 0}, {1, 4, 0}, {1, 4, 0}, {2, 2, 1}},     // decode
    {{2, 2, 1}, {2, 2, 1}, {2, 2, 1}, {2, 2, 1}, {2, 2, 1}},      // encode_batch
    {{4, 16, 1}, {4, 16, 1}, {4, 16, 1}, {4, 16, 1}, {4, 16, 1}}, // decode_batch
    {{2, 64, 0}, {2, 32, 0}, {1, 4, 0}, {1, 4, 0}, {2, 2, 1}},    // validate
    {{1, 8, 0}, {1, 64, 0}, {1, 8, 0}, {2, 64, 0}, {8, 1, 0}},    // line-wrapped encode
    {{2, 12, 0}, {2, 8, 0}, {2, 16, 0}, {1, 2, 1}, {2, 8, 1}},    // whitespace-skipping decode
    {{2, 64, 1}, {2, 64, 1}, {2, 64, 1}, {2, 64, 1}, {2, 64, 1}}, // fused decode
};
std::mutex g_mu;

int bucket_of(int64_t n)
{
    int b = 0;
    while (b < kBuckets - 1 && n >= kBucketLimit[b]) ++b;
    return b;
}

// Texts of at least this many bytes try the regular-line guess in the
// whitespace-skipping decode; shorter ones take the counted path alone.  On
// MI355X the two cross near 14 MB of MIME text (5.7 MB: 0.035 ms counted
// only against 0.042 ms with the guess; 23 MB: 0.052 against 0.045 ms).
constexpr int64_t kWsGuessMin = 14 << 20;
std::atomic<int64_t> g_ws_guess_min{kWsGuessMin};
std::atomic<int64_t> g_ws_small_max{kWsSmallMax};

// Shape of `op` for an input of n bytes (n < 0: the last bucket).
Shape shape_of(int op, int64_t n)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_shape[op][n < 0 ? kBuckets - 1 : bucket_of(n)];
}

}  // namespace

Shape b64hip::op_shape(int op, int64_t n) { return shape_of(op, n); }

namespace {

constexpr int kMaxDevices = 64;
// Compute units per device, asked once (threads may race to ask; they store
// the same value).
int g_cus[kMaxDevices];

hipError_t cu_count(int *cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    int c = __atomic_load_n(&g_cus[dev], __ATOMIC_RELAXED);
    if (c == 0) {
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        c = v > 0 ? v : 1;
        __atomic_store_n(&g_cus[dev], c, __ATOMIC_RELAXED);
    }
    *cus = c;
    return hipSuccess;
}

// Per thread and device: 2 int64 of device memory and of pinned host memory
// for the blocking b64_decode (held until the process ends).
struct StatusSlot { int64_t *d = nullptr; int64_t *h = nullptr; };
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
    }
    *out = &s;
    return hipSuccess;
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

hipError_t scratch_ptr(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t b64hip::device_cus(int *cus) { return cu_count(cus); }

namespace {

const char *const kBadAlphabet = "alphabet must be 64 distinct bytes without '='";

constexpr uint32_t kFlagsAll = kFlagNoPad | kFlagSkipWs;

// Argument checks shared by the decode / validate entry points; returns 0 or
// an error code with the message set.
int64_t check_decode_args(int64_t n, const char *alphabet, uint32_t flags)
{
    if (n < 0) return fail(B64_EARG, "negative length");
    if (flags & ~kFlagsAll) return fail(B64_EARG, "unknown flags");
    if (!alphabet_ok(alphabet)) return fail(B64_EARG, kBadAlphabet);
    if (flags & kFlagSkipWs)
        for (int v = 0; v < 64; ++v)
            if (is_ws((uint8_t)alphabet[v]))
                return fail(B64_EARG, "B64_SKIP_WS needs an alphabet without space, tab, CR or LF");
    return 0;
}

// Per thread and device: the device workspace of the blocking
// whitespace-skipping decode / validate, grown as needed (held until the
// process ends).
struct WsCache { void *d = nullptr; int64_t bytes = 0; };
thread_local WsCache g_ws[kMaxDevices];

hipError_t ws_cache(int64_t bytes, void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    WsCache &c = g_ws[dev];
    if (c.bytes < bytes) {
        if (c.d) {
            e = hipFree(c.d);
            if (e != hipSuccess) return e;
            c.d = nullptr;
            c.bytes = 0;
        }
        const int64_t want = bytes < 4096 ? 4096 : bytes;
        e = hipMalloc(&c.d, (size_t)want);
        if (e != hipSuccess) return e;
        c.bytes = want;
    }
    *out = c.d;
    return hipSuccess;
}

// Status slots of the single-launch decode / validation.  Work on one stream
// runs in order, so a stream's calls never overlap and can share one slot; the
// slot is back to zero after each call.  hipStreamPerThread names a different
// stream on every thread, so it gets a slot per thread.  Decodes captured into
// a graph get a slot per capture and capturing stream: the nodes captured from
// one stream run in order within a replay, and launches of one graph run one
// after another, so they never overlap either.  Slots are never given back (a
// slot is 4,224 bytes of device memory); once all kStatusSlots of a device are
// taken, further streams and captures use the three-launch form.
struct SlotTable {
    std::mutex mu;
    std::unordered_map<hipStream_t, int> idx;
    std::unordered_map<unsigned long long, std::unordered_map<hipStream_t, int>> captured;
    int next = 0;
};
SlotTable g_slot_tables[kMaxDevices];
thread_local int g_per_thread_slot[kMaxDevices];   // slot index + 1, 0 = none yet

// The status slot for a call on `stream` on the current device, or nullptr
// when every slot is taken (or the stream's capture has been invalidated).
int64_t *stream_slot(hipStream_t stream)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    unsigned long long capture_id = 0;
    if (hipStreamGetCaptureInfo(stream, &cs, &capture_id) != hipSuccess ||
        cs == hipStreamCaptureStatusInvalidated)
        return nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    SlotTable &t = g_slot_tables[dev];
    int idx = -1;
    if (cs == hipStreamCaptureStatusActive) {
        std::lock_guard<std::mutex> lk(t.mu);
        auto &per_stream = t.captured[capture_id];
        auto it = per_stream.find(stream);
        if (it != per_stream.end()) {
            idx = it->second;
        } else if (t.next < kStatusSlots) {
            idx = t.next++;
            per_stream.emplace(stream, idx);
        }
    } else if (stream == hipStreamPerThread) {
        if (!g_per_thread_slot[dev]) {
            std::lock_guard<std::mutex> lk(t.mu);
            if (t.next < kStatusSlots) g_per_thread_slot[dev] = ++t.next;
        }
        idx = g_per_thread_slot[dev] - 1;
    } else {
        std::lock_guard<std::mutex> lk(t.mu);
        auto it = t.idx.find(stream);
        if (it != t.idx.end()) {
            idx = it->second;
        } else if (t.next < kStatusSlots) {
            idx = t.next++;
            t.idx.emplace(stream, idx);
        }
    }
    if (idx < 0) return nullptr;
    int64_t *p = nullptr;
    return status_slot_addr(idx, &p) == hipSuccess ? p : nullptr;
}

// Enqueue one single-buffer decode (`write`) or validation (!`write`, dst
// unused), leaving the public status in *out_len / *first_bad.  Without
// B64_SKIP_WS and with a status slot (`sslot`, from stream_slot) this is one
// launch; without a slot it is three: reset first_bad, run k_decode /
// k_validate, turn the raw status into the public form.  With B64_SKIP_WS the
// whitespace path runs its own launches.
int64_t decode_enqueue(const uint8_t *src, int64_t n, uint8_t *dst, bool write, int64_t *out_len,
                       int64_t *first_bad, const char *alphabet, uint32_t flags, void *workspace,
                       int64_t *sslot, hipStream_t stream)
{
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    if (flags & kFlagSkipWs) {
        e = launch_decode_ws(src, n, dst, write, make_dec_ws(alphabet, flags & kFlagNoPad), out_len,
                             first_bad, flags, workspace, shape_of(6, n), cus,
                             g_ws_guess_min.load(std::memory_order_relaxed),
                             g_ws_small_max.load(std::memory_order_relaxed), stream);
        return e == hipSuccess ? 0 : hip_fail(e, "whitespace decode launch");
    }
    if (!sslot) {
        e = launch_fill(first_bad, 1, kNoError, stream);
        if (e != hipSuccess) return hip_fail(e, "fill launch");
    }
    const DecSink sink{out_len, first_bad, sslot};
    if (write)
        e = launch_decode(src, n, dst, make_enc(alphabet), sink, flags, shape_of(1, n), cus, stream);
    else
        e = launch_validate(src, n, make_enc(alphabet), sink, flags, shape_of(4, n), cus, stream);
    if (e != hipSuccess) return hip_fail(e, write ? "decode launch" : "validate launch");
    if (!sslot) {
        e = launch_finish(out_len, first_bad, 1, stream);
        if (e != hipSuccess) return hip_fail(e, "status launch");
    }
    return 0;
}

// Blocking decode / validation: returns the length, ~first_invalid_offset, or
// an error code.  With a status slot the kernel writes the public status
// straight into the per-thread pinned host words (one launch, then the
// stream is synchronized); otherwise the status goes to the per-thread device
// words and is copied back.
int64_t decode_blocking(const uint8_t *src, int64_t n, uint8_t *dst, bool write,
                        const char *alphabet, uint32_t flags, hipStream_t stream)
{
    StatusSlot *slot = nullptr;
    hipError_t e = status_slot(&slot);
    if (e != hipSuccess) return hip_fail(e, "status slot");
    void *ws = nullptr;
    int64_t *sslot = nullptr;
    if (flags & kFlagSkipWs) {
        e = ws_cache(ws_workspace_bytes(n), &ws);
        if (e != hipSuccess) return hip_fail(e, "workspace");
    } else {
        sslot = stream_slot(stream);
    }
    int64_t *words = sslot ? slot->h : slot->d;
    const int64_t r = decode_enqueue(src, n, dst, write, words, words + 1, alphabet, flags, ws,
                                     sslot, stream);
    if (r) return r;
    if (!sslot) {
        e = hipMemcpyAsync(slot->h, slot->d, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return hip_fail(e, "status copy");
    }
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    const int64_t len = ((volatile int64_t *)slot->h)[0], bad = ((volatile int64_t *)slot->h)[1];
    return bad == -1 ? len : ~bad;
}

}  // namespace

extern "C" {

int64_t b64_encoded_len(int64_t n)
{
    if (n < 0) return fail(B64_EARG, "negative length");
    return 4 * ((n + 2) / 3);
}

int64_t b64_decoded_max_len(int64_t n)
{
    if (n < 0) return fail(B64_EARG, "negative length");
    return 3 * (n / 4);
}

int64_t b64_encoded_len_mode(int64_t n, uint32_t flags, int64_t line_len)
{
    if (n < 0) return fail(B64_EARG, "negative length");
    if (flags & ~kFlagNoPad) return fail(B64_EARG, "encode takes no flag but B64_NOPAD");
    if (line_len < 0 || (line_len & 3)) return fail(B64_EARG, "line_len must be 0 or a positive multiple of 4");
    int64_t m = (flags & kFlagNoPad) ? (4 * n + 2) / 3 : 4 * ((n + 2) / 3);
    if (line_len > 0 && m > 0) m += 2 * ((m - 1) / line_len);
    return m;
}

int64_t b64_decoded_max_len_mode(int64_t n, uint32_t flags)
{
    if (n < 0) return fail(B64_EARG, "negative length");
    if (flags & ~kFlagsAll) return fail(B64_EARG, "unknown flags");
    const int64_t r = n & 3;
    return 3 * (n / 4) + ((flags & kFlagNoPad) && r > 1 ? r - 1 : 0);
}

int64_t b64_decode_workspace_size(int64_t n, uint32_t flags)
{
    if (n < 0) return fail(B64_EARG, "negative length");
    if (flags & ~kFlagsAll) return fail(B64_EARG, "unknown flags");
    return (flags & kFlagSkipWs) ? ws_workspace_bytes(n) : 0;
}

const char *b64_last_error(void) { return g_err; }

int64_t b64_tune_set_bucket(int op, int bucket, int unroll, int blocks_per_cu, int nontemporal)
{
    if (op < 0 || op >= kOps) return fail(B64_EARG, "bad op");
    if (bucket < -1 || bucket >= kBuckets) return fail(B64_EARG, "bad size bucket");
    if (!(unroll == 1 || unroll == 2 || unroll == 4 || unroll == 8))
        return fail(B64_EARG, "unroll must be 1, 2, 4 or 8");
    if (blocks_per_cu < 1 || blocks_per_cu > 64) return fail(B64_EARG, "blocks_per_cu out of range");
    if (nontemporal != 0 && nontemporal != 1) return fail(B64_EARG, "nontemporal must be 0 or 1");
    std::lock_guard<std::mutex> lk(g_mu);
    for (int b = 0; b < kBuckets; ++b)
        if (bucket < 0 || b == bucket) g_shape[op][b] = Shape{unroll, blocks_per_cu, nontemporal};
    return 0;
}

int64_t b64_tune_set(int op, int unroll, int blocks_per_cu, int nontemporal)
{
    return b64_tune_set_bucket(op, -1, unroll, blocks_per_cu, nontemporal);
}

int64_t b64_tune_bucket(int64_t n)
{
    if (n < 0) return fail(B64_EARG, "negative length");
    return bucket_of(n);
}

int64_t b64_tune_ws_small_max(int64_t max_chars)
{
    if (max_chars > kWsSmallMax) return fail(B64_EARG, "max_chars above the one-workgroup limit (65,536)");
    if (max_chars < 0) return g_ws_small_max.load(std::memory_order_relaxed);
    return g_ws_small_max.exchange(max_chars, std::memory_order_relaxed);
}

int64_t b64_tune_ws_guess_min(int64_t min_chars)
{
    if (min_chars < 0) return g_ws_guess_min.load(std::memory_order_relaxed);
    return g_ws_guess_min.exchange(min_chars, std::memory_order_relaxed);
}

int64_t b64_tune_get_bucket(int op, int bucket)
{
    if (op < 0 || op >= kOps) return fail(B64_EARG, "bad op");
    if (bucket < 0 || bucket >= kBuckets) return fail(B64_EARG, "bad size bucket");
    std::lock_guard<std::mutex> lk(g_mu);
    const Shape s = g_shape[op][bucket];
    return (int64_t)s.nt * 10000 + (int64_t)s.unroll * 100 + s.bpc;
}

int64_t b64_tune_get(int op) { return b64_tune_get_bucket(op, kBuckets - 1); }

int64_t b64_encode_mode(const uint8_t *src, int64_t n, uint8_t *dst, const char *alphabet,
                        uint32_t flags, int64_t line_len, hipStream_t stream)
{
    const int64_t m = b64_encoded_len_mode(n, flags, line_len);
    if (m < 0) return m;
    if (n > 0 && (!src || !dst)) return fail(B64_EARG, "null buffer");
    if (!alphabet_ok(alphabet)) return fail(B64_EARG, kBadAlphabet);
    if (n == 0) return 0;
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    if (line_len > 0 && line_len < m)
        e = launch_encode_wrap(src, n, dst, make_enc(alphabet), flags, line_len, shape_of(5, n), cus,
                               stream);
    else
        e = launch_encode(src, n, dst, make_enc(alphabet), flags, shape_of(0, n), cus, stream);
    if (e != hipSuccess) return hip_fail(e, "encode launch");
    return m;
}

int64_t b64_encode(const uint8_t *src, int64_t n, uint8_t *dst, const char *alphabet,
                   hipStream_t stream)
{
    return b64_encode_mode(src, n, dst, alphabet, 0, 0, stream);
}

int64_t b64_decode_mode_async(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *out_len,
                              int64_t *first_bad, const char *alphabet, uint32_t flags,
                              void *workspace, int64_t workspace_bytes, hipStream_t stream)
{
    const int64_t c = check_decode_args(n, alphabet, flags);
    if (c) return c;
    if ((n > 0 && (!src || !dst)) || !out_len || !first_bad) return fail(B64_EARG, "null pointer");
    if ((flags & kFlagSkipWs) && (!workspace || workspace_bytes < ws_workspace_bytes(n)))
        return fail(B64_EARG, "workspace smaller than b64_decode_workspace_size");
    return decode_enqueue(src, n, dst, true, out_len, first_bad, alphabet, flags, workspace,
                          (flags & kFlagSkipWs) ? nullptr : stream_slot(stream), stream);
}

int64_t b64_decode_ws_async_noalloc(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *out_len,
                                    int64_t *first_bad, const char *alphabet, uint32_t flags,
                                    hipStream_t stream)
{
    if (!(flags & kFlagSkipWs)) return fail(B64_EARG, "b64_decode_ws_async_noalloc needs B64_SKIP_WS");
    const int64_t c = check_decode_args(n, alphabet, flags);
    if (c) return c;
    if (ws_workspace_bytes(n) > kScratchBytes)
        return fail(B64_EARG, "input longer than B64_NOALLOC_MAX_CHARS (the 1 MiB scratch array)");
    if ((n > 0 && (!src || !dst)) || !out_len || !first_bad) return fail(B64_EARG, "null pointer");
    void *ws = nullptr;
    const hipError_t e = scratch_ptr(&ws);
    if (e != hipSuccess) return hip_fail(e, "scratch address");
    return decode_enqueue(src, n, dst, true, out_len, first_bad, alphabet, flags, ws, nullptr,
                          stream);
}

int64_t b64_decode_async(const uint8_t *src, int64_t n, uint8_t *dst, int64_t *out_len,
                         int64_t *first_bad, const char *alphabet, hipStream_t stream)
{
    return b64_decode_mode_async(src, n, dst, out_len, first_bad, alphabet, 0, nullptr, 0, stream);
}

int64_t b64_decode_mode(const uint8_t *src, int64_t n, uint8_t *dst, const char *alphabet,
                        uint32_t flags, hipStream_t stream)
{
    const int64_t c = check_decode_args(n, alphabet, flags);
    if (c) return c;
    if (n > 0 && (!src || !dst)) return fail(B64_EARG, "null buffer");
    return decode_blocking(src, n, dst, true, alphabet, flags, stream);
}

int64_t b64_decode(const uint8_t *src, int64_t n, uint8_t *dst, const char *alphabet,
                   hipStream_t stream)
{
    return b64_decode_mode(src, n, dst, alphabet, 0, stream);
}

int64_t b64_validate_mode(const uint8_t *src, int64_t n, const char *alphabet, uint32_t flags,
                          hipStream_t stream)
{
    const int64_t c = check_decode_args(n, alphabet, flags);
    if (c) return c;
    if (n > 0 && !src) return fail(B64_EARG, "null buffer");
    return decode_blocking(src, n, nullptr, false, alphabet, flags, stream);
}

int64_t b64_validate(const uint8_t *src, int64_t n, const char *alphabet, hipStream_t stream)
{
    return b64_validate_mode(src, n, alphabet, 0, stream);
}

int64_t b64_validate_mode_async(const uint8_t *src, int64_t n, int64_t *out_len, int64_t *first_bad,
                                const char *alphabet, uint32_t flags, void *workspace,
                                int64_t workspace_bytes, hipStream_t stream)
{
    const int64_t c = check_decode_args(n, alphabet, flags);
    if (c) return c;
    if ((n > 0 && !src) || !out_len || !first_bad) return fail(B64_EARG, "null pointer");
    if ((flags & kFlagSkipWs) && (!workspace || workspace_bytes < ws_workspace_bytes(n)))
        return fail(B64_EARG, "workspace smaller than b64_decode_workspace_size");
    return decode_enqueue(src, n, nullptr, false, out_len, first_bad, alphabet, flags, workspace,
                          (flags & kFlagSkipWs) ? nullptr : stream_slot(stream), stream);
}

int64_t b64_validate_async(const uint8_t *src, int64_t n, int64_t *out_len, int64_t *first_bad,
                           const char *alphabet, hipStream_t stream)
{
    return b64_validate_mode_async(src, n, out_len, first_bad, alphabet, 0, nullptr, 0, stream);
}

int64_t b64_encode_batch_mode(const uint8_t *src, const int64_t *in_off, int64_t nbuf, uint8_t *dst,
                              const int64_t *out_off, int64_t *out_len, const char *alphabet,
                              uint32_t flags, hipStream_t stream)
{
    if (nbuf < 0) return fail(B64_EARG, "negative buffer count");
    if (flags & ~kFlagNoPad) return fail(B64_EARG, "batched encode takes no flag but B64_NOPAD");
    if (nbuf == 0) return 0;
    if (!src || !in_off || !dst || !out_off || !out_len) return fail(B64_EARG, "null pointer");
    if (!alphabet_ok(alphabet)) return fail(B64_EARG, kBadAlphabet);
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    e = launch_encode_batch(src, in_off, nbuf, dst, out_off, out_len, make_enc(alphabet), flags,
                            shape_of(2, -1), cus, stream);
    return e == hipSuccess ? 0 : hip_fail(e, "encode_batch launch");
}

int64_t b64_encode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf, uint8_t *dst,
                         const int64_t *out_off, int64_t *out_len, const char *alphabet,
                         hipStream_t stream)
{
    return b64_encode_batch_mode(src, in_off, nbuf, dst, out_off, out_len, alphabet, 0, stream);
}

int64_t b64_decode_batch_mode(const uint8_t *src, const int64_t *in_off, int64_t nbuf, uint8_t *dst,
                              const int64_t *out_off, int64_t *out_len, int64_t *first_bad,
                              const char *alphabet, uint32_t flags, hipStream_t stream)
{
    if (nbuf < 0) return fail(B64_EARG, "negative buffer count");
    if (flags & ~kFlagNoPad) return fail(B64_EARG, "batched decode takes no flag but B64_NOPAD");
    if (nbuf == 0) return 0;
    if (!src || !in_off || !dst || !out_off || !out_len || !first_bad)
        return fail(B64_EARG, "null pointer");
    if (!alphabet_ok(alphabet)) return fail(B64_EARG, kBadAlphabet);
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    e = launch_fill(first_bad, nbuf, kNoError, stream);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    e = launch_decode_batch(src, in_off, nbuf, dst, out_off, out_len, first_bad,
                            make_dec(alphabet), flags, shape_of(3, -1), cus, stream);
    if (e != hipSuccess) return hip_fail(e, "decode_batch launch");
    e = launch_finish(out_len, first_bad, nbuf, stream);
    return e == hipSuccess ? 0 : hip_fail(e, "status launch");
}

int64_t b64_decode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf, uint8_t *dst,
                         const int64_t *out_off, int64_t *out_len, int64_t *first_bad,
                         const char *alphabet, hipStream_t stream)
{
    return b64_decode_batch_mode(src, in_off, nbuf, dst, out_off, out_len, first_bad, alphabet, 0,
                                 stream);
}

int64_t b64_decode_f32_bf16(const uint8_t *src, const int64_t *in_off, int64_t nrows, int64_t dim,
                            uint16_t *dst, int64_t *status, const char *alphabet, uint32_t flags,
                            hipStream_t stream)
{
    if (nrows < 0 || dim < 0) return fail(B64_EARG, "negative row count or dim");
    if (flags & ~kFlagNoPad) return fail(B64_EARG, "fused decode takes no flag but B64_NOPAD");
    if (nrows == 0) return 0;
    if (!src || !in_off || (dim > 0 && !dst) || !status) return fail(B64_EARG, "null pointer");
    if (!alphabet_ok(alphabet)) return fail(B64_EARG, kBadAlphabet);
    int cus = 0;
    hipError_t e = cu_count(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    e = launch_decode_f32_bf16(src, in_off, nrows, dim, dst, status, make_dec(alphabet), flags,
                               shape_of(7, -1), cus, stream);
    return e == hipSuccess ? 0 : hip_fail(e, "fused decode launch");
}

}  // extern "C"
