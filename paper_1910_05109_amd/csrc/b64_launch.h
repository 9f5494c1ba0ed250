// b64_launch.h -- host-side launchers shared by the C ABI (b64_abi.hip) and
// the kernel translation units (b64_single.hip, b64_batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <tuple>
#include <utility>

#include "b64_device.h"

namespace b64hip {

// Launch shape: lane chunks in flight per lane, workgroups per CU, and
// whether streaming loads / stores carry the nontemporal hint.
struct Shape { int unroll, bpc, nt; };

// An alphabet must be invertible and may not contain the pad character.
inline bool alphabet_ok(const char *alphabet)
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

// The kernel-argument tables of an alphabet: its 64 bytes (encode), and the
// 256-entry map from byte to value or kBad (decode).
inline EncTab make_enc(const char *alphabet)
{
    EncTab t;
    for (int i = 0; i < 16; ++i)
        t.w[i] = (uint32_t)(uint8_t)alphabet[4 * i] | (uint32_t)(uint8_t)alphabet[4 * i + 1] << 8 |
                 (uint32_t)(uint8_t)alphabet[4 * i + 2] << 16 |
                 (uint32_t)(uint8_t)alphabet[4 * i + 3] << 24;
    return t;
}

inline DecMap make_dec(const char *alphabet)
{
    DecMap d;
    uint8_t b[256];
    for (int i = 0; i < 256; ++i) b[i] = (uint8_t)kBad;
    for (int v = 0; v < 64; ++v) b[(uint8_t)alphabet[v]] = (uint8_t)v;
    for (int i = 0; i < 64; ++i)
        d.w[i] = (uint32_t)b[4 * i] | (uint32_t)b[4 * i + 1] << 8 | (uint32_t)b[4 * i + 2] << 16 |
                 (uint32_t)b[4 * i + 3] << 24;
    return d;
}

// The shape the library holds for operation `op` (the numbering of
// b64_tune_set) and an input of n bytes (n < 0: the largest size bucket), and
// the compute units of the current device.
Shape op_shape(int op, int64_t n);
hipError_t device_cus(int *cus);

// Blocks for a grid-stride launch over `nch` lane chunks: enough to cover
// them with `unroll` chunks per lane if that takes at most `bpc` per CU, else
// `bpc` per CU; a whole number per XCD.
int64_t grid_for(int64_t nch, Shape sh, int cus);

// `flags` carries kFlagNoPad (the other variant flags have kernels of their own).
hipError_t launch_encode(const uint8_t *src, int64_t n, uint8_t *dst, const EncTab &tab, uint32_t flags,
                         Shape sh, int cus, hipStream_t stream);
// Single-buffer decode (k_decode only), result in `sink`: in the raw form
// *first_bad must hold kNoError before it, and afterwards holds the first
// invalid offset or still kNoError, and *out_len the decoded length when the
// input is valid; in the slot form the launch leaves the public form.
// The kernel builds its map from the alphabet (`alpha`, the encode table).
hipError_t launch_decode(const uint8_t *src, int64_t n, uint8_t *dst, const EncTab &alpha,
                         const DecSink &sink, uint32_t flags, Shape sh, int cus, hipStream_t stream);
// Read-only validation (k_validate), result in `sink` as for launch_decode.
hipError_t launch_validate(const uint8_t *src, int64_t n, const EncTab &alpha, const DecSink &sink,
                           uint32_t flags, Shape sh, int cus, hipStream_t stream);
// Device address of status slot `idx` (0 <= idx < kStatusSlots) of the
// current device: kSlotWords int64 words, zero between calls (the slot form
// of DecSink).
constexpr int kStatusSlots = 1024;
hipError_t status_slot_addr(int idx, int64_t **out);
hipError_t launch_fill(int64_t *p, int64_t count, int64_t value, hipStream_t stream);
hipError_t launch_finish(int64_t *out_len, int64_t *first_bad, int64_t count, hipStream_t stream);
hipError_t launch_encode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                               uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                               const EncTab &tab, uint32_t flags, Shape sh, int cus, hipStream_t stream);
hipError_t launch_decode_batch(const uint8_t *src, const int64_t *in_off, int64_t nbuf,
                               uint8_t *dst, const int64_t *out_off, int64_t *out_len,
                               int64_t *first_bad, const DecMap &map, uint32_t flags, Shape sh,
                               int cus, hipStream_t stream);
// Line-wrapped encode (k_encode_wrap): line_len > 0, a multiple of 4.
hipError_t launch_encode_wrap(const uint8_t *src, int64_t n, uint8_t *dst, const EncTab &tab,
                              uint32_t flags, int64_t line_len, Shape sh, int cus, hipStream_t stream);
// Whitespace-skipping decode (`write`) or validation (!`write`, dst unused):
// five launches on `stream`, ending with the public status in *out_len and
// *first_bad.  `map` holds the codes of make_dec_ws (b64_abi.hip);
// `workspace` holds ws_workspace_bytes(n) bytes.
// Fused decode + float32 -> bfloat16 of `nrows` rows (k_decode_f32_bf16).
hipError_t launch_decode_f32_bf16(const uint8_t *src, const int64_t *in_off, int64_t nrows,
                                  int64_t dim, uint16_t *dst, int64_t *status, const DecMap &map,
                                  uint32_t flags, Shape sh, int cus, hipStream_t stream);
int64_t ws_tile_size(int64_t n);
int64_t ws_workspace_bytes(int64_t n);
// Texts of at most small_max (<= kWsSmallMax) characters take one launch of
// one workgroup (k_ws_small); longer ones the counted path, after the guess
// of regular lines from guess_min characters on.
constexpr int64_t kWsSmallMax = 64 << 10;
hipError_t launch_decode_ws(const uint8_t *src, int64_t n, uint8_t *dst, bool write, const DecMap &map,
                            int64_t *out_len, int64_t *first_bad, uint32_t flags, void *workspace,
                            Shape sh, int cus, int64_t guess_min, int64_t small_max,
                            hipStream_t stream);

}  // namespace b64hip

// Launches `kernel` through hipLaunchKernel with an array of argument
// addresses, each argument first converted to the kernel's parameter type.
// On MI355X hosts this enqueues a launch of the codec's kernels about 0.4 us
// faster than hipLaunchKernelGGL; a small call costs about as much on the
// host as on the GPU, so this shows in every latency-bound call.
template <class... P, class... A>
inline hipError_t launch_args(void (*kernel)(P...), dim3 grid, dim3 block, hipStream_t stream,
                              A &&...a)
{
    static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
    std::tuple<P...> args(static_cast<P>(std::forward<A>(a))...);
    return std::apply(
        [&](auto &...x) {
            void *p[] = {(void *)&x...};
            return hipLaunchKernel((const void *)kernel, grid, block, p, 0, stream);
        },
        args);
}

// (the launchers return hipGetLastError(), which also holds a launch error)
#define B64_LAUNCH(KERNEL, U_, NT_, GRID, STREAM, ...) \
    (void)launch_args(&KERNEL<U_, NT_>, dim3(GRID), dim3(kThreads), STREAM, __VA_ARGS__)
#define B64_DISPATCH_NT(KERNEL, U_, SH, GRID, STREAM, ...)                      \
    do {                                                                       \
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
