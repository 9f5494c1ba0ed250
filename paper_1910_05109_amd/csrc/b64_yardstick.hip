// b64_yardstick.hip -- streaming kernels with the codec's memory access
// pattern and none of its arithmetic: the attainable-bandwidth ceiling the
// encode and decode kernels are measured against (Section "Experiments" uses
// a memory copy as the yardstick of a codec; these are memory copies shaped
// like the codec's own loads and stores).
//
// Every kernel runs the single-buffer kernels' grid: lane chunk c of a round
// of U chunks per lane, consecutive lanes on consecutive chunks, the loads of
// round r+1 issued before round r is stored, the same grid size (grid_for)
// and nontemporal choice as the encode kernel's shape for that size.
//   kind 0  read only:   16 bytes loaded per lane chunk, one word stored per
//                        workgroup (their XOR, so the loads stay);
//   kind 1  write only:  16 bytes stored per lane chunk;
//   kind 2  12 -> 16:    encode's pattern (12 bytes loaded, 16 stored);
//   kind 3  16 -> 12:    decode's pattern (16 bytes loaded, 12 stored);
//   kind 4  16 -> 16:    a plain copy at the same grid.
#include "b64_launch.h"
#include "b64hip.h"

namespace b64hip {
namespace {

// Round loads and stores of the pattern: RIN bytes in (0: none) and WOUT
// bytes out (0: none, the XOR kept instead) per lane chunk.
template <int U, bool NT, int RIN>
__device__ __forceinline__ void yard_load(u32x4 (&v)[U], const uint8_t *s, int64_t c0,
                                          int64_t stride, int64_t nch)
{
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int64_t c = c0 + j * stride;
        const int64_t cc = c < nch ? c : nch - 1;
        if constexpr (RIN == 12) {
            const u32x3 w = load12<NT>(s + 12 * cc);
            v[j] = u32x4{w.x, w.y, w.z, w.x ^ w.z};
        } else if constexpr (RIN == 16) {
            v[j] = load16<NT>(s + 16 * cc);
        } else {
            v[j] = u32x4{(uint32_t)c, (uint32_t)(c >> 32), (uint32_t)j, 0x3D3D3D3Du};
        }
    }
}
template <int U, bool NT, int WOUT, bool GUARD>
__device__ __forceinline__ void yard_store(const u32x4 (&v)[U], uint8_t *d, int64_t c0,
                                           int64_t stride, int64_t nch, uint32_t &acc)
{
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int64_t c = c0 + j * stride;
        if (GUARD && c >= nch) continue;
        if constexpr (WOUT == 16) store16<NT>(d + 16 * c, v[j]);
        else if constexpr (WOUT == 12) store12<NT>(d + 12 * c, u32x3{v[j].x ^ v[j].w, v[j].y, v[j].z});
        else acc ^= v[j].x ^ v[j].y ^ v[j].z ^ v[j].w;
    }
}

// nch lane chunks, grid-stride in rounds of U per lane, software-pipelined as
// the codec's streams are: complete rounds alternate between two register
// sets, the loads of round r+1 issued before round r is stored; then the last,
// partial round with its loads clamped and its stores guarded.
template <int U, bool NT, int RIN, int WOUT>
__global__ __launch_bounds__(kThreads) void k_yardstick(const uint8_t *__restrict__ src,
                                                        uint8_t *__restrict__ dst, int64_t nch)
{
    const int64_t T = (int64_t)gridDim.x * kThreads;
    const int64_t t = logical_block() * kThreads + threadIdx.x;
    const int64_t rstep = U * T;
    const int64_t nfull = full_rounds(nch, rstep);
    uint32_t acc = 0;
    int64_t c0 = t;
    if (nfull > 0) {
        u32x4 A[U], B[U];
        yard_load<U, NT, RIN>(A, src, c0, T, nch);
        int64_t r = 0;
        for (; r + 2 < nfull; r += 2) {
            yard_load<U, NT, RIN>(B, src, c0 + rstep, T, nch);
            yard_store<U, NT, WOUT, false>(A, dst, c0, T, nch, acc);
            yard_load<U, NT, RIN>(A, src, c0 + 2 * rstep, T, nch);
            yard_store<U, NT, WOUT, false>(B, dst, c0 + rstep, T, nch, acc);
            c0 += 2 * rstep;
        }
        if (r + 1 < nfull) {
            yard_load<U, NT, RIN>(B, src, c0 + rstep, T, nch);
            yard_store<U, NT, WOUT, false>(A, dst, c0, T, nch, acc);
            yard_store<U, NT, WOUT, false>(B, dst, c0 + rstep, T, nch, acc);
            c0 += 2 * rstep;
        } else {
            yard_store<U, NT, WOUT, false>(A, dst, c0, T, nch, acc);
            c0 += rstep;
        }
    }
    if (c0 < nch || nfull * rstep < nch) {
        u32x4 v[U];
        yard_load<U, NT, RIN>(v, src, c0, T, nch);
        yard_store<U, NT, WOUT, true>(v, dst, c0, T, nch, acc);
    }
    if constexpr (WOUT == 0) {
        __shared__ uint32_t s_acc;
        if (threadIdx.x == 0) s_acc = 0;
        __syncthreads();
        atomicXor(&s_acc, acc);
        __syncthreads();
        if (threadIdx.x == 0) ((uint32_t *)dst)[blockIdx.x] = s_acc;
    }
}

template <int RIN, int WOUT>
hipError_t launch_kind(const uint8_t *src, uint8_t *dst, int64_t nch, Shape sh, int cus,
                       hipStream_t stream)
{
    const int64_t grid = grid_for(nch, sh, cus);
#define B64_YARD(U_)                                                                         \
    do {                                                                                    \
        if (sh.nt)                                                                          \
            (void)launch_args(&k_yardstick<U_, true, RIN, WOUT>, dim3(grid), dim3(kThreads), stream, \
                        src, dst, nch);                                                     \
        else                                                                                \
            (void)launch_args(&k_yardstick<U_, false, RIN, WOUT>, dim3(grid), dim3(kThreads), stream, \
                        src, dst, nch);                                                     \
    } while (0)
    switch (sh.unroll) {
    case 1: B64_YARD(1); break;
    case 2: B64_YARD(2); break;
    case 4: B64_YARD(4); break;
    default: B64_YARD(8); break;
    }
#undef B64_YARD
    return hipGetLastError();
}

}  // namespace
}  // namespace b64hip

using namespace b64hip;

extern "C" int64_t b64_yardstick(int kind, const uint8_t *src, uint8_t *dst, int64_t nch,
                                 hipStream_t stream)
{
    if (kind < 0 || kind > 4 || nch < 0) return B64_EARG;
    if (nch == 0) return 0;
    if ((kind != 1 && !src) || !dst) return B64_EARG;
    int cus = 0;
    hipError_t e = device_cus(&cus);
    if (e != hipSuccess) return B64_EHIP;
    // the shape of the codec kernel with this pattern (decode's for 16 -> 12,
    // encode's otherwise) for an input of the same size
    const Shape sh = kind == 3 ? op_shape(1, 16 * nch) : op_shape(0, 12 * nch);
    switch (kind) {
    case 0: e = launch_kind<16, 0>(src, dst, nch, sh, cus, stream); break;
    case 1: e = launch_kind<0, 16>(src, dst, nch, sh, cus, stream); break;
    case 2: e = launch_kind<12, 16>(src, dst, nch, sh, cus, stream); break;
    case 3: e = launch_kind<16, 12>(src, dst, nch, sh, cus, stream); break;
    default: e = launch_kind<16, 16>(src, dst, nch, sh, cus, stream); break;
    }
    return e == hipSuccess ? 0 : B64_EHIP;
}
