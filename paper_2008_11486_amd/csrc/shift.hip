// Bilinear sub-pixel shift onto the common overlap (Section 3.2.1 names bilinear
// interpolation as the cheaper alternative to the paper's bicubic spline).
//
// Streaming kernel: a thread makes 4 consecutive outputs in each row of a 16-row
// strip.  The integer part of the offset is applied in integer arithmetic, the
// fraction becomes per-frame bilinear weights evaluated in double and rounded once.
// Bytes per output pixel: 4 read (a strip fetches each input row once, plus one
// extra row per strip) + 4 write.
#include "common.h"
#include "shift_core.h"

namespace rd {

template <bool INTEGER>
__global__ __launch_bounds__(SH_BLOCK) void shift_kernel(
    const float *__restrict__ in, float *__restrict__ out, int32_t W, int32_t H,
    const float *__restrict__ offs, int32_t x0, int32_t y0, int32_t w, int32_t h, int vec_store, bool aligned)
{
    const int32_t k = blockIdx.z;
    shift_strip<INTEGER, SH_VEC>(in, out, W, H, k, offs[2 * k], offs[2 * k + 1], blockIdx.y, blockIdx.x, x0, y0, w,
                                 h, (int64_t)w * h, vec_store, aligned);
}

// Grid (N * ceil(w / 8192), h), the frame index fastest: the workgroups of one output
// row of all frames run together and read the same few map rows (one frame's offset
// apart) from L2.  A thread checks 32 consecutive outputs of a row: the map bytes of the
// 33 columns they read in each tap row come in as ten 4-byte words (when the span lies
// inside the row and the rows are 4-byte aligned; byte by byte, clamped, otherwise), a
// word's four bytes become four "bad" bits, and the thread writes only the outputs
// whose taps hold a bad pixel.
constexpr int MASK_PX = 32;

// bit i (i < 4) set when byte i of v is non-zero
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t v)
{
    const uint32_t t = (v | ((v & 0x7f7f7f7fu) + 0x7f7f7f7fu)) & 0x80808080u;
    return ((t >> 7) & 1u) | ((t >> 14) & 2u) | ((t >> 21) & 4u) | ((t >> 28) & 8u);
}

// bit e (e <= MASK_PX) set when map row r is bad at column clamp(c0 + e)
__device__ __forceinline__ uint64_t bad_columns(const uint8_t *__restrict__ r, int32_t c0, int32_t W, bool words)
{
    uint64_t m = 0;
    if (words && c0 >= 0 && c0 + 40 <= W) {
        const int32_t base = c0 & ~3, off = c0 - base;
        const uint32_t *p = reinterpret_cast<const uint32_t *>(r + base);
#pragma unroll
        for (int i = 0; i < 10; ++i) m |= (uint64_t)nonzero_bytes(p[i]) << (4 * i);
        return m >> off;
    }
#pragma unroll
    for (int e = 0; e <= MASK_PX; ++e) m |= (uint64_t)(r[clampi(c0 + e, 0, W - 1)] != 0) << e;
    return m;
}

__global__ __launch_bounds__(256) void mask_shifted_kernel(const uint8_t *__restrict__ mask, float *__restrict__ out,
                                                           int32_t W, int32_t H, const float *__restrict__ offs,
                                                           int32_t x0, int32_t y0, int32_t w, int32_t h,
                                                           int32_t N, int integer)
{
    // XCD-aware order: each XCD takes a contiguous run of rows, so a row of the map is
    // fetched into one L2 rather than eight
    const int32_t lid = xcd_logical_id((int32_t)(blockIdx.y * gridDim.x + blockIdx.x), (int32_t)(gridDim.x * gridDim.y));
    const int32_t v = lid / (int32_t)gridDim.x, r = lid - v * (int32_t)gridDim.x;
    const int32_t k = r % N, xb = r / N;
    const int32_t u0 = (xb * 256 + threadIdx.x) * MASK_PX;
    if (u0 >= w) return;
    const ShiftSetup ss = shift_setup(offs[2 * k], offs[2 * k + 1]);
    const bool sx = !integer && ss.a > 0.0, sy = !integer && ss.b > 0.0;
    const int32_t j = clampi(y0 + v + ss.iy, 0, H - 1);
    const int32_t j1 = sy ? clampi(j + 1, 0, H - 1) : j;
    const bool words = (W & 3) == 0 && (reinterpret_cast<uintptr_t>(mask) & 3u) == 0;
    const int32_t c0 = x0 + u0 + ss.ix;
    uint64_t bad = bad_columns(mask + (int64_t)j * W, c0, W, words);
    if (j1 != j) bad |= bad_columns(mask + (int64_t)j1 * W, c0, W, words);
    // output e reads the clamped columns of bits e and, when the x fraction is non-zero, e + 1
    const uint32_t hit = (uint32_t)(bad | (sx ? bad >> 1 : 0ull));
    if (!hit) return;
    float *row = out + ((int64_t)k * h + v) * w;
#pragma unroll 4
    for (int e = 0; e < MASK_PX; ++e)
        if (((hit >> e) & 1u) && u0 + e < w) row[u0 + e] = __builtin_nanf("");
}

}  // namespace rd

using namespace rd;

extern "C" int reduce_shift(const float *in, float *out, int32_t W, int32_t H, int32_t N,
                            const float *offs, const int32_t *rect, int32_t integer_mode, void *stream)
{
    if (!in || !out || !offs || !rect) return fail(REDUCE_ERR_NULL, "reduce_shift: NULL argument");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_shift: W, H, N must be >= 1");
    const int32_t x0 = rect[0], y0 = rect[1], w = rect[2], h = rect[3];
    if (w < 1 || h < 1 || w > W || h > H) return fail(REDUCE_ERR_SHAPE, "reduce_shift: empty or oversized rect");
    if (N > 65535 || h > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_shift: N or h above 65535");
    const int vec_store = shift_vec_store(w, reinterpret_cast<uintptr_t>(out));
    const bool aligned = (W % 4 == 0) && ((reinterpret_cast<uintptr_t>(in) & 15u) == 0);
    const dim3 grid((unsigned)ceil_div(w, (int64_t)SH_BLOCK * SH_VEC), (unsigned)ceil_div(h, SH_ROWS), (unsigned)N);
    ProfScope prof("shift", as_stream(stream));
    hipStream_t s = as_stream(stream);
    if (integer_mode)
        hipLaunchKernelGGL(shift_kernel<true>, grid, dim3(SH_BLOCK), 0, s, in, out, W, H, offs, x0, y0, w, h,
                           vec_store, aligned);
    else
        hipLaunchKernelGGL(shift_kernel<false>, grid, dim3(SH_BLOCK), 0, s, in, out, W, H, offs, x0, y0, w,
                           h, vec_store, aligned);
    return check_launch("reduce_shift");
}

extern "C" int reduce_mask_shifted(const uint8_t *mask, float *out, int32_t W, int32_t H, int32_t N,
                                   const float *offs, const int32_t *rect, int32_t integer_mode, void *stream)
{
    if (!mask || !out || !offs || !rect) return fail(REDUCE_ERR_NULL, "reduce_mask_shifted: NULL argument");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_mask_shifted: W, H, N must be >= 1");
    const int32_t x0 = rect[0], y0 = rect[1], w = rect[2], h = rect[3];
    if (w < 1 || h < 1 || w > W || h > H)
        return fail(REDUCE_ERR_SHAPE, "reduce_mask_shifted: empty or oversized rect");
    if (N > 65535 || h > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_mask_shifted: N or h above 65535");
    hipStream_t s = as_stream(stream);
    ProfScope prof("mask_shifted", s);
    hipLaunchKernelGGL(mask_shifted_kernel, dim3((unsigned)(N * ceil_div(w, 256 * MASK_PX)), (unsigned)h), dim3(256),
                       0, s, mask, out, W, H, offs, x0, y0, w, h, N, integer_mode ? 1 : 0);
    return check_launch("reduce_mask_shifted");
}
