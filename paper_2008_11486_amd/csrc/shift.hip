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

// Grid (ceil(w / 2048), h, N): a thread checks 8 consecutive outputs of a row against
// the bad-pixel map (the bytes of one mask row serve all 8), and writes only the outputs
// that read a bad pixel.
constexpr int MASK_PX = 8;

__global__ __launch_bounds__(256) void mask_shifted_kernel(const uint8_t *__restrict__ mask, float *__restrict__ out,
                                                           int32_t W, int32_t H, const float *__restrict__ offs,
                                                           int32_t x0, int32_t y0, int32_t w, int32_t h,
                                                           int integer)
{
    const int32_t u0 = (blockIdx.x * 256 + threadIdx.x) * MASK_PX, v = blockIdx.y, k = blockIdx.z;
    if (u0 >= w) return;
    const ShiftSetup ss = shift_setup(offs[2 * k], offs[2 * k + 1]);
    const bool sx = !integer && ss.a > 0.0, sy = !integer && ss.b > 0.0;
    const int32_t j = clampi(y0 + v + ss.iy, 0, H - 1);
    const int32_t j1 = sy ? clampi(j + 1, 0, H - 1) : j;
    const uint8_t *r0 = mask + (int64_t)j * W, *r1 = mask + (int64_t)j1 * W;
    // column c = x0 + u0 + ix + e, e = 0 .. MASK_PX: bad if either tap row has it
    uint32_t bad = 0;
#pragma unroll
    for (int e = 0; e <= MASK_PX; ++e) {
        const int32_t c = clampi(x0 + u0 + ss.ix + e, 0, W - 1);
        bad |= (uint32_t)((r0[c] | r1[c]) != 0) << e;
    }
    if (!bad) return;
    float *row = out + ((int64_t)k * h + v) * w;
#pragma unroll
    for (int e = 0; e < MASK_PX; ++e) {
        // output u0 + e reads the clamped columns of bits e and, when the x fraction is
        // non-zero, e + 1
        const bool hit = ((bad >> e) & 1u) || (sx && ((bad >> (e + 1)) & 1u));
        if (u0 + e < w && hit) row[u0 + e] = __builtin_nanf("");
    }
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
    dim3 grid((unsigned)ceil_div(w, (int64_t)SH_BLOCK * SH_VEC), (unsigned)ceil_div(h, SH_ROWS), (unsigned)N);
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
    hipLaunchKernelGGL(mask_shifted_kernel, dim3((unsigned)ceil_div(w, 256 * MASK_PX), (unsigned)h, (unsigned)N),
                       dim3(256), 0, s, mask, out, W, H, offs, x0, y0, w, h, integer_mode ? 1 : 0);
    return check_launch("reduce_mask_shifted");
}
