// Bilinear sub-pixel shift onto the common overlap (Section 3.2.1 names bilinear
// interpolation as the cheaper alternative to the paper's bicubic spline).
//
// Streaming kernel: a thread makes 4 consecutive outputs in each row of a 16-row
// strip.  The integer part of the offset is applied in integer arithmetic, the
// fraction becomes per-frame bilinear weights evaluated in double and rounded once.
// Bytes per output pixel: 4 read (a strip fetches each input row once, plus one
// extra row per strip) + 4 write.
#include "common.h"

namespace rd {

constexpr int SH_VEC = 4;
constexpr int SH_BLOCK = 256;
constexpr int SH_ROWS = 16;  // output rows per workgroup: each input row is fetched once per strip

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// The SH_VEC + 1 taps f[row][c0 + e], e = 0..SH_VEC, of one thread.  When the frame's
// rows are 16-byte aligned and the 8 floats from the aligned start lie inside the row,
// two aligned float4 loads serve all taps (the misalignment c0 & 3 is the same for
// every thread of the frame, so the select is uniform); otherwise clamped scalar loads.
__device__ __forceinline__ void load_taps(const float *__restrict__ row, int32_t c0, int32_t W, bool aligned,
                                          float (&t)[SH_VEC + 1])
{
    const int32_t al = c0 & 3;
    const int32_t b = c0 - al;
    if (aligned && b >= 0 && b + 8 <= W) {
        const float4 p = *reinterpret_cast<const float4 *>(row + b);
        const float4 q = *reinterpret_cast<const float4 *>(row + b + 4);
        const float v[8] = {p.x, p.y, p.z, p.w, q.x, q.y, q.z, q.w};
        switch (al) {
        case 0:
#pragma unroll
            for (int e = 0; e <= SH_VEC; ++e) t[e] = v[e];
            break;
        case 1:
#pragma unroll
            for (int e = 0; e <= SH_VEC; ++e) t[e] = v[e + 1];
            break;
        case 2:
#pragma unroll
            for (int e = 0; e <= SH_VEC; ++e) t[e] = v[e + 2];
            break;
        default:
#pragma unroll
            for (int e = 0; e <= SH_VEC; ++e) t[e] = v[e + 3];
            break;
        }
    } else {
#pragma unroll
        for (int e = 0; e <= SH_VEC; ++e) t[e] = row[clampi(c0 + e, 0, W - 1)];
    }
}

// Grid (x strips of SH_BLOCK * SH_VEC outputs, strips of SH_ROWS rows, frames).  A
// thread produces SH_VEC consecutive outputs in each of the strip's rows, keeping the
// lower tap row of one output row as the upper tap row of the next.
template <bool INTEGER>
__global__ __launch_bounds__(SH_BLOCK) void shift_kernel(
    const float *__restrict__ in, float *__restrict__ out, int32_t W, int32_t H,
    const float *__restrict__ offs, int32_t x0, int32_t y0, int32_t w, int32_t h, bool vec_store, bool aligned)
{
    const int32_t k = blockIdx.z;
    const int32_t v0 = blockIdx.y * SH_ROWS;
    const int32_t v1 = min(v0 + SH_ROWS, h);
    const int32_t u0 = (blockIdx.x * SH_BLOCK + threadIdx.x) * SH_VEC;
    if (u0 >= w) return;
    const ShiftSetup ss = shift_setup(offs[2 * k], offs[2 * k + 1]);
    const float *f = in + (int64_t)k * W * H;
    const int32_t c0 = x0 + u0 + ss.ix;
    const bool step = ss.a > 0.0;
    const bool down = ss.b > 0.0;
    float t0[SH_VEC + 1], t1[SH_VEC + 1];
    int32_t jt = -1;  // row held in t1
    for (int32_t v = v0; v < v1; ++v) {
        const int32_t j = clampi(y0 + v + ss.iy, 0, H - 1);
        float r[SH_VEC];
        if (INTEGER) {
            load_taps(f + (int64_t)j * W, c0, W, aligned, t0);
#pragma unroll
            for (int e = 0; e < SH_VEC; ++e) r[e] = t0[e];
        } else {
            if (jt == j) {
#pragma unroll
                for (int e = 0; e <= SH_VEC; ++e) t0[e] = t1[e];
            } else {
                load_taps(f + (int64_t)j * W, c0, W, aligned, t0);
            }
            const int32_t j1 = clampi(down ? j + 1 : j, 0, H - 1);
            load_taps(f + (int64_t)j1 * W, c0, W, aligned, t1);
            jt = j1;
#pragma unroll
            for (int e = 0; e < SH_VEC; ++e) {
                // the right-hand tap is the next column only when it carries weight
                const float f10 = step ? t0[e + 1] : t0[e];
                const float f11 = step ? t1[e + 1] : t1[e];
                r[e] = bilerp(ss.a, ss.b, t0[e], f10, t1[e], f11);
            }
        }
        float *o = out + ((int64_t)k * h + v) * w;
        if (vec_store && u0 + SH_VEC <= w) {
            *reinterpret_cast<float4 *>(o + u0) = make_float4(r[0], r[1], r[2], r[3]);
        } else {
#pragma unroll
            for (int e = 0; e < SH_VEC; ++e)
                if (u0 + e < w) o[u0 + e] = r[e];
        }
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
    const bool vec_store = (w % SH_VEC == 0) && ((reinterpret_cast<uintptr_t>(out) & 15u) == 0);
    const bool aligned = (W % 4 == 0) && ((reinterpret_cast<uintptr_t>(in) & 15u) == 0);
    dim3 grid((unsigned)ceil_div(w, (int64_t)SH_BLOCK * SH_VEC), (unsigned)ceil_div(h, SH_ROWS), (unsigned)N);
    ProfScope prof("shift", as_stream(stream));
    if (integer_mode)
        hipLaunchKernelGGL(shift_kernel<true>, grid, dim3(SH_BLOCK), 0, as_stream(stream), in, out, W, H, offs, x0,
                           y0, w, h, vec_store, aligned);
    else
        hipLaunchKernelGGL(shift_kernel<false>, grid, dim3(SH_BLOCK), 0, as_stream(stream), in, out, W, H, offs, x0,
                           y0, w, h, vec_store, aligned);
    return check_launch("reduce_shift");
}
