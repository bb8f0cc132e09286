// Dark subtraction and flat division of a stack of uint16 frames (Section 2.1/2.2).
//
// Streaming kernel: each thread owns 8 consecutive pixels of one row, loads the
// dark and flat values for them once (2 x 32 B), then walks the N frames with one
// 16 B uint16 load and two 16 B float stores per frame.  Bytes per input pixel:
// 2 (raw) + 4 (out) + 8/N (dark, flat).
#include "common.h"

namespace rd {

constexpr int CAL_VEC = 8;
constexpr int CAL_BLOCK = 256;

__global__ __launch_bounds__(CAL_BLOCK) void calibrate_vec8(
    const uint16_t *__restrict__ raw, int64_t rrp, int64_t rfp,
    const float *__restrict__ dark, const float *__restrict__ flat, int64_t crp,
    float *__restrict__ out, int32_t W, int32_t H, int32_t N)
{
    const int64_t groups_per_row = W / CAL_VEC;
    const int64_t g = (int64_t)blockIdx.x * CAL_BLOCK + threadIdx.x;
    if (g >= groups_per_row * H) return;
    const int32_t y = (int32_t)(g / groups_per_row);
    const int32_t x = (int32_t)(g - (int64_t)y * groups_per_row) * CAL_VEC;

    const float4 *dp = reinterpret_cast<const float4 *>(dark + (int64_t)y * crp + x);
    const float4 *fp = reinterpret_cast<const float4 *>(flat + (int64_t)y * crp + x);
    const float4 d0 = dp[0], d1 = dp[1], f0 = fp[0], f1 = fp[1];
    const float d[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    const float f[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};

    const uint16_t *rp = raw + (int64_t)y * rrp + x;
    float *op = out + (int64_t)y * W + x;
    const int64_t plane = (int64_t)W * H;
#pragma unroll 4
    for (int32_t k = 0; k < N; ++k) {
        const uint4 v = *reinterpret_cast<const uint4 *>(rp + (int64_t)k * rfp);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        float c[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c[2 * i] = calib_px((uint16_t)(w[i] & 0xffffu), d[2 * i], f[2 * i]);
            c[2 * i + 1] = calib_px((uint16_t)(w[i] >> 16), d[2 * i + 1], f[2 * i + 1]);
        }
        float4 *o = reinterpret_cast<float4 *>(op + (int64_t)k * plane);
        o[0] = make_float4(c[0], c[1], c[2], c[3]);
        o[1] = make_float4(c[4], c[5], c[6], c[7]);
    }
}

// Any pitch and alignment: one pixel per thread, frames looped.
__global__ __launch_bounds__(CAL_BLOCK) void calibrate_scalar(
    const uint16_t *__restrict__ raw, int64_t rrp, int64_t rfp,
    const float *__restrict__ dark, const float *__restrict__ flat, int64_t crp,
    float *__restrict__ out, int32_t W, int32_t H, int32_t N)
{
    const int64_t p = (int64_t)blockIdx.x * CAL_BLOCK + threadIdx.x;
    if (p >= (int64_t)W * H) return;
    const int32_t y = (int32_t)(p / W), x = (int32_t)(p - (int64_t)y * W);
    const float d = dark[(int64_t)y * crp + x], f = flat[(int64_t)y * crp + x];
    const int64_t plane = (int64_t)W * H;
    for (int32_t k = 0; k < N; ++k)
        out[k * plane + p] = calib_px(raw[(int64_t)k * rfp + (int64_t)y * rrp + x], d, f);
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace rd

using namespace rd;

extern "C" int reduce_calibrate(const uint16_t *raw, int64_t raw_row_pitch, int64_t raw_frame_pitch,
                                const float *dark, const float *flat, int64_t cal_row_pitch,
                                float *out, int32_t W, int32_t H, int32_t N, void *stream)
{
    if (!raw || !dark || !flat || !out) return fail(REDUCE_ERR_NULL, "reduce_calibrate: NULL buffer");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_calibrate: W, H, N must be >= 1");
    if (raw_row_pitch < W || raw_frame_pitch < raw_row_pitch * (int64_t)(H - 1) + W || cal_row_pitch < W)
        return fail(REDUCE_ERR_SHAPE, "reduce_calibrate: pitch smaller than the frame");
    hipStream_t s = as_stream(stream);
    const bool vec = (W % CAL_VEC == 0) && (raw_row_pitch % CAL_VEC == 0) && (raw_frame_pitch % CAL_VEC == 0) &&
                     (cal_row_pitch % 4 == 0) && aligned16(raw) && aligned16(dark) && aligned16(flat) &&
                     aligned16(out);
    ProfScope prof("calibrate", s);
    if (vec) {
        const int64_t groups = (int64_t)(W / CAL_VEC) * H;
        hipLaunchKernelGGL(calibrate_vec8, dim3((unsigned)ceil_div(groups, CAL_BLOCK)), dim3(CAL_BLOCK), 0, s,
                           raw, raw_row_pitch, raw_frame_pitch, dark, flat, cal_row_pitch, out, W, H, N);
    } else {
        hipLaunchKernelGGL(calibrate_scalar, dim3((unsigned)ceil_div((int64_t)W * H, CAL_BLOCK)), dim3(CAL_BLOCK), 0,
                           s, raw, raw_row_pitch, raw_frame_pitch, dark, flat, cal_row_pitch, out, W, H, N);
    }
    return check_launch("reduce_calibrate");
}
