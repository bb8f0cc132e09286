// Bias and dark subtraction and flat division of a stack of uint16 frames (Section
// 2.1/2.2).
//
// Streaming kernel: each thread owns 8 consecutive pixels of one row, loads the
// dark and flat values for them once (2 x 32 B), then walks the N frames with one
// 16 B uint16 load and two 16 B float stores per frame.  Bytes per input pixel:
// 2 (raw) + 4 (out) + 8/N (dark, flat).
#include "calibrate_core.h"
#include "common.h"

namespace rd {

__global__ __launch_bounds__(CAL_BLOCK) void calibrate_vec8(
    const uint16_t *__restrict__ raw, int64_t rrp, int64_t rfp, const float *__restrict__ bias,
    const float *__restrict__ dark, const float *__restrict__ flat, int64_t crp,
    float *__restrict__ out, int32_t W, int32_t H, int32_t N)
{
    calibrate_group8(raw, rrp, rfp, bias, dark, flat, crp, out, W, H, N,
                     (int64_t)blockIdx.x * CAL_BLOCK + threadIdx.x);
}

__global__ __launch_bounds__(CAL_BLOCK) void calibrate_scalar(
    const uint16_t *__restrict__ raw, int64_t rrp, int64_t rfp, const float *__restrict__ bias,
    const float *__restrict__ dark, const float *__restrict__ flat, int64_t crp,
    float *__restrict__ out, int32_t W, int32_t H, int32_t N)
{
    calibrate_pixel(raw, rrp, rfp, bias, dark, flat, crp, out, W, H, N,
                    (int64_t)blockIdx.x * CAL_BLOCK + threadIdx.x);
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace rd

using namespace rd;

extern "C" int reduce_calibrate(const uint16_t *raw, int64_t raw_row_pitch, int64_t raw_frame_pitch,
                                const float *bias, const float *dark, const float *flat, int64_t cal_row_pitch,
                                float *out, int32_t W, int32_t H, int32_t N, void *stream)
{
    if (!raw || !dark || !flat || !out) return fail(REDUCE_ERR_NULL, "reduce_calibrate: NULL buffer");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_calibrate: W, H, N must be >= 1");
    if (raw_row_pitch < W || raw_frame_pitch < raw_row_pitch * (int64_t)(H - 1) + W || cal_row_pitch < W)
        return fail(REDUCE_ERR_SHAPE, "reduce_calibrate: pitch smaller than the frame");
    hipStream_t s = as_stream(stream);
    const bool vec = (W % CAL_VEC == 0) && (raw_row_pitch % CAL_VEC == 0) && (raw_frame_pitch % CAL_VEC == 0) &&
                     (cal_row_pitch % 4 == 0) && aligned16(raw) && aligned16(dark) && aligned16(flat) &&
                     aligned16(out) && (!bias || aligned16(bias));
    ProfScope prof("calibrate", s);
    if (vec) {
        const int64_t groups = (int64_t)(W / CAL_VEC) * H;
        hipLaunchKernelGGL(calibrate_vec8, dim3((unsigned)ceil_div(groups, CAL_BLOCK)), dim3(CAL_BLOCK), 0, s,
                           raw, raw_row_pitch, raw_frame_pitch, bias, dark, flat, cal_row_pitch, out, W, H, N);
    } else {
        hipLaunchKernelGGL(calibrate_scalar, dim3((unsigned)ceil_div((int64_t)W * H, CAL_BLOCK)), dim3(CAL_BLOCK), 0,
                           s, raw, raw_row_pitch, raw_frame_pitch, bias, dark, flat, cal_row_pitch, out, W, H, N);
    }
    return check_launch("reduce_calibrate");
}
