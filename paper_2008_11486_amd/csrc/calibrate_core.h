// Device bodies of dark subtraction and flat division, shared by the stage-wise kernels
// and the batched path.
#pragma once

#include "common.h"

namespace rd {

constexpr int CAL_VEC = 8;
constexpr int CAL_BLOCK = 256;

// Group g of 8 pixels of one row, every frame (16-byte aligned rows and pitches).
// bias may be NULL (no bias frame).
__device__ __forceinline__ void calibrate_group8(const uint16_t *__restrict__ raw, int64_t rrp, int64_t rfp,
                                                 const float *__restrict__ bias, const float *__restrict__ dark,
                                                 const float *__restrict__ flat, int64_t crp,
                                                 float *__restrict__ out, int32_t W, int32_t H, int32_t N,
                                                 int64_t g)
{
    const int64_t groups_per_row = W / CAL_VEC;
    if (g >= groups_per_row * H) return;
    const int32_t y = (int32_t)(g / groups_per_row);
    const int32_t x = (int32_t)(g - (int64_t)y * groups_per_row) * CAL_VEC;

    const float4 *dp = reinterpret_cast<const float4 *>(dark + (int64_t)y * crp + x);
    const float4 *fp = reinterpret_cast<const float4 *>(flat + (int64_t)y * crp + x);
    const float4 d0 = dp[0], d1 = dp[1], f0 = fp[0], f1 = fp[1];
    const float d[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    const float f[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
    float b[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (bias) {
        const float4 *bp = reinterpret_cast<const float4 *>(bias + (int64_t)y * crp + x);
        const float4 b0 = bp[0], b1 = bp[1];
        b[0] = b0.x, b[1] = b0.y, b[2] = b0.z, b[3] = b0.w, b[4] = b1.x, b[5] = b1.y, b[6] = b1.z, b[7] = b1.w;
    }

    const uint16_t *rp = raw + (int64_t)y * rrp + x;
    float *op = out + (int64_t)y * W + x;
    const int64_t plane = (int64_t)W * H;
#pragma unroll 4
    for (int32_t k = 0; k < N; ++k) {
        const uint4 v = *reinterpret_cast<const uint4 *>(rp + (int64_t)k * rfp);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        float c[8];
        if (bias) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                c[2 * i] = calib_px((uint16_t)(w[i] & 0xffffu), b[2 * i], d[2 * i], f[2 * i]);
                c[2 * i + 1] = calib_px((uint16_t)(w[i] >> 16), b[2 * i + 1], d[2 * i + 1], f[2 * i + 1]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                c[2 * i] = calib_px((uint16_t)(w[i] & 0xffffu), d[2 * i], f[2 * i]);
                c[2 * i + 1] = calib_px((uint16_t)(w[i] >> 16), d[2 * i + 1], f[2 * i + 1]);
            }
        }
        float4 *o = reinterpret_cast<float4 *>(op + (int64_t)k * plane);
        o[0] = make_float4(c[0], c[1], c[2], c[3]);
        o[1] = make_float4(c[4], c[5], c[6], c[7]);
    }
}

// Pixel p of the frame, every frame (any pitch and alignment).
__device__ __forceinline__ void calibrate_pixel(const uint16_t *__restrict__ raw, int64_t rrp, int64_t rfp,
                                                const float *__restrict__ bias, const float *__restrict__ dark,
                                                const float *__restrict__ flat, int64_t crp,
                                                float *__restrict__ out, int32_t W, int32_t H, int32_t N, int64_t p)
{
    if (p >= (int64_t)W * H) return;
    const int32_t y = (int32_t)(p / W), x = (int32_t)(p - (int64_t)y * W);
    const float d = dark[(int64_t)y * crp + x], f = flat[(int64_t)y * crp + x];
    const int64_t plane = (int64_t)W * H;
    if (bias) {
        const float b = bias[(int64_t)y * crp + x];
        for (int32_t k = 0; k < N; ++k)
            out[k * plane + p] = calib_px(raw[(int64_t)k * rfp + (int64_t)y * rrp + x], b, d, f);
    } else {
        for (int32_t k = 0; k < N; ++k)
            out[k * plane + p] = calib_px(raw[(int64_t)k * rfp + (int64_t)y * rrp + x], d, f);
    }
}

}  // namespace rd
