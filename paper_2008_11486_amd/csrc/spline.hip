// Bicubic-spline sub-pixel shift onto the common overlap: the paper's own interpolation
// (Section 2.1 and 2.2; Section 3.2.1 prices its tridiagonal systems, one per image row
// or column).  The interpolant is the tensor-product natural cubic spline through the
// pixel values on the integer grid, evaluated at (x + s_x, y + s_y).
//
// Along one line of L values the natural spline's second derivatives M satisfy
//   M[i-1] + 4 M[i] + M[i+1] = g[i] := 6 (f[i+1] - 2 f[i] + f[i-1]),  0 < i < L-1,
//   M[0] = M[L-1] = 0.
// Instead of a sequential solve per line, every M[i] comes from a short stencil: on an
// unbounded line the inverse of the (1, 4, 1) operator is h[j] = z^|j| / (2 sqrt 3) with
// z = sqrt 3 - 2, so with g = 0 outside the interior, P = h * g satisfies every interior
// equation, and M = P + A z^i + B z^(L-1-i) adds the two homogeneous solutions whose
// coefficients make both ends zero.  |z| = 0.268, so h is cut at |j| <= 16 (the rest is
// below 2e-10 of g).  On [i, i+1], with t = x - i,
//   S(x) = (1-t) f[i] + t f[i+1] + ((1-t)^3 - (1-t)) M[i] / 6 + (t^3 - t) M[i+1] / 6.
// Positions are clamped into [0, L-1] (inside the overlap they never need it).
//
// Two streaming passes, FP32 arithmetic: rows (every frame row at the shifted x of every
// output column, into a workspace [N][H][w]), then columns of that result at the shifted
// y.  Each workgroup stages its line segment plus a 17-value halo in LDS, forms g, the
// 33-tap stencil and the end corrections, then evaluates its outputs.
#include <string>

#include "common.h"
#include "shift_core.h"  // clampi

namespace rd {

constexpr int SP_T = 16;                          // stencil half-width
constexpr double SP_Z = -0.26794919243112270;     // sqrt 3 - 2
constexpr double SP_C = 0.28867513459481287;      // 1 / (2 sqrt 3)

struct SpTaps {
    float v[SP_T + 1];
};
__host__ __device__ constexpr SpTaps sp_taps()
{
    SpTaps t{};
    double p = 1.0;
    for (int j = 0; j <= SP_T; ++j) {
        t.v[j] = (float)(SP_C * p);
        p *= SP_Z;
    }
    return t;
}

// z^n for n >= 0 (zero once it is far below single precision)
__device__ __forceinline__ float sp_zpow(int32_t n)
{
    if (n < 0 || n >= 64) return 0.0f;
    const float a = exp2f((float)n * -1.8999686269529916f);  // log2 |z|
    return (n & 1) ? -a : a;
}

// The end-correction coefficients (A, B) of one line from P[0] and P[L-1].
__device__ __forceinline__ void sp_ends(float P0, float PL, int32_t L, float &A, float &B)
{
    const float zL = sp_zpow(L - 1);
    const float den = 1.0f - zL * zL;
    A = (-P0 + PL * zL) / den;
    B = (-PL + P0 * zL) / den;
}

// P[0] (end 0) or P[L-1] (end 1) of a line read through get(i), i in [0, L).
template <typename Get>
__device__ __forceinline__ float sp_end_p(Get get, int32_t L, int end)
{
    constexpr SpTaps h = sp_taps();
    float p = 0.0f;
#pragma unroll
    for (int j = 1; j <= SP_T; ++j) {
        const int32_t m = end ? L - 1 - j : j;  // g[m] is zero outside 1 .. L-2
        if (m >= 1 && m <= L - 2) p += h.v[j] * (6.0f * (get(m + 1) - 2.0f * get(m) + get(m - 1)));
    }
    return p;
}

__device__ __forceinline__ float sp_eval(float fi, float fi1, float Mi, float Mi1, float t)
{
    const float u = 1.0f - t;
    return u * fi + t * fi1 + (u * u * u - u) * Mi * (1.0f / 6.0f) + (t * t * t - t) * Mi1 * (1.0f / 6.0f);
}

// Knot i and fraction t of position (xi + tf) clamped into [0, L-1], L >= 2.
__device__ __forceinline__ void sp_knot(int32_t xi, float tf, int32_t L, int32_t &i, float &t)
{
    if (xi < 0) {
        i = 0;
        t = 0.0f;
    } else if (xi >= L - 1) {
        i = L - 2;
        t = 1.0f;
    } else {
        i = xi;
        t = tf;
    }
}

// ---- pass 1: rows -------------------------------------------------------------------------
constexpr int SP_N = 256;                          // outputs per workgroup, one per thread
constexpr int SP_K = SP_N + 1;                     // knots those outputs touch
constexpr int SP_F = SP_K + 2 * SP_T + 2;          // staged values

__global__ __launch_bounds__(SP_N) void spline_rows(const float *__restrict__ in, float *__restrict__ R, int32_t W,
                                                    int32_t H, const float *__restrict__ offs, int32_t x0, int32_t w)
{
    constexpr SpTaps h = sp_taps();
    __shared__ float fs[SP_F], gs[SP_F], ms[SP_K];
    __shared__ float ends[2];
    const int32_t k = blockIdx.z, j = blockIdx.y, u0 = blockIdx.x * SP_N;
    const int t = threadIdx.x;
    const float sx = offs[2 * k];
    const float fl = floorf(sx);
    const float tf = sx - fl;
    const int32_t fx = (int32_t)fl;
    const float *row = in + ((int64_t)k * H + j) * W;
    float *dst = R + ((int64_t)k * H + j) * w;
    const int32_t L = W;
    if (L < 2) {
        for (int32_t u = u0 + t; u < min(u0 + SP_N, w); u += SP_N) dst[u] = row[0];
        return;
    }
    const int32_t ka = clampi(x0 + u0 + fx, 0, L - 2);  // first knot of the workgroup
    const int32_t base = ka - SP_T - 1;                // line index of fs[0]
    for (int e = t; e < SP_F; e += SP_N) fs[e] = row[clampi(base + e, 0, L - 1)];
    if (t < 2) {
        const float p = sp_end_p([&](int32_t i) { return row[i]; }, L, t);
        ends[t] = p;
    }
    __syncthreads();
    for (int e = t; e < SP_F; e += SP_N) {
        const int32_t m = base + e;
        gs[e] = (m >= 1 && m <= L - 2 && e >= 1 && e + 1 < SP_F) ? 6.0f * (fs[e + 1] - 2.0f * fs[e] + fs[e - 1]) : 0.0f;
    }
    float A, B;
    sp_ends(ends[0], ends[1], L, A, B);
    __syncthreads();
    for (int q = t; q < SP_K; q += SP_N) {
        float p = h.v[0] * gs[q + SP_T + 1];
#pragma unroll
        for (int jj = 1; jj <= SP_T; ++jj) p += h.v[jj] * (gs[q + SP_T + 1 - jj] + gs[q + SP_T + 1 + jj]);
        const int32_t i = ka + q;
        ms[q] = (i <= 0 || i >= L - 1) ? 0.0f : p + A * sp_zpow(i) + B * sp_zpow(L - 1 - i);
    }
    __syncthreads();
    const int32_t u = u0 + t;
    if (u < w) {
        int32_t i;
        float tt;
        sp_knot(x0 + u + fx, tf, L, i, tt);
        const int q = i - ka;
        dst[u] = sp_eval(fs[q + SP_T + 1], fs[q + SP_T + 2], ms[q], ms[q + 1], tt);
    }
}

// ---- pass 2: columns ----------------------------------------------------------------------
constexpr int SPC_C = 64;                          // columns per workgroup
constexpr int SPC_V = 64;                          // output rows per workgroup
constexpr int SPC_G = 4;                           // row groups (threads = SPC_C * SPC_G)
constexpr int SPC_K = SPC_V + 1;
constexpr int SPC_F = SPC_K + 2 * SP_T + 2;

__global__ __launch_bounds__(SPC_C *SPC_G) void spline_cols(const float *__restrict__ R, float *__restrict__ out,
                                                            int32_t H, const float *__restrict__ offs, int32_t y0,
                                                            int32_t w, int32_t h)
{
    constexpr SpTaps hh = sp_taps();
    __shared__ float fs[SPC_F][SPC_C];
    __shared__ float gs[SPC_F][SPC_C];  // g, then M of the knots
    __shared__ float endA[SPC_C], endB[SPC_C], endP[2][SPC_C];
    const int32_t k = blockIdx.z, v0 = blockIdx.y * SPC_V, c0 = blockIdx.x * SPC_C;
    const int c = threadIdx.x % SPC_C, rg = threadIdx.x / SPC_C;
    const float sy = offs[2 * k + 1];
    const float fl = floorf(sy);
    const float tf = sy - fl;
    const int32_t fy = (int32_t)fl;
    const int32_t L = H;
    const int32_t col = min(c0 + c, w - 1);
    const float *src = R + (int64_t)k * H * w + col;
    auto at = [&](int32_t i) { return src[(int64_t)i * w]; };
    if (L < 2) {
        for (int32_t v = v0 + rg; v < min(v0 + SPC_V, h); v += SPC_G)
            if (c0 + c < w) out[((int64_t)k * h + v) * w + c0 + c] = at(0);
        return;
    }
    const int32_t ka = clampi(y0 + v0 + fy, 0, L - 2);
    const int32_t base = ka - SP_T - 1;
    for (int e = rg; e < SPC_F; e += SPC_G) fs[e][c] = at(clampi(base + e, 0, L - 1));
    if (rg < 2) endP[rg][c] = sp_end_p(at, L, rg);
    __syncthreads();
    for (int e = rg; e < SPC_F; e += SPC_G) {
        const int32_t m = base + e;
        gs[e][c] = (m >= 1 && m <= L - 2 && e >= 1 && e + 1 < SPC_F)
                       ? 6.0f * (fs[e + 1][c] - 2.0f * fs[e][c] + fs[e - 1][c])
                       : 0.0f;
    }
    if (rg == 0) {
        float A, B;
        sp_ends(endP[0][c], endP[1][c], L, A, B);
        endA[c] = A;
        endB[c] = B;
    }
    __syncthreads();
    constexpr int QN = (SPC_K + SPC_G - 1) / SPC_G;
    float mv[QN];
#pragma unroll
    for (int r = 0; r < QN; ++r) {
        const int q = rg + SPC_G * r;
        float p = 0.0f;
        if (q < SPC_K) {
            p = hh.v[0] * gs[q + SP_T + 1][c];
#pragma unroll
            for (int jj = 1; jj <= SP_T; ++jj) p += hh.v[jj] * (gs[q + SP_T + 1 - jj][c] + gs[q + SP_T + 1 + jj][c]);
            const int32_t i = ka + q;
            p = (i <= 0 || i >= L - 1) ? 0.0f : p + endA[c] * sp_zpow(i) + endB[c] * sp_zpow(L - 1 - i);
        }
        mv[r] = p;
    }
    __syncthreads();  // every stencil has read g
#pragma unroll
    for (int r = 0; r < QN; ++r) {
        const int q = rg + SPC_G * r;
        if (q < SPC_K) gs[q][c] = mv[r];
    }
    __syncthreads();
    if (c0 + c >= w) return;
    for (int32_t v = v0 + rg; v < min(v0 + SPC_V, h); v += SPC_G) {
        int32_t i;
        float tt;
        sp_knot(y0 + v + fy, tf, L, i, tt);
        const int q = i - ka;
        out[((int64_t)k * h + v) * w + c0 + c] = sp_eval(fs[q + SP_T + 1][c], fs[q + SP_T + 2][c], gs[q][c],
                                                         gs[q + 1][c], tt);
    }
}

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_shift_spline_ws(int32_t W, int32_t H, int32_t N)
{
    if (W < 1 || H < 1 || N < 1) return 0;
    return (sizeof(float) * (size_t)N * H * W + 255) & ~(size_t)255;
}

extern "C" int reduce_shift_spline(const float *in, float *out, int32_t W, int32_t H, int32_t N, const float *offs,
                                   const int32_t *rect, void *ws, size_t ws_bytes, void *stream)
{
    if (!in || !out || !offs || !rect || !ws) return fail(REDUCE_ERR_NULL, "reduce_shift_spline: NULL argument");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_shift_spline: W, H, N must be >= 1");
    const int32_t x0 = rect[0], y0 = rect[1], w = rect[2], h = rect[3];
    if (w < 1 || h < 1 || w > W || h > H) return fail(REDUCE_ERR_SHAPE, "reduce_shift_spline: empty or oversized rect");
    if (N > 65535 || H > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_shift_spline: N or H above 65535");
    const size_t need = sizeof(float) * (size_t)N * H * w;
    if (ws_bytes < need)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_shift_spline: workspace needs " + std::to_string(need) + " bytes");
    hipStream_t s = as_stream(stream);
    float *R = static_cast<float *>(ws);
    ProfScope prof("shift_spline", s);
    hipLaunchKernelGGL(spline_rows, dim3((unsigned)ceil_div(w, SP_N), (unsigned)H, (unsigned)N), dim3(SP_N), 0, s, in,
                       R, W, H, offs, x0, w);
    hipLaunchKernelGGL(spline_cols, dim3((unsigned)ceil_div(w, SPC_C), (unsigned)ceil_div(h, SPC_V), (unsigned)N),
                       dim3(SPC_C * SPC_G), 0, s, R, out, H, offs, y0, w, h);
    return check_launch("reduce_shift_spline");
}
