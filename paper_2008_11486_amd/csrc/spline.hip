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
// y.  Each workgroup stages its line segment plus a 17-value halo in LDS; every thread
// forms g and runs the 33-tap stencil for a run of consecutive knots from a window of the
// staged values in registers; the end corrections are formed only by workgroups near a
// line end.
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

// Stencil P for NK consecutive knots from a window gw[NK + 2 SP_T] of g (gw[r + SP_T] at
// knot r), in registers.
template <int NK>
__device__ __forceinline__ void sp_stencil(const float (&gw)[NK + 2 * SP_T], float (&p)[NK])
{
    constexpr SpTaps h = sp_taps();
#pragma unroll
    for (int r = 0; r < NK; ++r) {
        float a = h.v[0] * gw[r + SP_T];
#pragma unroll
        for (int jj = 1; jj <= SP_T; ++jj) a += h.v[jj] * (gw[r + SP_T - jj] + gw[r + SP_T + jj]);
        p[r] = a;
    }
}

// End corrections are needed only within a few dozen knots of a line end (z^40 < 1e-22).
constexpr int SP_NEAR = 40;

// ---- pass 1: rows -------------------------------------------------------------------------
constexpr int SP_N = 256;                          // threads
constexpr int SP_V = 4;                            // outputs (and knots) per thread
constexpr int SP_K = SP_N * SP_V + 1;              // knots the workgroup's outputs touch
constexpr int SP_F = SP_K + 2 * SP_T + 2;          // staged values

__global__ __launch_bounds__(SP_N) void spline_rows(const float *__restrict__ in, float *__restrict__ R, int32_t W,
                                                    int32_t H, const float *__restrict__ offs, int32_t x0, int32_t w)
{
    __shared__ float fs[SP_F], ms[SP_K];
    __shared__ float ends[2];
    const int32_t k = blockIdx.z, j = blockIdx.y, u0 = blockIdx.x * SP_N * SP_V;
    const int t = threadIdx.x;
    const float sx = offs[2 * k];
    const float fl = floorf(sx);
    const float tf = sx - fl;
    const int32_t fx = (int32_t)fl;
    const float *row = in + ((int64_t)k * H + j) * W;
    float *dst = R + ((int64_t)k * H + j) * w;
    const int32_t L = W;
    if (L < 2) {
        for (int32_t u = u0 + t; u < min(u0 + SP_N * SP_V, w); u += SP_N) dst[u] = row[0];
        return;
    }
    const int32_t ka = clampi(x0 + u0 + fx, 0, L - 2);  // first knot of the workgroup
    const int32_t base = ka - SP_T - 1;                // line index of fs[0]
    const bool near0 = ka < SP_NEAR, nearL = ka + SP_K > L - 1 - SP_NEAR;  // uniform
    {
        // all of a thread's loads in flight before any is stored
        constexpr int NL = (SP_F + SP_N - 1) / SP_N;
        float v[NL];
#pragma unroll
        for (int r = 0; r < NL; ++r) v[r] = row[clampi(base + t + SP_N * r, 0, L - 1)];
#pragma unroll
        for (int r = 0; r < NL; ++r)
            if (t + SP_N * r < SP_F) fs[t + SP_N * r] = v[r];
    }
    if (t < 2) ends[t] = (t == 0 ? near0 : nearL) ? sp_end_p([&](int32_t i) { return row[i]; }, L, t) : 0.0f;
    __syncthreads();
    float A, B;
    sp_ends(ends[0], ends[1], L, A, B);
    {
        // knots q0 .. q0 + SP_V (the last one is also the next thread's first); g of knots
        // q0 - SP_T .. from the staged values in registers (zero outside the line's interior)
        const int q0 = SP_V * t;
        constexpr int NG = SP_V + 1 + 2 * SP_T;
        float fw[NG + 2], gw[NG], p[SP_V + 1];
#pragma unroll
        for (int r = 0; r < NG + 2; ++r) fw[r] = fs[q0 + r];
#pragma unroll
        for (int r = 0; r < NG; ++r) {
            const int32_t m = ka + q0 - SP_T + r;
            gw[r] = (m >= 1 && m <= L - 2) ? 6.0f * (fw[r + 2] - 2.0f * fw[r + 1] + fw[r]) : 0.0f;
        }
        sp_stencil<SP_V + 1>(gw, p);
#pragma unroll
        for (int r = 0; r < SP_V + 1; ++r) {
            const int32_t i = ka + q0 + r;
            const float m = (i <= 0 || i >= L - 1) ? 0.0f : p[r] + A * sp_zpow(i) + B * sp_zpow(L - 1 - i);
            if (r < SP_V || t == SP_N - 1) ms[q0 + r] = m;
        }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < SP_V; ++v) {
        const int32_t u = u0 + t + SP_N * v;  // consecutive threads write consecutive columns
        if (u < w) {
            int32_t i;
            float tt;
            sp_knot(x0 + u + fx, tf, L, i, tt);
            const int q = i - ka;
            dst[u] = sp_eval(fs[q + SP_T + 1], fs[q + SP_T + 2], ms[q], ms[q + 1], tt);
        }
    }
}

// ---- pass 2: columns ----------------------------------------------------------------------
constexpr int SPC_C = 64;                          // columns per workgroup
constexpr int SPC_G = 4;                           // row groups (threads = SPC_C * SPC_G)
constexpr int SPC_Q = 16;                          // knots (output rows) per thread
constexpr int SPC_V = SPC_G * SPC_Q;               // output rows per workgroup
constexpr int SPC_K = SPC_V + 1;
constexpr int SPC_F = SPC_K + 2 * SP_T + 2;

__global__ __launch_bounds__(SPC_C *SPC_G) void spline_cols(const float *__restrict__ R, float *__restrict__ out,
                                                            int32_t H, const float *__restrict__ offs, int32_t y0,
                                                            int32_t w, int32_t h)
{
    __shared__ float fs[SPC_F][SPC_C];
    __shared__ float ms[SPC_K][SPC_C];  // M of the knots
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
    const bool near0 = ka < SP_NEAR, nearL = ka + SPC_K > L - 1 - SP_NEAR;  // uniform
    {
        // all of a thread's loads in flight before any is stored
        constexpr int NL = (SPC_F + SPC_G - 1) / SPC_G;
        float v[NL];
#pragma unroll
        for (int r = 0; r < NL; ++r) v[r] = at(clampi(base + rg + SPC_G * r, 0, L - 1));
#pragma unroll
        for (int r = 0; r < NL; ++r)
            if (rg + SPC_G * r < SPC_F) fs[rg + SPC_G * r][c] = v[r];
    }
    if (rg < 2) endP[rg][c] = (rg == 0 ? near0 : nearL) ? sp_end_p(at, L, rg) : 0.0f;
    __syncthreads();
    if (rg == 0) {
        float A, B;
        sp_ends(endP[0][c], endP[1][c], L, A, B);
        endA[c] = A;
        endB[c] = B;
    }
    __syncthreads();
    // knots q0 .. q0 + SPC_Q of column c (the last one is also the next group's first)
    const int q0 = SPC_Q * rg;
    float p[SPC_Q + 1];
    {
        constexpr int NG = SPC_Q + 1 + 2 * SP_T;
        float fw[NG + 2], gw[NG];
#pragma unroll
        for (int r = 0; r < NG + 2; ++r) fw[r] = fs[q0 + r][c];
#pragma unroll
        for (int r = 0; r < NG; ++r) {
            const int32_t m = ka + q0 - SP_T + r;
            gw[r] = (m >= 1 && m <= L - 2) ? 6.0f * (fw[r + 2] - 2.0f * fw[r + 1] + fw[r]) : 0.0f;
        }
        sp_stencil<SPC_Q + 1>(gw, p);
#pragma unroll
        for (int r = 0; r < SPC_Q + 1; ++r) {
            const int32_t i = ka + q0 + r;
            p[r] = (i <= 0 || i >= L - 1) ? 0.0f : p[r] + endA[c] * sp_zpow(i) + endB[c] * sp_zpow(L - 1 - i);
        }
    }
#pragma unroll
    for (int r = 0; r < SPC_Q + 1; ++r)
        if (r < SPC_Q || rg == SPC_G - 1) ms[q0 + r][c] = p[r];
    __syncthreads();
    if (c0 + c >= w) return;
#pragma unroll 4
    for (int r = 0; r < SPC_Q; ++r) {
        const int32_t v = v0 + q0 + r;
        if (v >= h) break;
        int32_t i;
        float tt;
        sp_knot(y0 + v + fy, tf, L, i, tt);
        const int q = i - ka;
        out[((int64_t)k * h + v) * w + c0 + c] = sp_eval(fs[q + SP_T + 1][c], fs[q + SP_T + 2][c], ms[q][c],
                                                         ms[q + 1][c], tt);
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
    hipLaunchKernelGGL(spline_rows, dim3((unsigned)ceil_div(w, SP_N * SP_V), (unsigned)H, (unsigned)N), dim3(SP_N), 0,
                       s, in, R, W, H, offs, x0, w);
    hipLaunchKernelGGL(spline_cols, dim3((unsigned)ceil_div(w, SPC_C), (unsigned)ceil_div(h, SPC_V), (unsigned)N),
                       dim3(SPC_C * SPC_G), 0, s, R, out, H, offs, y0, w, h);
    return check_launch("reduce_shift_spline");
}
