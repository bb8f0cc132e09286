// Bicubic-spline sub-pixel shift onto the common overlap: the paper's own interpolation
// (Section 2.1 and 2.2; Section 3.2.1 prices its tridiagonal systems, one per image row
// or column).  The interpolant is the tensor-product natural cubic spline through the
// pixel values on the integer grid, evaluated at (x + s_x, y + s_y).
//
// Along one line of L values the natural spline's second derivatives M satisfy
//   M[i-1] + 4 M[i] + M[i+1] = g[i] := 6 (f[i+1] - 2 f[i] + f[i-1]),  0 < i < L-1,
//   M[0] = M[L-1] = 0.
// On an unbounded line the inverse of the (1, 4, 1) operator is h[j] = z^|j| / (2 sqrt 3)
// with z = sqrt 3 - 2, so with g = 0 outside the interior, P = h * g satisfies every
// interior equation, and M = P + A z^i + B z^(L-1-i) adds the two homogeneous solutions
// whose coefficients make both ends zero.  P is not formed as a sum over h: h factors into
// a causal and an anticausal first-order recursion (sp_recur), which a thread runs over
// its own run of knots, started 16 knots outside it (|z|^17 < 2e-10).  On [i, i+1], with
// t = x - i,
//   S(x) = (1-t) f[i] + t f[i+1] + ((1-t)^3 - (1-t)) M[i] / 6 + (t^3 - t) M[i+1] / 6.
// Positions are clamped into [0, L-1] (inside the overlap they never need it); a clamped
// position takes f[0] or f[L-1].
//
// Two streaming passes, FP32 arithmetic: rows (every frame row at the shifted x of every
// output column, into a workspace [N][H][w]), then columns of that result at the shifted
// y.  The shift is the same for the whole frame, so output u sits on knot x0 + fx + u
// (before clamping) with the same fraction: a thread that owns a run of knots holds in
// registers everything its run's outputs need.
#include <string>

#include "common.h"
#include "shift_core.h"  // clampi

namespace rd {

constexpr int SP_T = 16;                          // recursion warm-up, knots
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

// P[0] (end 0) or P[L-1] (end 1) of a line read through get(i), i in [0, L): h * g with
// g zero outside 1 .. L-2, which reaches 16 knots in.
template <typename Get>
__device__ __forceinline__ float sp_end_p(Get get, int32_t L, int end)
{
    constexpr SpTaps h = sp_taps();
    float p = 0.0f;
#pragma unroll
    for (int j = 1; j <= SP_T; ++j) {
        const int32_t m = end ? L - 1 - j : j;
        if (m >= 1 && m <= L - 2) p += h.v[j] * (6.0f * (get(m + 1) - 2.0f * get(m) + get(m - 1)));
    }
    return p;
}

// The four weights of S for a fixed fraction t: S = a f[i] + b f[i+1] + c M[i] + d M[i+1].
struct SpW {
    float a, b, c, d;
};
__device__ __forceinline__ SpW sp_weights(float t)
{
    const float u = 1.0f - t;
    return SpW{u, t, (u * u * u - u) * (1.0f / 6.0f), (t * t * t - t) * (1.0f / 6.0f)};
}
__device__ __forceinline__ float sp_apply(const SpW &wt, float fi, float fi1, float Mi, float Mi1)
{
    return fmaf(wt.d, Mi1, fmaf(wt.c, Mi, fmaf(wt.b, fi1, wt.a * fi)));
}

// P (up to the end corrections) of knots s .. s+K from fw[r] = f[s - SP_T - 1 + r]: the
// inverse of (1, 4, 1) on the unbounded line factors as (-z) / ((1 - z S^-1)(1 - z S)),
// S the shift, so P = -6 z d with c[m] = D2f[m] + z c[m-1] (causal) and
// d[m] = c[m] + z d[m+1] (anticausal), D2f[m] = f[m+1] - 2 f[m] + f[m-1].  Both
// recursions start SP_T knots outside the run with zero state; the state they miss is
// below z^17 (2e-10) of the data.
template <int K>
__device__ __forceinline__ void sp_recur(const float (&fw)[K + 2 * SP_T + 3], float (&p)[K + 1])
{
    const float z = (float)SP_Z, scale = (float)(-6.0 * SP_Z);
    float c[K + SP_T + 1];  // causal state at knots s .. s+K+SP_T
    float st = 0.0f;
#pragma unroll
    for (int r = 0; r <= K + 2 * SP_T; ++r) {  // knot s - SP_T + r
        const float g = fmaf(-2.0f, fw[r + 1], fw[r + 2] + fw[r]);
        st = fmaf(z, st, g);
        if (r >= SP_T) c[r - SP_T] = st;
    }
    float d = 0.0f;
#pragma unroll
    for (int r = K + SP_T; r >= 0; --r) {
        d = fmaf(z, d, c[r]);
        if (r <= K) p[r] = scale * d;
    }
}

// The recursion reads staged values clamped into the line, so next to an end its g holds
// D2f[0] = f[1] - f[0] and D2f[L-1] = f[L-2] - f[L-1] instead of zero (further out the
// clamped values give exactly zero).  Their responses, 6 h[i] e0 and 6 h[L-1-i] e1, have
// the shape of the two end corrections, so they are taken out of (A, B): returns the
// coefficients to add to P from P[0], P[L-1] of the true g and the four end values.
__device__ __forceinline__ void sp_ends_raw(float P0, float PL, int32_t L, float f0, float f1, float fl2, float fl1,
                                            float &A, float &B)
{
    sp_ends(P0, PL, L, A, B);
    const float c6 = (float)(6.0 * SP_C);
    A -= c6 * fmaf(-2.0f, f0, f1 + f0);    // the recursion's own g at knot 0
    B -= c6 * fmaf(-2.0f, fl1, fl1 + fl2);  // and at knot L-1
}

// End corrections are needed only within a few dozen knots of a line end (z^40 < 1e-22).
constexpr int SP_NEAR = 40;

// The outputs of a run of K knots s .. s+K-1 (M of knot s+K is p[K]): fw and p as in
// sp_recur.  Knots at or beyond an end first get their M (zero at both ends, plus the
// end corrections near them); a knot outside 0 .. L-2 is a clamped position, whose value
// is the staged (clamped) line value.
template <int K>
__device__ __forceinline__ void sp_outputs(const float (&fw)[K + 2 * SP_T + 3], float (&p)[K + 1], int32_t s,
                                           int32_t L, bool near, float A, float B, const SpW &wt, float (&o)[K])
{
    if (near) {
#pragma unroll
        for (int r = 0; r <= K; ++r) {
            const int32_t i = s + r;
            p[r] = (i <= 0 || i >= L - 1) ? 0.0f : p[r] + A * sp_zpow(i) + B * sp_zpow(L - 1 - i);
        }
    }
#pragma unroll
    for (int r = 0; r < K; ++r) {
        o[r] = sp_apply(wt, fw[r + SP_T + 1], fw[r + SP_T + 2], p[r], p[r + 1]);
        if (near) {
            const int32_t i = s + r;
            if (i < 0 || i > L - 2) o[r] = fw[r + SP_T + 1];
        }
    }
}

// LDS index of staged value (or output) e: a pad word every 16 puts the stride-16
// windows of the lanes on distinct banks.
__device__ __forceinline__ int sp_pad(int e) { return e + (e >> 4); }

// ---- pass 1: rows -------------------------------------------------------------------------
constexpr int SP_N = 64;                           // lanes: one wave per workgroup
constexpr int SP_Q = 16;                           // knots (outputs) per lane
constexpr int SP_U = SP_N * SP_Q;                  // outputs per workgroup
constexpr int SP_F = SP_U + 1 + 2 * SP_T + 2;      // staged values
constexpr int SP_NL = (SP_F + SP_N - 1) / SP_N;    // staged values per lane
constexpr int SP_FP = SP_F + (SP_F >> 4) + 1;

// A workgroup takes 1024 output columns of one row: it stages their knots' values plus a
// 17-value halo, every lane runs the two recursions over its 16 knots and forms their
// outputs, which go back through LDS so that consecutive lanes store consecutive columns.
__global__ __launch_bounds__(SP_N) void spline_rows(const float *__restrict__ in, float *__restrict__ R, int32_t W,
                                                    int32_t H, const float *__restrict__ offs, int32_t x0, int32_t w,
                                                    int32_t wp)
{
    __shared__ float fs[SP_FP];
    const int32_t k = blockIdx.z, j = blockIdx.y, u0 = blockIdx.x * SP_U;
    const int t = threadIdx.x;
    const float sx = offs[2 * k];
    const float fl = floorf(sx);
    const int32_t fx = (int32_t)fl;
    const float *row = in + ((int64_t)k * H + j) * W;
    float *dst = R + ((int64_t)k * H + j) * wp;
    const int32_t L = W;
    const int32_t un = min(u0 + SP_U, w) - u0;
    if (L < 2) {
        for (int32_t d = t; d < un; d += SP_N) dst[u0 + d] = row[0];
        return;
    }
    const int32_t ka = x0 + u0 + fx;     // knot of output u0 (before clamping)
    const int32_t base = ka - SP_T - 1;  // line index of staged value 0
    const bool near0 = ka < SP_NEAR, nearL = ka + SP_U + 1 > L - 1 - SP_NEAR;  // uniform
    {
        float v[SP_NL];
#pragma unroll
        for (int r = 0; r < SP_NL; ++r) v[r] = row[clampi(base + t + SP_N * r, 0, L - 1)];
#pragma unroll
        for (int r = 0; r < SP_NL; ++r)
            if (t + SP_N * r < SP_F) fs[sp_pad(t + SP_N * r)] = v[r];
    }
    float A = 0.0f, B = 0.0f;
    if (near0 || nearL) {
        auto get = [&](int32_t i) { return row[i]; };
        sp_ends_raw(near0 ? sp_end_p(get, L, 0) : 0.0f, nearL ? sp_end_p(get, L, 1) : 0.0f, L, row[0],
                    row[min(1, L - 1)], row[max(L - 2, 0)], row[L - 1], A, B);
    }
    __syncthreads();
    float o[SP_Q];
    {
        const int q0 = SP_Q * t;
        float fw[SP_Q + 2 * SP_T + 3], p[SP_Q + 1];
#pragma unroll
        for (int r = 0; r < SP_Q + 2 * SP_T + 3; ++r) fw[r] = fs[sp_pad(q0 + r)];
        sp_recur<SP_Q>(fw, p);
        sp_outputs<SP_Q>(fw, p, ka + q0, L, near0 || nearL, A, B, sp_weights(sx - fl), o);
    }
    __syncthreads();  // every lane has read its window
#pragma unroll
    for (int r = 0; r < SP_Q; ++r) fs[sp_pad(SP_Q * t + r)] = o[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < SP_Q; ++q) {
        const int d = t + SP_N * q;  // consecutive lanes store consecutive columns
        if (d < un) dst[u0 + d] = fs[sp_pad(d)];
    }
}

// ---- pass 2: columns ----------------------------------------------------------------------
constexpr int SPC_C = 64;                          // columns per workgroup
constexpr int SPC_G = 4;                           // row groups (threads = SPC_C * SPC_G)
constexpr int SPC_Q = 16;                          // knots (output rows) per thread and tile
constexpr int SPC_V = SPC_G * SPC_Q;               // output rows per tile
constexpr int SPC_F = SPC_V + 1 + 2 * SP_T + 2;    // line values a tile reads
constexpr int SPC_RING = 128;                      // LDS ring of line values (>= SPC_F)
constexpr int SPC_NT = 2;                          // tiles per workgroup (short walks keep the
                                                   // workgroups that run together on the same
                                                   // rows: 8-tile walks were 10% slower)
constexpr int SPC_NL0 = (SPC_F + SPC_G - 1) / SPC_G;
constexpr int SPC_NL = SPC_V / SPC_G;              // new lines per thread and tile
constexpr int SP_E = SP_T + 2;                     // values at each line end that P[0], P[L-1] read
static_assert(SPC_RING >= SPC_F && (SPC_RING & (SPC_RING - 1)) == 0, "ring");
static_assert(2 * SP_E <= SPC_RING, "the end values pass through the ring");

// A workgroup walks down SPC_NT tiles of 64 columns x 64 output rows.  Line value m of a
// column sits in ring row m mod 128; a tile whose first output row sits on knot kb reads
// lines kb - 17 .. kb + 81, so the next tile adds 64 new lines, loaded into registers
// while the current tile is computed and stored once its reads are done.  A thread's 16
// output rows are its own knots.  The end corrections are the same for every tile of a
// column: each thread forms them for its column at the start.
__global__ __launch_bounds__(SPC_C *SPC_G) void spline_cols(const float *__restrict__ R, float *__restrict__ out,
                                                            int32_t H, const float *__restrict__ offs, int32_t y0,
                                                            int32_t w, int32_t wp, int32_t h)
{
    __shared__ float ring[SPC_RING][SPC_C];
    const int32_t k = blockIdx.z, vs = blockIdx.y * SPC_V * SPC_NT, c0 = blockIdx.x * SPC_C;
    const int32_t ve = min(vs + SPC_V * SPC_NT, h);
    const int c = threadIdx.x % SPC_C, rg = threadIdx.x / SPC_C;
    const float sy = offs[2 * k + 1];
    const float fl = floorf(sy);
    const int32_t fy = (int32_t)fl;
    const int32_t L = H;
    const int32_t col = min(c0 + c, w - 1);
    const bool live = c0 + c < w;
    const float *src = R + (int64_t)k * H * wp + col;
    auto at = [&](int32_t i) { return src[(int64_t)clampi(i, 0, L - 1) * wp]; };
    if (L < 2) {
        for (int32_t v = vs + rg; v < ve; v += SPC_G)
            if (live) out[((int64_t)k * h + v) * w + c0 + c] = at(0);
        return;
    }
    int32_t kb = y0 + vs + fy;  // knot of the tile's first output row (before clamping)
    const bool near0 = kb < SP_NEAR, nearL = y0 + ve - 1 + fy + 1 > L - 1 - SP_NEAR;  // uniform
    float A = 0.0f, B = 0.0f;
    if (near0 || nearL) {
        // ring row e holds f[e] and ring row SP_E + e holds f[L - SP_E + e] (indices clamped
        // into the line) until the first tile is staged; sp_end_p reads only 0 .. L-1
        for (int e = rg; e < 2 * SP_E; e += SPC_G) ring[e][c] = at(e < SP_E ? e : L - 2 * SP_E + e);
        __syncthreads();
        auto lo = [&](int32_t i) { return ring[min(i, SP_E - 1)][c]; };
        auto hi = [&](int32_t i) { return ring[SP_E + max(i - (L - SP_E), 0)][c]; };
        sp_ends_raw(near0 ? sp_end_p(lo, L, 0) : 0.0f, nearL ? sp_end_p(hi, L, 1) : 0.0f, L, lo(0), lo(1),
                    hi(L - 2), hi(L - 1), A, B);
        __syncthreads();
    }
    {
        float v[SPC_NL0];
#pragma unroll
        for (int r = 0; r < SPC_NL0; ++r) v[r] = at(kb - SP_T - 1 + rg + SPC_G * r);
#pragma unroll
        for (int r = 0; r < SPC_NL0; ++r)
            if (rg + SPC_G * r < SPC_F) ring[(kb - SP_T - 1 + rg + SPC_G * r) & (SPC_RING - 1)][c] = v[r];
    }
    const SpW wt = sp_weights(sy - fl);
    const int q0 = SPC_Q * rg;
    for (int32_t v0 = vs; v0 < ve; v0 += SPC_V, kb += SPC_V) {
        __syncthreads();  // the ring holds this tile's lines
        // the next tile's new lines: hi .. hi + 63
        const int32_t hi = kb + SPC_F - SP_T - 1;
        const bool more = v0 + SPC_V < ve;
        float nv[SPC_NL];
        if (more) {
#pragma unroll
            for (int r = 0; r < SPC_NL; ++r) nv[r] = at(hi + rg + SPC_G * r);
        }
        float o[SPC_Q];
        {
            float fw[SPC_Q + 2 * SP_T + 3], p[SPC_Q + 1];
            const int32_t m0 = kb + q0 - SP_T - 1;
#pragma unroll
            for (int r = 0; r < SPC_Q + 2 * SP_T + 3; ++r) fw[r] = ring[(m0 + r) & (SPC_RING - 1)][c];
            sp_recur<SPC_Q>(fw, p);
            sp_outputs<SPC_Q>(fw, p, kb + q0, L, near0 || nearL, A, B, wt, o);
        }
        if (live) {
#pragma unroll
            for (int r = 0; r < SPC_Q; ++r)
                if (v0 + q0 + r < ve) out[((int64_t)k * h + v0 + q0 + r) * w + c0 + c] = o[r];
        }
        if (more) {
            __syncthreads();  // this tile's reads of the ring are done
#pragma unroll
            for (int r = 0; r < SPC_NL; ++r) ring[(hi + rg + SPC_G * r) & (SPC_RING - 1)][c] = nv[r];
        }
    }
}

}  // namespace rd

using namespace rd;

// row pitch of the workspace: whole 256-byte segments for the column pass's loads
static int32_t spline_pitch(int32_t w) { return (w + 63) & ~63; }

extern "C" size_t reduce_shift_spline_ws(int32_t W, int32_t H, int32_t N)
{
    if (W < 1 || H < 1 || N < 1) return 0;
    return sizeof(float) * (size_t)N * H * (size_t)spline_pitch(W);
}

extern "C" int reduce_shift_spline(const float *in, float *out, int32_t W, int32_t H, int32_t N, const float *offs,
                                   const int32_t *rect, void *ws, size_t ws_bytes, void *stream)
{
    if (!in || !out || !offs || !rect || !ws) return fail(REDUCE_ERR_NULL, "reduce_shift_spline: NULL argument");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_shift_spline: W, H, N must be >= 1");
    const int32_t x0 = rect[0], y0 = rect[1], w = rect[2], h = rect[3];
    if (w < 1 || h < 1 || w > W || h > H) return fail(REDUCE_ERR_SHAPE, "reduce_shift_spline: empty or oversized rect");
    if (N > 65535 || H > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_shift_spline: N or H above 65535");
    const int32_t wp = spline_pitch(w);
    const size_t need = sizeof(float) * (size_t)N * H * (size_t)wp;
    if (ws_bytes < need)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_shift_spline: workspace needs " + std::to_string(need) + " bytes");
    hipStream_t s = as_stream(stream);
    float *R = static_cast<float *>(ws);
    ProfScope prof("shift_spline", s);
    hipLaunchKernelGGL(spline_rows, dim3((unsigned)ceil_div(w, SP_U), (unsigned)H, (unsigned)N), dim3(SP_N), 0, s, in,
                       R, W, H, offs, x0, w, wp);
    hipLaunchKernelGGL(spline_cols,
                       dim3((unsigned)ceil_div(w, SPC_C), (unsigned)ceil_div(h, SPC_V * SPC_NT), (unsigned)N),
                       dim3(SPC_C * SPC_G), 0, s, R, out, H, offs, y0, w, wp, h);
    return check_launch("reduce_shift_spline");
}
