// Device body of the bilinear shift, shared by the stage-wise kernel and the batched
// path so that both produce the same bits.
#pragma once

#include "common.h"

namespace rd {

constexpr int SH_BLOCK = 256;
constexpr int SH_VEC = 4;     // outputs per thread and row
constexpr int SH_ROWS = 16;   // output rows per workgroup: each input row is fetched once per strip

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// V outputs of one row at o + u0: 16-byte stores when every output row starts 16-byte
// aligned (vec_store 4: w % 4 == 0), 8-byte stores when rows start 8-byte aligned
// (vec_store 2: w even), single floats otherwise and at the row end.
template <int V>
__device__ __forceinline__ void store_outputs(float *__restrict__ o, int32_t u0, int32_t w, int vec_store,
                                              const float (&r)[V])
{
    if (vec_store == 4 && u0 + V <= w) {
#pragma unroll
        for (int q = 0; q < V / 4; ++q)
            *reinterpret_cast<float4 *>(o + u0 + 4 * q) = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2],
                                                                      r[4 * q + 3]);
    } else if (vec_store == 2 && u0 + V <= w) {
#pragma unroll
        for (int q = 0; q < V / 2; ++q)
            *reinterpret_cast<float2 *>(o + u0 + 2 * q) = make_float2(r[2 * q], r[2 * q + 1]);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e)
            if (u0 + e < w) o[u0 + e] = r[e];
    }
}

// One tap row of a thread: the floats from the 16-byte aligned column b = c0 - (c0 & 3)
// on, so that tap e (column c0 + e) is raw[(c0 & 3) + e].  The misalignment is the same
// for every thread of a frame.  Rows whose aligned span lies inside the frame row come
// in as float4 loads; otherwise the taps are loaded one by one with clamped columns.
// The select happens only when the taps are used, so a prefetched row stays in flight.
template <int V>
struct TapRow {
    static constexpr int RAW = V + 4;  // covers (c0 & 3) + V + 1 taps
    float raw[RAW];

    __device__ __forceinline__ void load(const float *__restrict__ row, int32_t c0, int32_t W, bool aligned)
    {
        const int32_t al = c0 & 3;
        const int32_t b = c0 - al;
        if (aligned && b >= 0 && b + RAW <= W) {
#pragma unroll
            for (int q = 0; q < RAW / 4; ++q) {
                const float4 u = *reinterpret_cast<const float4 *>(row + b + 4 * q);
                raw[4 * q] = u.x;
                raw[4 * q + 1] = u.y;
                raw[4 * q + 2] = u.z;
                raw[4 * q + 3] = u.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < RAW; ++e) raw[e] = row[clampi(b + e, 0, W - 1)];
        }
    }

    template <int AL>
    __device__ __forceinline__ void taps_at(float (&t)[V + 1]) const
    {
#pragma unroll
        for (int e = 0; e <= V; ++e) t[e] = raw[AL + e];
    }

    __device__ __forceinline__ void taps(int32_t al, float (&t)[V + 1]) const
    {
        switch (al) {
        case 0: taps_at<0>(t); break;
        case 1: taps_at<1>(t); break;
        case 2: taps_at<2>(t); break;
        default: taps_at<3>(t); break;
        }
    }
};

// Grid (x strips of SH_BLOCK * V outputs, strips of SH_ROWS rows, frames).  A thread
// produces V consecutive outputs in each row of its strip.  The lower tap row of one
// output row is the upper tap row of the next, and the row the next output row needs
// is requested before the current one is computed.
// One thread's part of strip `strip` (SH_ROWS output rows) of x block `xblk` of frame k
// (offset (sx, sy)): V consecutive outputs in each row.  Output frame k's plane of h
// rows of w starts at out + k * pstride.
template <bool INTEGER, int V>
__device__ __forceinline__ void shift_strip(const float *__restrict__ in, float *__restrict__ out, int32_t W,
                                            int32_t H, int32_t k, float sx, float sy, int32_t strip, int32_t xblk,
                                            int32_t x0, int32_t y0, int32_t w, int32_t h, int64_t pstride,
                                            int vec_store, bool aligned)
{
    const int32_t v0 = strip * SH_ROWS;
    const int32_t v1 = min(v0 + SH_ROWS, h);
    const int32_t u0 = (xblk * SH_BLOCK + (int32_t)threadIdx.x) * V;
    if (u0 >= w || v0 >= h) return;
    const ShiftSetup ss = shift_setup(sx, sy);
    const float *f = in + (int64_t)k * W * H;
    const int32_t c0 = x0 + u0 + ss.ix;
    const int32_t al = c0 & 3;
    const bool step = ss.a > 0.0;
    const bool down = !INTEGER && ss.b > 0.0;
    auto row_of = [&](int32_t v) { return clampi(y0 + v + ss.iy, 0, H - 1); };
    auto low_of = [&](int32_t j) { return clampi(down ? j + 1 : j, 0, H - 1); };

    TapRow<V> up, lo, nx;
    int32_t j = row_of(v0);
    int32_t j1 = low_of(j);
    up.load(f + (int64_t)j * W, c0, W, aligned);
    if (j1 != j) lo.load(f + (int64_t)j1 * W, c0, W, aligned);
    for (int32_t v = v0; v < v1; ++v) {
        const bool more = v + 1 < v1;
        const int32_t jn = more ? row_of(v + 1) : j;
        const int32_t jn1 = more ? low_of(jn) : j1;
        // the next upper row is the current lower row whenever the rows advance by one
        const int32_t want = (jn == j1 && j1 != j) ? jn1 : jn;
        if (more) nx.load(f + (int64_t)want * W, c0, W, aligned);
        float t0[V + 1], t1[V + 1];
        up.taps(al, t0);
        if (j1 != j)
            lo.taps(al, t1);
        else
#pragma unroll
            for (int e = 0; e <= V; ++e) t1[e] = t0[e];
        float r[V];
        if (INTEGER) {
#pragma unroll
            for (int e = 0; e < V; ++e) r[e] = t0[e];
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                // the right-hand tap is the next column only when it carries weight
                const float f10 = step ? t0[e + 1] : t0[e];
                const float f11 = step ? t1[e + 1] : t1[e];
                r[e] = bilerp(ss.a, ss.b, t0[e], f10, t1[e], f11);
            }
        }
        float *o = out + (int64_t)k * pstride + (int64_t)v * w;
        store_outputs<V>(o, u0, w, vec_store, r);
        if (!more) break;
        if (jn == j1 && j1 != j) {
            up = lo;                      // rows advanced by one
            if (jn1 != jn) lo = nx;
        } else {
            up = nx;                      // integer mode, no vertical weight, or clamped rows
            if (jn1 != jn) lo.load(f + (int64_t)jn1 * W, c0, W, aligned);
        }
        j = jn;
        j1 = jn1;
    }
}

// Output rows of frames with 4-byte alignment of `out`: the widest store the rows allow.
__host__ __device__ inline int shift_vec_store(int32_t w, uintptr_t out_addr)
{
    return (w % 4 == 0 && (out_addr & 15u) == 0) ? 4 : (w % 2 == 0 && (out_addr & 7u) == 0) ? 2 : 1;
}

// Bad-pixel masking after the shift (the paper masks bad pixels before alignment,
// Section 2.1): output u of row v of frame k becomes NaN (missing) when one of the taps
// the bilinear shift read for it is a bad pixel of mask [H][W], the bad-pixel map
// shared by the frames (integer mode: the one pixel it copied).  The taps are those of
// shift_strip: rows j and j + 1 (when the y fraction is non-zero), columns i and i + 1
// (when the x fraction is non-zero), clamped into the frame as there.
__device__ __forceinline__ bool reads_bad_pixel(const uint8_t *__restrict__ mask, int32_t W, int32_t H,
                                                const ShiftSetup &ss, bool integer, int32_t x, int32_t y)
{
    const int32_t c = x + ss.ix;
    const int32_t i = clampi(c, 0, W - 1), j = clampi(y + ss.iy, 0, H - 1);
    const int32_t i1 = (!integer && ss.a > 0.0) ? clampi(c + 1, 0, W - 1) : i;
    const int32_t j1 = (!integer && ss.b > 0.0) ? clampi(j + 1, 0, H - 1) : j;
    const uint8_t *r0 = mask + (int64_t)j * W, *r1 = mask + (int64_t)j1 * W;
    return (r0[i] | r0[i1] | r1[i] | r1[i1]) != 0;
}

}  // namespace rd
