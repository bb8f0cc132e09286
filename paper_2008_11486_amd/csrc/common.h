// Shared host/device helpers of libreduce (gfx950).  Per-element arithmetic that
// both the stage-wise kernels and the fused batch kernel use lives here, so the two
// paths evaluate exactly the same operations in the same order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <string>

#include "reduce.h"

namespace rd {

// ---- host-side error reporting ------------------------------------------------
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);
int check_launch(const char *what);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ---- kernel timing (enabled by reduce_prof_enable) ----------------------------
// When enabled, ProfScope records a HIP event pair around a launch on its stream;
// reduce_prof_query() sums the elapsed times per kernel name.
bool prof_on();
void prof_record(const char *name, hipStream_t s, bool start);

struct ProfScope {
    const char *name;
    hipStream_t stream;
    bool on;
    ProfScope(const char *n, hipStream_t s) : name(n), stream(s), on(prof_on())
    {
        if (on) prof_record(name, stream, true);
    }
    ~ProfScope()
    {
        if (on) prof_record(name, stream, false);
    }
};

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---- XCD-aware work order ----------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous run of logical work items so that neighbouring items, which share input
// rows (the search tiles of one frame band, the frames of one masked row), hit the
// same L2.
__device__ __forceinline__ int32_t xcd_logical_id(int32_t lin, int32_t total)
{
    constexpr int32_t NXCD = 8;
    const int32_t per = total / NXCD, rem = total % NXCD;
    const int32_t x = lin % NXCD, slot = lin / NXCD;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + slot;
}

// ---- per-element arithmetic ----------------------------------------------------

// (raw - dark) / flat in float: the subtraction is exact whenever dark lies within a
// factor of two of raw, and the division is IEEE correctly rounded (no fast-math).
__device__ __forceinline__ float calib_px(uint16_t raw, float dark, float flat)
{
    return __fdiv_rn(__fsub_rn((float)raw, dark), flat);
}

// ((raw - bias) - dark) / flat: the cast happens at the bias subtraction (Section 2.1).
__device__ __forceinline__ float calib_px(uint16_t raw, float bias, float dark, float flat)
{
    return __fdiv_rn(__fsub_rn(__fsub_rn((float)raw, bias), dark), flat);
}

// Per-frame bilinear setup: integer part and exact fraction of the offset.
struct ShiftSetup {
    int32_t ix, iy;     // floor(s)
    double a, b;        // s - floor(s), exact in double
};

__device__ __forceinline__ ShiftSetup shift_setup(float sx, float sy)
{
    ShiftSetup s;
    const double dsx = (double)sx, dsy = (double)sy;
    const double fx = floor(dsx), fy = floor(dsy);
    s.ix = (int32_t)fx;
    s.iy = (int32_t)fy;
    s.a = dsx - fx;
    s.b = dsy - fy;
    return s;
}

// Bilinear combination of the four taps in double, rounded once to float.
__device__ __forceinline__ float bilerp(double a, double b, float f00, float f10, float f01, float f11)
{
    const double ra = 1.0 - a, rb = 1.0 - b;
    const double t0 = __dmul_rn(__dmul_rn(ra, rb), (double)f00);
    const double t1 = __dmul_rn(__dmul_rn(a, rb), (double)f10);
    const double t2 = __dmul_rn(__dmul_rn(ra, b), (double)f01);
    const double t3 = __dmul_rn(__dmul_rn(a, b), (double)f11);
    return (float)__dadd_rn(__dadd_rn(__dadd_rn(t0, t1), t2), t3);
}

}  // namespace rd
