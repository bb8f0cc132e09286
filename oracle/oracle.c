/*
 * FP64 CPU oracle for the CCD reduction hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Each function is the plain definition (or the algorithm's steps in order) of one
 * step, in double precision, with loops in the natural row-major order.  OpenMP
 * only distributes independent outputs (frames, rows, candidate offsets) over
 * threads; every output value is produced by one thread in a fixed order, so the
 * result does not depend on the thread count.  Nothing here is blocked, fused or
 * reordered for speed.  Only tests, the smoke check and the benchmark's CPU
 * baseline use it.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { O_OK = 0, O_NULL = 1, O_SHAPE = 2, O_RANGE = 3 };

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (the CPU baseline times 1 and all); the
 * result does not depend on it: every parallel loop writes disjoint outputs. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------------
 * Calibration (Section 2.1 and 2.2: the 16-bit to floating-point cast at the bias
 * subtraction, then dark subtraction and flat fielding).  Without a bias frame the
 * master dark is taken to contain the bias; the flat is normalised already.
 * ---------------------------------------------------------------------------- */
int oracle_calibrate(const uint16_t *raw, int64_t raw_row_pitch, int64_t raw_frame_pitch,
                     const double *bias, const double *dark, const double *flat, int64_t cal_row_pitch,
                     double *out, int32_t W, int32_t H, int32_t N)
{
    if (!raw || !dark || !flat || !out) return O_NULL;
    if (W < 1 || H < 1 || N < 1) return O_SHAPE;
    if (raw_row_pitch < W || raw_frame_pitch < raw_row_pitch * (int64_t)H || cal_row_pitch < W)
        return O_SHAPE;
#pragma omp parallel for collapse(2) schedule(static)
    for (int32_t k = 0; k < N; ++k)
        for (int32_t y = 0; y < H; ++y)
            for (int32_t x = 0; x < W; ++x) {
                double r = (double)raw[(int64_t)k * raw_frame_pitch + (int64_t)y * raw_row_pitch + x];
                if (bias) r = r - bias[(int64_t)y * cal_row_pitch + x];
                double d = dark[(int64_t)y * cal_row_pitch + x];
                double f = flat[(int64_t)y * cal_row_pitch + x];
                out[((int64_t)k * H + y) * W + x] = (r - d) / f;
            }
    return O_OK;
}

/* ------------------------------------------------------------------------------
 * Registration: zero-mean-template cross-correlation over a bounded window.
 *
 *   T      fixed template rectangle inside the reference (interior shrunk by Rmax
 *          unless given), the same for every candidate offset;
 *   r'     = ref - mean_T(ref), so the constant sky drops out of every score;
 *   S(d)   = sum over (x, y) in T of r'(x, y) * f(x + dx, y + dy);
 *   d*     = argmax S; equal scores go to the smaller dy, then the smaller dx;
 *   delta  = 3-point parabola vertex per axis, 0 when d* is on the window border;
 *   s      = d* + delta, rounded to float.
 * ---------------------------------------------------------------------------- */
static int better(double s, int32_t dy, int32_t dx, double best, int32_t bdy, int32_t bdx)
{
    if (s > best) return 1;
    if (s < best) return 0;
    if (dy != bdy) return dy < bdy;
    return dx < bdx;
}

static double parabola_vertex(double sm, double s0, double sp)
{
    double den = 2.0 * (sm - 2.0 * s0 + sp);
    if (!(den < 0.0)) return 0.0;
    double d = (sm - sp) / den;
    if (d > 0.5) d = 0.5;
    if (d < -0.5) d = -0.5;
    return d;
}

int oracle_register(const double *ref, const double *frames, int32_t W, int32_t H, int32_t N,
                    int32_t R, int32_t Rmax, const int32_t *centers, const int32_t *tmpl,
                    oracle_offset_t *out, double *scores)
{
    if (!ref || !frames || !out) return O_NULL;
    if (W < 1 || H < 1 || N < 1) return O_SHAPE;
    if (R < 0 || Rmax < 0) return O_RANGE;
    int32_t tx0, ty0, tw, th;
    if (tmpl) { tx0 = tmpl[0]; ty0 = tmpl[1]; tw = tmpl[2]; th = tmpl[3]; }
    else { tx0 = Rmax; ty0 = Rmax; tw = W - 2 * Rmax; th = H - 2 * Rmax; }
    if (tw < 1 || th < 1) return O_SHAPE;
    if (tx0 - Rmax < 0 || ty0 - Rmax < 0 || tx0 + tw + Rmax > W || ty0 + th + Rmax > H)
        return O_RANGE;
    const int32_t side = 2 * R + 1;

    /* mean of the reference over the template, then the zero-mean template */
    double sum = 0.0;
    for (int32_t y = ty0; y < ty0 + th; ++y)
        for (int32_t x = tx0; x < tx0 + tw; ++x) sum += ref[(int64_t)y * W + x];
    const double mean = sum / ((double)tw * (double)th);
    double *rp = (double *)malloc(sizeof(double) * (size_t)tw * (size_t)th);
    if (!rp) return O_RANGE;
    for (int32_t y = 0; y < th; ++y)
        for (int32_t x = 0; x < tw; ++x)
            rp[(int64_t)y * tw + x] = ref[(int64_t)(ty0 + y) * W + tx0 + x] - mean;

    double *S = (double *)malloc(sizeof(double) * (size_t)N * side * side);
    if (!S) { free(rp); return O_RANGE; }
    int status = O_OK;

    for (int32_t k = 0; k < N; ++k) {
        const int32_t cx = centers ? centers[2 * k] : 0, cy = centers ? centers[2 * k + 1] : 0;
        const int32_t lox = cx - R < -Rmax ? -Rmax : cx - R, hix = cx + R > Rmax ? Rmax : cx + R;
        const int32_t loy = cy - R < -Rmax ? -Rmax : cy - R, hiy = cy + R > Rmax ? Rmax : cy + R;
        if (lox > hix || loy > hiy) { status = O_RANGE; break; }
        const double *f = frames + (int64_t)k * W * H;
        double *Sk = S + (int64_t)k * side * side;
        /* the score of every candidate in the window */
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
        for (int32_t j = 0; j < side; ++j)
            for (int32_t i = 0; i < side; ++i) {
                const int32_t dy = cy - R + j, dx = cx - R + i;
                if (dx < lox || dx > hix || dy < loy || dy > hiy) { Sk[j * side + i] = -INFINITY; continue; }
                double acc = 0.0;
                for (int32_t y = 0; y < th; ++y) {
                    const double *frow = f + (int64_t)(ty0 + y + dy) * W + (tx0 + dx);
                    const double *rrow = rp + (int64_t)y * tw;
                    for (int32_t x = 0; x < tw; ++x) acc += rrow[x] * frow[x];
                }
                Sk[j * side + i] = acc;
            }
        /* argmax with the tie-break, and the best of the other candidates */
        int32_t bdx = 0, bdy = 0, have = 0;
        double best = -INFINITY;
        for (int32_t dy = loy; dy <= hiy; ++dy)
            for (int32_t dx = lox; dx <= hix; ++dx) {
                double s = Sk[(dy - cy + R) * side + (dx - cx + R)];
                if (!have || better(s, dy, dx, best, bdy, bdx)) { best = s; bdx = dx; bdy = dy; have = 1; }
            }
        double second = -INFINITY;
        for (int32_t dy = loy; dy <= hiy; ++dy)
            for (int32_t dx = lox; dx <= hix; ++dx) {
                if (dx == bdx && dy == bdy) continue;
                double s = Sk[(dy - cy + R) * side + (dx - cx + R)];
                if (s > second) second = s;
            }
        /* sub-pixel vertex on each axis through d* and its two neighbours */
        int32_t flags = 0;
        double delx = 0.0, dely = 0.0;
        if (bdx == lox || bdx == hix) flags |= ORACLE_EDGE_X;
        else delx = parabola_vertex(Sk[(bdy - cy + R) * side + (bdx - 1 - cx + R)], best,
                                    Sk[(bdy - cy + R) * side + (bdx + 1 - cx + R)]);
        if (bdy == loy || bdy == hiy) flags |= ORACLE_EDGE_Y;
        else dely = parabola_vertex(Sk[(bdy - 1 - cy + R) * side + (bdx - cx + R)], best,
                                    Sk[(bdy + 1 - cy + R) * side + (bdx - cx + R)]);
        if (lox != cx - R || hix != cx + R || loy != cy - R || hiy != cy + R) flags |= ORACLE_CLIPPED;
        double margin;
        if (second == -INFINITY) margin = INFINITY;
        else if (best == 0.0) margin = (best > second) ? INFINITY : 0.0;
        else margin = (best - second) / fabs(best);
        if (margin < 1e-9) flags |= ORACLE_NEAR_TIE;

        out[k].dx = bdx;
        out[k].dy = bdy;
        out[k].sx = (float)((double)bdx + delx);
        out[k].sy = (float)((double)bdy + dely);
        out[k].peak = best;
        out[k].second = second;
        out[k].margin = margin;
        out[k].flags = flags;
        out[k].pad = 0;
    }
    if (status == O_OK && scores) memcpy(scores, S, sizeof(double) * (size_t)N * side * side);
    free(S);
    free(rp);
    return status;
}

/* ------------------------------------------------------------------------------
 * Common overlap (the alignment crops to the area every frame covers; Section
 * 3.1.2, table of co-adding data sets).  Output pixel x samples frame k at x + s_k,
 * so x must satisfy 0 <= x + s_k <= W - 1 for every k.
 * ---------------------------------------------------------------------------- */
int oracle_valid_rect(const float *offs, int32_t N, int32_t W, int32_t H, int32_t *rect)
{
    if (!offs || !rect) return O_NULL;
    if (W < 1 || H < 1 || N < 1) return O_SHAPE;
    double xl = -INFINITY, xh = INFINITY, yl = -INFINITY, yh = INFINITY;
    for (int32_t k = 0; k < N; ++k) {
        double sx = offs[2 * k], sy = offs[2 * k + 1];
        if (!isfinite(sx) || !isfinite(sy)) return O_RANGE;
        double a = ceil(-sx), b = floor((double)(W - 1) - sx);
        double c = ceil(-sy), d = floor((double)(H - 1) - sy);
        if (a > xl) xl = a;
        if (b < xh) xh = b;
        if (c > yl) yl = c;
        if (d < yh) yh = d;
    }
    if (xl > xh || yl > yh) return O_RANGE;
    rect[0] = (int32_t)xl;
    rect[1] = (int32_t)yl;
    rect[2] = (int32_t)(xh - xl) + 1;
    rect[3] = (int32_t)(yh - yl) + 1;
    return O_OK;
}

/* ------------------------------------------------------------------------------
 * Bilinear shift (the paper shifts by bicubic splines and names bilinear as the
 * cheaper alternative, Section 3.2.1).  The source coordinate x + s splits into the
 * integer i = x + floor(s) and the exact fraction a = s - floor(s); a tap whose
 * weight is zero has its index clamped so that it never leaves the frame.
 * ---------------------------------------------------------------------------- */
int oracle_shift(const double *in, double *out, int32_t W, int32_t H, int32_t N,
                 const float *offs, const int32_t *rect, const uint8_t *mask)
{
    if (!in || !out || !offs || !rect) return O_NULL;
    if (W < 1 || H < 1 || N < 1) return O_SHAPE;
    const int32_t x0 = rect[0], y0 = rect[1], w = rect[2], h = rect[3];
    if (w < 1 || h < 1) return O_SHAPE;
    for (int32_t k = 0; k < N; ++k) {
        double sx = offs[2 * k], sy = offs[2 * k + 1];
        if (!isfinite(sx) || !isfinite(sy)) return O_RANGE;
        double fx = floor(sx), fy = floor(sy);
        if (x0 + fx < 0 || y0 + fy < 0) return O_RANGE;
        double ax = sx - fx, ay = sy - fy;
        if (x0 + w - 1 + fx + (ax > 0 ? 1 : 0) > W - 1) return O_RANGE;
        if (y0 + h - 1 + fy + (ay > 0 ? 1 : 0) > H - 1) return O_RANGE;
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int32_t k = 0; k < N; ++k)
        for (int32_t v = 0; v < h; ++v) {
            const double *f = in + (int64_t)k * W * H;
            const double sx = offs[2 * k], sy = offs[2 * k + 1];
            const double fx = floor(sx), fy = floor(sy);
            const double a = sx - fx, b = sy - fy;
            const int32_t j = y0 + v + (int32_t)fy;
            const int32_t j1 = (b > 0.0) ? j + 1 : j;
            for (int32_t u = 0; u < w; ++u) {
                const int32_t i = x0 + u + (int32_t)fx;
                const int32_t i1 = (a > 0.0) ? i + 1 : i;
                const double f00 = f[(int64_t)j * W + i], f10 = f[(int64_t)j * W + i1];
                const double f01 = f[(int64_t)j1 * W + i], f11 = f[(int64_t)j1 * W + i1];
                double val = (1.0 - a) * (1.0 - b) * f00 + a * (1.0 - b) * f10 +
                             (1.0 - a) * b * f01 + a * b * f11;
                /* bad-pixel masking: an output that reads a bad pixel is missing */
                if (mask && (mask[(int64_t)j * W + i] || mask[(int64_t)j * W + i1] ||
                             mask[(int64_t)j1 * W + i] || mask[(int64_t)j1 * W + i1]))
                    val = NAN;
                out[((int64_t)k * h + v) * w + u] = val;
            }
        }
    return O_OK;
}

/* ------------------------------------------------------------------------------
 * Sigma-clipped mean (Sections 2.1, 2.2 and 3.1.2).  Per pixel, over the N values:
 * start with all kept; up to max_iters times, take the mean m and the population
 * standard deviation sigma of the kept values and drop every kept value with
 * |x - m| > k sigma (all decided against the same m and sigma); stop early when an
 * iteration drops nothing; output the mean of what is kept.
 * ---------------------------------------------------------------------------- */
int oracle_combine(const double *aligned, int32_t w, int32_t h, int32_t N, double ksigma,
                   int32_t max_iters, double *out, uint8_t *keep, int64_t *n_rej,
                   uint8_t *near, double rel_band, int32_t missing)
{
    if (!aligned || !out) return O_NULL;
    if (w < 1 || h < 1 || N < 1 || N > 4096) return O_SHAPE;
    if (!(ksigma > 0.0) || max_iters < 0) return O_RANGE;
    const int64_t plane = (int64_t)w * h;
    int64_t rejected = 0;
#pragma omp parallel for schedule(static) reduction(+ : rejected)
    for (int64_t p = 0; p < plane; ++p) {
        uint8_t kept[4096];
        uint8_t close[4096];
        int32_t nk = 0;
        for (int32_t k = 0; k < N; ++k) {
            kept[k] = !(missing && isnan(aligned[k * plane + p]));
            nk += kept[k];
            close[k] = 0;
        }
        for (int32_t it = 0; it < max_iters; ++it) {
            double s = 0.0;
            for (int32_t k = 0; k < N; ++k)
                if (kept[k]) s += aligned[k * plane + p];
            const double m = s / nk;
            double q = 0.0;
            for (int32_t k = 0; k < N; ++k)
                if (kept[k]) { double d = aligned[k * plane + p] - m; q += d * d; }
            const double thr = ksigma * sqrt(q / nk);
            int32_t dropped = 0;
            for (int32_t k = 0; k < N; ++k) {
                if (!kept[k]) continue;
                const double dist = fabs(aligned[k * plane + p] - m);
                if (fabs(dist - thr) <= rel_band * thr) close[k] = 1;
                if (dist > thr) { kept[k] = 0; ++dropped; }
            }
            nk -= dropped;
            rejected += dropped;
            if (dropped == 0) break;
        }
        double s = 0.0;
        for (int32_t k = 0; k < N; ++k)
            if (kept[k]) s += aligned[k * plane + p];
        out[p] = s / nk;
        if (keep) for (int32_t k = 0; k < N; ++k) keep[k * plane + p] = kept[k];
        if (near) for (int32_t k = 0; k < N; ++k) near[k * plane + p] = close[k];
    }
    if (n_rej) *n_rej = rejected;
    return O_OK;
}

/* ------------------------------------------------------------------------------
 * 4x4 box downsample (input of the offset-proposal network).
 * ---------------------------------------------------------------------------- */
int oracle_downsample4(const double *in, int32_t W, int32_t H, double *out)
{
    if (!in || !out) return O_NULL;
    if (W < 4 || H < 4 || W % 4 || H % 4) return O_SHAPE;
    const int32_t w = W / 4, h = H / 4;
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < h; ++j)
        for (int32_t i = 0; i < w; ++i) {
            double s = 0.0;
            for (int32_t y = 0; y < 4; ++y)
                for (int32_t x = 0; x < 4; ++x) s += in[(int64_t)(4 * j + y) * W + 4 * i + x];
            out[(int64_t)j * w + i] = s / 16.0;
        }
    return O_OK;
}

/* ------------------------------------------------------------------------------
 * Input of the offset-proposal network: block mean, standardisation by the mean and
 * population standard deviation of the block-mean image, asinh to compress the
 * bright stars, and the bfloat16 rounding of the stored input (via float, ties to
 * even).
 * ---------------------------------------------------------------------------- */
static double to_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

int oracle_cnn_input(const double *in, int32_t W, int32_t H, double *out)
{
    int rc = oracle_downsample4(in, W, H, out);
    if (rc) return rc;
    const int64_t n = (int64_t)(W / 4) * (H / 4);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += out[i];
    const double mean = s / (double)n;
    double q = 0.0;
    for (int64_t i = 0; i < n; ++i) q += (out[i] - mean) * (out[i] - mean);
    const double sd = sqrt(q / (double)n);
    for (int64_t i = 0; i < n; ++i) out[i] = to_bf16(asinh(sd > 0.0 ? (out[i] - mean) / sd : 0.0));
    return O_OK;
}
