// Translation registration by brute-force cross-correlation over a bounded window.
//
//   S_k(d) = sum_{p in T} r'(p) f_k(p + d),   r' = ref - mean_T(ref),   d in window
//
// Work split.  A thread owns one window row dy and K consecutive dx candidates and
// keeps K double accumulators.  For one template row segment of K pixels it reads
// the K template values (LDS broadcast) and 2K-1 frame values (LDS), and performs
// K*K FMAs: the frame value at column m serves every (pixel i, candidate j) pair
// with i + j = m.  A workgroup owns a band of template rows x a column chunk of the
// template ("tile") for a group of candidate rows; the template and frame tiles are
// staged in LDS chunk by chunk (TY template rows at a time, plus the frame rows and
// columns the window needs).  When there are fewer candidates than threads, threads
// also split the chunk's (row, column-block) pairs ("sub-ranges") and their
// accumulators are summed in a fixed order at the end.  Each tile writes one FP64
// partial score per candidate; a second kernel sums the partials over tiles in tile
// order, and a third does the (score, index) max-reduction, the runner-up, the
// parabola vertex and the flags.  All sums are FP64 with FMA; the arithmetic is the
// same for any launch shape up to the summation order.
//
// Roofline: VALU (FP64 FMA).  Algorithmic work per frame: |T| * (2R+1)^2 FMA.
#include <algorithm>
#include <vector>

#include "common.h"
#include "register_plan.h"

namespace rd {

// ---- mean of the reference over the template ---------------------------------
constexpr int MEAN_BLOCK = 256;
constexpr int MEAN_ROWS = 16;

__device__ __forceinline__ double block_sum_f64(double v, double *scratch)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += scratch[i];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(MEAN_BLOCK) void tmpl_sum_rows(const float *__restrict__ ref, int32_t W, int32_t tx0,
                                                            int32_t ty0, int32_t tw, int32_t th,
                                                            double *__restrict__ part)
{
    __shared__ double scratch[MEAN_BLOCK / 64];
    const int32_t y0 = blockIdx.x * MEAN_ROWS;
    const int32_t y1 = min(y0 + MEAN_ROWS, th);
    double s = 0.0;
    for (int32_t y = y0; y < y1; ++y)
        for (int32_t x = threadIdx.x; x < tw; x += MEAN_BLOCK) s += (double)ref[(int64_t)(ty0 + y) * W + tx0 + x];
    s = block_sum_f64(s, scratch);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(MEAN_BLOCK) void tmpl_mean_final(const double *__restrict__ part, int32_t nparts,
                                                              double count, double *__restrict__ mean)
{
    __shared__ double scratch[MEAN_BLOCK / 64];
    double s = 0.0;
    for (int32_t i = threadIdx.x; i < nparts; i += MEAN_BLOCK) s += part[i];
    s = block_sum_f64(s, scratch);
    if (threadIdx.x == 0) *mean = s / count;
}

// ---- partial scores per template tile ------------------------------------------
struct ScoreArgs {
    const float *ref;
    const float *frames;
    const int32_t *centers;
    const double *mean;
    double *partial;        // [N][n_tiles][D*D]
    int32_t W, H, R, Rmax, D;
    int32_t tx0, ty0, tw, th;
    int32_t TY, TX, NXB, BR, NBX, C, CW, S, JS, FR, FC, n_xchunks, n_tiles, N, G;
};

// Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous run of logical work items (tile fastest, then candidate group, then
// frame) so that neighbouring tiles, which share frame rows and columns, hit the
// same L2.
__device__ __forceinline__ int32_t xcd_logical_id(int32_t lin, int32_t total)
{
    constexpr int32_t NXCD = 8;
    const int32_t per = total / NXCD, rem = total % NXCD;
    const int32_t x = lin % NXCD, slot = lin / NXCD;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + slot;
}

template <int K>
__global__ __launch_bounds__(512) void score_tiles(ScoreArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *rt = reinterpret_cast<double *>(smem);                         // [TY][TX]
    float *ft = reinterpret_cast<float *>(smem + sizeof(double) * a.TY * a.TX);  // [FR][FC]

    const int32_t G = a.G;
    const int32_t total = a.n_tiles * G * a.N;
    const int32_t lid = xcd_logical_id((int32_t)blockIdx.x, total);
    const int32_t tile = lid % a.n_tiles;
    const int32_t gk = lid / a.n_tiles;
    const int32_t g = gk % G;
    const int32_t k = gk / G;
    const int32_t band = tile / a.n_xchunks;
    const int32_t xc = tile - band * a.n_xchunks;
    const int32_t c0 = g * a.CW;
    const int32_t x_t = xc * a.TX;                 // first template column of the tile
    const int32_t yb0 = band * a.BR;               // first template row of the band
    const int32_t yb1 = min(yb0 + a.BR, a.th);
    const int32_t cx = a.centers ? a.centers[2 * k] : 0;
    const int32_t cy = a.centers ? a.centers[2 * k + 1] : 0;
    const int32_t j_lo = c0 / a.NBX;

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int nwaves = blockDim.x >> 6;
    const int cl = t % a.CW;
    const int s = t / a.CW;
    const int c = c0 + cl;
    const bool active = (s < a.S) && (cl < a.CW) && (c < a.C);
    const int j = active ? c / a.NBX : j_lo;
    const int bx = active ? c - j * a.NBX : 0;
    const int jr = j - j_lo;                       // frame-tile row offset of this thread

    const double mean = *a.mean;
    const float *f = a.frames + (int64_t)k * a.W * a.H;
    // frame tile origin: template row yc + (cy - R + j_lo), column x_t + (cx - R)
    const int32_t fx0 = a.tx0 + x_t + cx - a.R;

    double acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0;

    const int pairs = a.TY * a.NXB;
    for (int32_t yc = yb0; yc < yb1; yc += a.TY) {
        __syncthreads();
        // template tile, zero outside T (contributes exactly nothing); one wave per row
        for (int yy = wave; yy < a.TY; yy += nwaves) {
            const bool row_ok = yc + yy < yb1;
            const float *src = a.ref + (int64_t)(a.ty0 + yc + yy) * a.W + a.tx0 + x_t;
            for (int xx = lane; xx < a.TX; xx += 64) {
                double v = 0.0;
                if (row_ok && x_t + xx < a.tw) v = (double)src[xx] - mean;
                rt[yy * a.TX + xx] = v;
            }
        }
        // frame tile, zero outside the frame; one wave per row
        const int32_t fy0 = a.ty0 + yc + cy - a.R + j_lo;
        for (int rr = wave; rr < a.FR; rr += nwaves) {
            const int32_t gy = fy0 + rr;
            const bool row_ok = gy >= 0 && gy < a.H;
            const float *src = f + (int64_t)gy * a.W;
            for (int cc = lane; cc < a.FC; cc += 64) {
                const int32_t gx = fx0 + cc;
                float v = 0.0f;
                if (row_ok && gx >= 0 && gx < a.W) v = src[gx];
                ft[rr * a.FC + cc] = v;
            }
        }
        __syncthreads();
        if (active) {
            for (int pr = s; pr < pairs; pr += a.S) {
                const int yy = pr / a.NXB;
                const int xb = pr - yy * a.NXB;
                const double *rrow = rt + yy * a.TX + xb * K;
                const float *frow = ft + (yy + jr) * a.FC + (xb + bx) * K;
                double r[K];
#pragma unroll
                for (int i = 0; i < K; ++i) r[i] = rrow[i];
#pragma unroll
                for (int m = 0; m < 2 * K - 1; ++m) {
                    const double fv = (double)frow[m];
#pragma unroll
                    for (int i = 0; i < K; ++i) {
                        const int q = m - i;
                        if (q >= 0 && q < K) acc[q] = fma(r[i], fv, acc[q]);
                    }
                }
            }
        }
    }

    // sum the sub-ranges in order s = 0, 1, ... (only needed when S > 1)
    __syncthreads();
    double *red = reinterpret_cast<double *>(smem);  // [CW][K]
    if (a.S > 1) {
        for (int ss = 0; ss < a.S; ++ss) {
            if (active && s == ss) {
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    double *slot = red + cl * K + q;
                    *slot = (ss == 0) ? acc[q] : *slot + acc[q];
                }
            }
            __syncthreads();
        }
    }
    if (active && s == 0) {
        double *out = a.partial + ((int64_t)k * a.n_tiles + tile) * (int64_t)a.D * a.D + (int64_t)j * a.D;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int i = bx * K + q;
            if (i < a.D) out[i] = (a.S > 1) ? red[cl * K + q] : acc[q];
        }
    }
}

// ---- sum of partials over tiles, window clip --------------------------------------
__global__ __launch_bounds__(256) void sum_tiles(const double *__restrict__ partial, int32_t n_tiles, int32_t D,
                                                 int32_t R, int32_t Rmax, const int32_t *__restrict__ centers,
                                                 double *__restrict__ scores)
{
    const int32_t k = blockIdx.y;
    const int32_t cand = blockIdx.x * 256 + threadIdx.x;
    if (cand >= D * D) return;
    const int32_t jj = cand / D, ii = cand - jj * D;
    const int32_t cx = centers ? centers[2 * k] : 0, cy = centers ? centers[2 * k + 1] : 0;
    const int32_t dx = cx - R + ii, dy = cy - R + jj;
    double s = -INFINITY;
    if (dx >= -Rmax && dx <= Rmax && dy >= -Rmax && dy <= Rmax) {
        s = 0.0;
        const double *p = partial + (int64_t)k * n_tiles * D * D + cand;
        for (int32_t tI = 0; tI < n_tiles; ++tI) s += p[(int64_t)tI * D * D];
    }
    scores[(int64_t)k * D * D + cand] = s;
}

// ---- argmax, runner-up, parabola -------------------------------------------------
struct Best {
    double s;
    int32_t i;
};

__device__ __forceinline__ Best better_of(Best a, Best b)
{
    if (a.s > b.s) return a;
    if (b.s > a.s) return b;
    return a.i <= b.i ? a : b;
}

__device__ Best block_best(Best v, Best *scratch)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Best o;
        o.s = __shfl_xor(v.s, off, 64);
        o.i = __shfl_xor(v.i, off, 64);
        v = better_of(v, o);
    }
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    Best r = scratch[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = better_of(r, scratch[w]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double parabola_vertex(double sm, double s0, double sp)
{
    const double den = 2.0 * (sm - 2.0 * s0 + sp);
    if (!(den < 0.0)) return 0.0;
    double d = (sm - sp) / den;
    if (d > 0.5) d = 0.5;
    if (d < -0.5) d = -0.5;
    return d;
}

__global__ __launch_bounds__(256) void pick_offsets(const double *__restrict__ scores, int32_t D, int32_t R,
                                                    int32_t Rmax, const int32_t *__restrict__ centers,
                                                    reduce_offset_t *__restrict__ out)
{
    __shared__ Best scratch[4];
    const int32_t k = blockIdx.x;
    const double *S = scores + (int64_t)k * D * D;
    const int32_t cx = centers ? centers[2 * k] : 0, cy = centers ? centers[2 * k + 1] : 0;
    const int32_t lox = max(cx - R, -Rmax), hix = min(cx + R, Rmax);
    const int32_t loy = max(cy - R, -Rmax), hiy = min(cy + R, Rmax);
    const bool empty = lox > hix || loy > hiy;

    Best b{-INFINITY, 0x7fffffff};
    for (int32_t c = threadIdx.x; c < D * D; c += blockDim.x) {
        const int32_t jj = c / D, ii = c - jj * D;
        const int32_t dx = cx - R + ii, dy = cy - R + jj;
        if (dx < lox || dx > hix || dy < loy || dy > hiy) continue;
        b = better_of(b, Best{S[c], c});
    }
    const Best best = block_best(b, scratch);
    Best sb{-INFINITY, 0x7fffffff};
    for (int32_t c = threadIdx.x; c < D * D; c += blockDim.x) {
        const int32_t jj = c / D, ii = c - jj * D;
        const int32_t dx = cx - R + ii, dy = cy - R + jj;
        if (dx < lox || dx > hix || dy < loy || dy > hiy || c == best.i) continue;
        sb = better_of(sb, Best{S[c], c});
    }
    const Best second = block_best(sb, scratch);
    if (threadIdx.x != 0) return;

    reduce_offset_t o;
    if (empty) {
        o.dx = o.dy = 0;
        o.sx = o.sy = 0.0f;
        o.peak = o.second = -INFINITY;
        o.margin = 0.0;
        o.flags = REDUCE_CLIPPED | REDUCE_EDGE_X | REDUCE_EDGE_Y | REDUCE_NEAR_TIE;
        o.pad = 0;
        out[k] = o;
        return;
    }
    const int32_t bj = best.i / D, bi = best.i - bj * D;
    const int32_t bdx = cx - R + bi, bdy = cy - R + bj;
    int32_t flags = 0;
    double delx = 0.0, dely = 0.0;
    if (bdx == lox || bdx == hix) flags |= REDUCE_EDGE_X;
    else delx = parabola_vertex(S[best.i - 1], best.s, S[best.i + 1]);
    if (bdy == loy || bdy == hiy) flags |= REDUCE_EDGE_Y;
    else dely = parabola_vertex(S[best.i - D], best.s, S[best.i + D]);
    if (lox != cx - R || hix != cx + R || loy != cy - R || hiy != cy + R) flags |= REDUCE_CLIPPED;
    double margin;
    if (second.s == -INFINITY) margin = INFINITY;
    else if (best.s == 0.0) margin = (best.s > second.s) ? INFINITY : 0.0;
    else margin = (best.s - second.s) / fabs(best.s);
    if (margin < REDUCE_NEAR_TIE_MARGIN) flags |= REDUCE_NEAR_TIE;
    o.dx = bdx;
    o.dy = bdy;
    o.sx = (float)((double)bdx + delx);
    o.sy = (float)((double)bdy + dely);
    o.peak = best.s;
    o.second = second.s;
    o.margin = margin;
    o.flags = flags;
    o.pad = 0;
    out[k] = o;
}

// ---- host side ---------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct RegWs {
    size_t mean_parts, mean, partial, scores, total;
};

static RegWs reg_ws_layout(const RegPlan &p, int32_t N, int32_t th_max)
{
    RegWs w;
    const int32_t nparts = (int32_t)ceil_div(th_max, MEAN_ROWS);
    w.mean_parts = 0;
    w.mean = align256(sizeof(double) * nparts);
    w.partial = w.mean + 256;
    w.scores = w.partial + align256(sizeof(double) * (size_t)N * p.n_tiles * p.D * p.D);
    w.total = w.scores + align256(sizeof(double) * (size_t)N * p.D * p.D);
    return w;
}

template <int K>
static void launch_score(const ScoreArgs &a, const RegPlan &p, int32_t N, hipStream_t s)
{
    ProfScope prof("score_tiles", s);
    hipLaunchKernelGGL(score_tiles<K>, dim3((unsigned)((int64_t)p.n_tiles * p.G * N)), dim3(p.threads), p.lds, s,
                       a);
}

int register_launch(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N, int32_t R,
                    int32_t Rmax, const int32_t *centers, int32_t tx0, int32_t ty0, int32_t tw, int32_t th,
                    reduce_offset_t *out, double *scores, void *ws, const RegPlan &p, hipStream_t s)
{
    const RegWs L = reg_ws_layout(p, N, p.th_max);
    unsigned char *base = static_cast<unsigned char *>(ws);
    double *mean_parts = reinterpret_cast<double *>(base + L.mean_parts);
    double *mean = reinterpret_cast<double *>(base + L.mean);
    double *partial = reinterpret_cast<double *>(base + L.partial);
    double *sc = scores ? scores : reinterpret_cast<double *>(base + L.scores);

    const int32_t nparts = (int32_t)ceil_div(th, MEAN_ROWS);
    hipLaunchKernelGGL(tmpl_sum_rows, dim3(nparts), dim3(MEAN_BLOCK), 0, s, ref, W, tx0, ty0, tw, th, mean_parts);
    hipLaunchKernelGGL(tmpl_mean_final, dim3(1), dim3(MEAN_BLOCK), 0, s, mean_parts, nparts, (double)tw * (double)th,
                       mean);

    RegPlan q = p;
    q.n_bands = (int32_t)ceil_div(th, p.BR);
    q.n_xchunks = (int32_t)ceil_div(tw, p.TX);
    q.n_tiles = q.n_bands * q.n_xchunks;
    ScoreArgs a;
    a.ref = ref;
    a.frames = frames;
    a.centers = centers;
    a.mean = mean;
    a.partial = partial;
    a.W = W; a.H = H; a.R = R; a.Rmax = Rmax; a.D = p.D;
    a.tx0 = tx0; a.ty0 = ty0; a.tw = tw; a.th = th;
    a.TY = p.TY; a.TX = p.TX; a.NXB = p.NXB; a.BR = p.BR; a.NBX = p.NBX; a.C = p.C; a.CW = p.CW; a.S = p.S;
    a.JS = p.JS; a.FR = p.FR; a.FC = p.FC; a.n_xchunks = q.n_xchunks; a.n_tiles = q.n_tiles; a.N = N; a.G = p.G;
    switch (p.K) {
    case 5: launch_score<5>(a, q, N, s); break;
    case 9: launch_score<9>(a, q, N, s); break;
    case 12: launch_score<12>(a, q, N, s); break;
    case 17: launch_score<17>(a, q, N, s); break;
    case 18: launch_score<18>(a, q, N, s); break;
    default: launch_score<22>(a, q, N, s); break;
    }
    hipLaunchKernelGGL(sum_tiles, dim3((unsigned)ceil_div((int64_t)p.D * p.D, 256), N), dim3(256), 0, s, partial,
                       q.n_tiles, p.D, R, Rmax, centers, sc);
    hipLaunchKernelGGL(pick_offsets, dim3(N), dim3(256), 0, s, sc, p.D, R, Rmax, centers, out);
    return check_launch("reduce_register");
}

size_t register_ws_bytes(const RegPlan &p, int32_t N) { return reg_ws_layout(p, N, p.th_max).total; }

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_register_ws(int32_t W, int32_t H, int32_t N, int32_t radius, int32_t radius_max)
{
    if (W < 1 || H < 1 || N < 1 || radius < 0 || radius_max < 0) return 0;
    if (W - 2 * radius_max < 1 || H - 2 * radius_max < 1) return 0;
    const RegPlan p = reg_plan(W, H, N, radius, radius_max);
    if (p.D == 0) return 0;
    return register_ws_bytes(p, N);
}

extern "C" int reduce_register(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                               int32_t radius, int32_t radius_max, const int32_t *centers, const int32_t *tmpl,
                               reduce_offset_t *out, double *scores, void *ws, size_t ws_bytes, void *stream)
{
    if (!ref || !frames || !out) return fail(REDUCE_ERR_NULL, "reduce_register: NULL buffer");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_register: W, H, N must be >= 1");
    if (radius < 0 || radius_max < 0) return fail(REDUCE_ERR_RANGE, "reduce_register: negative radius");
    if (radius > 1024) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_register: radius above 1024");
    if (W - 2 * radius_max < 1 || H - 2 * radius_max < 1)
        return fail(REDUCE_ERR_RANGE, "reduce_register: radius_max leaves no template");
    int32_t tx0 = radius_max, ty0 = radius_max, tw = W - 2 * radius_max, th = H - 2 * radius_max;
    if (tmpl) {
        tx0 = tmpl[0]; ty0 = tmpl[1]; tw = tmpl[2]; th = tmpl[3];
        if (tw < 1 || th < 1) return fail(REDUCE_ERR_SHAPE, "reduce_register: empty template");
        if (tx0 - radius_max < 0 || ty0 - radius_max < 0 || (int64_t)tx0 + tw + radius_max > W ||
            (int64_t)ty0 + th + radius_max > H)
            return fail(REDUCE_ERR_RANGE, "reduce_register: template dilated by radius_max leaves the frame");
    }
    if (N > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_register: N above 65535");
    const RegPlan p = reg_plan(W, H, N, radius, radius_max);
    if (p.D == 0) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_register: window too large for any launch shape");
    const size_t need = register_ws_bytes(p, N);
    if (!ws || ws_bytes < need)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_register: workspace needs " + std::to_string(need) + " bytes");
    return register_launch(ref, frames, W, H, N, radius, radius_max, centers, tx0, ty0, tw, th, out, scores, ws, p,
                           as_stream(stream));
}
