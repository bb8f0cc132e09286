// Device bodies of the correlation search, shared by the stage-wise kernels and the
// persistent batch kernel so that both produce bit-identical scores and offsets:
//
//   S_k(d) = sum_{p in T} r'(p) f_k(p + d),   r' = ref - mean_T(ref),   d in window
//
// Work split.  A thread owns one window row dy and K consecutive dx candidates and
// keeps K double accumulators.  For one template row segment of K pixels it reads
// the K template values (LDS broadcast) and 2K-1 frame values, and performs K*K FMAs:
// the frame value at column m serves every (pixel i, candidate j) pair with
// i + j = m.  It walks the column blocks of a template row in order, so K - 1 of the
// frame values (already converted to FP64) carry over to the next block and only K
// are read anew.  A work item ("tile") is a band of template rows x a column chunk
// of the template for one group of candidate rows of one frame; the template and
// frame tiles are staged in LDS chunk by chunk (TY template rows at a time, plus the
// frame rows and columns the window needs).  When there are fewer candidates than
// threads, threads also split the chunk's template rows ("sub-ranges": rows s,
// s + S, ...) and their accumulators are summed in a fixed order.  Each tile writes one FP64
// partial score per candidate; partials are summed over tiles in tile order, and the
// (score, index) maximum, the runner-up, the parabola vertex and the flags follow.
// The decomposition depends only on (W, H, R, Rmax) and the launch shape, never on
// the number of frames, so every path that uses the same shape sums in the same
// order.
#pragma once

#include <type_traits>

#include "common.h"

namespace rd {

constexpr int MEAN_THREADS = 256;  // logical threads of the template-mean reduction
constexpr int MEAN_ROWS = 2;       // template rows per mean part
constexpr int MEAN_U = 4;          // columns per thread loaded together

struct ScoreArgs {
    const float *ref;
    const float *frames;     // frame k at frames + (k + (k >= skip)) * W * H
    const int32_t *centers;  // [N][2] or NULL (indexed by frame when map is set, else by k)
    const int32_t *map;      // [N] frame of work slot k (negative: nothing to do), or NULL
    const double *mean;
    double *partial;         // [N][n_tiles][D*D]
    int32_t W, H, R, Rmax, D;
    int32_t tx0, ty0, tw, th;
    int32_t TY, TX, NXB, BR, NBX, C, CW, S, JS, FR, FC, n_xchunks, n_tiles, N, G;
    int32_t threads;         // threads taking part (the first `threads` of the block)
    int32_t skip;            // index of a frame to step over (the reference), or a large value
};

// ---- template mean ---------------------------------------------------------------
// Sum over a wave then over the first `waves` waves in order; threads that have no
// data contribute exactly zero.
__device__ __forceinline__ double block_sum_f64(double v, double *scratch, int waves)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0 && w < waves) scratch[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < waves; ++i) t += scratch[i];
    __syncthreads();
    return t;
}

// Sum of template rows [MEAN_ROWS*part, +MEAN_ROWS) with MEAN_THREADS logical threads
// striding over columns; valid in thread 0.  A thread loads MEAN_U columns of a row
// before adding them, in column order.
__device__ __forceinline__ double tmpl_part_sum(const float *ref, int32_t W, int32_t tx0, int32_t ty0, int32_t tw,
                                                int32_t th, int32_t part, double *scratch)
{
    const int32_t y0 = part * MEAN_ROWS;
    const int32_t y1 = min(y0 + MEAN_ROWS, th);
    double s = 0.0;
    if (threadIdx.x < MEAN_THREADS)
        for (int32_t y = y0; y < y1; ++y) {
            const float *row = ref + (int64_t)(ty0 + y) * W + tx0;
            for (int32_t x0 = threadIdx.x; x0 < tw; x0 += MEAN_U * MEAN_THREADS) {
                float v[MEAN_U];
#pragma unroll
                for (int u = 0; u < MEAN_U; ++u) {
                    const int32_t x = x0 + u * MEAN_THREADS;
                    v[u] = row[x < tw ? x : 0];
                }
#pragma unroll
                for (int u = 0; u < MEAN_U; ++u)
                    if (x0 + u * MEAN_THREADS < tw) s += (double)v[u];
            }
        }
    return block_sum_f64(s, scratch, MEAN_THREADS / 64);
}

__device__ __forceinline__ double tmpl_mean_of_parts(const double *part, int32_t nparts, double count,
                                                     double *scratch)
{
    double s = 0.0;
    if (threadIdx.x < MEAN_THREADS)
        for (int32_t i = threadIdx.x; i < nparts; i += MEAN_THREADS) s += part[i];
    s = block_sum_f64(s, scratch, MEAN_THREADS / 64);
    return s / count;  // valid in thread 0
}

// ---- LDS staging -----------------------------------------------------------------------------
// Copy a rows x cols tile into LDS: element e = t, t + nthreads, ... is (e / cols, e % cols).
// Each thread issues STAGE_U loads before it stores any of them, so their latencies
// overlap; an element outside the source (ok == false) is loaded from offset 0 and
// stored as zero, which keeps the loads branch-free.
constexpr int STAGE_U = 8;

template <typename Addr, typename Store>
__device__ __forceinline__ void stage_tile(int rows, int cols, int nthreads, int t, Addr addr,
                                           const float *__restrict__ src, Store store)
{
    const int n = rows * cols;
    const int dr = nthreads / cols, dc = nthreads - dr * cols;
    int r = t / cols, c = t - r * cols;
    for (int e = t; e < n; e += STAGE_U * nthreads) {
        float v[STAGE_U];
        int lr[STAGE_U], lc[STAGE_U];
        bool ok[STAGE_U];
#pragma unroll
        for (int u = 0; u < STAGE_U; ++u) {
            lr[u] = r;
            lc[u] = c;
            bool in = false;
            const int64_t off = addr(r, c, in);
            ok[u] = in && e + u * nthreads < n;
            v[u] = src[ok[u] ? off : 0];
            c += dc;
            r += dr;
            if (c >= cols) {
                c -= cols;
                ++r;
            }
        }
#pragma unroll
        for (int u = 0; u < STAGE_U; ++u)
            if (e + u * nthreads < n) store(lr[u], lc[u], ok[u], v[u]);
    }
}

// ---- one tile of partial scores ----------------------------------------------------------
// lid in [0, n_tiles * G * N): tile fastest, then candidate group, then frame.
template <int K>
__device__ __forceinline__ void score_tile(const ScoreArgs &a, int32_t lid, unsigned char *smem)
{
    double *rt = reinterpret_cast<double *>(smem);                               // [TY][TX]
    float *ft = reinterpret_cast<float *>(smem + sizeof(double) * a.TY * a.TX);  // [FR][FC]

    const int32_t tile = lid % a.n_tiles;
    const int32_t gk = lid / a.n_tiles;
    const int32_t g = gk % a.G;
    const int32_t k = gk / a.G;
    const int32_t kf = a.map ? a.map[k] : k + (k >= a.skip ? 1 : 0);
    if (kf < 0) return;  // an idle slot: the whole workgroup leaves before any barrier
    const int32_t ci = a.map ? kf : k;
    const int32_t band = tile / a.n_xchunks;
    const int32_t xc = tile - band * a.n_xchunks;
    const int32_t c0 = g * a.CW;
    const int32_t x_t = xc * a.TX;                 // first template column of the tile
    const int32_t yb0 = band * a.BR;               // first template row of the band
    const int32_t yb1 = min(yb0 + a.BR, a.th);
    const int32_t cx = a.centers ? a.centers[2 * ci] : 0;
    const int32_t cy = a.centers ? a.centers[2 * ci + 1] : 0;
    const int32_t j_lo = c0 / a.NBX;

    const int t = threadIdx.x;
    const bool in_block = t < a.threads;
    const int cl = t % a.CW;
    const int s = t / a.CW;
    const int c = c0 + cl;
    const bool active = in_block && (s < a.S) && (c < a.C);
    const int j = active ? c / a.NBX : j_lo;
    const int bx = active ? c - j * a.NBX : 0;
    const int jr = j - j_lo;                       // frame-tile row offset of this thread

    const double mean = *a.mean;
    const float *f = a.frames + (int64_t)kf * a.W * a.H;
    // frame tile origin: template row yc + (cy - R + j_lo), column x_t + (cx - R)
    const int32_t fx0 = a.tx0 + x_t + cx - a.R;

    double acc[K];
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] = 0.0;

    // The frame tile is a ring of FR rows: chunk c (template rows yc = yb0 + c * TY ...) needs
    // frame rows fy(c) + [0, FR), fy(c) = fy(0) + c * TY, and keeps them in LDS rows
    // (c * TY + r) mod FR; from the second chunk on only the TY rows it adds are staged,
    // into the LDS rows of the TY rows the previous chunk alone needed.
    int32_t ring0 = 0;  // LDS row of the chunk's frame row 0
    for (int32_t yc = yb0; yc < yb1; yc += a.TY) {
        __syncthreads();
        if (in_block) {
            // template tile (zero outside T: contributes exactly nothing), then the frame
            // rows (zero outside the frame)
            stage_tile(a.TY, a.TX, a.threads, t, [&](int r, int c, bool &ok) -> int64_t {
                ok = yc + r < yb1 && x_t + c < a.tw;
                return (int64_t)(a.ty0 + yc + r) * a.W + a.tx0 + x_t + c;
            }, a.ref, [&](int r, int c, bool ok, float v) { rt[r * a.TX + c] = ok ? (double)v - mean : 0.0; });
            const int32_t fy0 = a.ty0 + yc + cy - a.R + j_lo;
            const int32_t r0 = yc == yb0 ? 0 : a.FR - a.TY;  // first chunk row to stage
            stage_tile(a.FR - r0, a.FC, a.threads, t, [&](int r, int c, bool &ok) -> int64_t {
                const int32_t gy = fy0 + r0 + r, gx = fx0 + c;
                ok = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
                return (int64_t)gy * a.W + gx;
            }, f, [&](int r, int c, bool ok, float v) {
                int32_t lr = ring0 + r0 + r;
                if (lr >= a.FR) lr -= a.FR;
                ft[lr * a.FC + c] = ok ? v : 0.0f;
            });
        }
        __syncthreads();
        if (active) {
            // rows s, s + S, ...: the column blocks of a row in order; the K - 1 frame values a
            // block shares with the next stay in registers, converted once
            constexpr int NXB = (64 + K - 1) / K;  // column blocks per tile row (TX = K * NXB)
            for (int yy = s; yy < a.TY; yy += a.S) {
                int32_t lr = ring0 + yy + jr;  // < 2 FR
                if (lr >= a.FR) lr -= a.FR;
                const double *rrow = rt + yy * a.TX;
                const float *frow = ft + lr * a.FC + bx * K;
                double w[2 * K - 1];
#pragma unroll
                for (int m = 0; m < K - 1; ++m) w[m] = (double)frow[m];
#pragma unroll
                for (int xb = 0; xb < NXB; ++xb) {
#pragma unroll
                    for (int m = K - 1; m < 2 * K - 1; ++m) w[m] = (double)frow[xb * K + m];
                    double r[K];
#pragma unroll
                    for (int i = 0; i < K; ++i) r[i] = rrow[xb * K + i];
#pragma unroll
                    for (int m = 0; m < 2 * K - 1; ++m) {
#pragma unroll
                        for (int i = 0; i < K; ++i) {
                            const int q = m - i;
                            if (q >= 0 && q < K) acc[q] = fma(r[i], w[m], acc[q]);
                        }
                    }
#pragma unroll
                    for (int m = 0; m < K - 1; ++m) w[m] = w[m + K];
                }
            }
        }
        ring0 += a.TY % a.FR;
        if (ring0 >= a.FR) ring0 -= a.FR;
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
    __syncthreads();  // LDS is reused by the caller's next item
}

// ---- small windows (side D <= 5) ------------------------------------------------------------
// A tile is BR template rows (the plan's, a multiple of SMALL_CH of at most SMALL_ROWS)
// x SMALL_COLS template columns for one workgroup of
// SMALL_COLS threads; thread t owns template column SMALL_COLS * colblock + t and walks down
// the tile with all D x D candidate sums in registers.  The frame rows a template row needs
// (D of them, one per window row) slide down with it in a register ring of D rows, converted
// to FP64 once; the newest row of the ring comes from LDS, where the workgroup stages the
// frame in chunks of SMALL_CH rows x SMALL_FC columns, double-buffered: the loads of the next
// chunk (and its template values) are issued before the current chunk is computed, so one
// barrier per chunk is the only wait.  At the end each sum is reduced over the wave with a
// fixed butterfly and over the waves in wave order, and written as the tile's partial in the
// layout of the general kernel.
constexpr int SMALL_COLS = 256;                       // template columns per tile, one per thread
constexpr int SMALL_CH = 15;                          // template rows per chunk (a multiple of every D)
constexpr int SMALL_ROWS = 16 * SMALL_CH;             // most template rows per tile
constexpr int SMALL_FC = SMALL_COLS + 4;              // frame columns per staged row (>= SMALL_COLS + D - 1)
constexpr int SMALL_LDS_FLOATS = 2 * SMALL_CH * SMALL_FC + SMALL_COLS;  // both chunk buffers, one spare slot per thread
constexpr int SMALL_D_MAX = 5;
static_assert(SMALL_CH % 15 == 0, "chunk rows must be a multiple of 1, 3 and 5");
static_assert(4 * SMALL_CH <= SMALL_COLS && SMALL_FC - SMALL_COLS == 4, "extra staged columns");
static_assert(SMALL_LDS_FLOATS * 4 >= 8 * (SMALL_COLS / 64) * SMALL_D_MAX * SMALL_D_MAX, "reduction scratch");

template <int D>
__device__ __forceinline__ void score_small_tile(const ScoreArgs &a, int32_t lid, float *__restrict__ fl)
{
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int32_t tile = lid % a.n_tiles, k = lid / a.n_tiles;
    const int32_t kf = a.map ? a.map[k] : k + (k >= a.skip ? 1 : 0);
    if (kf < 0) return;  // an idle slot: the whole workgroup leaves before any barrier
    const int32_t ci = a.map ? kf : k;
    const int32_t strip = tile / a.n_xchunks, colb = tile - strip * a.n_xchunks;
    const int32_t x = colb * SMALL_COLS + t;
    const bool col_ok = x < a.tw;
    const int32_t y0 = strip * a.BR, rows = min(y0 + a.BR, a.th) - y0;
    const int nch = (rows + SMALL_CH - 1) / SMALL_CH;
    const int32_t cx = a.centers ? a.centers[2 * ci] : 0, cy = a.centers ? a.centers[2 * ci + 1] : 0;
    const float *f = a.frames + (int64_t)kf * a.W * a.H;
    const double mean = *a.mean;
    // staged column c is frame column fx0 + c, clamped into the frame (an offset beyond
    // +-Rmax is discarded when the tiles are summed, so any in-frame value will do); frame
    // row of window row 0 at template row y0 is fy0; chunk ch holds frame rows
    // fy0 + D - 1 + ch * SMALL_CH + [0, SMALL_CH), clamped likewise
    const int32_t fx0 = a.tx0 + colb * SMALL_COLS + cx - a.R;
    const int32_t fy0 = a.ty0 + y0 + cy - a.R;
    // 32-bit element offsets (a frame holds fewer than 2^31 pixels)
    const uint32_t W = (uint32_t)a.W;
    const float *tcol = a.ref + a.tx0 + (col_ok ? x : 0);
    const int32_t ty_last = a.ty0 + y0 + rows - 1;

    // staging: thread t loads column t of every chunk row, and threads t < 4 * SMALL_CH also
    // one of the SMALL_FC - SMALL_COLS extra columns (row t / 4, column SMALL_COLS + t % 4);
    // row offsets are uniform over the workgroup
    const int32_t gxm = min(max(fx0 + t, 0), a.W - 1);
    const bool has_x = t < 4 * SMALL_CH;
    const int xr = has_x ? t >> 2 : 0, xc = SMALL_COLS + (t & 3);
    const int32_t gxx = min(max(fx0 + xc, 0), a.W - 1);
    float pf[SMALL_CH], pfx;
    auto load_chunk = [&](int ch) {
        const int32_t gy0 = fy0 + D - 1 + ch * SMALL_CH;
#pragma unroll
        for (int r = 0; r < SMALL_CH; ++r) pf[r] = f[(uint32_t)min(max(gy0 + r, 0), a.H - 1) * W + (uint32_t)gxm];
        pfx = f[(uint32_t)min(max(gy0 + xr, 0), a.H - 1) * W + (uint32_t)gxx];
    };
    // branch-free: a thread without an extra value writes it to its spare slot
    const int xslot = has_x ? xr * SMALL_FC + xc : 2 * SMALL_CH * SMALL_FC + t;
    auto store_chunk = [&](int buf) {
        float *dst = fl + buf * (SMALL_CH * SMALL_FC);
#pragma unroll
        for (int r = 0; r < SMALL_CH; ++r) dst[r * SMALL_FC + t] = pf[r];
        fl[has_x ? buf * (SMALL_CH * SMALL_FC) + xslot : xslot] = pfx;
    };
    // template value of row y0 + yl of this thread's column (rows past the tile repeat its last)
    auto tmpl_at = [&](int32_t yl) { return tcol[(uint32_t)min(a.ty0 + y0 + yl, ty_last) * W]; };

    load_chunk(0);  // in flight together with the ring's first rows and the first template values
    // the ring starts with frame rows fy0 .. fy0 + D - 2 (window rows 0 .. D-2 of template row 0)
    double ring[D][D];
#pragma unroll
    for (int i = 0; i + 1 < D; ++i) {
        const float *row = f + (uint32_t)min(max(fy0 + i, 0), a.H - 1) * W;
#pragma unroll
        for (int j = 0; j < D; ++j) ring[i][j] = (double)row[min(max(fx0 + t + j, 0), a.W - 1)];
    }
    double acc[D * D];
#pragma unroll
    for (int q = 0; q < D * D; ++q) acc[q] = 0.0;
    const double colw = col_ok ? 1.0 : 0.0;

    // template values one chunk ahead: tv[p] holds row ch * SMALL_CH + p while chunk ch is
    // computed and is refilled with row (ch + 1) * SMALL_CH + p right after its use
    float tv[SMALL_CH];
#pragma unroll
    for (int p = 0; p < SMALL_CH; ++p) tv[p] = tmpl_at(p);
    store_chunk(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        // the loads and stores of the next chunk are unconditional (rows are clamped into
        // the frame; after the last chunk they fill the idle buffer, which is not read), so
        // the loop body stays one block and the compiler keeps the computation in place
        load_chunk(ch + 1);
        const float *src = fl + (ch & 1) * (SMALL_CH * SMALL_FC) + t;
        // the staged row of template row p + 1 is read while row p is computed
        float nxt[D];
#pragma unroll
        for (int j = 0; j < D; ++j) nxt[j] = src[j];
#pragma unroll
        for (int p = 0; p < SMALL_CH; ++p) {
            // frame row of window row D-1 for template row ch * SMALL_CH + p enters the ring
#pragma unroll
            for (int j = 0; j < D; ++j) ring[(p + D - 1) % D][j] = (double)nxt[j];
            if (p + 1 < SMALL_CH) {
#pragma unroll
                for (int j = 0; j < D; ++j) nxt[j] = src[(p + 1) * SMALL_FC + j];
            }
            // zero weight for columns past the template and rows past the tile
            const double rv = ((double)tv[p] - mean) * (ch * SMALL_CH + p < rows ? colw : 0.0);
            tv[p] = tmpl_at((ch + 1) * SMALL_CH + p);
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) acc[i * D + j] = fma(rv, ring[(p + i) % D][j], acc[i * D + j]);
            __builtin_amdgcn_sched_barrier(0);  // one row at a time: bounds the registers in flight
        }
        store_chunk((ch + 1) & 1);
        __syncthreads();
    }
    // wave butterflies, then the waves in order
    double *red = reinterpret_cast<double *>(fl);
#pragma unroll
    for (int q = 0; q < D * D; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == q) red[wave * (D * D) + q] = v;
    }
    __syncthreads();
    if (t < D * D) {
        double v = red[t];
#pragma unroll
        for (int w = 1; w < SMALL_COLS / 64; ++w) v += red[w * (D * D) + t];
        a.partial[((int64_t)k * a.n_tiles + tile) * (int64_t)(D * D) + t] = v;
    }
    __syncthreads();  // LDS is reused by the caller's next item
}

template <typename F>
__device__ __forceinline__ void small_dispatch(int D, F &&f)
{
    switch (D) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    default: f(std::integral_constant<int, 5>{}); break;
    }
}

template <typename F>
__device__ __forceinline__ void score_dispatch(int K, F &&f)
{
    switch (K) {
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    case 17: f(std::integral_constant<int, 17>{}); break;
    case 18: f(std::integral_constant<int, 18>{}); break;
    default: f(std::integral_constant<int, 22>{}); break;
    }
}

// ---- sum of tile partials ------------------------------------------------------------------
// Candidates 64*cblock .. +63 of one frame, by a workgroup of 64*SUM_WAVES threads: wave w
// sums tiles w, w + SUM_WAVES, ... in order, then the SUM_WAVES partial sums are added in
// wave order, so every path that uses this routine gets the same bits.  -inf outside the
// clipped window.
constexpr int SUM_WAVES = 8;

__device__ __forceinline__ void sum_candidate_block(const double *__restrict__ partial_k, int32_t n_tiles,
                                                    int32_t D, int32_t R, int32_t Rmax, int32_t cx, int32_t cy,
                                                    int32_t cblock, double *__restrict__ scores_k,
                                                    double (*part)[64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t DD = D * D;
    const int32_t cand = cblock * 64 + lane;
    double s = 0.0;
    if (cand < DD && wave < SUM_WAVES) {
        const double *pk = partial_k + cand;
#pragma unroll 4
        for (int32_t t = wave; t < n_tiles; t += SUM_WAVES) s += pk[(int64_t)t * DD];
    }
    if (wave < SUM_WAVES) part[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && cand < DD) {
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < SUM_WAVES; ++w) tot += part[w][lane];
        const int32_t jj = cand / D, ii = cand - jj * D;
        const int32_t dx = cx - R + ii, dy = cy - R + jj;
        const bool inside = dx >= -Rmax && dx <= Rmax && dy >= -Rmax && dy <= Rmax;
        scores_k[cand] = inside ? tot : -INFINITY;
    }
    __syncthreads();
}

// ---- scores of one frame from its partials ------------------------------------------------
// Sum over tiles in tile order; -inf outside the clipped window.
__device__ __forceinline__ double candidate_score(const double *partial_k, int32_t n_tiles, int32_t D, int32_t R,
                                                  int32_t Rmax, int32_t cx, int32_t cy, int32_t cand)
{
    const int32_t jj = cand / D, ii = cand - jj * D;
    const int32_t dx = cx - R + ii, dy = cy - R + jj;
    if (dx < -Rmax || dx > Rmax || dy < -Rmax || dy > Rmax) return -INFINITY;
    double s = 0.0;
    for (int32_t tI = 0; tI < n_tiles; ++tI) s += partial_k[(int64_t)tI * D * D + cand];
    return s;
}

// ---- argmax, runner-up, parabola -------------------------------------------------
struct Best {
    double s;
    int32_t i;
};

// Larger score wins; equal scores go to the smaller linear index (smaller dy, then
// smaller dx).  A total order, so any reduction tree gives the same answer.
__device__ __forceinline__ Best better_of(Best a, Best b)
{
    if (a.s > b.s) return a;
    if (b.s > a.s) return b;
    return a.i <= b.i ? a : b;
}

__device__ __forceinline__ Best block_best(Best v, Best *scratch)
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

// Offsets of one frame from its score cube S [D*D]; every thread of the block takes
// part, thread 0 writes *out.  scratch holds one Best per wave.
__device__ __forceinline__ void pick_frame(const double *S, int32_t D, int32_t R, int32_t Rmax, int32_t cx,
                                           int32_t cy, reduce_offset_t *out, Best *scratch)
{
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
        *out = o;
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
    *out = o;
}

}  // namespace rd
