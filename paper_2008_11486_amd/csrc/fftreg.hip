// Correlation search evaluated through row spectra: the same scores S(d) over the same
// full window and template as the direct sums of register_core.h, for every offset, at a
// cost that no longer grows with the square of the window side.
//
// With the template T = [R, W-R) x [R, H-R) (tw x th), r' = ref - mean_T(ref) and the
// frame f, write b_y(x) = r'(R + x, R + y) for x < tw (0 up to P) and a_r(u) = f(u, r)
// for u < W (0 up to P), P >= W a power of two.  Then
//
//   S(dx, dy) = sum_y sum_x b_y(x) a_{y + R + dy}(x + R + dx)
//             = (1/P) sum_k Z_{R+dy}(k) e^{+2 pi i k (R + dx) / P},
//   Z_j(k)    = sum_y A_{y + j}(k) conj(B_y(k)),
//
// with A_r, B_y the length-P DFTs of the rows (no wrap-around: x + R + dx <= W - 1 < P).
// The rows are real, so only k = 0 .. P/2 is formed (Z at P - k is the conjugate).
// Four steps: row spectra (one P/2-point complex FFT per row of two packed real rows,
// Stockham radix-4 passes in LDS), the contraction Z over template rows (lags in register
// windows, frame spectra staged in LDS), the inverse at the 2R+1 lags needed, and the
// argmax.  The scores carry rounding of order 1e-13 relative to the largest, so the
// offsets are taken from exact direct sums: a +-1 window around the spectral argmax
// (moved while its maximum sits on an inner border), kept when its exact peak exceeds
// every spectral score outside the window by more than a bound on the spectral error,
// and otherwise the full direct search for that frame.  The results (integer and
// sub-pixel offsets, peak, flags) are therefore those of the direct search.
#include <algorithm>
#include <string>
#include <type_traits>

#include "common.h"
#include "register_core.h"
#include "register_plan.h"

namespace rd {

void register_mean(const float *ref, int32_t W, int32_t tx0, int32_t ty0, int32_t tw, int32_t th,
                   double *mean_parts, double *mean, hipStream_t s);
void register_scores(const RegPlan &p, const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                     int32_t R, int32_t Rmax, const int32_t *centers, const int32_t *map, int32_t tx0, int32_t ty0,
                     int32_t tw, int32_t th, const double *mean, double *partial, double *sc, reduce_offset_t *out,
                     hipStream_t s);

constexpr int FFT_THREADS = 256;
constexpr int32_t FFT_P_MAX = 8192;    // longest rows: P/2 = 4096 complex values in LDS (64 KB)
constexpr int CORR_KW = 64;            // spectrum columns per contraction workgroup (one per lane)
constexpr int CORR_LDS_MAX = 64 * 1024;
constexpr int32_t FFT_MAX_MOVES = 2;   // window moves of the exact refinement (then the full search)
constexpr size_t FFT_FALLBACK_BYTES = size_t(256) << 20;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// tw[t] = exp(-2 pi i t / P), t in [0, P)
__global__ void fft_twiddles(double2 *__restrict__ tw, int32_t P)
{
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P) return;
    double s, c;
    sincospi(-2.0 * (double)t / (double)P, &s, &c);
    tw[t] = make_double2(c, s);
}

// ---- row spectra -------------------------------------------------------------------------
// Rows of batch b: row r (r < nrows) holds x(u) = base[b * batch + r * pitch + u] - sub for
// u < ncols, 0 for ncols <= u < P; rows nrows <= r < rows_out are zero.  Output: the
// half spectrum X(k), k = 0 .. P/2, at spec + b * spec_batch + r * PS, and the sum of
// squares of each row at rowsq[b * rows_out + r].  A row of P real values is packed as
// z(n) = x(2n) + i x(2n+1), transformed with P/2-point Stockham passes (one radix-2 pass
// first when log2(P/2) is odd, then radix-4), and unpacked:
//   X(k) = E(k) - i w^k O(k),  E = (Z(k) + conj Z(N2-k)) / 2,  O = (Z(k) - conj Z(N2-k)) / 2,
// w = exp(-2 pi i / P).  Small rows share a workgroup (1024 / (P/2) rows each).
struct RowSrc {
    const float *base;
    int64_t batch, pitch;
    int32_t ncols, nrows;
    const double *sub;  // device scalar subtracted from every value, or NULL
};

template <int LOG2N2>
__global__ __launch_bounds__(FFT_THREADS) void fft_rows(RowSrc src, int32_t rows_out, const double2 *__restrict__ tw,
                                                        double2 *__restrict__ spec, int64_t spec_batch, int32_t PS,
                                                        double *__restrict__ rowsq)
{
    extern __shared__ __align__(16) double2 zl[];
    constexpr int32_t N2 = 1 << LOG2N2, P = 2 * N2;
    constexpr int rpw = N2 >= 1024 ? 1 : 1024 / N2;  // rows per workgroup
    constexpr int tpr = FFT_THREADS / rpw;           // threads per row
    const int t = threadIdx.x, lr = t / tpr, lt = t - lr * tpr;
    const int32_t b = blockIdx.y;
    const int32_t r = blockIdx.x * rpw + lr;
    double2 *z = zl + lr * N2;
    const bool live = r < rows_out;
    const bool data = r < src.nrows;
    const double sub = src.sub ? *src.sub : 0.0;
    const float *row = src.base + (int64_t)b * src.batch + (int64_t)(data ? r : 0) * src.pitch;

    // packed load and the row's sum of squares: the thread's NPT value pairs are loaded
    // together (addresses clamped into the row, values past it replaced by zero), then
    // converted and summed in the order of n
    constexpr int NPT = N2 / tpr;
    float f0[NPT], f1[NPT];
    if (data) {
        const int32_t last = src.ncols - 1;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int32_t u = 2 * (lt + i * tpr);
            f0[i] = row[min(u, last)];
            f1[i] = row[min(u + 1, last)];
        }
    }
    // twiddles of a radix-4 pass (see below): w[c][q - 1] = w_{4L}^{q k}, k = j mod L of the
    // thread's butterfly c.  Each pass's are loaded one pass ahead (the first pass's with
    // the row), so no pass waits on them.
    constexpr int32_t m4 = N2 >> 2;
    constexpr int NB4 = m4 / tpr;                   // radix-4 butterflies per thread
    constexpr int NP4 = LOG2N2 / 2;                 // radix-4 passes
    constexpr int32_t L0 = (LOG2N2 & 1) ? 2 : 1;    // L of the first of them
    static_assert(NP4 >= 1 && NB4 >= 1, "rows of at least 64 values");
    auto tw_pass = [&](int32_t Lp, double2(&w)[NB4][3]) {
#pragma unroll
        for (int c = 0; c < NB4; ++c) {
            const int32_t step = (P / 4 / Lp) * ((lt + c * tpr) & (Lp - 1));  // w_{4L}^k = tw[k P / (4L)]
#pragma unroll
            for (int q = 1; q < 4; ++q) w[c][q - 1] = tw[q * step];
        }
    };
    double2 wn[NB4][3];
    tw_pass(L0, wn);
    double sq = 0.0;
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int32_t n = lt + i * tpr, u = 2 * n;
        const double x0 = (data && u < src.ncols) ? (double)f0[i] - sub : 0.0;
        const double x1 = (data && u + 1 < src.ncols) ? (double)f1[i] - sub : 0.0;
        sq = fma(x0, x0, sq);
        sq = fma(x1, x1, sq);
        z[n] = make_double2(x0, x1);
    }
    // the row's sum of squares: over the row's threads in a fixed order
    {
        __shared__ double part[FFT_THREADS];
        part[t] = sq;
        __syncthreads();
        if (lt == 0 && live) {
            double s = 0.0;
            for (int i = 0; i < tpr; ++i) s += part[lr * tpr + i];
            rowsq[(int64_t)b * rows_out + r] = s;
        }
    }
    __syncthreads();

    // Stockham passes: L = product of the radices done so far; butterfly j reads
    // z[j + q m] (m = N2 / radix), twiddles input q by w_{L radix}^{q (j mod L)}, and writes
    // output q at (j / L) L radix + (j mod L) + q L.  Twiddle w_M^e = tw[e P / M].
    if (LOG2N2 & 1) {  // radix 2
        constexpr int32_t m = N2 >> 1;
        constexpr int NB2 = m / tpr;  // butterflies per thread
        double2 v[NB2][2];
#pragma unroll
        for (int c = 0; c < NB2; ++c) {
            const int32_t j = lt + c * tpr;
            v[c][0] = z[j];
            v[c][1] = z[j + m];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NB2; ++c) {
            const int32_t j = lt + c * tpr;
            z[2 * j] = cadd(v[c][0], v[c][1]);  // L = 1: output q at 2 j + q
            z[2 * j + 1] = csub(v[c][0], v[c][1]);
        }
        __syncthreads();
    }
    // the unpacking twiddles tw[k], k = lt, lt + tpr, ... <= N2, are loaded with the last
    // pass's LDS reads
    constexpr int NK = N2 / tpr + 1;
    double2 wk[NK];
#pragma unroll
    for (int p = 0; p < NP4; ++p) {
        const int32_t L = L0 << (2 * p);
        double2 w[NB4][3];
#pragma unroll
        for (int c = 0; c < NB4; ++c)
#pragma unroll
            for (int q = 0; q < 3; ++q) w[c][q] = wn[c][q];
        if (p + 1 < NP4) {
            tw_pass(4 * L, wn);
        } else {
#pragma unroll
            for (int i = 0; i < NK; ++i) wk[i] = tw[min(lt + i * tpr, N2)];
        }
        double2 v[NB4][4];
#pragma unroll
        for (int c = 0; c < NB4; ++c) {
            const int32_t j = lt + c * tpr;
            v[c][0] = z[j];
#pragma unroll
            for (int q = 1; q < 4; ++q) v[c][q] = cmul(z[j + q * m4], w[c][q - 1]);
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NB4; ++c) {
            const int32_t j = lt + c * tpr;
            const int32_t k = j & (L - 1);
            const double2 a = cadd(v[c][0], v[c][2]), bb = csub(v[c][0], v[c][2]);
            const double2 cc = cadd(v[c][1], v[c][3]), d = csub(v[c][1], v[c][3]);
            const int32_t o = (j - k) * 4 + k;  // (j / L) L 4 + k
            z[o] = cadd(a, cc);
            z[o + L] = make_double2(bb.x + d.y, bb.y - d.x);      // b - i d
            z[o + 2 * L] = csub(a, cc);
            z[o + 3 * L] = make_double2(bb.x - d.y, bb.y + d.x);  // b + i d
        }
        __syncthreads();
    }

    // unpack the two real transforms into the half spectrum of the row
    if (live) {
        double2 *out = spec + (int64_t)b * spec_batch + (int64_t)r * PS;
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const int32_t k = lt + i * tpr;
            if (k > N2) break;
            const double2 zk = z[k & (N2 - 1)];
            const double2 zc = z[(N2 - k) & (N2 - 1)];
            const double2 e = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y - zc.y));
            const double2 o = make_double2(0.5 * (zk.x - zc.x), 0.5 * (zk.y + zc.y));
            const double2 wo = cmul(wk[i], o);  // wk[i] = tw[k], k <= N2 < P
            out[k] = make_double2(e.x + wo.y, e.y - wo.x);  // E - i w O
        }
    }
}

// ---- contraction over template rows -------------------------------------------------------
// Zp[f][band][s][j][k] = sum over template rows y of sub-range s of band `band` of
// A_f[y + j][k] conj(B[y][k]), lags j in [0, D).  Lane = spectrum column k (CORR_KW per
// workgroup); wave w = (lag block within the group, sub-range s): a thread owns DY
// consecutive lags j0 .. j0 + DY - 1 and keeps the DY frame values its next template row
// needs in a register window (one new value per row).  The frame rows of a chunk of
// S * DY template rows (and the lags of the group) are staged in LDS; template values are
// read from the spectrum directly.  Rows beyond the data are zero in both spectra.
struct CorrArgs {
    const double2 *A;  // frame spectra: frame f at A + f * a_batch, row r at + r * PS
    const double2 *B;  // template spectrum [rows][PS]
    double2 *Zp;       // [F][n_band][S][D][PS]
    int64_t a_batch;
    int32_t PS, N2, D, NB, NBG, S, BY, n_band, n_kb;  // sub-ranges of DY template rows per chunk
};

template <int DY>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void spec_corr(CorrArgs a)
{
    extern __shared__ __align__(16) double2 al[];  // [YC + NBG * DY - 1][CORR_KW]
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int gb = w % a.NBG, s = w / a.NBG;       // lag block within the group, sub-range
    const int32_t kb = blockIdx.x % a.n_kb, grp = blockIdx.x / a.n_kb;
    const int32_t band = blockIdx.y, f = blockIdx.z;
    const int32_t k = kb * CORR_KW + lane;
    const int32_t blk = grp * a.NBG + gb;           // lag block
    const bool act = blk < a.NB;
    const int32_t j0 = blk * DY;                    // first lag of the thread
    const int32_t jg0 = grp * a.NBG * DY;           // first lag of the group
    const int32_t YC = a.S * DY;                   // template rows per chunk
    const int32_t rows = YC + a.NBG * DY - 1;       // staged frame rows per chunk
    const double2 *A = a.A + (int64_t)f * a.a_batch;
    const int nthr = blockDim.x;

    double2 acc[DY];
#pragma unroll
    for (int i = 0; i < DY; ++i) acc[i] = make_double2(0.0, 0.0);

    // The staged frame rows are a ring of `rows` LDS rows: frame row y_lo + jg0 + r of the
    // band sits in LDS row r mod rows.  Chunk y0 needs rows (y0 - y_lo) + [0, rows); from
    // the second chunk on only the YC rows it adds are staged, into the LDS rows of the YC
    // rows the previous chunk alone needed.  Those rows (chunk rows rows - YC + wv + u nw of
    // wave wv) are loaded into registers while the previous chunk is computed and stored
    // after its barrier, when each wave has at most NPF of them.
    constexpr int NPF = 4;
    const int wv = t >> 6, nw = nthr >> 6;
    const bool pipe = YC <= NPF * nw;  // every wave has at most NPF new rows per chunk
    double2 pf[NPF];
#pragma unroll
    for (int u = 0; u < NPF; ++u) pf[u] = make_double2(0.0, 0.0);
    const int32_t y_lo = band * a.BY, y_hi = y_lo + a.BY;
    int32_t ring0 = 0;  // LDS row of the chunk's first frame row
    for (int32_t y0 = y_lo; y0 < y_hi; y0 += YC) {
        __syncthreads();
        if (pipe && y0 != y_lo) {
#pragma unroll
            for (int u = 0; u < NPF; ++u) {  // a repeated last row stores the same value again
                int32_t lr = ring0 + rows - YC + min(wv + u * nw, YC - 1);
                if (lr >= rows) lr -= rows;
                al[lr * CORR_KW + lane] = pf[u];
            }
        } else {
            // frame rows y0 + jg0 + [r_lo, rows), columns kb * 64 ..: wave w stages rows
            // r_lo + w, r_lo + w + nw, ... (lane = column), eight rows loaded together, then
            // stored; a row index past the last is clamped to it on both sides (the same
            // value stored to the same place again), so no load waits behind a branch
            const int32_t r_lo = y0 == y_lo ? 0 : rows - YC;
            const double2 *src = A + (int64_t)(y0 + jg0) * a.PS + kb * CORR_KW + lane;
            for (int r0 = r_lo + wv; r0 < rows; r0 += 8 * nw) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)min(r0 + u * nw, rows - 1) * a.PS];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    int32_t lr = ring0 + min(r0 + u * nw, rows - 1);
                    if (lr >= rows) lr -= rows;
                    al[lr * CORR_KW + lane] = v[u];
                }
            }
        }
        __syncthreads();
        // the sub-range's template values (one window length, DY rows), then the next
        // chunk's new frame rows: both issued before any is used, the template values first
        // (the waits are in issue order).  Both unconditional: the last chunk reloads its own
        // rows, a wave's rows past its last repeat it, so the loads stay ahead of the compute.
        const int32_t ys = y0 + s * DY;  // first template row of this sub-range
        double2 bq[DY];
        {
            const double2 *bp = a.B + (int64_t)ys * a.PS + k;
#pragma unroll
            for (int q = 0; q < DY; ++q) bq[q] = bp[(int64_t)q * a.PS];
            __builtin_amdgcn_sched_barrier(0);  // keep the issue order
            const int32_t y0n = y0 + YC < y_hi ? y0 + YC : y0;
            const double2 *src = A + (int64_t)(y0n + jg0) * a.PS + kb * CORR_KW + lane;
#pragma unroll
            for (int u = 0; u < NPF; ++u) pf[u] = src[(int64_t)(rows - YC + min(wv + u * nw, YC - 1)) * a.PS];
            __builtin_amdgcn_sched_barrier(0);
        }
        if (act) {
            // window: chunk row of lag i at template row y is (y - y0) + (j0 - jg0) + i, in
            // LDS row ring0 + that, wrapped
            const int32_t c0 = ring0 + (ys - y0) + (j0 - jg0);
            auto at = [&](int32_t cr) {  // cr = chunk row - (ys - y0) - (j0 - jg0) < rows
                int32_t lr = c0 + cr;
                if (lr >= rows) lr -= rows;
                return al[lr * CORR_KW + lane];
            };
            double2 win[DY];
#pragma unroll
            for (int i = 0; i < DY - 1; ++i) win[i] = at(i);
#pragma unroll
            for (int q = 0; q < DY; ++q) {
                // row ys + q: the window holds lags 0 .. DY-1 in slots (q + i) mod DY
                win[(q + DY - 1) % DY] = at(q + DY - 1);
                const double2 bv = bq[q];
#pragma unroll
                for (int i = 0; i < DY; ++i) {
                    const double2 av = win[(q + i) % DY];
                    // acc += av * conj(bv)
                    acc[i].x = fma(av.x, bv.x, acc[i].x);
                    acc[i].x = fma(av.y, bv.y, acc[i].x);
                    acc[i].y = fma(av.y, bv.x, acc[i].y);
                    acc[i].y = fma(-av.x, bv.y, acc[i].y);
                }
            }
        }
        ring0 += YC % rows;
        if (ring0 >= rows) ring0 -= rows;
    }
    if (act && k <= a.N2) {
        double2 *zp = a.Zp + ((((int64_t)f * a.n_band + band) * a.S + s) * a.D) * a.PS + k;
#pragma unroll
        for (int i = 0; i < DY; ++i)
            if (j0 + i < a.D) zp[(int64_t)(j0 + i) * a.PS] = acc[i];
    }
}

// ---- scores at the lags of the window --------------------------------------------------
// S[f][j][m] = (1/P) sum_{k=0}^{N2} c_k Re(Z_j(k) e^{+2 pi i k m / P}), c_k = 1 at k = 0 and
// k = N2, else 2; Z_j(k) the sum of the partials over bands and sub-ranges in order.  One
// workgroup per (lag j, frame f); lanes stride over k; the D sums over m are reduced
// over the workgroup in a fixed order.  The twiddles of a pass over m0 .. m0 + EVAL_M - 1
// come from one table value and a recurrence, w(k, m + 1) = w(k, m) w(k, 1): scattered
// reads of the table for every (k, m) had bound the kernel by cache traffic.  A step adds
// at most sqrt(5) eps (the product) + 2 eps (the table value w(k, 1)) of relative error, so
// a twiddle is within 5 EVAL_M eps; the error bound of the decision below carries a term
// of 8 EVAL_M eps for it.
constexpr int EVAL_M = 16;  // lags m formed per pass

template <int LOG2N2>
__global__ __launch_bounds__(FFT_THREADS) void spec_eval(const double2 *__restrict__ Zp, int32_t n_part, int32_t D,
                                                         int32_t PS, const double2 *__restrict__ tw,
                                                         double *__restrict__ S)
{
    constexpr int32_t N2 = 1 << LOG2N2, P = 2 * N2;
    extern __shared__ __align__(16) double2 zs[];  // [N2 + 1]: c_k Z_j(k)
    __shared__ double red[FFT_THREADS / 64][EVAL_M];
    const int32_t j = blockIdx.x, f = blockIdx.y;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const double2 *z0 = Zp + (int64_t)f * n_part * D * PS + (int64_t)j * PS;
    for (int32_t k = t; k <= N2; k += FFT_THREADS) {
        // the partials added in order p = 0, 1, ...; eight loaded together at a time (a
        // partial index past the last is clamped and its value not added)
        double2 s = make_double2(0.0, 0.0);
        for (int32_t p0 = 0; p0 < n_part; p0 += 8) {
            double2 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = z0[(int64_t)min(p0 + u, n_part - 1) * D * PS + k];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (p0 + u < n_part) s = cadd(s, v[u]);
        }
        const double c = (k == 0 || k == N2) ? 1.0 : 2.0;
        zs[k] = make_double2(c * s.x, c * s.y);
    }
    __syncthreads();
    for (int32_t m0 = 0; m0 < D; m0 += EVAL_M) {
        double acc[EVAL_M];
#pragma unroll
        for (int q = 0; q < EVAL_M; ++q) acc[q] = 0.0;
        // EVAL_K values of k per iteration, their table values loaded together; a k past N2
        // is clamped for the loads and its spectrum value taken as zero (adding 0 * w to a
        // sum that started at +0 leaves it exact), so the sums are those of k in order
        constexpr int EVAL_K = 4;
#pragma unroll 1
        for (int32_t k0 = t; k0 <= N2; k0 += EVAL_K * FFT_THREADS) {
            double2 w[EVAL_K], w1[EVAL_K], z[EVAL_K];
#pragma unroll
            for (int e = 0; e < EVAL_K; ++e) {
                const int32_t kc = min(k0 + e * FFT_THREADS, N2);
                w[e] = tw[((int64_t)kc * m0) & (P - 1)];  // e^{-2 pi i k m / P} at m = m0
                w1[e] = tw[kc & (P - 1)];                 // and at m = 1
                z[e] = k0 + e * FFT_THREADS <= N2 ? zs[kc] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int e = 0; e < EVAL_K; ++e)
#pragma unroll
                for (int q = 0; q < EVAL_M; ++q) {
                    acc[q] = fma(z[e].x, w[e].x, acc[q]);  // Re(z conj(w))
                    acc[q] = fma(z[e].y, w[e].y, acc[q]);
                    if (q + 1 < EVAL_M) w[e] = cmul(w[e], w1[e]);
                }
        }
#pragma unroll
        for (int q = 0; q < EVAL_M; ++q) {
            double v = acc[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[wv][q] = v;
        }
        __syncthreads();
        if (t < EVAL_M && m0 + t < D) {
            double v = 0.0;
            for (int i = 0; i < FFT_THREADS / 64; ++i) v += red[i][t];
            S[((int64_t)f * D + j) * D + m0 + t] = v / (double)P;
        }
        __syncthreads();
    }
}

// Argmax of the spectral scores (full window, centre 0) and the window centre of the
// exact refinement.
__global__ __launch_bounds__(256) void spec_pick(const double *__restrict__ S, int32_t D, int32_t R,
                                                 reduce_offset_t *__restrict__ off, int32_t *__restrict__ centres)
{
    __shared__ Best scratch[4];
    const int32_t f = blockIdx.x;
    pick_frame(S + (int64_t)f * D * D, D, R, R, 0, 0, off + f, scratch);
    __syncthreads();
    if (threadIdx.x == 0) {
        centres[2 * f] = off[f].dx;
        centres[2 * f + 1] = off[f].dy;
    }
}

// One window move of the refinement: a frame whose exact maximum lies on a border of its
// +-1 window strictly inside +-R gets its centre on that maximum and its slot.
__global__ void spec_walk(const reduce_offset_t *__restrict__ offs, int32_t N, int32_t R, int32_t *__restrict__ centres,
                          int32_t *__restrict__ map)
{
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const reduce_offset_t o = offs[k];
    const bool bx = (o.flags & REDUCE_EDGE_X) && o.dx > -R && o.dx < R;
    const bool by = (o.flags & REDUCE_EDGE_Y) && o.dy > -R && o.dy < R;
    if (bx || by) {
        centres[2 * k] = o.dx;
        centres[2 * k + 1] = o.dy;
        map[k] = k;
    } else {
        map[k] = -1;
    }
}

// Decision per frame, one workgroup each.  Kept: the exact maximum is not on an inner
// border, and it exceeds the best spectral score outside its +-1 window by more than the
// bound on the spectral error
//   bound = factor ||a||_F ||b||_F,  factor = 4 eps (10 log2(P/2) + th + P + 18 + 2 EVAL_M),
// (eps = 2^-53; ||a||_F over the frame rows, ||b||_F over the template rows; first-order
// rounding of the row transforms, the contraction, the inverse sums and their twiddles).  A kept frame
// gets second = the larger of its window's runner-up and that spectral score, the margin
// and NEAR_TIE from it, and loses CLIPPED (its window is a step of the full search).
// fb[k] = 1 for the frames that take the full search; info[k] says why (1: inner border,
// 2: not clear of the bound).
__global__ __launch_bounds__(256) void spec_settle(reduce_offset_t *__restrict__ offs, const double *__restrict__ S,
                                                   int32_t D, int32_t R, const double *__restrict__ rowsq_a,
                                                   int32_t rows_a, const double *__restrict__ rowsq_b,
                                                   int32_t rows_b, double factor, int32_t *__restrict__ fb,
                                                   int32_t *__restrict__ info)
{
    __shared__ double red[4];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int32_t k = blockIdx.x;
    const reduce_offset_t o0 = offs[k];
    // ||a||^2, ||b||^2: threads stride over rows, then the waves in order
    auto block_sum = [&](const double *v, int32_t n) {
        double s = 0.0;
        for (int32_t r = t; r < n; r += 256) s += v[r];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[wv] = s;
        __syncthreads();
        const double tot = red[0] + red[1] + red[2] + red[3];
        __syncthreads();
        return tot;
    };
    const double aa = block_sum(rowsq_a + (int64_t)k * rows_a, rows_a);
    const double bb = block_sum(rowsq_b, rows_b);
    // best spectral score outside the +-1 window around the exact maximum
    const double *Sk = S + (int64_t)k * D * D;
    double best = -INFINITY;
    for (int32_t c = t; c < D * D; c += 256) {
        const int32_t jj = c / D, ii = c - jj * D;
        if (abs(ii - R - o0.dx) <= 1 && abs(jj - R - o0.dy) <= 1) continue;
        best = fmax(best, Sk[c]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off, 64));
    if (lane == 0) red[wv] = best;
    __syncthreads();
    if (t != 0) return;
    const double out_best = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    const double bound = factor * sqrt(aa) * sqrt(bb);
    reduce_offset_t o = o0;
    const bool border = ((o.flags & REDUCE_EDGE_X) && o.dx > -R && o.dx < R) ||
                        ((o.flags & REDUCE_EDGE_Y) && o.dy > -R && o.dy < R);
    const bool unsure = !(o.peak > out_best + bound);
    fb[k] = (border || unsure) ? 1 : 0;
    if (info) info[k] = (border ? 1 : 0) | (unsure ? 2 : 0);
    if (!border && !unsure) {
        o.second = fmax(o.second, out_best);
        if (o.second == -INFINITY) o.margin = INFINITY;
        else if (o.peak == 0.0) o.margin = (o.peak > o.second) ? INFINITY : 0.0;
        else o.margin = (o.peak - o.second) / fabs(o.peak);
        o.flags &= ~(REDUCE_CLIPPED | REDUCE_NEAR_TIE);
        if (o.margin < REDUCE_NEAR_TIE_MARGIN) o.flags |= REDUCE_NEAR_TIE;
        offs[k] = o;
    }
}

// The frames with fb[k] = 1 in increasing order: list[0, n) = those frames, list[n, N) = -1.
// One wave.
__global__ __launch_bounds__(64) void spec_list(const int32_t *__restrict__ fb, int32_t N, int32_t *__restrict__ list)
{
    const int lane = threadIdx.x;
    int32_t base = 0;
    for (int32_t c0 = 0; c0 < N; c0 += 64) {
        const int32_t k = c0 + lane;
        const bool f = k < N && fb[k] != 0;
        const uint64_t m = __ballot(f);
        if (f) list[base + __popcll(m & ((1ull << lane) - 1ull))] = k;
        base += __popcll(m);
    }
    for (int32_t k = base + lane; k < N; k += 64) list[k] = -1;
}

// ---- host side ---------------------------------------------------------------------------
static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

static int corr_dy(int32_t D)
{
    // lags per thread: the least padding of D, the larger block on ties
    int best = 8;
    int64_t waste = 1 << 30;
    for (int dy : {12, 11, 10, 9, 8}) {
        const int64_t wst = ceil_div(D, dy) * dy - D;
        if (wst < waste) {
            waste = wst;
            best = dy;
        }
    }
    return best;
}

struct FftLayout {
    int32_t P, N2, log2n2, PS, D, DY, NB, NBG, n_grp, S, YS, BY, n_band, th_pad, rows_a, F;
    size_t corr_lds, fft_lds;
    RegPlan refine, full;
    int32_t Ffull;
    size_t tw, mean_parts, mean, B, rowsq_b, A, rowsq_a, Zp, S_fft, cen, map, list, info, fb;
    size_t part_r, sc_r, part_f, sc_f, total;
};

static bool fft_layout(int32_t W, int32_t H, int32_t N, int32_t R, FftLayout *L)
{
    const int32_t tw = W - 2 * R, th = H - 2 * R;
    if (tw < 1 || th < 1) return false;
    int32_t P = 64;
    while (P < W) P <<= 1;
    if (P > FFT_P_MAX) return false;
    L->P = P;
    L->N2 = P / 2;
    L->log2n2 = 0;
    while ((1 << L->log2n2) < L->N2) ++L->log2n2;
    L->PS = (int32_t)(ceil_div(L->N2 + 1, CORR_KW) * CORR_KW);
    L->D = 2 * R + 1;
    L->DY = corr_dy(L->D);
    L->NB = (int32_t)ceil_div(L->D, L->DY);
    // lag blocks per workgroup (fewer restagings of the frame rows) and sub-ranges of
    // template rows (more waves on one chunk), each sub-range one window length per chunk,
    // with the staged rows within CORR_LDS_MAX
    L->YS = L->DY;
    L->NBG = 0;
    for (int32_t g = std::min<int32_t>(L->NB, 4); g >= 1 && !L->NBG; --g)
        for (int32_t sr = 4; sr >= 1; --sr) {
            const size_t lds = sizeof(double2) * CORR_KW * (size_t)(sr * L->YS + g * L->DY - 1);
            if (lds <= CORR_LDS_MAX && 64 * g * sr <= 512) {
                L->NBG = g;
                L->S = sr;
                L->corr_lds = lds;
                break;
            }
        }
    if (!L->NBG) return false;
    L->n_grp = (int32_t)ceil_div(L->NB, L->NBG);
    const int32_t YC = L->S * L->YS;
    // template rows in bands of whole chunks: about 16 bands
    L->BY = (int32_t)(ceil_div(ceil_div(th, 16), YC) * YC);
    L->n_band = (int32_t)ceil_div(th, L->BY);
    L->th_pad = L->n_band * L->BY;
    // >= H: every lag of every padded template row, lag groups padded to whole groups
    L->rows_a = L->th_pad + L->n_grp * L->NBG * L->DY;
    L->fft_lds = sizeof(double2) * (size_t)std::max<int32_t>(L->N2, 1024);
    // frames per round of spectra: their spectra and contraction partials in about 1 GB
    const size_t per_frame = sizeof(double2) * (size_t)L->PS *
                             ((size_t)L->rows_a + (size_t)L->n_band * L->S * L->D) + sizeof(double) * L->rows_a;
    L->F = (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)N, (size_t(1) << 30) / per_frame));
    L->refine = reg_plan(W, H, 1, R);
    L->full = reg_plan(W, H, R, R);
    if (L->refine.D == 0 || L->full.D == 0) return false;
    const size_t per_full = sizeof(double) * (size_t)L->full.n_tiles * L->full.D * L->full.D;
    L->Ffull = (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)N, FFT_FALLBACK_BYTES / per_full));
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += al256(std::max<size_t>(bytes, 1));
        return at;
    };
    L->tw = take(sizeof(double2) * P);
    L->mean_parts = take(sizeof(double) * (size_t)ceil_div(th, MEAN_ROWS));
    L->mean = take(sizeof(double));
    L->B = take(sizeof(double2) * (size_t)L->PS * L->th_pad);
    L->rowsq_b = take(sizeof(double) * (size_t)L->th_pad);
    L->A = take(sizeof(double2) * (size_t)L->PS * L->rows_a * L->F);
    L->rowsq_a = take(sizeof(double) * (size_t)L->rows_a * N);  // every frame's, for the decisions
    L->Zp = take(sizeof(double2) * (size_t)L->PS * L->n_band * L->S * L->D * L->F);
    L->S_fft = take(sizeof(double) * (size_t)N * L->D * L->D);
    L->cen = take(sizeof(int32_t) * 2 * (size_t)N);
    L->map = take(sizeof(int32_t) * (size_t)N);
    L->list = take(sizeof(int32_t) * (size_t)N);
    L->info = take(sizeof(int32_t) * (size_t)N);
    L->fb = take(sizeof(int32_t) * (size_t)N);
    const RegPlan &pr = L->refine, &pf = L->full;
    L->part_r = take(sizeof(double) * (size_t)N * pr.n_tiles * pr.D * pr.D);
    L->sc_r = take(sizeof(double) * (size_t)N * pr.D * pr.D);
    L->part_f = take(per_full * (size_t)L->Ffull);
    L->sc_f = take(sizeof(double) * (size_t)L->Ffull * pf.D * pf.D);
    L->total = o;
    return true;
}

static int fft_check(int32_t W, int32_t H, int32_t N, int32_t R, const char *who)
{
    const std::string w(who);
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, w + ": W, H, N must be >= 1");
    if (R < 1) return fail(REDUCE_ERR_RANGE, w + ": radius must be >= 1");
    if (W - 2 * R < 1 || H - 2 * R < 1) return fail(REDUCE_ERR_RANGE, w + ": radius leaves no template");
    if (W > FFT_P_MAX) return fail(REDUCE_ERR_UNSUPPORTED, w + ": rows longer than 8192");
    if (N > 65535) return fail(REDUCE_ERR_UNSUPPORTED, w + ": N above 65535");
    if (2 * R + 1 > 1024) return fail(REDUCE_ERR_UNSUPPORTED, w + ": radius above 511");
    return REDUCE_OK;
}

// P/2 from 32 (P = 64) to 4096 (P = 8192)
template <typename F>
static void log2_dispatch(int32_t log2n2, F &&f)
{
    switch (log2n2) {
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    case 11: f(std::integral_constant<int, 11>{}); break;
    default: f(std::integral_constant<int, 12>{}); break;
    }
}

static void launch_fft_rows(const FftLayout &L, const RowSrc &src, int32_t rows_out, int32_t batches,
                            const double2 *tw, double2 *spec, int64_t spec_batch, double *rowsq, hipStream_t s)
{
    const int rpw = L.N2 >= 1024 ? 1 : 1024 / L.N2;
    const dim3 grid((unsigned)ceil_div(rows_out, rpw), (unsigned)batches);
    log2_dispatch(L.log2n2, [&](auto Lc) {
        hipLaunchKernelGGL(fft_rows<decltype(Lc)::value>, grid, dim3(FFT_THREADS), L.fft_lds, s, src, rows_out, tw,
                           spec, spec_batch, L.PS, rowsq);
    });
}

template <int DY>
static void launch_corr(const CorrArgs &c, const FftLayout &L, int32_t nf, hipStream_t s)
{
    const dim3 grid((unsigned)(c.n_kb * L.n_grp), (unsigned)L.n_band, (unsigned)nf);
    hipLaunchKernelGGL(spec_corr<DY>, grid, dim3((unsigned)(64 * L.NBG * L.S)), L.corr_lds, s, c);
}

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_register_fft_ws(int32_t W, int32_t H, int32_t N, int32_t radius)
{
    if (W < 1 || H < 1 || N < 1 || N > 65535 || radius < 1 || W - 2 * radius < 1 || H - 2 * radius < 1 ||
        W > FFT_P_MAX || 2 * radius + 1 > 1024)
        return 0;
    FftLayout L;
    return fft_layout(W, H, N, radius, &L) ? L.total : 0;
}

extern "C" int reduce_register_fft(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                                   int32_t radius, reduce_offset_t *out, double *scores, int32_t *info, void *ws,
                                   size_t ws_bytes, void *stream)
{
    if (!ref || !frames || !out) return fail(REDUCE_ERR_NULL, "reduce_register_fft: NULL buffer");
    const int c = fft_check(W, H, N, radius, "reduce_register_fft");
    if (c != REDUCE_OK) return c;
    FftLayout L;
    if (!fft_layout(W, H, N, radius, &L))
        return fail(REDUCE_ERR_UNSUPPORTED, "reduce_register_fft: no launch shape for these sizes");
    if (!ws || ws_bytes < L.total)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_register_fft: workspace needs " + std::to_string(L.total) + " bytes");
    hipStream_t s = as_stream(stream);
    unsigned char *b = static_cast<unsigned char *>(ws);
    auto at = [&](size_t off) { return static_cast<void *>(b + off); };
    double2 *tw = static_cast<double2 *>(at(L.tw));
    double *mean = static_cast<double *>(at(L.mean));
    double2 *Bs = static_cast<double2 *>(at(L.B));
    double *rowsq_b = static_cast<double *>(at(L.rowsq_b));
    double2 *As = static_cast<double2 *>(at(L.A));
    double *rowsq_a = static_cast<double *>(at(L.rowsq_a));
    double2 *Zp = static_cast<double2 *>(at(L.Zp));
    double *Sf = scores ? scores : static_cast<double *>(at(L.S_fft));
    int32_t *cen = static_cast<int32_t *>(at(L.cen));
    int32_t *map = static_cast<int32_t *>(at(L.map));
    int32_t *list = static_cast<int32_t *>(at(L.list));
    int32_t *inf = info ? info : static_cast<int32_t *>(at(L.info));
    const int32_t R = radius, D = L.D;
    const int32_t tx0 = R, ty0 = R, tw_ = W - 2 * R, th = H - 2 * R;
    const int64_t a_batch = (int64_t)L.PS * L.rows_a;
    ProfScope prof("register_fft", s);

    hipLaunchKernelGGL(fft_twiddles, dim3((unsigned)ceil_div(L.P, 256)), dim3(256), 0, s, tw, L.P);
    register_mean(ref, W, tx0, ty0, tw_, th, static_cast<double *>(at(L.mean_parts)), mean, s);
    {
        ProfScope p2("fft_rows", s);
        const RowSrc tsrc{ref + (int64_t)ty0 * W + tx0, 0, W, tw_, th, mean};
        launch_fft_rows(L, tsrc, L.th_pad, 1, tw, Bs, 0, rowsq_b, s);
    }
    CorrArgs ca;
    ca.A = As;
    ca.B = Bs;
    ca.Zp = Zp;
    ca.a_batch = a_batch;
    ca.PS = L.PS;
    ca.N2 = L.N2;
    ca.D = D;
    ca.NB = L.NB;
    ca.NBG = L.NBG;
    ca.S = L.S;
    ca.BY = L.BY;
    ca.n_band = L.n_band;
    ca.n_kb = (int32_t)ceil_div(L.N2 + 1, CORR_KW);
    for (int32_t f0 = 0; f0 < N; f0 += L.F) {
        const int32_t nf = std::min(L.F, N - f0);
        {
            ProfScope p2("fft_rows", s);
            const RowSrc fsrc{frames + (int64_t)f0 * W * H, (int64_t)W * H, W, W, H, nullptr};
            launch_fft_rows(L, fsrc, L.rows_a, nf, tw, As, a_batch, rowsq_a + (int64_t)f0 * L.rows_a, s);
        }
        {
            ProfScope p2("spec_corr", s);
            switch (L.DY) {
            case 8: launch_corr<8>(ca, L, nf, s); break;
            case 9: launch_corr<9>(ca, L, nf, s); break;
            case 10: launch_corr<10>(ca, L, nf, s); break;
            case 11: launch_corr<11>(ca, L, nf, s); break;
            default: launch_corr<12>(ca, L, nf, s); break;
            }
        }
        {
            ProfScope p2("spec_eval", s);
            log2_dispatch(L.log2n2, [&](auto Lc) {
                hipLaunchKernelGGL(spec_eval<decltype(Lc)::value>, dim3((unsigned)D, (unsigned)nf),
                                   dim3(FFT_THREADS), sizeof(double2) * (L.N2 + 1), s, Zp, L.n_band * L.S, D, L.PS,
                                   tw, Sf + (int64_t)f0 * D * D);
            });
        }
        hipLaunchKernelGGL(spec_pick, dim3((unsigned)nf), dim3(256), 0, s, Sf + (int64_t)f0 * D * D, D, R, out + f0,
                           cen + 2 * f0);
    }
    // exact +-1 windows around the spectral maxima, moved while their maximum lies on an
    // inner border; the decisions; the full direct search for the frames not settled
    {
        ProfScope p2("fft_refine", s);
        double *part_r = static_cast<double *>(at(L.part_r));
        double *sc_r = static_cast<double *>(at(L.sc_r));
        register_scores(L.refine, ref, frames, W, H, N, 1, R, cen, nullptr, tx0, ty0, tw_, th, mean, part_r, sc_r,
                        out, s);
        for (int32_t mv = 0; mv < FFT_MAX_MOVES; ++mv) {
            hipLaunchKernelGGL(spec_walk, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, out, N, R, cen, map);
            register_scores(L.refine, ref, frames, W, H, N, 1, R, cen, map, tx0, ty0, tw_, th, mean, part_r, sc_r,
                            out, s);
        }
        const double eps = 1.1102230246251565e-16;  // 2^-53
        const double factor = 4.0 * eps * (10.0 * L.log2n2 + (double)th + (double)L.P + 18.0 + 2.0 * EVAL_M);
        int32_t *fb = static_cast<int32_t *>(at(L.fb));
        hipLaunchKernelGGL(spec_settle, dim3((unsigned)N), dim3(256), 0, s, out, Sf, D, R, rowsq_a, L.rows_a, rowsq_b,
                           L.th_pad, factor, fb, inf);
        hipLaunchKernelGGL(spec_list, dim3(1), dim3(64), 0, s, fb, N, list);
    }
    {
        ProfScope p2("fft_fallback", s);
        for (int32_t r0 = 0; r0 < N; r0 += L.Ffull) {
            const int32_t n = std::min(L.Ffull, N - r0);
            register_scores(L.full, ref, frames, W, H, n, R, R, nullptr, list + r0, tx0, ty0, tw_, th, mean,
                            static_cast<double *>(at(L.part_f)), static_cast<double *>(at(L.sc_f)), out, s);
        }
    }
    return check_launch("reduce_register_fft");
}
