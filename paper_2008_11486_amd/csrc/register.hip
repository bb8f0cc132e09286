// Translation registration by brute-force cross-correlation over a bounded window
// (stage-wise entry point).  The arithmetic lives in register_core.h; this file holds
// the kernels that wrap it and the host side of reduce_register.
//
// Roofline: VALU (FP64 FMA).  Algorithmic work per frame: |T| * (2R+1)^2 FMA.
#include <map>
#include <mutex>
#include <string>

#include "common.h"
#include "register_core.h"
#include "register_plan.h"

namespace rd {

__global__ __launch_bounds__(MEAN_THREADS) void tmpl_sum_rows(const float *__restrict__ ref, int32_t W, int32_t tx0,
                                                              int32_t ty0, int32_t tw, int32_t th,
                                                              double *__restrict__ part)
{
    __shared__ double scratch[MEAN_THREADS / 64];
    const double s = tmpl_part_sum(ref, W, tx0, ty0, tw, th, blockIdx.x, scratch);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(MEAN_THREADS) void tmpl_mean_final(const double *__restrict__ part, int32_t nparts,
                                                                double count, double *__restrict__ mean)
{
    __shared__ double scratch[MEAN_THREADS / 64];
    const double m = tmpl_mean_of_parts(part, nparts, count, scratch);
    if (threadIdx.x == 0) *mean = m;
}

template <int K>
__global__ __launch_bounds__(512) void score_tiles(ScoreArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t total = a.n_tiles * a.G * a.N;
    score_tile<K>(a, xcd_logical_id((int32_t)blockIdx.x, total), smem);
}

// Scores of each frame from its tile partials (64 candidates per workgroup).
// Slot k works on frame map[k] (nothing when negative), or on frame k without a map;
// centres and offsets are indexed by frame, partials and scores by slot.
__global__ __launch_bounds__(64 * SUM_WAVES) void sum_tiles(const double *__restrict__ partial, int32_t n_tiles,
                                                            int32_t D, int32_t R, int32_t Rmax,
                                                            const int32_t *__restrict__ centers,
                                                            const int32_t *__restrict__ map,
                                                            double *__restrict__ scores)
{
    __shared__ double part[SUM_WAVES][64];
    const int32_t k = blockIdx.y;
    const int32_t kf = map ? map[k] : k;
    if (kf < 0) return;
    const int32_t cx = centers ? centers[2 * kf] : 0, cy = centers ? centers[2 * kf + 1] : 0;
    sum_candidate_block(partial + (int64_t)k * n_tiles * D * D, n_tiles, D, R, Rmax, cx, cy, blockIdx.x,
                        scores + (int64_t)k * D * D, part);
}

__global__ __launch_bounds__(256) void pick_offsets(const double *__restrict__ scores, int32_t D, int32_t R,
                                                    int32_t Rmax, const int32_t *__restrict__ centers,
                                                    const int32_t *__restrict__ map,
                                                    reduce_offset_t *__restrict__ out)
{
    __shared__ Best scratch[4];
    const int32_t k = blockIdx.x;
    const int32_t kf = map ? map[k] : k;
    if (kf < 0) return;
    const int32_t cx = centers ? centers[2 * kf] : 0, cy = centers ? centers[2 * kf + 1] : 0;
    pick_frame(scores + (int64_t)k * D * D, D, R, Rmax, cx, cy, out + kf, scratch);
}

// ---- host side ---------------------------------------------------------------------
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct RegWs {
    size_t mean_parts, mean, partial, scores, total;
};

static RegWs reg_ws_layout(const RegPlan &p, int32_t N)
{
    RegWs w;
    const int32_t nparts = (int32_t)ceil_div(p.th_max, MEAN_ROWS);
    w.mean_parts = 0;
    w.mean = align256(sizeof(double) * nparts);
    w.partial = w.mean + 256;
    w.scores = w.partial + align256(sizeof(double) * (size_t)N * p.n_tiles * p.D * p.D);
    w.total = w.scores + align256(sizeof(double) * (size_t)N * p.D * p.D);
    return w;
}

ScoreArgs make_score_args(const RegPlan &p, const float *ref, const float *frames, const int32_t *centers,
                          const double *mean, double *partial, int32_t W, int32_t H, int32_t N, int32_t R,
                          int32_t Rmax, int32_t tx0, int32_t ty0, int32_t tw, int32_t th, int32_t skip)
{
    ScoreArgs a;
    a.ref = ref;
    a.frames = frames;
    a.centers = centers;
    a.mean = mean;
    a.partial = partial;
    a.W = W; a.H = H; a.R = R; a.Rmax = Rmax; a.D = p.D;
    a.tx0 = tx0; a.ty0 = ty0; a.tw = tw; a.th = th;
    a.TY = p.TY; a.TX = p.TX; a.NXB = p.NXB; a.BR = p.BR; a.NBX = p.NBX; a.C = p.C; a.CW = p.CW; a.S = p.S;
    a.JS = p.JS; a.FR = p.FR; a.FC = p.FC;
    a.n_xchunks = (int32_t)ceil_div(tw, p.TX);
    a.n_tiles = (int32_t)ceil_div(th, p.BR) * a.n_xchunks;
    a.N = N;
    a.G = p.G;
    a.threads = p.threads;
    a.skip = skip;
    a.map = nullptr;
    return a;
}

template <int D>
__global__ __launch_bounds__(SMALL_COLS) void score_small(ScoreArgs a)
{
    __shared__ __align__(16) float fl[SMALL_LDS_FLOATS];
    score_small_tile<D>(a, (int32_t)blockIdx.x, fl);
}

template <int K>
static void launch_score(const ScoreArgs &a, const RegPlan &p, hipStream_t s)
{
    ProfScope prof("score_tiles", s);
    hipLaunchKernelGGL(score_tiles<K>, dim3((unsigned)((int64_t)a.n_tiles * a.G * a.N)), dim3(p.threads), p.lds, s,
                       a);
}

// Template mean of the reference (two launches): parts [ceil(th / MEAN_ROWS)], mean [1].
void register_mean(const float *ref, int32_t W, int32_t tx0, int32_t ty0, int32_t tw, int32_t th,
                   double *mean_parts, double *mean, hipStream_t s)
{
    const int32_t nparts = (int32_t)ceil_div(th, MEAN_ROWS);
    hipLaunchKernelGGL(tmpl_sum_rows, dim3(nparts), dim3(MEAN_THREADS), 0, s, ref, W, tx0, ty0, tw, th, mean_parts);
    hipLaunchKernelGGL(tmpl_mean_final, dim3(1), dim3(MEAN_THREADS), 0, s, mean_parts, nparts,
                       (double)tw * (double)th, mean);
}

// Score tiles, tile sums and argmax for N work slots with a known template mean.
// map: slot -> frame (negative: idle slot) or NULL (slot k is frame k); partial holds
// [N][n_tiles][D*D] and scores [N][D*D] doubles.
void register_scores(const RegPlan &p, const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                     int32_t R, int32_t Rmax, const int32_t *centers, const int32_t *map, int32_t tx0, int32_t ty0,
                     int32_t tw, int32_t th, const double *mean, double *partial, double *sc, reduce_offset_t *out,
                     hipStream_t s)
{
    ScoreArgs a =
        make_score_args(p, ref, frames, centers, mean, partial, W, H, N, R, Rmax, tx0, ty0, tw, th, 0x7fffffff);
    a.map = map;
    if (p.K == 0) {
        ProfScope prof("score_tiles", s);
        // workgroups for this call's template (at most the plan's, which is sized for the largest)
        const dim3 grid((unsigned)((int64_t)a.n_tiles * N));
        switch (p.D) {
        case 1: hipLaunchKernelGGL(score_small<1>, grid, dim3(SMALL_COLS), 0, s, a); break;
        case 3: hipLaunchKernelGGL(score_small<3>, grid, dim3(SMALL_COLS), 0, s, a); break;
        default: hipLaunchKernelGGL(score_small<5>, grid, dim3(SMALL_COLS), 0, s, a); break;
        }
    } else {
    switch (p.K) {
    case 5: launch_score<5>(a, p, s); break;
    case 9: launch_score<9>(a, p, s); break;
    case 12: launch_score<12>(a, p, s); break;
    case 17: launch_score<17>(a, p, s); break;
    case 18: launch_score<18>(a, p, s); break;
    default: launch_score<22>(a, p, s); break;
    }
    }
    hipLaunchKernelGGL(sum_tiles, dim3((unsigned)ceil_div((int64_t)p.D * p.D, 64), N), dim3(64 * SUM_WAVES), 0, s,
                       partial, a.n_tiles, p.D, R, Rmax, centers, map, sc);
    hipLaunchKernelGGL(pick_offsets, dim3(N), dim3(256), 0, s, sc, p.D, R, Rmax, centers, map, out);
}

int register_launch(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N, int32_t R,
                    int32_t Rmax, const int32_t *centers, int32_t tx0, int32_t ty0, int32_t tw, int32_t th,
                    reduce_offset_t *out, double *scores, void *ws, const RegPlan &p, hipStream_t s)
{
    ProfScope prof_all("register", s);
    const RegWs L = reg_ws_layout(p, N);
    unsigned char *base = static_cast<unsigned char *>(ws);
    double *mean_parts = reinterpret_cast<double *>(base + L.mean_parts);
    double *mean = reinterpret_cast<double *>(base + L.mean);
    double *partial = reinterpret_cast<double *>(base + L.partial);
    double *sc = scores ? scores : reinterpret_cast<double *>(base + L.scores);
    register_mean(ref, W, tx0, ty0, tw, th, mean_parts, mean, s);
    register_scores(p, ref, frames, W, H, N, R, Rmax, centers, nullptr, tx0, ty0, tw, th, mean, partial, sc, out, s);
    return check_launch("reduce_register");
}

size_t register_ws_bytes(const RegPlan &p, int32_t N) { return reg_ws_layout(p, N).total; }

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_register_ws(int32_t W, int32_t H, int32_t N, int32_t radius, int32_t radius_max)
{
    if (W < 1 || H < 1 || N < 1 || radius < 0 || radius_max < 0) return 0;
    if (W - 2 * radius_max < 1 || H - 2 * radius_max < 1) return 0;
    const RegPlan p = reg_plan(W, H, radius, radius_max);
    if (p.D == 0) return 0;
    return register_ws_bytes(p, N);
}

// Argument checks shared by the search entry points; fills the template rectangle and the plan.
static int register_checks(const char *who, const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                           int32_t radius, int32_t radius_max, const int32_t *tmpl, const reduce_offset_t *out,
                           int32_t t[4], RegPlan *plan)
{
    const std::string w(who);
    if (!ref || !frames || !out) return fail(REDUCE_ERR_NULL, w + ": NULL buffer");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, w + ": W, H, N must be >= 1");
    if (radius < 0 || radius_max < 0) return fail(REDUCE_ERR_RANGE, w + ": negative radius");
    if (radius > 1024) return fail(REDUCE_ERR_UNSUPPORTED, w + ": radius above 1024");
    if (W - 2 * radius_max < 1 || H - 2 * radius_max < 1)
        return fail(REDUCE_ERR_RANGE, w + ": radius_max leaves no template");
    t[0] = radius_max; t[1] = radius_max; t[2] = W - 2 * radius_max; t[3] = H - 2 * radius_max;
    if (tmpl) {
        t[0] = tmpl[0]; t[1] = tmpl[1]; t[2] = tmpl[2]; t[3] = tmpl[3];
        if (t[2] < 1 || t[3] < 1) return fail(REDUCE_ERR_SHAPE, w + ": empty template");
        if (t[0] - radius_max < 0 || t[1] - radius_max < 0 || (int64_t)t[0] + t[2] + radius_max > W ||
            (int64_t)t[1] + t[3] + radius_max > H)
            return fail(REDUCE_ERR_RANGE, w + ": template dilated by radius_max leaves the frame");
    }
    if (N > 65535) return fail(REDUCE_ERR_UNSUPPORTED, w + ": N above 65535");
    *plan = reg_plan(W, H, radius, radius_max);
    if (plan->D == 0) return fail(REDUCE_ERR_UNSUPPORTED, w + ": window too large for any launch shape");
    return REDUCE_OK;
}

extern "C" int reduce_register(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                               int32_t radius, int32_t radius_max, const int32_t *centers, const int32_t *tmpl,
                               reduce_offset_t *out, double *scores, void *ws, size_t ws_bytes, void *stream)
{
    int32_t t[4];
    RegPlan p;
    const int c = register_checks("reduce_register", ref, frames, W, H, N, radius, radius_max, tmpl, out, t, &p);
    if (c != REDUCE_OK) return c;
    const size_t need = register_ws_bytes(p, N);
    if (!ws || ws_bytes < need)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_register: workspace needs " + std::to_string(need) + " bytes");
    return register_launch(ref, frames, W, H, N, radius, radius_max, centers, t[0], t[1], t[2], t[3], out, scores,
                           ws, p, as_stream(stream));
}

// ---- search without a caller workspace ---------------------------------------------------
// For callers that cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid allocation): the search's workspace (template mean parts,
// per-tile partial scores, score planes) lives in a fixed array of device memory that every
// GPU the library runs on holds until the process ends.  Host code never passes the array's
// name to a kernel: its device address, taken once per device with that device current,
// is what the kernels receive.  Every workspace word a call reads is written by that call
// first, so nothing needs clearing between calls.
namespace rd {
constexpr size_t REGISTER_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[REGISTER_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_addr;  // device -> address of its copy of scratch

static int scratch_address(const char *who, void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(REDUCE_ERR_HIP, std::string(who) + ": hipGetDevice: " + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) {
        *ptr = it->second;
        return REDUCE_OK;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(REDUCE_ERR_HIP, std::string(who) + ": hipGetSymbolAddress: " + hipGetErrorString(e));
    g_scratch_addr[dev] = p;
    *ptr = p;
    return REDUCE_OK;
}
}  // namespace rd

extern "C" size_t reduce_register_static_max(void) { return REGISTER_SCRATCH_BYTES; }

extern "C" int reduce_register_static(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                                      int32_t radius, int32_t radius_max, const int32_t *centers,
                                      const int32_t *tmpl, reduce_offset_t *out, double *scores, void *stream)
{
    int32_t t[4];
    RegPlan p;
    const int c =
        register_checks("reduce_register_static", ref, frames, W, H, N, radius, radius_max, tmpl, out, t, &p);
    if (c != REDUCE_OK) return c;
    const size_t need = register_ws_bytes(p, N);
    if (need > REGISTER_SCRATCH_BYTES)
        return fail(REDUCE_ERR_UNSUPPORTED, "reduce_register_static: these sizes need " + std::to_string(need) +
                                                " bytes of workspace, above the " +
                                                std::to_string(REGISTER_SCRATCH_BYTES) +
                                                " the library holds; search fewer frames per call");
    void *ws = nullptr;
    const int a = scratch_address("reduce_register_static", &ws);
    if (a != REDUCE_OK) return a;
    return register_launch(ref, frames, W, H, N, radius, radius_max, centers, t[0], t[1], t[2], t[3], out, scores,
                           ws, p, as_stream(stream));
}
