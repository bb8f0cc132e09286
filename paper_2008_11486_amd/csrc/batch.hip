// Many stacks of uneven frame counts and sizes in one persistent kernel launch,
// replayed from a cached HIP graph.
//
// The host turns the stacks into one ordered work queue of items:
//
//   CAL        calibrate a band of rows of one frame into the workspace
//   MEANPART   sum MEAN_ROWS template rows of the calibrated reference
//   MEANFINAL  template mean of the reference
//   SCORE      one tile of partial correlation scores (stack's tuned launch shape)
//   PICK       sum one frame's partials over tiles, argmax, runner-up, parabola
//   RECT       common overlap of the stack from its offsets
//   OUT        bilinear shift of every frame + sigma-clipped mean for OUT_TILES x 256
//              output pixels
//
// Items are listed phase by phase, so every item depends only on items earlier in
// the queue.  Workgroups take items in queue order with one atomic counter; before
// running an item a workgroup waits until the per-stack counter of the phase it
// depends on is complete, and after it publishes its results with a release and
// bumps its own phase counter.  The lowest unfinished item never waits on a later
// one and was taken by a running workgroup, so the queue always drains.  Every wait
// is bounded: past the spin limit the kernel raises an error flag and all
// workgroups leave.  Each item calls the same device bodies as the stage-wise
// kernels with the same launch shape, so results are bit-identical to them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "combine_core.h"
#include "common.h"
#include "register_core.h"
#include "register_plan.h"

namespace rd {

int combine_lanes_for(int32_t N);
ScoreArgs make_score_args(const RegPlan &p, const float *ref, const float *frames, const int32_t *centers,
                          const double *mean, double *partial, int32_t W, int32_t H, int32_t N, int32_t R,
                          int32_t Rmax, int32_t tx0, int32_t ty0, int32_t tw, int32_t th, int32_t skip);

constexpr int BATCH_THREADS = 512;
constexpr int CAL_ROWS = 32;    // rows of one frame per CAL item
constexpr int OUT_TILES = 4;    // combine tiles (of COMB_TILE pixels) per OUT item

enum ItemType : int32_t { IT_CAL = 0, IT_MEANPART, IT_MEANFINAL, IT_SCORE, IT_PICK, IT_RECT, IT_OUT };
enum Counter : int32_t { C_CAL = 0, C_MEANPART, C_MEAN, C_SCORE, C_PICK, C_RECT, C_COUNT };

struct Item {
    int32_t type, stack, a, pad;
};

struct StackDev {
    // caller buffers
    const uint16_t *raw;
    int64_t rrp, rfp;
    const float *dark, *flat;
    int64_t crp;
    float *out;
    int32_t *out_rect;
    reduce_offset_t *offsets;
    int64_t *n_rej;
    // sizes and parameters
    int32_t W, H, N, ref, R, max_iters, integer_mode, lanes, K;
    float ksigma;
    // workspace
    float *cal;           // [N][H][W]
    double *mean_parts;   // [n_mean_parts]
    double *mean;         // [1]
    double *partial;      // [N-1][n_tiles][D*D]
    double *scores;       // [N-1][D*D]
    float *soffs;         // [N][2] offsets applied by the shift
    int32_t *rect;        // [4]
    uint32_t *ctr;        // [C_COUNT]
    int32_t n_cal, n_mean_parts, n_score, n_pick;
    ScoreArgs sa;
};

struct BatchArgs {
    const Item *items;
    const StackDev *stacks;
    int32_t n_items;
    uint32_t *head;
    uint32_t *error;
    uint32_t spin_limit;
};

// ---- inter-workgroup signalling ------------------------------------------------------
__device__ __forceinline__ bool wait_count(const BatchArgs &a, uint32_t *ctr, uint32_t target, int *flag)
{
    if (threadIdx.x == 0) {
        uint32_t spins = 0;
        int ok = 1;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                ok = 0;
                break;
            }
            if (++spins > a.spin_limit) {
                __hip_atomic_store(a.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        // make the producers' released writes visible before anything is read
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *flag = ok;
    }
    __syncthreads();
    const bool ok = *flag != 0;
    __syncthreads();
    return ok;
}

__device__ __forceinline__ void signal_done(uint32_t *ctr)
{
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- item bodies ---------------------------------------------------------------------------
__device__ __noinline__ void do_cal(const StackDev &s, int32_t a)
{
    const int32_t bands = (int32_t)((s.H + CAL_ROWS - 1) / CAL_ROWS);
    const int32_t k = a / bands, y0 = (a - k * bands) * CAL_ROWS;
    const int32_t y1 = min(y0 + CAL_ROWS, s.H);
    const int64_t n = (int64_t)(y1 - y0) * s.W;
    for (int64_t i = threadIdx.x; i < n; i += BATCH_THREADS) {
        const int32_t y = y0 + (int32_t)(i / s.W), x = (int32_t)(i % s.W);
        const int64_t c = (int64_t)y * s.crp + x;
        s.cal[((int64_t)k * s.H + y) * s.W + x] =
            calib_px(s.raw[(int64_t)k * s.rfp + (int64_t)y * s.rrp + x], s.dark[c], s.flat[c]);
    }
}

__device__ __noinline__ void do_rect(const StackDev &s)
{
    if (threadIdx.x != 0) return;
    // reference frame: offset 0 by definition
    reduce_offset_t z;
    z.dx = z.dy = 0;
    z.sx = z.sy = 0.0f;
    z.peak = 0.0;
    z.second = -INFINITY;
    z.margin = INFINITY;
    z.flags = 0;
    z.pad = 0;
    s.offsets[s.ref] = z;
    double xl = -1e300, xh = 1e300, yl = -1e300, yh = 1e300;
    for (int32_t k = 0; k < s.N; ++k) {
        float sx = 0.0f, sy = 0.0f;
        if (k != s.ref) {
            const reduce_offset_t o = s.offsets[k];
            sx = s.integer_mode ? (float)o.dx : o.sx;
            sy = s.integer_mode ? (float)o.dy : o.sy;
        }
        s.soffs[2 * k] = sx;
        s.soffs[2 * k + 1] = sy;
        const double a = ceil(-(double)sx), b = floor((double)(s.W - 1) - (double)sx);
        const double c = ceil(-(double)sy), d = floor((double)(s.H - 1) - (double)sy);
        xl = a > xl ? a : xl;
        xh = b < xh ? b : xh;
        yl = c > yl ? c : yl;
        yh = d < yh ? d : yh;
    }
    int32_t r[4];
    if (xl > xh || yl > yh) {
        r[0] = r[1] = r[2] = r[3] = 0;  // no overlap: empty output
    } else {
        r[0] = (int32_t)xl;
        r[1] = (int32_t)yl;
        r[2] = (int32_t)(xh - xl) + 1;
        r[3] = (int32_t)(yh - yl) + 1;
    }
    for (int i = 0; i < 4; ++i) {
        s.rect[i] = r[i];
        s.out_rect[i] = r[i];
    }
}

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __noinline__ void do_out(const StackDev &s, int32_t a, float *tile)
{
    const int32_t x0 = s.rect[0], y0 = s.rect[1], w = s.rect[2], h = s.rect[3];
    const int64_t plane = (int64_t)w * h;
    unsigned dropped = 0;
    for (int32_t sub = 0; sub < OUT_TILES; ++sub) {
        const int64_t p0 = ((int64_t)a * OUT_TILES + sub) * COMB_TILE;
        if (p0 >= plane) break;  // uniform over the workgroup
        // aligned values of every frame for the tile's pixels, as the shift kernel makes them
        for (int32_t idx = threadIdx.x; idx < s.N * COMB_TILE; idx += BATCH_THREADS) {
            const int32_t k = idx / COMB_TILE, px = idx - k * COMB_TILE;
            const int64_t p = p0 + px;
            float v = 0.0f;
            if (p < plane) {
                const int32_t vv = (int32_t)(p / w), u = (int32_t)(p - (int64_t)vv * w);
                const ShiftSetup ss = shift_setup(s.soffs[2 * k], s.soffs[2 * k + 1]);
                const float *f = s.cal + (int64_t)k * s.W * s.H;
                const int32_t j = clampi(y0 + vv + ss.iy, 0, s.H - 1);
                const int32_t i = clampi(x0 + u + ss.ix, 0, s.W - 1);
                if (s.integer_mode) {
                    v = f[(int64_t)j * s.W + i];
                } else {
                    const int32_t j1 = clampi(ss.b > 0.0 ? j + 1 : j, 0, s.H - 1);
                    const int32_t i1 = ss.a > 0.0 ? clampi(x0 + u + ss.ix + 1, 0, s.W - 1) : i;
                    v = bilerp(ss.a, ss.b, f[(int64_t)j * s.W + i], f[(int64_t)j * s.W + i1],
                               f[(int64_t)j1 * s.W + i], f[(int64_t)j1 * s.W + i1]);
                }
            }
            tile[idx] = v;
        }
        __syncthreads();
        lanes_dispatch(s.lanes, s.N, [&](auto Lc, auto Vc) {
            constexpr int L = decltype(Lc)::value, V = decltype(Vc)::value;
            dropped += clip_tile<L, V>(tile, p0, plane, s.N, (double)s.ksigma, s.max_iters, s.out, nullptr);
        });
        __syncthreads();
    }
    if (s.n_rej && dropped) atomicAdd(reinterpret_cast<unsigned long long *>(s.n_rej), (unsigned long long)dropped);
}

__device__ __noinline__ void do_score(const StackDev &s, int32_t a, unsigned char *smem)
{
    score_dispatch(s.K, [&](auto Kc) { score_tile<decltype(Kc)::value>(s.sa, a, smem); });
}

__device__ __noinline__ void do_pick(const StackDev &s, int32_t k, Best *bscratch)
{
    const int32_t D = s.sa.D;
    double *S = s.scores + (int64_t)k * D * D;
    const double *pk = s.partial + (int64_t)k * s.sa.n_tiles * D * D;
    for (int32_t c = threadIdx.x; c < D * D; c += BATCH_THREADS)
        S[c] = candidate_score(pk, s.sa.n_tiles, D, s.R, s.R, 0, 0, c);
    __syncthreads();
    const int32_t kf = k + (k >= s.ref ? 1 : 0);
    pick_frame(S, D, s.R, s.R, 0, 0, s.offsets + kf, bscratch);
}

__device__ __noinline__ double do_meanpart(const StackDev &s, int32_t part, double *mscratch)
{
    return tmpl_part_sum(s.sa.ref, s.W, s.sa.tx0, s.sa.ty0, s.sa.tw, s.sa.th, part, mscratch);
}

__global__ __launch_bounds__(BATCH_THREADS, 4) void batch_kernel(BatchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t item_id;
    __shared__ int flag;
    __shared__ double mscratch[BATCH_THREADS / 64];
    __shared__ Best bscratch[BATCH_THREADS / 64];

    for (;;) {
        if (threadIdx.x == 0) {
            const bool err = __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
            item_id = err ? a.n_items : (int32_t)atomicAdd(a.head, 1u);
        }
        __syncthreads();
        const int32_t id = item_id;
        __syncthreads();
        if (id >= a.n_items) break;
        const Item it = a.items[id];
        const StackDev &s = a.stacks[it.stack];
        switch (it.type) {
        case IT_CAL:
            do_cal(s, it.a);
            signal_done(s.ctr + C_CAL);
            break;
        case IT_MEANPART: {
            if (!wait_count(a, s.ctr + C_CAL, (uint32_t)s.n_cal, &flag)) break;
            const double v = do_meanpart(s, it.a, mscratch);
            if (threadIdx.x == 0) s.mean_parts[it.a] = v;
            signal_done(s.ctr + C_MEANPART);
            break;
        }
        case IT_MEANFINAL: {
            if (!wait_count(a, s.ctr + C_MEANPART, (uint32_t)s.n_mean_parts, &flag)) break;
            const double m = tmpl_mean_of_parts(s.mean_parts, s.n_mean_parts, (double)s.sa.tw * (double)s.sa.th,
                                                mscratch);
            if (threadIdx.x == 0) *s.mean = m;
            signal_done(s.ctr + C_MEAN);
            break;
        }
        case IT_SCORE:
            if (!wait_count(a, s.ctr + C_MEAN, 1u, &flag)) break;
            do_score(s, it.a, smem);
            signal_done(s.ctr + C_SCORE);
            break;
        case IT_PICK: {
            if (!wait_count(a, s.ctr + C_SCORE, (uint32_t)s.n_score, &flag)) break;
            do_pick(s, it.a, bscratch);
            signal_done(s.ctr + C_PICK);
            break;
        }
        case IT_RECT:
            if (!wait_count(a, s.ctr + C_PICK, (uint32_t)s.n_pick, &flag)) break;
            do_rect(s);
            signal_done(s.ctr + C_RECT);
            break;
        case IT_OUT:
            if (!wait_count(a, s.ctr + C_RECT, 1u, &flag)) break;
            do_out(s, it.a, reinterpret_cast<float *>(smem));
            break;
        default:
            break;
        }
    }
}

__global__ void batch_reset(uint32_t *ctrs, int32_t n, int64_t *const *n_rej, int32_t n_stacks)
{
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) ctrs[i] = 0u;
    for (int32_t i = threadIdx.x; i < n_stacks; i += blockDim.x)
        if (n_rej[i]) *n_rej[i] = 0;
}

// ---- host side ---------------------------------------------------------------------------
static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

struct StackLayout {
    RegPlan plan;
    size_t cal, mean_parts, mean, partial, scores, soffs, rect;
    int32_t n_cal, n_mean_parts, n_score, n_pick, n_out;
};

struct BatchLayout {
    std::vector<StackLayout> st;
    size_t items, stacks, ctrs, head, nrej_ptrs, total;
    int32_t n_items;
    size_t lds;
};

static int32_t stack_ref(const reduce_stack_t &s) { return s.ref_index; }

static int validate(const reduce_stack_t *stacks, int32_t n)
{
    for (int32_t i = 0; i < n; ++i) {
        const reduce_stack_t &s = stacks[i];
        const std::string who = "reduce_stack_batch: stack " + std::to_string(i);
        if (!s.raw || !s.dark || !s.flat || !s.out || !s.out_rect || !s.offsets)
            return fail(REDUCE_ERR_NULL, who + ": NULL buffer");
        if (s.W < 1 || s.H < 1 || s.N < 1) return fail(REDUCE_ERR_SHAPE, who + ": W, H, N must be >= 1");
        if (s.raw_row_pitch < s.W || s.raw_frame_pitch < s.raw_row_pitch * (int64_t)(s.H - 1) + s.W ||
            s.cal_row_pitch < s.W)
            return fail(REDUCE_ERR_SHAPE, who + ": pitch smaller than the frame");
        if (s.N > COMB_MAX_N) return fail(REDUCE_ERR_UNSUPPORTED, who + ": N above 48");
        if (s.ref_index < 0 || s.ref_index >= s.N) return fail(REDUCE_ERR_RANGE, who + ": ref_index out of range");
        if (s.radius < 0 || s.W - 2 * s.radius < 1 || s.H - 2 * s.radius < 1)
            return fail(REDUCE_ERR_RANGE, who + ": radius leaves no template");
        if (!(s.ksigma > 0.0f) || s.max_iters < 0) return fail(REDUCE_ERR_RANGE, who + ": bad clip parameters");
        if (reg_plan(s.W, s.H, s.radius, s.radius).D == 0)
            return fail(REDUCE_ERR_UNSUPPORTED, who + ": radius too large for any launch shape");
    }
    return REDUCE_OK;
}

static BatchLayout layout_of(const reduce_stack_t *stacks, int32_t n)
{
    BatchLayout L;
    size_t off = 0;
    int64_t n_items = 0;
    L.lds = 0;
    for (int32_t i = 0; i < n; ++i) {
        const reduce_stack_t &s = stacks[i];
        StackLayout sl;
        sl.plan = reg_plan(s.W, s.H, s.radius, s.radius);
        const RegPlan &p = sl.plan;
        const int64_t fp = (int64_t)s.W * s.H;
        const int32_t nreg = s.N - 1;
        sl.cal = off;
        off += al(sizeof(float) * fp * s.N);
        sl.n_mean_parts = (int32_t)ceil_div(s.H - 2 * s.radius, MEAN_ROWS);
        sl.mean_parts = off;
        off += al(sizeof(double) * sl.n_mean_parts);
        sl.mean = off;
        off += 256;
        sl.partial = off;
        off += al(sizeof(double) * (size_t)std::max(nreg, 0) * p.n_tiles * p.D * p.D);
        sl.scores = off;
        off += al(sizeof(double) * (size_t)std::max(nreg, 0) * p.D * p.D);
        sl.soffs = off;
        off += al(sizeof(float) * 2 * s.N);
        sl.rect = off;
        off += 256;
        sl.n_cal = s.N * (int32_t)ceil_div(s.H, CAL_ROWS);
        sl.n_score = nreg * p.n_tiles * p.G;
        sl.n_pick = nreg;
        sl.n_out = (int32_t)ceil_div(fp, (int64_t)COMB_TILE * OUT_TILES);
        n_items += sl.n_cal + sl.n_mean_parts + 1 + sl.n_score + sl.n_pick + 1 + sl.n_out;
        L.lds = std::max(L.lds, std::max(p.lds, sizeof(float) * (size_t)s.N * COMB_TILE));
        L.st.push_back(sl);
    }
    L.n_items = (int32_t)n_items;
    L.items = off;
    off += al(sizeof(Item) * (size_t)n_items);
    L.stacks = off;
    off += al(sizeof(StackDev) * (size_t)n);
    L.ctrs = off;
    off += al(sizeof(uint32_t) * C_COUNT * (size_t)n);
    L.head = off;
    off += 256;  // head, error
    L.nrej_ptrs = off;
    off += al(sizeof(int64_t *) * (size_t)n);
    L.total = off;
    return L;
}

struct GraphEntry {
    uint64_t hash = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<unsigned char> host;  // uploaded descriptor bytes (kept alive with the entry)
    BatchArgs args{};
    uint32_t *ctrs = nullptr;
    int32_t n_ctrs = 0;
    int64_t *const *nrej = nullptr;
    int32_t n_stacks = 0;
    int grid = 0;
    size_t lds = 0;
};

static std::mutex g_batch_mu;
static std::map<void *, GraphEntry> g_graphs;  // by workspace address

static uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

static int build_entry(const reduce_stack_t *stacks, int32_t n, void *ws, const BatchLayout &L, GraphEntry *e,
                       hipStream_t s)
{
    unsigned char *base = static_cast<unsigned char *>(ws);
    std::vector<StackDev> sd(n);
    std::vector<Item> items;
    items.reserve(L.n_items);
    std::vector<int64_t *> nrej(n);
    for (int32_t i = 0; i < n; ++i) {
        const reduce_stack_t &st = stacks[i];
        const StackLayout &sl = L.st[i];
        StackDev &d = sd[i];
        d.raw = st.raw;
        d.rrp = st.raw_row_pitch;
        d.rfp = st.raw_frame_pitch;
        d.dark = st.dark;
        d.flat = st.flat;
        d.crp = st.cal_row_pitch;
        d.out = st.out;
        d.out_rect = st.out_rect;
        d.offsets = st.offsets;
        d.n_rej = st.n_rej;
        nrej[i] = st.n_rej;
        d.W = st.W;
        d.H = st.H;
        d.N = st.N;
        d.ref = stack_ref(st);
        d.R = st.radius;
        d.max_iters = st.max_iters;
        d.integer_mode = st.integer_mode ? 1 : 0;
        d.lanes = combine_lanes_for(st.N);
        d.K = sl.plan.K;
        d.ksigma = st.ksigma;
        d.cal = reinterpret_cast<float *>(base + sl.cal);
        d.mean_parts = reinterpret_cast<double *>(base + sl.mean_parts);
        d.mean = reinterpret_cast<double *>(base + sl.mean);
        d.partial = reinterpret_cast<double *>(base + sl.partial);
        d.scores = reinterpret_cast<double *>(base + sl.scores);
        d.soffs = reinterpret_cast<float *>(base + sl.soffs);
        d.rect = reinterpret_cast<int32_t *>(base + sl.rect);
        d.ctr = reinterpret_cast<uint32_t *>(base + L.ctrs) + (size_t)C_COUNT * i;
        d.n_cal = sl.n_cal;
        d.n_mean_parts = sl.n_mean_parts;
        d.n_score = sl.n_score;
        d.n_pick = sl.n_pick;
        const int32_t R = st.radius;
        const float *ref = d.cal + (int64_t)d.ref * st.W * st.H;
        d.sa = make_score_args(sl.plan, ref, d.cal, nullptr, d.mean, d.partial, st.W, st.H, std::max(st.N - 1, 1), R,
                               R, R, R, st.W - 2 * R, st.H - 2 * R, d.ref);
    }
    // the queue, phase by phase; search items of the largest stacks first
    for (int32_t i = 0; i < n; ++i)
        for (int32_t a = 0; a < L.st[i].n_cal; ++a) items.push_back({IT_CAL, i, a, 0});
    for (int32_t i = 0; i < n; ++i)
        for (int32_t a = 0; a < L.st[i].n_mean_parts; ++a) items.push_back({IT_MEANPART, i, a, 0});
    for (int32_t i = 0; i < n; ++i) items.push_back({IT_MEANFINAL, i, 0, 0});
    std::vector<int32_t> order(n);
    for (int32_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        const double cx = (double)L.st[x].n_score * L.st[x].plan.BR * L.st[x].plan.TX * L.st[x].plan.C;
        const double cy = (double)L.st[y].n_score * L.st[y].plan.BR * L.st[y].plan.TX * L.st[y].plan.C;
        return cx > cy;
    });
    for (int32_t i : order)
        for (int32_t a = 0; a < L.st[i].n_score; ++a) items.push_back({IT_SCORE, i, a, 0});
    for (int32_t i = 0; i < n; ++i)
        for (int32_t a = 0; a < L.st[i].n_pick; ++a) items.push_back({IT_PICK, i, a, 0});
    for (int32_t i = 0; i < n; ++i) items.push_back({IT_RECT, i, 0, 0});
    for (int32_t i : order)
        for (int32_t a = 0; a < L.st[i].n_out; ++a) items.push_back({IT_OUT, i, a, 0});
    if ((int32_t)items.size() != L.n_items) return fail(REDUCE_ERR_SHAPE, "reduce_stack_batch: item count");

    // descriptors into the workspace
    e->host.assign(L.total - L.items, 0);
    std::memcpy(e->host.data(), items.data(), sizeof(Item) * items.size());
    std::memcpy(e->host.data() + (L.stacks - L.items), sd.data(), sizeof(StackDev) * sd.size());
    std::memcpy(e->host.data() + (L.nrej_ptrs - L.items), nrej.data(), sizeof(int64_t *) * nrej.size());
    if (hipMemcpyAsync(base + L.items, e->host.data(), e->host.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(REDUCE_ERR_HIP, "reduce_stack_batch: descriptor upload");

    BatchArgs &a = e->args;
    a.items = reinterpret_cast<const Item *>(base + L.items);
    a.stacks = reinterpret_cast<const StackDev *>(base + L.stacks);
    a.n_items = L.n_items;
    a.head = reinterpret_cast<uint32_t *>(base + L.head);
    a.error = a.head + 1;
    const char *lim = std::getenv("REDUCE_BATCH_SPIN_LIMIT");
    a.spin_limit = lim ? (uint32_t)std::strtoul(lim, nullptr, 10) : (1u << 27);
    e->ctrs = reinterpret_cast<uint32_t *>(base + L.ctrs);
    e->n_ctrs = C_COUNT * n;
    e->nrej = reinterpret_cast<int64_t *const *>(base + L.nrej_ptrs);
    e->n_stacks = n;
    e->lds = L.lds;

    // persistent grid: as many workgroups as can be resident at once
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))
        return fail(REDUCE_ERR_HIP, "reduce_stack_batch: device query");
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel, BATCH_THREADS, L.lds) != hipSuccess ||
        per_cu < 1)
        return fail(REDUCE_ERR_HIP, "reduce_stack_batch: the kernel does not fit on a compute unit");
    e->grid = std::min<int64_t>((int64_t)cus * per_cu, std::max<int32_t>(L.n_items, 1));

    // graph: reset counters and error flag, then the persistent kernel
    if (hipGraphCreate(&e->graph, 0) != hipSuccess) return fail(REDUCE_ERR_HIP, "reduce_stack_batch: graph");
    uint32_t *ctr_all = e->ctrs;
    int32_t n_all = (int32_t)((L.head + 8 - L.ctrs) / sizeof(uint32_t));  // counters, head and error
    void *reset_args[] = {&ctr_all, &n_all, (void *)&e->nrej, &e->n_stacks};
    hipKernelNodeParams rp{};
    rp.func = reinterpret_cast<void *>(batch_reset);
    rp.gridDim = dim3(1);
    rp.blockDim = dim3(256);
    rp.sharedMemBytes = 0;
    rp.kernelParams = reset_args;
    hipGraphNode_t n_reset, n_main;
    if (hipGraphAddKernelNode(&n_reset, e->graph, nullptr, 0, &rp) != hipSuccess)
        return fail(REDUCE_ERR_HIP, "reduce_stack_batch: graph reset node");
    void *main_args[] = {&e->args};
    hipKernelNodeParams mp{};
    mp.func = reinterpret_cast<void *>(batch_kernel);
    mp.gridDim = dim3((unsigned)e->grid);
    mp.blockDim = dim3(BATCH_THREADS);
    mp.sharedMemBytes = (unsigned)L.lds;
    mp.kernelParams = main_args;
    if (hipGraphAddKernelNode(&n_main, e->graph, &n_reset, 1, &mp) != hipSuccess)
        return fail(REDUCE_ERR_HIP, "reduce_stack_batch: graph kernel node");
    if (hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(REDUCE_ERR_HIP, "reduce_stack_batch: graph instantiate");
    return REDUCE_OK;
}

static void destroy_entry(GraphEntry &e)
{
    if (e.exec) hipGraphExecDestroy(e.exec);
    if (e.graph) hipGraphDestroy(e.graph);
    e.exec = nullptr;
    e.graph = nullptr;
}

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_stack_batch_ws(const reduce_stack_t *stacks, int32_t n)
{
    if (!stacks || n < 1) return 0;
    if (validate(stacks, n) != REDUCE_OK) return 0;
    return layout_of(stacks, n).total;
}

extern "C" int reduce_stack_batch(const reduce_stack_t *stacks, int32_t n, void *ws, size_t ws_bytes, void *stream)
{
    if (!stacks) return fail(REDUCE_ERR_NULL, "reduce_stack_batch: NULL stacks");
    if (n < 1) return fail(REDUCE_ERR_SHAPE, "reduce_stack_batch: no stacks");
    const int v = validate(stacks, n);
    if (v != REDUCE_OK) return v;
    const BatchLayout L = layout_of(stacks, n);
    if (!ws || ws_bytes < L.total)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_stack_batch: workspace needs " + std::to_string(L.total) + " bytes");
    if (L.n_items < 0) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_stack_batch: too many work items");
    hipStream_t s = as_stream(stream);

    // a graph per workspace, rebuilt when the stacks or their launch shapes change
    uint64_t h = fnv1a(stacks, sizeof(reduce_stack_t) * (size_t)n);
    for (const StackLayout &sl : L.st) h = fnv1a(&sl.plan, sizeof(RegPlan), h);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t lanes = combine_lanes_for(stacks[i].N);
        h = fnv1a(&lanes, sizeof(lanes), h);
    }
    h = fnv1a(&L.total, sizeof(L.total), h);
    const char *lim = std::getenv("REDUCE_BATCH_SPIN_LIMIT");
    h = fnv1a(lim ? lim : "", lim ? std::strlen(lim) : 0, h);
    std::lock_guard<std::mutex> lk(g_batch_mu);
    GraphEntry &e = g_graphs[ws];
    if (!e.exec || e.hash != h) {
        if (e.exec && hipStreamSynchronize(s) != hipSuccess)  // the old graph may still run
            return fail(REDUCE_ERR_HIP, "reduce_stack_batch: synchronize before rebuilding");
        destroy_entry(e);
        e = GraphEntry{};
        const int rc = build_entry(stacks, n, ws, L, &e, s);
        if (rc != REDUCE_OK) {
            destroy_entry(e);
            g_graphs.erase(ws);
            return rc;
        }
        e.hash = h;
    }
    ProfScope prof("batch_kernel", s);
    if (hipGraphLaunch(e.exec, s) != hipSuccess) return fail(REDUCE_ERR_HIP, "reduce_stack_batch: graph launch");
    return check_launch("reduce_stack_batch");
}

extern "C" int reduce_stack_batch_check(const void *ws, size_t ws_bytes, const reduce_stack_t *stacks, int32_t n,
                                        void *stream)
{
    if (!ws || !stacks) return fail(REDUCE_ERR_NULL, "reduce_stack_batch_check: NULL argument");
    if (n < 1) return fail(REDUCE_ERR_SHAPE, "reduce_stack_batch_check: no stacks");
    const BatchLayout L = layout_of(stacks, n);
    if (ws_bytes < L.total) return fail(REDUCE_ERR_WORKSPACE, "reduce_stack_batch_check: workspace too small");
    uint32_t flag = 0;
    hipStream_t s = as_stream(stream);
    if (hipMemcpyAsync(&flag, static_cast<const unsigned char *>(ws) + L.head + 4, sizeof(flag),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(REDUCE_ERR_HIP, "reduce_stack_batch_check: read of the error flag");
    if (flag) return fail(REDUCE_ERR_HIP, "reduce_stack_batch: a dependency wait exceeded its spin limit");
    return REDUCE_OK;
}
