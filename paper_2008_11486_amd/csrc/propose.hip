// Learned registration on the stream, without host round trips: the network proposes a
// window centre per frame, the correlation search runs in a small window around it with
// the full search's template, windows whose maximum sits on an inner border walk onto that
// maximum, and the frames whose narrowed result cannot be trusted take the full-window
// search.  Every decision is taken by a kernel; the host only enqueues.
//
// Slots.  The search kernels take a slot -> frame map (register_core.h): the window walk
// maps slot k to frame k while frame k moves and to -1 otherwise, and the fallback search
// runs over a compacted list of the flagged frames, F slots per round, so its workspace
// holds F frames' partial scores rather than N.  Idle slots leave at once.
#include <algorithm>
#include <string>

#include "common.h"
#include "learned.h"
#include "register_core.h"
#include "register_plan.h"

namespace rd {

void register_mean(const float *ref, int32_t W, int32_t tx0, int32_t ty0, int32_t tw, int32_t th,
                   double *mean_parts, double *mean, hipStream_t s);
void register_scores(const RegPlan &p, const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                     int32_t R, int32_t Rmax, const int32_t *centers, const int32_t *map, int32_t tx0, int32_t ty0,
                     int32_t tw, int32_t th, const double *mean, double *partial, double *sc, reduce_offset_t *out,
                     hipStream_t s);

// Partial-score budget of the fallback search: the number of frames it scores at once is
// chosen so that their tile partials fit in this many bytes (at least one frame).
constexpr size_t PROPOSE_FALLBACK_BYTES = size_t(256) << 20;
constexpr int32_t PROPOSE_MAX_MOVES = 64;

// The window maximum lies on a border strictly inside +-rmax (a border at +-rmax is also
// the full search's border, where a move cannot help).
__device__ __forceinline__ bool inner_border(const reduce_offset_t &o, int32_t rmax)
{
    const bool bx = (o.flags & REDUCE_EDGE_X) && o.dx > -rmax && o.dx < rmax;
    const bool by = (o.flags & REDUCE_EDGE_Y) && o.dy > -rmax && o.dy < rmax;
    return bx || by;
}

// One window move: a frame with an inner-border maximum gets its centre on that maximum
// and its slot (map[k] = k); every other slot idles.
__global__ void propose_walk(const reduce_offset_t *__restrict__ offs, int32_t N, int32_t rmax,
                             int32_t *__restrict__ centres, int32_t *__restrict__ map, int32_t *__restrict__ info)
{
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const reduce_offset_t o = offs[k];
    if (inner_border(o, rmax)) {
        centres[2 * k] = min(max(o.dx, -rmax), rmax);
        centres[2 * k + 1] = min(max(o.dy, -rmax), rmax);
        map[k] = k;
        info[k] += 1;
    } else {
        map[k] = -1;
    }
}

// Fallback decision per frame (maximum still on an inner border, or a peak below
// peak_ratio times the reference's own zero-offset score) and the flagged frames in
// increasing order: list[0, n) = flagged frames, list[n, N) = -1.  One wave.
__global__ __launch_bounds__(64) void propose_flag(const reduce_offset_t *__restrict__ offs, int32_t N, int32_t rmax,
                                                   double peak_ratio, const reduce_offset_t *__restrict__ auto_off,
                                                   int32_t *__restrict__ list, int32_t *__restrict__ info)
{
    const int lane = threadIdx.x;
    const double s_auto = auto_off->peak;
    int32_t base = 0;
    for (int32_t c0 = 0; c0 < N; c0 += 64) {
        const int32_t k = c0 + lane;
        bool fb = false;
        if (k < N) {
            const reduce_offset_t o = offs[k];
            const bool border = inner_border(o, rmax);
            const bool weak = !(o.peak >= peak_ratio * s_auto);
            fb = border || weak;
            info[k] |= (border ? 1 << 8 : 0) | (weak ? 1 << 9 : 0);
        }
        const uint64_t m = __ballot(fb);
        if (fb) list[base + __popcll(m & ((1ull << lane) - 1ull))] = k;
        base += __popcll(m);
    }
    for (int32_t k = base + lane; k < N; k += 64) list[k] = -1;
}

// The flagged frames now hold the full search's result: mark them.
__global__ void propose_mark(const int32_t *__restrict__ list, int32_t N, reduce_offset_t *__restrict__ offs)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t k = list[i];
    if (k >= 0) offs[k].flags |= REDUCE_FALLBACK;
}

__global__ void propose_zero(int32_t *__restrict__ v, int32_t n)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = 0;
}

// ---- host side ---------------------------------------------------------------------
static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct ProposeLayout {
    RegPlan small, full, zero;
    int32_t F;  // frames per fallback round
    size_t inp_ref, inp, in_ws, cnn_ws, pred, cen, map, list, info, mean_parts, mean, auto_off;
    size_t part_s, sc_s, part_0, sc_0, part_f, sc_f, total;
    size_t in_ws_bytes, cnn_ws_bytes;
};

static bool propose_layout(int32_t W, int32_t H, int32_t N, int32_t R, int32_t Rmax, ProposeLayout *L)
{
    L->small = reg_plan(W, H, R, Rmax);
    L->full = reg_plan(W, H, Rmax, Rmax);
    L->zero = reg_plan(W, H, 0, Rmax);
    if (L->small.D == 0 || L->full.D == 0 || L->zero.D == 0) return false;
    const int32_t h = H / 4, w = W / 4;
    L->in_ws_bytes = reduce_cnn_input_ws(W, H, N);
    L->cnn_ws_bytes = reduce_cnn_ws(N, h, w);
    if (L->in_ws_bytes == 0 || L->cnn_ws_bytes == 0) return false;
    const size_t per_full = sizeof(double) * (size_t)L->full.n_tiles * L->full.D * L->full.D;
    L->F = (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)N, PROPOSE_FALLBACK_BYTES / per_full));
    const int32_t th = H - 2 * Rmax;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += al256(std::max<size_t>(bytes, 1));
        return at;
    };
    L->inp_ref = take(sizeof(uint16_t) * (size_t)h * w);
    L->inp = take(sizeof(uint16_t) * (size_t)N * h * w);
    L->in_ws = take(L->in_ws_bytes);
    L->cnn_ws = take(L->cnn_ws_bytes);
    L->pred = take(sizeof(float) * 2 * (size_t)N);
    L->cen = take(sizeof(int32_t) * 2 * (size_t)N);
    L->map = take(sizeof(int32_t) * (size_t)N);
    L->list = take(sizeof(int32_t) * (size_t)N);
    L->info = take(sizeof(int32_t) * (size_t)N);
    L->mean_parts = take(sizeof(double) * (size_t)ceil_div(th, MEAN_ROWS));
    L->mean = take(sizeof(double));
    L->auto_off = take(sizeof(reduce_offset_t));
    const RegPlan &ps = L->small, &pz = L->zero, &pf = L->full;
    L->part_s = take(sizeof(double) * (size_t)N * ps.n_tiles * ps.D * ps.D);
    L->sc_s = take(sizeof(double) * (size_t)N * ps.D * ps.D);
    L->part_0 = take(sizeof(double) * (size_t)pz.n_tiles * pz.D * pz.D);
    L->sc_0 = take(sizeof(double) * (size_t)pz.D * pz.D);
    L->part_f = take(per_full * (size_t)L->F);
    L->sc_f = take(sizeof(double) * (size_t)L->F * pf.D * pf.D);
    L->total = o;
    return true;
}

static int propose_check(int32_t W, int32_t H, int32_t N, int32_t R, int32_t Rmax, const char *who)
{
    const std::string w(who);
    if (W < 64 || H < 64 || N < 1) return fail(REDUCE_ERR_SHAPE, w + ": W, H >= 64 and N >= 1 needed");
    if (W % 4 || H % 4) return fail(REDUCE_ERR_SHAPE, w + ": W and H must be multiples of 4");
    if (N > 65535) return fail(REDUCE_ERR_UNSUPPORTED, w + ": N above 65535");
    if (R < 0 || Rmax < R) return fail(REDUCE_ERR_RANGE, w + ": 0 <= refine_radius <= radius_max needed");
    if (W - 2 * Rmax < 1 || H - 2 * Rmax < 1) return fail(REDUCE_ERR_RANGE, w + ": radius_max leaves no template");
    return REDUCE_OK;
}

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_propose_ws(int32_t W, int32_t H, int32_t N, int32_t refine_radius, int32_t radius_max)
{
    if (W < 64 || H < 64 || N < 1 || N > 65535 || W % 4 || H % 4 || refine_radius < 0 ||
        radius_max < refine_radius || W - 2 * radius_max < 1 || H - 2 * radius_max < 1)
        return 0;
    ProposeLayout L;
    return propose_layout(W, H, N, refine_radius, radius_max, &L) ? L.total : 0;
}

extern "C" int reduce_propose(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                              const float *params, int32_t refine_radius, int32_t radius_max, float peak_ratio,
                              int32_t max_moves, reduce_offset_t *out, int32_t *centres, int32_t *info, void *ws,
                              size_t ws_bytes, void *stream)
{
    if (!ref || !frames || !params || !out) return fail(REDUCE_ERR_NULL, "reduce_propose: NULL buffer");
    const int c = propose_check(W, H, N, refine_radius, radius_max, "reduce_propose");
    if (c != REDUCE_OK) return c;
    if (!std::isfinite(peak_ratio)) return fail(REDUCE_ERR_RANGE, "reduce_propose: peak_ratio must be finite");
    if (max_moves < 0 || max_moves > PROPOSE_MAX_MOVES)
        return fail(REDUCE_ERR_RANGE, "reduce_propose: max_moves outside [0, 64]");
    ProposeLayout L;
    if (!propose_layout(W, H, N, refine_radius, radius_max, &L))
        return fail(REDUCE_ERR_UNSUPPORTED, "reduce_propose: no launch shape for these sizes");
    if (!ws || ws_bytes < L.total)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_propose: workspace needs " + std::to_string(L.total) + " bytes");
    hipStream_t s = as_stream(stream);
    unsigned char *b = static_cast<unsigned char *>(ws);
    auto at = [&](size_t off) { return static_cast<void *>(b + off); };
    uint16_t *inp_ref = static_cast<uint16_t *>(at(L.inp_ref));
    uint16_t *inp = static_cast<uint16_t *>(at(L.inp));
    float *pred = static_cast<float *>(at(L.pred));
    int32_t *cen = static_cast<int32_t *>(at(L.cen));
    int32_t *map = static_cast<int32_t *>(at(L.map));
    int32_t *list = static_cast<int32_t *>(at(L.list));
    int32_t *inf = info ? info : static_cast<int32_t *>(at(L.info));
    double *mean_parts = static_cast<double *>(at(L.mean_parts));
    double *mean = static_cast<double *>(at(L.mean));
    reduce_offset_t *auto_off = static_cast<reduce_offset_t *>(at(L.auto_off));
    const int32_t h = H / 4, w = W / 4;
    const int32_t R = refine_radius, Rm = radius_max;
    const int32_t tx0 = Rm, ty0 = Rm, tw = W - 2 * Rm, th = H - 2 * Rm;
    ProfScope prof("propose", s);

    // network input and forward pass, window centres
    int rc = reduce_cnn_input(ref, W, H, 1, inp_ref, at(L.in_ws), L.in_ws_bytes, s);
    if (rc == REDUCE_OK) rc = reduce_cnn_input(frames, W, H, N, inp, at(L.in_ws), L.in_ws_bytes, s);
    if (rc == REDUCE_OK)
        rc = reduce_cnn_forward(inp_ref, 0, inp, N, h, w, params, pred, at(L.cnn_ws), L.cnn_ws_bytes, s);
    if (rc == REDUCE_OK) rc = reduce_cnn_centres(pred, N, 4.0f, Rm, cen, s);
    if (rc == REDUCE_OK && centres) rc = reduce_cnn_centres(pred, N, 4.0f, Rm, centres, s);
    if (rc != REDUCE_OK) return rc;
    hipLaunchKernelGGL(propose_zero, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, inf, N);

    // one template mean for every search below (they share the template)
    register_mean(ref, W, tx0, ty0, tw, th, mean_parts, mean, s);
    // the reference's own zero-offset score, and the narrowed search of every frame
    register_scores(L.zero, ref, ref, W, H, 1, 0, Rm, nullptr, nullptr, tx0, ty0, tw, th, mean,
                    static_cast<double *>(at(L.part_0)), static_cast<double *>(at(L.sc_0)), auto_off, s);
    double *part_s = static_cast<double *>(at(L.part_s));
    double *sc_s = static_cast<double *>(at(L.sc_s));
    register_scores(L.small, ref, frames, W, H, N, R, Rm, cen, nullptr, tx0, ty0, tw, th, mean, part_s, sc_s, out, s);
    // window moves: only the frames whose maximum is on an inner border are searched again
    for (int32_t m = 0; m < max_moves; ++m) {
        hipLaunchKernelGGL(propose_walk, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, out, N, Rm, cen, map, inf);
        register_scores(L.small, ref, frames, W, H, N, R, Rm, cen, map, tx0, ty0, tw, th, mean, part_s, sc_s, out, s);
    }
    // fallback: the full window for the flagged frames, F of them per round
    hipLaunchKernelGGL(propose_flag, dim3(1), dim3(64), 0, s, out, N, Rm, (double)peak_ratio, auto_off, list, inf);
    for (int32_t r0 = 0; r0 < N; r0 += L.F) {
        const int32_t n = std::min(L.F, N - r0);
        register_scores(L.full, ref, frames, W, H, n, Rm, Rm, nullptr, list + r0, tx0, ty0, tw, th, mean,
                        static_cast<double *>(at(L.part_f)), static_cast<double *>(at(L.sc_f)), out, s);
    }
    hipLaunchKernelGGL(propose_mark, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, list, N, out);
    return check_launch("reduce_propose");
}
