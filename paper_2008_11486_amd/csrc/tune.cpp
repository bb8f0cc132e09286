// Autotuner: times candidate launch shapes on the caller's data with HIP events and
// caches the fastest per problem size; the cache persists as JSON lines keyed by the
// device architecture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "common.h"
#include "register_plan.h"

namespace rd {

int register_launch(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N, int32_t R,
                    int32_t Rmax, const int32_t *centers, int32_t tx0, int32_t ty0, int32_t tw, int32_t th,
                    reduce_offset_t *out, double *scores, void *ws, const RegPlan &p, hipStream_t s);
size_t register_ws_bytes(const RegPlan &p, int32_t N);
void combine_dispatch(int lanes, const float *aligned, int64_t plane, int32_t N, double ksigma, int32_t max_iters,
                      float *out, uint8_t *keep, unsigned long long *n_rej, hipStream_t s);
int tune_save(const char *path, const char *arch);
int tune_load(const char *path, const char *arch);
void tune_clear();

static std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// Average milliseconds of `reps` calls of fn after one warm-up call.
template <typename F>
static int time_ms(hipStream_t s, int reps, F fn, double *ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(REDUCE_ERR_HIP, "autotune: event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(REDUCE_ERR_HIP, "autotune: event");
    }
    int rc = fn();
    if (rc == REDUCE_OK) {
        if (hipEventRecord(e0, s) != hipSuccess) rc = fail(REDUCE_ERR_HIP, "autotune: event record");
        for (int i = 0; i < reps && rc == REDUCE_OK; ++i) rc = fn();
        if (rc == REDUCE_OK && hipEventRecord(e1, s) != hipSuccess) rc = fail(REDUCE_ERR_HIP, "autotune: event record");
        if (rc == REDUCE_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(REDUCE_ERR_HIP, "autotune: synchronize");
    }
    float t = 0.0f;
    if (rc == REDUCE_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = fail(REDUCE_ERR_HIP, "autotune: time");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return rc;
}

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_tune_register_ws(int32_t W, int32_t H, int32_t N, int32_t radius, int32_t radius_max)
{
    if (W < 1 || H < 1 || N < 1 || radius < 0 || radius_max < 0) return 0;
    if (W - 2 * radius_max < 1 || H - 2 * radius_max < 1) return 0;
    size_t need = reduce_register_ws(W, H, N, radius, radius_max);
    RegPlan sp;
    if (reg_plan_small(W, H, radius, radius_max, &sp)) return need;
    constexpr int MAXC = 64;
    RegShape cand[MAXC];
    int n = 0;
    reg_shape_candidates(W, H, radius, radius_max, cand, &n, MAXC);
    for (int i = 0; i < n; ++i) {
        RegShape one = cand[i];
        one.CPT = 1;  // the most tiles this shape can have (the tuner also tries other tile heights)
        RegPlan p;
        if (reg_plan_from_shape(W, H, radius, radius_max, one, &p)) need = std::max(need, register_ws_bytes(p, N));
    }
    return need;
}

extern "C" int reduce_tune_register(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                                    int32_t radius, int32_t radius_max, reduce_offset_t *out, void *ws,
                                    size_t ws_bytes, int32_t reps, void *stream, int32_t *fields)
{
    if (!ref || !frames || !ws || !out) return fail(REDUCE_ERR_NULL, "reduce_tune_register: NULL buffer");
    if (W < 1 || H < 1 || N < 1 || radius < 0 || radius_max < 0 || W - 2 * radius_max < 1 ||
        H - 2 * radius_max < 1)
        return fail(REDUCE_ERR_RANGE, "reduce_tune_register: no template for these sizes");
    if (reps < 1) reps = 1;
    hipStream_t s = as_stream(stream);
    {
        RegPlan sp;
        if (reg_plan_small(W, H, radius, radius_max, &sp)) {  // small windows have one shape
            if (fields) {
                const int32_t v[16] = {sp.D, sp.K, sp.NBX, sp.C, sp.G, sp.CW, sp.S, sp.threads, sp.TX, sp.TY, sp.BR,
                                       sp.JS, sp.FR, sp.FC, (int32_t)sp.lds, sp.n_tiles};
                for (int i = 0; i < 16; ++i) fields[i] = v[i];
            }
            return REDUCE_OK;
        }
    }
    constexpr int MAXC = 64;
    RegShape cand[MAXC];
    int n = 0;
    reg_shape_candidates(W, H, radius, radius_max, cand, &n, MAXC);
    double best_ms = 1e30;
    RegShape best{};
    const int32_t tx0 = radius_max, ty0 = radius_max, tw = W - 2 * radius_max, th = H - 2 * radius_max;
    int rc = REDUCE_OK;
    auto time_shape = [&](const RegShape &sh, double *ms) -> int {
        RegPlan p;
        if (!reg_plan_from_shape(W, H, radius, radius_max, sh, &p) || register_ws_bytes(p, N) > ws_bytes) {
            *ms = 1e30;
            return REDUCE_OK;
        }
        const int r = time_ms(s, reps,
                              [&]() {
                                  return register_launch(ref, frames, W, H, N, radius, radius_max, nullptr, tx0, ty0,
                                                         tw, th, out, nullptr, ws, p, s);
                              },
                              ms);
        if (std::getenv("REDUCE_TUNE_VERBOSE"))
            std::fprintf(stderr, "tune register K=%d G=%d S=%d TY=%d BR=%d threads=%d tiles=%d: %.4f ms\n", p.K, p.G,
                         p.S, p.TY, p.BR, p.threads, p.n_tiles, *ms);
        return r;
    };
    // first round: every candidate once
    std::vector<std::pair<double, RegShape>> timed;
    for (int i = 0; i < n && rc == REDUCE_OK; ++i) {
        double ms = 0.0;
        rc = time_shape(cand[i], &ms);
        if (ms < 1e30) timed.push_back({ms, cand[i]});
    }
    if (rc != REDUCE_OK) return rc;
    if (timed.empty()) return fail(REDUCE_ERR_WORKSPACE, "reduce_tune_register: no candidate fits the workspace");
    std::stable_sort(timed.begin(), timed.end(),
                     [](const std::pair<double, RegShape> &x, const std::pair<double, RegShape> &y) {
                         return x.first < y.first;
                     });
    // contenders: the three fastest, and the fastest with other tile heights (up to four
    // chunks and kTileRowsMax rows)
    std::vector<RegShape> cont;
    for (size_t i = 0; i < timed.size() && cont.size() < 3; ++i) cont.push_back(timed[i].second);
    const RegShape top = timed[0].second;
    for (int32_t cpt : {top.CPT * 2, top.CPT * 3, top.CPT * 4, top.CPT / 2, 1}) {
        if (cpt < 1 || cpt > 4) continue;
        RegShape v = top;
        v.CPT = cpt;
        RegPlan pv;
        if (!reg_plan_from_shape(W, H, radius, radius_max, v, &pv) || pv.BR > kTileRowsMax) continue;
        bool dup = false;
        for (const RegShape &c : cont)
            dup = dup || (c.K == v.K && c.G == v.G && c.S == v.S && c.TY == v.TY && c.CPT == v.CPT);
        if (!dup) cont.push_back(v);
    }
    // then three interleaved rounds over the contenders (clock and temperature drift over a
    // long tuning run would otherwise favour whichever ran first); the least time wins
    std::vector<double> least(cont.size(), 1e30);
    for (int round = 0; round < 3 && rc == REDUCE_OK; ++round)
        for (size_t i = 0; i < cont.size() && rc == REDUCE_OK; ++i) {
            double ms = 0.0;
            rc = time_shape(cont[i], &ms);
            least[i] = std::min(least[i], ms);
        }
    for (size_t i = 0; i < cont.size(); ++i)
        if (least[i] < best_ms) {
            best_ms = least[i];
            best = cont[i];
        }
    if (rc != REDUCE_OK) return rc;
    if (best_ms >= 1e30) return fail(REDUCE_ERR_WORKSPACE, "reduce_tune_register: no candidate fits the workspace");
    set_tuned_reg_shape(W, H, radius, radius_max, best, best_ms);
    if (fields) {
        RegPlan p;
        reg_plan_from_shape(W, H, radius, radius_max, best, &p);
        const int32_t v[16] = {p.D, p.K, p.NBX, p.C, p.G, p.CW, p.S, p.threads, p.TX, p.TY, p.BR, p.JS, p.FR, p.FC,
                               (int32_t)p.lds, p.n_tiles};
        for (int i = 0; i < 16; ++i) fields[i] = v[i];
    }
    return REDUCE_OK;
}

extern "C" int reduce_tune_combine(const float *aligned, int32_t w, int32_t h, int32_t N, float ksigma,
                                   int32_t max_iters, float *out, int32_t reps, void *stream, int32_t *lanes)
{
    if (!aligned || !out) return fail(REDUCE_ERR_NULL, "reduce_tune_combine: NULL buffer");
    if (w < 1 || h < 1 || N < 1 || N > 48) return fail(REDUCE_ERR_SHAPE, "reduce_tune_combine: bad sizes");
    if (!(ksigma > 0.0f) || max_iters < 0) return fail(REDUCE_ERR_RANGE, "reduce_tune_combine: bad clip parameters");
    if (reps < 1) reps = 1;
    hipStream_t s = as_stream(stream);
    double best_ms = 1e30;
    int best = 1;
    for (int L : {1, 2, 4, 8, 16}) {
        double ms = 0.0;
        const int rc = time_ms(s, reps,
                               [&]() {
                                   combine_dispatch(L, aligned, (int64_t)w * h, N, (double)ksigma, max_iters, out,
                                                    nullptr, nullptr, s);
                                   return check_launch("reduce_tune_combine");
                               },
                               &ms);
        if (rc != REDUCE_OK) return rc;
        if (ms < best_ms) {
            best_ms = ms;
            best = L;
        }
    }
    set_tuned_combine_lanes(N, best, best_ms);
    if (lanes) *lanes = best;
    return REDUCE_OK;
}

extern "C" int reduce_tune_search(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                                  int32_t radius, reduce_offset_t *out, void *ws, size_t ws_bytes, int32_t reps,
                                  void *stream, int32_t *search, double *ms_direct, double *ms_spectral)
{
    if (!ref || !frames || !out || !ws || !search) return fail(REDUCE_ERR_NULL, "reduce_tune_search: NULL argument");
    if (W < 1 || H < 1 || N < 1 || radius < 1 || W - 2 * radius < 1 || H - 2 * radius < 1)
        return fail(REDUCE_ERR_RANGE, "reduce_tune_search: no template for these sizes");
    if (reps < 1) reps = 1;
    hipStream_t s = as_stream(stream);
    const size_t need_d = reduce_register_ws(W, H, N, radius, radius);
    const size_t need_s = reduce_register_fft_ws(W, H, N, radius);
    if (need_d == 0 || ws_bytes < need_d)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_tune_search: workspace needs " + std::to_string(need_d) + " bytes");
    double td = 0.0, ts = 1e30;
    int rc = time_ms(s, reps,
                     [&]() {
                         return reduce_register(ref, frames, W, H, N, radius, radius, nullptr, nullptr, out, nullptr,
                                                ws, ws_bytes, s);
                     },
                     &td);
    if (rc != REDUCE_OK) return rc;
    if (need_s != 0 && ws_bytes >= need_s) {
        rc = time_ms(s, reps,
                     [&]() {
                         return reduce_register_fft(ref, frames, W, H, N, radius, out, nullptr, nullptr, ws, ws_bytes,
                                                    s);
                     },
                     &ts);
        if (rc != REDUCE_OK) return rc;
    }
    *search = ts < td ? REDUCE_SEARCH_SPECTRAL : REDUCE_SEARCH_DIRECT;
    if (ms_direct) *ms_direct = td;
    if (ms_spectral) *ms_spectral = ts;
    return REDUCE_OK;
}

extern "C" int reduce_tune_save(const char *path)
{
    if (!path) return fail(REDUCE_ERR_NULL, "reduce_tune_save: NULL path");
    return tune_save(path, device_arch().c_str());
}

extern "C" int reduce_tune_load(const char *path)
{
    if (!path) return fail(REDUCE_ERR_NULL, "reduce_tune_load: NULL path");
    return tune_load(path, device_arch().c_str());
}

extern "C" int reduce_tune_clear(void)
{
    tune_clear();
    return REDUCE_OK;
}
