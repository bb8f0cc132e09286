// Host-side pieces of the C ABI: status strings, the thread-local error detail,
// launch checking and the host-only common-overlap computation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace rd {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg)
{
    g_last_error = msg;
    return status;
}

int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(REDUCE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return REDUCE_OK;
}

// ---- kernel timing ------------------------------------------------------------
struct ProfRec {
    std::string name;
    hipEvent_t start, stop;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_event_pool;

bool prof_on() { return g_prof_on; }

static hipEvent_t take_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_record(const char *name, hipStream_t s, bool start)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (start) {
        ProfRec r{name, take_event(), nullptr};
        if (r.start && hipEventRecord(r.start, s) != hipSuccess) {  // a record that failed is not timed
            g_event_pool.push_back(r.start);
            r.start = nullptr;
        }
        g_prof.push_back(r);
    } else {
        for (auto it = g_prof.rbegin(); it != g_prof.rend(); ++it)
            if (it->stop == nullptr && it->name == name) {
                it->stop = take_event();
                if (it->stop && hipEventRecord(it->stop, s) != hipSuccess) {
                    g_event_pool.push_back(it->stop);
                    it->stop = nullptr;
                }
                break;
            }
    }
}

static void prof_clear()
{
    for (auto &r : g_prof) {
        if (r.start) g_event_pool.push_back(r.start);
        if (r.stop) g_event_pool.push_back(r.stop);
    }
    g_prof.clear();
}

}  // namespace rd

extern "C" {

int reduce_prof_enable(int on)
{
    std::lock_guard<std::mutex> lk(rd::g_prof_mu);
    rd::prof_clear();
    rd::g_prof_on = on != 0;
    return REDUCE_OK;
}

int reduce_prof_query(const char *kernel, double *total_ms, int64_t *launches)
{
    using namespace rd;
    if (!kernel || !total_ms || !launches) return fail(REDUCE_ERR_NULL, "reduce_prof_query: NULL argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double t = 0.0;
    int64_t n = 0;
    for (auto &r : g_prof) {
        if (r.name != kernel || !r.start || !r.stop) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return fail(REDUCE_ERR_HIP, "reduce_prof_query: event");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            return fail(REDUCE_ERR_HIP, "reduce_prof_query: elapsed time");
        t += ms;
        ++n;
    }
    *total_ms = t;
    *launches = n;
    return REDUCE_OK;
}

int reduce_version(void) { return 1; }

const char *reduce_status_str(int status)
{
    switch (status) {
    case REDUCE_OK: return "ok";
    case REDUCE_ERR_NULL: return "null argument";
    case REDUCE_ERR_SHAPE: return "bad shape";
    case REDUCE_ERR_RANGE: return "parameter out of range";
    case REDUCE_ERR_WORKSPACE: return "workspace too small";
    case REDUCE_ERR_HIP: return "HIP runtime error";
    case REDUCE_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *reduce_last_error(void) { return rd::g_last_error.c_str(); }

int reduce_valid_rect(const float *offs, int32_t N, int32_t W, int32_t H, int32_t *rect)
{
    using namespace rd;
    if (!offs || !rect) return fail(REDUCE_ERR_NULL, "reduce_valid_rect: NULL argument");
    if (W < 1 || H < 1 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_valid_rect: W, H, N must be >= 1");
    int64_t xl = INT64_MIN, xh = INT64_MAX, yl = INT64_MIN, yh = INT64_MAX;
    for (int32_t k = 0; k < N; ++k) {
        const double sx = offs[2 * k], sy = offs[2 * k + 1];
        if (!std::isfinite(sx) || !std::isfinite(sy) || std::fabs(sx) > 1e9 || std::fabs(sy) > 1e9)
            return fail(REDUCE_ERR_RANGE, "reduce_valid_rect: offset not finite");
        const int64_t a = (int64_t)std::ceil(-sx), b = (int64_t)std::floor((double)(W - 1) - sx);
        const int64_t c = (int64_t)std::ceil(-sy), d = (int64_t)std::floor((double)(H - 1) - sy);
        xl = a > xl ? a : xl;
        xh = b < xh ? b : xh;
        yl = c > yl ? c : yl;
        yh = d < yh ? d : yh;
    }
    if (xl > xh || yl > yh) return fail(REDUCE_ERR_RANGE, "reduce_valid_rect: the frames do not overlap");
    rect[0] = (int32_t)xl;
    rect[1] = (int32_t)yl;
    rect[2] = (int32_t)(xh - xl + 1);
    rect[3] = (int32_t)(yh - yl + 1);
    return REDUCE_OK;
}

}  // extern "C"
