// Launch-plan selection for the correlation search and the combine kernel, and the
// cache of shapes chosen by the autotuner.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.h"
#include "register_plan.h"

namespace rd {

static const int32_t kRegK[] = {5, 9, 12, 17, 18, 22};
constexpr size_t kLdsLimit = 63 * 1024;  // leaves room for the batch kernel's static LDS
constexpr int32_t kMaxThreads = 512;

static int32_t env_int(const char *name)
{
    const char *v = std::getenv(name);
    return v ? std::atoi(v) : 0;
}

// ---- tuned-shape cache ------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::tuple<int32_t, int32_t, int32_t, int32_t>, std::pair<RegShape, double>> g_reg_tuned;
static std::map<int32_t, std::pair<int, double>> g_comb_tuned;

bool tuned_reg_shape(int32_t W, int32_t H, int32_t R, int32_t Rmax, RegShape *sh)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_reg_tuned.find(std::make_tuple(W, H, R, Rmax));
    if (it == g_reg_tuned.end()) return false;
    *sh = it->second.first;
    return true;
}

void set_tuned_reg_shape(int32_t W, int32_t H, int32_t R, int32_t Rmax, const RegShape &sh, double ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_reg_tuned[std::make_tuple(W, H, R, Rmax)] = {sh, ms};
}

int tuned_combine_lanes(int32_t N)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_comb_tuned.find(N);
    return it == g_comb_tuned.end() ? 0 : it->second.first;
}

void set_tuned_combine_lanes(int32_t N, int lanes, double ms)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_comb_tuned[N] = {lanes, ms};
}

// ---- plan construction ----------------------------------------------------------------
static int32_t group_span(int32_t C, int32_t CW, int32_t G, int32_t NBX)
{
    int32_t JS = 1;
    for (int32_t g = 0; g < G; ++g) {
        const int32_t c0 = g * CW, c1 = std::min(c0 + CW, C) - 1;
        if (c0 > c1) break;
        JS = std::max(JS, c1 / NBX - c0 / NBX + 1);
    }
    return JS;
}

bool reg_plan_from_shape(int32_t W, int32_t H, int32_t R, int32_t Rmax, const RegShape &sh, RegPlan *out)
{
    RegPlan p{};
    p.D = 2 * R + 1;
    p.K = sh.K;
    if (std::find(std::begin(kRegK), std::end(kRegK), p.K) == std::end(kRegK)) return false;
    p.NBX = (int32_t)ceil_div(p.D, p.K);
    p.C = p.D * p.NBX;
    p.TX = p.K * (int32_t)ceil_div(64, p.K);
    p.NXB = p.TX / p.K;
    p.G = sh.G;
    if (p.G < 1) return false;
    p.CW = (int32_t)ceil_div(p.C, p.G);
    if (p.CW > kMaxThreads || (int64_t)(p.G - 1) * p.CW >= p.C) return false;
    p.S = sh.S;
    if (p.S < 1 || (int64_t)p.CW * p.S > kMaxThreads) return false;
    p.threads = (int32_t)ceil_div((int64_t)p.CW * p.S, 64) * 64;
    p.JS = group_span(p.C, p.CW, p.G, p.NBX);
    p.FC = p.TX + p.NBX * p.K - 1;
    if ((p.FC & 1) == 0) p.FC += 1;
    p.TY = sh.TY;
    if (p.TY < 1 || p.TY > 256) return false;
    p.FR = p.TY + p.JS - 1;
    const size_t stage = sizeof(double) * (size_t)p.TY * p.TX + sizeof(float) * (size_t)p.FR * p.FC;
    const size_t red = p.S > 1 ? sizeof(double) * (size_t)p.CW * p.K : 0;
    p.lds = std::max(stage, red);
    if (p.lds > kLdsLimit) return false;

    // tile rows: CPT chunks, at most the template height; independent of the frame
    // count so that every path with the same shape sums partials in the same order
    const int32_t tw = W - 2 * Rmax, th = H - 2 * Rmax;
    if (tw < 1 || th < 1) return false;
    if (sh.CPT < 1) return false;
    p.th_max = th;
    p.n_xchunks = (int32_t)ceil_div(tw, p.TX);
    p.BR = (int32_t)std::min<int64_t>((int64_t)sh.CPT * p.TY, ceil_div(th, p.TY) * p.TY);
    p.n_bands = (int32_t)ceil_div(th, p.BR);
    p.n_tiles = p.n_bands * p.n_xchunks;
    p.wg_per_frame = p.n_tiles * p.G;
    *out = p;
    return true;
}

bool reg_plan_small(int32_t W, int32_t H, int32_t R, int32_t Rmax, RegPlan *out)
{
    constexpr int32_t COLS = 256, CH = 15, ROWS = 240;  // the device constants SMALL_COLS, SMALL_CH, SMALL_ROWS
    RegPlan p{};
    p.D = 2 * R + 1;
    if (p.D > 5) return false;
    const int32_t tw = W - 2 * Rmax, th = H - 2 * Rmax;
    if (tw < 1 || th < 1) return false;
    p.K = 0;
    p.NBX = 1;
    p.C = p.D;
    p.G = 1;
    p.CW = p.D;
    p.S = 1;
    p.threads = COLS;
    p.TX = COLS;
    p.NXB = 1;
    p.TY = CH;  // rows per staged chunk
    // tile rows: the most (shorter tiles were measured slower, single-frame calls included)
    p.n_xchunks = (int32_t)ceil_div(tw, COLS);
    p.BR = ROWS;
    const int32_t forced = env_int("REDUCE_SMALL_ROWS");  // for measurement: a multiple of 15, at most 240
    if (forced >= CH && forced <= ROWS && forced % CH == 0) p.BR = forced;
    p.JS = p.D;
    p.FR = CH;
    p.FC = COLS + 4;
    p.lds = 2 * CH * (COLS + 4) * sizeof(float);  // static in the kernel
    p.th_max = th;
    p.n_bands = (int32_t)ceil_div(th, p.BR);
    p.n_tiles = p.n_bands * p.n_xchunks;
    p.wg_per_frame = p.n_tiles;
    *out = p;
    return true;
}

// Useful FMAs per issued VALU instruction (higher is better): each (row, column
// block) pair costs K*K FMAs plus its LDS loads and converts, each staged element
// about a dozen instructions, and every candidate group restages the tiles.
static double shape_score(const RegPlan &p)
{
    const int32_t waves = p.threads / 64;
    const double valid = (double)p.D / (double)(p.NBX * p.K);
    const int64_t pairs = (int64_t)p.TY * p.NXB;
    const double per_wave = (double)ceil_div(pairs, p.S) * (p.K * p.K + 3 * p.K + 24) +
                            (double)ceil_div((int64_t)p.TY * p.TX, 64) * 10.0 / waves +
                            (double)ceil_div((int64_t)p.FR * p.FC, 64) * 8.0 / waves;
    const double useful = (double)p.C / p.G * p.K * valid * p.TY * p.TX / 64.0;
    return useful / (per_wave * waves);
}

// Chunks per tile aiming at about 2048 tiles x groups per frame.
static int32_t model_cpt(int32_t W, int32_t H, int32_t Rmax, int32_t TX, int32_t G, int32_t TY)
{
    const int64_t tw = W - 2 * Rmax, th = H - 2 * Rmax;
    const int64_t per_band = ceil_div(tw, TX) * G;
    const int64_t bands = std::max<int64_t>(1, std::min<int64_t>(ceil_div(2048, per_band), ceil_div(th, TY)));
    return (int32_t)std::max<int64_t>(1, ceil_div(ceil_div(th, bands), TY));
}

static void all_shapes(int32_t W, int32_t H, int32_t R, int32_t Rmax, int32_t K_only, int32_t TY_only,
                       std::vector<std::pair<double, RegShape>> *out)
{
    const int32_t D = 2 * R + 1;
    for (int32_t K : kRegK) {
        if (K_only && K != K_only) continue;
        const int32_t C = D * (int32_t)ceil_div(D, K);
        for (int32_t G = 1; G <= 64; ++G) {
            const int32_t CW = (int32_t)ceil_div(C, G);
            if (CW > kMaxThreads) continue;
            if ((int64_t)(G - 1) * CW >= C) break;
            for (int32_t S = 1; S <= std::min<int32_t>(16, kMaxThreads / CW); ++S)
                for (int32_t TY = 4; TY <= 64; ++TY) {
                    if (TY_only && TY != TY_only) continue;
                    RegPlan p;
                    const int32_t TX = K * (int32_t)ceil_div(64, K);
                    const RegShape sh{K, G, S, TY, model_cpt(W, H, Rmax, TX, G, TY)};
                    if (!reg_plan_from_shape(W, H, R, Rmax, sh, &p)) {
                        if (TY_only) continue;
                        break;  // larger TY only needs more LDS
                    }
                    out->push_back({shape_score(p), sh});
                }
        }
    }
}

RegPlan reg_plan(int32_t W, int32_t H, int32_t R, int32_t Rmax, int32_t K_force, int32_t TY_force)
{
    if (!K_force) K_force = env_int("REDUCE_REG_K");
    if (!TY_force) TY_force = env_int("REDUCE_REG_TY");
    RegPlan p{};
    RegShape sh{};
    if (!K_force && !TY_force && env_int("REDUCE_REG_GENERAL") != 1 && reg_plan_small(W, H, R, Rmax, &p)) return p;
    if (!K_force && !TY_force && tuned_reg_shape(W, H, R, Rmax, &sh) && reg_plan_from_shape(W, H, R, Rmax, sh, &p))
        return p;
    // the model's choice depends only on the arguments: searched once per key (the
    // search scores every candidate shape, milliseconds of host time)
    static std::mutex mu;
    static std::map<std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t>, RegPlan> chosen;
    const auto key = std::make_tuple(W, H, R, Rmax, K_force, TY_force);
    {
        std::lock_guard<std::mutex> lk(mu);
        const auto it = chosen.find(key);
        if (it != chosen.end()) return it->second;
    }
    std::vector<std::pair<double, RegShape>> shapes;
    all_shapes(W, H, R, Rmax, K_force, TY_force, &shapes);
    if (shapes.empty()) all_shapes(W, H, R, Rmax, 0, 0, &shapes);
    double best = -1.0;
    for (const auto &c : shapes)
        if (c.first > best * 1.005) {
            best = c.first;
            sh = c.second;
        }
    if (best < 0.0 || !reg_plan_from_shape(W, H, R, Rmax, sh, &p)) {
        // a window too large for any shape: leave D = 0 so the caller reports it
        p = RegPlan{};
    }
    std::lock_guard<std::mutex> lk(mu);
    chosen[key] = p;
    return p;
}

void reg_shape_candidates(int32_t W, int32_t H, int32_t R, int32_t Rmax, RegShape *out, int *count, int max_count)
{
    std::vector<std::pair<double, RegShape>> shapes;
    all_shapes(W, H, R, Rmax, 0, 0, &shapes);
    std::stable_sort(shapes.begin(), shapes.end(),
                     [](const std::pair<double, RegShape> &a, const std::pair<double, RegShape> &b) {
                         return a.first > b.first;
                     });
    // the best few per K with distinct (G, S)
    int n = 0;
    for (int32_t K : kRegK) {
        int taken = 0;
        std::vector<std::pair<int32_t, int32_t>> seen;
        for (const auto &c : shapes) {
            if (c.second.K != K || n >= max_count) continue;
            const auto gs = std::make_pair(c.second.G, c.second.S);
            if (std::find(seen.begin(), seen.end(), gs) != seen.end()) continue;
            seen.push_back(gs);
            out[n++] = c.second;
            if (++taken == 4) break;
        }
    }
    // smaller-LDS shapes per K, so that more workgroups share a compute unit (the model
    // counts instructions, not occupancy; the measurement decides)
    for (int32_t K : kRegK)
        for (size_t cap : {(size_t)52 * 1024, (size_t)39 * 1024, (size_t)30 * 1024}) {
            if (n >= max_count) break;
            for (const auto &c : shapes) {
                if (c.second.K != K) continue;
                RegPlan p;
                if (!reg_plan_from_shape(W, H, R, Rmax, c.second, &p) || p.lds > cap) continue;
                bool dup = false;
                for (int i = 0; i < n; ++i)
                    dup = dup || (out[i].K == c.second.K && out[i].G == c.second.G && out[i].S == c.second.S &&
                                  out[i].TY == c.second.TY && out[i].CPT == c.second.CPT);
                if (!dup) out[n++] = c.second;
                break;
            }
        }
    // tile-height variants of the model's overall best shape
    if (!shapes.empty()) {
        const RegShape b = shapes.front().second;
        for (int32_t m : {2, 4}) {
            if (n >= max_count) break;
            RegShape v = b;
            v.CPT = b.CPT * m;
            RegPlan p;
            if (reg_plan_from_shape(W, H, R, Rmax, v, &p) && p.BR > b.CPT * b.TY && p.BR <= kTileRowsMax)
                out[n++] = v;
        }
        if (b.CPT > 1 && n < max_count) {
            RegShape v = b;
            v.CPT = std::max(1, b.CPT / 2);
            out[n++] = v;
        }
    }
    *count = n;
}

int combine_lanes_for(int32_t N)
{
    const int32_t forced = env_int("REDUCE_COMBINE_LANES");
    if (forced == 1 || forced == 2 || forced == 4 || forced == 8 || forced == 16 || forced == 32 || forced == 64)
        return forced;
    const int tuned = tuned_combine_lanes(N);
    return tuned ? tuned : 1;
}

// ---- persistence ------------------------------------------------------------------------
int tune_save(const char *path, const char *arch)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(REDUCE_ERR_RANGE, std::string("reduce_tune_save: cannot write ") + path);
    for (const auto &e : g_reg_tuned) {
        const auto &k = e.first;
        const RegShape &s = e.second.first;
        std::fprintf(f,
                     "{\"arch\": \"%s\", \"op\": \"register\", \"W\": %d, \"H\": %d, \"R\": %d, \"Rmax\": %d, "
                     "\"K\": %d, \"G\": %d, \"S\": %d, \"TY\": %d, \"CPT\": %d, \"ms\": %.6f}\n",
                     arch, std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), s.K, s.G, s.S, s.TY, s.CPT,
                     e.second.second);
    }
    for (const auto &e : g_comb_tuned)
        std::fprintf(f, "{\"arch\": \"%s\", \"op\": \"combine\", \"N\": %d, \"lanes\": %d, \"ms\": %.6f}\n", arch,
                     e.first, e.second.first, e.second.second);
    std::fclose(f);
    return REDUCE_OK;
}

static bool json_int(const char *line, const char *key, int32_t *v)
{
    char pat[64];
    std::snprintf(pat, sizeof(pat), "\"%s\": ", key);
    const char *p = std::strstr(line, pat);
    if (!p) return false;
    return std::sscanf(p + std::strlen(pat), "%d", v) == 1;
}

static bool json_num(const char *line, const char *key, double *v)
{
    char pat[64];
    std::snprintf(pat, sizeof(pat), "\"%s\": ", key);
    const char *p = std::strstr(line, pat);
    if (!p) return false;
    return std::sscanf(p + std::strlen(pat), "%lf", v) == 1;
}

int tune_load(const char *path, const char *arch)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(REDUCE_ERR_RANGE, std::string("reduce_tune_load: cannot read ") + path);
    char line[512];
    char want[96];
    std::snprintf(want, sizeof(want), "\"arch\": \"%s\"", arch);
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strstr(line, want)) continue;  // entries of other devices are ignored
        double ms = 0.0;
        json_num(line, "ms", &ms);
        if (std::strstr(line, "\"op\": \"register\"")) {
            int32_t W, H, R, Rmax;
            RegShape s;
            if (json_int(line, "W", &W) && json_int(line, "H", &H) && json_int(line, "R", &R) &&
                json_int(line, "Rmax", &Rmax) && json_int(line, "K", &s.K) && json_int(line, "G", &s.G) &&
                json_int(line, "S", &s.S) && json_int(line, "TY", &s.TY) && json_int(line, "CPT", &s.CPT)) {
                RegPlan p;
                if (reg_plan_from_shape(W, H, R, Rmax, s, &p)) set_tuned_reg_shape(W, H, R, Rmax, s, ms);
            }
        } else if (std::strstr(line, "\"op\": \"combine\"")) {
            int32_t N, lanes;
            if (json_int(line, "N", &N) && json_int(line, "lanes", &lanes) &&
                (lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16 || lanes == 32 || lanes == 64))
                set_tuned_combine_lanes(N, lanes, ms);
        }
    }
    std::fclose(f);
    return REDUCE_OK;
}

void tune_clear()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_reg_tuned.clear();
    g_comb_tuned.clear();
}

}  // namespace rd

extern "C" int reduce_register_plan(int32_t W, int32_t H, int32_t N, int32_t radius, int32_t radius_max,
                                    int32_t *fields)
{
    using namespace rd;
    if (!fields) return fail(REDUCE_ERR_NULL, "reduce_register_plan: NULL argument");
    if (W < 1 || H < 1 || N < 1 || radius < 0 || radius_max < 0 || W - 2 * radius_max < 1 ||
        H - 2 * radius_max < 1)
        return fail(REDUCE_ERR_RANGE, "reduce_register_plan: no template for these sizes");
    const RegPlan p = reg_plan(W, H, radius, radius_max);
    (void)N;
    if (p.D == 0) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_register_plan: window too large");
    const int32_t v[16] = {p.D, p.K, p.NBX, p.C, p.G, p.CW, p.S, p.threads, p.TX, p.TY, p.BR, p.JS, p.FR, p.FC,
                           (int32_t)p.lds, p.n_tiles};
    for (int i = 0; i < 16; ++i) fields[i] = v[i];
    return REDUCE_OK;
}
