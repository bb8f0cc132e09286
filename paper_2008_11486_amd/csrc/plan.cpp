// Launch-plan selection for the correlation search and the combine kernel.
#include <algorithm>
#include <cstdlib>

#include "common.h"
#include "register_plan.h"

namespace rd {

static const int32_t kRegK[] = {5, 9, 12, 17, 18, 22};
constexpr size_t kLdsLimit = 64 * 1024;
constexpr int32_t kMaxThreads = 512;

static int32_t env_int(const char *name)
{
    const char *v = std::getenv(name);
    return v ? std::atoi(v) : 0;
}

static double k_score(int32_t D, int32_t K)
{
    const double fill = (double)D / (double)(ceil_div(D, K) * K);
    const double issue = (double)(K * K) / (double)(K * K + 4 * K);  // FMAs among LDS loads and converts
    return fill * issue;
}

RegPlan reg_plan(int32_t W, int32_t H, int32_t N, int32_t R, int32_t Rmax, int32_t K_force, int32_t TY_force)
{
    RegPlan p{};
    p.D = 2 * R + 1;
    if (!K_force) K_force = env_int("REDUCE_REG_K");
    if (!TY_force) TY_force = env_int("REDUCE_REG_TY");
    int32_t K = 0;
    for (int32_t k : kRegK) {
        if (K_force && k != K_force) continue;
        if (!K || k_score(p.D, k) > k_score(p.D, K) + 1e-12) K = k;
    }
    if (!K) K = 22;
    p.K = K;
    p.NBX = (int32_t)ceil_div(p.D, K);
    p.C = p.D * p.NBX;
    p.TX = K * (int32_t)ceil_div(64, K);
    p.NXB = p.TX / K;

    // candidate groups: maximise the share of launched lanes that do real work
    double best_eff = -1.0;
    for (int32_t G = 1; G <= 256; ++G) {
        const int32_t CW = (int32_t)ceil_div(p.C, G);
        if (CW > kMaxThreads) continue;
        if ((int64_t)(G - 1) * CW >= p.C) break;
        const int32_t S = std::max<int32_t>(1, kMaxThreads / CW);
        const int32_t threads = (int32_t)ceil_div((int64_t)CW * S, 64) * 64;
        const double eff = (double)p.C / (double)(G * CW) * (double)(CW * S) / (double)threads;
        if (eff > best_eff + 0.01) {
            best_eff = eff;
            p.G = G;
            p.CW = CW;
            p.S = S;
            p.threads = threads;
        }
    }
    // window rows spanned by one group
    p.JS = 1;
    for (int32_t g = 0; g < p.G; ++g) {
        const int32_t c0 = g * p.CW, c1 = std::min(c0 + p.CW, p.C) - 1;
        if (c0 > c1) break;
        p.JS = std::max(p.JS, c1 / p.NBX - c0 / p.NBX + 1);
    }
    p.FC = p.TX + p.NBX * K - 1;
    if ((p.FC & 1) == 0) p.FC += 1;

    // rows per LDS chunk: balance the (row, column block) pairs over the sub-ranges
    double best_bal = -1.0;
    for (int32_t TY = 4; TY <= 64; ++TY) {
        if (TY_force && TY != TY_force) continue;
        const int32_t FR = TY + p.JS - 1;
        const size_t stage = sizeof(double) * (size_t)TY * p.TX + sizeof(float) * (size_t)FR * p.FC;
        const size_t red = p.S > 1 ? sizeof(double) * (size_t)p.CW * K : 0;
        const size_t lds = std::max(stage, red);
        if (lds > kLdsLimit) break;
        const int64_t pairs = (int64_t)TY * p.NXB;
        const double bal = (double)pairs / (double)(p.S * ceil_div(pairs, p.S));
        // halo cost of restaging the window rows with every chunk
        const double halo = (double)TY / (double)(TY + p.JS - 1);
        const double score = bal * (0.9 + 0.1 * halo);
        if (score > best_bal + 1e-9) {
            best_bal = score;
            p.TY = TY;
            p.FR = FR;
            p.lds = lds;
        }
    }
    if (!p.TY) {  // forced TY did not fit: smallest legal chunk
        p.TY = 4;
        p.FR = p.TY + p.JS - 1;
        p.lds = std::max(sizeof(double) * (size_t)p.TY * p.TX + sizeof(float) * (size_t)p.FR * p.FC,
                         p.S > 1 ? sizeof(double) * (size_t)p.CW * K : (size_t)0);
    }

    // template rows per tile: enough workgroups to fill the chip a few times over
    const int32_t tw = W - 2 * Rmax, th = H - 2 * Rmax;
    p.th_max = th;
    p.n_xchunks = (int32_t)ceil_div(tw, p.TX);
    const int64_t per_band = (int64_t)p.n_xchunks * p.G * N;
    const int64_t target = 4096;
    int64_t bands = std::max<int64_t>(1, ceil_div(target, per_band));
    bands = std::min<int64_t>(bands, ceil_div(th, p.TY));
    p.BR = (int32_t)(ceil_div(ceil_div(th, bands), p.TY) * p.TY);
    p.n_bands = (int32_t)ceil_div(th, p.BR);
    p.n_tiles = p.n_bands * p.n_xchunks;
    return p;
}

int combine_lanes_for(int32_t N)
{
    const int32_t forced = env_int("REDUCE_COMBINE_LANES");
    if (forced == 1 || forced == 2 || forced == 4 || forced == 8 || forced == 16 || forced == 32 || forced == 64)
        return forced;
    (void)N;
    return 1;
}

}  // namespace rd
