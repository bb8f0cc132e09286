/*
 * FP64 CPU oracle of the offset-proposal network -- TEST INFRASTRUCTURE ONLY.
 *
 * Network: four 3x3 convolutions with stride 2 and zero padding 1 (2 -> 32 -> 32 -> 32
 * -> 32 channels), each followed by ReLU; the mean over all pixels of the last
 * activation; a linear layer 32 -> 2 that gives (dx, dy) in downsampled pixels.
 * Loss: Huber with threshold delta on pred - target, averaged over the batch and the
 * two components.
 *
 * Layout: activations [B][H][W][C] (channels contiguous); conv weights
 * W[t][cin][cout] with t = 3 ky + kx; conv bias [cout]; head Wl[2][32], bl[2].
 * The flat parameter vector is W1 b1 W2 b2 W3 b3 W4 b4 Wl bl (28418 values).
 *
 *   Z[b][oy][ox][co] = bias[co] + sum_{ky,kx,ci} X[b][2oy+ky-1][2ox+kx-1][ci] W[3ky+kx][ci][co]
 *
 * Everything is double.  With bf16 != 0 the values the device stores in bfloat16
 * are rounded the same way here (to float, then to bfloat16 with ties to even): the
 * conv weights, every activation after ReLU, and every gradient with respect to a
 * conv pre-activation.  With bf16 == 0 nothing is rounded (for finite-difference
 * and library cross-checks).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { O_OK = 0, O_NULL = 1, O_SHAPE = 2, O_RANGE = 3 };

#define NCH 32
static const int32_t CIN[4] = {2, NCH, NCH, NCH};

int64_t oracle_cnn_num_params(void)
{
    int64_t n = 0;
    for (int l = 0; l < 4; ++l) n += 9 * CIN[l] * NCH + NCH;
    return n + 2 * NCH + 2;
}

static double bf16r(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan unchanged */
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

int oracle_bf16_round(const double *in, double *out, int64_t n)
{
    if (!in || !out) return O_NULL;
    for (int64_t i = 0; i < n; ++i) out[i] = bf16r(in[i]);
    return O_OK;
}

/* ---- one convolution ---------------------------------------------------------------- */
int oracle_conv3x3s2_forward(const double *x, int32_t B, int32_t Cin, int32_t H, int32_t W, const double *w,
                             const double *bias, int32_t Cout, int32_t relu, double *y)
{
    if (!x || !w || !bias || !y) return O_NULL;
    if (B < 1 || Cin < 1 || Cout < 1 || H < 1 || W < 1) return O_SHAPE;
    const int32_t Ho = (H + 1) / 2, Wo = (W + 1) / 2;
#pragma omp parallel for collapse(2) schedule(static)
    for (int32_t b = 0; b < B; ++b)
        for (int32_t oy = 0; oy < Ho; ++oy)
            for (int32_t ox = 0; ox < Wo; ++ox)
                for (int32_t co = 0; co < Cout; ++co) {
                    double acc = bias[co];
                    for (int32_t ky = 0; ky < 3; ++ky)
                        for (int32_t kx = 0; kx < 3; ++kx) {
                            const int32_t iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
                            if (iy < 0 || iy >= H || ix < 0 || ix >= W) continue;
                            const double *xp = x + (((int64_t)b * H + iy) * W + ix) * Cin;
                            const double *wp = w + ((int64_t)(3 * ky + kx) * Cin) * Cout + co;
                            for (int32_t ci = 0; ci < Cin; ++ci) acc += xp[ci] * wp[(int64_t)ci * Cout];
                        }
                    if (relu && acc < 0.0) acc = 0.0;
                    y[(((int64_t)b * Ho + oy) * Wo + ox) * Cout + co] = acc;
                }
    return O_OK;
}

/* Gradients of one convolution given dz (gradient w.r.t. its pre-activation): dw, db,
 * and dx (gradient w.r.t. its input) if dx is not NULL.  y is unused (kept for the
 * interface); the caller applies the ReLU mask to dz. */
int oracle_conv3x3s2_backward(const double *x, int32_t B, int32_t Cin, int32_t H, int32_t W, const double *w,
                              int32_t Cout, const double *y, int32_t relu, const double *dz, double *dx, double *dw,
                              double *db)
{
    (void)y;
    (void)relu;
    if (!x || !w || !dz || !dw || !db) return O_NULL;
    if (B < 1 || Cin < 1 || Cout < 1 || H < 1 || W < 1) return O_SHAPE;
    const int32_t Ho = (H + 1) / 2, Wo = (W + 1) / 2;
    /* weight and bias gradients: one output element per thread, pixels in order */
#pragma omp parallel for collapse(2) schedule(static)
    for (int32_t t = 0; t < 9; ++t)
        for (int32_t ci = 0; ci < Cin; ++ci)
            for (int32_t co = 0; co < Cout; ++co) {
                const int32_t ky = t / 3, kx = t % 3;
                double acc = 0.0;
                for (int32_t b = 0; b < B; ++b)
                    for (int32_t oy = 0; oy < Ho; ++oy)
                        for (int32_t ox = 0; ox < Wo; ++ox) {
                            const int32_t iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
                            if (iy < 0 || iy >= H || ix < 0 || ix >= W) continue;
                            acc += x[(((int64_t)b * H + iy) * W + ix) * Cin + ci] *
                                   dz[(((int64_t)b * Ho + oy) * Wo + ox) * Cout + co];
                        }
                dw[((int64_t)t * Cin + ci) * Cout + co] = acc;
            }
    for (int32_t co = 0; co < Cout; ++co) {
        double acc = 0.0;
        for (int64_t p = 0; p < (int64_t)B * Ho * Wo; ++p) acc += dz[p * Cout + co];
        db[co] = acc;
    }
    if (dx) {
        /* input gradient: every output pixel whose 3x3 window covers the input pixel */
#pragma omp parallel for collapse(2) schedule(static)
        for (int32_t b = 0; b < B; ++b)
            for (int32_t iy = 0; iy < H; ++iy)
                for (int32_t ix = 0; ix < W; ++ix)
                    for (int32_t ci = 0; ci < Cin; ++ci) {
                        double acc = 0.0;
                        for (int32_t ky = 0; ky < 3; ++ky)
                            for (int32_t kx = 0; kx < 3; ++kx) {
                                const int32_t ny = iy + 1 - ky, nx = ix + 1 - kx;
                                if (ny < 0 || nx < 0 || (ny & 1) || (nx & 1)) continue;
                                const int32_t oy = ny / 2, ox = nx / 2;
                                if (oy >= Ho || ox >= Wo) continue;
                                const double *dzp = dz + (((int64_t)b * Ho + oy) * Wo + ox) * Cout;
                                const double *wp = w + ((int64_t)(3 * ky + kx) * Cin + ci) * Cout;
                                for (int32_t co = 0; co < Cout; ++co) acc += dzp[co] * wp[co];
                            }
                        dx[(((int64_t)b * H + iy) * W + ix) * Cin + ci] = acc;
                    }
    }
    return O_OK;
}

/* ---- whole network ------------------------------------------------------------------ */
typedef struct {
    const double *w[4], *b[4], *wl, *bl;
} net_t;

static void unpack(const double *params, net_t *n)
{
    const double *p = params;
    for (int l = 0; l < 4; ++l) {
        n->w[l] = p;
        p += 9 * CIN[l] * NCH;
        n->b[l] = p;
        p += NCH;
    }
    n->wl = p;
    p += 2 * NCH;
    n->bl = p;
}

int64_t oracle_cnn_act_size(int32_t B, int32_t H, int32_t W)
{
    int64_t total = 0;
    int32_t h = H, w = W;
    for (int l = 0; l < 4; ++l) {
        h = (h + 1) / 2;
        w = (w + 1) / 2;
        total += (int64_t)B * h * w * NCH;
    }
    return total + (int64_t)B * NCH; /* + pooled features */
}

/* Forward pass.  acts (optional, oracle_cnn_act_size doubles) receives X1..X4 and the
 * pooled features. */
static int forward_impl(const double *x, int32_t B, int32_t H, int32_t W, const double *params, int32_t bf16,
                        double *pred, double **X, int32_t *hs, int32_t *ws, double *pool, double **wr)
{
    net_t n;
    unpack(params, &n);
    int32_t h = H, w = W;
    const double *in = x;
    for (int l = 0; l < 4; ++l) {
        const int64_t nw = 9 * CIN[l] * NCH;
        wr[l] = (double *)malloc(sizeof(double) * nw);
        if (!wr[l]) return O_SHAPE;
        for (int64_t i = 0; i < nw; ++i) wr[l][i] = bf16 ? bf16r(n.w[l][i]) : n.w[l][i];
        const int32_t ho = (h + 1) / 2, wo = (w + 1) / 2;
        X[l] = (double *)malloc(sizeof(double) * (size_t)B * ho * wo * NCH);
        if (!X[l]) return O_SHAPE;
        oracle_conv3x3s2_forward(in, B, CIN[l], h, w, wr[l], n.b[l], NCH, 1, X[l]);
        if (bf16)
            for (int64_t i = 0; i < (int64_t)B * ho * wo * NCH; ++i) X[l][i] = bf16r(X[l][i]);
        h = ho;
        w = wo;
        hs[l] = h;
        ws[l] = w;
        in = X[l];
    }
    const int64_t P = (int64_t)h * w;
    for (int32_t b = 0; b < B; ++b)
        for (int32_t c = 0; c < NCH; ++c) {
            double s = 0.0;
            for (int64_t p = 0; p < P; ++p) s += X[3][((int64_t)b * P + p) * NCH + c];
            pool[b * NCH + c] = s / (double)P;
        }
    for (int32_t b = 0; b < B; ++b)
        for (int32_t j = 0; j < 2; ++j) {
            double s = n.bl[j];
            for (int32_t c = 0; c < NCH; ++c) s += pool[b * NCH + c] * n.wl[j * NCH + c];
            pred[2 * b + j] = s;
        }
    return O_OK;
}

static void free_all(double **X, double **wr)
{
    for (int l = 0; l < 4; ++l) {
        free(X[l]);
        free(wr[l]);
    }
}

int oracle_cnn_forward(const double *x, int32_t B, int32_t H, int32_t W, const double *params, int32_t bf16,
                       double *pred, double *acts)
{
    if (!x || !params || !pred) return O_NULL;
    if (B < 1 || H < 16 || W < 16) return O_SHAPE;
    double *X[4] = {0}, *wr[4] = {0};
    int32_t hs[4], ws[4];
    double *pool = (double *)malloc(sizeof(double) * B * NCH);
    int rc = pool ? forward_impl(x, B, H, W, params, bf16, pred, X, hs, ws, pool, wr) : O_SHAPE;
    if (rc == O_OK && acts) {
        double *a = acts;
        for (int l = 0; l < 4; ++l) {
            const int64_t n = (int64_t)B * hs[l] * ws[l] * NCH;
            memcpy(a, X[l], sizeof(double) * n);
            a += n;
        }
        memcpy(a, pool, sizeof(double) * B * NCH);
    }
    free_all(X, wr);
    free(pool);
    return rc;
}

int oracle_cnn_loss_backward(const double *x, int32_t B, int32_t H, int32_t W, const double *params, int32_t bf16,
                             const double *target, double huber_delta, double *loss, double *grad)
{
    if (!x || !params || !target || !loss || !grad) return O_NULL;
    if (B < 1 || H < 16 || W < 16 || !(huber_delta > 0.0)) return O_SHAPE;
    net_t n;
    unpack(params, &n);
    double *X[4] = {0}, *wr[4] = {0};
    int32_t hs[4], ws[4];
    double *pool = (double *)malloc(sizeof(double) * B * NCH);
    double *pred = (double *)malloc(sizeof(double) * B * 2);
    int rc = (pool && pred) ? forward_impl(x, B, H, W, params, bf16, pred, X, hs, ws, pool, wr) : O_SHAPE;
    if (rc != O_OK) goto done;
    {
        /* loss and its gradient with respect to the prediction */
        double L = 0.0;
        double *dpred = (double *)malloc(sizeof(double) * B * 2);
        for (int32_t i = 0; i < 2 * B; ++i) {
            const double e = pred[i] - target[i];
            const double ae = fabs(e);
            L += ae <= huber_delta ? 0.5 * e * e : huber_delta * (ae - 0.5 * huber_delta);
            const double g = ae <= huber_delta ? e : (e > 0 ? huber_delta : -huber_delta);
            dpred[i] = g / (2.0 * B);
        }
        *loss = L / (2.0 * B);

        /* gradient layout mirrors the parameters */
        double *gw[4], *gb[4], *gwl, *gbl;
        double *p = grad;
        for (int l = 0; l < 4; ++l) {
            gw[l] = p;
            p += 9 * CIN[l] * NCH;
            gb[l] = p;
            p += NCH;
        }
        gwl = p;
        p += 2 * NCH;
        gbl = p;

        /* head */
        double *dpool = (double *)malloc(sizeof(double) * B * NCH);
        for (int32_t j = 0; j < 2; ++j) {
            double sb = 0.0;
            for (int32_t b = 0; b < B; ++b) sb += dpred[2 * b + j];
            gbl[j] = sb;
            for (int32_t c = 0; c < NCH; ++c) {
                double s = 0.0;
                for (int32_t b = 0; b < B; ++b) s += dpred[2 * b + j] * pool[b * NCH + c];
                gwl[j * NCH + c] = s;
            }
        }
        for (int32_t b = 0; b < B; ++b)
            for (int32_t c = 0; c < NCH; ++c)
                dpool[b * NCH + c] = dpred[2 * b] * n.wl[c] + dpred[2 * b + 1] * n.wl[NCH + c];

        /* mean pool and the last ReLU */
        const int64_t P4 = (int64_t)hs[3] * ws[3];
        double *dz = (double *)malloc(sizeof(double) * (size_t)B * P4 * NCH);
        for (int32_t b = 0; b < B; ++b)
            for (int64_t q = 0; q < P4; ++q)
                for (int32_t c = 0; c < NCH; ++c) {
                    const int64_t i = ((int64_t)b * P4 + q) * NCH + c;
                    const double g = X[3][i] > 0.0 ? dpool[b * NCH + c] / (double)P4 : 0.0;
                    dz[i] = bf16 ? bf16r(g) : g;
                }
        /* the convolutions, last to first */
        for (int l = 3; l >= 0; --l) {
            const int32_t hin = l ? hs[l - 1] : H, win = l ? ws[l - 1] : W;
            const double *in = l ? X[l - 1] : x;
            double *dx = l ? (double *)malloc(sizeof(double) * (size_t)B * hin * win * CIN[l]) : NULL;
            oracle_conv3x3s2_backward(in, B, CIN[l], hin, win, wr[l], NCH, NULL, 1, dz, dx, gw[l], gb[l]);
            free(dz);
            dz = NULL;
            if (l) {
                const int64_t m = (int64_t)B * hin * win * CIN[l];
                for (int64_t i = 0; i < m; ++i) {
                    const double g = X[l - 1][i] > 0.0 ? dx[i] : 0.0;
                    dx[i] = bf16 ? bf16r(g) : g;
                }
                dz = dx;
            }
        }
        free(dpool);
        free(dpred);
    }
done:
    free_all(X, wr);
    free(pool);
    free(pred);
    return rc;
}

/* ------------------------------------------------------------------------------
 * One AdamW step (Loshchilov and Hutter, "Decoupled weight decay regularization",
 * ICLR 2019, Adam with decoupled weight decay; moments bias-corrected as in Kingma and
 * Ba, "Adam", ICLR 2015), in FP64:
 *   m <- beta1 m + (1 - beta1) g          first moment
 *   v <- beta2 v + (1 - beta2) g^2        second moment
 *   mhat = m / (1 - beta1^t), vhat = v / (1 - beta2^t)
 *   p <- p - lr (mhat / (sqrt(vhat) + eps) + wd p)
 * The weight decay acts on the parameter itself (not through the gradient), at the
 * parameter's value before the step.  t = step >= 1.
 * ---------------------------------------------------------------------------- */
int oracle_adamw(double *p, double *m, double *v, const double *g, int64_t n, double lr, double beta1,
                 double beta2, double eps, double wd, int32_t step)
{
    if (!p || !m || !v || !g) return O_NULL;
    if (n < 0 || step < 1 || !(eps > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return O_RANGE;
    const double c1 = 1.0 - pow(beta1, (double)step);
    const double c2 = 1.0 - pow(beta2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        const double mhat = m[i] / c1, vhat = v[i] / c2;
        p[i] = p[i] - lr * (mhat / (sqrt(vhat) + eps) + wd * p[i]);
    }
    return O_OK;
}
