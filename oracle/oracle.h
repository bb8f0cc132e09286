/*
 * FP64 CPU oracle for the CCD reduction hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct double-precision reference for every step of the
 * path: dark subtraction and flat division (Section 2.1/2.2), translation
 * registration against a reference frame, bilinear sub-pixel shifting onto the
 * common overlap (Section 2.2, and the cheaper-interpolation remark of Section
 * 3.2.1), sigma-clipped mean co-adding (Sections 2.1, 3.1.2), 4x4 box downsampling
 * and the small offset-proposal CNN.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library; the product path never
 * does.  It shares no code, header or constant with the HIP library.
 *
 * Every array is row-major with x contiguous; all pointers are host pointers.
 * Return value: 0 on success, 1 null argument, 2 bad shape, 3 bad range,
 * 6 unsupported.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_EDGE_X   1
#define ORACLE_EDGE_Y   2
#define ORACLE_NEAR_TIE 4
#define ORACLE_CLIPPED  16

typedef struct {
    int32_t dx, dy;          /* integer argmax of the score */
    float sx, sy;            /* sub-pixel offset, rounded to float */
    double peak, second;     /* best score, best score among the other candidates */
    double margin;           /* (peak - second) / |peak| */
    int32_t flags;
    int32_t pad;
} oracle_offset_t;

int oracle_num_threads(void);
void oracle_set_num_threads(int n);

/* out[k][y][x] = ((raw[k][y][x] - bias[y][x]) - dark[y][x]) / flat[y][x] in double
 * (bias may be NULL: no bias term).  raw has row pitch raw_row_pitch and frame pitch
 * raw_frame_pitch (elements); bias, dark and flat have row pitch cal_row_pitch; out is
 * dense [N][H][W]. */
int oracle_calibrate(const uint16_t *raw, int64_t raw_row_pitch, int64_t raw_frame_pitch,
                     const double *bias, const double *dark, const double *flat, int64_t cal_row_pitch,
                     double *out, int32_t W, int32_t H, int32_t N);

/* Register every frame against ref over the window [c-R, c+R]^2 clipped to
 * [-Rmax, Rmax]^2 (c = centers[k] or 0).  tmpl = {x0, y0, w, h} or NULL for the
 * interior shrunk by Rmax.  scores, if not NULL, receives [N][2R+1][2R+1] with
 * the window's (dy, dx) at index (dy-cy+R, dx-cx+R) and -inf outside the clip. */
int oracle_register(const double *ref, const double *frames, int32_t W, int32_t H, int32_t N,
                    int32_t R, int32_t Rmax, const int32_t *centers, const int32_t *tmpl,
                    oracle_offset_t *out, double *scores);

/* Common overlap of all frames: x in [max_k ceil(-s_kx), min_k floor(W-1-s_kx)], same
 * for y.  rect = {x0, y0, w, h}.  Returns 3 if the overlap is empty. */
int oracle_valid_rect(const float *offs, int32_t N, int32_t W, int32_t H, int32_t *rect);

/* Bilinear resample: out[k][v][u] = f_k(x0+u+sx_k, y0+v+sy_k) over rect.  mask (may
 * be NULL) is a bad-pixel map [H][W] shared by the frames: an output one of whose taps
 * is a bad pixel is NaN (missing). */
int oracle_shift(const double *in, double *out, int32_t W, int32_t H, int32_t N,
                 const float *offs, const int32_t *rect, const uint8_t *mask);

/* Sigma-clipped mean along the frame axis.  keep and near may be NULL: near marks
 * values whose distance from the mean lay within rel_band * k*sigma of the
 * threshold at some iteration in which they were tested.  With missing != 0 NaN
 * values are missing: never kept, not counted as rejected, and n is the number of
 * the pixel's other values (a pixel without any gives NaN). */
int oracle_combine(const double *aligned, int32_t w, int32_t h, int32_t N, double ksigma,
                   int32_t max_iters, double *out, uint8_t *keep, int64_t *n_rej,
                   uint8_t *near, double rel_band, int32_t missing);

/* 4x4 block mean: out[j][i] = mean of in[4j..4j+3][4i..4i+3]. */
int oracle_downsample4(const double *in, int32_t W, int32_t H, double *out);

/* Network input of one frame: 4x4 block mean, then asinh((x - mean) / std) with the
 * mean and population standard deviation of the block-mean image, rounded to
 * bfloat16 (via float, ties to even).  out is [H/4][W/4]. */
int oracle_cnn_input(const double *in, int32_t W, int32_t H, double *out);

/* ---- offset-proposal network (oracle_cnn.c) ---- */
int oracle_bf16_round(const double *in, double *out, int64_t n);
int oracle_conv3x3s2_forward(const double *x, int32_t B, int32_t Cin, int32_t H, int32_t W, const double *w,
                             const double *bias, int32_t Cout, int32_t relu, double *y);
int oracle_conv3x3s2_backward(const double *x, int32_t B, int32_t Cin, int32_t H, int32_t W, const double *w,
                              int32_t Cout, const double *y, int32_t relu, const double *dz, double *dx,
                              double *dw, double *db);
int64_t oracle_cnn_num_params(void);
int64_t oracle_cnn_act_size(int32_t B, int32_t H, int32_t W);
int oracle_cnn_forward(const double *x, int32_t B, int32_t H, int32_t W, const double *params, int32_t bf16,
                       double *pred, double *acts);
int oracle_cnn_loss_backward(const double *x, int32_t B, int32_t H, int32_t W, const double *params,
                             int32_t bf16, const double *target, double huber_delta, double *loss,
                             double *grad);
/* One AdamW step in place on p, m, v [n] (decoupled weight decay, bias-corrected moments). */
int oracle_adamw(double *p, double *m, double *v, const double *g, int64_t n, double lr, double beta1,
                 double beta2, double eps, double wd, int32_t step);

#ifdef __cplusplus
}
#endif
#endif
