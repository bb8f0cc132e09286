/*
 * libreduce -- CCD frame reduction on MI355X (gfx950): dark subtraction, flat
 * division, translation registration, bilinear shift and sigma-clipped co-adding
 * of a stack of 16-bit frames, as in the reduction pipeline of Niwano et al.
 * (PASJ 2020), Sections 2.1-2.2.
 *
 * Conventions shared by every entry point:
 *
 *  - Ownership: the caller allocates every buffer.  "device" pointers are HIP
 *    device memory, "host" pointers are ordinary host memory.  The library never
 *    allocates or frees memory inside a call; scratch space is a caller-provided
 *    device workspace whose size the matching *_ws() query returns.
 *  - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *    call only enqueues work on that stream and returns; results are ready when
 *    the stream is synchronised.  No call synchronises the device.
 *  - Errors: every call validates its arguments on the host before launching
 *    anything and returns one of the REDUCE_* status codes below; on failure
 *    nothing was enqueued (except REDUCE_ERR_HIP, which reports a failed launch).
 *    reduce_last_error() gives a thread-local description of the last failure.
 *    Faults inside kernels surface at the caller's next synchronisation.
 *  - Layout: images are row-major, x contiguous, row y = 0 first (the paper puts
 *    the origin at the lower-left corner, X horizontal, Y vertical; Section
 *    3.1.1).  Pitches are counted in elements.  W, H, N are int32.
 *  - Offsets: s = (sx, sy) is the offset with frame(x + s) ~ ref(x).
 *  - Preconditions not checked on the device: flat > 0 and finite, dark finite.
 */
#ifndef REDUCE_H
#define REDUCE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
#define REDUCE_OK               0
#define REDUCE_ERR_NULL         1  /* a required pointer is NULL */
#define REDUCE_ERR_SHAPE        2  /* sizes or pitches are inconsistent */
#define REDUCE_ERR_RANGE        3  /* a parameter is outside its valid range */
#define REDUCE_ERR_WORKSPACE    4  /* workspace missing or smaller than *_ws() */
#define REDUCE_ERR_HIP          5  /* the HIP runtime reported an error */
#define REDUCE_ERR_UNSUPPORTED  6  /* valid request the library does not serve */

/* ---- registration result ------------------------------------------------- */
#define REDUCE_EDGE_X    1   /* x argmax on the window border: no sub-pixel step */
#define REDUCE_EDGE_Y    2
#define REDUCE_NEAR_TIE  4   /* margin below REDUCE_NEAR_TIE_MARGIN */
#define REDUCE_FALLBACK  8   /* proposal path fell back to the full search */
#define REDUCE_CLIPPED   16  /* window [c-R, c+R] was clipped at +-radius_max */
#define REDUCE_NEAR_TIE_MARGIN 1e-9

typedef struct {
    int32_t dx, dy;        /* integer argmax of the score S(d) */
    float sx, sy;          /* d + parabola vertex, rounded to float */
    double peak;           /* S(d*) */
    double second;         /* best score among the other candidates (-inf if none) */
    double margin;         /* (peak - second) / |peak| (+inf if no other candidate) */
    int32_t flags;         /* REDUCE_EDGE_X | ... */
    int32_t pad;
} reduce_offset_t;         /* 48 bytes */

const char *reduce_status_str(int status);
const char *reduce_last_error(void);
int reduce_version(void);

/* Kernel timing: reduce_prof_enable(1) clears earlier records and makes every
 * following launch of a named kernel ("calibrate", "score_tiles", "shift",
 * "combine", ...) record a HIP event pair on its own stream; reduce_prof_query
 * waits for the recorded events and returns the summed elapsed milliseconds and the
 * number of launches of one kernel.  Host-side bookkeeping only; 0 disables. */
int reduce_prof_enable(int on);
int reduce_prof_query(const char *kernel, double *total_ms, int64_t *launches);

/* ---- calibrate ------------------------------------------------------------
 * Bias subtraction (where the 16-bit to float cast happens), dark subtraction and
 * flat fielding (Section 2.1; Section 2.2).  For every frame k:
 *   out[k][y][x] = ((float(raw[k][y][x]) - bias[y][x]) - dark[y][x]) / flat[y][x]
 * in IEEE single precision, each step correctly rounded.  bias may be NULL: then
 * out = (float(raw) - dark) / flat, the master dark carrying the bias.
 *   raw    device uint16, frame k row y at raw + k*raw_frame_pitch + y*raw_row_pitch
 *          (a pitch larger than W expresses the overscan cut of Section 2.1 as a
 *          zero-copy region of interest)
 *   bias, dark, flat  device float [H] rows of pitch cal_row_pitch (bias may be NULL)
 *   out    device float, dense [N][H][W]
 * Errors: NULL -> REDUCE_ERR_NULL; W, H, N < 1 or pitches too small -> SHAPE. */
int reduce_calibrate(const uint16_t *raw, int64_t raw_row_pitch, int64_t raw_frame_pitch,
                     const float *bias, const float *dark, const float *flat, int64_t cal_row_pitch,
                     float *out, int32_t W, int32_t H, int32_t N, void *stream);

/* ---- register -------------------------------------------------------------
 * Translation registration by brute-force cross-correlation (the paper takes the
 * relative positions from WCS headers, Section 2.2; this call replaces that step).
 * With the template T = tmpl (or the interior [Rmax, W-Rmax) x [Rmax, H-Rmax)),
 * r' = ref - mean_T(ref) and, for each frame k and every integer d in the window
 * [c_k - R, c_k + R]^2 clipped to [-Rmax, Rmax]^2 (c_k = centers[k] or 0):
 *     S_k(d) = sum_{p in T} r'(p) * frame_k(p + d)        (FP64 accumulation)
 * d* = argmax S_k (equal scores: smaller dy, then smaller dx); per axis the vertex
 * of the parabola through S at d*-1, d*, d*+1 refines d* unless d* is on the window
 * border (then the fraction is 0 and EDGE is set).
 *   ref     device float [H][W];  frames device float [N][H][W]
 *   centers device int32 [N][2] (cx, cy) or NULL
 *   tmpl    host int32 {x0, y0, w, h} or NULL; T dilated by Rmax must lie in the frame
 *   out     device reduce_offset_t [N]
 *   scores  device double [N][2R+1][2R+1] or NULL: S_k at (dy-cy+R, dx-cx+R), -inf
 *           outside the clipped window
 *   ws      device workspace of at least reduce_register_ws(W, H, N, R, Rmax) bytes
 * Errors: R < 0, Rmax < 0 or an invalid template -> RANGE; small ws -> WORKSPACE. */
size_t reduce_register_ws(int32_t W, int32_t H, int32_t N, int32_t radius, int32_t radius_max);

/* Launch plan the search would use for these sizes (host-only, for diagnostics and
 * tuning): fields = {D, K, NBX, C, G, CW, S, threads, TX, TY, BR, JS, FR, FC,
 * lds_bytes, n_tiles}.  Errors: no template for the sizes -> RANGE. */
int reduce_register_plan(int32_t W, int32_t H, int32_t N, int32_t radius, int32_t radius_max,
                         int32_t *fields);
int reduce_register(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                    int32_t radius, int32_t radius_max, const int32_t *centers,
                    const int32_t *tmpl, reduce_offset_t *out, double *scores,
                    void *ws, size_t ws_bytes, void *stream);

/* ---- search through row spectra -----------------------------------------------
 * The full-window search of reduce_register (radius_max = radius, the interior
 * template, no centres) with the scores S(d) of the whole window evaluated from row
 * spectra instead of direct sums, an alternative evaluation for large windows (the
 * paper's sweeps over image size and frame count, Section 3.2.2, motivate searches
 * whose cost must not grow with the window area).  With P >= W a power of two, the
 * rows of the mean-free template and of each frame are transformed (length-P DFT, the
 * half spectrum of real rows), Z_j(k) = sum_y A_{y+j}(k) conj(B_y(k)) is formed for the
 * 2R+1 row lags j, and S at the 2R+1 column lags is the inverse transform there.  The
 * offsets then come from exact direct sums: a +-1 window around the spectral argmax
 * (moved while its maximum lies on an inner border) is kept when its exact peak
 * exceeds every spectral score outside it by more than a bound on the spectral
 * rounding error, 4 eps (10 log2(P/2) + th + P + 50) ||frame rows|| ||template rows||
 * (eps = 2^-53, Frobenius norms), else the frame takes the full direct search.  So
 * dx, dy, sx, sy, peak and the EDGE and NEAR_TIE flags are those of reduce_register up
 * to the summation order of its direct sums; `second` may be a spectral score (within
 * the bound of the exact one).
 *   ref, frames, out as reduce_register (radius_max = radius);
 *   scores  device double [N][2R+1][2R+1] or NULL: the spectral scores (layout of
 *           reduce_register's), before the exact refinement;
 *   info    device int32 [N] or NULL: per frame 0 (kept), or 1 (maximum still on an
 *           inner border) | 2 (not clear of the error bound): the full search ran;
 *   ws      device workspace of reduce_register_fft_ws(W, H, N, radius) bytes.
 * Errors: radius < 1 or no template -> RANGE; W > 8192, N > 65535 or radius > 511 ->
 * UNSUPPORTED; small ws -> WORKSPACE. */
size_t reduce_register_fft_ws(int32_t W, int32_t H, int32_t N, int32_t radius);
int reduce_register_fft(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                        int32_t radius, reduce_offset_t *out, double *scores, int32_t *info, void *ws,
                        size_t ws_bytes, void *stream);

/* ---- search without a workspace ------------------------------------------------
 * For callers that cannot allocate device memory (code under graph capture, tight
 * serving loops, harnesses that forbid allocation): reduce_register with the same
 * arguments and results, but no ws.  The workspace is a fixed array of
 * reduce_register_static_max() bytes (64 MiB) of device memory that the library holds
 * on every GPU it runs on until the process ends; its device address is taken on the
 * first call on each device (with that device current).  The call allocates nothing.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams, or host threads) race and must be serialised by the caller.
 * Errors: as reduce_register; sizes whose workspace, reduce_register_ws(W, H, N, R,
 * Rmax), exceeds reduce_register_static_max() -> UNSUPPORTED (split the frames over
 * several calls); the symbol address cannot be taken -> HIP_ERROR. */
size_t reduce_register_static_max(void);
int reduce_register_static(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                           int32_t radius, int32_t radius_max, const int32_t *centers,
                           const int32_t *tmpl, reduce_offset_t *out, double *scores, void *stream);

/* ---- common overlap -------------------------------------------------------
 * The alignment crops every frame to the area all frames cover (Section 3.1.2,
 * note to the table of co-adding data sets).  Output x must satisfy
 * 0 <= x + s_kx <= W - 1 for every k:  x in [max_k ceil(-s_kx), min_k floor(W-1-s_kx)],
 * likewise y.  Host-only computation.
 *   offs  host float [N][2];  rect  host int32 out {x0, y0, w, h}
 * Errors: non-finite offsets or an empty overlap -> RANGE. */
int reduce_valid_rect(const float *offs, int32_t N, int32_t W, int32_t H, int32_t *rect);

/* ---- shift ----------------------------------------------------------------
 * Sub-pixel alignment by bilinear interpolation (the paper shifts by bicubic
 * splines and names bilinear interpolation as the cheaper alternative, Section
 * 3.2.1).  out[k][v][u] = f_k(x0 + u + sx_k, y0 + v + sy_k) with the integer part
 * floor(s) applied in integer arithmetic and the fraction a = s - floor(s) as
 * bilinear weights (computed in double, rounded once to float).
 *   in    device float [N][H][W];  out  device float dense [N][h][w]
 *   offs  device float [N][2];     rect host int32 {x0, y0, w, h}
 *   integer_mode != 0: exact copy f_k(x + floor(sx), y + floor(sy)).
 * Errors: an empty rect -> SHAPE.  The caller guarantees that rect lies inside the
 * overlap of the offsets (reduce_valid_rect); taps are clamped to the frame. */
int reduce_shift(const float *in, float *out, int32_t W, int32_t H, int32_t N,
                 const float *offs, const int32_t *rect, int32_t integer_mode, void *stream);

/* ---- bad-pixel masking ------------------------------------------------------------
 * Bad-pixel masking (Section 2.1 lists it between flat fielding and alignment; the
 * method is not given): mask [H][W] uint8 is the detector's bad-pixel map shared by
 * the N frames (nonzero = bad).  After reduce_shift with the same offs, rect and
 * integer_mode, every aligned value whose bilinear taps (rows j and j+1 when the y
 * fraction is non-zero, columns i and i+1 when the x fraction is non-zero; the one
 * copied pixel in integer mode) include a bad pixel is set to NaN in out, for the
 * missing-value combine (reduce_combine with missing = 1).
 *   mask  device uint8 [H][W];  out  device float dense [N][h][w] (reduce_shift's output)
 *   offs  device float [N][2];  rect host int32 {x0, y0, w, h}
 * Errors: NULL -> NULL; empty or oversized rect -> SHAPE; N or h above 65535 ->
 * UNSUPPORTED. */
int reduce_mask_shifted(const uint8_t *mask, float *out, int32_t W, int32_t H, int32_t N,
                        const float *offs, const int32_t *rect, int32_t integer_mode, void *stream);

/* ---- bicubic-spline shift ---------------------------------------------------------
 * The paper's own interpolation (Sections 2.1, 2.2; Section 3.2.1 prices its
 * tridiagonal system per image row or column): out[k][v][u] = S_k(x0 + u + sx_k,
 * y0 + v + sy_k), S_k the tensor-product natural cubic spline through frame k's pixels
 * on the integer grid (second derivative zero at both ends of every row and column).
 * Positions are clamped into the frame.  FP32 arithmetic; two passes (rows into the
 * workspace, then columns).
 *   in    device float [N][H][W];  out  device float dense [N][h][w]
 *   offs  device float [N][2];     rect host int32 {x0, y0, w, h}
 *   ws    device workspace of at least reduce_shift_spline_ws(W, H, N) bytes
 *         (the row pass's result, N * H rows of w floats at a pitch of w rounded up
 *         to 64 floats, so that the column pass reads whole 256-byte segments)
 * Errors: an empty or oversized rect -> SHAPE; N or H above 65535 -> UNSUPPORTED;
 * small ws -> WORKSPACE. */
size_t reduce_shift_spline_ws(int32_t W, int32_t H, int32_t N);
int reduce_shift_spline(const float *in, float *out, int32_t W, int32_t H, int32_t N,
                        const float *offs, const int32_t *rect, void *ws, size_t ws_bytes,
                        void *stream);

/* ---- combine --------------------------------------------------------------
 * Co-adding by sigma-clipped mean (Sections 2.1 and 3.1.2).  Per pixel, over the
 * N aligned values: up to max_iters times, take the mean m and population sigma of
 * the kept values (in double) and drop every kept value with |x - m| > ksigma*sigma;
 * stop when an iteration drops nothing; out = mean of the kept values.
 *   aligned  device float [N][h][w];  out device float [h][w]
 *   keep     device uint8 [N][h][w] (1 = kept) or NULL
 *   n_rej    device int64 [1], set to the number of dropped values, or NULL
 * Stacks of up to 48 frames hold a pixel's values in registers (or, with the tuned
 * lanes per column, in an LDS tile); 49 - 128 frames (the paper's co-adding sets
 * reach 97, Section 3.1.2) in the thread's own slice of LDS.
 * missing != 0: NaN values (bad pixels, see reduce_mask_shifted) are missing: never
 * kept (keep 0), not counted in n_rej, and the clip runs over the pixel's other
 * values; a pixel without any gives NaN.  missing == 0: a NaN poisons its pixel.
 * Errors: ksigma <= 0, max_iters < 0 -> RANGE; N > 128 -> UNSUPPORTED. */
int reduce_combine(const float *aligned, int32_t w, int32_t h, int32_t N, float ksigma,
                   int32_t max_iters, float *out, uint8_t *keep, int64_t *n_rej, int32_t missing,
                   void *stream);

/* ---- batched stacks -----------------------------------------------------------
 * The whole chain for many independent stacks (for instance the three bands of the
 * paper's cameras, Section 2.1, or many fields) of uneven frame counts and sizes
 * with one kernel launch per phase (calibrate, template mean, search tiles, tile
 * sums, argmax, overlap, shift + combine), each launch covering the phase's work
 * items of every stack, enqueued on `stream`.  For every stack:
 * calibrate all frames as reduce_calibrate; register every frame k != ref_index
 * against frame ref_index as reduce_register with radius_max = radius and the
 * interior template; the reference frame gets the offset 0 (peak 0, second -inf,
 * margin +inf, flags 0); the common overlap as reduce_valid_rect of the sub-pixel
 * offsets (of the integer offsets in integer_mode); shift as reduce_shift; combine
 * as reduce_combine.  With the same launch shapes (the autotuner's, if any) every
 * output is bit-identical to that stage-wise chain.
 *   out       device float, room for W*H values; the combined image, dense [h][w]
 *   out_rect  device int32[4] {x0, y0, w, h} of the overlap in reference pixels
 *   offsets   device reduce_offset_t [N]
 *   n_rej     device int64[1] (values dropped by the clip) or NULL
 * ws: device workspace of reduce_stack_batch_ws(stacks, n) bytes (calibrated frames,
 * partial scores, the work-item table); query again after tuning.  The stack
 * A stack with a bias frame calibrates as reduce_calibrate with it; a stack with a
 * bad-pixel map masks its aligned values as reduce_mask_shifted and combines with
 * missing = 1.  A stack with search = REDUCE_SEARCH_SPECTRAL (radius >= 1, W <= 8192)
 * registers as reduce_register_fft of its calibrated frames instead of
 * reduce_register (the same offsets; the choice is the caller's or the tuner's).  The stack
 * descriptors are copied into the workspace at every call (the host image is kept
 * per workspace and rebuilt, after synchronising `stream`, when the descriptors
 * change).  Calls sharing one workspace must not overlap.  Errors: as the stage-wise
 * calls, per stack; N > 128 -> UNSUPPORTED. */
typedef struct {
    const uint16_t *raw;
    int64_t raw_row_pitch, raw_frame_pitch;
    const float *dark, *flat;
    int64_t cal_row_pitch;
    int32_t W, H, N, ref_index, radius, max_iters;
    float ksigma;
    int32_t integer_mode;
    float *out;
    int32_t *out_rect;
    reduce_offset_t *offsets;
    int64_t *n_rej;
    const float *bias;      /* [H][W] at cal_row_pitch, or NULL (the dark carries the bias) */
    const uint8_t *mask;    /* bad-pixel map [H][W] (row pitch W, nonzero = bad) or NULL */
    int32_t search;         /* REDUCE_SEARCH_DIRECT (0) or REDUCE_SEARCH_SPECTRAL (1) */
    int32_t pad;
} reduce_stack_t;
#define REDUCE_SEARCH_DIRECT   0  /* scores by direct sums (reduce_register) */
#define REDUCE_SEARCH_SPECTRAL 1  /* scores from row spectra, offsets from exact sums (reduce_register_fft) */

size_t reduce_stack_batch_ws(const reduce_stack_t *stacks, int32_t n);
int reduce_stack_batch(const reduce_stack_t *stacks, int32_t n, void *ws, size_t ws_bytes, void *stream);

/* ---- offset-proposal network --------------------------------------------------
 * A small CNN proposes each frame's offset from 4x-downsampled frames, so that the
 * brute-force search can be narrowed to a +-2 px window around the proposal.
 *
 * reduce_cnn_input: network input of N calibrated frames: the 4x4 block mean (in
 *   double), standardised by the mean and population standard deviation of the
 *   block-mean image, asinh, rounded to bfloat16 (ties to even).  frames: device
 *   float [N][H][W] (W, H multiples of 4); out: device bfloat16 bits [N][H/4][W/4];
 *   ws: reduce_cnn_input_ws(W, H, N) bytes.
 *
 * Network: four 3x3 convolutions with stride 2 and zero padding 1 (2 -> 32 -> 32 ->
 * 32 -> 32 channels) with ReLU, the mean over pixels, a linear layer 32 -> 2 giving
 * (dx, dy) in downsampled pixels.  Input channel 0 is the reference, channel 1 the
 * frame.  params: device float, reduce_cnn_num_params() values in the order W1 b1 W2
 * b2 W3 b3 W4 b4 Wl bl with conv weights W[t][cin][cout], t = 3 ky + kx, Wl[2][32].
 * The convolutions run on bfloat16 matrix cores with FP32 accumulation; weights and
 * activations are stored in bfloat16.
 *
 * reduce_cnn_forward: ref device bfloat16 [h][w] per batch item at ref + b *
 *   ref_stride (ref_stride 0: one reference for all), img device bfloat16 [B][h][w];
 *   pred device float [B][2].  ws (reduce_cnn_ws(B, h, w) bytes) keeps the
 *   activations for reduce_cnn_backward.  reduce_cnn_ws_offsets fills offsets[6]
 *   with byte offsets inside ws: [0..3] the four activations [B][h_l][w_l][32]
 *   (h_l = ceil(h / 2^l)); [4] and [5] two bfloat16 gradient planes that, after
 *   reduce_cnn_backward, hold dLoss/dZ of layer 2 and of layer 1 respectively. */
size_t reduce_cnn_input_ws(int32_t W, int32_t H, int32_t N);
int reduce_cnn_input(const float *frames, int32_t W, int32_t H, int32_t N, uint16_t *out, void *ws,
                     size_t ws_bytes, void *stream);
int64_t reduce_cnn_num_params(void);
size_t reduce_cnn_ws(int32_t B, int32_t h, int32_t w);
int reduce_cnn_ws_offsets(int32_t B, int32_t h, int32_t w, int64_t *offsets);
int reduce_cnn_forward(const uint16_t *ref, int64_t ref_stride, const uint16_t *img, int32_t B, int32_t h,
                       int32_t w, const float *params, float *pred, void *ws, size_t ws_bytes, void *stream);

/* reduce_cnn_backward: loss and gradient of the Huber loss (threshold huber_delta) of
 *   pred - target, averaged over the B x 2 components, with respect to params.  Needs
 *   the activations the immediately preceding reduce_cnn_forward left in ws for the
 *   same inputs and params.  target device float [B][2]; loss device float [1]; grad
 *   device float [reduce_cnn_num_params()].  Gradients with respect to conv
 *   pre-activations are stored in bfloat16; weight gradients accumulate in FP32 and
 *   are summed over fixed pixel chunks in order.  B <= 1024.
 * reduce_cnn_adamw: one AdamW step (decoupled weight decay, bias-corrected moments)
 *   on n FP32 parameters with moments m, v, at 1-based step `step`. */
int reduce_cnn_backward(const uint16_t *ref, int64_t ref_stride, const uint16_t *img, int32_t B, int32_t h,
                        int32_t w, const float *params, const float *pred, const float *target,
                        float huber_delta, float *loss, float *grad, void *ws, size_t ws_bytes, void *stream);
int reduce_cnn_adamw(float *params, float *m, float *v, const float *grad, int64_t n, float lr, float beta1,
                     float beta2, float eps, float weight_decay, int32_t step, void *stream);

/* reduce_cnn_centres: search-window centres from the network's prediction:
 *   centres[b][j] = clamp(rint(scale * pred[b][j]), -radius_max, radius_max) as int32
 *   (device pred float [B][2], device centres int32 [B][2]), for the narrowed search
 *   of reduce_register (scale 4 maps the 4x-downsampled prediction to frame pixels).
 *   A NaN prediction gives -radius_max. */
int reduce_cnn_centres(const float *pred, int32_t B, float scale, int32_t radius_max, int32_t *centres,
                       void *stream);

/* reduce_recentre: for every frame whose narrowed-search maximum lies on a window
 *   border strictly inside +-radius_max (EDGE_X with |dx| < radius_max, or EDGE_Y
 *   with |dy| < radius_max; a border at +-radius_max is also the full search's border),
 *   set centres[k] to that maximum (dx, dy), clamped to +-radius_max; other centres
 *   are left alone.  Repeating
 *   reduce_register + reduce_recentre walks each +-R window towards the peak it
 *   sees rising at its border.  offs device reduce_offset_t [N], centres device
 *   int32 [N][2] (updated in place). */
int reduce_recentre(const reduce_offset_t *offs, int32_t N, int32_t radius_max, int32_t *centres, void *stream);

/* reduce_propose: learned registration of N frames against one reference, entirely on
 *   `stream` (no host round trip).  The network proposes each frame's offset from the
 *   4x-downsampled pair (reduce_cnn_input + reduce_cnn_forward with params; window centre
 *   c_k = clamp(rint(4 * pred_k), +-radius_max) as reduce_cnn_centres); the correlation
 *   search of reduce_register then runs in the window [c_k - refine_radius, c_k +
 *   refine_radius]^2 with the full search's template (the interior shrunk by radius_max),
 *   so its scores S_k(d) are those of the full search.  A frame whose maximum lies on a
 *   window border strictly inside +-radius_max moves its centre onto that maximum and is
 *   searched again (at most max_moves times; only those frames are searched).  The
 *   full-window search (radius radius_max) then replaces the result of every frame whose
 *   maximum is still on such a border or whose peak is below peak_ratio times the
 *   reference's own zero-offset score S_ref(0) = sum_T r' ref; those frames get
 *   REDUCE_FALLBACK in their flags.  The network only moves the window: the score,
 *   argmax and sub-pixel vertex are reduce_register's.
 *   ref     device float [H][W];  frames device float [N][H][W] (W, H multiples of 4, >= 64)
 *   params  device float, the network's reduce_cnn_num_params() values
 *   out     device reduce_offset_t [N]
 *   centres device int32 [N][2] (the network's window centres) or NULL
 *   info    device int32 [N] or NULL: number of window moves | 256 if the fallback was
 *           taken for a border maximum | 512 if it was taken for a weak peak
 *   ws      device workspace of at least reduce_propose_ws(W, H, N, refine_radius,
 *           radius_max) bytes (network input and activations, the narrowed and the
 *           fallback searches' partial scores; the fallback scores as many frames at a
 *           time as fit 256 MiB of partials)
 * Errors: NULL -> NULL; bad sizes -> SHAPE; refine_radius > radius_max, a radius that
 * leaves no template, max_moves outside [0, 64] or a non-finite peak_ratio -> RANGE;
 * small ws -> WORKSPACE. */
size_t reduce_propose_ws(int32_t W, int32_t H, int32_t N, int32_t refine_radius, int32_t radius_max);
int reduce_propose(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N, const float *params,
                   int32_t refine_radius, int32_t radius_max, float peak_ratio, int32_t max_moves,
                   reduce_offset_t *out, int32_t *centres, int32_t *info, void *ws, size_t ws_bytes, void *stream);

/* ---- training and evaluation frames --------------------------------------------
 * reduce_render_frames: F synthetic sky frames [F][H][W] (device float out) for the
 *   network's training and evaluation pairs: sky + sum over the frame's S catalogue
 *   stars of amp * exp(-r^2 / (2 sigma^2)) (sigma = fwhm / 2.3548; pixel centres at
 *   integer coordinates; each star reaches pixels within 8 px on both axes) + noise.
 *   stars: device float [F][S][4] = (x, y, amp, unused) (NULL allowed when S = 0); keys:
 *   device int64 [F].  With
 *   noise != 0 each pixel adds sqrt(max(signal, 0) + read_noise^2) * z, z standard
 *   normal by Box-Muller from Philox4x32-10 (key = seed, counter = (pixel index y*W + x
 *   as two words, keys[f] as two words)), so a frame is reproducible from its inputs.
 *   The paper times its pipeline on random-valued dummy frames (Section 3.2.2); these
 *   stand in for calibrated sky frames.  Errors: F > 65535 -> UNSUPPORTED. */
int reduce_render_frames(const float *stars, int32_t S, const int64_t *keys, int32_t F, int32_t W, int32_t H,
                         float sky, float fwhm, float read_noise, int32_t noise, uint64_t seed, float *out,
                         void *stream);

/* ---- autotuner --------------------------------------------------------------
 * Launch shapes (tiles, workgroup sizes, lanes per pixel) are chosen per problem
 * size by timing candidates on the caller's data with HIP events; the winner is
 * cached in the process and used by every later call of that size (including the
 * batched path).  Tuning calls synchronise `stream`.
 *   reduce_tune_register: candidates of the correlation search for (W, H, radius,
 *     radius_max), each run reps times on ref/frames, then the fastest three and the
 *     fastest with other tile heights timed again in three interleaved rounds (least
 *     time wins); only shapes whose workspace fits ws_bytes are tried; out receives the offsets (device reduce_offset_t [N]);
 *     fields (host int32[16] or NULL) receives the chosen plan as in
 *     reduce_register_plan.
 *   reduce_tune_register_ws: workspace bytes that fit every candidate shape of
 *     reduce_tune_register for these sizes (0 for sizes without a template); a
 *     workspace of reduce_register_ws bytes may exclude the faster shapes.
 *   reduce_tune_combine: lanes per pixel column L in {1, 2, 4, 8, 16} for N frames;
 *     out (device float [h][w]) is overwritten; lanes (host, or NULL) gets L.
 *   reduce_tune_save / reduce_tune_load: the cache as JSON lines tagged with the
 *     device architecture; entries of other architectures are ignored on load.
 * Errors: as the calls they time; no fitting candidate -> WORKSPACE; unreadable or
 * unwritable file -> RANGE. */
/*   reduce_tune_search: the full-window search of ref/frames (radius_max = radius)
 *     timed reps times with direct sums (reduce_register, the tuned launch shape if any)
 *     and through row spectra (reduce_register_fft, when ws_bytes covers its workspace);
 *     search (host) receives the faster, REDUCE_SEARCH_DIRECT or REDUCE_SEARCH_SPECTRAL,
 *     ms_direct / ms_spectral (host, or NULL) the times (1e30 for a search not timed);
 *     ws: device workspace of at least reduce_register_ws(W, H, N, radius, radius) bytes;
 *     out: device reduce_offset_t [N] (overwritten). */
int reduce_tune_search(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                       int32_t radius, reduce_offset_t *out, void *ws, size_t ws_bytes, int32_t reps,
                       void *stream, int32_t *search, double *ms_direct, double *ms_spectral);
size_t reduce_tune_register_ws(int32_t W, int32_t H, int32_t N, int32_t radius, int32_t radius_max);
int reduce_tune_register(const float *ref, const float *frames, int32_t W, int32_t H, int32_t N,
                         int32_t radius, int32_t radius_max, reduce_offset_t *out, void *ws,
                         size_t ws_bytes, int32_t reps, void *stream, int32_t *fields);
int reduce_tune_combine(const float *aligned, int32_t w, int32_t h, int32_t N, float ksigma,
                        int32_t max_iters, float *out, int32_t reps, void *stream, int32_t *lanes);
int reduce_tune_save(const char *path);
int reduce_tune_load(const char *path);
int reduce_tune_clear(void);

#ifdef __cplusplus
}
#endif
#endif /* REDUCE_H */
