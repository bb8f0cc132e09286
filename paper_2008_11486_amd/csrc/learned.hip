// Offset-proposal network: input preparation, BF16 matrix-core convolutions with FP32
// accumulation (forward and backward), mean pool, linear head, Huber loss and AdamW.
//
// Network: four 3x3 convolutions with stride 2 and zero padding 1 (2 -> 32 -> 32 -> 32
// -> 32 channels), each followed by ReLU; the mean over all pixels of the last
// activation; a linear layer 32 -> 2 giving (dx, dy) in downsampled pixels.
// Activations are [B][H][W][C] bfloat16 (channels contiguous).  Master parameters
// are one flat FP32 vector W1 b1 W2 b2 W3 b3 W4 b4 Wl bl with conv weights
// W[t][cin][cout], t = 3 ky + kx.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16: a wave computes 16
// output pixels x 16 output channels per instruction with K = 32 (one tap x 32 input
// channels, or all 18 (tap, channel) pairs of the 2-channel input layer).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "common.h"
#include "learned.h"

namespace rd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest, ties to even
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ bf16x8 zero8()
{
    const uint4 v = make_uint4(0u, 0u, 0u, 0u);
    return __builtin_bit_cast(bf16x8, v);
}

// ---- network input: 4x4 block mean, standardisation, asinh, bfloat16 --------------------
constexpr int DS_BLOCK = 256;

__device__ __forceinline__ double block_sum_d(double v, double *scratch)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < DS_BLOCK / 64; ++i) t += scratch[i];
    __syncthreads();
    return t;
}

// Block means (double) of one frame per blockIdx.y, and per-block partial sums.
__global__ __launch_bounds__(DS_BLOCK) void ds_boxmean(const float *__restrict__ frames, int32_t W, int32_t H,
                                                       double *__restrict__ m, double *__restrict__ part)
{
    __shared__ double scratch[DS_BLOCK / 64];
    const int32_t w = W / 4, h = H / 4;
    const int64_t n = (int64_t)w * h;
    const int32_t f = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * DS_BLOCK + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const int32_t jy = (int32_t)(i / w), jx = (int32_t)(i - (int64_t)jy * w);
        const float *src = frames + (int64_t)f * W * H + (int64_t)(4 * jy) * W + 4 * jx;
        double s = 0.0;
        for (int y = 0; y < 4; ++y)
            for (int x = 0; x < 4; ++x) s += (double)src[(int64_t)y * W + x];
        v = s / 16.0;
        m[(int64_t)f * n + i] = v;
    }
    const double t = block_sum_d(v, scratch);
    if (threadIdx.x == 0) part[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

// Per frame: stat = sum of the partials in order / n; with `sqrt_of` the square root.
__global__ __launch_bounds__(DS_BLOCK) void ds_finish(const double *__restrict__ part, int32_t nparts, double n,
                                                      double *__restrict__ stat, int sqrt_of)
{
    __shared__ double scratch[DS_BLOCK / 64];
    const int32_t f = blockIdx.x;
    double s = 0.0;
    for (int32_t i = threadIdx.x; i < nparts; i += DS_BLOCK) s += part[(int64_t)f * nparts + i];
    s = block_sum_d(s, scratch);
    if (threadIdx.x == 0) stat[f] = sqrt_of ? sqrt(s / n) : s / n;
}

__global__ __launch_bounds__(DS_BLOCK) void ds_sqdev(const double *__restrict__ m, int64_t n,
                                                     const double *__restrict__ mean, double *__restrict__ part)
{
    __shared__ double scratch[DS_BLOCK / 64];
    const int32_t f = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * DS_BLOCK + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        const double d = m[(int64_t)f * n + i] - mean[f];
        v = d * d;
    }
    const double t = block_sum_d(v, scratch);
    if (threadIdx.x == 0) part[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(DS_BLOCK) void ds_normalize(const double *__restrict__ m, int64_t n,
                                                         const double *__restrict__ mean,
                                                         const double *__restrict__ sd, uint16_t *__restrict__ out)
{
    const int32_t f = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * DS_BLOCK + threadIdx.x;
    if (i >= n) return;
    const double s = sd[f];
    const double z = asinh(s > 0.0 ? (m[(int64_t)f * n + i] - mean[f]) / s : 0.0);
    out[(int64_t)f * n + i] = f2bf((float)z);
}

// ---- weight packing ---------------------------------------------------------------------
// Forward operand of layer l: [ksteps][32 cout][32 k] bf16, k = input channel of tap
// kstep (3x3 layers with 32 inputs) or k = 2 t + c for the 2-channel input layer
// (one kstep, k >= 18 zero).  Backward-data operand of layers 2..4: [9][32 cin][32 cout].
__global__ void pack_weights(const float *__restrict__ params, uint16_t *__restrict__ wf,
                             uint16_t *__restrict__ wd)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // layer 1: 32 x 32 forward entries
    if (tid < 1024) {
        const int32_t co = (int32_t)(tid / 32), k = (int32_t)(tid % 32);
        float v = 0.0f;
        if (k < 18) v = params[(k >> 1) * 2 * CNN_CH + (k & 1) * CNN_CH + co];
        wf[tid] = f2bf(v);
        return;
    }
    int64_t r = tid - 1024;
    if (r < 3 * 9 * 1024) {  // layers 2..4, forward layout
        const int32_t l = (int32_t)(r / (9 * 1024));
        const int32_t rem = (int32_t)(r % (9 * 1024));
        const int32_t t = rem / 1024, co = (rem % 1024) / 32, ci = rem % 32;
        const float *w = params + cnn_weight_offset(l + 1);
        wf[1024 + r] = f2bf(w[(t * CNN_CH + ci) * CNN_CH + co]);
        return;
    }
    r -= 3 * 9 * 1024;
    if (r < 3 * 9 * 1024) {  // layers 2..4, backward-data layout [t][cin][cout]
        const int32_t l = (int32_t)(r / (9 * 1024));
        const int32_t rem = (int32_t)(r % (9 * 1024));
        const float *w = params + cnn_weight_offset(l + 1);
        wd[r] = f2bf(w[rem]);
    }
}

// ---- convolution forward ---------------------------------------------------------------------
// One wave: 16 consecutive output pixels of a row x 32 channels.  The workgroup's four
// waves cover 64 pixels; results go through LDS for 16-byte stores.
template <int CIN>
__global__ __launch_bounds__(256) void conv_fwd(const uint16_t *__restrict__ x, const uint16_t *__restrict__ ref,
                                                int64_t ref_stride, const uint16_t *__restrict__ img, int32_t H,
                                                int32_t W, const uint16_t *__restrict__ wf,
                                                const float *__restrict__ bias, uint16_t *__restrict__ y)
{
    __shared__ uint16_t tile[4][16 * CNN_CH];
    const int32_t Ho = (H + 1) / 2, Wo = (W + 1) / 2;
    const int32_t b = blockIdx.z, oy = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t ox0 = blockIdx.x * 64 + wave * 16;
    const int m = lane & 15, kg = lane >> 4;
    const int32_t ox = ox0 + m;

    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    if (CIN == 2) {
        // K = 18 (tap, channel) pairs + zeros, gathered element by element
        uint16_t e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = kg * 8 + j;
            uint16_t v = 0;
            if (k < 18 && ox < Wo) {
                const int t = k >> 1, c = k & 1;
                const int32_t iy = 2 * oy + t / 3 - 1, ix = 2 * ox + t % 3 - 1;
                if (iy >= 0 && iy < H && ix >= 0 && ix < W) {
                    const int64_t p = (int64_t)iy * W + ix;
                    v = c == 0 ? ref[(int64_t)b * ref_stride + p] : img[(int64_t)b * H * W + p];
                }
            }
            e[j] = v;
        }
        const uint4 pk = make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                                    e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
        const bf16x8 a = __builtin_bit_cast(bf16x8, pk);
        const bf16x8 b0 = load8(wf + (0 * 32 + m) * 32 + kg * 8);
        const bf16x8 b1 = load8(wf + (0 * 32 + 16 + m) * 32 + kg * 8);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc1, 0, 0, 0);
    } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int32_t iy = 2 * oy + t / 3 - 1, ix = 2 * ox + t % 3 - 1;
            bf16x8 a = zero8();
            if (ox < Wo && iy >= 0 && iy < H && ix >= 0 && ix < W)
                a = load8(x + (((int64_t)b * H + iy) * W + ix) * CNN_CH + kg * 8);
            const bf16x8 b0 = load8(wf + (t * 32 + m) * 32 + kg * 8);
            const bf16x8 b1 = load8(wf + (t * 32 + 16 + m) * 32 + kg * 8);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc1, 0, 0, 0);
        }
    }
    // lane holds pixels 4 kg + j, channel m (tile 0) and 16 + m (tile 1)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int px = 4 * kg + j;
        tile[wave][px * CNN_CH + m] = f2bf(fmaxf(acc0[j] + bias[m], 0.0f));
        tile[wave][px * CNN_CH + 16 + m] = f2bf(fmaxf(acc1[j] + bias[16 + m], 0.0f));
    }
    __syncthreads();
    const int px = lane >> 2, c8 = (lane & 3) * 8;
    const int32_t oxs = ox0 + px;
    if (oxs < Wo) {
        const uint4 v = *reinterpret_cast<const uint4 *>(&tile[wave][px * CNN_CH + c8]);
        *reinterpret_cast<uint4 *>(y + (((int64_t)b * Ho + oy) * Wo + oxs) * CNN_CH + c8) = v;
    }
}

// ---- mean pool and linear head ----------------------------------------------------------------
// One workgroup per image: pool[c] = mean over pixels (double, fixed order), then
// pred = Wl pool + bl.
__global__ __launch_bounds__(256) void pool_head(const uint16_t *__restrict__ x4, int64_t P,
                                                 const float *__restrict__ params, double *__restrict__ pool,
                                                 float *__restrict__ pred)
{
    __shared__ double part[8][CNN_CH];
    const int32_t b = blockIdx.x;
    const int c = threadIdx.x % CNN_CH, g = threadIdx.x / CNN_CH;  // 8 pixel groups
    double s = 0.0;
    for (int64_t p = g; p < P; p += 8) s += (double)bf2f(x4[((int64_t)b * P + p) * CNN_CH + c]);
    part[g][c] = s;
    __syncthreads();
    if (threadIdx.x < CNN_CH) {
        double t = 0.0;
        for (int i = 0; i < 8; ++i) t += part[i][c];
        pool[b * CNN_CH + c] = t / (double)P;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int j = threadIdx.x;
        const float *wl = params + cnn_head_offset();
        double v = (double)wl[2 * CNN_CH + j];
        for (int cc = 0; cc < CNN_CH; ++cc) v += pool[b * CNN_CH + cc] * (double)wl[j * CNN_CH + cc];
        pred[2 * b + j] = (float)v;
    }
}

// ---- host side -----------------------------------------------------------------------------------
static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

CnnLayout cnn_layout(int32_t B, int32_t h, int32_t w)
{
    CnnLayout L;
    size_t off = 0;
    L.wf = off;
    off += al(sizeof(uint16_t) * (1024 + 3 * 9 * 1024));
    L.wd = off;
    off += al(sizeof(uint16_t) * 3 * 9 * 1024);
    int32_t hh = h, ww = w;
    for (int l = 0; l < 4; ++l) {
        hh = (hh + 1) / 2;
        ww = (ww + 1) / 2;
        L.hs[l] = hh;
        L.ws[l] = ww;
        L.act[l] = off;
        off += al(sizeof(uint16_t) * (size_t)B * hh * ww * CNN_CH);
    }
    L.pool = off;
    off += al(sizeof(double) * (size_t)B * CNN_CH);
    L.fwd_total = off;
    // backward: two gradient planes the size of the largest activation, partial sums
    const size_t big = sizeof(uint16_t) * (size_t)B * L.hs[0] * L.ws[0] * CNN_CH;
    L.dz[0] = off;
    off += al(big);
    L.dz[1] = off;
    off += al(big);
    L.dpool = off;
    off += al(sizeof(double) * (size_t)B * CNN_CH);
    L.wpart = off;
    off += al(sizeof(float) * (size_t)CNN_WGRAD_CHUNKS * 9 * CNN_CH * CNN_CH);
    L.bpart = off;
    off += al(sizeof(float) * (size_t)CNN_WGRAD_CHUNKS * 9 * CNN_CH);
    L.total = off;
    return L;
}

int cnn_forward_launch(const uint16_t *ref, int64_t ref_stride, const uint16_t *img, int32_t B, int32_t h,
                       int32_t w, const float *params, float *pred, void *ws, hipStream_t s)
{
    const CnnLayout L = cnn_layout(B, h, w);
    unsigned char *base = static_cast<unsigned char *>(ws);
    uint16_t *wf = reinterpret_cast<uint16_t *>(base + L.wf);
    uint16_t *wd = reinterpret_cast<uint16_t *>(base + L.wd);
    hipLaunchKernelGGL(pack_weights, dim3((unsigned)ceil_div(1024 + 6 * 9 * 1024, 256)), dim3(256), 0, s, params, wf,
                       wd);
    ProfScope prof("cnn_forward", s);
    int32_t hh = h, ww = w;
    const uint16_t *in = nullptr;
    for (int l = 0; l < 4; ++l) {
        uint16_t *out = reinterpret_cast<uint16_t *>(base + L.act[l]);
        const float *bias = params + cnn_weight_offset(l) + 9 * (l == 0 ? 2 : CNN_CH) * CNN_CH;
        dim3 grid((unsigned)ceil_div(L.ws[l], 64), (unsigned)L.hs[l], (unsigned)B);
        if (l == 0)
            hipLaunchKernelGGL(conv_fwd<2>, grid, dim3(256), 0, s, nullptr, ref, ref_stride, img, hh, ww, wf, bias,
                               out);
        else
            hipLaunchKernelGGL(conv_fwd<32>, grid, dim3(256), 0, s, in, nullptr, 0, nullptr, hh, ww,
                               wf + 1024 + (size_t)(l - 1) * 9 * 1024, bias, out);
        in = out;
        hh = L.hs[l];
        ww = L.ws[l];
    }
    hipLaunchKernelGGL(pool_head, dim3(B), dim3(256), 0, s, in, (int64_t)L.hs[3] * L.ws[3], params,
                       reinterpret_cast<double *>(base + L.pool), pred);
    return check_launch("reduce_cnn_forward");
}

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_cnn_input_ws(int32_t W, int32_t H, int32_t N)
{
    if (W < 4 || H < 4 || W % 4 || H % 4 || N < 1) return 0;
    const int64_t n = (int64_t)(W / 4) * (H / 4);
    const int64_t nparts = ceil_div(n, DS_BLOCK);
    return al(sizeof(double) * n * N) + 2 * al(sizeof(double) * nparts * N) + 2 * al(sizeof(double) * N);
}

extern "C" int reduce_cnn_input(const float *frames, int32_t W, int32_t H, int32_t N, uint16_t *out, void *ws,
                                size_t ws_bytes, void *stream)
{
    if (!frames || !out) return fail(REDUCE_ERR_NULL, "reduce_cnn_input: NULL buffer");
    if (W < 4 || H < 4 || N < 1) return fail(REDUCE_ERR_SHAPE, "reduce_cnn_input: W, H >= 4 and N >= 1 needed");
    if (W % 4 || H % 4) return fail(REDUCE_ERR_SHAPE, "reduce_cnn_input: W and H must be multiples of 4");
    if (N > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_cnn_input: N above 65535");
    const size_t need = reduce_cnn_input_ws(W, H, N);
    if (!ws || ws_bytes < need)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_cnn_input: workspace needs " + std::to_string(need) + " bytes");
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)(W / 4) * (H / 4);
    const int32_t nparts = (int32_t)ceil_div(n, DS_BLOCK);
    unsigned char *base = static_cast<unsigned char *>(ws);
    double *m = reinterpret_cast<double *>(base);
    double *part = reinterpret_cast<double *>(base + al(sizeof(double) * n * N));
    double *mean = reinterpret_cast<double *>(base + al(sizeof(double) * n * N) + 2 * al(sizeof(double) * nparts * N));
    double *sd = mean + N;
    ProfScope prof("cnn_input", s);
    const dim3 grid((unsigned)nparts, (unsigned)N);
    hipLaunchKernelGGL(ds_boxmean, grid, dim3(DS_BLOCK), 0, s, frames, W, H, m, part);
    hipLaunchKernelGGL(ds_finish, dim3(N), dim3(DS_BLOCK), 0, s, part, nparts, (double)n, mean, 0);
    hipLaunchKernelGGL(ds_sqdev, grid, dim3(DS_BLOCK), 0, s, m, n, mean, part);
    hipLaunchKernelGGL(ds_finish, dim3(N), dim3(DS_BLOCK), 0, s, part, nparts, (double)n, sd, 1);
    hipLaunchKernelGGL(ds_normalize, grid, dim3(DS_BLOCK), 0, s, m, n, mean, sd, out);
    return check_launch("reduce_cnn_input");
}

extern "C" int64_t reduce_cnn_num_params(void) { return CNN_NPARAMS; }

extern "C" size_t reduce_cnn_ws(int32_t B, int32_t h, int32_t w)
{
    if (B < 1 || h < 16 || w < 16) return 0;
    return cnn_layout(B, h, w).total;
}

extern "C" int reduce_cnn_ws_offsets(int32_t B, int32_t h, int32_t w, int64_t *offsets)
{
    if (!offsets) return fail(REDUCE_ERR_NULL, "reduce_cnn_ws_offsets: NULL argument");
    if (B < 1 || h < 16 || w < 16) return fail(REDUCE_ERR_SHAPE, "reduce_cnn_ws_offsets: bad sizes");
    const CnnLayout L = cnn_layout(B, h, w);
    for (int l = 0; l < 4; ++l) offsets[l] = (int64_t)L.act[l];
    return REDUCE_OK;
}

extern "C" int reduce_cnn_forward(const uint16_t *ref, int64_t ref_stride, const uint16_t *img, int32_t B,
                                  int32_t h, int32_t w, const float *params, float *pred, void *ws, size_t ws_bytes,
                                  void *stream)
{
    if (!ref || !img || !params || !pred) return fail(REDUCE_ERR_NULL, "reduce_cnn_forward: NULL buffer");
    if (B < 1 || h < 16 || w < 16) return fail(REDUCE_ERR_SHAPE, "reduce_cnn_forward: B >= 1 and h, w >= 16 needed");
    if (ref_stride < 0) return fail(REDUCE_ERR_RANGE, "reduce_cnn_forward: negative ref_stride");
    if (B > 65535 || h > 65535) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_cnn_forward: B or h above 65535");
    const size_t need = cnn_layout(B, h, w).total;
    if (!ws || ws_bytes < need)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_cnn_forward: workspace needs " + std::to_string(need) + " bytes");
    return cnn_forward_launch(ref, ref_stride, img, B, h, w, params, pred, ws, as_stream(stream));
}
