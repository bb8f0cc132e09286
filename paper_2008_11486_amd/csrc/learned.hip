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

#include <algorithm>
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

// One pass per frame: the 4x4 block means (summed in double, stored as float), and per
// workgroup the sums of d = v - c and d^2, with c the frame's first block mean (a shift
// that keeps the one-pass variance free of cancellation; every workgroup recomputes it,
// the first one stores it).
__device__ __forceinline__ double box4(const float *__restrict__ src, int32_t W)
{
    double s = 0.0;
    for (int y = 0; y < 4; ++y)
        for (int x = 0; x < 4; ++x) s += (double)src[(int64_t)y * W + x];
    return s / 16.0;
}

__global__ __launch_bounds__(DS_BLOCK) void ds_boxmean(const float *__restrict__ frames, int32_t W, int32_t H,
                                                       float *__restrict__ m, double *__restrict__ part,
                                                       double *__restrict__ shift)
{
    __shared__ double scratch[DS_BLOCK / 64];
    const int32_t w = W / 4, h = H / 4;
    const int64_t n = (int64_t)w * h;
    const int32_t f = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * DS_BLOCK + threadIdx.x;
    const float *frame = frames + (int64_t)f * W * H;
    const double c = box4(frame, W);
    double d = 0.0;
    if (i < n) {
        const int32_t jy = (int32_t)(i / w), jx = (int32_t)(i - (int64_t)jy * w);
        const double v = box4(frame + (int64_t)(4 * jy) * W + 4 * jx, W);
        m[(int64_t)f * n + i] = (float)v;
        d = v - c;
    }
    const double t1 = block_sum_d(d, scratch);
    const double t2 = block_sum_d(d * d, scratch);
    if (threadIdx.x == 0) {
        double *pp = part + 2 * ((int64_t)f * gridDim.x + blockIdx.x);
        pp[0] = t1;
        pp[1] = t2;
        if (blockIdx.x == 0) shift[f] = c;
    }
}

// Per frame: mean = c + S1 / n and population sigma = sqrt(S2 / n - (S1 / n)^2), the
// partial sums added over workgroups in a fixed order.
__global__ __launch_bounds__(DS_BLOCK) void ds_finish(const double *__restrict__ part, int32_t nparts, double n,
                                                      const double *__restrict__ shift, double *__restrict__ mean,
                                                      double *__restrict__ sd)
{
    __shared__ double scratch[DS_BLOCK / 64];
    const int32_t f = blockIdx.x;
    double s1 = 0.0, s2 = 0.0;
    for (int32_t i = threadIdx.x; i < nparts; i += DS_BLOCK) {
        s1 += part[2 * ((int64_t)f * nparts + i)];
        s2 += part[2 * ((int64_t)f * nparts + i) + 1];
    }
    s1 = block_sum_d(s1, scratch);
    s2 = block_sum_d(s2, scratch);
    if (threadIdx.x == 0) {
        const double a = s1 / n;
        mean[f] = shift[f] + a;
        sd[f] = sqrt(fmax(s2 / n - a * a, 0.0));
    }
}

// Four values per thread: standardise, asinh, round to bfloat16.
__global__ __launch_bounds__(DS_BLOCK) void ds_normalize(const float *__restrict__ m, int64_t n,
                                                         const double *__restrict__ mean,
                                                         const double *__restrict__ sd, uint16_t *__restrict__ out)
{
    const int32_t f = blockIdx.y;
    const int64_t i0 = ((int64_t)blockIdx.x * DS_BLOCK + threadIdx.x) * 4;
    if (i0 >= n) return;
    const double s = sd[f], mu = mean[f];
    const float *src = m + (int64_t)f * n;
    uint16_t *dst = out + (int64_t)f * n;
    auto z = [&](float v) { return f2bf((float)asinh(s > 0.0 ? ((double)v - mu) / s : 0.0)); };
    if (i0 + 4 <= n && n % 4 == 0 && (reinterpret_cast<uintptr_t>(out) & 7u) == 0) {
        const float4 v = *reinterpret_cast<const float4 *>(src + i0);
        const uint32_t lo = (uint32_t)z(v.x) | ((uint32_t)z(v.y) << 16);
        const uint32_t hi = (uint32_t)z(v.z) | ((uint32_t)z(v.w) << 16);
        *reinterpret_cast<uint2 *>(dst + i0) = make_uint2(lo, hi);
    } else {
        for (int64_t i = i0; i < min(i0 + 4, n); ++i) dst[i] = z(src[i]);
    }
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
// One wave: 16 consecutive output pixels of a row x 32 channels per MFMA pair; results go
// through LDS for 16-byte stores.  Layer 1 (CIN = 2): the workgroup's four waves cover 64
// pixels, and the three input rows of both channels they need are staged in LDS with
// coalesced loads first.  Layers 2-4 (CIN = 32): a wave keeps the weights of all nine taps
// in registers and covers NG groups of 64 pixels (one group per pass of the workgroup), so
// the weights are read once per NG * 64 pixels.  The accumulation order (taps in order,
// one MFMA per tap and 16 channels) is the same in every case.
constexpr int CONV_NG = 4;  // 64-pixel groups per workgroup of the 32-channel layers

template <int CIN>
__global__ __launch_bounds__(256) void conv_fwd(const uint16_t *__restrict__ x, const uint16_t *__restrict__ ref,
                                                int64_t ref_stride, const uint16_t *__restrict__ img, int32_t H,
                                                int32_t W, const uint16_t *__restrict__ wf,
                                                const float *__restrict__ bias, uint16_t *__restrict__ y)
{
    constexpr int NG = CIN == 2 ? 1 : CONV_NG;
    constexpr int XC = 2 * 64 + 4;  // staged input columns (129 used)
    __shared__ __align__(16) uint16_t tile[4][16 * CNN_CH];
    __shared__ uint16_t in2[CIN == 2 ? 3 * 2 * XC : 1];
    const int32_t Ho = (H + 1) / 2, Wo = (W + 1) / 2;
    const int32_t b = blockIdx.z, oy = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kg = lane >> 4;

    bf16x8 wb0[CIN == 2 ? 1 : 9], wb1[CIN == 2 ? 1 : 9];
#pragma unroll
    for (int t = 0; t < (CIN == 2 ? 1 : 9); ++t) {
        wb0[t] = load8(wf + (t * 32 + m) * 32 + kg * 8);
        wb1[t] = load8(wf + (t * 32 + 16 + m) * 32 + kg * 8);
    }
    const float bias0 = bias[m], bias1 = bias[16 + m];

    for (int g = 0; g < NG; ++g) {
        const int32_t gx0 = (blockIdx.x * NG + g) * 64;  // first output pixel of the group
        if (gx0 >= Wo) break;                            // uniform over the workgroup
        const int32_t ox0 = gx0 + wave * 16;
        const int32_t ox = ox0 + m;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        if constexpr (CIN == 2) {
            // input rows 2 oy - 1 .. 2 oy + 1, columns 2 gx0 - 1 + c, both channels
            for (int e = threadIdx.x; e < 3 * 2 * (XC - 3); e += 256) {
                const int r = e / (2 * (XC - 3)), rem = e - r * 2 * (XC - 3);
                const int c = rem / (XC - 3), col = rem - c * (XC - 3);
                const int32_t iy = 2 * oy + r - 1, ix = 2 * gx0 - 1 + col;
                uint16_t v = 0;
                if (iy >= 0 && iy < H && ix >= 0 && ix < W) {
                    const int64_t p = (int64_t)iy * W + ix;
                    v = c == 0 ? ref[(int64_t)b * ref_stride + p] : img[(int64_t)b * H * W + p];
                }
                in2[(r * 2 + c) * XC + col] = v;
            }
            __syncthreads();
            // K = 18 (tap, channel) pairs + zeros
            uint16_t e8[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = kg * 8 + j;
                uint16_t v = 0;
                if (k < 18 && ox < Wo) {
                    const int t = k >> 1, c = k & 1;
                    v = in2[((t / 3) * 2 + c) * XC + 2 * (ox - gx0) + t % 3];
                }
                e8[j] = v;
            }
            const uint4 pk = make_uint4(e8[0] | ((uint32_t)e8[1] << 16), e8[2] | ((uint32_t)e8[3] << 16),
                                        e8[4] | ((uint32_t)e8[5] << 16), e8[6] | ((uint32_t)e8[7] << 16));
            const bf16x8 a = __builtin_bit_cast(bf16x8, pk);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wb0[0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wb1[0], acc1, 0, 0, 0);
        } else {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int32_t iy = 2 * oy + t / 3 - 1, ix = 2 * ox + t % 3 - 1;
                bf16x8 a = zero8();
                if (ox < Wo && iy >= 0 && iy < H && ix >= 0 && ix < W)
                    a = load8(x + (((int64_t)b * H + iy) * W + ix) * CNN_CH + kg * 8);
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wb0[t], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wb1[t], acc1, 0, 0, 0);
            }
        }
        // lane holds pixels 4 kg + j, channel m (tile 0) and 16 + m (tile 1)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int px = 4 * kg + j;
            tile[wave][px * CNN_CH + m] = f2bf(fmaxf(acc0[j] + bias0, 0.0f));
            tile[wave][px * CNN_CH + 16 + m] = f2bf(fmaxf(acc1[j] + bias1, 0.0f));
        }
        __syncthreads();
        const int px = lane >> 2, c8 = (lane & 3) * 8;
        const int32_t oxs = ox0 + px;
        if (oxs < Wo) {
            const uint4 v = *reinterpret_cast<const uint4 *>(&tile[wave][px * CNN_CH + c8]);
            *reinterpret_cast<uint4 *>(y + (((int64_t)b * Ho + oy) * Wo + oxs) * CNN_CH + c8) = v;
        }
        __syncthreads();  // the tiles (and staged rows) are reused by the next group
    }
}

// ---- mean pool and linear head ----------------------------------------------------------------
// pool_partial: workgroup (chunk, image) sums POOL_CHUNK pixels of every channel (eight
// pixel groups, then the groups in order, in double).  pool_head: one workgroup per
// image adds the chunk sums in chunk order, pool[c] = sum / P, then pred = Wl pool + bl.
constexpr int POOL_CHUNK = 128;

__global__ __launch_bounds__(256) void pool_partial(const uint16_t *__restrict__ x4, int64_t P, int32_t nchunk,
                                                    double *__restrict__ part)
{
    __shared__ double red[8][CNN_CH];
    const int32_t b = blockIdx.y, ch = blockIdx.x;
    const int c = threadIdx.x % CNN_CH, g = threadIdx.x / CNN_CH;  // 8 pixel groups
    const int64_t p0 = (int64_t)ch * POOL_CHUNK, p1 = min(p0 + POOL_CHUNK, P);
    double s = 0.0;
    for (int64_t p = p0 + g; p < p1; p += 8) s += (double)bf2f(x4[((int64_t)b * P + p) * CNN_CH + c]);
    red[g][c] = s;
    __syncthreads();
    if (threadIdx.x < CNN_CH) {
        double t = 0.0;
        for (int i = 0; i < 8; ++i) t += red[i][threadIdx.x];
        part[((int64_t)b * nchunk + ch) * CNN_CH + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(64) void pool_head(const double *__restrict__ part, int32_t nchunk, int64_t P,
                                                const float *__restrict__ params, double *__restrict__ pool,
                                                float *__restrict__ pred)
{
    __shared__ double pl[CNN_CH];
    const int32_t b = blockIdx.x;
    if (threadIdx.x < CNN_CH) {
        double t = 0.0;
        for (int32_t i = 0; i < nchunk; ++i) t += part[((int64_t)b * nchunk + i) * CNN_CH + threadIdx.x];
        pl[threadIdx.x] = t / (double)P;
        pool[b * CNN_CH + threadIdx.x] = pl[threadIdx.x];
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int j = threadIdx.x;
        const float *wl = params + cnn_head_offset();
        double v = (double)wl[2 * CNN_CH + j];
        for (int cc = 0; cc < CNN_CH; ++cc) v += pl[cc] * (double)wl[j * CNN_CH + cc];
        pred[2 * b + j] = (float)v;
    }
}

// ---- loss and head backward ------------------------------------------------------------------
// One workgroup: Huber loss, head gradients (double sums over the batch in order) and
// the gradient with respect to the pooled features.
__global__ __launch_bounds__(256) void head_backward(const float *__restrict__ pred, const float *__restrict__ target,
                                                     int32_t B, double delta, const double *__restrict__ pool,
                                                     const float *__restrict__ params, float *__restrict__ loss,
                                                     float *__restrict__ grad, double *__restrict__ dpool)
{
    __shared__ double dpred[2 * 1024];
    __shared__ double lpart[256];
    const float *wl = params + cnn_head_offset();
    double l = 0.0;
    for (int32_t i = threadIdx.x; i < 2 * B; i += 256) {
        const double e = (double)pred[i] - (double)target[i];
        const double ae = fabs(e);
        l += ae <= delta ? 0.5 * e * e : delta * (ae - 0.5 * delta);
        dpred[i] = (ae <= delta ? e : (e > 0 ? delta : -delta)) / (2.0 * B);
    }
    lpart[threadIdx.x] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 256; ++i) t += lpart[i];
        *loss = (float)(t / (2.0 * B));
    }
    float *gh = grad + cnn_head_offset();
    if (threadIdx.x < 2 * CNN_CH) {  // dWl[j][c]
        const int j = threadIdx.x / CNN_CH, c = threadIdx.x % CNN_CH;
        double sacc = 0.0;
        for (int32_t b = 0; b < B; ++b) sacc += dpred[2 * b + j] * pool[b * CNN_CH + c];
        gh[j * CNN_CH + c] = (float)sacc;
    } else if (threadIdx.x < 2 * CNN_CH + 2) {  // dbl[j]
        const int j = threadIdx.x - 2 * CNN_CH;
        double sacc = 0.0;
        for (int32_t b = 0; b < B; ++b) sacc += dpred[2 * b + j];
        gh[2 * CNN_CH + j] = (float)sacc;
    }
    for (int32_t i = threadIdx.x; i < B * CNN_CH; i += 256) {
        const int32_t b = i / CNN_CH, c = i % CNN_CH;
        dpool[i] = dpred[2 * b] * (double)wl[c] + dpred[2 * b + 1] * (double)wl[CNN_CH + c];
    }
}

// Gradient of the last pre-activation: the pool's 1/P spread, masked by ReLU.
__global__ void pool_backward(const uint16_t *__restrict__ x4, int64_t P, int32_t B,
                              const double *__restrict__ dpool, uint16_t *__restrict__ dz)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * P * CNN_CH) return;
    const int32_t c = (int32_t)(i % CNN_CH);
    const int32_t b = (int32_t)(i / (P * CNN_CH));
    const double g = bf2f(x4[i]) > 0.0f ? dpool[b * CNN_CH + c] / (double)P : 0.0;
    dz[i] = f2bf((float)g);
}

// ---- weight gradient ---------------------------------------------------------------------------
// dW[t][ci][co] = sum over output pixels of X[input pixel of tap t][ci] * dZ[pixel][co],
// as D[co][n] with K = 32 output pixels per step.  For the 2-channel input layer n =
// 2 t + ci (18 columns); otherwise n = ci for each of the 9 taps.  A chunk of pixel
// blocks per workgroup writes one partial; wgrad_reduce sums the partials in order.
template <int CIN>
__global__ __launch_bounds__(256) void wgrad(const uint16_t *__restrict__ x, const uint16_t *__restrict__ ref,
                                             int64_t ref_stride, const uint16_t *__restrict__ img, int32_t B,
                                             int32_t H, int32_t W, const uint16_t *__restrict__ dz,
                                             float *__restrict__ wpart, float *__restrict__ bpart)
{
    constexpr int TAPS = CIN == 2 ? 1 : 9;  // column groups of 32
    __shared__ uint16_t zt[32][CNN_CH + 2];      // [pixel][co]
    __shared__ uint16_t xt[TAPS][32][32 + 2];    // [group][pixel][n]
    const int32_t Ho = (H + 1) / 2, Wo = (W + 1) / 2;
    const int64_t P = (int64_t)B * Ho * Wo;
    const int64_t nblk = (P + 31) / 32;
    const int64_t per = (nblk + gridDim.x - 1) / gridDim.x;
    const int64_t blk0 = (int64_t)blockIdx.x * per, blk1 = min(blk0 + per, nblk);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mt = wave & 1, nt = wave >> 1;  // co tile, column tile
    f32x4 acc[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;

    for (int64_t blk = blk0; blk < blk1; ++blk) {
        __syncthreads();
        // dZ tile: 32 pixels x 32 channels
        for (int e = threadIdx.x; e < 32 * CNN_CH; e += 256) {
            const int pp = e / CNN_CH, c = e % CNN_CH;
            const int64_t p = blk * 32 + pp;
            zt[pp][c] = p < P ? dz[p * CNN_CH + c] : (uint16_t)0;
        }
        // input tiles
        for (int e = threadIdx.x; e < TAPS * 32 * 32; e += 256) {
            const int g = e / 1024, pp = (e / 32) % 32, n = e % 32;
            const int64_t p = blk * 32 + pp;
            uint16_t v = 0;
            if (p < P) {
                const int32_t b = (int32_t)(p / ((int64_t)Ho * Wo));
                const int32_t r = (int32_t)(p % ((int64_t)Ho * Wo));
                const int32_t oy = r / Wo, ox = r % Wo;
                int t, ci;
                if (CIN == 2) {
                    t = n >> 1;
                    ci = n & 1;
                } else {
                    t = g;
                    ci = n;
                }
                if (t < 9) {
                    const int32_t iy = 2 * oy + t / 3 - 1, ix = 2 * ox + t % 3 - 1;
                    if (iy >= 0 && iy < H && ix >= 0 && ix < W) {
                        if (CIN == 2) {
                            const int64_t q = (int64_t)iy * W + ix;
                            v = ci == 0 ? ref[(int64_t)b * ref_stride + q] : img[(int64_t)b * H * W + q];
                        } else {
                            v = x[(((int64_t)b * H + iy) * W + ix) * CNN_CH + ci];
                        }
                    }
                }
            }
            xt[g][pp][n] = v;
        }
        __syncthreads();
        if (threadIdx.x < CNN_CH) {
            const int c = threadIdx.x;
            for (int pp = 0; pp < 32; ++pp) bsum += bf2f(zt[pp][c]);
        }
        // A[m = co][k = pixel], B[k = pixel][n]
        const int m = lane & 15, kg = lane >> 4;
        uint16_t ae[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) ae[j] = zt[kg * 8 + j][mt * 16 + m];
        const uint4 apk = make_uint4(ae[0] | ((uint32_t)ae[1] << 16), ae[2] | ((uint32_t)ae[3] << 16),
                                     ae[4] | ((uint32_t)ae[5] << 16), ae[6] | ((uint32_t)ae[7] << 16));
        const bf16x8 a = __builtin_bit_cast(bf16x8, apk);
#pragma unroll
        for (int g = 0; g < TAPS; ++g) {
            uint16_t be[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) be[j] = xt[g][kg * 8 + j][nt * 16 + m];
            const uint4 bpk = make_uint4(be[0] | ((uint32_t)be[1] << 16), be[2] | ((uint32_t)be[3] << 16),
                                         be[4] | ((uint32_t)be[5] << 16), be[6] | ((uint32_t)be[7] << 16));
            acc[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bpk), acc[g], 0, 0, 0);
        }
    }
    // D[co = 16 mt + 4 kg + j][n = 16 nt + m]
    const int m = lane & 15, kg = lane >> 4;
    float *wp = wpart + (int64_t)blockIdx.x * 9 * CNN_CH * CNN_CH;
#pragma unroll
    for (int g = 0; g < TAPS; ++g)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = mt * 16 + kg * 4 + j, n = nt * 16 + m;
            int t, ci;
            if (CIN == 2) {
                t = n >> 1;
                ci = n & 1;
                if (n >= 18) continue;
            } else {
                t = g;
                ci = n;
            }
            wp[((int64_t)t * CIN + ci) * CNN_CH + co] = acc[g][j];
        }
    if (threadIdx.x < CNN_CH) bpart[(int64_t)blockIdx.x * CNN_CH + threadIdx.x] = bsum;
}

// Sum the chunk partials in chunk order: n_w weight and CNN_CH bias entries.
__global__ void wgrad_reduce(const float *__restrict__ wpart, const float *__restrict__ bpart, int32_t chunks,
                             int32_t n_w, float *__restrict__ gw, float *__restrict__ gb)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_w) {
        float s = 0.0f;
        for (int32_t c = 0; c < chunks; ++c) s += wpart[(int64_t)c * 9 * CNN_CH * CNN_CH + i];
        gw[i] = s;
    } else if (i < n_w + CNN_CH) {
        const int32_t co = i - n_w;
        float s = 0.0f;
        for (int32_t c = 0; c < chunks; ++c) s += bpart[(int64_t)c * CNN_CH + co];
        gb[co] = s;
    }
}

// ---- data gradient -------------------------------------------------------------------------------
// dX[iy][ix][ci] = sum over the taps whose output pixel exists of dZ[oy][ox][co] W[t][ci][co];
// the result times the ReLU mask of X is the previous layer's dZ.  A wave takes 16 input
// pixels of one row with the same x parity (ix = 2 j + px), so all 16 share the valid
// taps: one ky for even iy, two for odd; likewise kx.
__global__ __launch_bounds__(256) void dgrad(const uint16_t *__restrict__ dz, const uint16_t *__restrict__ wd,
                                             const uint16_t *__restrict__ xin, int32_t H, int32_t W,
                                             uint16_t *__restrict__ dzin)
{
    __shared__ __align__(16) uint16_t tile[4][16 * CNN_CH];
    const int32_t Ho = (H + 1) / 2, Wo = (W + 1) / 2;
    const int32_t b = blockIdx.z;
    const int32_t iy = blockIdx.y >> 1, px = blockIdx.y & 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t j0 = (blockIdx.x * 4 + wave) * 16;
    const int m = lane & 15, kg = lane >> 4;
    const int32_t jm = j0 + m, ixm = 2 * jm + px;

    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int ky = 0; ky < 3; ++ky) {
        const int32_t ny = iy + 1 - ky;
        if (ny < 0 || (ny & 1)) continue;
        const int32_t oy = ny >> 1;
        if (oy >= Ho) continue;
        for (int kx = 0; kx < 3; ++kx) {
            if ((px + 1 - kx) & 1) continue;
            const int t = 3 * ky + kx;
            const int32_t nx = ixm + 1 - kx;  // even by the parity of the tile
            bf16x8 a = zero8();
            if (ixm < W && nx >= 0 && (nx >> 1) < Wo)
                a = load8(dz + (((int64_t)b * Ho + oy) * Wo + (nx >> 1)) * CNN_CH + kg * 8);
            const bf16x8 b0 = load8(wd + ((int64_t)t * CNN_CH + m) * CNN_CH + kg * 8);
            const bf16x8 b1 = load8(wd + ((int64_t)t * CNN_CH + 16 + m) * CNN_CH + kg * 8);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc1, 0, 0, 0);
        }
    }
    // lane holds pixels 4 kg + j, input channel m (and 16 + m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int pp = 4 * kg + j;
        const int32_t ix = 2 * (j0 + pp) + px;
        float g0 = 0.0f, g1 = 0.0f;
        if (ix < W) {
            const uint16_t *xp = xin + (((int64_t)b * H + iy) * W + ix) * CNN_CH;
            g0 = bf2f(xp[m]) > 0.0f ? acc0[j] : 0.0f;
            g1 = bf2f(xp[16 + m]) > 0.0f ? acc1[j] : 0.0f;
        }
        tile[wave][pp * CNN_CH + m] = f2bf(g0);
        tile[wave][pp * CNN_CH + 16 + m] = f2bf(g1);
    }
    __syncthreads();
    const int pp = lane >> 2, c8 = (lane & 3) * 8;
    const int32_t ix = 2 * (j0 + pp) + px;
    if (ix < W) {
        const uint4 v = *reinterpret_cast<const uint4 *>(&tile[wave][pp * CNN_CH + c8]);
        *reinterpret_cast<uint4 *>(dzin + (((int64_t)b * H + iy) * W + ix) * CNN_CH + c8) = v;
    }
}

// ---- AdamW on the FP32 master parameters ------------------------------------------------------
__global__ void adamw(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                      const float *__restrict__ g, int64_t n, float lr, float beta1, float beta2, float eps, float wd,
                      float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    p[i] = p[i] - lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
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
    L.ppart = off;
    off += al(sizeof(double) * (size_t)B * ceil_div((int64_t)L.hs[3] * L.ws[3], POOL_CHUNK) * CNN_CH);
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
        dim3 grid((unsigned)ceil_div(L.ws[l], 64 * (l == 0 ? 1 : CONV_NG)), (unsigned)L.hs[l], (unsigned)B);
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
    const int64_t P4 = (int64_t)L.hs[3] * L.ws[3];
    const int32_t nchunk = (int32_t)ceil_div(P4, POOL_CHUNK);
    double *ppart = reinterpret_cast<double *>(base + L.ppart);
    hipLaunchKernelGGL(pool_partial, dim3((unsigned)nchunk, (unsigned)B), dim3(256), 0, s, in, P4, nchunk, ppart);
    hipLaunchKernelGGL(pool_head, dim3(B), dim3(64), 0, s, ppart, nchunk, P4, params,
                       reinterpret_cast<double *>(base + L.pool), pred);
    return check_launch("reduce_cnn_forward");
}

int cnn_backward_launch(const uint16_t *ref, int64_t ref_stride, const uint16_t *img, int32_t B, int32_t h,
                        int32_t w, const float *params, const float *pred, const float *target, double delta,
                        float *loss, float *grad, void *ws, hipStream_t s)
{
    const CnnLayout L = cnn_layout(B, h, w);
    unsigned char *base = static_cast<unsigned char *>(ws);
    const uint16_t *wd = reinterpret_cast<const uint16_t *>(base + L.wd);
    double *pool = reinterpret_cast<double *>(base + L.pool);
    double *dpool = reinterpret_cast<double *>(base + L.dpool);
    float *wpart = reinterpret_cast<float *>(base + L.wpart);
    float *bpart = reinterpret_cast<float *>(base + L.bpart);
    uint16_t *dz[2] = {reinterpret_cast<uint16_t *>(base + L.dz[0]), reinterpret_cast<uint16_t *>(base + L.dz[1])};
    ProfScope prof("cnn_backward", s);
    hipLaunchKernelGGL(head_backward, dim3(1), dim3(256), 0, s, pred, target, B, delta, pool, params, loss, grad,
                       dpool);
    const int64_t P4 = (int64_t)L.hs[3] * L.ws[3];
    const uint16_t *x4 = reinterpret_cast<const uint16_t *>(base + L.act[3]);
    hipLaunchKernelGGL(pool_backward, dim3((unsigned)ceil_div((int64_t)B * P4 * CNN_CH, 256)), dim3(256), 0, s, x4,
                       P4, B, dpool, dz[0]);
    int cur = 0;
    for (int l = 3; l >= 0; --l) {
        const int32_t hin = l ? L.hs[l - 1] : h, win = l ? L.ws[l - 1] : w;
        const uint16_t *xin = l ? reinterpret_cast<const uint16_t *>(base + L.act[l - 1]) : nullptr;
        const int64_t nblk = ceil_div((int64_t)B * L.hs[l] * L.ws[l], 32);
        const int32_t chunks = (int32_t)std::min<int64_t>(CNN_WGRAD_CHUNKS, nblk);
        if (l == 0)
            hipLaunchKernelGGL(wgrad<2>, dim3(chunks), dim3(256), 0, s, nullptr, ref, ref_stride, img, B, hin, win,
                               dz[cur], wpart, bpart);
        else
            hipLaunchKernelGGL(wgrad<32>, dim3(chunks), dim3(256), 0, s, xin, nullptr, 0, nullptr, B, hin, win,
                               dz[cur], wpart, bpart);
        const int32_t cin = l == 0 ? 2 : CNN_CH;
        const int32_t n_w = 9 * cin * CNN_CH;
        float *gw = grad + cnn_weight_offset(l);
        hipLaunchKernelGGL(wgrad_reduce, dim3((unsigned)ceil_div(n_w + CNN_CH, 256)), dim3(256), 0, s, wpart, bpart,
                           chunks, n_w, gw, gw + n_w);
        if (l > 0) {
            const int32_t jn = (win + 1) / 2;
            dim3 grid((unsigned)ceil_div(jn, 64), (unsigned)(2 * hin), (unsigned)B);
            hipLaunchKernelGGL(dgrad, grid, dim3(256), 0, s, dz[cur], wd + (size_t)(l - 1) * 9 * 1024, xin, hin, win,
                               dz[cur ^ 1]);
            cur ^= 1;
        }
    }
    return check_launch("reduce_cnn_backward");
}

}  // namespace rd

using namespace rd;

extern "C" size_t reduce_cnn_input_ws(int32_t W, int32_t H, int32_t N)
{
    if (W < 4 || H < 4 || W % 4 || H % 4 || N < 1) return 0;
    const int64_t n = (int64_t)(W / 4) * (H / 4);
    const int64_t nparts = ceil_div(n, DS_BLOCK);
    return al(sizeof(float) * n * N) + al(2 * sizeof(double) * nparts * N) + 3 * al(sizeof(double) * N);
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
    float *m = reinterpret_cast<float *>(base);
    unsigned char *b1 = base + al(sizeof(float) * n * N);
    double *part = reinterpret_cast<double *>(b1);
    unsigned char *b2 = b1 + al(2 * sizeof(double) * nparts * N);
    double *shift = reinterpret_cast<double *>(b2);
    double *mean = reinterpret_cast<double *>(b2 + al(sizeof(double) * N));
    double *sd = reinterpret_cast<double *>(b2 + 2 * al(sizeof(double) * N));
    ProfScope prof("cnn_input", s);
    hipLaunchKernelGGL(ds_boxmean, dim3((unsigned)nparts, (unsigned)N), dim3(DS_BLOCK), 0, s, frames, W, H, m, part,
                       shift);
    hipLaunchKernelGGL(ds_finish, dim3(N), dim3(DS_BLOCK), 0, s, part, nparts, (double)n, shift, mean, sd);
    hipLaunchKernelGGL(ds_normalize, dim3((unsigned)ceil_div(n, 4 * DS_BLOCK), (unsigned)N), dim3(DS_BLOCK), 0, s,
                       m, n, mean, sd, out);
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
    offsets[4] = (int64_t)L.dz[0];
    offsets[5] = (int64_t)L.dz[1];
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

extern "C" int reduce_cnn_backward(const uint16_t *ref, int64_t ref_stride, const uint16_t *img, int32_t B,
                                   int32_t h, int32_t w, const float *params, const float *pred, const float *target,
                                   float huber_delta, float *loss, float *grad, void *ws, size_t ws_bytes,
                                   void *stream)
{
    if (!ref || !img || !params || !pred || !target || !loss || !grad)
        return fail(REDUCE_ERR_NULL, "reduce_cnn_backward: NULL buffer");
    if (B < 1 || h < 16 || w < 16) return fail(REDUCE_ERR_SHAPE, "reduce_cnn_backward: B >= 1 and h, w >= 16 needed");
    if (B > 1024) return fail(REDUCE_ERR_UNSUPPORTED, "reduce_cnn_backward: B above 1024");
    if (!(huber_delta > 0.0f)) return fail(REDUCE_ERR_RANGE, "reduce_cnn_backward: huber_delta must be > 0");
    const size_t need = cnn_layout(B, h, w).total;
    if (!ws || ws_bytes < need)
        return fail(REDUCE_ERR_WORKSPACE, "reduce_cnn_backward: workspace needs " + std::to_string(need) + " bytes");
    return cnn_backward_launch(ref, ref_stride, img, B, h, w, params, pred, target, (double)huber_delta, loss, grad,
                               ws, as_stream(stream));
}

extern "C" int reduce_cnn_adamw(float *params, float *m, float *v, const float *grad, int64_t n, float lr,
                                float beta1, float beta2, float eps, float weight_decay, int32_t step, void *stream)
{
    if (!params || !m || !v || !grad) return fail(REDUCE_ERR_NULL, "reduce_cnn_adamw: NULL buffer");
    if (n < 1 || step < 1) return fail(REDUCE_ERR_RANGE, "reduce_cnn_adamw: n and step must be >= 1");
    if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(REDUCE_ERR_RANGE, "reduce_cnn_adamw: bad hyper-parameters");
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    hipLaunchKernelGGL(adamw, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, as_stream(stream), params, m, v, grad, n,
                       lr, beta1, beta2, eps, weight_decay, c1, c2);
    return check_launch("reduce_cnn_adamw");
}
