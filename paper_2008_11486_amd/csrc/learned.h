// Shapes, parameter offsets and workspace layout of the offset-proposal network.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace rd {

constexpr int CNN_CH = 32;
constexpr int64_t CNN_NPARAMS = (9 * 2 * 32 + 32) + 3 * (9 * 32 * 32 + 32) + 2 * 32 + 2;
constexpr int CNN_WGRAD_CHUNKS = 256;  // pixel chunks of the weight-gradient reduction

// offset of conv layer l's weights (l = 0..3) in the flat parameter vector; its bias
// follows the weights
__host__ __device__ constexpr int64_t cnn_weight_offset(int l)
{
    return l == 0 ? 0 : (9 * 2 * 32 + 32) + (int64_t)(l - 1) * (9 * 32 * 32 + 32);
}
__host__ __device__ constexpr int64_t cnn_head_offset() { return cnn_weight_offset(4); }

struct CnnLayout {
    size_t wf, wd;         // packed bf16 weights (forward, backward-data)
    size_t act[4];         // X1..X4 [B][h_l][w_l][32] bf16
    int32_t hs[4], ws[4];
    size_t pool;           // [B][32] double
    size_t ppart;          // [B][chunks][32] double pooling partial sums
    size_t fwd_total;
    size_t dz[2];          // gradient planes (bf16)
    size_t dpool;          // [B][32] double
    size_t wpart, bpart;   // per-chunk partial weight and bias gradients
    size_t total;
};

CnnLayout cnn_layout(int32_t B, int32_t h, int32_t w);

}  // namespace rd
