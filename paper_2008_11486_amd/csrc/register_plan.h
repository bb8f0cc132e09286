// Launch plan of the correlation-search kernel: how candidates and template pixels
// are split over threads and workgroups.  The plan depends only on (W, H, N, R,
// Rmax) so that the workspace size can be queried before the call.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace rd {

struct RegPlan {
    int32_t D;          // window side 2R+1
    int32_t K;          // dx candidates per thread (register block)
    int32_t NBX;        // dx blocks per window row
    int32_t C;          // (window row, dx block) combinations
    int32_t G;          // candidate groups (grid.y)
    int32_t CW;         // combinations per group
    int32_t S;          // sub-ranges of template pixels per combination
    int32_t threads;    // workgroup size
    int32_t TX;         // template columns per tile (multiple of K)
    int32_t NXB;        // TX / K
    int32_t TY;         // template rows per LDS chunk
    int32_t BR;         // template rows per tile (multiple of TY)
    int32_t JS;         // window rows spanned by one group
    int32_t FR, FC;     // frame tile rows and columns in LDS
    size_t lds;         // dynamic LDS bytes
    int32_t n_bands, n_xchunks, n_tiles;  // tiles of the largest template
    int32_t th_max;
};

// Override knobs (0 = automatic): K and TY; set by the autotuner or REDUCE_REG_K /
// REDUCE_REG_TY in the environment.
RegPlan reg_plan(int32_t W, int32_t H, int32_t N, int32_t R, int32_t Rmax, int32_t K_force = 0,
                 int32_t TY_force = 0);

}  // namespace rd
