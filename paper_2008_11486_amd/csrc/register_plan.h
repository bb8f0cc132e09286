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
    int32_t wg_per_frame;  // workgroups (work items) per frame
};

// The small-window plan (window side D <= 5): K = 0, tiles of 240 template rows x 256
// columns, one per workgroup of 256 threads, frame rows staged in 15-row chunks.
bool reg_plan_small(int32_t W, int32_t H, int32_t R, int32_t Rmax, RegPlan *out);

// Tallest tile made when other chunk counts are tried for a shape (template rows).  The
// cost model's own chunk count may give taller tiles (for wide windows it sizes tiles so
// that a frame has about 2048 workgroups, and their frame halo is shared by the chunks);
// the variants stop here because taller tiles, which stage the frame rows that
// consecutive chunks share once, lose in long batched launches what they gain in a call
// of one size: tiles of 196 rows for the 2048x2048 frames of a 64-stack batch (radius 17)
// ran its search 13% slower than tiles of 98 or 147 rows, which timed the same in the
// stage-wise calls.
constexpr int32_t kTileRowsMax = 150;

// Per-workgroup shape of a plan; everything else follows from it and the sizes.
struct RegShape {
    int32_t K, G, S, TY;
    int32_t CPT;        // LDS chunks per tile: tile rows BR = CPT * TY
};

// The plan for these sizes: the tuned shape if the autotuner cached one for
// (W, H, R, Rmax), else the cost model's choice.  K_force / TY_force (or
// REDUCE_REG_K / REDUCE_REG_TY in the environment) restrict the model's search.
RegPlan reg_plan(int32_t W, int32_t H, int32_t R, int32_t Rmax, int32_t K_force = 0, int32_t TY_force = 0);

// Complete a plan from a workgroup shape; returns false if it does not fit.
bool reg_plan_from_shape(int32_t W, int32_t H, int32_t R, int32_t Rmax, const RegShape &sh, RegPlan *out);

// Candidate shapes for the autotuner: the model's best few for every K.
void reg_shape_candidates(int32_t W, int32_t H, int32_t R, int32_t Rmax, RegShape *out, int *count, int max_count);

// Tuned-shape cache (keyed by W, H, R, Rmax on the current device).
bool tuned_reg_shape(int32_t W, int32_t H, int32_t R, int32_t Rmax, RegShape *sh);
void set_tuned_reg_shape(int32_t W, int32_t H, int32_t R, int32_t Rmax, const RegShape &sh, double ms);
int tuned_combine_lanes(int32_t N);
void set_tuned_combine_lanes(int32_t N, int lanes, double ms);

}  // namespace rd
