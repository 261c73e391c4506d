// internal.hpp -- types shared by the library's host code and its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace firesim {

enum : uint8_t { kUnburnable = 0, kFlammable = 1, kBurning = 2, kBurnt = 3 };

// Device copy of one env descriptor.  The env's cells also form
// ceil(H W / kLossChunk) runs of kLossChunk cells for the loss reductions,
// numbered from chunk0 in a batch-wide list.
struct EnvDev {
    int64_t offset;
    int32_t H, W;
    uint32_t env_id;
    float V, Vx, Vy;
    int32_t chunk0;
};
constexpr int kLossChunk = 4096;

// Scalar parameters of the stochastic step, as kernel arguments.
struct StepArgs {
    float p_base, alpha_gamma, alpha_w1, alpha_w2, alpha_s, p_continue;
    float inv_run_orth, inv_run_diag;  // 1/cell_size, 1/(cell_size sqrt 2)
    uint32_t key0, key1;               // Philox key (seed lo, seed hi)
    int32_t drop_mode;                 // 0: FLAMMABLE/BURNING -> UNBURNABLE, 1: BURNING -> BURNT
    int32_t drop_radius;               // drops cover (2R+1) x (2R+1) cells
    int32_t slope_mode;                // 0: S = rise / run; 1: S = atan(rise / run)
};

// Inputs of the step resident in HBM: fuel and elevation for the life of a
// handle; wind either static (per env in EnvDev, or per cell) or a series
// indexed by the absolute step t.
struct StaticFields {
    const float* g;         // fuel term (1 + veg[class]) (1 + den), fp32 [n_cells]
    const float* E;         // elevation, m [n_cells]
    const float* wind;      // [3][n_cells] (V | Vx | Vy), or [T][3][n_cells] when
                            // wind_stride != 0, or nullptr (per-env wind)
    int64_t n_cells;
    int64_t wind_stride;    // elements between the per-cell wind of steps t and t+1
    const float* env_wind;  // [T][n_env][3] per-env wind series or nullptr
    int32_t n_env;
};

// One workgroup tile of the stochastic step: env, first row, first column and
// tile width in cells (16, 32, 64, 128 or 256; narrow envs get narrow tiles).
// Its height is (256 / width) * rows_per_thread.
struct TileDesc {
    int32_t env, r0, c0, width;
};

constexpr int kBlock = 256;

// Launchers (stream-ordered, no synchronisation).
hipError_t launch_init_cells(hipStream_t s, int64_t n, const uint8_t* cls, const float* den,
                             const float* elev, const float* wind_in, const float veg[11],
                             uint32_t unburnable_mask, float* g, float* E, uint8_t* cls_out,
                             float* den_out, float* wind_out, uint8_t* states);
hipError_t launch_ignite(hipStream_t s, const int32_t* ign, int32_t n_ign, const EnvDev* envs,
                         uint8_t* states);
hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);
hipError_t launch_copy_u8(hipStream_t s, uint8_t* dst, const uint8_t* src, int64_t n);
// Copy the cells of envs env_list[0..n_list) from src to dst.
hipError_t launch_copy_envs(hipStream_t s, const EnvDev* envs, const int32_t* env_list, int32_t n_list,
                            uint8_t* dst, const uint8_t* src);

struct StepLaunch {
    const TileDesc* tiles;
    int32_t n_tiles;
    const EnvDev* envs;
    int32_t n_env;
    StaticFields fields;
    StepArgs args;
    bool aligned;       // every env has W % 4 == 0
    int rows_per_thread;
    bool skip_static;   // skip fuel/elevation loads of waves with no front
};

// Sparse scheduling of the step: a tile whose cells and neighbouring tiles
// held no burning cell after the previous step (and that no drop touches) is
// left as it is.  burn_prev / burn_next: per-tile marks (nonzero: run the
// step) set by the tiles that held a burning cell after the previous step /
// this step, on themselves and their neighbours; each tile clears its mark in
// burn_prev once read, so the two arrays alternate.  A stale mark only makes
// a tile run, which is always exact.  eq[tile] != 0 when both state buffers
// hold the same content on the tile; nbr: the 8 neighbouring tiles (-1 off
// the env).  burn_next == nullptr disables it; all_active forces every tile
// to run (first step of a call, when nothing is known about the caller's
// states).
struct SparseArgs {
    int32_t* burn_prev;
    int32_t* burn_next;
    int32_t* eq;
    const int32_t* nbr;
    int32_t all_active;
};

// One stochastic step t -> t+1 from src to dst, with t = *t_base + step.
// t_base lives in device memory so that a captured sequence of launches can be
// replayed for any starting step.
hipError_t launch_stoch_step(hipStream_t s, const StepLaunch& L, const uint8_t* src,
                             uint8_t* dst, const uint32_t* t_base, uint32_t step,
                             const int32_t* actions_row, int32_t* counts_row, const SparseArgs& sp);
// ksteps (<= K, K in {2, 4, 8}) steps from src to dst in one launch over
// tiles of tile_width (64 or 128) x 32 cells; actions and counts point at the
// rows of step step0 (or are NULL).  Requires W % 4 == 0 in every env.
constexpr int kTbTileRows = 32;
hipError_t launch_stoch_tb(hipStream_t s, const StepLaunch& L, int K, int tile_width, const uint8_t* src,
                           uint8_t* dst, const uint32_t* t_base, uint32_t step0, int32_t ksteps,
                           const int32_t* actions, int32_t* counts);
hipError_t launch_set_u32(hipStream_t s, uint32_t* p, uint32_t v);

hipError_t launch_debug_exp(hipStream_t s, const float* x, float* y, int64_t n);
// HBM streaming probe over n16 16-byte words with `blocks` workgroups of 256.
hipError_t launch_stream_probe(hipStream_t s, int mode, const void* src, void* dst, int64_t n16, int blocks);
hipError_t launch_debug_atan(hipStream_t s, const float* x, float* y, int64_t n);
hipError_t launch_debug_philox(hipStream_t s, const uint32_t* ctr, const uint32_t* key,
                               uint32_t* out, int64_t n);

}  // namespace firesim
