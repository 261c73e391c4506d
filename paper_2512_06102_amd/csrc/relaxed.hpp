// relaxed.hpp -- host interface of the relaxed (mean-field) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/firesim.h"
#include "internal.hpp"

namespace firesim {

// Tiles of the relaxed kernels (forward and adjoint): 64 x 32 cells, one wave
// each, one column per lane.
constexpr int kAdjW = 64, kAdjR = 32;
// Exchange record of an adjoint tile (doubles): Bbar terms for the rows
// just above and below the tile (64 each) and the columns just left and
// right of it (kAdjR + 2 each, corners included).
constexpr int kXTile = 200;

struct RelaxedTile {
    int32_t env, r0, c0, pad;
};

// The adjoint tiles of one env form a rows x cols grid starting at tile
// `first` (row-major); its (rows + 1) x (cols + 1) integral image of tiles
// holding initial burning mass starts at `ioff` (sparse adjoint).
struct TileGrid {
    int32_t first, rows, cols, ioff;
};

// Per-handle state of the relaxed path (built on first use).
struct RelaxedState {
    RelaxedTile* d_btiles = nullptr;  // tiles of the forward and the adjoint
    int32_t n_btiles = 0;
    int32_t n_env = 0;
    // pooled blocks of the BCE + pooled-MSE loss (built for one pool size)
    RelaxedTile* d_pool = nullptr;  // env, r0, c0 of each pool x pool block
    int32_t n_pool = 0, pool_k = 0;
    int32_t* d_env_blocks = nullptr;  // [n_env][2]: first block, number of blocks
    double* d_pool_vals = nullptr;    // [4][n_pool]: block means of S and Y, BCE sum, squared error
    double* d_bce_loss = nullptr;     // [n_env]: per-env loss in fp64
    // per-env grids of the adjoint tiles; sparse adjoint: per-tile
    // initial-mass flags and their integral images (sparse_lds: bytes of the
    // largest image; 0 when an image would not fit in LDS, and the adjoint
    // then stays dense)
    TileGrid* d_tgrid = nullptr;
    int32_t* d_tmass = nullptr;
    int32_t* d_tinteg = nullptr;
    int32_t sparse_lds = 0;
    // workspace whose segment slots hold the last segment's states, as the
    // last forward left them (the backward then skips that recompute)
    const void* last_segment_ws = nullptr;
};

struct RelaxedInputs {
    const RelaxedTile* tiles;
    int32_t n_tiles;
    const EnvDev* envs;
    int32_t n_env;
    const uint8_t* cls;
    const float* den;
    const float* E;
    const float* wind;  // [3][n_cells] (or a series of such planes, see wind_stride) or nullptr
    int64_t n_cells;
    int32_t form;       // 0: product form of p_ignite, 1: 1 - exp(-gamma sum B phi)
    int64_t wind_stride = 0;          // floats between the per-cell wind planes of steps t, t+1
    const float* env_wind = nullptr;  // per-env wind series [T][n_env][3] or nullptr
    int32_t sparse = 0;               // adjoint: skip tiles beyond the reach of the initial burning mass
};

int relaxed_prepare(RelaxedState& R, const std::vector<sim_env>& envs);
int relaxed_prepare_pool(RelaxedState& R, const std::vector<sim_env>& envs, int pool);
void relaxed_free(RelaxedState& R);
// Number of adjoint tiles of a batch (they size the workspace).
int64_t relaxed_adj_tiles(const std::vector<sim_env>& envs);
size_t relaxed_workspace_bytes(int64_t n_cells, int64_t n_adj_tiles, int32_t T, int32_t ckpt_every);

hipError_t launch_relaxed_init(hipStream_t s, const uint8_t* init_states, int64_t n, double* U,
                               double* B);
hipError_t relaxed_forward(hipStream_t s, const RelaxedInputs& in, const sim_params& p, double* U,
                           double* B, int32_t T, int32_t ckpt_every, void* workspace, RelaxedState& R);
// The batch as the loss kernels see it: envs with their chunk0, the env of
// every loss chunk, and the initial fire state (burnable cells).
struct LossBatch {
    const EnvDev* envs;
    int32_t n_env;
    const int32_t* chunk_env;
    int32_t n_chunks;
    const uint8_t* init_states;
};

// Scratch of the soft-IoU loss in doubles: per chunk 3 partial sums, per env
// 3 sums and its loss.
inline size_t loss_scratch_doubles(int32_t n_chunks, int32_t n_env)
{
    return 3 * (size_t)n_chunks + 4 * (size_t)n_env;
}

// Soft IoU per env, its fp64 objective scale * sum_e L_e (objective may be
// nullptr) and the seed scale * dL_e/dU_T (gU_T may be nullptr).  Every sum
// runs in a fixed order, so repeated calls give the same bits.
hipError_t relaxed_loss(hipStream_t s, const LossBatch& lb, const double* U_T, const uint8_t* target,
                        float* loss, double* gU_T, double scale, double* objective, double* scratch);
hipError_t relaxed_loss_bce(hipStream_t s, const RelaxedInputs& in, const uint8_t* init_states,
                            const double* U_T, const uint8_t* target, int pool, double mse_weight,
                            double eps, float* loss, double* gU_T, double scale, double* objective,
                            RelaxedState& R);
hipError_t relaxed_backward(hipStream_t s, const RelaxedInputs& in, const sim_params& p,
                            const double* gU_T, const double* gB_T, int32_t T, int32_t ckpt_every,
                            void* workspace, double* grad, RelaxedState& R);

}  // namespace firesim
