// rl.hpp -- device-side types and launchers of the reinforcement-learning layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace firesim {

// Same layout as sim_rl_agent of the C ABI.
struct RlAgent {
    int32_t row, col;    // position on the grid
    int32_t water;       // drops left
    int32_t steps;       // steps taken in the episode
    int32_t done;        // episode over (fire out or step limit)
    int32_t last_count;  // BURNING cells after the last step
    int32_t pad[2];
};

struct RlConfigDev {
    int32_t obs_radius;
    int32_t max_steps;
    float burn_penalty;
    float extinguish_bonus;
};

// Draws tried for a burnable ignition cell at a reset (after that, no fire).
constexpr uint32_t kRlIgnitionAttempts = 8;

// Shape of the fused RL step over a batch whose envs all have W % 4 == 0:
// the largest framed state, (H + 2)(W/4 + 2) dwords, rounded up to a
// multiple of 4, and the largest env in cells (at most 65536).  It fits when
// its dynamic LDS is at most kRlFusedMaxLds.
struct RlFusedShape {
    bool fits = false;
    int32_t frame_cap = 0;
    int32_t cell_cap = 0;
};
constexpr size_t kRlFusedMaxLds = 64 * 1024;
// Dwords of the dense new state, rounded up to keep what follows 16-byte aligned.
__host__ __device__ inline int32_t rl_fused_new_dwords(int32_t cell_cap) { return ((cell_cap / 4) + 3) & ~3; }
// Old state (framed), new state, one uniform, one list entry and one
// decision byte per cell.
inline size_t rl_fused_lds_bytes(const RlFusedShape& s)
{
    return 4 * ((size_t)s.frame_cap + (size_t)rl_fused_new_dwords(s.cell_cap) + 2 * (size_t)s.cell_cap) +
           (size_t)s.cell_cap;
}

hipError_t launch_rl_reset(hipStream_t s, const EnvDev* envs, int32_t n_env, const uint8_t* cls,
                           uint32_t unburnable_mask, uint8_t* states, RlAgent* agents,
                           const int32_t* reset_mask, uint32_t key0, uint32_t key1, uint64_t episode,
                           int32_t water);
hipError_t launch_rl_act(hipStream_t s, const EnvDev* envs, int32_t n_env, RlAgent* agents,
                         const int32_t* actions, int32_t* drop_row);
// One launch per RL step for envs that fit (see rl_fused_lds_dwords); the
// fire step is bit-identical to the step kernels' with a water drop.
hipError_t launch_rl_step_fused(hipStream_t s, const EnvDev* envs, int32_t n_env, const StaticFields& F,
                                const StepArgs& A, const RlFusedShape& shape, uint8_t* states, RlAgent* agents,
                                const int32_t* actions, const RlConfigDev& cfg, uint32_t t, uint8_t* obs,
                                float* reward, int32_t* done);
hipError_t launch_rl_obs(hipStream_t s, const EnvDev* envs, int32_t n_env, const uint8_t* states,
                         RlAgent* agents, const int32_t* counts, const RlConfigDev& cfg, uint8_t* obs,
                         float* reward, int32_t* done);

}  // namespace firesim
