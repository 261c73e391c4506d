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

hipError_t launch_rl_reset(hipStream_t s, const EnvDev* envs, int32_t n_env, const uint8_t* cls,
                           uint32_t unburnable_mask, uint8_t* states, RlAgent* agents,
                           const int32_t* reset_mask, uint32_t key0, uint32_t key1, uint64_t episode,
                           int32_t water);
hipError_t launch_rl_act(hipStream_t s, const EnvDev* envs, int32_t n_env, RlAgent* agents,
                         const int32_t* actions, int32_t* drop_row);
hipError_t launch_rl_obs(hipStream_t s, const EnvDev* envs, int32_t n_env, const uint8_t* states,
                         RlAgent* agents, const int32_t* counts, const RlConfigDev& cfg, uint8_t* obs,
                         float* reward, int32_t* done);

}  // namespace firesim
