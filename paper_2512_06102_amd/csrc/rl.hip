// rl.hip -- the reinforcement-learning layer over the batched step.
//
// Section 4 of the paper trains an air-tanker agent: it sees an egocentric
// window of the fire, moves, and opens a valve to drop a limited amount of
// water, which turns burning cells burnt; each step costs a penalty
// proportional to the number of burning cells, and putting the fire out
// earns a terminal bonus; episodes start from a random fire and agent
// position.  One RL step of every env is:
//   rl_act_kernel   move each agent, turn an open valve into a water drop
//                   (drop row of the step kernel), spend one unit of water;
//   the step kernel one stochastic step with those drops (water mode) and
//                   the BURNING count of every env;
//   rl_obs_kernel   reward and done from the count, then the (2R+1)^2
//                   window of the new state around each agent.
// rl_reset_kernel redraws the fire and the agent of selected envs.
#include "devmath.hpp"
#include "internal.hpp"
#include "rl.hpp"

namespace firesim {
namespace {

constexpr uint8_t kOutside = 4;  // observation code of cells beyond the grid

__device__ __forceinline__ int32_t scale_draw(uint32_t w, int32_t n)
{
    return (int32_t)(((uint64_t)w * (uint64_t)n) >> 32);  // uniform in 0..n-1
}

__global__ __launch_bounds__(256) void rl_reset_kernel(const EnvDev* __restrict__ envs,
                                                       const uint8_t* __restrict__ cls,
                                                       uint32_t unburnable_mask,
                                                       uint8_t* __restrict__ states, RlAgent* __restrict__ agents,
                                                       const int32_t* __restrict__ reset_mask, uint2 key,
                                                       uint64_t episode, int32_t water)
{
    const int e = blockIdx.x;
    if (reset_mask && reset_mask[e] == 0) return;
    const EnvDev ed = envs[e];
    const int64_t n = (int64_t)ed.H * ed.W;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t v = ed.offset + i;
        states[v] = ((unburnable_mask >> cls[v]) & 1u) ? kUnburnable : kFlammable;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    RlAgent a{};
    for (uint32_t attempt = 0; attempt < kRlIgnitionAttempts; ++attempt) {
        const uint4 w = philox4x32_10(make_uint4(ed.env_id, (uint32_t)episode, (uint32_t)(episode >> 32),
                                                 0x80000000u | attempt),
                                      key);
        if (attempt == 0) {
            a.row = scale_draw(w.z, ed.H);
            a.col = scale_draw(w.w, ed.W);
        }
        const int64_t v = ed.offset + (int64_t)scale_draw(w.x, ed.H) * ed.W + scale_draw(w.y, ed.W);
        if (!((unburnable_mask >> cls[v]) & 1u)) {
            states[v] = kBurning;
            break;
        }
    }
    a.water = water;
    a.steps = 0;
    a.done = 0;
    a.last_count = 0;
    agents[e] = a;
}

__global__ __launch_bounds__(256) void rl_act_kernel(const EnvDev* __restrict__ envs, RlAgent* __restrict__ agents,
                                                     const int32_t* __restrict__ actions,
                                                     int32_t* __restrict__ drop_row, int32_t n_env)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_env) return;
    RlAgent a = agents[e];
    int32_t drop = -1;
    if (!a.done) {
        const int32_t act = actions[e];
        const int32_t move = (act >= 0 && act < 32) ? (act & 15) : 0;
        const bool valve = act >= 0 && act < 32 && ((act >> 4) & 1);
        if (move >= 1 && move <= 8) {
            const EnvDev ed = envs[e];
            a.row = min(max(a.row + kDRow[move - 1], 0), ed.H - 1);
            a.col = min(max(a.col + kDCol[move - 1], 0), ed.W - 1);
        }
        if (valve && a.water > 0) {
            drop = (a.row << 16) | a.col;
            a.water -= 1;
        }
        agents[e] = a;
    }
    drop_row[e] = drop;
}

// counts == nullptr: observation only (after a reset), reward 0.
__global__ __launch_bounds__(256) void rl_obs_kernel(const EnvDev* __restrict__ envs,
                                                     const uint8_t* __restrict__ states,
                                                     RlAgent* __restrict__ agents,
                                                     const int32_t* __restrict__ counts, RlConfigDev cfg,
                                                     uint8_t* __restrict__ obs, float* __restrict__ reward,
                                                     int32_t* __restrict__ done)
{
    const int e = blockIdx.x;
    const EnvDev ed = envs[e];
    __shared__ int32_t s_row, s_col;
    if (threadIdx.x == 0) {
        RlAgent a = agents[e];
        float r = 0.0f;
        if (counts && !a.done) {
            const int32_t c = counts[e];
            r = -cfg.burn_penalty * (float)c;
            if (c == 0) r = r + cfg.extinguish_bonus;
            a.steps += 1;
            a.last_count = c;
            a.done = (c == 0 || a.steps >= cfg.max_steps) ? 1 : 0;
            agents[e] = a;
        }
        if (reward) reward[e] = r;
        if (done) done[e] = a.done;
        s_row = a.row;
        s_col = a.col;
    }
    __syncthreads();
    const int R = cfg.obs_radius, side = 2 * R + 1;
    const int n = side * side;
    uint8_t* o = obs + (int64_t)e * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int gi = s_row - R + i / side, gj = s_col - R + i % side;
        o[i] = (gi >= 0 && gi < ed.H && gj >= 0 && gj < ed.W) ? states[ed.offset + (int64_t)gi * ed.W + gj]
                                                              : kOutside;
    }
}

}  // namespace

hipError_t launch_rl_reset(hipStream_t s, const EnvDev* envs, int32_t n_env, const uint8_t* cls,
                           uint32_t unburnable_mask, uint8_t* states, RlAgent* agents,
                           const int32_t* reset_mask, uint32_t key0, uint32_t key1, uint64_t episode,
                           int32_t water)
{
    if (n_env <= 0) return hipSuccess;
    hipLaunchKernelGGL(rl_reset_kernel, dim3(n_env), dim3(256), 0, s, envs, cls, unburnable_mask, states, agents,
                       reset_mask, make_uint2(key0, key1), episode, water);
    return hipGetLastError();
}

hipError_t launch_rl_act(hipStream_t s, const EnvDev* envs, int32_t n_env, RlAgent* agents,
                         const int32_t* actions, int32_t* drop_row)
{
    if (n_env <= 0) return hipSuccess;
    hipLaunchKernelGGL(rl_act_kernel, dim3((n_env + 255) / 256), dim3(256), 0, s, envs, agents, actions,
                       drop_row, n_env);
    return hipGetLastError();
}

hipError_t launch_rl_obs(hipStream_t s, const EnvDev* envs, int32_t n_env, const uint8_t* states,
                         RlAgent* agents, const int32_t* counts, const RlConfigDev& cfg, uint8_t* obs,
                         float* reward, int32_t* done)
{
    if (n_env <= 0) return hipSuccess;
    const int side = 2 * cfg.obs_radius + 1;
    const int threads = side * side >= 256 ? 256 : ((side * side + 63) / 64) * 64;
    hipLaunchKernelGGL(rl_obs_kernel, dim3(n_env), dim3(threads), 0, s, envs, states, agents, counts, cfg, obs,
                       reward, done);
    return hipGetLastError();
}

}  // namespace firesim
