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
#include "framed.hpp"
#include "internal.hpp"
#include "rl.hpp"
#include "stepcell.hpp"

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

// One whole RL step of one env per 64-lane workgroup, the env's state
// resident in LDS: the agent's move and water drop, the fire step (same
// per-cell pieces, counters and operation order as the step kernels, hence
// the same bits), the BURNING count, reward and done, and the observation
// window.  Dynamic LDS (rl_fused_lds_bytes) holds the old state as (H + 2)
// rows of W/4 + 2 dwords with a zero frame (frame_cap dwords), the new
// state, the uniforms of the groups that draw, the list of front cells and
// their ignition decisions.  Every read of the old state comes from LDS, so
// the new state is stored in place.  A front cell's sources are read from
// HBM: few cells of an env are on the front, so staging every cell's fuel
// and elevation in LDS would cost more than it saves.
template <bool WIND_CELL>
__global__ __launch_bounds__(64) void rl_step_kernel(const EnvDev* __restrict__ envs, StaticFields F0, StepArgs A,
                                                     uint8_t* __restrict__ states, RlAgent* __restrict__ agents,
                                                     const int32_t* __restrict__ actions, RlConfigDev cfg,
                                                     uint32_t t, int32_t frame_cap, int32_t cell_cap,
                                                     uint8_t* __restrict__ obs,
                                                     float* __restrict__ reward, int32_t* __restrict__ done)
{
    extern __shared__ uint4 lds_dyn[];
    __shared__ float lds_ew[8];
    __shared__ int32_t s_drop, s_row, s_col;
    const int e = blockIdx.x, lane = threadIdx.x;
    const EnvDev ed = envs[e];
    const int H = ed.H, W = ed.W, WD = W >> 2, SW = WD + 2, n_dw = H * WD;
    const float inv_wd = 1.0f / (float)WD;
    const int64_t base = ed.offset;
    StaticFields F = F0;
    if (F0.wind_stride != 0) F.wind = F0.wind + (int64_t)t * F0.wind_stride;
    uint32_t* sS = reinterpret_cast<uint32_t*>(lds_dyn);  // old state, framed
    uint32_t* sN = sS + frame_cap;                       // new state, dense
    float* sU = reinterpret_cast<float*>(sN + rl_fused_new_dwords(cell_cap));  // uniforms per cell
    uint32_t* sL = reinterpret_cast<uint32_t*>(sU + cell_cap);  // front cells: cell | nbk << 16
    uint8_t* sD = reinterpret_cast<uint8_t*>(sL + cell_cap);    // ignition decision per cell

    // -- 1. the state into LDS; the agent acts (lane 0); per-env wind
    //       exponents (lanes 0-7); the zero frame
    const uint32_t* src = reinterpret_cast<const uint32_t*>(states + base);
    for (int i = lane; i < n_dw; i += 64) {
        const int r = small_div(i, WD, inv_wd);
        sS[i + 2 * r + SW + 1] = src[i];  // (r + 1) SW + (i - r WD) + 1
    }
    RlAgent a{};
    if (lane == 0) {
        a = agents[e];
        int32_t drop = -1;
        if (!a.done) {
            const int32_t act = actions[e];
            const int32_t move = (act >= 0 && act < 32) ? (act & 15) : 0;
            const bool valve = act >= 0 && act < 32 && ((act >> 4) & 1);
            if (move >= 1 && move <= 8) {
                a.row = min(max(a.row + kDRow[move - 1], 0), H - 1);
                a.col = min(max(a.col + kDCol[move - 1], 0), W - 1);
            }
            if (valve && a.water > 0) {
                drop = (a.row << 16) | a.col;
                a.water -= 1;
            }
        }
        s_drop = drop;
    }
    if (!WIND_CELL && lane < 8) {
        float V = ed.V, Vx = ed.Vx, Vy = ed.Vy;
        if (F.env_wind) {
            const float* w = F.env_wind + ((int64_t)t * F.n_env + e) * 3;
            V = w[0];
            Vx = w[1];
            Vy = w[2];
        }
        lds_ew[lane] = wind_exponent(lane, A.alpha_w1, A.alpha_w2, V, Vx, Vy);
    }
    for (int i = lane; i < 2 * SW; i += 64) sS[i < SW ? i : (H + 1) * SW + (i - SW)] = 0u;
    for (int i = lane; i < 2 * H; i += 64) sS[(1 + (i >> 1)) * SW + ((i & 1) ? SW - 1 : 0)] = 0u;
    __syncthreads();

    // -- 2. the drop, before the step: the dwords of its square
    const int32_t drop = s_drop;
    const int ar = (drop >> 16) & 0x7FFF, ac = drop & 0xFFFF;
    if (drop >= 0 && ar < H && ac < W) {
        const int R = A.drop_radius;
        const int r0 = max(ar - R, 0), r1 = min(ar + R, H - 1);
        const int d0 = max(ac - R, 0) >> 2, d1 = min(ac + R, W - 1) >> 2;
        const int nd = d1 - d0 + 1;
        for (int q = lane; q < (r1 - r0 + 1) * nd; q += 64) {
            const int r = r0 + q / nd, cd = d0 + q % nd;
            uint32_t* p = sS + (r + 1) * SW + cd + 1;
            *p = apply_drop(*p, r, 4 * cd, ar, ac, R, A.drop_mode);
        }
        __syncthreads();
    }

    // -- 2b. no BURNING cell after the drop: no cell can change (no front, no
    //        draw; the fire model only spreads from burning cells)
    uint32_t my_burn = 0;
    for (int i = lane; i < n_dw; i += 64) {
        const int r = small_div(i, WD, inv_wd);
        my_burn |= burning_flags(sS[i + 2 * r + SW + 1]);
    }
    const bool quiet = !__any(my_burn != 0u);

    // -- 3. draws of the groups that need one; front cells listed across the
    //       wave and evaluated by all lanes together, so that their fuel and
    //       elevation loads overlap instead of queueing on their owners
    const uint2 key = make_uint2(A.key0, A.key1);
    uint32_t my_front = 0;
    for (int i = lane; i < n_dw && !quiet; i += 64) {
        const int r = small_div(i, WD, inv_wd);
        const uint32_t* m = sS + i + 2 * r + SW + 1;
        const uint32_t burn = pack4(burning_flags(m[0]));
        const uint32_t front = pack4(flammable_flags(m[0])) & near_burning(m, SW);
        if (burn | front) {
            const uint4 w = group_words<true>(4 * i, t, ed.env_id, key);  // 4 i = r W + 4 (i - r WD)
            sU[4 * i + 0] = word_to_uniform(w.x);
            sU[4 * i + 1] = word_to_uniform(w.y);
            sU[4 * i + 2] = word_to_uniform(w.z);
            sU[4 * i + 3] = word_to_uniform(w.w);
        }
        my_front += __popc(front);
    }
    uint32_t n_front = 0;
    uint32_t slot = 0;
    if (__any(my_front != 0u)) slot = wave_exclusive_scan(my_front, n_front);
    if (my_front) {
        for (int i = lane; i < n_dw; i += 64) {
            const int r = small_div(i, WD, inv_wd);
            const uint32_t* m = sS + i + 2 * r + SW + 1;
            const uint32_t up6 = row_window(m[-SW - 1], m[-SW], m[-SW + 1]);
            const uint32_t md6 = row_window(m[-1], m[0], m[1]);
            const uint32_t dn6 = row_window(m[SW - 1], m[SW], m[SW + 1]);
            const uint32_t ud = up6 | dn6;
            const uint32_t near = (ud | (ud >> 1) | (ud >> 2) | md6 | (md6 >> 2)) & 0xFu;
            const uint32_t front = pack4(flammable_flags(m[0])) & near;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if ((front >> c) & 1u)
                    sL[slot++] = (uint32_t)(4 * i + c) | (direction_mask(up6, md6, dn6, c) << 16);
        }
    }
    if (n_front) {
        __syncthreads();
        for (uint32_t q = lane; q < n_front; q += 64) {
            const uint32_t entry = sL[q];
            const int v = entry & 0xFFFF;
            sD[v] = sU[v] < ignite_prob<WIND_CELL>(entry >> 16, base + v, W, F, A, lds_ew) ? 1 : 0;
        }
        __syncthreads();
    }

    // -- 4. new states and the BURNING count
    int cnt = 0;
    for (int i = lane; i < n_dw; i += 64) {
        const int r = small_div(i, WD, inv_wd);
        const uint32_t* m = sS + i + 2 * r + SW + 1;
        const uint32_t own = m[0];
        uint32_t out = own;
        const uint32_t burn = pack4(burning_flags(own));
        const uint32_t flam = pack4(flammable_flags(own));
        if (!quiet && (burn | flam)) {
            const uint32_t front = flam & near_burning(m, SW);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                uint32_t next;
                if ((burn >> c) & 1u)
                    next = sU[4 * i + c] < A.p_continue ? kBurning : kBurnt;
                else if ((front >> c) & 1u)
                    next = sD[4 * i + c] ? kBurning : kFlammable;
                else
                    continue;
                out = (out & ~(0xFFu << (8 * c))) | (next << (8 * c));
            }
        }
        sN[i] = out;
        cnt += __popc(pack4(burning_flags(out)));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);

    // -- 5. reward and done from the count (lane 0)
    if (lane == 0) {
        float rw = 0.0f;
        if (!a.done) {
            rw = -cfg.burn_penalty * (float)cnt;
            if (cnt == 0) rw = rw + cfg.extinguish_bonus;
            a.steps += 1;
            a.last_count = cnt;
            a.done = (cnt == 0 || a.steps >= cfg.max_steps) ? 1 : 0;
        }
        agents[e] = a;
        reward[e] = rw;
        done[e] = a.done;
        s_row = a.row;
        s_col = a.col;
    }
    __syncthreads();  // the new state and the agent's position

    // -- 6. the new state to HBM (a quiet env without a drop is unchanged
    //       there), the observation window from LDS
    uint32_t* dst = reinterpret_cast<uint32_t*>(states + base);
    if (!quiet || drop >= 0)
        for (int i = lane; i < n_dw; i += 64) dst[i] = sN[i];
    const int R = cfg.obs_radius, side = 2 * R + 1, n_obs = side * side;
    const float inv_side = 1.0f / (float)side;
    uint8_t* o = obs + (int64_t)e * n_obs;
    for (int i = lane; i < n_obs; i += 64) {
        const int di = small_div(i, side, inv_side);
        const int gi = s_row - R + di, gj = s_col - R + (i - di * side);
        o[i] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? (uint8_t)(sN[gi * WD + (gj >> 2)] >> (8 * (gj & 3)))
                                                        : kOutside;
    }
}

}  // namespace

hipError_t launch_rl_step_fused(hipStream_t s, const EnvDev* envs, int32_t n_env, const StaticFields& F,
                                const StepArgs& A, const RlFusedShape& shape, uint8_t* states, RlAgent* agents,
                                const int32_t* actions, const RlConfigDev& cfg, uint32_t t, uint8_t* obs,
                                float* reward, int32_t* done)
{
    if (n_env <= 0) return hipSuccess;
    if (!shape.fits) return hipErrorInvalidValue;
    const size_t lds = rl_fused_lds_bytes(shape);
    if (F.wind)
        hipLaunchKernelGGL((rl_step_kernel<true>), dim3(n_env), dim3(64), lds, s, envs, F, A, states, agents, actions,
                           cfg, t, shape.frame_cap, shape.cell_cap, obs, reward, done);
    else
        hipLaunchKernelGGL((rl_step_kernel<false>), dim3(n_env), dim3(64), lds, s, envs, F, A, states, agents,
                           actions, cfg, t, shape.frame_cap, shape.cell_cap, obs, reward, done);
    return hipGetLastError();
}

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
