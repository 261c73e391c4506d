// stepcell.hpp -- per-cell pieces of the stochastic step shared by the step
// kernels and the fused RL step: byte-SWAR state flags, burning-neighbour
// masks, the ignition probability of a front cell (Eqs. 1-4 of the paper,
// fixed fp32 operation order), the Philox words of a 4-cell group and the
// drops.  Every kernel that advances the fire goes through these, so their
// results agree bit for bit.
#pragma once

#include "devmath.hpp"
#include "internal.hpp"

namespace firesim {

// Byte-lane flags (bit 8b set for byte b); state codes are 0..3.
__device__ __forceinline__ uint32_t burning_flags(uint32_t w) { return (w >> 1) & ~w & 0x01010101u; }
__device__ __forceinline__ uint32_t flammable_flags(uint32_t w) { return w & ~(w >> 1) & 0x01010101u; }
// Gather the four byte-lane flags into bits 0..3.
__device__ __forceinline__ uint32_t pack4(uint32_t f) { return (f | (f >> 7) | (f >> 14) | (f >> 21)) & 0xFu; }

// Burning bits of a 6-cell row window: bit m <-> column (first own column - 1 + m).
__device__ __forceinline__ uint32_t row_window(uint32_t left, uint32_t own, uint32_t right)
{
    return ((burning_flags(left) >> 24) & 1u) | (pack4(burning_flags(own)) << 1) |
           ((burning_flags(right) & 1u) << 5);
}

// Burning-neighbour mask of own cell c: bit k set iff the source v - D_k burns.
__device__ __forceinline__ uint32_t direction_mask(uint32_t up6, uint32_t md6, uint32_t dn6, int c)
{
    return ((md6 >> c) & 1u) | (((dn6 >> c) & 1u) << 1) | (((dn6 >> (c + 1)) & 1u) << 2) |
           (((dn6 >> (c + 2)) & 1u) << 3) | (((md6 >> (c + 2)) & 1u) << 4) |
           (((up6 >> (c + 2)) & 1u) << 5) | (((up6 >> (c + 1)) & 1u) << 6) |
           (((up6 >> c) & 1u) << 7);
}

__device__ __forceinline__ uint32_t compu(const uint4& v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

// p_ignite of a target cell from its burning-neighbour mask (bit k: the
// source v - D_k burns), its own fuel term and elevation, and its sources'
// fuel, elevation and (per-cell) wind: lambda is summed in ascending
// direction order, then p = 1 - exp(-gamma lambda).
template <bool WIND_CELL>
__device__ __forceinline__ float ignite_prob_of(uint32_t nbk, float g_v, float E_v, const float (&g_u)[8],
                                                const float (&E_u)[8], const float (&V_u)[8],
                                                const float (&Vx_u)[8], const float (&Vy_u)[8],
                                                const StepArgs& A, const float* ew)
{
    float lambda = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!((nbk >> k) & 1u)) continue;
        float wexp;
        if constexpr (WIND_CELL)
            wexp = wind_exponent(k, A.alpha_w1, A.alpha_w2, V_u[k], Vx_u[k], Vy_u[k]);
        else
            wexp = ew[k];
        float slope = (E_v - E_u[k]) * ((k & 1) ? A.inv_run_diag : A.inv_run_orth);
        if (A.slope_mode) slope = atan_c(slope);  // the slope angle in radians
        const float x = wexp + A.alpha_s * slope;
        lambda = lambda + (A.p_base * g_u[k]) * exp_c(x);
    }
    if (!(lambda > 0.0f)) return 0.0f;
    const float gamma = A.alpha_gamma * g_v;
    return 1.0f - exp_c(-(gamma * lambda));
}

// p_ignite of target cell v (packed index) with its inputs read from HBM.
// The sources' fuel, elevation (and wind) are loaded together first so their
// latency is paid once.
template <bool WIND_CELL>
__device__ __forceinline__ float ignite_prob(uint32_t nbk, int64_t v, int W, const StaticFields& F,
                                             const StepArgs& A, const float* ew)
{
    float g_u[8], E_u[8], V_u[8], Vx_u[8], Vy_u[8];
    const float g_v = F.g[v], E_v = F.E[v];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        g_u[k] = E_u[k] = V_u[k] = Vx_u[k] = Vy_u[k] = 0.0f;
        if ((nbk >> k) & 1u) {
            const int64_t u = v - (int64_t)kDRow[k] * W - kDCol[k];
            g_u[k] = F.g[u];
            E_u[k] = F.E[u];
            if constexpr (WIND_CELL) {
                V_u[k] = F.wind[u];
                Vx_u[k] = F.wind[F.n_cells + u];
                Vy_u[k] = F.wind[2 * F.n_cells + u];
            }
        }
    }
    return ignite_prob_of<WIND_CELL>(nbk, g_v, E_v, g_u, E_u, V_u, Vx_u, Vy_u, A, ew);
}

// The four Philox words of a 4-cell group whose first cell has env-local
// index n0 (a group may straddle two counters when W % 4 != 0).
template <bool ALIGNED>
__device__ __forceinline__ uint4 group_words(int64_t n0, uint32_t t, uint32_t env_id, uint2 key)
{
    const uint4 w0 = philox4x32_10(make_uint4((uint32_t)(n0 >> 2), t, env_id, 0u), key);
    if constexpr (ALIGNED) {
        return w0;
    } else {
        const int64_t q0 = n0 >> 2;
        uint4 w1 = w0;
        if (((n0 + 3) >> 2) != q0)
            w1 = philox4x32_10(make_uint4((uint32_t)(q0 + 1), t, env_id, 0u), key);
        uint32_t w[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t n = n0 + c;
            w[c] = (n >> 2) == q0 ? compu(w0, (int)(n & 3)) : compu(w1, (int)(n & 3));
        }
        return make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Wave-wide exclusive scan of one 32-bit value per lane of a 64-lane wave;
// returns the lane's offset and the wave total.
__device__ __forceinline__ uint32_t wave_exclusive_scan(uint32_t x, uint32_t& total)
{
    const int lane = threadIdx.x & 63;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    total = __shfl(incl, 63);
    return incl - x;
}

// A drop on the (2R+1) x (2R+1) square centred at (ar, ac): mode 0 turns
// FLAMMABLE and BURNING cells UNBURNABLE (suppressant), mode 1 turns BURNING
// cells BURNT (water).
__device__ __forceinline__ uint32_t drop_cell(uint32_t s, int mode)
{
    if (mode == 0) return (s == kFlammable || s == kBurning) ? (uint32_t)kUnburnable : s;
    return s == kBurning ? (uint32_t)kBurnt : s;
}

// The drop on dword w (columns gj..gj+3 of row gi).
__device__ __forceinline__ uint32_t apply_drop(uint32_t w, int gi, int gj, int ar, int ac, int R, int mode)
{
    if (gi < ar - R || gi > ar + R) return w;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int j = gj + c;
        const uint32_t s = (w >> (8 * c)) & 0xFFu;
        if (j >= ac - R && j <= ac + R) w = (w & ~(0xFFu << (8 * c))) | (drop_cell(s, mode) << (8 * c));
    }
    return w;
}

}  // namespace firesim
