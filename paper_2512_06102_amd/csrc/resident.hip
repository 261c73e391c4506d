// resident.hip -- T stochastic steps in one launch for batches of small envs,
// each env resident in LDS for the whole call.
//
// One workgroup (64, 256, 512 or 1024 lanes) per env holds the env's state as
// two framed buffers (before and after the step; (H + 2) x (W/4 + 2) dwords
// with a zero frame), its fuel term and elevation (read from HBM once per
// call) and the step's uniforms and front list, and advances it T steps.
// Every step is the one of the step kernels (the paper's section 3, Eqs. 1-4
// and the "Stochastic update"): the step's drop on F_t, one Philox draw per
// cell at counter (n >> 2, t, env_id, 0) for the 4-cell groups that hold a
// burning or a front cell, the ignition probability of each front cell with
// the same per-cell pieces and fp32 operation order (stepcell.hpp), the
// transition and the BURNING count of the env after the step, so the results
// are bit-identical.
//
// Each wave owns a contiguous run of the env's dwords and takes them through
// the whole step on its own: one pass draws, writes the burning cells'
// transitions into F_{t+1} and lists the front cells with their uniforms;
// the wave's 64 lanes then evaluate that list together and write each
// ignition as a byte of F_{t+1}.  A wave reads only F_t (stable for the step)
// besides what it wrote itself, so a step costs one workgroup barrier
// (F_{t+1} complete before it becomes F_t), plus one after a drop.
// The drops and per-env wind exponents of kChunk steps are staged in LDS at
// once, so no step waits on HBM; per-wave prefix sums and counts go through
// ballots instead of lane shuffles.
#include "devmath.hpp"
#include "framed.hpp"
#include "internal.hpp"
#include "resident.hpp"
#include "stepcell.hpp"

namespace firesim {
namespace {

// Orders one wave's LDS writes before its later LDS reads by other lanes of
// the same wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix over the wave's lanes of x >= 0 and the wave total, bit
// plane by bit plane (one ballot and one masked popcount per bit of the
// largest x).
__device__ __forceinline__ uint32_t ballot_exclusive_scan(uint32_t x, uint32_t& total)
{
    const uint64_t below = (1ull << (threadIdx.x & 63)) - 1ull;
    uint32_t pre = 0, tot = 0;
    for (int b = 0;; ++b) {
        const uint64_t any = __ballot(x >> b);
        if (any == 0) break;
        const uint64_t bit = __ballot((x >> b) & 1u);
        pre += (uint32_t)__popcll(bit & below) << b;
        tot += (uint32_t)__popcll(bit) << b;
    }
    total = tot;
    return pre;
}

// Wave-wide sum of x >= 0, bit plane by bit plane.
__device__ __forceinline__ uint32_t ballot_sum(uint32_t x)
{
    uint32_t tot = 0;
    for (int b = 0;; ++b) {
        const uint64_t any = __ballot(x >> b);
        if (any == 0) break;
        tot += (uint32_t)__popcll(__ballot((x >> b) & 1u)) << b;
    }
    return tot;
}

constexpr int kChunk = 64;  // steps of drops and wind exponents staged at once

template <int NT, bool WIND_CELL>
__global__ __launch_bounds__(NT) void stoch_resident_kernel(
    const EnvDev* __restrict__ envs, const int32_t* __restrict__ env_list, StaticFields F0, StepArgs A,
    const uint8_t* src_states, uint8_t* dst_states, const int32_t* __restrict__ actions,
    int32_t* __restrict__ counts, int32_t n_env, const uint32_t* __restrict__ t_base, uint32_t step0, int32_t T,
    int32_t frame_cap, int32_t cell_cap)
{
    constexpr int NW = NT / 64;
    extern __shared__ uint4 lds_dyn[];
    __shared__ float s_ew[kChunk][8];  // per-env wind exponents of the chunk's steps
    __shared__ int32_t s_act[kChunk];  // the chunk's drops
    __shared__ uint32_t s_count[3];    // BURNING cells after step k, in slot k % 3
    const int e = env_list ? env_list[blockIdx.x] : (int)blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const EnvDev ed = envs[e];
    const int H = ed.H, W = ed.W, WD = W >> 2, SW = WD + 2, n_dw = H * WD;
    const float inv_wd = 1.0f / (float)WD;
    const int64_t base = ed.offset;
    const uint32_t t0 = *t_base + step0;
    uint32_t* cur = reinterpret_cast<uint32_t*>(lds_dyn);  // F_t, framed
    uint32_t* nxt = cur + frame_cap;                        // F_{t+1}, framed
    float* sG = reinterpret_cast<float*>(nxt + frame_cap);  // fuel term g(v)
    float* sE = sG + cell_cap;                              // elevation
    // front list: (cell | its 3x3 burning window << 16, the cell's Philox
    // word >> 8); the window holds bits c..c+2 of the up, middle and down row
    // windows of the cell's dword (c = cell & 3)
    uint2* sL = reinterpret_cast<uint2*>(sE + cell_cap);

    // this wave's dwords [d_lo, d_hi) and front-list segment (4 d_lo onwards)
    const int per_wave = (n_dw + NW - 1) / NW;
    const int d_lo = min(wv * per_wave, n_dw), d_hi = min(d_lo + per_wave, n_dw);

    // state, fuel and elevation into LDS; zero frames around both buffers
    {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(src_states + base);
        for (int i = tid; i < n_dw; i += NT) {
            const int r = small_div(i, WD, inv_wd);
            cur[i + 2 * r + SW + 1] = src[i];
        }
        const float4* g4 = reinterpret_cast<const float4*>(F0.g + base);
        const float4* e4 = reinterpret_cast<const float4*>(F0.E + base);
        for (int i = tid; i < n_dw; i += NT) {
            reinterpret_cast<float4*>(sG)[i] = g4[i];
            reinterpret_cast<float4*>(sE)[i] = e4[i];
        }
        for (int i = tid; i < 2 * SW; i += NT) {
            const int f = i < SW ? i : (H + 1) * SW + (i - SW);
            cur[f] = 0u;
            nxt[f] = 0u;
        }
        for (int i = tid; i < 2 * H; i += NT) {
            const int f = (1 + (i >> 1)) * SW + ((i & 1) ? SW - 1 : 0);
            cur[f] = 0u;
            nxt[f] = 0u;
        }
        if (tid < 3) s_count[tid] = 0u;
        // a static per-env wind gives every step the same exponents
        if (!WIND_CELL && !F0.env_wind && tid < 8)
            s_ew[0][tid] = wind_exponent(tid, A.alpha_w1, A.alpha_w2, ed.V, ed.Vx, ed.Vy);
    }
    const uint2 key = make_uint2(A.key0, A.key1);
    const bool ew_series = !WIND_CELL && F0.env_wind != nullptr;

    bool stopped = false;  // left the step loop early: every remaining step is a no-op
    for (int32_t k = 0; k < T; ++k) {
        const uint32_t t = t0 + (uint32_t)k;
        const int slot = k % 3, kc = k % kChunk;
        StaticFields F = F0;
        if (F0.wind_stride != 0) F.wind = F0.wind + (int64_t)t * F0.wind_stride;
        if (kc == 0 && (actions || ew_series)) {
            // stage the next kChunk steps' drops and wind exponents
            if (k > 0) __syncthreads();  // the last chunk's entries are read
            const int nk = min(kChunk, T - k);
            if (actions)
                for (int j = tid; j < nk; j += NT) s_act[j] = actions[(int64_t)(k + j) * n_env + e];
            if (ew_series)
                for (int q = tid; q < nk * 8; q += NT) {
                    const int j = q >> 3, d = q & 7;
                    const float* w = F0.env_wind + ((int64_t)(t + j) * F0.n_env + e) * 3;
                    s_ew[j][d] = wind_exponent(d, A.alpha_w1, A.alpha_w2, w[0], w[1], w[2]);
                }
        }
        __syncthreads();  // F_t complete, the chunk staged, the last step's count summed
        // the last step's count: read by every thread in this barrier phase;
        // the slot step k + 1 adds to (step k - 2's, read in the last phase)
        // is cleared meanwhile
        const uint32_t prev = s_count[(slot + 2) % 3];
        if (tid == 0) {
            if (counts && k > 0) counts[(int64_t)(k - 1) * n_env + e] = (int32_t)prev;
            s_count[(slot + 1) % 3] = 0u;
        }
        // F_t holds no BURNING cell: no cell can ignite or burn out any more,
        // only the drops can still change it (the counts of the remaining
        // steps stay 0 as cleared before the launch)
        const bool quiet = k > 0 && prev == 0u;
        if (quiet && !actions) {
            stopped = true;
            break;
        }
        const float* ew = s_ew[ew_series ? kc : 0];

        // -- the step's drop on F_t
        const int32_t act = actions ? s_act[kc] : -1;
        if (act >= 0) {
            const int ar = (act >> 16) & 0x7FFF, ac = act & 0xFFFF;
            if (ar < H && ac < W) {
                const int R = A.drop_radius;
                const int r0 = max(ar - R, 0), r1 = min(ar + R, H - 1);
                const int c0 = max(ac - R, 0) >> 2, c1 = min(ac + R, W - 1) >> 2;
                const int nd = c1 - c0 + 1;
                for (int q = tid; q < (r1 - r0 + 1) * nd; q += NT) {
                    const int r = r0 + q / nd, cd = c0 + q % nd;
                    uint32_t* p = cur + (r + 1) * SW + cd + 1;
                    *p = apply_drop(*p, r, 4 * cd, ar, ac, R, A.drop_mode);
                }
                __syncthreads();
            }
        }
        if (quiet) continue;  // F_{t+1} is F_t after the drop: cur keeps it

        // -- this wave's dwords: draws, the burning cells' transitions into
        //    F_{t+1} (front cells left FLAMMABLE there), the front list
        uint32_t cnt = 0;  // BURNING cells of F_{t+1} found by this lane
        uint32_t n_front = 0;
        for (int i0 = d_lo; i0 < d_hi; i0 += 64) {
            const int i = i0 + lane;
            uint32_t front = 0, up6 = 0, md6 = 0, dn6 = 0;
            uint4 w = make_uint4(0u, 0u, 0u, 0u);
            if (i < d_hi) {
                const int r = small_div(i, WD, inv_wd);
                const int f = i + 2 * r + SW + 1;
                const uint32_t* m = cur + f;
                up6 = row_window(m[-SW - 1], m[-SW], m[-SW + 1]);
                md6 = row_window(m[-1], m[0], m[1]);
                dn6 = row_window(m[SW - 1], m[SW], m[SW + 1]);
                const uint32_t ud = up6 | dn6;
                const uint32_t near = (ud | (ud >> 1) | (ud >> 2) | md6 | (md6 >> 2)) & 0xFu;
                const uint32_t own = m[0];
                const uint32_t burn = (md6 >> 1) & 0xFu;
                front = pack4(flammable_flags(own)) & near;
                uint32_t out = own;
                if (burn | front) {
                    w = group_words<true>(4 * i, t, ed.env_id, key);  // 4 i = r W + 4 (i - r WD)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (!((burn >> c) & 1u)) continue;
                        const bool stays = word_to_uniform(compu(w, c)) < A.p_continue;
                        out = (out & ~(0xFFu << (8 * c))) | ((stays ? kBurning : kBurnt) << (8 * c));
                        cnt += stays ? 1u : 0u;
                    }
                }
                nxt[f] = out;
            }
            uint32_t tot = 0;
            uint32_t slot = 4 * d_lo + n_front + ballot_exclusive_scan(__popc(front), tot);
            if (front) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if ((front >> c) & 1u) {
                        const uint32_t win = ((up6 >> c) & 7u) | (((md6 >> c) & 7u) << 3) | (((dn6 >> c) & 7u) << 6);
                        sL[slot++] = make_uint2((uint32_t)(4 * i + c) | (win << 16), compu(w, c) >> 8);
                    }
            }
            n_front += tot;
        }
        if (n_front) {
            wave_sync();
            // the wave's front cells, evaluated by its 64 lanes together; an
            // ignition sets the cell's byte of F_{t+1}
            for (uint32_t q = lane; q < n_front; q += 64) {
                const uint2 entry = sL[4 * d_lo + q];
                const int v = entry.x & 0xFFFF;
                const uint32_t win = entry.x >> 16;
                const uint32_t nbk = direction_mask(win & 7u, (win >> 3) & 7u, (win >> 6) & 7u, 0);
                float g_u[8], E_u[8], V_u[8], Vx_u[8], Vy_u[8];
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    g_u[d] = E_u[d] = V_u[d] = Vx_u[d] = Vy_u[d] = 0.0f;
                    if ((nbk >> d) & 1u) {
                        const int u = v - kDRow[d] * W - kDCol[d];
                        g_u[d] = sG[u];
                        E_u[d] = sE[u];
                        if constexpr (WIND_CELL) {
                            V_u[d] = F.wind[base + u];
                            Vx_u[d] = F.wind[F.n_cells + base + u];
                            Vy_u[d] = F.wind[2 * F.n_cells + base + u];
                        }
                    }
                }
                const float p = ignite_prob_of<WIND_CELL>(nbk, sG[v], sE[v], g_u, E_u, V_u, Vx_u, Vy_u, A, ew);
                if (word_to_uniform(entry.y << 8) < p) {
                    const int iv = v >> 2, r = small_div(iv, WD, inv_wd);
                    reinterpret_cast<uint8_t*>(nxt)[4 * (iv + 2 * r + SW + 1) + (v & 3)] = kBurning;
                    ++cnt;
                }
            }
        }
        cnt = ballot_sum(cnt);
        if (lane == 0 && cnt) atomicAdd(&s_count[slot], cnt);
        uint32_t* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    __syncthreads();
    if (tid == 0 && counts && !stopped) counts[(int64_t)(T - 1) * n_env + e] = (int32_t)s_count[(T - 1) % 3];
    uint32_t* dst = reinterpret_cast<uint32_t*>(dst_states + base);
    for (int i = tid; i < n_dw; i += NT) {
        const int r = small_div(i, WD, inv_wd);
        dst[i] = cur[i + 2 * r + SW + 1];
    }
}

template <int NT>
hipError_t set_lds_limit(int bytes)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&stoch_resident_kernel<NT, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&stoch_resident_kernel<NT, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
}

template <int NT>
hipError_t launch_nt(hipStream_t s, const EnvDev* envs, int32_t n_env, const int32_t* env_list, int32_t n_list,
                     const StaticFields& F, const StepArgs& A, const ResidentShape& shape, const uint8_t* src,
                     uint8_t* dst, const uint32_t* t_base, uint32_t step0, int32_t T, const int32_t* actions,
                     int32_t* counts)
{
    const size_t lds = resident_lds_bytes(shape);
    if (F.wind)  // per-cell wind (static or a series)
        hipLaunchKernelGGL((stoch_resident_kernel<NT, true>), dim3(n_list), dim3(NT), lds, s, envs, env_list, F, A,
                           src, dst, actions, counts, n_env, t_base, step0, T, shape.frame_cap, shape.cell_cap);
    else
        hipLaunchKernelGGL((stoch_resident_kernel<NT, false>), dim3(n_list), dim3(NT), lds, s, envs, env_list, F, A,
                           src, dst, actions, counts, n_env, t_base, step0, T, shape.frame_cap, shape.cell_cap);
    return hipGetLastError();
}

}  // namespace

hipError_t resident_set_lds_limit(int bytes)
{
    hipError_t e = set_lds_limit<64>(bytes);
    if (e == hipSuccess) e = set_lds_limit<256>(bytes);
    if (e == hipSuccess) e = set_lds_limit<512>(bytes);
    if (e == hipSuccess) e = set_lds_limit<1024>(bytes);
    return e;
}

hipError_t launch_stoch_resident(hipStream_t s, const EnvDev* envs, int32_t n_env, const int32_t* env_list,
                                 int32_t n_list, const StaticFields& F, const StepArgs& A, const ResidentShape& shape,
                                 int threads, const uint8_t* src, uint8_t* dst, const uint32_t* t_base,
                                 uint32_t step0, int32_t T, const int32_t* actions, int32_t* counts)
{
    if (!shape.fits || T < 1 || n_list < 1) return hipErrorInvalidValue;
#define RESIDENT_ARGS s, envs, n_env, env_list, n_list, F, A, shape, src, dst, t_base, step0, T, actions, counts
    switch (threads) {
    case 64: return launch_nt<64>(RESIDENT_ARGS);
    case 256: return launch_nt<256>(RESIDENT_ARGS);
    case 512: return launch_nt<512>(RESIDENT_ARGS);
    case 1024: return launch_nt<1024>(RESIDENT_ARGS);
    default: return hipErrorInvalidValue;
    }
#undef RESIDENT_ARGS
}

}  // namespace firesim
