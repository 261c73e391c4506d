// resident.hip -- T stochastic steps in one launch for batches of small envs,
// each env's state resident in LDS for the whole call.
//
// One workgroup (256, 512 or 1024 lanes) per env holds the env in LDS as two framed buffers
// (the state before and after the step; (H + 2) x (W/4 + 2) dwords with a
// zero frame) and advances it T steps, with a workgroup barrier between the
// phases of a step instead of a launch per step.  Every step is the one of the
// step kernels (the paper's section 3, Eqs. 1-4 and the "Stochastic update"):
// the step's drop on F_t, one Philox draw per cell at counter (n >> 2, t,
// env_id, 0) for the 4-cell groups that hold a burning or a front cell, the
// ignition probability of each front cell with the same per-cell pieces and
// fp32 operation order (stepcell.hpp), the transition, and the BURNING count
// of the env after the step.  The results are therefore bit-identical.  The
// fuel, elevation and wind of front cells and their sources are read from
// HBM (the env's few kilobytes of them stay in L2 across the call).
#include "devmath.hpp"
#include "framed.hpp"
#include "internal.hpp"
#include "resident.hpp"
#include "stepcell.hpp"

namespace firesim {
namespace {

template <int NT, bool WIND_CELL>
__global__ __launch_bounds__(NT) void stoch_resident_kernel(
    const EnvDev* __restrict__ envs, StaticFields F0, StepArgs A, const uint8_t* src_states,
    uint8_t* dst_states, const int32_t* __restrict__ actions, int32_t* __restrict__ counts,
    int32_t n_env, const uint32_t* __restrict__ t_base, uint32_t step0, int32_t T, int32_t frame_cap,
    int32_t cell_cap)
{
    constexpr int kResidentThreads = NT;
    extern __shared__ uint4 lds_dyn[];
    __shared__ float lds_ew[8];
    __shared__ uint32_t s_wave[NT / 64];
    const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const EnvDev ed = envs[e];
    const int H = ed.H, W = ed.W, WD = W >> 2, SW = WD + 2, n_dw = H * WD;
    const float inv_wd = 1.0f / (float)WD;
    const int64_t base = ed.offset;
    const uint32_t t0 = *t_base + step0;
    uint32_t* cur = reinterpret_cast<uint32_t*>(lds_dyn);  // F_t, framed
    uint32_t* nxt = cur + frame_cap;                        // F_{t+1}, framed
    float* sU = reinterpret_cast<float*>(nxt + frame_cap);  // uniform of each cell that draws
    uint32_t* sL = reinterpret_cast<uint32_t*>(sU + cell_cap);  // front cells: cell | nbk << 16
    uint8_t* sD = reinterpret_cast<uint8_t*>(sL + cell_cap);    // ignition decision per front cell

    // the state into `cur`; zero frames around both buffers
    const uint32_t* src = reinterpret_cast<const uint32_t*>(src_states + base);
    for (int i = tid; i < n_dw; i += kResidentThreads) {
        const int r = small_div(i, WD, inv_wd);
        cur[i + 2 * r + SW + 1] = src[i];
    }
    for (int i = tid; i < 2 * SW; i += kResidentThreads) {
        const int f = i < SW ? i : (H + 1) * SW + (i - SW);
        cur[f] = 0u;
        nxt[f] = 0u;
    }
    for (int i = tid; i < 2 * H; i += kResidentThreads) {
        const int f = (1 + (i >> 1)) * SW + ((i & 1) ? SW - 1 : 0);
        cur[f] = 0u;
        nxt[f] = 0u;
    }
    const uint2 key = make_uint2(A.key0, A.key1);

    for (int32_t k = 0; k < T; ++k) {
        const uint32_t t = t0 + (uint32_t)k;
        StaticFields F = F0;
        if (F0.wind_stride != 0) F.wind = F0.wind + (int64_t)t * F0.wind_stride;
        if (!WIND_CELL && tid < 8) {
            float V = ed.V, Vx = ed.Vx, Vy = ed.Vy;
            if (F.env_wind) {
                const float* w = F.env_wind + ((int64_t)t * F.n_env + e) * 3;
                V = w[0];
                Vx = w[1];
                Vy = w[2];
            }
            lds_ew[tid] = wind_exponent(tid, A.alpha_w1, A.alpha_w2, V, Vx, Vy);
        }
        __syncthreads();  // cur complete (load or last step), lds_ew written

        // -- the step's drop on F_t
        const int32_t act = actions ? actions[(int64_t)k * n_env + e] : -1;
        if (act >= 0) {
            const int ar = (act >> 16) & 0x7FFF, ac = act & 0xFFFF;
            if (ar < H && ac < W) {
                const int R = A.drop_radius;
                const int r0 = max(ar - R, 0), r1 = min(ar + R, H - 1);
                const int d0 = max(ac - R, 0) >> 2, d1 = min(ac + R, W - 1) >> 2;
                const int nd = d1 - d0 + 1;
                for (int q = tid; q < (r1 - r0 + 1) * nd; q += kResidentThreads) {
                    const int r = r0 + q / nd, cd = d0 + q % nd;
                    uint32_t* p = cur + (r + 1) * SW + cd + 1;
                    *p = apply_drop(*p, r, 4 * cd, ar, ac, R, A.drop_mode);
                }
                __syncthreads();
            }
        }

        // -- draws of the groups that need one; front cells counted per lane
        uint32_t my_front = 0;
        for (int i = tid; i < n_dw; i += kResidentThreads) {
            const int r = small_div(i, WD, inv_wd);
            const uint32_t* m = cur + i + 2 * r + SW + 1;
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
        // workgroup-wide exclusive scan of the front counts
        uint32_t wave_total = 0;
        uint32_t slot = wave_exclusive_scan(my_front, wave_total);
        if (lane == 0) s_wave[wv] = wave_total;
        __syncthreads();
        uint32_t n_front = 0;
#pragma unroll
        for (int w = 0; w < kResidentThreads / 64; ++w) {
            const uint32_t c = s_wave[w];
            if (w < wv) slot += c;
            n_front += c;
        }
        if (n_front) {
            if (my_front) {
                for (int i = tid; i < n_dw; i += kResidentThreads) {
                    const int r = small_div(i, WD, inv_wd);
                    const uint32_t* m = cur + i + 2 * r + SW + 1;
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
            __syncthreads();
            // front cells evaluated by all lanes together
            for (uint32_t q = tid; q < n_front; q += kResidentThreads) {
                const uint32_t entry = sL[q];
                const int v = entry & 0xFFFF;
                sD[v] = sU[v] < ignite_prob<WIND_CELL>(entry >> 16, base + v, W, F, A, lds_ew) ? 1 : 0;
            }
            __syncthreads();
        }

        // -- F_{t+1} and its BURNING count
        int cnt = 0;
        for (int i = tid; i < n_dw; i += kResidentThreads) {
            const int r = small_div(i, WD, inv_wd);
            const uint32_t* m = cur + i + 2 * r + SW + 1;
            const uint32_t own = m[0];
            uint32_t out = own;
            const uint32_t burn = pack4(burning_flags(own));
            const uint32_t flam = pack4(flammable_flags(own));
            if (burn | flam) {
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
            nxt[i + 2 * r + SW + 1] = out;
            cnt += __popc(pack4(burning_flags(out)));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
        __syncthreads();  // every lane has read the scan totals and written nxt
        if (lane == 0) s_wave[wv] = (uint32_t)cnt;
        __syncthreads();
        if (counts && tid == 0) {
            uint32_t total = 0;
#pragma unroll
            for (int w = 0; w < kResidentThreads / 64; ++w) total += s_wave[w];
            counts[(int64_t)k * n_env + e] = (int32_t)total;
        }
        uint32_t* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    __syncthreads();
    uint32_t* dst = reinterpret_cast<uint32_t*>(dst_states + base);
    for (int i = tid; i < n_dw; i += kResidentThreads) {
        const int r = small_div(i, WD, inv_wd);
        dst[i] = cur[i + 2 * r + SW + 1];
    }
}

template <int NT>
hipError_t launch_nt(hipStream_t s, const EnvDev* envs, int32_t n_env, const StaticFields& F, const StepArgs& A,
                     const ResidentShape& shape, const uint8_t* src, uint8_t* dst, const uint32_t* t_base,
                     uint32_t step0, int32_t T, const int32_t* actions, int32_t* counts)
{
    const size_t lds = resident_lds_bytes(shape);
    if (F.wind)  // per-cell wind (static or a series)
        hipLaunchKernelGGL((stoch_resident_kernel<NT, true>), dim3(n_env), dim3(NT), lds, s, envs, F, A, src, dst,
                           actions, counts, n_env, t_base, step0, T, shape.frame_cap, shape.cell_cap);
    else
        hipLaunchKernelGGL((stoch_resident_kernel<NT, false>), dim3(n_env), dim3(NT), lds, s, envs, F, A, src, dst,
                           actions, counts, n_env, t_base, step0, T, shape.frame_cap, shape.cell_cap);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stoch_resident(hipStream_t s, const EnvDev* envs, int32_t n_env, const StaticFields& F,
                                 const StepArgs& A, const ResidentShape& shape, int threads, const uint8_t* src,
                                 uint8_t* dst, const uint32_t* t_base, uint32_t step0, int32_t T,
                                 const int32_t* actions, int32_t* counts)
{
    if (!shape.fits || T < 1) return hipErrorInvalidValue;
    switch (threads) {
    case 256: return launch_nt<256>(s, envs, n_env, F, A, shape, src, dst, t_base, step0, T, actions, counts);
    case 512: return launch_nt<512>(s, envs, n_env, F, A, shape, src, dst, t_base, step0, T, actions, counts);
    case 1024: return launch_nt<1024>(s, envs, n_env, F, A, shape, src, dst, t_base, step0, T, actions, counts);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace firesim
