// stoch.hip -- the stochastic fire-spread step and the set-up kernels.
//
// Model (JaxWildfire, arXiv 2512.06102, section 3): a FLAMMABLE cell v
// ignites with p = 1 - exp(-gamma(v) lambda(v)) (Eq. 4), where lambda sums
// phi(u, D_{u->v}) over its BURNING Moore neighbours u (Eq. 3, with the wind
// and slope factors of Eqs. 1-2 evaluated at the source u), and gamma(v) =
// alpha_gamma (1 + mu_veg(v)) (1 + mu_den(v)); a BURNING cell keeps burning
// with p_continue, else becomes BURNT ("Stochastic update").  All draws of a
// step use the state before it (synchronous update).
//
// One step is one launch of 64-lane workgroups (one wave64 each).  A
// workgroup owns a tile of one env: `width` (64/128/256) columns by
// (256/width) * RT rows.  Lane (tx, ty) owns the 4-cell column group at
// column c0 + 4 tx (one dword of uint8 states) in the RT consecutive rows
// r0 + ty RT + m.
//  1. Each lane loads its RT state dwords and the dwords directly above and
//     below them (those repeats hit L2: the neighbouring lanes load the same
//     lines), and in the dense plan the fuel term and elevation of its cells
//     (the step's 10 bytes per cell).  The left / right neighbour bytes come
//     from the adjacent lanes of the row segment by a lane shuffle; only the
//     segment's end lanes load the halo byte beyond the tile.  Nothing is
//     staged in LDS and no barrier waits on the loads.
//  2. A suppression drop, if any, is applied to the loaded dwords.
//  3. Burning / flammable flags come four cells at a time from byte SWAR.
//     Front cells (flammable with a burning neighbour) and 4-cell groups that
//     need a draw (a front or burning cell) are counted, scanned across the
//     wave and listed in LDS.
//  4. The wave then works through the lists: one Philox block per listed
//     group, then lambda and p of each listed front cell (its neighbours'
//     fuel and elevation loaded together, then the ordered sum of phi).  Fires
//     cover a few percent of the cells, so packing their arithmetic onto every
//     lane, instead of leaving it to the lanes that own the cells, keeps the
//     step at memory speed.  A wave whose lists would overflow falls back to
//     each lane handling its own cells.
//  5. Owners assemble the new dwords and store them (nontemporal in the
//     dense plan); the BURNING count is reduced across the wave and added
//     to the env's counter with one atomic.
// Workgroup b runs on XCD b % 8; tiles are dealt so that each XCD walks a
// contiguous run of the tile list (neighbouring tiles share lines in that
// XCD's L2).
#include "devmath.hpp"
#include "internal.hpp"
#include "stepcell.hpp"

namespace firesim {
namespace {

constexpr int kWave = 64;
constexpr int kCellCap = 256;    // listed front cells per wave
constexpr int kGroupCap = 128;   // listed 4-cell groups per wave

__device__ __forceinline__ void keep_loaded(const float4& v)
{
    asm volatile("" ::"v"(v.x), "v"(v.y), "v"(v.z), "v"(v.w));
}

// x of lane - 1 / lane + 1 of the wave by a DPP wave shift (0 where that
// lane does not exist); every lane must be active
__device__ __forceinline__ uint32_t from_lane_below(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_lane_above(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130 /* wave_shl:1 */, 0xF, 0xF, false);
}

constexpr int bit_width(int v) { return v == 0 ? 0 : 1 + bit_width(v >> 1); }

// Exclusive prefix sum across the wave of a per-lane value below 2^NB, and
// the wave total: one ballot per bit plane (no LDS round trips)
template <int NB>
__device__ __forceinline__ uint32_t ballot_exclusive_scan(uint32_t x, uint32_t& total)
{
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const uint64_t m = __ballot((x >> b) & 1u);
        off += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
        tot += (uint32_t)__popcll(m) << b;
    }
    total = tot;
    return off;
}

// Wave total of a per-lane value below 2^NB
template <int NB>
__device__ __forceinline__ uint32_t ballot_sum(uint32_t x)
{
    uint32_t tot = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) tot += (uint32_t)__popcll(__ballot((x >> b) & 1u)) << b;
    return tot;
}

// State dword of the 4-cell group at (gi, gj); 0 (not burning) off the grid.
template <bool ALIGNED>
__device__ __forceinline__ uint32_t load_group(const uint8_t* __restrict__ env_src, int gi, int gj, int H,
                                               int W)
{
    if (gi < 0 || gi >= H || gj >= W) return 0u;
    const uint8_t* p = env_src + (uint32_t)(gi * W + gj);  // envs hold < 2^30 cells
    if constexpr (ALIGNED) {
        return *reinterpret_cast<const uint32_t*>(p);
    } else {
        uint32_t v = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (gj + c < W) v |= (uint32_t)p[c] << (8 * c);
        return v;
    }
}

// Waves per SIMD the front-skipping kernels with up to 4 rows per lane are
// compiled for: with per-env wind they fit 64 VGPRs without spilling, so 8
// waves share each SIMD (7 at the compiler's own choice of 65), and with
// per-cell wind 80 (6 waves instead of 5).  These plans wait on chains of
// dependent loads, and the extra wave hides latency (6.6% faster on 1024
// envs of 256x256).  The dense plan streams instead and runs slower when
// capped, and 8 rows per lane would spill: both keep the compiler's choice.
constexpr int step_waves_per_eu(bool wind_cell, int rt, bool skip)
{
    return (skip && rt <= 4) ? (wind_cell ? 6 : 8) : 1;
}

template <bool ALIGNED, bool WIND_CELL, int RT, bool SKIP>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(step_waves_per_eu(WIND_CELL, RT, SKIP))))
void stoch_step_kernel(
    const TileDesc* __restrict__ tiles, int32_t n_tiles, int32_t tiles_per_xcd,
    const EnvDev* __restrict__ envs, StaticFields F0, StepArgs A, const uint8_t* __restrict__ src,
    uint8_t* __restrict__ dst, const uint32_t* __restrict__ t_base, uint32_t step,
    const int32_t* __restrict__ actions_row, int32_t* __restrict__ counts_row, SparseArgs SP)
{
    __shared__ uint32_t lds_cell[kCellCap];   // lane | m << 6 | c << 9 | 3x3 window << 11 | group << 20
    __shared__ uint16_t lds_group[kGroupCap]; // lane | m << 6
    __shared__ float lds_u[kGroupCap * 4];    // uniforms of each listed group's cells
    __shared__ uint8_t lds_dec[kCellCap];     // ignition decision of each listed cell
    __shared__ float lds_ew[8];

    const int b = blockIdx.x;
    const int tile = (b & 7) * tiles_per_xcd + (b >> 3);
    if (tile >= n_tiles) return;
    const int lane = threadIdx.x;
    const TileDesc td = tiles[tile];
    const EnvDev ed = envs[td.env];  // issued early; an inactive tile does not wait for it
    const int gx_log = td.width == 256 ? 6 : (td.width == 128 ? 5 : (td.width == 64 ? 4 : (td.width == 32 ? 3 : 2)));
    const int GX = 1 << gx_log;  // lanes per row segment
    const int tx = lane & (GX - 1), ty = lane >> gx_log;
    const int row0 = td.r0 + ty * RT;  // first own row
    const int gj0 = td.c0 + 4 * tx;    // first own column

    // -- 0. sparse scheduling: a tile runs when it or one of its 8 neighbours
    //       held a burning cell after the previous step (those tiles marked
    //       it), when a drop may reach it, or on the first step of a call;
    //       an inactive tile keeps its cells.  Each tile clears its own mark
    //       once read, so the array takes the marks of the step after next.
    if (SP.burn_next) {
        bool active = SP.all_active != 0 || SP.burn_prev[tile] != 0;
        if (lane == 0) SP.burn_prev[tile] = 0;
        const int32_t a0 = (!active && actions_row) ? actions_row[td.env] : -1;
        if (a0 >= 0) {
            // the drop square reaches the tile or its one-cell ring (a drop
            // off the grid changes nothing: running the tile is still exact)
            const int ar = (a0 >> 16) & 0x7FFF, ac = a0 & 0xFFFF;
            const int R = A.drop_radius, TH = (kWave >> gx_log) * RT;
            active = ar + R >= td.r0 - 1 && ar - R <= td.r0 + TH && ac + R >= td.c0 - 1 &&
                     ac - R <= td.c0 + td.width;
        }
        if (!active) {
            if (SP.eq[tile] == 0) {  // the other buffer is stale on this tile: copy it over
                const EnvDev& ed0 = ed;
                const int H0 = ed0.H, W0 = ed0.W;
#pragma unroll
                for (int m = 0; m < RT; ++m) {
                    const int gi = row0 + m;
                    if (!(gi < H0 && gj0 < W0)) continue;
                    const int64_t c0 = ed0.offset + (int64_t)gi * W0 + gj0;
                    if constexpr (ALIGNED) {
                        *reinterpret_cast<uint32_t*>(dst + c0) = *reinterpret_cast<const uint32_t*>(src + c0);
                    } else {
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            if (gj0 + c < W0) dst[c0 + c] = src[c0 + c];
                    }
                }
            }
            if (lane == 0) SP.eq[tile] = 1;
            return;
        }
    }

    const int H = ed.H, W = ed.W;
    const uint32_t t = *t_base + step;
    StaticFields F = F0;
    if (F0.wind_stride != 0) F.wind = F0.wind + (int64_t)t * F0.wind_stride;
    const int64_t base = ed.offset;
    const uint8_t* env_src = src + base;
    const uint2 key = make_uint2(A.key0, A.key1);

    // -- 1. loads: RT own dwords plus the one above and below; halo bytes at
    //       the segment ends; fuel and elevation of own cells (dense plan)
    uint32_t s[RT + 2], hl[RT + 2], hr[RT + 2];
    if constexpr (ALIGNED) {
        // branch-free: every lane loads from a clamped in-grid address and
        // zeroes what lies off the grid (W % 4 == 0, so W >= 4)
        const int gjc = min(gj0, W - 4);
#pragma unroll
        for (int j = 0; j < RT + 2; ++j) {
            const int gi = row0 - 1 + j, gic = min(max(gi, 0), H - 1);
            const uint32_t w = *reinterpret_cast<const uint32_t*>(env_src + (uint32_t)(gic * W + gjc));
            s[j] = (gi >= 0 && gi < H && gj0 < W) ? w : 0u;
        }
    } else {
#pragma unroll
        for (int j = 0; j < RT + 2; ++j) s[j] = load_group<ALIGNED>(env_src, row0 - 1 + j, gj0, H, W);
    }
    const int cl = td.c0 - 1, cr = td.c0 + td.width;
#pragma unroll
    for (int j = 0; j < RT + 2; ++j) {
        const int gi = row0 - 1 + j;
        const bool row_in = gi >= 0 && gi < H;
        hl[j] = (tx == 0 && row_in && cl >= 0) ? (uint32_t)env_src[(uint32_t)(gi * W + cl)] : 0u;
        hr[j] = (tx == GX - 1 && row_in && cr < W) ? (uint32_t)env_src[(uint32_t)(gi * W + cr)] : 0u;
    }
    float4 gv[RT], ev[RT];
#pragma unroll
    for (int m = 0; m < RT; ++m) {
        gv[m] = make_float4(0.f, 0.f, 0.f, 0.f);
        ev[m] = gv[m];
        if constexpr (!SKIP) {
            const int gi = row0 + m;
            if (ALIGNED || (gi < H && gj0 < W)) {
                const int64_t c0 = base + (int64_t)gi * W + gj0;
                if constexpr (ALIGNED) {
                    // uniform env bases plus 32-bit byte offsets (envs hold < 2^30
                    // cells), clamped into the grid so that no lane branches
                    const uint32_t bo = 4u * (uint32_t)(min(gi, H - 1) * W + min(gj0, W - 4));
                    gv[m] = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(F.g + base) + bo);
                    ev[m] = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(F.E + base) + bo);
                    if constexpr (WIND_CELL) {
                        keep_loaded(*reinterpret_cast<const float4*>(reinterpret_cast<const char*>(F.wind + base) + bo));
                        keep_loaded(*reinterpret_cast<const float4*>(
                            reinterpret_cast<const char*>(F.wind + F.n_cells + base) + bo));
                        keep_loaded(*reinterpret_cast<const float4*>(
                            reinterpret_cast<const char*>(F.wind + 2 * F.n_cells + base) + bo));
                    }
                } else {
                    float tg[4] = {0.f, 0.f, 0.f, 0.f}, te[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (gj0 + c < W) {
                            tg[c] = F.g[c0 + c];
                            te[c] = F.E[c0 + c];
                        }
                    gv[m] = make_float4(tg[0], tg[1], tg[2], tg[3]);
                    ev[m] = make_float4(te[0], te[1], te[2], te[3]);
                }
            }
        }
    }
    if constexpr (!SKIP) {
        // the loaded values are not needed by this lane (front cells reload
        // through the cache), only their arrival
#pragma unroll
        for (int m = 0; m < RT; ++m) {
            keep_loaded(gv[m]);
            keep_loaded(ev[m]);
        }
    }
    if constexpr (!WIND_CELL) {
        if (lane < 8) {
            float V = ed.V, Vx = ed.Vx, Vy = ed.Vy;
            if (F.env_wind) {
                const float* w = F.env_wind + ((int64_t)t * F.n_env + td.env) * 3;
                V = w[0];
                Vx = w[1];
                Vy = w[2];
            }
            lds_ew[lane] = wind_exponent(lane, A.alpha_w1, A.alpha_w2, V, Vx, Vy);
        }
    }

    // -- 2. suppression drop on the loaded dwords and halo bytes, before the step
    const int32_t act = actions_row ? actions_row[td.env] : -1;
    if (act >= 0) {
        const int ar = (act >> 16) & 0x7FFF, ac = act & 0xFFFF;
        if (ar < H && ac < W) {
            const int R = A.drop_radius, mode = A.drop_mode;
#pragma unroll
            for (int j = 0; j < RT + 2; ++j) {
                const int gi = row0 - 1 + j;
                s[j] = apply_drop(s[j], gi, gj0, ar, ac, R, mode);
                if (gi >= ar - R && gi <= ar + R) {
                    if (cl >= ac - R && cl <= ac + R) hl[j] = drop_cell(hl[j], mode);
                    if (cr >= ac - R && cr <= ac + R) hr[j] = drop_cell(hr[j], mode);
                }
            }
        }
    }

    // -- 2b. no burning cell in the tile or its one-cell halo: no cell of the
    //        tile can change (a drop only removes fire); store the state and stop
    {
        uint32_t any_burn = 0;
#pragma unroll
        for (int j = 0; j < RT + 2; ++j) any_burn |= burning_flags(s[j]) | burning_flags(hl[j]) | burning_flags(hr[j]);
        if (!__any(any_burn != 0u)) {
#pragma unroll
            for (int m = 0; m < RT; ++m) {
                const int gi = row0 + m;
                if (!(gi < H && gj0 < W)) continue;
                uint8_t* o = (dst + base) + (uint32_t)(gi * W + gj0);
                if constexpr (ALIGNED && !SKIP) {
                    __builtin_nontemporal_store(s[m + 1], reinterpret_cast<uint32_t*>(o));
                } else if constexpr (ALIGNED) {
                    *reinterpret_cast<uint32_t*>(o) = s[m + 1];
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (gj0 + c < W) o[c] = (uint8_t)(s[m + 1] >> (8 * c));
                }
            }
            if (SP.burn_next && lane == 0) SP.eq[tile] = 0;
            return;
        }
    }

    // -- 3. neighbour dwords across the row segment, then flags of own cells:
    //       burning (bits 0-3) and front (bits 4-7)
    uint32_t win[RT + 2];  // burning bits of the 6-cell window of each loaded row
#pragma unroll
    for (int j = 0; j < RT + 2; ++j) {
        // the segment's end lanes take the halo bytes instead
        uint32_t left = from_lane_below(s[j]), right = from_lane_above(s[j]);
        if (tx == 0) left = hl[j] << 24;
        if (tx == GX - 1) right = hr[j];
        win[j] = row_window(left, s[j], right);
    }
    uint32_t flags[RT];
    uint32_t my_cells = 0, my_groups = 0;
#pragma unroll
    for (int m = 0; m < RT; ++m) {
        flags[m] = 0;
        if (!(row0 + m < H && gj0 < W)) continue;
        const uint32_t up6 = win[m], md6 = win[m + 1], dn6 = win[m + 2];
        const uint32_t ud = up6 | dn6;
        const uint32_t near = (ud | (ud >> 1) | (ud >> 2) | md6 | (md6 >> 2)) & 0xFu;
        const uint32_t burn = pack4(burning_flags(s[m + 1]));
        const uint32_t front = pack4(flammable_flags(s[m + 1])) & near;
        flags[m] = burn | (front << 4);
        my_cells += __popc(front);
        my_groups += (burn | front) != 0u;
    }
    // the row windows, 6 bits each, packed five to a register for the list
    // and the overflow path after the scan (the empty asm keeps the compiler
    // from reading the unpacked copies instead, which would hold one
    // register per row until the end of the kernel)
    constexpr int kWinRegs = (RT + 2 + 4) / 5;
    uint32_t wpk[kWinRegs];
#pragma unroll
    for (int i = 0; i < kWinRegs; ++i) wpk[i] = 0;
#pragma unroll
    for (int j = 0; j < RT + 2; ++j) wpk[j / 5] |= win[j] << (6 * (j % 5));
#pragma unroll
    for (int i = 0; i < kWinRegs; ++i) asm volatile("" : "+v"(wpk[i]));
    auto row_win = [&](int j) { return (wpk[j / 5] >> (6 * (j % 5))) & 0x3Fu; };
    __syncthreads();  // lds_ew visible (one wave: no waiting on other waves)

    // -- 4. list front cells and draw groups across the wave
    constexpr int kCellBits = bit_width(4 * RT), kGroupBits = bit_width(RT);
    uint32_t totals = 0, off = 0;
    if (__any(my_groups != 0u)) {
        uint32_t tc, tg;
        const uint32_t oc = ballot_exclusive_scan<kCellBits>(my_cells, tc);
        const uint32_t og = ballot_exclusive_scan<kGroupBits>(my_groups, tg);
        off = oc | (og << 16);
        totals = tc | (tg << 16);
    }
    const uint32_t n_cells = totals & 0xFFFFu, n_groups = totals >> 16;
    const bool listed = n_cells <= (uint32_t)kCellCap && n_groups <= (uint32_t)kGroupCap;
    uint32_t slot[RT];  // per row: group index | first cell index << 16
#pragma unroll
    for (int m = 0; m < RT; ++m) slot[m] = 0;
    if (listed && totals != 0u) {
        uint32_t ci = off & 0xFFFFu, gidx = off >> 16;
#pragma unroll
        for (int m = 0; m < RT; ++m) {
            const uint32_t burn = flags[m] & 0xFu, front = flags[m] >> 4;
            if (!(burn | front)) continue;
            slot[m] = gidx | (ci << 16);
            lds_group[gidx] = (uint16_t)(lane | (m << 6));
            // each front cell is listed with its 3x3 burning window (bits
            // c..c+2 of the up, middle and down row windows); its direction
            // mask is derived where the list is evaluated, on every lane
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if ((front >> c) & 1u) {
                    const uint32_t w9 = ((row_win(m) >> c) & 7u) | (((row_win(m + 1) >> c) & 7u) << 3) |
                                        (((row_win(m + 2) >> c) & 7u) << 6);
                    lds_cell[ci++] = (uint32_t)lane | ((uint32_t)m << 6) | ((uint32_t)c << 9) | (w9 << 11) |
                                     (gidx << 20);
                }
            ++gidx;
        }
        __syncthreads();
        // one Philox block per listed group
        for (uint32_t gq = lane; gq < n_groups; gq += kWave) {
            const uint32_t e = lds_group[gq];
            const int olane = e & 63, m = e >> 6;
            const int gi = td.r0 + (olane >> gx_log) * RT + m;
            const int gj = td.c0 + 4 * (olane & (GX - 1));
            const uint4 w = group_words<ALIGNED>((int64_t)gi * W + gj, t, ed.env_id, key);
            lds_u[gq * 4 + 0] = word_to_uniform(w.x);
            lds_u[gq * 4 + 1] = word_to_uniform(w.y);
            lds_u[gq * 4 + 2] = word_to_uniform(w.z);
            lds_u[gq * 4 + 3] = word_to_uniform(w.w);
        }
        __syncthreads();
        // lambda and p of each listed front cell
        for (uint32_t cq = lane; cq < n_cells; cq += kWave) {
            const uint32_t e = lds_cell[cq];
            const int olane = e & 63, m = (e >> 6) & 7, c = (e >> 9) & 3;
            const uint32_t w9 = (e >> 11) & 0x1FFu, gq = e >> 20;
            const uint32_t nbk = direction_mask(w9 & 7u, (w9 >> 3) & 7u, (w9 >> 6) & 7u, 0);
            const int gi = td.r0 + (olane >> gx_log) * RT + m;
            const int gj = td.c0 + 4 * (olane & (GX - 1)) + c;
            const float p = ignite_prob<WIND_CELL>(nbk, base + (int64_t)gi * W + gj, W, F, A, lds_ew);
            lds_dec[cq] = lds_u[gq * 4 + c] < p ? 1 : 0;
        }
        __syncthreads();
    }

    // -- 5. new states, store, count
    int cnt = 0;
#pragma unroll
    for (int m = 0; m < RT; ++m) {
        const int gi = row0 + m;
        if (!(gi < H && gj0 < W)) continue;
        const uint32_t own = s[m + 1];
        const uint32_t burn = flags[m] & 0xFu, front = flags[m] >> 4;
        uint32_t out = own;
        if (burn | front) {
            if (listed) {
                const uint32_t gq = slot[m] & 0xFFFFu;
                uint32_t ci = slot[m] >> 16;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    uint32_t next;
                    if ((burn >> c) & 1u)
                        next = lds_u[gq * 4 + c] < A.p_continue ? kBurning : kBurnt;
                    else if ((front >> c) & 1u)
                        next = lds_dec[ci++] ? kBurning : kFlammable;
                    else
                        continue;
                    out = (out & ~(0xFFu << (8 * c))) | (next << (8 * c));
                }
            } else {
                // list overflow: this lane draws and evaluates its own cells
                const int64_t n0 = (int64_t)gi * W + gj0;
                const uint4 w = group_words<ALIGNED>(n0, t, ed.env_id, key);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float u = word_to_uniform(compu(w, c));
                    uint32_t next;
                    if ((burn >> c) & 1u)
                        next = u < A.p_continue ? kBurning : kBurnt;
                    else if ((front >> c) & 1u)
                        next = u < ignite_prob<WIND_CELL>(direction_mask(row_win(m), row_win(m + 1), row_win(m + 2), c),
                                                          base + n0 + c, W, F, A, lds_ew)
                                   ? kBurning
                                   : kFlammable;
                    else
                        continue;
                    out = (out & ~(0xFFu << (8 * c))) | (next << (8 * c));
                }
            }
        }
        uint8_t* o = (dst + base) + (uint32_t)(gi * W + gj0);
        if constexpr (ALIGNED && !SKIP) {
            // dense plan: nontemporal, as the fuel and elevation streamed
            // through every step evict the state from the caches anyway, and
            // nothing in this launch reads the new state (about 2% faster on
            // the 1024 x 256^2 batch).  The front-skipping plans move a few
            // bytes per cell and find the state still cached the next step.
            __builtin_nontemporal_store(out, reinterpret_cast<uint32_t*>(o));
        } else if constexpr (ALIGNED) {
            *reinterpret_cast<uint32_t*>(o) = out;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (gj0 + c < W) o[c] = (uint8_t)(out >> (8 * c));
        }
        cnt += __popc(pack4(burning_flags(out)));
    }

    // -- BURNING count of the env (and of the tile) after the step --
    if (counts_row || SP.burn_next) {
        const int tile_cnt = (int)ballot_sum<bit_width(4 * RT)>((uint32_t)cnt);
        if (lane == 0) {
            if (counts_row && tile_cnt) atomicAdd(counts_row + td.env, tile_cnt);
            if (SP.burn_next) SP.eq[tile] = 0;
        }
        // a tile that still burns marks itself and its 8 neighbours to run
        // the next step
        if (SP.burn_next && tile_cnt && lane < 9) {
            const int nb = lane == 0 ? tile : SP.nbr[8 * tile + lane - 1];
            if (nb >= 0) SP.burn_next[nb] = 1;
        }
    }
}

__global__ void init_cells_kernel(int64_t n, const uint8_t* __restrict__ cls,
                                  const float* __restrict__ den, const float* __restrict__ elev,
                                  const float* __restrict__ wind_in, float v0, float v1, float v2,
                                  float v3, float v4, float v5, float v6, float v7, float v8,
                                  float v9, float v10, uint32_t mask, float* __restrict__ g,
                                  float* __restrict__ E, uint8_t* __restrict__ cls_out,
                                  float* __restrict__ den_out, float* __restrict__ wind_out,
                                  uint8_t* __restrict__ states)
{
    __shared__ float veg[11];
    if (threadIdx.x == 0) {
        veg[0] = v0; veg[1] = v1; veg[2] = v2; veg[3] = v3; veg[4] = v4; veg[5] = v5;
        veg[6] = v6; veg[7] = v7; veg[8] = v8; veg[9] = v9; veg[10] = v10;
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cls[i] > 10 ? 10u : cls[i];
        const float d = den[i];
        g[i] = (1.0f + veg[c]) * (1.0f + d);
        E[i] = elev[i];
        cls_out[i] = (uint8_t)c;
        den_out[i] = d;
        states[i] = ((mask >> c) & 1u) ? kUnburnable : kFlammable;
        if (wind_in) {
            wind_out[i] = wind_in[i];
            wind_out[n + i] = wind_in[n + i];
            wind_out[2 * n + i] = wind_in[2 * n + i];
        }
    }
}

__global__ void ignite_kernel(const int32_t* __restrict__ ign, int32_t n_ign,
                              const EnvDev* __restrict__ envs, uint8_t* __restrict__ states)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_ign) return;
    const EnvDev e = envs[ign[3 * q]];
    const int64_t idx = e.offset + (int64_t)ign[3 * q + 1] * e.W + ign[3 * q + 2];
    if (states[idx] == kFlammable) states[idx] = kBurning;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void copy_u8_kernel(uint8_t* __restrict__ dst, const uint8_t* __restrict__ src, int64_t n)
{
    const int64_t n16 = n >> 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * blockDim.x)
        reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
    for (int64_t i = (n16 << 4) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void set_u32_kernel(uint32_t* p, uint32_t v) { *p = v; }

__global__ void debug_exp_kernel(const float* x, float* y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = exp_c(x[i]);
}

__global__ void debug_atan_kernel(const float* x, float* y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = atan_c(x[i]);
}

__global__ void debug_philox_kernel(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint4 r = philox4x32_10(make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]),
                                      make_uint2(key[2 * i], key[2 * i + 1]));
        out[4 * i] = r.x;
        out[4 * i + 1] = r.y;
        out[4 * i + 2] = r.z;
        out[4 * i + 3] = r.w;
    }
}

// ---------------------------------------------------------------------------
// Temporal blocking: `ksteps` (<= K) steps per launch.  A 256-lane workgroup
// loads the state of its tile (TWD dwords x kTbRows rows of one env) with a
// halo of K rows and HX dwords (>= K cells) into LDS once, advances the whole
// region ksteps times in LDS, and stores only the tile.  After s steps the
// cells within s of the region border are stale (their neighbours were not
// loaded); each step computes the dwords that are still valid, so the tile
// itself is exact after K steps.  Draws, drops, counts and the arithmetic are
// those of the one-step kernel (same counters, same operation order), so the
// results are bit-identical; fuel and elevation are read only where a front
// cell needs them.  Envs must have W % 4 == 0.
constexpr int kTbRows = kTbTileRows;
constexpr int kTbListCap = 1024;  // listed front cells per tile and step

template <bool WIND_CELL, int TWD, int K>
__global__ __launch_bounds__(256) void stoch_tb_kernel(
    const TileDesc* __restrict__ tiles, int32_t n_tiles, int32_t tiles_per_xcd,
    const EnvDev* __restrict__ envs, StaticFields F0, StepArgs A, const uint8_t* __restrict__ src,
    uint8_t* __restrict__ dst, const uint32_t* __restrict__ t_base, uint32_t step0, int32_t ksteps,
    const int32_t* __restrict__ actions, int32_t* __restrict__ counts, int32_t n_env)
{
    constexpr int HX = (K + 3) / 4;        // halo in dwords
    constexpr int RWD = TWD + 2 * HX;      // region width in dwords
    constexpr int RW = 4 * RWD;            // ... in cells
    constexpr int RH = kTbRows + 2 * K;    // region rows
    constexpr int G = 256 / RWD;           // row strips: lane (g, cd) walks strip g of column cd
    __shared__ uint32_t buf[2][RH * RWD];
    __shared__ float lds_ew[2][8];
    // Row activity, rotating over three slots (written during step j, read
    // during step j + 1, cleared during step j + 2): bit r of burn_rows says
    // row r may hold a burning cell; bit r of diff_rows says the two buffers
    // may differ on row r.  A row with no burning cell within one row cannot
    // change, so it is skipped (copied if the buffers differ).
    __shared__ unsigned long long burn_rows[3], diff_rows[3];
    // Front cells of the step, listed so that their neighbour loads are
    // issued by all lanes together: row | column dword << 6 | cell << 12 |
    // burning-neighbour mask << 14, with the cell's uniform.  A full list
    // leaves further cells to their lane.
    __shared__ uint32_t list_key[kTbListCap];
    __shared__ float list_u[kTbListCap];
    __shared__ int32_t n_list[3];

    const int b = blockIdx.x;
    const int tile = (b & 7) * tiles_per_xcd + (b >> 3);
    if (tile >= n_tiles) return;
    const TileDesc td = tiles[tile];
    const EnvDev ed = envs[td.env];
    const int H = ed.H, W = ed.W, Wd = W >> 2;
    const int tid = threadIdx.x, lane = tid & 63;
    const int r0 = td.r0 - K, d0 = (td.c0 >> 2) - HX;  // region origin (row, dword column)
    const int64_t base = ed.offset;
    const uint32_t* src32 = reinterpret_cast<const uint32_t*>(src + base);
    uint32_t* dst32 = reinterpret_cast<uint32_t*>(dst + base);
    const uint2 key = make_uint2(A.key0, A.key1);
    const int cd = tid % RWD, grp = tid / RWD;  // this lane's column and row strip
    const int gj = 4 * (d0 + cd);
    const bool col_in = gj >= 0 && gj < W;
    const bool col_tile = cd >= HX && cd < HX + TWD;

    if (tid < 3) {
        burn_rows[tid] = 0ull;
        diff_rows[tid] = tid == 0 ? ~0ull : 0ull;  // the second buffer holds nothing yet
        n_list[tid] = 0;
    }
    __syncthreads();
    for (int idx = tid; idx < RH * RWD; idx += 256) {
        const int gi = r0 + idx / RWD, gd = d0 + idx % RWD;
        const uint32_t w = (gi >= 0 && gi < H && gd >= 0 && gd < Wd) ? src32[(int64_t)gi * Wd + gd] : 0u;
        buf[0][idx] = w;
        if (burning_flags(w)) atomicOr(&burn_rows[0], 1ull << (idx / RWD));
    }

    for (int j = 0; j < ksteps; ++j) {
        const uint32_t t = *t_base + step0 + (uint32_t)j;
        StaticFields F = F0;
        if (F0.wind_stride != 0) F.wind = F0.wind + (int64_t)t * F0.wind_stride;
        uint32_t* cur = buf[j & 1];
        uint32_t* nxt = buf[(j + 1) & 1];
        float* ew = lds_ew[j & 1];  // double-buffered: the previous step may still read the other
        if constexpr (!WIND_CELL) {
            if (tid < 8) {
                float V = ed.V, Vx = ed.Vx, Vy = ed.Vy;
                if (F.env_wind) {
                    const float* w = F.env_wind + ((int64_t)t * F.n_env + td.env) * 3;
                    V = w[0];
                    Vx = w[1];
                    Vy = w[2];
                }
                ew[tid] = wind_exponent(tid, A.alpha_w1, A.alpha_w2, V, Vx, Vy);
            }
        }
        const int32_t act = actions ? actions[(int64_t)j * n_env + td.env] : -1;
        const int sc = j % 3, sn = (j + 1) % 3, sz = (j + 2) % 3;
        __syncthreads();  // region loaded / previous step complete; wind exponents visible
        unsigned long long bmask = burn_rows[sc], dmask = diff_rows[sc];
        if (tid == 0) {
            burn_rows[sz] = 0ull;
            diff_rows[sz] = 0ull;
            n_list[sn] = 0;  // the counter of the next step (last read two steps ago)
        }
        if (act >= 0) {
            const int ar = (act >> 16) & 0x7FFF, ac = act & 0xFFFF;
            if (ar < H && ac < W) {
                // rows the drop may change differ from the other buffer afterwards
                for (int r = max(ar - A.drop_radius - r0, 0); r <= min(ar + A.drop_radius - r0, RH - 1); ++r)
                    dmask |= 1ull << r;
                // the dwords of the square inside the region
                const int R = A.drop_radius;
                const int ya = max(ar - R - r0, 0), yb = min(ar + R - r0, RH - 1);
                const int xa = max(ac - R - 4 * d0, 0), xb = min(ac + R - 4 * d0, RW - 1);
                if (ya <= yb && xa <= xb) {
                    const int da = xa >> 2, nw = (xb >> 2) - da + 1;
                    for (int q = tid; q < (yb - ya + 1) * nw; q += 256) {
                        const int rr = ya + q / nw, cdq = da + q % nw;
                        cur[rr * RWD + cdq] =
                            apply_drop(cur[rr * RWD + cdq], r0 + rr, 4 * (d0 + cdq), ar, ac, R, A.drop_mode);
                    }
                }
                __syncthreads();
            }
        }
        // dwords still valid after this step: rows [s, RH - s), cells [s, RW - s), s = j + 1
        const int s1 = j + 1;
        const int row_lo = s1, nrows = RH - 2 * s1;
        const int per = (nrows + G - 1) / G;
        const int ra = row_lo + grp * per, rb = min(ra + per, row_lo + nrows);
        const unsigned long long active = bmask | (bmask << 1) | (bmask >> 1);
        unsigned long long my_burn = 0ull, my_diff = 0ull;
        int cnt = 0;
        if (grp < G && cd >= (s1 >> 2) && cd <= ((RW - s1 - 1) >> 2) && ra < rb) {
            const bool hasl = cd > 0, hasr = cd < RWD - 1;
            auto window = [&](int rr, uint32_t& own) {
                const uint32_t* r = cur + rr * RWD;
                own = r[cd];
                return row_window(hasl ? r[cd - 1] : 0u, own, hasr ? r[cd + 1] : 0u);
            };
            uint32_t own_up, own = 0u, own_dn, up6 = 0u, md6 = 0u;
            bool have = false;  // up6 / md6 / own hold rows rr - 1 and rr
            for (int rr = ra; rr < rb; ++rr) {
                if (!((active >> rr) & 1ull)) {  // no burning cell within one row: unchanged
                    if ((dmask >> rr) & 1ull) nxt[rr * RWD + cd] = cur[rr * RWD + cd];
                    have = false;
                    continue;
                }
                if (!have) {
                    up6 = window(rr - 1, own_up);
                    md6 = window(rr, own);
                }
                const uint32_t dn6 = window(rr + 1, own_dn);
                const uint32_t ud = up6 | dn6;
                const uint32_t near = (ud | (ud >> 1) | (ud >> 2) | md6 | (md6 >> 2)) & 0xFu;
                const uint32_t burn = pack4(burning_flags(own));
                const uint32_t front = pack4(flammable_flags(own)) & near;
                uint32_t out = own;
                const int gi = r0 + rr;
                if ((burn | front) && col_in && gi >= 0 && gi < H) {
                    const int64_t n0 = (int64_t)gi * W + gj;
                    const uint4 w = group_words<true>(n0, t, ed.env_id, key);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const float u = word_to_uniform(compu(w, c));
                        uint32_t next;
                        if ((burn >> c) & 1u) {
                            next = u < A.p_continue ? kBurning : kBurnt;
                        } else if ((front >> c) & 1u) {
                            const uint32_t nbk = direction_mask(up6, md6, dn6, c);
                            const int slot = atomicAdd(&n_list[sc], 1);
                            if (slot < kTbListCap) {  // decided below, with the other listed cells
                                list_key[slot] = (uint32_t)rr | ((uint32_t)cd << 6) | ((uint32_t)c << 12) | (nbk << 14);
                                list_u[slot] = u;
                                continue;
                            }
                            next = u < ignite_prob<WIND_CELL>(nbk, base + n0 + c, W, F, A, ew) ? kBurning
                                                                                                : kFlammable;
                        } else {
                            continue;
                        }
                        out = (out & ~(0xFFu << (8 * c))) | (next << (8 * c));
                    }
                }
                nxt[rr * RWD + cd] = out;
                const uint32_t bo = burning_flags(out);
                if (bo) my_burn |= 1ull << rr;
                if (out != own) my_diff |= 1ull << rr;  // every valid dword of the row is rewritten
                if (col_tile && rr >= K && rr < K + kTbRows && gi < H) cnt += __popc(pack4(bo));
                up6 = md6;
                md6 = dn6;
                own = own_dn;
                have = true;
            }
        }
        __syncthreads();  // list complete, non-listed cells written
        {
            const int n = min(n_list[sc], kTbListCap);
            uint8_t* nxt8 = reinterpret_cast<uint8_t*>(nxt);
            for (int q = tid; q < n; q += 256) {
                const uint32_t e = list_key[q];
                const int rr = e & 63, cdq = (e >> 6) & 63, c = (e >> 12) & 3;
                const uint32_t nbk = e >> 14;
                const int gi = r0 + rr, gjc = 4 * (d0 + cdq) + c;
                if (list_u[q] < ignite_prob<WIND_CELL>(nbk, base + (int64_t)gi * W + gjc, W, F, A, ew)) {
                    nxt8[(rr * RWD + cdq) * 4 + c] = kBurning;
                    my_burn |= 1ull << rr;
                    my_diff |= 1ull << rr;
                    if (cdq >= HX && cdq < HX + TWD && rr >= K && rr < K + kTbRows && gi < H) ++cnt;
                }
            }
        }
        // row masks of the next step, OR-reduced over the wave first
#pragma unroll
        for (int o2 = 32; o2 > 0; o2 >>= 1) {
            my_burn |= __shfl_xor(my_burn, o2);
            my_diff |= __shfl_xor(my_diff, o2);
        }
        if (lane == 0) {
            if (my_burn) atomicOr(&burn_rows[sn], my_burn);
            if (my_diff) atomicOr(&diff_rows[sn], my_diff);
        }
        if (counts) {
#pragma unroll
            for (int o2 = 32; o2 > 0; o2 >>= 1) cnt += __shfl_xor(cnt, o2);
            if (lane == 0 && cnt) atomicAdd(counts + (int64_t)j * n_env + td.env, cnt);
        }
    }
    __syncthreads();
    const uint32_t* fin = buf[ksteps & 1];
    for (int idx = tid; idx < kTbRows * TWD; idx += 256) {
        const int rr = K + idx / TWD, cdo = HX + idx % TWD;
        const int gi = r0 + rr, gd = d0 + cdo;
        if (gi < H && gd < Wd) dst32[(int64_t)gi * Wd + gd] = fin[rr * RWD + cdo];
    }
}

template <bool WC, int TWD, int K>
hipError_t launch_tb(hipStream_t s, const StepLaunch& L, const uint8_t* src, uint8_t* dst, const uint32_t* t_base,
                     uint32_t step0, int32_t ksteps, const int32_t* act, int32_t* cnt)
{
    const int32_t per_xcd = (L.n_tiles + 7) / 8;
    hipLaunchKernelGGL((stoch_tb_kernel<WC, TWD, K>), dim3(8 * per_xcd), dim3(256), 0, s, L.tiles, L.n_tiles,
                       per_xcd, L.envs, L.fields, L.args, src, dst, t_base, step0, ksteps, act, cnt, L.n_env);
    return hipGetLastError();
}

template <bool WC, int TWD>
hipError_t launch_tb_k(hipStream_t s, const StepLaunch& L, int K, const uint8_t* src, uint8_t* dst,
                       const uint32_t* t_base, uint32_t step0, int32_t ksteps, const int32_t* act, int32_t* cnt)
{
    switch (K) {
    case 2: return launch_tb<WC, TWD, 2>(s, L, src, dst, t_base, step0, ksteps, act, cnt);
    case 4: return launch_tb<WC, TWD, 4>(s, L, src, dst, t_base, step0, ksteps, act, cnt);
    default: return launch_tb<WC, TWD, 8>(s, L, src, dst, t_base, step0, ksteps, act, cnt);
    }
}

int grid_for(int64_t n, int block)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

template <bool AL, bool WC, int RT, bool SK>
hipError_t launch_variant(hipStream_t s, const StepLaunch& L, const uint8_t* src, uint8_t* dst,
                          const uint32_t* t_base, uint32_t step, const int32_t* act, int32_t* cnt,
                          const SparseArgs& sp)
{
    const int32_t per_xcd = (L.n_tiles + 7) / 8;
    hipLaunchKernelGGL((stoch_step_kernel<AL, WC, RT, SK>), dim3(8 * per_xcd), dim3(kWave), 0, s,
                       L.tiles, L.n_tiles, per_xcd, L.envs, L.fields, L.args, src, dst, t_base,
                       step, act, cnt, sp);
    return hipGetLastError();
}

template <bool AL, bool WC, bool SK>
hipError_t launch_rt(hipStream_t s, const StepLaunch& L, const uint8_t* src, uint8_t* dst,
                     const uint32_t* t_base, uint32_t step, const int32_t* act, int32_t* cnt,
                     const SparseArgs& sp)
{
    switch (L.rows_per_thread) {
    case 1: return launch_variant<AL, WC, 1, SK>(s, L, src, dst, t_base, step, act, cnt, sp);
    case 2: return launch_variant<AL, WC, 2, SK>(s, L, src, dst, t_base, step, act, cnt, sp);
    case 8: return launch_variant<AL, WC, 8, SK>(s, L, src, dst, t_base, step, act, cnt, sp);
    default: return launch_variant<AL, WC, 4, SK>(s, L, src, dst, t_base, step, act, cnt, sp);
    }
}

}  // namespace

hipError_t launch_stoch_step(hipStream_t s, const StepLaunch& L, const uint8_t* src, uint8_t* dst,
                             const uint32_t* t_base, uint32_t step, const int32_t* actions_row,
                             int32_t* counts_row, const SparseArgs& sp)
{
    const bool wc = L.fields.wind != nullptr;
    if (L.aligned) {
        if (wc)
            return L.skip_static
                       ? launch_rt<true, true, true>(s, L, src, dst, t_base, step, actions_row, counts_row, sp)
                       : launch_rt<true, true, false>(s, L, src, dst, t_base, step, actions_row, counts_row, sp);
        return L.skip_static
                   ? launch_rt<true, false, true>(s, L, src, dst, t_base, step, actions_row, counts_row, sp)
                   : launch_rt<true, false, false>(s, L, src, dst, t_base, step, actions_row, counts_row, sp);
    }
    if (wc)
        return L.skip_static
                   ? launch_rt<false, true, true>(s, L, src, dst, t_base, step, actions_row, counts_row, sp)
                   : launch_rt<false, true, false>(s, L, src, dst, t_base, step, actions_row, counts_row, sp);
    return L.skip_static
               ? launch_rt<false, false, true>(s, L, src, dst, t_base, step, actions_row, counts_row, sp)
               : launch_rt<false, false, false>(s, L, src, dst, t_base, step, actions_row, counts_row, sp);
}

hipError_t launch_stoch_tb(hipStream_t s, const StepLaunch& L, int K, int tile_width, const uint8_t* src,
                           uint8_t* dst, const uint32_t* t_base, uint32_t step0, int32_t ksteps,
                           const int32_t* actions, int32_t* counts)
{
    const bool wc = L.fields.wind != nullptr;
    if (tile_width == 64)
        return wc ? launch_tb_k<true, 16>(s, L, K, src, dst, t_base, step0, ksteps, actions, counts)
                  : launch_tb_k<false, 16>(s, L, K, src, dst, t_base, step0, ksteps, actions, counts);
    return wc ? launch_tb_k<true, 32>(s, L, K, src, dst, t_base, step0, ksteps, actions, counts)
              : launch_tb_k<false, 32>(s, L, K, src, dst, t_base, step0, ksteps, actions, counts);
}

hipError_t launch_init_cells(hipStream_t s, int64_t n, const uint8_t* cls, const float* den,
                             const float* elev, const float* wind_in, const float veg[11],
                             uint32_t mask, float* g, float* E, uint8_t* cls_out, float* den_out,
                             float* wind_out, uint8_t* states)
{
    hipLaunchKernelGGL(init_cells_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, n, cls, den, elev,
                       wind_in, veg[0], veg[1], veg[2], veg[3], veg[4], veg[5], veg[6], veg[7],
                       veg[8], veg[9], veg[10], mask, g, E, cls_out, den_out, wind_out, states);
    return hipGetLastError();
}

hipError_t launch_ignite(hipStream_t s, const int32_t* ign, int32_t n_ign, const EnvDev* envs,
                         uint8_t* states)
{
    if (n_ign <= 0) return hipSuccess;
    hipLaunchKernelGGL(ignite_kernel, dim3((n_ign + 255) / 256), dim3(256), 0, s, ign, n_ign, envs,
                       states);
    return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy_u8(hipStream_t s, uint8_t* dst, const uint8_t* src, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_u8_kernel, dim3(grid_for((n >> 4) + 1, 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_set_u32(hipStream_t s, uint32_t* p, uint32_t v)
{
    hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_debug_exp(hipStream_t s, const float* x, float* y, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(debug_exp_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_debug_atan(hipStream_t s, const float* x, float* y, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(debug_atan_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_debug_philox(hipStream_t s, const uint32_t* ctr, const uint32_t* key,
                               uint32_t* out, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(debug_philox_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, ctr, key, out, n);
    return hipGetLastError();
}

}  // namespace firesim
