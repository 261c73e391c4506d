// relaxed.hip -- the relaxed (mean-field) fire-spread step, its soft-IoU
// loss and its adjoint, for gradient-based calibration of the model's
// parameters (JaxWildfire, arXiv 2512.06102, section 3, "Deterministic
// (raw-probabilities) update", Eqs. 5-10; Eq. 4 for the ignition term).
//
// State per cell: U = p_un, B = p_burn.  One step:
//   q_k(v) = 1 - exp(-gamma(v) phi(u_k, k)),  u_k = v - D_k   (Eqs. 1-4)
//   P(v)   = 1 - prod_k (1 - q_k(v) B(u_k))
//   N = U P,  U' = U - N,  B' = N + p_continue B             (Eqs. 5-10)
//
// Adjoint of one step (bars are adjoints, primes are step t+1):
//   Nbar = B'bar - U'bar,   Ubar = U'bar + Nbar P,   Pbar = Nbar U,
//   Bbar(u) = p_c B'bar(u) + sum_k c_k(u + D_k),  c_k(v) = Pbar(v) q_k(v) E_k(v),
//   qbar_k(v) = Pbar(v) B(u_k) E_k(v),  E_k = prod_{j != k} (1 - q_j B(u_j))
// (exclusive products from prefix and suffix products, no division since
// q B can be 1), then through q = 1 - exp(-y), y = gamma phi (dq/dy =
// exp(-y)), phi = p_base g(u) exp(x), x = wind exponent + alpha_s S,
// gamma(v) = alpha_gamma g(v), g = (1 + veg[class]) (1 + den), to the 17
// parameters.
//
// Both directions work on 64 x 32 tiles (kAdjW x kAdjR) whose lanes own
// columns and walk the rows, passing neighbouring values and terms by DPP
// lane shifts, so each cell is loaded once per step.  The forward cuts a tile
// into four 8-row bands, one wave each.  The adjoint's transpose stencil
// (Bbar(u) gathers the terms of the targets around u, and those need B two
// cells away) runs one wave per tile, one launch per step; terms that cross
// into another tile go through an exchange record that the owning tile adds
// in the next step.  Every sum runs in a fixed order (no atomics), so the gradient
// is the same bits on every run.  Parameter gradients are summed per lane,
// reduced per wave and added to the tile's own row of partial sums; a last
// kernel sums the rows.
//
// Precision: the recurrence amplifies small burning mass exponentially (in
// the mean-field model every region reachable from a burning cell
// eventually ignites), so an fp32 state underflows and rounds its way onto a
// different trajectory within ~100 steps on a 128 x 128 grid.  U, B, the
// adjoint and the gradient sums are therefore fp64; the per-edge factors
// exp(x), phi, q = 1 - exp(-y) and exp(-y) are fp32 from the hardware base-2
// exponential (relative error ~1e-6 for |x| < 20), with q from its Taylor
// series below y = 1/16 so that small rates keep their relative accuracy.
#include <algorithm>
#include <vector>

#include "devmath.hpp"
#include "relaxed.hpp"

// Unlike the stochastic step, whose fp32 operation sequence is fixed so that
// it reproduces the oracle bit for bit, the relaxed path is held to a
// tolerance against an fp64 recurrence: from here on multiplies and adds may
// fuse into FMAs.
#pragma clang fp contract(fast)

namespace firesim {
namespace {

struct RelaxedArgs {
    float p_base, alpha_gamma, alpha_w1, alpha_w2, alpha_s, p_continue;
    float inv_orth, inv_diag;
    int32_t slope_mode;  // 0: S = rise / run; 1: S = atan(rise / run)
};

// The per-env wind of the current step: row env of a series row [n_env][3],
// or the env's static wind.
__device__ __forceinline__ float3 env_wind_of(const EnvDev& ed, const float* env_wind, int env)
{
    if (env_wind) return make_float3(env_wind[3 * env], env_wind[3 * env + 1], env_wind[3 * env + 2]);
    return make_float3(ed.V, ed.Vx, ed.Vy);
}

RelaxedArgs relaxed_args(const sim_params& p)
{
    RelaxedArgs a;
    a.p_base = p.p_base;
    a.alpha_gamma = p.alpha_gamma;
    a.alpha_w1 = p.alpha_w1;
    a.alpha_w2 = p.alpha_w2;
    a.alpha_s = p.alpha_s;
    a.p_continue = p.p_continue;
    a.inv_orth = (float)(1.0 / (double)p.cell_size);
    a.inv_diag = (float)(1.0 / ((double)p.cell_size * 1.41421356237309504880));
    a.slope_mode = (int32_t)p.slope_mode;
    return a;
}

struct Veg11 {
    float v[11];
};

// e^x by the hardware base-2 exponential.
__device__ __forceinline__ float hexp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// 1 - e^{-y} for y >= 0: Taylor series through y^5 below 1/16 (relative
// error < 2e-9 there), 1 - e^{-y} above (where it is at least 0.06).
__device__ __forceinline__ float one_minus_exp_neg(float y)
{
    if (y < 0.0625f)
        return y * (1.0f - y * (0.5f - y * ((float)(1.0 / 6.0) - y * ((float)(1.0 / 24.0) - y * (float)(1.0 / 120.0)))));
    return 1.0f - hexp(-y);
}

// q = 1 - e^{-y} as above and the survival e^{-y}: 1 - q below y = 1/16
// (where e^{-y} > 0.94, so the subtraction loses nothing), else from the
// one exponential.
__device__ __forceinline__ float2 q_and_survival(float y)
{
    const float qs = y * (1.0f - y * (0.5f - y * ((float)(1.0 / 6.0) - y * ((float)(1.0 / 24.0) - y * (float)(1.0 / 120.0)))));
    float el = hexp(-y);
    float qt = qs;
    // both are computed: a select, not a divergent branch
    asm volatile("" : "+v"(el), "+v"(qt));
    return y < 0.0625f ? make_float2(qt, 1.0f - qt) : make_float2(1.0f - el, el);
}


__global__ __launch_bounds__(256) void relaxed_init_kernel(const uint8_t* __restrict__ st, int64_t n,
                                                           double* __restrict__ U, double* __restrict__ B)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t s = st[i];
        U[i] = s == kFlammable ? 1.0 : 0.0;
        B[i] = s == kBurning ? 1.0 : 0.0;
    }
}

__global__ __launch_bounds__(256) void fuel_kernel(const uint8_t* __restrict__ cls,
                                                   const float* __restrict__ den, int64_t n,
                                                   Veg11 veg, float* __restrict__ g)
{
    __shared__ float sveg[11];
    if (threadIdx.x < 11) sveg[threadIdx.x] = veg.v[threadIdx.x];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        g[i] = (1.0f + sveg[cls[i]]) * (1.0f + den[i]);
}

__global__ __launch_bounds__(256) void copy_f64_kernel(double* __restrict__ dst,
                                                       const double* __restrict__ src, int64_t n)
{
    const int64_t n2 = n >> 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
         i += (int64_t)gridDim.x * blockDim.x)
        reinterpret_cast<double2*>(dst)[i] = reinterpret_cast<const double2*>(src)[i];
    for (int64_t i = (n2 << 1) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Wind exponent of direction k at source cell u (per env from LDS, or per cell).
template <bool WC>
__device__ __forceinline__ float source_wind(int k, const float* ew, const float* wind, int64_t n_cells,
                                             int64_t u, const RelaxedArgs& A)
{
    if constexpr (WC)
        return wind_exponent(k, A.alpha_w1, A.alpha_w2, wind[u], wind[n_cells + u], wind[2 * n_cells + u]);
    else
        return ew[k];
}

// ---------------------------------------------------------------- adjoint
// Adjoint tiles are AW = 64 columns (one wave, one column per lane) by AR
// rows.  A wave walks its tile's rows top to bottom with the target row r in
// the middle of a three-row window of sources (rows r-1, r, r+1).  Each lane
// loads its own column; the left and right columns come from the
// neighbouring lanes by wave-wide DPP shifts, and lanes 0 and 63 load the
// column just outside the tile (the "ghost" column) themselves.
//
// Every target is evaluated once, by the tile that holds it.  Its terms c_k
// (into Bbar of source u_k) and d_k (into the fuel adjoint of u_k) go to
// running sums of the three source rows of the own column and, by the same
// DPP shifts, of the two neighbouring columns, always added in the same
// order.  Row r-1 is complete once target row r is done and is finished
// then.  Sums that belong to cells of another tile (the rows just above and
// below the tile and the ghost columns) are written to the tile's exchange
// record; the tile that owns those cells adds them, in a fixed order, to
// Bbar_{t+1} when it reads it in the next adjoint step.  Their fuel-adjoint
// part is turned into veg gradient by the producing lane, which reads the
// land-cover class and density of the foreign cell.  No atomics: Bbar, Ubar
// and the gradient are the same bits on every run.
constexpr int AW = kAdjW, AR = kAdjR;
constexpr int kFwdSplit = 4;  // row bands (waves) per tile in the forward
static_assert(AR % kFwdSplit == 0, "forward row bands");
constexpr int kXTop = 0, kXBot = AW, kXLeft = 2 * AW, kXRight = 2 * AW + AR + 2;
static_assert(kXRight + AR + 2 <= kXTile, "exchange record");

// Wave-wide shifts (DPP wave_shr:1 / wave_shl:1): from_left gives lane i the
// value of lane i-1, from_right that of lane i+1.  The lane with no source
// (0, resp. 63) reads 0 in the *0 forms and keeps `edge` in the *_or forms.
template <bool ZERO>
__device__ __forceinline__ int shr1(int old, int v) { return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, ZERO); }
template <bool ZERO>
__device__ __forceinline__ int shl1(int old, int v) { return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, ZERO); }
__device__ __forceinline__ float from_left_or(float edge, float v)
{
    return __int_as_float(shr1<false>(__float_as_int(edge), __float_as_int(v)));
}
__device__ __forceinline__ float from_right_or(float edge, float v)
{
    return __int_as_float(shl1<false>(__float_as_int(edge), __float_as_int(v)));
}
__device__ __forceinline__ int lo32(double v) { return (int)(unsigned)(unsigned long long)__double_as_longlong(v); }
__device__ __forceinline__ int hi32(double v) { return (int)(__double_as_longlong(v) >> 32); }
__device__ __forceinline__ double mk64(int lo, int hi)
{
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double from_left_or(double edge, double v)
{
    return mk64(shr1<false>(lo32(edge), lo32(v)), shr1<false>(hi32(edge), hi32(v)));
}
__device__ __forceinline__ double from_right_or(double edge, double v)
{
    return mk64(shl1<false>(lo32(edge), lo32(v)), shl1<false>(hi32(edge), hi32(v)));
}
__device__ __forceinline__ double from_left0(double v) { return mk64(shr1<true>(0, lo32(v)), shr1<true>(0, hi32(v))); }
__device__ __forceinline__ double from_right0(double v) { return mk64(shl1<true>(0, lo32(v)), shl1<true>(0, hi32(v))); }

// Sum over the 64 lanes of a wave by xor butterflies (every lane receives the
// same bits: each level adds the same two values, only their order differs).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// A source cell as the adjoint reads it: B, fuel g, elevation E and (per-cell
// wind only) V, Vx, Vy.  Off-grid cells are all zero.
struct AdjCell {
    double B;
    float g, E, V, Vx, Vy;
};

// An env's arrays from its first cell (wave-uniform pointers).  Cells are
// addressed by a 32-bit byte offset from them, so loads take a scalar base;
// the relaxed path therefore accepts envs of fewer than 2^29 cells.
struct AdjEnv {
    const double *U, *B, *gU1, *gB1;
    double *gU0, *gB0;
    const float *g, *E, *V, *Vx, *Vy, *den;
    const uint8_t* cls;
};

template <class T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t i)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st_at(T* base, uint32_t i, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T)) = v;
}

template <bool WC>
__device__ __forceinline__ AdjCell load_adj_cell(const AdjEnv& P, uint32_t o, bool in)
{
    AdjCell c{0.0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (in) {
        c.B = ld_at(P.B, o);
        c.g = ld_at(P.g, o);
        c.E = ld_at(P.E, o);
        if constexpr (WC) {
            c.V = ld_at(P.V, o);
            c.Vx = ld_at(P.Vx, o);
            c.Vy = ld_at(P.Vy, o);
        }
    }
    return c;
}

// The left (right) neighbour of each lane's cell: the neighbouring lane's
// cell, or for lane 0 (63) its ghost cell, the column just outside the tile.
template <bool WC>
__device__ __forceinline__ AdjCell left_of(const AdjCell& x, const AdjCell& ghost)
{
    AdjCell r{from_left_or(ghost.B, x.B), from_left_or(ghost.g, x.g), from_left_or(ghost.E, x.E), 0.0f, 0.0f, 0.0f};
    if constexpr (WC) {
        r.V = from_left_or(ghost.V, x.V);
        r.Vx = from_left_or(ghost.Vx, x.Vx);
        r.Vy = from_left_or(ghost.Vy, x.Vy);
    }
    return r;
}

template <bool WC>
__device__ __forceinline__ AdjCell right_of(const AdjCell& x, const AdjCell& ghost)
{
    AdjCell r{from_right_or(ghost.B, x.B), from_right_or(ghost.g, x.g), from_right_or(ghost.E, x.E), 0.0f, 0.0f, 0.0f};
    if constexpr (WC) {
        r.V = from_right_or(ghost.V, x.V);
        r.Vx = from_right_or(ghost.Vx, x.Vx);
        r.Vy = from_right_or(ghost.Vy, x.Vy);
    }
    return r;
}

// Running sums of one source cell: c into Bbar, d into the fuel adjoint.
struct CD {
    double c, d;
};

__device__ __forceinline__ CD cd_add(CD a, CD b) { return CD{a.c + b.c, a.d + b.d}; }
// a + m b with m = 1 or 0 (the ghost sums of lanes 0 and 63)
__device__ __forceinline__ CD cd_fma(CD b, double m, CD a) { return CD{fma(b.c, m, a.c), fma(b.d, m, a.d)}; }
__device__ __forceinline__ CD cd_from_left(CD a) { return CD{from_left0(a.c), from_left0(a.d)}; }
__device__ __forceinline__ CD cd_from_right(CD a) { return CD{from_right0(a.c), from_right0(a.d)}; }

// Sparse adjoint.  The parameter gradient of step s sums over edges u -> v
// with B_s(u) != 0, so u lies within s cells (Chebyshev) of S_0, the cells
// with initial burning mass, and v within s + 1; it needs Bbar_{s+1} and
// Ubar_{s+1} there.  Bbar_s(u) in turn needs the terms of the targets next
// to u, whose inputs are one cell further out, and so on up to the seed at
// T: the adjoint step s must be exact within s + 1 cells of S_0, and it
// evaluates targets within s + 2.  A tile with no cell within s + 2 of S_0 is
// skipped: whatever its cells and exchange record hold (finite: the buffers
// start at zero) only ever meets B = 0 in the gradient sums, so only the
// parameter gradient is returned.
//
// tile_mass_kernel flags the adjoint tiles holding initial burning mass;
// tile_integral_kernel builds each env's integral image of the flags (one
// workgroup per env, in LDS).
__global__ __launch_bounds__(256) void tile_mass_kernel(const RelaxedTile* __restrict__ tiles,
                                                        const EnvDev* __restrict__ envs,
                                                        const double* __restrict__ B, int32_t* __restrict__ mass)
{
    const RelaxedTile td = tiles[blockIdx.x];
    const EnvDev ed = envs[td.env];
    int any = 0;
    for (int idx = threadIdx.x; idx < AW * AR; idx += 256) {
        const int gi = td.r0 + idx / AW, gj = td.c0 + idx % AW;
        if (gi < ed.H && gj < ed.W && B[ed.offset + (int64_t)gi * ed.W + gj] != 0.0) any = 1;
    }
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) mass[blockIdx.x] = any ? 1 : 0;
}

__global__ __launch_bounds__(256) void tile_integral_kernel(const TileGrid* __restrict__ grids,
                                                            const int32_t* __restrict__ mass,
                                                            int32_t* __restrict__ integ)
{
    extern __shared__ int32_t sI[];
    const TileGrid tg = grids[blockIdx.x];
    const int W1 = tg.cols + 1, n = (tg.rows + 1) * W1;
    for (int i = threadIdx.x; i < n; i += 256) {
        const int r = i / W1, c = i % W1;
        sI[i] = (r && c) ? mass[tg.first + (r - 1) * tg.cols + (c - 1)] : 0;
    }
    __syncthreads();
    for (int r = threadIdx.x + 1; r <= tg.rows; r += 256) {
        int run = 0;
        for (int c = 1; c <= tg.cols; ++c) sI[r * W1 + c] = (run += sI[r * W1 + c]);
    }
    __syncthreads();
    for (int c = threadIdx.x + 1; c <= tg.cols; c += 256) {
        int run = 0;
        for (int r = 1; r <= tg.rows; ++r) sI[r * W1 + c] = (run += sI[r * W1 + c]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) integ[tg.ioff + i] = sI[i];
}

// Does the adjoint step s need tile (band i, strip j): is a tile with initial
// mass within a = floor((s + 1) / AR) + 1 bands and b = floor((s + 1) / AW) + 1
// strips (the tiles whose nearest cells are at most s + 2 apart)?
__device__ __forceinline__ bool adj_tile_in_reach(int i, int j, const TileGrid& tg, const int32_t* integ, int32_t s)
{
    const int a = (s + 1) / AR + 1, b = (s + 1) / AW + 1;
    const int i0 = max(i - a, 0), i1 = min(i + a, tg.rows - 1);
    const int j0 = max(j - b, 0), j1 = min(j + b, tg.cols - 1);
    const int32_t* I = integ + tg.ioff;
    const int W1 = tg.cols + 1;
    return I[(i1 + 1) * W1 + (j1 + 1)] - I[i0 * W1 + (j1 + 1)] - I[(i1 + 1) * W1 + j0] + I[i0 * W1 + j0] > 0;
}

// One adjoint step: (U_t, B_t), (Ubar_{t+1}, Bbar_{t+1}) -> (Ubar_t, Bbar_t)
// and the step's terms of the parameter gradient, added to the tile's row of
// gsum.  Both forms reduce to per-edge phibar_k and per-target gammabar:
//   FORM 0: ybar_k = Pbar B_k E_k exp(-y_k), phibar_k = ybar_k gamma,
//           gammabar = sum_k ybar_k phi_k, c_k = Pbar q_k E_k;
//   FORM 1: lambdabar = Pbar gamma (1 - P), phibar_k = lambdabar B_k,
//           gammabar = Pbar lambda (1 - P), c_k = lambdabar phi_k;
// d_k = phibar_k p_base exp(x_k) (dphi/dg of the source).  Far ahead of the
// fire (B = 0, U = 1) the adjoint state grows by about p_c + sum_k q_k per
// step backward and can pass the fp64 range after a few hundred steps.  It
// only ever meets B = 0 there: every gradient term it enters carries a factor
// B of a source or of the target, so those terms are 0.  The kernel takes a
// non-finite Pbar as 0 and adds the p_continue term only where B != 0, so the
// overflow never turns into inf x 0 = NaN.
// Four tiles (waves)
// per workgroup, dealt to the XCDs in contiguous runs of the tile list.
// SL: slope S = rise / run (0) or atan(rise / run) (1).
template <bool WC, int FORM, int SL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void relaxed_adj_kernel(
    const RelaxedTile* __restrict__ tiles, int32_t n_tiles, int32_t groups_per_xcd,
    const TileGrid* __restrict__ grids, const EnvDev* __restrict__ envs, const float* __restrict__ g,
    const float* __restrict__ E, const float* __restrict__ wind, const uint8_t* __restrict__ cls,
    const float* __restrict__ den, int64_t n_cells, RelaxedArgs A, const double* __restrict__ U,
    const double* __restrict__ B, const double* __restrict__ gU1, const double* __restrict__ gB1,
    double* __restrict__ gU0, double* __restrict__ gB0, const double* __restrict__ Xin,
    double* __restrict__ Xout, double* __restrict__ gsum, const float* __restrict__ env_wind,
    const int32_t* __restrict__ integ, int32_t step)
{
    __shared__ double sveg[4][11][64];  // per lane: fuel adjoint x (1 + den) by land-cover class
    __shared__ double sxc[4][AR][2];    // incoming Bbar terms of the first and last column, per row
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: tile values in SGPRs
    const int b = blockIdx.x;
    const int tix = (((b & 7) * groups_per_xcd + (b >> 3)) << 2) + wv;
    if (tix >= n_tiles) return;
    const RelaxedTile td = tiles[tix];
    const TileGrid tg = grids[td.env];
    const int tb = td.r0 / AR, ts = td.c0 / AW;  // band and strip of the tile
    if (integ && !adj_tile_in_reach(tb, ts, tg, integ, step)) return;  // sparse: the whole wave
    const EnvDev ed = envs[td.env];
    const int H = ed.H, W = ed.W;
    const int r0 = td.r0;
    const int rows = min(AR, H - r0);
    const int c = td.c0 + lane;
    const bool act = c < W;
    // ghost column: c0 - 1 for lane 0, c0 + 64 for lane 63 (if on the grid)
    const int cg = lane == 0 ? td.c0 - 1 : td.c0 + AW;
    const bool ghost = (lane == 0 && td.c0 > 0) || (lane == 63 && td.c0 + AW < W);
    const double mL = lane == 0 ? 1.0 : 0.0, mR = lane == 63 ? 1.0 : 0.0;
    const int64_t base = ed.offset;
    AdjEnv P;
    P.U = U + base;
    P.B = B + base;
    P.gU1 = gU1 + base;
    P.gB1 = gB1 + base;
    P.gU0 = gU0 + base;
    P.gB0 = gB0 + base;
    P.g = g + base;
    P.E = E + base;
    P.den = den + base;
    P.cls = cls + base;
    if constexpr (WC) {
        P.V = wind + base;
        P.Vx = wind + n_cells + base;
        P.Vy = wind + 2 * n_cells + base;
    } else {
        P.V = P.Vx = P.Vy = nullptr;
    }
    // cell (r, col) of the env; wraps for the row above row 0, which is never read
    auto at = [&](int r, int col) { return (uint32_t)(r * W + col); };
    auto tile_of = [&](int bi, int sj) { return (int64_t)(tg.first + bi * tg.cols + sj) * kXTile; };
    const int64_t xrec = (int64_t)tix * kXTile;

#pragma unroll
    for (int j = 0; j < 11; ++j) sveg[wv][j][lane] = 0.0;
    // each lane touches only its own slots, in program order: no barrier
    auto veg_add = [&](double fbar, uint32_t cl, float dn, bool on) {
        if (on) {
            double& slot = sveg[wv][cl][lane];
            slot += fbar * (1.0 + (double)dn);
        }
    };

    // this step's per-env wind; the exponent of direction k is
    // (alpha_w1 - alpha_w2) V + cos_k alpha_w2 Vx + sin_k alpha_w2 Vy
    const float3 wenv = env_wind_of(ed, env_wind, td.env);
    const float wA0 = (A.alpha_w1 - A.alpha_w2) * wenv.x, wA1 = A.alpha_w2 * wenv.y, wA2 = A.alpha_w2 * wenv.z;
    const float gp = A.alpha_gamma * A.p_base;

    // Bbar terms that neighbouring tiles added to this tile's cells in the
    // previous step: for the first and last row one per lane (xt, xb, corners
    // included), for the first and last column one per row (lanes 0 and 63,
    // fetched by lanes 0..15 and 32..47 into LDS)
    double xt = 0.0, xb = 0.0;
    if (Xin) {
        const bool up = tb > 0, dn = tb + 1 < tg.rows;
        if (act && up) xt = Xin[tile_of(tb - 1, ts) + kXBot + lane];
        if (act && dn) xb = Xin[tile_of(tb + 1, ts) + kXTop + lane];
        if (lane == 0 && ts > 0) {
            if (up) xt += Xin[tile_of(tb - 1, ts - 1) + kXRight + AR + 1];
            if (dn) xb += Xin[tile_of(tb + 1, ts - 1) + kXRight];
        }
        if (lane == 63 && ts + 1 < tg.cols) {
            if (up) xt += Xin[tile_of(tb - 1, ts + 1) + kXLeft + AR + 1];
            if (dn) xb += Xin[tile_of(tb + 1, ts + 1) + kXLeft];
        }
        const int side = lane >> 5, ii = lane & 31;
        double x = 0.0;
        if (ii < rows) {
            if (side == 0 && ts > 0) x = Xin[tile_of(tb, ts - 1) + kXRight + ii + 1];
            if (side == 1 && ts + 1 < tg.cols) x = Xin[tile_of(tb, ts + 1) + kXLeft + ii + 1];
        }
        if (ii < AR) sxc[wv][ii][side] = x;
        // the wave reads what its own lanes wrote: order the LDS accesses
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // the window: own column (X) and ghost column (G, lanes 0 and 63) of
    // source rows r - 1 (a), r (m), r + 1 (b)
    AdjCell X0 = load_adj_cell<WC>(P, at(r0 - 1, c), act && r0 > 0);
    AdjCell X1 = load_adj_cell<WC>(P, at(r0, c), act);
    AdjCell X2 = load_adj_cell<WC>(P, at(r0 + 1, c), act && r0 + 1 < H);
    AdjCell G0 = load_adj_cell<WC>(P, at(r0 - 1, cg), ghost && r0 > 0);
    AdjCell G1 = load_adj_cell<WC>(P, at(r0, cg), ghost);
    AdjCell G2 = load_adj_cell<WC>(P, at(r0 + 1, cg), ghost && r0 + 1 < H);

    // running sums (c, d) of the own column and the ghost column (lanes 0 and
    // 63) for source rows r - 1 (a), r (m), r + 1 (b): slots below
    double gB_prev = 0.0;
    // sums of t0 = phibar dphi/dp_base and of t0 S; per-cell wind: of t0 V
    // and t0 ((cos Vx + sin Vy) - V) of the source (acc_w1, acc_w2); per-env
    // wind: of t0 cos_k and t0 sin_k
    double acc_pb = 0.0, acc_w1 = 0.0, acc_w2 = 0.0, acc_s = 0.0, acc_gw = 0.0, acc_pc = 0.0;
    const double p_c = A.p_continue;

    // loaded one row ahead: the target's U, Ubar, Bbar, and the class and
    // density of the source row finished next (own and ghost column)
    double nU = 0.0, ngU = 0.0, ngB = 0.0;
    if (act) {
        nU = ld_at(P.U, at(r0, c));
        ngU = ld_at(P.gU1, at(r0, c));
        ngB = ld_at(P.gB1, at(r0, c));
    }
    uint32_t fcl = 0, gcl = 0;
    float fdn = 0.0f, gdn = 0.0f;
    if (act && r0 > 0) {
        fcl = ld_at(P.cls, at(r0 - 1, c));
        fdn = ld_at(P.den, at(r0 - 1, c));
    }
    if (ghost && r0 > 0) {
        gcl = ld_at(P.cls, at(r0 - 1, cg));
        gdn = ld_at(P.den, at(r0 - 1, cg));
    }

    CD acc_a{0.0, 0.0}, acc_m{0.0, 0.0}, acc_b{0.0, 0.0};
    CD gh_a{0.0, 0.0}, gh_m{0.0, 0.0}, gh_b{0.0, 0.0};
    AdjCell Xa = X0, Xm = X1, Xb = X2, Ga = G0, Gm = G1, Gb = G2;
#pragma unroll 1
    for (int i = 0; i < rows; ++i) {
        const int r = r0 + i;
        const uint32_t v = at(r, c);
        // the target's adjoint inputs, and what other tiles added to Bbar_{t+1}
        // of this cell in the previous step
        const double Uv = nU, gU = ngU;
        double gB = ngB;
        if (act && Xin)
            gB += ((i == 0 ? xt : 0.0) + (i == rows - 1 ? xb : 0.0)) +
                  (lane == 0 ? sxc[wv][i][0] : (lane == 63 ? sxc[wv][i][1] : 0.0));
        const uint32_t cl_a = fcl, gcl_a = gcl;  // row r - 1
        const float dn_a = fdn, gdn_a = gdn;
        if (act && i + 1 < rows) {
            nU = ld_at(P.U, v + W);
            ngU = ld_at(P.gU1, v + W);
            ngB = ld_at(P.gB1, v + W);
        }
        if (act) {
            fcl = ld_at(P.cls, v);
            fdn = ld_at(P.den, v);
        }
        if (ghost) {
            gcl = ld_at(P.cls, at(r, cg));
            gdn = ld_at(P.den, at(r, cg));
        }
        // next window row (r + 2)
        const bool more = i + 1 < rows && r + 2 < H;
        const AdjCell Xn = load_adj_cell<WC>(P, at(r + 2, c), act && more);
        const AdjCell Gn = load_adj_cell<WC>(P, at(r + 2, cg), ghost && more);

        // ---- the target v = (r, c); its source in direction k is u_k = v - D_k
        const AdjCell La = left_of<WC>(Xa, Ga), Lm = left_of<WC>(Xm, Gm), Lb = left_of<WC>(Xb, Gb);
        const AdjCell Ra = right_of<WC>(Xa, Ga), Rm = right_of<WC>(Xm, Gm), Rb = right_of<WC>(Xb, Gb);
        const double sB[8] = {Lm.B, Lb.B, Xb.B, Rb.B, Rm.B, Ra.B, Xa.B, La.B};
        const float sg[8] = {Lm.g, Lb.g, Xb.g, Rb.g, Rm.g, Ra.g, Xa.g, La.g};
        const float sE[8] = {Lm.E, Lb.E, Xb.E, Rb.E, Rm.E, Ra.E, Xa.E, La.E};
        const float sV[8] = {Lm.V, Lb.V, Xb.V, Rb.V, Rm.V, Ra.V, Xa.V, La.V};
        const float sVx[8] = {Lm.Vx, Lb.Vx, Xb.Vx, Rb.Vx, Rm.Vx, Ra.Vx, Xa.Vx, La.Vx};
        const float sVy[8] = {Lm.Vy, Lb.Vy, Xb.Vy, Rb.Vy, Rm.Vy, Ra.Vy, Xa.Vy, La.Vy};
        const double nbar = gB - gU;
        // a non-finite Pbar comes only from an overflowed far-field adjoint
        // (see above), whose terms all carry B = 0: they are 0, not inf x 0
        const double Pbar = __builtin_isfinite(nbar * Uv) ? nbar * Uv : 0.0;
        const float gv = Xm.g, Ev = Xm.E;
        const float gam = A.alpha_gamma * gv, gpe = gp * gv;  // gamma(v), gamma(v) p_base
        const double gam64 = gam;
        // per-cell wind: the wind term (cos Vx + sin Vy) - V of direction k at the source
        auto wterm = [&](int k) -> float { return (kCos[k] * sVx[k] + kSin[k] * sVy[k]) - sV[k]; };
        auto slope_k = [&](int k) {
            const float rr = (Ev - sE[k]) * ((k & 1) ? A.inv_diag : A.inv_orth);
            return SL ? atanf(rr) : rr;
        };
        float q[8], em[8], ex[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            // the exponent sums onto the slope term first, so that the
            // per-env wind constants are not kept per direction
            float x = A.alpha_s * slope_k(k);
            if constexpr (WC) {
                x = x + (A.alpha_w1 * sV[k] + A.alpha_w2 * wterm(k));
            } else {
                x = x + wA0;
                if (kCos[k] != 0.0f) x = x + kCos[k] * wA1;
                if (kSin[k] != 0.0f) x = x + kSin[k] * wA2;
            }
            // off-grid sources have zero fuel and zero B, so their terms
            // vanish; the exponent is capped so that 0 x e^x stays 0
            ex[k] = hexp(fminf(x, 88.0f));
            if constexpr (FORM == 0) {
                const float2 qe = q_and_survival(gam * (A.p_base * (sg[k] * ex[k])));
                q[k] = qe.x;
                em[k] = qe.y;
            }
        }
        // the terms of edge k from ybar_k = phibar_k / gamma: the gradient
        // sums, then c_k and d_k into the running sums of source u_k (own
        // column now, neighbouring lanes by DPP; lane 0 also keeps its k = 7,
        // 0, 1 terms for the ghost column on its left, lane 63 its k = 5, 4, 3
        // terms for the one on its right)
        double gam_w = 0.0;  // sum_k ybar_k dphi_k/dp_base (gammabar / p_base)
        auto emit = [&](int k, double cterm, double ybar) {
            const double yw = ybar * (double)(sg[k] * ex[k]);
            gam_w += yw;
            const double t0 = yw * gam64;  // phibar dphi/dp_base
            acc_pb += t0;
            acc_s += t0 * (double)slope_k(k);
            if constexpr (WC) {
                acc_w1 += t0 * (double)sV[k];
                acc_w2 += t0 * (double)wterm(k);
            } else {  // the env's wind is applied at the end
                if (kCos[k] != 0.0f) acc_w1 += t0 * (double)kCos[k];
                if (kSin[k] != 0.0f) acc_w2 += t0 * (double)kSin[k];
            }
            const CD o{cterm, ybar * (double)(gpe * ex[k])};  // d = phibar p_base e^x
            switch (k) {
            case 0: acc_m = cd_add(acc_m, cd_from_right(o)); gh_m = cd_fma(o, mL, gh_m); break;
            case 1: acc_b = cd_add(acc_b, cd_from_right(o)); gh_b = cd_fma(o, mL, gh_b); break;
            case 2: acc_b = cd_add(acc_b, o); break;
            case 3: acc_b = cd_add(acc_b, cd_from_left(o)); gh_b = cd_fma(o, mR, gh_b); break;
            case 4: acc_m = cd_add(acc_m, cd_from_left(o)); gh_m = cd_fma(o, mR, gh_m); break;
            case 5: acc_a = cd_add(acc_a, cd_from_left(o)); gh_a = cd_fma(o, mR, gh_a); break;
            case 6: acc_a = cd_add(acc_a, o); break;
            default: acc_a = cd_add(acc_a, cd_from_right(o)); gh_a = cd_fma(o, mL, gh_a); break;
            }
        };
        double Pv;
        if constexpr (FORM == 0) {
            double pre[8], run = 1.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                pre[k] = run;
                run = run * (1.0 - (double)q[k] * sB[k]);
            }
            Pv = 1.0 - run;
            double suf = 1.0;
#pragma unroll
            for (int k = 7; k >= 0; --k) {
                const double excl = pre[k] * suf;  // prod over j != k, no division
                suf = suf * (1.0 - (double)q[k] * sB[k]);
                const double pe = Pbar * excl;
                emit(k, pe * (double)q[k], (pe * sB[k]) * (double)em[k]);  // ybar = qbar dq/dy
            }
        } else {
            double lam = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) lam = lam + (double)(A.p_base * (sg[k] * ex[k])) * sB[k];
            const double surv = exp(-(double)gam * lam);
            Pv = -expm1(-(double)gam * lam);
            const double lbar = Pbar * gam64 * surv;  // phibar_k = lbar B_k, ybar_k = phibar_k / gamma
            const double ls = Pbar * surv;
#pragma unroll
            for (int k = 7; k >= 0; --k) emit(k, lbar * (double)(A.p_base * (sg[k] * ex[k])), ls * sB[k]);
        }
        // gammabar = p_base gam_w; gamma(v) = alpha_gamma g(v)
        const double gam_bar = (double)A.p_base * gam_w;
        acc_gw += gam_w * (double)gv;
        if (Xm.B != 0.0) acc_pc += gB * Xm.B;
        acc_m.d += gam_bar * (double)A.alpha_gamma;
        if (act) st_at(P.gU0, v, gU + nbar * Pv);

        // ---- source row r - 1 is complete
        if (i == 0) {  // the row above the tile: the band above owns it
            if (r0 > 0) {
                if (act) Xout[xrec + kXTop + lane] = acc_a.c;
                veg_add(acc_a.d, cl_a, dn_a, act);
                if (ghost) Xout[xrec + (lane == 0 ? kXLeft : kXRight)] = gh_a.c;
                veg_add(gh_a.d, gcl_a, gdn_a, ghost);
            }
        } else {
            if (act) st_at(P.gB0, v - W, p_c * gB_prev + acc_a.c);
            veg_add(acc_a.d, cl_a, dn_a, act);
            if (ghost) Xout[xrec + (lane == 0 ? kXLeft : kXRight) + i] = gh_a.c;
            veg_add(gh_a.d, gcl_a, gdn_a, ghost);
        }
        acc_a = acc_m;
        acc_m = acc_b;
        acc_b = CD{0.0, 0.0};
        gh_a = gh_m;
        gh_m = gh_b;
        gh_b = CD{0.0, 0.0};
        gB_prev = gB;
        Xa = Xm;
        Xm = Xb;
        Xb = Xn;
        Ga = Gm;
        Gm = Gb;
        Gb = Gn;
        }
    // the tile's last row, and the row below it (owned by the band below)
    const int rl = r0 + rows - 1;
    if (act) st_at(P.gB0, at(rl, c), p_c * gB_prev + acc_a.c);
    veg_add(acc_a.d, fcl, fdn, act);
    if (ghost) Xout[xrec + (lane == 0 ? kXLeft : kXRight) + rows] = gh_a.c;
    veg_add(gh_a.d, gcl, gdn, ghost);
    if (rl + 1 < H) {
        const bool on = act, gon = ghost;
        const uint32_t cl = on ? (uint32_t)ld_at(P.cls, at(rl + 1, c)) : 0u;
        const float dn = on ? ld_at(P.den, at(rl + 1, c)) : 0.0f;
        const uint32_t gc = gon ? (uint32_t)ld_at(P.cls, at(rl + 1, cg)) : 0u;
        const float gd = gon ? ld_at(P.den, at(rl + 1, cg)) : 0.0f;
        if (act) Xout[xrec + kXBot + lane] = acc_m.c;
        veg_add(acc_m.d, cl, dn, on);
        if (ghost) Xout[xrec + (lane == 0 ? kXLeft : kXRight) + rows + 1] = gh_m.c;
        veg_add(gh_m.d, gc, gd, gon);
    }

    // ---- the tile's 17 gradient terms (fixed order), added to its gsum row.
    // dphi/dx = phi = p_base dphi/dp_base, so the wind and slope terms are
    // p_base times sums of t0
    const double p_base = A.p_base;
    double acc[17];
    acc[0] = acc_pb;
    if constexpr (WC) {
        acc[1] = p_base * acc_w1;
        acc[2] = p_base * acc_w2;
    } else {
        acc[1] = p_base * ((double)wenv.x * acc_pb);
        acc[2] = p_base * (((double)wenv.y * acc_w1 + (double)wenv.z * acc_w2) - (double)wenv.x * acc_pb);
    }
    acc[3] = p_base * acc_s;
    acc[4] = p_base * acc_gw;  // sum gammabar g(v)
    acc[5] = acc_pc;
#pragma unroll
    for (int j = 0; j < 11; ++j) acc[6 + j] = sveg[wv][j][lane];
#pragma unroll
    for (int j = 0; j < 17; ++j) acc[j] = wave_sum(acc[j]);
    if (lane == 0) {
        double* row = gsum + (int64_t)tix * 17;
#pragma unroll
        for (int j = 0; j < 17; ++j) row[j] += acc[j];
    }
}

// One relaxed forward step on the adjoint's 64 x AR tiles, each cut into
// kFwdSplit row bands of one wave (four per workgroup, so that enough loads
// are in flight): lanes own columns and walk the rows with the same
// window as the adjoint (left and right sources by DPP from the neighbouring
// lanes, the ghost columns for lanes 0 and 63), so each cell is loaded once.
// FORM 0: p_ignite = 1 - prod_k (1 - q_k B_k); FORM 1: p_ignite = 1 -
// exp(-gamma sum_k B_k phi_k).  Rows where no lane sees burning mass skip the
// edge terms (P = 0 exactly there).
template <bool WC, int FORM, int SL>
__global__ __launch_bounds__(256) void relaxed_fwd_kernel(
    const RelaxedTile* __restrict__ tiles, int32_t n_tiles, int32_t groups_per_xcd,
    const EnvDev* __restrict__ envs, const float* __restrict__ g, const float* __restrict__ E,
    const float* __restrict__ wind, int64_t n_cells, RelaxedArgs A, const double* __restrict__ U,
    const double* __restrict__ B, double* __restrict__ Uo, double* __restrict__ Bo,
    const float* __restrict__ env_wind)
{
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int b = blockIdx.x;
    const int wix = (((b & 7) * groups_per_xcd + (b >> 3)) << 2) + wv;
    if (wix >= n_tiles * kFwdSplit) return;
    const RelaxedTile td = tiles[wix / kFwdSplit];
    const EnvDev ed = envs[td.env];
    const int H = ed.H, W = ed.W, r0 = td.r0 + (wix % kFwdSplit) * (AR / kFwdSplit);
    if (r0 >= H) return;
    const int rows = min(AR / kFwdSplit, H - r0);
    const int c = td.c0 + lane;
    const bool act = c < W;
    const int cg = lane == 0 ? td.c0 - 1 : td.c0 + AW;
    const bool ghost = (lane == 0 && td.c0 > 0) || (lane == 63 && td.c0 + AW < W);
    const int64_t base = ed.offset;
    AdjEnv P{};
    P.U = U + base;
    P.B = B + base;
    P.g = g + base;
    P.E = E + base;
    if constexpr (WC) {
        P.V = wind + base;
        P.Vx = wind + n_cells + base;
        P.Vy = wind + 2 * n_cells + base;
    }
    double* const Uoe = Uo + base;
    double* const Boe = Bo + base;
    auto at = [&](int r, int col) { return (uint32_t)(r * W + col); };
    const float3 wenv = env_wind_of(ed, env_wind, td.env);
    const float wA0 = (A.alpha_w1 - A.alpha_w2) * wenv.x, wA1 = A.alpha_w2 * wenv.y, wA2 = A.alpha_w2 * wenv.z;
    const double p_c = A.p_continue;

    AdjCell Xa = load_adj_cell<WC>(P, at(r0 - 1, c), act && r0 > 0);
    AdjCell Xm = load_adj_cell<WC>(P, at(r0, c), act);
    AdjCell Xb = load_adj_cell<WC>(P, at(r0 + 1, c), act && r0 + 1 < H);
    AdjCell Ga = load_adj_cell<WC>(P, at(r0 - 1, cg), ghost && r0 > 0);
    AdjCell Gm = load_adj_cell<WC>(P, at(r0, cg), ghost);
    AdjCell Gb = load_adj_cell<WC>(P, at(r0 + 1, cg), ghost && r0 + 1 < H);
    double nU = act ? ld_at(P.U, at(r0, c)) : 0.0;

#pragma unroll 1
    for (int i = 0; i < rows; ++i) {
        const int r = r0 + i;
        const uint32_t v = at(r, c);
        const double Uv = nU;
        if (act && i + 1 < rows) nU = ld_at(P.U, v + W);
        const bool more = i + 1 < rows && r + 2 < H;
        const AdjCell Xn = load_adj_cell<WC>(P, at(r + 2, c), act && more);
        const AdjCell Gn = load_adj_cell<WC>(P, at(r + 2, cg), ghost && more);

        double Pv = 0.0;
        const bool any_burning = Xa.B != 0.0 || Xm.B != 0.0 || Xb.B != 0.0 || Ga.B != 0.0 || Gm.B != 0.0 ||
                                 Gb.B != 0.0;
        if (__any(any_burning)) {  // wave-uniform
            const AdjCell La = left_of<WC>(Xa, Ga), Lm = left_of<WC>(Xm, Gm), Lb = left_of<WC>(Xb, Gb);
            const AdjCell Ra = right_of<WC>(Xa, Ga), Rm = right_of<WC>(Xm, Gm), Rb = right_of<WC>(Xb, Gb);
            const double sB[8] = {Lm.B, Lb.B, Xb.B, Rb.B, Rm.B, Ra.B, Xa.B, La.B};
            const float sg[8] = {Lm.g, Lb.g, Xb.g, Rb.g, Rm.g, Ra.g, Xa.g, La.g};
            const float sE[8] = {Lm.E, Lb.E, Xb.E, Rb.E, Rm.E, Ra.E, Xa.E, La.E};
            const float sV[8] = {Lm.V, Lb.V, Xb.V, Rb.V, Rm.V, Ra.V, Xa.V, La.V};
            const float sVx[8] = {Lm.Vx, Lb.Vx, Xb.Vx, Rb.Vx, Rm.Vx, Ra.Vx, Xa.Vx, La.Vx};
            const float sVy[8] = {Lm.Vy, Lb.Vy, Xb.Vy, Rb.Vy, Rm.Vy, Ra.Vy, Xa.Vy, La.Vy};
            const float Ev = Xm.E, gam = A.alpha_gamma * Xm.g;
            double prod = 1.0, lam = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float rr = (Ev - sE[k]) * ((k & 1) ? A.inv_diag : A.inv_orth);
                float x = A.alpha_s * (SL ? atanf(rr) : rr);
                if constexpr (WC) {
                    x = x + (A.alpha_w1 * sV[k] + A.alpha_w2 * ((kCos[k] * sVx[k] + kSin[k] * sVy[k]) - sV[k]));
                } else {
                    x = x + wA0;
                    if (kCos[k] != 0.0f) x = x + kCos[k] * wA1;
                    if (kSin[k] != 0.0f) x = x + kSin[k] * wA2;
                }
                // off-grid sources read 0: no fuel, no burning mass
                const float phi = A.p_base * (sg[k] * hexp(fminf(x, 88.0f)));
                if constexpr (FORM == 0)
                    prod = prod * (1.0 - (double)one_minus_exp_neg(gam * phi) * sB[k]);
                else
                    lam = lam + (double)phi * sB[k];
            }
            Pv = FORM == 0 ? 1.0 - prod : -expm1(-(double)gam * lam);
        }
        if (act) {
            const double N = Uv * Pv;
            st_at(Uoe, v, Uv - N);
            st_at(Boe, v, N + p_c * Xm.B);
        }
        Xa = Xm;
        Xm = Xb;
        Xb = Xn;
        Ga = Gm;
        Gm = Gb;
        Gb = Gn;
    }
}

// grad[j] = sum over tiles of gsum[tile][j], one workgroup per j, in a fixed order.
__global__ __launch_bounds__(256) void gsum_reduce_kernel(const double* __restrict__ gsum, int32_t n_tiles,
                                                          double* __restrict__ grad)
{
    __shared__ double red[4];
    const int j = blockIdx.x;
    double a = 0.0;
    for (int t = threadIdx.x; t < n_tiles; t += 256) a += gsum[(int64_t)t * 17 + j];
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) grad[j] = ((red[0] + red[1]) + red[2]) + red[3];
}
// ---------------------------------------------------------------- losses
// Every reduction below runs in a fixed order (lane-strided partial sums,
// xor butterflies, then the four wave sums in order), so the losses, the
// objective and the seed are the same bits on every call.

// Sum over a 256-lane workgroup, returned to every lane.
__device__ __forceinline__ double block_sum256(double v, double* red)
{
    v = wave_sum(v);
    __syncthreads();  // red may still be read by a previous call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red[0] + red[1]) + red[2]) + red[3];
}

// Soft IoU, stage 1: per loss chunk (kLossChunk cells of one env), the sums
// I = sum S Y, sum S and sum Y, with S = 1 - U_T on burnable cells.
__global__ __launch_bounds__(256) void iou_partials_kernel(const int32_t* __restrict__ chunk_env,
                                                           const EnvDev* __restrict__ envs,
                                                           const uint8_t* __restrict__ init_states,
                                                           const double* __restrict__ U_T,
                                                           const uint8_t* __restrict__ target,
                                                           double* __restrict__ partial)
{
    __shared__ double red[4];
    const int c = blockIdx.x;
    const EnvDev ed = envs[chunk_env[c]];
    const int64_t n = (int64_t)ed.H * ed.W;
    const int64_t first = (int64_t)(c - ed.chunk0) * kLossChunk;
    const int64_t last = min(first + (int64_t)kLossChunk, n);
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int64_t i = first + threadIdx.x; i < last; i += 256) {
        const int64_t v = ed.offset + i;
        const double S = init_states[v] != kUnburnable ? 1.0 - U_T[v] : 0.0;
        const double Y = target[v] ? 1.0 : 0.0;
        sy += S * Y;
        ss += S;
        yy += Y;
    }
    sy = block_sum256(sy, red);
    ss = block_sum256(ss, red);
    yy = block_sum256(yy, red);
    if (threadIdx.x == 0) {
        partial[3 * c] = sy;
        partial[3 * c + 1] = ss;
        partial[3 * c + 2] = yy;
    }
}

// Soft IoU, stage 2 (one wave per env): the env's sums over its chunks and
// L_e = 1 - I / D, D = sum S + sum Y - I (0 when D = 0).
__global__ __launch_bounds__(64) void iou_env_kernel(const EnvDev* __restrict__ envs,
                                                     const double* __restrict__ partial,
                                                     double* __restrict__ sums, double* __restrict__ env_loss,
                                                     float* __restrict__ loss)
{
    const int e = blockIdx.x, lane = threadIdx.x;
    const EnvDev ed = envs[e];
    const int nch = (int)(((int64_t)ed.H * ed.W + kLossChunk - 1) / kLossChunk);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int c = lane; c < nch; c += 64) {
        const double* p = partial + 3 * (int64_t)(ed.chunk0 + c);
        a0 += p[0];
        a1 += p[1];
        a2 += p[2];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
        const double D = (a1 + a2) - a0;
        const double L = D > 0.0 ? 1.0 - a0 / D : 0.0;
        sums[3 * e] = a0;
        sums[3 * e + 1] = a1;
        sums[3 * e + 2] = a2;
        env_loss[e] = L;
        loss[e] = (float)L;
    }
}

// The objective scale * sum_e L_e (one workgroup).
__global__ __launch_bounds__(256) void objective_kernel(const double* __restrict__ env_loss, int32_t n_env,
                                                        double scale, double* __restrict__ objective)
{
    __shared__ double red[4];
    double a = 0.0;
    for (int e = threadIdx.x; e < n_env; e += 256) a += env_loss[e];
    a = block_sum256(a, red);
    if (threadIdx.x == 0) objective[0] = scale * a;
}

// Soft IoU, stage 3: the seed scale * dL_e/dU_T = scale (Y D - I (1 - Y)) / D^2
// on burnable cells (dL/dU = -dL/dS), 0 elsewhere.
__global__ __launch_bounds__(256) void iou_seed_kernel(const int32_t* __restrict__ chunk_env,
                                                       const EnvDev* __restrict__ envs,
                                                       const uint8_t* __restrict__ init_states,
                                                       const uint8_t* __restrict__ target,
                                                       const double* __restrict__ sums, double scale,
                                                       double* __restrict__ gU_T)
{
    const int c = blockIdx.x;
    const int e = chunk_env[c];
    const EnvDev ed = envs[e];
    const int64_t n = (int64_t)ed.H * ed.W;
    const int64_t first = (int64_t)(c - ed.chunk0) * kLossChunk;
    const int64_t last = min(first + (int64_t)kLossChunk, n);
    const double I = sums[3 * e], D = (sums[3 * e + 1] + sums[3 * e + 2]) - I;
    for (int64_t i = first + threadIdx.x; i < last; i += 256) {
        const int64_t v = ed.offset + i;
        double gv = 0.0;
        if (D > 0.0 && init_states[v] != kUnburnable) {
            const double Y = target[v] ? 1.0 : 0.0;
            gv = scale * (Y * D - I * (1.0 - Y)) / (D * D);
        }
        gU_T[v] = gv;
    }
}

// The paper's calibration loss: BCE of the clipped soft scar plus the mean
// squared error of pool x pool block averages.  One lane per pooled block:
// the block means of S and Y, the block's BCE sum and squared error.
__global__ __launch_bounds__(256) void bce_pool_sums_kernel(
    const RelaxedTile* __restrict__ blocks, int32_t n_pool, int32_t pool, const EnvDev* __restrict__ envs,
    const uint8_t* __restrict__ init_states, const double* __restrict__ U_T,
    const uint8_t* __restrict__ target, double eps, double* __restrict__ vals)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_pool) return;
    const RelaxedTile pb = blocks[b];
    const EnvDev ed = envs[pb.env];
    const int i1 = min(pb.r0 + pool, ed.H), j1 = min(pb.c0 + pool, ed.W);
    double sS = 0.0, sY = 0.0, bce = 0.0;
    for (int i = pb.r0; i < i1; ++i)
        for (int j = pb.c0; j < j1; ++j) {
            const int64_t v = ed.offset + (int64_t)i * ed.W + j;
            const double S = init_states[v] != kUnburnable ? 1.0 - U_T[v] : 0.0;
            const double Y = target[v] ? 1.0 : 0.0;
            const double Sc = fmin(fmax(S, eps), 1.0 - eps);
            bce -= Y * log(Sc) + (1.0 - Y) * log(1.0 - Sc);
            sS += S;
            sY += Y;
        }
    const double cnt = (double)(i1 - pb.r0) * (double)(j1 - pb.c0);
    const double pS = sS / cnt, pY = sY / cnt;
    vals[b] = pS;
    vals[n_pool + b] = pY;
    vals[2 * (int64_t)n_pool + b] = bce;
    vals[3 * (int64_t)n_pool + b] = (pS - pY) * (pS - pY);
}

// Per env (one wave): BCE over its cells plus mse_weight times the mean
// squared error over its blocks.
__global__ __launch_bounds__(64) void bce_env_kernel(const EnvDev* __restrict__ envs,
                                                     const int32_t* __restrict__ env_blocks, int32_t n_pool,
                                                     const double* __restrict__ vals, double mse_weight,
                                                     double* __restrict__ env_loss, float* __restrict__ loss)
{
    const int e = blockIdx.x, lane = threadIdx.x;
    const int first = env_blocks[2 * e], nb = env_blocks[2 * e + 1];
    double bce = 0.0, sq = 0.0;
    for (int b = lane; b < nb; b += 64) {
        bce += vals[2 * (int64_t)n_pool + first + b];
        sq += vals[3 * (int64_t)n_pool + first + b];
    }
    bce = wave_sum(bce);
    sq = wave_sum(sq);
    if (lane == 0) {
        const double n_e = (double)envs[e].H * (double)envs[e].W;
        const double L = bce / n_e + mse_weight * sq / (double)nb;
        env_loss[e] = L;
        loss[e] = (float)L;
    }
}

__global__ __launch_bounds__(256) void bce_pool_grad_kernel(
    const RelaxedTile* __restrict__ blocks, int32_t n_pool, int32_t pool, const EnvDev* __restrict__ envs,
    const int32_t* __restrict__ env_blocks, const uint8_t* __restrict__ init_states,
    const double* __restrict__ U_T, const uint8_t* __restrict__ target, double eps, double mse_weight,
    const double* __restrict__ vals, double scale, double* __restrict__ gU_T)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_pool) return;
    const RelaxedTile pb = blocks[b];
    const EnvDev ed = envs[pb.env];
    const int i1 = min(pb.r0 + pool, ed.H), j1 = min(pb.c0 + pool, ed.W);
    const double n_e = (double)ed.H * (double)ed.W, m_e = (double)env_blocks[2 * pb.env + 1];
    const double cnt = (double)(i1 - pb.r0) * (double)(j1 - pb.c0);
    const double dmse = 2.0 * (vals[b] - vals[n_pool + b]) / m_e / cnt;  // d mse / d S of each cell
    for (int i = pb.r0; i < i1; ++i)
        for (int j = pb.c0; j < j1; ++j) {
            const int64_t v = ed.offset + (int64_t)i * ed.W + j;
            double gv = 0.0;
            if (init_states[v] != kUnburnable) {
                const double S = 1.0 - U_T[v];
                const double Y = target[v] ? 1.0 : 0.0;
                const double dbce = (S > eps && S < 1.0 - eps) ? (-(Y / S) + (1.0 - Y) / (1.0 - S)) / n_e : 0.0;
                gv = -scale * (dbce + mse_weight * dmse);  // dL/dU = -dL/dS
            }
            gU_T[v] = gv;
        }
}

int blocks_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

hipError_t copy_f64(hipStream_t s, double* dst, const double* src, int64_t n)
{
    hipLaunchKernelGGL(copy_f64_kernel, dim3(blocks_for((n >> 1) + 1)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t fill_f64(hipStream_t s, double* p, int64_t n, double v)
{
    hipLaunchKernelGGL(fill_f64_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Workspace layout (all offsets 256-byte aligned).
struct WsLayout {
    size_t g, ckpt, seg, fwd, adj, xchg, gsum, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout layout(int64_t n, int64_t n_adj_tiles, int32_t T, int32_t k)
{
    const size_t d = 8 * (size_t)n;
    const size_t n_ckpt = T > 0 ? (size_t)((T + k - 1) / k) : 1;
    WsLayout L;
    size_t o = 0;
    L.g = o;
    o = align256(o + 4 * (size_t)n);
    L.ckpt = o;
    o = align256(o + n_ckpt * 2 * d);
    L.seg = o;
    o = align256(o + (size_t)k * 2 * d);
    L.fwd = o;
    o = align256(o + 2 * d);
    L.adj = o;
    o = align256(o + 4 * d);
    L.xchg = o;  // two exchange records per adjoint tile (steps of either parity)
    o = align256(o + sizeof(double) * 2 * (size_t)n_adj_tiles * kXTile);
    L.gsum = o;  // 17 gradient partial sums per adjoint tile
    o = align256(o + sizeof(double) * 17 * (size_t)n_adj_tiles);
    L.total = o;
    return L;
}

hipError_t fuel(hipStream_t s, const RelaxedInputs& in, const sim_params& p, float* g)
{
    Veg11 veg;
    for (int c = 0; c < 11; ++c) veg.v[c] = p.veg[c];
    hipLaunchKernelGGL(fuel_kernel, dim3(blocks_for(in.n_cells)), dim3(256), 0, s, in.cls, in.den,
                       in.n_cells, veg, g);
    return hipGetLastError();
}

// The inputs of relaxed step t: a wind series (per env or per cell) moves to
// its row t; static wind is returned as it is.
RelaxedInputs at_step(const RelaxedInputs& in, int32_t t)
{
    RelaxedInputs r = in;
    if (in.wind && in.wind_stride) r.wind = in.wind + (int64_t)t * in.wind_stride;
    if (in.env_wind) r.env_wind = in.env_wind + (int64_t)t * in.n_env * 3;
    return r;
}

template <bool WC, int FORM>
void launch_fwd(hipStream_t s, const RelaxedInputs& in, const RelaxedArgs& A, const float* g,
                const double* U, const double* B, double* Uo, double* Bo)
{
    const int32_t groups = (in.n_tiles * kFwdSplit + 3) / 4;
    const int32_t per_xcd = (groups + 7) / 8;
    auto kernel = A.slope_mode ? relaxed_fwd_kernel<WC, FORM, 1> : relaxed_fwd_kernel<WC, FORM, 0>;
    hipLaunchKernelGGL(kernel, dim3(8 * per_xcd), dim3(256), 0, s, in.tiles, in.n_tiles, per_xcd, in.envs, g,
                       in.E, in.wind, in.n_cells, A, U, B, Uo, Bo, in.env_wind);
}

hipError_t fwd_step(hipStream_t s, const RelaxedInputs& in, const RelaxedArgs& A, const float* g,
                    const double* U, const double* B, double* Uo, double* Bo)
{
    if (in.wind)
        in.form ? launch_fwd<true, 1>(s, in, A, g, U, B, Uo, Bo) : launch_fwd<true, 0>(s, in, A, g, U, B, Uo, Bo);
    else
        in.form ? launch_fwd<false, 1>(s, in, A, g, U, B, Uo, Bo) : launch_fwd<false, 0>(s, in, A, g, U, B, Uo, Bo);
    return hipGetLastError();
}

template <bool WC, int FORM>
void launch_adj(hipStream_t s, const RelaxedInputs& in, const RelaxedState& R, const RelaxedArgs& A,
                const float* g, const double* U, const double* B, const double* gU1, const double* gB1,
                double* gU0, double* gB0, const double* Xin, double* Xout, double* gsum, const int32_t* integ,
                int32_t step)
{
    const int32_t groups = (R.n_btiles + 3) / 4;
    const int32_t per_xcd = (groups + 7) / 8;
    auto kernel = A.slope_mode ? relaxed_adj_kernel<WC, FORM, 1> : relaxed_adj_kernel<WC, FORM, 0>;
    hipLaunchKernelGGL(kernel, dim3(8 * per_xcd), dim3(256), 0, s, R.d_btiles, R.n_btiles, per_xcd, R.d_tgrid,
                       in.envs, g, in.E, in.wind, in.cls, in.den, in.n_cells, A, U, B, gU1, gB1, gU0, gB0, Xin,
                       Xout, gsum, in.env_wind, integ, step);
}

}  // namespace

int64_t relaxed_adj_tiles(const std::vector<sim_env>& envs)
{
    int64_t n = 0;
    for (const sim_env& v : envs) n += (int64_t)((v.H + AR - 1) / AR) * ((v.W + AW - 1) / AW);
    return n;
}

int relaxed_prepare(RelaxedState& R, const std::vector<sim_env>& envs)
{
    if (R.d_btiles) return 0;
    std::vector<RelaxedTile> btiles;
    std::vector<TileGrid> grids;
    int64_t ioff = 0, max_img = 0;
    for (int32_t e = 0; e < (int32_t)envs.size(); ++e) {
        TileGrid tg{(int32_t)btiles.size(), (envs[e].H + AR - 1) / AR, (envs[e].W + AW - 1) / AW, (int32_t)ioff};
        for (int r0 = 0; r0 < envs[e].H; r0 += AR)
            for (int c0 = 0; c0 < envs[e].W; c0 += AW) btiles.push_back(RelaxedTile{e, r0, c0, 0});
        const int64_t img = (int64_t)(tg.rows + 1) * (tg.cols + 1);
        ioff += img;
        max_img = std::max(max_img, img);
        grids.push_back(tg);
    }
    if (hipMalloc(&R.d_btiles, btiles.size() * sizeof(RelaxedTile)) != hipSuccess) return -1;
    if (hipMemcpy(R.d_btiles, btiles.data(), btiles.size() * sizeof(RelaxedTile),
                  hipMemcpyHostToDevice) != hipSuccess)
        return -1;
    if (hipMalloc(&R.d_tgrid, grids.size() * sizeof(TileGrid)) != hipSuccess) return -1;
    if (hipMemcpy(R.d_tgrid, grids.data(), grids.size() * sizeof(TileGrid), hipMemcpyHostToDevice) != hipSuccess)
        return -1;
    R.n_btiles = (int32_t)btiles.size();
    R.n_env = (int32_t)envs.size();
    if (ioff < INT32_MAX && 4 * max_img <= 64 * 1024) {
        if (hipMalloc(&R.d_tmass, btiles.size() * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&R.d_tinteg, (size_t)ioff * sizeof(int32_t)) != hipSuccess)
            return -1;
        R.sparse_lds = (int32_t)(4 * max_img);
    }
    return 0;
}

int relaxed_prepare_pool(RelaxedState& R, const std::vector<sim_env>& envs, int pool)
{
    if (R.d_pool && R.pool_k == pool) return 0;
    for (void** p : {(void**)&R.d_pool, (void**)&R.d_env_blocks, (void**)&R.d_pool_vals,
                     (void**)&R.d_bce_loss}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    std::vector<RelaxedTile> blocks;
    std::vector<int32_t> per_env;  // first block, number of blocks
    for (int32_t e = 0; e < (int32_t)envs.size(); ++e) {
        const size_t before = blocks.size();
        for (int r0 = 0; r0 < envs[e].H; r0 += pool)
            for (int c0 = 0; c0 < envs[e].W; c0 += pool) blocks.push_back(RelaxedTile{e, r0, c0, 0});
        per_env.push_back((int32_t)before);
        per_env.push_back((int32_t)(blocks.size() - before));
    }
    R.n_pool = (int32_t)blocks.size();
    if (hipMalloc(&R.d_pool, blocks.size() * sizeof(RelaxedTile)) != hipSuccess ||
        hipMalloc(&R.d_env_blocks, per_env.size() * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&R.d_pool_vals, 4 * blocks.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&R.d_bce_loss, envs.size() * sizeof(double)) != hipSuccess)
        return -1;
    if (hipMemcpy(R.d_pool, blocks.data(), blocks.size() * sizeof(RelaxedTile), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(R.d_env_blocks, per_env.data(), per_env.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess)
        return -1;
    R.pool_k = pool;
    return 0;
}

void relaxed_free(RelaxedState& R)
{
    for (void* p : {(void*)R.d_btiles, (void*)R.d_pool,
                    (void*)R.d_env_blocks, (void*)R.d_pool_vals, (void*)R.d_bce_loss, (void*)R.d_tgrid,
                    (void*)R.d_tmass, (void*)R.d_tinteg})
        if (p) (void)hipFree(p);
    R = RelaxedState{};
}

size_t relaxed_workspace_bytes(int64_t n_cells, int64_t n_adj_tiles, int32_t T, int32_t ckpt_every)
{
    return layout(n_cells, n_adj_tiles, T, ckpt_every).total;
}

hipError_t launch_relaxed_init(hipStream_t s, const uint8_t* init_states, int64_t n, double* U, double* B)
{
    hipLaunchKernelGGL(relaxed_init_kernel, dim3(blocks_for(n)), dim3(256), 0, s, init_states, n, U, B);
    return hipGetLastError();
}

// The forward writes each step's output where it is needed next: the
// checkpoint slot of every k-th state, the segment slots 1.. of the last
// segment's states (so the backward need not recompute that segment), the
// caller's U, B for the final state, and otherwise one of two scratch states
// (the forward buffer and segment slot 0, which the backward never uses).
hipError_t relaxed_forward(hipStream_t s, const RelaxedInputs& in, const sim_params& p, double* U,
                           double* B, int32_t T, int32_t k, void* workspace, RelaxedState& R)
{
    R.last_segment_ws = nullptr;
    if (T == 0) return hipSuccess;
    const int64_t n = in.n_cells;
    const WsLayout L = layout(n, R.n_btiles, T, k);
    char* ws = static_cast<char*>(workspace);
    float* g = reinterpret_cast<float*>(ws + L.g);
    double* ckpt = reinterpret_cast<double*>(ws + L.ckpt);
    double* seg = reinterpret_cast<double*>(ws + L.seg);
    double* spare[2] = {reinterpret_cast<double*>(ws + L.fwd), seg};
    const RelaxedArgs A = relaxed_args(p);
    const int32_t t_last = ((T - 1) / k) * k;  // first step of the last segment
    hipError_t e = fuel(s, in, p, g);
    if (e == hipSuccess) e = copy_f64(s, ckpt, U, n);
    if (e == hipSuccess) e = copy_f64(s, ckpt + n, B, n);
    const double* cu = ckpt;  // state t
    const double* cb = ckpt + n;
    for (int32_t t = 0; t < T && e == hipSuccess; ++t) {
        const int32_t t1 = t + 1;
        double *nu, *nb;
        if (t1 == T) {
            nu = U;
            nb = B;
        } else if (t1 % k == 0) {
            nu = ckpt + (size_t)(t1 / k) * 2 * n;
            nb = nu + n;
        } else if (t1 > t_last) {
            nu = seg + (size_t)(t1 - t_last) * 2 * n;
            nb = nu + n;
        } else {
            nu = spare[0] == cu ? spare[1] : spare[0];
            nb = nu + n;
        }
        e = fwd_step(s, at_step(in, t), A, g, cu, cb, nu, nb);
        cu = nu;
        cb = nb;
    }
    if (e == hipSuccess) R.last_segment_ws = workspace;
    return e;
}

hipError_t relaxed_loss(hipStream_t s, const LossBatch& lb, const double* U_T, const uint8_t* target,
                        float* loss, double* gU_T, double scale, double* objective, double* scr)
{
    double* partial = scr;
    double* sums = partial + 3 * (size_t)lb.n_chunks;
    double* env_loss = sums + 3 * (size_t)lb.n_env;
    hipLaunchKernelGGL(iou_partials_kernel, dim3(lb.n_chunks), dim3(256), 0, s, lb.chunk_env, lb.envs,
                       lb.init_states, U_T, target, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(iou_env_kernel, dim3(lb.n_env), dim3(64), 0, s, lb.envs, partial, sums, env_loss, loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (objective) {
        hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(256), 0, s, env_loss, lb.n_env, scale, objective);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (gU_T) {
        hipLaunchKernelGGL(iou_seed_kernel, dim3(lb.n_chunks), dim3(256), 0, s, lb.chunk_env, lb.envs,
                           lb.init_states, target, sums, scale, gU_T);
        e = hipGetLastError();
    }
    return e;
}

hipError_t relaxed_loss_bce(hipStream_t s, const RelaxedInputs& in, const uint8_t* init_states,
                            const double* U_T, const uint8_t* target, int pool, double mse_weight,
                            double eps, float* loss, double* gU_T, double scale, double* objective,
                            RelaxedState& R)
{
    const int nb = (R.n_pool + 255) / 256;
    hipLaunchKernelGGL(bce_pool_sums_kernel, dim3(nb), dim3(256), 0, s, R.d_pool, R.n_pool, pool, in.envs,
                       init_states, U_T, target, eps, R.d_pool_vals);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bce_env_kernel, dim3(in.n_env), dim3(64), 0, s, in.envs, R.d_env_blocks, R.n_pool,
                       R.d_pool_vals, mse_weight, R.d_bce_loss, loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (objective) {
        hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(256), 0, s, R.d_bce_loss, in.n_env, scale, objective);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (gU_T) {
        hipLaunchKernelGGL(bce_pool_grad_kernel, dim3(nb), dim3(256), 0, s, R.d_pool, R.n_pool, pool, in.envs,
                           R.d_env_blocks, init_states, U_T, target, eps, mse_weight, R.d_pool_vals, scale,
                           gU_T);
        e = hipGetLastError();
    }
    return e;
}

hipError_t relaxed_backward(hipStream_t s, const RelaxedInputs& in, const sim_params& p,
                            const double* gU_T, const double* gB_T, int32_t T, int32_t k,
                            void* workspace, double* grad, RelaxedState& R)
{
    const int64_t n = in.n_cells;
    const WsLayout L = layout(n, R.n_btiles, T, k);
    char* ws = static_cast<char*>(workspace);
    float* g = reinterpret_cast<float*>(ws + L.g);
    double* ckpt = reinterpret_cast<double*>(ws + L.ckpt);
    double* seg = reinterpret_cast<double*>(ws + L.seg);
    double* adj = reinterpret_cast<double*>(ws + L.adj);
    double* xchg = reinterpret_cast<double*>(ws + L.xchg);
    double* gsum = reinterpret_cast<double*>(ws + L.gsum);
    const int64_t xrecs = (int64_t)R.n_btiles * kXTile;
    const RelaxedArgs A = relaxed_args(p);
    hipError_t e = fill_f64(s, gsum, (int64_t)R.n_btiles * 17, 0.0);
    // exchange records start at zero: a tile that the sparse adjoint skips
    // leaves finite values for its neighbours to read
    if (e == hipSuccess) e = fill_f64(s, xchg, 2 * xrecs, 0.0);
    if (e == hipSuccess) e = fuel(s, in, p, g);
    double* cu = adj;  // adjoint at t+1: (Ubar, Bbar)
    double* cb = adj + n;
    double* nu = adj + 2 * n;  // adjoint at t
    double* nb = adj + 3 * n;
    if (e == hipSuccess) e = copy_f64(s, cu, gU_T, n);
    if (e == hipSuccess) e = gB_T ? copy_f64(s, cb, gB_T, n) : fill_f64(s, cb, n, 0.0);
    // sparse adjoint: tiles with initial burning mass (checkpoint 0 holds B_0),
    // their integral images, and zeroed output buffers (skipped tiles keep them)
    const int32_t* integ = nullptr;
    if (in.sparse && R.sparse_lds > 0 && T > 0 && e == hipSuccess) {
        hipLaunchKernelGGL(tile_mass_kernel, dim3(R.n_btiles), dim3(256), 0, s, R.d_btiles, in.envs, ckpt + n,
                           R.d_tmass);
        hipLaunchKernelGGL(tile_integral_kernel, dim3(R.n_env), dim3(256), (size_t)R.sparse_lds, s, R.d_tgrid,
                           R.d_tmass, R.d_tinteg);
        e = hipGetLastError();
        if (e == hipSuccess) e = fill_f64(s, nu, 2 * n, 0.0);
        integ = R.d_tinteg;
    }
    const int32_t n_seg = T > 0 ? (T + k - 1) / k : 0;
    for (int32_t sg = n_seg - 1; sg >= 0 && e == hipSuccess; --sg) {
        const int32_t t0 = sg * k, t1 = std::min(T, t0 + k);
        const double* base = ckpt + (size_t)sg * 2 * n;
        // states t0 .. t1-1 of the segment: slot 0 is the checkpoint itself
        auto state_u = [&](int32_t j) -> const double* { return j == 0 ? base : seg + (size_t)j * 2 * n; };
        auto state_b = [&](int32_t j) -> const double* {
            return j == 0 ? base + n : seg + (size_t)j * 2 * n + n;
        };
        // the last segment's states are in place after the forward, until an
        // earlier segment's recompute overwrites them
        const bool stored = sg == n_seg - 1 && R.last_segment_ws == workspace;
        if (sg < n_seg - 1) R.last_segment_ws = nullptr;
        for (int32_t j = 1; j < t1 - t0 && !stored && e == hipSuccess; ++j)
            e = fwd_step(s, at_step(in, t0 + j - 1), A, g, state_u(j - 1), state_b(j - 1),
                         seg + (size_t)j * 2 * n, seg + (size_t)j * 2 * n + n);
        for (int32_t t = t1 - 1; t >= t0 && e == hipSuccess; --t) {
            const int32_t j = t - t0;
            const double *Ut = state_u(j), *Bt = state_b(j);
            const RelaxedInputs it = at_step(in, t);
            // step t writes the exchange record of parity t; step t - 1 adds it
            const double* Xin = t == T - 1 ? nullptr : xchg + ((t + 1) & 1) * xrecs;
            double* Xout = xchg + (t & 1) * xrecs;
            if (it.wind)
                it.form ? launch_adj<true, 1>(s, it, R, A, g, Ut, Bt, cu, cb, nu, nb, Xin, Xout, gsum, integ, t)
                        : launch_adj<true, 0>(s, it, R, A, g, Ut, Bt, cu, cb, nu, nb, Xin, Xout, gsum, integ, t);
            else
                it.form ? launch_adj<false, 1>(s, it, R, A, g, Ut, Bt, cu, cb, nu, nb, Xin, Xout, gsum, integ, t)
                        : launch_adj<false, 0>(s, it, R, A, g, Ut, Bt, cu, cb, nu, nb, Xin, Xout, gsum, integ, t);
            e = hipGetLastError();
            std::swap(cu, nu);
            std::swap(cb, nb);
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(gsum_reduce_kernel, dim3(17), dim3(256), 0, s, gsum, R.n_btiles, grad);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace firesim
