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
// The forward works on 32 x 16 tiles, the adjoint on 32 x 20 tiles (256 lanes).
// The adjoint's transpose stencil (Bbar(u) gathers from the targets around
// u, and those need B two cells away) is done in one launch per step: the
// tile stages B, g and E (and per-cell wind) with a two-cell halo in LDS;
// phase 1 evaluates every target of the tile plus a one-cell ring and adds
// c_k and the source-side fuel adjoint d_k into LDS slots of the sources in
// the tile (LDS atomics: the summation order of a slot is not fixed);
// phase 2 finishes the tile's own cells.  Parameter
// gradients are summed per lane, reduced per workgroup, and added to one of
// 64 fp64 stripes with atomics; a last kernel sums the stripes.
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

// S of Eq. 2 from the rise over the run (or its angle).
__device__ __forceinline__ float slope_of(float rise_over_run, const RelaxedArgs& A)
{
    return A.slope_mode ? atanf(rise_over_run) : rise_over_run;
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
    const float el = hexp(-y);
    return y < 0.0625f ? make_float2(qs, 1.0f - qs) : make_float2(1.0f - el, el);
}

// Sums of 17 values over the 64 lanes of a wave, written to out[0..16].
// Recursive halving: at the exchange with lane ^ 32 the lower half keeps the
// sums of values 0-7 and the upper half those of 8-15, and so on down to one
// value per lane at lane ^ 4; lanes ^ 2 and ^ 1 finish it.  Lane l then
// holds value 8 b5 + 4 b4 + 2 b3 + b2 (bits of l).  Value 16 is summed on
// its own.  17 + 6 exchanges instead of 17 x 6.
__device__ __forceinline__ void wave_sum17(const double (&a)[17], int lane, double* out)
{
    double b8[8], b4[4], b2[2];
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
    for (int j = 0; j < 8; ++j) b8[j] = (h5 ? a[8 + j] : a[j]) + __shfl_xor(h5 ? a[j] : a[8 + j], 32);
#pragma unroll
    for (int j = 0; j < 4; ++j) b4[j] = (h4 ? b8[4 + j] : b8[j]) + __shfl_xor(h4 ? b8[j] : b8[4 + j], 16);
#pragma unroll
    for (int j = 0; j < 2; ++j) b2[j] = (h3 ? b4[2 + j] : b4[j]) + __shfl_xor(h3 ? b4[j] : b4[2 + j], 8);
    double b1 = (h2 ? b2[1] : b2[0]) + __shfl_xor(h2 ? b2[0] : b2[1], 4);
    b1 += __shfl_xor(b1, 2);
    b1 += __shfl_xor(b1, 1);
    double last = a[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) last += __shfl_xor(last, off);
    if ((lane & 3) == 0) out[((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1)] = b1;
    if (lane == 0) out[16] = last;
}

constexpr int TW = kRelaxTW, TH = kRelaxTH;  // forward tile
constexpr int BW = kRelaxBW, BH = kRelaxBH;  // adjoint tile

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

// One relaxed forward step on a 32 x 16 tile.  FORM 0: p_ignite = 1 -
// prod_k (1 - q_k B_k); FORM 1: p_ignite = 1 - exp(-gamma sum_k B_k phi_k).
template <bool WC, int FORM>
__global__ __launch_bounds__(256) void relaxed_fwd_kernel(
    const RelaxedTile* __restrict__ tiles, const EnvDev* __restrict__ envs, const float* __restrict__ g,
    const float* __restrict__ E, const float* __restrict__ wind, int64_t n_cells, RelaxedArgs A,
    const double* __restrict__ U, const double* __restrict__ B, double* __restrict__ Uo,
    double* __restrict__ Bo, const float* __restrict__ env_wind)
{
    constexpr int EW = TW + 2, EH = TH + 2;
    __shared__ double sB[EH * EW];
    __shared__ float sg[EH * EW], sE[EH * EW];
    __shared__ float ew[8];
    const RelaxedTile td = tiles[blockIdx.x];
    const EnvDev ed = envs[td.env];
    const int H = ed.H, W = ed.W, tid = threadIdx.x;
    for (int idx = tid; idx < EH * EW; idx += 256) {
        const int gi = td.r0 - 1 + idx / EW, gj = td.c0 - 1 + idx % EW;
        const bool in = gi >= 0 && gi < H && gj >= 0 && gj < W;
        const int64_t v = ed.offset + (int64_t)gi * W + gj;
        sB[idx] = in ? B[v] : 0.0;
        sg[idx] = in ? g[v] : 0.0f;
        sE[idx] = in ? E[v] : 0.0f;
    }
    if (!WC && tid < 8) {
        const float3 w = env_wind_of(ed, env_wind, td.env);
        ew[tid] = wind_exponent(tid, A.alpha_w1, A.alpha_w2, w.x, w.y, w.z);
    }
    __syncthreads();
    for (int idx = tid; idx < TW * TH; idx += 256) {
        const int rr = idx / TW, cc = idx % TW;
        const int gi = td.r0 + rr, gj = td.c0 + cc;
        if (gi >= H || gj >= W) continue;
        const int64_t v = ed.offset + (int64_t)gi * W + gj;
        const int a = rr + 1, b = cc + 1;
        const double Uv = U[v], Bv = sB[a * EW + b];
        double P = 0.0;
        if (Uv != 0.0) {
            const float gam = A.alpha_gamma * sg[a * EW + b];
            const float Ev = sE[a * EW + b];
            double prod = 1.0, lam = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int s = (a - kDRow[k]) * EW + (b - kDCol[k]);
                const double Bu = sB[s];
                if (Bu == 0.0) continue;  // off-grid sources read 0
                const int64_t u = v - (int64_t)kDRow[k] * W - kDCol[k];
                const float x = source_wind<WC>(k, ew, wind, n_cells, u, A) +
                                A.alpha_s * slope_of((Ev - sE[s]) * ((k & 1) ? A.inv_diag : A.inv_orth), A);
                const float phi = A.p_base * sg[s] * hexp(x);
                if constexpr (FORM == 0)
                    prod = prod * (1.0 - (double)one_minus_exp_neg(gam * phi) * Bu);
                else
                    lam = lam + (double)phi * Bu;
            }
            P = FORM == 0 ? 1.0 - prod : -expm1(-(double)gam * lam);
        }
        const double N = Uv * P;
        Uo[v] = Uv - N;
        Bo[v] = N + (double)A.p_continue * Bv;
    }
}

// Sparse adjoint.  The parameter gradient of step s sums over edges u -> v
// with B_s(u) != 0, so u lies within s cells (Chebyshev) of S_0, the cells
// with initial burning mass, and v within s + 1; it needs the adjoint of
// step s + 1 there.  That in turn is exact wherever its inputs of step s + 2
// are, one cell further out, and so on up to the seed at T.  So the adjoint
// step s must be exact only within s + 1 cells of S_0, and a tile farther
// from every cell of S_0 can be skipped: whatever its cells hold (finite:
// the buffers start at zero) only ever meets B = 0 in the gradient sums.
// Its cells' adjoint values are then not those of the dense sweep; only
// the parameter gradient is returned.
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
    for (int idx = threadIdx.x; idx < BW * BH; idx += 256) {
        const int gi = td.r0 + idx / BW, gj = td.c0 + idx % BW;
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

// Does the adjoint step s need this tile: is a tile with initial mass within
// a = floor(s / BH) + 1 tile rows and b = floor(s / BW) + 1 tile columns
// (the tile bands whose nearest cells are at most s + 1 apart)?
__device__ __forceinline__ bool tile_in_reach(const RelaxedTile& td, const TileGrid* grids, const int32_t* integ,
                                              int32_t s)
{
    const TileGrid tg = grids[td.env];
    const int i = td.r0 / BH, j = td.c0 / BW;
    const int a = s / BH + 1, b = s / BW + 1;
    const int i0 = max(i - a, 0), i1 = min(i + a, tg.rows - 1);
    const int j0 = max(j - b, 0), j1 = min(j + b, tg.cols - 1);
    const int32_t* I = integ + tg.ioff;
    const int W1 = tg.cols + 1;
    return I[(i1 + 1) * W1 + (j1 + 1)] - I[i0 * W1 + (j1 + 1)] - I[(i1 + 1) * W1 + j0] + I[i0 * W1 + j0] > 0;
}

// Atomic add to a double in LDS (ds_add_f64).
__device__ __forceinline__ void lds_add(double* p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wind exponent of direction k at a staged source cell (per env, or from the
// staged per-cell wind).
template <bool WC>
__device__ __forceinline__ float staged_wind(int k, const float* ew, const float* sW, int s, int nx,
                                             const RelaxedArgs& A)
{
    if constexpr (WC)
        return wind_exponent(k, A.alpha_w1, A.alpha_w2, sW[s], sW[nx + s], sW[2 * nx + s]);
    else
        return ew[k];
}

// One adjoint step on a 32 x 20 tile: (U_t, B_t), (Ubar_{t+1}, Bbar_{t+1})
// -> (Ubar_t, Bbar_t), and the step's contribution to the parameter gradient.
// Both forms reduce to per-edge phibar_k and per-target gammabar:
//   FORM 0: ybar_k = Pbar B_k E_k exp(-y_k), phibar_k = ybar_k gamma,
//           gammabar = sum_k ybar_k phi_k, c_k = Pbar q_k E_k;
//   FORM 1: lambdabar = Pbar gamma (1 - P), phibar_k = lambdabar B_k,
//           gammabar = Pbar lambda (1 - P), c_k = lambdabar phi_k.
// The targets are the tile and its one-cell ring (34 x 22 = 748, three
// passes of 256 lanes); each target adds c_k and the source-side fuel adjoint to
// the LDS slots of its sources inside the tile, so per tile cell only two
// doubles of LDS are needed and occupancy is set by registers.
template <bool WC, int FORM>
__global__ __launch_bounds__(256) void relaxed_bwd_kernel(
    const RelaxedTile* __restrict__ tiles, const EnvDev* __restrict__ envs, const float* __restrict__ g,
    const float* __restrict__ E, const float* __restrict__ wind, const uint8_t* __restrict__ cls,
    const float* __restrict__ den, int64_t n_cells, RelaxedArgs A, const double* __restrict__ U,
    const double* __restrict__ B, const double* __restrict__ gU1, const double* __restrict__ gB1,
    double* __restrict__ gU0, double* __restrict__ gB0, double* __restrict__ stripes,
    const float* __restrict__ env_wind, const TileGrid* __restrict__ grids, const int32_t* __restrict__ integ,
    int32_t step)
{
    constexpr int XW = BW + 4, XH = BH + 4;  // staged: the targets' sources
    constexpr int EW = BW + 2, EH = BH + 2;  // targets: the tile and its ring
    constexpr int NX = XW * XH, NE = EW * EH, NT = BW * BH;
    __shared__ double sB[NX];
    __shared__ float sg[NX], sE[NX];
    __shared__ float sW[WC ? 3 * NX : 1];      // per-cell wind V, Vx, Vy of the staged cells
    __shared__ double sBbar[NT], sFbar[NT];  // per tile cell: sum_k c_k, fuel adjoint
    __shared__ float ew[8];
    __shared__ double sred[4][17];
    const RelaxedTile td = tiles[blockIdx.x];
    if (integ && !tile_in_reach(td, grids, integ, step)) return;  // sparse: the whole workgroup
    const EnvDev ed = envs[td.env];
    const int H = ed.H, W = ed.W, tid = threadIdx.x;
    for (int idx = tid; idx < NX; idx += 256) {
        const int gi = td.r0 - 2 + idx / XW, gj = td.c0 - 2 + idx % XW;
        const bool in = gi >= 0 && gi < H && gj >= 0 && gj < W;
        const int64_t v = ed.offset + (int64_t)gi * W + gj;
        sB[idx] = in ? B[v] : 0.0;
        sg[idx] = in ? g[v] : 0.0f;
        sE[idx] = in ? E[v] : 0.0f;
        if constexpr (WC) {
            sW[idx] = in ? wind[v] : 0.0f;
            sW[NX + idx] = in ? wind[n_cells + v] : 0.0f;
            sW[2 * NX + idx] = in ? wind[2 * n_cells + v] : 0.0f;
        }
    }
    for (int idx = tid; idx < NT; idx += 256) sBbar[idx] = sFbar[idx] = 0.0;
    const float3 wenv = env_wind_of(ed, env_wind, td.env);  // this step's per-env wind
    if (!WC && tid < 8) ew[tid] = wind_exponent(tid, A.alpha_w1, A.alpha_w2, wenv.x, wenv.y, wenv.z);
    __syncthreads();

    double acc[17];
#pragma unroll
    for (int j = 0; j < 17; ++j) acc[j] = 0.0;
    double xbar_sin = 0.0;  // per-env wind: sum of xbar sin(k pi / 4)
    const double p_base = A.p_base, a_gamma = A.alpha_gamma;

    // phase 1: every target of the tile, then its ring (top and bottom rows,
    // left and right columns), so that waves of ring targets, which only
    // feed the few edges into the tile, mostly skip the edge work together
    for (int idx = tid; idx < NE; idx += 256) {
        int er, ec;
        if (idx < NT) {
            er = 1 + idx / BW;
            ec = 1 + idx % BW;
        } else {
            const int r = idx - NT;
            if (r < 2 * EW) {
                er = r < EW ? 0 : EH - 1;
                ec = r < EW ? r : r - EW;
            } else {
                er = 1 + (r - 2 * EW) % BH;
                ec = r < 2 * EW + BH ? 0 : EW - 1;
            }
        }
        const int gi = td.r0 - 1 + er, gj = td.c0 - 1 + ec;
        if (gi < 0 || gi >= H || gj < 0 || gj >= W) continue;
        const int64_t v = ed.offset + (int64_t)gi * W + gj;
        const int a = er + 1, b = ec + 1;  // staged coordinates of v
        const double Uv = U[v];
        const double gU = gU1[v], gB = gB1[v];
        const double nbar = gB - gU;
        const double Pbar = nbar * Uv;
        const float gv = sg[a * XW + b], Ev = sE[a * XW + b];
        const float gam = A.alpha_gamma * gv;
        float q[8], em[8], ex[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int s = (a - kDRow[k]) * XW + (b - kDCol[k]);
            // Off-grid sources are staged with zero fuel and zero B, so their
            // q, c and phibar vanish without a bounds check; the exponent is
            // capped below fp32 overflow so that their elevation term cannot
            // turn 0 x e^x into 0 x inf.
            const float x = staged_wind<WC>(k, ew, sW, s, NX, A) +
                            A.alpha_s * slope_of((Ev - sE[s]) * ((k & 1) ? A.inv_diag : A.inv_orth), A);
            ex[k] = hexp(fminf(x, 88.0f));
            if constexpr (FORM == 0) {
                const float2 qe = q_and_survival(gam * (A.p_base * sg[s] * ex[k]));
                q[k] = qe.x;
                em[k] = qe.y;
            }
        }
        // The later loops read B, g (and E) of the sources from LDS again
        // instead of keeping them in registers across the loops.
        asm volatile("" ::: "memory");
        // FORM 0: exclusive products from stored prefixes and a running suffix
        double pre[8];
        double P, gam_bar = 0.0, lbar = 0.0;
        if constexpr (FORM == 0) {
            double run = 1.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                pre[k] = run;
                run = run * (1.0 - (double)q[k] * sB[(a - kDRow[k]) * XW + (b - kDCol[k])]);
            }
            P = 1.0 - run;
        } else {
            double lam = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int s = (a - kDRow[k]) * XW + (b - kDCol[k]);
                lam = lam + (double)(A.p_base * sg[s] * ex[k]) * sB[s];
            }
            const double surv = exp(-(double)gam * lam);
            P = -expm1(-(double)gam * lam);
            lbar = Pbar * (double)gam * surv;
            gam_bar = Pbar * lam * surv;
        }
        const bool interior = idx < NT;
        double suf = 1.0;
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 7; k >= 0; --k) {
            const int s = (a - kDRow[k]) * XW + (b - kDCol[k]);
            const double Bu = sB[s];
            // the source u = v - D_k in tile coordinates
            const int tr = er - 1 - kDRow[k], tc = ec - 1 - kDCol[k];
            const bool to_tile = tr >= 0 && tr < BH && tc >= 0 && tc < BW;
            double excl = 0.0;
            if constexpr (FORM == 0) {
                excl = pre[k] * suf;
                suf = suf * (1.0 - (double)q[k] * Bu);
            }
            // a ring target only feeds the edges whose source is in the tile
            if (!interior && !to_tile) continue;
            const float ph = A.p_base * sg[s] * ex[k];
            double c, phibar;
            if constexpr (FORM == 0) {
                const double pe = Pbar * excl;
                const double ybar = pe * Bu * (double)em[k];  // qbar dq/dy
                c = pe * (double)q[k];
                phibar = ybar * (double)gam;
                gam_bar += ybar * (double)ph;
            } else {
                c = lbar * (double)ph;
                phibar = lbar * Bu;
            }
            const double d = phibar * (p_base * (double)ex[k]);  // -> gbar(source)
            if (to_tile) {
                const int t = tr * BW + tc;
                lds_add(&sBbar[t], c);
                lds_add(&sFbar[t], d);
            }
            if (interior) {
                const double gu = sg[s];
                const double xbar = d * gu;  // phibar dphi/dx
                acc[0] += phibar * (gu * (double)ex[k]);
                if constexpr (WC) {
                    const float V = sW[s], Vx = sW[NX + s], Vy = sW[2 * NX + s];
                    acc[1] += xbar * (double)V;
                    acc[2] += xbar * (double)((kCos[k] * Vx + kSin[k] * Vy) - V);
                } else {  // the env's wind is common to the tile: factored out below
                    acc[1] += xbar;
                    acc[2] += xbar * (double)kCos[k];
                    xbar_sin += xbar * (double)kSin[k];
                }
                acc[3] += xbar * (double)slope_of((Ev - sE[s]) * ((k & 1) ? A.inv_diag : A.inv_orth), A);
            }
        }
        if (interior) {
            gU0[v] = gU + nbar * P;
            acc[4] += gam_bar * (double)gv;
            acc[5] += gB * sB[a * XW + b];
            lds_add(&sFbar[(er - 1) * BW + (ec - 1)], gam_bar * a_gamma);
        }
    }
    __syncthreads();

    // phase 2: the tile's own cells
    for (int idx = tid; idx < NT; idx += 256) {
        const int rr = idx / BW, cc = idx % BW;
        const int gi = td.r0 + rr, gj = td.c0 + cc;
        if (gi >= H || gj >= W) continue;
        const int64_t u = ed.offset + (int64_t)gi * W + gj;
        gB0[u] = (double)A.p_continue * gB1[u] + sBbar[idx];
        const double gb = sFbar[idx] * (1.0 + (double)den[u]);
        const int c = cls[u];
#pragma unroll
        for (int j = 0; j < 11; ++j) acc[6 + j] += (c == j) ? gb : 0.0;
    }

    if constexpr (!WC) {
        // acc[1] and acc[2] hold the sums of xbar and xbar cos(k pi / 4)
        const double V = wenv.x, Vx = wenv.y, Vy = wenv.z, s0 = acc[1];
        acc[1] = s0 * V;
        acc[2] = (acc[2] * Vx + xbar_sin * Vy) - s0 * V;
    }

    // workgroup reduction of the 17 partial sums, then one fp64 stripe
    wave_sum17(acc, tid & 63, sred[tid >> 6]);
    __syncthreads();
    if (tid < 17) {
        const double total = sred[0][tid] + sred[1][tid] + sred[2][tid] + sred[3][tid];
        if (total != 0.0) unsafeAtomicAdd(stripes + (blockIdx.x % kGradStripes) * 17 + tid, total);
    }
}

__global__ void stripes_sum_kernel(const double* __restrict__ stripes, double* __restrict__ grad)
{
    const int j = threadIdx.x;
    if (j >= 17) return;
    double s = 0.0;
    for (int r = 0; r < kGradStripes; ++r) s += stripes[r * 17 + j];
    grad[j] = s;
}

// ---------------------------------------------------------------- losses
// Every reduction below runs in a fixed order (lane-strided partial sums,
// xor butterflies, then the four wave sums in order), so the losses, the
// objective and the seed are the same bits on every call.

// Sum over the 64 lanes of a wave (every lane receives it).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

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
    size_t g, ckpt, seg, fwd, adj, stripes, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WsLayout layout(int64_t n, int32_t T, int32_t k)
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
    L.stripes = o;
    o = align256(o + sizeof(double) * kGradStripes * 17);
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
    hipLaunchKernelGGL((relaxed_fwd_kernel<WC, FORM>), dim3(in.n_tiles), dim3(256), 0, s, in.tiles,
                       in.envs, g, in.E, in.wind, in.n_cells, A, U, B, Uo, Bo, in.env_wind);
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
void launch_bwd(hipStream_t s, const RelaxedInputs& in, const RelaxedState& R, const RelaxedArgs& A,
                const float* g, const double* U, const double* B, const double* gU1, const double* gB1,
                double* gU0, double* gB0, double* stripes, const int32_t* integ, int32_t step)
{
    hipLaunchKernelGGL((relaxed_bwd_kernel<WC, FORM>), dim3(R.n_btiles), dim3(256), 0, s, R.d_btiles,
                       in.envs, g, in.E, in.wind, in.cls, in.den, in.n_cells, A, U, B, gU1, gB1, gU0,
                       gB0, stripes, in.env_wind, R.d_tgrid, integ, step);
}

}  // namespace

int relaxed_prepare(RelaxedState& R, const std::vector<sim_env>& envs)
{
    if (R.d_tiles) return 0;
    std::vector<RelaxedTile> tiles, btiles;
    std::vector<TileGrid> grids;
    int64_t ioff = 0, max_img = 0;
    for (int32_t e = 0; e < (int32_t)envs.size(); ++e) {
        for (int r0 = 0; r0 < envs[e].H; r0 += TH)
            for (int c0 = 0; c0 < envs[e].W; c0 += TW) tiles.push_back(RelaxedTile{e, r0, c0, 0});
        TileGrid tg{(int32_t)btiles.size(), (envs[e].H + BH - 1) / BH, (envs[e].W + BW - 1) / BW, (int32_t)ioff};
        for (int r0 = 0; r0 < envs[e].H; r0 += BH)
            for (int c0 = 0; c0 < envs[e].W; c0 += BW) btiles.push_back(RelaxedTile{e, r0, c0, 0});
        const int64_t img = (int64_t)(tg.rows + 1) * (tg.cols + 1);
        ioff += img;
        max_img = std::max(max_img, img);
        grids.push_back(tg);
    }
    if (hipMalloc(&R.d_tiles, tiles.size() * sizeof(RelaxedTile)) != hipSuccess) return -1;
    if (hipMemcpy(R.d_tiles, tiles.data(), tiles.size() * sizeof(RelaxedTile), hipMemcpyHostToDevice) !=
        hipSuccess)
        return -1;
    if (hipMalloc(&R.d_btiles, btiles.size() * sizeof(RelaxedTile)) != hipSuccess) return -1;
    if (hipMemcpy(R.d_btiles, btiles.data(), btiles.size() * sizeof(RelaxedTile),
                  hipMemcpyHostToDevice) != hipSuccess)
        return -1;
    R.n_tiles = (int32_t)tiles.size();
    R.n_btiles = (int32_t)btiles.size();
    R.n_env = (int32_t)envs.size();
    if (ioff < INT32_MAX && 4 * max_img <= 64 * 1024) {
        if (hipMalloc(&R.d_tgrid, grids.size() * sizeof(TileGrid)) != hipSuccess ||
            hipMalloc(&R.d_tmass, btiles.size() * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&R.d_tinteg, (size_t)ioff * sizeof(int32_t)) != hipSuccess)
            return -1;
        if (hipMemcpy(R.d_tgrid, grids.data(), grids.size() * sizeof(TileGrid), hipMemcpyHostToDevice) !=
            hipSuccess)
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
    for (void* p : {(void*)R.d_tiles, (void*)R.d_btiles, (void*)R.d_pool,
                    (void*)R.d_env_blocks, (void*)R.d_pool_vals, (void*)R.d_bce_loss, (void*)R.d_tgrid,
                    (void*)R.d_tmass, (void*)R.d_tinteg})
        if (p) (void)hipFree(p);
    R = RelaxedState{};
}

size_t relaxed_workspace_bytes(int64_t n_cells, int32_t T, int32_t ckpt_every)
{
    return layout(n_cells, T, ckpt_every).total;
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
    const WsLayout L = layout(n, T, k);
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
    const WsLayout L = layout(n, T, k);
    char* ws = static_cast<char*>(workspace);
    float* g = reinterpret_cast<float*>(ws + L.g);
    double* ckpt = reinterpret_cast<double*>(ws + L.ckpt);
    double* seg = reinterpret_cast<double*>(ws + L.seg);
    double* adj = reinterpret_cast<double*>(ws + L.adj);
    double* stripes = reinterpret_cast<double*>(ws + L.stripes);
    const RelaxedArgs A = relaxed_args(p);
    hipError_t e = fill_f64(s, stripes, (int64_t)kGradStripes * 17, 0.0);
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
            if (it.wind)
                it.form ? launch_bwd<true, 1>(s, it, R, A, g, Ut, Bt, cu, cb, nu, nb, stripes, integ, t)
                        : launch_bwd<true, 0>(s, it, R, A, g, Ut, Bt, cu, cb, nu, nb, stripes, integ, t);
            else
                it.form ? launch_bwd<false, 1>(s, it, R, A, g, Ut, Bt, cu, cb, nu, nb, stripes, integ, t)
                        : launch_bwd<false, 0>(s, it, R, A, g, Ut, Bt, cu, cb, nu, nb, stripes, integ, t);
            e = hipGetLastError();
            std::swap(cu, nu);
            std::swap(cb, nb);
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(stripes_sum_kernel, dim3(1), dim3(64), 0, s, stripes, grad);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace firesim
