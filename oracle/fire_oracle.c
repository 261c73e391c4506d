/*
 * fire_oracle.c -- CPU oracle for the stochastic fire-spread cellular automaton.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP implementation: every constant below is derived here from its
 * mathematical definition.
 *
 * It is deliberately plain: one env after another, one cell after another,
 * no blocking and no fusion beyond what the model itself states.  It follows
 * the paper (JaxWildfire, arXiv 2512.06102) section 3, "JaxWildfire Simulator":
 *
 *   state layers (fire state, wind, vegetation, density, slope)  -- "State
 *     representation";
 *   kappa_wind, kappa_slope, phi                                    -- Eqs. 1-3;
 *   p_ignite = 1 - exp(-gamma(v) * lambda), lambda = sum b(u) phi     -- Eq. 4
 *     with gamma(v) = alpha_gamma (1 + mu_veg(v)) (1 + mu_den(v));
 *   stochastic update (independent Bernoulli draws; burning cells continue
 *     with p_continue, otherwise burn out)                           -- "Stochastic
 *     update" paragraph.
 *
 * Fixed readings (the paper does not pin these; the HIP path uses the same):
 *   - 4 states: 0 UNBURNABLE (no fuel, never changes), 1 FLAMMABLE (the paper's
 *     "unburned"), 2 BURNING, 3 BURNT.
 *   - Directions k = 0..7 at angle k*pi/4 counter-clockwise from east; rows
 *     grow southward, so k=1 (north-east) is (di,dj) = (-1,+1).
 *   - Theta is the direction the wind blows toward.
 *   - Slope S(u,k) = (E(u+D_k) - E(u)) / distance, distance = cs or cs*sqrt(2).
 *   - kappa_wind * kappa_slope is evaluated as one exponential of the summed
 *     exponents (exp(a) exp(b) exp(c) = exp(a+b+c)), and
 *     V cos(phi_k - Theta) = cos(phi_k) Vx + sin(phi_k) Vy with the wind given
 *     as (V, Vx = V cos Theta, Vy = V sin Theta).
 *   - Off-grid neighbours are not burning (no wrap).
 *   - One uniform per cell per step from Philox4x32-10 (Salmon et al., SC'11)
 *     at counter (n>>2, t, env_id, 0), key (seed lo, seed hi), word n&3,
 *     u = (word >> 8) * 2^-24; ignite iff u < p_ignite; a burning cell burns
 *     out iff !(u < p_continue).
 *   - Synchronous update: every read comes from the state after the step's
 *     suppression action; newly ignited cells spread from the next step on.
 *   - Suppression action a = (r<<16)|c (or -1 for none): every FLAMMABLE or
 *     BURNING cell of the 5x5 square centred on (r,c), clipped to the grid,
 *     becomes UNBURNABLE before the step; a centre outside the grid is a no-op.
 *   - Arithmetic is fp32, in the order written, with no contraction into FMA
 *     (built with -ffp-contract=off) and with denormals kept.
 *   - exp is this file's own exp_c: Cody-Waite range reduction and a degree-7
 *     Taylor polynomial (Cody & Waite, "Software Manual for the Elementary
 *     Functions", 1980), valid on [-87, 88]; below -87 it returns 0, above 88
 *     it returns exp_c(88).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ST_UNBURNABLE = 0, ST_FLAMMABLE = 1, ST_BURNING = 2, ST_BURNT = 3 };

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11, section 4.2).                                     */
/* ------------------------------------------------------------------------- */
#define PHILOX_MUL_A 0xD2511F53u
#define PHILOX_MUL_B 0xCD9E8D57u
#define PHILOX_WEYL_A 0x9E3779B9u /* golden ratio */
#define PHILOX_WEYL_B 0xBB67AE85u /* sqrt(3) - 1   */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_WEYL_A;
            k1 += PHILOX_WEYL_B;
        }
        uint64_t pa = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
        uint64_t pb = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)pb;
        uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)pa;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void oracle_philox_blocks(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) oracle_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* Uniform in [0, 1 - 2^-24] for cell n of env env_id at absolute step t. */
static float cell_uniform(uint64_t seed, uint32_t env_id, uint64_t t, uint64_t n)
{
    uint32_t ctr[4] = {(uint32_t)(n >> 2), (uint32_t)t, env_id, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    uint32_t word = out[n & 3u];
    return (float)(word >> 8) * (1.0f / 16777216.0f);
}

/* ------------------------------------------------------------------------- */
/* exp_c: Cody-Waite reduction x = n ln2 + r, |r| <~ ln2/2, then             */
/* e^r by its Taylor series to degree 7 (truncation < r^8/8! < 6e-9) and      */
/* e^x = 2^n e^r.  ln2 is split as LN2_HI (15 significant bits, so n*LN2_HI   */
/* is exact for |n| < 2^9) plus LN2_LO.                                       */
/* ------------------------------------------------------------------------- */
static const double LN2_D = 0.69314718055994530942;
static const float LN2_HI = 0.693145751953125f; /* 22713 / 2^15 */

float oracle_exp_c(float x)
{
    const float log2e = (float)1.44269504088896340736; /* 1/ln2 */
    const float ln2_lo = (float)(LN2_D - 0.693145751953125);
    const float c0 = 1.0f, c1 = 1.0f, c2 = 0.5f;
    const float c3 = (float)(1.0 / 6.0), c4 = (float)(1.0 / 24.0);
    const float c5 = (float)(1.0 / 120.0), c6 = (float)(1.0 / 720.0);
    const float c7 = (float)(1.0 / 5040.0);
    if (x != x) return x;
    if (x < -87.0f) return 0.0f;
    if (x > 88.0f) x = 88.0f;
    float n = rintf(x * log2e);
    float r = (x - n * LN2_HI) - n * ln2_lo;
    float p = c7;
    p = p * r + c6;
    p = p * r + c5;
    p = p * r + c4;
    p = p * r + c3;
    p = p * r + c2;
    p = p * r + c1;
    p = p * r + c0;
    /* 2^n as an fp32 bit pattern; n is in [-126, 127] on the clamped range */
    union { uint32_t u; float f; } scale;
    scale.u = (uint32_t)((int)n + 127) << 23;
    return p * scale.f;
}

void oracle_exp_c_batch(const float* x, float* y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = oracle_exp_c(x[i]);
}

/* ------------------------------------------------------------------------- */
/* atan_c: the arctangent of the slope-angle variant (S = atan(rise / run)),  */
/* in fp32 from the mathematics: atan is odd; for |x| > 1 use                 */
/* atan(x) = pi/2 - atan(1/x); above tan(pi/8) use                            */
/* atan(a) = pi/4 + atan((a - 1) / (a + 1)); on the remaining |t| <= tan(pi/8) */
/* the Taylor series t - t^3/3 + ... - t^19/19 (Horner in t^2, coefficients   */
/* rounded to fp32, separate multiply and add).  Divisions are IEEE.          */
/* ------------------------------------------------------------------------- */
float oracle_atan_c(float x)
{
    const float tan_pi8 = (float)0.41421356237309504880;
    const float pi4 = (float)0.78539816339744830962, pi2 = (float)1.57079632679489661923;
    if (x != x) return x;
    const int neg = x < 0.0f;
    float a = neg ? -x : x;
    const int inv = a > 1.0f;
    if (inv) a = 1.0f / a;
    float base = 0.0f, t = a;
    if (a > tan_pi8) {
        t = (a - 1.0f) / (a + 1.0f);
        base = pi4;
    }
    const float t2 = t * t;
    float p = (float)(-1.0 / 19.0);
    p = p * t2 + (float)(1.0 / 17.0);
    p = p * t2 + (float)(-1.0 / 15.0);
    p = p * t2 + (float)(1.0 / 13.0);
    p = p * t2 + (float)(-1.0 / 11.0);
    p = p * t2 + (float)(1.0 / 9.0);
    p = p * t2 + (float)(-1.0 / 7.0);
    p = p * t2 + (float)(1.0 / 5.0);
    p = p * t2 + (float)(-1.0 / 3.0);
    p = p * t2 + 1.0f;
    float r = base + t * p;
    if (inv) r = pi2 - r;
    return neg ? -r : r;
}

void oracle_atan_c_batch(const float* x, float* y, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = oracle_atan_c(x[i]);
}

/* Error of exp_c against the fp64 exp, in units of the fp32 ulp of the true  */
/* value, over every fp32 in [lo, hi]; multi-threaded over bit-pattern        */
/* ranges.  Returns the max error; *worst receives its argument.              */
typedef struct { uint32_t b0, b1; int neg; double maxerr; float worst; } sweep_job;

static double ulp_of(double v)
{
    int e;
    frexp(v, &e);               /* v = m 2^e, m in [0.5,1) */
    if (e - 24 < -149) return ldexp(1.0, -149);
    return ldexp(1.0, e - 24);
}

static void* sweep_worker(void* arg)
{
    sweep_job* j = (sweep_job*)arg;
    double mx = 0.0;
    float worst = 0.0f;
    for (uint64_t b = j->b0; b <= j->b1; ++b) {
        union { uint32_t u; float f; } v;
        v.u = (uint32_t)b | (j->neg ? 0x80000000u : 0u);
        double ref = exp((double)v.f);
        double err = fabs((double)oracle_exp_c(v.f) - ref) / ulp_of(ref);
        if (err > mx) { mx = err; worst = v.f; }
    }
    j->maxerr = mx;
    j->worst = worst;
    return NULL;
}

/* Sweep the fp32 values of one sign between magnitudes |a| <= |x| <= |b|.   */
double oracle_exp_c_sweep(float amag, float bmag, int negative, int n_threads, float* worst)
{
    union { float f; uint32_t u; } a, b;
    a.f = amag; b.f = bmag;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 64) n_threads = 64;
    pthread_t th[64];
    sweep_job jobs[64];
    uint64_t span = (uint64_t)b.u - a.u + 1;
    for (int i = 0; i < n_threads; ++i) {
        jobs[i].b0 = (uint32_t)(a.u + span * i / n_threads);
        jobs[i].b1 = (uint32_t)(a.u + span * (i + 1) / n_threads - 1);
        jobs[i].neg = negative;
        pthread_create(&th[i], NULL, sweep_worker, &jobs[i]);
    }
    double mx = 0.0;
    float w = 0.0f;
    for (int i = 0; i < n_threads; ++i) {
        pthread_join(th[i], NULL);
        if (jobs[i].maxerr > mx) { mx = jobs[i].maxerr; w = jobs[i].worst; }
    }
    if (worst) *worst = w;
    return mx;
}

/* ------------------------------------------------------------------------- */
/* Model inputs                                                               */
/* ------------------------------------------------------------------------- */
typedef struct {
    float p_base;      /* Eq. 3 base propagation factor                 */
    float alpha_gamma; /* susceptibility scale, gamma(v)                */
    float alpha_w1;    /* Eq. 1                                         */
    float alpha_w2;    /* Eq. 1                                         */
    float alpha_s;     /* Eq. 2                                         */
    float p_continue;  /* stochastic update: burning stays burning      */
    float cell_size;   /* metres per cell edge (slope denominator)      */
    int32_t slope_mode; /* 0: S = rise / run; 1: S = atan(rise / run)   */
} oracle_params;

typedef struct {
    int64_t offset;  /* first cell of this env in the packed arrays   */
    int32_t H, W;    /* rows, columns                                 */
    uint32_t env_id; /* RNG stream id                                 */
    float V, Vx, Vy; /* per-env wind: speed and V cos/sin Theta       */
} oracle_env;

/* Neighbour offsets: direction k points from a source u to its target       */
/* v = u + D_k; angle k*pi/4 counter-clockwise from east, rows grow south.   */
static const int DI[8] = {0, -1, -1, -1, 0, 1, 1, 1};
static const int DJ[8] = {1, 1, 0, -1, -1, -1, 0, 1};

/* cos and sin of k*pi/4, rounded to fp32 from their exact values. */
static void direction_cos_sin(float cx[8], float sy[8])
{
    const float h = (float)sqrt(0.5);
    const float c[8] = {1.0f, h, 0.0f, -h, -1.0f, -h, 0.0f, h};
    const float s[8] = {0.0f, h, 1.0f, h, 0.0f, -h, -1.0f, -h};
    for (int k = 0; k < 8; ++k) { cx[k] = c[k]; sy[k] = s[k]; }
}

/* Fuel term (1 + mu_veg(u)) (1 + mu_den(u)) shared by Eq. 3 and gamma(v). */
void oracle_fuel(int64_t n, const uint8_t* cls, const float* den, const float* veg11, float* g)
{
    for (int64_t i = 0; i < n; ++i) g[i] = (1.0f + veg11[cls[i]]) * (1.0f + den[i]);
}

/* Initial fire state: classes in unburnable_mask (bit c set) hold no fuel;   */
/* every other cell is FLAMMABLE; each ignition (env, i, j) sets a FLAMMABLE */
/* cell BURNING.                                                             */
int oracle_init_states(int32_t n_env, const oracle_env* envs, const uint8_t* cls,
                       uint32_t unburnable_mask, const int32_t* ign, int32_t n_ign,
                       uint8_t* states)
{
    for (int32_t e = 0; e < n_env; ++e) {
        int64_t n = (int64_t)envs[e].H * envs[e].W;
        for (int64_t c = 0; c < n; ++c) {
            int64_t idx = envs[e].offset + c;
            states[idx] = ((unburnable_mask >> cls[idx]) & 1u) ? ST_UNBURNABLE : ST_FLAMMABLE;
        }
    }
    for (int32_t q = 0; q < n_ign; ++q) {
        int32_t e = ign[3 * q], i = ign[3 * q + 1], j = ign[3 * q + 2];
        if (e < 0 || e >= n_env || i < 0 || i >= envs[e].H || j < 0 || j >= envs[e].W) return -1;
        int64_t idx = envs[e].offset + (int64_t)i * envs[e].W + j;
        if (states[idx] == ST_FLAMMABLE) states[idx] = ST_BURNING;
    }
    return 0;
}

/* Wind at the source cell u: per env (V, Vx, Vy of the current step), or   */
/* per cell when wind_cell is given as three planes [V | Vx | Vy] of n_cells */
/* each (the planes of the current step).                                    */
typedef struct {
    const oracle_params* P;
    const oracle_env* env;
    const float* g;
    const float* E;
    const float* wind_cell;
    int64_t n_cells;
    float V, Vx, Vy;
    float cx[8], sy[8], invd[8];
} step_ctx;

static void init_ctx(step_ctx* c, const oracle_params* P, const oracle_env* env, const float* g,
                     const float* E, const float* wind_cell, int64_t n_cells)
{
    c->P = P;
    c->env = env;
    c->g = g;
    c->E = E;
    c->wind_cell = wind_cell;
    c->n_cells = n_cells;
    c->V = env->V;
    c->Vx = env->Vx;
    c->Vy = env->Vy;
    direction_cos_sin(c->cx, c->sy);
    for (int k = 0; k < 8; ++k)
        c->invd[k] = (k & 1) ? (float)(1.0 / ((double)P->cell_size * sqrt(2.0)))
                             : (float)(1.0 / (double)P->cell_size);
}

/* phi(u, k): Eq. 3 with Eqs. 1-2, source u (packed index), target v. */
static float phi_uk(const step_ctx* c, int64_t u, int64_t v, int k)
{
    const oracle_params* P = c->P;
    float V, Vx, Vy;
    if (c->wind_cell) {
        V = c->wind_cell[u];
        Vx = c->wind_cell[c->n_cells + u];
        Vy = c->wind_cell[2 * c->n_cells + u];
    } else {
        V = c->V;
        Vx = c->Vx;
        Vy = c->Vy;
    }
    /* exponent of kappa_wind: alpha_w1 V + alpha_w2 V (cos(phi_k - Theta) - 1) */
    float wind_exp = P->alpha_w1 * V + P->alpha_w2 * ((c->cx[k] * Vx + c->sy[k] * Vy) - V);
    /* exponent of kappa_slope: alpha_s S(u, k), S = rise over run toward v   */
    /* (or its angle, in radians)                                             */
    float slope = (c->E[v] - c->E[u]) * c->invd[k];
    if (P->slope_mode) slope = oracle_atan_c(slope);
    float x = wind_exp + P->alpha_s * slope;
    return (P->p_base * c->g[u]) * oracle_exp_c(x);
}

/* p_ignite(v) for a FLAMMABLE cell v=(i,j) of state array F (Eq. 4). */
static float ignite_prob(const step_ctx* c, const uint8_t* F, int32_t i, int32_t j)
{
    const oracle_env* e = c->env;
    int64_t v = e->offset + (int64_t)i * e->W + j;
    float lambda = 0.0f;
    for (int k = 0; k < 8; ++k) {
        int32_t ui = i - DI[k], uj = j - DJ[k];
        if (ui < 0 || ui >= e->H || uj < 0 || uj >= e->W) continue;
        int64_t u = e->offset + (int64_t)ui * e->W + uj;
        if (F[u] != ST_BURNING) continue;
        lambda = lambda + phi_uk(c, u, v, k);
    }
    if (!(lambda > 0.0f)) return 0.0f;
    float gamma = c->P->alpha_gamma * c->g[v];
    return 1.0f - oracle_exp_c(-(gamma * lambda));
}

/* Exposed for the closed-form tests: p_ignite of one cell of one env. */
float oracle_cell_prob(const oracle_params* P, const oracle_env* env, const float* g, const float* E,
                       const float* wind_cell, int64_t n_cells, const uint8_t* states, int32_t i, int32_t j)
{
    step_ctx c;
    init_ctx(&c, P, env, g, E, wind_cell, n_cells);
    return ignite_prob(&c, states, i, j);
}

/* A drop on the (2R+1) x (2R+1) square centred at (r, col), clipped to the  */
/* grid: mode 0 (suppressant) makes FLAMMABLE and BURNING cells UNBURNABLE,  */
/* mode 1 (water, section 4) makes BURNING cells BURNT.                      */
static void apply_action(const oracle_env* e, uint8_t* F, int32_t a, int32_t mode, int32_t R)
{
    if (a < 0) return;
    int32_t r = (a >> 16) & 0x7FFF, col = a & 0xFFFF;
    if (r >= e->H || col >= e->W) return;
    for (int32_t i = r - R; i <= r + R; ++i) {
        if (i < 0 || i >= e->H) continue;
        for (int32_t j = col - R; j <= col + R; ++j) {
            if (j < 0 || j >= e->W) continue;
            uint8_t* s = &F[e->offset + (int64_t)i * e->W + j];
            if (mode == 0) {
                if (*s == ST_FLAMMABLE || *s == ST_BURNING) *s = ST_UNBURNABLE;
            } else {
                if (*s == ST_BURNING) *s = ST_BURNT;
            }
        }
    }
}

/* Advance one env by T steps from absolute step t0.  actions/counts are    */
/* [T][n_env] (row s holds step t0+s) or NULL.  A wind series, when given,   */
/* is indexed by the absolute step t: env_series [t][n_env][3] or            */
/* cell_series [t][3][n_cells]; it replaces the static wind of that step.    */
static void run_env(const oracle_params* P, int32_t n_env, int32_t e, const oracle_env* envs,
                    const float* g, const float* E, const float* wind_cell, int64_t n_cells,
                    uint8_t* states, uint64_t t0, int32_t T, const int32_t* actions, int32_t* counts,
                    uint64_t seed, const float* env_series, const float* cell_series, int32_t drop_mode,
                    int32_t drop_radius)
{
    const oracle_env* env = &envs[e];
    int64_t n = (int64_t)env->H * env->W;
    uint8_t* next = (uint8_t*)malloc((size_t)n);
    step_ctx c;
    init_ctx(&c, P, env, g, E, wind_cell, n_cells);
    uint8_t* F = states; /* F indexed by packed index; this env's cells only */
    for (int32_t s = 0; s < T; ++s) {
        uint64_t t = t0 + (uint64_t)s;
        if (env_series) {
            const float* w = env_series + ((int64_t)t * n_env + e) * 3;
            c.V = w[0];
            c.Vx = w[1];
            c.Vy = w[2];
        }
        if (cell_series) c.wind_cell = cell_series + (int64_t)t * 3 * n_cells;
        if (actions) apply_action(env, F, actions[(int64_t)s * n_env + e], drop_mode, drop_radius);
        int32_t burning = 0;
        for (int32_t i = 0; i < env->H; ++i) {
            for (int32_t j = 0; j < env->W; ++j) {
                int64_t local = (int64_t)i * env->W + j;
                uint8_t cur = F[env->offset + local], nxt = cur;
                if (cur == ST_FLAMMABLE) {
                    float p = ignite_prob(&c, F, i, j);
                    float u = cell_uniform(seed, env->env_id, t, (uint64_t)local);
                    if (u < p) nxt = ST_BURNING;
                } else if (cur == ST_BURNING) {
                    float u = cell_uniform(seed, env->env_id, t, (uint64_t)local);
                    if (!(u < P->p_continue)) nxt = ST_BURNT;
                }
                next[local] = nxt;
                burning += (nxt == ST_BURNING);
            }
        }
        memcpy(F + env->offset, next, (size_t)n);
        if (counts) counts[(int64_t)s * n_env + e] = burning;
    }
    free(next);
}

typedef struct {
    const oracle_params* P;
    int32_t n_env;
    const oracle_env* envs;
    const float *g, *E, *wind_cell;
    int64_t n_cells;
    uint8_t* states;
    uint64_t t0;
    int32_t T;
    const int32_t* actions;
    int32_t* counts;
    uint64_t seed;
    int32_t first, stride;
    const float *env_series, *cell_series;
    int32_t drop_mode, drop_radius;
} run_job;

static void* run_worker(void* arg)
{
    run_job* j = (run_job*)arg;
    for (int32_t e = j->first; e < j->n_env; e += j->stride)
        run_env(j->P, j->n_env, e, j->envs, j->g, j->E, j->wind_cell, j->n_cells, j->states, j->t0,
                j->T, j->actions, j->counts, j->seed, j->env_series, j->cell_series, j->drop_mode,
                j->drop_radius);
    return NULL;
}

/* Run T steps on every env.  Envs are independent, so n_threads > 1 only   */
/* spreads whole envs over threads; each env is still stepped as above.     */
void oracle_run_ex(const oracle_params* P, int32_t n_env, const oracle_env* envs, const float* g,
                   const float* E, const float* wind_cell, int64_t n_cells, uint8_t* states,
                   uint64_t t0, int32_t T, const int32_t* actions, int32_t* counts, uint64_t seed,
                   int32_t n_threads, const float* env_series, const float* cell_series,
                   int32_t drop_mode, int32_t drop_radius)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    run_job jobs[256];
    pthread_t th[256];
    for (int32_t i = 0; i < n_threads; ++i) {
        run_job j = {P, n_env, envs, g, E, wind_cell, n_cells, states, t0, T, actions, counts, seed, i,
                     n_threads, env_series, cell_series, drop_mode, drop_radius};
        jobs[i] = j;
    }
    if (n_threads == 1) {
        run_worker(&jobs[0]);
        return;
    }
    for (int32_t i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, run_worker, &jobs[i]);
    for (int32_t i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
}

void oracle_run(const oracle_params* P, int32_t n_env, const oracle_env* envs, const float* g,
                const float* E, const float* wind_cell, int64_t n_cells, uint8_t* states, uint64_t t0,
                int32_t T, const int32_t* actions, int32_t* counts, uint64_t seed, int32_t n_threads)
{
    oracle_run_ex(P, n_env, envs, g, E, wind_cell, n_cells, states, t0, T, actions, counts, seed,
                  n_threads, NULL, NULL, 0, 2);
}
