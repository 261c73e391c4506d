/*
 * firesim.h -- C ABI of the MI355X (gfx950) batched fire-spread library.
 *
 * The library runs the probabilistic cellular-automaton fire-spread model of
 * JaxWildfire (arXiv 2512.06102, section 3) over a batch of independent
 * grids ("envs") on one GPU: the stochastic step (Eqs. 1-4 and the
 * "Stochastic update" paragraph) and a relaxed mean-field step with its
 * adjoint (the "Deterministic (raw-probabilities) update", Eqs. 5-10) for
 * gradient-based calibration.  Around the step: time-varying wind
 * (sim_set_wind_series), retardant or water drops (sim_set_drop), per-step
 * history (sim_step_history), the air-tanker reinforcement-learning scenario
 * of section 4 (sim_rl_reset / sim_rl_step), launch plans with temporal
 * blocking and sparse tiles, and an autotuner (sim_set_plan, sim_autotune).
 *
 * Conventions
 *  - Every pointer marked "device" is memory the caller allocated on the
 *    handle's GPU; the library never frees caller memory.  "host" pointers
 *    are read before the call returns.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *    on it and return without synchronising, except sim_init, which
 *    synchronises once at the end (its host inputs are copied in).
 *  - Return 0 on success, a negative SIM_E* code on failure; no exception
 *    crosses the ABI.  sim_last_error() gives the message of the last failure
 *    (per handle; with h == NULL the calling thread's last sim_init failure).
 *  - Layout: per-cell arrays are packed env after env (env e starts at
 *    envs[e].offset), each env row-major with H rows of W cells; row 0 is the
 *    northern edge, so row index grows southward and column index eastward.
 *  - Cell states are uint8: SIM_UNBURNABLE (no fuel), SIM_FLAMMABLE (the
 *    paper's "unburned"), SIM_BURNING, SIM_BURNT.
 *  - A handle lives on the device that was current at sim_init.  Every call
 *    on it makes that device current while it runs and restores the
 *    caller's device on return, so handles on several GPUs can be driven
 *    from one thread; `stream` must belong to the handle's device.  Calls on
 *    one handle must not overlap (they share its internal buffers and its
 *    step counter).
 *  - Each call shows as a range named after it in a marker trace
 *    (roctx; rocprofv3 --marker-trace).
 */
#ifndef FIRESIM_H
#define FIRESIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK 0
#define SIM_EINVAL (-1) /* bad argument: sizes, pointers, ranges         */
#define SIM_ENOMEM (-2) /* device allocation failed                       */
#define SIM_EHIP (-3)   /* a HIP runtime call failed (message has the why) */
#define SIM_ESTATE (-4) /* call not valid in the handle's current state   */

enum { SIM_UNBURNABLE = 0, SIM_FLAMMABLE = 1, SIM_BURNING = 2, SIM_BURNT = 3 };

#define SIM_N_CLASSES 11 /* the WorldCover legend: tree, shrub, grass, crop, built,
                            bare, snow, water, wetland, mangrove, lichen */
#define SIM_N_THETA 17   /* p_base, alpha_w1, alpha_w2, alpha_s, alpha_gamma,
                            p_continue, veg[0..10] */

/* Model parameters, named as in the paper.
 *  p_base       base propagation factor of phi (Eq. 3)
 *  alpha_gamma  susceptibility scale: gamma(v) = alpha_gamma (1+veg)(1+den) (Eq. 4)
 *  alpha_w1/w2  wind factor (Eq. 1); alpha_s slope factor (Eq. 2)
 *  p_continue   probability that a burning cell keeps burning
 *  veg[c]       mu_veg of land-cover class c, in [-1, 1]
 *  cell_size    cell edge in metres (slope = rise / run, run = cell_size or
 *               cell_size * sqrt(2) on diagonals)
 *  unburnable_mask  bit c set: class c holds no fuel (starts UNBURNABLE)
 *  slope_mode   SIM_SLOPE_RATIO: S of Eq. 2 is rise / run; SIM_SLOPE_ANGLE:
 *               S is the slope angle atan(rise / run) in radians (the paper
 *               says only that S is the slope toward the neighbour, positive
 *               uphill); other values are SIM_EINVAL */
#define SIM_SLOPE_RATIO 0
#define SIM_SLOPE_ANGLE 1
typedef struct {
    float p_base, alpha_gamma, alpha_w1, alpha_w2, alpha_s, p_continue;
    float veg[SIM_N_CLASSES];
    float cell_size;
    uint32_t unburnable_mask;
    uint32_t slope_mode;
} sim_params;

/* One env of the batch.  (V, Vx, Vy) is its wind: speed V (m/s) and
 * Vx = V cos Theta, Vy = V sin Theta, Theta the direction the wind blows
 * toward, counter-clockwise from east.  Ignored when per-cell wind is given.
 * env_id selects the env's random stream (two envs with equal env_id, seed
 * and inputs evolve identically). */
typedef struct {
    int64_t offset;
    int32_t H, W;
    uint32_t env_id;
    float V, Vx, Vy;
} sim_env;

typedef struct sim_handle sim_handle;

/* sim_init -- set up a batch (the static layers of the paper's "State
 * representation") and write the initial fire state.
 *  out        receives the new handle (host).
 *  p          parameters (host); copied.
 *  n_env, envs  host array of n_env descriptors; 1 <= H, W <= 32767; env
 *             cell ranges must not overlap and must lie in [0, n_cells).
 *  n_cells    total packed cells.
 *  landcover  device uint8[n_cells], class 0..10.
 *  density    device float[n_cells], mu_den in [-1, 1].
 *  elevation  device float[n_cells], metres.
 *  wind_cell  device float[3][n_cells] planes (V | Vx | Vy), or NULL for the
 *             per-env wind of envs[].
 *  ignitions  host int32[n_ign][3] (env, row, col); a FLAMMABLE cell there
 *             starts BURNING, an UNBURNABLE one stays UNBURNABLE.
 *  seed       Philox key of the random streams.
 *  states_out device uint8[n_cells]: the initial fire state.
 * The handle keeps its own copies of everything it needs (fuel term
 * g = (1+veg)(1+den) in fp32, elevation, class, density, wind); the inputs
 * may be freed after the call.  The step counter starts at 0. */
int sim_init(sim_handle** out, const sim_params* p, int32_t n_env, const sim_env* envs,
             int64_t n_cells, const uint8_t* landcover, const float* density,
             const float* elevation, const float* wind_cell, const int32_t* ignitions,
             int32_t n_ign, uint64_t seed, uint8_t* states_out, void* stream);

/* sim_step -- T stochastic steps F_t -> F_{t+1} of every env (section 3,
 * Eqs. 1-4, "Stochastic update"), starting at the handle's step counter t,
 * which then advances by T.
 *  states   device uint8[n_cells], updated in place.
 *  actions  device int32[T][n_env] or NULL: before step s, env e makes a
 *           drop on the square centred at (a>>16, a&0xFFFF) for a =
 *           actions[s][e] >= 0, clipped to the grid; by default (see
 *           sim_set_drop) the square is 5x5 and every FLAMMABLE or BURNING
 *           cell in it becomes UNBURNABLE.  a < 0 or a centre outside the
 *           grid means no drop.
 *  counts   device int32[T][n_env] or NULL: number of BURNING cells of each
 *           env after each step (overwritten).
 * The random draw of cell n = i*W + j of env e at absolute step t is
 * Philox4x32-10 with key (seed lo, seed hi), counter (n>>2, t, env_id, 0),
 * word n&3, u = (word >> 8) 2^-24; a FLAMMABLE cell ignites iff u <
 * p_ignite, a BURNING cell burns out iff !(u < p_continue).  Results are
 * bit-exact to that definition whatever the launch plan. T = 0 is a no-op;
 * T < 0 is SIM_EINVAL. */
int sim_step(sim_handle* h, uint8_t* states, const int32_t* actions, int32_t T, int32_t* counts,
             void* stream);

/* sim_set_wind_series -- time-varying wind (section 3, state representation:
 * wind speed and direction are per-step fields; section 4 mentions weather
 * given as a time series).  Step t (F_t -> F_{t+1}, absolute t) takes its
 * wind from row t of the series instead of the static wind:
 *  env_wind   device float[series_T][n_env][3] (V, V cos Theta, V sin Theta)
 *             per env and step, or NULL;
 *  cell_wind  device float[series_T][3][n_cells] (the V | Vx | Vy planes of
 *             step t, packed like sim_init's wind_cell), or NULL.
 * At most one of the two; both NULL returns to the static wind.  A handle
 * created with per-cell wind accepts only a per-cell series.  The memory is
 * the caller's and must stay valid while steps run.  sim_step and
 * sim_autotune fail with SIM_EINVAL when a call would read past row
 * series_T - 1.  The relaxed calls use the same series: relaxed step t
 * (counted from the relaxed initial state) takes row t, and a relaxed call
 * with T > series_T is SIM_EINVAL. */
int sim_set_wind_series(sim_handle* h, const float* env_wind, const float* cell_wind, int64_t series_T);

/* sim_step_history -- sim_step that also keeps every intermediate state
 * (the scan form of the rollout): history is device uint8[T][n_cells] and
 * row k receives F_{t+k+1}; states ends equal to row T-1.  The steps write
 * straight into the rows, so the history costs no extra pass.  Same
 * arguments and errors as sim_step otherwise; history NULL is SIM_EINVAL. */
int sim_step_history(sim_handle* h, uint8_t* states, const int32_t* actions, int32_t T, int32_t* counts,
                     uint8_t* history, void* stream);

/* sim_set_drop -- what a drop (the actions of sim_step) does to the cells of
 * its (2 radius + 1)^2 square: SIM_DROP_SUPPRESS turns FLAMMABLE and BURNING
 * cells UNBURNABLE (a retardant line; the default, radius 2), SIM_DROP_WATER
 * turns BURNING cells BURNT (section 4: water changes a burning cell to
 * burned).  radius in 0..255; other values are SIM_EINVAL. */
#define SIM_DROP_SUPPRESS 0
#define SIM_DROP_WATER 1
int sim_set_drop(sim_handle* h, int32_t mode, int32_t radius);

/* ---- Reinforcement-learning layer (section 4, the air-tanker scenario) ----
 * One agent per env flies over the grid, sees an egocentric window of the
 * fire, and can open a valve to drop water, which turns the BURNING cells
 * of a square footprint BURNT.  A step costs burn_penalty per BURNING cell
 * after it; the step that leaves no BURNING cell earns extinguish_bonus and
 * ends the episode, as does reaching max_steps.  Episodes start from one
 * random ignition and a random agent position (sim_rl_reset). */
typedef struct {
    int32_t obs_radius;      /* observation window (2R+1)^2, R in 0..31 */
    int32_t drop_radius;     /* water footprint (2r+1)^2, r in 0..255 */
    int32_t water_capacity;  /* drops per episode, >= 0 */
    int32_t max_steps;       /* episode length, >= 1 */
    float burn_penalty;      /* reward -= burn_penalty * (BURNING cells) */
    float extinguish_bonus;  /* reward += bonus on the step that puts the fire out */
    int32_t single_launch;   /* nonzero: sim_rl_step runs as one kernel launch
                                when every env fits it (W % 4 == 0 and about
                                11 bytes of LDS per cell of the largest env
                                within 64 KB: up to about 5,900 cells, e.g.
                                64 x 64), the env's state resident in LDS and
                                stepped in place; otherwise, or with 0,
                                separate act, step (under the launch plan)
                                and observation launches.  Results are
                                identical. */
} sim_rl_config;

/* Per-env agent state, device memory, 32 bytes. */
typedef struct {
    int32_t row, col;    /* position */
    int32_t water;       /* drops left */
    int32_t steps;       /* steps taken this episode */
    int32_t done;        /* 1 once the episode is over; the agent then stays idle */
    int32_t last_count;  /* BURNING cells after the last step */
    int32_t pad[2];
} sim_rl_agent;

/* Observation codes: the four cell states, and 4 for cells beyond the grid. */
#define SIM_OBS_OUTSIDE 4

/* sim_rl_reset -- start new episodes in the envs with reset_mask[e] != 0
 * (device int32[n_env]; NULL resets every env).  Each such env's states
 * become FLAMMABLE (UNBURNABLE where the land cover is unburnable), one
 * ignition is drawn uniformly over the grid (the first of 8 draws that lands
 * on a burnable cell; none burns if all 8 miss), the agent is placed
 * uniformly at random with water_capacity drops, steps = done = 0.  The
 * draws are Philox4x32-10 with the handle's key and counter (env_id,
 * episode lo, episode hi, 0x80000000 | attempt): row = (word0 * H) >> 32,
 * col = (word1 * W) >> 32 for the ignition, words 2 and 3 of attempt 0 for
 * the agent.  obs (device uint8[n_env][(2R+1)^2], row-major window centred
 * on the agent) is written for every env; reset envs get done = 0 in
 * done_out (device int32[n_env] or NULL). */
int sim_rl_reset(sim_handle* h, const sim_rl_config* cfg, uint8_t* states, sim_rl_agent* agents,
                 const int32_t* reset_mask, uint64_t episode, uint8_t* obs, int32_t* done_out, void* stream);

/* sim_rl_step -- one RL step of every env.
 *  actions  device int32[n_env]: bits 0-3 move (0 stay, 1..8 one cell in
 *           direction k = move-1 of the paper's eight directions, k = 0
 *           east, counter-clockwise; clipped to the grid), bit 4 opens the
 *           valve: one drop of water at the agent's new position if water is
 *           left.  Values outside 0..31 or moves above 8 act as 0.
 *  Then one stochastic step (sim_step semantics, drops in water mode of
 *  radius drop_radius), the handle's step counter advancing by 1.
 *  reward   device float[n_env]: -burn_penalty * count (+ extinguish_bonus
 *           when count == 0), count = BURNING cells after the step, in fp32;
 *           0 for envs whose episode was already over.
 *  done     device int32[n_env]: episode over after this step.
 *  obs      as in sim_rl_reset, after the step.
 * Envs whose episode is over still step (their fire keeps its course) until
 * they are reset. */
int sim_rl_step(sim_handle* h, const sim_rl_config* cfg, uint8_t* states, sim_rl_agent* agents,
                const int32_t* actions, uint8_t* obs, float* reward, int32_t* done, void* stream);

/* Step counter: get it, or set it to resume a saved run (states saved by
 * the caller, same handle inputs and seed). */
int sim_get_step(const sim_handle* h, uint64_t* t);
int sim_set_step(sim_handle* h, uint64_t t);

/* Launch plan of sim_step, and of sim_step_relaxed_bwd for `sparse` (results
 * never depend on it, up to the summation order of the relaxed gradient).
 * A new handle starts with {tile_rows 4, tile_width 64, temporal 1,
 * skip_static 1, sparse 1, graph 0, resident r}: fuel and elevation are read only at
 * front cells and tiles with no fire in reach are skipped.  r is 0 unless
 * every env fits the resident plan (see below) and the batch needs at most
 * two rounds of its workgroups across the device; then r follows the largest
 * env: 1024 when it has at least 4096 cells and there are no more envs than
 * CUs, else 512 from 2048 cells, 256 from 512 cells and 64 below.  The dense plan
 * {4, 256, 1, 0, 0, 0, 0} streams every cell's state, fuel and elevation each
 * step (the HBM roofline reference).
 *  tile_rows    rows of 4-cell groups each lane owns in its tile (1, 2, 4 or 8),
 *               0 = default (4)
 *  tile_width   widest tile in cells (64, 128 or 256), 0 = default (256);
 *               an env of width W gets the smallest of 16, 32, 64, 128, 256
 *               that covers W, capped at tile_width
 *  temporal     steps per launch (1, 2, 4 or 8; 0 = default 1).  Above 1 each
 *               256-lane workgroup loads a tile_width x 32 tile of states
 *               with a halo of `temporal` cells into LDS, advances it that
 *               many steps there and stores the tile; fuel and elevation are
 *               read only at front cells.  Needs W % 4 == 0 in every env,
 *               tile_width 64 or 128 and sparse 0 (else SIM_EINVAL);
 *               tile_rows and skip_static are then unused.  sim_step_history
 *               runs such plans one step per launch.
 *  skip_static  1: only cells with a burning neighbour read fuel and
 *               elevation; 0: every cell reads its 10 bytes every step
 *  sparse       1: after the first step of a call, a tile with no burning
 *               cell in it or in its 8 neighbouring tiles, and no drop on it,
 *               is not computed (its cells cannot change); 0: every tile runs.
 *               In sim_step_relaxed_bwd, 1 skips the adjoint step s on tiles
 *               farther than s + 1 cells from every cell with initial burning
 *               mass (B_0 != 0): the parameter gradient is unchanged, since
 *               it only sums terms carrying B_s, which is zero there.
 *  graph        1: capture the T launches of a call into a HIP graph and
 *               replay it (re-captured when T, the pointers or the plan
 *               change); 0: launch directly
 *  resident     0: off; 64, 256, 512 or 1024: sim_step runs all T steps
 *               of a call in ONE launch, one workgroup of that many lanes per
 *               env holding the env's state, fuel and elevation in LDS for
 *               the whole call (per-cell wind read from HBM at front cells),
 *               with results bit-identical to the other plans.  For batches
 *               of small envs: needs W % 4 == 0 and offset % 4 == 0 in every
 *               env, at most 65536 cells and (H + 2)(W/4 + 2) 8 + 16 H W
 *               bytes of LDS per env within the device's LDS per workgroup
 *               less 2.5 KiB (160 KiB on MI355X: up to 92 x 92; a 64 x 64
 *               env takes 75040), and temporal 1 (else SIM_EINVAL); tile_rows, tile_width and skip_static are then
 *               unused by the stochastic step (sparse still applies to
 *               sim_step_relaxed_bwd).  sim_step_history runs it one step per
 *               launch. */
typedef struct {
    int32_t tile_rows, tile_width, temporal, skip_static, sparse, graph, resident;
} sim_plan;
int sim_set_plan(sim_handle* h, const sim_plan* plan);
int sim_get_plan(const sim_handle* h, sim_plan* plan);

/* Autotuner: times every candidate plan (tile_rows 1/2/4/8 x tile_width
 * 64/256, with skip_static 0 and, if allow_skip, 1; sparse = allow_sparse;
 * and, if allow_skip and every env has W % 4 == 0, temporal 2/4/8 x
 * tile_width 64/128; and, if allow_skip and the batch fits it, resident
 * 64/256/512/1024)
 * for T_probe steps of this batch starting from `states` (device, read only)
 * at the handle's step counter, and makes the fastest the handle's plan
 * (graph flag kept).  Plans are ranked on those steps alone, and which plan
 * wins depends on how much of each env is burning: probe a representative
 * stretch of the run (on the 4096-env uneven batch, 50 steps from the
 * initial fires pick a plan 13% slower over 300 steps than a 150-step probe).
 * Neither `states` nor the step counter change; the handle allocates and
 * frees one scratch state buffer.  Synchronises `stream`.
 *  results      host array of max_results entries or NULL: the plans tried,
 *               fastest first, with their measured milliseconds per step
 *  n_results    receives the number of entries written (may be NULL) */
typedef struct {
    sim_plan plan;
    float ms_per_step;
} sim_tune_result;
int sim_autotune(sim_handle* h, const uint8_t* states, int32_t T_probe, int32_t allow_skip,
                 int32_t allow_sparse, sim_tune_result* results, int32_t max_results,
                 int32_t* n_results, void* stream);

/* ----------------------------------------------------------- size classes */
/* Per-size-class plans.  An env's size class is set by its larger side:
 * class c holds the envs with 2^(c+4) < max(H, W) <= 2^(c+5), class 0 also
 * the smaller ones and class SIM_N_SIZE_CLASSES - 1 the larger ones (so
 * 0: <= 32, 1: <= 64, 2: <= 128, 3: <= 256, 4: <= 512, 5: <= 1024,
 * 6: <= 2048, 7: above).  With class plans set, sim_step, sim_step_history
 * and the multi-launch path of sim_rl_step run the envs of each class with
 * that class's plan, the classes concurrently on streams of the handle's
 * that fork from the caller's stream and join it again before the call's
 * later work (the results stay bit-identical: envs never interact).  The handle-wide graph flag
 * still applies (the launches of all classes form one graph), and the
 * handle-wide plan's sparse flag still drives sim_step_relaxed_bwd.
 * sim_set_plan and sim_autotune drop the class plans (one plan for all envs
 * again). */
#define SIM_N_SIZE_CLASSES 8
typedef struct {
    int32_t size_class;  /* 0 .. SIM_N_SIZE_CLASSES - 1 */
    int32_t n_env;       /* envs of the batch in the class */
    int64_t n_cells;     /* their cells */
    sim_plan plan;       /* the class's plan (its graph field is not used) */
    float ms_per_step;   /* the autotuner's time for the class alone; 0 if not timed */
    int32_t from_cache;  /* 1: sim_autotune_classes took the plan from its cache */
} sim_class_plan;

/* Set the plan of one size class.  The first call splits the batch into its
 * classes, each starting from the handle-wide plan.  SIM_EINVAL if the batch
 * has no env in the class or the plan does not suit its envs (as
 * sim_set_plan, checked against the class's envs alone: a class of small envs can
 * take a resident plan that the whole batch cannot). */
int sim_set_class_plan(sim_handle* h, int32_t size_class, const sim_plan* plan);

/* The size classes present in the batch, in ascending order, with their
 * plans (the handle-wide plan for each when no class plans are set).
 *  out      host array of max_out entries (may be NULL if max_out is 0)
 *  n_out    receives the number of classes present */
int sim_get_class_plans(const sim_handle* h, sim_class_plan* out, int32_t max_out, int32_t* n_out);

/* Per-size-class autotuner: for each class, times the candidates of
 * sim_autotune (with the class's own fit for temporal and resident plans)
 * on the class's envs alone for T_probe steps from `states` at the handle's
 * step counter, and gives the class its fastest plan.  Neither `states` nor
 * the step counter change; synchronises `stream`.
 *  cache_path  a text file of tuned plans, or NULL for none.  Each line
 *              holds a key -- the GPU architecture, the class, its env
 *              count, cells and largest H and W, whether all its envs have
 *              W % 4 == 0 and 4-aligned offsets, the wind kind (per env,
 *              per cell, per-env series, per-cell series), T_probe,
 *              allow_skip and allow_sparse -- and a plan.  A class whose key
 *              is in the file (the last such line wins) takes its plan
 *              without timing; each class timed is appended as one line.
 *              SIM_EINVAL if the file exists but cannot be read, or cannot
 *              be appended to; a malformed line is ignored.
 *  out, max_out, n_out  as in sim_get_class_plans */
int sim_autotune_classes(sim_handle* h, const uint8_t* states, int32_t T_probe, int32_t allow_skip,
                         int32_t allow_sparse, const char* cache_path, sim_class_plan* out,
                         int32_t max_out, int32_t* n_out, void* stream);

/* ---------------------------------------------------------------- relaxed */
/* The relaxed (mean-field) state: per cell U = P(unburned), B = P(burning)
 * (the paper's p_un and p_burn; p_bd = 1 - U - B is not carried).  One step:
 *   q_k(v) = 1 - exp(-gamma(v) phi(v - D_k, k))          (per neighbour, Eq. 4)
 *   P(v)   = 1 - prod_k (1 - q_k(v) B(v - D_k))          (product form)
 *   N = U P;  U' = U - N;  B' = N + p_continue B        (Eqs. 5-10)
 * which equals Eq. 4 whenever B is 0/1.
 * U, B and their adjoints are fp64: the recurrence amplifies small burning
 * mass exponentially, so an fp32 state drifts onto a different trajectory
 * within ~100 steps (the per-edge exp terms are fp32). */

/* Initial relaxed state from the handle's initial fire state: U = 1, B = 0
 * on FLAMMABLE cells, U = 0, B = 1 on BURNING ones, 0 elsewhere.
 * U, B: device double[n_cells]. */
int sim_relaxed_init(sim_handle* h, double* U, double* B, void* stream);

/* Workspace bytes the relaxed forward/backward need for T steps with a
 * checkpoint every ckpt_every steps (ckpt_every >= 1). */
size_t sim_relaxed_workspace_bytes(const sim_handle* h, int32_t T, int32_t ckpt_every);

/* T relaxed steps in place on (U, B) with parameters p (host; veg, p_base,
 * alpha_* and p_continue may differ from sim_init's; unburnable_mask and
 * cell_size must match).  Stores the checkpoints the backward needs in
 * `workspace` (device, >= sim_relaxed_workspace_bytes).
 *  form  SIM_FORM_PRODUCT: P = 1 - prod_k (1 - q_k B(u_k)) as above;
 *        SIM_FORM_EXP: P = 1 - exp(-gamma(v) sum_k B(u_k) phi(u_k, k)), Eq. 4
 *        with the burning indicator replaced by B (the paper's soft reading).
 *        Both equal Eq. 4 on 0/1 states. */
#define SIM_FORM_PRODUCT 0
#define SIM_FORM_EXP 1
int sim_step_relaxed_fwd(sim_handle* h, const sim_params* p, double* U, double* B, int32_t T,
                         int32_t ckpt_every, int32_t form, void* workspace, size_t workspace_bytes,
                         void* stream);

/* Soft-IoU loss of the final relaxed state against a binary target scar.
 * Per env e: S = 1 - U_T on burnable cells, I = sum S Y, D = sum S + sum Y - I,
 * loss[e] = 1 - I / D (0 when D = 0) (the calibration objective of section 4
 * with the IoU as its score).
 *  target     device uint8[n_cells], nonzero = burnt in the target scar.
 *  loss       device float[n_env]: the per-env losses (rounded from fp64).
 *  gU_T       device double[n_cells] or NULL: scale * d loss[e] / d U_T, the
 *             seed of sim_step_relaxed_bwd for the objective below.
 *  objective  device double[1] or NULL: scale * sum_e loss[e] in fp64 (scale
 *             = 1 / n_env gives the mean over envs).
 * Every sum runs in a fixed order, so equal inputs give equal bits.  On the
 * first call the handle allocates its scratch (3 doubles per 4096-cell chunk
 * of every env and 4 per env). */
int sim_relaxed_loss(sim_handle* h, const double* U_T, const uint8_t* target, float* loss,
                     double* gU_T, double scale, double* objective, void* stream);

/* sim_relaxed_loss for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and arguments, with the partial sums kept in a static device
 * array of 4 MiB (2^19 doubles) per GPU instead of handle memory.  It calls
 * no hipMalloc or hipFree, ever.
 *  Limit: 3 doubles per 4096-cell chunk of every env plus 4 per env must fit
 *  2^19 (e.g. 128 Mi cells in 8 envs, or 4096 envs of 512 x 512); a larger
 *  batch gets SIM_EINVAL and a message naming sim_relaxed_loss.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (every slot is written before it is read): calls that overlap in
 * time on one GPU, on any streams or handles, race and must be ordered by the
 * caller.  Results equal sim_relaxed_loss's bit for bit. */
int sim_relaxed_loss_noalloc(sim_handle* h, const double* U_T, const uint8_t* target, float* loss,
                             double* gU_T, double scale, double* objective, void* stream);

/* The paper's calibration loss (section 4): per env e, binary cross-entropy
 * of S = clip(1 - U_T on burnable cells, 0 elsewhere; eps, 1 - eps) against
 * the target scar Y, averaged over the env's cells, plus mse_weight times the
 * mean squared error between the pool x pool block averages of S and Y
 * (blocks at the far edges cover what is left).  loss[e], gU_T (or NULL; zero
 * where S is clipped) and objective (or NULL) as for sim_relaxed_loss.
 * 1 <= pool <= 64, 0 < eps < 0.5. */
int sim_relaxed_loss_bce(sim_handle* h, const double* U_T, const uint8_t* target, int32_t pool,
                         double mse_weight, double eps, float* loss, double* gU_T, double scale,
                         double* objective, void* stream);

/* Gradient of a scalar objective J(U_T, B_T) with respect to the parameter
 * vector (p_base, alpha_w1, alpha_w2, alpha_s, alpha_gamma, p_continue,
 * veg[0..10]) through the T relaxed steps of the last sim_step_relaxed_fwd
 * call on the same workspace (same p, T, ckpt_every, form): recomputes each
 * checkpoint segment forward, then runs the adjoint step backward.
 *  gU_T, gB_T  device double[n_cells]: dJ/dU_T, dJ/dB_T (gB_T may be NULL = 0).
 *  grad        device double[SIM_N_THETA], overwritten. */
int sim_step_relaxed_bwd(sim_handle* h, const sim_params* p, const double* gU_T,
                         const double* gB_T, int32_t T, int32_t ckpt_every, int32_t form,
                         void* workspace,
                         size_t workspace_bytes, double* grad, void* stream);

/* ------------------------------------------------------------- diagnostics */
/* The device exp and Philox the step uses, applied elementwise (for parity
 * tests of the building blocks).  x, y: device float[n]; ctr: device
 * uint32[n][4], key: device uint32[n][2], out: device uint32[n][4]. */
int sim_debug_exp(const float* x, float* y, int64_t n, void* stream);
/* The device arctangent of the slope-angle variant, elementwise. */
int sim_debug_atan(const float* x, float* y, int64_t n, void* stream);
int sim_debug_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n,
                     void* stream);

/* HBM streaming probe, the attainable-bandwidth reference for the roofline
 * figures: mode 0 reads src, 1 writes dst, 2 copies src to dst, with 16-byte
 * accesses by `blocks` workgroups of 256 lanes (grid-stride).
 *  src, dst   device, 16-byte aligned; bytes a multiple of 16.  Mode 0 writes
 *             nothing (it only may, for an xor of the data no real input has,
 *             write dst[blocks * 256] words); mode 1 ignores src.
 * Returns SIM_EINVAL for a bad mode, size, alignment or block count. */
int sim_debug_stream(int32_t mode, const void* src, void* dst, int64_t bytes, int32_t blocks, void* stream);

const char* sim_last_error(const sim_handle* h);
void sim_destroy(sim_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* FIRESIM_H */
