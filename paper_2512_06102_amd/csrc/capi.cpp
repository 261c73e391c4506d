// capi.cpp -- the C ABI (include/firesim.h): argument checking, the handle's
// device memory, the tile list, step sequencing and graph replay.  All model
// arithmetic runs in the kernels (stoch.hip, relaxed.hip).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/firesim.h"
#include "rl.hpp"
#include "internal.hpp"
#include "relaxed.hpp"
#include "resident.hpp"

using namespace firesim;

namespace {

thread_local std::string g_init_error;

// Scratch of sim_relaxed_loss_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself (on the host it only
// names the variable); sim_init looks up its device address once per device
// with hipGetSymbolAddress and the entry point uses that address.
constexpr size_t kNoallocScratchDoubles = (size_t)1 << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be current.
hipError_t noalloc_scratch(int dev, double** out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// A set of envs stepped with one plan: the whole batch, or one size class
// when class plans are set.  Its tile list is built for its plan.
struct PlanGroup {
    std::vector<int32_t> envs;       // global env indices (empty: the whole batch)
    int32_t* d_list = nullptr;       // device copy of envs (nullptr: the whole batch)
    int32_t size_class = -1;         // -1: the whole batch
    int64_t n_cells = 0;             // cells of its envs
    int32_t max_h = 0, max_w = 0;    // largest H and W among them
    bool aligned = true;             // every env W % 4 == 0 with a 4-aligned offset
    ResidentShape res;               // the resident kernel's LDS layout over its envs
    sim_plan plan{4, 64, 1, 1, 1, 0, 0};
    float tuned_ms = 0.0f;           // the autotuner's time per step (0: not timed)
    bool from_cache = false;
    TileDesc* d_tiles = nullptr;
    int32_t* d_tile_nbr = nullptr;   // [n_tiles][8] neighbouring tiles (-1 off the env)
    int32_t* d_tile_burn = nullptr;  // [2][n_tiles] burning cells per tile (sparse plan)
    int32_t* d_tile_eq = nullptr;    // [n_tiles] both state buffers agree on the tile
    int32_t n_tiles = 0;
    int32_t tiles_rt = 0;            // tile_rows the tile list was built for
    int32_t tiles_tw = 0;            // tile_width the tile list was built for
};

void free_group(PlanGroup& g)
{
    for (void* p : {(void*)g.d_list, (void*)g.d_tiles, (void*)g.d_tile_nbr, (void*)g.d_tile_burn,
                    (void*)g.d_tile_eq})
        if (p) (void)hipFree(p);
    g.d_list = nullptr;
    g.d_tiles = nullptr;
    g.d_tile_nbr = g.d_tile_burn = g.d_tile_eq = nullptr;
    g.n_tiles = g.tiles_rt = g.tiles_tw = 0;
}

struct GraphCache {
    hipGraphExec_t exec = nullptr;
    int32_t T = -1;
    const void* states = nullptr;
    const void* actions = nullptr;
    const void* counts = nullptr;
    const void* history = nullptr;
    sim_plan plan{};
    bool valid = false;
};

}  // namespace

struct sim_handle {
    int device = 0;
    sim_params params{};
    int32_t n_env = 0;
    int64_t n_cells = 0;
    std::vector<sim_env> envs;
    bool aligned = true;
    bool wind_cell = false;
    uint64_t seed = 0;
    uint64_t t = 0;
    // default launch plan: fuel and elevation read only at front cells, and
    // tiles with no fire in reach skipped (the dense plan, which streams every
    // cell's 10 bytes each step, is {4, 256, 1, 0, 0, 0})
    sim_plan plan{4, 64, 1, 1, 1, 0, 0};
    // the whole batch under `plan`, or (when non-empty) its size classes under their own plans
    PlanGroup all;
    std::vector<PlanGroup> classes;
    // the classes run concurrently: one stream each, forked from and joined
    // to the caller's stream by events (one per class, plus the fork)
    std::vector<hipStream_t> class_streams;
    std::vector<hipEvent_t> class_events;
    // wind series (caller-owned device memory, indexed by the absolute step)
    const float* series_env = nullptr;   // [series_T][n_env][3]
    const float* series_cell = nullptr;  // [series_T][3][n_cells]
    int64_t series_T = 0;
    // drops of sim_step: mode 0 suppressant (FLAMMABLE/BURNING -> UNBURNABLE),
    // mode 1 water (BURNING -> BURNT), square of side 2 radius + 1
    int32_t drop_mode = 0, drop_radius = 2;
    // reinforcement-learning layer: drop row and burning counts of one step
    int32_t* d_rl_drop = nullptr;
    int32_t* d_rl_counts = nullptr;
    RlFusedShape rl_shape;  // the fused RL step's LDS layout (fits: every env fits it)

    EnvDev* d_envs = nullptr;
    int32_t* d_chunk_env = nullptr;    // env of every loss chunk (kLossChunk cells)
    int32_t n_chunks = 0;
    double* d_loss_scratch = nullptr;  // soft-IoU loss partial sums (allocated on first use)
    double* noalloc_scratch = nullptr; // this device's static scratch (sim_relaxed_loss_noalloc)
    int64_t n_adj_tiles = 0;           // tiles of the relaxed adjoint (they size its workspace)
    float* d_g = nullptr;
    float* d_E = nullptr;
    uint8_t* d_cls = nullptr;
    float* d_den = nullptr;
    float* d_wind = nullptr;
    uint8_t* d_init_states = nullptr;  // initial fire state (for the relaxed initial state)
    uint8_t* d_tmp = nullptr;          // ping-pong state buffer
    uint32_t* d_t = nullptr;           // step counter base read by the step kernels
    hipStream_t cap_stream = nullptr;
    GraphCache graph;
    RelaxedState relaxed;
    std::string err;
};

namespace {

int fail(sim_handle* h, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_init_error = buf;
    return code;
}

// Every entry point runs with the handle's GPU current (the caller's
// current device is restored on return) and shows as a named range in a
// marker trace (rocprofv3 --marker-trace).
class CallScope {
public:
    CallScope(const char* name, const sim_handle* h)
    {
        roctxRangePushA(name);
        if (h && hipGetDevice(&prev_) == hipSuccess && prev_ != h->device)
            switched_ = hipSetDevice(h->device) == hipSuccess;
    }
    ~CallScope()
    {
        if (switched_) (void)hipSetDevice(prev_);
        roctxRangePop();
    }
    CallScope(const CallScope&) = delete;
    CallScope& operator=(const CallScope&) = delete;

private:
    int prev_ = 0;
    bool switched_ = false;
};

#define HIP_OR_FAIL(h, expr)                                                              \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((h), SIM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

void free_all(sim_handle* h)
{
    void* ptrs[] = {h->d_envs, h->d_chunk_env, h->d_loss_scratch, h->d_g, h->d_E, h->d_cls, h->d_den, h->d_wind, h->d_init_states,
                    h->d_tmp, h->d_t, h->d_rl_drop, h->d_rl_counts};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    free_group(h->all);
    for (PlanGroup& g : h->classes) free_group(g);
    for (hipStream_t cs : h->class_streams) (void)hipStreamDestroy(cs);
    for (hipEvent_t ev : h->class_events) (void)hipEventDestroy(ev);
    if (h->graph.exec) (void)hipGraphExecDestroy(h->graph.exec);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    relaxed_free(h->relaxed);
}

StepArgs step_args(const sim_handle* h)
{
    StepArgs a;
    const sim_params& p = h->params;
    a.p_base = p.p_base;
    a.alpha_gamma = p.alpha_gamma;
    a.alpha_w1 = p.alpha_w1;
    a.alpha_w2 = p.alpha_w2;
    a.alpha_s = p.alpha_s;
    a.p_continue = p.p_continue;
    a.inv_run_orth = (float)(1.0 / (double)p.cell_size);
    a.inv_run_diag = (float)(1.0 / ((double)p.cell_size * std::sqrt(2.0)));
    a.key0 = (uint32_t)h->seed;
    a.key1 = (uint32_t)(h->seed >> 32);
    a.drop_mode = h->drop_mode;
    a.drop_radius = h->drop_radius;
    a.slope_mode = (int32_t)p.slope_mode;
    return a;
}

// Widest tile width (64, 128, 256) not above max_width that W needs.
int tile_width_for(int W, int max_width)
{
    const int w = W > 128 ? 256 : (W > 64 ? 128 : (W > 32 ? 64 : (W > 16 ? 32 : 16)));
    return w < max_width ? w : max_width;
}

// Tile list of group g: env-major, then row band, then column band; with
// each tile's 8 neighbouring tiles (same env) for the sparse plan.
// rt > 0: one-step tiles (one wave64: 256 / width lane rows of rt rows, width
// narrowed for narrow envs); rt < 0: temporal-blocking tiles of max_width x
// kTbTileRows for every env.
int build_tiles(sim_handle* h, PlanGroup& g, int rt, int max_width)
{
    std::vector<TileDesc> tiles;
    std::vector<int32_t> nbr;
    const int32_t n_members = g.envs.empty() ? h->n_env : (int32_t)g.envs.size();
    for (int32_t q = 0; q < n_members; ++q) {
        const int32_t e = g.envs.empty() ? q : g.envs[q];
        const int H = h->envs[e].H, W = h->envs[e].W;
        const int width = rt < 0 ? max_width : tile_width_for(W, max_width);
        const int th = rt < 0 ? kTbTileRows : (256 / width) * rt;
        const int nr = (H + th - 1) / th, nc = (W + width - 1) / width;
        const int32_t first = (int32_t)tiles.size();
        for (int i = 0; i < nr; ++i)
            for (int j = 0; j < nc; ++j) {
                tiles.push_back(TileDesc{e, i * th, j * width, width});
                for (int di = -1; di <= 1; ++di)
                    for (int dj = -1; dj <= 1; ++dj) {
                        if (di == 0 && dj == 0) continue;
                        const int a = i + di, b = j + dj;
                        nbr.push_back(a >= 0 && a < nr && b >= 0 && b < nc ? first + a * nc + b : -1);
                    }
            }
    }
    for (void** p : {(void**)&g.d_tiles, (void**)&g.d_tile_nbr, (void**)&g.d_tile_burn, (void**)&g.d_tile_eq}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    g.n_tiles = g.tiles_rt = g.tiles_tw = 0;
    const size_t nt = tiles.size();
    if (hipMalloc(&g.d_tiles, nt * sizeof(TileDesc)) != hipSuccess ||
        hipMalloc(&g.d_tile_nbr, nt * 8 * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&g.d_tile_burn, nt * 2 * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&g.d_tile_eq, nt * sizeof(int32_t)) != hipSuccess)
        return fail(h, SIM_ENOMEM, "tile list allocation failed");
    HIP_OR_FAIL(h, hipMemcpy(g.d_tiles, tiles.data(), nt * sizeof(TileDesc), hipMemcpyHostToDevice));
    HIP_OR_FAIL(h, hipMemcpy(g.d_tile_nbr, nbr.data(), nt * 8 * sizeof(int32_t), hipMemcpyHostToDevice));
    g.n_tiles = (int32_t)tiles.size();
    g.tiles_rt = rt;
    g.tiles_tw = max_width;
    return SIM_OK;
}

int tiles_key(const sim_plan& p) { return p.temporal > 1 ? -1 : p.tile_rows; }

// The groups sim_step runs: the size classes if class plans are set, else the whole batch.
std::vector<PlanGroup*> active_groups(sim_handle* h)
{
    std::vector<PlanGroup*> out;
    if (h->classes.empty()) {
        out.push_back(&h->all);
    } else {
        for (PlanGroup& g : h->classes) out.push_back(&g);
    }
    return out;
}

// Rebuild a group's tile list if its plan changed the geometry.
int ensure_group_tiles(sim_handle* h, PlanGroup& g)
{
    if (g.tiles_rt == tiles_key(g.plan) && g.tiles_tw == g.plan.tile_width) return SIM_OK;
    h->graph.valid = false;
    return build_tiles(h, g, tiles_key(g.plan), g.plan.tile_width);
}

int ensure_tiles(sim_handle* h)
{
    for (PlanGroup* g : active_groups(h)) {
        const int rc = ensure_group_tiles(h, *g);
        if (rc != SIM_OK) return rc;
    }
    return SIM_OK;
}

// The resident kernel's dynamic-LDS limit is an attribute of the kernel
// functions, shared by every handle in the process: it is raised once per
// device to everything the device allows beside the kernel's static LDS, so
// that no batch lowers it under another's.  Returns whether that worked.
constexpr size_t kResidentStaticLds = 2560;
bool resident_lds_allowed(int device, int max_lds)
{
    static std::mutex mu;
    static int state[kMaxDevices] = {};  // 0 not tried, 1 set, 2 refused
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lock(mu);
    if (state[device] == 0) {
        const bool ok = resident_set_lds_limit(max_lds - (int)kResidentStaticLds) == hipSuccess;
        if (!ok) (void)hipGetLastError();  // not sticky: the batches just do not take the plan
        state[device] = ok ? 1 : 2;
    }
    return state[device] == 1;
}

// The resident workgroup size a new handle starts with, 0 for the tiled
// plans.  Measured on 64 x 64 envs: 1024 lanes for up to 256 envs (0.43 ms
// per 200 steps for 64 envs, against 1.2 ms for the tiled plan), 512 for
// 1024 envs (1.26 against 2.1 ms); 64 lanes for 20 x 20 envs.  Beyond two
// rounds of workgroups (4096 envs of 64 x 64) the tiled plan wins.
int default_resident(sim_handle* h, const PlanGroup& g)
{
    if (!g.res.fits) return 0;
    int cus = 0, max_lds = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) != hipSuccess ||
        cus < 1)
        return 0;
    const int dwords = g.res.cell_cap / 4;
    const int nt = dwords >= 1024 && h->n_env <= cus ? 1024 : (dwords >= 512 ? 512 : (dwords >= 128 ? 256 : 64));
    const int64_t by_lds = (int64_t)max_lds / (int64_t)(resident_lds_bytes(g.res) + kResidentStaticLds);
    const int64_t by_waves = 32 / (nt / 64);  // 32 wave slots per CU
    const int64_t per_round = (int64_t)cus * std::max<int64_t>(1, std::min(by_lds, by_waves));
    return (int64_t)h->n_env <= 2 * per_round ? nt : 0;
}

// Size class of an env (see SIM_N_SIZE_CLASSES).
int size_class_of(int H, int W)
{
    const int side = std::max(H, W);
    int c = 0;
    while (c < SIM_N_SIZE_CLASSES - 1 && side > (32 << c)) ++c;
    return c;
}

// Alignment, sizes and the resident kernel's fit over a group's envs.
void describe_group(sim_handle* h, PlanGroup& g)
{
    const int32_t n_members = g.envs.empty() ? h->n_env : (int32_t)g.envs.size();
    int64_t cells = 0, max_cells = 0, max_frame = 0;
    g.aligned = !(h->wind_cell && h->n_cells % 4 != 0);
    g.max_h = g.max_w = 0;
    for (int32_t q = 0; q < n_members; ++q) {
        const sim_env& v = h->envs[g.envs.empty() ? q : g.envs[q]];
        if (v.W % 4 != 0 || v.offset % 4 != 0) g.aligned = false;
        cells += (int64_t)v.H * v.W;
        max_cells = std::max<int64_t>(max_cells, (int64_t)v.H * v.W);
        max_frame = std::max<int64_t>(max_frame, ((int64_t)v.H + 2) * (v.W / 4 + 2));
        g.max_h = std::max(g.max_h, v.H);
        g.max_w = std::max(g.max_w, v.W);
    }
    g.n_cells = cells;
    g.res = ResidentShape{};
    int max_lds = 0;
    if (g.aligned && max_cells <= 65536 &&
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess &&
        max_frame <= max_lds) {
        g.res.frame_cap = (int32_t)((max_frame + 3) & ~3);
        g.res.cell_cap = (int32_t)max_cells;
        // the kernel's own static LDS (under 2.5 KiB) comes on top of the dynamic part
        const size_t need = resident_lds_bytes(g.res);
        g.res.fits = need + kResidentStaticLds <= (size_t)max_lds && resident_lds_allowed(h->device, max_lds);

    }
}

StepLaunch step_launch(const sim_handle* h, const PlanGroup& g)
{
    StepLaunch L;
    L.tiles = g.d_tiles;
    L.n_tiles = g.n_tiles;
    L.envs = h->d_envs;
    L.n_env = h->n_env;
    L.fields = StaticFields{h->d_g, h->d_E, h->wind_cell ? h->d_wind : nullptr, h->n_cells, 0, nullptr,
                            h->n_env};
    if (h->series_cell) {
        L.fields.wind = h->series_cell;
        L.fields.wind_stride = 3 * h->n_cells;
    } else if (h->series_env) {
        L.fields.env_wind = h->series_env;
    }
    L.args = step_args(h);
    L.aligned = g.aligned;
    L.rows_per_thread = g.plan.tile_rows;
    L.skip_static = g.plan.skip_static != 0;
    return L;
}

// Copy the cells of group g from src to dst (all cells for the whole batch).
hipError_t copy_group(sim_handle* h, hipStream_t s, const PlanGroup& g, uint8_t* dst, const uint8_t* src)
{
    if (!g.d_list) return launch_copy_u8(s, dst, src, h->n_cells);
    return launch_copy_envs(s, h->d_envs, g.d_list, (int32_t)g.envs.size(), dst, src);
}

// Enqueue the launches of T steps of group g's envs (if T is odd the result
// is copied back from the ping-pong buffer).  With a history buffer, step k
// reads row k-1 (states for k = 0) and writes row k, and the last row is
// copied to states.  drop overrides the handle's drop setting.
hipError_t enqueue_group(sim_handle* h, PlanGroup& g, hipStream_t s, uint8_t* states, const int32_t* actions,
                         int32_t T, int32_t* counts, uint8_t* history, const int32_t* drop)
{
    hipError_t e;
    StepLaunch L = step_launch(h, g);
    if (drop) {
        L.args.drop_mode = drop[0];
        L.args.drop_radius = drop[1];
    }
    const sim_plan& plan = g.plan;
    const int32_t n_members = g.envs.empty() ? h->n_env : (int32_t)g.envs.size();
    uint8_t* cur = states;
    uint8_t* nxt = history ? history : h->d_tmp;
    if (plan.resident) {
        // all T steps in one launch, in place (one launch per step with a history)
        if (!history)
            return launch_stoch_resident(s, h->d_envs, h->n_env, g.d_list, n_members, L.fields, L.args, g.res,
                                         plan.resident, states, states, h->d_t, 0u, T, actions, counts);
        for (int32_t k = 0; k < T; ++k) {
            e = launch_stoch_resident(s, h->d_envs, h->n_env, g.d_list, n_members, L.fields, L.args, g.res,
                                      plan.resident, cur, nxt, h->d_t, (uint32_t)k, 1,
                                      actions ? actions + (int64_t)k * h->n_env : nullptr,
                                      counts ? counts + (int64_t)k * h->n_env : nullptr);
            if (e != hipSuccess) return e;
            cur = nxt;
            nxt = history + (int64_t)(k + 1) * h->n_cells;
        }
        return copy_group(h, s, g, states, cur);
    }
    const bool sparse = plan.sparse != 0;
    if (sparse) {  // nothing is known yet about how the two buffers compare
        e = launch_fill_i32(s, g.d_tile_eq, g.n_tiles, 0);
        if (e != hipSuccess) return e;
    }
    if (plan.temporal > 1) {
        // temporal blocking: K steps per launch (one per launch with a history)
        const int K = plan.temporal;
        for (int32_t k = 0; k < T;) {
            const int32_t ks = history ? 1 : std::min<int32_t>(K, T - k);
            e = launch_stoch_tb(s, L, K, plan.tile_width, cur, nxt, h->d_t, (uint32_t)k, ks,
                                actions ? actions + (int64_t)k * h->n_env : nullptr,
                                counts ? counts + (int64_t)k * h->n_env : nullptr);
            if (e != hipSuccess) return e;
            k += ks;
            if (history) {
                cur = nxt;
                nxt = history + (int64_t)k * h->n_cells;
            } else {
                std::swap(cur, nxt);
            }
        }
        if (cur != states) return copy_group(h, s, g, states, cur);
        return hipSuccess;
    }
    for (int32_t k = 0; k < T; ++k) {
        SparseArgs sp{nullptr, nullptr, nullptr, nullptr, 0};
        if (sparse) {
            // a history row starts empty: an inactive tile must copy its cells
            if (history && k > 0 && (e = launch_fill_i32(s, g.d_tile_eq, g.n_tiles, 0)) != hipSuccess)
                return e;
            sp = SparseArgs{g.d_tile_burn + (k & 1) * g.n_tiles, g.d_tile_burn + ((k + 1) & 1) * g.n_tiles,
                            g.d_tile_eq, g.d_tile_nbr, k == 0 ? 1 : 0};
        }
        e = launch_stoch_step(s, L, cur, nxt, h->d_t, (uint32_t)k,
                              actions ? actions + (int64_t)k * h->n_env : nullptr,
                              counts ? counts + (int64_t)k * h->n_env : nullptr, sp);
        if (e != hipSuccess) return e;
        if (history) {
            cur = nxt;
            nxt = history + (int64_t)(k + 1) * h->n_cells;
        } else {
            std::swap(cur, nxt);
        }
    }
    if (cur != states) return copy_group(h, s, g, states, cur);
    return hipSuccess;
}

// Enqueue one sim_step call: counts cleared, then each active group's steps.
// Size classes touch disjoint cells (and count rows), so each runs on its own
// stream, forked from s after the clear and joined back to s.
hipError_t enqueue_steps(sim_handle* h, hipStream_t s, uint8_t* states, const int32_t* actions,
                         int32_t T, int32_t* counts, uint8_t* history = nullptr,
                         const int32_t* drop = nullptr)
{
    hipError_t e;
    if (counts && (e = launch_fill_i32(s, counts, (int64_t)T * h->n_env, 0)) != hipSuccess) return e;
    const std::vector<PlanGroup*> groups = active_groups(h);
    if (groups.size() == 1 || h->class_streams.size() != groups.size() ||
        h->class_events.size() != groups.size() + 1)
        for (PlanGroup* g : groups) {
            if ((e = enqueue_group(h, *g, s, states, actions, T, counts, history, drop)) != hipSuccess) return e;
        }
    else {
        hipEvent_t fork = h->class_events.back();
        if ((e = hipEventRecord(fork, s)) != hipSuccess) return e;
        for (size_t i = 0; i < groups.size(); ++i) {
            hipStream_t cs = h->class_streams[i];
            if ((e = hipStreamWaitEvent(cs, fork, 0)) != hipSuccess) return e;
            if ((e = enqueue_group(h, *groups[i], cs, states, actions, T, counts, history, drop)) != hipSuccess)
                return e;
            if ((e = hipEventRecord(h->class_events[i], cs)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s, h->class_events[i], 0)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

bool same_plan(const sim_plan& a, const sim_plan& b)
{
    return a.tile_rows == b.tile_rows && a.tile_width == b.tile_width && a.temporal == b.temporal &&
           a.skip_static == b.skip_static && a.sparse == b.sparse && a.graph == b.graph &&
           a.resident == b.resident;
}

int validate_plan(sim_handle* h, const PlanGroup& g, sim_plan& p)
{
    if (p.tile_rows == 0) p.tile_rows = 4;
    if (p.tile_width == 0) p.tile_width = 256;
    if (p.temporal == 0) p.temporal = 1;
    if (!(p.tile_rows == 1 || p.tile_rows == 2 || p.tile_rows == 4 || p.tile_rows == 8))
        return fail(h, SIM_EINVAL, "tile_rows must be 1, 2, 4 or 8");
    if (!(p.tile_width == 64 || p.tile_width == 128 || p.tile_width == 256))
        return fail(h, SIM_EINVAL, "tile_width must be 64, 128 or 256");
    if (!(p.temporal == 1 || p.temporal == 2 || p.temporal == 4 || p.temporal == 8))
        return fail(h, SIM_EINVAL, "temporal must be 1, 2, 4 or 8");
    if (p.temporal > 1) {
        if (!g.aligned) return fail(h, SIM_EINVAL, "temporal blocking needs W %% 4 == 0 in every env");
        if (p.sparse) return fail(h, SIM_EINVAL, "temporal blocking and the sparse plan do not combine");
        if (p.tile_width != 64 && p.tile_width != 128)
            return fail(h, SIM_EINVAL, "temporal blocking takes tile_width 64 or 128");
    }
    if (p.skip_static != 0 && p.skip_static != 1) return fail(h, SIM_EINVAL, "skip_static must be 0 or 1");
    if (p.sparse != 0 && p.sparse != 1) return fail(h, SIM_EINVAL, "sparse must be 0 or 1");
    if (p.graph != 0 && p.graph != 1) return fail(h, SIM_EINVAL, "graph must be 0 or 1");
    if (p.resident != 0) {
        if (!(p.resident == 64 || p.resident == 256 || p.resident == 512 || p.resident == 1024))
            return fail(h, SIM_EINVAL, "resident must be 0, 64, 256, 512 or 1024");
        if (p.temporal > 1) return fail(h, SIM_EINVAL, "resident and temporal blocking do not combine");
        if (!g.res.fits)
            return fail(h, SIM_EINVAL,
                        "resident plan needs W %% 4 == 0 and 4-aligned offsets in every env, at most 65536 "
                        "cells and (H + 2)(W/4 + 2) 8 + 16 H W bytes of LDS per env within the device's "
                        "LDS per workgroup less 2.5 KiB");
    }
    return SIM_OK;
}

}  // namespace

extern "C" {

int sim_init(sim_handle** out, const sim_params* p, int32_t n_env, const sim_env* envs,
             int64_t n_cells, const uint8_t* landcover, const float* density,
             const float* elevation, const float* wind_cell, const int32_t* ignitions,
             int32_t n_ign, uint64_t seed, uint8_t* states_out, void* stream)
{
    CallScope scope("sim_init", nullptr);
    g_init_error.clear();
    if (!out) return fail(nullptr, SIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p || !envs || n_env < 1) return fail(nullptr, SIM_EINVAL, "need params and n_env >= 1 envs");
    if (!landcover || !density || !elevation || !states_out)
        return fail(nullptr, SIM_EINVAL, "landcover, density, elevation and states_out are required");
    if (n_ign < 0 || (n_ign > 0 && !ignitions)) return fail(nullptr, SIM_EINVAL, "bad ignition list");
    if (!(p->cell_size > 0.0f) || !std::isfinite(p->cell_size))
        return fail(nullptr, SIM_EINVAL, "cell_size must be positive");
    if (p->slope_mode != SIM_SLOPE_RATIO && p->slope_mode != SIM_SLOPE_ANGLE)
        return fail(nullptr, SIM_EINVAL, "slope_mode must be SIM_SLOPE_RATIO or SIM_SLOPE_ANGLE");
    if (n_cells < 1) return fail(nullptr, SIM_EINVAL, "n_cells must be >= 1");
    // envs: sizes and disjoint in-range cell ranges
    std::vector<std::pair<int64_t, int64_t>> ranges;
    for (int32_t e = 0; e < n_env; ++e) {
        const sim_env& v = envs[e];
        if (v.H < 1 || v.W < 1 || v.H > 32767 || v.W > 32767)
            return fail(nullptr, SIM_EINVAL, "env %d: H, W must be in [1, 32767]", e);
        const int64_t cells = (int64_t)v.H * v.W;
        if (v.offset < 0 || v.offset + cells > n_cells)
            return fail(nullptr, SIM_EINVAL, "env %d: cells [%lld, %lld) outside [0, %lld)", e,
                        (long long)v.offset, (long long)(v.offset + cells), (long long)n_cells);
        ranges.push_back({v.offset, v.offset + cells});
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].second)
            return fail(nullptr, SIM_EINVAL, "env cell ranges overlap");
    for (int32_t q = 0; q < n_ign; ++q) {
        const int32_t e = ignitions[3 * q], i = ignitions[3 * q + 1], j = ignitions[3 * q + 2];
        if (e < 0 || e >= n_env || i < 0 || i >= envs[e].H || j < 0 || j >= envs[e].W)
            return fail(nullptr, SIM_EINVAL, "ignition %d (%d, %d, %d) outside its env", q, e, i, j);
    }

    sim_handle* h = new (std::nothrow) sim_handle();
    if (!h) return fail(nullptr, SIM_ENOMEM, "host allocation failed");
    hipStream_t s = (hipStream_t)stream;
    auto bail = [&](int code) {
        g_init_error = h->err;
        free_all(h);
        delete h;
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) {
        h->err = "hipGetDevice failed (no GPU?)";
        return bail(SIM_EHIP);
    }
    {
        const hipError_t e = noalloc_scratch(h->device, &h->noalloc_scratch);
        if (e != hipSuccess) {
            fail(h, SIM_EHIP, "static scratch lookup on device %d failed: %s", h->device, hipGetErrorString(e));
            return bail(SIM_EHIP);
        }
    }
    h->params = *p;
    h->n_env = n_env;
    h->n_cells = n_cells;
    h->envs.assign(envs, envs + n_env);
    h->wind_cell = wind_cell != nullptr;
    h->seed = seed;
    // 4-cell vector loads need every row start (and each wind plane) on a 4-cell boundary
    for (const sim_env& v : h->envs)
        if (v.W % 4 != 0 || v.offset % 4 != 0) h->aligned = false;
    if (h->wind_cell && n_cells % 4 != 0) h->aligned = false;
    if (h->aligned) {
        int64_t max_cells = 0, max_frame = 0;
        for (const sim_env& v : h->envs) {
            max_cells = std::max<int64_t>(max_cells, (int64_t)v.H * v.W);
            max_frame = std::max<int64_t>(max_frame, ((int64_t)v.H + 2) * (v.W / 4 + 2));
        }
        RlFusedShape& rs = h->rl_shape;
        if (max_cells <= 65536 && max_frame <= (int64_t)kRlFusedMaxLds) {
            rs.frame_cap = (int32_t)((max_frame + 3) & ~3);
            rs.cell_cap = (int32_t)max_cells;
            rs.fits = rl_fused_lds_bytes(rs) <= kRlFusedMaxLds;
        }
    }
    h->all.plan = h->plan;
    describe_group(h, h->all);
    // small envs: default to the resident plan when the batch fits it and
    // needs at most two rounds of workgroups across the chip
    h->plan.resident = default_resident(h, h->all);
    h->all.plan = h->plan;

    std::vector<EnvDev> ed(n_env);
    std::vector<int32_t> chunk_env;
    for (int32_t e = 0; e < n_env; ++e) {
        ed[e] = EnvDev{envs[e].offset, envs[e].H, envs[e].W, envs[e].env_id,
                       envs[e].V, envs[e].Vx, envs[e].Vy, (int32_t)chunk_env.size()};
        const int64_t nch = ((int64_t)envs[e].H * envs[e].W + kLossChunk - 1) / kLossChunk;
        chunk_env.insert(chunk_env.end(), (size_t)nch, e);
    }
    h->n_chunks = (int32_t)chunk_env.size();
    h->n_adj_tiles = relaxed_adj_tiles(h->envs);
    const size_t n = (size_t)n_cells;
    int rc;
#define ALLOC(ptr, bytes)                                                                   \
    if (hipMalloc(&(ptr), (bytes)) != hipSuccess) {                                         \
        fail(h, SIM_ENOMEM, "device allocation of %zu bytes failed", (size_t)(bytes));      \
        return bail(SIM_ENOMEM);                                                            \
    }
    ALLOC(h->d_envs, sizeof(EnvDev) * n_env);
    ALLOC(h->d_chunk_env, sizeof(int32_t) * chunk_env.size());
    ALLOC(h->d_g, 4 * n);
    ALLOC(h->d_E, 4 * n);
    ALLOC(h->d_cls, n);
    ALLOC(h->d_den, 4 * n);
    ALLOC(h->d_init_states, n);
    ALLOC(h->d_tmp, n);
    ALLOC(h->d_t, 256);
    if (h->wind_cell) ALLOC(h->d_wind, 12 * n);
#undef ALLOC
    int32_t* d_ign = nullptr;
    if (hipMemcpy(h->d_envs, ed.data(), sizeof(EnvDev) * n_env, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_chunk_env, chunk_env.data(), sizeof(int32_t) * chunk_env.size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
        fail(h, SIM_EHIP, "env table upload failed");
        return bail(SIM_EHIP);
    }
    if (n_ign > 0) {
        if (hipMalloc(&d_ign, 12 * (size_t)n_ign) != hipSuccess) {
            fail(h, SIM_ENOMEM, "ignition list allocation failed");
            return bail(SIM_ENOMEM);
        }
        if (hipMemcpy(d_ign, ignitions, 12 * (size_t)n_ign, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d_ign);
            fail(h, SIM_EHIP, "ignition list upload failed");
            return bail(SIM_EHIP);
        }
    }
    hipError_t e = launch_init_cells(s, n_cells, landcover, density, elevation, wind_cell,
                                     p->veg, p->unburnable_mask, h->d_g, h->d_E, h->d_cls,
                                     h->d_den, h->d_wind, states_out);
    if (e == hipSuccess) e = launch_ignite(s, d_ign, n_ign, h->d_envs, states_out);
    if (e == hipSuccess) e = launch_copy_u8(s, h->d_init_states, states_out, n_cells);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (d_ign) (void)hipFree(d_ign);
    if (e != hipSuccess) {
        fail(h, SIM_EHIP, "initialisation kernels failed: %s", hipGetErrorString(e));
        return bail(SIM_EHIP);
    }
    if ((rc = build_tiles(h, h->all, tiles_key(h->all.plan), h->all.plan.tile_width)) != SIM_OK) return bail(rc);
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        fail(h, SIM_EHIP, "stream creation failed");
        return bail(SIM_EHIP);
    }
    *out = h;
    return SIM_OK;
}

namespace {

int step_common(sim_handle* h, uint8_t* states, const int32_t* actions, int32_t T, int32_t* counts,
                uint8_t* history, void* stream)
{
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (T < 0) return fail(h, SIM_EINVAL, "T must be >= 0");
    if (!states) return fail(h, SIM_EINVAL, "states is NULL");
    if (T == 0) return SIM_OK;
    if (h->t + (uint64_t)T > 0xFFFFFFFFull)
        return fail(h, SIM_ESTATE, "step counter would pass 2^32");
    if ((h->series_env || h->series_cell) && h->t + (uint64_t)T > (uint64_t)h->series_T)
        return fail(h, SIM_EINVAL, "the wind series covers steps 0..%lld, the call needs up to step %llu",
                    (long long)h->series_T - 1, (unsigned long long)(h->t + T - 1));
    hipStream_t s = (hipStream_t)stream;
    {
        const int rc = ensure_tiles(h);
        if (rc != SIM_OK) return rc;
    }
    HIP_OR_FAIL(h, launch_set_u32(s, h->d_t, (uint32_t)h->t));
    if (h->plan.graph) {
        GraphCache& G = h->graph;
        if (!(G.valid && G.T == T && G.states == states && G.actions == actions &&
              G.counts == counts && G.history == history && same_plan(G.plan, h->plan))) {
            if (G.exec) (void)hipGraphExecDestroy(G.exec);
            G.exec = nullptr;
            G.valid = false;
            hipGraph_t graph = nullptr;
            HIP_OR_FAIL(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_steps(h, h->cap_stream, states, actions, T, counts, history);
            hipError_t e2 = hipStreamEndCapture(h->cap_stream, &graph);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return fail(h, SIM_EHIP, "graph capture failed: %s",
                            hipGetErrorString(e != hipSuccess ? e : e2));
            }
            e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(h, SIM_EHIP, "graph instantiate failed: %s", hipGetErrorString(e));
            G.T = T;
            G.states = states;
            G.actions = actions;
            G.counts = counts;
            G.history = history;
            G.plan = h->plan;
            G.valid = true;
        }
        HIP_OR_FAIL(h, hipGraphLaunch(G.exec, s));
    } else {
        HIP_OR_FAIL(h, enqueue_steps(h, s, states, actions, T, counts, history));
    }
    h->t += (uint64_t)T;
    return SIM_OK;
}

}  // namespace

int sim_step(sim_handle* h, uint8_t* states, const int32_t* actions, int32_t T, int32_t* counts,
             void* stream)
{
    CallScope scope("sim_step", h);
    return step_common(h, states, actions, T, counts, nullptr, stream);
}

int sim_step_history(sim_handle* h, uint8_t* states, const int32_t* actions, int32_t T, int32_t* counts,
                     uint8_t* history, void* stream)
{
    CallScope scope("sim_step_history", h);
    if (h && !history) return fail(h, SIM_EINVAL, "history is NULL");
    return step_common(h, states, actions, T, counts, history, stream);
}

static_assert(sizeof(sim_rl_agent) == sizeof(RlAgent), "agent layout");

namespace {

int rl_check(sim_handle* h, const sim_rl_config* cfg, const void* states, const void* agents, const void* obs)
{
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (!cfg || !states || !agents || !obs) return fail(h, SIM_EINVAL, "cfg, states, agents and obs are required");
    if (cfg->obs_radius < 0 || cfg->obs_radius > 31) return fail(h, SIM_EINVAL, "obs_radius must be in 0..31");
    if (cfg->drop_radius < 0 || cfg->drop_radius > 255) return fail(h, SIM_EINVAL, "drop_radius must be in 0..255");
    if (cfg->water_capacity < 0) return fail(h, SIM_EINVAL, "water_capacity must be >= 0");
    if (cfg->max_steps < 1) return fail(h, SIM_EINVAL, "max_steps must be >= 1");
    if (!h->d_rl_drop) {
        if (hipMalloc(&h->d_rl_drop, (size_t)h->n_env * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&h->d_rl_counts, (size_t)h->n_env * sizeof(int32_t)) != hipSuccess)
            return fail(h, SIM_ENOMEM, "RL buffers allocation failed");
    }
    return SIM_OK;
}

RlConfigDev rl_dev(const sim_rl_config* cfg)
{
    return RlConfigDev{cfg->obs_radius, cfg->max_steps, cfg->burn_penalty, cfg->extinguish_bonus};
}

}  // namespace

int sim_rl_reset(sim_handle* h, const sim_rl_config* cfg, uint8_t* states, sim_rl_agent* agents,
                 const int32_t* reset_mask, uint64_t episode, uint8_t* obs, int32_t* done_out, void* stream)
{
    CallScope scope("sim_rl_reset", h);
    int rc = rl_check(h, cfg, states, agents, obs);
    if (rc != SIM_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    RlAgent* ag = reinterpret_cast<RlAgent*>(agents);
    HIP_OR_FAIL(h, launch_rl_reset(s, h->d_envs, h->n_env, h->d_cls, h->params.unburnable_mask, states, ag,
                                   reset_mask, (uint32_t)h->seed, (uint32_t)(h->seed >> 32), episode,
                                   cfg->water_capacity));
    HIP_OR_FAIL(h, launch_rl_obs(s, h->d_envs, h->n_env, states, ag, nullptr, rl_dev(cfg), obs, nullptr,
                                 done_out));
    return SIM_OK;
}

int sim_rl_step(sim_handle* h, const sim_rl_config* cfg, uint8_t* states, sim_rl_agent* agents,
                const int32_t* actions, uint8_t* obs, float* reward, int32_t* done, void* stream)
{
    CallScope scope("sim_rl_step", h);
    int rc = rl_check(h, cfg, states, agents, obs);
    if (rc != SIM_OK) return rc;
    if (!actions || !reward || !done) return fail(h, SIM_EINVAL, "actions, reward and done are required");
    if (h->t + 1 > 0xFFFFFFFFull) return fail(h, SIM_ESTATE, "step counter would pass 2^32");
    if ((h->series_env || h->series_cell) && h->t + 1 > (uint64_t)h->series_T)
        return fail(h, SIM_EINVAL, "the wind series does not cover step %llu", (unsigned long long)h->t);
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ensure_tiles(h)) != SIM_OK) return rc;
    RlAgent* ag = reinterpret_cast<RlAgent*>(agents);
    if (cfg->single_launch && h->rl_shape.fits) {
        StepLaunch L = step_launch(h, h->all);
        L.args.drop_mode = SIM_DROP_WATER;
        L.args.drop_radius = cfg->drop_radius;
        HIP_OR_FAIL(h, launch_rl_step_fused(s, h->d_envs, h->n_env, L.fields, L.args, h->rl_shape, states, ag,
                                            actions, rl_dev(cfg), (uint32_t)h->t, obs, reward, done));
        h->t += 1;
        return SIM_OK;
    }
    const int32_t water[2] = {SIM_DROP_WATER, cfg->drop_radius};
    HIP_OR_FAIL(h, launch_set_u32(s, h->d_t, (uint32_t)h->t));
    HIP_OR_FAIL(h, launch_rl_act(s, h->d_envs, h->n_env, ag, actions, h->d_rl_drop));
    HIP_OR_FAIL(h, enqueue_steps(h, s, states, h->d_rl_drop, 1, h->d_rl_counts, nullptr, water));
    HIP_OR_FAIL(h, launch_rl_obs(s, h->d_envs, h->n_env, states, ag, h->d_rl_counts, rl_dev(cfg), obs, reward,
                                 done));
    h->t += 1;
    return SIM_OK;
}

int sim_set_drop(sim_handle* h, int32_t mode, int32_t radius)
{
    CallScope scope("sim_set_drop", h);
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (mode != SIM_DROP_SUPPRESS && mode != SIM_DROP_WATER) return fail(h, SIM_EINVAL, "unknown drop mode");
    if (radius < 0 || radius > 255) return fail(h, SIM_EINVAL, "drop radius must be in 0..255");
    h->drop_mode = mode;
    h->drop_radius = radius;
    h->graph.valid = false;  // the drop setting is a kernel argument
    return SIM_OK;
}

int sim_set_wind_series(sim_handle* h, const float* env_wind, const float* cell_wind, int64_t series_T)
{
    CallScope scope("sim_set_wind_series", h);
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (env_wind && cell_wind) return fail(h, SIM_EINVAL, "give a per-env or a per-cell series, not both");
    if ((env_wind || cell_wind) && series_T < 1) return fail(h, SIM_EINVAL, "series_T must be >= 1");
    if (!env_wind && !cell_wind) series_T = 0;
    if (env_wind && h->wind_cell)
        return fail(h, SIM_EINVAL, "this handle has per-cell wind: give a per-cell series");
    h->series_env = env_wind;
    h->series_cell = cell_wind;
    h->series_T = series_T;
    h->graph.valid = false;  // the series pointers are kernel arguments
    return SIM_OK;
}

int sim_get_step(const sim_handle* h, uint64_t* t)
{
    if (!h || !t) return SIM_EINVAL;
    *t = h->t;
    return SIM_OK;
}

int sim_set_step(sim_handle* h, uint64_t t)
{
    CallScope scope("sim_set_step", h);
    if (!h) return SIM_EINVAL;
    if (t > 0xFFFFFFFFull) return fail(h, SIM_EINVAL, "step counter must be < 2^32");
    h->t = t;
    return SIM_OK;
}

}  // extern "C"

namespace {

void drop_classes(sim_handle* h)
{
    for (PlanGroup& g : h->classes) free_group(g);
    h->classes.clear();
    for (hipStream_t cs : h->class_streams) (void)hipStreamDestroy(cs);
    for (hipEvent_t ev : h->class_events) (void)hipEventDestroy(ev);
    h->class_streams.clear();
    h->class_events.clear();
    h->graph.valid = false;
}

// Split the batch into its size classes, each under the handle-wide plan;
// all or nothing (on an error the handle keeps one plan for all envs).
int make_classes_or_partial(sim_handle* h);
int make_classes(sim_handle* h)
{
    const int rc = make_classes_or_partial(h);
    if (rc != SIM_OK) {
        const std::string err = h->err;
        drop_classes(h);
        h->err = err;
    }
    return rc;
}

int make_classes_or_partial(sim_handle* h)
{
    std::vector<PlanGroup> cls(SIM_N_SIZE_CLASSES);
    for (int32_t e = 0; e < h->n_env; ++e) cls[size_class_of(h->envs[e].H, h->envs[e].W)].envs.push_back(e);
    drop_classes(h);
    for (int c = 0; c < SIM_N_SIZE_CLASSES; ++c) {
        PlanGroup& g = cls[c];
        if (g.envs.empty()) continue;
        g.size_class = c;
        g.plan = h->plan;
        describe_group(h, g);
        const size_t bytes = g.envs.size() * sizeof(int32_t);
        if (hipMalloc(&g.d_list, bytes) != hipSuccess) return fail(h, SIM_ENOMEM, "size-class env list allocation failed");
        h->classes.push_back(g);  // owns d_list from here
        HIP_OR_FAIL(h, hipMemcpy(h->classes.back().d_list, g.envs.data(), bytes, hipMemcpyHostToDevice));
    }
    if (h->classes.size() > 1) {
        // default-priority streams (no priority is ever set on them)
        for (size_t i = 0; i < h->classes.size(); ++i) {
            hipStream_t cs = nullptr;
            HIP_OR_FAIL(h, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            h->class_streams.push_back(cs);
        }
        for (size_t i = 0; i <= h->classes.size(); ++i) {
            hipEvent_t ev = nullptr;
            HIP_OR_FAIL(h, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            h->class_events.push_back(ev);
        }
    }
    return SIM_OK;
}

PlanGroup* find_class(sim_handle* h, int32_t c)
{
    for (PlanGroup& g : h->classes)
        if (g.size_class == c) return &g;
    return nullptr;
}

// Time every candidate plan on group g alone (T_probe steps from `states`
// in `work`) and give g the fastest; `tried` receives the plans, fastest
// first.  g's graph field is kept.
int tune_group(sim_handle* h, PlanGroup& g, hipStream_t s, const uint8_t* states, uint8_t* work, int32_t T_probe,
               int32_t allow_skip, int32_t allow_sparse, std::vector<sim_tune_result>& tried)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(h, SIM_EHIP, "event creation failed");
    }
    const sim_plan saved = g.plan;
    std::vector<sim_plan> cands;
    for (int skip = 0; skip <= (allow_skip ? 1 : 0); ++skip)
        for (int width : {64, 256})
            for (int rows : {1, 2, 4, 8})
                cands.push_back(sim_plan{rows, width, 1, skip, allow_sparse ? 1 : 0, 0, 0});
    if (allow_skip && g.aligned)  // temporal blocking reads fuel and elevation only at fronts, like skip
        for (int width : {64, 128})
            for (int k : {2, 4, 8}) cands.push_back(sim_plan{4, width, k, 1, 0, 0, 0});
    if (allow_skip && g.res.fits)  // so does the resident kernel
        for (int nt : {64, 256, 512, 1024}) cands.push_back(sim_plan{4, 64, 1, 1, allow_sparse ? 1 : 0, 0, nt});
    tried.clear();
    int rc = SIM_OK;
    for (const sim_plan& cand : cands) {
        g.plan = cand;
        if ((rc = ensure_group_tiles(h, g)) != SIM_OK) break;
        hipError_t e = hipSuccess;
        float best = 0.0f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first pass warms up
            e = launch_copy_u8(s, work, states, h->n_cells);
            if (e == hipSuccess) e = launch_set_u32(s, h->d_t, (uint32_t)h->t);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = enqueue_group(h, g, s, work, nullptr, T_probe, nullptr, nullptr, nullptr);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&best, e0, e1);
        }
        if (e != hipSuccess) {
            rc = fail(h, SIM_EHIP, "autotune run failed: %s", hipGetErrorString(e));
            break;
        }
        tried.push_back(sim_tune_result{g.plan, best / (float)T_probe});
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(tried.begin(), tried.end(),
              [](const sim_tune_result& a, const sim_tune_result& b) { return a.ms_per_step < b.ms_per_step; });
    g.plan = saved;
    if (rc == SIM_OK && !tried.empty()) {
        g.plan = tried[0].plan;
        g.plan.graph = saved.graph;
        g.tuned_ms = tried[0].ms_per_step;
    }
    h->graph.valid = false;
    const int built = ensure_group_tiles(h, g);
    return rc == SIM_OK ? built : rc;
}

int check_tune_args(sim_handle* h, const uint8_t* states, int32_t T_probe)
{
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (!states || T_probe < 1) return fail(h, SIM_EINVAL, "need states and T_probe >= 1");
    if ((h->series_env || h->series_cell) && h->t + (uint64_t)T_probe > (uint64_t)h->series_T)
        return fail(h, SIM_EINVAL, "T_probe steps from the current step run past the wind series");
    return SIM_OK;
}

// The tuning-cache key of a size class (one line of text, no ':').
std::string class_key(const sim_handle* h, const PlanGroup& g, int32_t T_probe, int32_t allow_skip,
                      int32_t allow_sparse)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    for (char& c : arch)
        if (c == ' ' || c == ':') c = '_';
    const char* wind = h->series_cell ? "cell_series" : (h->series_env ? "env_series" : (h->wind_cell ? "cell" : "env"));
    std::ostringstream k;
    k << "firesim-plan-v1 arch=" << arch << " class=" << g.size_class << " n_env=" << g.envs.size()
      << " cells=" << g.n_cells << " max_h=" << g.max_h << " max_w=" << g.max_w << " aligned=" << (g.aligned ? 1 : 0)
      << " wind=" << wind << " T_probe=" << T_probe << " allow_skip=" << (allow_skip ? 1 : 0)
      << " allow_sparse=" << (allow_sparse ? 1 : 0);
    return k.str();
}

void class_entry(const PlanGroup& g, sim_class_plan& out)
{
    out.size_class = g.size_class;
    out.n_env = (int32_t)g.envs.size();
    out.n_cells = g.n_cells;
    out.plan = g.plan;
    out.ms_per_step = g.tuned_ms;
    out.from_cache = g.from_cache ? 1 : 0;
}

}  // namespace

extern "C" {

int sim_set_plan(sim_handle* h, const sim_plan* plan)
{
    CallScope scope("sim_set_plan", h);
    if (!h || !plan) return SIM_EINVAL;
    sim_plan p = *plan;
    const int rc = validate_plan(h, h->all, p);
    if (rc != SIM_OK) return rc;
    drop_classes(h);
    h->plan = p;
    h->all.plan = p;
    return SIM_OK;
}

int sim_get_plan(const sim_handle* h, sim_plan* plan)
{
    if (!h || !plan) return SIM_EINVAL;
    *plan = h->plan;
    return SIM_OK;
}

int sim_autotune(sim_handle* h, const uint8_t* states, int32_t T_probe, int32_t allow_skip,
                 int32_t allow_sparse, sim_tune_result* results, int32_t max_results,
                 int32_t* n_results, void* stream)
{
    CallScope scope("sim_autotune", h);
    int rc = check_tune_args(h, states, T_probe);
    if (rc != SIM_OK) return rc;
    if (max_results < 0 || (max_results > 0 && !results))
        return fail(h, SIM_EINVAL, "need a results array for max_results > 0");
    drop_classes(h);
    uint8_t* work = nullptr;
    if (hipMalloc(&work, (size_t)h->n_cells) != hipSuccess)
        return fail(h, SIM_ENOMEM, "autotune scratch allocation failed");
    std::vector<sim_tune_result> tried;
    h->all.plan = h->plan;
    rc = tune_group(h, h->all, (hipStream_t)stream, states, work, T_probe, allow_skip, allow_sparse, tried);
    (void)hipFree(work);
    h->plan = h->all.plan;
    const int n = std::min<int>((int)tried.size(), max_results);
    for (int i = 0; i < n; ++i) results[i] = tried[i];
    if (n_results) *n_results = n;
    return rc;
}

int sim_set_class_plan(sim_handle* h, int32_t size_class, const sim_plan* plan)
{
    CallScope scope("sim_set_class_plan", h);
    if (!h || !plan) return fail(h, SIM_EINVAL, "handle and plan are required");
    int rc;
    if (h->classes.empty() && (rc = make_classes(h)) != SIM_OK) return rc;
    PlanGroup* g = find_class(h, size_class);
    if (!g) return fail(h, SIM_EINVAL, "the batch has no env in size class %d", size_class);
    sim_plan p = *plan;
    if ((rc = validate_plan(h, *g, p)) != SIM_OK) return rc;
    g->plan = p;
    g->tuned_ms = 0.0f;
    g->from_cache = false;
    h->graph.valid = false;
    return SIM_OK;
}

int sim_get_class_plans(const sim_handle* h, sim_class_plan* out, int32_t max_out, int32_t* n_out)
{
    if (!h || max_out < 0 || (max_out > 0 && !out)) return SIM_EINVAL;
    std::vector<sim_class_plan> list;
    if (!h->classes.empty()) {
        for (const PlanGroup& g : h->classes) {
            sim_class_plan c{};
            class_entry(g, c);
            list.push_back(c);
        }
    } else {
        std::vector<sim_class_plan> all(SIM_N_SIZE_CLASSES);
        for (const sim_env& v : h->envs) {
            sim_class_plan& c = all[size_class_of(v.H, v.W)];
            c.n_env += 1;
            c.n_cells += (int64_t)v.H * v.W;
        }
        for (int c = 0; c < SIM_N_SIZE_CLASSES; ++c)
            if (all[c].n_env) {
                all[c].size_class = c;
                all[c].plan = h->plan;
                list.push_back(all[c]);
            }
    }
    const int n = std::min<int>((int)list.size(), max_out);
    for (int i = 0; i < n; ++i) out[i] = list[i];
    if (n_out) *n_out = (int32_t)list.size();
    return SIM_OK;
}

int sim_autotune_classes(sim_handle* h, const uint8_t* states, int32_t T_probe, int32_t allow_skip,
                         int32_t allow_sparse, const char* cache_path, sim_class_plan* out,
                         int32_t max_out, int32_t* n_out, void* stream)
{
    CallScope scope("sim_autotune_classes", h);
    int rc = check_tune_args(h, states, T_probe);
    if (rc != SIM_OK) return rc;
    if (max_out < 0 || (max_out > 0 && !out)) return fail(h, SIM_EINVAL, "need an out array for max_out > 0");
    // the cache: key -> plan, the last line of a key winning
    std::vector<std::pair<std::string, std::string>> cached;
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "r");
        if (!f && errno != ENOENT) return fail(h, SIM_EINVAL, "cannot read the tuning cache %s", cache_path);
        if (f) {
            char line[1024];
            while (std::fgets(line, sizeof line, f)) {
                const char* sep = std::strstr(line, " : ");
                if (!sep || std::strncmp(line, "firesim-plan-v1 ", 16) != 0) continue;
                cached.emplace_back(std::string(line, (size_t)(sep - line)), std::string(sep + 3));
            }
            std::fclose(f);
        }
    }
    if ((rc = make_classes(h)) != SIM_OK) return rc;
    uint8_t* work = nullptr;
    std::vector<sim_tune_result> tried;
    std::string appended;
    for (PlanGroup& g : h->classes) {
        const std::string key = class_key(h, g, T_probe, allow_skip, allow_sparse);
        bool hit = false;
        for (auto it = cached.rbegin(); it != cached.rend() && !hit; ++it) {
            if (it->first != key) continue;
            sim_plan p{};
            float ms = 0.0f;
            if (std::sscanf(it->second.c_str(), "%d %d %d %d %d %d %f", &p.tile_rows, &p.tile_width, &p.temporal,
                            &p.skip_static, &p.sparse, &p.resident, &ms) != 7)
                continue;
            p.graph = h->plan.graph;
            const std::string err = h->err;
            if (validate_plan(h, g, p) != SIM_OK) {  // a line this batch cannot take is skipped
                h->err = err;
                continue;
            }
            g.plan = p;
            g.tuned_ms = ms;
            g.from_cache = true;
            hit = true;
        }
        if (hit) continue;
        if (!work && hipMalloc(&work, (size_t)h->n_cells) != hipSuccess) {
            rc = fail(h, SIM_ENOMEM, "autotune scratch allocation failed");
            break;
        }
        if ((rc = tune_group(h, g, (hipStream_t)stream, states, work, T_probe, allow_skip, allow_sparse, tried)) !=
            SIM_OK)
            break;
        char val[160];
        std::snprintf(val, sizeof val, "%d %d %d %d %d %d %.6g\n", g.plan.tile_rows, g.plan.tile_width,
                      g.plan.temporal, g.plan.skip_static, g.plan.sparse, g.plan.resident, (double)g.tuned_ms);
        appended += key + " : " + val;
    }
    if (work) (void)hipFree(work);
    if (rc == SIM_OK && cache_path && !appended.empty()) {
        FILE* f = std::fopen(cache_path, "a");
        if (!f || std::fputs(appended.c_str(), f) < 0) rc = fail(h, SIM_EINVAL, "cannot append to the tuning cache %s", cache_path);
        if (f && std::fclose(f) != 0 && rc == SIM_OK)
            rc = fail(h, SIM_EINVAL, "cannot append to the tuning cache %s", cache_path);
    }
    h->graph.valid = false;
    if (rc == SIM_OK) rc = ensure_tiles(h);
    int32_t n = 0;
    const int rc2 = sim_get_class_plans(h, out, max_out, &n);
    if (n_out) *n_out = n;
    return rc != SIM_OK ? rc : rc2;
}

int sim_relaxed_init(sim_handle* h, double* U, double* B, void* stream)
{
    CallScope scope("sim_relaxed_init", h);
    if (!h || !U || !B) return fail(h, SIM_EINVAL, "handle, U and B are required");
    HIP_OR_FAIL(h, launch_relaxed_init(
                       (hipStream_t)stream, h->d_init_states, h->n_cells, U, B));
    return SIM_OK;
}

size_t sim_relaxed_workspace_bytes(const sim_handle* h, int32_t T, int32_t ckpt_every)
{
    if (!h || T < 0 || ckpt_every < 1) return 0;
    return relaxed_workspace_bytes(h->n_cells, h->n_adj_tiles, T, ckpt_every);
}

static RelaxedInputs relaxed_inputs(const sim_handle* h, int32_t form = 0)
{
    RelaxedInputs in;
    in.form = form;
    in.tiles = h->relaxed.d_btiles;
    in.n_tiles = h->relaxed.n_btiles;
    in.envs = h->d_envs;
    in.n_env = h->n_env;
    in.cls = h->d_cls;
    in.den = h->d_den;
    in.E = h->d_E;
    in.wind = h->wind_cell ? h->d_wind : nullptr;
    in.n_cells = h->n_cells;
    in.sparse = h->plan.sparse;
    if (h->series_cell) {  // relaxed step t takes row t of the wind series
        in.wind = h->series_cell;
        in.wind_stride = 3 * h->n_cells;
    } else if (h->series_env) {
        in.env_wind = h->series_env;
    }
    return in;
}

static int check_relaxed_params(sim_handle* h, const sim_params* p)
{
    if (!p) return fail(h, SIM_EINVAL, "params are NULL");
    if (p->cell_size != h->params.cell_size || p->unburnable_mask != h->params.unburnable_mask)
        return fail(h, SIM_EINVAL, "cell_size and unburnable_mask must match sim_init");
    if (p->slope_mode != SIM_SLOPE_RATIO && p->slope_mode != SIM_SLOPE_ANGLE)
        return fail(h, SIM_EINVAL, "slope_mode must be SIM_SLOPE_RATIO or SIM_SLOPE_ANGLE");
    return SIM_OK;
}

int sim_step_relaxed_fwd(sim_handle* h, const sim_params* p, double* U, double* B, int32_t T,
                         int32_t ckpt_every, int32_t form, void* workspace, size_t workspace_bytes,
                         void* stream)
{
    CallScope scope("sim_step_relaxed_fwd", h);
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    int rc = check_relaxed_params(h, p);
    if (rc) return rc;
    if (form != SIM_FORM_PRODUCT && form != SIM_FORM_EXP) return fail(h, SIM_EINVAL, "unknown form");
    if ((h->series_env || h->series_cell) && (int64_t)T > h->series_T)
        return fail(h, SIM_EINVAL, "the wind series covers %lld steps, the relaxed run needs %d",
                    (long long)h->series_T, T);
    if (!U || !B || T < 0 || ckpt_every < 1) return fail(h, SIM_EINVAL, "bad U/B/T/ckpt_every");
    if (T > 0 && (!workspace || workspace_bytes < relaxed_workspace_bytes(h->n_cells, h->n_adj_tiles, T, ckpt_every)))
        return fail(h, SIM_EINVAL, "workspace too small (%zu < %zu)", workspace_bytes,
                    relaxed_workspace_bytes(h->n_cells, h->n_adj_tiles, T, ckpt_every));
    if ((rc = relaxed_prepare(h->relaxed, h->envs)) != 0)
        return fail(h, SIM_ENOMEM, "relaxed tile list allocation failed");
    hipError_t e = relaxed_forward((hipStream_t)stream, relaxed_inputs(h, form), *p, U, B, T, ckpt_every,
                                   workspace, h->relaxed);
    if (e != hipSuccess) return fail(h, SIM_EHIP, "relaxed forward failed: %s", hipGetErrorString(e));
    return SIM_OK;
}

static LossBatch loss_batch(const sim_handle* h)
{
    return LossBatch{h->d_envs, h->n_env, h->d_chunk_env, h->n_chunks, h->d_init_states};
}

int sim_relaxed_loss(sim_handle* h, const double* U_T, const uint8_t* target, float* loss,
                     double* gU_T, double scale, double* objective, void* stream)
{
    CallScope scope("sim_relaxed_loss", h);
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (!U_T || !target || !loss) return fail(h, SIM_EINVAL, "U_T, target and loss are required");
    if (!h->d_loss_scratch &&
        hipMalloc(&h->d_loss_scratch, sizeof(double) * loss_scratch_doubles(h->n_chunks, h->n_env)) != hipSuccess) {
        h->d_loss_scratch = nullptr;
        return fail(h, SIM_ENOMEM, "loss scratch allocation failed");
    }
    hipError_t e = relaxed_loss((hipStream_t)stream, loss_batch(h), U_T, target, loss, gU_T, scale, objective,
                                h->d_loss_scratch);
    if (e != hipSuccess) return fail(h, SIM_EHIP, "relaxed loss failed: %s", hipGetErrorString(e));
    return SIM_OK;
}

int sim_relaxed_loss_noalloc(sim_handle* h, const double* U_T, const uint8_t* target, float* loss,
                             double* gU_T, double scale, double* objective, void* stream)
{
    CallScope scope("sim_relaxed_loss_noalloc", h);
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (!U_T || !target || !loss) return fail(h, SIM_EINVAL, "U_T, target and loss are required");
    const size_t need = loss_scratch_doubles(h->n_chunks, h->n_env);
    if (need > kNoallocScratchDoubles)
        return fail(h, SIM_EINVAL,
                    "the batch needs %zu scratch doubles (3 per 4096-cell chunk, 4 per env), "
                    "the static scratch holds %zu: use sim_relaxed_loss",
                    need, kNoallocScratchDoubles);
    hipError_t e = relaxed_loss((hipStream_t)stream, loss_batch(h), U_T, target, loss, gU_T, scale, objective,
                                h->noalloc_scratch);
    if (e != hipSuccess) return fail(h, SIM_EHIP, "relaxed loss failed: %s", hipGetErrorString(e));
    return SIM_OK;
}

int sim_relaxed_loss_bce(sim_handle* h, const double* U_T, const uint8_t* target, int32_t pool,
                         double mse_weight, double eps, float* loss, double* gU_T, double scale,
                         double* objective, void* stream)
{
    CallScope scope("sim_relaxed_loss_bce", h);
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    if (!U_T || !target || !loss) return fail(h, SIM_EINVAL, "U_T, target and loss are required");
    if (pool < 1 || pool > 64 || !(eps > 0.0 && eps < 0.5) || !(mse_weight >= 0.0))
        return fail(h, SIM_EINVAL, "need 1 <= pool <= 64, 0 < eps < 0.5, mse_weight >= 0");
    if (relaxed_prepare(h->relaxed, h->envs) != 0 || relaxed_prepare_pool(h->relaxed, h->envs, pool) != 0)
        return fail(h, SIM_ENOMEM, "relaxed tables allocation failed");
    hipError_t e = relaxed_loss_bce((hipStream_t)stream, relaxed_inputs(h), h->d_init_states, U_T,
                                    target, pool, mse_weight, eps, loss, gU_T, scale, objective, h->relaxed);
    if (e != hipSuccess) return fail(h, SIM_EHIP, "relaxed loss failed: %s", hipGetErrorString(e));
    return SIM_OK;
}

int sim_step_relaxed_bwd(sim_handle* h, const sim_params* p, const double* gU_T, const double* gB_T,
                         int32_t T, int32_t ckpt_every, int32_t form, void* workspace,
                         size_t workspace_bytes, double* grad, void* stream)
{
    CallScope scope("sim_step_relaxed_bwd", h);
    if (!h) return fail(nullptr, SIM_EINVAL, "handle is NULL");
    int rc = check_relaxed_params(h, p);
    if (rc) return rc;
    if (form != SIM_FORM_PRODUCT && form != SIM_FORM_EXP) return fail(h, SIM_EINVAL, "unknown form");
    if ((h->series_env || h->series_cell) && (int64_t)T > h->series_T)
        return fail(h, SIM_EINVAL, "the wind series covers %lld steps, the relaxed run needs %d",
                    (long long)h->series_T, T);
    if (!gU_T || !grad || T < 0 || ckpt_every < 1) return fail(h, SIM_EINVAL, "bad gU_T/grad/T/ckpt_every");
    if (T > 0 && (!workspace || workspace_bytes < relaxed_workspace_bytes(h->n_cells, h->n_adj_tiles, T, ckpt_every)))
        return fail(h, SIM_EINVAL, "workspace too small");
    if ((rc = relaxed_prepare(h->relaxed, h->envs)) != 0)
        return fail(h, SIM_ENOMEM, "relaxed tile list allocation failed");
    hipError_t e = relaxed_backward((hipStream_t)stream, relaxed_inputs(h, form), *p, gU_T, gB_T, T,
                                    ckpt_every, workspace, grad, h->relaxed);
    if (e != hipSuccess) return fail(h, SIM_EHIP, "relaxed backward failed: %s", hipGetErrorString(e));
    return SIM_OK;
}

int sim_debug_atan(const float* x, float* y, int64_t n, void* stream)
{
    CallScope scope("sim_debug_atan", nullptr);
    if (n < 0 || (n > 0 && (!x || !y))) return SIM_EINVAL;
    return launch_debug_atan((hipStream_t)stream, x, y, n) == hipSuccess ? SIM_OK : SIM_EHIP;
}

int sim_debug_exp(const float* x, float* y, int64_t n, void* stream)
{
    CallScope scope("sim_debug_exp", nullptr);
    if (n < 0 || (n > 0 && (!x || !y))) return SIM_EINVAL;
    return launch_debug_exp((hipStream_t)stream, x, y, n) == hipSuccess ? SIM_OK : SIM_EHIP;
}

int sim_debug_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n, void* stream)
{
    CallScope scope("sim_debug_philox", nullptr);
    if (n < 0 || (n > 0 && (!ctr || !key || !out))) return SIM_EINVAL;
    return launch_debug_philox((hipStream_t)stream, ctr, key, out, n) == hipSuccess ? SIM_OK : SIM_EHIP;
}

int sim_debug_stream(int32_t mode, const void* src, void* dst, int64_t bytes, int32_t blocks, void* stream)
{
    CallScope scope("sim_debug_stream", nullptr);
    if (mode < 0 || mode > 2 || bytes < 16 || bytes % 16 != 0 || blocks < 1 || blocks > (1 << 20))
        return SIM_EINVAL;
    if ((mode != 1 && (!src || (uintptr_t)src % 16)) || !dst || (uintptr_t)dst % 16) return SIM_EINVAL;
    return launch_stream_probe((hipStream_t)stream, mode, src, dst, bytes / 16, blocks) == hipSuccess ? SIM_OK
                                                                                                     : SIM_EHIP;
}

const char* sim_last_error(const sim_handle* h)
{
    return h ? h->err.c_str() : g_init_error.c_str();
}

void sim_destroy(sim_handle* h)
{
    CallScope scope("sim_destroy", h);
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
}

}  // extern "C"
