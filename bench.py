"""Benchmark of the batched fire-spread step on one MI355X.

One benchmark step = one pass of the hot path over the batch: the 1024 envs
of 256 x 256 cells are reset to their initial fire state and advanced 200
stochastic steps (one sim_step call, in-kernel burning counts).  `value` is
cell-updates per second over the timed steps (1024 * 65536 * 200 per step),
with the dense plan (every step reads the whole state, fuel and elevation).

Reported beside it, each in its own object:
  variants    - the same workload under the front-skipping plans (static
                fields skipped off the front, sparse active tiles, autotuned);
                effective rates, not roofline evidence;
  dense_front - an ALU-bound case: a stationary checkerboard front where every
                cell evaluates its neighbourhood each step;
  relaxed     - the relaxed forward + adjoint on 256 envs of 128 x 128 (T 100)
                and on one 2048 x 2048 env (T 500), checkpoints every 10;
  paper_setting, rl, uneven, large - the paper's 64 x 64^2 vectorised
                setting, the RL layer on 65536 envs of 20 x 20, the 4096-env
                uneven batch with drops, and 8 envs of 2048 x 2048 with
                per-cell wind (1000 steps);
  product_plan - the same workload under the library's default plan (fuel
                read at fronts, quiet tiles skipped), with counter-measured HBM
                bytes;
  stream_probe - the library's HBM streaming probe (read, write, copy of
                1 GiB) and torch's copy: the attainable bandwidth;
  cpu_baseline - the CPU oracle on the same stochastic workload.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# 256 CUs x 64 lanes x 2.4 GHz: one non-packed 32-bit VALU op per lane per cycle
ALU_PEAK_GOPS = 256 * 64 * 2.4
STOCH_BYTES_PER_CELL = 10      # state r/w 2 B + fuel 4 B + elevation 4 B per cell-update
STOCH_WIND_CELL_BYTES = 12     # per-cell wind adds V, Vx, Vy (3 x 4 B) per cell-update
# relaxed, fp64 state, per cell-step: forward 40 B (U,B r/w 32 + fuel,
# elevation 8) and adjoint 61 B (U,B 16, adjoint r/w 32, fuel, elevation,
# density 12, class 1); per-cell wind adds V, Vx, Vy (12 B) to each pass
RELAXED_FWD_BYTES, RELAXED_ADJ_BYTES, RELAXED_WIND_BYTES = 40, 61, 12
# the same accounting for an fp32 state (what the method must move): forward
# 24 B (U,B r/w 16 + fuel, elevation 8), adjoint 32 B (U,B 8, adjoint r/w 16,
# fuel, elevation 8); forward + recompute + adjoint = 80 B per cell-step
RELAXED_ALG_FWD_BYTES, RELAXED_ALG_ADJ_BYTES = 24, 32
RELAXED_ALG_BYTES = 2 * RELAXED_ALG_FWD_BYTES + RELAXED_ALG_ADJ_BYTES


def relaxed_bytes_per_cell_step(T: int, k: int, wind_cell: bool) -> float:
    """Forward, adjoint and the recompute of every checkpoint segment but the
    last (whose states the forward leaves in place): (ceil(T/k) - 1)(k - 1)
    recomputed steps; plus copying the initial state into checkpoint 0."""
    recomputed = ((T + k - 1) // k - 1) * (k - 1) / T
    w = RELAXED_WIND_BYTES if wind_cell else 0
    return (RELAXED_FWD_BYTES + w) * (1 + recomputed) + RELAXED_ADJ_BYTES + w + 32.0 / T
# fp32/int32 operations of the method (separate multiply and add, as the step
# is specified): one phi term 30 (slope 2, exponent 2, exp 23, scale 2, sum 1),
# the ignition probability 26 (gamma 1, product 1, exp 23, 1-e 1), one draw 29
# (a quarter of a Philox4x32-10 block 25, uniform 2, compare 2)
OPS_PHI, OPS_PROB, OPS_DRAW = 30, 26, 29
KERNEL_SOURCES = ("paper_2512_06102_amd/csrc/stoch.hip", "paper_2512_06102_amd/csrc/stepcell.hpp",
                  "paper_2512_06102_amd/csrc/devmath.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stoch_step_batch256_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(plan_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter records, if
    one was taken on the current kernel source and this plan."""
    try:
        recs = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    for rec in recs.get("records", []):
        if rec.get("kernel_hash") == kernel_hash() and rec.get("plan") == plan_key:
            return rec.get("bytes_per_launch")
    return None


def plan_key_of(plan: dict) -> str:
    return "tile_rows=%d,tile_width=%d,skip_static=%d,sparse=%d" % (
        plan["tile_rows"], plan["tile_width"], plan["skip_static"], plan["sparse"])


def stream_probe(torch, fs):
    """Attainable HBM bandwidth on this GPU: the library's streaming probe
    (16-byte accesses, nontemporal stores) reading, writing and copying 1 GiB,
    and torch's 1 GiB device copy beside it."""
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()

    def best_ms(fn):
        fn()
        best = float("inf")
        for _ in range(5):
            with StepTimer(torch, stream) as tm:
                fn()
            best = min(best, tm.ms())
        return best

    out = {"kind": "1 GiB streams; best of 5 at each of 16384, 32768 and 65536 workgroups"}
    for name, mode, moved in (("read", 0, 1), ("write", 1, 1), ("copy", 2, 2)):
        ms, blocks = min((best_ms(lambda: fs.debug_stream(mode, None if mode == 1 else a, b, blocks=nb)), nb)
                         for nb in (16384, 32768, 65536))
        gbs = moved * a.numel() / (ms / 1e3) / 1e9
        out[name] = {"ms": round(ms, 4), "GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                     "workgroups": blocks}
        log("[bench] stream probe %s: 1 GiB in %.3f ms = %.0f GB/s" % (name, ms, gbs))
    ms = best_ms(lambda: b.copy_(a))
    gbs = 2 * a.numel() / (ms / 1e3) / 1e9
    out["torch_copy"] = {"ms": round(ms, 4), "GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
    log("[bench] torch copy_: 1 GiB in %.3f ms = %.0f GB/s (read + write)" % (ms, gbs))
    del a, b
    return out


def cpu_baseline(batch, params, T, seed):
    """The oracle, as written, on a bounded sample of the same workload."""
    import oracle

    threads = min(16, len(os.sched_getaffinity(0)))
    n_env = min(batch.n_env, 64 * threads)
    sub = batch.subset(range(n_env))
    sim = oracle.Sim(sub, params, seed=seed)
    t0 = time.perf_counter()
    sim.step(T, counts=True, threads=threads)
    dt = time.perf_counter() - t0
    cells = float(sub.n_cells) * T
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the 1024 envs (256x256), %d steps from the initial state, "
                      "one env per thread at a time, %.1f s" % (n_env, T, dt)}


class StepTimer:
    """HIP events on the launch stream around a region."""

    def __init__(self, torch, stream):
        self.torch, self.stream = torch, stream

    def __enter__(self):
        ev = self.torch.cuda.Event
        self.a, self.b = ev(enable_timing=True), ev(enable_timing=True)
        self.a.record(self.stream)
        return self

    def __exit__(self, *exc):
        self.b.record(self.stream)

    def ms(self):
        self.torch.cuda.synchronize()
        return self.a.elapsed_time(self.b)


def timed_runs(torch, stream, sim, init, T, steps, warmup):
    """Reset + T steps, `warmup` untimed then `steps` timed; returns (ms per
    reset+T-steps, ms per step launch of the last timed run)."""
    def one():
        sim.states.copy_(init)
        sim.t = 0
        sim.step(T, counts=True)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    with StepTimer(torch, stream) as whole:
        for i in range(steps - 1):
            one()
        sim.states.copy_(init)
        sim.t = 0
        with StepTimer(torch, stream) as last:
            sim.step(T, counts=True)
    return whole.ms() / steps, last.ms() / T


def bench_stochastic(args, torch, fs, firegen):
    batch, params, T, seed = firegen.workload_batch256()
    log("[bench] workload generated: %d envs, %d cells" % (batch.n_env, batch.n_cells))
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    plan = {"tile_rows": args.tile_rows, "tile_width": args.tile_width,
            "skip_static": args.skip_static, "sparse": args.sparse, "graph": args.graph}
    sim.set_plan(**plan)
    init = sim.states.clone()
    stream = torch.cuda.current_stream()
    if args.no_stochastic:
        return dict(batch=batch, params=params, T=T, seed=seed, value=None, ms=float("nan"), roof=None,
                    plan=plan, burning=None, sim=sim, init=init)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ms, launch_ms = timed_runs(torch, stream, sim, init, T, args.steps, args.warmup)
    wall = time.perf_counter() - wall0
    cells = float(batch.n_cells)
    value = cells * T / (ms / 1e3)
    achieved = STOCH_BYTES_PER_CELL * cells / (launch_ms / 1e3) / 1e9
    plan_key = plan_key_of(sim.plan())
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(plan_key),
            "kernel": "stoch_step_kernel", "launch_ms": round(launch_ms, 5),
            "algorithmic_bytes_per_launch": STOCH_BYTES_PER_CELL * int(cells),
            "note": "one step per tile load with every cell's state, fuel and elevation streamed (the "
                    "k=1 roofline probe); front cells read their neighbours' fuel and elevation again "
                    "through the cache, so the fuel and elevation of non-front cells are loaded unused; "
                    "the library's default plan skips them (product_plan)"}
    log("[bench] stochastic: %.3f ms/step, %.3e cell-updates/s, kernel %.4f ms = %.0f GB/s (wall %.2fs)"
        % (ms, value, launch_ms, achieved, wall))
    sim.states.copy_(init)
    sim.t = 0
    burning = int(sim.step(T, counts=True).sum())
    return dict(batch=batch, params=params, T=T, seed=seed, value=value, ms=ms, roof=roof, plan=plan,
                burning=burning, sim=sim, init=init)


# the library's default launch plan (what sim_init sets), graph-replayed here
PRODUCT_PLAN = dict(tile_rows=4, tile_width=64, skip_static=1, sparse=1, graph=1)


def bench_product_plan(args, torch, fs, st):
    """The default plan on the same workload: fuel and elevation read only at
    front cells, tiles with no fire in reach skipped.  Its roofline uses the
    HBM bytes the counters measured for it (an effective rate: it moves fewer
    than the 10 B per cell-update the dense probe streams)."""
    sim, init, T = st["sim"], st["init"], st["T"]
    cells = float(st["batch"].n_cells)
    stream = torch.cuda.current_stream()
    sim.set_plan(**PRODUCT_PLAN)
    ms, launch_ms = timed_runs(torch, stream, sim, init, T, args.steps, 1)
    traffic = stored_traffic(plan_key_of(sim.plan()))
    roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
            "traffic": traffic, "kernel": "stoch_step_kernel", "launch_ms": round(launch_ms, 5),
            "bytes_per_cell_update": None if traffic is None else round(traffic / cells, 3)}
    if traffic is not None:
        roof["achieved"] = round(traffic / (launch_ms / 1e3) / 1e9, 1)
        roof["frac"] = round(roof["achieved"] / HBM_PEAK_GBS, 4)
    out = {"plan": PRODUCT_PLAN, "ms_per_step": round(ms, 4), "value": cells * T / (ms / 1e3),
           "unit": "cell-updates/s", "roofline": roof,
           "note": "the library's default plan; bit-identical states; achieved = counter-measured HBM bytes "
                   "per launch / launch time"}
    log("[bench] product plan: %.3f ms/step, %.3e cell-updates/s, launch %.4f ms, traffic %s"
        % (ms, out["value"], launch_ms, traffic))
    return out


def bench_variants(args, torch, fs, st):
    """The same workload under the front-skipping plans: effective rates."""
    sim, init, T = st["sim"], st["init"], st["T"]
    cells = float(st["batch"].n_cells)
    stream = torch.cuda.current_stream()
    out = {}
    for name, plan in (("skip_static", dict(tile_rows=4, tile_width=64, skip_static=1, graph=1)),
                       ("sparse", dict(tile_rows=4, tile_width=64, skip_static=1, sparse=1, graph=1)),
                       ("temporal4", dict(tile_width=128, temporal=4, graph=1)),
                       ("temporal8", dict(tile_width=128, temporal=8, graph=1))):
        sim.set_plan(**plan)
        ms, launch_ms = timed_runs(torch, stream, sim, init, T, args.steps, 1)
        out[name] = {"plan": plan, "ms_per_step": round(ms, 4), "value": cells * T / (ms / 1e3),
                     "launch_ms_last_run": round(launch_ms * plan.get("temporal", 1), 5)}
        log("[bench] variant %s: %.3f ms/step, %.3e cell-updates/s" % (name, ms, out[name]["value"]))
    sim.states.copy_(init)
    sim.t = 0
    tuned = sim.autotune(T_probe=T, allow_skip=True, allow_sparse=True)
    best = sim.plan()
    keys = ("tile_rows", "tile_width", "temporal", "skip_static", "sparse", "resident")
    sim.set_plan(**{k: best[k] for k in keys}, graph=1)
    ms, launch_ms = timed_runs(torch, stream, sim, init, T, args.steps, 1)
    out["autotuned"] = {"plan": {k: best[k] for k in keys},
                        "candidates": len(tuned), "ms_per_step": round(ms, 4),
                        "value": cells * T / (ms / 1e3)}
    log("[bench] autotuned %s: %.3f ms/step" % (out["autotuned"]["plan"], ms))
    out["note"] = ("effective rates: these plans read fuel and elevation only near burning cells, "
                   "skip quiescent tiles (sparse) or advance 4 / 8 steps per tile load (temporal), so "
                   "their bytes moved per cell-update are below the 10 B the roofline counts; not "
                   "roofline evidence")
    return out


def dense_front_ops(batch, states, firegen):
    """Operations of one step of the method on a state (count of phi terms,
    ignition probabilities and draws), priced with OPS_*."""
    import numpy as np

    n_phi = n_front = n_draw = 0
    for e in range(batch.n_env):
        st = batch.env_view(states, e)
        burn = np.pad(st == firegen.BURNING, 1)
        H, W = st.shape
        nb = np.zeros((H, W), np.int32)
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                if di or dj:
                    nb += burn[1 + di:1 + di + H, 1 + dj:1 + dj + W]
        flam = st == firegen.FLAMMABLE
        front = flam & (nb > 0)
        n_phi += int(nb[flam].sum())
        n_front += int(front.sum())
        n_draw += int(front.sum() + (st == firegen.BURNING).sum())
    return n_phi, n_front, n_draw, OPS_PHI * n_phi + OPS_PROB * n_front + OPS_DRAW * n_draw


def bench_dense_front(args, torch, fs, firegen, st):
    """A stationary dense front: p_continue 1 keeps burning cells burning and a
    negligible p_base keeps flammable ones flammable, while every cell still
    evaluates its burning neighbours each step."""
    batch, seed = st["batch"], st["seed"]
    params = st["params"].replace(p_base=1e-30, p_continue=1.0)
    dense = firegen.dense_front_states(batch)
    n_phi, n_front, n_draw, ops = dense_front_ops(batch, dense, firegen)
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    sim.set_plan(tile_rows=args.tile_rows, tile_width=args.tile_width, skip_static=0, sparse=0, graph=1)
    init = torch.from_numpy(dense).to(sim.states.device)
    T = 20
    stream = torch.cuda.current_stream()
    ms, launch_ms = timed_runs(torch, stream, sim, init, T, args.steps, 1)
    same = bool(torch.equal(sim.states, init))
    cells = float(batch.n_cells)
    gops = ops / (launch_ms / 1e3) / 1e9
    log("[bench] dense front: %.4f ms per launch, %.3e cell-updates/s, %.0f Gop/s (stationary %s)"
        % (launch_ms, cells / (launch_ms / 1e3), gops, same))
    return {"workload": "1024 envs x 256x256, checkerboard BURNING/FLAMMABLE front, p_continue 1, "
                        "p_base 1e-30 (stationary), 20 steps per call",
            "value": cells / (launch_ms / 1e3), "unit": "cell-updates/s", "stationary": same,
            "roofline": {"bound": "alu", "achieved": round(gops, 1), "peak": ALU_PEAK_GOPS,
                         "unit": "Gop/s", "frac": round(gops / ALU_PEAK_GOPS, 4),
                         "ops_per_launch": ops, "phi_terms": n_phi, "front_cells": n_front,
                         "draws": n_draw, "launch_ms": round(launch_ms, 5),
                         "hbm_GBs_at_10B": round(STOCH_BYTES_PER_CELL * cells / (launch_ms / 1e3) / 1e9, 1)}}


def bench_paper_config(args, torch, fs, firegen):
    """The paper's vectorised-throughput setting: 64 envs of 64 x 64, 200
    steps, timed with the dense plan and with the autotuner's choice."""
    import numpy as np

    batch = firegen.landscape_batch(7, [(64, 64)] * 64)
    params = firegen.Params(veg=tuple(float(v) for v in firegen.veg_table(np.random.default_rng(7))))
    sim = fs.FireSim.from_batch(batch, params, seed=0)
    init = sim.states.clone()
    stream = torch.cuda.current_stream()
    T = 200
    out = {"workload": "64 envs x 64x64, 200 steps (the paper's vmap throughput setting)"}
    sim.set_plan(tile_rows=4, tile_width=256, temporal=1, skip_static=0, sparse=0, graph=1)
    ms, _ = timed_runs(torch, stream, sim, init, T, args.steps, 2)
    out["dense"] = {"ms_per_200_steps": round(ms, 4), "env_steps_per_s": 64 * T / (ms / 1e3)}
    sim.states.copy_(init)
    sim.t = 0
    sim.autotune(T_probe=T, allow_skip=True, allow_sparse=True)
    best = sim.plan()
    keys = ("tile_rows", "tile_width", "temporal", "skip_static", "sparse", "resident")
    sim.set_plan(**{k: best[k] for k in keys}, graph=1)
    ms, _ = timed_runs(torch, stream, sim, init, T, args.steps, 2)
    out["autotuned"] = {"plan": {k: best[k] for k in keys}, "ms_per_200_steps": round(ms, 4),
                        "env_steps_per_s": 64 * T / (ms / 1e3)}
    out["unit"] = "env-steps/s"
    out["note"] = ("context only: the paper quotes its peak on an NVIDIA A100 in a garbled form; "
                   "its literal reading is 2.5^16 = 2.3e6 env-steps/s")
    # the paper's throughput-versus-batch curve: 200 steps of n envs of 64 x 64, autotuned each
    sweep = []
    for n in (1, 4, 16, 64, 256, 1024, 4096) if args.paper_sweep else ():
        b = firegen.landscape_batch(7, [(64, 64)] * n)
        s2 = fs.FireSim.from_batch(b, params, seed=0)
        i2 = s2.states.clone()
        s2.autotune(T_probe=T, allow_skip=True, allow_sparse=True)
        p2 = s2.plan()
        s2.set_plan(**{k: p2[k] for k in keys}, graph=1)
        ms2, _ = timed_runs(torch, stream, s2, i2, T, max(2, args.steps), 1)
        sweep.append({"n_env": n, "plan": {k: p2[k] for k in keys}, "ms_per_200_steps": round(ms2, 4),
                      "env_steps_per_s": n * T / (ms2 / 1e3)})
        log("[bench] paper sweep %4d envs of 64x64: %s %.3f ms per 200 steps, %.3e env-steps/s"
            % (n, {k: p2[k] for k in keys if p2[k]}, ms2, n * T / (ms2 / 1e3)))
        del s2, i2, b
    if sweep:
        out["sweep"] = sweep
    log("[bench] paper setting 64 x 64^2: dense %.3f ms, autotuned %s %.3f ms per 200 steps"
        % (out["dense"]["ms_per_200_steps"], out["autotuned"]["plan"], ms))
    return out


def bench_uneven(args, torch, fs, firegen):
    """The uneven batch: 4096 envs with sides in {64, 128, 256, 512}, 300
    steps, one 5 x 5 suppression drop per env per step, in-kernel counts; the
    dense plan, the autotuner's one plan for the batch and its per-size-class
    plans."""
    batch, params, T, seed, act = firegen.workload_uneven()
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    acts = torch.from_numpy(act).cuda()
    init = sim.states.clone()
    stream = torch.cuda.current_stream()
    cells = float(batch.n_cells)

    def run(reps):
        for _ in range(reps):
            sim.states.copy_(init)
            sim.t = 0
            sim.step(T, actions=acts, counts=True)

    out = {"workload": "4096 envs, sides in {64,128,256,512} (%d cells), 300 steps, one 5x5 drop per "
                       "env per step, in-kernel counts" % int(cells), "unit": "cell-updates/s"}
    sim.set_plan(tile_rows=4, tile_width=256, temporal=1, skip_static=0, sparse=0, graph=1)
    run(1)
    torch.cuda.synchronize()
    with StepTimer(torch, stream) as tm:
        run(2)
    ms = tm.ms() / 2
    rate = cells * T / (ms / 1e3)
    out["dense"] = {"ms_per_pass": round(ms, 3), "value": rate,
                    "hbm_GBs_at_10B": round(STOCH_BYTES_PER_CELL * rate / 1e9, 1),
                    "hbm_frac_at_10B": round(STOCH_BYTES_PER_CELL * rate / 1e9 / HBM_PEAK_GBS, 4)}
    sim.states.copy_(init)
    sim.t = 0
    # both tuners probe 150 steps: long enough for the fires to reach the sizes
    # that decide between plans (a 50-step probe picks 256-wide tiles for the
    # 512^2 envs, which lose later in the run)
    keys = ("tile_rows", "tile_width", "temporal", "skip_static", "sparse", "resident")
    if args.tune:
        sim.autotune(T_probe=150, allow_skip=True, allow_sparse=True)
        best = sim.plan()
    else:  # the library's default tiled plan, which the tuner picks here (short profiles)
        best = dict(tile_rows=4, tile_width=64, temporal=1, skip_static=1, sparse=1, resident=0)
    sim.set_plan(**{k: best[k] for k in keys}, graph=1)
    run(1)
    torch.cuda.synchronize()
    with StepTimer(torch, stream) as tm:
        run(2)
    ms2 = tm.ms() / 2
    tag = "autotuned" if args.tune else "default_plan"
    out[tag] = {"plan": {k: best[k] for k in keys}, "ms_per_pass": round(ms2, 3),
                "value": cells * T / (ms2 / 1e3)}
    ms3 = float("nan")
    if args.tune:
        # one plan per size class (sides 64 / 128 / 256 / 512), each class tuned alone
        sim.states.copy_(init)
        sim.t = 0
        cls = sim.autotune_classes(T_probe=150, allow_skip=True, allow_sparse=True)
        run(1)
        torch.cuda.synchronize()
        with StepTimer(torch, stream) as tm:
            run(2)
        ms3 = tm.ms() / 2
        out["per_class"] = {"classes": [{"size_class": c["size_class"], "n_env": c["n_env"], "plan": c["plan"],
                                         "tuned_ms_per_step": round(c["ms_per_step"], 4)} for c in cls],
                            "ms_per_pass": round(ms3, 3), "value": cells * T / (ms3 / 1e3)}
    log("[bench] uneven: dense %.2f ms (%.3e cell-updates/s, %.0f GB/s at 10 B), %s %s %.2f ms, "
        "per-class %.2f ms" % (ms, rate, STOCH_BYTES_PER_CELL * rate / 1e9, tag, out[tag]["plan"], ms2, ms3))
    return out


def bench_rl(args, torch, fs, firegen):
    """RL air-tanker layer: 65536 envs of 20 x 20, 100 steps of random actions
    (agent move + water drop + fire step + reward + 5 x 5 observation), as one
    launch per step (the env resident in LDS) and as separate act / step /
    observation launches."""
    n = 65536
    batch = firegen.uniform_batch(20, 20, n_env=n, ignitions=())
    params = firegen.Params(p_base=0.45)
    sim = fs.FireSim.from_batch(batch, params, seed=0)
    sim.set_plan(tile_rows=4, tile_width=64, graph=0)
    steps = 100
    g = torch.Generator(device="cuda").manual_seed(0)
    acts = torch.randint(0, 32, (steps, n), dtype=torch.int32, device="cuda", generator=g)
    stream = torch.cuda.current_stream()
    ms = {}
    for single in (True, False):
        env = fs.RLEnv(sim, obs_radius=2, drop_radius=1, water_capacity=20, max_steps=1000,
                       single_launch=single)
        env.reset(episode=0)
        for i in range(5):
            env.step(acts[i])
        torch.cuda.synchronize()
        env.reset(episode=1)
        with StepTimer(torch, stream) as tm:
            for i in range(steps):
                env.step(acts[i])
        ms[single] = tm.ms()
    rate = n * steps / (ms[True] / 1e3)
    log("[bench] rl: %.3f ms per step of %d envs (one launch), %.3f ms (separate launches), %.3e env-steps/s"
        % (ms[True] / steps, n, ms[False] / steps, rate))
    return {"workload": "65536 envs x 20x20, 100 RL steps, random moves and valve, 5x5 observations",
            "value": rate, "unit": "env-steps/s", "ms_per_step": round(ms[True] / steps, 4),
            "cell_updates_per_s": rate * 400,
            "separate_launches": {"ms_per_step": round(ms[False] / steps, 4),
                                  "value": n * steps / (ms[False] / 1e3)}}


def bench_large(args, torch, fs, firegen):
    """8 envs of 2048 x 2048 with fractal terrain (0-2000 m), 11-class land
    cover and per-cell wind, 1000 steps: the dense plan (22 algorithmic bytes
    per cell-update) and the autotuner's choice."""
    batch, params, T, seed = firegen.workload_large()
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    init = sim.states.clone()
    stream = torch.cuda.current_stream()
    cells = float(batch.n_cells)
    bpc = STOCH_BYTES_PER_CELL + STOCH_WIND_CELL_BYTES

    def run():
        sim.states.copy_(init)
        sim.t = 0
        sim.step(T)

    out = {"workload": "8 envs x 2048x2048, fractal terrain 0-2000 m, 11-class land cover, per-cell "
                       "wind, 1000 steps", "unit": "cell-updates/s", "algorithmic_bytes_per_cell": bpc}
    sim.set_plan(tile_rows=4, tile_width=256, temporal=1, skip_static=0, sparse=0, graph=1)
    run()
    torch.cuda.synchronize()
    with StepTimer(torch, stream) as tm:
        run()
    ms = tm.ms()
    rate = cells * T / (ms / 1e3)
    out["dense"] = {"ms_per_pass": round(ms, 3), "value": rate,
                    "hbm_GBs_at_22B": round(bpc * rate / 1e9, 1),
                    "hbm_frac_at_22B": round(bpc * rate / 1e9 / HBM_PEAK_GBS, 4)}
    sim.states.copy_(init)
    sim.t = 0
    keys = ("tile_rows", "tile_width", "temporal", "skip_static", "sparse", "resident")
    if args.tune:
        # the whole run: the fires grow for most of the 1000 steps, and a short probe
        # from the initial fires ranks the plans by their cost on small fronts
        sim.autotune(T_probe=T, allow_skip=True, allow_sparse=True)
        best = sim.plan()
    else:  # the library's default tiled plan, which the tuner picks here (short profiles)
        best = dict(tile_rows=4, tile_width=64, temporal=1, skip_static=1, sparse=1, resident=0)
    sim.set_plan(**{k: best[k] for k in keys}, graph=1)
    run()
    torch.cuda.synchronize()
    with StepTimer(torch, stream) as tm:
        run()
    ms2 = tm.ms()
    tag = "autotuned" if args.tune else "default_plan"
    out[tag] = {"plan": {k: best[k] for k in keys}, "ms_per_pass": round(ms2, 3),
                "value": cells * T / (ms2 / 1e3)}
    log("[bench] large: dense %.2f ms (%.3e cell-updates/s, %.0f GB/s at 22 B), %s %s %.2f ms"
        % (ms, rate, bpc * rate / 1e9, tag, out[tag]["plan"], ms2))
    return out


def relaxed_case(args, torch, fs, firegen, batch, params, T, k, label, roofline):
    sim = fs.FireSim.from_batch(batch, params, seed=0)
    sim.step(T)   # target scar: a stochastic run at the known parameters
    Y = ((sim.states == firegen.BURNING) | (sim.states == firegen.BURNT)).to(torch.uint8)
    sim.set_plan(sparse=0)  # the dense adjoint: every tile, every step
    theta = fs.params_with_theta(sim.params, [params.p_base * 1.2, params.alpha_w1 * 1.2,
                                              params.alpha_w2 * 1.2, params.alpha_s * 1.2,
                                              params.alpha_gamma, params.p_continue, *params.veg])
    stream = torch.cuda.current_stream()
    wind = batch.wind_cell is not None

    def fwd_bwd(T, k, ws):
        U, B = sim.relaxed_init()
        sim.relaxed_fwd(theta, U, B, T, k, ws)
        loss, gU, _ = sim.relaxed_loss(U, Y, scale=1.0 / batch.n_env)
        return loss, gU, sim.relaxed_bwd(theta, gU, None, T, k, ws)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        reps = max(1, args.relaxed_reps)
        with StepTimer(torch, stream) as tm:
            for _ in range(reps):
                out = fn()
        return tm.ms() / reps, out

    ws = sim.relaxed_workspace(T, k)
    ms, (loss, _, grad) = timed(lambda: fwd_bwd(T, k, ws))   # dense adjoint
    cs = float(batch.n_cells) * T / (ms / 1e3)
    bpc = round(relaxed_bytes_per_cell_step(T, k, wind), 2)
    log("[bench] relaxed %s: %.2f ms per fwd+bwd, %.3e cell-steps/s (%.1f%% of HBM at %d B, %.1f%% at the "
        "fp64 state's %.1f B), loss %.4f" % (label, ms, cs, 100 * cs * RELAXED_ALG_BYTES / 1e9 / HBM_PEAK_GBS,
                                          RELAXED_ALG_BYTES, 100 * cs * bpc / 1e9 / HBM_PEAK_GBS, bpc,
                                          float(loss.mean())))
    out = {"value": cs, "unit": "cell-steps/s", "ms_per_fwd_bwd": round(ms, 3), "workload": label,
           "loss": round(float(loss.mean()), 6), "gradient_norm": float(grad.norm())}
    if roofline:
        out["hbm_frac_at_80B"] = round(cs * RELAXED_ALG_BYTES / 1e9 / HBM_PEAK_GBS, 4)
        out["fp64_state"] = {"bytes_per_cell_step": bpc, "achieved_GBs": round(cs * bpc / 1e9, 1),
                             "hbm_frac": round(cs * bpc / 1e9 / HBM_PEAK_GBS, 4)}
        # per kernel: every step checkpointed (no recompute); the difference
        # of T- and T/2-step calls removes the fixed costs, leaving T/2 launches
        half = T // 2
        ws1 = sim.relaxed_workspace(T, 1)
        launches = {}
        for name, T_ in (("full", T), ("half", half)):
            U0, B0 = sim.relaxed_init()
            t_f, _ = timed(lambda: sim.relaxed_fwd(theta, U0.clone(), B0.clone(), T_, 1, ws1))
            U, B = sim.relaxed_init()
            sim.relaxed_fwd(theta, U, B, T_, 1, ws1)
            _, gU, _ = sim.relaxed_loss(U, Y, scale=1.0 / batch.n_env)
            t_b, _ = timed(lambda: sim.relaxed_bwd(theta, gU, None, T_, 1, ws1))
            launches[name] = (t_f, t_b)
        # store-all: every state kept (checkpoint every step), so nothing is
        # recomputed; the method's count is then 56 B per cell-step (fwd 24 + adj 32)
        ms_sa, (_, _, grad_sa) = timed(lambda: fwd_bwd(T, 1, ws1))
        cs_sa = float(batch.n_cells) * T / (ms_sa / 1e3)
        out["store_all"] = {"ms_per_fwd_bwd": round(ms_sa, 3), "value": cs_sa,
                            "workspace_GB": round(ws1.numel() / 1e9, 1),
                            "hbm_frac_at_56B": round(cs_sa * 56 / 1e9 / HBM_PEAK_GBS, 4),
                            "grad_max_abs_diff_vs_recompute": float((grad_sa - grad).abs().max())}
        log("[bench] relaxed %s store-all (checkpoint every step): %.2f ms per fwd+bwd, %.3e cell-steps/s"
            % (label.split(":")[0], ms_sa, cs_sa))
        del ws1
        kern = {}
        w = RELAXED_WIND_BYTES if wind else 0
        for i, (kname, fp64_b, alg_b) in enumerate((("relaxed_fwd_kernel", RELAXED_FWD_BYTES + w,
                                                      RELAXED_ALG_FWD_BYTES + w),
                                                     ("relaxed_adj_kernel", RELAXED_ADJ_BYTES + w,
                                                      RELAXED_ALG_ADJ_BYTES + w))):
            us = (launches["full"][i] - launches["half"][i]) / (T - half) * 1e3
            kern[kname] = {"launch_us": round(us, 2), "bytes_per_cell": fp64_b,
                           "achieved_GBs": round(batch.n_cells * fp64_b / us / 1e3, 1),
                           "frac": round(batch.n_cells * fp64_b / us / 1e3 / HBM_PEAK_GBS, 4),
                           "frac_at_fp32_state_bytes": round(batch.n_cells * alg_b / us / 1e3 / HBM_PEAK_GBS, 4),
                           "fp32_state_bytes_per_cell": alg_b}
            log("[bench] relaxed %s %s: %.1f us per launch, %.0f GB/s at %d B (fp64 state)"
                % (label.split(":")[0], kname, us, kern[kname]["achieved_GBs"], fp64_b))
        out["kernels"] = kern
    else:
        out["note"] = "the whole working set fits the 256 MB Infinity Cache: not an HBM roofline configuration"
    if args.relaxed_sparse:
        # sparse adjoint (tiles beyond the reach of the initial fire skipped):
        # an effective rate, same gradient
        sim.set_plan(sparse=1)
        ms_sp, (_, _, grad_sp) = timed(lambda: fwd_bwd(T, k, ws))
        sim.set_plan(sparse=0)
        same = bool(torch.equal(grad_sp, grad))
        log("[bench] relaxed %s, sparse adjoint: %.2f ms (gradient %s)" % (label, ms_sp,
                                                                         "bit-identical" if same else "DIFFERS"))
        out["sparse_adjoint"] = {"ms_per_fwd_bwd": round(ms_sp, 3),
                                 "value": float(batch.n_cells) * T / (ms_sp / 1e3),
                                 "gradient_bit_identical": same,
                                 "note": "effective rate: adjoint tiles beyond the reach of the initial "
                                         "burning mass are skipped"}
    return out


def bench_relaxed(args, torch, fs, firegen):
    batch, params, T, k = firegen.workload_relaxed()
    small = relaxed_case(args, torch, fs, firegen, batch, params, T, k,
                         "relaxed128: 256 envs x 128x128, T=100, checkpoint every 10, fp64 state", False)
    del batch
    batch, params, T, k = firegen.workload_relaxed_large()
    large = relaxed_case(args, torch, fs, firegen, batch, params, T, k,
                         "relaxed2048: 1 env 2048x2048, per-cell wind, T=%d, checkpoint every %d, "
                         "fp64 state" % (T, k), True)
    adj = large["kernels"]["relaxed_adj_kernel"]
    large["roofline"] = {"bound": "hbm", "achieved": round(large["value"] * RELAXED_ALG_BYTES / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": large["hbm_frac_at_80B"],
                         "bytes_per_cell_step": RELAXED_ALG_BYTES,
                         "dominant_kernel": "relaxed_adj_kernel", "dominant_launch_us": adj["launch_us"],
                         "note": "whole fwd+bwd (forward, recompute, adjoint, loss) at the method's 80 B per "
                                 "cell-step (fp32 state); the adjoint is VALU-bound, see the kernel profiles"}
    return {"relaxed128": small, "relaxed2048": large}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tile-rows", type=int, default=4)
    ap.add_argument("--tile-width", type=int, default=256)
    ap.add_argument("--skip-static", type=int, default=0)
    ap.add_argument("--sparse", type=int, default=0)
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--relaxed-reps", type=int, default=2)
    ap.add_argument("--relaxed-sparse", type=int, default=1, help="also time the sparse adjoint")
    ap.add_argument("--no-stochastic", action="store_true",
                    help="skip the timed headline run (profiling of the other parts)")
    ap.add_argument("--no-relaxed", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the front-skipping plans")
    ap.add_argument("--no-dense-front", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the paper-setting, RL, uneven and large objects")
    ap.add_argument("--extras", default="paper,rl,uneven,large",
                    help="comma-separated subset of the extra objects to run")
    ap.add_argument("--tune", type=int, default=1,
                    help="0: time the uneven and large workloads under the default tiled plan instead of "
                         "autotuning them (short profiles)")
    ap.add_argument("--paper-sweep", type=int, default=1,
                    help="0: time the paper setting without the 1-4096-env sweep (shorter profiles)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(envs shard across GPUs with no communication; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import firegen
    import paper_2512_06102_amd as fs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    fs.lib()
    st = bench_stochastic(args, torch, fs, firegen)
    product = bench_product_plan(args, torch, fs, st) if st["value"] is not None else None
    variants = None if args.no_variants else bench_variants(args, torch, fs, st)
    dense = None if args.no_dense_front else bench_dense_front(args, torch, fs, firegen, st)
    st.pop("sim")
    extras = set() if args.no_extra else set(args.extras.split(","))
    paper = bench_paper_config(args, torch, fs, firegen) if "paper" in extras else None
    rl = bench_rl(args, torch, fs, firegen) if "rl" in extras else None
    uneven = bench_uneven(args, torch, fs, firegen) if "uneven" in extras else None
    large = bench_large(args, torch, fs, firegen) if "large" in extras else None
    relaxed = None if args.no_relaxed else bench_relaxed(args, torch, fs, firegen)
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    probe = stream_probe(torch, fs)
    cpu = None if args.no_cpu else cpu_baseline(st["batch"], st["params"], st["T"], st["seed"])
    batch = st["batch"]
    out = {"metric": "cell-updates/s stochastic step + relaxed fwd+bwd cell-steps/s, % HBM peak",
           "value": st["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(st["ms"], 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch256: 1024 envs x 256x256 cells (uint8 state), 200 steps, "
                                  "11-class land cover, fractal terrain, per-env wind, 1-5 ignitions",
                      "n_env": int(batch.n_env), "H": 256, "W": 256, "T": st["T"], "plan": st["plan"],
                      "burning_cell_steps": st["burning"]},
           "roofline": st["roof"], "product_plan": product, "variants": variants, "dense_front": dense, "relaxed": relaxed,
           "paper_setting": paper, "rl": rl, "uneven": uneven, "large": large, "stream_probe": probe,
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
