"""Benchmark of the batched fire-spread step on one MI355X.

One benchmark step = one pass of the hot path over the batch: the 1024 envs
of 256 x 256 cells are reset to their initial fire state and advanced 200
stochastic steps (one sim_step call, in-kernel burning counts).  `value` is
cell-updates per second over the timed steps (1024 * 65536 * 200 per step).
The relaxed forward + adjoint (256 envs of 128 x 128, 100 steps, checkpoints
every 10) is timed after it and reported in its own object.

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
STOCH_BYTES_PER_CELL = 10      # state r/w 2 B + fuel 4 B + elevation 4 B per cell-update
# relaxed, fp64 state: forward 40 B (U,B r/w 32 + fuel, elevation 8); adjoint
# 61 B (U,B 16, adjoint r/w 32, fuel, elevation, density 12, class 1); the
# forward is recomputed from checkpoints (40 B) and every 10th state stored (1.6 B)
RELAXED_BYTES_PER_CELL_STEP = 40 + 40 + 61 + 1.6
KERNEL_SOURCES = ("paper_2512_06102_amd/csrc/stoch.hip", "paper_2512_06102_amd/csrc/devmath.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stoch_step_batch256_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(plan_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source and plan."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash() or rec.get("plan") != plan_key:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(batch, params, T, seed):
    """The oracle, as written, on a bounded sample of the same workload."""
    import oracle

    threads = min(16, len(os.sched_getaffinity(0)))
    n_env = min(batch.n_env, 24 * threads)
    sub = batch.subset(range(n_env))
    sim = oracle.Sim(sub, params, seed=seed)
    t0 = time.perf_counter()
    sim.step(T, counts=True, threads=threads)
    dt = time.perf_counter() - t0
    cells = float(sub.n_cells) * T
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "%d of the 1024 envs (256x256), %d steps from the initial state, "
                      "one env per thread, %.1f s" % (n_env, T, dt)}


def bench_stochastic(args, torch, fs, firegen):
    batch, params, T, seed = firegen.workload_batch256()
    log("[bench] workload generated: %d envs, %d cells" % (batch.n_env, batch.n_cells))
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    plan = {"tile_rows": args.tile_rows, "tile_width": args.tile_width,
            "skip_static": args.skip_static, "sparse": args.sparse, "graph": args.graph}
    sim.set_plan(**plan)
    init = sim.states.clone()
    stream = torch.cuda.current_stream()

    def one_step():
        sim.states.copy_(init)
        sim.t = 0
        return sim.step(T, counts=True)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # kernel-only events around the launches of the last timed step
    k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        sim.states.copy_(init)
        sim.t = 0
        if i == args.steps - 1:
            k0.record(stream)
        sim.step(T, counts=True)
        if i == args.steps - 1:
            k1.record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = start.elapsed_time(stop) / args.steps
    launch_ms = k0.elapsed_time(k1) / T       # average step-kernel duration (fill/set kernels included)
    cells = float(batch.n_cells)
    value = cells * T / (ms / 1e3)
    achieved = STOCH_BYTES_PER_CELL * cells / (launch_ms / 1e3) / 1e9
    plan_key = "tile_rows=%d,tile_width=%d,skip_static=%d,sparse=%d" % (
        sim.plan()["tile_rows"], sim.plan()["tile_width"], args.skip_static, args.sparse)
    traffic = stored_traffic(plan_key)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "stoch_step_kernel", "launch_ms": round(launch_ms, 5),
            "algorithmic_bytes_per_launch": STOCH_BYTES_PER_CELL * int(cells)}
    log("[bench] stochastic: %.3f ms/step, %.3e cell-updates/s, kernel %.4f ms = %.0f GB/s (wall %.2fs)"
        % (ms, value, launch_ms, achieved, wall))
    counts = one_step().cpu()
    return batch, params, T, seed, value, ms, roof, plan, int(counts.sum())


def bench_relaxed(args, torch, fs, firegen):
    batch, params, T, k = firegen.workload_relaxed()
    sim = fs.FireSim.from_batch(batch, params, seed=0)
    sim.step(T)   # target scar: a stochastic run at the known parameters
    Y = ((sim.states == firegen.BURNING) | (sim.states == firegen.BURNT)).to(torch.uint8)
    theta = fs.params_with_theta(sim.params, [params.p_base * 1.2, params.alpha_w1 * 1.2,
                                              params.alpha_w2 * 1.2, params.alpha_s * 1.2,
                                              params.alpha_gamma, params.p_continue, *params.veg])
    ws = sim.relaxed_workspace(T, k)

    def fwd_bwd():
        U, B = sim.relaxed_init()
        sim.relaxed_fwd(theta, U, B, T, k, ws)
        loss, gU = sim.relaxed_loss(U, Y, scale=1.0 / batch.n_env)
        return loss, sim.relaxed_bwd(theta, gU, None, T, k, ws)

    fwd_bwd()
    torch.cuda.synchronize()
    reps = max(1, args.relaxed_reps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        loss, grad = fwd_bwd()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    cs = float(batch.n_cells) * T / (ms / 1e3)
    gbs = cs * RELAXED_BYTES_PER_CELL_STEP / 1e9
    log("[bench] relaxed: %.2f ms per fwd+bwd, %.3e cell-steps/s, loss %.4f"
        % (ms, cs, float(loss.mean())))
    return {"value": cs, "unit": "cell-steps/s", "ms_per_fwd_bwd": round(ms, 3),
            "workload": "relaxed128: 256 envs x 128x128, T=100, checkpoint every 10, fp64 state",
            "algorithmic_bytes_per_cell_step": RELAXED_BYTES_PER_CELL_STEP,
            "achieved_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "loss": round(float(loss.mean()), 6)}


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
    ap.add_argument("--relaxed-reps", type=int, default=3)
    ap.add_argument("--no-relaxed", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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
    batch, params, T, seed, value, ms, roof, plan, burning = bench_stochastic(args, torch, fs, firegen)
    relaxed = None if args.no_relaxed else bench_relaxed(args, torch, fs, firegen)
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    cpu = None if args.no_cpu else cpu_baseline(batch, params, T, seed)
    out = {"metric": "cell-updates/s stochastic step + relaxed fwd+bwd cell-steps/s, % HBM peak",
           "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch256: 1024 envs x 256x256 cells (uint8 state), 200 steps, "
                                  "11-class land cover, fractal terrain, per-env wind, 1-5 ignitions",
                      "n_env": int(batch.n_env), "H": 256, "W": 256, "T": T, "plan": plan,
                      "burning_cell_steps": burning},
           "roofline": roof, "relaxed": relaxed, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
