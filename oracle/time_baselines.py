"""CPU baselines of the oracle (test infrastructure; never used by the library).

Times the plain oracle, as written, on the host cores: the stochastic step on
the 64 x 64 single-grid workload and on 16 envs of the 1024 x 256^2 batch on
one core; the whole 1024 x 256^2 batch and the 4096-env uneven batch (with
drops) with one env per thread on every core; and the fp64 relaxed forward +
adjoint on 8 envs of the 256 x 128^2 workload on one core and with one env
per process.  Prints a markdown report (progress lines go to stderr).

Usage: python oracle/time_baselines.py [--threads N] > report.md
"""
from __future__ import annotations

import argparse
import os
import platform
import subprocess
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import firegen  # noqa: E402
import oracle  # noqa: E402
from oracle import relaxed64  # noqa: E402


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, check=False).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def stoch(batch, params, T, seed, threads, actions=None):
    sim = oracle.Sim(batch, params, seed=seed)
    t0 = time.perf_counter()
    sim.step(T, actions=actions, counts=True, threads=threads)
    dt = time.perf_counter() - t0
    return float(batch.n_cells) * T / dt, dt


def relaxed_env(args):
    batch, params, T, e, Y = args
    theta = relaxed64.theta_from_params(params)
    t0 = time.perf_counter()
    relaxed64.loss_and_grad(batch, theta, T, [Y], env_ids=[e])
    return time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=min(16, len(os.sched_getaffinity(0))))
    a = ap.parse_args()
    n = a.threads
    rows = []

    b1, p1, T1, s1 = firegen.workload_single64()
    r, dt = stoch(b1, p1, T1, s1, 1)
    rows.append(("64x64 single grid, 100 steps", "1", r, "cell-updates/s", dt))
    log("[baseline] single64 done")

    b2, p2, T2, s2 = firegen.workload_batch256()
    sub = b2.subset(range(16))
    r, dt = stoch(sub, p2, T2, s2, 1)
    rows.append(("16 envs of 1024 x 256^2, 200 steps", "1", r, "cell-updates/s", dt))
    log("[baseline] batch256 subset done")
    r, dt = stoch(b2, p2, T2, s2, n)
    rows.append(("1024 x 256^2, 200 steps", str(n), r, "cell-updates/s", dt))
    log("[baseline] batch256 all cores done")
    del b2, sub

    b3, p3, T3, s3, act = firegen.workload_uneven()
    log("[baseline] uneven workload generated")
    r, dt = stoch(b3, p3, T3, s3, n, actions=act)
    rows.append(("4096 uneven envs, 300 steps, drops", str(n), r, "cell-updates/s", dt))
    log("[baseline] uneven all cores done")
    del b3, act

    b4, p4, T4, k4 = firegen.workload_relaxed()
    sub = b4.subset(range(8))
    ref = oracle.Sim(sub, p4, seed=0)
    ref.step(T4, threads=min(n, 8))
    Y = ((ref.states == firegen.BURNING) | (ref.states == firegen.BURNT))
    jobs = [(sub, p4, T4, e, sub.env_view(Y, e)) for e in range(8)]
    t0 = time.perf_counter()
    relaxed_env(jobs[0])
    dt = time.perf_counter() - t0
    rows.append(("relaxed fp64 fwd+adjoint, 1 env of 256 x 128^2, T=100", "1",
                 128 * 128 * T4 / dt, "cell-steps/s", dt))
    workers = min(n, 8)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers) as ex:
        list(ex.map(relaxed_env, jobs))
    dt = time.perf_counter() - t0
    rows.append(("relaxed fp64 fwd+adjoint, 8 envs of 256 x 128^2, T=100", str(workers),
                 8 * 128 * 128 * T4 / dt, "cell-steps/s", dt))
    log("[baseline] relaxed done")

    print("# CPU oracle baselines\n")
    print("Host: %s, %d threads used at most (os reports %d CPUs)." % (cpu_model(), n, os.cpu_count()))
    print("The oracle as written (plain C, one env per thread; numpy fp64 for the relaxed path, "
          "one env per process).\n")
    print("| workload | threads | rate | unit | seconds |")
    print("|---|---|---|---|---|")
    for w, th, r, u, dt in rows:
        print("| %s | %s | %.3e | %s | %.1f |" % (w, th, r, u, dt))


if __name__ == "__main__":
    main()
