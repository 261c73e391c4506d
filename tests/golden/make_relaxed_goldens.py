"""Write the fp64 oracle's losses and parameter gradients of the full relaxed
workloads to tests/golden/*.json (the GPU tests compare the whole 17-entry
gradient with them).  Calls only the oracle and the input generators.

    python tests/golden/make_relaxed_goldens.py [relaxed128] [relaxed2048_T<T> ...]

Setups (the benchmark's):
  relaxed128        256 envs of 128 x 128, T = 100, checkpoints every 10.
  relaxed2048_T100  1 env of 2048 x 2048 with per-cell wind, T = 100.
  relaxed2048_T<T>  the same env at T = 200, 300, 400 or 500 (the large
                    workload's horizon); the fp64 forward keeps every state:
                    about 7.4 GB of RAM per 100 steps.
Target scar Y: BURNING or BURNT after a stochastic oracle run of T steps with
the workload's parameters and Philox seed 0.  The gradient is taken at
p_base, alpha_w1, alpha_w2, alpha_s times 1.2 (the others unchanged), on the
fp32-rounded parameter vector the GPU kernels receive; the loss is the soft
IoU, averaged over the envs.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import firegen  # noqa: E402
import oracle  # noqa: E402
from oracle import relaxed64  # noqa: E402


def perturbed(params):
    return params.replace(p_base=params.p_base * 1.2, alpha_w1=params.alpha_w1 * 1.2,
                          alpha_w2=params.alpha_w2 * 1.2, alpha_s=params.alpha_s * 1.2)


def target(batch, params, T):
    ref = oracle.Sim(batch, params, seed=0)
    ref.step(T, threads=min(16, os.cpu_count() or 1))
    return ((ref.states == firegen.BURNING) | (ref.states == firegen.BURNT)).astype(np.uint8)


def golden(name, batch, params, T, k):
    t0 = time.time()
    Y = target(batch, params, T)
    p = perturbed(params)
    theta32 = relaxed64.theta_from_params(p).astype(np.float32).astype(np.float64)
    Ys = [batch.env_view(Y, e).astype(bool) for e in range(batch.n_env)]
    L, g, finals = relaxed64.loss_and_grad(batch, theta32, T, Ys, cell_size=p.cell_size)
    out = {"workload": name, "T": T, "ckpt_every": k, "n_env": int(batch.n_env),
           "theta": [float(x) for x in theta32], "theta_names": list(relaxed64.THETA_NAMES),
           "loss": float(L), "grad": [float(x) for x in g],
           "target_burnt_cells": int(Y.sum()),
           "U_T_sum": float(sum(float(f[0].sum()) for f in finals)),
           "B_T_sum": float(sum(float(f[1].sum()) for f in finals)),
           "seconds": round(time.time() - t0, 1),
           "made_by": "tests/golden/make_relaxed_goldens.py " + name}
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "loss %.9f |g| %.6e in %.0f s" % (L, float(np.linalg.norm(g)), out["seconds"]), flush=True)


def main(names):
    for name in names:
        if name == "relaxed128":
            batch, params, T, k = firegen.workload_relaxed()
            golden(name, batch, params, T, k)
        elif name.startswith("relaxed2048_T"):
            batch, params, _, k = firegen.workload_relaxed_large()
            golden(name, batch, params, int(name.split("_T")[1]), k)
        else:
            raise SystemExit("unknown golden " + name)


if __name__ == "__main__":
    main(sys.argv[1:] or ["relaxed128", "relaxed2048_T100"])
