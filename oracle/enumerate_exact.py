"""Exact law of the stochastic fire-spread process on tiny grids (float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Given the fire state F_t, the paper's stochastic update (section 3,
"Stochastic update") moves every cell independently: a FLAMMABLE cell ignites
with p_ignite(v) = 1 - exp(-gamma(v) lambda(v)), lambda = sum over burning
neighbours of phi(u, D_{u->v}) (Eq. 4, phi from Eqs. 1-3); a BURNING cell
burns out with probability 1 - p_continue; UNBURNABLE and BURNT cells stay.
So F_t is a Markov chain, and its full distribution can be propagated exactly
on a handful of cells.  Configurations are coded two bits per cell (the state
code), and each step expands every configuration into all its successors.
"""
from __future__ import annotations

import numpy as np

from . import relaxed64

UNBURNABLE, FLAMMABLE, BURNING, BURNT = 0, 1, 2, 3


def _decode(codes: np.ndarray, n: int) -> np.ndarray:
    shifts = (2 * np.arange(n, dtype=np.int64))[None, :]
    return ((codes[:, None] >> shifts) & 3).astype(np.int8)


def exact_marginals(env: relaxed64.Env64, theta, F0: np.ndarray, T: int,
                    max_configs: int = 50_000_000) -> np.ndarray:
    """P(F_t(v) = s) for t = 0..T, every cell v and state s: [T+1, H, W, 4]."""
    theta = np.asarray(theta, np.float64)
    H, W = F0.shape
    n = H * W
    if n > 31:
        raise ValueError("grid too large for exact enumeration")
    terms = relaxed64.edge_terms(env, theta)
    phi = np.stack([terms["phi"][k].ravel() for k in range(8)])        # [8, n]
    gamma = terms["gamma"].ravel()                                     # [n]
    src = np.full((8, n), -1, np.int64)
    for k, (di, dj) in enumerate(relaxed64.DIRS):
        for i in range(H):
            for j in range(W):
                ui, uj = i - di, j - dj
                if 0 <= ui < H and 0 <= uj < W:
                    src[k, i * W + j] = ui * W + uj
    p_c = theta[5]
    code0 = int(sum(int(F0.ravel()[v]) << (2 * v) for v in range(n)))
    codes = np.array([code0], np.int64)
    probs = np.array([1.0])
    out = np.zeros((T + 1, n, 4))
    out[0, np.arange(n), F0.ravel()] = 1.0
    for t in range(T):
        S = _decode(codes, n)                                           # [M, n]
        burning = (S == BURNING).astype(np.float64)
        lam = np.zeros(S.shape)
        for k in range(8):
            valid = src[k] >= 0
            b = np.zeros(S.shape)
            b[:, valid] = burning[:, src[k, valid]]
            lam += b * phi[k][None, :]
        p_ign = -np.expm1(-gamma[None, :] * lam)
        adv = np.where(S == FLAMMABLE, p_ign, np.where(S == BURNING, 1.0 - p_c, 0.0))
        cur_code = codes.copy()
        cur_w = probs.copy()
        row = np.arange(codes.size)
        for v in range(n):
            a = adv[row, v]
            split = (a > 0.0) & (a < 1.0)
            full = a >= 1.0
            step_bit = np.int64(1) << np.int64(2 * v)
            moved_code = cur_code[split] + step_bit
            moved_w = cur_w[split] * a[split]
            moved_row = row[split]
            cur_w = np.where(split, cur_w * (1.0 - a), cur_w)
            cur_code = np.where(full, cur_code + step_bit, cur_code)
            cur_code = np.concatenate([cur_code, moved_code])
            cur_w = np.concatenate([cur_w, moved_w])
            row = np.concatenate([row, moved_row])
            if cur_code.size > max_configs:
                raise MemoryError("enumeration exceeds max_configs")
        uniq, inv = np.unique(cur_code, return_inverse=True)
        codes = uniq
        probs = np.bincount(inv, weights=cur_w, minlength=uniq.size)
        keep = probs > 0.0
        codes, probs = codes[keep], probs[keep]
        S = _decode(codes, n)
        for s in range(4):
            out[t + 1, :, s] = ((S == s) * probs[:, None]).sum(axis=0)
    return out.reshape(T + 1, H, W, 4)
