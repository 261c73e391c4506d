"""Relaxed (mean-field) fire spread, its soft-IoU loss and its adjoint, in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's deterministic "raw-probabilities" routine (section 3, Eqs. 5-10)
carries per cell the probabilities (p_un, p_burn, p_bd) and updates

    newly  = p_un * p_ignite,  continuing = p_burn * p_continue,
    p_burn' = newly + continuing,   p_un' = p_un - newly,
    p_bd'   = p_bd + p_burn (1 - p_continue).

Here U = p_un, B = p_burn; p_bd = 1 - U - B never feeds back, so it is not
carried.  The ignition term takes b(u) = B(u) in the product form

    p_ignite(v) = 1 - prod_k (1 - q_k(v) B(u_k)),
    q_k(v)      = 1 - exp(-gamma(v) phi(u_k, k)),   u_k = v - D_k,

which is Eq. 4 exactly whenever B is 0/1 (prod_k exp(-gamma phi_k b_k) =
exp(-gamma lambda)).  phi follows Eqs. 1-3 with the wind and slope exponent
written as in the paper: kappa_wind = exp(a_w1 V) exp(a_w2 V (cos(ang_k -
Theta) - 1)), kappa_slope = exp(a_s S).

The loss is one minus the soft intersection-over-union of the soft scar
S = 1 - U_T (burnable cells) with a binary target scar Y, averaged over envs.

The adjoint is reverse-mode differentiation of exactly these formulas.  q does
not change over time, so its adjoint is summed over all steps first and then
taken through q -> (phi, gamma) -> parameters once.

Parameter vector (THETA_NAMES): p_base, alpha_w1, alpha_w2, alpha_s,
alpha_gamma, p_continue, veg[0..10].
"""
from __future__ import annotations

import math

import numpy as np

# direction k: from source u to target v = u + (di, dj); angle k pi/4
# counter-clockwise from east; rows grow southward.
DIRS = ((0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1))
THETA_NAMES = ("p_base", "alpha_w1", "alpha_w2", "alpha_s", "alpha_gamma", "p_continue") + \
    tuple("veg%d" % c for c in range(11))
N_THETA = len(THETA_NAMES)


def theta_from_params(p) -> np.ndarray:
    return np.array([p.p_base, p.alpha_w1, p.alpha_w2, p.alpha_s, p.alpha_gamma, p.p_continue,
                     *p.veg], np.float64)


def shift_from_source(A: np.ndarray, k: int, fill: float = 0.0) -> np.ndarray:
    """out[v] = A[v - D_k] (the source of direction k), `fill` off the grid."""
    di, dj = DIRS[k]
    H, W = A.shape
    out = np.full_like(A, fill)
    si0, si1 = max(0, -di), min(H, H - di)
    sj0, sj1 = max(0, -dj), min(W, W - dj)
    out[si0 + di:si1 + di, sj0 + dj:sj1 + dj] = A[si0:si1, sj0:sj1]
    return out


def scatter_to_source(C: np.ndarray, k: int) -> np.ndarray:
    """Adjoint of shift_from_source: out[u] = C[u + D_k] (0 off the grid)."""
    di, dj = DIRS[k]
    H, W = C.shape
    out = np.zeros_like(C)
    si0, si1 = max(0, -di), min(H, H - di)
    sj0, sj1 = max(0, -dj), min(W, W - dj)
    out[si0:si1, sj0:sj1] = C[si0 + di:si1 + di, sj0 + dj:sj1 + dj]
    return out


class Env64:
    """One env's static inputs in float64 arrays of shape [H, W]."""

    def __init__(self, cls, den, elev, wind, cell_size):
        self.cls = np.asarray(cls).astype(np.int64)
        self.den = np.asarray(den, np.float64)
        self.E = np.asarray(elev, np.float64)
        H, W = self.cls.shape
        w = np.asarray(wind, np.float64)
        if w.ndim == 1:  # per env (V, Vx, Vy)
            self.V = np.full((H, W), w[0])
            self.Vx = np.full((H, W), w[1])
            self.Vy = np.full((H, W), w[2])
        else:  # [3, H, W]
            self.V, self.Vx, self.Vy = w[0], w[1], w[2]
        self.cs = float(cell_size)
        self.valid = [shift_from_source(np.ones((H, W)), k) > 0 for k in range(8)]


def from_batch(batch, e, cell_size) -> Env64:
    H, W = int(batch.H[e]), int(batch.W[e])
    sl = batch.env_slice(e)
    if batch.wind_cell is not None:
        wind = batch.wind_cell[:, sl].reshape(3, H, W)
    else:
        wind = batch.wind_env[e]
    return Env64(batch.cls[sl].reshape(H, W), batch.den[sl].reshape(H, W),
                 batch.elev[sl].reshape(H, W), wind, cell_size)


def edge_terms(env: Env64, theta: np.ndarray) -> dict:
    """Per direction k, on the target grid: phi(u_k, k) (Eqs. 1-3) and
    q_k(v) = 1 - exp(-gamma(v) phi), plus the factors the adjoint needs."""
    p_base, a_w1, a_w2, a_s, a_gamma = theta[0], theta[1], theta[2], theta[3], theta[4]
    veg = theta[6:17]
    g = (1.0 + veg[env.cls]) * (1.0 + env.den)
    gamma = a_gamma * g
    out = {"g": g, "gamma": gamma, "phi": [], "q": [], "kappa": [], "g_src": [], "V_src": [],
           "cosdev": [], "S": []}
    for k in range(8):
        ang = k * math.pi / 4.0
        ca = math.cos(ang) if k % 2 == 1 else float(round(math.cos(ang)))
        sa = math.sin(ang) if k % 2 == 1 else float(round(math.sin(ang)))
        dist = env.cs * (math.sqrt(2.0) if k % 2 == 1 else 1.0)
        V = shift_from_source(env.V, k)
        Vx = shift_from_source(env.Vx, k)
        Vy = shift_from_source(env.Vy, k)
        Eu = shift_from_source(env.E, k)
        gu = shift_from_source(g, k)
        # V cos(ang_k - Theta) - V, with V cos Theta = Vx, V sin Theta = Vy
        cosdev = (ca * Vx + sa * Vy) - V
        S = (env.E - Eu) / dist
        kappa_wind = np.exp(a_w1 * V) * np.exp(a_w2 * cosdev)
        kappa_slope = np.exp(a_s * S)
        kappa = kappa_wind * kappa_slope
        phi = p_base * gu * kappa
        q = np.where(env.valid[k], -np.expm1(-gamma * phi), 0.0)
        out["phi"].append(np.where(env.valid[k], phi, 0.0))
        out["q"].append(q)
        out["kappa"].append(kappa)
        out["g_src"].append(gu)
        out["V_src"].append(V)
        out["cosdev"].append(cosdev)
        out["S"].append(S)
    return out


def ignite_prob(q: list, B: np.ndarray) -> np.ndarray:
    """p_ignite = 1 - prod_k (1 - q_k B(u_k))."""
    prod = np.ones_like(B)
    for k in range(8):
        prod = prod * (1.0 - q[k] * shift_from_source(B, k))
    return 1.0 - prod


def step(U, B, q, p_continue):
    """One relaxed step (Eqs. 5-10 with the product-form ignition)."""
    P = ignite_prob(q, B)
    newly = U * P
    return U - newly, newly + p_continue * B


def initial_state(batch, e) -> tuple:
    """U = 1, B = 0 on burnable cells; U = 0, B = 1 on ignition cells;
    U = B = 0 on unburnable cells."""
    H, W = int(batch.H[e]), int(batch.W[e])
    cls = batch.cls[batch.env_slice(e)].reshape(H, W)
    burnable = ((batch.unburnable_mask >> cls.astype(np.int64)) & 1) == 0
    U = burnable.astype(np.float64)
    B = np.zeros((H, W))
    for row in batch.ignitions[batch.ignitions[:, 0] == e]:
        i, j = int(row[1]), int(row[2])
        if burnable[i, j]:
            U[i, j], B[i, j] = 0.0, 1.0
    return U, B, burnable


def forward(env: Env64, theta, U0, B0, T) -> tuple:
    """Return the lists U[0..T], B[0..T] and the edge terms."""
    terms = edge_terms(env, theta)
    Us, Bs = [U0.astype(np.float64)], [B0.astype(np.float64)]
    for _ in range(T):
        U, B = step(Us[-1], Bs[-1], terms["q"], theta[5])
        Us.append(U)
        Bs.append(B)
    return Us, Bs, terms


def soft_iou_loss(U_T, Y, burnable) -> tuple:
    """Per env: L = 1 - I/D, S = (1 - U_T) on burnable cells, I = sum S Y,
    D = sum S + sum Y - I.  Returns (L, dL/dU_T)."""
    S = np.where(burnable, 1.0 - U_T, 0.0)
    Yf = Y.astype(np.float64)
    I = float(np.sum(S * Yf))
    D = float(np.sum(S) + np.sum(Yf) - I)
    if D <= 0.0:
        return 0.0, np.zeros_like(U_T)
    L = 1.0 - I / D
    dL_dS = -(Yf * D - I * (1.0 - Yf)) / (D * D)
    return L, np.where(burnable, -dL_dS, 0.0)


def adjoint(env: Env64, theta, Us, Bs, terms, gU_T, gB_T=None) -> np.ndarray:
    """Reverse-mode gradient of a scalar loss with dL/dU_T = gU_T (and dL/dB_T
    = gB_T, default 0) with respect to THETA."""
    T = len(Us) - 1
    p_c = theta[5]
    q = terms["q"]
    gU = gU_T.astype(np.float64).copy()
    gB = np.zeros_like(gU) if gB_T is None else gB_T.astype(np.float64).copy()
    Qbar = [np.zeros_like(gU) for _ in range(8)]
    grad = np.zeros(N_THETA)
    for t in range(T - 1, -1, -1):
        U, B = Us[t], Bs[t]
        Bsrc = [shift_from_source(B, k) for k in range(8)]
        fac = [1.0 - q[k] * Bsrc[k] for k in range(8)]
        # exclusive products prod_{j != k} fac_j by prefix and suffix products
        pre = [np.ones_like(U)]
        for k in range(8):
            pre.append(pre[-1] * fac[k])
        suf = [np.ones_like(U)] * 9
        for k in range(7, -1, -1):
            suf[k] = suf[k + 1] * fac[k]
        P = 1.0 - pre[8]
        nbar = gB - gU                   # adjoint of newly = U P
        gU_new = gU + nbar * P
        Pbar = nbar * U
        grad[5] += float(np.sum(gB * B))  # B' = newly + p_c B
        gB_new = p_c * gB
        for k in range(8):
            excl = pre[k] * suf[k + 1]
            gB_new = gB_new + scatter_to_source(Pbar * q[k] * excl, k)
            Qbar[k] += Pbar * Bsrc[k] * excl
        gU, gB = gU_new, gB_new
    # through q_k = 1 - exp(-gamma phi_k)
    p_base, a_gamma = theta[0], theta[4]
    g = terms["g"]
    gamma = terms["gamma"]
    gbar = np.zeros_like(g)       # adjoint of the fuel term g per cell
    gamma_bar = np.zeros_like(g)
    for k in range(8):
        ybar = Qbar[k] * (1.0 - q[k])          # dq/dy = exp(-y) = 1 - q
        phi = terms["phi"][k]
        phibar = ybar * gamma
        gamma_bar += ybar * phi
        kappa = np.where(env.valid[k], terms["kappa"][k], 0.0)
        grad[0] += float(np.sum(phibar * terms["g_src"][k] * kappa))
        xbar = phibar * phi                       # phi = p_base g_u exp(x)
        grad[1] += float(np.sum(xbar * terms["V_src"][k]))
        grad[2] += float(np.sum(xbar * terms["cosdev"][k]))
        grad[3] += float(np.sum(xbar * np.where(env.valid[k], terms["S"][k], 0.0)))
        gbar += scatter_to_source(phibar * p_base * kappa, k)
    grad[4] += float(np.sum(gamma_bar * g))
    gbar += gamma_bar * a_gamma
    contrib = gbar * (1.0 + env.den)             # g = (1 + veg[c]) (1 + den)
    grad[6:17] += np.bincount(env.cls.ravel(), weights=contrib.ravel(), minlength=11)[:11]
    return grad


def loss_and_grad(batch, theta, T, Y_list, env_ids=None, cell_size=30.0) -> tuple:
    """Mean soft-IoU loss over the given envs after T relaxed steps, its
    gradient, and the final U_T per env."""
    theta = np.asarray(theta, np.float64)
    env_ids = range(batch.n_env) if env_ids is None else env_ids
    env_ids = list(env_ids)
    n = len(env_ids)
    L = 0.0
    grad = np.zeros(N_THETA)
    finals = []
    for idx, e in enumerate(env_ids):
        env = from_batch(batch, e, cell_size)
        U0, B0, burnable = initial_state(batch, e)
        Us, Bs, terms = forward(env, theta, U0, B0, T)
        Le, gU = soft_iou_loss(Us[-1], Y_list[idx], burnable)
        L += Le / n
        grad += adjoint(env, theta, Us, Bs, terms, gU / n)
        finals.append((Us[-1], Bs[-1]))
    return L, grad, finals


def loss_only(batch, theta, T, Y_list, env_ids=None, cell_size=30.0) -> float:
    theta = np.asarray(theta, np.float64)
    env_ids = list(range(batch.n_env) if env_ids is None else env_ids)
    n = len(env_ids)
    L = 0.0
    for idx, e in enumerate(env_ids):
        env = from_batch(batch, e, cell_size)
        U0, B0, burnable = initial_state(batch, e)
        Us, Bs, _ = forward(env, theta, U0, B0, T)
        L += soft_iou_loss(Us[-1], Y_list[idx], burnable)[0] / n
    return L
