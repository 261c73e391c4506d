"""Relaxed (mean-field) fire spread, its calibration losses and its adjoint, in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's deterministic "raw-probabilities" routine (section 3, Eqs. 5-10)
carries per cell the probabilities (p_un, p_burn, p_bd) and updates

    newly  = p_un * p_ignite,  continuing = p_burn * p_continue,
    p_burn' = newly + continuing,   p_un' = p_un - newly,
    p_bd'   = p_bd + p_burn (1 - p_continue).

Here U = p_un, B = p_burn; p_bd = 1 - U - B never feeds back, so it is not
carried.  Two readings of p_ignite with b(u) = B(u):

  form "product":  p_ignite(v) = 1 - prod_k (1 - q_k(v) B(u_k)),
                   q_k(v) = 1 - exp(-gamma(v) phi(u_k, k)),  u_k = v - D_k;
  form "exp":      p_ignite(v) = 1 - exp(-gamma(v) sum_k B(u_k) phi(u_k, k))
                   (Eq. 4 with the burning indicator replaced by B).

Both equal Eq. 4 when B is 0/1.  phi follows Eqs. 1-3 with the wind and slope
factors written as in the paper: kappa_wind = exp(a_w1 V) exp(a_w2 V
(cos(ang_k - Theta) - 1)), kappa_slope = exp(a_s S).

Losses of the final state, S = 1 - U_T on burnable cells (0 elsewhere) against
a binary target scar Y, averaged over envs:
  "iou":  1 - sum S Y / (sum S + sum Y - sum S Y);
  "bce":  binary cross-entropy of clip(S, eps, 1 - eps) against Y (mean over
          cells) plus w times the mean squared error between k x k average
          pools of S and Y (the paper's calibration loss, section 4).

The adjoint is reverse-mode differentiation of exactly these formulas.  The
per-edge phi and the per-cell gamma do not change over time, so their
adjoints are summed over all steps first and then taken to the parameters
once.

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
FORMS = ("product", "exp")


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

    def __init__(self, cls, den, elev, wind, cell_size, slope_mode=0, wind_series=None):
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
        self.slope_mode = int(slope_mode)  # 0: S = rise / run; 1: S = atan(rise / run)
        # time-varying wind: [S, 3] (per env) or [S, 3, H, W] (per cell), row t for step t
        self.wind_series = None if wind_series is None else np.asarray(wind_series, np.float64)
        self.valid = [shift_from_source(np.ones((H, W)), k) > 0 for k in range(8)]


def from_batch(batch, e, cell_size, slope_mode=0, wind_env_series=None, wind_cell_series=None) -> Env64:
    H, W = int(batch.H[e]), int(batch.W[e])
    sl = batch.env_slice(e)
    if batch.wind_cell is not None:
        wind = batch.wind_cell[:, sl].reshape(3, H, W)
    else:
        wind = batch.wind_env[e]
    series = None
    if wind_env_series is not None:
        series = np.asarray(wind_env_series)[:, e, :]
    elif wind_cell_series is not None:
        series = np.asarray(wind_cell_series)[:, :, sl].reshape(-1, 3, H, W)
    return Env64(batch.cls[sl].reshape(H, W), batch.den[sl].reshape(H, W),
                 batch.elev[sl].reshape(H, W), wind, cell_size, slope_mode, series)


def env_at_step(env: Env64, t: int) -> Env64:
    """The env with the wind of step t of its series (itself without one)."""
    if env.wind_series is None:
        return env
    out = Env64.__new__(Env64)
    out.__dict__.update(env.__dict__)
    w = env.wind_series[t]
    H, W = env.cls.shape
    if w.ndim == 1:
        out.V, out.Vx, out.Vy = (np.full((H, W), w[i]) for i in range(3))
    else:
        out.V, out.Vx, out.Vy = w[0], w[1], w[2]
    out.wind_series = None
    return out


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
        if env.slope_mode:
            S = np.arctan(S)  # the slope angle (radians)
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


def ignite_prob(terms: dict, B: np.ndarray, form: str = "product") -> np.ndarray:
    """p_ignite of every cell from the soft burning mass B."""
    if form == "product":
        prod = np.ones_like(B)
        for k in range(8):
            prod = prod * (1.0 - terms["q"][k] * shift_from_source(B, k))
        return 1.0 - prod
    if form == "exp":
        lam = np.zeros_like(B)
        for k in range(8):
            lam = lam + terms["phi"][k] * shift_from_source(B, k)
        return -np.expm1(-terms["gamma"] * lam)
    raise ValueError(form)


def step(U, B, terms, p_continue, form="product"):
    """One relaxed step (Eqs. 5-10)."""
    P = ignite_prob(terms, B, form)
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


def forward(env: Env64, theta, U0, B0, T, form="product") -> tuple:
    """Return the lists U[0..T], B[0..T] and the edge terms (one dict, or a
    list of per-step dicts when the wind varies with time)."""
    if env.wind_series is None:
        terms = edge_terms(env, theta)
        per_step = [terms] * T
    else:
        per_step = [edge_terms(env_at_step(env, t), theta) for t in range(T)]
        terms = per_step
    Us, Bs = [U0.astype(np.float64)], [B0.astype(np.float64)]
    for t in range(T):
        U, B = step(Us[-1], Bs[-1], per_step[t], theta[5], form)
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


def _pool(A, k):
    """Mean over the k x k blocks of A (blocks at the far edges may be smaller)."""
    H, W = A.shape
    nb_r, nb_c = -(-H // k), -(-W // k)
    out = np.zeros((nb_r, nb_c))
    cnt = np.zeros((nb_r, nb_c))
    ii, jj = np.meshgrid(np.arange(H) // k, np.arange(W) // k, indexing="ij")
    np.add.at(out, (ii, jj), A)
    np.add.at(cnt, (ii, jj), 1.0)
    return out / cnt, cnt, (ii, jj)


def bce_pool_loss(U_T, Y, burnable, pool=8, mse_weight=1.0, eps=1e-6) -> tuple:
    """BCE of clip(S, eps, 1-eps) against Y over all cells plus mse_weight x
    MSE of the pool x pool block means of S and Y.  Returns (L, dL/dU_T)."""
    S = np.where(burnable, 1.0 - U_T, 0.0)
    Yf = Y.astype(np.float64)
    n = S.size
    Sc = np.clip(S, eps, 1.0 - eps)
    bce = -np.sum(Yf * np.log(Sc) + (1.0 - Yf) * np.log(1.0 - Sc)) / n
    inside = (S > eps) & (S < 1.0 - eps)
    dbce_dS = np.where(inside, (-(Yf / Sc) + (1.0 - Yf) / (1.0 - Sc)) / n, 0.0)
    pS, cnt, idx = _pool(S, pool)
    pY, _, _ = _pool(Yf, pool)
    m = pS.size
    mse = np.sum((pS - pY) ** 2) / m
    dmse_dpS = 2.0 * (pS - pY) / m
    dmse_dS = (dmse_dpS / cnt)[idx]
    dL_dS = dbce_dS + mse_weight * dmse_dS
    return bce + mse_weight * mse, np.where(burnable, -dL_dS, 0.0)


def loss_fn(kind, U_T, Y, burnable, **kw):
    if kind == "iou":
        return soft_iou_loss(U_T, Y, burnable)
    if kind == "bce":
        return bce_pool_loss(U_T, Y, burnable, **kw)
    raise ValueError(kind)


def _param_chain(env: Env64, theta, terms, phibar, gamma_bar) -> np.ndarray:
    """Gradient from the adjoints of phi_k (per edge) and gamma (per cell)
    through phi_k = p_base g(u) kappa_k and gamma = alpha_gamma g(v)."""
    grad = np.zeros(N_THETA)
    p_base, a_gamma = theta[0], theta[4]
    phi_k = terms["phi"]
    g = terms["g"]
    gbar = np.zeros_like(g)       # adjoint of the fuel term g per cell
    for k in range(8):
        kappa = np.where(env.valid[k], terms["kappa"][k], 0.0)
        grad[0] += float(np.sum(phibar[k] * terms["g_src"][k] * kappa))
        xbar = phibar[k] * phi_k[k]                  # phi = p_base g_u exp(x)
        grad[1] += float(np.sum(xbar * terms["V_src"][k]))
        grad[2] += float(np.sum(xbar * terms["cosdev"][k]))
        grad[3] += float(np.sum(xbar * np.where(env.valid[k], terms["S"][k], 0.0)))
        gbar += scatter_to_source(phibar[k] * p_base * kappa, k)
    grad[4] += float(np.sum(gamma_bar * g))
    gbar += gamma_bar * a_gamma
    contrib = gbar * (1.0 + env.den)             # g = (1 + veg[c]) (1 + den)
    grad[6:17] += np.bincount(env.cls.ravel(), weights=contrib.ravel(), minlength=11)[:11]
    return grad


def adjoint(env: Env64, theta, Us, Bs, terms, gU_T, gB_T=None, form="product") -> np.ndarray:
    """Reverse-mode gradient of a scalar loss with dL/dU_T = gU_T (and dL/dB_T
    = gB_T, default 0) with respect to THETA.  With per-step edge terms (a
    wind series) the parameter chain is applied step by step.

    Every gradient term carries a factor B: of the source (qbar = Pbar B(u)
    prod_{w != u}(1 - q B(w)), phibar = lambdabar B(u)) or of the target
    (the p_continue term Bbar' B).  Where that factor is 0 the term is 0.  It
    is evaluated so: far ahead of the fire (B = 0, U = 1) the adjoint state
    grows by about p_c + sum_k q_k per step backward and can pass the fp64
    range, and inf x 0 would otherwise make the sum NaN."""
    with np.errstate(over="ignore", invalid="ignore"):
        return _adjoint(env, theta, Us, Bs, terms, gU_T, gB_T, form)


def _adjoint(env, theta, Us, Bs, terms, gU_T, gB_T, form):
    T = len(Us) - 1
    p_c = theta[5]
    per_step = isinstance(terms, list)
    gU = gU_T.astype(np.float64).copy()
    gB = np.zeros_like(gU) if gB_T is None else gB_T.astype(np.float64).copy()
    phibar = [np.zeros_like(gU) for _ in range(8)]   # summed over time (static terms)
    gamma_bar = np.zeros_like(gU)
    grad = np.zeros(N_THETA)
    for t in range(T - 1, -1, -1):
        tt = terms[t] if per_step else terms
        q, phi_k, gamma = tt["q"], tt["phi"], tt["gamma"]
        if per_step:
            phibar = [np.zeros_like(gU) for _ in range(8)]
            gamma_bar = np.zeros_like(gU)
        U, B = Us[t], Bs[t]
        Bsrc = [shift_from_source(B, k) for k in range(8)]
        gB_new = p_c * gB
        if form == "product":
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
            Pbar = nbar * U
            for k in range(8):
                excl = pre[k] * suf[k + 1]
                gB_new = gB_new + scatter_to_source(Pbar * q[k] * excl, k)
                # qbar dq/dy, y = gamma phi; 0 where the source has no burning mass
                ybar = np.where(Bsrc[k] == 0.0, 0.0, Pbar * Bsrc[k] * excl * (1.0 - q[k]))
                phibar[k] += ybar * gamma
                gamma_bar += ybar * phi_k[k]
        else:
            lam = np.zeros_like(U)
            for k in range(8):
                lam = lam + phi_k[k] * Bsrc[k]
            P = -np.expm1(-gamma * lam)
            nbar = gB - gU
            Pbar = nbar * U
            lbar = Pbar * gamma * (1.0 - P)               # dP/dlambda = gamma exp(-gamma lambda)
            gamma_bar += np.where(lam == 0.0, 0.0, Pbar * lam * (1.0 - P))
            for k in range(8):
                gB_new = gB_new + scatter_to_source(lbar * phi_k[k], k)
                phibar[k] += np.where(Bsrc[k] == 0.0, 0.0, lbar * Bsrc[k])
        grad[5] += float(np.sum(np.where(B == 0.0, 0.0, gB * B)))  # B' = newly + p_c B
        if per_step:
            grad += _param_chain(env, theta, tt, phibar, gamma_bar)
        gU, gB = gU + nbar * P, gB_new
    if not per_step:
        grad += _param_chain(env, theta, terms, phibar, gamma_bar)
    return grad


def loss_and_grad(batch, theta, T, Y_list, env_ids=None, cell_size=30.0, form="product",
                  loss="iou", slope_mode=0, wind_env_series=None, wind_cell_series=None,
                  **loss_kw) -> tuple:
    """Mean loss over the given envs after T relaxed steps, its gradient,
    and the final (U_T, B_T) per env."""
    theta = np.asarray(theta, np.float64)
    env_ids = list(range(batch.n_env) if env_ids is None else env_ids)
    n = len(env_ids)
    L = 0.0
    grad = np.zeros(N_THETA)
    finals = []
    for idx, e in enumerate(env_ids):
        env = from_batch(batch, e, cell_size, slope_mode, wind_env_series, wind_cell_series)
        U0, B0, burnable = initial_state(batch, e)
        Us, Bs, terms = forward(env, theta, U0, B0, T, form)
        Le, gU = loss_fn(loss, Us[-1], Y_list[idx], burnable, **loss_kw)
        L += Le / n
        grad += adjoint(env, theta, Us, Bs, terms, gU / n, form=form)
        finals.append((Us[-1], Bs[-1]))
    return L, grad, finals


def loss_only(batch, theta, T, Y_list, env_ids=None, cell_size=30.0, form="product", loss="iou",
              slope_mode=0, wind_env_series=None, wind_cell_series=None, **loss_kw) -> float:
    theta = np.asarray(theta, np.float64)
    env_ids = list(range(batch.n_env) if env_ids is None else env_ids)
    n = len(env_ids)
    L = 0.0
    for idx, e in enumerate(env_ids):
        env = from_batch(batch, e, cell_size, slope_mode, wind_env_series, wind_cell_series)
        U0, B0, burnable = initial_state(batch, e)
        Us, Bs, _ = forward(env, theta, U0, B0, T, form)
        L += loss_fn(loss, Us[-1], Y_list[idx], burnable, **loss_kw)[0] / n
    return L
