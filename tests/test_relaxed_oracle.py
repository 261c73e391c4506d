"""Pins of the fp64 relaxed oracle (forward, soft-IoU loss, adjoint).

* adjoint versus fp64 central finite differences of the forward + loss;
* adjoint versus torch autograd (fp64, CPU) through the same forward;
* one relaxed step from a binary state equals the exact one-step marginal of
  the stochastic process (exact enumeration, Eq. 4);
* with q in {0, 1} and p_continue = 0 the relaxed step is the deterministic CA
  (Chebyshev square);
* probability mass: U non-increasing, U + B <= 1, unburnable cells fixed.
"""
import math

import numpy as np
import pytest
import torch

import firegen
from oracle import enumerate_exact, relaxed64


def _small_batch(seed=1, sizes=((16, 16),), per_cell_wind=False):
    return firegen.landscape_batch(seed, list(sizes), per_cell_wind=per_cell_wind, elev_max=60.0)


def _params(seed=0):
    rng = np.random.default_rng(seed)
    return firegen.Params(p_base=0.5, alpha_w1=0.05, alpha_w2=0.12, alpha_s=3.0, alpha_gamma=1.1,
                          p_continue=0.55, veg=tuple(float(v) for v in firegen.veg_table(rng)))


def _target(batch, T, seed):
    """A binary scar: a random blob around each env's ignitions."""
    rng = np.random.default_rng(seed)
    Ys = []
    for e in range(batch.n_env):
        H, W = int(batch.H[e]), int(batch.W[e])
        ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        Y = np.zeros((H, W), bool)
        for row in batch.ignitions[batch.ignitions[:, 0] == e]:
            r = rng.uniform(2, 2 + T / 2)
            Y |= (ii - row[1]) ** 2 + (jj - row[2]) ** 2 <= r * r
        Ys.append(Y)
    return Ys


@pytest.mark.parametrize("per_cell_wind", [False, True])
@pytest.mark.parametrize("form", ["product", "exp"])
@pytest.mark.parametrize("loss", ["iou", "bce"])
def test_adjoint_matches_central_differences(per_cell_wind, form, loss):
    b = _small_batch(3, ((16, 16), (12, 20)), per_cell_wind)
    prm = _params(1)
    T = 12
    Y = _target(b, T, 2)
    theta = relaxed64.theta_from_params(prm)
    kw = dict(form=form, loss=loss, **({"pool": 4} if loss == "bce" else {}))
    L, grad, _ = relaxed64.loss_and_grad(b, theta, T, Y, **kw)
    assert 0 < L < (1 if loss == "iou" else 20)
    fd = np.zeros_like(grad)
    for i in range(theta.size):
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (relaxed64.loss_only(b, tp, T, Y, **kw) - relaxed64.loss_only(b, tm, T, Y, **kw)) / (2 * h)
    scale = np.max(np.abs(fd))
    assert scale > 0
    for i in range(theta.size):
        assert abs(grad[i] - fd[i]) <= 1e-6 * scale + 1e-6 * abs(fd[i]), \
            (relaxed64.THETA_NAMES[i], grad[i], fd[i])
    for c in firegen.UNBURNABLE_CLASSES:
        assert grad[6 + c] == 0.0


def _torch_forward_loss(env, theta_t, U0, B0, T, Y, burnable, form="product", loss="iou"):
    """The relaxed forward in torch (fp64), to differentiate with autograd."""
    p_base, a_w1, a_w2, a_s, a_g, p_c = (theta_t[i] for i in range(6))
    veg = theta_t[6:17]
    cls = torch.from_numpy(env.cls)
    den = torch.from_numpy(env.den)
    g = (1 + veg[cls]) * (1 + den)
    gamma = a_g * g
    H, W = env.cls.shape
    q, phis = [], []
    for k, (di, dj) in enumerate(relaxed64.DIRS):
        pad = torch.nn.functional.pad

        def src(A, fill=0.0):
            Ap = pad(A[None, None], (1, 1, 1, 1), value=fill)[0, 0]
            return Ap[1 - di:1 - di + H, 1 - dj:1 - dj + W]
        V = src(torch.from_numpy(env.V))
        Vx = src(torch.from_numpy(env.Vx))
        Vy = src(torch.from_numpy(env.Vy))
        ang = k * math.pi / 4
        ca, sa = (math.cos(ang), math.sin(ang)) if k % 2 else (round(math.cos(ang)), round(math.sin(ang)))
        dist = env.cs * (math.sqrt(2) if k % 2 else 1.0)
        S = (torch.from_numpy(env.E) - src(torch.from_numpy(env.E))) / dist
        phi = p_base * src(g) * torch.exp(a_w1 * V + a_w2 * ((ca * Vx + sa * Vy) - V) + a_s * S)
        valid = torch.from_numpy(env.valid[k])
        q.append(torch.where(valid, -torch.expm1(-gamma * phi), torch.zeros_like(phi)))
        phis.append(torch.where(valid, phi, torch.zeros_like(phi)))
    U = torch.from_numpy(U0)
    B = torch.from_numpy(B0)
    for _ in range(T):
        Bp = torch.nn.functional.pad(B[None, None], (1, 1, 1, 1))[0, 0]
        if form == "product":
            prod = torch.ones_like(U)
            for k, (di, dj) in enumerate(relaxed64.DIRS):
                prod = prod * (1 - q[k] * Bp[1 - di:1 - di + H, 1 - dj:1 - dj + W])
            P = 1 - prod
        else:
            lam = torch.zeros_like(U)
            for k, (di, dj) in enumerate(relaxed64.DIRS):
                lam = lam + phis[k] * Bp[1 - di:1 - di + H, 1 - dj:1 - dj + W]
            P = -torch.expm1(-gamma * lam)
        newly = U * P
        U, B = U - newly, newly + p_c * B
    Sg = torch.where(torch.from_numpy(burnable), 1 - U, torch.zeros_like(U))
    Yt = torch.from_numpy(Y.astype(np.float64))
    if loss == "iou":
        I = (Sg * Yt).sum()
        D = Sg.sum() + Yt.sum() - I
        return 1 - I / D
    Sc = torch.clamp(Sg, 1e-6, 1 - 1e-6)
    bce = -(Yt * torch.log(Sc) + (1 - Yt) * torch.log(1 - Sc)).mean()
    pool = torch.nn.functional.avg_pool2d
    pS = pool(Sg[None, None], 4, ceil_mode=True, count_include_pad=False)
    pY = pool(Yt[None, None], 4, ceil_mode=True, count_include_pad=False)
    return bce + ((pS - pY) ** 2).mean()


@pytest.mark.parametrize("form,loss", [("product", "iou"), ("exp", "iou"), ("product", "bce"),
                                       ("exp", "bce")])
def test_adjoint_matches_torch_autograd(form, loss):
    b = _small_batch(5, ((20, 14),))
    prm = _params(2)
    T = 15
    Y = _target(b, T, 3)
    theta = relaxed64.theta_from_params(prm)
    kw = dict(form=form, loss=loss, **({"pool": 4} if loss == "bce" else {}))
    L, grad, _ = relaxed64.loss_and_grad(b, theta, T, Y, **kw)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    env = relaxed64.from_batch(b, 0, 30.0)
    U0, B0, burnable = relaxed64.initial_state(b, 0)
    Lt = _torch_forward_loss(env, th, U0, B0, T, Y[0], burnable, form, loss)
    Lt.backward()
    assert abs(Lt.item() - L) < 1e-13
    assert np.allclose(th.grad.numpy(), grad, rtol=1e-10, atol=1e-14)


def test_one_step_from_binary_state_is_exact_marginal():
    """B(v) after one relaxed step from a binary state equals P(F_1(v) =
    BURNING), U(v) equals P(F_1(v) = FLAMMABLE) (exact enumeration of Eq. 4)."""
    rng = np.random.default_rng(7)
    prm = _params(3)
    b = firegen.uniform_batch(3, 4, wind=(6.0, 1.1), ignitions=())
    b.cls[:] = rng.choice([0, 1, 2, 3, 8], 12).astype(np.uint8)
    b.den[:] = rng.uniform(-0.3, 0.3, 12).astype(np.float32)
    b.elev[:] = rng.uniform(0, 10, 12).astype(np.float32)
    F0 = np.full((3, 4), firegen.FLAMMABLE)
    F0[0, 1] = F0[2, 2] = F0[1, 3] = firegen.BURNING
    theta = relaxed64.theta_from_params(prm)
    env = relaxed64.from_batch(b, 0, 30.0)
    exact = enumerate_exact.exact_marginals(env, theta, F0, 1)
    U0 = (F0 == firegen.FLAMMABLE).astype(np.float64)
    B0 = (F0 == firegen.BURNING).astype(np.float64)
    for form in relaxed64.FORMS:
        Us, Bs, _ = relaxed64.forward(env, theta, U0, B0, 1, form)
        assert np.allclose(Us[1], exact[1, :, :, firegen.FLAMMABLE], atol=1e-14), form
        assert np.allclose(Bs[1], exact[1, :, :, firegen.BURNING], atol=1e-14), form


def test_saturated_relaxed_step_is_deterministic_ca():
    """q = 1 (p_base large) and p_continue = 0: B_t is the Chebyshev ring at
    distance t and U is zero inside it, exactly."""
    b = firegen.uniform_batch(15, 15)
    prm = firegen.Params(p_base=64.0, p_continue=0.0)
    theta = relaxed64.theta_from_params(prm)
    env = relaxed64.from_batch(b, 0, 30.0)
    U0, B0, _ = relaxed64.initial_state(b, 0)
    Us, Bs, _ = relaxed64.forward(env, theta, U0, B0, 9)
    ii, jj = np.meshgrid(np.arange(15), np.arange(15), indexing="ij")
    d = np.maximum(abs(ii - 7), abs(jj - 7))
    for t in range(10):
        assert np.array_equal(Bs[t], (d == t).astype(float))
        assert np.array_equal(Us[t], (d > t).astype(float))


def test_mass_invariants():
    b = _small_batch(9, ((24, 24),))
    prm = _params(4)
    theta = relaxed64.theta_from_params(prm)
    env = relaxed64.from_batch(b, 0, 30.0)
    U0, B0, burnable = relaxed64.initial_state(b, 0)
    Us, Bs, _ = relaxed64.forward(env, theta, U0, B0, 30)
    for t in range(30):
        assert np.all(Us[t + 1] <= Us[t] + 1e-15)
        assert np.all(Us[t + 1] + Bs[t + 1] <= 1 + 1e-12)
        assert np.all(Us[t + 1][~burnable] == 0) and np.all(Bs[t + 1][~burnable] == 0)


@pytest.mark.parametrize("form", ["product", "exp"])
def test_adjoint_matches_central_differences_slope_angle(form):
    """The slope-angle variant (S = atan(rise / run)): the adjoint against
    fp64 central differences, on steep terrain where atan departs from its
    argument."""
    b = firegen.landscape_batch(4, ((14, 18),), elev_max=400.0)
    prm = _params(7)
    T = 10
    Y = _target(b, T, 5)
    theta = relaxed64.theta_from_params(prm)
    kw = dict(form=form, slope_mode=1)
    L, grad, _ = relaxed64.loss_and_grad(b, theta, T, Y, **kw)
    L0, _, _ = relaxed64.loss_and_grad(b, theta, T, Y, form=form)
    assert L != L0   # the mode changes the model
    fd = np.zeros_like(grad)
    for i in range(theta.size):
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (relaxed64.loss_only(b, tp, T, Y, **kw) - relaxed64.loss_only(b, tm, T, Y, **kw)) / (2 * h)
    scale = np.max(np.abs(fd))
    for i in range(theta.size):
        assert abs(grad[i] - fd[i]) <= 1e-6 * scale + 1e-6 * abs(fd[i]), (relaxed64.THETA_NAMES[i], grad[i], fd[i])


@pytest.mark.parametrize("per_cell", [False, True])
def test_wind_series_adjoint(per_cell):
    """Time-varying wind in the relaxed step: a constant series reproduces the
    static run (loss and gradient), and with a varying series the adjoint
    (parameter chain applied step by step) matches fp64 central differences."""
    b = _small_batch(6, ((14, 16), (10, 12)), per_cell)
    prm = _params(9)
    T = 9
    Y = _target(b, T, 7)
    theta = relaxed64.theta_from_params(prm)
    if per_cell:
        const = {"wind_cell_series": np.repeat(b.wind_cell[None], T, 0)}
    else:
        const = {"wind_env_series": np.repeat(b.wind_env[None], T, 0)}
    L0, g0, _ = relaxed64.loss_and_grad(b, theta, T, Y)
    L1, g1, _ = relaxed64.loss_and_grad(b, theta, T, Y, **const)
    assert abs(L1 - L0) < 1e-14 and np.allclose(g1, g0, rtol=1e-12, atol=1e-15)
    ser = firegen.wind_series(3, b, T, per_cell=per_cell, speed_step=1.5, turn_step=0.4)
    kw = {"wind_cell_series" if per_cell else "wind_env_series": ser}
    L, grad, _ = relaxed64.loss_and_grad(b, theta, T, Y, **kw)
    assert abs(L - L0) > 1e-6   # the series matters
    fd = np.zeros_like(grad)
    for i in range(theta.size):
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (relaxed64.loss_only(b, tp, T, Y, **kw) - relaxed64.loss_only(b, tm, T, Y, **kw)) / (2 * h)
    scale = np.max(np.abs(fd))
    for i in range(theta.size):
        assert abs(grad[i] - fd[i]) <= 1e-6 * scale + 1e-6 * abs(fd[i]), (relaxed64.THETA_NAMES[i], grad[i], fd[i])


@pytest.mark.parametrize("form", ["product", "exp"])
def test_far_field_adjoint_overflow_keeps_the_light_cone_gradient(form):
    """A 3 x 1000 strip burning from its west end with nearly saturated q:
    ahead of the fire (B = 0, U = 1) the adjoint state grows by at least
    p_c + sum_k q_k per step backward, past the fp64 range within 450 steps.
    It only ever meets B = 0, so the gradient must stay finite and equal that
    of the same strip cut at 460 columns, where no cell lies beyond the reach
    of the burning mass (light cone: after T steps it has spread T columns)."""
    T = 450
    params = firegen.Params(p_base=8.0, alpha_gamma=1.0, alpha_w1=0.0, alpha_w2=0.0, alpha_s=0.0,
                            p_continue=0.5)
    theta = relaxed64.theta_from_params(params)
    grads = []
    for W in (1000, 460):
        batch = firegen.uniform_batch(3, W, ignitions=[(0, 1, 0)])
        env = relaxed64.from_batch(batch, 0, params.cell_size)
        U0, B0, burnable = relaxed64.initial_state(batch, 0)
        Us, Bs, terms = relaxed64.forward(env, theta, U0, B0, T, form)
        Y = np.zeros((3, W), bool)
        Y[:, :300] = True
        L, gU = relaxed64.soft_iou_loss(Us[-1], Y, burnable)
        if W == 1000:
            # the regime: an interior cell of the middle row gains more than
            # 10^(308/T) per step, so its adjoint passes 1e308 within T steps
            gain = params.p_continue + sum(float(terms["q"][k][1, 700]) for k in range(8))
            assert T * math.log10(gain) > 320
            # nothing burns beyond column T
            assert np.all(Bs[-1][:, T + 1:] == 0.0) and np.all(Us[-1][:, T + 1:] == 1.0)
        grads.append((L, relaxed64.adjoint(env, theta, Us, Bs, terms, gU, form=form)))
    (L_full, g_full), (L_cut, g_cut) = grads
    assert np.all(np.isfinite(g_full))
    assert abs(L_full - L_cut) <= 1e-12
    assert np.allclose(g_full, g_cut, rtol=1e-9, atol=1e-12 * np.max(np.abs(g_cut)))
