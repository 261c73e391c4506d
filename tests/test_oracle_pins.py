"""Pins of the stochastic CPU oracle against what the model and mathematics fix.

None of these compare the oracle with itself: each checks it against a
published generator (rocRAND's Philox, Random123's known answers), the
fp64 exp, a closed form the paper's Eq. 4 gives by hand, a geometric fact
(the p=1 Chebyshev square), an invariant, or exact enumeration of the
Markov chain.
"""
import ctypes
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import firegen
import oracle
from oracle import enumerate_exact, relaxed64

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- Philox ---
# Known-answer vectors published with Random123 (Salmon et al., SC'11) for
# philox4x32 with 10 rounds: (counter, key) -> output.
PHILOX_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,want", PHILOX_KAT)
def test_philox_known_answers(ctr, key, want):
    assert tuple(int(x) for x in oracle.philox4x32_10(ctr, key)) == want


def _rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    out = os.path.join(tempfile.mkdtemp(), "librocrand_probe.so")
    subprocess.check_call([hipcc, "-O2", "-fPIC", "-shared", "-o", out,
                           os.path.join(HERE, "rocrand_philox_probe.cpp")])
    L = ctypes.CDLL(out)
    L.rocrand_philox_blocks.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_long]
    return L


def test_philox_matches_rocrand_on_random_counters():
    L = _rocrand_probe()
    rng = np.random.default_rng(11)
    n = 1 << 16
    ctr = rng.integers(0, 2**32, (n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, (n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[:256, 1:] = 0      # also the counter layout the model uses: (n>>2, t, env, 0)
    ctr[:256, 3] = 0
    want = np.zeros_like(ctr)
    L.rocrand_philox_blocks(ctr.ctypes.data, key.ctypes.data, want.ctypes.data, n)
    got = oracle.philox_blocks(ctr, key)
    assert np.array_equal(got, want)


# ---------------------------------------------------------------- exp_c ---
@pytest.mark.parametrize("negative", [False, True])
def test_exp_c_exhaustive_within_2ulp(negative):
    """Every fp32 with |x| in [2^-149, 87] (88 for x>0) against fp64 exp."""
    hi = 87.0 if negative else 88.0
    err, worst = oracle.exp_c_sweep(1e-45, hi, negative, threads=os.cpu_count() or 8)
    assert err <= 2.0, (err, worst)


def test_exp_c_special_values():
    x = np.array([0.0, -0.0, -87.0, -87.00001, -100.0, -np.inf, 88.0, 88.5, 1e30, np.inf],
                 np.float32)
    y = oracle.exp_c(x)
    assert y[0] == 1.0 and y[1] == 1.0
    assert y[2] > 0 and y[3] == 0.0 and y[4] == 0.0 and y[5] == 0.0
    assert y[6] == y[7] == y[8] == y[9] == oracle.exp_c(np.array([88.0], np.float32))[0]
    assert np.isfinite(y[6])


def test_philox_uniform_is_24bit_and_below_one():
    """The draw u = (word >> 8) 2^-24 is exact and < 1 for every word."""
    words = np.array([0, 255, 256, 0xffffffff, 0x80000000], np.uint64)
    u = (words >> 8).astype(np.float32) * np.float32(2.0 ** -24)
    assert u[0] == 0.0 and u[1] == 0.0 and u[2] == np.float32(2.0 ** -24)
    assert u[3] == np.float32(1.0 - 2.0 ** -24) and u[3] < 1.0 and u[4] == 0.5


# ------------------------------------------------- Eq. 4 closed forms ------
def _one_cell_batch(burning_dirs, *, V=0.0, theta=0.0, slope_rise=None, den=0.0, cls=firegen.GRASS):
    """3x3 env with the centre FLAMMABLE and the sources of the listed
    directions k BURNING (source of k is centre - D_k)."""
    b = firegen.uniform_batch(3, 3, cls=cls, den=den, wind=(V, theta), ignitions=())
    st = np.full(9, firegen.FLAMMABLE, np.uint8)
    for k in burning_dirs:
        di, dj = relaxed64.DIRS[k]
        st[(1 - di) * 3 + (1 - dj)] = firegen.BURNING
    if slope_rise is not None:
        b.elev[:] = slope_rise.ravel()
    return b, st


def test_textbook_n_neighbours_flat_no_wind():
    """g = 1, V = 0, flat: p = 1 - exp(-n p_base alpha_gamma) (Eq. 4)."""
    params = firegen.Params(p_base=0.58, alpha_gamma=1.0)
    for n in range(1, 9):
        b, st = _one_cell_batch(range(n))
        sim = oracle.Sim(b, params)
        p = sim.cell_prob(0, 1, 1, st)
        want = 1.0 - math.exp(-n * 0.58)
        assert abs(p - want) <= 4 * 2.0 ** -24, (n, p, want)


def test_wind_blows_toward_theta():
    """Wind toward east (Theta = 0): a burning west neighbour spreads east with
    kappa_wind = exp(a_w1 V); an east neighbour spreading west gets
    exp(a_w1 V) exp(-2 a_w2 V); a south neighbour spreading north gets
    exp(a_w1 V) exp(-a_w2 V) (Eq. 1, angle 0 = east, counter-clockwise)."""
    prm = firegen.Params(alpha_w1=0.045, alpha_w2=0.131, p_base=0.3)
    V = 7.0
    cases = {0: 0.045 * V, 4: 0.045 * V - 2 * 0.131 * V, 2: 0.045 * V - 0.131 * V,
             6: 0.045 * V - 0.131 * V, 1: 0.045 * V + 0.131 * V * (math.cos(math.pi / 4) - 1)}
    for k, expo in cases.items():
        b, st = _one_cell_batch([k], V=V, theta=0.0)
        p = oracle.Sim(b, prm).cell_prob(0, 1, 1, st)
        want = 1.0 - math.exp(-0.3 * math.exp(expo))
        assert abs(p - want) < 3e-7, (k, p, want)


def test_wind_toward_north():
    """Theta = pi/2 (toward north, i.e. decreasing row): the burning cell
    south of v spreads north with the full factor exp(a_w1 V)."""
    prm = firegen.Params(alpha_w1=0.05, alpha_w2=0.2, p_base=0.2)
    b, st = _one_cell_batch([2], V=5.0, theta=math.pi / 2)  # k=2 north, source is south
    p = oracle.Sim(b, prm).cell_prob(0, 1, 1, st)
    assert abs(p - (1.0 - math.exp(-0.2 * math.exp(0.25)))) < 3e-7


def test_slope_uphill_and_diagonal_distance():
    """Eq. 2 with S = rise / run: spreading uphill by h over one cell gives
    exp(a_s h / cs); over a diagonal the run is cs sqrt(2)."""
    prm = firegen.Params(alpha_s=4.5, p_base=0.25, cell_size=30.0)
    E = np.zeros((3, 3), np.float32)
    E[1, 1] = 6.0                              # target 6 m above its neighbours
    for k, run in [(2, 30.0), (1, 30.0 * math.sqrt(2)), (4, 30.0)]:
        b, st = _one_cell_batch([k], slope_rise=E)
        p = oracle.Sim(b, prm).cell_prob(0, 1, 1, st)
        want = 1.0 - math.exp(-0.25 * math.exp(4.5 * 6.0 / run))
        assert abs(p - want) < 3e-7, (k, p, want)


def test_fuel_terms_source_and_target():
    """phi uses the source's (1+veg)(1+den); gamma the target's (Eq. 3, 4)."""
    veg = [0.0] * 11
    veg[firegen.TREE] = 0.3
    veg[firegen.GRASS] = -0.2
    prm = firegen.Params(p_base=0.4, alpha_gamma=1.7, veg=tuple(veg))
    b, st = _one_cell_batch([0])
    b.cls[:] = firegen.GRASS
    b.cls[3] = firegen.TREE                    # west neighbour = source of k=0
    b.den[:] = 0.1
    b.den[3] = -0.25
    p = oracle.Sim(b, prm).cell_prob(0, 1, 1, st)
    phi = 0.4 * (1 + 0.3) * (1 - 0.25)
    gamma = 1.7 * (1 - 0.2) * (1 + 0.1)
    assert abs(p - (1 - math.exp(-gamma * phi))) < 3e-7


def test_random_neighbourhoods_against_fp64_closed_form():
    """Random wind, fuel, terrain and burning subsets: oracle fp32 p versus
    Eq. 4 in fp64 written with the paper's separate exponentials."""
    rng = np.random.default_rng(5)
    veg = tuple(float(v) for v in rng.uniform(-0.4, 0.4, 11))
    for trial in range(300):
        prm = firegen.Params(p_base=float(rng.uniform(0.05, 1.5)),
                             alpha_gamma=float(rng.uniform(0.5, 2.0)),
                             alpha_w1=float(rng.uniform(0, 0.1)),
                             alpha_w2=float(rng.uniform(0, 0.3)),
                             alpha_s=float(rng.uniform(0, 6.0)), veg=veg)
        dirs = [k for k in range(8) if rng.random() < 0.4] or [int(rng.integers(8))]
        V, th = float(rng.uniform(0, 10)), float(rng.uniform(0, 2 * math.pi))
        b, st = _one_cell_batch(dirs, V=V, theta=th)
        b.cls[:] = rng.integers(0, 11, 9).astype(np.uint8)
        b.den[:] = rng.uniform(-0.3, 0.3, 9).astype(np.float32)
        b.elev[:] = rng.uniform(0, 20, 9).astype(np.float32)
        p = oracle.Sim(b, prm).cell_prob(0, 1, 1, st)
        g = [(1 + np.float32(veg[b.cls[c]]).astype(np.float64)) * (1 + float(b.den[c]))
             for c in range(9)]
        Vx, Vy = float(b.wind_env[0, 1]), float(b.wind_env[0, 2])
        Vv = float(b.wind_env[0, 0])
        th32 = math.atan2(Vy, Vx)
        lam = 0.0
        for k in dirs:
            di, dj = relaxed64.DIRS[k]
            u = (1 - di) * 3 + (1 - dj)
            kw = math.exp(prm.alpha_w1 * Vv) * math.exp(
                prm.alpha_w2 * Vv * (math.cos(k * math.pi / 4 - th32) - 1))
            S = (float(b.elev[4]) - float(b.elev[u])) / (30.0 * (math.sqrt(2) if k % 2 else 1.0))
            lam += prm.p_base * g[u] * kw * math.exp(prm.alpha_s * S)
        want = 1.0 - math.exp(-prm.alpha_gamma * g[4] * lam)
        # fp32 evaluation: a few ulp of (1 - p) plus input rounding of the parameters
        assert abs(p - want) <= 2e-6 * max(1.0, lam), (trial, p, want)


# -------------------------------------------------- whole-grid pins --------
def _cheb(H, W, ci, cj):
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return np.maximum(abs(ii - ci), abs(jj - cj))


@pytest.mark.parametrize("p_c", [0.0, 0.5])
def test_p_one_chebyshev_square(p_c):
    """p_base = 64 makes gamma lambda >= 64, so p rounds to 1.0f: the burning
    front is the Chebyshev ring at distance t from the ignition, clipped by
    the grid (64x64, 100 steps)."""
    b, prm, T, seed = firegen.workload_single64()
    prm = prm.replace(p_base=64.0, p_continue=p_c)
    sim = oracle.Sim(b, prm, seed)
    d = _cheb(64, 64, 32, 32)
    for t in range(1, T + 1):
        sim.step(1)
        F = sim.states.reshape(64, 64)
        assert np.all(F[d > t] == firegen.FLAMMABLE)
        assert np.all(F[d == t] == firegen.BURNING)
        inner = F[d < t]
        if p_c == 0.0:
            assert np.all(inner == firegen.BURNT)
        else:
            assert np.all((inner == firegen.BURNING) | (inner == firegen.BURNT))


def test_p_zero_never_spreads_and_burning_decays_binomially():
    """p_base = 0: the FLAMMABLE set never changes; each ignition cell is still
    BURNING after t steps with probability p_c^t."""
    R, T, p_c = 20000, 3, 0.6
    b = firegen.uniform_batch(5, 5, n_env=R)
    prm = firegen.Params(p_base=0.0, p_continue=p_c)
    sim = oracle.Sim(b, prm, seed=9)
    flam0 = sim.states == firegen.FLAMMABLE
    sim.step(T)
    assert np.array_equal(sim.states == firegen.FLAMMABLE, flam0)
    centre = sim.states.reshape(R, 25)[:, 12]
    frac = np.mean(centre == firegen.BURNING)
    want = p_c ** T
    assert abs(frac - want) < 5 * math.sqrt(want * (1 - want) / R)


def test_invariants_on_landscape_with_actions():
    """States only move FLAMMABLE -> BURNING -> BURNT or to UNBURNABLE by a
    drop; UNBURNABLE and BURNT never change; counts equal a recount; no cell
    of a drop square is FLAMMABLE/BURNING after its step."""
    b = firegen.landscape_batch(7, [(40, 56), (33, 17), (64, 64)])
    prm = firegen.Params(veg=tuple(firegen.veg_table(np.random.default_rng(1))))
    acts = firegen.random_actions(8, b, 12, p_none=0.3)
    sim = oracle.Sim(b, prm, seed=4)
    for s in range(12):
        before = sim.states.copy()
        cnt = sim.step(1, actions=acts[s:s + 1], counts=True)
        after = sim.states
        ok = ((after == before) |
              ((before == firegen.FLAMMABLE) & (after == firegen.BURNING)) |
              ((before == firegen.BURNING) & (after == firegen.BURNT)) |
              (((before == firegen.FLAMMABLE) | (before == firegen.BURNING)) &
               (after == firegen.UNBURNABLE)))
        assert ok.all()
        assert np.all(after[before == firegen.UNBURNABLE] == firegen.UNBURNABLE)
        assert np.all(after[before == firegen.BURNT] == firegen.BURNT)
        for e in range(b.n_env):
            Fe = b.env_view(after, e)
            assert cnt[0, e] == int(np.sum(Fe == firegen.BURNING))
            a = int(acts[s, e])
            if a >= 0:
                r, c = a >> 16, a & 0xFFFF
                box = Fe[max(0, r - 2):r + 3, max(0, c - 2):c + 3]
                assert not np.any((box == firegen.FLAMMABLE) | (box == firegen.BURNING))


def test_resume_split_is_bit_identical():
    """Counter-based draws: T1 + T2 steps equal T1+T2 steps in one call."""
    b = firegen.landscape_batch(3, [(48, 48)] * 3)
    prm = firegen.Params(veg=tuple(firegen.veg_table(np.random.default_rng(2))))
    a = oracle.Sim(b, prm, seed=77)
    a.step(25)
    c = oracle.Sim(b, prm, seed=77)
    c.step(10)
    c.step(15)
    assert np.array_equal(a.states, c.states)


def test_threads_do_not_change_results():
    b = firegen.landscape_batch(4, [(32, 40)] * 6)
    prm = firegen.Params()
    a = oracle.Sim(b, prm, seed=1)
    a.step(20)
    c = oracle.Sim(b, prm, seed=1)
    c.step(20, threads=4)
    assert np.array_equal(a.states, c.states)


# --------------------------------------------- Monte Carlo vs closed form --
def test_single_cell_ignition_frequency():
    """Over many replica envs (distinct env_id) the ignition frequency of one
    flammable cell matches Eq. 4 in fp64 within 5 sigma; the continuation
    frequency of the burning neighbours matches p_continue."""
    R = 1 << 17
    rng = np.random.default_rng(3)
    prm = firegen.Params(p_base=0.35, alpha_s=3.0, p_continue=0.37,
                         veg=tuple(float(v) for v in rng.uniform(-0.4, 0.4, 11)))
    dirs = [0, 3, 6]
    b1, st = _one_cell_batch(dirs, V=6.0, theta=2.0)
    b1.cls[:] = rng.integers(0, 5, 9).astype(np.uint8)
    b1.den[:] = rng.uniform(-0.3, 0.3, 9).astype(np.float32)
    b1.elev[:] = rng.uniform(0, 15, 9).astype(np.float32)
    b = firegen.uniform_batch(3, 3, n_env=R, ignitions=())
    b.cls[:] = np.tile(b1.cls, R)
    b.den[:] = np.tile(b1.den, R)
    b.elev[:] = np.tile(b1.elev, R)
    b.wind_env[:] = b1.wind_env[0]
    sim = oracle.Sim(b, prm, seed=123)
    sim.states[:] = np.tile(st, R)
    env = relaxed64.from_batch(b1, 0, 30.0)
    theta = relaxed64.theta_from_params(prm)
    theta32 = theta.astype(np.float32).astype(np.float64)
    terms = relaxed64.edge_terms(env, theta32)
    lam = sum(terms["phi"][k][1, 1] for k in dirs)
    p = -math.expm1(-terms["gamma"][1, 1] * lam)
    sim.step(1)
    F = sim.states.reshape(R, 9)
    freq = np.mean(F[:, 4] == firegen.BURNING)
    assert abs(freq - p) < 5 * math.sqrt(p * (1 - p) / R), (freq, p)
    src = [(1 - relaxed64.DIRS[k][0]) * 3 + (1 - relaxed64.DIRS[k][1]) for k in dirs]
    cont = np.mean(F[:, src] == firegen.BURNING)
    n = R * len(src)
    assert abs(cont - 0.37) < 5 * math.sqrt(0.37 * 0.63 / n)


def _replicate(b1, R):
    H, W = int(b1.H[0]), int(b1.W[0])
    b = firegen.uniform_batch(H, W, n_env=R, ignitions=())
    b.cls[:] = np.tile(b1.cls, R)
    b.den[:] = np.tile(b1.den, R)
    b.elev[:] = np.tile(b1.elev, R)
    b.wind_env[:] = b1.wind_env[0]
    return b


@pytest.mark.parametrize("H,W,T,ign", [(3, 3, 6, [(1, 1)]), (4, 4, 3, [(0, 0)]),
                                       (3, 4, 3, [(0, 1), (2, 3)])])
def test_exact_enumeration_matches_monte_carlo(H, W, T, ign):
    """Exact Markov-chain marginals P(F_t(v) = s) (fp64, Eq. 4) against the
    oracle's frequencies over 2^17 replica envs, every cell, state and step,
    within 5 sigma; one unburnable cell included."""
    R = 1 << 17
    rng = np.random.default_rng(H * 100 + W + T)
    prm = firegen.Params(p_base=0.3, alpha_w1=0.04, alpha_w2=0.15, alpha_s=4.0, p_continue=0.45,
                         veg=tuple(float(v) for v in firegen.veg_table(rng)))
    b1 = firegen.uniform_batch(H, W, wind=(5.0, 0.7), ignitions=())
    b1.cls[:] = rng.choice([0, 1, 2, 3, 8], H * W).astype(np.uint8)
    b1.cls[H * W - 2] = firegen.WATER
    b1.den[:] = rng.uniform(-0.3, 0.3, H * W).astype(np.float32)
    b1.elev[:] = rng.uniform(0, 10, H * W).astype(np.float32)
    F0 = np.where(((b1.unburnable_mask >> b1.cls.astype(np.int64)) & 1) == 1,
                  firegen.UNBURNABLE, firegen.FLAMMABLE).reshape(H, W)
    for i, j in ign:
        F0[i, j] = firegen.BURNING
    theta32 = relaxed64.theta_from_params(prm).astype(np.float32).astype(np.float64)
    exact = enumerate_exact.exact_marginals(relaxed64.from_batch(b1, 0, 30.0), theta32, F0, T)
    sim = oracle.Sim(_replicate(b1, R), prm, seed=31)
    sim.states[:] = np.tile(F0.ravel(), R)
    worst = 0.0
    for t in range(1, T + 1):
        sim.step(1)
        F = sim.states.reshape(R, H, W)
        for s in range(4):
            freq = np.mean(F == s, axis=0)
            p = exact[t, :, :, s]
            sd = np.sqrt(np.maximum(p * (1 - p), 1e-12) / R)
            z = np.abs(freq - p) / sd
            worst = max(worst, float(z.max()))
    assert worst < 5.0, worst


def test_directional_sanity():
    """Flat, no wind: the mean scar is D4-symmetric.  Wind toward east moves
    the burnt centroid to +j; terrain rising northward moves it to -i."""
    R, n = 2000, 21
    prm = firegen.Params(p_base=0.35, p_continue=0.6, alpha_w1=0.05, alpha_w2=0.3, alpha_s=8.0)

    def scar(b, T=8):
        s = oracle.Sim(b, prm, seed=5)
        s.step(T)
        F = s.states.reshape(R, n, n)
        return np.mean((F == firegen.BURNING) | (F == firegen.BURNT), axis=0)

    flat = scar(firegen.uniform_batch(n, n, n_env=R))
    for m in (np.flip(flat, 0), np.flip(flat, 1), flat.T):
        assert np.max(np.abs(m - flat)) < 0.06
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    east = scar(firegen.uniform_batch(n, n, n_env=R, wind=(8.0, 0.0)))
    assert (east * jj).sum() / east.sum() > n // 2 + 1.0
    b = firegen.uniform_batch(n, n, n_env=R)
    b.elev[:] = np.tile(((n - 1 - ii) * 3.0).astype(np.float32).ravel(), R)
    north = scar(b)
    assert (north * ii).sum() / north.sum() < n // 2 - 1.0


# ------------------------------------------------------ time-varying wind --
def _with_env_wind(b, wind):
    import dataclasses
    return dataclasses.replace(b, wind_env=np.ascontiguousarray(wind, np.float32))


def test_wind_series_constant_equals_static():
    """A series repeating the static wind gives the static run, per env and
    per cell."""
    prm = firegen.Params(veg=tuple(firegen.veg_table(np.random.default_rng(4))))
    b = firegen.landscape_batch(8, [(40, 40), (24, 56)])
    a = oracle.Sim(b, prm, seed=3)
    a.step(30)
    c = oracle.Sim(b, prm, seed=3)
    c.step(30, wind_env_series=np.repeat(b.wind_env[None], 30, axis=0))
    assert np.array_equal(a.states, c.states)
    bc = firegen.landscape_batch(8, [(40, 40), (24, 56)], per_cell_wind=True)
    a = oracle.Sim(bc, prm, seed=3)
    a.step(30)
    c = oracle.Sim(bc, prm, seed=3)
    c.step(30, wind_cell_series=np.repeat(bc.wind_cell[None], 30, axis=0))
    assert np.array_equal(a.states, c.states)


def test_wind_series_is_indexed_by_absolute_step():
    """Wind A for steps 0..k-1 and B from step k equals k static steps under A
    followed by static steps under B from step k (also when the series run is
    itself split), and a per-cell series that broadcasts each env's wind
    equals the per-env series."""
    prm = firegen.Params(p_base=0.7, veg=tuple(firegen.veg_table(np.random.default_rng(5))))
    b = firegen.landscape_batch(9, [(48, 48), (30, 50), (40, 20)])
    A = firegen.wind_components(np.array([9.0, 2.0, 6.0]), np.array([0.0, 2.0, 4.0]))
    B = firegen.wind_components(np.array([3.0, 8.0, 6.0]), np.array([3.0, 1.0, 4.5]))
    k, T = 7, 20
    ser = np.concatenate([np.repeat(A[None], k, 0), np.repeat(B[None], T - k, 0)])
    ref = oracle.Sim(_with_env_wind(b, A), prm, seed=11)
    ref.step(k)
    ref2 = oracle.Sim(_with_env_wind(b, B), prm, seed=11)
    ref2.states[:] = ref.states
    ref2.t = k
    ref2.step(T - k)
    only_a = oracle.Sim(_with_env_wind(b, A), prm, seed=11)
    only_a.step(T)
    assert not np.array_equal(only_a.states, ref2.states)  # the switch matters
    s = oracle.Sim(b, prm, seed=11)
    s.step(12, wind_env_series=ser)
    s.step(T - 12, wind_env_series=ser)
    assert np.array_equal(s.states, ref2.states)
    cell = np.empty((T, 3, b.n_cells), np.float32)
    for e in range(b.n_env):
        cell[:, :, b.env_slice(e)] = ser[:, e, :, None]
    c = oracle.Sim(b, prm, seed=11)
    c.step(T, wind_cell_series=cell)
    assert np.array_equal(c.states, ref2.states)
    with pytest.raises(ValueError):
        oracle.Sim(b, prm).step(T + 1, wind_env_series=ser)


# ------------------------------------------------------------- drop modes --
@pytest.mark.parametrize("radius", [0, 1, 3])
def test_water_drop_extinguishes_square_before_the_step(radius):
    """Water (mode 1) turns the BURNING cells of the (2R+1)^2 square BURNT
    before the transition: with p = 1 spread and p_continue = 1, cells outside
    the square keep burning and spread, the square's burning cells are BURNT,
    its flammable cells stay flammable unless a burning cell outside the
    square touches them; the suppressant (mode 0) makes the square's
    flammable and burning cells UNBURNABLE."""
    n = 15
    b = firegen.uniform_batch(n, n, ignitions=())
    prm = firegen.Params(p_base=64.0, p_continue=1.0)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    F0 = np.where((ii + jj) % 3 == 0, firegen.BURNING, firegen.FLAMMABLE).astype(np.uint8)
    F0[0, :] = firegen.BURNT
    r, c = 7, 6
    inside = (abs(ii - r) <= radius) & (abs(jj - c) <= radius)
    for mode in (1, 0):
        s = oracle.Sim(b, prm)
        s.states[:] = F0.ravel()
        s.step(1, actions=np.array([[(r << 16) | c]], np.int32), drop_mode=mode, drop_radius=radius)
        F1 = s.states.reshape(n, n)
        Fd = F0.copy()
        if mode == 1:
            Fd[inside & (F0 == firegen.BURNING)] = firegen.BURNT
        else:
            Fd[inside & ((F0 == firegen.BURNING) | (F0 == firegen.FLAMMABLE))] = firegen.UNBURNABLE
        burn = np.pad(Fd == firegen.BURNING, 1)
        nb = sum(burn[1 + di:1 + di + n, 1 + dj:1 + dj + n] for di in (-1, 0, 1) for dj in (-1, 0, 1)
                 if di or dj)
        want = Fd.copy()
        want[(Fd == firegen.FLAMMABLE) & (nb > 0)] = firegen.BURNING
        assert np.array_equal(F1, want), (mode, radius)


# ---------------------------------------------------- slope-angle variant --
def _ulp32(v):
    v = np.abs(v)
    e = np.floor(np.log2(np.maximum(v, 2.0 ** -126)))
    return 2.0 ** (e - 23)


def test_atan_c_within_3ulp_and_odd():
    """atan_c against fp64 atan on every 64th fp32 bit pattern of [0, 2^24]
    plus powers of two up to 2^100, in units of the result's fp32 ulp; odd and
    monotone; atan(+-inf) = +-pi/2."""
    bits = np.arange(0, np.float32(2.0 ** 24).view(np.uint32), 64, dtype=np.uint32)
    x = np.concatenate([bits.view(np.float32), (2.0 ** np.arange(-100, 101)).astype(np.float32)])
    y = oracle.atan_c(x).astype(np.float64)
    want = np.arctan(x.astype(np.float64))
    err = np.abs(y - want) / _ulp32(want)
    assert np.max(err[want != 0]) <= 3.0, (x[np.argmax(err)], np.max(err))
    assert np.array_equal(oracle.atan_c(-x), -oracle.atan_c(x))
    xs = np.sort(x)
    assert np.all(np.diff(oracle.atan_c(xs).astype(np.float64)) >= 0)
    inf = oracle.atan_c(np.array([np.inf, -np.inf], np.float32))
    assert inf[0] == np.float32(math.pi / 2) and inf[1] == -np.float32(math.pi / 2)


def test_slope_angle_mode():
    """slope_mode 1: S is the slope angle atan(rise / run) in radians, so
    spreading uphill by h over one cell gives exp(a_s atan(h / cs)) (Eq. 2),
    diagonals with run cs sqrt(2); and downhill the mirror image."""
    prm = firegen.Params(alpha_s=3.0, p_base=0.25, cell_size=30.0, slope_mode=1)
    for h in (6.0, 45.0, -20.0, 300.0):
        E = np.zeros((3, 3), np.float32)
        E[1, 1] = h
        for k, run in [(2, 30.0), (1, 30.0 * math.sqrt(2)), (4, 30.0)]:
            b, st = _one_cell_batch([k], slope_rise=E)
            p = oracle.Sim(b, prm).cell_prob(0, 1, 1, st)
            want = 1.0 - math.exp(-0.25 * math.exp(3.0 * math.atan(h / run)))
            assert abs(p - want) < 4e-7, (h, k, p, want)
