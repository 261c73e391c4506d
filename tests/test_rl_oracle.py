"""Pins of the RL-layer oracle (section 4's air-tanker scenario) on small,
hand-checked cases: moves and clipping, water drops and their budget, the
reward, the terminal bonus and episode end, observation windows, and the
uniformity of the random resets."""
import numpy as np
import pytest

import firegen
from oracle import rl


def _envs(F, cfg, p_base=0.0, p_continue=1.0, n_env=1, seed=0):
    H, W = F.shape
    b = firegen.uniform_batch(H, W, n_env=n_env, ignitions=())
    prm = firegen.Params(p_base=p_base, p_continue=p_continue)
    env = rl.RLEnvs(b, prm, seed, cfg)
    env.sim.states[:] = np.tile(F.ravel(), n_env)
    return env


def _place(env, e, row, col, water):
    env.agents[e] = rl.Agent(row=row, col=col, water=water)


def test_moves_clip_to_the_grid():
    F = np.full((5, 6), firegen.FLAMMABLE, np.uint8)
    F[4, 5] = firegen.BURNING
    env = _envs(F, rl.Config(obs_radius=1, max_steps=50))
    _place(env, 0, 0, 0, 0)
    path = []
    # NW (clipped), E, E, SE x5 (clipped twice), S (clipped), N, stay, SW, W
    for move in (4, 1, 1, 8, 8, 8, 8, 8, 7, 3, 0, 6, 5):
        env.step(np.array([move]))
        a = env.agents[0]
        path.append((a.row, a.col))
    assert path == [(0, 0), (0, 1), (0, 2), (1, 3), (2, 4), (3, 5), (4, 5), (4, 5), (4, 5), (3, 5),
                    (3, 5), (4, 4), (4, 3)]


def test_water_turns_burning_square_burnt_and_is_limited():
    """p_base 0, p_continue 1: nothing spreads or burns out by itself; each
    drop turns the burning cells of its 3x3 square burnt; the reward is
    -0.5 x the burning cells left; no water, no drop."""
    F = np.full((7, 7), firegen.FLAMMABLE, np.uint8)
    F[1:6, 1:6] = firegen.BURNING
    cfg = rl.Config(obs_radius=1, drop_radius=1, water_capacity=2, burn_penalty=0.5, max_steps=50)
    env = _envs(F, cfg)
    _place(env, 0, 2, 2, 2)
    obs, r, d = env.step(np.array([16]))           # stay, valve open: 3x3 around (2,2)
    G = F.copy()
    G[1:4, 1:4] = firegen.BURNT
    assert np.array_equal(env.sim.states.reshape(7, 7), G)
    assert r[0] == np.float32(-0.5 * 16) and d[0] == 0 and env.agents[0].water == 1
    obs, r, d = env.step(np.array([16 | 7]))       # south, drop around (3,2)
    G[2:5, 1:4] = np.where(G[2:5, 1:4] == firegen.BURNING, firegen.BURNT, G[2:5, 1:4])
    assert np.array_equal(env.sim.states.reshape(7, 7), G)
    assert r[0] == np.float32(-0.5 * 13) and env.agents[0].water == 0
    obs, r, d = env.step(np.array([16 | 7]))       # no water left: nothing dropped
    assert np.array_equal(env.sim.states.reshape(7, 7), G)
    assert (env.agents[0].row, env.agents[0].col) == (4, 2)
    assert r[0] == np.float32(-0.5 * 13)


def test_extinguishing_ends_the_episode_with_the_bonus():
    F = np.full((6, 6), firegen.FLAMMABLE, np.uint8)
    F[2, 2] = F[3, 3] = firegen.BURNING
    cfg = rl.Config(obs_radius=2, drop_radius=1, water_capacity=3, burn_penalty=0.25,
                    extinguish_bonus=10.0, max_steps=50)
    env = _envs(F, cfg)
    _place(env, 0, 0, 0, 3)
    obs, r, d = env.step(np.array([8]))            # SE to (1,1), no drop
    assert r[0] == np.float32(-0.5) and d[0] == 0
    obs, r, d = env.step(np.array([16 | 8]))       # SE to (2,2) and drop: both fires out
    assert r[0] == np.float32(10.0) and d[0] == 1
    assert env.agents[0].water == 2 and env.agents[0].last_count == 0
    obs, r, d = env.step(np.array([16 | 1]))       # episode over: idle, no reward
    assert r[0] == 0.0 and d[0] == 1
    assert (env.agents[0].row, env.agents[0].col, env.agents[0].water) == (2, 2, 2)


def test_step_limit_ends_the_episode():
    F = np.full((4, 4), firegen.FLAMMABLE, np.uint8)
    F[0, 0] = firegen.BURNING
    env = _envs(F, rl.Config(max_steps=3, burn_penalty=1.0))
    _place(env, 0, 3, 3, 0)
    dones = [int(env.step(np.array([0]))[2][0]) for _ in range(5)]
    assert dones == [0, 0, 1, 1, 1]
    assert env.agents[0].steps == 3


def test_observation_window_and_outside_code():
    F = (np.arange(30) % 4).astype(np.uint8).reshape(5, 6)
    env = _envs(F, rl.Config(obs_radius=2))
    _place(env, 0, 0, 5, 0)
    obs = env.observe().reshape(5, 5)
    want = np.full((5, 5), rl.OUTSIDE, np.uint8)
    want[2:5, 0:3] = F[0:3, 3:6]
    assert np.array_equal(obs, want)
    assert obs[2, 2] == F[0, 5]


def test_reset_draws_are_uniform_and_skip_unburnable_cells():
    """Over 4096 envs of 8 x 8 the ignition row and column and the agent row
    and column are uniform (chi-square at the 1e-4 level); with the left half
    of every grid water, fires start only on the right half and a grid is
    left without fire with probability 2^-8 (binomial, 5 sigma)."""
    from scipy.stats import chi2
    n = 4096
    b = firegen.uniform_batch(8, 8, n_env=n, ignitions=())
    env = rl.RLEnvs(b, firegen.Params(), 3, rl.Config())
    env.reset(episode=11)
    st = env.sim.states.reshape(n, 8, 8)
    assert np.all((st == firegen.BURNING).sum(axis=(1, 2)) == 1)
    e, i, j = np.nonzero(st == firegen.BURNING)
    rows = np.array([a.row for a in env.agents])
    cols = np.array([a.col for a in env.agents])
    for x in (i, j, rows, cols):
        cnt = np.bincount(x, minlength=8)
        assert np.sum((cnt - n / 8) ** 2 / (n / 8)) < chi2.ppf(1 - 1e-4, 7)
    b.cls[:] = np.tile(np.where(np.arange(64) % 8 < 4, firegen.WATER, firegen.GRASS), n).astype(np.uint8)
    env = rl.RLEnvs(b, firegen.Params(), 3, rl.Config())
    env.reset(episode=5)
    st = env.sim.states.reshape(n, 8, 8)
    assert np.all(st[:, :, :4] == firegen.UNBURNABLE)
    fires = (st == firegen.BURNING).sum(axis=(1, 2))
    assert set(np.unique(fires)) <= {0, 1}
    none = int((fires == 0).sum())
    mu, sd = n / 256, np.sqrt(n / 256 * (1 - 1 / 256))
    assert abs(none - mu) <= 5 * sd + 1


def test_reset_mask_and_episode_key():
    """A reset depends only on (seed, env_id, episode): repeating it repeats
    the draws; a masked reset leaves the other envs alone and gives the
    masked ones what a full reset with that episode gives them."""
    n = 6
    b = firegen.uniform_batch(16, 16, n_env=n, ignitions=())
    env = rl.RLEnvs(b, firegen.Params(), 9, rl.Config())
    env.reset(episode=1)
    s1 = env.sim.states.copy()
    a1 = [(a.row, a.col) for a in env.agents]
    env.reset(episode=1)
    assert np.array_equal(env.sim.states, s1)
    full = rl.RLEnvs(b, firegen.Params(), 9, rl.Config())
    full.reset(episode=2)
    mask = np.array([1, 0, 1, 0, 0, 1])
    env.reset(episode=2, mask=mask)
    for e in range(n):
        src, pos = (full.sim.states, (full.agents[e].row, full.agents[e].col)) if mask[e] else (s1, a1[e])
        assert np.array_equal(b.env_view(env.sim.states, e), b.env_view(src, e))
        assert (env.agents[e].row, env.agents[e].col) == pos
