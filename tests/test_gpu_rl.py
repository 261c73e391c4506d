"""GPU parity of the RL layer (section 4's air-tanker scenario) against the
oracle: resets, moves, water drops, fire steps, rewards, episode ends and
observations, bit-exact, through the C ABI."""
import numpy as np
import pytest
import torch

import firegen
from oracle import rl

pytestmark = pytest.mark.gpu

fs = pytest.importorskip("paper_2512_06102_amd")


def _agents_np(env):
    return np.array([[a.row, a.col, a.water, a.steps, a.done, a.last_count] for a in env.agents], np.int32)


# Batches: 20 x 20 envs (one launch per step holds 2 dwords per lane); envs
# with W % 4 != 0 (the separate launches, whatever single_launch says); up to
# 64 x 64 (16 dwords per lane); 32 x 32 (4 dwords per lane); per-cell wind;
# per-env and per-cell wind series; per-size-class plans (resident for the
# 20 x 20 envs) in a graph.
@pytest.mark.parametrize("single_launch", [True, False])
@pytest.mark.parametrize("sizes,plan,wind", [
    ([(20, 20)] * 96, dict(graph=0), None),
    ([(20, 20)] * 40 + [(33, 17), (64, 64), (7, 9)], dict(graph=0, tile_width=64, tile_rows=2,
                                                           skip_static=1, sparse=1), None),
    ([(20, 20)] * 30 + [(64, 64), (32, 48)], dict(graph=0, tile_width=64, temporal=4), None),
    ([(32, 32)] * 12 + [(20, 20)] * 12, dict(graph=0), "cell"),
    ([(20, 20)] * 24 + [(28, 16)], dict(graph=0), "env_series"),
    ([(20, 20)] * 24 + [(12, 36)], dict(graph=0), "cell_series"),
    ([(20, 20)] * 30 + [(64, 64), (32, 48)],
     dict(graph=1, classes={0: dict(resident=64), 1: dict(tile_rows=2, tile_width=64, skip_static=1, sparse=1)}),
     "env_series"),
])
def test_rl_episodes_match_oracle(sizes, plan, wind, single_launch):
    batch = firegen.landscape_batch(31, sizes, per_cell_wind=wind in ("cell", "cell_series"))
    params = firegen.Params(p_base=0.45, veg=tuple(firegen.veg_table(np.random.default_rng(31))))
    cfg = rl.Config(obs_radius=3, drop_radius=1, water_capacity=6, max_steps=25, burn_penalty=0.1,
                    extinguish_bonus=10.0)
    ser = None
    if wind in ("env_series", "cell_series"):
        ser = firegen.wind_series(8, batch, 40, per_cell=wind == "cell_series", speed_step=1.0, turn_step=0.3)
    ref = rl.RLEnvs(batch, params, 77, cfg, wind_env_series=ser if wind == "env_series" else None,
                    wind_cell_series=ser if wind == "cell_series" else None)
    sim = fs.FireSim.from_batch(batch, params, seed=77)
    plan = dict(plan)
    classes = plan.pop("classes", {})
    sim.set_plan(**plan)
    for c, cp in classes.items():  # per-size-class plans (the multi-launch path runs them)
        sim.set_class_plan(c, **cp)
    if ser is not None:
        dev = torch.from_numpy(ser).cuda()
        sim.set_wind_series(cell_series=dev) if wind == "cell_series" else sim.set_wind_series(env_series=dev)
    env = fs.RLEnv(sim, obs_radius=cfg.obs_radius, drop_radius=cfg.drop_radius,
                   water_capacity=cfg.water_capacity, max_steps=cfg.max_steps,
                   burn_penalty=cfg.burn_penalty, extinguish_bonus=cfg.extinguish_bonus,
                   single_launch=single_launch)
    ref.sim.t = 0
    want_obs, want_done = ref.reset(episode=5)
    obs, done = env.reset(episode=5)
    torch.cuda.synchronize()
    assert np.array_equal(sim.states.cpu().numpy(), ref.sim.states)
    assert np.array_equal(obs.cpu().numpy(), want_obs)
    assert np.array_equal(env.agents.cpu().numpy()[:, :6], _agents_np(ref))
    rng = np.random.default_rng(3)
    episode = 5
    for step in range(40):
        act = rng.integers(0, 32, batch.n_env).astype(np.int32)
        act[rng.random(batch.n_env) < 0.1] = -7      # invalid actions act as "stay, valve closed"
        want_obs, want_r, want_d = ref.step(act)
        obs, r, d = env.step(torch.from_numpy(act))
        torch.cuda.synchronize()
        assert np.array_equal(sim.states.cpu().numpy(), ref.sim.states), step
        assert np.array_equal(obs.cpu().numpy(), want_obs), step
        assert np.array_equal(r.cpu().numpy(), want_r), step
        assert np.array_equal(d.cpu().numpy(), want_d), step
        assert np.array_equal(env.agents.cpu().numpy()[:, :6], _agents_np(ref)), step
        if step % 10 == 9:      # restart finished episodes
            episode += 1
            m = want_d.copy()
            want_obs, _ = ref.reset(episode=episode, mask=m)
            obs, _ = env.reset(episode=episode, mask=torch.from_numpy(m))
            torch.cuda.synchronize()
            assert np.array_equal(sim.states.cpu().numpy(), ref.sim.states), step
            assert np.array_equal(obs.cpu().numpy(), want_obs), step
    assert sim.t == ref.sim.t == 40


def test_rl_rejects_bad_config():
    batch = firegen.landscape_batch(32, [(20, 20)] * 4)
    sim = fs.FireSim.from_batch(batch, firegen.Params(), seed=0)
    for kw in (dict(obs_radius=32), dict(obs_radius=-1), dict(drop_radius=256), dict(max_steps=0),
               dict(water_capacity=-1)):
        env = fs.RLEnv(sim, **kw)
        with pytest.raises(fs.SimError):
            env.reset(0)
        with pytest.raises(fs.SimError):
            env.step(torch.zeros(4, dtype=torch.int32))
    torch.cuda.synchronize()


@pytest.mark.parametrize("single_launch", [True, False])
@pytest.mark.parametrize("obs_radius,drop_radius,water,max_steps", [(0, 0, 3, 4), (31, 255, 2, 30), (5, 2, 0, 1)])
def test_rl_edge_configs(obs_radius, drop_radius, water, max_steps, single_launch):
    """Edge cases of the RL layer against the oracle: a one-cell and a 63 x 63
    window, a drop of radius 0 and one covering the grid, no water, one-step
    episodes; grids down to 1 x 4 and 4 x 4, and a 64 x 64 one."""
    sizes = [(20, 20)] * 6 + [(1, 4), (4, 4), (3, 8), (64, 64), (12, 44)]
    batch = firegen.landscape_batch(45, sizes)
    params = firegen.Params(p_base=0.9, veg=tuple(firegen.veg_table(np.random.default_rng(45))))
    cfg = rl.Config(obs_radius=obs_radius, drop_radius=drop_radius, water_capacity=water,
                    max_steps=max_steps, burn_penalty=0.25, extinguish_bonus=3.0)
    ref = rl.RLEnvs(batch, params, 5, cfg)
    sim = fs.FireSim.from_batch(batch, params, seed=5)
    env = fs.RLEnv(sim, obs_radius=cfg.obs_radius, drop_radius=cfg.drop_radius,
                   water_capacity=cfg.water_capacity, max_steps=cfg.max_steps,
                   burn_penalty=cfg.burn_penalty, extinguish_bonus=cfg.extinguish_bonus,
                   single_launch=single_launch)
    want_obs, _ = ref.reset(episode=2)
    obs, _ = env.reset(episode=2)
    torch.cuda.synchronize()
    assert np.array_equal(obs.cpu().numpy(), want_obs)
    rng = np.random.default_rng(11)
    for step in range(12):
        act = rng.integers(0, 32, batch.n_env).astype(np.int32)
        want_obs, want_r, want_d = ref.step(act)
        obs, r, d = env.step(torch.from_numpy(act))
        torch.cuda.synchronize()
        assert np.array_equal(sim.states.cpu().numpy(), ref.sim.states), step
        assert np.array_equal(obs.cpu().numpy(), want_obs), step
        assert np.array_equal(r.cpu().numpy(), want_r), step
        assert np.array_equal(d.cpu().numpy(), want_d), step
        assert np.array_equal(env.agents.cpu().numpy()[:, :6], _agents_np(ref)), step


@pytest.mark.parametrize("single_launch", [True, False])
def test_rl_benchmark_configuration_sampled(single_launch):
    """The benchmark's RL configuration at full size (65536 envs of 20 x 20,
    its plan and settings): 12 steps of random actions, with 16 sampled envs
    (first and last included) checked bit-exactly against the oracle run on
    those envs alone (envs are independent; draws are keyed by env_id)."""
    n = 65536
    batch = firegen.uniform_batch(20, 20, n_env=n, ignitions=())
    params = firegen.Params(p_base=0.45)
    sim = fs.FireSim.from_batch(batch, params, seed=0)
    sim.set_plan(tile_rows=4, tile_width=64, graph=0)
    env = fs.RLEnv(sim, obs_radius=2, drop_radius=1, water_capacity=20, max_steps=1000,
                   single_launch=single_launch)
    rng = np.random.default_rng(17)
    pick = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 14)]))
    cfg = rl.Config(obs_radius=2, drop_radius=1, water_capacity=20, max_steps=1000)
    ref = rl.RLEnvs(batch.subset(pick), params, 0, cfg)
    cells = np.concatenate([np.arange(e * 400, (e + 1) * 400) for e in pick])
    want_obs, _ = ref.reset(episode=1)
    obs, _ = env.reset(episode=1)
    torch.cuda.synchronize()
    assert np.array_equal(obs.cpu().numpy()[pick], want_obs)
    for step in range(12):
        act = rng.integers(0, 32, n).astype(np.int32)
        want_obs, want_r, want_d = ref.step(act[pick])
        obs, r, d = env.step(torch.from_numpy(act))
        torch.cuda.synchronize()
        assert np.array_equal(sim.states.cpu().numpy()[cells], ref.sim.states), step
        assert np.array_equal(obs.cpu().numpy()[pick], want_obs), step
        assert np.array_equal(r.cpu().numpy()[pick], want_r), step
        assert np.array_equal(d.cpu().numpy()[pick], want_d), step
        assert np.array_equal(env.agents.cpu().numpy()[pick, :6], _agents_np(ref)), step
