"""Oracle of the reinforcement-learning layer (test infrastructure only).

Section 4 of the paper: an air-tanker agent per env with partial egocentric
observations, a valve that drops a limited amount of water turning burning
cells burnt, a per-step penalty proportional to the number of burning cells,
a terminal +10 when the fire is out, and random initial fire and agent
positions.  The fire itself advances with the stochastic-step oracle
(`oracle.Sim.step`, drops in water mode).  Plain Python loops over envs.

Readings (the paper gives no more detail): the agent moves one cell per step
in one of the eight directions of section 3 (or stays), clipped to the grid;
an open valve with water left drops on the square of side 2 r + 1 centred on
the agent's new position before the fire step; an episode ends when no cell
burns or after max_steps steps; observations are the fire-state codes of the
(2R+1)^2 window centred on the agent, 4 outside the grid.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import firegen
import oracle

# the eight directions of section 3: k = 0 east, counter-clockwise, rows grow south
DIRS = ((0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1))
OUTSIDE = 4
ATTEMPTS = 8


@dataclasses.dataclass
class Config:
    obs_radius: int = 2
    drop_radius: int = 1
    water_capacity: int = 10
    max_steps: int = 100
    burn_penalty: float = 0.1
    extinguish_bonus: float = 10.0


@dataclasses.dataclass
class Agent:
    row: int = 0
    col: int = 0
    water: int = 0
    steps: int = 0
    done: int = 0
    last_count: int = 0


class RLEnvs:
    """Batched RL envs over an oracle.Sim."""

    def __init__(self, batch, params, seed: int, cfg: Config, wind_env_series=None, wind_cell_series=None):
        self.batch, self.cfg, self.seed = batch, cfg, int(seed)
        self.sim = oracle.Sim(batch, params, seed=seed)
        self.wind = {}  # optional wind series of the fire steps, row = absolute step
        if wind_env_series is not None:
            self.wind["wind_env_series"] = wind_env_series
        if wind_cell_series is not None:
            self.wind["wind_cell_series"] = wind_cell_series
        self.agents = [Agent() for _ in range(batch.n_env)]
        self.burnable = ((batch.unburnable_mask >> batch.cls.astype(np.int64)) & 1) == 0

    def _draw(self, e, episode, attempt):
        ctr = [int(self.batch.env_id[e]), episode & 0xFFFFFFFF, (episode >> 32) & 0xFFFFFFFF,
               0x80000000 | attempt]
        key = [self.seed & 0xFFFFFFFF, (self.seed >> 32) & 0xFFFFFFFF]
        return [int(w) for w in oracle.philox4x32_10(ctr, key)]

    def reset(self, episode: int, mask=None):
        b = self.batch
        for e in range(b.n_env):
            if mask is not None and not mask[e]:
                continue
            H, W = int(b.H[e]), int(b.W[e])
            sl = b.env_slice(e)
            self.sim.states[sl] = np.where(self.burnable[sl], firegen.FLAMMABLE, firegen.UNBURNABLE)
            a = Agent(water=self.cfg.water_capacity)
            for attempt in range(ATTEMPTS):
                w = self._draw(e, episode, attempt)
                if attempt == 0:
                    a.row, a.col = (w[2] * H) >> 32, (w[3] * W) >> 32
                i, j = (w[0] * H) >> 32, (w[1] * W) >> 32
                if self.burnable[sl][i * W + j]:
                    self.sim.states[sl.start + i * W + j] = firegen.BURNING
                    break
            self.agents[e] = a
        return self.observe(), np.array([a.done for a in self.agents], np.int32)

    def observe(self):
        b, R = self.batch, self.cfg.obs_radius
        side = 2 * R + 1
        out = np.full((b.n_env, side, side), OUTSIDE, np.uint8)
        for e, a in enumerate(self.agents):
            F = b.env_view(self.sim.states, e)
            H, W = F.shape
            for di in range(side):
                for dj in range(side):
                    i, j = a.row - R + di, a.col - R + dj
                    if 0 <= i < H and 0 <= j < W:
                        out[e, di, dj] = F[i, j]
        return out.reshape(b.n_env, side * side)

    def step(self, actions):
        b, cfg = self.batch, self.cfg
        drops = np.full((1, b.n_env), -1, np.int32)
        for e, a in enumerate(self.agents):
            if a.done:
                continue
            act = int(actions[e])
            move = act & 15 if 0 <= act < 32 else 0
            valve = 0 <= act < 32 and (act >> 4) & 1
            if 1 <= move <= 8:
                di, dj = DIRS[move - 1]
                a.row = min(max(a.row + di, 0), int(b.H[e]) - 1)
                a.col = min(max(a.col + dj, 0), int(b.W[e]) - 1)
            if valve and a.water > 0:
                drops[0, e] = (a.row << 16) | a.col
                a.water -= 1
        counts = self.sim.step(1, actions=drops, counts=True, drop_mode=1, drop_radius=cfg.drop_radius,
                               **self.wind)[0]
        reward = np.zeros(b.n_env, np.float32)
        for e, a in enumerate(self.agents):
            if a.done:
                continue
            c = int(counts[e])
            r = np.float32(-cfg.burn_penalty) * np.float32(c)
            if c == 0:
                r = np.float32(r + np.float32(cfg.extinguish_bonus))
            reward[e] = r
            a.steps += 1
            a.last_count = c
            a.done = int(c == 0 or a.steps >= cfg.max_steps)
        return self.observe(), reward, np.array([a.done for a in self.agents], np.int32)
