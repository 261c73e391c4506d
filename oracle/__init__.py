"""CPU oracle for the fire-spread cellular automaton -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it; it shares no code
with the HIP implementation.

* `fire_oracle.c` (bound here through ctypes): the stochastic step in fp32
  with its own Philox4x32-10 and its own exp, following the paper's section 3
  (Eqs. 1-4 and the stochastic-update paragraph).
* `relaxed64.py`: the relaxed (mean-field) step, its soft-IoU loss and its
  adjoint in float64 numpy.
* `enumerate_exact.py`: exact Markov-chain marginals of the stochastic
  process on tiny grids, from the fp64 closed form of Eq. 4.
* `rl.py`: the reinforcement-learning layer of section 4 (air-tanker agent,
  water drops, reward, egocentric observations, random resets) in plain
  Python over the stochastic-step oracle.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build_oracle

_lib = None


class OracleParams(ctypes.Structure):
    _fields_ = [("p_base", ctypes.c_float), ("alpha_gamma", ctypes.c_float),
                ("alpha_w1", ctypes.c_float), ("alpha_w2", ctypes.c_float),
                ("alpha_s", ctypes.c_float), ("p_continue", ctypes.c_float),
                ("cell_size", ctypes.c_float), ("slope_mode", ctypes.c_int32)]


class OracleEnv(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("env_id", ctypes.c_uint32), ("V", ctypes.c_float), ("Vx", ctypes.c_float),
                ("Vy", ctypes.c_float)]


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        path = build_oracle.LIB
        if not os.path.exists(path):
            build_oracle.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox_blocks.argtypes = [P, P, P, ctypes.c_int64]
        L.oracle_exp_c.argtypes = [ctypes.c_float]
        L.oracle_exp_c.restype = ctypes.c_float
        L.oracle_exp_c_batch.argtypes = [P, P, ctypes.c_int64]
        L.oracle_exp_c_sweep.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_int,
                                         ctypes.c_int, P]
        L.oracle_atan_c_batch.argtypes = [P, P, ctypes.c_int64]
        L.oracle_exp_c_sweep.restype = ctypes.c_double
        L.oracle_fuel.argtypes = [ctypes.c_int64, P, P, P, P]
        L.oracle_init_states.argtypes = [ctypes.c_int32, P, P, ctypes.c_uint32, P, ctypes.c_int32, P]
        L.oracle_init_states.restype = ctypes.c_int
        L.oracle_cell_prob.argtypes = [P, P, P, P, P, ctypes.c_int64, P, ctypes.c_int32,
                                       ctypes.c_int32]
        L.oracle_cell_prob.restype = ctypes.c_float
        L.oracle_run.argtypes = [P, ctypes.c_int32, P, P, P, P, ctypes.c_int64, P, ctypes.c_uint64,
                                 ctypes.c_int32, P, P, ctypes.c_uint64, ctypes.c_int32]
        L.oracle_run_ex.argtypes = L.oracle_run.argtypes + [P, P, ctypes.c_int32, ctypes.c_int32]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_blocks(ctr, key):
    """Philox4x32-10 of n counters [n,4] under keys [n,2] -> [n,4] uint32."""
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros_like(c)
    lib().oracle_philox_blocks(_ptr(c), _ptr(k), _ptr(out), c.shape[0])
    return out


def atan_c(x):
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().oracle_atan_c_batch(_ptr(x), _ptr(y), x.size)
    return y


def exp_c(x):
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().oracle_exp_c_batch(_ptr(x), _ptr(y), x.size)
    return y


def exp_c_sweep(amag: float, bmag: float, negative: bool, threads: int = 8):
    worst = ctypes.c_float(0.0)
    err = lib().oracle_exp_c_sweep(amag, bmag, int(negative), threads, ctypes.byref(worst))
    return err, worst.value


def params_struct(p) -> OracleParams:
    return OracleParams(p.p_base, p.alpha_gamma, p.alpha_w1, p.alpha_w2, p.alpha_s,
                        p.p_continue, p.cell_size, int(getattr(p, "slope_mode", 0)))


def envs_struct(batch):
    arr = (OracleEnv * batch.n_env)()
    for e in range(batch.n_env):
        arr[e] = OracleEnv(int(batch.offset[e]), int(batch.H[e]), int(batch.W[e]),
                           int(batch.env_id[e]), float(batch.wind_env[e, 0]),
                           float(batch.wind_env[e, 1]), float(batch.wind_env[e, 2]))
    return arr


def fuel(batch, params) -> np.ndarray:
    veg = np.asarray(params.veg, np.float32)
    g = np.empty(batch.n_cells, np.float32)
    lib().oracle_fuel(batch.n_cells, _ptr(np.ascontiguousarray(batch.cls)),
                      _ptr(np.ascontiguousarray(batch.den)), _ptr(veg), _ptr(g))
    return g


def init_states(batch) -> np.ndarray:
    st = np.empty(batch.n_cells, np.uint8)
    ign = np.ascontiguousarray(batch.ignitions, np.int32)
    rc = lib().oracle_init_states(batch.n_env, envs_struct(batch), _ptr(batch.cls),
                                  batch.unburnable_mask, _ptr(ign), ign.shape[0], _ptr(st))
    if rc != 0:
        raise ValueError("ignition outside its env")
    return st


class Sim:
    """Oracle simulation of a batch: fp32 fuel, initial states, step counter."""

    def __init__(self, batch, params, seed: int = 0):
        self.batch = batch
        self.params = params
        self.seed = int(seed)
        self.P = params_struct(params)
        self.envs = envs_struct(batch)
        self.g = fuel(batch, params)
        self.E = np.ascontiguousarray(batch.elev, np.float32)
        self.wind_cell = (None if batch.wind_cell is None
                          else np.ascontiguousarray(batch.wind_cell, np.float32))
        self.states = init_states(batch)
        self.t = 0

    def step(self, T: int, actions=None, counts: bool = False, threads: int = 1,
             wind_env_series=None, wind_cell_series=None, drop_mode: int = 0, drop_radius: int = 2,
             history: bool = False):
        """T steps from the current step t.  A wind series (float32
        [S][n_env][3] per env, or [S][3][n_cells] per cell, row = absolute
        step) replaces the static wind for steps t .. t+T-1.  Drops (actions)
        cover (2 drop_radius + 1)^2 cells; drop_mode 0 makes FLAMMABLE and
        BURNING cells UNBURNABLE, 1 makes BURNING cells BURNT.  With history
        the states after every step are returned ([T, n_cells]) instead of
        the counts; counts then come second."""
        if history:
            rows, cnts = [], []
            for _ in range(T):
                c = self.step(1, None if actions is None else np.asarray(actions)[len(rows):len(rows) + 1],
                              counts, threads, wind_env_series, wind_cell_series, drop_mode, drop_radius)
                rows.append(self.states.copy())
                cnts.append(c)
            return np.stack(rows), (np.concatenate(cnts) if counts else None)
        n_env = self.batch.n_env
        act = None if actions is None else np.ascontiguousarray(actions, np.int32)
        if act is not None and act.shape != (T, n_env):
            raise ValueError("actions must be [T, n_env]")
        es = None if wind_env_series is None else np.ascontiguousarray(wind_env_series, np.float32)
        cs = None if wind_cell_series is None else np.ascontiguousarray(wind_cell_series, np.float32)
        if es is not None and (es.ndim != 3 or es.shape[1:] != (n_env, 3) or es.shape[0] < self.t + T):
            raise ValueError("wind_env_series must be [>= t+T, n_env, 3]")
        if cs is not None and (cs.ndim != 3 or cs.shape[1:] != (3, self.batch.n_cells)
                               or cs.shape[0] < self.t + T):
            raise ValueError("wind_cell_series must be [>= t+T, 3, n_cells]")
        cnt = np.zeros((T, n_env), np.int32) if counts else None
        lib().oracle_run_ex(ctypes.byref(self.P), n_env, self.envs, _ptr(self.g), _ptr(self.E),
                            _ptr(self.wind_cell), self.batch.n_cells, _ptr(self.states), self.t, T,
                            _ptr(act), _ptr(cnt), self.seed, threads, _ptr(es), _ptr(cs),
                            int(drop_mode), int(drop_radius))
        self.t += T
        return cnt

    def cell_prob(self, e: int, i: int, j: int, states=None) -> float:
        st = self.states if states is None else np.ascontiguousarray(states, np.uint8)
        return lib().oracle_cell_prob(ctypes.byref(self.P), ctypes.byref(self.envs[e]),
                                      _ptr(self.g), _ptr(self.E), _ptr(self.wind_cell),
                                      self.batch.n_cells, _ptr(st), i, j)
