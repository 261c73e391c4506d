"""Batched probabilistic fire-spread cellular automaton on AMD MI355X (gfx950).

Thin ctypes binding of the HIP library libfiresim.so (C ABI in
include/firesim.h).  Python only marshals arguments: PyTorch provides device
memory and the current stream; every step of the model runs in the library's
kernels.  Importing works without a GPU; creating a simulator needs the built
library and a GPU, and fails loudly otherwise.

    sim = FireSim.from_batch(batch, params, seed=0)    # batch: packed envs (firegen.Batch)
    counts = sim.step(200, counts=True)                 # [200, n_env] burning cells
    sim.autotune(T_probe=50)                            # pick the fastest launch plan
    hist, _ = sim.step_history(20)                      # every state of 20 steps

    U, B = sim.relaxed_init()                           # relaxed (mean-field) path
    theta, losses = calibrate(sim, target_scar, T=100, theta0=theta0, loss="bce",
                              loss_kw={"pool": 8})      # Adam through the adjoint

    env = RLEnv(sim, obs_radius=2, water_capacity=10)   # air-tanker scenario
    obs, done = env.reset(episode=0)
    obs, reward, done = env.step(actions)               # int32 [n_env]: move | valve << 4
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfiresim.so")

SIM_OK = 0
UNBURNABLE, FLAMMABLE, BURNING, BURNT = 0, 1, 2, 3
N_CLASSES = 11
N_THETA = 17
THETA_NAMES = ("p_base", "alpha_w1", "alpha_w2", "alpha_s", "alpha_gamma", "p_continue") + \
    tuple("veg%d" % c for c in range(N_CLASSES))

EXPORTED = ("sim_init", "sim_step", "sim_get_step", "sim_set_step", "sim_set_plan", "sim_get_plan",
            "sim_autotune", "sim_set_class_plan", "sim_get_class_plans", "sim_autotune_classes",
            "sim_set_wind_series", "sim_step_history", "sim_set_drop",
            "sim_rl_reset", "sim_rl_step",
            "sim_relaxed_init", "sim_relaxed_workspace_bytes", "sim_step_relaxed_fwd",
            "sim_relaxed_loss", "sim_relaxed_loss_noalloc", "sim_relaxed_loss_bce", "sim_step_relaxed_bwd", "sim_debug_exp", "sim_debug_atan", "sim_debug_philox", "sim_debug_stream",
            "sim_last_error", "sim_destroy")


class SimParams(ctypes.Structure):
    _fields_ = [("p_base", ctypes.c_float), ("alpha_gamma", ctypes.c_float),
                ("alpha_w1", ctypes.c_float), ("alpha_w2", ctypes.c_float),
                ("alpha_s", ctypes.c_float), ("p_continue", ctypes.c_float),
                ("veg", ctypes.c_float * N_CLASSES), ("cell_size", ctypes.c_float),
                ("unburnable_mask", ctypes.c_uint32), ("slope_mode", ctypes.c_uint32)]


class SimEnv(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("env_id", ctypes.c_uint32), ("V", ctypes.c_float), ("Vx", ctypes.c_float),
                ("Vy", ctypes.c_float)]


class SimPlan(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("tile_width", ctypes.c_int32),
                ("temporal", ctypes.c_int32), ("skip_static", ctypes.c_int32),
                ("sparse", ctypes.c_int32), ("graph", ctypes.c_int32), ("resident", ctypes.c_int32)]


class SimTuneResult(ctypes.Structure):
    _fields_ = [("plan", SimPlan), ("ms_per_step", ctypes.c_float)]


class SimClassPlan(ctypes.Structure):
    _fields_ = [("size_class", ctypes.c_int32), ("n_env", ctypes.c_int32), ("n_cells", ctypes.c_int64),
                ("plan", SimPlan), ("ms_per_step", ctypes.c_float), ("from_cache", ctypes.c_int32)]


N_SIZE_CLASSES = 8
PLAN_KEYS = ("tile_rows", "tile_width", "temporal", "skip_static", "sparse", "resident")


def _plan_dict(p) -> dict:
    return {k: int(getattr(p, k)) for k in PLAN_KEYS}


class SimError(RuntimeError):
    pass


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SimError("libfiresim.so is not built (run __graft_entry__.build() or "
                           "python paper_2512_06102_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, U64, SZ = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                ctypes.c_size_t)
        L.sim_init.argtypes = [ctypes.POINTER(P), P, I32, P, I64, P, P, P, P, P, I32, U64, P, P]
        L.sim_step.argtypes = [P, P, P, I32, P, P]
        L.sim_get_step.argtypes = [P, ctypes.POINTER(U64)]
        L.sim_set_step.argtypes = [P, U64]
        L.sim_set_plan.argtypes = [P, P]
        L.sim_get_plan.argtypes = [P, P]
        L.sim_set_wind_series.argtypes = [P, P, P, I64]
        L.sim_step_history.argtypes = [P, P, P, I32, P, P, P]
        L.sim_set_drop.argtypes = [P, I32, I32]
        L.sim_rl_reset.argtypes = [P, P, P, P, P, U64, P, P, P]
        L.sim_rl_step.argtypes = [P, P, P, P, P, P, P, P, P]
        L.sim_autotune.argtypes = [P, P, I32, I32, I32, P, I32, ctypes.POINTER(I32), P]
        L.sim_set_class_plan.argtypes = [P, I32, P]
        L.sim_get_class_plans.argtypes = [P, P, I32, ctypes.POINTER(I32)]
        L.sim_autotune_classes.argtypes = [P, P, I32, I32, I32, ctypes.c_char_p, P, I32, ctypes.POINTER(I32), P]
        L.sim_relaxed_init.argtypes = [P, P, P, P]
        L.sim_relaxed_workspace_bytes.argtypes = [P, I32, I32]
        L.sim_relaxed_workspace_bytes.restype = SZ
        D = ctypes.c_double
        L.sim_step_relaxed_fwd.argtypes = [P, P, P, P, I32, I32, I32, P, SZ, P]
        L.sim_relaxed_loss.argtypes = [P, P, P, P, P, D, P, P]
        L.sim_relaxed_loss_noalloc.argtypes = [P, P, P, P, P, D, P, P]
        L.sim_relaxed_loss_bce.argtypes = [P, P, P, I32, D, D, P, P, D, P, P]
        L.sim_step_relaxed_bwd.argtypes = [P, P, P, P, I32, I32, I32, P, SZ, P, P]
        L.sim_debug_exp.argtypes = [P, P, I64, P]
        L.sim_debug_atan.argtypes = [P, P, I64, P]
        L.sim_debug_philox.argtypes = [P, P, P, I64, P]
        L.sim_debug_stream.argtypes = [I32, P, P, I64, I32, P]
        L.sim_last_error.argtypes = [P]
        L.sim_last_error.restype = ctypes.c_char_p
        L.sim_destroy.argtypes = [P]
        _lib = L
    return _lib


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _form(form: str) -> int:
    if form not in ("product", "exp"):
        raise ValueError("form must be 'product' or 'exp', got %r" % (form,))
    return 0 if form == "product" else 1


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(rc: int, handle=None):
    if rc != SIM_OK:
        msg = lib().sim_last_error(handle)
        raise SimError("firesim error %d: %s" % (rc, msg.decode() if msg else ""))


def make_params(p) -> SimParams:
    """SimParams from any object with the paper's parameter names."""
    from_mask = getattr(p, "unburnable_mask", None)
    s = SimParams()
    s.p_base, s.alpha_gamma = p.p_base, p.alpha_gamma
    s.alpha_w1, s.alpha_w2, s.alpha_s = p.alpha_w1, p.alpha_w2, p.alpha_s
    s.p_continue, s.cell_size = p.p_continue, p.cell_size
    for c in range(N_CLASSES):
        s.veg[c] = float(p.veg[c])
    s.unburnable_mask = int(from_mask) if from_mask is not None else 0
    s.slope_mode = int(getattr(p, "slope_mode", 0))
    return s


def params_with_theta(base: SimParams, theta: Sequence[float]) -> SimParams:
    """Copy of `base` with the 17 calibrated parameters taken from theta."""
    s = SimParams()
    ctypes.pointer(s)[0] = base
    s.p_base, s.alpha_w1, s.alpha_w2, s.alpha_s, s.alpha_gamma, s.p_continue = \
        (float(x) for x in theta[:6])
    for c in range(N_CLASSES):
        s.veg[c] = float(theta[6 + c])
    return s


def debug_atan(x: torch.Tensor) -> torch.Tensor:
    """The slope-angle arctangent of the step applied to a float32 CUDA tensor."""
    x = x.contiguous()
    y = torch.empty_like(x)
    _check(lib().sim_debug_atan(_ptr(x), _ptr(y), x.numel(), ctypes.c_void_p(_stream(x.device))))
    return y


def debug_exp(x: torch.Tensor) -> torch.Tensor:
    """The step's device exp applied to a float32 CUDA tensor."""
    x = x.contiguous()
    y = torch.empty_like(x)
    _check(lib().sim_debug_exp(_ptr(x), _ptr(y), x.numel(), ctypes.c_void_p(_stream(x.device))))
    return y


def debug_stream(mode: int, src: Optional[torch.Tensor], dst: torch.Tensor, blocks: int = 8192):
    """The library's HBM streaming probe (0 read src, 1 write dst, 2 copy) on
    the current stream; src and dst are byte-sized views of device memory."""
    n = dst.numel() * dst.element_size() if src is None else src.numel() * src.element_size()
    _check(lib().sim_debug_stream(int(mode), _ptr(src), _ptr(dst), int(n), int(blocks), _stream(dst.device)))


def debug_philox(ctr: torch.Tensor, key: torch.Tensor) -> torch.Tensor:
    """Philox4x32-10 blocks of int32 CUDA tensors ctr [n,4], key [n,2]."""
    ctr, key = ctr.contiguous(), key.contiguous()
    out = torch.empty_like(ctr)
    _check(lib().sim_debug_philox(_ptr(ctr), _ptr(key), _ptr(out), ctr.shape[0],
                                  ctypes.c_void_p(_stream(ctr.device))))
    return out


class FireSim:
    """A batch of envs on one GPU: static layers, fire state, step counter.

    Arguments are CUDA tensors in the packed layout of include/firesim.h:
    landcover uint8 [n_cells], density / elevation float32 [n_cells],
    wind_cell float32 [3, n_cells] or None; envs is a list of
    (offset, H, W, env_id, V, Vx, Vy); ignitions an int32 array [n, 3]."""

    def __init__(self, params, envs, landcover, density, elevation, wind_cell=None,
                 ignitions=(), seed: int = 0, unburnable_mask: Optional[int] = None):
        L = lib()
        self.device = landcover.device
        self.params = make_params(params)
        if unburnable_mask is not None:
            self.params.unburnable_mask = int(unburnable_mask)
        self.n_env = len(envs)
        self.n_cells = int(landcover.numel())
        arr = (SimEnv * self.n_env)()
        for e, (off, H, W, eid, V, Vx, Vy) in enumerate(envs):
            arr[e] = SimEnv(int(off), int(H), int(W), int(eid), float(V), float(Vx), float(Vy))
        self.envs = arr
        self.env_tuples = [tuple(x) for x in envs]
        ign = list(ignitions)
        ign_arr = (ctypes.c_int32 * max(1, 3 * len(ign)))()
        for q, (e, i, j) in enumerate(ign):
            ign_arr[3 * q], ign_arr[3 * q + 1], ign_arr[3 * q + 2] = int(e), int(i), int(j)
        self.states = torch.empty(self.n_cells, dtype=torch.uint8, device=self.device)
        self._keep = (landcover, density, elevation, wind_cell)
        h = ctypes.c_void_p()
        rc = L.sim_init(ctypes.byref(h), ctypes.byref(self.params), self.n_env, arr, self.n_cells,
                        _ptr(landcover.contiguous()), _ptr(density.contiguous()),
                        _ptr(elevation.contiguous()),
                        _ptr(None if wind_cell is None else wind_cell.contiguous()),
                        ign_arr if ign else None, len(ign), int(seed), _ptr(self.states),
                        ctypes.c_void_p(_stream(self.device)))
        _check(rc)
        self.handle = h
        self._keep = None

    @classmethod
    def from_batch(cls, batch, params, seed: int = 0, device="cuda"):
        """Build from a host batch (numpy arrays: cls, den, elev, wind_cell,
        offsets, sizes, env_id, wind_env, ignitions)."""
        dev = torch.device(device)
        envs = [(int(batch.offset[e]), int(batch.H[e]), int(batch.W[e]), int(batch.env_id[e]),
                 float(batch.wind_env[e, 0]), float(batch.wind_env[e, 1]),
                 float(batch.wind_env[e, 2])) for e in range(batch.n_env)]
        wc = None if batch.wind_cell is None else torch.from_numpy(batch.wind_cell).to(dev)
        return cls(params, envs, torch.from_numpy(batch.cls).to(dev),
                   torch.from_numpy(batch.den).to(dev), torch.from_numpy(batch.elev).to(dev),
                   wc, [tuple(int(x) for x in r) for r in batch.ignitions], seed,
                   unburnable_mask=batch.unburnable_mask)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.sim_destroy(h)
            self.handle = None

    def _s(self):
        return ctypes.c_void_p(_stream(self.device))

    # ---------------------------------------------------------- stochastic
    def step(self, T: int, actions: Optional[torch.Tensor] = None, counts: bool = False,
             states: Optional[torch.Tensor] = None):
        """Advance T stochastic steps in place; returns counts [T, n_env] or None."""
        st = self.states if states is None else states
        cnt = torch.empty((T, self.n_env), dtype=torch.int32, device=self.device) if counts else None
        if actions is not None:
            actions = actions.to(device=self.device, dtype=torch.int32).contiguous()
            if tuple(actions.shape) != (T, self.n_env):
                raise ValueError("actions must be [T, n_env]")
        _check(lib().sim_step(self.handle, _ptr(st), _ptr(actions), int(T), _ptr(cnt), self._s()),
               self.handle)
        return cnt

    def set_wind_series(self, env_series: Optional[torch.Tensor] = None,
                        cell_series: Optional[torch.Tensor] = None):
        """Time-varying wind: float32 device [S][n_env][3] per env or
        [S][3][n_cells] per cell, (V, V cos Theta, V sin Theta), row = absolute
        step.  None for both restores the static wind.  The tensor is kept
        alive by the simulator until replaced."""
        S = 0
        for ser, shape in ((env_series, (self.n_env, 3)), (cell_series, (3, self.n_cells))):
            if ser is None:
                continue
            if ser.dtype != torch.float32 or ser.device != self.device or ser.dim() != 3 \
                    or tuple(ser.shape[1:]) != shape or not ser.is_contiguous():
                raise ValueError("wind series must be a contiguous float32 [S, %d, %d] tensor on %s"
                                 % (shape + (self.device,)))
            S = int(ser.shape[0])
        _check(lib().sim_set_wind_series(self.handle, _ptr(env_series), _ptr(cell_series), S), self.handle)
        self._wind_series = (env_series, cell_series)

    def step_history(self, T: int, actions: Optional[torch.Tensor] = None, counts: bool = False,
                     history: Optional[torch.Tensor] = None):
        """T steps keeping every state: returns (history [T, n_cells] uint8,
        counts or None); the states end equal to history[T-1]."""
        if history is None:
            history = torch.empty((T, self.n_cells), dtype=torch.uint8, device=self.device)
        if history.dtype != torch.uint8 or history.device != self.device or not history.is_contiguous() \
                or tuple(history.shape) != (T, self.n_cells):
            raise ValueError("history must be a contiguous uint8 [T, n_cells] tensor on %s" % self.device)
        cnt = torch.empty((T, self.n_env), dtype=torch.int32, device=self.device) if counts else None
        if actions is not None:
            actions = actions.to(device=self.device, dtype=torch.int32).contiguous()
            if tuple(actions.shape) != (T, self.n_env):
                raise ValueError("actions must be [T, n_env]")
        _check(lib().sim_step_history(self.handle, _ptr(self.states), _ptr(actions), int(T), _ptr(cnt),
                                      _ptr(history), self._s()), self.handle)
        return history, cnt

    DROP_SUPPRESS, DROP_WATER = 0, 1

    def set_drop(self, mode: int = 0, radius: int = 2):
        """What drops do: mode 0 (suppressant) FLAMMABLE/BURNING -> UNBURNABLE,
        mode 1 (water) BURNING -> BURNT, on (2 radius + 1)^2 cells."""
        _check(lib().sim_set_drop(self.handle, int(mode), int(radius)), self.handle)

    @property
    def t(self) -> int:
        v = ctypes.c_uint64()
        _check(lib().sim_get_step(self.handle, ctypes.byref(v)), self.handle)
        return int(v.value)

    @t.setter
    def t(self, value: int):
        _check(lib().sim_set_step(self.handle, int(value)), self.handle)

    def set_plan(self, tile_rows=0, tile_width=0, temporal=0, skip_static=0, sparse=0, graph=0, resident=0):
        p = SimPlan(tile_rows, tile_width, temporal, skip_static, sparse, graph, resident)
        _check(lib().sim_set_plan(self.handle, ctypes.byref(p)), self.handle)

    def plan(self) -> dict:
        p = SimPlan()
        _check(lib().sim_get_plan(self.handle, ctypes.byref(p)), self.handle)
        return {"tile_rows": p.tile_rows, "tile_width": p.tile_width, "temporal": p.temporal,
                "sparse": p.sparse,
                "skip_static": p.skip_static, "graph": p.graph, "resident": p.resident}

    def autotune(self, T_probe: int = 10, allow_skip: bool = True, allow_sparse: bool = False) -> list:
        """Time every candidate plan on this batch (states and step counter
        unchanged) and adopt the fastest; returns [(plan dict, ms/step)].
        Plans are ranked on the T_probe steps alone: probe a representative
        stretch of the run (the fire sizes decide between plans)."""
        res = (SimTuneResult * 32)()
        n = ctypes.c_int32(0)
        _check(lib().sim_autotune(self.handle, _ptr(self.states), int(T_probe), int(allow_skip),
                                  int(allow_sparse), res, 32, ctypes.byref(n), self._s()), self.handle)
        out = []
        for i in range(n.value):
            p = res[i].plan
            out.append(({"tile_rows": p.tile_rows, "tile_width": p.tile_width,
                         "skip_static": p.skip_static, "sparse": p.sparse, "temporal": p.temporal,
                         "resident": p.resident},
                        float(res[i].ms_per_step)))
        return out

    # ---------------------------------------------------------- size classes
    @staticmethod
    def _classes(arr, n) -> list:
        return [{"size_class": int(c.size_class), "n_env": int(c.n_env), "n_cells": int(c.n_cells),
                 "plan": _plan_dict(c.plan), "ms_per_step": float(c.ms_per_step),
                 "from_cache": bool(c.from_cache)} for c in arr[:n]]

    def set_class_plan(self, size_class: int, tile_rows=0, tile_width=0, temporal=0, skip_static=0, sparse=0,
                       resident=0):
        """Give the envs of one size class (larger side in (2^(c+4), 2^(c+5)])
        their own plan; sim_step then runs the classes in turn."""
        p = SimPlan(tile_rows, tile_width, temporal, skip_static, sparse, 0, resident)
        _check(lib().sim_set_class_plan(self.handle, int(size_class), ctypes.byref(p)), self.handle)

    def class_plans(self) -> list:
        """The size classes present and their plans."""
        arr = (SimClassPlan * N_SIZE_CLASSES)()
        n = ctypes.c_int32(0)
        _check(lib().sim_get_class_plans(self.handle, arr, N_SIZE_CLASSES, ctypes.byref(n)), self.handle)
        return self._classes(arr, n.value)

    def autotune_classes(self, T_probe: int = 10, allow_skip: bool = True, allow_sparse: bool = False,
                         cache_path: str = None) -> list:
        """Tune a plan per size class (each class timed alone; states and step
        counter unchanged), looking plans up in / appending them to the text
        file cache_path when given; returns class_plans()."""
        arr = (SimClassPlan * N_SIZE_CLASSES)()
        n = ctypes.c_int32(0)
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().sim_autotune_classes(self.handle, _ptr(self.states), int(T_probe), int(allow_skip),
                                          int(allow_sparse), path, arr, N_SIZE_CLASSES, ctypes.byref(n),
                                          self._s()), self.handle)
        return self._classes(arr, n.value)

    # ------------------------------------------------------------- relaxed
    def relaxed_init(self):
        U = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        B = torch.empty_like(U)
        _check(lib().sim_relaxed_init(self.handle, _ptr(U), _ptr(B), self._s()), self.handle)
        return U, B

    def relaxed_workspace(self, T: int, ckpt_every: int) -> torch.Tensor:
        n = lib().sim_relaxed_workspace_bytes(self.handle, int(T), int(ckpt_every))
        return torch.empty(max(int(n), 1), dtype=torch.uint8, device=self.device)

    def relaxed_fwd(self, params: SimParams, U, B, T, ckpt_every, ws, form: str = "product"):
        _check(lib().sim_step_relaxed_fwd(self.handle, ctypes.byref(params), _ptr(U), _ptr(B),
                                          int(T), int(ckpt_every), _form(form), _ptr(ws), ws.numel(),
                                          self._s()), self.handle)

    def relaxed_loss(self, U_T, target, scale: float = 1.0, want_grad: bool = True):
        """Soft-IoU loss: (per-env losses float32 [n_env], seed scale x dL/dU_T
        or None, objective float64 [1] = scale x sum of the per-env losses)."""
        loss = torch.empty(self.n_env, dtype=torch.float32, device=self.device)
        obj = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.empty_like(U_T) if want_grad else None
        _check(lib().sim_relaxed_loss(self.handle, _ptr(U_T), _ptr(target), _ptr(loss), _ptr(g),
                                      float(scale), _ptr(obj), self._s()), self.handle)
        return loss, g, obj

    def relaxed_loss_noalloc(self, U_T, target, loss, gU_T, objective, scale: float = 1.0):
        """Soft-IoU loss into caller-given outputs (loss float32 [n_env], gU_T
        float64 like U_T or None, objective float64 [1] or None), with the
        library's static scratch: no device allocation on this path."""
        _check(lib().sim_relaxed_loss_noalloc(self.handle, _ptr(U_T), _ptr(target), _ptr(loss), _ptr(gU_T),
                                              float(scale), _ptr(objective), self._s()), self.handle)

    def relaxed_loss_bce(self, U_T, target, pool: int = 8, mse_weight: float = 1.0, eps: float = 1e-6,
                         scale: float = 1.0, want_grad: bool = True):
        """Per-env BCE of the clipped soft scar plus mse_weight x MSE of its
        pool x pool block means; returns (losses, scale x dL/dU_T or None,
        objective float64 [1] = scale x sum of the losses)."""
        loss = torch.empty(self.n_env, dtype=torch.float32, device=self.device)
        obj = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.empty_like(U_T) if want_grad else None
        _check(lib().sim_relaxed_loss_bce(self.handle, _ptr(U_T), _ptr(target), int(pool),
                                          float(mse_weight), float(eps), _ptr(loss), _ptr(g),
                                          float(scale), _ptr(obj), self._s()), self.handle)
        return loss, g, obj

    def relaxed_loss_any(self, kind: str, U_T, target, scale: float = 1.0, **kw):
        if kind == "iou":
            return self.relaxed_loss(U_T, target, scale=scale)
        if kind == "bce":
            return self.relaxed_loss_bce(U_T, target, scale=scale, **kw)
        raise ValueError("loss must be 'iou' or 'bce', got %r" % (kind,))

    def relaxed_bwd(self, params: SimParams, gU_T, gB_T, T, ckpt_every, ws,
                    form: str = "product") -> torch.Tensor:
        grad = torch.empty(N_THETA, dtype=torch.float64, device=self.device)
        _check(lib().sim_step_relaxed_bwd(self.handle, ctypes.byref(params), _ptr(gU_T), _ptr(gB_T),
                                          int(T), int(ckpt_every), _form(form), _ptr(ws), ws.numel(),
                                          _ptr(grad), self._s()), self.handle)
        return grad


class SimRlConfig(ctypes.Structure):
    _fields_ = [("obs_radius", ctypes.c_int32), ("drop_radius", ctypes.c_int32),
                ("water_capacity", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("burn_penalty", ctypes.c_float), ("extinguish_bonus", ctypes.c_float),
                ("single_launch", ctypes.c_int32)]


class RLEnv:
    """The air-tanker scenario over a FireSim: one agent per env, egocentric
    observations, water drops (BURNING -> BURNT), reward -burn_penalty x
    burning cells and +extinguish_bonus when the fire is out.  Every part of
    reset and step runs in the library's kernels on the simulator's stream.

    Actions: int32 [n_env], bits 0-3 move (0 stay, 1..8 direction k = move-1,
    k = 0 east, counter-clockwise), bit 4 opens the valve.  Agents: int32
    [n_env, 8] (row, col, water, steps, done, last_count, pad, pad).

    single_launch: each step is one kernel launch when every env fits it
    (W % 4 == 0 and up to about 5,900 cells, e.g. 64 x 64: the env's state
    is held in LDS and stepped in place); otherwise, or with
    single_launch=False, the act, step (under the simulator's launch plan)
    and observation kernels run apart.  Both give the same results."""

    def __init__(self, sim: "FireSim", obs_radius: int = 2, drop_radius: int = 1, water_capacity: int = 10,
                 max_steps: int = 100, burn_penalty: float = 0.1, extinguish_bonus: float = 10.0,
                 single_launch: bool = True):
        self.sim = sim
        self.cfg = SimRlConfig(obs_radius, drop_radius, water_capacity, max_steps, burn_penalty,
                               extinguish_bonus, int(bool(single_launch)))
        dev = sim.device
        side = 2 * obs_radius + 1
        self.agents = torch.zeros((sim.n_env, 8), dtype=torch.int32, device=dev)
        self.obs = torch.empty((sim.n_env, side * side), dtype=torch.uint8, device=dev)
        self.reward = torch.zeros(sim.n_env, dtype=torch.float32, device=dev)
        self.done = torch.zeros(sim.n_env, dtype=torch.int32, device=dev)

    def reset(self, episode: int, mask: Optional[torch.Tensor] = None):
        if mask is not None:
            mask = mask.to(device=self.sim.device, dtype=torch.int32).contiguous()
            if tuple(mask.shape) != (self.sim.n_env,):
                raise ValueError("mask must be [n_env]")
        _check(lib().sim_rl_reset(self.sim.handle, ctypes.byref(self.cfg), _ptr(self.sim.states),
                                  _ptr(self.agents), _ptr(mask), int(episode), _ptr(self.obs),
                                  _ptr(self.done), self.sim._s()), self.sim.handle)
        return self.obs, self.done

    def step(self, actions: torch.Tensor):
        actions = actions.to(device=self.sim.device, dtype=torch.int32).contiguous()
        if tuple(actions.shape) != (self.sim.n_env,):
            raise ValueError("actions must be [n_env]")
        _check(lib().sim_rl_step(self.sim.handle, ctypes.byref(self.cfg), _ptr(self.sim.states),
                                 _ptr(self.agents), _ptr(actions), _ptr(self.obs), _ptr(self.reward),
                                 _ptr(self.done), self.sim._s()), self.sim.handle)
        return self.obs, self.reward, self.done


class RelaxedCalibrationLoss(torch.autograd.Function):
    """Mean per-env loss of T relaxed steps as a function of the 17
    parameters theta (float64 CPU tensor), with the library's adjoint as the
    backward.  forward(theta, sim, target, T, ckpt_every, form, loss, loss_kw)
    -> scalar; form is "product" or "exp", loss "iou" (soft IoU) or "bce"
    (BCE + pooled MSE, loss_kw: pool, mse_weight, eps)."""

    @staticmethod
    def forward(ctx, theta, sim: FireSim, target, T: int, ckpt_every: int = 10, form: str = "product",
                loss: str = "iou", loss_kw: Optional[dict] = None):
        p = params_with_theta(sim.params, theta.detach().cpu().tolist())
        U, B = sim.relaxed_init()
        ws = sim.relaxed_workspace(T, ckpt_every)
        sim.relaxed_fwd(p, U, B, T, ckpt_every, ws, form)
        _, gU, obj = sim.relaxed_loss_any(loss, U, target, scale=1.0 / sim.n_env, **(loss_kw or {}))
        ctx.sim, ctx.p, ctx.T, ctx.k, ctx.ws, ctx.gU, ctx.form = sim, p, T, ckpt_every, ws, gU, form
        return obj.cpu().reshape(())   # the library's fp64 mean over envs

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.sim.relaxed_bwd(ctx.p, ctx.gU, None, ctx.T, ctx.k, ctx.ws, ctx.form)
        return g.cpu() * grad_out, None, None, None, None, None, None, None


def calibrate(sim: FireSim, target, T: int, theta0, steps: int = 50, lr: float = 0.02,
              ckpt_every: int = 10, form: str = "product", loss: str = "iou",
              loss_kw: Optional[dict] = None, fixed: Sequence[int] = (),
              lower=None, upper=None, callback=None):
    """Gradient-based parameter calibration: Adam on the 17 parameters against
    the observed scars `target`, each iteration one relaxed forward + adjoint
    in the library.  Parameters listed in `fixed` are not updated; after each
    update theta is clamped to [lower, upper] (default: p_continue and the
    probabilities in [0, 1], the rest unbounded, p_base >= 0).  Returns
    (theta, losses)."""
    theta = torch.tensor([float(v) for v in theta0], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([theta], lr=lr)
    lo = torch.full((N_THETA,), -float("inf"), dtype=torch.float64)
    hi = torch.full((N_THETA,), float("inf"), dtype=torch.float64)
    lo[0], lo[4], lo[5], hi[5] = 0.0, 0.0, 0.0, 1.0
    lo[6:] = -0.99
    if lower is not None:
        lo = torch.as_tensor(lower, dtype=torch.float64)
    if upper is not None:
        hi = torch.as_tensor(upper, dtype=torch.float64)
    mask = torch.ones(N_THETA, dtype=torch.float64)
    for i in fixed:
        mask[i] = 0.0
    losses = []
    for it in range(steps):
        opt.zero_grad()
        L = RelaxedCalibrationLoss.apply(theta, sim, target, T, ckpt_every, form, loss, loss_kw)
        L.backward()
        theta.grad.mul_(mask)
        opt.step()
        with torch.no_grad():
            theta.copy_(torch.maximum(torch.minimum(theta, hi), lo))
        losses.append(float(L.detach()))
        if callback is not None:
            callback(it, losses[-1], theta.detach().clone())
    return theta.detach(), losses
