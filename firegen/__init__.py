"""Seeded synthetic inputs for the fire-spread cellular automaton.

This module only *generates inputs* (land cover, fuel density, elevation,
wind, ignitions, suppression actions, parameter sets).  It holds none of the
model's arithmetic, so both the CPU oracle and the GPU library may be fed from
it.  The real inputs of the paper (ESA WorldCover land cover, a Copernicus
DEM, the Bear 2020 fire) are not available; these generators stand in for them
with the same structure: an 11-class land-cover legend in spatially coherent
patches, a density modifier in [-1, 1], fractal terrain, and per-env or
per-cell wind given by speed and direction.

Layout of a batch: every per-cell array is packed env after env, each env
row-major (H rows of W cells); env e occupies cells [offset[e], offset[e] +
H[e]*W[e]).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

try:
    import scipy.fft as _fft

    def _rfft2(a):
        return _fft.rfft2(a, workers=8)

    def _irfft2(a, s):
        return _fft.irfft2(a, s=s, workers=8)
except ImportError:  # pragma: no cover
    def _rfft2(a):
        return np.fft.rfft2(a)

    def _irfft2(a, s):
        return np.fft.irfft2(a, s=s)


# The 11-class WorldCover legend, in the paper's colour-definition order.
CLASS_NAMES = ("tree", "shrub", "grass", "crop", "built", "bare", "snow", "water",
               "wetland", "mangrove", "lichen")
N_CLASSES = 11
TREE, SHRUB, GRASS, CROP, BUILT, BARE, SNOW, WATER, WETLAND, MANGROVE, LICHEN = range(11)
# Classes that hold no fuel (the model's "no fuel" cells).
UNBURNABLE_CLASSES = (BARE, SNOW, WATER)
UNBURNABLE_MASK = sum(1 << c for c in UNBURNABLE_CLASSES)

# Rank-quantisation of a smoothed noise field into classes: classes are laid
# out along the noise value in this order, each taking this fraction of cells.
CLASS_ORDER = (WATER, WETLAND, MANGROVE, CROP, GRASS, SHRUB, TREE, BUILT, LICHEN, BARE, SNOW)
CLASS_FRACTION = (0.06, 0.05, 0.02, 0.12, 0.20, 0.15, 0.25, 0.05, 0.04, 0.04, 0.02)

# State codes (inputs to tests only; the model's transitions live elsewhere).
UNBURNABLE, FLAMMABLE, BURNING, BURNT = 0, 1, 2, 3


@dataclasses.dataclass
class Params:
    """Model parameters (names follow the paper's notation)."""
    p_base: float = 0.58
    alpha_gamma: float = 1.0
    alpha_w1: float = 0.045
    alpha_w2: float = 0.131
    alpha_s: float = 4.5
    p_continue: float = 0.5
    veg: Sequence[float] = tuple([0.0] * N_CLASSES)
    cell_size: float = 30.0
    slope_mode: int = 0  # 0: S = rise / run; 1: S = atan(rise / run) (radians)

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Batch:
    H: np.ndarray          # int32 [n_env]
    W: np.ndarray          # int32 [n_env]
    offset: np.ndarray     # int64 [n_env]
    env_id: np.ndarray     # uint32 [n_env]
    cls: np.ndarray        # uint8 [n_cells]   land-cover class 0..10
    den: np.ndarray        # float32 [n_cells] density modifier mu_den
    elev: np.ndarray       # float32 [n_cells] elevation (m)
    wind_env: np.ndarray   # float32 [n_env, 3]  (V, V cos Theta, V sin Theta)
    wind_cell: Optional[np.ndarray]  # float32 [3, n_cells] or None
    ignitions: np.ndarray  # int32 [n_ign, 3]  (env, row, col)
    unburnable_mask: int = UNBURNABLE_MASK

    @property
    def n_env(self) -> int:
        return int(self.H.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cls.shape[0])

    def env_slice(self, e: int) -> slice:
        o = int(self.offset[e])
        return slice(o, o + int(self.H[e]) * int(self.W[e]))

    def env_view(self, arr: np.ndarray, e: int) -> np.ndarray:
        return arr[self.env_slice(e)].reshape(int(self.H[e]), int(self.W[e]))

    def subset(self, envs: Sequence[int]) -> "Batch":
        """A batch made of the given envs (keeping their env_id)."""
        envs = list(envs)
        H = self.H[envs].copy()
        W = self.W[envs].copy()
        sizes = H.astype(np.int64) * W
        offset = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        take = np.concatenate([np.arange(self.env_slice(e).start, self.env_slice(e).stop)
                               for e in envs]) if envs else np.zeros(0, np.int64)
        ign = []
        for new, e in enumerate(envs):
            rows = self.ignitions[self.ignitions[:, 0] == e]
            for r in rows:
                ign.append((new, r[1], r[2]))
        return Batch(H=H, W=W, offset=offset, env_id=self.env_id[envs].copy(),
                     cls=self.cls[take].copy(), den=self.den[take].copy(),
                     elev=self.elev[take].copy(), wind_env=self.wind_env[envs].copy(),
                     wind_cell=None if self.wind_cell is None else self.wind_cell[:, take].copy(),
                     ignitions=np.array(ign, np.int32).reshape(-1, 3),
                     unburnable_mask=self.unburnable_mask)


# --------------------------------------------------------------------------
# fields
# --------------------------------------------------------------------------
def _freq_radius(H: int, W: int) -> np.ndarray:
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    return np.sqrt(fy * fy + fx * fx)


def smoothed_noise(rng: np.random.Generator, n: int, H: int, W: int, sigma: float) -> np.ndarray:
    """White noise blurred by a periodic Gaussian of std `sigma` cells, [n,H,W] float32."""
    white = rng.standard_normal((n, H, W), dtype=np.float32)
    f = _freq_radius(H, W)
    kernel = np.exp(-2.0 * (math.pi * sigma) ** 2 * f * f).astype(np.float32)
    out = _irfft2(_rfft2(white) * kernel, s=(H, W)).astype(np.float32)
    return out


def fractal_field(rng: np.random.Generator, n: int, H: int, W: int, beta: float = 3.2) -> np.ndarray:
    """Spectral fractal: power spectrum ~ 1/f^beta (amplitude f^(-beta/2)), [n,H,W] float32.
    beta = 2 H + 2 for a fractional Brownian surface of Hurst exponent H; the
    default 3.2 (H = 0.6) is in the range measured for real topography."""
    white = rng.standard_normal((n, H, W), dtype=np.float32)
    f = _freq_radius(H, W)
    f[0, 0] = 1.0
    amp = (f ** (-beta / 2.0)).astype(np.float32)
    amp[0, 0] = 0.0
    return _irfft2(_rfft2(white) * amp, s=(H, W)).astype(np.float32)


def _rescale(a: np.ndarray, lo: float, hi: float) -> np.ndarray:
    amin = a.min(axis=(1, 2), keepdims=True)
    amax = a.max(axis=(1, 2), keepdims=True)
    span = np.where(amax > amin, amax - amin, 1.0)
    return (lo + (a - amin) / span * (hi - lo)).astype(np.float32)


def quantise_classes(field: np.ndarray) -> np.ndarray:
    """Rank-quantise each [H,W] slice into the 11 classes by CLASS_FRACTION."""
    n, H, W = field.shape
    flat = field.reshape(n, -1)
    m = flat.shape[1]
    cum = np.cumsum(CLASS_FRACTION)
    cum[-1] = 1.0 + 1e-9
    q = (np.arange(m, dtype=np.float64) + 0.5) / m
    by_rank = np.asarray(CLASS_ORDER, np.uint8)[np.minimum(np.searchsorted(cum, q, side="right"),
                                                           N_CLASSES - 1)]
    order = np.argsort(flat, axis=1)
    out = np.empty_like(order, dtype=np.uint8)
    np.put_along_axis(out, order, np.broadcast_to(by_rank, order.shape), axis=1)
    return out.reshape(n, H, W)


def veg_table(rng: np.random.Generator) -> np.ndarray:
    """Per-class vegetation modifier mu_veg in [-0.4, 0.4]; 0 for unburnable classes."""
    v = rng.uniform(-0.4, 0.4, N_CLASSES).astype(np.float32)
    for c in UNBURNABLE_CLASSES:
        v[c] = 0.0
    return v


def wind_components(V: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """(V, V cos Theta, V sin Theta) as float32, products taken in float64."""
    V32 = np.asarray(V, np.float32)
    V64 = V32.astype(np.float64)
    th = np.asarray(theta, np.float64)
    return np.stack([V32, (V64 * np.cos(th)).astype(np.float32),
                     (V64 * np.sin(th)).astype(np.float32)], axis=-1)


def wind_series(seed: int, batch: "Batch", S: int, per_cell: bool = False,
                speed_step: float = 0.3, turn_step: float = 0.05) -> np.ndarray:
    """Time-varying wind for steps 0..S-1, as random walks from the batch's
    static wind: per env, V_t = clip(V_0 + walk, 0, 15) m/s and Theta_t =
    Theta_0 + walk (float32 [S][n_env][3]); per cell, every cell's static
    speed is scaled by a common factor walk and its direction turned by a
    common angle walk (float32 [S][3][n_cells])."""
    rng = np.random.default_rng(seed)
    if not per_cell:
        V0 = batch.wind_env[:, 0].astype(np.float64)
        th0 = np.arctan2(batch.wind_env[:, 2], batch.wind_env[:, 1]).astype(np.float64)
        V = np.clip(V0[None, :] + np.cumsum(rng.normal(0, speed_step, (S, batch.n_env)), axis=0), 0, 15)
        th = th0[None, :] + np.cumsum(rng.normal(0, turn_step, (S, batch.n_env)), axis=0)
        return np.ascontiguousarray(wind_components(V, th))
    if batch.wind_cell is not None:
        V0 = batch.wind_cell[0].astype(np.float64)
        th0 = np.arctan2(batch.wind_cell[2], batch.wind_cell[1]).astype(np.float64)
    else:
        V0 = np.concatenate([np.full(int(batch.H[e]) * int(batch.W[e]), batch.wind_env[e, 0], np.float64)
                             for e in range(batch.n_env)])
        th0 = np.concatenate([np.full(int(batch.H[e]) * int(batch.W[e]),
                                      np.arctan2(batch.wind_env[e, 2], batch.wind_env[e, 1]), np.float64)
                              for e in range(batch.n_env)])
    scale = np.clip(1.0 + np.cumsum(rng.normal(0, speed_step / 10, S)), 0.0, 2.0)
    turn = np.cumsum(rng.normal(0, turn_step, S))
    out = np.empty((S, 3, batch.n_cells), np.float32)
    for t in range(S):
        out[t] = wind_components(V0 * scale[t], th0 + turn[t]).T
    return out


# --------------------------------------------------------------------------
# batches
# --------------------------------------------------------------------------
def _pack(sizes: Sequence[tuple]) -> tuple:
    H = np.array([s[0] for s in sizes], np.int32)
    W = np.array([s[1] for s in sizes], np.int32)
    cells = H.astype(np.int64) * W
    offset = np.concatenate([[0], np.cumsum(cells)[:-1]]).astype(np.int64)
    return H, W, offset, int(cells.sum())


def landscape_batch(seed: int, sizes: Sequence[tuple], *, elev_max: float = 500.0,
                    class_sigma: float = 6.0, den_sigma: float = 4.0,
                    ign_range=(1, 5), per_cell_wind: bool = False,
                    env_id_base: int = 0) -> Batch:
    """Land cover from smoothed noise quantised into 11 classes, density in
    [-0.3, 0.3], fractal elevation 0..elev_max m, wind V~U(0,10) m/s and
    Theta~U(0, 2 pi) per env (or a smooth per-cell field), and K~U{ign_range}
    ignitions on burnable cells."""
    rng = np.random.default_rng(seed)
    H, W, offset, n_cells = _pack(sizes)
    n_env = len(sizes)
    cls = np.empty(n_cells, np.uint8)
    den = np.empty(n_cells, np.float32)
    elev = np.empty(n_cells, np.float32)
    wind_cell = np.empty((3, n_cells), np.float32) if per_cell_wind else None
    # group envs of one shape so each group is generated in one batched FFT
    shapes = {}
    for e, s in enumerate(sizes):
        shapes.setdefault((int(s[0]), int(s[1])), []).append(e)
    for (h, w), envs in sorted(shapes.items()):
        for chunk_start in range(0, len(envs), max(1, (1 << 24) // (h * w))):
            chunk = envs[chunk_start:chunk_start + max(1, (1 << 24) // (h * w))]
            m = len(chunk)
            c = quantise_classes(smoothed_noise(rng, m, h, w, class_sigma))
            d = _rescale(smoothed_noise(rng, m, h, w, den_sigma), -0.3, 0.3)
            z = _rescale(fractal_field(rng, m, h, w), 0.0, elev_max)
            if per_cell_wind:
                sp = _rescale(smoothed_noise(rng, m, h, w, max(h, w) / 8.0), 0.0, 10.0)
                th = _rescale(smoothed_noise(rng, m, h, w, max(h, w) / 8.0), 0.0, 2.0 * math.pi)
                wc = wind_components(sp, th)  # [m,h,w,3]
            for k, e in enumerate(chunk):
                sl = slice(int(offset[e]), int(offset[e]) + h * w)
                cls[sl] = c[k].ravel()
                den[sl] = d[k].ravel()
                elev[sl] = z[k].ravel()
                if per_cell_wind:
                    for q in range(3):
                        wind_cell[q, sl] = wc[k, :, :, q].ravel()
    V = rng.uniform(0.0, 10.0, n_env)
    theta = rng.uniform(0.0, 2.0 * math.pi, n_env)
    wind_env = wind_components(V, theta)
    burnable = np.ones(N_CLASSES, bool)
    burnable[list(UNBURNABLE_CLASSES)] = False
    ign = []
    for e in range(n_env):
        sl = slice(int(offset[e]), int(offset[e]) + int(H[e]) * int(W[e]))
        cand = np.flatnonzero(burnable[cls[sl]])
        if cand.size == 0:
            continue
        k = int(rng.integers(ign_range[0], ign_range[1] + 1))
        pick = rng.choice(cand, size=min(k, cand.size), replace=False)
        for p in np.sort(pick):
            ign.append((e, int(p) // int(W[e]), int(p) % int(W[e])))
    return Batch(H=H, W=W, offset=offset,
                 env_id=(np.arange(n_env, dtype=np.uint64) + env_id_base).astype(np.uint32),
                 cls=cls, den=den, elev=elev, wind_env=wind_env, wind_cell=wind_cell,
                 ignitions=np.array(ign, np.int32).reshape(-1, 3))


def uniform_batch(H: int, W: int, *, n_env: int = 1, cls: int = GRASS, den: float = 0.0,
                  elev: float = 0.0, wind=(0.0, 0.0), ignitions=None,
                  env_id_base: int = 0) -> Batch:
    """Flat, homogeneous envs (one class, constant density and elevation, one
    wind (V, Theta)); ignitions default to the centre (H//2, W//2) of every env."""
    Ha, Wa, offset, n_cells = _pack([(H, W)] * n_env)
    if ignitions is None:
        ignitions = [(e, None, None) for e in range(n_env)]
    ign = []
    for e, i, j in ignitions:
        ign.append((e, H // 2 if i is None else i, W // 2 if j is None else j))
    return Batch(H=Ha, W=Wa, offset=offset,
                 env_id=(np.arange(n_env, dtype=np.uint64) + env_id_base).astype(np.uint32),
                 cls=np.full(n_cells, cls, np.uint8), den=np.full(n_cells, den, np.float32),
                 elev=np.full(n_cells, elev, np.float32),
                 wind_env=np.repeat(wind_components(np.array([wind[0]]), np.array([wind[1]])),
                                    n_env, axis=0),
                 wind_cell=None, ignitions=np.array(ign, np.int32).reshape(-1, 3))


def random_actions(seed: int, batch: Batch, T: int, p_none: float = 0.0) -> np.ndarray:
    """One 5x5 suppression drop per env per step at a uniform random centre,
    encoded (row << 16) | col; -1 (no drop) with probability p_none."""
    rng = np.random.default_rng(seed)
    r = (rng.random((T, batch.n_env)) * batch.H[None, :]).astype(np.int32)
    c = (rng.random((T, batch.n_env)) * batch.W[None, :]).astype(np.int32)
    a = (r << 16) | c
    if p_none > 0:
        a = np.where(rng.random((T, batch.n_env)) < p_none, -1, a)
    return a.astype(np.int32)


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def workload_single64() -> tuple:
    """1 env 64x64, all grass (veg 0), density 0, flat, no wind, ignition at
    (32, 32); p_base 0.58, alpha_gamma 1, p_continue 0.5; 100 steps; seed 0."""
    return uniform_batch(64, 64), Params(), 100, 0


def workload_batch256(n_env: int = 1024, side: int = 256, seed: int = 2) -> tuple:
    """1024 envs of 256x256 at 30 m cells, 200 steps, generator seed 2, Philox seed 0."""
    rng = np.random.default_rng(seed + 1000)
    params = Params(veg=tuple(float(v) for v in veg_table(rng)))
    return landscape_batch(seed, [(side, side)] * n_env), params, 200, 0


def uneven_sizes(n_env: int, seed: int, sides=(64, 128, 256, 512)) -> list:
    rng = np.random.default_rng(seed)
    s = rng.choice(np.asarray(sides), size=n_env)
    return [(int(x), int(x)) for x in s]


def workload_uneven(n_env: int = 4096, seed: int = 3, T: int = 300) -> tuple:
    """4096 envs with sides drawn from {64,128,256,512}, 300 steps, one 5x5
    drop per env per step (seed 3)."""
    rng = np.random.default_rng(seed + 1000)
    params = Params(veg=tuple(float(v) for v in veg_table(rng)))
    batch = landscape_batch(seed, uneven_sizes(n_env, seed))
    return batch, params, T, 0, random_actions(seed, batch, T)


def workload_relaxed(n_env: int = 256, side: int = 128, seed: int = 4) -> tuple:
    """256 envs of 128x128 for the relaxed path, T = 100, checkpoints every 10."""
    rng = np.random.default_rng(seed + 1000)
    params = Params(veg=tuple(float(v) for v in veg_table(rng)))
    return landscape_batch(seed, [(side, side)] * n_env), params, 100, 10


def workload_large(n_env: int = 8, side: int = 2048, seed: int = 5) -> tuple:
    """8 envs of 2048x2048, fractal terrain 0..2000 m, per-cell wind, 1000 steps."""
    rng = np.random.default_rng(seed + 1000)
    params = Params(veg=tuple(float(v) for v in veg_table(rng)))
    batch = landscape_batch(seed, [(side, side)] * n_env, elev_max=2000.0, per_cell_wind=True,
                            class_sigma=12.0)
    return batch, params, 1000, 0


def workload_relaxed_large(side: int = 2048, seed: int = 6) -> tuple:
    """1 env of 2048x2048 for the relaxed path (fractal terrain 0..2000 m,
    per-cell wind), T = 500, checkpoints every 10."""
    rng = np.random.default_rng(seed + 1000)
    params = Params(veg=tuple(float(v) for v in veg_table(rng)))
    batch = landscape_batch(seed, [(side, side)], elev_max=2000.0, per_cell_wind=True, class_sigma=12.0)
    return batch, params, 500, 10


def dense_front_states(batch: Batch) -> np.ndarray:
    """A checkerboard of BURNING and FLAMMABLE over every burnable cell
    (UNBURNABLE cells kept): every flammable cell then touches a burning one.
    With p_continue = 1 and a negligible p_base the pattern is stationary, so
    each step evaluates the whole neighbourhood arithmetic at every cell."""
    out = np.empty(batch.n_cells, np.uint8)
    for e in range(batch.n_env):
        H, W = int(batch.H[e]), int(batch.W[e])
        ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        st = np.where((ii + jj) % 2 == 0, BURNING, FLAMMABLE).astype(np.uint8)
        burnable = ~np.isin(batch.env_view(batch.cls, e), UNBURNABLE_CLASSES)
        st[~burnable] = UNBURNABLE
        batch.env_view(out, e)[...] = st
    return out
