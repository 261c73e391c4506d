"""The stochastic-step oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/oracle_sanitize_driver.c and oracle/fire_oracle.c are compiled together
with gcc -fsanitize=address,undefined (host code only, no GPU) and run on
batches that exercise every path of the oracle's step: ragged and odd grids,
drops of both modes at corners and off the grid, per-env and per-cell wind
series, static per-cell wind, several threads.  Any sanitizer report aborts
the driver; its final states and counts must equal the regular oracle's.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import firegen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")
OUT_DIR = os.path.join(ROOT, "oracle", "_build")
EXE = os.path.join(OUT_DIR, "oracle_sanitize")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


@pytest.fixture(scope="module")
def driver():
    os.makedirs(OUT_DIR, exist_ok=True)
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-pthread", "-ffp-contract=off",
                           "-fno-fast-math", "-frounding-math", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", EXE, DRIVER, "-lm"])
    return EXE


def _write_input(path, batch, params, seed, T, t0=0, threads=1, actions=None, env_series=None,
                 cell_series=None, drop_mode=0, drop_radius=2):
    flags = (1 if actions is not None else 0) | (2 if env_series is not None else 0) | \
        (4 if cell_series is not None else 0) | (8 if batch.wind_cell is not None else 0)
    ign = np.ascontiguousarray(batch.ignitions, np.int32).reshape(-1, 3)
    with open(path, "wb") as f:
        f.write(np.array([batch.n_env, ign.shape[0], T, threads, drop_mode, drop_radius, flags],
                         np.int32).tobytes())
        f.write(np.array([batch.n_cells], np.int64).tobytes())
        f.write(np.array([seed, t0], np.uint64).tobytes())
        f.write(bytes(oracle.params_struct(params)))
        f.write(np.asarray(params.veg, np.float32).tobytes())
        f.write(np.array([batch.unburnable_mask], np.uint32).tobytes())
        f.write(bytes(oracle.envs_struct(batch)))
        f.write(np.ascontiguousarray(batch.cls, np.uint8).tobytes())
        f.write(np.ascontiguousarray(batch.den, np.float32).tobytes())
        f.write(np.ascontiguousarray(batch.elev, np.float32).tobytes())
        if batch.wind_cell is not None:
            f.write(np.ascontiguousarray(batch.wind_cell, np.float32).tobytes())
        f.write(ign.tobytes())
        for a in (actions, env_series, cell_series):
            if a is not None:
                f.write(np.ascontiguousarray(a).tobytes())


def _run(driver, tmp_path, batch, params, seed, T, **kw):
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(inp, batch, params, seed, T, **kw)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, inp, out], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    raw = open(out, "rb").read()
    n, ne = batch.n_cells, batch.n_env
    states = np.frombuffer(raw[:n], np.uint8)
    counts = np.frombuffer(raw[n:n + 4 * T * ne], np.int32).reshape(T, ne)
    rest = np.frombuffer(raw[n + 4 * T * ne:], np.float32)
    return states, counts, rest[:4096], rest[4096:]


def _reference(batch, params, seed, T, threads=1, actions=None, env_series=None, cell_series=None,
               drop_mode=0, drop_radius=2):
    sim = oracle.Sim(batch, params, seed=seed)
    cnt = sim.step(T, actions=actions, counts=True, threads=threads, wind_env_series=env_series,
                   wind_cell_series=cell_series, drop_mode=drop_mode, drop_radius=drop_radius)
    return sim.states, cnt


def _params(seed=0, **kw):
    rng = np.random.default_rng(seed)
    return firegen.Params(p_base=0.9, veg=tuple(float(v) for v in firegen.veg_table(rng))).replace(**kw)


def test_sanitized_oracle_ragged_batch_with_drops(driver, tmp_path):
    batch = firegen.landscape_batch(31, [(1, 1), (3, 5), (37, 53), (16, 16), (7, 257)])
    params = _params(1)
    T = 30
    acts = firegen.random_actions(5, batch, T, p_none=0.3)
    acts[3, 2] = (36 << 16) | 52          # far corner
    acts[4, 2] = (40 << 16) | 3           # row off the grid: no drop
    for mode, radius in ((0, 2), (1, 0), (1, 3)):
        got = _run(driver, tmp_path, batch, params, 11, T, threads=3, actions=acts, drop_mode=mode,
                   drop_radius=radius)
        want = _reference(batch, params, 11, T, threads=1, actions=acts, drop_mode=mode,
                          drop_radius=radius)
        assert np.array_equal(got[0], want[0])
        assert np.array_equal(got[1], want[1])


def test_sanitized_oracle_wind_series_and_cell_wind(driver, tmp_path):
    params = _params(2, slope_mode=1)
    batch = firegen.landscape_batch(32, [(20, 24), (9, 12)])
    T = 20
    es = firegen.wind_series(3, batch, T)
    got = _run(driver, tmp_path, batch, params, 5, T, env_series=es)
    want = _reference(batch, params, 5, T, env_series=es)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])

    cb = firegen.landscape_batch(33, [(24, 20), (12, 8)], per_cell_wind=True)
    cs = firegen.wind_series(4, cb, T, per_cell=True)
    got = _run(driver, tmp_path, cb, params, 6, T, threads=2, cell_series=cs)
    want = _reference(cb, params, 6, T, threads=2, cell_series=cs)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    got = _run(driver, tmp_path, cb, params, 6, T)
    want = _reference(cb, params, 6, T)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_sanitized_exp_and_atan_match(driver, tmp_path):
    batch = firegen.uniform_batch(4, 4)
    _, _, ye, ya = _run(driver, tmp_path, batch, firegen.Params(), 0, 1)
    xs = np.array([np.float32(-100.0) + np.float32(0.05) * np.float32(i) for i in range(4096)], np.float32)
    assert np.array_equal(ye.view(np.uint32), oracle.exp_c(xs).view(np.uint32))
    assert np.array_equal(ya.view(np.uint32), oracle.atan_c(xs).view(np.uint32))
