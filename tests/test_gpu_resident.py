"""GPU parity of the resident multi-step kernel (plan field `resident`): all
T steps of a sim_step call in one launch, each env held in LDS by one
workgroup.  Bit-exact against the CPU oracle: states, burning counts and
history rows, for every workgroup size.
"""
import numpy as np
import pytest
import torch

import firegen
import oracle

pytestmark = pytest.mark.gpu

fs = pytest.importorskip("paper_2512_06102_amd")

THREADS = [64, 256, 512, 1024]


def _veg(seed):
    return tuple(float(v) for v in firegen.veg_table(np.random.default_rng(seed)))


def _check(sim, ref, got, want, what):
    torch.cuda.synchronize()
    assert np.array_equal(sim.states.cpu().numpy(), ref.states), what
    assert np.array_equal(got, want), what


@pytest.mark.parametrize("threads", THREADS)
@pytest.mark.parametrize("mode,radius", [(0, 2), (1, 2)])
def test_paper_setting_64x64_with_drops(threads, mode, radius):
    """64 envs of 64 x 64 (the paper's vectorised setting), 200 steps with a
    drop in most envs at most steps, split into two calls, in a graph and
    directly."""
    batch = firegen.landscape_batch(61, [(64, 64)] * 64)
    params = firegen.Params(p_base=0.8, veg=_veg(61))
    T = 200
    act = firegen.random_actions(21, batch, T, p_none=0.3)
    ref = oracle.Sim(batch, params, seed=3)
    want = ref.step(T, actions=act, counts=True, threads=8, drop_mode=mode, drop_radius=radius)
    for graph in (1, 0):
        sim = fs.FireSim.from_batch(batch, params, seed=3)
        sim.set_plan(resident=threads, graph=graph)
        sim.set_drop(mode, radius)
        c1 = sim.step(77, actions=torch.from_numpy(act[:77]), counts=True).cpu().numpy()
        c2 = sim.step(T - 77, actions=torch.from_numpy(act[77:]), counts=True).cpu().numpy()
        _check(sim, ref, np.concatenate([c1, c2]), want, (threads, graph))
        assert sim.plan()["resident"] == threads
        assert sim.t == T


@pytest.mark.parametrize("threads", THREADS)
def test_fires_burn_out_without_drops(threads):
    """The paper setting's batch with no drops: every fire is out well before
    step 200, after which an env stops stepping and leaves its count rows at
    0; 200 steps in one call and as 120 + 80 (the second call starts after
    every fire is out), counts after every step and the final states equal
    the oracle's."""
    batch = firegen.landscape_batch(7, [(64, 64)] * 64)
    params = firegen.Params(veg=_veg(7))
    T = 200
    ref = oracle.Sim(batch, params, seed=0)
    want = ref.step(T, counts=True, threads=8)
    last = max(int(np.flatnonzero(want[:, e]).max(initial=-1)) for e in range(batch.n_env))
    assert 0 < last < 120, last  # every fire is out before the split
    for split in ((T,), (120, 80)):
        sim = fs.FireSim.from_batch(batch, params, seed=0)
        sim.set_plan(resident=threads, graph=1)
        got = np.concatenate([sim.step(n, counts=True).cpu().numpy() for n in split])
        _check(sim, ref, got, want, (threads, split))


@pytest.mark.parametrize("threads", THREADS)
def test_many_20x20_envs_with_drops(threads):
    """1024 envs of 20 x 20 (the RL layer's size), water drops, 60 steps."""
    batch = firegen.landscape_batch(62, [(20, 20)] * 1024)
    params = firegen.Params(p_base=0.9, veg=_veg(62))
    T = 60
    act = firegen.random_actions(22, batch, T, p_none=0.2)
    ref = oracle.Sim(batch, params, seed=8)
    want = ref.step(T, actions=act, counts=True, threads=8, drop_mode=1, drop_radius=2)
    sim = fs.FireSim.from_batch(batch, params, seed=8)
    sim.set_plan(resident=threads)
    sim.set_drop(1, 2)
    got = sim.step(T, actions=torch.from_numpy(act), counts=True).cpu().numpy()
    _check(sim, ref, got, want, threads)


MIXED = [(64, 64), (20, 20), (8, 8), (36, 52), (4, 4), (92, 92), (12, 100), (1, 4), (5, 8)]


@pytest.mark.parametrize("threads", THREADS)
def test_mixed_small_envs_edges_and_corners(threads):
    """Envs from 1 x 4 up to the largest square that fits in 160 KiB of LDS
    (92 x 92), drops at the
    corners and centres outside the grid, a steep spread probability."""
    batch = firegen.landscape_batch(63, MIXED)
    params = firegen.Params(p_base=0.95, veg=_veg(63))
    T = 90
    act = firegen.random_actions(23, batch, T, p_none=0.3)
    act[3, :] = 0                                     # top-left corner
    act[4, :] = ((batch.H - 1) << 16) | (batch.W - 1)  # bottom-right corner
    act[5, :] = (batch.H + 3) << 16                   # outside the grid: no drop
    ref = oracle.Sim(batch, params, seed=9)
    want = ref.step(T, actions=act, counts=True, threads=8, drop_mode=0, drop_radius=4)
    sim = fs.FireSim.from_batch(batch, params, seed=9)
    sim.set_plan(resident=threads)
    sim.set_drop(0, 4)
    got = sim.step(T, actions=torch.from_numpy(act), counts=True).cpu().numpy()
    _check(sim, ref, got, want, threads)


def test_no_actions_no_counts_and_resume():
    """Calls without actions or counts; a second handle resumes from the
    saved states at the saved step counter."""
    batch = firegen.landscape_batch(64, [(64, 64)] * 8 + [(32, 48)] * 8)
    params = firegen.Params(p_base=0.75, veg=_veg(64))
    ref = oracle.Sim(batch, params, seed=11)
    ref.step(50, threads=8)
    sim = fs.FireSim.from_batch(batch, params, seed=11)
    sim.set_plan(resident=512)
    sim.step(20)
    saved = sim.states.clone()
    sim2 = fs.FireSim.from_batch(batch, params, seed=11)
    sim2.set_plan(resident=256, graph=1)
    sim2.states.copy_(saved)
    sim2.t = 20
    sim2.step(30)
    torch.cuda.synchronize()
    assert np.array_equal(sim2.states.cpu().numpy(), ref.states)


@pytest.mark.parametrize("per_cell", [False, True])
def test_wind_series_and_history(per_cell):
    """A per-env or per-cell wind series indexed by the absolute step, and
    sim_step_history (one launch per step) against the oracle's rows."""
    batch = firegen.landscape_batch(65, [(64, 64), (40, 60), (20, 20)], per_cell_wind=per_cell)
    params = firegen.Params(p_base=0.9, veg=_veg(65))
    T = 40
    ser = firegen.wind_series(7, batch, T, per_cell=per_cell, speed_step=1.0, turn_step=0.3)
    kw = {"wind_cell_series" if per_cell else "wind_env_series": ser}
    act = firegen.random_actions(24, batch, T, p_none=0.4)
    ref = oracle.Sim(batch, params, seed=12)
    rows, want = ref.step(T, actions=act, counts=True, threads=6, drop_mode=1, drop_radius=3, history=True, **kw)
    dev = torch.from_numpy(ser).cuda()
    for hist_mode in (False, True):
        sim = fs.FireSim.from_batch(batch, params, seed=12)
        sim.set_plan(resident=256, graph=1)
        sim.set_drop(1, 3)
        sim.set_wind_series(cell_series=dev) if per_cell else sim.set_wind_series(env_series=dev)
        if hist_mode:
            hist, cnt = sim.step_history(T, actions=torch.from_numpy(act), counts=True)
            torch.cuda.synchronize()
            assert np.array_equal(hist.cpu().numpy(), rows)
            assert np.array_equal(cnt.cpu().numpy(), want)
            assert np.array_equal(sim.states.cpu().numpy(), rows[-1])
        else:
            got = sim.step(T, actions=torch.from_numpy(act), counts=True).cpu().numpy()
            _check(sim, ref, got, want, per_cell)


def test_static_per_cell_wind_and_slope_angle():
    batch = firegen.landscape_batch(66, [(64, 64)] * 4 + [(24, 36)] * 4, per_cell_wind=True)
    params = firegen.Params(p_base=0.85, veg=_veg(66), slope_mode=1)
    T = 70
    ref = oracle.Sim(batch, params, seed=13)
    want = ref.step(T, counts=True, threads=8)
    sim = fs.FireSim.from_batch(batch, params, seed=13)
    sim.set_plan(resident=1024)
    got = sim.step(T, counts=True).cpu().numpy()
    _check(sim, ref, got, want, "per-cell wind")


def test_rejections():
    """Batches the kernel cannot hold and bad plan values raise SimError; the
    handle keeps its previous plan."""
    for sizes in ([(128, 128)], [(96, 96)], [(64, 64), (40, 42)], [(1, 30000)]):
        sim = fs.FireSim.from_batch(firegen.landscape_batch(67, sizes), firegen.Params(), seed=0)
        with pytest.raises(fs.SimError):
            sim.set_plan(resident=256)
        assert sim.plan()["resident"] == 0
    sim = fs.FireSim.from_batch(firegen.landscape_batch(68, [(64, 64)]), firegen.Params(), seed=0)
    for kw in (dict(resident=300), dict(resident=128), dict(resident=256, temporal=4, tile_width=64)):
        with pytest.raises(fs.SimError):
            sim.set_plan(**kw)
    sim.set_plan(resident=512)
    sim.step(3)
    torch.cuda.synchronize()


def test_autotune_tries_resident_plans():
    batch = firegen.landscape_batch(69, [(64, 64)] * 16)
    sim = fs.FireSim.from_batch(batch, firegen.Params(), seed=0)
    res = sim.autotune(T_probe=20, allow_skip=True, allow_sparse=True)
    assert sorted(p["resident"] for p, _ in res if p["resident"]) == THREADS
    big = fs.FireSim.from_batch(firegen.landscape_batch(70, [(128, 128)]), firegen.Params(), seed=0)
    res = big.autotune(T_probe=5, allow_skip=True, allow_sparse=True)
    assert all(p["resident"] == 0 for p, _ in res)


@pytest.mark.parametrize("per_cell", [False, True])
def test_long_wind_series_across_staging_chunks(per_cell):
    """Drops and wind exponents are staged 64 steps at a time: a 150-step
    per-env (or per-cell) wind series with drops, split 70 + 80 so that both
    calls cross a chunk boundary at a step that is not a multiple of 64 of
    the run."""
    batch = firegen.landscape_batch(73, [(64, 64)] * 6 + [(20, 20)] * 10, per_cell_wind=per_cell)
    params = firegen.Params(p_base=0.7, veg=_veg(73))
    T = 150
    ser = firegen.wind_series(10, batch, T, per_cell=per_cell, speed_step=1.5, turn_step=0.4)
    kw = {"wind_cell_series" if per_cell else "wind_env_series": ser}
    act = firegen.random_actions(25, batch, T, p_none=0.6)
    ref = oracle.Sim(batch, params, seed=14)
    want = ref.step(T, actions=act, counts=True, threads=8, **kw)
    sim = fs.FireSim.from_batch(batch, params, seed=14)
    sim.set_plan(resident=512, graph=1)
    dev = torch.from_numpy(ser).cuda()
    sim.set_wind_series(cell_series=dev) if per_cell else sim.set_wind_series(env_series=dev)
    got = [sim.step(n, actions=torch.from_numpy(np.ascontiguousarray(a)), counts=True).cpu().numpy()
           for n, a in ((70, act[:70]), (T - 70, act[70:]))]
    _check(sim, ref, np.concatenate(got), want, per_cell)


def test_handles_of_different_sizes_share_the_kernel():
    """The kernel's LDS limit is shared by all handles: a handle of 64 x 64
    envs still runs its resident plan after a handle of 20 x 20 envs was
    created (and stepped) after it."""
    big = firegen.landscape_batch(74, [(64, 64)] * 8)
    small = firegen.landscape_batch(75, [(20, 20)] * 8)
    params = firegen.Params(p_base=0.8, veg=_veg(74))
    sim_big = fs.FireSim.from_batch(big, params, seed=15)
    sim_big.set_plan(resident=1024)
    sim_small = fs.FireSim.from_batch(small, params, seed=15)
    sim_small.set_plan(resident=64)
    sim_small.step(20)
    got = sim_big.step(40, counts=True).cpu().numpy()
    ref = oracle.Sim(big, params, seed=15)
    want = ref.step(40, counts=True, threads=8)
    _check(sim_big, ref, got, want, "big after small")
    ref_s = oracle.Sim(small, params, seed=15)
    ref_s.step(20, threads=8)
    torch.cuda.synchronize()
    assert np.array_equal(sim_small.states.cpu().numpy(), ref_s.states)


def test_default_plan_takes_resident_for_small_envs():
    """A new handle starts with the resident plan when every env fits it and
    the batch needs at most two rounds of workgroups (the measured choices:
    1024 lanes for 64 envs of 64 x 64, 512 for 1024 of them, none for 4096,
    64 lanes for 20 x 20 envs), and with the tiled plan otherwise."""
    params = firegen.Params()
    cases = [([(64, 64)] * 64, 1024), ([(64, 64)] * 1024, 512), ([(64, 64)] * 4096, 0),
             ([(20, 20)] * 512, 64), ([(40, 40)] * 64, 256), ([(128, 128)] * 4, 0), ([(64, 64), (40, 42)], 0)]
    for sizes, want in cases:
        sim = fs.FireSim.from_batch(firegen.landscape_batch(76, sizes), params, seed=0)
        plan = sim.plan()
        assert plan["resident"] == want, (sizes[0], len(sizes), plan)
        assert (plan["tile_rows"], plan["tile_width"], plan["skip_static"], plan["sparse"]) == (4, 64, 1, 1)
        del sim
