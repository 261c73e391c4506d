"""GPU parity of the stochastic step: bit-exact against the CPU oracle.

Every test drives the HIP library through its C ABI (ctypes binding) and
compares states and burning counts byte for byte with the oracle on the same
seeded inputs.
"""
import numpy as np
import pytest
import torch

import firegen
import oracle

pytestmark = pytest.mark.gpu

fs = pytest.importorskip("paper_2512_06102_amd")


def _veg(seed):
    return tuple(float(v) for v in firegen.veg_table(np.random.default_rng(seed)))


def _run_both(batch, params, T, seed=0, actions=None, plan=None, split=None):
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    if plan:
        sim.set_plan(**plan)
    ref = oracle.Sim(batch, params, seed=seed)
    assert np.array_equal(sim.states.cpu().numpy(), ref.states), "initial states differ"
    splits = split or [T]
    got_c, want_c = [], []
    s0 = 0
    for Tk in splits:
        a = None if actions is None else actions[s0:s0 + Tk]
        c = sim.step(Tk, actions=None if a is None else torch.from_numpy(np.ascontiguousarray(a)),
                     counts=True)
        got_c.append(c.cpu().numpy())
        want_c.append(ref.step(Tk, actions=a, counts=True, threads=8))
        s0 += Tk
    torch.cuda.synchronize()
    return sim, ref, np.concatenate(got_c), np.concatenate(want_c)


def test_exp_bit_exact_exhaustive():
    """Device exp equals the oracle's on every fp32 in [-87, 88] (and a tail)."""
    lo = np.array([-87.5], np.float32).view(np.uint32)[0]
    hi = np.array([88.5], np.float32).view(np.uint32)[0]
    chunk = 1 << 26
    for neg, top in ((False, hi), (True, lo)):
        for start in range(0, int(top & 0x7FFFFFFF) + 1, chunk):
            bits = np.arange(start, min(start + chunk, int(top & 0x7FFFFFFF) + 1), dtype=np.uint32)
            if neg:
                bits |= np.uint32(0x80000000)
            x = bits.view(np.float32)
            want = oracle.exp_c(x)
            got = fs.debug_exp(torch.from_numpy(x).cuda()).cpu().numpy()
            bad = np.flatnonzero(got.view(np.uint32) != want.view(np.uint32))
            assert bad.size == 0, (x[bad[:5]], got[bad[:5]], want[bad[:5]])


def test_philox_bit_exact():
    rng = np.random.default_rng(0)
    n = 1 << 20
    ctr = rng.integers(0, 2**32, (n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, (n, 2), dtype=np.uint64).astype(np.uint32)
    got = fs.debug_philox(torch.from_numpy(ctr.view(np.int32)).cuda(),
                          torch.from_numpy(key.view(np.int32)).cuda()).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.philox_blocks(ctr, key))


def test_single_grid_64_every_step():
    """1 env 64x64, all grass, flat, no wind, ignition at (32, 32), p_base 0.58,
    p_continue 0.5, seed 0: states equal after every one of 100 steps."""
    batch, params, T, seed = firegen.workload_single64()
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    ref = oracle.Sim(batch, params, seed=seed)
    for t in range(T):
        c = sim.step(1, counts=True)
        rc = ref.step(1, counts=True)
        assert np.array_equal(sim.states.cpu().numpy(), ref.states), "step %d" % t
        assert np.array_equal(c.cpu().numpy(), rc), "count at step %d" % t
    assert sim.t == T


def test_p_one_chebyshev_square_on_gpu():
    batch, params, T, seed = firegen.workload_single64()
    params = params.replace(p_base=64.0, p_continue=0.0)
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    ii, jj = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    d = np.maximum(abs(ii - 32), abs(jj - 32))
    for t in range(1, 41):
        sim.step(1)
        F = sim.states.cpu().numpy().reshape(64, 64)
        assert np.all(F[d == t] == firegen.BURNING) and np.all(F[d > t] == firegen.FLAMMABLE)
        assert np.all(F[d < t] == firegen.BURNT)


ODD_SIZES = [(1, 1), (3, 5), (37, 53), (64, 64), (100, 130), (300, 17), (7, 257), (129, 65)]


def test_odd_and_ragged_grids_with_actions():
    """Widths that are not multiples of 4 (byte path), partial tiles, 1x1
    envs, drops at edges and corners, counts."""
    batch = firegen.landscape_batch(21, ODD_SIZES)
    params = firegen.Params(p_base=0.7, veg=_veg(3))
    acts = firegen.random_actions(5, batch, 40, p_none=0.4)
    acts[3, :] = (0 << 16) | 0               # corner drops
    acts[4, :] = ((batch.H - 1) << 16) | (batch.W - 1)
    acts[5, :] = (batch.H + 3) << 16         # centre outside the grid: no drop
    sim, ref, got, want = _run_both(batch, params, 40, seed=5, actions=acts)
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(got, want)


ALIGNED_SIZES = [(64, 64), (128, 256), (256, 256), (512, 128), (96, 192), (256, 72), (20, 68)]


@pytest.mark.parametrize("tile_rows", [1, 2, 4, 8])
@pytest.mark.parametrize("skip_static", [0, 1])
@pytest.mark.parametrize("tile_width", [64, 256])
def test_aligned_batch_every_plan(tile_rows, skip_static, tile_width):
    """Same bits whatever the tile shape and load mode."""
    batch = firegen.landscape_batch(31, ALIGNED_SIZES)
    params = firegen.Params(p_base=0.8, veg=_veg(4))
    acts = firegen.random_actions(6, batch, 30, p_none=0.5)
    sim, ref, got, want = _run_both(batch, params, 30, seed=9, actions=acts,
                                    plan={"tile_rows": tile_rows, "skip_static": skip_static,
                                          "tile_width": tile_width})
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("tile_rows", [2, 8])
def test_dense_fronts_overflow_the_lists(tile_rows):
    """A checkerboard of burning cells makes half of every tile a front cell,
    more than a workgroup lists; those workgroups fall back to per-lane work
    and must give the same bits."""
    batch = firegen.landscape_batch(35, [(256, 256), (128, 128), (64, 200)])
    params = firegen.Params(p_base=0.3, veg=_veg(9))
    sim = fs.FireSim.from_batch(batch, params, seed=13)
    sim.set_plan(tile_rows=tile_rows)
    ref = oracle.Sim(batch, params, seed=13)
    st = ref.states.copy()
    for e in range(batch.n_env):
        v = batch.env_view(st, e)
        ii, jj = np.meshgrid(np.arange(v.shape[0]), np.arange(v.shape[1]), indexing="ij")
        v[((ii + jj) % 2 == 0) & (v == firegen.FLAMMABLE)] = firegen.BURNING
    ref.states[:] = st
    sim.states.copy_(torch.from_numpy(st))
    c = sim.step(4, counts=True).cpu().numpy()
    rc = ref.step(4, counts=True)
    torch.cuda.synchronize()
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(c, rc)


def test_stationary_dense_front_benchmark_case():
    """The benchmark's ALU-bound case (checkerboard front, p_base 1e-30,
    p_continue 1) on envs of the 1024 x 256^2 workload in the benchmark's plan:
    bit-exact against the oracle and stationary."""
    batch, params, T, seed = firegen.workload_batch256(n_env=6)
    params = params.replace(p_base=1e-30, p_continue=1.0)
    dense = firegen.dense_front_states(batch)
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    sim.set_plan(tile_rows=4, tile_width=256, skip_static=0, sparse=0, graph=1)
    ref = oracle.Sim(batch, params, seed=seed)
    ref.states[:] = dense
    sim.states.copy_(torch.from_numpy(dense))
    c = sim.step(5, counts=True).cpu().numpy()
    rc = ref.step(5, counts=True, threads=6)
    torch.cuda.synchronize()
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(c, rc)
    assert np.array_equal(ref.states, dense)


def test_graph_replay_and_resume_split():
    """Graph-captured calls replayed several times, and T1 + T2 + T3 split
    calls, equal one oracle run of T1 + T2 + T3 steps."""
    batch = firegen.landscape_batch(41, [(128, 128)] * 5 + [(64, 192)])
    params = firegen.Params(p_base=0.9, veg=_veg(5))
    acts = firegen.random_actions(7, batch, 36, p_none=0.5)
    sim, ref, got, want = _run_both(batch, params, 36, seed=3, actions=acts,
                                    plan={"graph": 1}, split=[12, 12, 12])
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(got, want)


def test_per_cell_wind():
    batch = firegen.landscape_batch(51, [(128, 128), (64, 256), (50, 50)], per_cell_wind=True,
                                    elev_max=2000.0)
    params = firegen.Params(p_base=0.6, veg=_veg(6))
    for skip in (0, 1):
        sim, ref, got, want = _run_both(batch, params, 40, seed=2, plan={"skip_static": skip})
        assert np.array_equal(sim.states.cpu().numpy(), ref.states)
        assert np.array_equal(got, want)


def test_resume_with_saved_states_and_counter():
    """Interrupt and resume: save states and t, destroy, re-init, restore."""
    batch = firegen.landscape_batch(61, [(96, 96)] * 3)
    params = firegen.Params(p_base=0.8, veg=_veg(7))
    a = fs.FireSim.from_batch(batch, params, seed=11)
    a.step(17)
    saved, t = a.states.clone(), a.t
    del a
    b = fs.FireSim.from_batch(batch, params, seed=11)
    b.states.copy_(saved)
    b.t = t
    b.step(13)
    ref = oracle.Sim(batch, params, seed=11)
    ref.step(30)
    torch.cuda.synchronize()
    assert np.array_equal(b.states.cpu().numpy(), ref.states)


def test_batch_order_does_not_matter():
    """An env evolves the same (same env_id) whatever its position in the batch."""
    batch = firegen.landscape_batch(71, [(64, 64), (128, 64), (64, 128), (32, 96)])
    params = firegen.Params(p_base=0.8, veg=_veg(8))
    full = fs.FireSim.from_batch(batch, params, seed=4)
    full.step(25)
    sub = batch.subset([3, 1])
    part = fs.FireSim.from_batch(sub, params, seed=4)
    part.step(25)
    torch.cuda.synchronize()
    f = full.states.cpu().numpy()
    p = part.states.cpu().numpy()
    assert np.array_equal(sub.env_view(p, 0), batch.env_view(f, 3))
    assert np.array_equal(sub.env_view(p, 1), batch.env_view(f, 1))


# launch plans of the full-size checks: the dense one-step plan (the
# roofline probe), the library's default plan, and the plans the benchmark's
# autotuner picked for the uneven and the large workloads
DENSE = dict(tile_rows=4, tile_width=256, skip_static=0, sparse=0, graph=1)
DEFAULT = dict(tile_rows=4, tile_width=64, skip_static=1, sparse=1, graph=1)
TUNED_UNEVEN = dict(tile_rows=8, tile_width=256, skip_static=1, sparse=1, graph=1)
TUNED_LARGE = dict(tile_rows=4, tile_width=256, skip_static=1, sparse=1, graph=1)


def _spread_sample(n, k, seed):
    """k distinct envs out of n: the first, the last and k - 2 seeded draws."""
    rng = np.random.default_rng(seed)
    rest = rng.choice(np.arange(1, n - 1), size=k - 2, replace=False)
    return [0, n - 1] + sorted(int(e) for e in rest)


@pytest.mark.parametrize("plan", [DENSE, DEFAULT], ids=["dense", "default"])
def test_full_size_batch256_sampled_envs(plan):
    """The full 1024 envs of 256x256, 200 steps, in the dense plan (the
    benchmark's headline launch plan) and in the default plan: 32 sampled
    envs equal the oracle bit for bit, counts of those envs too."""
    batch, params, T, seed = firegen.workload_batch256()
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    sim.set_plan(**plan)
    cnt = sim.step(T, counts=True).cpu().numpy()
    torch.cuda.synchronize()
    got = sim.states.cpu().numpy()
    sample = _spread_sample(batch.n_env, 32, 1)
    sub = batch.subset(sample)
    ref = oracle.Sim(sub, params, seed=seed)
    rc = ref.step(T, counts=True, threads=16)
    for k, e in enumerate(sample):
        assert np.array_equal(batch.env_view(got, e), sub.env_view(ref.states, k)), e
        assert np.array_equal(cnt[:, e], rc[:, k]), e


def test_rejects_bad_arguments():
    batch = firegen.landscape_batch(81, [(16, 16)])
    params = firegen.Params()
    with pytest.raises(fs.SimError):
        fs.FireSim(params, [(0, 16, 16, 0, 0, 0, 0)], torch.zeros(100, dtype=torch.uint8, device="cuda"),
                   torch.zeros(100, device="cuda"), torch.zeros(100, device="cuda"))
    with pytest.raises(fs.SimError):
        fs.FireSim(params, [(0, 16, 16, 0, 0, 0, 0)], torch.zeros(256, dtype=torch.uint8, device="cuda"),
                   torch.zeros(256, device="cuda"), torch.zeros(256, device="cuda"),
                   ignitions=[(0, 16, 3)])
    sim = fs.FireSim.from_batch(batch, params)
    with pytest.raises(fs.SimError):
        sim.step(-1)
    with pytest.raises(fs.SimError):
        sim.set_plan(tile_rows=3)
    assert sim.step(0) is None


def test_uneven_batch_with_drops_sampled_envs():
    """The full uneven workload: 4096 envs with sides drawn from {64, 128, 256,
    512}, one 5x5 drop per env per step, 300 steps, counts; in the dense plan,
    the default plan and the benchmark's tuned plan.  8 sampled envs of each
    side equal the oracle bit for bit, counts too."""
    batch, params, T, seed, acts = firegen.workload_uneven()
    rng = np.random.default_rng(7)
    sample = []
    for side in (64, 128, 256, 512):
        of_side = np.flatnonzero(batch.H == side)
        sample += [int(of_side[0]), int(of_side[-1])] + [int(e) for e in rng.choice(of_side[1:-1], 6, replace=False)]
    sample = sorted(sample)
    sub = batch.subset(sample)
    ref = oracle.Sim(sub, params, seed=seed)
    rc = ref.step(T, actions=np.ascontiguousarray(acts[:, sample]), counts=True, threads=16)
    acts_d = torch.from_numpy(acts).cuda()
    for plan in (DENSE, DEFAULT, TUNED_UNEVEN):
        sim = fs.FireSim.from_batch(batch, params, seed=seed)
        sim.set_plan(**plan)
        cnt = sim.step(T, actions=acts_d, counts=True).cpu().numpy()
        torch.cuda.synchronize()
        got = sim.states.cpu().numpy()
        for k, e in enumerate(sample):
            assert np.array_equal(batch.env_view(got, e), sub.env_view(ref.states, k)), (plan, e)
            assert np.array_equal(cnt[:, e], rc[:, k]), (plan, e)
        del sim


def test_large_grids_per_cell_wind_full_run():
    """The full large workload: 8 envs of 2048x2048 with per-cell wind and
    0-2000 m terrain, all 1000 steps, in the dense plan, the default plan and
    the benchmark's tuned plan; one env against the oracle over the whole
    run, states and counts."""
    batch, params, T, seed = firegen.workload_large()
    e = 5
    sub = batch.subset([e])
    ref = oracle.Sim(sub, params, seed=seed)
    rc = ref.step(T, counts=True, threads=1)
    for plan in (DENSE, DEFAULT, TUNED_LARGE):
        sim = fs.FireSim.from_batch(batch, params, seed=seed)
        sim.set_plan(**plan)
        cnt = sim.step(T, counts=True).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(batch.env_view(sim.states.cpu().numpy(), e), sub.env_view(ref.states, 0)), plan
        assert np.array_equal(cnt[:, e], rc[:, 0]), plan
        del sim


def test_autotune_keeps_state_and_results():
    """The autotuner leaves states and step counter alone, adopts its fastest
    plan, and the run continues bit-exact."""
    batch = firegen.landscape_batch(91, [(256, 256)] * 6 + [(128, 200)])
    params = firegen.Params(p_base=0.8, veg=_veg(10))
    sim = fs.FireSim.from_batch(batch, params, seed=21)
    sim.step(7)
    before = sim.states.clone()
    res = sim.autotune(T_probe=4)
    torch.cuda.synchronize()
    assert torch.equal(sim.states, before) and sim.t == 7
    # 16 one-step plans + 6 temporal-blocking plans (every width is a multiple of 4)
    assert len(res) == 22 and all(res[i][1] <= res[i + 1][1] for i in range(21))
    assert sum(r[0]["temporal"] > 1 for r in res) == 6
    best = res[0][0]
    plan = sim.plan()
    keys = ("tile_width", "temporal") if best["temporal"] > 1 else ("tile_rows", "tile_width", "skip_static")
    assert all(plan[k] == best[k] for k in keys), (plan, best)
    sim.step(13)
    ref = oracle.Sim(batch, params, seed=21)
    ref.step(20, threads=8)
    torch.cuda.synchronize()
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)


@pytest.mark.parametrize("skip_static", [0, 1])
@pytest.mark.parametrize("tile_width,tile_rows", [(64, 1), (64, 4), (256, 2), (256, 8)])
def test_sparse_plan_with_drops_graph_and_splits(skip_static, tile_width, tile_rows):
    """Sparse scheduling (tiles without fire nearby are not computed) gives
    the same bits across drops, graph replay and split calls."""
    batch = firegen.landscape_batch(33, [(256, 256), (512, 128), (64, 64), (96, 200), (37, 300)])
    params = firegen.Params(p_base=0.7, veg=_veg(11))
    acts = firegen.random_actions(17, batch, 60, p_none=0.7)
    sim, ref, got, want = _run_both(batch, params, 60, seed=19, actions=acts,
                                    plan={"tile_rows": tile_rows, "tile_width": tile_width,
                                          "skip_static": skip_static, "sparse": 1, "graph": 1},
                                    split=[7, 20, 20, 13])
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("per_cell", [False, True])
def test_wind_series(per_cell):
    """Time-varying wind (per env or per cell, indexed by the absolute step):
    bit-exact against the oracle across split calls, graph replays and a
    sparse plan; a call reaching past the series is rejected."""
    batch = firegen.landscape_batch(21, [(128, 128), (64, 200), (37, 53)], per_cell_wind=per_cell)
    params = firegen.Params(p_base=0.8, veg=_veg(21))
    S = 40
    ser = firegen.wind_series(5, batch, S, per_cell=per_cell, speed_step=1.0, turn_step=0.3)
    kw = {"wind_cell_series" if per_cell else "wind_env_series": ser}
    ref = oracle.Sim(batch, params, seed=9)
    want = [ref.step(15, counts=True, threads=6, **kw), ref.step(25, counts=True, threads=6, **kw)]
    for plan in (dict(graph=1), dict(graph=0, tile_width=64, tile_rows=2, skip_static=1, sparse=1)):
        sim = fs.FireSim.from_batch(batch, params, seed=9)
        sim.set_plan(**plan)
        dev = torch.from_numpy(ser).cuda()
        sim.set_wind_series(cell_series=dev) if per_cell else sim.set_wind_series(env_series=dev)
        got = [sim.step(15, counts=True).cpu().numpy(), sim.step(25, counts=True).cpu().numpy()]
        torch.cuda.synchronize()
        assert np.array_equal(sim.states.cpu().numpy(), ref.states), plan
        for g, w in zip(got, want):
            assert np.array_equal(g, w), plan
        with pytest.raises(fs.SimError):
            sim.step(1)
        sim.set_wind_series()          # back to the static wind
        sim.step(1)
    static = oracle.Sim(batch, params, seed=9)
    static.step(40, threads=6)
    assert not np.array_equal(static.states, ref.states)


def test_wind_series_argument_checks():
    batch = firegen.landscape_batch(22, [(32, 32)] * 2, per_cell_wind=True)
    sim = fs.FireSim.from_batch(batch, firegen.Params(), seed=0)
    env_ser = torch.zeros((4, 2, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(fs.SimError):   # per-cell handle takes only a per-cell series
        sim.set_wind_series(env_series=env_ser)
    with pytest.raises(ValueError):
        sim.set_wind_series(cell_series=torch.zeros((4, 3, 7), dtype=torch.float32, device="cuda"))
    cell = torch.zeros((4, 3, batch.n_cells), dtype=torch.float32, device="cuda")
    with pytest.raises(fs.SimError):
        fs._check(fs.lib().sim_set_wind_series(sim.handle, fs._ptr(env_ser), fs._ptr(cell), 4), sim.handle)
    sim.set_wind_series(cell_series=cell)
    sim.step(4)
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode,radius", [(1, 0), (1, 2), (1, 5), (0, 1), (0, 4)])
def test_drop_modes_and_radii(mode, radius):
    """Water (BURNING -> BURNT) and suppressant drops of several radii, with
    drops in every env at every step: bit-exact against the oracle, in a
    graph and in the sparse plan."""
    batch = firegen.landscape_batch(23, [(128, 128), (60, 200), (33, 47)])
    params = firegen.Params(p_base=0.9, veg=_veg(23))
    T = 30
    act = firegen.random_actions(7, batch, T, p_none=0.3)
    ref = oracle.Sim(batch, params, seed=4)
    want = ref.step(T, actions=act, counts=True, threads=6, drop_mode=mode, drop_radius=radius)
    for plan in (dict(graph=1), dict(graph=0, tile_width=64, tile_rows=8, skip_static=1, sparse=1)):
        sim = fs.FireSim.from_batch(batch, params, seed=4)
        sim.set_plan(**plan)
        sim.set_drop(mode, radius)
        got = sim.step(T, actions=torch.from_numpy(act), counts=True).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(sim.states.cpu().numpy(), ref.states), plan
        assert np.array_equal(got, want), plan
    with pytest.raises(fs.SimError):
        sim.set_drop(2, 1)
    with pytest.raises(fs.SimError):
        sim.set_drop(1, -1)


@pytest.mark.parametrize("plan", [dict(graph=1), dict(graph=0, sparse=1, skip_static=1, tile_width=64)])
def test_history_rows_are_every_step(plan):
    """sim_step_history: row k is the state after step k, bit-exact, for a
    call that starts mid-run, with drops; the states end at the last row."""
    batch = firegen.landscape_batch(24, [(96, 96), (40, 130)])
    params = firegen.Params(p_base=0.8, veg=_veg(24))
    act = firegen.random_actions(8, batch, 25, p_none=0.5)
    ref = oracle.Sim(batch, params, seed=6)
    ref.step(5, actions=act[:5])
    rows, want_c = ref.step(20, actions=act[5:], counts=True, history=True)
    sim = fs.FireSim.from_batch(batch, params, seed=6)
    sim.set_plan(**plan)
    sim.step(5, actions=torch.from_numpy(act[:5]))
    for rep in range(2):   # the second call starts from a saved row, at step 10
        if rep:
            sim.states.copy_(torch.from_numpy(hist0[4]))
            sim.t = 10
            rows, want_c = rows[5:], want_c[5:]
            hist, cnt = sim.step_history(15, actions=torch.from_numpy(act[10:]), counts=True)
        else:
            hist, cnt = sim.step_history(20, actions=torch.from_numpy(act[5:]), counts=True)
            hist0 = hist.cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(hist.cpu().numpy(), rows)
        assert np.array_equal(cnt.cpu().numpy(), want_c)
        assert np.array_equal(sim.states.cpu().numpy(), rows[-1])


@pytest.mark.parametrize("temporal", [2, 4, 8])
@pytest.mark.parametrize("tile_width", [64, 128])
def test_temporal_blocking(temporal, tile_width):
    """Several steps per launch with the state tile in LDS: bit-exact against
    the oracle with drops, counts, a T that is not a multiple of the depth,
    split calls, graph replay and envs narrower, wider and shorter than a
    tile."""
    batch = firegen.landscape_batch(51, [(128, 128), (64, 200), (36, 52), (300, 20), (8, 8), (97, 132)])
    params = firegen.Params(p_base=0.85, veg=_veg(51))
    T = 23
    act = firegen.random_actions(12, batch, T, p_none=0.4)
    ref = oracle.Sim(batch, params, seed=17)
    want = ref.step(T, actions=act, counts=True, threads=6)
    for graph in (1, 0):
        sim = fs.FireSim.from_batch(batch, params, seed=17)
        sim.set_plan(tile_width=tile_width, temporal=temporal, graph=graph)
        c1 = sim.step(9, actions=torch.from_numpy(act[:9]), counts=True).cpu().numpy()
        c2 = sim.step(T - 9, actions=torch.from_numpy(act[9:]), counts=True).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(sim.states.cpu().numpy(), ref.states), graph
        assert np.array_equal(np.concatenate([c1, c2]), want), graph
        assert sim.plan()["temporal"] == temporal


@pytest.mark.parametrize("per_cell", [False, True])
def test_temporal_blocking_with_wind_series_water_and_history(per_cell):
    batch = firegen.landscape_batch(52, [(128, 128), (60, 200)], per_cell_wind=per_cell)
    params = firegen.Params(p_base=0.9, veg=_veg(52))
    T = 19
    ser = firegen.wind_series(6, batch, T, per_cell=per_cell, speed_step=1.0, turn_step=0.3)
    kw = {"wind_cell_series" if per_cell else "wind_env_series": ser}
    act = firegen.random_actions(13, batch, T, p_none=0.3)
    ref = oracle.Sim(batch, params, seed=5)
    rows, want = ref.step(T, actions=act, counts=True, threads=6, drop_mode=1, drop_radius=3, history=True,
                          **kw)
    sim = fs.FireSim.from_batch(batch, params, seed=5)
    sim.set_plan(tile_width=128, temporal=8, graph=1)
    sim.set_drop(1, 3)
    dev = torch.from_numpy(ser).cuda()
    sim.set_wind_series(cell_series=dev) if per_cell else sim.set_wind_series(env_series=dev)
    got = sim.step(T, actions=torch.from_numpy(act), counts=True).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(got, want)
    sim2 = fs.FireSim.from_batch(batch, params, seed=5)
    sim2.set_plan(tile_width=64, temporal=4)
    sim2.set_drop(1, 3)
    sim2.set_wind_series(cell_series=dev) if per_cell else sim2.set_wind_series(env_series=dev)
    hist, cnt = sim2.step_history(T, actions=torch.from_numpy(act), counts=True)
    torch.cuda.synchronize()
    assert np.array_equal(hist.cpu().numpy(), rows)
    assert np.array_equal(cnt.cpu().numpy(), want)


def test_temporal_blocking_rejections():
    ragged = firegen.landscape_batch(53, [(40, 42)])
    sim = fs.FireSim.from_batch(ragged, firegen.Params(), seed=0)
    with pytest.raises(fs.SimError):
        sim.set_plan(temporal=4, tile_width=64)
    batch = firegen.landscape_batch(54, [(64, 64)])
    sim = fs.FireSim.from_batch(batch, firegen.Params(), seed=0)
    for kw in (dict(temporal=3, tile_width=64), dict(temporal=4, tile_width=256),
               dict(temporal=4, tile_width=64, sparse=1)):
        with pytest.raises(fs.SimError):
            sim.set_plan(**kw)
    sim.set_plan(temporal=2, tile_width=64)
    sim.step(3)
    torch.cuda.synchronize()


@pytest.mark.parametrize("plan", [dict(graph=1), dict(tile_rows=1, skip_static=1, sparse=1, graph=0),
                                  dict(tile_rows=8, tile_width=64)])
def test_narrow_envs_use_narrow_tiles(plan):
    """Envs of width <= 32 run on 16- and 32-column tiles (4 or 8 lanes per
    row segment): bit-exact with drops, including the RL scenario's 20 x 20."""
    sizes = [(20, 20)] * 5 + [(12, 28), (32, 32), (16, 48), (40, 16), (9, 4), (33, 36)]
    batch = firegen.landscape_batch(61, sizes)
    params = firegen.Params(p_base=0.9, veg=_veg(61))
    T = 25
    act = firegen.random_actions(14, batch, T, p_none=0.5)
    sim, ref, got, want = _run_both(batch, params, T, seed=3, actions=act, plan=plan)
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(got, want)


def test_atan_bit_exact():
    """The device arctangent of the slope-angle variant equals the oracle's
    on every third fp32 in (-2^24, 2^24) and on +-0, +-inf, NaN-free powers."""
    top = int(np.float32(2.0 ** 24).view(np.uint32))
    chunk = 1 << 26
    for neg in (False, True):
        for start in range(0, top, chunk):
            bits = np.arange(start, min(start + chunk, top), 3, dtype=np.uint32)
            if neg:
                bits |= np.uint32(0x80000000)
            x = bits.view(np.float32)
            want = oracle.atan_c(x)
            got = fs.debug_atan(torch.from_numpy(x).cuda()).cpu().numpy()
            bad = np.flatnonzero(got.view(np.uint32) != want.view(np.uint32))
            assert bad.size == 0, (x[bad[:5]], got[bad[:5]], want[bad[:5]])
    x = np.array([0.0, -0.0, np.inf, -np.inf, 2.0 ** 100, -2.0 ** -100], np.float32)
    assert np.array_equal(fs.debug_atan(torch.from_numpy(x).cuda()).cpu().numpy().view(np.uint32),
                          oracle.atan_c(x).view(np.uint32))


@pytest.mark.parametrize("per_cell_wind", [False, True])
@pytest.mark.parametrize("plan", [dict(graph=1), dict(tile_width=128, temporal=4)])
def test_slope_angle_mode(per_cell_wind, plan):
    """S = atan(rise / run) on steep terrain (0-2000 m): bit-exact."""
    batch = firegen.landscape_batch(71, [(128, 128), (64, 200), (36, 52)], elev_max=2000.0,
                                    per_cell_wind=per_cell_wind)
    params = firegen.Params(p_base=0.8, alpha_s=3.0, slope_mode=1, veg=_veg(71))
    T = 30
    sim, ref, got, want = _run_both(batch, params, T, seed=8, plan=plan)
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(got, want)
    flat = oracle.Sim(batch, params.replace(slope_mode=0), seed=8)
    flat.step(T, threads=6)
    assert not np.array_equal(flat.states, ref.states)   # the mode matters here


@pytest.mark.parametrize("plan", [dict(graph=1), dict(tile_rows=1, tile_width=64, skip_static=1, sparse=1)])
def test_maximum_side_lengths(plan):
    """Envs at the largest side the ABI accepts (32767) in either direction,
    with drops at the far edges: bit-exact."""
    sizes = [(6, 32767), (32767, 5), (1, 32767), (32767, 1), (3, 32764)]
    batch = firegen.landscape_batch(81, sizes, class_sigma=3.0)
    for e, (H, W) in enumerate(sizes):   # ignite along the long axis too
        far = (H - 1, W - 1)
        batch.ignitions = np.concatenate([batch.ignitions, np.array([[e, far[0] // 2, far[1] // 2],
                                                                     [e, far[0], far[1]]], np.int32)])
    params = firegen.Params(p_base=1.5, veg=_veg(81))
    T = 20
    act = firegen.random_actions(15, batch, T, p_none=0.6)
    act[5] = ((batch.H - 1) << 16) | (batch.W - 1)      # a drop on every far corner
    sim, ref, got, want = _run_both(batch, params, T, seed=12, actions=act, plan=plan)
    assert np.array_equal(sim.states.cpu().numpy(), ref.states)
    assert np.array_equal(got, want)
    assert want.sum() > 0
