"""The allocation-free soft-IoU loss (sim_relaxed_loss_noalloc) through the C
ABI: equal bits to sim_relaxed_loss on two calls in a row, the second on a
smaller batch, both within tolerance of the fp64 oracle's soft IoU, and a
clear error for a batch beyond its static scratch."""
import numpy as np
import pytest
import torch

import firegen
from oracle import relaxed64

pytestmark = pytest.mark.gpu

fs = pytest.importorskip("paper_2512_06102_amd")


def _relaxed_state(sizes, seed, T=15):
    batch = firegen.landscape_batch(seed, sizes, elev_max=80.0)
    params = firegen.Params(p_base=0.6, veg=tuple(float(v) for v in firegen.veg_table(np.random.default_rng(seed))))
    sim = fs.FireSim.from_batch(batch, params, seed=seed)
    burnable = sim.states.cpu().numpy() != firegen.UNBURNABLE  # the initial state
    p = fs.make_params(params)
    p.unburnable_mask = batch.unburnable_mask
    U, B = sim.relaxed_init()
    ws = sim.relaxed_workspace(T, 5)
    sim.relaxed_fwd(p, U, B, T, 5, ws)
    rng = np.random.default_rng(seed + 100)
    Y = (rng.random(batch.cls.size) < 0.3).astype(np.uint8)
    return batch, sim, U, torch.from_numpy(Y).cuda(), Y, burnable


def _both(sim, U, Y, scale):
    loss_a, g_a, obj_a = sim.relaxed_loss(U, Y, scale=scale)
    loss_b = torch.full((sim.n_env,), -1.0, dtype=torch.float32, device=U.device)
    g_b = torch.full_like(U, -1.0)
    obj_b = torch.full((1,), -1.0, dtype=torch.float64, device=U.device)
    sim.relaxed_loss_noalloc(U, Y, loss_b, g_b, obj_b, scale=scale)
    torch.cuda.synchronize()
    return (loss_a.cpu().numpy(), g_a.cpu().numpy(), obj_a.item()), \
        (loss_b.cpu().numpy(), g_b.cpu().numpy(), obj_b.item())


def _check_against_oracle(batch, U, Y, burnable, loss, g, obj, scale):
    Un = U.cpu().numpy()
    Ls = []
    for e in range(batch.n_env):
        L64, gU64 = relaxed64.soft_iou_loss(batch.env_view(Un, e), batch.env_view(Y, e).astype(bool),
                                            batch.env_view(burnable, e))
        Ls.append(L64)
        assert abs(loss[e] - L64) <= 1e-6
        assert np.max(np.abs(batch.env_view(g, e) - scale * gU64)) <= 1e-12
    assert abs(obj - scale * sum(Ls)) <= 1e-12


def test_noalloc_loss_equals_regular_on_two_calls():
    # first call: four ragged envs spanning several 4096-cell chunks
    batch, sim, U, Yd, Y, burn = _relaxed_state([(200, 150), (64, 64), (33, 300), (5, 7)], 31)
    reg, noa = _both(sim, U, Yd, 0.25)
    for a, b in zip(reg, noa):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    _check_against_oracle(batch, U, Y, burn, *noa, 0.25)
    # second call, a smaller batch: the scratch keeps the first call's sums,
    # which must not leak into this one
    batch2, sim2, U2, Yd2, Y2, burn2 = _relaxed_state([(40, 50), (17, 3)], 32)
    reg2, noa2 = _both(sim2, U2, Yd2, 0.5)
    for a, b in zip(reg2, noa2):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    _check_against_oracle(batch2, U2, Y2, burn2, *noa2, 0.5)


def test_noalloc_loss_without_seed_or_objective():
    batch, sim, U, Yd, Y, _ = _relaxed_state([(70, 90)], 33)
    loss_a, _, obj_a = sim.relaxed_loss(U, Yd)
    loss_b = torch.empty(1, dtype=torch.float32, device=U.device)
    sim.relaxed_loss_noalloc(U, Yd, loss_b, None, None)
    torch.cuda.synchronize()
    assert np.array_equal(loss_a.cpu().numpy(), loss_b.cpu().numpy())


def test_noalloc_loss_rejects_batch_beyond_scratch():
    # 150000 one-cell envs need 7 doubles each, beyond the 2^19 of the scratch
    n = 150000
    dev = torch.device("cuda")
    envs = [(e, 1, 1, e, 0.0, 0.0, 0.0) for e in range(n)]
    lc = torch.full((n,), firegen.GRASS, dtype=torch.uint8, device=dev)
    zero = torch.zeros(n, dtype=torch.float32, device=dev)
    sim = fs.FireSim(firegen.Params(), envs, lc, zero, zero)
    U = torch.rand(n, dtype=torch.float64, device=dev)
    Y = torch.ones(n, dtype=torch.uint8, device=dev)
    loss = torch.empty(n, dtype=torch.float32, device=dev)
    with pytest.raises(fs.SimError, match="static scratch"):
        sim.relaxed_loss_noalloc(U, Y, loss, None, None)
    loss_a, _, _ = sim.relaxed_loss(U, Y, want_grad=False)  # the allocating call still serves it
    torch.cuda.synchronize()
    assert torch.all(torch.isfinite(loss_a))
