"""Hand-worked values of the two calibration losses of the fp64 oracle.

Each expected number below was computed by hand from the definitions
(soft IoU with S = 1 - U_T on burnable cells; the paper's section 4 loss:
BCE of the clipped soft scar plus the squared error of pool x pool block
means), not by re-evaluating the oracle's formulas.  A misread denominator,
an S / U swap, a wrong edge-block divisor or a wrong sign of the seed fails
one of them.
"""
import math

import numpy as np
import pytest

from oracle import relaxed64

# 2 x 3 worked example.  U_T -> S = 1 - U_T:
#   U = [[0.2, 0.5, 1.0],      S = [[0.8, 0.5, 0.0],      Y = [[1, 1, 0],
#        [0.9, 0.0, 0.6]]           [0.1, 1.0, 0.4]]           [0, 1, 0]]
# I = 0.8 + 0.5 + 1.0 = 2.3, sum S = 2.8, sum Y = 3, D = 2.8 + 3 - 2.3 = 3.5,
# L = 1 - 2.3 / 3.5 = 12/35.
U23 = np.array([[0.2, 0.5, 1.0], [0.9, 0.0, 0.6]])
Y23 = np.array([[1, 1, 0], [0, 1, 0]], bool)
ALL = np.ones((2, 3), bool)


def test_soft_iou_identical_scars_is_zero():
    Y = np.array([[1, 0, 1], [1, 1, 0]], bool)
    U = np.where(Y, 0.0, 1.0)          # S = Y exactly
    L, _ = relaxed64.soft_iou_loss(U, Y, ALL)
    assert L == 0.0


def test_soft_iou_disjoint_scars_is_one():
    Y = np.array([[1, 1, 0], [0, 0, 0]], bool)
    U = np.array([[1.0, 1.0, 0.3], [0.0, 0.5, 1.0]])   # S = 0 wherever Y = 1
    L, _ = relaxed64.soft_iou_loss(U, Y, ALL)
    assert L == 1.0


def test_soft_iou_worked_2x3():
    L, g = relaxed64.soft_iou_loss(U23, Y23, ALL)
    assert L == pytest.approx(12.0 / 35.0, abs=1e-15)
    # dL/dU = (Y D - I (1 - Y)) / D^2: Y = 1 -> 3.5 / 12.25 = 2/7,
    # Y = 0 -> -2.3 / 12.25 = -46/245
    want = np.where(Y23, 2.0 / 7.0, -46.0 / 245.0)
    np.testing.assert_allclose(g, want, rtol=0, atol=1e-15)


def test_soft_iou_unburnable_cell_is_not_scar():
    # cell (1, 2) unburnable: S there is 0 whatever U says, and its seed is 0.
    # sum S = 2.4, D = 2.4 + 3 - 2.3 = 3.1, L = 0.8 / 3.1 = 8/31
    burnable = ALL.copy()
    burnable[1, 2] = False
    L, g = relaxed64.soft_iou_loss(U23, Y23, burnable)
    assert L == pytest.approx(8.0 / 31.0, abs=1e-15)
    assert g[1, 2] == 0.0
    # D = 3.1, I = 2.3: Y = 1 -> 3.1 / 9.61 = 10/31, Y = 0 -> -2.3 / 9.61 = -230/961
    assert g[0, 0] == pytest.approx(10.0 / 31.0, abs=1e-15)
    assert g[0, 2] == pytest.approx(-230.0 / 961.0, abs=1e-15)


def test_bce_constant_field_closed_form():
    # S = 1 - 0.75 = 0.25 everywhere, Y has 2 ones among 6 cells:
    # BCE = -(2 ln 0.25 + 4 ln 0.75) / 6 = (4 ln 2 + 4 ln 4/3) / 6 = (2/3) ln (8/3)
    U = np.full((2, 3), 0.75)
    Y = np.array([[1, 0, 0], [0, 0, 1]], bool)
    L, g = relaxed64.bce_pool_loss(U, Y, ALL, pool=1, mse_weight=0.0, eps=1e-6)
    assert L == pytest.approx((2.0 / 3.0) * math.log(8.0 / 3.0), abs=1e-14)
    # dL/dU = -dL/dS = (Y / S - (1 - Y) / (1 - S)) / n: Y = 1 -> 4 / 6 = 2/3,
    # Y = 0 -> -(4/3) / 6 = -2/9
    np.testing.assert_allclose(g, np.where(Y, 2.0 / 3.0, -2.0 / 9.0), rtol=0, atol=1e-14)


def test_bce_clip_freezes_the_gradient():
    # S = 0 (U = 1) and S = 1 (U = 0) are clipped to eps and 1 - eps: the loss
    # takes the clipped value and the gradient there is 0
    eps = 1e-3
    U = np.array([[1.0, 0.0]])
    Y = np.array([[1, 0]], bool)
    L, g = relaxed64.bce_pool_loss(U, Y, np.ones((1, 2), bool), pool=1, mse_weight=0.0, eps=eps)
    assert L == pytest.approx(-math.log(eps), rel=1e-12)   # (-ln eps - ln eps) / 2
    assert np.all(g == 0.0)


def _ragged_5x6():
    # S(i, j) = 0.05 + 0.1 i + 0.01 j on a 5 x 6 grid; Y = 1 on columns 0, 1.
    # pool 4 -> blocks rows {0..3}, {4} x cols {0..3}, {4, 5}: 16, 8, 4, 2 cells.
    # Block means of S: 0.05 + 0.1 mean(i) + 0.01 mean(j):
    #   (0,0): 0.05 + 0.15 + 0.015 = 0.215   (0,1): 0.05 + 0.15 + 0.045 = 0.245
    #   (1,0): 0.05 + 0.40 + 0.015 = 0.465   (1,1): 0.05 + 0.40 + 0.045 = 0.495
    # Block means of Y: 8/16, 0, 2/4, 0.
    # MSE = ((0.285)^2 + 0.245^2 + 0.035^2 + 0.495^2) / 4
    #     = (0.081225 + 0.060025 + 0.001225 + 0.245025) / 4 = 0.096875
    ii, jj = np.meshgrid(np.arange(5), np.arange(6), indexing="ij")
    S = 0.05 + 0.1 * ii + 0.01 * jj
    Y = jj < 2
    return 1.0 - S, Y


def test_pooled_mse_ragged_blocks_by_hand():
    U, Y = _ragged_5x6()
    burn = np.ones((5, 6), bool)
    L0, g0 = relaxed64.bce_pool_loss(U, Y, burn, pool=4, mse_weight=0.0)
    L1, g1 = relaxed64.bce_pool_loss(U, Y, burn, pool=4, mse_weight=1.0)
    L3, _ = relaxed64.bce_pool_loss(U, Y, burn, pool=4, mse_weight=3.0)
    assert L1 - L0 == pytest.approx(0.096875, abs=1e-14)
    assert L3 - L0 == pytest.approx(3 * 0.096875, abs=1e-14)
    # d MSE / d S(cell) = 2 (pS - pY) / 4 / (cells of its block); dL/dU = -that
    #   block (0,0): 2 (0.215 - 0.5) / 4 / 16 = -0.00890625 -> +0.00890625
    #   block (0,1): 2 (0.245) / 4 / 8 = 0.0153125          -> -0.0153125
    #   block (1,0): 2 (0.465 - 0.5) / 4 / 4 = -0.004375    -> +0.004375
    #   block (1,1): 2 (0.495) / 4 / 2 = 0.12375             -> -0.12375
    d = g1 - g0
    assert d[0, 0] == pytest.approx(0.00890625, abs=1e-15)
    assert d[3, 5] == pytest.approx(-0.0153125, abs=1e-15)
    assert d[4, 3] == pytest.approx(0.004375, abs=1e-15)
    assert d[4, 5] == pytest.approx(-0.12375, abs=1e-15)


def test_loss_mean_over_envs():
    # T = 0: U_T is the initial state, so S = 1 exactly on the ignition cell
    # and 0 elsewhere.  Env 0's target is its ignition cell (L = 0), env 1's
    # a cell away from it (I = 0, L = 1): the mean over the two envs is 1/2,
    # and with no step taken the parameter gradient is 0.
    import firegen
    b = firegen.uniform_batch(4, 5, n_env=2, ignitions=[(0, 1, 1), (1, 2, 3)])
    Y0 = np.zeros((4, 5), bool)
    Y0[1, 1] = True
    Y1 = np.zeros((4, 5), bool)
    Y1[0, 0] = True
    theta = relaxed64.theta_from_params(firegen.Params())
    L, grad, _ = relaxed64.loss_and_grad(b, theta, 0, [Y0, Y1])
    assert L == 0.5
    assert np.all(grad == 0.0)
