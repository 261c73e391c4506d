"""Host-side checks of the benchmark's accounting (no GPU): the operation
count of the dense-front case on hand-counted states, and the one-GPU guard."""
import os
import subprocess
import sys

import numpy as np

import firegen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_dense_front_ops_hand_counted():
    """A 3 x 4 grid: burning cells at (0,0) and (2,3).  Front cells and their
    burning neighbours counted by hand: (0,1) 1, (1,0) 1, (1,1) 1, (1,2) 1,
    (1,3) 1, (2,2) 1 -> 6 phi terms on 6 front cells; draws = 6 front + 2
    burning."""
    b = firegen.uniform_batch(3, 4, ignitions=())
    st = np.full(12, firegen.FLAMMABLE, np.uint8)
    st[0] = st[11] = firegen.BURNING
    st[8] = firegen.BURNT
    n_phi, n_front, n_draw, ops = bench.dense_front_ops(b, st, firegen)
    assert (n_phi, n_front, n_draw) == (6, 6, 8)
    assert ops == bench.OPS_PHI * 6 + bench.OPS_PROB * 6 + bench.OPS_DRAW * 8


def test_dense_front_checkerboard_counts():
    """Checkerboard on an all-burnable 6 x 6 grid: every flammable cell is a
    front cell; its burning neighbours are its in-grid orthogonal ones."""
    b = firegen.uniform_batch(6, 6, ignitions=())
    st = firegen.dense_front_states(b)
    F = st.reshape(6, 6)
    assert np.all(F[(np.add.outer(np.arange(6), np.arange(6)) % 2) == 0] == firegen.BURNING)
    n_phi, n_front, n_draw, _ = bench.dense_front_ops(b, st, firegen)
    assert n_front == 18 and n_draw == 36
    # orthogonal in-grid neighbours of the 18 flammable cells
    want = sum(((i > 0) + (i < 5) + (j > 0) + (j < 5)) for i in range(6) for j in range(6) if (i + j) % 2)
    assert n_phi == want


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_relaxed_bytes_per_cell_step():
    """T = 100, checkpoints every 10: 9 of the 10 segments are recomputed, 9
    steps each (81 of 100); the forward's last segment stays in place."""
    assert abs(bench.relaxed_bytes_per_cell_step(100, 10, False) - (40 * 1.81 + 61 + 0.32)) < 1e-9
    assert abs(bench.relaxed_bytes_per_cell_step(100, 10, True) - (52 * 1.81 + 73 + 0.32)) < 1e-9
    # a single segment is never recomputed
    assert abs(bench.relaxed_bytes_per_cell_step(21, 40, False) - (40 + 61 + 32 / 21)) < 1e-9
