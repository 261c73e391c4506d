"""The library's HBM streaming probe (sim_debug_stream) moves what it says:
copy reproduces the source, write leaves its pattern, read writes nothing;
bad arguments are rejected."""
import pytest
import torch

pytestmark = pytest.mark.gpu

fs = pytest.importorskip("paper_2512_06102_amd")


def test_stream_probe_modes():
    n = (1 << 20) + 48  # bytes: not a multiple of the grid's stride
    a = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    b = torch.zeros(n, dtype=torch.uint8, device="cuda")
    fs.debug_stream(2, a, b, blocks=37)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    c = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    fs.debug_stream(0, a, c, blocks=64)  # read only
    torch.cuda.synchronize()
    assert bool((c == 7).all())
    fs.debug_stream(1, None, c, blocks=5)
    torch.cuda.synchronize()
    w = c.view(torch.int32).view(-1, 4).cpu()
    idx = torch.arange(w.shape[0], dtype=torch.int32)
    assert torch.equal(w[:, 0], idx) and bool((w[:, 1] == 1).all()) and bool((w[:, 3] == 3).all())


def test_stream_probe_rejects_bad_arguments():
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    L = fs.lib()
    s = torch.cuda.current_stream().cuda_stream
    import ctypes
    p = ctypes.c_void_p(a.data_ptr())
    assert L.sim_debug_stream(3, p, p, 64, 1, ctypes.c_void_p(s)) != 0          # mode
    assert L.sim_debug_stream(2, p, p, 40, 1, ctypes.c_void_p(s)) != 0          # size
    assert L.sim_debug_stream(2, ctypes.c_void_p(a.data_ptr() + 4), p, 48, 1, ctypes.c_void_p(s)) != 0  # alignment
    assert L.sim_debug_stream(2, p, p, 64, 0, ctypes.c_void_p(s)) != 0          # blocks
    torch.cuda.synchronize()
