"""The C ABI without a GPU: the library loads, exports every function the
header declares, its structs have the header's layout, and argument errors
are reported before any device work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "firesim.h")

fs = pytest.importorskip("paper_2512_06102_amd")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = fs.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fs.EXPORTED)


def test_struct_layout_matches_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "firesim.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(sim_params), sizeof(sim_env), sizeof(sim_plan),
         offsetof(sim_params, veg), offsetof(sim_params, unburnable_mask),
         offsetof(sim_env, env_id), offsetof(sim_env, Vy), sizeof(sim_rl_config),
         offsetof(sim_rl_config, single_launch));
  return 0;
}
"""
    d = tempfile.mkdtemp()
    c = os.path.join(d, "layout.c")
    open(c, "w").write(src)
    exe = os.path.join(d, "layout")
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), c, "-o", exe])
    got = [int(x) for x in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(fs.SimParams), ctypes.sizeof(fs.SimEnv), ctypes.sizeof(fs.SimPlan),
            fs.SimParams.veg.offset, fs.SimParams.unburnable_mask.offset, fs.SimEnv.env_id.offset,
            fs.SimEnv.Vy.offset, ctypes.sizeof(fs.SimRlConfig), fs.SimRlConfig.single_launch.offset]
    assert got == want


def test_header_compiles_as_c_and_cpp():
    for comp, ext in (("gcc", "c"), ("g++", "cpp")):
        d = tempfile.mkdtemp()
        f = os.path.join(d, "inc." + ext)
        open(f, "w").write('#include "firesim.h"\nint main(void){return SIM_OK;}\n')
        subprocess.check_call([comp, "-Wall", "-Werror", "-I", os.path.dirname(HEADER), f, "-o",
                               os.path.join(d, "a.out")])


def _bad_init(**over):
    L = fs.lib()
    p = fs.SimParams()
    p.cell_size = 30.0
    env = (fs.SimEnv * 1)(fs.SimEnv(0, 4, 4, 0, 0, 0, 0))
    args = dict(p=ctypes.byref(p), n_env=1, envs=env, n_cells=16, lc=ctypes.c_void_p(16),
                den=ctypes.c_void_p(16), elev=ctypes.c_void_p(16), ign=None, n_ign=0,
                out=ctypes.c_void_p(16))
    args.update(over)
    h = ctypes.c_void_p()
    rc = L.sim_init(ctypes.byref(h), args["p"], args["n_env"], args["envs"], args["n_cells"],
                    args["lc"], args["den"], args["elev"], None, args["ign"], args["n_ign"], 0,
                    args["out"], None)
    return rc, L.sim_last_error(None).decode()


@pytest.mark.parametrize("over,needle", [
    (dict(n_env=0), "n_env"),
    (dict(n_cells=15), "outside"),
    (dict(lc=None), "required"),
    (dict(envs=(fs.SimEnv * 1)(fs.SimEnv(0, 0, 4, 0, 0, 0, 0))), "H, W"),
    (dict(envs=(fs.SimEnv * 2)(fs.SimEnv(0, 4, 4, 0, 0, 0, 0), fs.SimEnv(8, 4, 4, 1, 0, 0, 0)),
          n_env=2, n_cells=32), "overlap"),
    (dict(ign=(ctypes.c_int32 * 3)(0, 4, 0), n_ign=1), "ignition"),
    (dict(ign=(ctypes.c_int32 * 3)(1, 0, 0), n_ign=1), "ignition"),
])
def test_init_rejects_bad_arguments_without_touching_the_gpu(over, needle):
    rc, msg = _bad_init(**over)
    assert rc == -1 and needle in msg, (rc, msg)


def test_null_handle_calls_fail_cleanly():
    L = fs.lib()
    assert L.sim_step(None, None, None, 1, None, None) == -1
    assert L.sim_set_step(None, 0) == -1
    assert L.sim_relaxed_workspace_bytes(None, 10, 5) == 0
    assert L.sim_debug_exp(None, None, -1, None) == -1
    L.sim_destroy(None)
