"""Host-side checks of arithmetic shortcuts that the kernels rely on."""
import os
import subprocess
import tempfile

SRC = r"""
#include <stdio.h>
/* The fused RL kernel's row of a dword index: q / d as (int)((q + 0.5f) * fl(1/d))
   in fp32 (no contraction), for every 0 <= q < 2^14 and 1 <= d <= 2^14. */
int main(void) {
    long bad = 0;
    for (int d = 1; d <= 16384; ++d) {
        volatile float inv = 1.0f / (float)d;
        for (int q = 0; q < 16384; ++q) {
            volatile float x = (float)q + 0.5f;
            volatile float y = x * inv;
            if ((int)y != q / d) ++bad;
        }
    }
    printf("%ld\n", bad);
    return 0;
}
"""


def test_small_division_is_exact_over_its_range():
    d = tempfile.mkdtemp()
    c = os.path.join(d, "div.c")
    open(c, "w").write(SRC)
    exe = os.path.join(d, "div")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", c, "-o", exe])
    assert subprocess.check_output([exe]).strip() == b"0"
