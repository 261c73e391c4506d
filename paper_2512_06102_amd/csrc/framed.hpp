// framed.hpp -- an env's state resident in LDS as (H + 2) rows of W/4 + 2
// dwords (4 cells each) with a zero frame, as the kernels that keep whole
// envs in LDS (the fused RL step, the resident multi-step kernel) hold it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stepcell.hpp"

namespace firesim {

// q / d by one fp32 multiply, inv_d = fl(1 / d): the rounding error of
// (q + 1/2) inv_d stays below the 1/(2d) distance of (q + 1/2)/d from an
// integer.  Exact for 0 <= q < 2^14 and 1 <= d <= 2^14 (checked over every
// pair); here q is a dword index (an env has at most 2^16 cells) or an
// observation index (side at most 63).
__device__ __forceinline__ int small_div(int q, int d, float inv_d) { return (int)(((float)q + 0.5f) * inv_d); }

// Cells of the 4-cell group at framed position m (row stride SW) with a
// burning Moore neighbour, bits 0-3.
__device__ __forceinline__ uint32_t near_burning(const uint32_t* m, int SW)
{
    const uint32_t up6 = row_window(m[-SW - 1], m[-SW], m[-SW + 1]);
    const uint32_t md6 = row_window(m[-1], m[0], m[1]);
    const uint32_t dn6 = row_window(m[SW - 1], m[SW], m[SW + 1]);
    const uint32_t ud = up6 | dn6;
    return (ud | (ud >> 1) | (ud >> 2) | md6 | (md6 >> 2)) & 0xFu;
}

}  // namespace firesim
