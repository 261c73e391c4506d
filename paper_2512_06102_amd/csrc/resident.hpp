// resident.hpp -- host interface of the resident multi-step kernel (T steps
// of a batch of small envs in one launch, each env held in LDS).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace firesim {

// Shape of the resident kernel over a batch whose envs all have W % 4 == 0
// and 4-aligned offsets: the largest framed state, (H + 2)(W/4 + 2) dwords
// rounded up to a multiple of 4, and the largest env in cells (at most
// 65536).  It fits when its dynamic LDS is at most the device's LDS per
// workgroup (160 KiB on gfx950) less the kernel's static LDS (under 2.5 KiB).
struct ResidentShape {
    bool fits = false;
    int32_t frame_cap = 0;
    int32_t cell_cap = 0;
};
// Two framed states; fuel term, elevation and an 8-byte front-list entry per cell.
inline size_t resident_lds_bytes(const ResidentShape& s)
{
    return 8 * (size_t)s.frame_cap + 16 * (size_t)s.cell_cap;
}
// Allows every instance of the kernel `bytes` of dynamic LDS.
hipError_t resident_set_lds_limit(int bytes);

// T steps of the n_list envs env_list[0..n_list) (env_list NULL: envs
// 0..n_list) from src to dst (which may be the same buffer), the first at the
// absolute step *t_base + step0 (t_base in device memory, so a captured
// launch serves any starting step), by workgroups of `threads` lanes (64,
// 256, 512 or 1024); actions and counts point at the rows of the first step
// (n_env entries per step, indexed by the global env index) or are NULL.
// The count rows must hold 0 on entry: an env whose fire is out stops
// stepping (applying only the remaining drops) and leaves its later rows.
hipError_t launch_stoch_resident(hipStream_t s, const EnvDev* envs, int32_t n_env, const int32_t* env_list,
                                 int32_t n_list, const StaticFields& F, const StepArgs& A, const ResidentShape& shape,
                                 int threads, const uint8_t* src, uint8_t* dst, const uint32_t* t_base,
                                 uint32_t step0, int32_t T, const int32_t* actions, int32_t* counts);

}  // namespace firesim
