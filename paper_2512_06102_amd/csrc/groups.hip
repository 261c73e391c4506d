// groups.hip -- device helpers of the size-class groups: copying the cells of
// a list of envs (the last ping-pong copy of a group's call).
#include "internal.hpp"

namespace firesim {
namespace {

// Block b copies envs b, b + gridDim.x, ... of the list, 16 bytes per lane
// where the env's cells allow it.
__global__ __launch_bounds__(256) void copy_envs_kernel(const EnvDev* __restrict__ envs,
                                                        const int32_t* __restrict__ env_list, int32_t n_list,
                                                        uint8_t* __restrict__ dst, const uint8_t* __restrict__ src)
{
    for (int32_t j = blockIdx.x; j < n_list; j += gridDim.x) {
        const EnvDev ed = envs[env_list[j]];
        const int64_t n = (int64_t)ed.H * ed.W, off = ed.offset;
        int64_t head = 0;
        if (off % 16 == 0) {
            const int64_t n16 = n / 16;
            const uint4* s4 = reinterpret_cast<const uint4*>(src + off);
            uint4* d4 = reinterpret_cast<uint4*>(dst + off);
            for (int64_t i = threadIdx.x; i < n16; i += blockDim.x) d4[i] = s4[i];
            head = n16 * 16;
        }
        for (int64_t i = head + threadIdx.x; i < n; i += blockDim.x) dst[off + i] = src[off + i];
    }
}

}  // namespace

hipError_t launch_copy_envs(hipStream_t s, const EnvDev* envs, const int32_t* env_list, int32_t n_list,
                            uint8_t* dst, const uint8_t* src)
{
    if (n_list <= 0) return hipSuccess;
    const int blocks = n_list < 8192 ? n_list : 8192;
    hipLaunchKernelGGL(copy_envs_kernel, dim3(blocks), dim3(256), 0, s, envs, env_list, n_list, dst, src);
    return hipGetLastError();
}

}  // namespace firesim
