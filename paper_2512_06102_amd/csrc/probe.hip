// probe.hip -- HBM streaming probe: the attainable-bandwidth reference that
// the roofline figures of the step kernels are read against.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace firesim {
namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// HBM streaming probe: 16-byte accesses, four per lane in flight, grid-stride,
// nontemporal stores (the data is not read again).  MODE 0 reads src (a lane
// stores only if its xor equals a value no input here produces, so the loads
// stay), 1 writes dst, 2 copies src to dst.
template <int MODE>
__global__ __launch_bounds__(256) void stream_probe_kernel(const v4u* __restrict__ src, v4u* __restrict__ dst,
                                                           int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    v4u acc = {0u, 0u, 0u, 0u};
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        if constexpr (MODE == 1) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const v4u v = {(unsigned)(i + u * stride), 1u, 2u, 3u};
                __builtin_nontemporal_store(v, &dst[i + u * stride]);
            }
        } else {
            v4u v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = src[i + u * stride];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if constexpr (MODE == 2)
                    __builtin_nontemporal_store(v[u], &dst[i + u * stride]);
                else
                    acc ^= v[u];
            }
        }
    }
    for (; i < n; i += stride) {
        if constexpr (MODE == 1) {
            const v4u v = {(unsigned)i, 1u, 2u, 3u};
            __builtin_nontemporal_store(v, &dst[i]);
        } else if constexpr (MODE == 2) {
            __builtin_nontemporal_store(src[i], &dst[i]);
        } else {
            acc ^= src[i];
        }
    }
    if constexpr (MODE == 0)
        if (acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0xf39cc060u && acc.w == 0x5ced1fa1u)
            dst[blockIdx.x * 256 + threadIdx.x] = acc;
}

}  // namespace

hipError_t launch_stream_probe(hipStream_t s, int mode, const void* src, void* dst, int64_t n16, int blocks)
{
    const v4u* a = static_cast<const v4u*>(src);
    v4u* b = static_cast<v4u*>(dst);
    if (mode == 0)
        hipLaunchKernelGGL(stream_probe_kernel<0>, dim3(blocks), dim3(256), 0, s, a, b, n16);
    else if (mode == 1)
        hipLaunchKernelGGL(stream_probe_kernel<1>, dim3(blocks), dim3(256), 0, s, a, b, n16);
    else
        hipLaunchKernelGGL(stream_probe_kernel<2>, dim3(blocks), dim3(256), 0, s, a, b, n16);
    return hipGetLastError();
}

}  // namespace firesim
