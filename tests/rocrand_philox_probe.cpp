// Independent Philox4x32-10: rocRAND's host-callable engine, exposed for the
// oracle's Philox test.  Built by the test with hipcc as host code.
#include <rocrand/rocrand_philox4x32_10.h>

namespace {
struct Probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
}  // namespace

extern "C" void rocrand_philox_blocks(const unsigned* ctr, const unsigned* key, unsigned* out, long n)
{
    Probe p;
    for (long i = 0; i < n; ++i) {
        uint4 c = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
        uint2 k = {key[2 * i], key[2 * i + 1]};
        uint4 r = p.block(c, k);
        out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
    }
}
