// philox.hpp -- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) for gfx950.
// Ten rounds of two 32x32->64 multiplies with the published multipliers and
// Weyl key increments.  Used by the draw contract: key = (seed lo, seed hi),
// counter top byte = draw domain (1 gap, 2 branch, 3 random measurement,
// 4 active-measurement uniform).
#pragma once

#include <hip/hip_runtime.h>

namespace symft {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

}  // namespace symft
