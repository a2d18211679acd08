// Workspace of the cooperative factor, per chain of a subdomain (host and device).
#pragma once
#include <cstdint>

namespace sfdd {

constexpr int F2_WAVES = 4;         // waves per factor workgroup
constexpr int F2_BLOCKS = 13;       // 16x16 accumulator blocks per wave

constexpr int F2_COUNTERS = 1;      // per chain counters: column parts published

// doubles per chain: full symmetric inverse (mp x mp), two exchange columns
// of NT 32x32 tiles, two pivot-block and two pivot-inverse slots of tagged
// words (2 words per entry), build scratch of ceil(NT/2) ranks
__host__ __device__ inline int64_t f2_chain_doubles(int mp, int NT) {
    return (int64_t)mp * mp + 2ll * NT * 1024 + 8ll * 1024 + (int64_t)((NT + 1) / 2) * F2_WAVES * F2_BLOCKS * 256;
}

}  // namespace sfdd
