// Workspace of the cooperative factor, per chain of a subdomain (host and device).
#pragma once
#include <cstdint>

namespace sfdd {

constexpr int F2_WAVES = 4;         // waves per factor workgroup
constexpr int F2_BLOCKS = 13;       // 16x16 accumulator blocks per wave

constexpr int F2_COUNTERS = 1;      // per chain counters: column parts published

// Block rows NT of a line matrix are owned in pairs (r, NT-1-r).  Up to 12
// block rows one workgroup ("rank") owns a pair; beyond that two ranks share
// a pair, one taking the tiles of even block columns and one of odd ones, so
// that a rank never holds more than 13 tiles.
constexpr int F2_SPLIT_NT = 12;
__host__ __device__ inline int f2_split(int NT) { return NT > F2_SPLIT_NT ? 2 : 1; }
__host__ __device__ inline int f2_ranks(int NT) { return f2_split(NT) * ((NT + 1) / 2); }

// doubles per chain: full symmetric inverse (mp x mp), two exchange columns
// of NT 32x32 tiles, two pivot-block and two pivot-inverse slots of tagged
// words (2 words per entry), build scratch of every rank
__host__ __device__ inline int64_t f2_chain_doubles(int mp, int NT) {
    return (int64_t)mp * mp + 2ll * NT * 1024 + 8ll * 1024 + (int64_t)f2_ranks(NT) * F2_WAVES * F2_BLOCKS * 256;
}

}  // namespace sfdd
