// The seed expansion of the multiplier c and the addend d on the device: word
// i of the stream of seed s is SplitMix64 output i (Steele, Lea and Flood,
// OOPSLA 2014), computed from its counter, so any word can be drawn alone.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

// SplitMix64 output i for `seed` (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace pa
