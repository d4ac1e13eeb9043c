// Host check of the LDS tile layout in swizzle.h, for every tile size the
// pass kernels use (2^k residues up to 2^14, and 3 2^k for the factor-3
// pass): the map must permute the tile onto itself (else a step would read or
// write LDS outside its tile), keep aligned 4-element groups whole and in
// order (the 16-byte tile loads and stores), and be linear over GF(2) (the
// steps form an index as swz(base) ^ swz(n nstep)).  Maps that break each
// property are run through the same checks, which must reject them.
#include <stdio.h>
#include <stdint.h>

#include <vector>

#include "swizzle.h"

namespace {

constexpr uint32_t kMaxTile = 1u << 14;

template <typename F>
int failures(F f)
{
    int bad = 0;
    std::vector<uint32_t> sizes;
    for (int k = 0; k <= 14; ++k) sizes.push_back(1u << k);
    for (int k = 2; k <= 12; ++k) sizes.push_back(3u << k);
    for (uint32_t N : sizes) {
        std::vector<char> seen(N, 0);
        for (uint32_t e = 0; e < N; ++e) {
            const uint32_t s = f(e);
            if (s >= N || seen[s]) {
                ++bad;
                break;
            }
            seen[s] = 1;
        }
    }
    for (uint32_t e = 0; e < kMaxTile; ++e)
        if (f(e) != (f(e & ~3u) | (e & 3u)) || (f(e & ~3u) & 3u) != 0) {
            ++bad;
            break;
        }
    if (f(0) != 0) ++bad;
    for (uint32_t e = 0; e < kMaxTile; ++e)
        for (uint32_t j = 1; j < kMaxTile; j <<= 1)
            if (f(e ^ j) != (f(e) ^ f(j))) {
                ++bad;
                e = kMaxTile;
                break;
            }
    return bad;
}

}  // namespace

int main()
{
    const int real = failures(pa::swz);
    // each breaks one property: leaves small tiles (element 8 of a 96-element
    // tile goes to 136); splits 4-groups; not linear; not injective
    const int planted[4] = {
        failures([](uint32_t e) { return e ^ (((e >> 2) & 15u) << 6); }),
        failures([](uint32_t e) { return e ^ (((e >> 6) & 15u) << 1); }),
        failures([](uint32_t e) { return e ^ ((((e >> 6) & 15u) + 1u) & 15u) << 2; }),
        failures([](uint32_t e) { return e & ~((e >> 6) & 1u); }),
    };
    if (real != 0) {
        fprintf(stderr, "swz fails %d checks\n", real);
        return 1;
    }
    for (int i = 0; i < 4; ++i)
        if (planted[i] == 0) {
            fprintf(stderr, "planted map %d passed the checks\n", i);
            return 1;
        }
    printf("ok: swz permutes every tile, keeps 4-groups, is linear; 4 planted maps rejected\n");
    return 0;
}
