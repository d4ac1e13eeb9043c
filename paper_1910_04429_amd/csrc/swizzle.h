// LDS layout of a transform tile, shared by the pass kernels and a host check.
#pragma once

#include <stdint.h>

namespace pa {

// LDS index of tile element e: XOR of bits 2..5 with bits 6..9.  It only
// permutes the 16 aligned 4-element groups of each 64-element block (by one
// value per block), so it maps every tile, 2^k or 3 2^k elements, onto
// itself, keeps 4-element groups together for the 16-byte tile loads and
// stores, and spreads the step accesses over the banks: a wave's lanes
// differ in bits 4..9 in the radix-16 step of stride 16 and in the unit-stride
// steps of the strided tiles, and bits 6..9 land on bank bits 2..5.  It is
// linear over GF(2): the elements of one small DFT sit at base + n nstep with
// base and n nstep on disjoint bits, so their indices are
// swz(base) ^ swz(n nstep), one vector XOR with a wave-uniform term.
//
// A plain constexpr function, so the host can check those properties for
// every tile size.
constexpr uint32_t swz(uint32_t e) { return e ^ (((e >> 6) & 15u) << 2); }

}  // namespace pa
