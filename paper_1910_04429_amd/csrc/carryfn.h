// Carry-transfer functions of the carry scan (Alg. 1, combine and carry).
//
// Position k of the product has a column sum s_k < 2^34 and takes a carry
// c in {0..3} from below; it passes on (s_k + c) >> 32, also in {0..3}.  With
// s = hi 2^32 + lo that is
//
//     f(c) = hi + [c >= t],  t = 2^32 - lo,
//
// a non-decreasing step of at most one: a base b = f(0) and a threshold t
// (t >= 4: no step within {0..3}).  Such functions are closed under
// composition: if f has range {b_f, b_f + 1} and g is one of them, then
//
//     (g o f)(c) = g(b_f) + [c >= t_f] (g(b_f + 1) - g(b_f)),
//     g(b_f) = b_g + [b_f >= t_g],  g(b_f + 1) - g(b_f) = [b_f + 1 == t_g],
//
// so a run of positions also maps its carry-in to its carry-out by one such
// function.  A function is stored as b | t << 2 (b in 0..3, t in 1..4); the
// identity c -> c, which is not of this form, is kCarryIdentity.  These are
// plain constexpr functions, usable on the host as well as in kernels.
#pragma once

#include <stdint.h>

namespace pa {

constexpr uint32_t kCarryIdentity = 0x80u;

// The function of one position with column sum s (s + 3 < 2^34).
constexpr uint32_t carry_fn_of_sum(uint64_t s)
{
    const uint32_t hi = (uint32_t)(s >> 32);
    const uint32_t lo = (uint32_t)s;
    const uint32_t t = (lo > 0xFFFFFFFCu) ? (0u - lo) : 4u;   // 2^32 - lo when below 4
    return hi | (t << 2);
}

// f applied to the carry c.
constexpr uint32_t carry_apply(uint32_t f, uint32_t c)
{
    return (f & kCarryIdentity) ? c : (f & 3u) + (c >= (f >> 2) ? 1u : 0u);
}

// f, then g.
constexpr uint32_t carry_compose(uint32_t f, uint32_t g)
{
    const uint32_t bf = f & 3u, tf = (f >> 2) & 7u;
    const uint32_t bg = g & 3u, tg = (g >> 2) & 7u;
    const uint32_t b = bg + (bf >= tg ? 1u : 0u);
    const uint32_t t = (bf + 1u == tg) ? tf : 4u;
    const uint32_t h = b | (t << 2);
    return (f & kCarryIdentity) ? g : ((g & kCarryIdentity) ? f : h);
}

}  // namespace pa
