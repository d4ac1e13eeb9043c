// Prime-field arithmetic for the exact number-theoretic-transform multiply.
//
// The hash needs the low n bits of c*x (Section 2.3, the g_{c,d} definition;
// Section 3.2.2, the large multiply done by an NTT convolution as in Alg. 1).
// Operands are cut into digits of W = 2 or 3 32-bit words (64 or 96 bits); the
// convolution coefficients sum_{i+j=k} x_i c_j are below D 2^{64 W} and are
// recovered exactly by CRT from 2 W + 1 NTTs over 31-bit primes: five primes
// (product 2^153.4 > 2^23 2^128) for 64-bit digits, seven (product 2^215.2 >
// 2^22.5 2^192) for 96-bit digits, at every n up to 2^29 bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

constexpr int kNumPrimes = 7;
constexpr int kLogMaxLen = 25;                 // min 2-adicity of the first five primes
// Twiddle exponents are counted in units of one root of order kOrder =
// 3 * 2^25.  The first five primes are all the primes k 3 2^25 + 1 below 2^31
// (quotients 20, 18, 21, 17 and 11), so they have such a root and serve every
// length 2^k and 3 * 2^k up to kOrder.  The last two only have roots of order
// kOrder / 8 = 3 * 2^22: their root r stands for w^8, exponent E of w is power
// E / 8 of r, which is exact for every length L that divides 3 * 2^22 (all
// exponents used are multiples of kOrder / L, hence of 8).  They serve the
// 96-bit-digit layout only, whose transform lengths divide that order.
constexpr uint32_t kOrder = 3u << kLogMaxLen;
constexpr uint32_t kPrimes[kNumPrimes] = {
    2013265921u,  // 15 * 2^27 + 1
    1811939329u,  // 27 * 2^26 + 1
    2113929217u,  // 63 * 2^25 + 1
    1711276033u,  // 51 * 2^25 + 1
    1107296257u,  // 33 * 2^25 + 1
    2088763393u,  // 249 * 2^23 + 1
    2025848833u,  // 483 * 2^22 + 1
};
// log2 of kOrder / (order of the prime's root): 0 or 3.
constexpr int kRootShift[kNumPrimes] = {0, 0, 0, 0, 0, 3, 3};
// Every transform length of the seven-prime (96-bit digit) layout divides
// this; the five-prime layout's divide kOrder.  (2^23 <= 3 * 2^22 does not
// divide it: at L = 2^23 the exponent unit kOrder / L is 12.)
constexpr uint32_t kOrder96 = kOrder >> 3;

// -p^{-1} mod 2^32 by Newton iteration (each step doubles the correct bits).
constexpr uint32_t neg_inverse_u32(uint32_t p)
{
    uint32_t inv = p;  // correct to 3 bits for odd p
    for (int i = 0; i < 5; ++i)
        inv *= 2u - p * inv;
    return 0u - inv;
}

constexpr uint32_t kNegInv[kNumPrimes] = {
    neg_inverse_u32(kPrimes[0]), neg_inverse_u32(kPrimes[1]), neg_inverse_u32(kPrimes[2]),
    neg_inverse_u32(kPrimes[3]), neg_inverse_u32(kPrimes[4]), neg_inverse_u32(kPrimes[5]),
    neg_inverse_u32(kPrimes[6])};

constexpr uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t p)
{
    uint64_t r = 1 % p;
    b %= p;
    while (e) {
        if (e & 1) r = r * b % p;
        b = b * b % p;
        e >>= 1;
    }
    return r;
}

constexpr uint32_t inv_mod(uint64_t a, uint64_t p) { return (uint32_t)pow_mod(a, p - 2, p); }

// Montgomery form x 2^32 mod p of a constant.
constexpr uint32_t to_mont(uint64_t x, uint64_t p) { return (uint32_t)(((x % p) << 32) % p); }

// Smallest generator of the multiplicative group mod the prime p: g with
// g^((p-1)/q) != 1 for every prime q dividing p - 1 (trial division).
constexpr uint32_t primitive_root(uint64_t p)
{
    uint64_t f[8] = {};
    int nf = 0;
    uint64_t q = p - 1;
    for (uint64_t d = 2; d * d <= q; ++d) {
        if (q % d == 0) {
            f[nf++] = d;
            while (q % d == 0) q /= d;
        }
    }
    if (q > 1) f[nf++] = q;
    for (uint64_t g = 2; g < p; ++g) {
        bool ok = true;
        for (int i = 0; i < nf && ok; ++i)
            ok = pow_mod(g, (p - 1) / f[i], p) != 1;
        if (ok) return (uint32_t)g;
    }
    return 0;
}

// The root of unity of order kOrder that every twiddle is a power of.
constexpr uint32_t order_root(uint64_t p, int shift)
{
    return (uint32_t)pow_mod(primitive_root(p), (p - 1) / (kOrder >> shift), p);
}

constexpr uint32_t kRoot[kNumPrimes] = {
    order_root(kPrimes[0], kRootShift[0]), order_root(kPrimes[1], kRootShift[1]),
    order_root(kPrimes[2], kRootShift[2]), order_root(kPrimes[3], kRootShift[3]),
    order_root(kPrimes[4], kRootShift[4]), order_root(kPrimes[5], kRootShift[5]),
    order_root(kPrimes[6], kRootShift[6])};

// Shoup quotient floor(w 2^32 / p) of a constant w < p.
constexpr uint32_t shoup_quotient(uint64_t w, uint64_t p) { return (uint32_t)((w << 32) / p); }

// Garner's mixed-radix CRT over the first P primes: with v_0 = r_0 and
//   v_i = (...((r_i - v_0) p_0^{-1} - v_1) p_1^{-1} ... - v_{i-1}) p_{i-1}^{-1}  mod p_i,
// the coefficient is v_0 + p_0 (v_1 + p_1 (v_2 + ... + p_{P-2} v_{P-1})).
// kGarner.inv[i][j] is p_j^{-1} mod p_i (j < i) and q[i][j] its Shoup quotient.
struct GarnerTable {
    uint32_t inv[kNumPrimes][kNumPrimes];
    uint32_t q[kNumPrimes][kNumPrimes];
};
constexpr GarnerTable make_garner()
{
    GarnerTable t{};
    for (int i = 0; i < kNumPrimes; ++i)
        for (int j = 0; j < i; ++j) {
            t.inv[i][j] = inv_mod(kPrimes[j] % kPrimes[i], kPrimes[i]);
            t.q[i][j] = shoup_quotient(t.inv[i][j], kPrimes[i]);
        }
    return t;
}
constexpr GarnerTable kGarner = make_garner();

constexpr bool primes_ok()
{
    for (int i = 0; i < kNumPrimes; ++i) {
        const uint64_t p = kPrimes[i];
        // odd, 2^30 < p < 2^31: a residue of any of the primes is below 2 p
        if (p % 2 == 0 || p <= (1ull << 30) || p >= (1ull << 31)) return false;
        const uint64_t order = kOrder >> kRootShift[i];
        if ((p - 1) % order != 0) return false;
        if ((uint32_t)(kNegInv[i] * (uint32_t)p) != 0xFFFFFFFFu) return false;
        // the root has order exactly 3 * 2^25 (or 3 * 2^22)
        if (pow_mod(kRoot[i], order, p) != 1 || pow_mod(kRoot[i], order / 2, p) == 1 ||
            pow_mod(kRoot[i], order / 3, p) == 1)
            return false;
        for (int j = 0; j < i; ++j)
            if (kPrimes[j] == p) return false;
    }
    return true;
}
static_assert(primes_ok(), "seven distinct primes in (2^30, 2^31) with roots of order 3 * 2^25 "
                           "(the first five) or 3 * 2^22");

// ---------------------------------------------------------------------------
// Canonical residues in [0, p), p < 2^31.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t fadd(uint32_t a, uint32_t b, uint32_t p)
{
    uint32_t s = a + b;          // < 2p < 2^32
    return min(s, s - p);        // s - p wraps above s when s < p
}

__device__ __forceinline__ uint32_t fsub(uint32_t a, uint32_t b, uint32_t p)
{
    uint32_t d = a - b;          // wraps when a < b
    return min(d, d + p);
}

// x w mod p for any 32-bit x, with wq = floor(w 2^32 / p) precomputed (Shoup).
__device__ __forceinline__ uint32_t fmul_shoup(uint32_t x, uint32_t w, uint32_t wq, uint32_t p)
{
    uint32_t q = __umulhi(x, wq);
    uint32_t r = x * w - q * p;  // in [0, 2p)
    return min(r, r - p);
}

// a b 2^{-32} mod p (Montgomery reduction), a < p and b < 2p (t < 2 p^2).
__device__ __forceinline__ uint32_t fmul_mont(uint32_t a, uint32_t b, uint32_t p, uint32_t pneg)
{
    uint64_t t = (uint64_t)a * b;
    uint32_t m = (uint32_t)t * pneg;
    uint32_t u = (uint32_t)((t + (uint64_t)m * p) >> 32);  // < 2p
    return min(u, u - p);
}

// a b 2^{-32} mod p, left in [0, 2p): for a < 2p and b < p the sum t + m p is
// below 2 p^2 + 2^32 p, so the result is below p (2p / 2^32 + 1) < 2p.  Used
// for chains of twiddle powers, which feed another multiply, never an add.
__device__ __forceinline__ uint32_t fmul_mont_lazy(uint32_t a, uint32_t b, uint32_t p, uint32_t pneg)
{
    uint64_t t = (uint64_t)a * b;
    uint32_t m = (uint32_t)t * pneg;
    return (uint32_t)((t + (uint64_t)m * p) >> 32);
}

// v mod p for any 32-bit v: p > 2^30, so v < 4p and three conditional
// subtractions suffice (two when 3p > 2^32 - 1).
__device__ __forceinline__ uint32_t freduce32(uint32_t v, uint32_t p)
{
    if (3ull * p <= 0xFFFFFFFFull) {
        v = min(v, v - 2 * p);
        return min(v, v - p);
    }
    v = min(v, v - p);
    return min(v, v - p);
}

}  // namespace pa
