// Device code of the carry step (CRT, column sums, carry scan, addend, mod
// 2^n and top-m extraction), shared by the carry kernels and the persistent
// batch kernel.  See carry.hip for the method.
#pragma once

#include "carryfn.h"
#include "kernels.h"
#include "splitmix.h"

namespace pa {
namespace {

// Inclusive scan of one function per lane over a wavefront, in lane order.
__device__ __forceinline__ uint32_t wave_scan(uint32_t f, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t prev = __shfl_up(f, d);
        if (lane >= d)
            f = carry_compose(prev, f);
    }
    return f;
}

// Addend digits t and t + 1 (t even: the two halves of one 64-bit word of
// d), low digit in the low half; 0 at and past D, the top digit masked to n bits.
__device__ __forceinline__ uint64_t addend_pair(const CarryArgs& a, uint32_t t)
{
    const uint32_t D = a.num_digits;
    if (t >= D)
        return 0;
    uint64_t w;
    if (a.addend_src == kSrcDigits) {
        const uint32_t lo = *gmem(a.addend + t);
        const uint32_t hi = (t + 1 < D) ? *gmem(a.addend + t + 1) : 0u;
        w = ((uint64_t)hi << 32) | lo;
    } else {
        w = splitmix64(a.seed, t >> 1);
    }
    // bits at and past n (the top digit's high bits, and digit t + 1 when t is
    // the last digit)
    const uint64_t keep = (uint64_t)D * 32 - a.n;   // bits of the top digit past n
    const uint32_t last = D - 1;
    if (t == last)
        w &= (0xFFFFFFFFull >> keep);
    else if (t + 1 == last)
        w &= ~0ull >> keep;
    return w;
}

// Exact coefficient from its residues over the first NP primes (Garner's mixed
// radix, then Horner in 32-bit words): z[0..NP), least significant first.
template <int NP>
__device__ __forceinline__ void crt(const uint32_t (&r)[NP], uint32_t (&z)[NP])
{
    uint32_t v[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const uint32_t p = kPrimes[i];
        uint32_t t = r[i];
#pragma unroll
        for (int j = 0; j < i; ++j) {
            // v_j < p_j < 2 p_i (every prime is above 2^30): reduce it, then
            // t + p - v_j < 2 p < 2^32 goes into Shoup's multiply unreduced
            const uint32_t vj = (kPrimes[j] > p) ? min(v[j], v[j] - p) : v[j];
            t = fmul_shoup(t + p - vj, kGarner.inv[i][j], kGarner.q[i][j], p);
        }
        v[i] = t;
    }
    z[0] = v[NP - 1];
#pragma unroll
    for (int i = NP - 2; i >= 0; --i) {
        const int words = NP - 1 - i;             // words of the accumulator so far
        uint64_t carry = v[i];
#pragma unroll
        for (int w = 0; w < words; ++w) {
            const uint64_t t = (uint64_t)z[w] * kPrimes[i] + carry;   // < 2^63 + 2^32
            z[w] = (uint32_t)t;
            carry = t >> 32;
        }
        z[words] = (uint32_t)carry;
    }
}

// Chunk-local digit i in [0, kChunk + 2) <-> LDS slot of the resolved digit,
// padded so that threads writing consecutive runs of kPer digits hit distinct
// banks.
template <int kPer>
__device__ __forceinline__ int slot(int i)
{
    return i + i / kPer;
}

// Batch mode: take the block's sizes, addend, state and output from its job.
__device__ __forceinline__ void bind_job(CarryArgs& a, uint32_t job)
{
    const auto* j = gmem(a.jobs + job);
    a.res = j->B;
    a.num_digits = j->num_digits;
    a.n = j->n;
    a.m = j->m;
    if (j->d) {
        a.addend_src = kSrcDigits;
        a.addend = j->d;
    } else {
        a.addend_src = kSrcSeed;
        a.seed = j->seed_b;
    }
    a.desc = j->carry;
    a.sums = j->A;
    a.out = j->out;
    a.chunks = j->chunks;
}

// Residues of coefficient K (0 outside [0, ceil(D / W))).
template <int W>
__device__ __forceinline__ void load_res(const CarryArgs& a, int64_t K, uint32_t (&r)[2 * W + 1])
{
    const int64_t coeffs = (a.num_digits + W - 1) / W;
#pragma unroll
    for (int pi = 0; pi < 2 * W + 1; ++pi)
        r[pi] = (K < 0 || K >= coeffs) ? 0u : *gmem(a.res + (size_t)pi * a.L + K);
}

// Exact coefficient K (0 outside the product's coefficients).
template <int W>
__device__ __forceinline__ void load_coeff(const CarryArgs& a, int64_t K, uint32_t (&z)[2 * W + 1])
{
    uint32_t r[2 * W + 1];
    load_res<W>(a, K, r);
    crt<2 * W + 1>(r, z);
}

// The LDS of one chunk: its resolved digits, the high words each thread passes
// to the next, the coefficient past the chunk and the per-wavefront scans.
template <int kPer, int W>
struct CarryShared {
    static constexpr int kChunk = kCarryThreads * kPer;
    static constexpr int kSlots = kChunk + 2 + (kChunk + 2) / kPer + 1;
    uint32_t val[kSlots];
    uint32_t hw[kCarryThreads + 1][W + 2];
    uint32_t tail[2];
    uint32_t wtot[kCarryThreads / 64];
    uint32_t wpre[kCarryThreads / 64];
};

// Column sums s[i] of digits kf + i, i < count (0 at and past D), from the
// residues: CRT of this thread's coefficients, the high words of the two
// before its first from the previous thread through LDS.
template <int kPer, int W>
__device__ __forceinline__ void column_sums(const CarryArgs& a, int64_t k0, int64_t kf, int count,
                                            uint64_t (&s)[kPer + 2], CarryShared<kPer, W>& sh)
{
    constexpr int NP = 2 * W + 1;
    constexpr int kExtra = 2;
    constexpr int kChunk = kCarryThreads * kPer;
    constexpr int kCo = kPer / W;              // coefficients per thread
    const int tid = threadIdx.x;
    const uint32_t D = a.num_digits;
    const int64_t K0 = kf / W;
    const int64_t coeffs = (D + W - 1) / W;
    // this thread's residues, vector loads when its coefficients lie inside
    // (K0 is a multiple of kCo, so they are aligned)
    uint32_t r[NP][kCo];
    if (K0 + kCo <= coeffs) {
#pragma unroll
        for (int pi = 0; pi < NP; ++pi) {
            const uint32_t* src = a.res + (size_t)pi * a.L + K0;
            if constexpr (kCo == 2) {
                const u32x2 q = *gmem(reinterpret_cast<const u32x2*>(src));
                r[pi][0] = q.x;
                r[pi][1] = q.y;
            } else {
#pragma unroll
                for (int v = 0; v < kCo / 4; ++v) {
                    const u32x4 q = *gmem(reinterpret_cast<const u32x4*>(src) + v);
                    r[pi][4 * v] = q.x;
                    r[pi][4 * v + 1] = q.y;
                    r[pi][4 * v + 2] = q.z;
                    r[pi][4 * v + 3] = q.w;
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < kCo; ++i) {
            uint32_t q[NP];
            load_res<W>(a, K0 + i, q);
#pragma unroll
            for (int pi = 0; pi < NP; ++pi) r[pi][i] = q[pi];
        }
    }
    // Exact coefficients of this thread.  The high words of the two before its
    // first come from the previous thread through LDS; for thread 0 they are
    // the chunk's boundary coefficients, and the last thread's two extra digits
    // need the coefficient past the chunk: lanes 0, 1 and 2 of wave 0 compute
    // one each, in one pass of the wave (a single lane in each of three waves
    // would cost three waves a pass each).
    uint32_t z[kCo][NP];
#pragma unroll
    for (int ci = 0; ci < kCo; ++ci) {
        uint32_t q[NP];
#pragma unroll
        for (int pi = 0; pi < NP; ++pi) q[pi] = r[pi][ci];
        crt<NP>(q, z[ci]);
    }
    // hw[t + 1] = words W .. 2 W of thread t's last coefficient, then word 2 W
    // of the one before it; hw[0] the same for the two coefficients before the
    // chunk
    auto& hw = sh.hw;
    auto& tail = sh.tail;
#pragma unroll
    for (int w = 0; w <= W; ++w) hw[tid + 1][w] = z[kCo - 1][W + w];
    hw[tid + 1][W + 1] = z[kCo - 2][2 * W];
    if (tid < 3) {
        const int64_t Kc = k0 / W;             // first coefficient of the chunk
        const int64_t K = tid == 0 ? Kc - 1 : (tid == 1 ? Kc - 2 : Kc + kChunk / W);
        uint32_t q[NP];
        load_coeff<W>(a, K, q);
        if (tid == 0) {
#pragma unroll
            for (int w = 0; w <= W; ++w) hw[0][w] = q[W + w];
        } else if (tid == 1) {
            hw[0][W + 1] = q[2 * W];
        } else {
            tail[0] = q[0];
            tail[1] = q[1];
        }
    }
    __syncthreads();
    {
        // prev[w] = word W + w of the previous coefficient (w <= W), prev2 =
        // word 2 W of the one before it
        uint32_t prev[W + 1];
#pragma unroll
        for (int w = 0; w <= W; ++w) prev[w] = hw[tid][w];
        uint32_t prev2 = hw[tid][W + 1];
        uint64_t dpair = 0;                    // addend digits i and i + 1, i even
#pragma unroll
        for (int ci = 0; ci < kCo + 1; ++ci) {
            const bool own = ci < kCo;
#pragma unroll
            for (int rr = 0; rr < W; ++rr) {
                const int i = W * ci + rr;
                if (i < count && i < kPer + kExtra) {
                    const uint32_t zw = own ? z[ci % kCo][rr] : (rr < 2 ? tail[rr % 2] : 0u);
                    const int64_t k = kf + i;
                    // kf is even (kPer is), so digit pairs are word-aligned
                    if ((i & 1) == 0)
                        dpair = (k < (int64_t)D) ? addend_pair(a, (uint32_t)k) : 0ull;
                    const uint32_t d = (i & 1) ? (uint32_t)(dpair >> 32) : (uint32_t)dpair;
                    s[i % (kPer + kExtra)] = (k < (int64_t)D)
                        ? (uint64_t)zw + prev[rr] + (rr == 0 ? prev2 : 0u) + d : 0ull;
                }
            }
            if (own) {
                prev2 = prev[W];
#pragma unroll
                for (int w = 0; w <= W; ++w) prev[w] = z[ci % kCo][W + w];
            }
        }
    }
}

// Store the column sums of this thread's kPer digits (those below D) for the
// apply kernel: their low words at digit positions, their bits 32..33 packed
// in one word per thread.  s < 2^34 (four terms below 2^32 each).
template <int kPer>
__device__ __forceinline__ void store_sums(const CarryArgs& a, int64_t kf, const uint64_t (&s)[kPer + 2])
{
    static_assert(kPer <= 16, "2 bits per digit in one word");
    const uint32_t D = a.num_digits;
    uint32_t hi = 0;
#pragma unroll
    for (int i = 0; i < kPer; ++i) hi |= (uint32_t)(s[i] >> 32) << (2 * i);
    if (kf + kPer <= (int64_t)D && kPer % 4 == 0) {
#pragma unroll
        for (int v = 0; v < kPer / 4; ++v)
            *gword<u32x4>(a.sums, (uint32_t)kf + 4 * v) =
                u32x4{(uint32_t)s[4 * v], (uint32_t)s[4 * v + 1], (uint32_t)s[4 * v + 2],
                      (uint32_t)s[4 * v + 3]};
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            if (kf + i < (int64_t)D)
                *gword(a.sums, (uint32_t)(kf + i)) = (uint32_t)s[i];
    }
    if (kf < (int64_t)D)
        *gword(a.sums, sums_hi_offset(D) + (uint32_t)(kf / kPer)) = hi;
}

// The column sums stored by the local kernel: this thread's kPer digits, and
// for the last thread of the chunk the two after them (the next chunk's first
// two, stored by its first thread); 0 at and past D.
template <int kPer>
__device__ __forceinline__ void load_sums(const CarryArgs& a, int64_t kf, int count, uint64_t (&s)[kPer + 2])
{
    const uint32_t D = a.num_digits;
#pragma unroll
    for (int i = 0; i < kPer + 2; ++i) s[i] = 0;
    if (kf >= (int64_t)D)
        return;
    const uint32_t hi = *gword(a.sums, sums_hi_offset(D) + (uint32_t)(kf / kPer));
    if (kf + kPer <= (int64_t)D && kPer % 4 == 0) {
#pragma unroll
        for (int v = 0; v < kPer / 4; ++v) {
            const u32x4 q = *gword<const u32x4>(a.sums, (uint32_t)kf + 4 * v);
            s[4 * v] = q.x;
            s[4 * v + 1] = q.y;
            s[4 * v + 2] = q.z;
            s[4 * v + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i)
            if (kf + i < (int64_t)D) s[i] = *gword(a.sums, (uint32_t)(kf + i));
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) s[i] |= (uint64_t)((hi >> (2 * i)) & 3u) << 32;
    if (count > kPer && kf + kPer < (int64_t)D) {
        const uint32_t nhi = *gword(a.sums, sums_hi_offset(D) + (uint32_t)(kf / kPer) + 1u);
#pragma unroll
        for (int i = 0; i < 2; ++i)
            if (kf + kPer + i < (int64_t)D)
                s[kPer + i] = *gword(a.sums, (uint32_t)(kf + kPer + i)) |
                              ((uint64_t)((nhi >> (2 * i)) & 3u) << 32);
    }
}

// One chunk of one block (job) of 256 threads.  kApply = false: write the
// chunk's carry function.  kApply = true: resolve the chunk with its carry-in
// and write its output words.  Returns early (uniformly) for chunks with
// nothing to do.
template <int kPer, bool kApply, int W>
__device__ __forceinline__ void carry_chunk(CarryArgs a, uint32_t chunk, uint32_t job,
                                            CarryShared<kPer, W>& sh)
{
    static_assert(kPer % W == 0, "a thread owns whole coefficients");
    if (a.jobs) {
        bind_job(a, job);
        if (chunk >= a.chunks)
            return;
    }
    constexpr int kChunk = kCarryThreads * kPer;
    auto& val = sh.val;

    const int tid = threadIdx.x;
    const int64_t k0 = (int64_t)chunk * kChunk;
    const uint32_t D = a.num_digits;
    // A chunk below bit n - m writes no output word (none starts in it): its
    // digits reach the output only through its carry function, which the local
    // kernel has written.
    if (kApply && (uint64_t)(k0 + kChunk) * 32 <= a.n - a.m)
        return;

    // column sums of this thread's kPer digits (and, for the last thread, the
    // two digits past the chunk, which it resolves with the chunk's carry-out);
    // its digits W K + r come from coefficients K, K - 1 and K - 2
    constexpr int kExtra = 2;
    uint64_t s[kPer + kExtra];
    const int first = tid * kPer;
    const int count = kPer + (tid == kCarryThreads - 1 ? kExtra : 0);
    const int64_t kf = k0 + first;             // a multiple of W
    // The apply kernel resolves only the chunks that reach the output window
    // (it returned above for the others); the local kernel stores their sums.
    if constexpr (kApply) {
        load_sums<kPer>(a, kf, count, s);
    } else {
        column_sums<kPer, W>(a, k0, kf, count, s, sh);
        if ((uint64_t)(k0 + kChunk) * 32 > a.n - a.m)
            store_sums<kPer>(a, kf, s);
    }
    uint32_t f = carry_fn_of_sum(s[0]);
#pragma unroll
    for (int i = 1; i < kPer; ++i)
        f = carry_compose(f, carry_fn_of_sum(s[i]));

    // inclusive scan of the thread functions in thread order: within each
    // wavefront by lane shuffles, then across the four wavefronts through LDS
    const int lane = tid & 63, wave = tid >> 6;
    f = wave_scan(f, lane);
    auto& wtot = sh.wtot;
    if (lane == 63)
        wtot[wave] = f;
    __syncthreads();
    uint32_t before = kCarryIdentity;              // the wavefronts before this one
    for (int w = 0; w < wave; ++w)
        before = carry_compose(before, wtot[w]);

    if (!kApply) {
        if (tid == kCarryThreads - 1)
            *gmem(a.desc + chunk) = carry_compose(before, f);
        return;
    }
    // carry entering this chunk: the functions of chunks 0 .. chunk-1 (written
    // by the local kernel) composed in order and applied to carry 0; each
    // workgroup reads the few thousand bytes itself instead of waiting for a
    // separate scan launch
    auto& wpre = sh.wpre;
    uint32_t cin_chunk;
    {
        const uint32_t per_t = (chunk + kCarryThreads - 1) / kCarryThreads;
        const uint32_t lo = (uint32_t)tid * per_t;
        uint32_t g = kCarryIdentity;
        for (uint32_t k = lo; k < lo + per_t && k < chunk; ++k)
            g = carry_compose(g, *gmem(a.desc + k));
        g = wave_scan(g, lane);
        if (lane == 63)
            wpre[wave] = g;
        __syncthreads();
        uint32_t all = kCarryIdentity;
#pragma unroll
        for (int w = 0; w < kCarryThreads / 64; ++w)
            all = carry_compose(all, wpre[w]);
        cin_chunk = carry_apply(all, 0u);
    }

    // resolve this thread's digits; V digits of the chunk (and two past it) to LDS
    uint32_t excl = __shfl_up(f, 1);          // inclusive scan of the lane before
    if (lane == 0)
        excl = kCarryIdentity;
    uint64_t carry = carry_apply(carry_compose(before, excl), cin_chunk);
    const uint32_t top = (uint32_t)(a.n & 31);
#pragma unroll
    for (int i = 0; i < kPer + kExtra; ++i) {
        if (i < count) {
            const int li = first + i;
            const int64_t k = k0 + li;
            const uint64_t t = s[i] + carry;
            uint32_t v = (uint32_t)t;
            carry = t >> 32;
            if (k >= (int64_t)D)
                v = 0;
            else if (k == (int64_t)D - 1 && top)
                v &= (1u << top) - 1u;
            val[slot<kPer>(li)] = v;
        }
    }
    __syncthreads();

    // output words whose first bit lies in this chunk: word j starts at bit
    // b_j = n - m + 64 j, in digit b_j / 32
    const uint64_t words = (a.m + 63) >> 6;
    const uint64_t base = a.n - a.m;
    const uint64_t lo_bit = (uint64_t)k0 * 32, hi_bit = lo_bit + (uint64_t)kChunk * 32;
    const uint64_t j_lo = lo_bit > base ? (lo_bit - base + 63) >> 6 : 0;
    uint64_t j_hi = hi_bit > base ? (hi_bit - base + 63) >> 6 : 0;
    if (j_hi > words) j_hi = words;
    for (uint64_t j = j_lo + tid; j < j_hi; j += kCarryThreads) {
        const uint64_t bit = base + 64 * j;
        const int q = (int)((bit >> 5) - (uint64_t)k0);   // in [0, kChunk)
        const uint32_t sh = (uint32_t)(bit & 31);
        const uint64_t v0 = val[slot<kPer>(q)], v1 = val[slot<kPer>(q + 1)],
                       v2 = val[slot<kPer>(q + 2)];
        uint64_t w = (v0 | (v1 << 32)) >> sh;
        if (sh) w |= v2 << (64 - sh);
        if (j == words - 1 && (a.m & 63))
            w &= (1ull << (a.m & 63)) - 1ull;
        *gmem(a.out + j) = w;
    }
}

}  // namespace
}  // namespace pa
