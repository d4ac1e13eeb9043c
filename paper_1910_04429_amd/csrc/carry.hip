// CRT, carry propagation, addend, mod 2^n and top-m extraction in one pass.
//
// After the inverse transform, position k < D holds the convolution
// coefficient z_k = sum_{i+j=k} x_i c_j modulo each prime.  Garner's CRT turns
// the three residues into the exact z_k < 2^93 (three 32-bit words).  Then
// (Alg. 1, combine and carry; the addition of mpz_addmul; the mod 2^n of
// Section 3.2.3; the export and top-r selection of Sections 3.2.4-3.2.5)
//
//   s_k = lo32(z_k) + mid32(z_{k-1}) + hi32(z_{k-2}) + d_k        (s_k < 2^34)
//   V_k = (s_k + carry_k) mod 2^32,   carry_{k+1} = (s_k + carry_k) >> 32,
//
// with carry_0 = 0 and every carry in [0, 3].  Digits k >= D are discarded
// (mod 2^n), the top digit is masked to n bits, and bits [n - m, n) of V are the
// output.  The chain is a scan of carry-transfer functions f_k : {0..3} ->
// {0..3}, f_k(c) = (s_k + c) >> 32, packed 2 bits per input in one byte;
// composition is associative.
//
// Two launches, none of which waits on another workgroup: (1) every chunk of
// digits loads its threads' residues, forms its column sums and scans its
// threads' carry functions into the chunk's function; (2) every chunk composes
// the functions of the chunks before it (a few thousand bytes) into its
// carry-in, redoes (1), resolves its digits (and two past its end) and writes
// every output word that starts inside the chunk.  Workgroups on different
// XCDs never exchange data inside a kernel.
#include "kernels.h"

namespace pa {
namespace {

constexpr uint32_t kIdentity = 0xE4u;   // f(c) = c for c = 0..3

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Apply f then g.
__device__ __forceinline__ uint32_t compose(uint32_t f, uint32_t g)
{
    uint32_t h = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        h |= ((g >> (2 * ((f >> (2 * c)) & 3u))) & 3u) << (2 * c);
    return h;
}

__device__ __forceinline__ uint32_t apply(uint32_t f, uint32_t c) { return (f >> (2 * c)) & 3u; }

__device__ __forceinline__ uint32_t digit_function(uint64_t s)
{
    uint32_t f = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c)
        f |= (uint32_t)((s + (uint64_t)c) >> 32) << (2 * c);
    return f;
}

__device__ __forceinline__ uint32_t addend_digit(const CarryArgs& a, uint32_t t)
{
    if (t >= a.num_digits)
        return 0;
    uint32_t v;
    if (a.addend_src == kSrcDigits) {
        v = a.addend[t];
    } else {
        const uint64_t w = splitmix64(a.seed, t >> 1);
        v = (t & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
    }
    const uint32_t top = (uint32_t)(a.n & 31);
    if (t == a.num_digits - 1 && top)
        v &= (1u << top) - 1u;
    return v;
}

// Exact coefficient from its three residues (Garner).
__device__ __forceinline__ void crt(uint32_t r0, uint32_t r1, uint32_t r2, uint32_t& z0,
                                    uint32_t& z1, uint32_t& z2)
{
    constexpr uint32_t p0 = kPrimes[0], p1 = kPrimes[1], p2 = kPrimes[2];
    const uint32_t v0 = r0;
    const uint32_t v1 = fmul_mont(fsub(r1, min(v0, v0 - p1), p1), kInvP0ModP1M, p1, kNegInv[1]);
    const uint32_t t = fsub(r2, v0, p2);
    const uint32_t u = fmul_mont(v1, kP0ModP2M, p2, kNegInv[2]);
    const uint32_t v2 = fmul_mont(fsub(t, u, p2), kInvP01ModP2M, p2, kNegInv[2]);
    const uint64_t a = (uint64_t)p0 * v1 + v0;          // < p0 p1 < 2^62
    const uint64_t lo = kP01 * (uint64_t)v2;
    uint64_t hi = __umul64hi(kP01, (uint64_t)v2);
    const uint64_t zl = a + lo;
    hi += (zl < a);
    z0 = (uint32_t)zl;
    z1 = (uint32_t)(zl >> 32);
    z2 = (uint32_t)hi;
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
    const JobDesc& j = a.jobs[job];
    a.res = j.B;
    a.num_digits = j.num_digits;
    a.n = j.n;
    a.m = j.m;
    if (j.d) {
        a.addend_src = kSrcDigits;
        a.addend = j.d;
    } else {
        a.addend_src = kSrcSeed;
        a.seed = j.seed_b;
    }
    a.desc = j.carry;
    a.out = j.out;
    a.chunks = j.chunks;
}

// Residues of digit k (0 outside [0, D)).
__device__ __forceinline__ void load_res(const CarryArgs& a, int64_t k, uint32_t& r0, uint32_t& r1,
                                         uint32_t& r2)
{
    if (k < 0 || k >= (int64_t)a.num_digits) {
        r0 = r1 = r2 = 0;
        return;
    }
    r0 = a.res[k];
    r1 = a.res[(size_t)a.L + k];
    r2 = a.res[2 * (size_t)a.L + k];
}

// kApply = false: write the chunk's carry function.  kApply = true: resolve the
// chunk with its carry-in and write its output words.
template <int kPer, bool kApply>
__global__ __launch_bounds__(kCarryThreads) void k_carry(CarryArgs a)
{
    if (a.jobs) {
        bind_job(a, blockIdx.y);
        if (blockIdx.x >= a.chunks)
            return;
    }
    constexpr int kChunk = kCarryThreads * kPer;
    constexpr int kSlots = kChunk + 2 + (kChunk + 2) / kPer + 1;
    __shared__ uint32_t val[kSlots];
    __shared__ uint32_t scan[kCarryThreads];

    const int tid = threadIdx.x;
    const uint32_t chunk = blockIdx.x;
    const int64_t k0 = (int64_t)chunk * kChunk;
    const uint32_t D = a.num_digits;

    // column sums of this thread's kPer digits (and, for the last thread, the
    // two digits past the chunk, which it resolves with the chunk's carry-out)
    constexpr int kExtra = 2;
    uint64_t s[kPer + kExtra];
    const int first = tid * kPer;
    const int count = kPer + (tid == kCarryThreads - 1 ? kExtra : 0);
    const int64_t kf = k0 + first;
    // this thread's residues, 16-byte loads when the run lies inside [0, D)
    uint32_t r[3][kPer];
    if (kf + kPer <= (int64_t)D) {
#pragma unroll
        for (int pi = 0; pi < kNumPrimes; ++pi) {
            const uint4* src = reinterpret_cast<const uint4*>(a.res + (size_t)pi * a.L + kf);
#pragma unroll
            for (int v = 0; v < kPer / 4; ++v) {
                const uint4 q = src[v];
                r[pi][4 * v] = q.x;
                r[pi][4 * v + 1] = q.y;
                r[pi][4 * v + 2] = q.z;
                r[pi][4 * v + 3] = q.w;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < kPer; ++i) load_res(a, kf + i, r[0][i], r[1][i], r[2][i]);
    }
    {
        uint32_t z0, z1, z2, q0, q1, q2;
        load_res(a, kf - 2, q0, q1, q2);
        crt(q0, q1, q2, z0, z1, z2);
        uint32_t prev2_hi = z2;
        load_res(a, kf - 1, q0, q1, q2);
        crt(q0, q1, q2, z0, z1, z2);
        uint32_t prev_mid = z1, prev_hi = z2;
#pragma unroll
        for (int i = 0; i < kPer + kExtra; ++i) {
            if (i < count) {
                if (i < kPer) {
                    crt(r[0][i], r[1][i], r[2][i], z0, z1, z2);
                } else {
                    load_res(a, kf + i, q0, q1, q2);
                    crt(q0, q1, q2, z0, z1, z2);
                }
                const int64_t k = kf + i;
                const uint32_t d = (k < (int64_t)D) ? addend_digit(a, (uint32_t)k) : 0u;
                s[i] = (k < (int64_t)D) ? (uint64_t)z0 + prev_mid + prev2_hi + d : 0ull;
                prev2_hi = prev_hi;
                prev_mid = z1;
                prev_hi = z2;
            }
        }
    }
    uint32_t f = kIdentity;
#pragma unroll
    for (int i = 0; i < kPer; ++i)
        f = compose(f, digit_function(s[i]));

    // inclusive scan of the thread functions in thread order
    scan[tid] = f;
    __syncthreads();
    for (int d = 1; d < kCarryThreads; d <<= 1) {
        const uint32_t prev = (tid >= d) ? scan[tid - d] : kIdentity;
        __syncthreads();
        f = compose(prev, f);
        scan[tid] = f;
        __syncthreads();
    }

    if (!kApply) {
        if (tid == kCarryThreads - 1)
            a.desc[chunk] = f;
        return;
    }
    // carry entering this chunk: the functions of chunks 0 .. chunk-1 (written
    // by the local kernel) composed in order and applied to carry 0; each
    // workgroup reads the few thousand bytes itself instead of waiting for a
    // separate scan launch
    __shared__ uint32_t pre[kCarryThreads];
    {
        const uint32_t per_t = (chunk + kCarryThreads - 1) / kCarryThreads;
        const uint32_t lo = (uint32_t)tid * per_t;
        uint32_t g = kIdentity;
        for (uint32_t k = lo; k < lo + per_t && k < chunk; ++k)
            g = compose(g, a.desc[k]);
        pre[tid] = g;
        __syncthreads();
        for (int d = 1; d < kCarryThreads; d <<= 1) {
            if ((tid & (2 * d - 1)) == 0)
                pre[tid] = compose(pre[tid], pre[tid + d]);
            __syncthreads();
        }
    }
    const uint32_t cin_chunk = apply(pre[0], 0u);

    // resolve this thread's digits; V digits of the chunk (and two past it) to LDS
    uint64_t carry = tid ? apply(scan[tid - 1], cin_chunk) : cin_chunk;
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
        a.out[j] = w;
    }
}

}  // namespace

#ifndef PA_CARRY_PER_LARGE
#define PA_CARRY_PER_LARGE 8
#endif

int carry_digits_per_thread(uint32_t num_digits)
{
    return num_digits >= (1u << 18) ? PA_CARRY_PER_LARGE : 4;
}

template <typename K>
void launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t stream, const LaunchEvents& ev,
                  const CarryArgs& a)
{
    if (ev.start)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, ev.start, ev.stop, 0, a);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, stream, a);
}

template <bool kApply>
void launch_chunks(const CarryArgs& a, hipStream_t stream, unsigned batch, const LaunchEvents& ev)
{
    const dim3 grid(a.chunks, batch);
    switch (a.per) {
    case 16: launch_timed(k_carry<16, kApply>, grid, dim3(kCarryThreads), stream, ev, a); break;
    case 8: launch_timed(k_carry<8, kApply>, grid, dim3(kCarryThreads), stream, ev, a); break;
    default: launch_timed(k_carry<4, kApply>, grid, dim3(kCarryThreads), stream, ev, a); break;
    }
}

hipError_t launch_carry_local(const CarryArgs& a, hipStream_t stream, unsigned batch,
                              const LaunchEvents& ev)
{
    launch_chunks<false>(a, stream, batch, ev);
    return hipGetLastError();
}

hipError_t launch_carry_apply(const CarryArgs& a, hipStream_t stream, unsigned batch,
                              const LaunchEvents& ev)
{
    launch_chunks<true>(a, stream, batch, ev);
    return hipGetLastError();
}

}  // namespace pa
