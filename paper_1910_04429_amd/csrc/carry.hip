// CRT, carry propagation, addend, mod 2^n and top-m extraction.
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
// output.  The carry chain is resolved as a scan of carry-transfer functions
// f_k : {0..3} -> {0..3}, f_k(c) = (s_k + c) >> 32, packed 2 bits per input in
// one byte; composition is associative, so chunks and threads scan in parallel.
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

// Exact coefficient z_k from its residues (Garner).  k < D <= L.
__device__ __forceinline__ void crt(const uint32_t* res, uint32_t L, uint32_t k, uint32_t& z0,
                                    uint32_t& z1, uint32_t& z2)
{
    constexpr uint32_t p0 = kPrimes[0], p1 = kPrimes[1], p2 = kPrimes[2];
    const uint32_t r0 = res[k], r1 = res[L + k], r2 = res[2 * (size_t)L + k];
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

// Column sums s_k for this thread's kCarryPerThread digits starting at k0.
__device__ void column_sums(const CarryArgs& a, uint32_t k0, uint64_t* s)
{
    uint32_t zm1_1 = 0, zm1_2 = 0, zm2_2 = 0;   // mid/hi words of z_{k-1}, hi of z_{k-2}
    // Halo: z_{k0-2} and z_{k0-1}.
    if (k0 >= 2) {
        uint32_t a0, a1, a2;
        crt(a.res, a.L, k0 - 2, a0, a1, a2);
        zm2_2 = a2;
    }
    if (k0 >= 1) {
        uint32_t a0, a1, a2;
        crt(a.res, a.L, k0 - 1, a0, a1, a2);
        zm1_1 = a1;
        zm1_2 = a2;
        // z_{k0-1} is k-1 for digit k0, and k-2 for digit k0+1
    }
    uint32_t prev_mid = zm1_1, prev_hi = zm1_2, prev2_hi = zm2_2;
    for (int i = 0; i < kCarryPerThread; ++i) {
        const uint32_t k = k0 + i;
        if (k >= a.num_digits) {
            s[i] = 0;
            continue;
        }
        uint32_t z0, z1, z2;
        crt(a.res, a.L, k, z0, z1, z2);
        s[i] = (uint64_t)z0 + prev_mid + prev2_hi + addend_digit(a, k);
        prev2_hi = prev_hi;
        prev_mid = z1;
        prev_hi = z2;
    }
}

// Inclusive scan of carry functions over the block, in thread order.
__device__ uint32_t block_scan_inclusive(uint32_t f, uint32_t* sh)
{
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int d = 1; d < (int)blockDim.x; d <<= 1) {
        uint32_t prev = (threadIdx.x >= (unsigned)d) ? sh[threadIdx.x - d] : kIdentity;
        __syncthreads();
        f = compose(prev, f);
        sh[threadIdx.x] = f;
        __syncthreads();
    }
    return f;
}

__global__ __launch_bounds__(kCarryThreads) void k_carry_chunk(CarryArgs a)
{
    __shared__ uint32_t sh[kCarryThreads];
    const uint32_t k0 = blockIdx.x * kCarryChunk + threadIdx.x * kCarryPerThread;
    uint64_t s[kCarryPerThread];
    column_sums(a, k0, s);
    uint32_t f = kIdentity;
    for (int i = 0; i < kCarryPerThread; ++i)
        f = compose(f, digit_function(s[i]));
    f = block_scan_inclusive(f, sh);
    if (threadIdx.x == kCarryThreads - 1)
        a.desc[blockIdx.x] = (uint8_t)f;
}

// One block: carry into every chunk from the chunk functions.
__global__ __launch_bounds__(1024) void k_carry_scan(CarryArgs a)
{
    __shared__ uint32_t sh[1024];
    const uint32_t per = (a.chunks + 1023) / 1024;
    const uint32_t j0 = threadIdx.x * per;
    uint32_t f = kIdentity;
    for (uint32_t j = j0; j < j0 + per && j < a.chunks; ++j)
        f = compose(f, a.desc[j]);
    const uint32_t incl = block_scan_inclusive(f, sh);
    __syncthreads();
    sh[threadIdx.x] = incl;
    __syncthreads();
    uint32_t c = threadIdx.x ? apply(sh[threadIdx.x - 1], 0) : 0u;
    for (uint32_t j = j0; j < j0 + per && j < a.chunks; ++j) {
        a.carry_in[j] = (uint8_t)c;
        c = apply(a.desc[j], c);
    }
}

__global__ __launch_bounds__(kCarryThreads) void k_carry_apply(CarryArgs a)
{
    __shared__ uint32_t sh[kCarryThreads];
    const uint32_t k0 = blockIdx.x * kCarryChunk + threadIdx.x * kCarryPerThread;
    uint64_t s[kCarryPerThread];
    column_sums(a, k0, s);
    uint32_t f = kIdentity;
    for (int i = 0; i < kCarryPerThread; ++i)
        f = compose(f, digit_function(s[i]));
    const uint32_t incl = block_scan_inclusive(f, sh);
    __syncthreads();
    sh[threadIdx.x] = incl;
    __syncthreads();
    const uint32_t cin_chunk = a.carry_in[blockIdx.x];
    uint64_t carry = threadIdx.x ? apply(sh[threadIdx.x - 1], cin_chunk) : cin_chunk;

    const uint32_t first = (uint32_t)((a.n - a.m) >> 5);   // lowest digit of the output
    const uint32_t top = (uint32_t)(a.n & 31);
    for (int i = 0; i < kCarryPerThread; ++i) {
        const uint32_t k = k0 + i;
        if (k >= a.num_digits)
            break;
        const uint64_t t = s[i] + carry;
        uint32_t v = (uint32_t)t;
        carry = t >> 32;
        if (k == a.num_digits - 1 && top)
            v &= (1u << top) - 1u;
        if (k >= first)
            a.value[k] = v;
    }
}

// Output word j = bits [n - m + 64 j, n - m + 64 j + 64) of V, masked to m bits.
__global__ __launch_bounds__(256) void k_extract(CarryArgs a)
{
    const uint64_t words = (a.m + 63) >> 6;
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= words)
        return;
    const uint64_t bit = (a.n - a.m) + 64 * j;
    const uint32_t q = (uint32_t)(bit >> 5);
    const uint32_t sh = (uint32_t)(bit & 31);
    const uint32_t D = a.num_digits;
    const uint64_t v0 = q < D ? a.value[q] : 0;
    const uint64_t v1 = q + 1 < D ? a.value[q + 1] : 0;
    const uint64_t v2 = q + 2 < D ? a.value[q + 2] : 0;
    uint64_t w = (v0 | (v1 << 32)) >> sh;
    if (sh)
        w |= v2 << (64 - sh);
    if (j == words - 1 && (a.m & 63))
        w &= (1ull << (a.m & 63)) - 1ull;
    a.out[j] = w;
}

}  // namespace

hipError_t launch_carry_chunk(const CarryArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_carry_chunk, dim3(a.chunks), dim3(kCarryThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_carry_scan(const CarryArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_carry_scan, dim3(1), dim3(1024), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_carry_apply(const CarryArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_carry_apply, dim3(a.chunks), dim3(kCarryThreads), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_extract(const CarryArgs& a, hipStream_t stream)
{
    const uint64_t words = (a.m + 63) >> 6;
    hipLaunchKernelGGL(k_extract, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace pa
