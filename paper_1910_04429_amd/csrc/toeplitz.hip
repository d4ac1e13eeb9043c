// Kernels of the Toeplitz-hash variant that the transform passes do not cover.
//
// The Toeplitz hash y = T x over GF(2), T[i][j] = t[i - j + n - 1], is the
// parity of a slice of the integer convolution of the bit sequences t and x:
// y_i = (t * x)[i + n - 1] mod 2.  The convolution runs on the transform passes
// with one element per bit over one prime (its coefficients are at most n, far
// below the prime, so the residues are the coefficients themselves); these
// kernels draw a seeded t and turn the coefficient residues into packed bits.
#include "kernels.h"
#include "splitmix.h"

namespace pa {
namespace {

__global__ __launch_bounds__(256) void k_stream_words(uint64_t seed, uint64_t words, uint64_t* out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words)
        out[i] = splitmix64(seed, i);
}

// One wavefront per output word: lane l reads coefficient base + 64 j + l and
// the wave's ballot of the low bits is the word.
__global__ __launch_bounds__(256) void k_parity(const uint32_t* __restrict__ res, uint64_t base,
                                                uint64_t m, uint64_t* __restrict__ out,
                                                int accumulate)
{
    const uint64_t words = (m + 63) >> 6;
    const uint64_t j = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (j >= words)
        return;                              // whole wavefronts leave together
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t i = 64 * j + lane;
    const int bit = (i < m) ? (int)(res[base + i] & 1u) : 0;
    const uint64_t word = __ballot(bit);
    if (lane == 0)
        out[j] = accumulate ? (out[j] ^ word) : word;
}

}  // namespace

hipError_t launch_parity(const uint32_t* res, uint64_t base, uint64_t m, uint64_t* out,
                         int accumulate, hipStream_t stream)
{
    const uint64_t words = (m + 63) >> 6;
    const unsigned blocks = (unsigned)((words + 3) / 4);
    hipLaunchKernelGGL(k_parity, dim3(blocks), dim3(256), 0, stream, res, base, m, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_stream_words(uint64_t seed, uint64_t words, uint64_t* out, hipStream_t stream)
{
    const unsigned blocks = (unsigned)((words + 255) / 256);
    hipLaunchKernelGGL(k_stream_words, dim3(blocks), dim3(256), 0, stream, seed, words, out);
    return hipGetLastError();
}

}  // namespace pa
