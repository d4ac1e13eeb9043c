// CRT, carry propagation, addend, mod 2^n and top-m extraction in one pass.
//
// After the inverse transform, position K < ceil(n / 32 W) holds the
// convolution coefficient Z_K = sum_{i+j=K} x_i c_j of the digits of W 32-bit
// words modulo each of the P = 2 W + 1 primes.  Garner's CRT turns the
// residues into the exact Z_K (below 2^{64 W + 23}), P 32-bit words z_K[0..P)
// that sit at 32-bit digit positions W K .. W K + 2 W of the product.  Then
// (Alg. 1, combine and carry; the addition of mpz_addmul; the mod 2^n of
// Section 3.2.3; the export and top-r selection of Sections 3.2.4-3.2.5), over
// 32-bit digit positions k = W K + r, r < W,
//
//   s_k = z_K[r] + z_{K-1}[r + W] + (r == 0 ? z_{K-2}[2 W] : 0) + d_k   (s < 2^34)
//   V_k = (s_k + carry_k) mod 2^32,   carry_{k+1} = (s_k + carry_k) >> 32,
//
// with carry_0 = 0 and every carry in [0, 3].  Digits k >= D = ceil(n/32) are
// discarded (mod 2^n), the top digit is masked to n bits, and bits [n - m, n)
// of V are the output.  The chain is a scan of the carry-transfer functions
// f_k(c) = (s_k + c) >> 32 of carryfn.h; composition is associative.
//
// Two launches, none of which waits on another workgroup: (1) every chunk of
// digits loads its threads' residues, forms its column sums and scans its
// threads' carry functions into the chunk's function; a chunk that reaches the
// output window also stores its column sums (34 bits each, in the multiplier
// spectrum's array, free by then); (2) every such chunk composes the functions
// of the chunks before it (a few thousand bytes) into its carry-in, reloads
// its column sums, resolves its digits (and two past its end) and writes every
// output word that starts inside the chunk.  Workgroups on different XCDs
// never exchange data inside a kernel.
#include "carry_body.h"

namespace pa {
namespace {

template <int kPer, bool kApply, int W>
__global__ __launch_bounds__(kCarryThreads) void k_carry(CarryArgs a)
{
    __shared__ CarryShared<kPer, W> sh;
    carry_chunk<kPer, kApply, W>(a, blockIdx.x, blockIdx.y, sh);
}

}  // namespace

#ifndef PA_CARRY_PER_LARGE
#define PA_CARRY_PER_LARGE 8
#endif

int carry_digits_per_thread(uint32_t num_digits, int W)
{
    if (W == 3)
        return num_digits >= (1u << 20) ? 12 : 6;
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
    if (a.dwords == 3) {
        if (a.per == 12)
            launch_timed(k_carry<12, kApply, 3>, grid, dim3(kCarryThreads), stream, ev, a);
        else
            launch_timed(k_carry<6, kApply, 3>, grid, dim3(kCarryThreads), stream, ev, a);
        return;
    }
    switch (a.per) {
    case 16: launch_timed(k_carry<16, kApply, 2>, grid, dim3(kCarryThreads), stream, ev, a); break;
    case 8: launch_timed(k_carry<8, kApply, 2>, grid, dim3(kCarryThreads), stream, ev, a); break;
    default: launch_timed(k_carry<4, kApply, 2>, grid, dim3(kCarryThreads), stream, ev, a); break;
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
