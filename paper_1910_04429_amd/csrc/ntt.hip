// Multi-pass number-theoretic transform over the primes of field.h (five for
// 64-bit digits, seven for 96-bit digits).
//
// The product c*x is a cyclic convolution of the two digit vectors padded to a
// length L >= 2D - 1 (Alg. 1: fill zero, split, evaluate, pointwise multiply,
// interpolate).  A length-L transform is a short sequence of passes; each pass
// works on LDS tiles of at most 2^14 residues of one prime (64 KB) and reads
// and writes its array once.
//
// Pass structure (decimation in frequency).  With the array seen as L/(R S)
// blocks of R rows by S contiguous columns, a pass does a length-R transform
// down every column and multiplies output row k of column j by omega_{RS}^{j k}.
// The last pass has S = 1 (contiguous blocks of R); earlier passes take C
// adjacent columns per tile so that every row segment is a full 128-byte line.
//
// Inside a tile the length-R transform is itself split into steps of radix
// 2^r <= 16 (64 to 68 vector registers per lane: seven waves per SIMD).  A
// step loads each of its small DFTs from LDS into registers, runs the radix-2
// butterflies there with the omega_64 powers (compile-time constants of the
// prime), multiplies output k by b^k for a per-DFT base b, and writes back.
// The first step of a pass whose input is a residue array may read its DFTs
// straight from HBM, and the last step of a contiguous or inverse strided
// pass may write straight to HBM (see pass_tile).  The kernel body is
// instantiated once per prime and the workgroup picks its prime from
// blockIdx.y.
// For DIF step s on sub-blocks of size B split as n = n_s sigma + o the base is
// omega_B^o; a strided pass also folds its omega_{RS}^{j k} factor into the
// bases of its steps, so there is no separate twiddle sweep.
//
// Lengths L = 3 * 2^k put the factor 3 in the rows of the first pass, whose
// first register step is then a radix-3 DFT; all other index arithmetic stays
// in powers of two.  Twiddle exponents are counted in units of one root of
// order kOrder = 3 * 2^25, so every length shares one table.
//
// Outputs stay in the digit-reversed order that the steps produce; the inverse
// transform runs the same passes and steps backwards (decimation in time, with
// inverse roots and pre-multiplication), so no explicit reordering is done:
// both operands share the same scrambled spectrum, which the pointwise product
// does not care about.
#include "pass_body.h"

namespace pa {
namespace {

// One kernel per layout: W = 2 (64-bit digits, the first five primes; also the
// Toeplitz variant's bit sources over prime 0) and W = 3 (96-bit digits, all
// seven), so that neither carries the other's primes and sources.
// Each kind of pass (pass_kind) has its own instance, one for single blocks
// and one for batches (block from the job table; kJobs of block_view), so a
// kernel holds only the code of one kind.  The one-pass fused kind, which
// serves short blocks only, has one instance for both (kJobs 2): compiled for
// single blocks alone, its register allocation put scalar-spill reloads in
// its arithmetic loop.
template <int W, int kKind, int kJobs>
__global__ __launch_bounds__(kPassThreads) void k_pass(const PassArgs a)
{
    extern __shared__ uint32_t sm[];          // 4 N bytes
    pass_tile_kind<W, kKind, kJobs>(a, sm, blockIdx.y,
                                    TileCoord{blockIdx.x, gridDim.x, blockIdx.z, true});
}

template <int W, int kJobs>
void (*pass_kernel(int kind))(PassArgs)
{
    switch (kind) {
    case kKindFirst: return k_pass<W, kKindFirst, kJobs>;
    case kKindForward: return k_pass<W, kKindForward, kJobs>;
    case kKindFusedFirst: return k_pass<W, kKindFusedFirst, 2>;
    case kKindFused: return k_pass<W, kKindFused, kJobs>;
    default: return k_pass<W, kKindInverse, kJobs>;
    }
}

}  // namespace

hipError_t launch_pass(const PassArgs& a, hipStream_t stream, unsigned batch, const LaunchEvents& ev)
{
    const uint32_t N = ((uint32_t)a.f << a.r) << a.logC;
    const unsigned tiles = a.L / N;
    // one DFT of the first step per thread, between 1 and 4 waves
    const uint32_t first = a.f == 3 ? 3u : (1u << (a.steps_code & 15u));
    uint32_t threads = N / first;
    threads = threads < 64 ? 64 : (threads > kPassThreads ? kPassThreads : threads);
    const bool w3 = a.dwords == 3;
    if (a.primes < 1 || a.primes > (w3 ? 7 : 5)) return hipErrorInvalidValue;
    const unsigned primes = (unsigned)a.primes;
    const int kind = pass_kind(a);
    if (!pass_kind_fits(a, kind)) return hipErrorInvalidValue;
    const bool jobs = a.jobs != nullptr;
    auto kernel = w3 ? (jobs ? pass_kernel<3, 1>(kind) : pass_kernel<3, 0>(kind))
                     : (jobs ? pass_kernel<2, 1>(kind) : pass_kernel<2, 0>(kind));
    if (ev.start)
        hipExtLaunchKernelGGL(kernel, dim3(tiles, primes, batch), dim3(threads),
                              sizeof(uint32_t) * N, stream, ev.start, ev.stop, 0, a);
    else
        hipLaunchKernelGGL(kernel, dim3(tiles, primes, batch), dim3(threads),
                           sizeof(uint32_t) * N, stream, a);
    return hipGetLastError();
}

}  // namespace pa
