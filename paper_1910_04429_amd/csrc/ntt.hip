// Multi-pass number-theoretic transform over the three primes of field.h.
//
// The product c*x is a cyclic convolution of the two digit vectors padded to a
// length L >= 2D - 1 (Alg. 1: fill zero, split, evaluate, pointwise multiply,
// interpolate).  A length-L transform is done as a sequence of passes: pass i
// takes length-R_i transforms down the rows of R_i x S_i blocks (S_i the
// product of the later radices) and multiplies output row k of column c by
// omega_{R_i S_i}^{c k}; the last pass (S = 1) works on contiguous blocks and
// leaves them in bit-reversed order.  The inverse runs the passes in reverse
// with inverse roots, pre-twiddles and decimation in time, so no explicit
// reordering is ever done: both operands share the same scrambled spectrum
// layout, which the pointwise product does not care about.
#include "kernels.h"

namespace pa {
namespace {

// SplitMix64 output i for `seed` (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t bitrev(uint32_t x, int bits)
{
    return bits == 0 ? 0u : (__brev(x) >> (32 - bits));
}

// Digit t of the operand described by the pass source (0 beyond the top digit).
__device__ __forceinline__ uint32_t source_digit(const PassArgs& a, uint32_t t)
{
    if (t >= a.num_digits)
        return 0;
    uint32_t v;
    if (a.src == kSrcDigits) {
        v = a.digits[t];
    } else {
        uint64_t w = splitmix64(a.seed, t >> 1);
        v = (t & 1) ? (uint32_t)(w >> 32) : (uint32_t)w;
        if (t == 0)
            v |= 1u;  // the multiplier must be odd (eq. (6))
    }
    const uint32_t top = (uint32_t)(a.n & 31);
    if (t == a.num_digits - 1 && top)
        v &= (1u << top) - 1u;
    return v;
}

// Montgomery form of omega_{2^25}^E.
__device__ __forceinline__ uint32_t pass_twiddle(const Tables& tb, int pi, uint32_t E,
                                                 uint32_t p, uint32_t pneg)
{
    const uint32_t lo = tb.pass_lo[pi * 4096 + (E & 4095u)];
    const uint32_t hi = tb.pass_hi[pi * 8192 + (E >> 12)];
    return fmul_mont(lo, hi, p, pneg);
}

// Radix-2 decimation-in-frequency transforms of length R = 2^r down the rows of
// `ncols` columns held in LDS as (g, row, cc) -> (g R + row) C + cc, col = g C + cc.
// Natural-order input, bit-reversed output.
template <bool kInv>
__device__ void lds_dif(uint32_t* sm, int r, int logC, int ncols, const uint2* tw, uint32_t p)
{
    const int halfR = (1 << r) >> 1;
    const int total = ncols * halfR;
    const bool colfast = logC >= 5;
    const int C = 1 << logC;
    for (int lh = r - 1; lh >= 0; --lh) {
        const int h = 1 << lh;
        const int tshift = kTileLog - 1 - lh;
        for (int bi = threadIdx.x; bi < total; bi += blockDim.x) {
            int col, j;
            if (colfast) {
                col = bi % ncols;
                j = bi / ncols;
            } else {
                j = bi & (halfR - 1);
                col = bi >> (r - 1);
            }
            const int g = col >> logC, cc = col & (C - 1);
            const int jl = j & (h - 1);
            const int i = ((j >> lh) << (lh + 1)) + jl;
            uint32_t* base = sm + ((g << r) << logC) + cc;
            const uint32_t x0 = base[i << logC], x1 = base[(i + h) << logC];
            int e = jl << tshift;
            if (kInv)
                e = (kTile - e) & (kTile - 1);
            const uint2 w = tw[e];
            base[i << logC] = fadd(x0, x1, p);
            base[(i + h) << logC] = fmul_shoup(fsub(x0, x1, p), w.x, w.y, p);
        }
        __syncthreads();
    }
}

// Radix-2 decimation-in-time transforms, bit-reversed input, natural output.
template <bool kInv>
__device__ void lds_dit(uint32_t* sm, int r, int logC, int ncols, const uint2* tw, uint32_t p)
{
    const int halfR = (1 << r) >> 1;
    const int total = ncols * halfR;
    const bool colfast = logC >= 5;
    const int C = 1 << logC;
    for (int lh = 0; lh < r; ++lh) {
        const int h = 1 << lh;
        const int tshift = kTileLog - 1 - lh;
        for (int bi = threadIdx.x; bi < total; bi += blockDim.x) {
            int col, j;
            if (colfast) {
                col = bi % ncols;
                j = bi / ncols;
            } else {
                j = bi & (halfR - 1);
                col = bi >> (r - 1);
            }
            const int g = col >> logC, cc = col & (C - 1);
            const int jl = j & (h - 1);
            const int i = ((j >> lh) << (lh + 1)) + jl;
            uint32_t* base = sm + ((g << r) << logC) + cc;
            int e = jl << tshift;
            if (kInv)
                e = (kTile - e) & (kTile - 1);
            const uint2 w = tw[e];
            const uint32_t x0 = base[i << logC];
            const uint32_t x1 = fmul_shoup(base[(i + h) << logC], w.x, w.y, p);
            base[i << logC] = fadd(x0, x1, p);
            base[(i + h) << logC] = fsub(x0, x1, p);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kPassThreads) void k_pass(PassArgs a)
{
    __shared__ uint32_t sm[kTile];

    const int pi = blockIdx.y;
    const uint32_t p = kPrimes[pi], pneg = kNegInv[pi];
    const uint2* tw = a.tb.tile_tw + pi * kTile;
    uint32_t* data = a.data + ((size_t)pi << a.logL);

    const int logT = min(kTileLog, a.logL);
    const int T = 1 << logT;
    const int r = a.r, s = a.s;
    const int logC = min(s, logT - r);
    const int logG = logT - r - logC;
    const int C = 1 << logC;
    const int logM = r + s;
    const int logCgs = s - logC;                 // column groups per block
    const int bg = blockIdx.x >> logCgs;
    const int cg = blockIdx.x & ((1 << logCgs) - 1);
    const int ncols = 1 << (logG + logC);
    const int twshift = kLogMaxLen - logM;

    // ---- load ----
    for (int li = threadIdx.x; li < T; li += kPassThreads) {
        const int cc = li & (C - 1);
        const int row = (li >> logC) & ((1 << r) - 1);
        const int g = li >> (r + logC);
        const uint32_t col = (uint32_t)(cg << logC) + cc;
        const uint32_t pos = ((uint32_t)((bg << logG) + g) << logM) + ((uint32_t)row << s) + col;
        if (a.mode == kInverse) {
            uint32_t v = data[pos];
            if (s > 0) {
                uint32_t E = (col * (uint32_t)row) << twshift;
                E = (0u - E) & ((1u << kLogMaxLen) - 1u);
                v = fmul_mont(v, pass_twiddle(a.tb, pi, E, p, pneg), p, pneg);
            }
            sm[(((g << r) + (int)bitrev(row, r)) << logC) + cc] = v;
        } else {
            sm[li] = (a.src == kSrcArray) ? data[pos] : freduce32(source_digit(a, pos), p);
        }
    }
    __syncthreads();

    // ---- transform ----
    if (a.mode == kInverse) {
        lds_dit<true>(sm, r, logC, ncols, tw, p);
    } else {
        lds_dif<false>(sm, r, logC, ncols, tw, p);
        if (a.mode == kFused) {
            // Pointwise product with the pre-scaled c-hat (stored in the same
            // bit-reversed block layout), then the inverse of this pass.
            const uint32_t* other = a.other + ((size_t)pi << a.logL);
            for (int li = threadIdx.x; li < T; li += kPassThreads) {
                const uint32_t pos = ((uint32_t)((bg << logG)) << logM) + (uint32_t)li;
                sm[li] = fmul_mont(sm[li], other[pos], p, pneg);
            }
            __syncthreads();
            lds_dit<true>(sm, r, logC, ncols, tw, p);
        }
    }

    // ---- store ----
    for (int li = threadIdx.x; li < T; li += kPassThreads) {
        const int cc = li & (C - 1);
        const int row = (li >> logC) & ((1 << r) - 1);
        const int g = li >> (r + logC);
        const uint32_t col = (uint32_t)(cg << logC) + cc;
        const uint32_t pos = ((uint32_t)((bg << logG) + g) << logM) + ((uint32_t)row << s) + col;
        uint32_t v;
        if (a.mode == kForward && s > 0) {
            v = sm[(((g << r) + (int)bitrev(row, r)) << logC) + cc];
            const uint32_t E = (col * (uint32_t)row) << twshift;
            v = fmul_mont(v, pass_twiddle(a.tb, pi, E, p, pneg), p, pneg);
        } else {
            v = sm[li];
        }
        if (a.scale)
            v = fmul_shoup(v, a.scale_w[pi], a.scale_q[pi], p);
        data[pos] = v;
    }
}

}  // namespace

hipError_t launch_pass(const PassArgs& a, hipStream_t stream)
{
    const int logT = a.logL < kTileLog ? a.logL : kTileLog;
    const unsigned tiles = 1u << (a.logL - logT);
    hipLaunchKernelGGL(k_pass, dim3(tiles, kNumPrimes), dim3(kPassThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace pa
