// Device code of one transform pass tile, shared by the pass kernel (one
// launch per pass) and the persistent batch kernel (tiles taken from a work
// queue).  See ntt.hip for the transform's structure.
#pragma once

#include "kernels.h"
#include "splitmix.h"
#include "swizzle.h"

namespace pa {
namespace {

constexpr int bitrev_c(int x, int bits)
{
    int r = 0;
    for (int i = 0; i < bits; ++i)
        r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

// Compile-time constants of prime PI: the modulus, -p^{-1} mod 2^32, and the
// small roots with their Shoup quotients, omega_64^{+-e} (e < 32) and the cube
// roots of unity, all powers of the order-kOrder root so that they agree with
// the run-time tables.  Indexed with constants after unrolling, they become
// scalar immediates instead of registers.
template <int PI>
struct PrimeConst {
    static constexpr uint32_t p = kPrimes[PI];
    static constexpr uint32_t pneg = kNegInv[PI];
    static constexpr uint64_t order = kOrder >> kRootShift[PI];   // of the prime's root
    static constexpr uint64_t w64 = pow_mod(kRoot[PI], order / 64, kPrimes[PI]);
    static constexpr uint64_t w64inv = pow_mod(w64, kPrimes[PI] - 2, kPrimes[PI]);
    static constexpr uint64_t w3 = pow_mod(kRoot[PI], order / 3, kPrimes[PI]);
    static constexpr uint64_t w3sq = w3 * w3 % kPrimes[PI];
    // 2^32 and 2^64 mod p with their Shoup quotients: a digit of words
    // (w0, w1, w2) is w0 + w1 (2^32 mod p) + w2 (2^64 mod p) mod p
    static constexpr uint32_t r32 = (uint32_t)((1ull << 32) % kPrimes[PI]);
    static constexpr uint32_t r32q = shoup_quotient(r32, kPrimes[PI]);
    static constexpr uint32_t r64 = (uint32_t)((uint64_t)r32 * r32 % kPrimes[PI]);
    static constexpr uint32_t r64q = shoup_quotient(r64, kPrimes[PI]);
};

// A 64-bit digit (lo, hi) reduced mod prime PI.
template <int PI>
__device__ __forceinline__ uint32_t reduce64(uint32_t lo, uint32_t hi)
{
    constexpr uint32_t p = PrimeConst<PI>::p;
    return fadd(freduce32(lo, p), fmul_shoup(hi, PrimeConst<PI>::r32, PrimeConst<PI>::r32q, p), p);
}

// A 96-bit digit (w0, w1, w2) reduced mod prime PI.
template <int PI>
__device__ __forceinline__ uint32_t reduce96(uint32_t w0, uint32_t w1, uint32_t w2)
{
    constexpr uint32_t p = PrimeConst<PI>::p;
    return fadd(reduce64<PI>(w0, w1), fmul_shoup(w2, PrimeConst<PI>::r64, PrimeConst<PI>::r64q, p), p);
}

// omega_64^e (kInv: omega_64^{-e}) and its Shoup quotient, e < 32.
template <int PI, bool kInv>
struct W64 {
    struct Table {
        uint32_t w[32], q[32];
    };
    static constexpr Table make()
    {
        Table t{};
        const uint64_t pp = PrimeConst<PI>::p;
        const uint64_t b = kInv ? PrimeConst<PI>::w64inv : PrimeConst<PI>::w64;
        for (int e = 0; e < 32; ++e) {
            t.w[e] = (uint32_t)pow_mod(b, (uint64_t)e, pp);
            t.q[e] = shoup_quotient(t.w[e], pp);
        }
        return t;
    }
    static constexpr Table table = make();
};

// What one workgroup reads and writes: the scalar fields of the pass, or the
// fields of its block in batch mode.  Kept apart from the kernel argument so
// the argument is never copied to private memory.
struct BlockView {
    uint32_t* data;
    const uint32_t* other;
    const uint32_t* digits;
    uint64_t seed;
    uint64_t n;
    uint64_t bit_off;
    uint32_t num_digits;
    uint32_t store_limit;
    int src;
};

// Where a workgroup's tile sits in its launch: the tile index and the tile
// count of one prime's array, and the job (batch) or operand (dual launch).
struct TileCoord {
    uint32_t tile;
    uint32_t tiles;
    uint32_t z;
    bool xcd_order;   // tiles were dealt to the XCDs round-robin by index
};

// The block a workgroup works on.  kJobs 0: a single block (the scalar
// fields, or the dual launch's second operand); 1: a batch's block from the
// job table (a.jobs set); 2: either, decided from a.jobs at run time.  The
// kernels of most kinds are compiled apart for single blocks and batches, so
// that the single-block ones carry no job-table code.
__device__ __forceinline__ void job_view(const PassArgs& a, uint32_t z, BlockView& v)
{
    const auto* j = gmem(a.jobs + z);
    v.n = j->n;
    v.num_digits = j->num_digits;
    v.data = (a.role == kRoleMul) ? j->A : j->B;
    v.other = j->A;
    if (a.src != kSrcArray) {             // first pass: the operand's digits
        if (a.role == kRoleKey) {
            v.src = kSrcDigits;
            v.digits = j->key;
        } else if (j->c) {
            v.src = kSrcDigits;
            v.digits = j->c;
        } else {
            v.src = kSrcSeed;
            v.seed = j->seed_a;
        }
    }
    if (a.limit_to_digits)
        v.store_limit = ((j->num_digits + a.dwords - 1u) / a.dwords + 3u) & ~3u;
}

template <int kJobs>
__device__ __forceinline__ BlockView block_view(const PassArgs& a, uint32_t z)
{
    BlockView v{a.data, a.other, a.digits, a.seed, a.n, a.bit_off, a.num_digits, a.store_limit, a.src};
    if (kJobs == 1 || (kJobs == 2 && a.jobs)) {
        job_view(a, z, v);
    } else if (a.dual && z == 1) {
        v.data = const_cast<uint32_t*>(a.other);
        v.src = kSrcDigits;
    }
    return v;
}

// Digits pos .. pos + 3 (pos a multiple of 4) of W 32-bit words each of the
// operand described by the block's source, as 4 W words, low word first, 0
// beyond bit n: W 16-byte loads of key words, or 2 W SplitMix64 words of a
// seeded multiplier (bit 0 forced to 1, eq. (6)).
template <int W>
__device__ __forceinline__ void source_quad(const BlockView& a, uint32_t pos, uint32_t (&v)[4 * W])
{
    const uint32_t D = a.num_digits;          // 32-bit words of the operand
    const uint32_t d0 = W * pos;              // even: pos is a multiple of 4
#pragma unroll
    for (int i = 0; i < 4 * W; ++i) v[i] = 0u;
    if (d0 >= D)
        return;
    if (a.src == kSrcDigits) {
        if (d0 + 4 * W <= D && (reinterpret_cast<uintptr_t>(a.digits) & 15u) == 0) {
#pragma unroll
            for (int q = 0; q < W; ++q) {
                const u32x4 t = *gword<const u32x4>(a.digits, d0 + 4 * q);
                v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4 * W; ++i)
                if (d0 + i < D) v[i] = *gword(a.digits, d0 + i);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 2 * W; ++e) {
            if (d0 + 2 * e < D) {
                const uint32_t idx = (d0 >> 1) + e;
                const uint64_t w = splitmix64(a.seed, idx);
                v[2 * e] = (uint32_t)w | ((idx == 0) ? 1u : 0u);
                v[2 * e + 1] = (d0 + 2 * e + 1 < D) ? (uint32_t)(w >> 32) : 0u;
            }
        }
    }
    // bits past n in the top 32-bit word
    const uint32_t top = (uint32_t)(a.n & 31);
    if (top) {
        const uint32_t mask = (1u << top) - 1u;
#pragma unroll
        for (int i = 0; i < 4 * W; ++i)
            if (d0 + i == D - 1) v[i] &= mask;
    }
}

// Element t of a bit source: bit bit_off + t of the 32-bit word array, 0 for t >= n.
__device__ __forceinline__ uint32_t source_bit(const BlockView& a, uint32_t t)
{
    if (t >= a.n)
        return 0;
    const uint64_t b = a.bit_off + t;
    return (*gmem(a.digits + (b >> 5)) >> (b & 31)) & 1u;
}

// Montgomery form of w^E for the root w of order kOrder, E < kOrder (for a
// prime whose root has order kOrder / 8: r^(E / 8), E a multiple of 8).
template <int PI>
__device__ __forceinline__ uint32_t root_pow(const Tables& tb, uint32_t E)
{
    const uint32_t lo = *gmem(tb.pass_lo + PI * 4096 + (E & 4095u));
    const uint32_t hi = *gmem(tb.pass_hi + PI * kRootHi + (E >> 12));
    return fmul_mont(lo, hi, PrimeConst<PI>::p, PrimeConst<PI>::pneg);
}

// Radix-2^R DIF butterflies in registers: natural input, bit-reversed output,
// with the constant powers of omega_64 of prime PI.  kHalfZero: the upper half
// of the input is zero, so the first level is x[j + h] = x[j] w^j.
template <int R, int PI, bool kHalfZero = false>
__device__ __forceinline__ void dif_regs(uint32_t* x)
{
    constexpr uint32_t p = PrimeConst<PI>::p;
    constexpr auto& tw = W64<PI, false>::table;
    constexpr int N = 1 << R;
#pragma unroll
    for (int lh = R - 1; lh >= 0; --lh) {
        const int h = 1 << lh;
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const uint32_t a = x[i0 + j], b = x[i0 + j + h];
                if (kHalfZero && lh == R - 1) {
                    const int e = j << (5 - lh);
                    x[i0 + j + h] = j ? fmul_shoup(a, tw.w[e], tw.q[e], p) : a;
                    continue;
                }
                x[i0 + j] = fadd(a, b, p);
                if (j == 0) {
                    x[i0 + j + h] = fsub(a, b, p);
                } else {
                    // a - b + p < 2p < 2^32 needs no reduction before Shoup's
                    // multiply, which takes any 32-bit input
                    const int e = j << (5 - lh);
                    x[i0 + j + h] = fmul_shoup(a - b + p, tw.w[e], tw.q[e], p);
                }
            }
        }
    }
}

// Radix-2^R DIT butterflies with inverse roots: bit-reversed input, natural
// output.
template <int R, int PI>
__device__ __forceinline__ void dit_regs(uint32_t* x)
{
    constexpr uint32_t p = PrimeConst<PI>::p;
    constexpr auto& tw = W64<PI, true>::table;
    constexpr int N = 1 << R;
#pragma unroll
    for (int lh = 0; lh < R; ++lh) {
        const int h = 1 << lh;
#pragma unroll
        for (int i0 = 0; i0 < N; i0 += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const uint32_t a = x[i0 + j];
                uint32_t b = x[i0 + j + h];
                if (j != 0) {
                    const int e = j << (5 - lh);
                    b = fmul_shoup(b, tw.w[e], tw.q[e], p);
                }
                x[i0 + j] = fadd(a, b, p);
                x[i0 + j + h] = fsub(a, b, p);
            }
        }
    }
}

// Geometry of one step inside a tile of R rows x C columns.  Element n of DFT
// (beta, o, c) sits at row beta B + n sigma + o, column c.  After a forward step
// output k is multiplied by b^k, b = w^E with
//   E = o (kOrder / B)                [the inner twiddle omega_B^o, if inner]
//     + (col0 + c) colmul (kOrder / M)  [the pass twiddle, strided passes]
struct StepGeo {
    int logC;       // columns
    int logSig;     // row stride of the DFT elements
    int logB;       // sub-block rows = radix * stride (power-of-two steps)
    int inner;
    uint32_t colmul;
    uint32_t unitB, unitM;
    uint32_t col0;  // global column of tile column 0
};

__device__ __forceinline__ uint32_t step_exponent(const StepGeo& g, uint32_t o, uint32_t c, bool inv)
{
    uint32_t E = g.inner ? o * g.unitB : 0u;
    if (g.colmul) {
        E += (g.col0 + c) * g.colmul * g.unitM;
        if (E >= kOrder) E -= kOrder;
    }
    if (inv && E) E = kOrder - E;
    return E;
}

// One DIF (forward) or DIT (inverse) step of radix 2^R over every DFT of the tile.
// Where a step's data comes from and goes to besides LDS (kIO, bit flags):
// kIoIn reads the step's inputs from HBM, kIoOut writes its outputs to HBM
// (positions below `limit`), in the order the step would have read or written
// the tile (natural for a forward step's inputs and an inverse step's outputs,
// bit-reversed within each DFT for the others).  `in` and `out` point to the
// tile's row 0, column 0 in the array, whose rows are 2^shift residues apart
// (the pass's S; 0 for a contiguous pass, one column).
constexpr int kIoIn = 1, kIoOut = 2;
struct GlobalIO {
    const uint32_t* in;
    uint32_t* out;
    uint32_t limit;
    int shift;
};

// kHalf (the first register step of an operand's first pass, or the last one
// of the final inverse pass, power-of-two rows): elements n >= 2^R / 2 of every
// DFT are rows >= R / 2 of the pass, positions >= L / 2 >= D: zero on input
// (forward: not read) or never stored (inverse: not written).
// kStrided: the tile has 4 or more columns and its rows are 2^io.shift apart
// in the array; else it is one contiguous column (tile and array offsets agree).
template <int R, bool kInv, int PI, int kIO = 0, bool kHalf = false, bool kStrided = false>
__device__ __forceinline__ void run_step(uint32_t* sm, int N, const StepGeo& g, const Tables& tb,
                                         const GlobalIO& io = GlobalIO{nullptr, nullptr, 0u, 0})
{
    constexpr uint32_t p = PrimeConst<PI>::p, pneg = PrimeConst<PI>::pneg;
    constexpr int RHO = 1 << R;
    const int ndft = N >> R;
    const uint32_t cmask = (1u << g.logC) - 1u;
    const uint32_t omask = (1u << g.logSig) - 1u;
    const bool twiddle = g.inner || g.colmul;
    // Without the inner twiddle the base depends only on the column, which is
    // the same for all of a thread's DFTs when the block is a whole number of
    // rows of columns: compute it once.
    const bool fixed_base = twiddle && !g.inner && (blockDim.x & cmask) == 0;
    uint32_t b_fixed = 0;
    if (fixed_base && (int)threadIdx.x < ndft)
        b_fixed = root_pow<PI>(tb, step_exponent(g, 0u, threadIdx.x & cmask, kInv));
    for (int q = threadIdx.x; q < ndft; q += blockDim.x) {
        const uint32_t c = (uint32_t)q & cmask;
        const uint32_t o = ((uint32_t)q >> g.logC) & omask;
        const uint32_t beta = (uint32_t)q >> (g.logC + g.logSig);
        const uint32_t base = (((beta << g.logB) + o) << g.logC) + c;
        const uint32_t nstep = 1u << (g.logSig + g.logC);
        const uint32_t sb = swz(base);
        // the same elements in the array (kIO): rows 2^shift apart
        uint32_t gbase = base, gstep = nstep;
        if constexpr (kStrided) {
            gbase = (((beta << g.logB) + o) << io.shift) + c;
            gstep = 1u << (g.logSig + io.shift);
        }
        uint32_t x[RHO];
        uint32_t b = b_fixed;  // Montgomery form of the twiddle base
        if (twiddle && !fixed_base)
            b = root_pow<PI>(tb, step_exponent(g, o, c, kInv));
        if (!kInv) {
#pragma unroll
            for (int n = 0; n < RHO; ++n) {
                if (kHalf && n >= RHO / 2)
                    x[n] = 0u;
                else
                    x[n] = (kIO & kIoIn) ? *gword(io.in, gbase + n * gstep) : sm[sb ^ swz(n * nstep)];
            }
            dif_regs<R, PI, kHalf>(x);
            if (twiddle) {
                uint32_t w = b;
#pragma unroll
                for (int k = 1; k < RHO; ++k) {
                    const int j = bitrev_c(k, R);
                    x[j] = fmul_mont(x[j], w, p, pneg);
                    if (k + 1 < RHO) w = fmul_mont_lazy(w, b, p, pneg);
                }
            }
#pragma unroll
            for (int j = 0; j < RHO; ++j) {
                if (kIO & kIoOut) {
                    const uint32_t gi = gbase + bitrev_c(j, R) * gstep;
                    if (gi < io.limit) *gword(io.out, gi) = x[j];
                } else {
                    sm[sb ^ swz(bitrev_c(j, R) * nstep)] = x[j];
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < RHO; ++j)
                x[j] = (kIO & kIoIn) ? *gword(io.in, gbase + bitrev_c(j, R) * gstep)
                                     : sm[sb ^ swz(bitrev_c(j, R) * nstep)];
            if (twiddle) {
                uint32_t w = b;
#pragma unroll
                for (int k = 1; k < RHO; ++k) {
                    const int j = bitrev_c(k, R);
                    x[j] = fmul_mont(x[j], w, p, pneg);
                    if (k + 1 < RHO) w = fmul_mont_lazy(w, b, p, pneg);
                }
            }
            dit_regs<R, PI>(x);
#pragma unroll
            for (int n = 0; n < RHO; ++n) {
                if (kHalf && n >= RHO / 2)
                    continue;
                if (kIO & kIoOut) {
                    if (gbase + n * gstep < io.limit) *gword(io.out, gbase + n * gstep) = x[n];
                } else {
                    sm[sb ^ swz(n * nstep)] = x[n];
                }
            }
        }
    }
}

// The radix-3 step that opens a pass whose R rows carry the factor 3: one
// block of B = R rows, sigma = R / 3.  With w3 a primitive cube root of unity
// (w3^2 = -1 - w3), the DFT of (x0, x1, x2) is
//   y0 = x0 + x1 + x2,  y1 = x0 - x2 + v,  y2 = x0 - x1 - v,  v = w3 (x1 - x2);
// the inverse uses w3^2 in place of w3.  w3p = (w3 or w3^2, Shoup quotient).
template <bool kInv, int PI>
__device__ __forceinline__ void run_step3(uint32_t* sm, int N, const StepGeo& g, const Tables& tb)
{
    constexpr uint32_t p = PrimeConst<PI>::p, pneg = PrimeConst<PI>::pneg;
    constexpr uint32_t w3 = (uint32_t)(kInv ? PrimeConst<PI>::w3sq : PrimeConst<PI>::w3);
    constexpr uint32_t w3q = shoup_quotient(w3, PrimeConst<PI>::p);
    const int ndft = N / 3;
    const uint32_t cmask = (1u << g.logC) - 1u;
    const bool twiddle = g.inner || g.colmul;
    for (int q = threadIdx.x; q < ndft; q += blockDim.x) {
        const uint32_t c = (uint32_t)q & cmask;
        const uint32_t o = (uint32_t)q >> g.logC;
        const uint32_t base = (o << g.logC) + c;
        const uint32_t nstep = 1u << (g.logSig + g.logC);
        uint32_t b = 0, b2 = 0;
        if (twiddle) {
            b = root_pow<PI>(tb, step_exponent(g, o, c, kInv));
            b2 = fmul_mont_lazy(b, b, p, pneg);
        }
        const uint32_t s0 = swz(base), s1 = s0 ^ swz(nstep), s2 = s0 ^ swz(2 * nstep);
        uint32_t x0 = sm[s0], x1 = sm[s1], x2 = sm[s2];
        if (kInv && twiddle) {
            x1 = fmul_mont(x1, b, p, pneg);
            x2 = fmul_mont(x2, b2, p, pneg);
        }
        const uint32_t v = fmul_shoup(x1 - x2 + p, w3, w3q, p);
        uint32_t y0 = fadd(fadd(x0, x1, p), x2, p);
        uint32_t y1 = fadd(fsub(x0, x2, p), v, p);
        uint32_t y2 = fsub(fsub(x0, x1, p), v, p);
        if (!kInv && twiddle) {
            y1 = fmul_mont(y1, b, p, pneg);
            y2 = fmul_mont(y2, b2, p, pneg);
        }
        sm[s0] = y0;
        sm[s1] = y1;
        sm[s2] = y2;
    }
}

template <bool kInv, int PI>
__device__ __forceinline__ void dispatch_step(int r, uint32_t* sm, int N, const StepGeo& g, const Tables& tb)
{
    switch (r) {
    case 1: run_step<1, kInv, PI>(sm, N, g, tb); break;
    case 2: run_step<2, kInv, PI>(sm, N, g, tb); break;
    case 3: run_step<3, kInv, PI>(sm, N, g, tb); break;
    case 4: run_step<4, kInv, PI>(sm, N, g, tb); break;
    default: break;
    }
}

template <bool kInv, int PI>
__device__ __forceinline__ void dispatch_step_half(int r, uint32_t* sm, int N, const StepGeo& g,
                                                   const Tables& tb)
{
    switch (r) {
    case 2: run_step<2, kInv, PI, 0, true>(sm, N, g, tb); break;
    case 3: run_step<3, kInv, PI, 0, true>(sm, N, g, tb); break;
    case 4: run_step<4, kInv, PI, 0, true>(sm, N, g, tb); break;
    default: run_step<1, kInv, PI>(sm, N, g, tb); break;
    }
}

// Geometry of step si of a pass (si counts the radix-3 step, if any, as 0).
__device__ __forceinline__ StepGeo step_geo(const PassArgs& a, int si, uint32_t col0)
{
    const int has3 = a.f == 3;
    const int total = a.nsteps + has3;
    const uint32_t M = (uint32_t)a.f << (a.r + a.s);
    StepGeo g;
    g.logC = a.logC;
    g.col0 = col0;
    g.unitM = kOrder / M;
    g.inner = si + 1 < total;
    if (has3 && si == 0) {                    // B = R = 3 2^r, sigma = 2^r
        g.logB = -1;
        g.logSig = a.r;
        g.unitB = kOrder / (3u << a.r);
        g.colmul = a.s > 0 ? 1u : 0u;
        return g;
    }
    const int j = si - has3;
    const int above = (int)((a.above_code >> (4 * j)) & 15u);
    g.logB = a.r - above;
    g.logSig = g.logB - (int)((a.steps_code >> (4 * j)) & 15u);
    g.unitB = kOrder >> g.logB;
    // the pass factor omega_M^{col k} with k = k_0 + rho_0 (k_1 + rho_1 (k_2 + ...)):
    // step s takes omega_M^{col rho_0 ... rho_{s-1} k_s}
    g.colmul = a.s > 0 ? ((uint32_t)a.f << above) : 0u;
    return g;
}

// A step of radix 2^r with HBM input or output (kIO), kHalf as for run_step
// (radix >= 4).
template <bool kInv, int PI, int kIO, bool kHalf = false, bool kStrided = false>
__device__ __forceinline__ void dispatch_step_io(int r, uint32_t* sm, int N, const StepGeo& g,
                                                 const Tables& tb, const GlobalIO& io)
{
    switch (r) {
    case 1: if constexpr (!kHalf) run_step<1, kInv, PI, kIO, false, kStrided>(sm, N, g, tb, io); break;
    case 2: run_step<2, kInv, PI, kIO, kHalf, kStrided>(sm, N, g, tb, io); break;
    case 3: run_step<3, kInv, PI, kIO, kHalf, kStrided>(sm, N, g, tb, io); break;
    case 4: run_step<4, kInv, PI, kIO, kHalf, kStrided>(sm, N, g, tb, io); break;
    default: break;
    }
}

// Steps first .. count-1 of the pass (forward), or their inverse count-1 ..
// first.  io_in: the first step run reads its inputs from HBM (no LDS load
// before it); io_out: the last step run writes its outputs to HBM (and no
// barrier follows it).  Both need power-of-two steps at those ends, and
// count - first >= 2.
template <bool kInv, int PI, bool kStrided = false>
__device__ __forceinline__ void run_pass_steps(const PassArgs& a, uint32_t* sm, int N, uint32_t col0,
                                               int count, int first = 0, bool half = false,
                                               const GlobalIO& io = GlobalIO{nullptr, nullptr, 0u, 0},
                                               bool io_in = false, bool io_out = false)
{
    const int has3 = a.f == 3;
    for (int k = first; k < count; ++k) {
        const int si = kInv ? count - 1 - (k - first) : k;
        const StepGeo g = step_geo(a, si, col0);
        const int r = (int)((a.steps_code >> (4 * (si - has3))) & 15u);
        const bool in = io_in && k == first, out = io_out && k == count - 1;
        if (has3 && si == 0)
            run_step3<kInv, PI>(sm, N, g, a.tb);
        else if (in)
            dispatch_step_io<kInv, PI, kIoIn, false, kStrided>(r, sm, N, g, a.tb, io);
        else if (out && half && si == 0)
            dispatch_step_io<kInv, PI, kIoOut, true, kStrided>(r, sm, N, g, a.tb, io);
        else if (out)
            dispatch_step_io<kInv, PI, kIoOut, false, kStrided>(r, sm, N, g, a.tb, io);
        else if (half && si == 0)
            dispatch_step_half<kInv, PI>(r, sm, N, g, a.tb);
        else
            dispatch_step<kInv, PI>(r, sm, N, g, a.tb);
        if (!out)
            __syncthreads();
    }
}

// The middle of the fused pass in registers: the last forward step of a
// contiguous pass (radix 2^R over 2^R consecutive residues, no twiddles), the
// pointwise product with c-hat (same positions) and the first inverse step,
// which reads exactly the registers the forward step would have written.
template <int R, int PI>
__device__ __forceinline__ void fused_middle(uint32_t* sm, int N, const uint32_t* chat)
{
    constexpr uint32_t p = PrimeConst<PI>::p, pneg = PrimeConst<PI>::pneg;
    constexpr int RHO = 1 << R;
    const int ndft = N >> R;
    for (int q = threadIdx.x; q < ndft; q += blockDim.x) {
        const uint32_t base = (uint32_t)q << R;
        const uint32_t sb = swz(base);
        uint32_t x[RHO];
#pragma unroll
        for (int n = 0; n < RHO; ++n)
            x[n] = sm[sb ^ swz((uint32_t)n)];
        dif_regs<R, PI>(x);
        uint32_t c[RHO];
        if (RHO >= 4) {
#pragma unroll
            for (int v = 0; v < RHO / 4; ++v) {
                const u32x4 w = *gword<const u32x4>(chat, base + 4 * v);
                c[4 * v] = w.x;
                c[4 * v + 1] = w.y;
                c[4 * v + 2] = w.z;
                c[4 * v + 3] = w.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < RHO; ++k) c[k] = *gword(chat, base + k);
        }
#pragma unroll
        for (int k = 0; k < RHO; ++k) {
            const int j = bitrev_c(k, R);
            x[j] = fmul_mont(x[j], c[k], p, pneg);
        }
        dit_regs<R, PI>(x);
#pragma unroll
        for (int n = 0; n < RHO; ++n)
            sm[sb ^ swz((uint32_t)n)] = x[n];
    }
}

// The last step of a forward contiguous pass (radix 2^R >= 4 over 2^R
// consecutive residues, no twiddles) straight to HBM: output k of the DFT at
// base goes to position base + bitrev(k), so each thread writes 2^R
// consecutive residues with 16-byte stores and the tile skips its last LDS
// round trip and the store sweep.
template <int R, int PI>
__device__ __forceinline__ void last_step_store(const uint32_t* sm, int N, uint32_t* out,
                                                uint32_t limit)
{
    constexpr int RHO = 1 << R;
    static_assert(RHO >= 4, "16-byte stores");
    const int ndft = N >> R;
    for (int q = threadIdx.x; q < ndft; q += blockDim.x) {
        const uint32_t base = (uint32_t)q << R;
        const uint32_t sb = swz(base);
        uint32_t x[RHO];
#pragma unroll
        for (int n = 0; n < RHO; ++n)
            x[n] = sm[sb ^ swz((uint32_t)n)];
        dif_regs<R, PI>(x);
        uint32_t y[RHO];
#pragma unroll
        for (int k = 0; k < RHO; ++k) y[k] = x[bitrev_c(k, R)];
#pragma unroll
        for (int v = 0; v < RHO / 4; ++v)
            if (base + 4 * v < limit)
                *gword<u32x4>(out, base + 4 * v) =
                    u32x4{y[4 * v], y[4 * v + 1], y[4 * v + 2], y[4 * v + 3]};
    }
}

template <int PI>
__device__ __forceinline__ void dispatch_fused_middle(int r, uint32_t* sm, int N, const uint32_t* chat)
{
    switch (r) {
    case 1: fused_middle<1, PI>(sm, N, chat); break;
    case 2: fused_middle<2, PI>(sm, N, chat); break;
    case 3: fused_middle<3, PI>(sm, N, chat); break;
    case 4: fused_middle<4, PI>(sm, N, chat); break;
    default: break;
    }
}

// One pass over the tile of prime PI owned by this workgroup; digit sources
// have W 32-bit words per digit.  kMode is the pass's mode (a.mode) and kSrc
// whether its input is an operand source rather than a residue array
// (a.src != kSrcArray): fixed at compile time, so each kernel carries only
// the code of its own kind of pass.  kStrided: the pass is known to be strided
// (a.s > 0, 4 or more columns per tile; the inverse passes after the fused
// one), else the layout is read from the arguments.
template <int PI, int W, int kMode, bool kSrc, bool kStrided, int kJobs>
__device__ __forceinline__ void pass_tile(const PassArgs& a, uint32_t* sm, const TileCoord& tc)
{
    constexpr uint32_t p = PrimeConst<PI>::p;
    const BlockView bv = block_view<kJobs>(a, tc.z);
    uint32_t* data = bv.data + (size_t)PI * a.L;

    const int logC = a.logC;                  // columns per tile
    const uint32_t R = (uint32_t)a.f << a.r;
    const int N = (int)(R << logC);           // tile residues
    const uint32_t M = R << a.s;              // pass block length
    const int logCgs = a.s - logC;            // column groups per block
    // Workgroups of a launch are dealt to the 8 XCDs round-robin by index, and
    // each XCD has its own L2.  Adjacent column groups of a strided pass share
    // 128-byte lines when a tile row is shorter than a line, so consecutive
    // tiles go to one XCD (tile = (id mod 8) tiles/8 + id / 8, a bijection
    // when the tile count is a multiple of 8) and each line is fetched once.
    uint32_t tile = tc.tile;
    if (tc.xcd_order && (tc.tiles & 7u) == 0)
        tile = (tile & 7u) * (tc.tiles >> 3) + (tile >> 3);
    const uint32_t bg = tile >> logCgs;
    const uint32_t col0 = (tile & ((1u << logCgs) - 1u)) << logC;
    const uint32_t blk0 = bg * M;             // global offset of the block

    // A contiguous pass (one column) whose input is already a residue array
    // reads its first register step straight from HBM: lanes take consecutive
    // positions, so those loads coalesce, and the load sweep and its barrier go.
    const int total = a.nsteps + (a.f == 3);
    const bool many_cols = kStrided || logC >= 2;
    const bool contig = !kStrided && a.f == 1 && logC == 0 && a.nsteps >= 2;
    const bool hbm_in = !kSrc && kMode != kInverse && contig;
    const StepGeo g0 = step_geo(a, 0, col0);
    const int r0 = (int)(a.steps_code & 15u);
    const uint32_t org = blk0 + col0;         // tile row 0, column 0 in the array
    const GlobalIO io{data + org, data + org, bv.store_limit > org ? bv.store_limit - org : 0u,
                      kStrided ? a.s : 0};
    // An inverse strided pass likewise reads its first step's inputs from HBM
    // and writes its last step's outputs (power-of-two rows) to HBM, instead
    // of the load and store sweeps through LDS.  (Measured: the inverse pass
    // at n = 10^8 44.7 -> 41.2 us; the same store in a forward strided pass,
    // the operands' first passes, made them 2.5 us slower.)
    const bool strided = kStrided && kMode == kInverse && total >= 2;
    const bool s_in = strided;
    const bool s_out = strided && a.f == 1;

    // An operand's first pass covers the whole array in one block of R rows;
    // rows >= R / 2 are positions >= L / 2 >= D, all zero: they are neither
    // loaded nor read by the first step.  The final inverse pass stores only
    // positions below D, so its last step leaves rows >= R / 2 unwritten.
    // (Power-of-two rows, a first or last step of radix >= 4; in the 96-bit
    // layout's kernel only: the 64-bit one serves the short, latency-bound
    // blocks, where the larger kernel measured slower than the saved work.)
    const bool half_in = W == 3 && kSrc && (bv.src == kSrcDigits || bv.src == kSrcSeed) &&
                         a.f == 1 && r0 >= 2 && (kMode != kFused || total >= 2);
    const bool half_out = W == 3 && kMode == kInverse && a.limit_to_digits && a.f == 1 && r0 >= 2;

    // Tile element (row, c) <-> global position blk0 + row S + col0 + c; moved
    // in groups of 4 consecutive columns (C >= 4) or rows (C == 1); quad u
    // holds tile elements 4u .. 4u + 3.
    const int nq = N >> 2;
    const int nq_in = half_in ? nq >> 1 : nq;
    // the multiplier's factor on its source values (not the key's, which the
    // dual launch runs as operand z = 1 with the same arguments)
    const bool scale_in = kSrc && a.scale_in && !(a.dual && tc.z == 1);
    const uint32_t sw_in = a.scale_w[PI], sq_in = a.scale_q[PI];
    for (int u = threadIdx.x; u < nq_in && !hbm_in && !s_in; u += blockDim.x) {
        uint32_t e, pos;
        if (many_cols) {
            const uint32_t row = (uint32_t)u >> (logC - 2);
            const uint32_t c = ((uint32_t)u << 2) & ((1u << logC) - 1u);
            e = (row << logC) + c;
            pos = blk0 + (row << a.s) + col0 + c;
        } else {
            e = (uint32_t)u << 2;
            pos = blk0 + e;
        }
        uint4 v;
        if constexpr (!kSrc) {
            const u32x4 t = *gword<const u32x4>(data, pos);
            v = make_uint4(t.x, t.y, t.z, t.w);
        } else if (bv.src == kSrcBits) {
            v.x = source_bit(bv, pos + 0);
            v.y = source_bit(bv, pos + 1);
            v.z = source_bit(bv, pos + 2);
            v.w = source_bit(bv, pos + 3);
        } else if constexpr (W == 3) {
            uint32_t h[12];
            source_quad<3>(bv, pos, h);
            v.x = reduce96<PI>(h[0], h[1], h[2]);
            v.y = reduce96<PI>(h[3], h[4], h[5]);
            v.z = reduce96<PI>(h[6], h[7], h[8]);
            v.w = reduce96<PI>(h[9], h[10], h[11]);
        } else {
            uint32_t h[8];
            source_quad<2>(bv, pos, h);
            v.x = reduce64<PI>(h[0], h[1]);
            v.y = reduce64<PI>(h[2], h[3]);
            v.z = reduce64<PI>(h[4], h[5]);
            v.w = reduce64<PI>(h[6], h[7]);
        }
        if constexpr (kSrc) {
            if (scale_in) {
                v.x = fmul_shoup(v.x, sw_in, sq_in, p);
                v.y = fmul_shoup(v.y, sw_in, sq_in, p);
                v.z = fmul_shoup(v.z, sw_in, sq_in, p);
                v.w = fmul_shoup(v.w, sw_in, sq_in, p);
            }
        }
        *reinterpret_cast<uint4*>(&sm[swz(e)]) = v;
    }
    if (hbm_in) {
        dispatch_step_io<false, PI, kIoIn>(r0, sm, N, g0, a.tb, io);
    }
    if (!s_in)
        __syncthreads();

    if constexpr (kMode == kInverse) {
        run_pass_steps<true, PI, kStrided>(a, sm, N, col0, total, 0, half_out, io, s_in, s_out);
        if (s_out)
            return;
    } else if (kMode == kFused && hbm_in) {
        // as below, with the first forward step read from HBM and the last
        // inverse step (its inverse) written to HBM
        run_pass_steps<false, PI>(a, sm, N, col0, total - 1, 1);
        const int rl = (int)((a.steps_code >> (4 * (a.nsteps - 1))) & 15u);
        dispatch_fused_middle<PI>(rl, sm, N, bv.other + (size_t)PI * a.L + blk0);
        __syncthreads();
        run_pass_steps<true, PI>(a, sm, N, col0, total - 1, 1);
        dispatch_step_io<true, PI, kIoOut>(r0, sm, N, step_geo(a, 0, col0), a.tb, io);
        return;
    } else if (kMode == kFused) {
        // Forward steps but the last, then the last forward step, the
        // pointwise product with the pre-scaled c-hat (same layout) and the
        // first inverse step together in registers, then the other inverse
        // steps.  The fused pass is the contiguous last pass (f = 1, no pass
        // twiddle), so its last step carries no twiddles.
        run_pass_steps<false, PI>(a, sm, N, col0, total - 1, 0, half_in);
        const int rl = (int)((a.steps_code >> (4 * (a.nsteps - 1))) & 15u);
        dispatch_fused_middle<PI>(rl, sm, N, bv.other + (size_t)PI * a.L + blk0);
        __syncthreads();
        run_pass_steps<true, PI>(a, sm, N, col0, total - 1);
    } else if (!kStrided && a.f == 1 && logC == 0 && a.nsteps >= 2 &&
               ((a.steps_code >> (4 * (a.nsteps - 1))) & 15u) >= 2) {
        // forward contiguous pass: all steps but the last through LDS, the
        // last straight to HBM
        run_pass_steps<false, PI>(a, sm, N, col0, total - 1, hbm_in ? 1 : 0, half_in);
        const int rl = (int)((a.steps_code >> (4 * (a.nsteps - 1))) & 15u);
        const uint32_t lim = bv.store_limit > blk0 ? bv.store_limit - blk0 : 0u;
        if (rl == 2)
            last_step_store<2, PI>(sm, N, data + blk0, lim);
        else if (rl == 3)
            last_step_store<3, PI>(sm, N, data + blk0, lim);
        else
            last_step_store<4, PI>(sm, N, data + blk0, lim);
        return;
    } else {
        run_pass_steps<false, PI>(a, sm, N, col0, total, hbm_in ? 1 : 0, half_in);
    }

    for (int u = threadIdx.x; u < (half_out ? nq >> 1 : nq); u += blockDim.x) {
        uint32_t e, pos;
        if (many_cols) {
            const uint32_t row = (uint32_t)u >> (logC - 2);
            const uint32_t c = ((uint32_t)u << 2) & ((1u << logC) - 1u);
            e = (row << logC) + c;
            pos = blk0 + (row << a.s) + col0 + c;
        } else {
            e = (uint32_t)u << 2;
            pos = blk0 + e;
        }
        const uint4 v = *reinterpret_cast<const uint4*>(&sm[swz(e)]);
        if (pos < bv.store_limit)
            *gword<u32x4>(data, pos) = u32x4{v.x, v.y, v.z, v.w};
    }
}

// One pass tile of prime `prime` of a layout: W = 2 (64-bit digits, the first
// five primes; also the Toeplitz variant's bit sources over prime 0) or W = 3
// (96-bit digits, all seven).  The body is instantiated once per prime, so
// that the prime's constants are immediates.
template <int W, int kMode, bool kSrc, bool kStrided, int kJobs>
__device__ __forceinline__ void pass_tile_any(const PassArgs& a, uint32_t* sm, uint32_t prime,
                                              const TileCoord& tc)
{
    if constexpr (W == 3) {
        switch (prime) {
        case 0: pass_tile<0, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        case 1: pass_tile<1, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        case 2: pass_tile<2, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        case 3: pass_tile<3, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        case 4: pass_tile<4, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        case 5: pass_tile<5, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        default: pass_tile<6, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        }
    } else {
        switch (prime) {
        case 0: pass_tile<0, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        case 1: pass_tile<1, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        case 2: pass_tile<2, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        case 3: pass_tile<3, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        default: pass_tile<4, W, kMode, kSrc, kStrided, kJobs>(a, sm, tc); break;
        }
    }
}

// The kinds of pass a plan has: (mode, operand source), see pass_tile.  Every
// pass but the last of a transform is strided and the last is contiguous, so
// the inverse passes after the fused one (the last) are all strided.
enum PassKind : int {
    kKindFirst = 0,        // forward, from the operand (its first pass)
    kKindForward = 1,      // forward, residue array in place
    kKindFusedFirst = 2,   // fused, from the key (a one-pass transform)
    kKindFused = 3,        // fused, residue array in place
    kKindInverse = 4,      // inverse, strided
    kPassKinds = 5,
};

__host__ __device__ inline int pass_kind(const PassArgs& a)
{
    const bool src = a.src != kSrcArray;
    if (a.mode == kInverse) return kKindInverse;
    if (a.mode == kFused) return src ? kKindFusedFirst : kKindFused;
    return src ? kKindFirst : kKindForward;
}

// Whether launch arguments fit their kind's kernel (the host checks before a
// launch): the inverse kind needs a strided pass (a.s > 0, 4 or more columns).
__host__ __device__ inline bool pass_kind_fits(const PassArgs& a, int kind)
{
    return kind != kKindInverse || (a.s > 0 && a.logC >= 2);
}

template <int W, int kKind, int kJobs>
__device__ __forceinline__ void pass_tile_kind(const PassArgs& a, uint32_t* sm, uint32_t prime,
                                               const TileCoord& tc)
{
    constexpr int kMode = kKind == kKindInverse ? kInverse
                        : (kKind == kKindFused || kKind == kKindFusedFirst) ? kFused : kForward;
    constexpr bool kSrc = kKind == kKindFirst || kKind == kKindFusedFirst;
    pass_tile_any<W, kMode, kSrc, kKind == kKindInverse, kJobs>(a, sm, prime, tc);
}

}  // namespace
}  // namespace pa
