// Internal interface between the runtime and the kernels of libpa.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.h"

namespace pa {

// Global-memory views of the buffers the kernels read and write.  Loads and
// stores through them compile to global_* instructions instead of flat_*
// ones: a flat access also counts against the LDS wait counter, so every wait
// for an LDS result would also wait for the outstanding HBM accesses.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// Word i of an array whose base is the same for the whole wave, as a V (a
// word or a vector of words), addressed by the base plus a 32-bit byte offset:
// the form of global access that takes a scalar base and one vector register
// per address, where base + i computed in 64 bits takes two vector registers
// per address (and a 64-bit add), or a scalar-register pair per distinct
// uniform offset.  The array must be shorter than 2^30 words.
template <class V = uint32_t, class T>
__device__ __forceinline__ __attribute__((address_space(1))) V* gword(T* base, uint32_t i)
{
    using Byte = __attribute__((address_space(1))) char;
    return (__attribute__((address_space(1))) V*)((Byte*)base + i * 4u);
}

constexpr int kTileLog = 14;                 // largest LDS tile: 2^14 residues, 64 KB
constexpr int kTileMinLog = 10;              // smallest tile of a multi-pass transform
constexpr int kStridedMaxLog = 9;            // strided passes: <= 512 rows
constexpr int kMaxSteps = 4;
constexpr int kPassThreads = 256;

constexpr int kRootHi = (int)(kOrder >> 12);   // 24576 high-table entries

// Device tables shared by every plan, one block per prime.
struct Tables {
    // Montgomery form of w^i (i < 4096) and w^{4096 j} (j < kRootHi), w the
    // root of order kOrder: any power w^E = lo[E & 4095] * hi[E >> 12].
    const uint32_t* pass_lo;  // [kNumPrimes][4096]
    const uint32_t* pass_hi;  // [kNumPrimes][kRootHi]
};

enum Source : int {
    kSrcArray = 0,   // residues already in `data`
    kSrcDigits = 1,  // digits of W 32-bit words of an n-bit operand in memory
    kSrcSeed = 2,    // words of the SplitMix64 stream of `seed`, bit 0 forced to 1
    kSrcBits = 3,    // element e = bit bit_off + e of `digits` for e < n, else 0
};

// One block of a batch: where its operands, spectra, carry state and output
// live.  Kernels launched for a batch take the block from blockIdx.z (passes)
// or blockIdx.y (carry) and read these fields instead of the scalar ones.
struct JobDesc {
    const uint32_t* key;       // key digits (32-bit view of the key words)
    const uint32_t* c;         // explicit multiplier digits, or null: seeded
    const uint32_t* d;         // explicit addend digits, or null: seeded
    uint64_t seed_a, seed_b;
    uint64_t n, m;
    uint32_t num_digits;       // ceil(n / 32)
    uint32_t chunks;           // carry chunks
    uint32_t* A;               // c-hat [primes][L]
    uint32_t* B;               // x-hat, then the product [primes][L]
    uint32_t* carry;           // carry state: the carry function of each chunk
    uint64_t* out;             // ceil(m / 64) words
};

enum Role : int {
    kRoleMul = 0,    // transform of the multiplier c into A
    kRoleKey = 1,    // transform of the key x into B (last pass fused)
    kRoleInv = 2,    // inverse passes on B
};

enum PassMode : int {
    kForward = 0,    // load, DIF, post-twiddle, store (last pass: keep bit-reversed)
    kInverse = 1,    // load, pre-twiddle, DIT, store natural order
    kFused = 2,      // last forward pass of x, pointwise with c-hat, first inverse pass
};

// One LDS pass of a multi-pass transform over L points (L = 2^k or 3 * 2^k).
// The array is viewed as L / (R S) blocks of R rows by S contiguous columns
// (R = f 2^r with f = 1 or 3, S = 2^s); the pass transforms along the rows of
// every column.  A tile holds R rows by 2^logC adjacent columns.  Inside the
// tile the length-R transform runs as register steps: a radix-3 step first when
// f = 3, then nsteps steps of radix 2^steps[i].
struct PassArgs {
    uint32_t* data;            // [primes][L]
    const uint32_t* other;     // kFused: pre-scaled c-hat, same layout
    const uint32_t* digits;    // kSrcDigits: the operand's words as ceil(n/32) 32-bit halves
    uint64_t seed;             // kSrcSeed
    uint64_t n;                // operand bits (sources only); kSrcBits: elements
    uint64_t bit_off;          // kSrcBits: bit of `digits` that element 0 takes
    uint32_t num_digits;       // ceil(n / 32)
    uint32_t store_limit;      // positions >= this are not stored (L if all)
    uint32_t L;
    int f, r, s, logC;
    int nsteps;
    int steps[kMaxSteps];
    // the same as 4-bit fields (step j at bits 4j): radix logs, and the sum of
    // the logs of the steps before j; read with shifts so that no array of the
    // kernel argument is ever indexed at run time
    uint32_t steps_code, above_code;
    int mode, src;
    int scale_in;              // multiply the source values by scale_w (Shoup; an
                               // operand's first pass, not the dual launch's second
                               // operand)
    uint32_t scale_w[kNumPrimes], scale_q[kNumPrimes];
    Tables tb;
    int primes;                // primes transformed (grid.y): 2 W + 1, or 1 (Toeplitz)
    int dwords;                // W: 32-bit words per digit of a kSrcDigits/kSrcSeed source
    // dual launch (single block, grid.z = 2, seeded multiplier): workgroups with
    // blockIdx.z == 1 run the key's first pass, of the same geometry, with the
    // key digits in `digits` and its spectrum in `other` (both unused by the
    // multiplier's seeded forward pass)
    int dual;
    // batch mode (jobs != null): per-block fields come from jobs[blockIdx.z]
    const JobDesc* jobs;
    int role;
    int limit_to_digits;       // store only the product's coefficients: positions
                               // below ceil(ceil(D / W) / 4) * 4
};

// CRT, carry propagation, addend and bit extraction over the product.
constexpr int kCarryThreads = 256;

struct CarryArgs {
    const uint32_t* res;       // [2 W + 1][L] residues of the product (natural order)
    uint32_t L;
    int dwords;                // W: a coefficient sits at 32-bit positions W K .. W K + 2 W
    uint32_t num_digits;       // D = ceil(n / 32)
    uint64_t n, m;
    int addend_src;            // kSrcDigits or kSrcSeed (no forced odd bit)
    const uint32_t* addend;    // kSrcDigits
    uint64_t seed;             // kSrcSeed
    uint32_t* desc;            // [chunks] carry function of each chunk
    // column sums of the chunks the apply kernel resolves, written by the
    // local kernel: word k = bits 0..31 of s_k (k < D), then from word
    // sums_hi_offset(D) one word per thread holding bits 32..33 of each of its
    // digits' sums (2 bits per digit, its first digit lowest).  The multiplier
    // spectrum's array, free once the pointwise product is taken.
    uint32_t* sums;
    uint64_t* out;             // ceil(m / 64) words
    uint32_t chunks;           // grid width (the largest chunk count in a batch)
    int per;                   // digits per thread (W = 2: 4 or 8; W = 3: 6 or 12)
    const JobDesc* jobs;       // batch mode: per-block fields from jobs[blockIdx.y]
};

// First word of the packed high bits in CarryArgs::sums for D digits.
__host__ __device__ inline uint32_t sums_hi_offset(uint32_t num_digits)
{
    return (num_digits + 63u) & ~63u;
}

// Optional timing of one launch: events stamped by the dispatch itself
// (hipExtLaunchKernelGGL), so no extra packets sit between the kernels.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// 32-bit digits per thread of the carry kernel for a block of D of them, with
// coefficients of W words (a multiple of W).
int carry_digits_per_thread(uint32_t num_digits, int W);

hipError_t launch_pass(const PassArgs& a, hipStream_t stream, unsigned batch = 1,
                       const LaunchEvents& ev = {});

// Toeplitz variant: out[j] (or out[j] ^ ..., accumulate) = the 64 bits
// res[base + 64 j + l] & 1, l < 64, of the first m positions.
hipError_t launch_parity(const uint32_t* res, uint64_t base, uint64_t m, uint64_t* out,
                         int accumulate, hipStream_t stream);
// out[i] = SplitMix64 output i of `seed`, i < words.
hipError_t launch_stream_words(uint64_t seed, uint64_t words, uint64_t* out, hipStream_t stream);
hipError_t launch_carry_local(const CarryArgs& a, hipStream_t stream, unsigned batch = 1,
                              const LaunchEvents& ev = {});
hipError_t launch_carry_apply(const CarryArgs& a, hipStream_t stream, unsigned batch = 1,
                              const LaunchEvents& ev = {});

}  // namespace pa
