// libpa internals shared by the runtime, the batch path and the server.
#pragma once

#include "../../include/pa.h"
#include "kernels.h"

// The state behind a pa_ctx handle.
struct pa_ctx {
    int device = 0;
    hipStream_t stream = nullptr;     // used by the synchronous entry points
    // tables
    uint32_t* pass_lo = nullptr;
    uint32_t* pass_hi = nullptr;
    // workspace: cap_L residues per array (all primes), carry state for cap_D digits
    uint64_t cap_L = 0, cap_D = 0;
    uint32_t* A = nullptr;            // c-hat   [primes][L]
    uint32_t* B = nullptr;            // x-hat, then the product residues [primes][L]
    uint32_t* status = nullptr;       // carry state: the carry function of each chunk
    // device address of this GPU's copy of the allocation-free entry point's
    // scratch (taken with hipGetSymbolAddress in pa_init)
    uint8_t* scratch = nullptr;
    // staging for the synchronous (host memory) entry points
    uint64_t cap_words = 0;
    uint64_t* d_key = nullptr;
    uint64_t* d_c = nullptr;
    uint64_t* d_d = nullptr;
    uint64_t* d_out = nullptr;
    // the seeded t of the Toeplitz variant
    uint64_t cap_tbits = 0;
    uint64_t* tbits = nullptr;
    // chosen plan geometry per transform length (slot: k, or 32 + k for 3 2^k);
    // t == 0: the defaults
    static constexpr int kPlanSlots = 128;   // (W == 3) 64 + (f == 3) 32 + k
    struct PlanChoice {
        int t = 0, ts = 0, r0 = 0;
    } plans[kPlanSlots];
    // side streams (default priority) on which batch groups run concurrently
    static constexpr int kSide = 4;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSide] = {};
    hipEvent_t ev[2 * PA_PROFILE_MAX] = {};
    bool have_events = false;
    char err[512] = {0};
    // pa_opts: the device bytes the context may hold for itself (0: no limit)
    // and what it holds now; the file of tuned geometries ("" for none)
    uint64_t budget = 0;
    uint64_t held = 0;
    char tune_cache[1024] = {0};
    char arch[64] = {0};
};

namespace pa {

// Device buffers of one block: the operands (32-bit digit views; c and d null
// when seeded), the two spectra, the carry state and the output words.
struct BlockBufs {
    const uint32_t* key = nullptr;
    const uint32_t* c = nullptr;
    const uint32_t* d = nullptr;
    uint64_t seed_a = 0, seed_b = 0, n = 0, m = 0;
    uint32_t* A = nullptr;
    uint32_t* B = nullptr;
    uint32_t* carry = nullptr;
    uint64_t* out = nullptr;
};

// Device bytes of A, B and the carry state for a block of n bits, and their
// placement from `base` (256-byte aligned pieces).
uint64_t block_workspace_bytes(uint64_t n);
void block_layout(uint64_t n, uint8_t* base, BlockBufs* b);

// Queue every kernel of one block's hash on `stream` (buffers given).
int enqueue_block(pa_ctx* ctx, const BlockBufs& b, hipStream_t stream);

// Record a failure on ctx and return `code`.
int set_error(pa_ctx* ctx, int code, const char* what);

}  // namespace pa
