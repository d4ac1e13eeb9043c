// Interface between the runtime and the persistent batch kernel (persist.hip).
#pragma once

#include "kernels.h"

namespace pa {

enum PersistKind : int {
    kPersistPass = 0,        // one tile of one prime of one block's pass
    kPersistCarryLocal = 1,  // one carry chunk: write its carry function
    kPersistCarryApply = 2,  // one carry chunk: resolve it, write its output words
};

// One launch of the grouped path, as items of the work queue.  Its items are
// numbered first .. first + gx gy gz - 1 with x fastest and z (the block of
// the group) slowest; an item of block z may run when launches dep0 and dep1
// (indices into the launch table, -1 for none) are complete for block z.
struct PersistLaunch {
    int kind;
    int W;                   // digit words of the launch's blocks (2 or 3)
    uint32_t gx, gy, gz;     // tiles, primes, blocks (carry: chunks, 1, blocks)
    uint32_t first;          // queue number of its first item
    uint32_t ctr_base;       // its done counts: ctr[kPersistCounters + ctr_base + z]
    int dep0, dep1;
    PassArgs pass;           // kind == kPersistPass (batch mode: jobs set)
    CarryArgs carry;         // carry kinds (batch mode: jobs set)
};

// ctr[0]: next item; ctr[1]: abort flag; then one done count per launch and block.
constexpr uint32_t kPersistCounters = 2;

struct PersistArgs {
    const PersistLaunch* launches;   // sorted by `first`
    uint32_t nlaunch;
    uint32_t total;                  // items
    uint32_t* ctr;                   // kPersistCounters + ncounters words
    uint32_t ncounters;
    uint64_t wait_ticks;             // device clock ticks before a wait gives up
    int force_abort;                 // every wait for a dependency gives up at once
};

// Carry digits per thread in the persistent kernel (the short chunks of each
// layout: the carry variant with the fewest registers).
constexpr int kPersistPer2 = 4;
constexpr int kPersistPer3 = 6;

// Dynamic LDS bytes of a carry chunk of W-word digits in the persistent kernel.
uint32_t persist_carry_lds_bytes(int W);

// Workgroups of the persistent kernel that fit on the device at once.
hipError_t persist_grid(uint32_t lds_bytes, int device, uint32_t* workgroups);

// Reset the counters, then run the queue with min(workgroups, total) workgroups.
hipError_t launch_persist(const PersistArgs& a, uint32_t workgroups, uint32_t lds_bytes,
                          hipStream_t stream);

}  // namespace pa
