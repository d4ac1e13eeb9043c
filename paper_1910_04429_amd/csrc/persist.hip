// Persistent batch kernel: every launch of a batch (the transform passes and
// the carry kernels of all its blocks) run by one grid of resident workgroups
// that take work items from a device queue.
//
// An item is what one workgroup of the per-launch kernels does: one tile of
// one prime of one block's pass, or one carry chunk of one block.  The host
// lists the launches of every block group (the same launches the grouped path
// makes, with the same arguments) and orders them by level (the length of the
// longest dependency chain before them); items are numbered in that order,
// launch by launch, block by block.  A workgroup takes the next item number
// from a device counter, waits until the launches its item depends on are
// complete for the item's block, runs it, and counts it done for that block.
//
// Dependencies (a pass reads what the previous pass of the same array wrote;
// the fused pass also reads the multiplier's spectrum; the carry kernels read
// the product; the apply kernel reads every chunk function) always point to
// launches of a lower level, whose items have smaller numbers.  An item is
// taken only after every item before it was taken by a running workgroup, so
// every wait ends without any workgroup being resident for it.  Waits are
// bounded all the same: after wait_ticks of the device clock it raises the abort
// flag, every later wait gives up at once, and the host reports the run as
// failed (pa_batch_result); the grid always drains.
//
// Memory order: every wave of a workgroup ends an item by waiting for its
// stores to reach its XCD's L2, then the workgroup's barrier, then thread 0
// adds the count with an agent-scope release (which writes that L2 back).  A
// waiting workgroup's thread 0 polls the count with relaxed loads and, once
// it is complete, fences with an agent-scope acquire (which drops stale L1
// and L2 lines) before the barrier after which the workgroup loads.
#include "carry_body.h"
#include "pass_body.h"
#include "persist.h"

namespace pa {
namespace {

// The launch table as constant memory: it is written by the host before the
// run and only read here, so its uniform fields go to scalar registers through
// scalar loads, as a kernel argument's would.  (The address space exists in
// the device compilation only; the host compilation of this source sees a
// plain pointer and never runs these functions.)
#if defined(__HIP_DEVICE_COMPILE__)
using ConstLaunch = const __attribute__((address_space(4))) PersistLaunch;
#else
using ConstLaunch = const PersistLaunch;
#endif

__device__ __forceinline__ ConstLaunch* launch_table(const PersistArgs& a)
{
    return (ConstLaunch*)a.launches;
}

// Thread 0: wait until launch `dep` is complete for job z.  Returns false if
// the run was aborted (now or before).  The count is polled with relaxed loads
// (an acquire load would invalidate the XCD's L2 on every poll); the caller
// fences once when every wait has succeeded.  A wait gives up after
// wait_ticks of the device's constant-rate clock, and then every later wait
// gives up at once.
__device__ bool wait_for(const PersistArgs& a, int dep, uint32_t z)
{
    if (dep < 0) return true;
    uint32_t* abort_flag = a.ctr + 1;
    if (a.force_abort) {
        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
    }
    ConstLaunch& d = launch_table(a)[dep];
    const uint32_t need = d.gx * d.gy;
    uint32_t* cnt = a.ctr + kPersistCounters + d.ctr_base + z;
    if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need)
        return true;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
            wall_clock64() - t0 > a.wait_ticks) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return true;
}

// s_waitcnt vmcnt(0), with lgkmcnt and expcnt left at their maxima (no wait).
constexpr int kWaitVmcnt0 = (0xF << 8) | (0x7 << 4);

// A scalar (wavefront-uniform) copy of a pointer, so that loads through it are
// scalar loads.
__device__ __forceinline__ ConstLaunch* uniform(ConstLaunch* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (ConstLaunch*)(((uint64_t)hi << 32) | lo);
}

// One item of a block of W-word digits, out of line: inlined into the queue
// loop, the constants and arguments of every pass and carry variant would be
// hoisted out of that loop and held in registers for the whole kernel.  Its
// arguments are uniform; the copies of the launch's arguments are kept in
// scalar registers.  The carry runs with the short chunks of each layout (4 or
// 6 digits per thread), the variant with the fewest registers.
template <int W>
__device__ __attribute__((noinline)) void run_item(ConstLaunch* Lp, uint32_t x, uint32_t y,
                                                   uint32_t z)
{
    extern __shared__ __align__(16) uint32_t sm[];
    constexpr int kPer = W == 3 ? kPersistPer3 : kPersistPer2;
    ConstLaunch* L = uniform(Lp);
    x = __builtin_amdgcn_readfirstlane(x);
    y = __builtin_amdgcn_readfirstlane(y);
    z = __builtin_amdgcn_readfirstlane(z);
    if (L->kind == kPersistPass) {
        const PassArgs pa = L->pass;
        const TileCoord tc{x, L->gx, z, false};
        switch (pass_kind(pa)) {
        case kKindFirst: pass_tile_kind<W, kKindFirst, 1>(pa, sm, y, tc); break;
        case kKindForward: pass_tile_kind<W, kKindForward, 1>(pa, sm, y, tc); break;
        case kKindFusedFirst: pass_tile_kind<W, kKindFusedFirst, 1>(pa, sm, y, tc); break;
        case kKindFused: pass_tile_kind<W, kKindFused, 1>(pa, sm, y, tc); break;
        default: pass_tile_kind<W, kKindInverse, 1>(pa, sm, y, tc); break;
        }
    } else {
        const CarryArgs ca = L->carry;
        auto& sh = *reinterpret_cast<CarryShared<kPer, W>*>(sm);
        if (L->kind == kPersistCarryLocal)
            carry_chunk<kPer, false, W>(ca, x, z, sh);
        else
            carry_chunk<kPer, true, W>(ca, x, z, sh);
    }
}

// The launch of queue item `item`: the last one whose first item is <= it.
__device__ __forceinline__ ConstLaunch* launch_of(const PersistArgs& a, uint32_t item)
{
    ConstLaunch* table = launch_table(a);
    uint32_t lo = 0, hi = a.nlaunch;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (table[mid].first <= item) lo = mid;
        else hi = mid;
    }
    return table + lo;
}

// The queue loop.  Seven waves per SIMD, as for the pass kernel.
//
// Each iteration has one region that only thread 0 runs (count the previous
// item done, take the next item, wait for its dependencies), then a barrier,
// then code that every thread runs alike.  With the done count at the end of
// an iteration and the take at the start of the next as two separate
// thread-0 regions, the compiler joined them across the loop's back edge and
// ran the other threads' next iteration (barrier, read of the item number)
// before thread 0's take: the workgroup then repeated one item forever.
__global__ __launch_bounds__(kPassThreads) __attribute__((amdgpu_waves_per_eu(7, 8)))
void k_persist(const PersistArgs a)
{
    __shared__ uint32_t s_item;
    __shared__ uint32_t s_go;
    uint32_t prev_ctr = 0xFFFFFFFFu;   // done counter of the previous item, if any
    for (;;) {
        if (threadIdx.x == 0) {
            if (prev_ctr != 0xFFFFFFFFu)
                __hip_atomic_fetch_add(a.ctr + kPersistCounters + prev_ctr, 1u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t item =
                __hip_atomic_fetch_add(a.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t go = 0;
            if (item < a.total) {
                ConstLaunch* L = launch_of(a, item);
                const uint32_t z = (item - L->first) / (L->gx * L->gy);
                go = (wait_for(a, L->dep0, z) && wait_for(a, L->dep1, z)) ? 1u : 0u;
                // acquire: the CU's L1 and the XCD's L2 drop lines that the
                // awaited items (possibly on other XCDs) have rewritten,
                // before any wave of the workgroup loads
                if (go && (L->dep0 >= 0 || L->dep1 >= 0))
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_item = item;
            s_go = go;
        }
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= a.total)
            break;
        ConstLaunch* L = uniform(launch_of(a, item));
        const uint32_t li = item - L->first;
        const uint32_t z = li / (L->gx * L->gy);
        const uint32_t x = li % L->gx;
        const uint32_t y = (li / L->gx) % L->gy;
        if (__builtin_amdgcn_readfirstlane(s_go)) {
            if (L->W == 3)
                run_item<3>(L, x, y, z);
            else
                run_item<2>(L, x, y, z);
        }
        // each wave waits until its stores have reached its XCD's L2 (vmcnt
        // 0); after the barrier, thread 0's release at the start of the next
        // iteration writes the L2 back and publishes the count
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        prev_ctr = L->ctr_base + z;
    }
}

// The queue counter, the abort flag and the done counts start at zero.
__global__ __launch_bounds__(256) void k_persist_reset(uint32_t* ctr, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        ctr[i] = 0u;
}

}  // namespace

uint32_t persist_carry_lds_bytes(int W)
{
    return W == 3 ? sizeof(CarryShared<kPersistPer3, 3>) : sizeof(CarryShared<kPersistPer2, 2>);
}

hipError_t persist_grid(uint32_t lds_bytes, int device, uint32_t* workgroups)
{
    int per_cu = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persist, kPassThreads,
                                                                lds_bytes);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    *workgroups = (uint32_t)per_cu * (uint32_t)cus;
    return hipSuccess;
}

hipError_t launch_persist(const PersistArgs& a, uint32_t workgroups, uint32_t lds_bytes,
                          hipStream_t stream)
{
    const uint32_t count = kPersistCounters + a.ncounters;
    hipLaunchKernelGGL(k_persist_reset, dim3((count + 255) / 256 < 64 ? (count + 255) / 256 : 64),
                       dim3(256), 0, stream, a.ctr, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t wg = workgroups < a.total ? workgroups : a.total;
    if (wg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_persist, dim3(wg), dim3(kPassThreads), lds_bytes, stream, a);
    return hipGetLastError();
}

}  // namespace pa
