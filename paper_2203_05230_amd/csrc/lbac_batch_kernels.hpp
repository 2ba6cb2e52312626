// Batched form of the step (kernels): many independent lattices advanced by
// one persistent launch.  Host side in lbac_batch.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbac_kernels.hpp"

// ---------------------------------------------------------------------------
// Batched form: many independent lattices advanced by ONE persistent launch.
//
// Work is split into items = (instance, tile of at most kBatchTile columns,
// strip of rows).  A run is two persistent launches: the first takes the full
// passes of kBatchS steps each (the multi-step tile function, the populations
// between the steps in LDS), the second the remaining nsteps mod kBatchS steps
// as one-step passes of the same tile function.  A pass of an item reads its
// tile grown by kBatchGrow nodes (its own rows and the rows of the items
// around it) and writes its own tile once.
//
// Schedule.  The (pass, item) slots of a launch are numbered so that every
// slot of pass p of an instance comes before any slot of its pass p + 1 (the
// passes of all instances interleaved in proportion to their lengths, see
// BatchSlots) and each workgroup of the launch takes one slot number from a
// single atomic counter when it starts.
// Before slot (p, I) runs it waits until I and the items whose tiles overlap
// I's read region have published pass p - 1: they wrote the rows I reads, and
// (the relation is symmetric) they have finished reading the part of the
// buffer I is about to overwrite.  Every slot waited for has a smaller
// number, so it is finished or held by a workgroup that has started and stays
// resident until it is done: the lowest unfinished slot can always proceed,
// whatever number of workgroups the device keeps resident, and the schedule
// cannot deadlock.  Every wait is also bounded in wall-clock time and sets an
// error flag that makes all later workgroups exit at once.
namespace lbac {

constexpr int kBatchTile = 224;          // widest item tile (columns)
constexpr int kBatchS = 3;               // steps per full pass
constexpr int kBatchGrow = 2 * kBatchS;  // read region: the tile grown by this many nodes
constexpr int kBatchThreads = stepS_threads<kBatchTile, kBatchS>();
constexpr int kBatchDeps = 16;           // items a slot waits for (itself included)

struct BatchInst {
    StepArgs a;       // entry 2k: instance k as seen by even passes; 2k + 1: by odd passes (src, dst swapped)
    int64_t nsteps;   // steps of this instance in this run
};

struct BatchItem {
    int32_t inst;       // instance
    int32_t x0, w;      // columns [x0, x0 + w)
    int32_t ys, hh;     // rows [ys, ys + hh)
    int32_t down;       // march direction of the strip
    // the items whose pass p - 1 must be published before this item's pass p:
    // itself and every item whose tile overlaps its read region (periodic);
    // repeats pad the list
    int32_t dep[kBatchDeps];
};

struct BatchCtl {
    uint64_t ticket[2];     // next slot of the first and of the second launch
    int64_t timeout_ticks;  // wall-clock ticks a wait may take before giving up
    int32_t dry;            // 1: every pass reads the current state and writes the other buffer (state untouched)
    int32_t err;            // set to 1 when a wait gave up
    int32_t test_stall;     // 1: waits ask for a pass that never completes (tests the time-out path)
    int32_t pad;
};

// Passes of an instance: full passes of kBatchS steps, then one-step passes.
__host__ __device__ constexpr int64_t batch_passes(int64_t nsteps) { return nsteps / kBatchS + nsteps % kBatchS; }

// Waits until every item of dep has published pass `need` (or the time-out
// or another workgroup's error ends the wait: returns false).  Lanes 0..15 of
// each wavefront read one entry each.
__device__ __forceinline__ bool batch_wait(const int32_t* done, const int32_t* dep, int32_t need, BatchCtl* ctl) {
    const int32_t* p = done + dep[threadIdx.x & (kBatchDeps - 1)];
    if (ctl->test_stall) need += (1 << 30);
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const int32_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__all(v >= need)) break;
        if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() - t0 > (uint64_t)ctl->timeout_ticks) {
            __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    // the rows this slot reads are loaded after the counters were seen (the
    // loop consumed them); the tile function reads them with device-scope
    // loads (IoCoherent), so no cache needs invalidating.  A compiler barrier
    // keeps the loads below this point.
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return true;
}

// Slot tables of a launch.  A pass of an instance is an entry (instance, p)
// with the slots of all the instance's items; entries are ordered by the
// fraction of its run the instance has done after the pass, (p + 1) / passes
// (ties by instance), so every instance advances in proportion to its length
// and all finish together, while every pass still comes after the previous
// pass of its instance (the order stays a topological order of the
// dependencies).  start[e] is the first slot number of entry e, start[n] the
// slot count; the items of an instance are the contiguous ids first_item[k] ..
// first_item[k + 1] - 1.  coarse[c] is the entry that holds slot c * 2^B
// (B = kBatchCoarseBits; n - 1 where that slot does not exist), so the entry
// of a slot is found among the few entries between two coarse values instead
// of by a search over all of them, a chain of dependent loads as long as
// log2 n that every workgroup runs before its wait.
constexpr int kBatchCoarseBits = 6;
struct BatchSlots {
    const int32_t* entry;       // 2 per entry: instance, pass
    const int64_t* start;       // n + 1 values
    const int32_t* first_item;  // count + 1 values
    const int32_t* nentries;    // n (device memory: a captured graph's arguments stay valid)
    const int32_t* coarse;      // (start[n] >> kBatchCoarseBits) + 2 values
};

// Maps slot number T of a launch (T < start[n]) to its pass p and item.
__host__ __device__ inline int32_t batch_slot_item(const BatchSlots& s, int64_t T, int32_t n, int32_t& p) {
    const int64_t c = T >> kBatchCoarseBits;
    int32_t lo = s.coarse[c], hi = s.coarse[c + 1] + 1;  // start[lo] <= T < start[hi]
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) / 2;
        if (s.start[mid] <= T) lo = mid;
        else hi = mid;
    }
    p = s.entry[2 * lo + 1];
    return s.first_item[s.entry[2 * lo]] + (int32_t)(T - s.start[lo]);
}

// One workgroup per slot: a workgroup takes the next slot number from the
// launch's counter when it starts (so the slot numbers are taken in the order
// the workgroups start, and every smaller number belongs to a workgroup that
// has started), waits for the slot's dependencies, runs it and publishes.
// The grid has one workgroup per slot of the launch; the hardware dispatcher
// refills the device as workgroups finish.  S = kBatchS: the full passes;
// S = 1: the remaining one-step passes (launch L = 1).  Both use the tile
// function of the multi-step kernel, so one block shape serves both and the
// results are those of the single-instance kernels.  Three waves per SIMD:
// 157 registers, no scratch.
template <int MODEL, int S>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(3))) void batch_kernel(
    const BatchInst* __restrict__ insts, const BatchItem* __restrict__ items, BatchSlots slots, int32_t* done,
    BatchCtl* ctl) {
    static_assert(stepS_threads<kBatchTile, S>() == kBatchThreads, "one block size serves both launches");
    constexpr int L = S == 1 ? 1 : 0;
    __shared__ TileSLds<kBatchTile, S> lds;
    __shared__ int64_t slot;
    const int32_t nent = *slots.nentries;
    const int64_t total = slots.start[nent];
    if (threadIdx.x == 0) {
        const bool stop = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        slot = stop ? total : (int64_t)atomicAdd((unsigned long long*)&ctl->ticket[L], 1ull);
    }
    __syncthreads();
    // read as a uniform value, so that the item and its instance's arguments
    // are scalar loads into scalar registers
    const int64_t T = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(slot >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)slot));
    if (T >= total) return;
    int32_t p;
    const int32_t id = batch_slot_item(slots, T, nent, p);
    const BatchItem& item = items[id];
    if (p > 0) {
        const bool ok = batch_wait(done, item.dep, p - 1, ctl);
        if (__syncthreads_or(!ok)) return;  // every wavefront leaves together
    }
    const bool dry = ctl->dry != 0;
    const int64_t nfull = insts[2 * item.inst].nsteps / kBatchS;
    const int64_t gp = S == 1 ? nfull + p : p;  // pass index within the run
    const StepArgs& a = insts[2 * item.inst + (int)(gp & 1)].a;
    const int64_t t = a.t_dev[0] + (dry ? 0 : (S == 1 ? nfull * kBatchS + p : (int64_t)p * kBatchS));
    stepS_tile_lds<MODEL, kBatchTile, S, ST_PLAIN, true>(a, item.x0, item.w, item.ys, item.hh, t, item.down != 0,
                                                         lds);
    // publish: every wavefront waits until its device-scope stores have
    // completed (vmcnt counts stores on this architecture), then the counter
    // moves; no writeback of the whole L2 is needed
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(done + id, p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Resets the progress counters and the slot counter of launch L and, if
// asked, the error flag (a kernel, not a memset, so that the whole run can be
// replayed from a captured graph).
static __global__ void batch_reset_kernel(int32_t* done, int32_t nitems, BatchCtl* ctl, int32_t L, int32_t reset_err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nitems) done[i] = -1;
    if (i == 0) {
        ctl->ticket[L] = 0;
        if (reset_err) ctl->err = 0;
    }
}

// Advances every instance's step counter by its step count (skipped on dry runs).
static __global__ void batch_advance_kernel(const BatchInst* __restrict__ insts, int32_t count, const BatchCtl* ctl) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count && ctl->dry == 0 && ctl->err == 0)
        const_cast<int64_t*>(insts[2 * k].a.t_dev)[0] += insts[2 * k].nsteps;
}

}  // namespace lbac
