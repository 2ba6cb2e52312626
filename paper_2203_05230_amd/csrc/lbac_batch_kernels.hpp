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
// strip of rows; one storage, FP32 or shifted 16-bit, for every instance).
// A run is two persistent launches: the first takes the full
// passes of kBatchS steps each (the multi-step tile function, the populations
// between the steps in LDS), the second the remaining nsteps mod kBatchS steps
// as one-step passes of the same tile function.  A pass of an item reads its
// tile grown by kBatchGrow nodes (its own rows and the rows of the items
// around it) and writes its own tile once.
//
// Schedule.  The instances are dealt to kBatchClasses classes of about equal
// work, one per XCD.  The (pass, item) slots of a class are numbered so that
// every slot of pass p of an instance comes before any slot of its pass p + 1
// (the passes of the class's instances interleaved in proportion to their
// lengths, see BatchSlots), and each class has its own atomic counter.  A
// workgroup takes one slot at a time: from the counter of its own class,
// blockIdx mod kBatchClasses (the dispatcher hands workgroups to the XCDs in
// turn, so a class's tiles, and the halo lines neighbouring tiles share, stay
// in one XCD's L2), or, once that class is used up, from the next class that
// is not.
// Before slot (p, I) runs it waits until I and the items whose tiles overlap
// I's read region have published pass p - 1: they wrote the rows I reads, and
// (the relation is symmetric) they have finished reading the part of the
// buffer I is about to overwrite.  Every slot waited for belongs to the same
// class and has a smaller number there, so it is finished or held by a
// running workgroup that stays resident until it is done (a slot is taken
// only by a running workgroup): the lowest unfinished slot of a class can
// always proceed, whatever number of workgroups the device keeps resident and
// whichever class a workgroup takes from, and the schedule cannot deadlock.
// Every wait is also bounded in wall-clock time and sets an error flag that
// makes all later workgroups exit at once.
namespace lbac {

constexpr int kBatchTile = 240;          // widest item tile (columns)
constexpr int kBatchS = 3;               // steps per full pass
constexpr int kBatchGrow = 2 * kBatchS;  // read region: the tile grown by this many nodes
constexpr int kBatchThreads = stepS_threads<kBatchTile, kBatchS>();
constexpr int kBatchDeps = 16;           // items a slot waits for (itself included)
constexpr int kBatchClasses = 8;         // slot classes: one per XCD

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
    uint64_t ticket[2][kBatchClasses];  // next slot of each class, first and second launch
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
// with the slots of all the instance's items.  The entries of class c come
// as one block, slots cls[c] .. cls[c + 1] - 1, ordered by the fraction of
// its run the instance has done after the pass, (p + 1) / passes (ties by
// instance), so every instance of a class advances in proportion to its
// length and all finish together, while every pass still comes after the
// previous pass of its instance (the order stays a topological order of the
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
    const int64_t* cls;         // kBatchClasses + 1 values: first slot of each class, then start[n]
};

// The slot a workgroup of class x0 takes: the next one of its own class, or,
// once that class is used up, of the next class in turn that is not; cls[C]
// (every slot taken) if none is left.  take(c, n) returns the next number of
// class c's counter and advances it (n: the class's slot count, at or above
// which the counter need not move).
template <typename Take>
__host__ __device__ inline int64_t batch_take(const int64_t* cls, int x0, Take take) {
    for (int k = 0; k < kBatchClasses; ++k) {
        const int c = (x0 + k) % kBatchClasses;
        const int64_t n = cls[c + 1] - cls[c];
        const int64_t l = take(c, n);
        if (l < n) return cls[c] + l;
    }
    return cls[kBatchClasses];
}

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

// A workgroup takes a slot from its class's counter (so the slot numbers of
// a class are taken in the order its workgroups ask for them), waits for the
// slot's dependencies, runs it, publishes, and takes the next slot, until
// none is left.  A slot is only ever taken by a running workgroup, which
// holds it until it is done, so every smaller number of a class belongs to a
// slot that is finished or held by a running workgroup, however many
// workgroups of the grid the device keeps resident (the grid, about the
// resident count, only sets how many run at once; a workgroup keeps its
// XCD, and so its class, for all its slots).  S = kBatchS: the full passes;
// S = 1: the remaining one-step passes (launch L = 1).  Both use the tile
// function of the multi-step kernel, so one block shape serves both and the
// results are those of the single-instance kernels.  Three waves per SIMD;
// the few registers spilled (36 bytes per lane) are per-slot values, outside
// the row loop.
// Everything a batch launch reads, in device memory behind one pointer: the
// workgroup loop reads it again per slot, so that the tile function has the
// scalar registers to itself instead of sharing them with a dozen pointers
// held across it (held, they spilled).
struct BatchDev {
    const BatchInst* insts;
    const BatchItem* items;
    BatchSlots slots[2];  // of the first and of the second launch
    int32_t* done;
    BatchCtl* ctl;
};

// ST: the storage of every instance of the batch (FP32, or shifted FP16 or
// BF16 with the populations in FP32 between the steps of a pass).
template <int MODEL, int S, int ST>
__global__ __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(3))) void batch_kernel(
    const BatchDev* dv) {
    static_assert(stepS_threads<kBatchTile, S>() == kBatchThreads, "one block size serves both launches");
#if defined(__HIP_DEVICE_COMPILE__)  // (copies out of the constant address space exist on the device only)
    constexpr int L = S == 1 ? 1 : 0;
    // the argument block, the items and the instances' arguments are not
    // written during a launch: read through the constant address space, as
    // scalar loads
    using C4 = const __attribute__((address_space(4))) BatchDev;
    using I4 = const __attribute__((address_space(4))) BatchItem;
    using N4 = const __attribute__((address_space(4))) BatchInst;
    __shared__ TileSLds<kBatchTile, S> lds;
    __shared__ int64_t slot;
    for (;;) {
        // an opaque zero, so that the block is read again per slot instead
        // of being held in registers across the tile function
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        C4& D = ((C4*)dv)[z];
        const BatchSlots slots = D.slots[L];
        BatchCtl* ctl = D.ctl;
        const int32_t nent = *slots.nentries;
        const int64_t total = slots.start[nent];
        if (threadIdx.x == 0) {
            const bool stop = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            slot = stop ? total : batch_take(slots.cls, (int)(blockIdx.x % kBatchClasses), [&](int c, int64_t n) -> int64_t {
                uint64_t* tk = &ctl->ticket[L][c];
                // a used-up class is passed over without moving its counter
                if ((int64_t)__hip_atomic_load(tk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) return n;
                return (int64_t)atomicAdd((unsigned long long*)tk, 1ull);
            });
        }
        __syncthreads();
        // read as a uniform value (thread 0 writes `slot` again only after
        // the publishing barrier below, which every thread reaches after
        // this read)
        const int64_t T = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(slot >> 32)) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane((int)slot));
        if (T >= total) return;
        int32_t p;
        const int32_t id = batch_slot_item(slots, T, nent, p);
        I4& item = ((I4*)D.items)[id];
        if (p > 0) {
            const bool ok = batch_wait(D.done, (const int32_t*)item.dep, p - 1, ctl);
            if (__syncthreads_or(!ok)) return;  // every wavefront leaves together
        }
        const bool dry = ctl->dry != 0;
        N4* insts = (N4*)D.insts;
        const int32_t inst = item.inst;
        const int64_t nfull = insts[2 * inst].nsteps / kBatchS;
        const int64_t gp = S == 1 ? nfull + p : p;  // pass index within the run
        const StepArgs a = insts[2 * inst + (int)(gp & 1)].a;
        const int64_t t = a.t_dev[0] + (dry ? 0 : (S == 1 ? nfull * kBatchS + p : (int64_t)p * kBatchS));
        stepS_tile_lds<MODEL, kBatchTile, S, ST, true>(a, item.x0, item.w, item.ys, item.hh, t, item.down != 0, lds);
        // publish: every wavefront waits until its device-scope stores have
        // completed (vmcnt counts stores on this architecture), then the
        // counter moves; no writeback of the whole L2 is needed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(D.done + id, p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#endif
}

// Resets the progress counters and the slot counter of launch L and, if
// asked, the error flag (a kernel, not a memset, so that the whole run can be
// replayed from a captured graph).
static __global__ void batch_reset_kernel(int32_t* done, int32_t nitems, BatchCtl* ctl, int32_t L, int32_t reset_err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nitems) done[i] = -1;
    if (i == 0) {
        for (int c = 0; c < kBatchClasses; ++c) ctl->ticket[L][c] = 0;
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
