// Batched form of the step (kernels): many independent lattices advanced by
// one persistent launch.  Host side in lbac_batch.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbac_kernels.hpp"

// ---------------------------------------------------------------------------
// Batched form: many independent lattices advanced by ONE persistent launch.
//
// Work is split into items = (instance, kBatchTile-column block, strip).
// Each workgroup (the block layout: kBatchTile column threads and one halo
// wavefront) owns a fixed list of items and walks them in pass-major order.
// A run is two persistent launches: the first takes the full passes of
// kBatchS steps each with the multi-step tile function, the second the
// remaining nsteps mod kBatchS steps as one-step passes of the block tile
// function.  An item reads its tile grown by 2 kBatchS nodes and writes its
// own tile once per pass.  Before item I runs pass p it waits until the
// items of the same instance whose tiles overlap I's grown tile have
// completed pass p-1: they wrote the rows and columns I reads, and (the
// relation is symmetric) they have finished reading the part of the buffer I
// is about to overwrite.  With every workgroup resident (the grid never
// exceeds the occupancy limit) the lowest pending pass can always proceed,
// so the schedule cannot deadlock; every wait is also bounded in wall-clock
// time and sets an error flag that makes all workgroups exit.
namespace lbac {

constexpr int kBatchTile = 128;  // columns per item
constexpr int kBatchS = 3;       // steps per full pass
constexpr int kBatchGrow = 2 * kBatchS;  // read region: the tile grown by this many nodes

struct BatchInst {
    StepArgs a;       // entry 2k: instance k as seen by even passes; 2k + 1: by odd passes (src, dst swapped)
    int64_t nsteps;   // steps of this instance in this run
};

struct BatchItem {
    int32_t inst, bxi, syi, down;
    // ids of the items whose tiles overlap this item's read region (its tile
    // grown by kBatchGrow nodes, periodic), itself excluded; repeats pad the list
    int32_t nbr[16];
};

struct BatchCtl {
    int64_t max_full, max_rest;  // passes of the first and of the second launch, largest over the instances
    int64_t timeout_ticks;  // wall-clock ticks a wait may take before giving up
    int32_t dry;            // 1: every pass reads src and writes dst (state untouched)
    int32_t err;            // set to 1 when a wait gave up
    int32_t test_stall;     // 1: waits ask for a pass that never completes (tests the time-out path)
};

__host__ __device__ constexpr int64_t batch_passes(int64_t nsteps) { return nsteps / kBatchS + nsteps % kBatchS; }

__device__ __forceinline__ bool batch_wait(const int32_t* done, const BatchItem* item, int32_t need, BatchCtl* ctl) {
    const int32_t* p = done + item->nbr[threadIdx.x & 15];
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
    // make the neighbours' rows visible to this wavefront's loads
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// S = kBatchS: the full passes; S = 1: the remaining one-step passes.  Three
// waves per SIMD are asked for: the loop over items around the multi-step
// tile function would otherwise take 190 registers (two waves per SIMD); at
// 168 a few values of the prologue spill, and the batch runs 1.33x faster.
template <int MODEL, int S>
__global__ __launch_bounds__(block_threads<kBatchTile>()) __attribute__((amdgpu_waves_per_eu(3))) void batch_kernel(const BatchInst* __restrict__ insts,
                                                                          const BatchItem* __restrict__ items,
                                                                          const int32_t* __restrict__ wg_off,
                                                                          const int32_t* __restrict__ wg_items,
                                                                          int32_t* done, BatchCtl* ctl) {
    __shared__ typename std::conditional<S == 1, TileLds<float, kBatchTile>, TileSLds<kBatchTile, kBatchS>>::type lds;
    if (S == 1 && __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int beg = wg_off[blockIdx.x], end = wg_off[blockIdx.x + 1];
    const int64_t max_passes = S == 1 ? ctl->max_rest : ctl->max_full;
    const bool dry = ctl->dry != 0;
    for (int64_t p = 0; p < max_passes; ++p) {
        bool any = false;
        for (int i = beg; i < end; ++i) {
            const int id = wg_items[i];
            const BatchItem* item = items + id;
            const int64_t nsteps = insts[2 * item->inst].nsteps;
            const int64_t nfull = nsteps / kBatchS;
            if (p >= (S == 1 ? nsteps % kBatchS : nfull)) continue;
            any = true;
            if (p > 0) {
                const bool ok = batch_wait(done, item, (int32_t)(p - 1), ctl);
                if (__syncthreads_or(!ok)) return;  // every wavefront leaves together
            }
            const int64_t gp = S == 1 ? nfull + p : p;  // pass index within the run
            const StepArgs& a = insts[2 * item->inst + (int)(gp & 1)].a;
            const int64_t t = a.t_dev[0] + (dry ? 0 : (S == 1 ? nfull * kBatchS + p : p * kBatchS));
            if constexpr (S == 1)
                step_tile_lds<float, ST_PLAIN, MODEL, kBatchTile, 2>(a, item->bxi, item->syi, t, item->down != 0, lds);
            else {
                static_assert(stepS_threads<kBatchTile, kBatchS>() == block_threads<kBatchTile>(),
                              "one block size serves both tile functions");
                stepS_tile_lds<MODEL, kBatchTile, kBatchS>(a, item->bxi, item->syi, t, item->down != 0, lds);
            }
            // publish: every wavefront's stores are visible before the counter moves
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (threadIdx.x == 0) __hip_atomic_store(done + id, (int32_t)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!any) break;
    }
}

// Resets the progress counters and, if asked, the error flag (a kernel, not
// a memset, so that the whole run can be replayed from a captured graph).
static __global__ void batch_reset_kernel(int32_t* done, int32_t nitems, BatchCtl* ctl, int32_t reset_err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nitems) done[i] = -1;
    if (i == 0 && reset_err) ctl->err = 0;
}

// Advances every instance's step counter by its step count (skipped on dry runs).
static __global__ void batch_advance_kernel(const BatchInst* __restrict__ insts, int32_t count, const BatchCtl* ctl) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count && ctl->dry == 0 && ctl->err == 0)
        const_cast<int64_t*>(insts[2 * k].a.t_dev)[0] += insts[2 * k].nsteps;
}

}  // namespace lbac
