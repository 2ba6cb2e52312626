// Batched form: many independent lattices advanced by one persistent kernel
// launch per run phase, replayed from a captured HIP graph (see batch_kernel
// in lbac_batch_kernels.hpp for the slot schedule and its dependency rule).
//
// Host side: the work list of (instance, column tile, strip) items with their
// dependency lists, the classes and pass-major slot tables of the two
// launches, graph capture of reset -> full passes -> reset -> one-step passes
// -> time advance, and an autotuner over the strip height.
// It also exports a host-only check of the schedule (lbac_batch_schedule_check)
// that runs the kernel's slot protocol on the CPU with a bounded number of
// concurrently running workgroups.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "lbac_batch_kernels.hpp"
#include "lbac_internal.hpp"

using namespace lbac;
using namespace lbac_host;

namespace {

// Rows per strip at least (an instance with fewer rows is one strip).
constexpr int kBatchMinStrip = kBatchGrow + 2;
// Slots of one batch launch at most (bounds the host tables).
constexpr int64_t kBatchMaxSlots = int64_t(1) << 36;

struct Geometry {
    int nx, ny;
};

// An item of the schedule (host form).
struct ItemH {
    int inst, x0, w, ys, hh, down;
    std::vector<int32_t> dep;  // itself first, then the items overlapping its read region
};

// Column tiles of an instance nx columns wide: widths that are multiples of 16
// columns (every tile starts on a 64-byte boundary in FP32 storage, 32 bytes
// in 16-bit storage; the tile function gives the columns before the first
// 128-byte line to its halo wavefront), at most kBatchTile, the last one
// ragged; chosen to minimise the wavefronts that run per row
// (ceil((w + 4S) / 64) per tile), then the number of tiles, the widest tiles
// first (a 512-column instance: 240 + 240 + 32, nine wavefronts per row
// against ten with multiples of 32).
std::vector<std::pair<int, int>> column_tiles(int nx) {
    constexpr int U = 16;
    const int n = (nx + U - 1) / U;
    std::vector<std::pair<int, int>> best(n + 1, {INT_MAX, INT_MAX});
    std::vector<int> next(n + 1, n);
    best[n] = {0, 0};
    for (int c = n - 1; c >= 0; --c)
        for (int k = std::min(kBatchTile / U, n - c); k >= 1; --k) {
            const int w = std::min(nx, (c + k) * U) - c * U;
            const std::pair<int, int> cand(best[c + k].first + (w + 4 * kBatchS + 63) / 64, best[c + k].second + 1);
            if (cand < best[c]) {
                best[c] = cand;
                next[c] = c + k;
            }
        }
    std::vector<std::pair<int, int>> t;
    for (int c = 0; c < n; c = next[c]) t.push_back({c * U, std::min(nx, next[c] * U) - c * U});
    return t;
}

// Items of every instance (instance-major, strips, tiles) and their dependency
// lists: an item depends on itself and on every item of its instance whose
// tile overlaps its read region, columns x0 - G .. x0 + w - 1 + G and rows
// ys - G .. ys + hh - 1 + G (G = kBatchGrow, periodic).  Returns false if an
// item would need more than kBatchDeps entries.
bool build_items(const std::vector<Geometry>& geo, int strip_h, std::vector<ItemH>& items) {
    constexpr int G = kBatchGrow;
    items.clear();
    for (int k = 0; k < (int)geo.size(); ++k) {
        const int nx = geo[k].nx, ny = geo[k].ny;
        const std::vector<std::pair<int, int>> ct = column_tiles(nx);
        // the nearest whole number of strips to ny / strip_h (at least one,
        // at most ny / kBatchMinStrip), of balanced heights: strip j covers
        // rows [j ny / nby, (j + 1) ny / nby); each strip costs its rows plus
        // the pipeline's fill, so a ragged last strip is avoided
        const int nby = std::max(1, std::min((int)std::lround((double)ny / strip_h), ny / kBatchMinStrip));
        const int nbx = (int)ct.size();
        auto strip_y0 = [&](int j) { return (int)((int64_t)j * ny / nby); };
        std::vector<int> tile_of_col(nx), strip_of_row(ny);
        for (int i = 0; i < nbx; ++i)
            for (int c = ct[i].first; c < ct[i].first + ct[i].second; ++c) tile_of_col[c] = i;
        for (int j = 0; j < nby; ++j)
            for (int r = strip_y0(j); r < strip_y0(j + 1); ++r) strip_of_row[r] = j;
        const int base = (int)items.size();
        for (int j = 0; j < nby; ++j)
            for (int i = 0; i < nbx; ++i) {
                ItemH it;
                it.inst = k;
                it.x0 = ct[i].first;
                it.w = ct[i].second;
                it.ys = strip_y0(j);
                it.hh = strip_y0(j + 1) - strip_y0(j);
                it.down = j & 1;
                std::vector<int> tx, ty;
                for (int c = it.x0 - G; c <= it.x0 + it.w - 1 + G; ++c) tx.push_back(tile_of_col[((c % nx) + nx) % nx]);
                for (int r = it.ys - G; r <= it.ys + it.hh - 1 + G; ++r) ty.push_back(strip_of_row[((r % ny) + ny) % ny]);
                std::sort(tx.begin(), tx.end());
                tx.erase(std::unique(tx.begin(), tx.end()), tx.end());
                std::sort(ty.begin(), ty.end());
                ty.erase(std::unique(ty.begin(), ty.end()), ty.end());
                it.dep.push_back(base + j * nbx + i);
                for (int jj : ty)
                    for (int ii : tx)
                        if (ii != i || jj != j) it.dep.push_back(base + jj * nbx + ii);
                if ((int)it.dep.size() > kBatchDeps) return false;
                items.push_back(std::move(it));
            }
    }
    return true;
}

// Classes of the instances (see batch_kernel): instances dealt largest work
// first (node-updates of the run, ties by index) to the class with the least
// work so far (ties: the lowest class).
std::vector<int> assign_classes(const std::vector<Geometry>& geo, const int64_t* nsteps) {
    const int count = (int)geo.size();
    std::vector<int> order(count), cls(count, 0);
    std::vector<double> work(count);
    for (int k = 0; k < count; ++k) work[k] = (double)geo[k].nx * geo[k].ny * (double)nsteps[k];
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    double load[kBatchClasses] = {};
    for (int k : order) {
        const int c = (int)(std::min_element(load, load + kBatchClasses) - load);
        cls[k] = c;
        load[c] += work[k];
    }
    return cls;
}

// Slot tables of a launch (see BatchSlots): per class, in class order, the
// entries (instance, pass) of the class's instances in the order of the
// fraction of its run the instance has done after the pass, (p + 1) /
// passes[k], ties by instance (a merge of the instances' pass sequences; the
// fractions are compared exactly in integers); the first slot of each entry
// and of each class, and the first item of each instance.
struct Slots {
    std::vector<int32_t> entry;       // 2 per entry: instance, pass
    std::vector<int64_t> start;       // entries + 1
    std::vector<int32_t> first_item;  // instances + 1
    std::vector<int32_t> coarse;      // (slots >> kBatchCoarseBits) + 2
    std::vector<int64_t> cls;         // kBatchClasses + 1
};

void build_slots(const std::vector<ItemH>& items, const std::vector<int64_t>& passes, const std::vector<int>& cls_of,
                 Slots& sl) {
    const int count = (int)passes.size();
    sl.first_item.assign(count + 1, 0);
    for (const ItemH& it : items) sl.first_item[it.inst + 1] += 1;
    for (int k = 0; k < count; ++k) sl.first_item[k + 1] += sl.first_item[k];
    // merge: the next pass of instance k is due at fraction (next[k] + 1) / passes[k]
    std::vector<int64_t> next(count, 0);
    auto later = [&](int a, int b) {  // heap order: the smallest fraction on top
        const __int128 fa = (__int128)(next[a] + 1) * passes[b], fb = (__int128)(next[b] + 1) * passes[a];
        return fa != fb ? fa > fb : a > b;
    };
    sl.entry.clear();
    sl.start.assign(1, 0);
    sl.cls.assign(kBatchClasses + 1, 0);
    for (int c = 0; c < kBatchClasses; ++c) {
        sl.cls[c] = sl.start.back();
        std::vector<int> heap;
        for (int k = 0; k < count; ++k)
            if (cls_of[k] == c && passes[k] > 0 && sl.first_item[k + 1] > sl.first_item[k]) heap.push_back(k);
        std::make_heap(heap.begin(), heap.end(), later);
        while (!heap.empty()) {
            std::pop_heap(heap.begin(), heap.end(), later);
            const int k = heap.back();
            sl.entry.push_back(k);
            sl.entry.push_back((int32_t)next[k]);
            sl.start.push_back(sl.start.back() + (sl.first_item[k + 1] - sl.first_item[k]));
            if (++next[k] < passes[k])
                std::push_heap(heap.begin(), heap.end(), later);
            else
                heap.pop_back();
        }
    }
    sl.cls[kBatchClasses] = sl.start.back();
    // coarse index: the entry holding slot c << kBatchCoarseBits
    const int32_t n = (int32_t)(sl.entry.size() / 2);
    const int64_t total = sl.start.back();
    sl.coarse.assign((size_t)((total >> kBatchCoarseBits) + 2), n - 1);
    int32_t e = 0;
    for (size_t c = 0; c < sl.coarse.size(); ++c) {
        const int64_t T = (int64_t)c << kBatchCoarseBits;
        if (T >= total) break;
        while (sl.start[e + 1] <= T) ++e;
        sl.coarse[c] = e;
    }
}

}  // namespace

struct lbac_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<lbac_ctx*> inst;
    int strip_h = 40;   // >= kBatchMinStrip
    int max_wgs = 0;    // workgroups the device keeps resident at once: the grid of a launch
    int st = ST_PLAIN;  // storage of every instance
    double ticks_per_s = 1e8;
    double timeout_s = 20.0;
    int test_stall = 0;
    bool failed = false;  // a run timed out: the state is undefined until the instances are set again
    // schedule
    int items_h = -1;  // strip height the item list was built for
    std::vector<ItemH> items;
    int nitems = 0;
    int64_t nslots[2] = {0, 0};  // slots of the two launches of the current run
    BatchInst* d_inst = nullptr;
    BatchItem* d_items = nullptr;
    int32_t* d_entry[2] = {nullptr, nullptr};
    int64_t* d_start[2] = {nullptr, nullptr};
    int32_t* d_coarse[2] = {nullptr, nullptr};
    int64_t* d_cls = nullptr;     // first slot of each class, per launch (2 x (kBatchClasses + 1))
    BatchDev* d_dev = nullptr;    // the batch launches' argument block
    BatchDev* h_dev = nullptr;    // pinned
    int32_t* d_first = nullptr;   // first item of each instance
    int32_t* d_done = nullptr;
    BatchCtl* d_ctl = nullptr;
    BatchCtl* h_ctl = nullptr;    // pinned
    BatchInst* h_inst = nullptr;  // pinned
    int32_t* d_nent = nullptr;    // entries of the two launches (read by the kernels)
    int32_t* h_nent = nullptr;    // pinned
    int cap_items = 0;
    int64_t cap_ent[2] = {0, 0};
    int64_t cap_coarse[2] = {0, 0};
    hipGraphExec_t gexec = nullptr;
    int64_t g_slots[2] = {-1, -1};  // grids the captured graph was made for
    std::string err;
};

namespace {

int bfail(lbac_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    return code;
}

#define BHIP(b, call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return bfail(b, LBAC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void drop_graph(lbac_batch* b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->g_slots[0] = b->g_slots[1] = -1;
}

void free_tables(lbac_batch* b) {
    drop_graph(b);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_done);
    b->d_items = nullptr;
    b->d_done = nullptr;
    b->cap_items = 0;
    for (int L = 0; L < 2; ++L) {
        (void)hipFree(b->d_entry[L]);
        (void)hipFree(b->d_start[L]);
        (void)hipFree(b->d_coarse[L]);
        b->d_entry[L] = nullptr;
        b->d_start[L] = nullptr;
        b->d_coarse[L] = nullptr;
        b->cap_ent[L] = 0;
        b->cap_coarse[L] = 0;
    }
}

void release(lbac_batch* b) {
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_tables(b);
    (void)hipFree(b->d_inst);
    (void)hipFree(b->d_ctl);
    (void)hipFree(b->d_nent);
    (void)hipFree(b->d_first);
    (void)hipFree(b->d_cls);
    (void)hipFree(b->d_dev);
    if (b->h_dev) (void)hipHostFree(b->h_dev);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
    if (b->h_inst) (void)hipHostFree(b->h_inst);
    if (b->h_nent) (void)hipHostFree(b->h_nent);
    for (lbac_ctx* c : b->inst) {
        if (c) {
            c->in_batch = false;
            destroy(c);
        }
    }
    b->inst.clear();
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

// Device tables large enough for the items and for the entries and coarse
// index of each launch; a reallocation invalidates the captured graph (its
// kernel arguments).
int ensure_tables(lbac_batch* b, const int64_t nent[2], const int64_t ncoarse[2]) {
    if (b->cap_items < b->nitems) {
        drop_graph(b);
        (void)hipFree(b->d_items);
        (void)hipFree(b->d_done);
        b->d_items = nullptr;
        b->d_done = nullptr;
        b->cap_items = 0;
        const int ci = std::max(b->nitems, 1);
        BHIP(b, hipMalloc(&b->d_items, sizeof(BatchItem) * ci));
        BHIP(b, hipMalloc(&b->d_done, sizeof(int32_t) * ci));
        b->cap_items = ci;
    }
    for (int L = 0; L < 2; ++L)
        if (b->cap_ent[L] < nent[L] + 1) {
            drop_graph(b);
            (void)hipFree(b->d_entry[L]);
            (void)hipFree(b->d_start[L]);
            b->d_entry[L] = nullptr;
            b->d_start[L] = nullptr;
            b->cap_ent[L] = 0;
            const int64_t c = std::max<int64_t>(nent[L] + 1, 64);
            BHIP(b, hipMalloc(&b->d_entry[L], 2 * sizeof(int32_t) * c));
            BHIP(b, hipMalloc(&b->d_start[L], sizeof(int64_t) * c));
            b->cap_ent[L] = c;
        }
    for (int L = 0; L < 2; ++L)
        if (b->cap_coarse[L] < ncoarse[L]) {
            drop_graph(b);
            (void)hipFree(b->d_coarse[L]);
            b->d_coarse[L] = nullptr;
            b->cap_coarse[L] = 0;
            const int64_t c = std::max<int64_t>(ncoarse[L], 64);
            BHIP(b, hipMalloc(&b->d_coarse[L], sizeof(int32_t) * c));
            b->cap_coarse[L] = c;
        }
    return LBAC_OK;
}

// The batch kernel of storage st for launch L (L = 0: full passes; 1: one-step passes).
template <int ST>
void launch_batch_st(int L, dim3 grid, hipStream_t stream, const BatchDev* dev) {
    if (L == 0)
        hipLaunchKernelGGL((batch_kernel<MODEL_IMPROVED, kBatchS, ST>), grid, dim3(kBatchThreads), 0, stream, dev);
    else
        hipLaunchKernelGGL((batch_kernel<MODEL_IMPROVED, 1, ST>), grid, dim3(kBatchThreads), 0, stream, dev);
}
void launch_batch(int st, int L, dim3 grid, hipStream_t stream, const BatchDev* dev) {
    if (st == ST_F16) launch_batch_st<ST_F16>(L, grid, stream, dev);
    else if (st == ST_BF16) launch_batch_st<ST_BF16>(L, grid, stream, dev);
    else launch_batch_st<ST_PLAIN>(L, grid, stream, dev);
}
const void* batch_kernel_of(int st) {
    if (st == ST_F16) return (const void*)batch_kernel<MODEL_IMPROVED, kBatchS, ST_F16>;
    if (st == ST_BF16) return (const void*)batch_kernel<MODEL_IMPROVED, kBatchS, ST_BF16>;
    return (const void*)batch_kernel<MODEL_IMPROVED, kBatchS, ST_PLAIN>;
}

// Workgroups of a batch launch: as many as the device keeps resident, fewer
// if the launch has fewer slots (each workgroup takes slots until none is
// left; a grid beyond the resident count would only add workgroups that
// start when the slots are gone).
int64_t batch_grid(const lbac_batch* b, int L) { return std::min<int64_t>(b->nslots[L], b->max_wgs); }

// The run as one graph; it is captured again when a launch's grid changes.
int capture(lbac_batch* b) {
    if (b->gexec && b->g_slots[0] == batch_grid(b, 0) && b->g_slots[1] == batch_grid(b, 1)) return LBAC_OK;
    drop_graph(b);
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int count = (int)b->inst.size();
    const int nreset = std::max(b->cap_items, 1);
    // full passes, then (counters reset, error flag kept) the one-step passes
    hipLaunchKernelGGL(batch_reset_kernel, dim3((nreset + 255) / 256), dim3(256), 0, b->stream, b->d_done, nreset,
                       b->d_ctl, 0, 1);
    hipError_t e = hipGetLastError();
    auto launch_slots = [&](int L) {
        const int64_t g = batch_grid(b, L);
        if (g <= 0 || e != hipSuccess) return;
        launch_batch(b->st, L, dim3((unsigned)g), b->stream, b->d_dev);
        e = hipGetLastError();
    };
    launch_slots(0);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_reset_kernel, dim3((nreset + 255) / 256), dim3(256), 0, b->stream, b->d_done, nreset,
                           b->d_ctl, 1, 0);
        e = hipGetLastError();
    }
    launch_slots(1);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_advance_kernel, dim3((count + 255) / 256), dim3(256), 0, b->stream, b->d_inst, count,
                           b->d_ctl);
        e = hipGetLastError();
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, LBAC_EDEVICE, std::string("batch graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return bfail(b, LBAC_EDEVICE, std::string("batch graph instantiate: ") + hipGetErrorString(e));
    b->g_slots[0] = batch_grid(b, 0);
    b->g_slots[1] = batch_grid(b, 1);
    return LBAC_OK;
}

void mark_failed(lbac_batch* b) {
    b->failed = true;
    for (lbac_ctx* c : b->inst) c->failed = true;
}

// One run over all instances.  dry: steps read the current state and write
// the scratch buffer (state and time untouched).
int run(lbac_batch* b, const int64_t* nsteps, bool dry, float* ms_out) {
    if (b->failed) return bfail(b, LBAC_ESTATE, "a previous run timed out; the batch state is undefined");
    const int count = (int)b->inst.size();
    for (int k = 0; k < count; ++k)
        if (nsteps[k] < 0 || nsteps[k] > (int64_t)INT32_MAX) return bfail(b, LBAC_EINVAL, "step count out of range");
    if (b->strip_h < kBatchMinStrip) return bfail(b, LBAC_EINVAL, "strip height too small");
    if (b->items_h != b->strip_h) {
        std::vector<Geometry> geo(count);
        for (int k = 0; k < count; ++k) geo[k] = {b->inst[k]->p.nx, b->inst[k]->p.ny};
        if (!build_items(geo, b->strip_h, b->items)) return bfail(b, LBAC_EINVAL, "item dependency list too long");
        b->nitems = (int)b->items.size();
        b->items_h = b->strip_h;
    }
    std::vector<int64_t> pf(count), pr(count);
    for (int k = 0; k < count; ++k) {
        pf[k] = nsteps[k] / kBatchS;
        pr[k] = nsteps[k] % kBatchS;
    }
    std::vector<Geometry> geo(count);
    for (int k = 0; k < count; ++k) geo[k] = {b->inst[k]->p.nx, b->inst[k]->p.ny};
    const std::vector<int> cls_of = assign_classes(geo, nsteps);
    Slots sl[2];
    build_slots(b->items, pf, cls_of, sl[0]);
    build_slots(b->items, pr, cls_of, sl[1]);
    int64_t nent[2], ncoarse[2];
    for (int L = 0; L < 2; ++L) {
        nent[L] = (int64_t)sl[L].entry.size() / 2;
        ncoarse[L] = (int64_t)sl[L].coarse.size();
        b->nslots[L] = sl[L].start.back();
        if (nent[L] > INT32_MAX || b->nslots[L] > kBatchMaxSlots)
            return bfail(b, LBAC_EINVAL, "too many slots");
    }
    int rc = ensure_tables(b, nent, ncoarse);
    if (rc != LBAC_OK) return rc;
    std::vector<BatchItem> di(b->nitems);
    for (int i = 0; i < b->nitems; ++i) {
        const ItemH& it = b->items[i];
        BatchItem& d = di[i];
        d.inst = it.inst;
        d.x0 = it.x0;
        d.w = it.w;
        d.ys = it.ys;
        d.hh = it.hh;
        d.down = it.down;
        for (int m = 0; m < kBatchDeps; ++m) d.dep[m] = it.dep[m % it.dep.size()];
    }
    for (int k = 0; k < count; ++k) {
        lbac_ctx* c = b->inst[k];
        // even passes read pop[cur] and write the other buffer, odd passes the
        // reverse (a dry run reads pop[cur] on every pass)
        const StepArgs a = make_args(c, c->cur, 0);
        const StepArgs o = make_args(c, dry ? c->cur : c->cur ^ 1, 0);
        b->h_inst[2 * k].a = a;
        b->h_inst[2 * k + 1].a = o;
        b->h_inst[2 * k].nsteps = b->h_inst[2 * k + 1].nsteps = nsteps[k];
    }
    std::memset(b->h_ctl->ticket, 0, sizeof(b->h_ctl->ticket));
    b->h_ctl->timeout_ticks = (int64_t)(b->timeout_s * b->ticks_per_s);
    b->h_ctl->dry = dry ? 1 : 0;
    b->h_ctl->err = 0;
    b->h_ctl->test_stall = b->test_stall;
    b->h_nent[0] = (int32_t)nent[0];
    b->h_nent[1] = (int32_t)nent[1];
    b->h_dev->insts = b->d_inst;
    b->h_dev->items = b->d_items;
    for (int L = 0; L < 2; ++L)
        b->h_dev->slots[L] = BatchSlots{b->d_entry[L],  b->d_start[L], b->d_first, b->d_nent + L, b->d_coarse[L],
                                        b->d_cls + L * (kBatchClasses + 1)};
    b->h_dev->done = b->d_done;
    b->h_dev->ctl = b->d_ctl;
    BHIP(b, hipMemcpyAsync(b->d_dev, b->h_dev, sizeof(BatchDev), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_inst, b->h_inst, sizeof(BatchInst) * 2 * count, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_ctl, b->h_ctl, sizeof(BatchCtl), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_nent, b->h_nent, 2 * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_first, sl[0].first_item.data(), sizeof(int32_t) * (count + 1), hipMemcpyHostToDevice,
                           b->stream));
    BHIP(b, hipMemcpyAsync(b->d_items, di.data(), sizeof(BatchItem) * b->nitems, hipMemcpyHostToDevice, b->stream));
    for (int L = 0; L < 2; ++L) {
        if (nent[L] > 0)
            BHIP(b, hipMemcpyAsync(b->d_entry[L], sl[L].entry.data(), sizeof(int32_t) * sl[L].entry.size(),
                                   hipMemcpyHostToDevice, b->stream));
        BHIP(b, hipMemcpyAsync(b->d_start[L], sl[L].start.data(), sizeof(int64_t) * sl[L].start.size(),
                               hipMemcpyHostToDevice, b->stream));
        BHIP(b, hipMemcpyAsync(b->d_coarse[L], sl[L].coarse.data(), sizeof(int32_t) * sl[L].coarse.size(),
                               hipMemcpyHostToDevice, b->stream));
        BHIP(b, hipMemcpyAsync(b->d_cls + L * (kBatchClasses + 1), sl[L].cls.data(),
                               sizeof(int64_t) * (kBatchClasses + 1), hipMemcpyHostToDevice, b->stream));
    }
    rc = capture(b);
    if (rc != LBAC_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms_out) {
        BHIP(b, hipEventCreate(&e0));
        BHIP(b, hipEventCreate(&e1));
        BHIP(b, hipEventRecord(e0, b->stream));
    }
    BHIP(b, hipGraphLaunch(b->gexec, b->stream));
    if (ms_out) BHIP(b, hipEventRecord(e1, b->stream));
    BHIP(b, hipMemcpyAsync(b->h_ctl, b->d_ctl, sizeof(BatchCtl), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));  // host vectors above must outlive the copies
    if (ms_out) {
        BHIP(b, hipEventElapsedTime(ms_out, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    if (b->h_ctl->err) {
        // passes that did run have overwritten both buffers of some instances
        if (!dry) mark_failed(b);
        return bfail(b, LBAC_EDEVICE, "batch schedule stalled: a dependency wait timed out");
    }
    if (!dry)
        for (int k = 0; k < count; ++k) {
            b->inst[k]->cur ^= (int)(batch_passes(nsteps[k]) & 1);  // one buffer swap per pass
            b->inst[k]->t += nsteps[k];
        }
    return LBAC_OK;
}

}  // namespace

extern "C" {

int lbac_batch_init(const lbac_params* params, const double* const* phi0, int32_t count, lbac_batch** out) {
    if (!out) return LBAC_EINVAL;
    *out = nullptr;
    if (!params || !phi0 || count < 1) return LBAC_EINVAL;
    const int prec = params[0].precision;
    if (prec != LBAC_F32 && prec != LBAC_F32_F16STORE && prec != LBAC_F32_BF16STORE) return LBAC_EINVAL;
    for (int k = 0; k < count; ++k) {
        if (params[k].precision != prec || params[k].model != LBAC_MODEL_IMPROVED) return LBAC_EINVAL;
        if (!phi0[k]) return LBAC_EINVAL;
        // nine FP32 planes of at least nx * ny values each must stay below
        // 2^31 bytes (checked exactly, padding included, once allocated)
        if ((int64_t)params[k].nx * params[k].ny * 9 * (int64_t)sizeof(float) >= (int64_t)0x7FFFFFFF) return LBAC_EINVAL;
    }
    lbac_batch* b = new (std::nothrow) lbac_batch();
    if (!b) return LBAC_ENOMEM;
    auto bail = [&](int code) {
        release(b);
        delete b;
        return code;
    };
    if (hipGetDevice(&b->device) != hipSuccess) return bail(LBAC_EDEVICE);
    if (params[0].stream) {
        b->stream = (hipStream_t)params[0].stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return bail(LBAC_EDEVICE);
        b->own_stream = true;
    }
    b->inst.assign(count, nullptr);
    for (int k = 0; k < count; ++k) {
        lbac_params p = params[k];
        p.stream = b->stream;
        lbac_ctx* c = nullptr;
        const int rc = create(&p, phi0[k], false, &c);
        if (rc != LBAC_OK) return bail(rc);
        c->in_batch = true;
        b->inst[k] = c;
        // the batch kernel addresses the planes of a buffer through one
        // buffer resource with 32-bit offsets below 2^31
        if (c->plane_stride * c->nplanes * (int64_t)c->elem_bytes >= (int64_t)0x7FFFFFFF) return bail(LBAC_EINVAL);
    }
    b->st = b->inst[0]->storage;
    int per_cu = 0, cus = 0, khz = 0;
    // the default grid: as many workgroups as the device keeps resident (the
    // schedule itself does not depend on residency); the multi-step launch
    // has the lower occupancy and sets it for both
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel_of(b->st), kBatchThreads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
        return bail(LBAC_EDEVICE);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) == hipSuccess && khz > 0)
        b->ticks_per_s = 1000.0 * khz;
    b->max_wgs = std::max(1, per_cu * cus);
    if (hipMalloc(&b->d_inst, sizeof(BatchInst) * 2 * count) != hipSuccess ||
        hipMalloc(&b->d_ctl, sizeof(BatchCtl)) != hipSuccess || hipMalloc(&b->d_nent, 64) != hipSuccess ||
        hipMalloc(&b->d_first, sizeof(int32_t) * (count + 1)) != hipSuccess ||
        hipMalloc(&b->d_cls, sizeof(int64_t) * 2 * (kBatchClasses + 1)) != hipSuccess ||
        hipMalloc(&b->d_dev, sizeof(BatchDev)) != hipSuccess ||
        hipHostMalloc((void**)&b->h_dev, sizeof(BatchDev), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_ctl, sizeof(BatchCtl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_nent, 2 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_inst, sizeof(BatchInst) * 2 * count, hipHostMallocDefault) != hipSuccess)
        return bail(LBAC_ENOMEM);
    std::memset(b->h_ctl, 0, sizeof(BatchCtl));
    *out = b;
    return LBAC_OK;
}

int lbac_batch_free(lbac_batch* b) {
    if (!b) return LBAC_OK;
    DeviceGuard g(b->device);
    release(b);
    delete b;
    return LBAC_OK;
}

int lbac_batch_run(lbac_batch* b, const int64_t* nsteps) {
    if (!b || !nsteps) return LBAC_EINVAL;
    DeviceGuard g(b->device);
    return run(b, nsteps, false, nullptr);
}

int lbac_batch_instance(lbac_batch* b, int32_t k, lbac_ctx** ctx) {
    if (!b || !ctx || k < 0 || k >= (int)b->inst.size()) return LBAC_EINVAL;
    *ctx = b->inst[k];
    return LBAC_OK;
}

int lbac_batch_phi(lbac_batch* b, int32_t k, double* out) {
    if (!b || !out || k < 0 || k >= (int)b->inst.size()) return LBAC_EINVAL;
    return lbac_phi(b->inst[k], out);
}

int lbac_batch_mass(lbac_batch* b, double* per_instance) {
    if (!b || !per_instance) return LBAC_EINVAL;
    for (size_t k = 0; k < b->inst.size(); ++k) {
        const int rc = lbac_mass(b->inst[k], per_instance + k);
        if (rc != LBAC_OK) return rc;
    }
    return LBAC_OK;
}

int lbac_batch_count(lbac_batch* b, int32_t* count) {
    if (!b || !count) return LBAC_EINVAL;
    *count = (int32_t)b->inst.size();
    return LBAC_OK;
}

int lbac_batch_set_shape(lbac_batch* b, int32_t strip_h) {
    if (!b) return LBAC_EINVAL;
    if (strip_h < kBatchMinStrip) return bfail(b, LBAC_EINVAL, "strip height must be >= 8");
    b->strip_h = strip_h;
    return LBAC_OK;
}

int lbac_batch_get_shape(lbac_batch* b, int32_t* strip_h, int32_t* resident_workgroups) {
    if (!b) return LBAC_EINVAL;
    if (strip_h) *strip_h = b->strip_h;
    if (resident_workgroups) *resident_workgroups = b->max_wgs;
    return LBAC_OK;
}

int lbac_batch_autotune(lbac_batch* b, const int64_t* nsteps, double* ms) {
    if (!b || !nsteps) return LBAC_EINVAL;
    if (b->failed) return bfail(b, LBAC_ESTATE, "a previous run timed out; the batch state is undefined");
    DeviceGuard g(b->device);
    const int count = (int)b->inst.size();
    std::vector<int64_t> ns(nsteps, nsteps + count);
    const int keep_h = b->strip_h;
    const int hs[13] = {16, 24, 32, 40, 48, 56, 64, 72, 80, 88, 96, 128, 192};
    float best = 1e30f;
    int best_h = keep_h;
    for (int h : hs) {
        b->strip_h = h;
        float t = 0.f;
        const int rc = run(b, ns.data(), true, &t);
        if (rc != LBAC_OK) {
            b->strip_h = keep_h;
            return rc;
        }
        if (t < best) {
            best = t;
            best_h = h;
        }
    }
    b->strip_h = best_h;
    if (ms) *ms = best;
    return LBAC_OK;
}

int lbac_batch_set_timeout(lbac_batch* b, double seconds, int32_t test_stall) {
    if (!b || !(seconds > 0.0) || seconds > 3600.0) return LBAC_EINVAL;
    b->timeout_s = seconds;
    b->test_stall = test_stall ? 1 : 0;
    return LBAC_OK;
}

const char* lbac_batch_last_error(lbac_batch* b) { return b ? b->err.c_str() : "no batch"; }

int lbac_batch_schedule_check(const int32_t* nx, const int32_t* ny, const int64_t* nsteps, int32_t count,
                              int32_t strip_h, int32_t workers, int32_t protocol, uint64_t seed, int32_t* verdict,
                              int64_t* slots_run) {
    if (!nx || !ny || !nsteps || !verdict || count < 1 || strip_h < kBatchMinStrip || workers < 1 || protocol < 0 ||
        protocol > 2)
        return LBAC_EINVAL;
    std::vector<Geometry> geo(count);
    std::vector<int64_t> pf(count), pr(count);
    for (int k = 0; k < count; ++k) {
        if (nx[k] < 1 || ny[k] < 1 || nsteps[k] < 0 || nsteps[k] > (int64_t)INT32_MAX) return LBAC_EINVAL;
        geo[k] = {nx[k], ny[k]};
        pf[k] = nsteps[k] / kBatchS;
        pr[k] = nsteps[k] % kBatchS;
    }
    std::vector<ItemH> items;
    if (!build_items(geo, strip_h, items)) return LBAC_EINVAL;
    const int n = (int)items.size();
    const std::vector<int> cls_of = assign_classes(geo, nsteps);
    // The state, per buffer and item tile: the pass (run-wide index) that last
    // wrote it; the initial state is in buffer 0 (pass -1), buffer 1 holds
    // nothing valid.  Pass gp reads buffer gp & 1 and writes the other one.
    std::vector<int64_t> ver[2] = {std::vector<int64_t>(n, -1), std::vector<int64_t>(n, -3)};
    std::mt19937_64 rng(seed);
    *verdict = 0;
    if (slots_run) *slots_run = 0;
    int64_t ran = 0;
    struct Slot {
        int32_t p, id;
        int64_t gp;
        bool started;
    };
    for (int L = 0; L < 2 && *verdict == 0; ++L) {
        const std::vector<int64_t>& passes = L == 0 ? pf : pr;
        Slots sl;
        build_slots(items, passes, cls_of, sl);
        const int32_t nent = (int32_t)(sl.entry.size() / 2);
        const int64_t total = sl.start.back();
        const BatchSlots tab{sl.entry.data(), sl.start.data(), sl.first_item.data(), &nent, sl.coarse.data(),
                             sl.cls.data()};
        // every instance's entries lie in its class's block of slots
        for (int64_t e = 0; e < nent; ++e) {
            const int c = cls_of[sl.entry[2 * e]];
            if (sl.start[e] < sl.cls[c] || sl.start[e + 1] > sl.cls[c + 1]) {
                *verdict = 3;
                return LBAC_OK;
            }
        }
        // the kernel's slot lookup (coarse index, then a search) against the
        // entry list walked slot by slot
        for (int64_t T = 0, e = 0; T < total && protocol != 2; ++T) {
            while (sl.start[e + 1] <= T) ++e;
            int32_t p = -1;
            const int32_t id = batch_slot_item(tab, T, nent, p);
            const int k = sl.entry[2 * e], pe = sl.entry[2 * e + 1];
            const int want = sl.first_item[k] + (int)(T - sl.start[e]);
            if (p != pe || id != want || items[want].inst != k) {
                *verdict = 3;
                return LBAC_OK;
            }
        }
        int32_t npass = 0;
        for (int64_t v : passes) npass = std::max<int32_t>(npass, (int32_t)v);
        // protocol 2: fixed item lists of 2 * workers workgroups (items dealt
        // longest-first to the least loaded list, each list walked pass by
        // pass), of which `workers` run at once; a list's workgroup starts
        // when a running one has finished its whole list
        const int lists = 2 * workers;
        std::vector<std::vector<int32_t>> list(lists);
        if (protocol == 2) {
            std::vector<int32_t> order(n);
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return passes[items[a].inst] > passes[items[b].inst]; });
            std::vector<double> load(lists, 0.0);
            for (int32_t id : order) {
                const int m = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                list[m].push_back(id);
                load[m] += (double)items[id].w * items[id].hh * std::max<int64_t>(passes[items[id].inst], 1);
            }
            for (auto& l : list) std::sort(l.begin(), l.end());
        }
        std::vector<int32_t> done(n, -1);
        std::vector<Slot> slot(workers);
        std::vector<bool> busy(workers, false);
        // protocol 2 state of a worker: its list, pass and position in the list
        std::vector<int> wl(workers, -1), wpos(workers, 0);
        std::vector<int32_t> wpass(workers, 0);
        int next_list = 0;
        int64_t finished = 0, taken = 0;
        std::vector<int64_t> tk(kBatchClasses, 0);  // the classes' counters
        // the next (pass, item) of worker w under protocol 2, or false at the
        // end of its list (the worker then takes the next list, if any)
        auto static_next = [&](int w, Slot& s) -> bool {
            for (;;) {
                if (wl[w] < 0) {
                    if (next_list >= lists) return false;
                    wl[w] = next_list++;
                    wpos[w] = 0;
                    wpass[w] = 0;
                }
                const std::vector<int32_t>& l = list[wl[w]];
                while (wpass[w] < npass) {
                    while (wpos[w] < (int)l.size() && passes[items[l[wpos[w]]].inst] <= wpass[w]) ++wpos[w];
                    if (wpos[w] < (int)l.size()) {
                        s.id = l[wpos[w]++];
                        s.p = wpass[w];
                        return true;
                    }
                    ++wpass[w];
                    wpos[w] = 0;
                }
                wl[w] = -1;
            }
        };
        // Each worker is a resident workgroup running the kernel's loop: take
        // a slot (the next of its class, else of another class, as the kernel
        // does), wait until every dependency has published p - 1, work
        // (reading its read region and writing its tile anywhere in that
        // interval), publish.  The interleaving of the workers' actions is
        // random; a state in which no worker can act before every slot has
        // finished is a deadlock.  A worker that starts working checks that
        // every tile it reads holds the previous pass and that no working
        // worker writes a tile it reads or reads the tile it writes.
        while (finished < total && *verdict == 0) {
            std::vector<int> can;
            for (int w = 0; w < workers; ++w) {
                if (!busy[w]) {
                    if (protocol == 2 ? (wl[w] >= 0 || next_list < lists) : taken < total) can.push_back(w);
                } else if (slot[w].started) {
                    can.push_back(w);
                } else {
                    bool ready = true;
                    if (slot[w].p > 0 && protocol != 1)
                        for (int32_t d : items[slot[w].id].dep) ready = ready && done[d] >= slot[w].p - 1;
                    if (ready) can.push_back(w);
                }
            }
            if (can.empty()) {
                *verdict = 1;
                break;
            }
            const int w = can[rng() % can.size()];
            Slot& s = slot[w];
            if (!busy[w]) {
                if (protocol == 2) {
                    if (!static_next(w, s)) continue;
                } else {
                    // worker w is workgroup w of the grid: class w mod kBatchClasses
                    const int64_t T = batch_take(sl.cls.data(), w % kBatchClasses,
                                                 [&](int c, int64_t nn) { return tk[c] < nn ? tk[c]++ : nn; });
                    s.id = batch_slot_item(tab, T, nent, s.p);
                    ++taken;
                }
                s.gp = (L == 0 ? 0 : pf[items[s.id].inst]) + s.p;
                s.started = false;
                busy[w] = true;
            } else if (!s.started) {
                const int rb = (int)(s.gp & 1), wb = rb ^ 1;
                for (int32_t d : items[s.id].dep)
                    if (ver[rb][d] != s.gp - 1) *verdict = 2;
                for (int v = 0; v < workers; ++v) {
                    if (v == w || !busy[v] || !slot[v].started) continue;
                    const Slot& o = slot[v];
                    const int orb = (int)(o.gp & 1), owb = orb ^ 1;
                    for (int32_t d : items[s.id].dep)
                        if (owb == rb && o.id == d) *verdict = 2;  // o writes a tile s reads
                    for (int32_t d : items[o.id].dep)
                        if (wb == orb && s.id == d) *verdict = 2;  // s writes a tile o reads
                    if (wb == owb && s.id == o.id) *verdict = 2;  // both write one tile
                }
                s.started = true;
            } else {
                ver[(s.gp & 1) ^ 1][s.id] = s.gp;
                done[s.id] = s.p;
                busy[w] = false;
                ++finished;
                ++ran;
            }
        }
    }
    if (slots_run) *slots_run = ran;
    return LBAC_OK;
}

}  // extern "C"
