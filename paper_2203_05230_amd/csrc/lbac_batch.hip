// Batched form: many independent lattices advanced by one persistent kernel
// launch, replayed from a captured HIP graph (see batch_kernel in
// lbac_kernels.hpp for the dependency protocol).
//
// Host side: the work list of (instance, 128-column block, strip) items, a
// longest-processing-time-first assignment of items to workgroups (work =
// nodes x steps), occupancy-limited workgroup count so that every workgroup
// is resident, graph capture of reset -> persistent kernel -> time advance,
// and an autotuner over the strip height and the workgroup count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "lbac_batch_kernels.hpp"
#include "lbac_internal.hpp"

using namespace lbac;
using namespace lbac_host;

// rows per strip at least: a pass reads kBatchGrow rows beyond its strip on
// each side, and the neighbour lists hold at most four strips per axis
constexpr int kBatchMinStrip = kBatchGrow + 2;

struct lbac_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<lbac_ctx*> inst;
    int strip_h = 32;  // >= kBatchMinStrip
    int wgs = 0;        // 0: occupancy limit
    int max_wgs = 0;    // occupancy limit (resident workgroups)
    double ticks_per_s = 1e8;
    double timeout_s = 20.0;
    int test_stall = 0;
    // schedule
    int nitems = 0, nwg = 0;
    std::vector<BatchItem> items;
    std::vector<int64_t> item_nodes;
    BatchInst* d_inst = nullptr;
    BatchItem* d_items = nullptr;
    int32_t* d_wg_off = nullptr;
    int32_t* d_wg_items = nullptr;
    int32_t* d_done = nullptr;
    BatchCtl* d_ctl = nullptr;
    BatchCtl* h_ctl = nullptr;  // pinned
    BatchInst* h_inst = nullptr;  // pinned
    int cap_items = 0, cap_wg = 0;
    hipGraphExec_t gexec = nullptr;
    int g_nwg = -1, g_nitems = -1;
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
    b->g_nwg = b->g_nitems = -1;
}

void free_tables(lbac_batch* b) {
    drop_graph(b);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_wg_off);
    (void)hipFree(b->d_wg_items);
    (void)hipFree(b->d_done);
    b->d_items = nullptr;
    b->d_wg_off = b->d_wg_items = b->d_done = nullptr;
    b->cap_items = b->cap_wg = 0;
}

void release(lbac_batch* b) {
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    free_tables(b);
    (void)hipFree(b->d_inst);
    (void)hipFree(b->d_ctl);
    if (b->h_ctl) (void)hipHostFree(b->h_ctl);
    if (b->h_inst) (void)hipHostFree(b->h_inst);
    for (lbac_ctx* c : b->inst) {
        if (c) {
            c->in_batch = false;
            destroy(c);
        }
    }
    b->inst.clear();
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

// Work items and their neighbour lists for the current strip height.  The
// neighbours of an item are the items whose tiles overlap its read region,
// columns x0-G .. x0+w-1+G and rows ys-G .. ys+hh-1+G (G = kBatchGrow,
// periodic).
void build_items(lbac_batch* b) {
    constexpr int W = kBatchTile, G = kBatchGrow;
    b->items.clear();
    b->item_nodes.clear();
    for (int k = 0; k < (int)b->inst.size(); ++k) {
        const lbac_ctx* c = b->inst[k];
        const int nx = c->p.nx, ny = c->p.ny;
        const int sh = std::min(b->strip_h, ny);
        const int nbx = (nx + W - 1) / W, nby = (ny + sh - 1) / sh;
        const int base = (int)b->items.size();
        for (int j = 0; j < nby; ++j)
            for (int i = 0; i < nbx; ++i) {
                const int w = std::min(W, nx - i * W), h = std::min(sh, ny - j * sh);
                std::vector<int> tx, ty;
                for (int cx = i * W - G; cx <= i * W + w - 1 + G; ++cx) tx.push_back(((cx % nx) + nx) % nx / W);
                for (int ry = j * sh - G; ry <= j * sh + h - 1 + G; ++ry) ty.push_back(((ry % ny) + ny) % ny / sh);
                std::sort(tx.begin(), tx.end());
                tx.erase(std::unique(tx.begin(), tx.end()), tx.end());
                std::sort(ty.begin(), ty.end());
                ty.erase(std::unique(ty.begin(), ty.end()), ty.end());
                std::vector<int32_t> nb;
                for (int jj : ty)
                    for (int ii : tx)
                        if (ii != i || jj != j) nb.push_back(base + jj * nbx + ii);
                BatchItem it{};
                it.inst = k;
                it.bxi = i;
                it.syi = j;
                it.down = j & 1;
                // at most 4 tiles per axis (strips are at least G + 2 rows high and
                // tiles 128 columns wide; only the last tile or strip can be narrower)
                for (int m = 0; m < 16; ++m) it.nbr[m] = nb.empty() ? base + j * nbx + i : nb[m % nb.size()];
                b->items.push_back(it);
                b->item_nodes.push_back((int64_t)w * h);
            }
    }
    b->nitems = (int)b->items.size();
}

// Longest processing time first: items by work (nodes x steps), each to the
// least loaded workgroup; each workgroup then walks its items in id order.
void lpt(const lbac_batch* b, const int64_t* nsteps, int nwg, std::vector<int32_t>& off, std::vector<int32_t>& list) {
    std::vector<int> order(b->nitems);
    std::iota(order.begin(), order.end(), 0);
    auto work = [&](int i) { return (double)b->item_nodes[i] * (double)std::max<int64_t>(nsteps[b->items[i].inst], 1); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    using E = std::pair<double, int>;
    std::priority_queue<E, std::vector<E>, std::greater<E>> pq;
    for (int w = 0; w < nwg; ++w) pq.push({0.0, w});
    std::vector<std::vector<int32_t>> per(nwg);
    for (int i : order) {
        E e = pq.top();
        pq.pop();
        per[e.second].push_back(i);
        e.first += work(i);
        pq.push(e);
    }
    off.assign(nwg + 1, 0);
    list.clear();
    for (int w = 0; w < nwg; ++w) {
        std::sort(per[w].begin(), per[w].end());
        off[w] = (int32_t)list.size();
        list.insert(list.end(), per[w].begin(), per[w].end());
    }
    off[nwg] = (int32_t)list.size();
}

int ensure_tables(lbac_batch* b, int nwg) {
    if (b->cap_items < b->nitems || b->cap_wg < nwg) {
        free_tables(b);
        const int ci = std::max(b->nitems, 1), cw = std::max(nwg, 1);
        BHIP(b, hipMalloc(&b->d_items, sizeof(BatchItem) * ci));
        BHIP(b, hipMalloc(&b->d_wg_items, sizeof(int32_t) * ci));
        BHIP(b, hipMalloc(&b->d_done, sizeof(int32_t) * ci));
        BHIP(b, hipMalloc(&b->d_wg_off, sizeof(int32_t) * (cw + 1)));
        b->cap_items = ci;
        b->cap_wg = cw;
    }
    return LBAC_OK;
}

int capture(lbac_batch* b) {
    if (b->gexec && b->g_nwg == b->nwg && b->g_nitems == b->nitems) return LBAC_OK;
    drop_graph(b);
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int count = (int)b->inst.size();
    // full passes, then (counters reset, error flag kept) the one-step passes
    hipLaunchKernelGGL(batch_reset_kernel, dim3((b->nitems + 255) / 256), dim3(256), 0, b->stream, b->d_done,
                       b->nitems, b->d_ctl, 1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL((batch_kernel<MODEL_IMPROVED, kBatchS>), dim3(b->nwg), dim3(block_threads<kBatchTile>()), 0,
                           b->stream, b->d_inst, b->d_items, b->d_wg_off, b->d_wg_items, b->d_done, b->d_ctl);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(batch_reset_kernel, dim3((b->nitems + 255) / 256), dim3(256), 0, b->stream, b->d_done,
                           b->nitems, b->d_ctl, 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL((batch_kernel<MODEL_IMPROVED, 1>), dim3(b->nwg), dim3(block_threads<kBatchTile>()), 0,
                           b->stream, b->d_inst, b->d_items, b->d_wg_off, b->d_wg_items, b->d_done, b->d_ctl);
        e = hipGetLastError();
    }
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
    b->g_nwg = b->nwg;
    b->g_nitems = b->nitems;
    return LBAC_OK;
}

// One persistent launch over all instances.  dry: steps read the current
// state and write the scratch buffer (state and time untouched).
int run(lbac_batch* b, const int64_t* nsteps, bool dry, float* ms_out) {
    const int count = (int)b->inst.size();
    int64_t max_full = 0, max_rest = 0;
    for (int k = 0; k < count; ++k) {
        if (nsteps[k] < 0 || nsteps[k] > (int64_t)INT32_MAX) return bfail(b, LBAC_EINVAL, "step count out of range");
        max_full = std::max(max_full, nsteps[k] / kBatchS);
        max_rest = std::max(max_rest, nsteps[k] % kBatchS);
    }
    if (b->strip_h < kBatchMinStrip) return bfail(b, LBAC_EINVAL, "strip height too small");
    build_items(b);
    const int nwg = std::max(1, std::min(b->wgs > 0 ? std::min(b->wgs, b->max_wgs) : b->max_wgs, b->nitems));
    b->nwg = nwg;
    int rc = ensure_tables(b, nwg);
    if (rc != LBAC_OK) return rc;
    std::vector<int32_t> off, list;
    lpt(b, nsteps, nwg, off, list);
    for (int k = 0; k < count; ++k) {
        lbac_ctx* c = b->inst[k];
        // even passes read pop[cur] and write the other buffer, odd passes the
        // reverse (a dry run reads pop[cur] on every pass)
        StepArgs a = make_args(c, c->cur, 0);
        a.strip_h = std::min(b->strip_h, c->p.ny);
        StepArgs o = make_args(c, dry ? c->cur : c->cur ^ 1, 0);
        o.strip_h = a.strip_h;
        b->h_inst[2 * k].a = a;
        b->h_inst[2 * k + 1].a = o;
        b->h_inst[2 * k].nsteps = b->h_inst[2 * k + 1].nsteps = nsteps[k];
    }
    b->h_ctl->max_full = max_full;
    b->h_ctl->max_rest = max_rest;
    b->h_ctl->timeout_ticks = (int64_t)(b->timeout_s * b->ticks_per_s);
    b->h_ctl->dry = dry ? 1 : 0;
    b->h_ctl->err = 0;
    b->h_ctl->test_stall = b->test_stall;
    BHIP(b, hipMemcpyAsync(b->d_inst, b->h_inst, sizeof(BatchInst) * 2 * count, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_ctl, b->h_ctl, sizeof(BatchCtl), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_items, b->items.data(), sizeof(BatchItem) * b->nitems, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_wg_items, list.data(), sizeof(int32_t) * list.size(), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_wg_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, b->stream));
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
    if (b->h_ctl->err) return bfail(b, LBAC_EDEVICE, "batch schedule stalled: a dependency wait timed out");
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
    for (int k = 0; k < count; ++k) {
        if (params[k].precision != LBAC_F32 || params[k].model != LBAC_MODEL_IMPROVED) return LBAC_EINVAL;
        if (!phi0[k]) return LBAC_EINVAL;
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
    }
    int per_cu = 0, cus = 0, khz = 0;
    // the multi-step launch has the lower occupancy; both launches use its grid
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<MODEL_IMPROVED, kBatchS>,
                                                     block_threads<kBatchTile>(), 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
        return bail(LBAC_EDEVICE);
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) == hipSuccess && khz > 0)
        b->ticks_per_s = 1000.0 * khz;
    b->max_wgs = std::max(1, per_cu * cus);
    if (hipMalloc(&b->d_inst, sizeof(BatchInst) * 2 * count) != hipSuccess ||
        hipMalloc(&b->d_ctl, sizeof(BatchCtl)) != hipSuccess ||
        hipHostMalloc((void**)&b->h_ctl, sizeof(BatchCtl), hipHostMallocDefault) != hipSuccess ||
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

int lbac_batch_count(lbac_batch* b, int32_t* count) {
    if (!b || !count) return LBAC_EINVAL;
    *count = (int32_t)b->inst.size();
    return LBAC_OK;
}

int lbac_batch_set_shape(lbac_batch* b, int32_t strip_h, int32_t workgroups) {
    if (!b) return LBAC_EINVAL;
    if (strip_h < kBatchMinStrip) return bfail(b, LBAC_EINVAL, "strip height must be >= 8");
    if (workgroups < 0) return bfail(b, LBAC_EINVAL, "workgroups must be >= 0 (0: occupancy limit)");
    b->strip_h = strip_h;
    b->wgs = workgroups;
    return LBAC_OK;
}

int lbac_batch_get_shape(lbac_batch* b, int32_t* strip_h, int32_t* workgroups, int32_t* max_workgroups) {
    if (!b) return LBAC_EINVAL;
    if (strip_h) *strip_h = b->strip_h;
    if (workgroups) *workgroups = b->wgs > 0 ? std::min(b->wgs, b->max_wgs) : b->max_wgs;
    if (max_workgroups) *max_workgroups = b->max_wgs;
    return LBAC_OK;
}

int lbac_batch_autotune(lbac_batch* b, int32_t steps, double* ms) {
    if (!b || steps < 1) return LBAC_EINVAL;
    DeviceGuard g(b->device);
    const int count = (int)b->inst.size();
    std::vector<int64_t> ns(count, steps);
    const int keep_h = b->strip_h, keep_w = b->wgs;
    const int hs[7] = {16, 32, 64, 96, 128, 192, 256};
    const int fr[3] = {4, 3, 2};  // workgroups = max * fr / 4
    float best = 1e30f;
    int best_h = keep_h, best_w = keep_w;
    for (int h : hs)
        for (int f : fr) {
            b->strip_h = h;
            b->wgs = std::max(1, b->max_wgs * f / 4);
            float t = 0.f;
            const int rc = run(b, ns.data(), true, &t);
            if (rc != LBAC_OK) {
                b->strip_h = keep_h;
                b->wgs = keep_w;
                return rc;
            }
            if (t < best) {
                best = t;
                best_h = h;
                best_w = b->wgs;
            }
        }
    b->strip_h = best_h;
    b->wgs = best_w;
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

}  // extern "C"
