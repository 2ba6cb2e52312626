// Internal declarations shared by the translation units of the library
// (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "lbac.h"
#include "lbac_kernels.hpp"

namespace lbac_host {

constexpr int kPlanePadBytes = 4096 + 256;  // staggers plane bases across HBM channels
constexpr int kXcds = 8;                    // MI355X: workgroups go round-robin over 8 XCDs
constexpr int kClosureBlocks = 512;         // blocks of the closure correction pass (grid-stride over the band list)
constexpr uint64_t kStateMagic = 0x4c42414353543031ull;  // "LBACST01"

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace lbac_host

struct lbac_ctx {
    lbac_params p{};
    lbac_allocator alloc{};
    bool has_alloc = false;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int storage = lbac::ST_PLAIN;
    int elem_bytes = 8;
    int nplanes = 9;
    int32_t pitch = 0;
    int64_t plane_stride = 0;
    void* pop[2] = {nullptr, nullptr};
    float* phis[2] = {nullptr, nullptr};
    double* vtab = nullptr;
    float* vtabf = nullptr;  // vtab rounded to FP32
    int64_t* t_dev = nullptr;
    void* rows = nullptr;    // per-row partial sums (working precision)
    double* red5 = nullptr;
    double* dtmp = nullptr;  // ny*nx doubles (phi0 upload, phi output, reference field)
    double* host5 = nullptr; // pinned
    int cur = 0;
    int64_t t = 0;
    int variant = LBAC_KERNEL_BLOCK;
    int bx = 256, strip_h = 64;
    int graph_chunk = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gexec_chunk[2] = {0, 0};
    int gexec_flips[2] = {0, 0};  // parity of the launches in each graph
    bool in_batch = false;   // owned by a batch: lbac_free refuses it
    bool failed = false;     // its batch's run timed out: the state is undefined
    // learned closure (FP32 plain storage only)
    bool closure = false;
    float cl_theta = 0.f;
    float* cl_param = nullptr;   // FP32 parameters as given
    uint16_t* cl_w = nullptr;    // packed BF16 weights
    float* cl_b = nullptr;       // padded biases
    uint64_t* cl_mask = nullptr;  // band masks written by the step kernel
    int32_t* cl_list = nullptr;   // band node list (up to nx * ny entries)
    uint32_t* cl_count = nullptr; // entries in cl_list
    int32_t cl_words = 0;         // mask words per row
    std::string err;
};

namespace lbac_host {

int fail(lbac_ctx* h, int code, const std::string& msg);
void* dev_alloc(lbac_ctx* h, size_t bytes);
void dev_free(lbac_ctx* h, void* ptr);
lbac::StepArgs make_args(const lbac_ctx* h, int src, int32_t k);
int create(const lbac_params* p, const double* phi0, bool phi0_on_device, lbac_ctx** out);
void destroy(lbac_ctx* h);

}  // namespace lbac_host

#define HIPCHK(h, call)                                                                                      \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return ::lbac_host::fail(h, LBAC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)
