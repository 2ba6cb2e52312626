// Training data for the learned closure, computed on the GPU from a fine
// field (for example lbac_phi_device of a run r times finer):
//   phi_c  = mean of each r x r block of phi_f                      (restriction)
//   target = mean_block(r S_f n_f) - S_c(phi_c) n_c(phi_c)          (flux the fine field
//            carries, per coarse lattice unit, minus the flux the coarse scheme computes)
// with S n the sharpening flux of Eq. (6), (7), (13) (isotropic gradient of
// psi, regulariser delta), and one sample per coarse node of the interface
// band theta < clip(phi_c) < 1 - theta: the 5x5 neighbourhood of phi_c
// (dy = -2..2 outer, dx = -2..2 inner, periodic) and the target, optionally
// with its 7 images under the symmetries of the square (neighbourhood
// permuted, target vector transformed).  Samples are written in row-major
// node order, so the output is deterministic.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <mutex>
#include <string>

#include "lbac.h"

namespace {

__device__ __forceinline__ int wrapi(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// S n at node (i, j) of a periodic double field (FP64, correctly rounded functions)
__device__ void flux_at(const double* phi, int nx, int ny, int i, int j, double eps, double delta, double& fx,
                        double& fy) {
    double ps[3][3];
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const double p = phi[(int64_t)wrapi(j + dy, ny) * nx + wrapi(i + dx, nx)];
            const double pc = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
            ps[dy + 1][dx + 1] = eps * log((pc + delta) / (1.0 - pc + delta));
        }
    const double gx = (ps[1][2] - ps[1][0]) / 3.0 + ((ps[2][2] - ps[2][0]) + (ps[0][2] - ps[0][0])) / 12.0;
    const double gy = (ps[2][1] - ps[0][1]) / 3.0 + ((ps[2][2] + ps[2][0]) - (ps[0][2] + ps[0][0])) / 12.0;
    const double inv = 1.0 / (sqrt(gx * gx + gy * gy) + delta);
    const double p = phi[(int64_t)j * nx + i];
    const double pc = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
    const double S = (pc + delta) * (1.0 - pc + delta) / (eps * (1.0 + 2.0 * delta) * (1.0 + 2.0 * delta));
    fx = S * gx * inv;
    fy = S * gy * inv;
}

// coarse phi and block mean of r S_f n_f
__global__ void restrict_kernel(const double* __restrict__ phif, int nxf, int nyf, int r, double eps_f, double delta,
                                double* __restrict__ phic, double* __restrict__ tx, double* __restrict__ ty) {
    const int nxc = nxf / r, nyc = nyf / r;
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= nxc || j >= nyc) return;
    double sp = 0.0, sx = 0.0, sy = 0.0;
    for (int b = 0; b < r; ++b)
        for (int a = 0; a < r; ++a) {
            const int fi = i * r + a, fj = j * r + b;
            sp += phif[(int64_t)fj * nxf + fi];
            double fx, fy;
            flux_at(phif, nxf, nyf, fi, fj, eps_f, delta, fx, fy);
            sx += fx;
            sy += fy;
        }
    const double inv = 1.0 / (double)(r * r);
    phic[(int64_t)j * nxc + i] = sp * inv;
    tx[(int64_t)j * nxc + i] = r * sx * inv;
    ty[(int64_t)j * nxc + i] = r * sy * inv;
}

__device__ __forceinline__ bool in_band(double p, float theta) {
    const double pc = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
    return pc > (double)theta && pc < 1.0 - (double)theta;
}

// per coarse row: number of band nodes
__global__ void count_kernel(const double* __restrict__ phic, int nxc, float theta, int* __restrict__ rows) {
    __shared__ int sh[256];
    const int j = blockIdx.x;
    int c = 0;
    for (int i = threadIdx.x; i < nxc; i += blockDim.x) c += in_band(phic[(int64_t)j * nxc + i], theta) ? 1 : 0;
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) rows[j] = sh[0];
}

// exclusive prefix sum of the row counts (one thread; rows <= 65536)
__global__ void scan_kernel(int* __restrict__ rows, int nyc, long long* __restrict__ total) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long long s = 0;
    for (int j = 0; j < nyc; ++j) {
        const int c = rows[j];
        rows[j] = (int)s;
        s += c;
    }
    total[0] = s;
}

// the 8 symmetries of the square as integer matrices (a b; c d) acting on (dx, dy)
__constant__ int kD4[8][4] = {{1, 0, 0, 1},  {0, -1, 1, 0}, {-1, 0, 0, -1}, {0, 1, -1, 0},
                              {-1, 0, 0, 1}, {1, 0, 0, -1}, {0, 1, 1, 0},   {0, -1, -1, 0}};

// one block per coarse row, nodes of the row handled in order by thread 0's
// running index (a row has at most a few hundred band nodes)
__global__ void emit_kernel(const double* __restrict__ phic, const double* __restrict__ tfx,
                            const double* __restrict__ tfy, int nxc, int nyc, double eps_c, double delta, float theta,
                            const int* __restrict__ rows, int copies, float* __restrict__ X, float* __restrict__ Y,
                            long long base, long long capacity) {
    const int j = blockIdx.x;
    __shared__ int order[1024];
    __shared__ int nband;
    if (threadIdx.x == 0) {
        int m = 0;
        for (int i = 0; i < nxc && m < 1024; ++i)
            if (in_band(phic[(int64_t)j * nxc + i], theta)) order[m++] = i;
        nband = m;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < nband * copies; s += blockDim.x) {
        const int i = order[s / copies], g = s % copies;
        const long long idx = base + ((long long)rows[j] + s / copies) * copies + g;
        if (idx >= capacity) continue;
        double cfx, cfy;
        flux_at(phic, nxc, nyc, i, j, eps_c, delta, cfx, cfy);
        const double tx = tfx[(int64_t)j * nxc + i] - cfx, ty = tfy[(int64_t)j * nxc + i] - cfy;
        const int a = kD4[g][0], b = kD4[g][1], c = kD4[g][2], d = kD4[g][3];
        // image: X'(p) = X(T^-1 p) with T^-1 = T^T; target' = T target
        for (int dy = -2; dy <= 2; ++dy)
            for (int dx = -2; dx <= 2; ++dx) {
                const int sx = a * dx + c * dy, sy = b * dx + d * dy;
                X[idx * 25 + (dy + 2) * 5 + (dx + 2)] =
                    (float)phic[(int64_t)wrapi(j + sy, nyc) * nxc + wrapi(i + sx, nxc)];
            }
        Y[idx * 2] = (float)(a * tx + b * ty);
        Y[idx * 2 + 1] = (float)(c * tx + d * ty);
    }
}

}  // namespace

// Workspace of lbac_closure_extract_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends.  Host code never uses its name
// as an address (that is a host-side stand-in): the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// The current device's address of `scratch`, or nullptr on a HIP error.
void* scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    void* p = g_scratch[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (!p) {
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch[dev].store(p, std::memory_order_release);
    }
    return p;
}

int64_t workspace_bytes(int32_t nxf, int32_t nyf, int32_t r) {
    if (r < 1 || nxf < r || nyf < r) return -1;
    const int64_t nc = (int64_t)(nxf / r) * (nyf / r);
    return (int64_t)(3 * nc * sizeof(double) + (nyf / r + 64) * sizeof(int) + 64);
}

// The extraction with a given workspace (device memory of workspace_bytes).
int extract(const double* phi_f_dev, int32_t nxf, int32_t nyf, int32_t r, double eps_f, double eps_c, double delta,
            float theta, int32_t augment, void* workspace, float* x_dev, float* y_dev, int64_t base, int64_t capacity,
            int64_t* count, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const int nxc = nxf / r, nyc = nyf / r;
    const int64_t nc = (int64_t)nxc * nyc;
    double* phic = (double*)workspace;
    double* tx = phic + nc;
    double* ty = tx + nc;
    int* rows = (int*)(ty + nc);
    long long* total = (long long*)(rows + ((nyc + 63) / 64) * 64);
    hipLaunchKernelGGL(restrict_kernel, dim3((nxc + 127) / 128, nyc), dim3(128), 0, s, phi_f_dev, nxf, nyf, r, eps_f,
                       delta, phic, tx, ty);
    hipLaunchKernelGGL(count_kernel, dim3(nyc), dim3(256), 0, s, phic, nxc, theta, rows);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(64), 0, s, rows, nyc, total);
    long long host_total = 0;
    if (hipMemcpyAsync(&host_total, total, sizeof(long long), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LBAC_EDEVICE;
    const int copies = augment ? 8 : 1;
    if (x_dev && y_dev && capacity > base)
        hipLaunchKernelGGL(emit_kernel, dim3(nyc), dim3(256), 0, s, phic, tx, ty, nxc, nyc, eps_c, delta, theta, rows,
                           copies, x_dev, y_dev, (long long)base, (long long)capacity);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return LBAC_EDEVICE;
    *count = host_total * copies;
    return LBAC_OK;
}

int check_args(const double* phi_f_dev, int32_t nxf, int32_t nyf, int32_t r, double eps_f, double eps_c,
               double delta, float theta, int64_t base, int64_t* count) {
    if (!phi_f_dev || !count || r < 1 || nxf % r || nyf % r || nxf / r < 5 || nyf / r < 5) return LBAC_EINVAL;
    if (!(eps_f > 0.0) || !(eps_c > 0.0) || !(delta >= 0.0) || !(theta >= 0.f) || !(theta < 0.5f) || base < 0)
        return LBAC_EINVAL;
    if (nxf / r > 1024 * 16) return LBAC_EINVAL;
    return LBAC_OK;
}

}  // namespace

extern "C" {

int64_t lbac_closure_workspace_bytes(int32_t nxf, int32_t nyf, int32_t r) { return workspace_bytes(nxf, nyf, r); }

int lbac_closure_extract(const double* phi_f_dev, int32_t nxf, int32_t nyf, int32_t r, double eps_f, double eps_c,
                         double delta, float theta, int32_t augment, void* workspace, float* x_dev, float* y_dev,
                         int64_t base, int64_t capacity, int64_t* count, void* stream) {
    const int rc = check_args(phi_f_dev, nxf, nyf, r, eps_f, eps_c, delta, theta, base, count);
    if (rc != LBAC_OK || !workspace) return LBAC_EINVAL;
    return extract(phi_f_dev, nxf, nyf, r, eps_f, eps_c, delta, theta, augment, workspace, x_dev, y_dev, base,
                   capacity, count, stream);
}

int lbac_closure_extract_noalloc(const double* phi_f_dev, int32_t nxf, int32_t nyf, int32_t r, double eps_f,
                                 double eps_c, double delta, float theta, int32_t augment, float* x_dev, float* y_dev,
                                 int64_t base, int64_t capacity, int64_t* count, void* stream) {
    const int rc = check_args(phi_f_dev, nxf, nyf, r, eps_f, eps_c, delta, theta, base, count);
    if (rc != LBAC_OK) return rc;
    if (workspace_bytes(nxf, nyf, r) > (int64_t)kNoAllocScratchBytes) return LBAC_EINVAL;
    void* ws = scratch_ptr();
    if (!ws) return LBAC_EDEVICE;
    return extract(phi_f_dev, nxf, nyf, r, eps_f, eps_c, delta, theta, augment, ws, x_dev, y_dev, base, capacity,
                   count, stream);
}

}  // extern "C"
