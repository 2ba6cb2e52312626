// Training of the learned closure's network on the GPU: a 25 -> 64 -> 64 -> 2
// multilayer perceptron with tanh-GELU, mean-squared-error loss and Adam.
//
// Kernels (FP32 throughout, all reductions in a fixed order so a training
// run is reproducible):
//   mlp_forward_kernel  one thread per sample; weights in LDS; keeps the
//                       pre-activations z1, z2 and the outputs
//   mlp_backward_kernel one thread per sample: d3 = 2 (out - y) / B,
//                       d2 = (W3^T d3) * gelu'(z2), d1 = (W2^T d2) * gelu'(z1)
//   mlp_wgrad_kernel    one thread per parameter, summing over the batch
//   mlp_loss_kernel     sum of squared errors (one block)
//   mlp_adam_kernel     one thread per parameter (Kingma & Ba, Algorithm 1)
// Parameter layout: W1[64][25], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbac.h"

namespace {

constexpr int kIn = 25, kH = 64, kOut = 2;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH,
              ob3 = oW3 + kOut * kH, kNParam = ob3 + kOut;
static_assert(kNParam == LBAC_MLP_NPARAM, "parameter count");
constexpr int kAct = 2 * kH + kOut;  // per-sample scratch: z1, z2, out
constexpr float kGeluK = 0.7978845608028654f;  // sqrt(2/pi)

__device__ __forceinline__ float gelu(float x) {
    return 0.5f * x * (1.0f + tanhf(kGeluK * (x + 0.044715f * x * x * x)));
}
__device__ __forceinline__ float gelu_grad(float x) {
    const float t = tanhf(kGeluK * (x + 0.044715f * x * x * x));
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * kGeluK * (1.0f + 3.0f * 0.044715f * x * x);
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ w, const float* __restrict__ x,
                                                          int64_t batch, float* __restrict__ act,
                                                          float* __restrict__ out) {
    __shared__ float sw[kNParam];
    for (int i = threadIdx.x; i < kNParam; i += blockDim.x) sw[i] = w[i];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= batch) return;
    float xi[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) xi[k] = x[s * kIn + k];
    float h1[kH];
    float* a = act + s * kAct;
    for (int o = 0; o < kH; ++o) {
        float z = sw[ob1 + o];
#pragma unroll
        for (int k = 0; k < kIn; ++k) z += sw[oW1 + o * kIn + k] * xi[k];
        a[o] = z;
        h1[o] = gelu(z);
    }
    float o0 = sw[ob3], o1 = sw[ob3 + 1];
    for (int o = 0; o < kH; ++o) {
        float z = sw[ob2 + o];
#pragma unroll 16
        for (int k = 0; k < kH; ++k) z += sw[oW2 + o * kH + k] * h1[k];
        a[kH + o] = z;
        const float h2 = gelu(z);
        o0 += sw[oW3 + o] * h2;
        o1 += sw[oW3 + kH + o] * h2;
    }
    a[2 * kH] = o0;
    a[2 * kH + 1] = o1;
    if (out) {
        out[s * kOut] = o0;
        out[s * kOut + 1] = o1;
    }
}

// dl: per-sample deltas d1 (64), d2 (64), d3 (2)
__global__ __launch_bounds__(256) void mlp_backward_kernel(const float* __restrict__ w, const float* __restrict__ y,
                                                           int64_t batch, const float* __restrict__ act,
                                                           float* __restrict__ dl) {
    __shared__ float sw[kNParam];
    for (int i = threadIdx.x; i < kNParam; i += blockDim.x) sw[i] = w[i];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= batch) return;
    const float* a = act + s * kAct;
    float* d = dl + s * kAct;
    const float inv_b = 1.0f / (float)batch;
    const float d30 = 2.0f * (a[2 * kH] - y[s * kOut]) * inv_b;
    const float d31 = 2.0f * (a[2 * kH + 1] - y[s * kOut + 1]) * inv_b;
    d[2 * kH] = d30;
    d[2 * kH + 1] = d31;
    float d2[kH];
    for (int o = 0; o < kH; ++o) {
        d2[o] = (sw[oW3 + o] * d30 + sw[oW3 + kH + o] * d31) * gelu_grad(a[kH + o]);
        d[kH + o] = d2[o];
    }
    for (int i = 0; i < kH; ++i) {
        float g = 0.f;
#pragma unroll 16
        for (int o = 0; o < kH; ++o) g += sw[oW2 + o * kH + i] * d2[o];
        d[i] = g * gelu_grad(a[i]);
    }
}

// gradient of parameter p: sum over the batch in sample order
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(const float* __restrict__ x, int64_t batch,
                                                        const float* __restrict__ act, const float* __restrict__ dl,
                                                        float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    float g = 0.f;
    if (p < ob1) {  // W1[o][k] = sum d1[o] x[k]
        const int o = p / kIn, k = p % kIn;
        for (int64_t s = 0; s < batch; ++s) g += dl[s * kAct + o] * x[s * kIn + k];
    } else if (p < oW2) {  // b1
        const int o = p - ob1;
        for (int64_t s = 0; s < batch; ++s) g += dl[s * kAct + o];
    } else if (p < ob2) {  // W2[o][k] = sum d2[o] gelu(z1[k])
        const int o = (p - oW2) / kH, k = (p - oW2) % kH;
        for (int64_t s = 0; s < batch; ++s) g += dl[s * kAct + kH + o] * gelu(act[s * kAct + k]);
    } else if (p < oW3) {  // b2
        const int o = p - ob2;
        for (int64_t s = 0; s < batch; ++s) g += dl[s * kAct + kH + o];
    } else if (p < ob3) {  // W3[o][k] = sum d3[o] gelu(z2[k])
        const int o = (p - oW3) / kH, k = (p - oW3) % kH;
        for (int64_t s = 0; s < batch; ++s) g += dl[s * kAct + 2 * kH + o] * gelu(act[s * kAct + kH + k]);
    } else {  // b3
        const int o = p - ob3;
        for (int64_t s = 0; s < batch; ++s) g += dl[s * kAct + 2 * kH + o];
    }
    grad[p] = g;
}

__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* __restrict__ y, int64_t batch,
                                                       const float* __restrict__ act, double* __restrict__ loss) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t s = threadIdx.x; s < batch; s += blockDim.x) {
        const double e0 = (double)act[s * kAct + 2 * kH] - y[s * kOut];
        const double e1 = (double)act[s * kAct + 2 * kH + 1] - y[s * kOut + 1];
        acc += e0 * e0 + e1 * e1;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = sh[0] / (double)batch;
}

__global__ void mlp_adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

}  // namespace

struct lbac_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    float *act = nullptr, *dl = nullptr;
    double* loss = nullptr;
    double* host_loss = nullptr;
    int64_t cap = 0;
    int64_t t = 0;
    std::string err;
};

namespace {

int mfail(lbac_mlp* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define MHIP(h, call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess) return mfail(h, LBAC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int ensure(lbac_mlp* h, int64_t batch) {
    if (batch <= h->cap) return LBAC_OK;
    (void)hipFree(h->act);
    (void)hipFree(h->dl);
    h->act = h->dl = nullptr;
    h->cap = 0;
    MHIP(h, hipMalloc(&h->act, sizeof(float) * kAct * batch));
    MHIP(h, hipMalloc(&h->dl, sizeof(float) * kAct * batch));
    h->cap = batch;
    return LBAC_OK;
}

int forward_backward(lbac_mlp* h, const float* x, const float* y, int64_t batch) {
    int rc = ensure(h, batch);
    if (rc != LBAC_OK) return rc;
    const int blocks = (int)((batch + 255) / 256);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(256), 0, h->stream, h->w, x, batch, h->act,
                       (float*)nullptr);
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(blocks), dim3(256), 0, h->stream, h->w, y, batch, h->act, h->dl);
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, h->stream, x, batch, h->act,
                       h->dl, h->g);
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(256), 0, h->stream, y, batch, h->act, h->loss);
    MHIP(h, hipGetLastError());
    return LBAC_OK;
}

}  // namespace

extern "C" {

int lbac_mlp_create(const float* init, void* stream, lbac_mlp** out) {
    if (!out || !init) return LBAC_EINVAL;
    *out = nullptr;
    for (int i = 0; i < kNParam; ++i)
        if (!std::isfinite(init[i])) return LBAC_EINVAL;
    lbac_mlp* h = new (std::nothrow) lbac_mlp();
    if (!h) return LBAC_ENOMEM;
    auto bail = [&](int code) {
        lbac_mlp_free(h);
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) return bail(LBAC_EDEVICE);
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return bail(LBAC_EDEVICE);
        h->own_stream = true;
    }
    const size_t pb = sizeof(float) * kNParam;
    if (hipMalloc(&h->w, pb) != hipSuccess || hipMalloc(&h->g, pb) != hipSuccess ||
        hipMalloc(&h->m, pb) != hipSuccess || hipMalloc(&h->v, pb) != hipSuccess ||
        hipMalloc(&h->loss, sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&h->host_loss, sizeof(double), hipHostMallocDefault) != hipSuccess)
        return bail(LBAC_ENOMEM);
    std::vector<float> zero(kNParam, 0.f);
    if (hipMemcpyAsync(h->w, init, pb, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->m, zero.data(), pb, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->v, zero.data(), pb, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return bail(LBAC_EDEVICE);
    *out = h;
    return LBAC_OK;
}

int lbac_mlp_free(lbac_mlp* h) {
    if (!h) return LBAC_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->w);
    (void)hipFree(h->g);
    (void)hipFree(h->m);
    (void)hipFree(h->v);
    (void)hipFree(h->act);
    (void)hipFree(h->dl);
    (void)hipFree(h->loss);
    if (h->host_loss) (void)hipHostFree(h->host_loss);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return LBAC_OK;
}

int lbac_mlp_get_weights(lbac_mlp* h, float* out) {
    if (!h || !out) return LBAC_EINVAL;
    MHIP(h, hipMemcpyAsync(out, h->w, sizeof(float) * kNParam, hipMemcpyDeviceToHost, h->stream));
    MHIP(h, hipStreamSynchronize(h->stream));
    return LBAC_OK;
}

int lbac_mlp_set_weights(lbac_mlp* h, const float* in) {
    if (!h || !in) return LBAC_EINVAL;
    MHIP(h, hipMemcpyAsync(h->w, in, sizeof(float) * kNParam, hipMemcpyHostToDevice, h->stream));
    MHIP(h, hipStreamSynchronize(h->stream));
    return LBAC_OK;
}

int lbac_mlp_forward(lbac_mlp* h, const float* x_dev, int64_t batch, float* out_dev) {
    if (!h || !x_dev || !out_dev || batch < 1) return LBAC_EINVAL;
    int rc = ensure(h, batch);
    if (rc != LBAC_OK) return rc;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((int)((batch + 255) / 256)), dim3(256), 0, h->stream, h->w, x_dev,
                       batch, h->act, out_dev);
    MHIP(h, hipGetLastError());
    return LBAC_OK;
}

int lbac_mlp_loss_grad(lbac_mlp* h, const float* x_dev, const float* y_dev, int64_t batch, double* loss,
                       float* grad) {
    if (!h || !x_dev || !y_dev || batch < 1) return LBAC_EINVAL;
    int rc = forward_backward(h, x_dev, y_dev, batch);
    if (rc != LBAC_OK) return rc;
    if (grad) MHIP(h, hipMemcpyAsync(grad, h->g, sizeof(float) * kNParam, hipMemcpyDeviceToHost, h->stream));
    MHIP(h, hipMemcpyAsync(h->host_loss, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    MHIP(h, hipStreamSynchronize(h->stream));
    if (loss) *loss = *h->host_loss;
    return LBAC_OK;
}

int lbac_mlp_train_step(lbac_mlp* h, const float* x_dev, const float* y_dev, int64_t batch, float lr, double* loss) {
    if (!h || !x_dev || !y_dev || batch < 1 || !(lr > 0.f)) return LBAC_EINVAL;
    int rc = forward_backward(h, x_dev, y_dev, batch);
    if (rc != LBAC_OK) return rc;
    h->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)h->t)), c2 = (float)(1.0 - std::pow(0.999, (double)h->t));
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, h->stream, h->w, h->g, h->m,
                       h->v, lr, b1, b2, 1e-8f, c1, c2);
    MHIP(h, hipGetLastError());
    if (loss) {
        MHIP(h, hipMemcpyAsync(h->host_loss, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        MHIP(h, hipStreamSynchronize(h->stream));
        *loss = *h->host_loss;
    }
    return LBAC_OK;
}

const char* lbac_mlp_last_error(lbac_mlp* h) { return h ? h->err.c_str() : "no network"; }

}  // extern "C"
