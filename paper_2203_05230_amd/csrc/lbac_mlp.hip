// Training of the learned closure's network on the GPU: a 25 -> 64 -> 64 -> 2
// multilayer perceptron with tanh-GELU, mean-squared-error loss and Adam.
//
// FP32 throughout, on the FP32 matrix cores (16x16x4 MFMA, FP32 products and
// sums), every reduction in a fixed order so a training run is reproducible:
//   mlp_block_kernel   one wavefront per 16 samples: the forward pass
//                      (Z1 = W1 X + b1, H1 = gelu(Z1), Z2 = W2 H1 + b2,
//                      H2 = gelu(Z2), out = W3 H2 + b3), and for training the
//                      backward pass (d3 = 2 (out - y) / B,
//                      d2 = (W3^T d3) * gelu'(Z2), d1 = (W2^T d2) * gelu'(Z1))
//                      and the block's share of the gradient
//                      (dW1 = d1 X^T, dW2 = d2 H1^T, dW3 = d3 H2^T, db = row
//                      sums of d) and of the loss, written to per-block rows
//   mlp_reduce_kernel  the gradient as the sum of the blocks' rows in a
//                      fixed order, then (training) the Adam update (Kingma
//                      & Ba, Algorithm 1); the loss as the sum of the blocks'
//                      shares in a fixed order
// MFMA operands: lane l of a 16x16x4 product supplies A[l % 16][k] and
// B[k][l % 16] with k the lane group l / 16 of the K-step, and receives
// D[4 (l / 16) + i][l % 16], i = 0..3.  The forward products keep features on
// the M side and samples on N, so the accumulator of a layer holds, in lane
// (g, n), features 16 mt + 4 g + i of sample n, which is directly the next
// layer's B operand for the K-steps (mt, i); the weight products take the
// block's 16 samples as K from LDS.
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
constexpr float kGeluK = 0.7978845608028654f;  // sqrt(2/pi)
constexpr int kNS = 16;                        // samples per block (one wavefront)
constexpr int kKin = 28;                       // inputs padded to whole K-steps of 4

typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu(float x) {
    return 0.5f * x * (1.0f + tanhf(kGeluK * (x + 0.044715f * x * x * x)));
}
__device__ __forceinline__ float gelu_grad(float x) {
    const float t = tanhf(kGeluK * (x + 0.044715f * x * x * x));
    return 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * kGeluK * (1.0f + 3.0f * 0.044715f * x * x);
}

__device__ __forceinline__ f32x4_t mfma(float a, float b, f32x4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct MlpLds {
    float w[kNParam];
    float x[kNS][32];   // inputs of the block's samples (25..31 zero)
    float h1[kH][kNS];  // gelu(z1), features x samples
    float h2[kH][kNS];
    float d1[kH][kNS];
    float d2[kH][kNS];
    float d3[kOut][kNS];
};

// grad_rows: per block kNParam floats; loss_rows: per block one double; out
// (forward only, may be null): batch x 2.  With train == false only the
// forward pass runs.
template <bool TRAIN>
__global__ __launch_bounds__(64) void mlp_block_kernel(const float* __restrict__ w, const float* __restrict__ x,
                                                       const float* __restrict__ y, int64_t batch, float inv_b,
                                                       float* __restrict__ out, float* __restrict__ grad_rows,
                                                       double* __restrict__ loss_rows) {
    __shared__ MlpLds L;
    const int l = threadIdx.x, r = l % 16, g = l / 16;
    const int64_t s0 = (int64_t)blockIdx.x * kNS;
    for (int i = l; i < kNParam; i += 64) L.w[i] = w[i];
    for (int i = l; i < kNS * 32; i += 64) {
        const int n = i / 32, k = i % 32;
        L.x[n][k] = (k < kIn && s0 + n < batch) ? x[(s0 + n) * kIn + k] : 0.f;
    }
    __syncthreads();

    // ---- forward: lane (g, r) holds features 16 mt + 4 g + i of sample r
    f32x4_t z1[4], z2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4_t acc;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = L.w[ob1 + 16 * mt + 4 * g + i];
#pragma unroll
        for (int ks = 0; ks < kKin / 4; ++ks) {
            const int k = 4 * ks + g;
            acc = mfma(k < kIn ? L.w[oW1 + (16 * mt + r) * kIn + k] : 0.f, L.x[r][k], acc);
        }
        z1[mt] = acc;
    }
    float h1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) h1[mt][i] = gelu(z1[mt][i]);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4_t acc;
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = L.w[ob2 + 16 * mt + 4 * g + i];
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                acc = mfma(L.w[oW2 + (16 * mt + r) * kH + 16 * kt + 4 * g + i], h1[kt][i], acc);
        z2[mt] = acc;
    }
    float h2[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) h2[mt][i] = gelu(z2[mt][i]);
    // layer 3 on the vector units: each lane's 16 features, then the four
    // lane groups of a sample summed pairwise (the same order on every lane)
    float o[2];
#pragma unroll
    for (int c = 0; c < kOut; ++c) {
        float p = 0.f;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) p = __builtin_fmaf(L.w[oW3 + c * kH + 16 * mt + 4 * g + i], h2[mt][i], p);
        p += __shfl_xor(p, 16, 64);
        p += __shfl_xor(p, 32, 64);
        o[c] = L.w[ob3 + c] + p;
    }
    const int64_t s = s0 + r;
    const bool real = s < batch;
    if (!TRAIN) {
        if (out && g == 0 && real) {
            out[s * kOut] = o[0];
            out[s * kOut + 1] = o[1];
        }
        return;
    }

    // ---- loss and backward
    const float e0 = real ? o[0] - y[s * kOut] : 0.f;
    const float e1 = real ? o[1] - y[s * kOut + 1] : 0.f;
    const float d30 = 2.0f * e0 * inv_b, d31 = 2.0f * e1 * inv_b;
    float d2r[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 16 * mt + 4 * g + i;
            d2r[mt][i] = (L.w[oW3 + k] * d30 + L.w[oW3 + kH + k] * d31) * gelu_grad(z2[mt][i]);
        }
    // d1 = (W2^T d2) * gelu'(z1): A[row k1][feature k] = W2[k][k1]
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc = mfma(L.w[oW2 + (16 * kt + 4 * g + i) * kH + 16 * mt + r], d2r[kt][i], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 16 * mt + 4 * g + i;
            L.d1[k][r] = acc[i] * gelu_grad(z1[mt][i]);
            L.h1[k][r] = h1[mt][i];
            L.h2[k][r] = h2[mt][i];
            L.d2[k][r] = d2r[mt][i];
        }
    }
    if (g == 0) {
        L.d3[0][r] = d30;
        L.d3[1][r] = d31;
    }
    // the block's loss share: squared errors of its samples in sample order
    {
        const double se = (double)e0 * e0 + (double)e1 * e1;
        double t = 0.0;
        for (int n = 0; n < kNS; ++n) t += __shfl(se, n, 64);
        if (l == 0) loss_rows[blockIdx.x] = t;
    }
    __syncthreads();

    // ---- the block's gradient rows: K = the block's 16 samples
    float* G = grad_rows + (int64_t)blockIdx.x * kNParam;
    // dW1 [64 x 25] = d1 X^T (N-tiles of 16 inputs)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < kNS / 4; ++ks) acc = mfma(L.d1[16 * mt + r][4 * ks + g], L.x[4 * ks + g][16 * nt + r], acc);
            const int k = 16 * nt + r;
            if (k < kIn)
#pragma unroll
                for (int i = 0; i < 4; ++i) G[oW1 + (16 * mt + 4 * g + i) * kIn + k] = acc[i];
        }
    // dW2 [64 x 64] = d2 H1^T
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < kNS / 4; ++ks)
                acc = mfma(L.d2[16 * mt + r][4 * ks + g], L.h1[16 * nt + r][4 * ks + g], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) G[oW2 + (16 * mt + 4 * g + i) * kH + 16 * nt + r] = acc[i];
        }
    // dW3 [2 x 64] = d3 H2^T and the bias rows: sums over samples in order
    {
        float a0 = 0.f, a1 = 0.f, b1s = 0.f, b2s = 0.f;
        for (int n = 0; n < kNS; ++n) {
            a0 = __builtin_fmaf(L.d3[0][n], L.h2[l][n], a0);
            a1 = __builtin_fmaf(L.d3[1][n], L.h2[l][n], a1);
            b1s += L.d1[l][n];
            b2s += L.d2[l][n];
        }
        G[oW3 + l] = a0;
        G[oW3 + kH + l] = a1;
        G[ob1 + l] = b1s;
        G[ob2 + l] = b2s;
        if (l < kOut) {
            float b3s = 0.f;
            for (int n = 0; n < kNS; ++n) b3s += L.d3[l][n];
            G[ob3 + l] = b3s;
        }
    }
}

// The gradient as the sum of the blocks' rows, in a fixed order: a block of
// 256 threads takes 64 parameters; thread (q, p) sums the rows b = q mod 4
// with four running sums (rows q, q + 4, q + 8, q + 12 modulo 16), which
// are then added pairwise, and the four quarters are added pairwise again.
// With adam != 0 the Adam update of the weights follows.  Block 0 also sums
// the loss shares (thread t the rows t mod 256, then a pairwise tree) into
// *loss (divided by the batch size).
constexpr int kRedParams = 64;
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ grad_rows,
                                                         const double* __restrict__ loss_rows, int nblk,
                                                         int64_t batch, float* __restrict__ grad,
                                                         double* __restrict__ loss, int adam, float* __restrict__ w,
                                                         float* __restrict__ m, float* __restrict__ v, float lr,
                                                         float b1, float b2, float eps, float c1, float c2) {
    __shared__ float part[4][kRedParams];
    __shared__ double lsum[256];
    const int t = threadIdx.x, q = t / kRedParams, pl = t % kRedParams;
    const int p = blockIdx.x * kRedParams + pl;
    if (blockIdx.x == 0) {
        double a = 0.0;
        for (int b = t; b < nblk; b += 256) a += loss_rows[b];
        lsum[t] = a;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (t < h) lsum[t] += lsum[t + h];
            __syncthreads();
        }
        if (t == 0) loss[0] = lsum[0] / (double)batch;
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (p < kNParam) {
        int b = q;
        for (; b + 12 < nblk; b += 16)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += grad_rows[(int64_t)(b + 4 * u) * kNParam + p];
        for (int u = 0; b < nblk; b += 4, ++u) acc[u] += grad_rows[(int64_t)b * kNParam + p];
    }
    part[q][pl] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (q != 0 || p >= kNParam) return;
    const float gp = (part[0][pl] + part[1][pl]) + (part[2][pl] + part[3][pl]);
    grad[p] = gp;
    if (!adam) return;
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
    float* grad_rows = nullptr;   // per block of 16 samples: its share of the gradient
    double* loss_rows = nullptr;  // per block: its share of the loss
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

int64_t blocks_of(int64_t batch) { return (batch + kNS - 1) / kNS; }

int ensure(lbac_mlp* h, int64_t batch) {
    const int64_t nb = blocks_of(batch);
    if (nb <= h->cap) return LBAC_OK;
    (void)hipFree(h->grad_rows);
    (void)hipFree(h->loss_rows);
    h->grad_rows = nullptr;
    h->loss_rows = nullptr;
    h->cap = 0;
    MHIP(h, hipMalloc(&h->grad_rows, sizeof(float) * kNParam * nb));
    MHIP(h, hipMalloc(&h->loss_rows, sizeof(double) * nb));
    h->cap = nb;
    return LBAC_OK;
}

// Gradient of the loss into h->g and the loss into h->loss; with lr > 0 also
// the Adam update of the weights.
int gradient_step(lbac_mlp* h, const float* x, const float* y, int64_t batch, float lr) {
    if (batch > ((int64_t)1 << 31) * kNS) return mfail(h, LBAC_EINVAL, "batch too large");
    int rc = ensure(h, batch);
    if (rc != LBAC_OK) return rc;
    const int nb = (int)blocks_of(batch);
    hipLaunchKernelGGL(mlp_block_kernel<true>, dim3(nb), dim3(64), 0, h->stream, h->w, x, y, batch,
                       1.0f / (float)batch, (float*)nullptr, h->grad_rows, h->loss_rows);
    float c1 = 1.f, c2 = 1.f;
    if (lr > 0.f) {
        h->t += 1;
        c1 = (float)(1.0 - std::pow(0.9, (double)h->t));
        c2 = (float)(1.0 - std::pow(0.999, (double)h->t));
    }
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kNParam + kRedParams - 1) / kRedParams), dim3(256), 0, h->stream,
                       h->grad_rows,
                       h->loss_rows, nb, batch, h->g, h->loss, lr > 0.f ? 1 : 0, h->w, h->m, h->v, lr, 0.9f, 0.999f,
                       1e-8f, c1, c2);
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
    (void)hipFree(h->grad_rows);
    (void)hipFree(h->loss_rows);
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
    if (batch > ((int64_t)1 << 31) * kNS) return mfail(h, LBAC_EINVAL, "batch too large");
    hipLaunchKernelGGL(mlp_block_kernel<false>, dim3((unsigned)blocks_of(batch)), dim3(64), 0, h->stream, h->w, x_dev,
                       (const float*)nullptr, batch, 1.0f / (float)batch, out_dev, (float*)nullptr, (double*)nullptr);
    MHIP(h, hipGetLastError());
    return LBAC_OK;
}

int lbac_mlp_loss_grad(lbac_mlp* h, const float* x_dev, const float* y_dev, int64_t batch, double* loss,
                       float* grad) {
    if (!h || !x_dev || !y_dev || batch < 1) return LBAC_EINVAL;
    int rc = gradient_step(h, x_dev, y_dev, batch, 0.f);
    if (rc != LBAC_OK) return rc;
    if (grad) MHIP(h, hipMemcpyAsync(grad, h->g, sizeof(float) * kNParam, hipMemcpyDeviceToHost, h->stream));
    MHIP(h, hipMemcpyAsync(h->host_loss, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    MHIP(h, hipStreamSynchronize(h->stream));
    if (loss) *loss = *h->host_loss;
    return LBAC_OK;
}

int lbac_mlp_train_step(lbac_mlp* h, const float* x_dev, const float* y_dev, int64_t batch, float lr, double* loss) {
    if (!h || !x_dev || !y_dev || batch < 1 || !(lr > 0.f)) return LBAC_EINVAL;
    int rc = gradient_step(h, x_dev, y_dev, batch, lr);
    if (rc != LBAC_OK) return rc;
    if (loss) {
        MHIP(h, hipMemcpyAsync(h->host_loss, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        MHIP(h, hipStreamSynchronize(h->stream));
        *loss = *h->host_loss;
    }
    return LBAC_OK;
}

const char* lbac_mlp_last_error(lbac_mlp* h) { return h ? h->err.c_str() : "no network"; }

}  // extern "C"
