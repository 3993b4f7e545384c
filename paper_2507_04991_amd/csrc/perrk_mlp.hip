// perrk_mlp.hip -- the learned initial guess of the relaxation solve: a small
// multilayer perceptron 8 -> 32 -> 32 -> 1 (tanh hidden layers) in single
// precision, with forward, gradient and Adam kernels for training it on the
// GPU from the method's own Newton solves.
//
// Parameters are packed as W1[32][8], b1[32], W2[32][32], b2[32], W3[1][32],
// b3[1] (1377 floats).  The loss is the mean squared error over N samples.
// Gradients: each workgroup back-propagates 64 samples, stores their layer
// activations and sensitivities in LDS and sums the per-sample parameter
// gradients of its chunk in sample order; a second kernel adds the chunk sums
// in chunk order in double precision.  The result is independent of the
// launch and bitwise reproducible.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "perrk.h"

namespace {

constexpr int NW = 1377;
constexpr int OW1 = 0, OB1 = 256, OW2 = 288, OB2 = 1312, OW3 = 1344, OB3 = 1376;
constexpr int CH = 64;  // samples per workgroup in the gradient kernel

__device__ __forceinline__ void load_weights(float *sw, const float *w)
{
    for (int i = threadIdx.x; i < NW; i += blockDim.x) sw[i] = w[i];
    __syncthreads();
}

__device__ __forceinline__ float forward_one(const float *sw, const float *x, float *h1, float *h2)
{
#pragma unroll 4
    for (int o = 0; o < 32; ++o) {
        float s = sw[OB1 + o];
#pragma unroll
        for (int i = 0; i < 8; ++i) s += sw[OW1 + o * 8 + i] * x[i];
        h1[o] = tanhf(s);
    }
#pragma unroll 4
    for (int o = 0; o < 32; ++o) {
        float s = sw[OB2 + o];
#pragma unroll 8
        for (int i = 0; i < 32; ++i) s += sw[OW2 + o * 32 + i] * h1[i];
        h2[o] = tanhf(s);
    }
    float y = sw[OB3];
#pragma unroll 8
    for (int i = 0; i < 32; ++i) y += sw[OW3 + i] * h2[i];
    return y;
}

__global__ void __launch_bounds__(256) mlp_forward_kernel(const float *w, const float *x, int64_t n, float *y)
{
    __shared__ float sw[NW];
    load_weights(sw, w);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float xi[8], h1[32], h2[32];
#pragma unroll
    for (int k = 0; k < 8; ++k) xi[k] = x[i * 8 + k];
    y[i] = forward_one(sw, xi, h1, h2);
}

// One chunk of CH samples per workgroup of CH threads.
__global__ void __launch_bounds__(CH) mlp_grad_chunk_kernel(const float *w, const float *x, const float *t, int64_t n,
                                                          float inv_n, float *part)
{
    __shared__ float sw[NW];
    __shared__ float sx[CH][9];
    __shared__ float sh1[CH][33], sh2[CH][33], sd1[CH][33], sd2[CH][33];
    __shared__ float sd3[CH], sl[CH];
    load_weights(sw, w);
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * CH + tid;
    const bool valid = i < n;
    float xi[8], h1[32], h2[32];
#pragma unroll
    for (int k = 0; k < 8; ++k) xi[k] = valid ? x[i * 8 + k] : 0.0f;
    const float y = forward_one(sw, xi, h1, h2);
    const float r = valid ? y - t[i] : 0.0f;
    const float d3 = 2.0f * r * inv_n;  // dL/dy
    float d2[32];
#pragma unroll
    for (int o = 0; o < 32; ++o) d2[o] = d3 * sw[OW3 + o] * (1.0f - h2[o] * h2[o]);
#pragma unroll 4
    for (int k = 0; k < 32; ++k) {
        float s = 0.0f;
#pragma unroll 8
        for (int o = 0; o < 32; ++o) s += sw[OW2 + o * 32 + k] * d2[o];
        sd1[tid][k] = s * (1.0f - h1[k] * h1[k]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) sx[tid][k] = xi[k];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        sh1[tid][k] = h1[k];
        sh2[tid][k] = h2[k];
        sd2[tid][k] = d2[k];
    }
    sd3[tid] = d3;
    sl[tid] = r * r * inv_n;
    __syncthreads();
    float *out = part + (size_t)blockIdx.x * (NW + 1);
    for (int p = tid; p < NW; p += CH) {
        float s = 0.0f;
        if (p < OB1) {
            const int o = p / 8, k = p % 8;
            for (int m = 0; m < CH; ++m) s += sd1[m][o] * sx[m][k];
        } else if (p < OW2) {
            const int o = p - OB1;
            for (int m = 0; m < CH; ++m) s += sd1[m][o];
        } else if (p < OB2) {
            const int o = (p - OW2) / 32, k = (p - OW2) % 32;
            for (int m = 0; m < CH; ++m) s += sd2[m][o] * sh1[m][k];
        } else if (p < OW3) {
            const int o = p - OB2;
            for (int m = 0; m < CH; ++m) s += sd2[m][o];
        } else if (p < OB3) {
            const int k = p - OW3;
            for (int m = 0; m < CH; ++m) s += sd3[m] * sh2[m][k];
        } else {
            for (int m = 0; m < CH; ++m) s += sd3[m];
        }
        out[p] = s;
    }
    if (tid == 0) {
        float s = 0.0f;
        for (int m = 0; m < CH; ++m) s += sl[m];
        out[NW] = s;
    }
}

__global__ void __launch_bounds__(256) mlp_grad_reduce_kernel(const float *part, int64_t nchunk, float *grad,
                                                              double *loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NW) return;
    double s = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) s += (double)part[(size_t)c * (NW + 1) + p];
    if (p < NW) grad[p] = (float)s;
    else if (loss) *loss = s;
}

__global__ void __launch_bounds__(256) mlp_adam_kernel(float *w, const float *g, float *m, float *v, float lr, float b1,
                                                       float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NW) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// Scratch of perrk_mlp_loss_grad_static: the per-chunk partial sums of up to
// PERRK_MLP_STATIC_MAX_N samples (11.3 MB), one copy per device, held until the
// process ends.  Host code never passes this name to a kernel (on the host it
// is a stand-in, not a device address): it uses the per-device address that
// hipGetSymbolAddress returns.
constexpr int64_t STATIC_CHUNKS = PERRK_MLP_STATIC_MAX_N / CH;
static_assert(PERRK_MLP_STATIC_MAX_N % CH == 0, "whole chunks");
__device__ __align__(256) float scratch[STATIC_CHUNKS * (NW + 1)];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[MAX_DEVICES] = {};

// Device address of the current device's scratch, looked up once per device.
int scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return PERRK_EHIP;
    if (dev < 0 || dev >= MAX_DEVICES) return PERRK_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PERRK_EHIP;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return PERRK_OK;
}

// The two gradient kernels on a workspace of at least nchunk chunks.
int launch_loss_grad(const float *w_dev, const float *x_dev, const float *t_dev, int64_t n, float *grad_dev,
                     double *loss_dev, float *work, hipStream_t s)
{
    const int64_t nchunk = (n + CH - 1) / CH;
    hipLaunchKernelGGL(mlp_grad_chunk_kernel, dim3((unsigned)nchunk), dim3(CH), 0, s, w_dev, x_dev, t_dev, n,
                       1.0f / (float)n, work);
    if (hipGetLastError() != hipSuccess) return PERRK_EHIP;
    hipLaunchKernelGGL(mlp_grad_reduce_kernel, dim3((NW + 1 + 255) / 256), dim3(256), 0, s,
                       static_cast<const float *>(work), nchunk, grad_dev, loss_dev);
    return hipGetLastError() == hipSuccess ? PERRK_OK : PERRK_EHIP;
}

}  // namespace

extern "C" {

size_t perrk_mlp_workspace_bytes(int64_t n)
{
    const int64_t nchunk = n > 0 ? (n + CH - 1) / CH : 0;
    return (size_t)nchunk * (NW + 1) * sizeof(float);
}

int perrk_mlp_forward(const float *w_dev, const float *x_dev, int64_t n, float *y_dev, void *stream)
{
    if (!w_dev || (n > 0 && (!x_dev || !y_dev)) || n < 0) return PERRK_EINVAL;
    if (n == 0) return PERRK_OK;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       w_dev, x_dev, n, y_dev);
    return hipGetLastError() == hipSuccess ? PERRK_OK : PERRK_EHIP;
}

int perrk_mlp_loss_grad(const float *w_dev, const float *x_dev, const float *t_dev, int64_t n, float *grad_dev,
                        double *loss_dev, void *work_dev, size_t work_bytes, void *stream)
{
    if (!w_dev || !x_dev || !t_dev || !grad_dev || n <= 0) return PERRK_EINVAL;
    if (!work_dev || work_bytes < perrk_mlp_workspace_bytes(n)) return PERRK_EINVAL;
    return launch_loss_grad(w_dev, x_dev, t_dev, n, grad_dev, loss_dev, static_cast<float *>(work_dev),
                            (hipStream_t)stream);
}

int perrk_mlp_loss_grad_static(const float *w_dev, const float *x_dev, const float *t_dev, int64_t n,
                               float *grad_dev, double *loss_dev, void *stream)
{
    if (!w_dev || !x_dev || !t_dev || !grad_dev || n <= 0) return PERRK_EINVAL;
    if (n > PERRK_MLP_STATIC_MAX_N) return PERRK_ENOMEM;
    void *work = nullptr;
    const int st = scratch_address(&work);
    if (st != PERRK_OK) return st;
    return launch_loss_grad(w_dev, x_dev, t_dev, n, grad_dev, loss_dev, static_cast<float *>(work),
                            (hipStream_t)stream);
}

int perrk_mlp_adam(float *w_dev, const float *grad_dev, float *m_dev, float *v_dev, int32_t step, float lr,
                   float beta1, float beta2, float eps, void *stream)
{
    if (!w_dev || !grad_dev || !m_dev || !v_dev || step < 1) return PERRK_EINVAL;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NW + 255) / 256), dim3(256), 0, (hipStream_t)stream, w_dev, grad_dev, m_dev,
                       v_dev, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? PERRK_OK : PERRK_EHIP;
}

}  // extern "C"
