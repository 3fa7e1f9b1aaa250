// Training and batch inference of the learned car-following closure.
//
// Training step on a batch of n samples (features x[8], label a_idm):
//   k_mlp_fwdbwd  one wave per sample, lane j = hidden unit j: forward pass,
//                 squared error, and the per-sample deltas of both hidden
//                 layers (backpropagation through GELU);
//   k_mlp_partial one thread per parameter and slice of the batch: sums of
//                 delta x input over the slice;
//   k_mlp_sum     adds the slices into the gradient and the loss;
//   k_mlp_adam    Adam update of the FP32 master parameters.
// In bfloat16 mode the weights and layer inputs are rounded to bfloat16 as in
// the simulator's inference; gradients are taken with respect to the rounded
// weights and applied to the master copy.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/moss.h"
#include "moss_internal.h"
#include "moss_mlp.h"

using namespace moss;

namespace {

constexpr int kSlice = 256;         // samples per partial gradient sum

__device__ __forceinline__ float rnd(float x, bool bf) { return bf ? bf2f(f2bf(x)) : x; }

// network input as the simulator feeds it: a pair of bfloat16 numbers
__device__ __forceinline__ float rnd2(float x, bool bf)
{
    if (!bf)
        return x;
    const float hi = bf2f(f2bf(x));
    return hi + bf2f(f2bf(x - hi));
}

// exact tanh-form GELU and its derivative for training (FP32)
__device__ __forceinline__ float gelu_t(float x, float &dgdx)
{
    const float k0 = 0.7978845608f, k1 = 0.044715f;
    const float u = k0 * (x + k1 * (x * x * x));
    const float t = tanhf(u);
    dgdx = 0.5f * (1.0f + t) + 0.5f * x * (1.0f - t * t) * k0 * (1.0f + 3.0f * k1 * (x * x));
    return 0.5f * x * (1.0f + t);
}

// Scratch per sample: z[8], h1q[64], h2q[64], da1[64], da2[64], dy, sq.
struct Scratch {
    float *z, *h1, *h2, *da1, *da2, *dy, *sq, *part;
};

__global__ void __launch_bounds__(256) k_mlp_fwdbwd(const float *feat, const float *label,
                                                   const int32_t *idx, int n, const float *theta,
                                                   const float *norm, int bf, float out_lo,
                                                   float out_hi, Scratch sc)
{
    __shared__ float W2s[kMlpH * kMlpH];
    const bool b16 = bf != 0;
    for (int q = threadIdx.x; q < kMlpH * kMlpH; q += blockDim.x)
        W2s[q] = rnd(theta[kOffW2 + q], b16);
    __syncthreads();
    const int j = __lane_id();
    const int waves = gridDim.x * (blockDim.x >> 6);
    float w1[kMlpIn];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i)
        w1[i] = rnd(theta[kOffW1 + j * kMlpIn + i], b16);
    const float b1 = theta[kOffB1 + j], b2 = theta[kOffB2 + j];
    const float w3 = rnd(theta[kOffW3 + j], b16), b3 = theta[kOffB3];
    for (int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < n; b += waves) {
        const int src = idx ? idx[b] : b;
        float z[kMlpIn];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i)
            z[i] = rnd2(mlp_in(i, feat[(size_t)src * kMlpIn + i], norm), b16);
        float a1 = b1;
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i)
            a1 += w1[i] * z[i];
        float g1;
        const float h1 = rnd(gelu_t(a1, g1), b16);
        float a2 = b2;
        for (int i = 0; i < kMlpH; ++i)
            a2 += W2s[j * kMlpH + i] * __shfl(h1, i);
        float g2;
        const float h2 = rnd(gelu_t(a2, g2), b16);
        float y = w3 * h2;
        for (int off = 32; off > 0; off >>= 1)
            y += __shfl_xor(y, off);
        y += b3;
        // residual of the output as the simulator uses it, limited to
        // [lo_out, hi_out]; beyond the limits on the label's side the limit
        // already matches and no gradient flows
        const float lab = label[src];
        const float yc = fminf(fmaxf(y, out_lo), out_hi);
        const float r = yc - lab;
        const float dy = (y == yc) ? 2.0f * r / (float)n : 0.0f;
        const float da2 = dy * w3 * g2;
        float s = 0.0f;
        for (int k = 0; k < kMlpH; ++k)
            s += __shfl(da2, k) * W2s[k * kMlpH + j];
        const float da1 = s * g1;
        const size_t o = (size_t)b * kMlpH + j;
        sc.h1[o] = h1;
        sc.h2[o] = h2;
        sc.da1[o] = da1;
        sc.da2[o] = da2;
        if (j < kMlpIn)
            sc.z[(size_t)b * kMlpIn + j] = z[j];
        if (j == 0) {
            sc.dy[b] = dy;
            sc.sq[b] = r * r;
        }
    }
}

// part[slice][param]: sum over the slice's samples of the parameter's gradient
__global__ void __launch_bounds__(256) k_mlp_partial(int n, Scratch sc)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int slice = blockIdx.y;
    if (p >= kMlpParams)
        return;
    const int b0 = slice * kSlice, b1 = min(n, b0 + kSlice);
    float acc = 0.0f;
    if (p < kOffB1) {                     // W1[j][i]
        const int jj = p / kMlpIn, ii = p % kMlpIn;
        for (int b = b0; b < b1; ++b)
            acc += sc.da1[(size_t)b * kMlpH + jj] * sc.z[(size_t)b * kMlpIn + ii];
    } else if (p < kOffW2) {              // b1[j]
        const int jj = p - kOffB1;
        for (int b = b0; b < b1; ++b)
            acc += sc.da1[(size_t)b * kMlpH + jj];
    } else if (p < kOffB2) {              // W2[j][i]
        const int q = p - kOffW2, jj = q / kMlpH, ii = q % kMlpH;
        for (int b = b0; b < b1; ++b)
            acc += sc.da2[(size_t)b * kMlpH + jj] * sc.h1[(size_t)b * kMlpH + ii];
    } else if (p < kOffW3) {              // b2[j]
        const int jj = p - kOffB2;
        for (int b = b0; b < b1; ++b)
            acc += sc.da2[(size_t)b * kMlpH + jj];
    } else if (p < kOffB3) {              // w3[i]
        const int ii = p - kOffW3;
        for (int b = b0; b < b1; ++b)
            acc += sc.dy[b] * sc.h2[(size_t)b * kMlpH + ii];
    } else {                              // b3
        for (int b = b0; b < b1; ++b)
            acc += sc.dy[b];
    }
    sc.part[(size_t)slice * kMlpParams + p] = acc;
}

__global__ void __launch_bounds__(256) k_mlp_sum(int n, int nslice, Scratch sc, float *grad,
                                                float *loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) {
        float acc = 0.0f;
        for (int s = 0; s < nslice; ++s)
            acc += sc.part[(size_t)s * kMlpParams + p];
        grad[p] = acc;
    }
    if (blockIdx.x == 0) {
        __shared__ float red[256];
        float s = 0.0f;
        for (int b = threadIdx.x; b < n; b += blockDim.x)
            s += sc.sq[b];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off)
                red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0 && loss)
            *loss = red[0] / (float)n;
    }
}

__global__ void k_mlp_adam(float *theta, float *m, float *v, const float *grad, float lr,
                           float beta1, float beta2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams)
        return;
    const float g = grad[p];
    const float mm = beta1 * m[p] + (1.0f - beta1) * g;
    const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / c1, vh = vv / c2;
    theta[p] = theta[p] - lr * mh / (sqrtf(vh) + eps);
}

// Batch inference with the simulator's matrix-core path (one wave per 64
// samples).
__global__ void __launch_bounds__(256) k_mlp_predict(const float *feat, int n, const float *theta,
                                                    const float *norm, float *out)
{
    __shared__ MlpLds w;
    __shared__ __attribute__((aligned(16))) uint16_t zs[4 * kMlpStage];
    mlp_pack(w, theta, norm);
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int i = base + threadIdx.x;
        float z[kMlpIn];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k)
            z[k] = (i < n) ? mlp_in(k, feat[(size_t)i * kMlpIn + k], w.norm) : 0.0f;
        const float y = wave_mlp(w, zs + wv * kMlpStage, z);
        if (i < n)
            out[i] = y;
        __syncthreads();
    }
}


// Argument checks shared by both gradient entry points.
int check_grad_args(const char *who, const float *feat, const float *label, int32_t n,
                    const float *theta, const float *norm, float out_lo, float out_hi,
                    const float *grad)
{
    if (n <= 0)
        return set_error(MOSS_EINVAL, "%s: n = %d, needs at least one sample", who, n);
    if (!feat || !label || !theta || !norm || !grad)
        return set_error(MOSS_EINVAL, "%s: null buffer", who);
    if (!(out_lo < out_hi))
        return set_error(MOSS_EINVAL, "%s: out_lo %g not below out_hi %g", who, out_lo, out_hi);
    return MOSS_OK;
}

// The gradient's three kernels on a scratch area of at least
// moss_mlp_scratch_bytes(n) bytes.  Every scratch element the kernels read is
// written earlier in the same call, so the area needs no clearing.
int launch_grad(const float *d_feat, const float *d_label, const int32_t *d_idx, int32_t n,
                const float *d_theta, const float *d_norm, int32_t bf16, float out_lo,
                float out_hi, float *d_grad, float *d_loss, void *d_scratch, hipStream_t st)
{
    const size_t b = (size_t)n;
    const int nslice = (n + kSlice - 1) / kSlice;
    Scratch sc;
    float *f = (float *)d_scratch;
    sc.z = f;
    f += b * kMlpIn;
    sc.h1 = f;
    f += b * kMlpH;
    sc.h2 = f;
    f += b * kMlpH;
    sc.da1 = f;
    f += b * kMlpH;
    sc.da2 = f;
    f += b * kMlpH;
    sc.dy = f;
    f += b;
    sc.sq = f;
    f += b;
    sc.part = f;
    unsigned g = (unsigned)((n + 3) / 4);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3(g), dim3(256), 0, st, d_feat, d_label, d_idx, n,
                       d_theta, d_norm, bf16, out_lo, out_hi, sc);
    hipLaunchKernelGGL(k_mlp_partial, dim3((kMlpParams + 255) / 256, nslice), dim3(256), 0, st,
                       n, sc);
    hipLaunchKernelGGL(k_mlp_sum, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, n, nslice,
                       sc, d_grad, d_loss);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MOSS_OK
                           : set_error(MOSS_EDEVICE, "launch failed: %s", hipGetErrorString(e));
}

}  // namespace

// Scratch of moss_mlp_grad_static: room for MOSS_MLP_STATIC_MAX_SAMPLES
// samples (about 9 MB), one copy per GPU, held until the process ends.
constexpr size_t kStaticSlices = (MOSS_MLP_STATIC_MAX_SAMPLES + kSlice - 1) / kSlice;
constexpr size_t kStaticScratchBytes =
    4 * ((size_t)MOSS_MLP_STATIC_MAX_SAMPLES * (kMlpIn + 4 * kMlpH + 2) +
         kStaticSlices * kMlpParams) + 1024;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Device address of this GPU's copy of `scratch`, looked up once per device
// (with that device current).  In host code the array's name is not a device
// address; only the pointer returned here may be passed to kernels.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return set_error(MOSS_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(MOSS_EDEVICE, "device %d beyond the %d the library tracks", dev,
                         kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(MOSS_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                             hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MOSS_OK;
}

}  // namespace

extern "C" {

size_t moss_mlp_scratch_bytes(int32_t n)
{
    const size_t b = n > 0 ? (size_t)n : 1;
    const size_t nslice = (b + kSlice - 1) / kSlice;
    return 4 * (b * (kMlpIn + 4 * kMlpH + 2) + nslice * kMlpParams) + 1024;
}

int moss_mlp_grad(const float *d_feat, const float *d_label, const int32_t *d_idx, int32_t n,
                  const float *d_theta, const float *d_norm, int32_t bf16, float out_lo,
                  float out_hi, float *d_grad, float *d_loss, void *d_scratch,
                  size_t scratch_bytes, void *stream)
{
    clear_error();
    int rc = check_grad_args("moss_mlp_grad", d_feat, d_label, n, d_theta, d_norm, out_lo,
                             out_hi, d_grad);
    if (rc)
        return rc;
    if (!d_scratch)
        return set_error(MOSS_EINVAL, "moss_mlp_grad: null buffer");
    if (scratch_bytes < moss_mlp_scratch_bytes(n))
        return set_error(MOSS_ENOMEM, "moss_mlp_grad: scratch of %zu bytes, needs %zu",
                         scratch_bytes, moss_mlp_scratch_bytes(n));
    return launch_grad(d_feat, d_label, d_idx, n, d_theta, d_norm, bf16, out_lo, out_hi, d_grad,
                       d_loss, d_scratch, (hipStream_t)stream);
}

int moss_mlp_grad_static(const float *d_feat, const float *d_label, const int32_t *d_idx,
                         int32_t n, const float *d_theta, const float *d_norm, int32_t bf16,
                         float out_lo, float out_hi, float *d_grad, float *d_loss, void *stream)
{
    clear_error();
    int rc = check_grad_args("moss_mlp_grad_static", d_feat, d_label, n, d_theta, d_norm,
                             out_lo, out_hi, d_grad);
    if (rc)
        return rc;
    if (n > MOSS_MLP_STATIC_MAX_SAMPLES)
        return set_error(MOSS_EINVAL,
                         "moss_mlp_grad_static: %d samples, at most %d (the size of the "
                         "library's static scratch); use moss_mlp_grad with a workspace",
                         n, MOSS_MLP_STATIC_MAX_SAMPLES);
    void *ptr = nullptr;
    rc = static_scratch(&ptr);
    if (rc)
        return rc;
    return launch_grad(d_feat, d_label, d_idx, n, d_theta, d_norm, bf16, out_lo, out_hi, d_grad,
                       d_loss, ptr, (hipStream_t)stream);
}

int moss_mlp_adam(float *d_theta, float *d_m, float *d_v, const float *d_grad, int32_t step,
                  float lr, float beta1, float beta2, float eps, void *stream)
{
    clear_error();
    if (!d_theta || !d_m || !d_v || !d_grad)
        return set_error(MOSS_EINVAL, "moss_mlp_adam: null buffer");
    if (step < 1)
        return set_error(MOSS_EINVAL, "moss_mlp_adam: step %d, counts from 1", step);
    const double c1 = 1.0 - std::pow((double)beta1, (double)step);
    const double c2 = 1.0 - std::pow((double)beta2, (double)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, d_theta, d_m, d_v, d_grad, lr, beta1, beta2, eps,
                       (float)c1, (float)c2);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MOSS_OK
                           : set_error(MOSS_EDEVICE, "launch failed: %s", hipGetErrorString(e));
}

int moss_mlp_predict(const float *d_feat, int32_t n, const float *d_theta, const float *d_norm,
                     float *d_out, void *stream)
{
    clear_error();
    if (n < 0)
        return set_error(MOSS_EINVAL, "moss_mlp_predict: n = %d", n);
    if (n == 0)
        return MOSS_OK;
    if (!d_feat || !d_theta || !d_norm || !d_out)
        return set_error(MOSS_EINVAL, "moss_mlp_predict: null buffer");
    unsigned g = (unsigned)((n + 255) / 256);
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_mlp_predict, dim3(g), dim3(256), 0, (hipStream_t)stream, d_feat, n,
                       d_theta, d_norm, d_out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MOSS_OK
                           : set_error(MOSS_EDEVICE, "launch failed: %s", hipGetErrorString(e));
}

}  // extern "C"
