// Learned car-following closure: an 8 -> 64 -> 64 -> 1 network with GELU
// (tanh form) evaluated per wave of 64 vehicles on the matrix cores, with
// bfloat16 weights and activations and FP32 accumulation.
//
// Layout of the parameter vector (FP32 master copy, kMlpParams values):
//   W1[64][8], b1[64], W2[64][64], b2[64], w3[64], b3[1]
// and of the input description (kMlpNorm values):
//   mean[8], inv_std[8], lo[8], hi[8]   (normalisation and envelope).
//
// The network is evaluated transposed, H^T = W * X^T, with the weights as the
// A operand of the matrix-core products (16x16x16 for the 8-input layer,
// 16x16x32 for the 64-wide ones) and the activations as B.  With that
// orientation the 16x16 FP32 result tile a lane holds (column = its lane mod
// 16, rows 4*(lane/16)+j) supplies the B fragment the next layer needs (with
// the K order of mlp_khid), so activations never leave registers between
// layers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace moss {

constexpr int kMlpIn = 8, kMlpH = 64;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;   // 4801
constexpr int kMlpNorm = 4 * kMlpIn;
constexpr int kOffW1 = 0, kOffB1 = 512, kOffW2 = 576, kOffB2 = 4672, kOffW3 = 4736, kOffB3 = 4800;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));

// float -> bfloat16 bits, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// GELU, tanh form (Hendrycks & Gimpel 2016), written as
//   g(x) = 0.5 x (1 + tanh u) = x / (1 + e^{-2u}),  u = sqrt(2/pi) (x + 0.044715 x^3),
// with e^{-2u} = 2^{x (c0 + c1 x^2)}: five VALU operations, one exp2, one rcp.
// For large |x| the exp2 saturates to 0 or +inf and g tends to x or -0.
__device__ __forceinline__ float gelu_fast(float x)
{
    constexpr float kLog2e = 1.4426950408889634f;
    constexpr float c0 = -2.0f * 0.7978845608028654f * kLog2e;
    constexpr float c1 = -2.0f * 0.7978845608028654f * 0.044715f * kLog2e;
    const float p = __builtin_fmaf(x * x, c1, c0);
    const float e = __builtin_amdgcn_exp2f(x * p);
    return x * __builtin_amdgcn_rcpf(1.0f + e);
}

// Input preparation: the three distances (leader gap, red stop line, lane
// end; inputs 0, 4, 6) enter as ln(max(x, 0.5 m)), the other inputs as they
// are; then z = (x' - mean) * inv_std.  The envelope applies to the raw x.
__device__ __forceinline__ float mlp_in(int q, float x, const float *norm)
{
    const float xt = (q == 0 || q == 4 || q == 6) ? logf(fmaxf(x, 0.5f)) : x;
    return (xt - norm[q]) * norm[kMlpIn + q];
}

// Hidden-unit order of the K dimension in the 16x16x32 products.  Lane group
// g (= lane / 16) supplies elements e = 0..7 of K block kb; with
//   hidden(kb, g, e) = 32 kb + 4 g + e          (e < 4)
//                      32 kb + 16 + 4 g + e - 4  (e >= 4)
// the four values a lane holds of each of two consecutive 16-row result
// tiles of the previous layer form its B fragment directly.  The weight
// rows are stored in the same order (A fragment = one 16-byte LDS read).
__host__ __device__ constexpr int mlp_khid(int p)      // p = 32 kb + 8 g + e
{
    return 32 * (p >> 5) + ((p & 7) < 4 ? 4 * ((p >> 3) & 3) + (p & 7)
                                         : 16 + 4 * ((p >> 3) & 3) + (p & 7) - 4);
}

constexpr int kW2Stride = kMlpH + 8;    // padded row (bf16): 144 B, no bank aliasing of rows

// Network image in the layout the kernels read: bfloat16 weights in the K
// order above, FP32 biases and input description.  Built once per network
// (in global memory at creation, or directly in LDS) by mlp_pack.
struct __attribute__((aligned(16))) MlpLds {
    uint16_t W2[kMlpH * kW2Stride];   // [out][K position], padded
    uint16_t W1[kMlpH * kMlpIn];      // [hidden][input]
    uint16_t w3[kMlpH];               // [K position]
    float b1[kMlpH], b2[kMlpH];
    float norm[kMlpNorm];
    float b3, pad_[3];
};
static_assert(sizeof(MlpLds) % 16 == 0, "MlpLds is copied in 16-byte units");

// Cooperative build of the image from the FP32 parameters (all threads of
// the block).
__device__ __forceinline__ void mlp_pack(MlpLds &w, const float *theta, const float *norm)
{
    for (int q = threadIdx.x; q < kMlpH * kW2Stride; q += blockDim.x) {
        const int o = q / kW2Stride, p = q - o * kW2Stride;
        w.W2[q] = p < kMlpH ? f2bf(theta[kOffW2 + o * kMlpH + mlp_khid(p)]) : (uint16_t)0;
    }
    for (int q = threadIdx.x; q < kMlpH * kMlpIn; q += blockDim.x)
        w.W1[q] = f2bf(theta[kOffW1 + q]);
    for (int q = threadIdx.x; q < kMlpH; q += blockDim.x) {
        w.w3[q] = f2bf(theta[kOffW3 + mlp_khid(q)]);
        w.b1[q] = theta[kOffB1 + q];
        w.b2[q] = theta[kOffB2 + q];
    }
    for (int q = threadIdx.x; q < kMlpNorm; q += blockDim.x)
        w.norm[q] = norm[q];
    if (threadIdx.x == 0) {
        w.b3 = theta[kOffB3];
        w.pad_[0] = w.pad_[1] = w.pad_[2] = 0.0f;
    }
}

// Cooperative copy of a packed image from global memory (all threads).
__device__ __forceinline__ void mlp_copy(MlpLds &w, const MlpLds *g)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(g);
    uint4 *dst = reinterpret_cast<uint4 *>(&w);
    for (int q = threadIdx.x; q < (int)(sizeof(MlpLds) / 16); q += blockDim.x)
        dst[q] = src[q];
}

__device__ __forceinline__ bf16x8 cvt8(const f32x4 &a, const f32x4 &b)
{
    const f32x8 v = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    return __builtin_convertvector(v, bf16x8);
}

__device__ __forceinline__ f32x4 gelu4(f32x4 c)
{
    return f32x4{gelu_fast(c.x), gelu_fast(c.y), gelu_fast(c.z), gelu_fast(c.w)};
}

// Staging elements of one wave's network inputs (64 vehicles x 8 inputs as
// bfloat16 pairs).
constexpr int kMlpStage = 64 * 2 * kMlpIn;

// Network output for the 64 vehicles of a wave: lane L passes the
// normalised inputs z[8] of its vehicle and receives that vehicle's output.
// zs is this wave's kMlpStage-element bfloat16 staging area in LDS.  Every
// thread of the block must call it (it synchronises the block; inactive
// vehicles pass zeros).  The wave works through its four 16-vehicle blocks
// one at a time; biases enter as the accumulators' initial values.
//
// Inputs as bfloat16 pairs: the first product has K = 16 for 8 inputs, so
// its second half carries the rounding remainders, z = bf16(z) +
// bf16(z - bf16(z)), against a second copy of W1.  Relative input precision
// is about 2^-16 instead of 2^-8 at no extra cost; it matters where IDM's
// interaction term (s*/gap)^2 is large, which amplifies small gap and speed
// errors.
__device__ __forceinline__ float wave_mlp(const MlpLds &w, uint16_t *zs, const float z[8])
{
    const int lane = __lane_id();
    const int r16 = lane & 15, q4 = lane >> 4;
    {
        const f32x4 z0 = {z[0], z[1], z[2], z[3]}, z1 = {z[4], z[5], z[6], z[7]};
        const bf16x8 hi = cvt8(z0, z1);
        f32x4 r0, r1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r0[k] = z0[k] - (float)hi[k];
            r1[k] = z1[k] - (float)hi[4 + k];
        }
        bf16x8 *dst = reinterpret_cast<bf16x8 *>(zs + lane * 2 * kMlpIn);
        dst[0] = hi;
        dst[1] = cvt8(r0, r1);
    }
    __syncthreads();

    const bf16x8 zero8 = {};
    // layer-1 weights (A fragments: lane groups 0-1 and 2-3 hold the same W1
    // columns, against the high and low parts of the inputs) and bias rows
    bf16x4 a1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
        a1[mt] = *reinterpret_cast<const bf16x4 *>(w.W1 + (16 * mt + r16) * kMlpIn + 4 * (q4 & 1));
    float out = 0.0f;
#pragma unroll 1
    for (int nt = 0; nt < 4; ++nt) {
        // layer 1: H1^T[16 hidden][16 veh] per tile mt
        const bf16x4 bz = *reinterpret_cast<const bf16x4 *>(zs + (16 * nt + r16) * 2 * kMlpIn + 4 * q4);
        f32x4 g[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const f32x4 b = *reinterpret_cast<const f32x4 *>(w.b1 + 16 * mt + 4 * q4);
            g[mt] = gelu4(__builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[mt], bz, b, 0, 0, 0));
        }
        const bf16x8 h1[2] = {cvt8(g[0], g[1]), cvt8(g[2], g[3])};
        // layer 2 per pair of 16-row output tiles, then layer 3 (row 0 = w3)
        // on the pair
        f32x4 y = {w.b3, w.b3, w.b3, w.b3};
#pragma unroll 1
        for (int kb3 = 0; kb3 < 2; ++kb3) {
            f32x4 h2[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int mo = 2 * kb3 + h;
                f32x4 c = *reinterpret_cast<const f32x4 *>(w.b2 + 16 * mo + 4 * q4);
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(w.W2 + (16 * mo + r16) * kW2Stride + 32 * kb + 8 * q4);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, h1[kb], c, 0, 0, 0);
                }
                h2[h] = gelu4(c);
            }
            const bf16x8 a3 = (r16 == 0) ? *reinterpret_cast<const bf16x8 *>(w.w3 + 32 * kb3 + 8 * q4)
                                         : zero8;
            y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, cvt8(h2[0], h2[1]), y, 0, 0, 0);
        }
        // output row 0 of this vehicle block: lanes 0..15, element x
        const float yn = __shfl(y.x, r16);
        if (q4 == nt)
            out = yn;
    }
    return out;
}

}  // namespace moss
