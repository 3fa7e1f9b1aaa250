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
// A operand of v_mfma_f32_16x16x16_bf16 and the activations as B.  With that
// orientation the 16x16 FP32 result tile a lane holds (column = its lane mod
// 16, rows 4*(lane/16)+j) is exactly the B fragment the next layer needs, so
// activations never leave registers between layers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace moss {

constexpr int kMlpIn = 8, kMlpH = 64;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH + 1;   // 4801
constexpr int kMlpNorm = 4 * kMlpIn;
constexpr int kOffW1 = 0, kOffB1 = 512, kOffW2 = 576, kOffB2 = 4672, kOffW3 = 4736, kOffB3 = 4800;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// GELU, tanh form (Hendrycks & Gimpel 2016), with tanh(u) = 1 - 2/(1 + e^{2u})
__device__ __forceinline__ float gelu_fast(float x)
{
    const float u = 0.7978845608f * (x + 0.044715f * (x * x * x));
    const float e = __expf(2.0f * u);
    const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
    return 0.5f * x * (1.0f + t);
}

// Input preparation: the three distances (leader gap, red stop line, lane
// end; inputs 0, 4, 6) enter as ln(max(x, 0.5 m)), the other inputs as they
// are; then z = (x' - mean) * inv_std.  The envelope applies to the raw x.
__device__ __forceinline__ float mlp_in(int q, float x, const float *norm)
{
    const float xt = (q == 0 || q == 4 || q == 6) ? logf(fmaxf(x, 0.5f)) : x;
    return (xt - norm[q]) * norm[kMlpIn + q];
}

// Weights of one block, converted to bfloat16 once per block.
struct MlpLds {
    uint16_t W1[kMlpH * kMlpIn];   // [hidden][input]
    uint16_t W2[kMlpH * kMlpH];    // [out][in]
    uint16_t w3[kMlpH];
    float b1[kMlpH], b2[kMlpH], b3;
    float norm[kMlpNorm];
};

// Cooperative load of the parameters into LDS (all threads of the block).
__device__ __forceinline__ void mlp_load(MlpLds &w, const float *theta, const float *norm)
{
    for (int q = threadIdx.x; q < kMlpH * kMlpIn; q += blockDim.x)
        w.W1[q] = f2bf(theta[kOffW1 + q]);
    for (int q = threadIdx.x; q < kMlpH * kMlpH; q += blockDim.x)
        w.W2[q] = f2bf(theta[kOffW2 + q]);
    for (int q = threadIdx.x; q < kMlpH; q += blockDim.x) {
        w.w3[q] = f2bf(theta[kOffW3 + q]);
        w.b1[q] = theta[kOffB1 + q];
        w.b2[q] = theta[kOffB2 + q];
    }
    for (int q = threadIdx.x; q < kMlpNorm; q += blockDim.x)
        w.norm[q] = norm[q];
    if (threadIdx.x == 0)
        w.b3 = theta[kOffB3];
}

__device__ __forceinline__ bf16x4 load4(const uint16_t *p)
{
    bf16x4 r;
    r.x = (short)p[0];
    r.y = (short)p[1];
    r.z = (short)p[2];
    r.w = (short)p[3];
    return r;
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d)
{
    bf16x4 r;
    r.x = (short)f2bf(a);
    r.y = (short)f2bf(b);
    r.z = (short)f2bf(c);
    r.w = (short)f2bf(d);
    return r;
}

// Network output for the 64 vehicles of a wave: lane L passes the
// normalised inputs z[8] of its vehicle and receives that vehicle's output.
// zs is this wave's 64*8 bfloat16 staging area in LDS.  Every thread of the
// block must call it (it synchronises the block; inactive vehicles pass
// zeros).
__device__ __forceinline__ float wave_mlp(const MlpLds &w, uint16_t *zs, const float z[8])
{
    const int lane = __lane_id();
    const int r16 = lane & 15, q4 = lane >> 4;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k)
        zs[lane * kMlpIn + k] = f2bf(z[k]);
    __syncthreads();

    const bf16x4 zero4 = {0, 0, 0, 0};
    const f32x4 zf = {0.0f, 0.0f, 0.0f, 0.0f};
    // layer 1: H1^T[hidden][veh] = W1[hidden][in16] * Z^T[in16][veh]
    bf16x4 h1[4][4];      // [k-block of hidden][vehicle block]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const bf16x4 bz = (q4 < 2) ? load4(zs + (16 * nt + r16) * kMlpIn + 4 * q4) : zero4;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x4 aw = (q4 < 2) ? load4(w.W1 + (16 * mt + r16) * kMlpIn + 4 * q4) : zero4;
            f32x4 c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aw, bz, zf, 0, 0, 0);
            const int hr = 16 * mt + 4 * q4;
            h1[mt][nt] = pack4(gelu_fast(c.x + w.b1[hr]), gelu_fast(c.y + w.b1[hr + 1]),
                               gelu_fast(c.z + w.b1[hr + 2]), gelu_fast(c.w + w.b1[hr + 3]));
        }
    }
    // layers 2 and 3: H2^T = W2 * H1^T, then y = w3 * H2^T one hidden block at a time
    f32x4 y[4] = {zf, zf, zf, zf};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        bf16x4 a2[4];
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
            a2[kt] = load4(w.W2 + (16 * mt + r16) * kMlpH + 16 * kt + 4 * q4);
        const bf16x4 a3 = (r16 == 0) ? load4(w.w3 + 16 * mt + 4 * q4) : zero4;
        const int hr = 16 * mt + 4 * q4;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 c = zf;
#pragma unroll
            for (int kt = 0; kt < 4; ++kt)
                c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[kt], h1[kt][nt], c, 0, 0, 0);
            const bf16x4 h2 = pack4(gelu_fast(c.x + w.b2[hr]), gelu_fast(c.y + w.b2[hr + 1]),
                                    gelu_fast(c.z + w.b2[hr + 2]), gelu_fast(c.w + w.b2[hr + 3]));
            y[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3, h2, y[nt], 0, 0, 0);
        }
    }
    // row 0 of output block nt sits in lanes 0..15, element x
    const float y0 = __shfl(y[0].x, r16), y1 = __shfl(y[1].x, r16);
    const float y2 = __shfl(y[2].x, r16), y3 = __shfl(y[3].x, r16);
    const float out = (q4 == 0) ? y0 : (q4 == 1) ? y1 : (q4 == 2) ? y2 : y3;
    return out + w.b3;
}

}  // namespace moss
