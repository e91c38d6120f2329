// Device code of the start-proposal network shared by the step kernels and
// the training kernels: parameter layout, bfloat16 rounding, the matrix-core
// forward pass and the chart-table lookup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slw {

// Offsets in the FP32 parameter vector: W1 (5 x 64), b1, W2 (64 x 64), b2,
// W3 (64 x 2), b3; W stored input-major (W[i][j] at i * n_out + j); a layer
// computes act(h W + b).
constexpr int kOW1 = 0, kOB1 = 320, kOW2 = 384, kOB2 = 4480, kOW3 = 4544, kOB3 = 4672;
// bfloat16 operand pack: 4 (layer 1) + 16 (layer 2) + 4 (layer 3) blocks of
// 64 lanes x 4 values; biases in accumulator order: b1 (64), b2 (64), b3 padded to 16
constexpr int kWpackHalves = 24 * 64 * 4;
constexpr int kBiasFloats = 144;

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline uint16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even (finite inputs)
    return (uint16_t)(u >> 16);
}

__device__ inline bf16x4_t pack4(float a, float b, float c, float d)
{
    bf16x4_t r;
    r[0] = (short)to_bf16(a);
    r[1] = (short)to_bf16(b);
    r[2] = (short)to_bf16(c);
    r[3] = (short)to_bf16(d);
    return r;
}

// features normalised in FP32: (f - shift) * scale
__device__ inline void mlp_normalise(const float *__restrict__ norm, float f[5])
{
#pragma unroll
    for (int i = 0; i < 5; ++i)
        f[i] = (f[i] - norm[i]) * norm[5 + i];
}

// Forward pass for the 64 points of a wavefront on the matrix cores
// (v_mfma_f32_16x16x16_bf16: bfloat16 operands, FP32 accumulation).  The
// transposed products H^T = W^T X^T put the points along N, so a layer's
// accumulator layout (lane l holds rows 4 (l / 16) .. + 3 of column l % 16)
// is the next layer's B-operand layout: activations stay in registers.
// feat: this lane's normalised features; returns this lane's outputs.
// Every lane of the wavefront must call it.
__device__ inline float2 mlp_forward_wave(const uint16_t *__restrict__ wpack, const float *__restrict__ bias,
                                          const float feat[5])
{
    const int l = threadIdx.x & 63;
    const int grp = l >> 4, col = l & 15;
    const bf16x4_t *A1 = (const bf16x4_t *)wpack;  // [mt][lane]
    const bf16x4_t *A2 = A1 + 4 * 64;              // [mt2][kk][lane]
    const bf16x4_t *A3 = A2 + 16 * 64;             // [kk][lane]
    float u_nt[4], v_nt[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        // layer-1 B operand: features 4 grp .. 4 grp + 3 of point 16 nt + col
        const int src = 16 * nt + col;
        float f[5];
#pragma unroll
        for (int i = 0; i < 5; ++i)
            f[i] = __shfl(feat[i], src, 64);
        const bf16x4_t b0 = grp == 0 ? pack4(f[0], f[1], f[2], f[3])
                                     : (grp == 1 ? pack4(f[4], 0.f, 0.f, 0.f) : pack4(0.f, 0.f, 0.f, 0.f));
        bf16x4_t B1[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const float4 bb = *(const float4 *)(bias + 16 * mt + 4 * grp);
            f32x4_t acc = {bb.x, bb.y, bb.z, bb.w};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A1[mt * 64 + l], b0, acc, 0, 0, 0);
            B1[mt] = pack4(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f), fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
        }
        bf16x4_t B2[4];
#pragma unroll
        for (int mt2 = 0; mt2 < 4; ++mt2) {
            const float4 bb = *(const float4 *)(bias + 64 + 16 * mt2 + 4 * grp);
            f32x4_t acc = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A2[(mt2 * 4 + kk) * 64 + l], B1[kk], acc, 0, 0, 0);
            B2[mt2] = pack4(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f), fmaxf(acc[2], 0.f), fmaxf(acc[3], 0.f));
        }
        const float4 bb = *(const float4 *)(bias + 128 + 4 * grp);
        f32x4_t acc = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A3[kk * 64 + l], B2[kk], acc, 0, 0, 0);
        // lanes 0..15 hold outputs 0 and 1 of points 16 nt .. 16 nt + 15
        u_nt[nt] = acc[0];
        v_nt[nt] = acc[1];
    }
    float u = 0.f, v = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float uu = __shfl(u_nt[nt], col, 64), vv = __shfl(v_nt[nt], col, 64);
        if (grp == nt) {
            u = uu;
            v = vv;
        }
    }
    return make_float2(u, v);
}

// chart coordinates -> start triangle (internal id) through the G x G table;
// outputs are clamped to [0, 1) (a NaN output lands in cell 0)
__device__ inline int32_t chart_lookup(const int32_t *__restrict__ table, int g, float2 uv)
{
    const float u = fminf(fmaxf(uv.x, 0.f), 0.99999994f), v = fminf(fmaxf(uv.y, 0.f), 0.99999994f);
    const int bu = min((int)(u * (float)g), g - 1), bv = min((int)(v * (float)g), g - 1);
    return table[bu * g + bv];
}

}  // namespace slw
