// pd_mlp_dev.h -- device code of the closure's MLP on the matrix cores,
// shared by the standalone forward (training, checks) and the fused step of
// the reduced learned closure: bfloat16 conversion, the activation, and one
// 16-row block's three layers on v_mfma_f32_16x16x32_bf16.
#pragma once

#include "pd_internal.h"

namespace pd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }

__device__ __forceinline__ float dsilu_f(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// the MLP on one 16-row block, on the matrix cores (v_mfma_f32_16x16x32_bf16:
// lane l holds A[l % 16][8 (l / 16) + t] and B[8 (l / 16) + t][l % 16],
// t = 0..7, and receives D[4 (l / 16) + t][l % 16], t = 0..3).  The NW
// wavefronts of a workgroup split the output columns of each layer (256 / NW
// hidden units each; the two 16-column tiles of the last layer go to waves 0
// and 1) and the layers meet in LDS, as bfloat16 rows padded by 16 bytes so
// that the 16 rows of an operand load fall in different banks.
// ---------------------------------------------------------------------------
constexpr int kXsStride = kClModes + 8;   // LDS row strides, bfloat16 elements
constexpr int kHStride = kClHidden + 8;

// eight consecutive bfloat16 values (16-byte aligned) as one MFMA operand
__device__ __forceinline__ bf16x8 load8(const uint16_t *p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// one wavefront's weight fragments and biases, read in fragment order (one
// contiguous 1 KB load per wavefront operand)
template <int NW>
struct MlpWave {
    static constexpr int TPW = kClHidden / 16 / NW;  // hidden column tiles per wave
    bf16x8 w1[TPW][kClModes / 32], w2[TPW][kClHidden / 32], w3[kClHidden / 32];
    float b1[TPW], b2[TPW], b3;
};

template <int NW>
__device__ __forceinline__ void mlp_load(MlpWave<NW> &W, const uint16_t *F, const float *Wf, int wv,
                                         int l) {
    constexpr int TPW = MlpWave<NW>::TPW;
    const int r = l & 15;
    auto frag = [&](int base, int f) { return load8(F + base + f * kFragElems + 8 * l); };
#pragma unroll
    for (int jj = 0; jj < TPW; ++jj) {
        const int tile = TPW * wv + jj;
#pragma unroll
        for (int ks = 0; ks < kClModes / 32; ++ks) W.w1[jj][ks] = frag(kFragW1, tile * (kClModes / 32) + ks);
        W.b1[jj] = Wf[kOffB1 + 16 * tile + r];
    }
#pragma unroll
    for (int jj = 0; jj < TPW; ++jj) {
        const int tile = TPW * wv + jj;
#pragma unroll
        for (int ks = 0; ks < kClHidden / 32; ++ks) W.w2[jj][ks] = frag(kFragW2, tile * (kClHidden / 32) + ks);
        W.b2[jj] = Wf[kOffB2 + 16 * tile + r];
    }
    W.b3 = 0.0f;
    if (wv < kClModes / 16) {
#pragma unroll
        for (int ks = 0; ks < kClHidden / 32; ++ks) W.w3[ks] = frag(kFragW3, wv * (kClHidden / 32) + ks);
        W.b3 = Wf[kOffB3 + 16 * wv + r];
    }
}

// a hidden layer: Hout = bfloat16(silu(Hin W^T + b)) on this wave's column
// tiles; the pre-activation and the activation also go to the training
// caches zc, hc (rows first .. first + cnt - 1) when given
template <int TPW, int KS>
__device__ __forceinline__ void mlp_hidden(const uint16_t *Hin, int in_stride,
                                           const bf16x8 (&w)[TPW][KS], const float (&b)[TPW],
                                           uint16_t *Hout, int wv, int l, int first, int cnt,
                                           float *zc, uint16_t *hc) {
    const int r = l & 15, kq = 4 * (l >> 4), k8 = 8 * (l >> 4);
    bf16x8 ah[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) ah[ks] = load8(Hin + r * in_stride + 32 * ks + k8);
#pragma unroll
    for (int jj = 0; jj < TPW; ++jj) {
        const int n = 16 * (TPW * wv + jj) + r;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) acc = mfma32(ah[ks], w[jj][ks], acc);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = kq + t;
            const float z = acc[t] + b[jj];
            const uint16_t h = f2bf(silu_f(z));
            Hout[row * kHStride + n] = h;
            if (zc && row < cnt) {
                zc[(size_t)(first + row) * kClHidden + n] = z;
                hc[(size_t)(first + row) * kClHidden + n] = h;
            }
        }
    }
}

// the last layer (waves 0 and 1): y[kq + t] of column 16 wv + l % 16
template <int NW>
__device__ __forceinline__ f32x4 mlp_out(const uint16_t *H2, const MlpWave<NW> &W, int l) {
    const int r = l & 15, k8 = 8 * (l >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kClHidden / 32; ++ks)
        acc = mfma32(load8(H2 + r * kHStride + 32 * ks + k8), W.w3[ks], acc);
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] += W.b3;
    return acc;
}

}  // namespace pd
