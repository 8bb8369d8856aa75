// Pointwise subgrid-closure network 20 -> 64 -> 64 -> 15 (GELU) evaluated
// with bfloat16 matrix-core instructions (v_mfma_f32_16x16x32_bf16) and FP32
// accumulation.  The paper names subgrid modelling for large-eddy runs as
// the next step of the code (Summary) and already treats entropy diffusion
// as a parameterisation of unresolved motion (Section 2); this network
// supplies a learned subgrid flux added to the total flux.
//
// The network runs transposed, hidden units as matrix rows and points as
// columns, so each layer's accumulator fragment (lane l: rows 4(l/16)+i of a
// 16-row tile, column l%16) is already the next layer's B fragment (lane l:
// 8 consecutive K values of column l%16) once two row tiles are
// concatenated.  The K order that this produces is folded into the packed
// weights, so no data moves between lanes or through LDS between layers.
//
// Packed model image (built by chorus_closure_pack):
//   14 A fragments of 64 lanes x 8 bf16 (16 B per lane): layer 1 row tiles
//   0..3 (K = features 0..31, 20..31 zero); layer 2 row tile mt, K step ks at
//   4 + 2 mt + ks; layer 3 K steps at 12, 13 (rows 15 zero);
//   then FP32: b1[64], b2[64], b3[16], x_mean[20], x_inv_std[20],
//   y_mean[16], y_std[16]; then an int32 "all finite" flag.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chorus {

constexpr int kMlpIn = 20, kMlpHid = 64, kMlpOut = 15;
constexpr int kMlpParams = kMlpHid * kMlpIn + kMlpHid + kMlpHid * kMlpHid + kMlpHid + kMlpOut * kMlpHid + kMlpOut;
constexpr int kMlpFrags = 14;
constexpr int kMlpFragBytes = 64 * 16;
constexpr int kMlpFloatOff = kMlpFrags * kMlpFragBytes;  // 14336
constexpr int kMlpB1 = 0, kMlpB2 = 64, kMlpB3 = 128, kMlpXMean = 144, kMlpXInv = 164, kMlpYMean = 184,
              kMlpYStd = 200, kMlpNFloat = 216;
constexpr int kMlpFlagOff = kMlpFloatOff + kMlpNFloat * 4;  // 15200
constexpr int kMlpModelBytes = 15360;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// two floats -> two bfloat16 (low half: lo), round to nearest even: one
// packed conversion instruction on gfx950
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{lo, hi}, bf16x2_t));
}

// GELU z Phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2, for the bfloat16
// inference, with erf by the rational
// approximation 7.1.26 of Abramowitz and Stegun (Handbook of Mathematical
// Functions, 1964): erf(x) = 1 - q, q = t (a1 + t (a2 + t (a3 + t (a4 +
// t a5)))) exp(-x^2), t = 1 / (1 + p x) for x >= 0 (odd extension),
// |error| <= 1.5e-7, far below the bfloat16 rounding (2^-9 relative) the
// activations receive.  With x = |z| / sqrt 2 the odd extension folds into
// z Phi(z) = max(z, 0) - |z| q / 2: one reciprocal, one exponential, four
// multiply-adds for the polynomial (coefficients halved) and four more
// operations, no sign handling.
__device__ __forceinline__ float gelu_bf(float z) {
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, az, 1.0f));
    float h = fmaf(0.5f * 1.061405429f, t, 0.5f * -1.453152027f);
    h = fmaf(h, t, 0.5f * 1.421413741f);
    h = fmaf(h, t, 0.5f * -0.284496736f);
    h = fmaf(h, t, 0.5f * 0.254829592f);
    // exp(-z^2 / 2) as a power of two
    const float e = __builtin_amdgcn_exp2f(z * z * (-0.5f * 1.4426950408889634f));
    // max(z, 0) as a signed-integer max of the bit pattern (a negative float
    // is a negative integer): the same value for every non-NaN z, one
    // instruction, where a float max of an accumulator first canonicalises it
    const float zp = __builtin_bit_cast(float, max(__builtin_bit_cast(int, z), 0));
    return fmaf(-az, h * t * e, zp);
}

// K index held by lane group g (= lane / 16), slot i (0..7) of the B
// fragment of K step ks for layers 2 and 3: hidden unit of the previous
// layer's accumulator that lands there
__host__ __device__ constexpr int mlp_kperm(int ks, int g, int i) {
    return 32 * ks + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
}

// Evaluate the network for NT points of one wave: lane l owns point tile
// pt's column l % 16; xb[pt] is the lane's B fragment of normalised
// features (features 8 (l/16) .. +7 of its point).  out[pt][i] receives
// output 4 (l/16) + i of that point (i = 0..3; output 15 is padding).
template <int NPT>
__device__ __forceinline__ void mlp_eval(const unsigned char *__restrict__ model, const u32x4_t (&xb)[NPT],
                                         f32x4_t (&out)[NPT]) {
    const int lane = threadIdx.x & 63, g = lane >> 4;
    const u32x4_t *fr = reinterpret_cast<const u32x4_t *>(model);
    const float *fl = reinterpret_cast<const float *>(model + kMlpFloatOff);
    // layer 1
    u32x4_t h1[2][NPT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x8_t a = __builtin_bit_cast(bf16x8_t, fr[mt * 64 + lane]);
        f32x4_t b;  // bias as the accumulator's initial value
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = fl[kMlpB1 + 16 * mt + 4 * g + i];
#pragma unroll
        for (int pt = 0; pt < NPT; ++pt) {
            const f32x4_t c =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8_t, xb[pt]), b, 0, 0, 0);
            const int ks = mt >> 1, half = (mt & 1) * 2;
            h1[ks][pt][half] = bf16_pair(gelu_bf(c[0]), gelu_bf(c[1]));
            h1[ks][pt][half + 1] = bf16_pair(gelu_bf(c[2]), gelu_bf(c[3]));
        }
    }
    // layer 2
    u32x4_t h2[2][NPT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const bf16x8_t a0 = __builtin_bit_cast(bf16x8_t, fr[(4 + 2 * mt) * 64 + lane]);
        const bf16x8_t a1 = __builtin_bit_cast(bf16x8_t, fr[(5 + 2 * mt) * 64 + lane]);
        f32x4_t b;
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = fl[kMlpB2 + 16 * mt + 4 * g + i];
#pragma unroll
        for (int pt = 0; pt < NPT; ++pt) {
            f32x4_t c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, __builtin_bit_cast(bf16x8_t, h1[0][pt]), b, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, __builtin_bit_cast(bf16x8_t, h1[1][pt]), c, 0, 0, 0);
            const int ks = mt >> 1, half = (mt & 1) * 2;
            h2[ks][pt][half] = bf16_pair(gelu_bf(c[0]), gelu_bf(c[1]));
            h2[ks][pt][half + 1] = bf16_pair(gelu_bf(c[2]), gelu_bf(c[3]));
        }
    }
    // layer 3 (linear) and output scaling
    const bf16x8_t a0 = __builtin_bit_cast(bf16x8_t, fr[12 * 64 + lane]);
    const bf16x8_t a1 = __builtin_bit_cast(bf16x8_t, fr[13 * 64 + lane]);
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
        f32x4_t c = {0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, __builtin_bit_cast(bf16x8_t, h2[0][pt]), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, __builtin_bit_cast(bf16x8_t, h2[1][pt]), c, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            out[pt][i] = fl[kMlpYMean + k] + fl[kMlpYStd + k] * (c[i] + fl[kMlpB3 + k]);
        }
    }
}

// normalised feature -> float (FP64 arithmetic, then rounded to FP32)
__device__ __forceinline__ float mlp_norm_feature(const unsigned char *__restrict__ model, int f, double x) {
    const float *fl = reinterpret_cast<const float *>(model + kMlpFloatOff);
    return (float)((x - (double)fl[kMlpXMean + f]) * (double)fl[kMlpXInv + f]);
}

}  // namespace chorus
