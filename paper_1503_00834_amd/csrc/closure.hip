// Kernels of the learned subgrid closure that are not part of the SD
// residual: packing the network for the bfloat16 matrix cores, FP32
// training (forward, backward, Adam) and the per-element filter that makes
// training targets from a higher-order solution.  The fused inference
// lives with the residual kernels.
//
// Training is a sequence of small fixed-order kernels (no atomics), so a
// run is bitwise reproducible:
//   k_fwd_bwd    one wave per 16 samples, every layer on the FP32 matrix
//                cores: forward pass, loss terms, and the pre-activation
//                gradients dZ1, dZ2, dY (activations and gradients kept per
//                sample, [t][64] rows; the GELU derivatives stay in
//                registers)
//   k_wgrad      one block per chunk of 64 samples: the chunk's partial
//                weight and bias gradients and its loss as matrix-core
//                products over the chunk's samples
//   k_wgrad_sum  chunk partials summed (the gradient alone)
//   k_wgrad_sum_adam  chunk partials summed and the Adam update (Kingma &
//                Ba 2015, with bias correction) applied at once (training)
// (every sum in a fixed order: the matrix-core products in their instruction
// order, the other sums as four interleaved running sums, then pairwise)
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"
#include "mlp_bf16.hpp"

namespace chorus {

// parameter vector offsets
constexpr int kW1 = 0, kB1 = 1280, kW2 = 1344, kB2 = 5440, kW3 = 5504, kB3 = 6464;
static_assert(kB3 + kMlpOut == kMlpParams, "parameter layout");

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_pack(const float *__restrict__ W, const float *__restrict__ norm,
                                             unsigned char *__restrict__ model) {
    const int lane = threadIdx.x, g = lane >> 4, r = lane & 15;
    bool ok = true;
    for (int q = lane; q < kMlpParams; q += 64) ok = ok && isfinite(W[q]);
    for (int q = lane; q < 70; q += 64) ok = ok && isfinite(norm[q]);
    uint32_t *fr = reinterpret_cast<uint32_t *>(model);
    for (int f = 0; f < kMlpFrags; ++f) {
        float a[8];
        for (int i = 0; i < 8; ++i) {
            float v = 0.0f;
            if (f < 4) {
                const int row = 16 * f + r, k = 8 * g + i;
                v = (k < kMlpIn) ? W[kW1 + row * kMlpIn + k] : 0.0f;
            } else if (f < 12) {
                const int mt = (f - 4) >> 1, ks = (f - 4) & 1;
                v = W[kW2 + (16 * mt + r) * kMlpHid + mlp_kperm(ks, g, i)];
            } else {
                const int ks = f - 12;
                v = (r < kMlpOut) ? W[kW3 + r * kMlpHid + mlp_kperm(ks, g, i)] : 0.0f;
            }
            a[i] = v;
        }
        uint32_t *dst = fr + (f * 64 + lane) * 4;
        for (int w = 0; w < 4; ++w) dst[w] = bf16_pair(a[2 * w], a[2 * w + 1]);
    }
    float *fl = reinterpret_cast<float *>(model + kMlpFloatOff);
    for (int q = lane; q < kMlpNFloat; q += 64) {
        float v = 0.0f;
        if (q < kMlpB2) v = W[kB1 + q];
        else if (q < kMlpB3) v = W[kB2 + q - kMlpB2];
        else if (q < kMlpXMean) v = (q - kMlpB3 < kMlpOut) ? W[kB3 + q - kMlpB3] : 0.0f;
        else if (q < kMlpXInv) v = norm[q - kMlpXMean];
        else if (q < kMlpYMean) v = norm[20 + q - kMlpXInv];
        else if (q < kMlpYStd) v = (q - kMlpYMean < kMlpOut) ? norm[40 + q - kMlpYMean] : 0.0f;
        else v = (q - kMlpYStd < kMlpOut) ? norm[55 + q - kMlpYStd] : 0.0f;
        fl[q] = v;
    }
    const bool all_ok = __all(ok);
    if (lane == 0) reinterpret_cast<int *>(model + kMlpFlagOff)[0] = all_ok ? 1 : 0;
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
// GELU h = z Phi(z) and its derivative Phi(z) + z phi(z) in FP32, with
// erf by the rational approximation 7.1.26 of Abramowitz and Stegun (as in
// the inference; |error| <= 1.5e-7, the size of an FP32 rounding at these
// magnitudes; hardware reciprocal and exponential): with x = |z| / sqrt 2,
// 1 - erf(x) = t (a1 + a2 t + ... + a5 t^4) exp(-x^2), t = 1 / (1 + p x);
// exp(-x^2) = exp(-z^2 / 2) is also the normal density's factor, so one
// exponential serves both
__device__ __forceinline__ void gelu_and_prime(float z, float &h, float &gp) {
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, az, 1.0f));
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(z * z * (-0.5f * 1.4426950408889634f));
    const float tail = 0.5f * q * t * e;            // Phi(-|z|)
    const float Phi = (z >= 0.0f) ? 1.0f - tail : tail;
    h = z * Phi;
    gp = fmaf(z * 0.39894228040143268f, e, Phi);
}

// One wave per 16 samples: every layer as FP32 matrix-core products
// (v_mfma_f32_16x16x4f32) with hidden units as rows and the wave's samples as
// columns.  Operand layout of the instruction (A 16 x 4, B 4 x 16, C 16 x
// 16): lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and C[4 (l / 16) +
// i][l % 16], i = 0..3.  A layer's accumulator (lane l: units 16 mt + 4 (l /
// 16) + i of sample l % 16) serves as the next product's B operand when the
// K steps run over (mt, i): the step (mt, i) takes unit 16 mt + 4 (l / 16) + i
// from lane group l / 16, and the weight operand is read at the same unit,
// so no data moves between lanes.
__global__ __launch_bounds__(64) void k_fwd_bwd(const float *__restrict__ X, const float *__restrict__ Y,
                                                const int32_t *__restrict__ idx, int64_t base, int nb,
                                                const float *__restrict__ W, TrainBufs T) {
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    const int t = blockIdx.x * 16 + c;  // this lane's sample (column)
    const bool ok = t < nb;
    // lanes past the batch compute on its first sample and store nothing
    const int64_t s = idx ? (int64_t)idx[base + (ok ? t : 0)] : base + (ok ? t : 0);
    // layer 1: z1[mt][i] = unit 16 mt + 4 g + i; K = the 20 features
    f32x4_t h1[4], gp1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) h1[mt][i] = W[kB1 + 16 * mt + 4 * g + i];
#pragma unroll
    for (int ks = 0; ks < kMlpIn / 4; ++ks) {
        const float b = X[s * kMlpIn + 4 * ks + g];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            h1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(W[kW1 + (16 * mt + c) * kMlpIn + 4 * ks + g], b, h1[mt],
                                                        0, 0, 0);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float h, gp;
            gelu_and_prime(h1[mt][i], h, gp);
            h1[mt][i] = h;
            gp1[mt][i] = gp;
        }
    // layer 2: K steps over the layer-1 units
    f32x4_t h2[4], gp2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) h2[mt][i] = W[kB2 + 16 * mt + 4 * g + i];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int ki = 0; ki < 4; ++ki) {
            const int k = 16 * kt + 4 * g + ki;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                h2[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(W[kW2 + (16 * mt + c) * kMlpHid + k], h1[kt][ki], h2[mt],
                                                            0, 0, 0);
        }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float h, gp;
            gelu_and_prime(h2[mt][i], h, gp);
            h2[mt][i] = h;
            gp2[mt][i] = gp;
        }
    // layer 3: outputs 4 g + i (row 15 padding)
    f32x4_t y;
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = (4 * g + i < kMlpOut) ? W[kB3 + 4 * g + i] : 0.0f;
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int ki = 0; ki < 4; ++ki) {
            const int k = 16 * kt + 4 * g + ki;
            const float a = (c < kMlpOut) ? W[kW3 + c * kMlpHid + k] : 0.0f;
            y = __builtin_amdgcn_mfma_f32_16x16x4f32(a, h2[kt][ki], y, 0, 0, 0);
        }
    // loss terms and dY
    const float sc = 2.0f / ((float)T.n_mean * (float)kMlpOut);
    f32x4_t dy;
    float l = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * g + i;
        const float e = (k < kMlpOut) ? y[i] - Y[s * kMlpOut + (k < kMlpOut ? k : 0)] : 0.0f;
        l += e * e;
        dy[i] = sc * e;
    }
    // the sample's loss: the four lane groups summed in a fixed order
    const float l1 = __shfl_xor(l, 16), l2 = __shfl_xor(l, 32), l3 = __shfl_xor(l, 48);
    const float lsum = (g == 0) ? (l + l1) + (l2 + l3) : 0.0f;
    // back through layer 3: dH2 = W3^T dY, K = the 16 (15 + padding) outputs
    f32x4_t dz2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) dz2[mt] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ki = 0; ki < 4; ++ki) {
        const int k = 4 * g + ki;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const float a = (k < kMlpOut) ? W[kW3 + (k < kMlpOut ? k : 0) * kMlpHid + 16 * mt + c] : 0.0f;
            dz2[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, dy[ki], dz2[mt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) dz2[mt][i] *= gp2[mt][i];
    // back through layer 2: dH1 = W2^T dZ2
    f32x4_t dz1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) dz1[mt] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int ki = 0; ki < 4; ++ki) {
            const int k = 16 * kt + 4 * g + ki;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
                dz1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(W[kW2 + k * kMlpHid + 16 * mt + c], dz2[kt][ki], dz1[mt],
                                                             0, 0, 0);
        }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) dz1[mt][i] *= gp1[mt][i];
    if (!ok) return;
    // [t][64] rows: four consecutive units per lane and row tile
    const int64_t r64 = (int64_t)t * 64 + 4 * g;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        *reinterpret_cast<f32x4_t *>(T.H1 + r64 + 16 * mt) = h1[mt];
        *reinterpret_cast<f32x4_t *>(T.H2 + r64 + 16 * mt) = h2[mt];
        *reinterpret_cast<f32x4_t *>(T.dZ1 + r64 + 16 * mt) = dz1[mt];
        *reinterpret_cast<f32x4_t *>(T.dZ2 + r64 + 16 * mt) = dz2[mt];
    }
    *reinterpret_cast<f32x4_t *>(T.dY + (int64_t)t * 16 + 4 * g) = dy;
    if (g == 0) T.lossv[t] = lsum;
}

// partial sums over chunk c (samples 64c .. 64c+63) of each parameter's
// gradient and (q = kMlpParams) of the losses: part[c][q].  The weight
// gradients are products over the chunk's samples on the FP32 matrix cores
// (operand layout as in k_fwd_bwd; K = the samples, 16 steps of 4): dW2 =
// dZ2^T H1 (waves 0 and 1, 8 tiles each), dW1 = dZ1^T X (wave 2, features
// padded to 32), dW3 = dY^T H2 (wave 3, outputs padded to 16).  The bias
// gradients are the same products with a column of ones (feature 20 of the
// padded X; one more column tile for dW2 and dW3), and the loss rides in
// the padding row 15 of dY^T.  Samples past the batch enter as zeros.
__global__ __launch_bounds__(256) void k_wgrad(const float *__restrict__ X, const int32_t *__restrict__ idx,
                                               int64_t base, int nb, TrainBufs T) {
    const int c = blockIdx.x, w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int t0 = 64 * c, t1 = min(nb, t0 + 64);
    float *part = T.part + (int64_t)c * (kMlpParams + 1);
    // operand of sample t0 + 4 ks + g: row t of a [t][ld] array at column col
    auto opnd = [&](const float *A, int ld, int ks, int col) {
        const int t = t0 + 4 * ks + g;
        return (t < t1) ? A[(int64_t)t * ld + col] : 0.0f;
    };
    if (w < 2) {
        // dW2[j][k] = sum_t dZ2[t][j] H1[t][k], rows j in tiles 2w, 2w + 1;
        // column tile 4: a column of ones (db2)
        f32x4_t acc[2][5];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int nt = 0; nt < 5; ++nt) acc[a][nt] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        // every operand of the chunk first (one wait), then the products
        float av[16][2], bv[16][4];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
#pragma unroll
            for (int a = 0; a < 2; ++a) av[ks][a] = opnd(T.dZ2, 64, ks, 16 * (2 * w + a) + r);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bv[ks][nt] = opnd(T.H1, 64, ks, 16 * nt + r);
        }
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const float one = (r == 0 && t0 + 4 * ks + g < t1) ? 1.0f : 0.0f;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[a][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][a], bv[ks][nt], acc[a][nt], 0, 0, 0);
                acc[a][4] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][a], one, acc[a][4], 0, 0, 0);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 16 * (2 * w + a) + 4 * g + i;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) part[kW2 + j * kMlpHid + 16 * nt + r] = acc[a][nt][i];
                if (r == 0) part[kB2 + j] = acc[a][4][i];
            }
    } else if (w == 2) {
        // dW1[j][i] = sum_t dZ1[t][j] X[s_t][i]
        f32x4_t acc[4][2];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        // every operand of the chunk first (sample indices, then the rest)
        int64_t smp[16];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int t = t0 + 4 * ks + g;
            const int tc = (t < t1) ? t : t0;
            smp[ks] = idx ? (int64_t)idx[base + tc] : base + tc;
        }
        float av[16][4], bv[16][2];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const bool in = t0 + 4 * ks + g < t1;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) av[ks][mt] = opnd(T.dZ1, 64, ks, 16 * mt + r);
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int f = 16 * nt + r;
                bv[ks][nt] = !in ? 0.0f : (f < kMlpIn) ? X[smp[ks] * kMlpIn + f] : (f == kMlpIn) ? 1.0f : 0.0f;
            }
        }
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks][mt], bv[ks][nt], acc[mt][nt], 0, 0, 0);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int f = 16 * nt + r, j = 16 * mt + 4 * g + i;
                    if (f < kMlpIn) part[kW1 + j * kMlpIn + f] = acc[mt][nt][i];
                    else if (f == kMlpIn) part[kB1 + j] = acc[mt][nt][i];
                }
    } else {
        // dW3[k][j] = sum_t dY[t][k] H2[t][j]; row 15 carries the sample
        // losses, column tile 4 a column of ones (db3 and the loss)
        f32x4_t acc[5];
#pragma unroll
        for (int nt = 0; nt < 5; ++nt) acc[nt] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
        float av[16], bv[16][4];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            av[ks] = (r < kMlpOut) ? opnd(T.dY, 16, ks, r) : opnd(T.lossv, 1, ks, 0);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) bv[ks][nt] = opnd(T.H2, 64, ks, 16 * nt + r);
        }
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks], bv[ks][nt], acc[nt], 0, 0, 0);
            const float one = (r == 0 && t0 + 4 * ks + g < t1) ? 1.0f : 0.0f;
            acc[4] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ks], one, acc[4], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            if (k < kMlpOut) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) part[kW3 + k * kMlpHid + 16 * nt + r] = acc[nt][i];
                if (r == 0) part[kB3 + k] = acc[4][i];
            } else if (r == 0) {
                part[kMlpParams] = acc[4][i];
            }
        }
    }
}

// sum over the chunks of quantity q in a fixed order: four running sums on
// four lanes (lane 4 q' + r sums chunks r, r + 4, ... in turn), combined
// pairwise as (s0 + s1) + (s2 + s3)
__device__ __forceinline__ float chunk_sum(int nchunk, const float *__restrict__ part, int q) {
    const int r = threadIdx.x & 3;
    float a = 0.0f;
    // 16 chunks per lane and round, every load of a round issued first
    for (int c0 = r; c0 < nchunk; c0 += 64) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = c0 + 4 * u;
            v[u] = part[(int64_t)(c < nchunk ? c : r) * (kMlpParams + 1) + q];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (c0 + 4 * u < nchunk) a += v[u];
    }
    const float p = a + __shfl_xor(a, 1);
    return p + __shfl_xor(p, 2);
}

// four lanes per quantity (parameter, or the loss for q = kMlpParams)
__global__ __launch_bounds__(64) void k_wgrad_sum(int nchunk, const float *__restrict__ part, int64_t n_mean,
                                                  float *__restrict__ grad, float *__restrict__ loss) {
    const int qq = (blockIdx.x * 64 + (int)threadIdx.x) >> 2, q = qq <= kMlpParams ? qq : kMlpParams;
    const float s = chunk_sum(nchunk, part, q);
    if ((threadIdx.x & 3) != 0 || qq > kMlpParams) return;
    if (q < kMlpParams) grad[q] = s;
    else loss[0] = s / ((float)n_mean * (float)kMlpOut);
}

__device__ __forceinline__ void adam_update(float *__restrict__ W, float *__restrict__ m, float *__restrict__ v,
                                            float g, const AdamArgs &a, int q) {
    const float mq = a.b1 * m[q] + (1.0f - a.b1) * g;
    const float vq = a.b2 * v[q] + (1.0f - a.b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    W[q] -= a.lr * (mq * a.inv_bc1) / (sqrtf(vq * a.inv_bc2) + a.eps);
}

__global__ __launch_bounds__(64) void k_wgrad_sum_adam(int nchunk, const float *__restrict__ part, int64_t n_mean,
                                                       float *__restrict__ W, float *__restrict__ m,
                                                       float *__restrict__ v, AdamArgs a, float *__restrict__ loss) {
    const int qq = (blockIdx.x * 64 + (int)threadIdx.x) >> 2, q = qq <= kMlpParams ? qq : kMlpParams;
    const float s = chunk_sum(nchunk, part, q);
    if ((threadIdx.x & 3) != 0 || qq > kMlpParams) return;
    if (q < kMlpParams) adam_update(W, m, v, s, a, q);
    else loss[0] = s / ((float)n_mean * (float)kMlpOut);
}

// ---------------------------------------------------------------------------
// filter: per element L2 projection of |J| U to degree Nc - 1
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cart_flux(const double q[5], double gm1, double F[15]) {
    const double r = q[0], m[3] = {q[1], q[2], q[3]}, E = q[4];
    const double ir = 1.0 / r;
    const double p = gm1 * (E - 0.5 * (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) * ir);
    for (int c = 0; c < 3; ++c) {
        F[c] = m[c];
        for (int i = 0; i < 3; ++i) F[3 * (1 + i) + c] = m[i] * m[c] * ir + (i == c ? p : 0.0);
        F[12 + c] = (E + p) * m[c] * ir;
    }
}

__global__ __launch_bounds__(64) void k_filter(FilterArgs A) {
    constexpr int MAXF = 6, MAXC = 3;
    __shared__ double U[20][MAXF * MAXF * MAXF];   // |J| Q (5) and |J| F(Q) (15) at the fine points
    __shared__ double T1[20][MAXC * MAXF * MAXF];  // after the xi pass
    __shared__ double T2[20][MAXC * MAXC * MAXF];  // after the eta pass
    const int64_t e = blockIdx.x;
    const int nf = A.nf, nc = A.nc, NPF = nf * nf * nf, NPC = nc * nc * nc;
    const double gm1 = A.gamma - 1.0;
    for (int p = threadIdx.x; p < NPF; p += 64) {
        double q[5], F[15];
        for (int v = 0; v < 5; ++v) q[v] = A.Qf[((int64_t)v * A.E + e) * NPF + p];
        const double J = 1.0 / A.solgeo_f[(e * 13 + 9) * NPF + p];
        cart_flux(q, gm1, F);
        for (int v = 0; v < 5; ++v) U[v][p] = J * q[v];
        for (int k = 0; k < 15; ++k) U[5 + k][p] = J * F[k];
    }
    __syncthreads();
    // xi: (a, j, k) <- sum_i P[a][i] U(i, j, k)
    for (int it = threadIdx.x; it < 20 * nc * nf * nf; it += 64) {
        const int f = it / (nc * nf * nf), r = it % (nc * nf * nf), a = r % nc, jk = r / nc;
        double s = 0.0;
        for (int i = 0; i < nf; ++i) s += A.P[a][i] * U[f][i + nf * jk];
        T1[f][a + nc * jk] = s;
    }
    __syncthreads();
    // eta: (a, b, k) <- sum_j P[b][j] T1(a, j, k)
    for (int it = threadIdx.x; it < 20 * nc * nc * nf; it += 64) {
        const int f = it / (nc * nc * nf), r = it % (nc * nc * nf), a = r % nc, b = (r / nc) % nc, k = r / (nc * nc);
        double s = 0.0;
        for (int j = 0; j < nf; ++j) s += A.P[b][j] * T1[f][a + nc * (j + nf * k)];
        T2[f][a + nc * (b + nc * k)] = s;
    }
    __syncthreads();
    // zeta, divide by the coarse |J|, subgrid flux
    for (int p = threadIdx.x; p < NPC; p += 64) {
        const int a = p % nc, b = (p / nc) % nc, c = p / (nc * nc);
        double g[20];
        for (int f = 0; f < 20; ++f) {
            double s = 0.0;
            for (int k = 0; k < nf; ++k) s += A.P[c][k] * T2[f][a + nc * (b + nc * k)];
            g[f] = s;
        }
        const double iJ = A.solgeo_c[(e * 13 + 9) * NPC + p];
        double qb[5], F[15];
        for (int v = 0; v < 5; ++v) qb[v] = g[v] * iJ;
        cart_flux(qb, gm1, F);
        for (int v = 0; v < 5; ++v) A.Qbar[((int64_t)v * A.E + e) * NPC + p] = qb[v];
        for (int k = 0; k < 15; ++k)
            A.tau[((int64_t)k * A.E + e) * NPC + p] = (k < 3) ? 0.0 : g[5 + k] * iJ - F[k];
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_pack(const float *W, const float *norm, unsigned char *model, hipStream_t s) {
    hipLaunchKernelGGL(k_pack, dim3(1), dim3(64), 0, s, W, norm, model);
    return hipGetLastError();
}

// forward/backward and the chunk partials of the gradient and the loss
static hipError_t launch_train_partials(const float *X, const float *Y, const int32_t *idx, int64_t base, int nb,
                                        const float *W, const TrainBufs &T, hipStream_t s) {
    const int nchunk = (nb + 63) / 64;
    hipLaunchKernelGGL(k_fwd_bwd, dim3((nb + 15) / 16), dim3(64), 0, s, X, Y, idx, base, nb, W, T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad, dim3(nchunk), dim3(256), 0, s, X, idx, base, nb, T);
    return hipGetLastError();
}

hipError_t launch_train_grad(const float *X, const float *Y, const int32_t *idx, int64_t base, int nb,
                             const float *W, const TrainBufs &T, float *grad, float *loss, hipStream_t s) {
    hipError_t e = launch_train_partials(X, Y, idx, base, nb, W, T, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_sum, dim3((4 * (kMlpParams + 1) + 63) / 64), dim3(64), 0, s, (nb + 63) / 64,
                       (const float *)T.part, T.n_mean, grad, loss);
    return hipGetLastError();
}

hipError_t launch_train_step(const float *X, const float *Y, const int32_t *idx, int64_t base, int nb, float *W,
                             float *m, float *v, const TrainBufs &T, const AdamArgs &a, float *loss, hipStream_t s) {
    hipError_t e = launch_train_partials(X, Y, idx, base, nb, W, T, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_sum_adam, dim3((4 * (kMlpParams + 1) + 63) / 64), dim3(64), 0, s, (nb + 63) / 64,
                       (const float *)T.part, T.n_mean, W, m, v, a, loss);
    return hipGetLastError();
}

// flag[0] = 1 if a sample index lies outside [0, n) (flag cleared first)
__global__ __launch_bounds__(256) void k_check_idx(const int32_t *__restrict__ idx, int64_t count, int64_t n,
                                                   int *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const int32_t v = idx[i];
    if (v < 0 || v >= n) flag[0] = 1;
}

hipError_t launch_check_idx(const int32_t *idx, int64_t count, int64_t n, int *flag, hipStream_t s) {
    hipError_t e = launch_clear_flag(flag, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_check_idx, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, idx, count, n, flag);
    return hipGetLastError();
}

hipError_t launch_filter(const FilterArgs &A, hipStream_t s) {
    hipLaunchKernelGGL(k_filter, dim3((unsigned)A.E), dim3(64), 0, s, A);
    return hipGetLastError();
}

}  // namespace chorus
