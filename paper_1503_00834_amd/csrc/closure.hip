// Kernels of the learned subgrid closure that are not part of the SD
// residual: packing the network for the bfloat16 matrix cores, FP32
// training (forward, backward, Adam) and the per-element filter that makes
// training targets from a higher-order solution.  The fused inference
// lives with the residual kernels.
//
// Training is a sequence of small fixed-order kernels (no atomics), so a
// run is bitwise reproducible:
//   k_fwd_bwd    a block of eight waves per 64 samples (lane = sample, wave
//                = an eighth of the hidden units of every layer): forward
//                pass, loss terms, and the pre-activation gradients dZ1,
//                dZ2, dY (activations and gradients kept per sample, [t][64]
//                rows; the GELU derivatives stay in registers)
//   k_wgrad      one thread per (parameter or loss, chunk of 64 samples):
//                partial sums of the outer products and of the losses
//   k_wgrad_sum  chunk partials summed (the gradient alone)
//   k_wgrad_sum_adam  chunk partials summed and the Adam update (Kingma &
//                Ba 2015, with bias correction) applied at once (training)
// (every sum in a fixed order: four interleaved running sums, then pairwise)
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
__device__ __forceinline__ float gelu_prime_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

constexpr int kTrainWaves = 8;  // waves per 64 samples in the forward/backward pass

__global__ __launch_bounds__(64 * kTrainWaves) void k_fwd_bwd(const float *__restrict__ X, const float *__restrict__ Y,
                                                 const int32_t *__restrict__ idx, int64_t base, int nb,
                                                 const float *__restrict__ W, TrainBufs T) {
    constexpr int NW = kTrainWaves, QU = kMlpHid / NW;  // hidden units per wave
    __shared__ float sh1[kMlpHid][64];              // h1[unit][sample]
    __shared__ float syq[NW][kMlpOut][64];          // layer-3 sums over each wave's units
    __shared__ float sdz2[kMlpHid][64];             // dz2[unit][sample]
    const int lane = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int t = blockIdx.x * 64 + lane;
    const bool ok = t < nb;
    // lanes past the batch compute on its first sample and store nothing
    const int64_t s = idx ? (int64_t)idx[base + (ok ? t : 0)] : base + (ok ? t : 0);
    float x[kMlpIn];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) x[i] = X[s * kMlpIn + i];
    float *H1 = T.H1 + (int64_t)t * 64, *H2 = T.H2 + (int64_t)t * 64;
    // layer 1, this wave's units
    float g1[QU];
#pragma unroll
    for (int jj = 0; jj < QU; ++jj) {
        const int j = QU * q + jj;
        float z = W[kB1 + j];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) z += W[kW1 + j * kMlpIn + i] * x[i];
        const float h = gelu_f(z);
        g1[jj] = gelu_prime_f(z);
        sh1[j][lane] = h;
        if (ok) H1[j] = h;
    }
    __syncthreads();
    // layer 2, this wave's units, and their share of layer 3
    float g2[QU], yq[kMlpOut];
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k) yq[k] = 0.0f;
#pragma unroll 4
    for (int jj = 0; jj < QU; ++jj) {
        const int j = QU * q + jj;
        float z = W[kB2 + j];
#pragma unroll
        for (int k = 0; k < kMlpHid; ++k) z += W[kW2 + j * kMlpHid + k] * sh1[k][lane];
        const float h = gelu_f(z);
        g2[jj] = gelu_prime_f(z);
        if (ok) H2[j] = h;
#pragma unroll
        for (int k = 0; k < kMlpOut; ++k) yq[k] += W[kW3 + k * kMlpHid + j] * h;
    }
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k) syq[q][k][lane] = yq[k];
    __syncthreads();
    // outputs, loss and dY (every wave forms them for its own backward pass)
    float l = 0.0f, dy[kMlpOut];
    const float sc = 2.0f / ((float)T.n_mean * (float)kMlpOut);
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k) {
        float p[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) p[w] = syq[w][k][lane];
#pragma unroll
        for (int h = NW / 2; h > 0; h /= 2)  // pairwise, fixed order
#pragma unroll
            for (int w = 0; w < h; ++w) p[w] += p[w + h];
        const float y = W[kB3 + k] + p[0];
        const float e = y - Y[s * kMlpOut + k];
        l += e * e;
        dy[k] = sc * e;
    }
    if (q == 0 && ok) {
#pragma unroll
        for (int k = 0; k < kMlpOut; ++k) T.dY[(int64_t)t * 16 + k] = dy[k];
        T.lossv[t] = l;
    }
    // back through layer 3 to this wave's layer-2 units:
    // dZ2_j = (sum_k W3[k][j] dY_k) gelu'(z2_j)
    float *dZ2 = T.dZ2 + (int64_t)t * 64, *dZ1 = T.dZ1 + (int64_t)t * 64;
#pragma unroll
    for (int jj = 0; jj < QU; ++jj) {
        const int j = QU * q + jj;
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < kMlpOut; ++k) a += W[kW3 + k * kMlpHid + j] * dy[k];
        const float dz = a * g2[jj];
        sdz2[j][lane] = dz;
        if (ok) dZ2[j] = dz;
    }
    __syncthreads();
    // back through layer 2 to this wave's layer-1 units:
    // dZ1_k = (sum_j W2[j][k] dZ2_j) gelu'(z1_k)
#pragma unroll 4
    for (int kk = 0; kk < QU; ++kk) {
        const int k = QU * q + kk;
        float dh = 0.0f;
#pragma unroll
        for (int j = 0; j < kMlpHid; ++j) dh += W[kW2 + j * kMlpHid + k] * sdz2[j][lane];
        if (ok) dZ1[k] = dh * g1[kk];
    }
}

// sum of f(t) for t0 <= t < t1 in a fixed order: four interleaved running
// sums (t = t0 + 4u + r in sum r), combined pairwise
template <typename Fn>
__device__ __forceinline__ float fixed_sum(int t0, int t1, Fn f) {
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    int t = t0;
    for (; t + 3 < t1; t += 4) {
        a0 += f(t);
        a1 += f(t + 1);
        a2 += f(t + 2);
        a3 += f(t + 3);
    }
    if (t < t1) a0 += f(t);
    if (t + 1 < t1) a1 += f(t + 1);
    if (t + 2 < t1) a2 += f(t + 2);
    return (a0 + a1) + (a2 + a3);
}

// partial sums over chunk c (samples 64c .. 64c+63) of each parameter's
// gradient and (q = kMlpParams) of the losses: part[c][q]
__global__ __launch_bounds__(64) void k_wgrad(const float *__restrict__ X, const int32_t *__restrict__ idx,
                                              int64_t base, int nb, TrainBufs T) {
    const int q = blockIdx.x * 64 + threadIdx.x, c = blockIdx.y;
    if (q > kMlpParams) return;
    const int t0 = 64 * c, t1 = min(nb, t0 + 64);
    float s;
    if (q == kMlpParams) {
        s = fixed_sum(t0, t1, [&](int t) { return T.lossv[t]; });
    } else if (q < kB1) {
        const int j = q / kMlpIn, i = q % kMlpIn;
        s = fixed_sum(t0, t1, [&](int t) {
            const int64_t smp = idx ? (int64_t)idx[base + t] : base + t;
            return T.dZ1[(int64_t)t * 64 + j] * X[smp * kMlpIn + i];
        });
    } else if (q < kW2) {
        const int j = q - kB1;
        s = fixed_sum(t0, t1, [&](int t) { return T.dZ1[(int64_t)t * 64 + j]; });
    } else if (q < kB2) {
        const int j = (q - kW2) / kMlpHid, k = (q - kW2) % kMlpHid;
        s = fixed_sum(t0, t1, [&](int t) { return T.dZ2[(int64_t)t * 64 + j] * T.H1[(int64_t)t * 64 + k]; });
    } else if (q < kW3) {
        const int j = q - kB2;
        s = fixed_sum(t0, t1, [&](int t) { return T.dZ2[(int64_t)t * 64 + j]; });
    } else if (q < kB3) {
        const int k = (q - kW3) / kMlpHid, j = (q - kW3) % kMlpHid;
        s = fixed_sum(t0, t1, [&](int t) { return T.dY[(int64_t)t * 16 + k] * T.H2[(int64_t)t * 64 + j]; });
    } else {
        const int k = q - kB3;
        s = fixed_sum(t0, t1, [&](int t) { return T.dY[(int64_t)t * 16 + k]; });
    }
    T.part[(int64_t)c * (kMlpParams + 1) + q] = s;
}

__global__ __launch_bounds__(64) void k_wgrad_sum(int nchunk, const float *__restrict__ part, int64_t n_mean,
                                                  float *__restrict__ grad, float *__restrict__ loss) {
    const int q = blockIdx.x * 64 + threadIdx.x;
    if (q > kMlpParams) return;
    const float s = fixed_sum(0, nchunk, [&](int c) { return part[(int64_t)c * (kMlpParams + 1) + q]; });
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
    const int q = blockIdx.x * 64 + threadIdx.x;
    if (q > kMlpParams) return;
    const float s = fixed_sum(0, nchunk, [&](int c) { return part[(int64_t)c * (kMlpParams + 1) + q]; });
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
    hipLaunchKernelGGL(k_fwd_bwd, dim3(nchunk), dim3(64 * kTrainWaves), 0, s, X, Y, idx, base, nb, W, T);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad, dim3((kMlpParams + 1 + 63) / 64, nchunk), dim3(64), 0, s, X, idx, base, nb, T);
    return hipGetLastError();
}

hipError_t launch_train_grad(const float *X, const float *Y, const int32_t *idx, int64_t base, int nb,
                             const float *W, const TrainBufs &T, float *grad, float *loss, hipStream_t s) {
    hipError_t e = launch_train_partials(X, Y, idx, base, nb, W, T, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_sum, dim3((kMlpParams + 1 + 63) / 64), dim3(64), 0, s, (nb + 63) / 64,
                       (const float *)T.part, T.n_mean, grad, loss);
    return hipGetLastError();
}

hipError_t launch_train_step(const float *X, const float *Y, const int32_t *idx, int64_t base, int nb, float *W,
                             float *m, float *v, const TrainBufs &T, const AdamArgs &a, float *loss, hipStream_t s) {
    hipError_t e = launch_train_partials(X, Y, idx, base, nb, W, T, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wgrad_sum_adam, dim3((kMlpParams + 1 + 63) / 64), dim3(64), 0, s, (nb + 63) / 64,
                       (const float *)T.part, T.n_mean, W, m, v, a, loss);
    return hipGetLastError();
}

hipError_t launch_filter(const FilterArgs &A, hipStream_t s) {
    hipLaunchKernelGGL(k_filter, dim3((unsigned)A.E), dim3(64), 0, s, A);
    return hipGetLastError();
}

}  // namespace chorus
