// Mixed-precision SD kernels (gfx950): FP64 state and SSP-RK3 accumulation,
// FP32 interpolation, fluxes and derivatives on perturbations about a
// hydrostatic background at rest (Q0 with zero momentum).
//
// Split of the residual (exact algebra, rounding aside):
//   R(Q) = R0 + dR,   R0 = inviscid + source residual of Q0 (computed once in
//   FP64 by the FP64 kernels, stored as FP32), and
//   dR   = [inviscid + source](Q) - [inviscid + source](Q0) + viscous(Q).
// The inviscid difference is evaluated without cancellation from the
// perturbation P = Q - Q0:
//   mass      m'.S
//   momentum  m' (m'.S)/rho + p' S,        p' = (g-1)(E' - |m'|^2 / (2 rho))
//   energy    (gamma E0 + E' + p') (m'.S)/rho
//   Rusanov   1/2 (dF_L + dF_R) - 1/2 |S| [lam (P_R - P_L) + (lam - lam0)(Q0_R - Q0_L)]
//   source    M(P) (M is linear in Q)
// so FP32 rounding is relative to perturbation sizes; the viscous residual
// (scaled by nu, kappa) is evaluated from the full state in FP32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"
#include "sd_common.hpp"

namespace chorus {

template <int N>
using OpsF = OpsT<float, N>;

// ---------------------------------------------------------------------------
// pointwise perturbation fluxes
// ---------------------------------------------------------------------------
// (F(Q) - F(Q0)) . S with m0 = 0, from the full density and energy and the
// perturbation momentum and energy
__device__ __forceinline__ void dflux_inviscid(float rho, const float m[3], float E, float Ep,
                                               const float S[3], float gm1, float gam, float out[5]) {
    const float inv = 1.0f / rho;
    const float mS = m[0] * S[0] + m[1] * S[1] + m[2] * S[2];
    const float mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    const float pp = gm1 * (Ep - 0.5f * mm * inv);
    const float uS = mS * inv;
    out[0] = mS;
    out[1] = m[0] * uS + pp * S[0];
    out[2] = m[1] * uS + pp * S[1];
    out[3] = m[2] * uS + pp * S[2];
    out[4] = (gam * E - gm1 * Ep + pp) * uS;
}

// viscous part of the wall flux (normal traction only, energy flux
// F_bottom |S| at the inner wall, interior diffusive flux at the outer wall),
// returned with the sign of a flux: (0, -tau_nn S, -e)
__device__ __forceinline__ void flux_wall_viscous(const float q[5], const float g[5][3], const float S[3],
                                                  bool outer, const PhysParams &P, float out[5]) {
    PrimGrad<float> pg;
    prim_grad(q, g, P, pg);
    const float mu = pg.rho * (float)P.nu;
    const float div = pg.du[0][0] + pg.du[1][1] + pg.du[2][2];
    const float A2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
    float ngn = 0.0f;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) ngn += S[a] * pg.du[a][b] * S[b];
    const float tnn = mu * (2.0f * ngn / A2 - (2.0f / 3.0f) * div);
    float ev;
    if (outer) {
        const float dSS = pg.dS[0] * S[0] + pg.dS[1] * S[1] + pg.dS[2] * S[2];
        const float dTS = pg.dT[0] * S[0] + pg.dT[1] * S[1] + pg.dT[2] * S[2];
        ev = (float)P.kappa * pg.rho * pg.Tmp * dSS + (float)P.kappa_r * pg.rho * (float)P.cp * dTS;
    } else {
        ev = (float)P.F_bottom * sqrtf(A2);
    }
    out[0] = 0.0f;
    for (int a = 0; a < 3; ++a) out[1 + a] = -tnn * S[a];
    out[4] = -ev;
}

// ---------------------------------------------------------------------------
// views
// ---------------------------------------------------------------------------
struct GeoF {
    const float *solgeo;   // [E][13][NP]
    const float *fluxgeo;  // [E][3][3][NFL]
    const int32_t *link;   // [E][6]
    const int32_t *info;   // [E][6]
    int64_t E;
};

struct MixedBufs {
    const float *bg;    // [E][2][NP]  rho0, E0 at solution points
    const float *bgT;   // [E][6][2][NF2] rho0, E0 face traces (FP64 interpolation, rounded)
    const float *R0;    // [5][E][NP]  background residual
};

// sol-point field slots in LDS: full rho, m' (3), full E, rho', E'
enum { F_RHO = 0, F_MX = 1, F_MY = 2, F_MZ = 3, F_E = 4, F_RP = 5, F_EP = 6, NFIELD = 7 };

template <int N, int EPB, int NT>
__device__ __forceinline__ void load_fields(const double *__restrict__ Pq, const MixedBufs &B, int64_t E,
                                            int64_t e0, float (*sf)[NFIELD][N * N * N]) {
    constexpr int NP = N * N * N;
    for (int it = threadIdx.x; it < EPB * NP; it += NT) {
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= E) {
            sf[el][F_RHO][p] = 1.0f;
            sf[el][F_MX][p] = sf[el][F_MY][p] = sf[el][F_MZ][p] = 0.0f;
            sf[el][F_E][p] = 1.0f;
            sf[el][F_RP][p] = sf[el][F_EP][p] = 0.0f;
            continue;
        }
        const double pr = Pq[(0 * E + e) * NP + p], pe = Pq[(4 * E + e) * NP + p];
        const float r0 = B.bg[(e * 2 + 0) * NP + p], E0 = B.bg[(e * 2 + 1) * NP + p];
        sf[el][F_RHO][p] = (float)((double)r0 + pr);
        sf[el][F_MX][p] = (float)Pq[(1 * E + e) * NP + p];
        sf[el][F_MY][p] = (float)Pq[(2 * E + e) * NP + p];
        sf[el][F_MZ][p] = (float)Pq[(3 * E + e) * NP + p];
        sf[el][F_E][p] = (float)((double)E0 + pe);
        sf[el][F_RP][p] = (float)pr;
        sf[el][F_EP][p] = (float)pe;
    }
}

// neighbour face data: perturbation trace (5) and background trace (2)
template <int N, int EPB, int NT>
__device__ __forceinline__ void load_neighbours(const GeoF &G, const MixedBufs &B, const float *__restrict__ TQ,
                                                int64_t e0, float (*snb)[6][7][N * N]) {
    constexpr int NF2 = N * N;
    for (int it = threadIdx.x; it < EPB * 6 * 7 * NF2; it += NT) {
        const int el = it / (6 * 7 * NF2), r = it % (6 * 7 * NF2);
        const int f = r / (7 * NF2), v = (r / NF2) % 7, pn = r % NF2;
        const int64_t e = e0 + el;
        float val = 0.0f;
        if (e < G.E) {
            const int32_t nb = G.link[e * 6 + f];
            if (nb >= 0) {
                const int f2 = G.info[e * 6 + f] & 7;
                val = (v < 5) ? TQ[(((int64_t)nb * 6 + f2) * 5 + v) * NF2 + pn]
                              : B.bgT[(((int64_t)nb * 6 + f2) * 2 + (v - 5)) * NF2 + pn];
            }
        }
        snb[el][f][v][pn] = val;  // stored in the neighbour's point order
    }
}

// own face values of the listed sol fields at face point (f, t1, t2)
template <int N>
__device__ __forceinline__ float face_interp(const OpsF<N> &op, const float *fld, int f, int t1, int t2) {
    const int d = f >> 1, m = (f & 1) ? N : 0;
    const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b < N; ++b) s += op.I[m][b] * fld[base + b * st];
    return s;
}

// full state on both sides of face point (f, pp): own from interpolation,
// neighbour from its traces; also the own perturbation and background.
struct FaceStates {
    float qL[5], qR[5];     // full
    float pL[5], pR[5];     // perturbation
    float r0L, E0L, r0R, E0R;
};

template <int N>
__device__ __forceinline__ void face_states(const OpsF<N> &op, const float (*sf)[N * N * N],
                                            const float (*nbf)[N * N], int o, int f, int t1, int t2,
                                            FaceStates &s) {
    const float rho = face_interp<N>(op, sf[F_RHO], f, t1, t2);
    const float E = face_interp<N>(op, sf[F_E], f, t1, t2);
    s.pL[0] = face_interp<N>(op, sf[F_RP], f, t1, t2);
    s.pL[4] = face_interp<N>(op, sf[F_EP], f, t1, t2);
    for (int a = 0; a < 3; ++a) s.pL[1 + a] = face_interp<N>(op, sf[F_MX + a], f, t1, t2);
    s.qL[0] = rho;
    s.qL[1] = s.pL[1];
    s.qL[2] = s.pL[2];
    s.qL[3] = s.pL[3];
    s.qL[4] = E;
    s.r0L = rho - s.pL[0];
    s.E0L = E - s.pL[4];
    const int pn = map_face_point<N>(o, t1, t2);
    for (int v = 0; v < 5; ++v) s.pR[v] = nbf[v][pn];
    s.r0R = nbf[5][pn];
    s.E0R = nbf[6][pn];
    s.qR[0] = s.r0R + s.pR[0];
    s.qR[1] = s.pR[1];
    s.qR[2] = s.pR[2];
    s.qR[3] = s.pR[3];
    s.qR[4] = s.E0R + s.pR[4];
}

// BR1 common solution (full variables) at every face point
template <int N, int EPB, int NT>
__device__ __forceinline__ void common_solution_mixed(const OpsF<N> &op, const GeoF &G, const PhysParams &P,
                                                      int64_t e0, float (*sf)[NFIELD][N * N * N],
                                                      float (*snb)[6][7][N * N], float (*sqs)[6][5][N * N]) {
    constexpr int NF2 = N * N, NFL = (N + 1) * N * N;
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int t1 = pp % N, t2 = pp / N;
        const int32_t nb = G.link[e * 6 + f], inf = G.info[e * 6 + f];
        const int bc = (inf >> 6) - 1;
        float qs[5];
        if (nb >= 0) {
            FaceStates s;
            face_states<N>(op, sf[el], snb[el][f], (inf >> 3) & 7, f, t1, t2, s);
            for (int v = 0; v < 5; ++v) qs[v] = 0.5f * (s.qL[v] + s.qR[v]);
        } else {
            float q[5];
            q[0] = face_interp<N>(op, sf[el][F_RHO], f, t1, t2);
            for (int a = 0; a < 3; ++a) q[1 + a] = face_interp<N>(op, sf[el][F_MX + a], f, t1, t2);
            q[4] = face_interp<N>(op, sf[el][F_E], f, t1, t2);
            const int d = f >> 1, m = (f & 1) ? N : 0;
            const int fl = m + (N + 1) * (t1 + N * t2);
            const float sg = (f & 1) ? 1.0f : -1.0f;
            float S[3];
            for (int c = 0; c < 3; ++c) S[c] = sg * G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
            wall_state(q, S, bc == CHORUS_BC_OUTER, P, qs);
        }
        for (int v = 0; v < 5; ++v) sqs[el][f][v][pp] = qs[v];
    }
}

// gradients of the full conserved variables at the solution points
template <int N, int EPB, int NT>
__device__ __forceinline__ void gradients_mixed(const OpsF<N> &op, const GeoF &G, int64_t e0,
                                                float (*sf)[NFIELD][N * N * N], float (*sqs)[6][5][N * N],
                                                float (*sgr)[15][N * N * N]) {
    constexpr int NP = N * N * N;
    for (int it = threadIdx.x; it < EPB * NP; it += NT) {
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        float dq[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d), pp = t1 + N * t2;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                float s = op.D[a][0] * sqs[el][2 * d][v][pp] + op.D[a][N] * sqs[el][2 * d + 1][v][pp];
#pragma unroll
                for (int b = 0; b < N; ++b) s += op.B[a][b] * sf[el][v][base + b * st];
                dq[d][v] = s;
            }
        }
        const float *gs = G.solgeo + e * 13 * NP + p;
        float Gm[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) Gm[t] = gs[t * NP];
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                sgr[el][v * 3 + c][p] = Gm[c] * dq[0][v] + Gm[3 + c] * dq[1][v] + Gm[6 + c] * dq[2][v];
    }
}

// gradient at a flux point (m along d) by interpolation along the line
template <int N>
__device__ __forceinline__ void grad_at(const OpsF<N> &op, const float (*gr)[N * N * N], int m, int base, int st,
                                        float g[5][3]) {
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float t = 0.0f;
#pragma unroll
            for (int b = 0; b < N; ++b) t += op.I[m][b] * gr[v * 3 + c][base + b * st];
            g[v][c] = t;
        }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// P = Q - Q0 (FP64) and the FP32 face traces of P
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_pert_begin(OpsF<N> op, GeoF G, const double *__restrict__ Q,
                                                   const double *__restrict__ Q0, double *__restrict__ Pq,
                                                   float *__restrict__ TQ) {
    constexpr int NP = N * N * N, NF2 = N * N;
    __shared__ float sp[EPB][5][NP];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    for (int it = threadIdx.x; it < EPB * 5 * NP; it += NT) {
        const int el = it / (5 * NP), r = it % (5 * NP), v = r / NP, p = r % NP;
        const int64_t e = e0 + el;
        float val = 0.0f;
        if (e < G.E) {
            const int64_t gi = ((int64_t)v * G.E + e) * NP + p;
            const double d = Q[gi] - Q0[gi];
            Pq[gi] = d;
            val = (float)d;
        }
        sp[el][v][p] = val;
    }
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        for (int v = 0; v < 5; ++v)
            TQ[((e * 6 + f) * 5 + v) * NF2 + pp] = face_interp<N>(op, sp[el][v], f, pp % N, pp / N);
    }
}

// viscous flux of the own side (full state, FP32) at interior interface
// points along the outward area vector: TV[e][f][v][pp]
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_grad_mixed(OpsF<N> op, GeoF G, MixedBufs B, PhysParams P,
                                                   const double *__restrict__ Pq, const float *__restrict__ TQ,
                                                   float *__restrict__ TV) {
    constexpr int NP = N * N * N, NF2 = N * N, NFL = (N + 1) * N * N;
    __shared__ float sf[EPB][NFIELD][NP];
    __shared__ float snb[EPB][6][7][NF2];
    __shared__ float sqs[EPB][6][5][NF2];
    __shared__ float sgr[EPB][15][NP];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    load_neighbours<N, EPB, NT>(G, B, TQ, e0, snb);
    load_fields<N, EPB, NT>(Pq, B, G.E, e0, sf);
    __syncthreads();
    common_solution_mixed<N, EPB, NT>(op, G, P, e0, sf, snb, sqs);
    __syncthreads();
    gradients_mixed<N, EPB, NT>(op, G, e0, sf, sqs, sgr);
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E || G.link[e * 6 + f] < 0) continue;
        const int d = f >> 1, m = (f & 1) ? N : 0, t1 = pp % N, t2 = pp / N;
        const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        float q[5], g[5][3];
        q[0] = face_interp<N>(op, sf[el][F_RHO], f, t1, t2);
        for (int a = 0; a < 3; ++a) q[1 + a] = face_interp<N>(op, sf[el][F_MX + a], f, t1, t2);
        q[4] = face_interp<N>(op, sf[el][F_E], f, t1, t2);
        grad_at<N>(op, sgr[el], m, base, st, g);
        const int fl = m + (N + 1) * (t1 + N * t2);
        const float sg = (f & 1) ? 1.0f : -1.0f;
        float S[3], fv[5];
        for (int c = 0; c < 3; ++c) S[c] = sg * G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
        flux_viscous(q, g, S, P, fv);
        for (int v = 0; v < 5; ++v) TV[((e * 6 + f) * 5 + v) * NF2 + pp] = fv[v];
    }
}

struct MixedStage {
    const double *Pn;  // step-start perturbation (may alias Pout)
    double *Pout;      // stage output (or dQ/dt in mode 0)
    float *TQout;      // FP32 face traces of Pout (RK mode)
    double ca, cb, dt;
    int mode;          // 0 residual (R0 + dR), 1 RK stage
};

template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_resid_mixed(OpsF<N> op, GeoF G, MixedBufs B, PhysParams P,
                                                    const double *Pq, const float *__restrict__ TQ,
                                                    const float *__restrict__ TV, MixedStage S_) {
    constexpr int NP = N * N * N, NF2 = N * N, NFL = (N + 1) * N * N;
    __shared__ float sf[EPB][NFIELD][NP];
    __shared__ float snb[EPB][6][7][NF2];
    __shared__ float snv[EPB][6][5][NF2];
    __shared__ float sqs[EPB][6][5][NF2];
    __shared__ float sgr[EPB][15][NP];
    __shared__ float sft[EPB][3][5][NFL];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const float gm1 = (float)(P.gamma - 1.0), gam = (float)P.gamma;
    load_neighbours<N, EPB, NT>(G, B, TQ, e0, snb);
    for (int it = threadIdx.x; it < EPB * 6 * 5 * NF2; it += NT) {
        const int el = it / (6 * 5 * NF2), r = it % (6 * 5 * NF2);
        const int f = r / (5 * NF2), v = (r / NF2) % 5, pn = r % NF2;
        const int64_t e = e0 + el;
        float val = 0.0f;
        if (e < G.E) {
            const int32_t nb = G.link[e * 6 + f];
            if (nb >= 0) val = TV[(((int64_t)nb * 6 + (G.info[e * 6 + f] & 7)) * 5 + v) * NF2 + pn];
        }
        snv[el][f][v][pn] = val;
    }
    load_fields<N, EPB, NT>(Pq, B, G.E, e0, sf);
    __syncthreads();
    common_solution_mixed<N, EPB, NT>(op, G, P, e0, sf, snb, sqs);
    __syncthreads();
    gradients_mixed<N, EPB, NT>(op, G, e0, sf, sqs, sgr);
    __syncthreads();
    // transformed perturbation flux at every flux point of all directions
    for (int it = threadIdx.x; it < EPB * 3 * NFL; it += NT) {
        const int el = it / (3 * NFL), r = it % (3 * NFL), d = r / NFL, fl = r % NFL;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int m = fl % (N + 1), t1 = (fl / (N + 1)) % N, t2 = fl / ((N + 1) * N);
        const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        float Sv[3], F[5];
        for (int c = 0; c < 3; ++c) Sv[c] = G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
        float g[5][3];
        grad_at<N>(op, sgr[el], m, base, st, g);
        if (m > 0 && m < N) {
            float q[5], Ep = 0.0f;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                float s = 0.0f;
#pragma unroll
                for (int b = 0; b < N; ++b) s += op.I[m][b] * sf[el][v][base + b * st];
                q[v] = s;
            }
#pragma unroll
            for (int b = 0; b < N; ++b) Ep += op.I[m][b] * sf[el][F_EP][base + b * st];
            float fi[5], fv[5];
            dflux_inviscid(q[0], &q[1], q[4], Ep, Sv, gm1, gam, fi);
            flux_viscous(q, g, Sv, P, fv);
            for (int v = 0; v < 5; ++v) F[v] = fi[v] - fv[v];
        } else {
            const int f = 2 * d + (m == N ? 1 : 0);
            const float sg = (m == N) ? 1.0f : -1.0f;
            float So[3] = {sg * Sv[0], sg * Sv[1], sg * Sv[2]}, phi[5];
            const int32_t nb = G.link[e * 6 + f], inf = G.info[e * 6 + f];
            const int bc = (inf >> 6) - 1;
            if (nb >= 0) {
                FaceStates s;
                const int o = (inf >> 3) & 7;
                face_states<N>(op, sf[el], snb[el][f], o, f, t1, t2, s);
                float fL[5], fR[5], fvL[5];
                dflux_inviscid(s.qL[0], &s.qL[1], s.qL[4], s.pL[4], So, gm1, gam, fL);
                dflux_inviscid(s.qR[0], &s.qR[1], s.qR[4], s.pR[4], So, gm1, gam, fR);
                const float A = sqrtf(So[0] * So[0] + So[1] * So[1] + So[2] * So[2]);
                const float iA = 1.0f / A;
                const float unL = fabsf((s.qL[1] * So[0] + s.qL[2] * So[1] + s.qL[3] * So[2]) * iA / s.qL[0]);
                const float unR = fabsf((s.qR[1] * So[0] + s.qR[2] * So[1] + s.qR[3] * So[2]) * iA / s.qR[0]);
                const float cL = sqrtf(gam * pressure_of(s.qL, gm1) / s.qL[0]);
                const float cR = sqrtf(gam * pressure_of(s.qR, gm1) / s.qR[0]);
                const float c0L = sqrtf(gam * gm1 * s.E0L / s.r0L), c0R = sqrtf(gam * gm1 * s.E0R / s.r0R);
                const float lam = fmaxf(unL + cL, unR + cR), lam0 = fmaxf(c0L, c0R);
                const float hl = 0.5f * lam * A, hd = 0.5f * (lam - lam0) * A;
                const float dq0[5] = {s.r0R - s.r0L, 0.0f, 0.0f, 0.0f, s.E0R - s.E0L};
                for (int v = 0; v < 5; ++v)
                    phi[v] = 0.5f * (fL[v] + fR[v]) - hl * (s.pR[v] - s.pL[v]) - hd * dq0[v];
                flux_viscous(s.qL, g, So, P, fvL);
                const int pn = map_face_point<N>(o, t1, t2);
                for (int v = 0; v < 5; ++v) phi[v] -= 0.5f * (fvL[v] + (-snv[el][f][v][pn]));
            } else {
                // wall: inviscid perturbation (0, p' S, 0) + viscous wall flux
                float q[5], Ep = 0.0f;
                for (int v = 0; v < 5; ++v) {
                    float s = 0.0f;
                    for (int b = 0; b < N; ++b) s += op.I[m][b] * sf[el][v][base + b * st];
                    q[v] = s;
                }
                for (int b = 0; b < N; ++b) Ep += op.I[m][b] * sf[el][F_EP][base + b * st];
                const float mm = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
                const float pp = gm1 * (Ep - 0.5f * mm / q[0]);
                flux_wall_viscous(q, g, So, bc == CHORUS_BC_OUTER, P, phi);
                for (int a = 0; a < 3; ++a) phi[1 + a] += pp * So[a];
            }
            for (int v = 0; v < 5; ++v) F[v] = sg * phi[v];
        }
        for (int v = 0; v < 5; ++v) sft[el][d][v][fl] = F[v];
    }
    __syncthreads();
    // divergence, source, background residual and stage update
    for (int it = threadIdx.x; it < EPB * NP; it += NT) {
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        float div[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int fb = (N + 1) * (t1 + N * t2);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                float s = 0.0f;
#pragma unroll
                for (int mm = 0; mm <= N; ++mm) s += op.D[a][mm] * sft[el][d][v][fb + mm];
                div[v] += s;
            }
        }
        const float *gs = G.solgeo + e * 13 * NP + p;
        const float iJ = gs[9 * NP];
        const float GMf = (float)P.GM, Om = (float)P.omega;
        const float g0 = GMf * gs[10 * NP], g1 = GMf * gs[11 * NP], g2 = GMf * gs[12 * NP];
        const float rp = sf[el][F_RP][p], mx = sf[el][F_MX][p], my = sf[el][F_MY][p], mz = sf[el][F_MZ][p];
        float M[5];
        M[0] = 0.0f;
        M[1] = rp * g0 - 2.0f * Om * my;
        M[2] = rp * g1 + 2.0f * Om * mx;
        M[3] = rp * g2;
        M[4] = mx * g0 + my * g1 + mz * g2;
        float newp[5];
        for (int v = 0; v < 5; ++v) {
            const int64_t gi = ((int64_t)v * G.E + e) * NP + p;
            const double R = (double)B.R0[gi] + (double)(-div[v] * iJ - M[v]);
            if (S_.mode == 0) {
                S_.Pout[gi] = R;
            } else {
                const double pn = (S_.ca != 0.0) ? S_.Pn[gi] : 0.0;
                const double pv = S_.ca * pn + S_.cb * (Pq[gi] + S_.dt * R);
                S_.Pout[gi] = pv;
                newp[v] = (float)pv;
            }
        }
        if (S_.mode != 0) {
            sf[el][F_RP][p] = newp[0];
            sf[el][F_MX][p] = newp[1];
            sf[el][F_MY][p] = newp[2];
            sf[el][F_MZ][p] = newp[3];
            sf[el][F_EP][p] = newp[4];
        }
    }
    if (S_.mode == 0 || S_.TQout == nullptr) return;
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int t1 = pp % N, t2 = pp / N;
        float* out = S_.TQout + (e * 6 + f) * 5 * NF2 + pp;
        out[0 * NF2] = face_interp<N>(op, sf[el][F_RP], f, t1, t2);
        out[1 * NF2] = face_interp<N>(op, sf[el][F_MX], f, t1, t2);
        out[2 * NF2] = face_interp<N>(op, sf[el][F_MY], f, t1, t2);
        out[3 * NF2] = face_interp<N>(op, sf[el][F_MZ], f, t1, t2);
        out[4 * NF2] = face_interp<N>(op, sf[el][F_EP], f, t1, t2);
    }
}

// Q = Q0 + P
__global__ void k_pert_end(const double *__restrict__ Q0, const double *__restrict__ Pq, double *__restrict__ Q,
                           int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Q[i] = Q0[i] + Pq[i];
}

// background setup: rho0, E0 (FP32) at solution points, their face traces
// (FP64 interpolation, rounded), and a flag if Q0 has non-zero momentum
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_bg_setup(Ops<N> op, int64_t E, const double *__restrict__ Q0,
                                                 float *__restrict__ bg, float *__restrict__ bgT,
                                                 int *__restrict__ flag) {
    constexpr int NP = N * N * N, NF2 = N * N;
    __shared__ double s0[EPB][2][NP];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    for (int it = threadIdx.x; it < EPB * NP; it += NT) {
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= E) continue;
        const double r = Q0[(0 * E + e) * NP + p], en = Q0[(4 * E + e) * NP + p];
        const double mx = Q0[(1 * E + e) * NP + p], my = Q0[(2 * E + e) * NP + p], mz = Q0[(3 * E + e) * NP + p];
        if (mx != 0.0 || my != 0.0 || mz != 0.0) flag[0] = 1;
        s0[el][0][p] = r;
        s0[el][1][p] = en;
        bg[(e * 2 + 0) * NP + p] = (float)r;
        bg[(e * 2 + 1) * NP + p] = (float)en;
    }
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= E) continue;
        const int d = f >> 1, m = (f & 1) ? N : 0, t1 = pp % N, t2 = pp / N;
        const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        for (int v = 0; v < 2; ++v) {
            double s = 0.0;
            for (int b = 0; b < N; ++b) s += op.I[m][b] * s0[el][v][base + b * st];
            bgT[((e * 6 + f) * 2 + v) * NF2 + pp] = (float)s;
        }
    }
}

__global__ void k_to_float(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N>
struct CfgM;
template <> struct CfgM<2> { static constexpr int EPB = 8, NT = 64; };
template <> struct CfgM<3> { static constexpr int EPB = 2, NT = 64; };
template <> struct CfgM<4> { static constexpr int EPB = 1, NT = 64; };
template <> struct CfgM<5> { static constexpr int EPB = 1, NT = 128; };
template <> struct CfgM<6> { static constexpr int EPB = 1, NT = 256; };

static GeoF geof_of(const GeoM &g) {
    GeoF o;
    o.solgeo = g.solgeo32;
    o.fluxgeo = g.fluxgeo32;
    o.link = g.link;
    o.info = g.info;
    o.E = g.E;
    return o;
}
static MixedBufs bufs_of(const GeoM &g) {
    MixedBufs b;
    b.bg = g.bg;
    b.bgT = g.bgT;
    b.R0 = g.R0;
    return b;
}

template <int N>
static hipError_t pert_begin_t(const Mesh &m, const GeoM &g, const double *Q, double *Pq, float *TQ, hipStream_t s) {
    constexpr int EPB = CfgM<N>::EPB, NT = CfgM<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_pert_begin<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, make_ops_t<float, N>(m.basis),
                       geof_of(g), Q, g.Q0, Pq, TQ);
    return hipGetLastError();
}
template <int N>
static hipError_t grad_mixed_t(const Mesh &m, const GeoM &g, const PhysParams &P, const double *Pq, const float *TQ,
                               float *TV, hipStream_t s) {
    constexpr int EPB = CfgM<N>::EPB, NT = CfgM<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_grad_mixed<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, make_ops_t<float, N>(m.basis),
                       geof_of(g), bufs_of(g), P, Pq, TQ, TV);
    return hipGetLastError();
}
template <int N>
static hipError_t resid_mixed_t(const Mesh &m, const GeoM &g, const PhysParams &P, const double *Pq,
                                const float *TQ, const float *TV, const MixedStageArgs &a, hipStream_t s) {
    constexpr int EPB = CfgM<N>::EPB, NT = CfgM<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    MixedStage st{a.Pn, a.Pout, a.TQout, a.ca, a.cb, a.dt, a.mode};
    hipLaunchKernelGGL((k_resid_mixed<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, make_ops_t<float, N>(m.basis),
                       geof_of(g), bufs_of(g), P, Pq, TQ, TV, st);
    return hipGetLastError();
}
template <int N>
static hipError_t bg_setup_t(const Mesh &m, const double *Q0, float *bg, float *bgT, int *flag, hipStream_t s) {
    constexpr int EPB = CfgM<N>::EPB, NT = CfgM<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_bg_setup<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, make_ops_t<double, N>(m.basis), m.E, Q0,
                       bg, bgT, flag);
    return hipGetLastError();
}

#define CHORUS_DISPATCH_M(N_, CALL)          \
    switch (N_) {                            \
        case 2: return CALL(2);              \
        case 3: return CALL(3);              \
        case 4: return CALL(4);              \
        case 5: return CALL(5);              \
        case 6: return CALL(6);              \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_pert_begin(const Mesh &m, const GeoM &g, const double *Q, double *Pq, float *TQ, hipStream_t s) {
#define C_(n) pert_begin_t<n>(m, g, Q, Pq, TQ, s)
    CHORUS_DISPATCH_M(m.N, C_)
#undef C_
}
hipError_t launch_grad_mixed(const Mesh &m, const GeoM &g, const PhysParams &P, const double *Pq, const float *TQ,
                             float *TV, hipStream_t s) {
#define C_(n) grad_mixed_t<n>(m, g, P, Pq, TQ, TV, s)
    CHORUS_DISPATCH_M(m.N, C_)
#undef C_
}
hipError_t launch_resid_mixed(const Mesh &m, const GeoM &g, const PhysParams &P, const double *Pq, const float *TQ,
                              const float *TV, const MixedStageArgs &a, hipStream_t s) {
#define C_(n) resid_mixed_t<n>(m, g, P, Pq, TQ, TV, a, s)
    CHORUS_DISPATCH_M(m.N, C_)
#undef C_
}
hipError_t launch_bg_setup(const Mesh &m, const double *Q0, float *bg, float *bgT, int *flag, hipStream_t s) {
#define C_(n) bg_setup_t<n>(m, Q0, bg, bgT, flag, s)
    CHORUS_DISPATCH_M(m.N, C_)
#undef C_
}
hipError_t launch_pert_end(const double *Q0, const double *Pq, double *Q, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_pert_end, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Q0, Pq, Q, n);
    return hipGetLastError();
}
hipError_t launch_to_float(const double *a, float *b, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_float, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

}  // namespace chorus
