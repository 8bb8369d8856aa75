// HIP kernels (gfx950) of the spectral-difference residual and the SSP-RK3
// update (Section 3 of the paper; SSP-RK3 as the explicit integrator).
//
// One residual evaluation is split in two element passes because BR1 needs
// two neighbour exchanges (Section 3, viscous treatment):
//
//   k_grad   Q (own element) + neighbours' Q face traces
//            -> common interface solution, gradients at solution points,
//               viscous flux of the own side at interior interface points
//               (written as the viscous face trace TV)
//   k_resid  Q + neighbours' Q and viscous traces
//            -> gradients again, fluxes at all flux points, Rusanov + averaged
//               viscous common fluxes at interfaces, divergence of the flux
//               polynomials, source, and either dQ/dt or the fused SSP-RK3
//               stage combination; in RK mode it also writes the face traces
//               of the new stage value for the next pass.
//
// Work mapping: a workgroup of NT threads owns EPB elements; every phase is a
// strided loop over (element, point) items with all element data staged in
// LDS.  No atomics: every output is written by exactly one thread in a fixed
// summation order, so results are bitwise run-to-run deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"
#include "mlp_bf16.hpp"
#include "sd_common.hpp"

namespace chorus {

// ---------------------------------------------------------------------------
// shared phases
// ---------------------------------------------------------------------------
template <int N, int EPB, int NT>
__device__ __forceinline__ void load_q(const double *__restrict__ Q, int64_t E, int64_t e0,
                                       double (*sq)[5][N * N * N]) {
    constexpr int NP = N * N * N;
    for (int it = threadIdx.x; it < EPB * 5 * NP; it += NT) {
        const int el = it / (5 * NP), r = it % (5 * NP), v = r / NP, p = r % NP;
        const int64_t e = e0 + el;
        sq[el][v][p] = (e < E) ? Q[((int64_t)v * E + e) * NP + p] : (v == 0 || v == 4 ? 1.0 : 0.0);
    }
}

// common interface solution Q* at the 6 N^2 face points (BR1 average with
// the neighbour trace, wall state, or average with the far-field state)
template <int N, int EPB, int NT>
__device__ __forceinline__ void common_solution(const Ops<N> &op, const Geo &G, const PhysParams &P,
                                                const double *__restrict__ TQ, int64_t e0,
                                                double (*sq)[5][N * N * N],
                                                double (*sqs)[6][5][N * N]) {
    constexpr int NF2 = N * N, NFL = (N + 1) * N * N;
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int d = f >> 1, m = (f & 1) ? N : 0, t1 = pp % N, t2 = pp / N;
        const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        double qo[5], qs[5];
        for (int v = 0; v < 5; ++v) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) s += op.I[m][b] * sq[el][v][base + b * st];
            qo[v] = s;
        }
        const int32_t nb = G.link[e * 6 + f];
        const int32_t inf = G.info[e * 6 + f];
        const int bc = (inf >> 6) - 1;
        if (nb >= 0) {
            const int f2 = inf & 7, o = (inf >> 3) & 7;
            const int pn = map_face_point<N>(o, t1, t2);
            const double *tq = TQ + ((int64_t)nb * 6 + f2) * 5 * NF2;
            for (int v = 0; v < 5; ++v) qs[v] = 0.5 * (qo[v] + tq[v * NF2 + pn]);
        } else if (bc == CHORUS_BC_INNER || bc == CHORUS_BC_OUTER) {
            const int fl = m + (N + 1) * (t1 + N * t2);
            const double sg = (f & 1) ? 1.0 : -1.0;
            double S[3];
            for (int c = 0; c < 3; ++c) S[c] = sg * G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
            wall_state(qo, S, bc == CHORUS_BC_OUTER, P, qs);
        } else {
            for (int v = 0; v < 5; ++v) qs[v] = 0.5 * (qo[v] + P.bc_state[v]);
        }
        for (int v = 0; v < 5; ++v) sqs[el][f][v][pp] = qs[v];
    }
}

// gradients of the conserved variables at the solution points:
// dQ/dxi_d = B q_line + D[.,0] Q*_0 + D[.,N] Q*_N, then grad_x = sum_d G_d dQ/dxi_d
template <int N, int EPB, int NT>
__device__ __forceinline__ void gradients(const Ops<N> &op, const Geo &G, int64_t e0,
                                          double (*sq)[5][N * N * N], double (*sqs)[6][5][N * N],
                                          double (*sgr)[15][N * N * N]) {
    constexpr int NP = N * N * N;
    for (int it = threadIdx.x; it < EPB * NP; it += NT) {
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        double dq[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d), pp = t1 + N * t2;
            for (int v = 0; v < 5; ++v) {
                double s = op.D[a][0] * sqs[el][2 * d][v][pp] + op.D[a][N] * sqs[el][2 * d + 1][v][pp];
#pragma unroll
                for (int b = 0; b < N; ++b) s += op.B[a][b] * sq[el][v][base + b * st];
                dq[d][v] = s;
            }
        }
        const double *gs = G.solgeo + e * 13 * NP + p;
        double Gm[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) Gm[t] = gs[t * NP];
        for (int v = 0; v < 5; ++v)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                sgr[el][v * 3 + c][p] = Gm[c] * dq[0][v] + Gm[3 + c] * dq[1][v] + Gm[6 + c] * dq[2][v];
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// face traces of Q: TQ[e][f][v][pp]
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_trace(Ops<N> opa, Geo G, const double *__restrict__ Q,
                                              double *__restrict__ TQ) {
    constexpr int NP = N * N * N, NF2 = N * N;
    __shared__ double sq[EPB][5][NP];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    __shared__ Ops<N> op;
    ops_to_lds(opa, op);
    load_q<N, EPB, NT>(Q, G.E, e0, sq);
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int d = f >> 1, m = (f & 1) ? N : 0, t1 = pp % N, t2 = pp / N;
        const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        for (int v = 0; v < 5; ++v) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) s += op.I[m][b] * sq[el][v][base + b * st];
            TQ[((e * 6 + f) * 5 + v) * NF2 + pp] = s;
        }
    }
}

// viscous flux of the own side at interior interface points, along the
// outward area vector: TV[e][f][v][pp]
// learned subgrid flux at the solution points of the block's elements (one
// wave, all points in 16-point tiles): features (Q, grad Q) -> network ->
// stau (LDS) and tau[k][E][NP] (global)
template <int N, int EPB, int NT>
__device__ __forceinline__ void closure_tau(const ClosureArgs &C, int64_t E, int64_t e0,
                                            double (*sq)[5][N * N * N], double (*sgr)[15][N * N * N],
                                            float (*stau)[15][N * N * N]) {
    constexpr int NP = N * N * N, NPTS = EPB * NP, NPT = (NPTS + 15) / 16;
    static_assert(NT == 64, "the closure runs one wave per block");
    const int lane = threadIdx.x, g = lane >> 4;
    u32x4_t xb[NPT];
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
        const int pidx = 16 * pt + (lane & 15);
        const int el = pidx / NP, sp = pidx % NP;
        const bool ok = pidx < NPTS && e0 + el < E;
        float x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int f = 8 * g + i;
            double raw = 0.0;
            if (ok && f < 5) raw = sq[el][f][sp];
            else if (ok && f < 20) raw = sgr[el][f - 5][sp];
            x[i] = (ok && f < 20) ? mlp_norm_feature(C.model, f, raw) : 0.0f;
        }
        xb[pt] = u32x4_t{bf16_pair(x[0], x[1]), bf16_pair(x[2], x[3]), bf16_pair(x[4], x[5]), bf16_pair(x[6], x[7])};
    }
    f32x4_t out[NPT];
    mlp_eval<NPT>(C.model, xb, out);
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
        const int pidx = 16 * pt + (lane & 15);
        const int el = pidx / NP, sp = pidx % NP;
        if (pidx >= NPTS || e0 + el >= E) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            if (k >= kMlpOut) continue;
            stau[el][k][sp] = out[pt][i];
            C.tau[((int64_t)k * E + e0 + el) * NP + sp] = out[pt][i];
        }
    }
}

template <int N, int EPB, int NT, bool CL>
__global__ __launch_bounds__(NT) void k_grad(Ops<N> opa, Geo G, PhysParams P, const double *__restrict__ Q,
                                             const double *__restrict__ TQ, double *__restrict__ TV,
                                             ClosureArgs C) {
    constexpr int NP = N * N * N, NF2 = N * N, NFL = (N + 1) * N * N;
    __shared__ double sq[EPB][5][NP];
    __shared__ double sqs[EPB][6][5][NF2];
    __shared__ double sgr[EPB][15][NP];
    __shared__ float stau[CL ? EPB : 1][15][CL ? NP : 1];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    __shared__ Ops<N> op;
    ops_to_lds(opa, op);
    load_q<N, EPB, NT>(Q, G.E, e0, sq);
    __syncthreads();
    common_solution<N, EPB, NT>(op, G, P, TQ, e0, sq, sqs);
    __syncthreads();
    gradients<N, EPB, NT>(op, G, e0, sq, sqs, sgr);
    __syncthreads();
    if constexpr (CL) {
        closure_tau<N, EPB, NT>(C, G.E, e0, sq, sgr, stau);
        __syncthreads();
    }
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int32_t nb = G.link[e * 6 + f], inf = G.info[e * 6 + f];
        const int d = f >> 1, m = (f & 1) ? N : 0, t1 = pp % N, t2 = pp / N;
        const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        double q[5], g[5][3];
        for (int v = 0; v < 5; ++v) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) s += op.I[m][b] * sq[el][v][base + b * st];
            q[v] = s;
            for (int c = 0; c < 3; ++c) {
                double t = 0.0;
#pragma unroll
                for (int b = 0; b < N; ++b) t += op.I[m][b] * sgr[el][v * 3 + c][base + b * st];
                g[v][c] = t;
            }
        }
        const int fl = m + (N + 1) * (t1 + N * t2);
        const double sg = (f & 1) ? 1.0 : -1.0;
        const int bc = (inf >> 6) - 1;
        double S[3], fv[5], phi[5];
        for (int c = 0; c < 3; ++c) S[c] = sg * G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
        if (nb >= 0) {
            flux_viscous(q, g, S, P, fv);
            if constexpr (CL) {
                // the own-side subgrid flux enters the trace with the sign of -F_v
                for (int v = 0; v < 5; ++v)
                    for (int c = 0; c < 3; ++c) {
                        double t = 0.0;
#pragma unroll
                        for (int b = 0; b < N; ++b) t += op.I[m][b] * (double)stau[el][v * 3 + c][base + b * st];
                        fv[v] -= t * S[c];
                    }
            }
            for (int v = 0; v < 5; ++v) TV[((e * 6 + f) * 5 + v) * NF2 + pp] = fv[v];
            // own-side part of the common flux: Rusanov minus half the own
            // viscous (minus subgrid) flux; the residual pass adds the
            // neighbour's half from its trace
            const int f2 = inf & 7, o = (inf >> 3) & 7;
            const int pn = map_face_point<N>(o, t1, t2);
            const double *tq = TQ + ((int64_t)nb * 6 + f2) * 5 * NF2;
            double qn[5];
            for (int v = 0; v < 5; ++v) qn[v] = tq[v * NF2 + pn];
            flux_rusanov(q, qn, S, P, phi);
            for (int v = 0; v < 5; ++v) phi[v] -= 0.5 * fv[v];
        } else if (bc == CHORUS_BC_INNER || bc == CHORUS_BC_OUTER) {
            flux_wall(q, g, S, bc == CHORUS_BC_OUTER, P, phi);
        } else {
            flux_viscous(q, g, S, P, fv);
            flux_rusanov(q, P.bc_state, S, P, phi);
            for (int v = 0; v < 5; ++v) phi[v] -= 0.5 * fv[v];
        }
        for (int v = 0; v < 5; ++v) G.FF[((e * 6 + f) * 5 + v) * NF2 + pp] = phi[v];
    }
}

// raw closure features at the solution points: X[e NP + p][20] = (Q, grad Q)
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_features(Ops<N> opa, Geo G, PhysParams P, const double *__restrict__ Q,
                                                 const double *__restrict__ TQ, float *__restrict__ X) {
    constexpr int NP = N * N * N, NF2 = N * N;
    __shared__ double sq[EPB][5][NP];
    __shared__ double sqs[EPB][6][5][NF2];
    __shared__ double sgr[EPB][15][NP];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    __shared__ Ops<N> op;
    ops_to_lds(opa, op);
    load_q<N, EPB, NT>(Q, G.E, e0, sq);
    __syncthreads();
    common_solution<N, EPB, NT>(op, G, P, TQ, e0, sq, sqs);
    __syncthreads();
    gradients<N, EPB, NT>(op, G, e0, sq, sqs, sgr);
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * NP * 20; it += NT) {
        const int el = it / (NP * 20), r = it % (NP * 20), p = r / 20, f = r % 20;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        X[(e * NP + p) * 20 + f] = (float)(f < 5 ? sq[el][f][p] : sgr[el][f - 5][p]);
    }
}



template <int N, int EPB, int NT, bool CL>
__global__ __launch_bounds__(NT) void k_resid(Ops<N> opa, Geo G, PhysParams P, const double *Q,
                                              const double *__restrict__ TQ,
                                              const double *__restrict__ TV, StageArgs S_, ClosureArgs C) {
    constexpr int NP = N * N * N, NF2 = N * N, NFL = (N + 1) * N * N;
    constexpr int IT_SOL = (EPB * NP + NT - 1) / NT;
    __shared__ double sq[EPB][5][NP];
    __shared__ double sgr[EPB][15][NP];
    // the common solution is consumed by the gradients before the first
    // direction's fluxes are written
    __shared__ union {
        double sqs[EPB][6][5][NF2];
        double sft[EPB][5][NFL];
    } U;
    __shared__ float stau[CL ? EPB : 1][15][CL ? NP : 1];
    auto &sqs = U.sqs;
    auto &sft = U.sft;
    double div[IT_SOL][5];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const double gm1 = P.gamma - 1.0;
    if constexpr (CL) {
        for (int it = threadIdx.x; it < EPB * 15 * NP; it += NT) {
            const int el = it / (15 * NP), r = it % (15 * NP), k = r / NP, p = r % NP;
            const int64_t e = e0 + el;
            stau[el][k][p] = (e < G.E) ? C.tau[((int64_t)k * G.E + e) * NP + p] : 0.0f;
        }
    }
    __shared__ Ops<N> op;
    ops_to_lds(opa, op);
    load_q<N, EPB, NT>(Q, G.E, e0, sq);
    __syncthreads();
    common_solution<N, EPB, NT>(op, G, P, TQ, e0, sq, sqs);
    __syncthreads();
    gradients<N, EPB, NT>(op, G, e0, sq, sqs, sgr);
    __syncthreads();
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        // interface points of direction d: own-side common flux from the
        // gradient pass plus half the neighbour's viscous flux (stored along
        // its own outward area vector, -So)
        for (int it = threadIdx.x; it < EPB * 2 * NF2; it += NT) {
            const int el = it / (2 * NF2), side = (it / NF2) & 1, pp = it % NF2;
            const int64_t e = e0 + el;
            if (e >= G.E) continue;
            const int f = 2 * d + side, m = side ? N : 0, t1 = pp % N, t2 = pp / N;
            const double sg = side ? 1.0 : -1.0;
            const int32_t nb = G.link[e * 6 + f];
            double phi[5];
            for (int v = 0; v < 5; ++v) phi[v] = G.FF[((e * 6 + f) * 5 + v) * NF2 + pp];
            if (nb >= 0) {
                const int32_t inf = G.info[e * 6 + f];
                const int f2 = inf & 7, o = (inf >> 3) & 7;
                const int pn = map_face_point<N>(o, t1, t2);
                const double *tv = TV + ((int64_t)nb * 6 + f2) * 5 * NF2;
                for (int v = 0; v < 5; ++v) phi[v] += 0.5 * tv[v * NF2 + pn];
            }
            for (int v = 0; v < 5; ++v) sft[el][v][m + (N + 1) * pp] = sg * phi[v];
        }
        // interior d-flux points: transformed flux
        for (int it = threadIdx.x; it < EPB * (N - 1) * NF2; it += NT) {
            const int el = it / ((N - 1) * NF2), r = it % ((N - 1) * NF2);
            const int64_t e = e0 + el;
            if (e >= G.E) continue;
            const int m = 1 + r % (N - 1), tt = r / (N - 1), t1 = tt % N, t2 = tt / N;
            const int fl = m + (N + 1) * tt;
            const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
            double q[5], g[5][3], S[3], F[5];
            for (int v = 0; v < 5; ++v) {
                double s = 0.0;
#pragma unroll
                for (int b = 0; b < N; ++b) s += op.I[m][b] * sq[el][v][base + b * st];
                q[v] = s;
                for (int c = 0; c < 3; ++c) {
                    double t = 0.0;
#pragma unroll
                    for (int b = 0; b < N; ++b) t += op.I[m][b] * sgr[el][v * 3 + c][base + b * st];
                    g[v][c] = t;
                }
            }
            for (int c = 0; c < 3; ++c) S[c] = G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
            // learned subgrid flux along S (interpolated like the gradients)
            double ts[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if constexpr (CL) {
                for (int v = 0; v < 5; ++v)
                    for (int c = 0; c < 3; ++c) {
                        double t = 0.0;
#pragma unroll
                        for (int b = 0; b < N; ++b) t += op.I[m][b] * (double)stau[el][v * 3 + c][base + b * st];
                        ts[v] += t * S[c];
                    }
            }
            double fi[5], fv[5];
            flux_inviscid(q, S, gm1, fi);
            flux_viscous(q, g, S, P, fv);
            for (int v = 0; v < 5; ++v) F[v] = fi[v] - fv[v] + ts[v];
            for (int v = 0; v < 5; ++v) sft[el][v][fl] = F[v];
        }
        __syncthreads();
        // derivative of the flux polynomial along d at the solution points
#pragma unroll
        for (int k = 0; k < IT_SOL; ++k) {
            const int it = threadIdx.x + k * NT;
            if (it >= EPB * NP) break;
            const int el = it / NP, p = it % NP;
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int fb = (N + 1) * (t1 + N * t2);
            for (int v = 0; v < 5; ++v) {
                double s = 0.0;
#pragma unroll
                for (int mm = 0; mm <= N; ++mm) s += op.D[a][mm] * sft[el][v][fb + mm];
                div[k][v] = (d == 0) ? s : div[k][v] + s;
            }
        }
        __syncthreads();
    }
    // source and output
#pragma unroll
    for (int k = 0; k < IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const double *gs = G.solgeo + e * 13 * NP + p;
        const double iJ = gs[9 * NP];
        const double g0 = P.GM * gs[10 * NP], g1 = P.GM * gs[11 * NP], g2 = P.GM * gs[12 * NP];
        const double rho = sq[el][0][p], mx = sq[el][1][p], my = sq[el][2][p], mz = sq[el][3][p];
        double M[5];
        M[0] = 0.0;
        M[1] = rho * g0 - 2.0 * P.omega * my;
        M[2] = rho * g1 + 2.0 * P.omega * mx;
        M[3] = rho * g2;
        M[4] = mx * g0 + my * g1 + mz * g2;
        for (int v = 0; v < 5; ++v) {
            const double R = -div[k][v] * iJ - M[v];
            const int64_t gi = ((int64_t)v * G.E + e) * NP + p;
            if (S_.mode == 0) {
                S_.Qout[gi] = R;
            } else {
                const double q = sq[el][v][p];
                if (S_.Tout) {
                    const double qb = (S_.d0 != 0.0) ? S_.B[gi] : 0.0;
                    S_.Tout[gi] = S_.d0 * qb + S_.d1 * (q + S_.d2 * R);
                }
                const double qa = (S_.c0 != 0.0) ? S_.A[gi] : 0.0;
                const double qv = S_.c0 * qa + S_.c1 * (q + S_.c2 * R);
                S_.Qout[gi] = qv;
                sq[el][v][p] = qv;
            }
        }
    }
    if (S_.mode == 0 || S_.TQout == nullptr) return;
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int d = f >> 1, m = (f & 1) ? N : 0, t1 = pp % N, t2 = pp / N;
        const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        for (int v = 0; v < 5; ++v) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) s += op.I[m][b] * sq[el][v][base + b * st];
            S_.TQout[((e * 6 + f) * 5 + v) * NF2 + pp] = s;
        }
    }
}

// entropy gradient of a state at rest along the flux-point metric:
// out[e][d][fl] = grad S . (|J| grad xi_d) at the d-flux points, with the BR1
// gradients of the FP64 path (S = c_p ln(p^(1/gamma)/rho), p = (gamma-1) E
// for zero momentum); used by the mixed-precision path
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_bg_entropy(Ops<N> opa, Geo G, PhysParams P, const double *__restrict__ Q0,
                                                   const double *__restrict__ TQ, float *__restrict__ out) {
    constexpr int NP = N * N * N, NF2 = N * N, NFL = (N + 1) * N * N;
    __shared__ double sq[EPB][5][NP];
    __shared__ double sqs[EPB][6][5][NF2];
    __shared__ double sgr[EPB][15][NP];
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    __shared__ Ops<N> op;
    ops_to_lds(opa, op);
    load_q<N, EPB, NT>(Q0, G.E, e0, sq);
    __syncthreads();
    common_solution<N, EPB, NT>(op, G, P, TQ, e0, sq, sqs);
    __syncthreads();
    gradients<N, EPB, NT>(op, G, e0, sq, sqs, sgr);
    __syncthreads();
    const double gm1 = P.gamma - 1.0;
    for (int it = threadIdx.x; it < EPB * 3 * NFL; it += NT) {
        const int el = it / (3 * NFL), r = it % (3 * NFL), d = r / NFL, fl = r % NFL;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int m = fl % (N + 1), t1 = (fl / (N + 1)) % N, t2 = fl / ((N + 1) * N);
        const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        double rho = 0.0, E = 0.0, gr = 0.0, gE = 0.0;
        for (int b = 0; b < N; ++b) {
            const double w = op.I[m][b];
            rho += w * sq[el][0][base + b * st];
            E += w * sq[el][4][base + b * st];
        }
        for (int c = 0; c < 3; ++c) {
            const double S = G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
            double a = 0.0, b2 = 0.0;
            for (int b = 0; b < N; ++b) {
                const double w = op.I[m][b];
                a += w * sgr[el][0 * 3 + c][base + b * st];
                b2 += w * sgr[el][4 * 3 + c][base + b * st];
            }
            gr += a * S;
            gE += b2 * S;
        }
        const double p = gm1 * E;
        out[(e * 3 + d) * NFL + fl] = (float)(P.cp * (gm1 * gE / (P.gamma * p) - gr / rho));
    }
}

// fixed-order partial sums of w w w |J| Q_v over element blocks
template <int NT>
__global__ __launch_bounds__(NT) void k_sums_partial(const double *__restrict__ Q,
                                                     const double *__restrict__ solw, int64_t n,
                                                     int64_t chunk, double *__restrict__ part) {
    __shared__ double red[NT];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = (lo + chunk < n) ? lo + chunk : n;
    for (int v = 0; v < 5; ++v) {
        double s = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += NT) s += solw[i] * Q[(int64_t)v * n + i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)v * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_sums_final(const double *__restrict__ part, int nb, int rows,
                                                   double *__restrict__ out) {
    __shared__ double red[NT];
    for (int v = 0; v < rows; ++v) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nb; i += NT) s += part[(int64_t)v * nb + i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[v] = red[0];
        __syncthreads();
    }
}

// angular momentum L = sum w|J| x cross m and the diagonal moments of
// inertia I_c = sum w|J| rho (|x|^2 - x_c^2) (Section 6): block partials
// part[q][block], q = Lx, Ly, Lz, Ix, Iy, Iz, over contiguous chunks of
// solution points, fixed tree order
template <int NT>
__global__ __launch_bounds__(NT) void k_am_partial(const double *__restrict__ Q, const double *__restrict__ solw,
                                                   const double *__restrict__ xsol, int64_t E, int NP,
                                                   int64_t chunk, double *__restrict__ part) {
    __shared__ double red[6][NT];
    const int64_t n = E * NP;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = (lo + chunk < n) ? lo + chunk : n;
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
        const int64_t e = i / NP, p = i % NP;
        const double x = xsol[(e * 3 + 0) * NP + p], y = xsol[(e * 3 + 1) * NP + p], z = xsol[(e * 3 + 2) * NP + p];
        const double w = solw[i], rho = Q[i], mx = Q[n + i], my = Q[2 * n + i], mz = Q[3 * n + i];
        s[0] += w * (y * mz - z * my);
        s[1] += w * (z * mx - x * mz);
        s[2] += w * (x * my - y * mx);
        s[3] += w * rho * (y * y + z * z);
        s[4] += w * rho * (x * x + z * z);
        s[5] += w * rho * (x * x + y * y);
    }
    for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

// u <- u - dOmega x x at fixed rho and pressure (E changes by the kinetic
// energy change)
__global__ void k_am_apply(double *__restrict__ Q, const double *__restrict__ xsol, int64_t E, int NP, double dx,
                           double dy, double dz) {
    const int64_t n = E * NP;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t e = i / NP, p = i % NP;
    const double x = xsol[(e * 3 + 0) * NP + p], y = xsol[(e * 3 + 1) * NP + p], z = xsol[(e * 3 + 2) * NP + p];
    const double rho = Q[i];
    const double u = Q[n + i] / rho, v = Q[2 * n + i] / rho, w = Q[3 * n + i] / rho;
    const double un = u - (dy * z - dz * y), vn = v - (dz * x - dx * z), wn = w - (dx * y - dy * x);
    const double dke = 0.5 * rho * ((un * un + vn * vn + wn * wn) - (u * u + v * v + w * w));
    Q[n + i] = rho * un;
    Q[2 * n + i] = rho * vn;
    Q[3 * n + i] = rho * wn;
    Q[4 * n + i] += dke;
}

// non-finite / non-positive density or pressure check: flag[0] set to 1
__global__ void k_check(const double *__restrict__ Q, int64_t n, double gm1, int *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double r = Q[i], mx = Q[n + i], my = Q[2 * n + i], mz = Q[3 * n + i], E = Q[4 * n + i];
    const double p = gm1 * (E - 0.5 * (mx * mx + my * my + mz * mz) / r);
    const bool ok = (r > 0.0) && (p > 0.0) && (r < 1e300) && (p < 1e300) && (mx == mx) && (my == my) &&
                    (mz == mz);
    if (!ok) flag[0] = 1;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
struct LaunchCfg {
    int epb, nt;
};

template <int N>
static Ops<N> make_ops(const Basis1D &b) {
    return make_ops_t<double, N>(b);
}

// elements per block / threads per block for each order
template <int N>
struct Cfg;
template <> struct Cfg<2> { static constexpr int EPB = 8, NT = 64; };
template <> struct Cfg<3> { static constexpr int EPB = 2, NT = 64; };
template <> struct Cfg<4> { static constexpr int EPB = 1, NT = 64; };
template <> struct Cfg<5> { static constexpr int EPB = 1, NT = 128; };
template <> struct Cfg<6> { static constexpr int EPB = 1, NT = 256; };

struct Bufs {
    const double *Q;
    const double *TQ;
    double *TQw;
    double *TV;
};

template <int N>
static hipError_t launch_trace_t(const Mesh &m, const Geo &G, const double *Q, double *TQ, hipStream_t s) {
    constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
    const Ops<N> op = make_ops<N>(m.basis);
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_trace<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, op, G, Q, TQ);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_grad_t(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q,
                                const double *TQ, double *TV, const ClosureArgs &C, hipStream_t s) {
    constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
    const Ops<N> op = make_ops<N>(m.basis);
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    if (C.model) {
        if constexpr (N == 3)
            hipLaunchKernelGGL((k_grad<N, EPB, NT, true>), dim3(nb), dim3(NT), 0, s, op, G, P, Q, TQ, TV, C);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_grad<N, EPB, NT, false>), dim3(nb), dim3(NT), 0, s, op, G, P, Q, TQ, TV, C);
    }
    return hipGetLastError();
}

template <int N>
static hipError_t launch_resid_t(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q,
                                 const double *TQ, const double *TV, const StageArgs &sa, const ClosureArgs &C,
                                 hipStream_t s) {
    constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
    const Ops<N> op = make_ops<N>(m.basis);
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    if (C.model) {
        if constexpr (N == 3)
            hipLaunchKernelGGL((k_resid<N, EPB, NT, true>), dim3(nb), dim3(NT), 0, s, op, G, P, Q, TQ, TV, sa, C);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_resid<N, EPB, NT, false>), dim3(nb), dim3(NT), 0, s, op, G, P, Q, TQ, TV, sa, C);
    }
    return hipGetLastError();
}

template <int N>
static hipError_t launch_features_t(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q,
                                    const double *TQ, float *X, hipStream_t s) {
    constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
    const Ops<N> op = make_ops<N>(m.basis);
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_features<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, op, G, P, Q, TQ, X);
    return hipGetLastError();
}

#define CHORUS_DISPATCH(N_, CALL)            \
    switch (N_) {                            \
        case 2: return CALL(2);              \
        case 3: return CALL(3);              \
        case 4: return CALL(4);              \
        case 5: return CALL(5);              \
        case 6: return CALL(6);              \
        default: return hipErrorInvalidValue; \
    }

hipError_t launch_trace(const Mesh &m, const Geo &G, const double *Q, double *TQ, hipStream_t s) {
#define C_(n) launch_trace_t<n>(m, G, Q, TQ, s)
    CHORUS_DISPATCH(m.N, C_)
#undef C_
}
hipError_t launch_grad(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q, const double *TQ,
                       double *TV, const ClosureArgs &C, hipStream_t s) {
#define C_(n) launch_grad_t<n>(m, G, P, Q, TQ, TV, C, s)
    CHORUS_DISPATCH(m.N, C_)
#undef C_
}
hipError_t launch_resid(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q, const double *TQ,
                        const double *TV, const StageArgs &sa, const ClosureArgs &C, hipStream_t s) {
#define C_(n) launch_resid_t<n>(m, G, P, Q, TQ, TV, sa, C, s)
    CHORUS_DISPATCH(m.N, C_)
#undef C_
}
hipError_t launch_features(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q, const double *TQ,
                           float *X, hipStream_t s) {
#define C_(n) launch_features_t<n>(m, G, P, Q, TQ, X, s)
    CHORUS_DISPATCH(m.N, C_)
#undef C_
}

template <int N>
static hipError_t launch_bg_entropy_t(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q0,
                                      const double *TQ, float *out, hipStream_t s) {
    constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
    const Ops<N> op = make_ops<N>(m.basis);
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_bg_entropy<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, op, G, P, Q0, TQ, out);
    return hipGetLastError();
}

hipError_t launch_bg_entropy(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q0, const double *TQ,
                             float *out, hipStream_t s) {
#define C_(n) launch_bg_entropy_t<n>(m, G, P, Q0, TQ, out, s)
    CHORUS_DISPATCH(m.N, C_)
#undef C_
}

hipError_t launch_sums(const double *Q, const double *solw, int64_t n, double *part, int nblocks, double *out,
                       hipStream_t s) {
    const int64_t chunk = (n + nblocks - 1) / nblocks;
    hipLaunchKernelGGL((k_sums_partial<256>), dim3(nblocks), dim3(256), 0, s, Q, solw, n, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sums_final<256>), dim3(1), dim3(256), 0, s, part, nblocks, 5, out);
    return hipGetLastError();
}

hipError_t launch_am_sums(const double *Q, const double *solw, const double *xsol, int64_t E, int NP, double *part,
                          int nblocks, double *out, hipStream_t s) {
    const int64_t n = E * NP;
    const int64_t chunk = (n + nblocks - 1) / nblocks;
    hipLaunchKernelGGL((k_am_partial<256>), dim3(nblocks), dim3(256), 0, s, Q, solw, xsol, E, NP, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_sums_final<256>), dim3(1), dim3(256), 0, s, part, nblocks, 6, out);
    return hipGetLastError();
}

hipError_t launch_am_apply(double *Q, const double *xsol, int64_t E, int NP, const double dO[3], hipStream_t s) {
    const int64_t n = E * NP;
    hipLaunchKernelGGL(k_am_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Q, xsol, E, NP, dO[0], dO[1],
                       dO[2]);
    return hipGetLastError();
}

__global__ void k_clear_flag(int *flag) { flag[0] = 0; }

hipError_t launch_clear_flag(int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, s, flag);
    return hipGetLastError();
}

hipError_t launch_check(const double *Q, int64_t n, double gm1, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, s, flag);
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_check, dim3(nb), dim3(256), 0, s, Q, n, gm1, flag);
    return hipGetLastError();
}

}  // namespace chorus
