// HIP kernels (gfx950) of the FP64 spectral-difference residual and the
// explicit Runge-Kutta update (Section 3 of the paper).
//
// One stage is split in two element passes because BR1 needs two
// neighbour exchanges (Section 3, viscous treatment):
//
//   k_flux64   Q (own element) + neighbours' Q face traces
//              -> common interface solution, gradients, [learned subgrid
//                 flux], own-side common fluxes and own viscous face flux
//                 (pushed to the neighbours), fluxes at the interior flux
//                 points, divergence, source, and the stage combination with
//                 this partial residual
//   k_lift64   neighbours' viscous face fluxes -> the missing residual part
//              added in place; face traces of the new state pushed to the
//              neighbours for the next stage.
//
// k_trace (traces indexed by their own element) serves the closure features
// and the background set-up of the mixed path; the flux pass's network-only
// variant serves closure inference.
//
// Work mapping: a workgroup of NT threads owns EPB elements; every phase is
// a loop over (element, point) items with all element data staged in LDS.
// No atomics: every output is written by exactly one thread in a fixed
// summation order, so results are bitwise run-to-run deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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

// learned subgrid flux at the solution points of the block's elements (one
// wave, all points in 16-point tiles): features (Q, grad Q) -> network ->
// tau[k][E][NP] (global), or into the block's LDS copy stau when given
template <int N, int EPB, int NT, typename GT>
__device__ __forceinline__ void closure_tau(const ClosureArgs &C, int64_t E, int64_t e0,
                                            double (*sq)[5][N * N * N], GT (*sgr)[15][N * N * N],
                                            float (*stau)[15][N * N * N] = nullptr) {
    constexpr int NP = N * N * N, NPTS = EPB * NP, NPT = (NPTS + 15) / 16;
    // point tiles evaluated together (fewer live accumulators than all of
    // the block's tiles at once)
    constexpr int TB = NPT < 2 ? NPT : 2;
    static_assert(NT == 64, "the closure runs one wave per block");
    const int lane = threadIdx.x, g = lane >> 4;
#pragma unroll
    for (int t0 = 0; t0 < NPT; t0 += TB) {
        u32x4_t xb[TB];
#pragma unroll
        for (int j = 0; j < TB; ++j) {
            const int pidx = 16 * (t0 + j) + (lane & 15);
            const int el = pidx / NP, sp = pidx % NP;
            const bool ok = pidx < NPTS && e0 + el < E;
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int f = 8 * g + i;
                double raw = 0.0;
                if (ok && f < 5) raw = sq[el][f][lds_sol<N>(sp)];
                else if (ok && f < 20) raw = (double)sgr[el][f - 5][lds_sol<N>(sp)];
                x[i] = (ok && f < 20) ? mlp_norm_feature(C.model, f, raw) : 0.0f;
            }
            xb[j] = u32x4_t{bf16_pair(x[0], x[1]), bf16_pair(x[2], x[3]), bf16_pair(x[4], x[5]), bf16_pair(x[6], x[7])};
        }
        f32x4_t out[TB];
        mlp_eval<TB>(C.model, xb, out);
#pragma unroll
        for (int j = 0; j < TB; ++j) {
            const int pidx = 16 * (t0 + j) + (lane & 15);
            const int el = pidx / NP, sp = pidx % NP;
            if (pidx >= NPTS || e0 + el >= E) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = 4 * g + i;
                if (k >= kMlpOut) continue;
                if (stau) stau[el][k][sp] = out[j][i];
                else C.tau[((int64_t)k * E + e0 + el) * NP + sp] = out[j][i];
            }
        }
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



// ---------------------------------------------------------------------------
// flux pass + lift pass (the stage split used by the solver)
// ---------------------------------------------------------------------------
// Per stage: the flux pass takes every step that needs the gradients --
// common interface solution, gradients, [learned subgrid flux], at the face
// points the own viscous flux (pushed to the neighbour's viscous mailbox)
// and the own-side common flux (Rusanov minus half the own viscous flux,
// the wall flux, or the far-field flux), at the interior flux points the
// transformed flux, the divergence with the own-side face fluxes at the line
// ends, the source -- and enters the stage combination with this partial
// residual.  The lift pass adds the neighbours' viscous halves in place and
// pushes the face traces of the new state to the neighbours' mailboxes.
// Mailboxes are indexed by the receiving element, face and point (in the
// receiver's point order), so each element reads its own contiguous block.
template <int N, int EPB, int NT>
struct Sh64 {
    static constexpr int NP = N * N * N, NF2 = N * N, NFL = (N + 1) * N * N, NINTD = (N - 1) * N * N;
    static constexpr int IT_SOL = (EPB * NP + NT - 1) / NT;
    static constexpr int IT_FACE = (EPB * 6 * NF2 + NT - 1) / NT;
    static constexpr int IT_INTD = (EPB * NINTD + NT - 1) / NT;
};

// launch shape of the flux/lift passes per order: elements per block,
// threads, minimum waves per SIMD of the flux pass
template <int N>
struct Cfg64;
template <> struct Cfg64<2> { static constexpr int EPB = 8, NT = 64, MINW = 1; };
template <> struct Cfg64<3> { static constexpr int EPB = 2, NT = 64, MINW = 1; };
template <> struct Cfg64<4> { static constexpr int EPB = 1, NT = 64, MINW = 3; };
template <> struct Cfg64<5> { static constexpr int EPB = 1, NT = 128, MINW = 1; };
template <> struct Cfg64<6> { static constexpr int EPB = 1, NT = 256, MINW = 1; };

// face traces of the element block's state (LDS) pushed to the neighbours
template <int N, int EPB, int NT, bool SW = false>
__device__ __forceinline__ void push_traces64(const Ops<N> &op, const Geo &G, int64_t e0, const int32_t (*lk)[6],
                                              const int32_t (*inf)[6], const double (*sq)[5][N * N * N],
                                              double *__restrict__ TQout) {
    constexpr int NF2 = N * N;
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int32_t nb = lk[el][f];
        if (e0 + el >= G.E || nb < 0) continue;
        const int d = f >> 1, m = (f & 1) ? N : 0;
        const int base = sol_of<N>(d, 0, pp % N, pp / N), st = stride_of<N>(d);
        double *out = TQout + mailbox_slot<N>(nb, inf[el][f], pp);
        for (int v = 0; v < 5; ++v) {
            double t = 0.0;
#pragma unroll
            for (int b = 0; b < N; ++b) t += op.I[m][b] * sq[el][v][SW ? lds_line<N>(base, b, st) : base + b * st];
            st_once(&out[v * NF2], t);
        }
    }
}

// face traces of Q pushed to the neighbours' mailboxes (start of a call)
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_trace_push(Ops<N> opa, Geo G, const double *__restrict__ Q,
                                                   double *__restrict__ TQ) {
    constexpr int NP = N * N * N;
    __shared__ double sq[EPB][5][NP];
    __shared__ int32_t lk[EPB][6], inf[EPB][6];
    __shared__ Ops<N> op;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    ops_to_lds(opa, op);
    load_q<N, EPB, NT>(Q, G.E, e0, sq);
    if ((int)threadIdx.x < EPB * 6) {
        const bool ok = e0 + threadIdx.x / 6 < G.E;
        lk[threadIdx.x / 6][threadIdx.x % 6] = ok ? G.link[e0 * 6 + threadIdx.x] : -1;
        inf[threadIdx.x / 6][threadIdx.x % 6] = ok ? G.info[e0 * 6 + threadIdx.x] : 0;
    }
    __syncthreads();
    push_traces64<N, EPB, NT>(op, G, e0, lk, inf, sq, TQ);
}

// line interpolation of an LDS field at flux point m of the line (base, st)
template <int N, typename T>
__device__ __forceinline__ double line_interp(const Ops<N> &op, const T *fld, int m, int base, int st) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) t += op.I[m][b] * (double)fld[base + b * st];
    return t;
}
// the same over a field stored in the lds_sol layout
template <int N, typename T>
__device__ __forceinline__ double line_interp_s(const Ops<N> &op, const T *fld, int m, int base, int st) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) t += op.I[m][b] * (double)fld[lds_line<N>(base, b, st)];
    return t;
}

// PART 0: the flux pass; PART 1: only the learned subgrid flux (common
// solution, gradients, network -> C.tau: chorus_closure_infer); PART 2: the
// flux pass with the learned subgrid flux evaluated in the pass (network on
// the gradients in LDS, its output kept in LDS)
// RAD: radiative diffusivity varying with radius (radius of each flux point
// read with its geometry), else the constant P.kappa_r
template <int N, int EPB, int NT, int PART, bool RAD>
__global__ __launch_bounds__(NT, Cfg64<N>::MINW) void k_flux64(Ops<N> opa, Geo G, PhysParams P, const double *__restrict__ Q,
                                               const double *__restrict__ TQ, double *__restrict__ TV,
                                               StageArgs S_, ClosureArgs C) {
    constexpr bool CL = PART != 0;
    using Sh = Sh64<N, EPB, NT>;
    constexpr int NP = Sh::NP, NF2 = Sh::NF2, NFL = Sh::NFL, NINTD = Sh::NINTD;
    __shared__ double sq[EPB][5][NP];
    // gradients at the solution points (the network-only pass keeps them in
    // FP32: they are network inputs, rounded to bfloat16 after
    // normalisation)
    __shared__ std::conditional_t<PART == 1, float, double> sgr[EPB][15][NP];
    // the common solution is consumed by the gradients before the subgrid
    // flux (PART 2) and the first direction's fluxes are written
    __shared__ union {
        double sqs[EPB][6][5][NF2];
        struct {
            double sft[EPB][5][NFL];
            float stau[PART == 2 ? EPB : 1][15][PART == 2 ? NP : 1];  // subgrid flux (PART 2)
        } F;
    } U;
    auto &stau = U.F.stau;
    __shared__ int32_t lk[EPB][6], inf[EPB][6];
    __shared__ Ops<N> op;
    const int64_t e0 = (int64_t)blockIdx.x * EPB, E = G.E;
    const double gm1 = P.gamma - 1.0;
    // every global input of the element block before the first wait;
    // unpredicated loads through clamped indices (items past the end read
    // element 0 and are never stored)
    double qv[Sh::IT_SOL][5], Gm[Sh::IT_SOL][9];
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / NP, p = it % NP;
        const int64_t e = (it < EPB * NP && e0 + el < E) ? e0 + el : 0;
        for (int v = 0; v < 5; ++v) qv[k][v] = Q[((int64_t)v * E + e) * NP + p];
        for (int t = 0; t < 9; ++t) Gm[k][t] = G.solgeo[(e * 13 + t) * NP + p];
    }
    // radiative diffusivity at the face and interior flux points
    double nq[Sh::IT_FACE][5], Sf[Sh::IT_FACE][3], krf[Sh::IT_FACE];
#pragma unroll
    for (int k = 0; k < Sh::IT_FACE; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = (it < EPB * 6 * NF2 && e0 + el < E) ? e0 + el : 0;
        for (int v = 0; v < 5; ++v) nq[k][v] = TQ[((e * 6 + f) * 5 + v) * NF2 + pp];
        const int d = f >> 1, fl = ((f & 1) ? N : 0) + (N + 1) * pp;
        const double sg = (f & 1) ? 1.0 : -1.0;
        for (int c = 0; c < 3; ++c) Sf[k][c] = sg * G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
        krf[k] = RAD ? G.rflux[(e * 3 + d) * NFL + fl] : P.kappa_r;
    }
    // interior flux-point metrics: one direction at a time, the next one
    // issued while the current one is used (fewer registers in flight)
    double Si[2][Sh::IT_INTD][3], kri[2][Sh::IT_INTD];
    auto load_si = [&](int d, int slot) {
#pragma unroll
        for (int k = 0; k < Sh::IT_INTD; ++k) {
            const int it = threadIdx.x + k * NT;
            const int el = it / NINTD, q = it % NINTD;
            const int fl = 1 + q % (N - 1) + (N + 1) * (q / (N - 1));
            const int64_t e = (it < EPB * NINTD && e0 + el < E) ? e0 + el : 0;
            for (int c = 0; c < 3; ++c) Si[slot][k][c] = G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
            kri[slot][k] = RAD ? G.rflux[(e * 3 + d) * NFL + fl] : P.kappa_r;
        }
    };
    if constexpr (PART != 1) load_si(0, 0);
    {
        const bool okl = (int)threadIdx.x < EPB * 6 && e0 + threadIdx.x / 6 < E;
        const int32_t l = G.link[okl ? e0 * 6 + threadIdx.x : 0], i = G.info[okl ? e0 * 6 + threadIdx.x : 0];
        if ((int)threadIdx.x < EPB * 6) {
            lk[threadIdx.x / 6][threadIdx.x % 6] = okl ? l : -1;
            inf[threadIdx.x / 6][threadIdx.x % 6] = okl ? i : 0;
        }
    }
    ops_to_lds(opa, op);
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        for (int v = 0; v < 5; ++v) sq[it / NP][v][lds_sol<N>(it % NP)] = qv[k][v];
    }
    __syncthreads();
    // common interface solution (the own face values are formed again in
    // the face-flux phase: fewer registers live across the gradients)
#pragma unroll
    for (int k = 0; k < Sh::IT_FACE; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * 6 * NF2) break;
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        if (e0 + el >= E) continue;
        const int d = f >> 1, m = (f & 1) ? N : 0;
        const int base = sol_of<N>(d, 0, pp % N, pp / N), st = stride_of<N>(d);
        double fo[5];
        for (int v = 0; v < 5; ++v) fo[v] = line_interp_s<N>(op, sq[el][v], m, base, st);
        const int32_t nb = lk[el][f];
        const int bc = (inf[el][f] >> 6) - 1;
        double qs[5];
        if (nb >= 0) {
            for (int v = 0; v < 5; ++v) qs[v] = 0.5 * (fo[v] + nq[k][v]);
        } else if (bc == CHORUS_BC_INNER || bc == CHORUS_BC_OUTER) {
            wall_state(fo, Sf[k], bc == CHORUS_BC_OUTER, P, qs);  // (the same along +-S)
        } else {
            for (int v = 0; v < 5; ++v) qs[v] = 0.5 * (fo[v] + P.bc_state[v]);
        }
        for (int v = 0; v < 5; ++v) U.sqs[el][f][v][pp] = qs[v];
    }
    __syncthreads();
    // gradients at the solution points
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        const int el = it / NP, p = it % NP;
        double dq[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d), pp = t1 + N * t2;
            for (int v = 0; v < 5; ++v) {
                double t = op.D[a][0] * U.sqs[el][2 * d][v][pp] + op.D[a][N] * U.sqs[el][2 * d + 1][v][pp];
#pragma unroll
                for (int b = 0; b < N; ++b) t += op.B[a][b] * sq[el][v][lds_line<N>(base, b, st)];
                dq[d][v] = t;
            }
        }
        for (int v = 0; v < 5; ++v)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                sgr[el][v * 3 + c][lds_sol<N>(p)] = Gm[k][c] * dq[0][v] + Gm[k][3 + c] * dq[1][v] + Gm[k][6 + c] * dq[2][v];
    }
    __syncthreads();
    if constexpr (PART == 1) {
        // subgrid flux at the solution points -> C.tau
        closure_tau<N, EPB, NT>(C, E, e0, sq, sgr);
        return;
    }
    if constexpr (PART == 2) {
        // subgrid flux at the solution points -> LDS
        closure_tau<N, EPB, NT>(C, E, e0, sq, sgr, stau);
        __syncthreads();
    }
    // face points: own viscous flux to the neighbour, own-side common flux
    // kept in registers for the divergence
    double ffc[Sh::IT_FACE][5];
#pragma unroll
    for (int k = 0; k < Sh::IT_FACE; ++k) {
        const int it = threadIdx.x + k * NT;
        for (int v = 0; v < 5; ++v) ffc[k][v] = 0.0;
        if (it >= EPB * 6 * NF2) break;
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        if (e0 + el >= E) continue;
        const int d = f >> 1, m = (f & 1) ? N : 0;
        const int base = sol_of<N>(d, 0, pp % N, pp / N), st = stride_of<N>(d);
        double fo[5], g[5][3];
        for (int v = 0; v < 5; ++v) {
            fo[v] = line_interp_s<N>(op, sq[el][v], m, base, st);
            for (int c = 0; c < 3; ++c) g[v][c] = line_interp_s<N>(op, sgr[el][v * 3 + c], m, base, st);
        }
        const int32_t nb = lk[el][f];
        const int bc = (inf[el][f] >> 6) - 1;
        const double kr = RAD ? kappa_r_at(P, krf[k]) : krf[k];
        double fv[5];
        if (nb >= 0) {
            flux_viscous(fo, g, Sf[k], P, kr, fv);
            if constexpr (CL) {
                // the own-side subgrid flux enters the trace with the sign of -F_v
                for (int v = 0; v < 5; ++v)
                    for (int c = 0; c < 3; ++c) fv[v] -= line_interp<N>(op, stau[el][v * 3 + c], m, base, st) * Sf[k][c];
            }
            // the viscous mass flux is zero: four components per point
            // unless the subgrid flux (with a mass part) rides along
            constexpr int NV = CL ? 5 : 4;
            double *tv = TV + mailbox_slot<N, NV>(nb, inf[el][f], pp);
            for (int v = 5 - NV; v < 5; ++v) st_once(&tv[(v - (5 - NV)) * NF2], fv[v]);
            flux_rusanov(fo, nq[k], Sf[k], P, ffc[k]);
            for (int v = 0; v < 5; ++v) ffc[k][v] -= 0.5 * fv[v];
        } else if (bc == CHORUS_BC_INNER || bc == CHORUS_BC_OUTER) {
            flux_wall(fo, g, Sf[k], bc == CHORUS_BC_OUTER, P, kr, ffc[k]);
        } else {
            flux_viscous(fo, g, Sf[k], P, kr, fv);
            flux_rusanov(fo, P.bc_state, Sf[k], P, ffc[k]);
            for (int v = 0; v < 5; ++v) ffc[k][v] -= 0.5 * fv[v];
        }
    }
    // per direction: transformed flux at the d-flux points, its derivative
    // added to the divergence at the solution points
    double div[Sh::IT_SOL][5];
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k)
        for (int v = 0; v < 5; ++v) div[k][v] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int cur = d & 1;
        if (d < 2) load_si(d + 1, cur ^ 1);
#pragma unroll
        for (int k = 0; k < Sh::IT_INTD; ++k) {
            const int it = threadIdx.x + k * NT;
            if (it >= EPB * NINTD) break;
            const int el = it / NINTD, q = it % NINTD;
            const int m = 1 + q % (N - 1), tt = q / (N - 1);
            if (e0 + el >= E) continue;
            const int base = sol_of<N>(d, 0, tt % N, tt / N), st = stride_of<N>(d);
            double qf[5], g[5][3], fi[5], fv[5];
            for (int v = 0; v < 5; ++v) {
                qf[v] = line_interp_s<N>(op, sq[el][v], m, base, st);
                for (int c = 0; c < 3; ++c) g[v][c] = line_interp_s<N>(op, sgr[el][v * 3 + c], m, base, st);
            }
            flux_inviscid(qf, Si[cur][k], gm1, fi);
            flux_viscous(qf, g, Si[cur][k], P, RAD ? kappa_r_at(P, kri[cur][k]) : kri[cur][k], fv);
            double ts[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if constexpr (CL) {
                for (int v = 0; v < 5; ++v)
                    for (int c = 0; c < 3; ++c) ts[v] += line_interp<N>(op, stau[el][v * 3 + c], m, base, st) * Si[cur][k][c];
            }
            const int fl = m + (N + 1) * tt;
            for (int v = 0; v < 5; ++v) U.F.sft[el][v][fl] = fi[v] - fv[v] + ts[v];
        }
#pragma unroll
        for (int k = 0; k < Sh::IT_FACE; ++k) {
            const int it = threadIdx.x + k * NT;
            if (it >= EPB * 6 * NF2) break;
            const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
            if ((f >> 1) != d || e0 + el >= E) continue;
            const double sg = (f & 1) ? 1.0 : -1.0;
            const int fl = ((f & 1) ? N : 0) + (N + 1) * pp;
            for (int v = 0; v < 5; ++v) U.F.sft[el][v][fl] = sg * ffc[k][v];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < Sh::IT_SOL; ++k) {
            const int it = threadIdx.x + k * NT;
            if (it >= EPB * NP) break;
            const int el = it / NP, p = it % NP;
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int fb = (N + 1) * (t1 + N * t2);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double t = 0.0;
#pragma unroll
                for (int mm = 0; mm <= N; ++mm) t += op.D[a][mm] * U.F.sft[el][v][fb + mm];
                div[k][v] += t;
            }
        }
        __syncthreads();
    }
    // source and the stage combination with the partial residual (operands
    // loaded before the first store: the outputs may alias them)
    const bool rk = S_.mode != 0;
    const bool useA = rk && S_.c0 != 0.0, useT = rk && S_.Tout != nullptr, useB = useT && S_.d0 != 0.0;
    double gq[Sh::IT_SOL][4], av[Sh::IT_SOL][5], bv[Sh::IT_SOL][5];
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / NP, p = it % NP;
        const int64_t e = (it < EPB * NP && e0 + el < E) ? e0 + el : 0;
        for (int c = 0; c < 4; ++c) gq[k][c] = G.solgeo[(e * 13 + 9 + c) * NP + p];
        for (int v = 0; v < 5; ++v) {
            const int64_t gi = ((int64_t)v * E + e) * NP + p;
            av[k][v] = useA ? S_.A[gi] : 0.0;
            bv[k][v] = useB ? S_.B[gi] : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= E) continue;
        const double iJ = gq[k][0];
        const double g0 = P.GM * gq[k][1], g1 = P.GM * gq[k][2], g2 = P.GM * gq[k][3];
        const int ps = lds_sol<N>(p);
        const double rho = sq[el][0][ps], mx = sq[el][1][ps], my = sq[el][2][ps], mz = sq[el][3][ps];
        double M[5];
        M[0] = 0.0;
        M[1] = rho * g0 - 2.0 * P.omega * my;
        M[2] = rho * g1 + 2.0 * P.omega * mx;
        M[3] = rho * g2;
        M[4] = mx * g0 + my * g1 + mz * g2;
        for (int v = 0; v < 5; ++v) {
            const double R = -div[k][v] * iJ - M[v];
            const int64_t gi = ((int64_t)v * E + e) * NP + p;
            if (!rk) {
                S_.Qout[gi] = R;
                continue;
            }
            const double q = sq[el][v][ps];
            if (useT) S_.Tout[gi] = S_.d0 * bv[k][v] + S_.d1 * (q + S_.d2 * R);
            S_.Qout[gi] = S_.c0 * av[k][v] + S_.c1 * (q + S_.c2 * R);
        }
    }
}

// Lift pass: the neighbours' viscous halves at interior interface points
// enter the divergence through the end columns of the derivative matrix;
// -(1/|J|) times that lift is added in place to the flux pass's outputs
// with their stage weights (Qout: c1 c2, Tout: d1 d2; residual mode: 1);
// the face traces of the new state are pushed to the neighbours.
// NV: components per mailbox point (4: momentum and energy; 5 with the
// subgrid flux, whose mass part need not vanish)
template <int N, int EPB, int NT, int NV>
__global__ __launch_bounds__(NT) void k_lift64(Ops<N> opa, Geo G, const double *__restrict__ TV, StageArgs S_) {
    constexpr int NP = N * N * N, NF2 = N * N, MBE = 6 * NV * NF2;
    constexpr int IT_MB = (EPB * MBE + NT - 1) / NT, IT_SOL = (EPB * NP + NT - 1) / NT;
    __shared__ double nv[EPB][6][NV][NF2];  // neighbours' viscous flux at own face points, 0 off interfaces
    __shared__ double sq[EPB][5][NP];      // the new state, for the traces
    __shared__ int32_t lk[EPB][6], inf[EPB][6];
    __shared__ Ops<N> op;
    // blocks walk the elements from the last to the first: the flux pass
    // before ran from the first to the last, so the first blocks here read
    // its latest writes, which are still in the memory-side cache; the next
    // flux pass starts where this pass ends, for the same reason
    const int64_t e0 = (int64_t)(gridDim.x - 1 - blockIdx.x) * EPB, E = G.E;
    const bool useT = S_.mode != 0 && S_.Tout != nullptr;
    // every global input first (unpredicated, clamped; the mailbox slots of
    // boundary faces are never written and are selected away below)
    int32_t rl, ri;
    {
        const bool okl = (int)threadIdx.x < EPB * 6 && e0 + threadIdx.x / 6 < E;
        const int32_t l = G.link[okl ? e0 * 6 + threadIdx.x : 0], i = G.info[okl ? e0 * 6 + threadIdx.x : 0];
        rl = okl ? l : -1;
        ri = okl ? i : 0;
    }
    double mb[IT_MB];
#pragma unroll
    for (int k = 0; k < IT_MB; ++k) {
        const int it = threadIdx.x + k * NT;
        const bool ok = it < EPB * MBE && e0 + it / MBE < E;
        mb[k] = ld_once(&TV[ok ? e0 * MBE + it : 0]);
    }
    double qo[IT_SOL][5], to[IT_SOL][5], iJ[IT_SOL], r0[IT_SOL][5];
    const bool bal = S_.R0 != nullptr;
#pragma unroll
    for (int k = 0; k < IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / NP, p = it % NP;
        const int64_t e = (it < EPB * NP && e0 + el < E) ? e0 + el : 0;
        iJ[k] = ld_once(&G.solgeo[(e * 13 + 9) * NP + p]);
        for (int v = 0; v < 5; ++v) {
            const int64_t gi = ((int64_t)v * E + e) * NP + p;
            qo[k][v] = S_.Qout[gi];
            to[k][v] = useT ? S_.Tout[gi] : 0.0;
            r0[k][v] = bal ? S_.R0[gi] : 0.0;
        }
    }
    ops_to_lds(opa, op);
    if ((int)threadIdx.x < EPB * 6) {
        lk[threadIdx.x / 6][threadIdx.x % 6] = rl;
        inf[threadIdx.x / 6][threadIdx.x % 6] = ri;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IT_MB; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * MBE) break;
        const int el = it / MBE, r = it % MBE, f = r / (NV * NF2);
        (&nv[el][0][0][0])[r] = (lk[el][f] >= 0) ? mb[k] : 0.0;
    }
    __syncthreads();
    const double wP = (S_.mode == 0) ? 1.0 : S_.c1 * S_.c2, wT = S_.d1 * S_.d2;
#pragma unroll
    for (int k = 0; k < IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= E) continue;
        double corr[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int pp = t1 + N * t2;
            const double wl = -0.5 * op.D[a][0], wu = 0.5 * op.D[a][N];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                corr[v + 5 - NV] += wl * nv[el][2 * d][v][pp] + wu * nv[el][2 * d + 1][v][pp];
        }
        for (int v = 0; v < 5; ++v) {
            const int64_t gi = ((int64_t)v * E + e) * NP + p;
            const double x = -iJ[k] * corr[v];
            // balanced mode: the background residual leaves R after the
            // lift (at Q = Q0 a residual call then gives exactly zero)
            const double qn = bal ? (qo[k][v] + wP * x) - wP * r0[k][v] : qo[k][v] + wP * x;
            S_.Qout[gi] = qn;
            if (useT) S_.Tout[gi] = bal ? (to[k][v] + wT * x) - wT * r0[k][v] : to[k][v] + wT * x;
            sq[el][v][lds_sol<N>(p)] = qn;
        }
    }
    if (S_.mode == 0 || S_.TQout == nullptr) return;
    __syncthreads();
    push_traces64<N, EPB, NT, true>(op, G, e0, lk, inf, sq, S_.TQout);
}

// entropy gradient of a state at rest along the flux-point metric:
// out[e][d][fl] = grad S . (|J| grad xi_d) at the d-flux points, with the BR1
// gradients of the FP64 path (S = c_p ln(p^(1/gamma)/rho), p = (gamma-1) E
// for zero momentum); used by the mixed-precision path
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_bg_entropy(Ops<N> opa, Geo G, PhysParams P, const double *__restrict__ Q0,
                                                   const double *__restrict__ TQ, float *__restrict__ out,
                                                   float *__restrict__ gout) {
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
    // gradient of rho0 at the solution points: gout[e][3][NP]
    for (int it = threadIdx.x; it < EPB * 3 * NP; it += NT) {
        const int el = it / (3 * NP), r = it % (3 * NP), k = r / NP, p = r % NP;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        gout[(e * 3 + k) * NP + p] = (float)sgr[el][k][p];
    }
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
static hipError_t launch_trace_push_t(const Mesh &m, const Geo &G, const double *Q, double *TQ, hipStream_t s) {
    constexpr int EPB = Cfg64<N>::EPB, NT = Cfg64<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_trace_push<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, make_ops<N>(m.basis), G, Q, TQ);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_flux64_t(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q,
                                  const double *TQ, double *TV, const StageArgs &sa, const ClosureArgs &C,
                                  hipStream_t s) {
    constexpr int EPB = Cfg64<N>::EPB, NT = Cfg64<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    const bool rad = P.kappa_r1 != 0.0 || P.kappa_r2 != 0.0;
    if (C.model) {
        // the flux pass with the network inside
        if constexpr (N == 3) {
            if (rad)
                hipLaunchKernelGGL((k_flux64<N, EPB, NT, 2, true>), dim3(nb), dim3(NT), 0, s, make_ops<N>(m.basis),
                                   G, P, Q, TQ, TV, sa, C);
            else
                hipLaunchKernelGGL((k_flux64<N, EPB, NT, 2, false>), dim3(nb), dim3(NT), 0, s, make_ops<N>(m.basis),
                                   G, P, Q, TQ, TV, sa, C);
        } else {
            return hipErrorInvalidValue;
        }
    } else if (rad) {
        hipLaunchKernelGGL((k_flux64<N, EPB, NT, 0, true>), dim3(nb), dim3(NT), 0, s, make_ops<N>(m.basis), G, P, Q,
                           TQ, TV, sa, C);
    } else {
        hipLaunchKernelGGL((k_flux64<N, EPB, NT, 0, false>), dim3(nb), dim3(NT), 0, s, make_ops<N>(m.basis), G, P, Q,
                           TQ, TV, sa, C);
    }
    return hipGetLastError();
}

template <int N>
static hipError_t launch_lift64_t(const Mesh &m, const Geo &G, const double *TV, const StageArgs &sa, bool closure,
                                  hipStream_t s) {
    constexpr int EPB = Cfg64<N>::EPB, NT = Cfg64<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    if (closure)
        hipLaunchKernelGGL((k_lift64<N, EPB, NT, 5>), dim3(nb), dim3(NT), 0, s, make_ops<N>(m.basis), G, TV, sa);
    else
        hipLaunchKernelGGL((k_lift64<N, EPB, NT, 4>), dim3(nb), dim3(NT), 0, s, make_ops<N>(m.basis), G, TV, sa);
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
template <int N>
static hipError_t launch_closure_tau_t(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q,
                                       const double *TQ, const ClosureArgs &C, hipStream_t s) {
    if constexpr (N == 3) {
        constexpr int EPB = Cfg64<N>::EPB, NT = Cfg64<N>::NT;
        const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
        const StageArgs none{nullptr, nullptr, nullptr, 0.0, 0.0, 0.0, nullptr, nullptr, 0.0, 0.0, 0.0, 0};
        hipLaunchKernelGGL((k_flux64<N, EPB, NT, 1, false>), dim3(nb), dim3(NT), 0, s, make_ops<N>(m.basis), G, P, Q,
                           TQ, nullptr, none, C);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_closure_tau(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q, const double *TQ,
                              const ClosureArgs &C, hipStream_t s) {
#define C_(n) launch_closure_tau_t<n>(m, G, P, Q, TQ, C, s)
    CHORUS_DISPATCH(m.N, C_)
#undef C_
}
hipError_t launch_trace_push(const Mesh &m, const Geo &G, const double *Q, double *TQ, hipStream_t s) {
#define C_(n) launch_trace_push_t<n>(m, G, Q, TQ, s)
    CHORUS_DISPATCH(m.N, C_)
#undef C_
}
hipError_t launch_flux64(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q, const double *TQ,
                         double *TV, const StageArgs &sa, const ClosureArgs &C, hipStream_t s) {
#define C_(n) launch_flux64_t<n>(m, G, P, Q, TQ, TV, sa, C, s)
    CHORUS_DISPATCH(m.N, C_)
#undef C_
}
hipError_t launch_lift64(const Mesh &m, const Geo &G, const double *TV, const StageArgs &sa, bool closure,
                         hipStream_t s) {
#define C_(n) launch_lift64_t<n>(m, G, TV, sa, closure, s)
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
                                      const double *TQ, float *out, float *gout, hipStream_t s) {
    constexpr int EPB = Cfg<N>::EPB, NT = Cfg<N>::NT;
    const Ops<N> op = make_ops<N>(m.basis);
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_bg_entropy<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, op, G, P, Q0, TQ, out, gout);
    return hipGetLastError();
}

hipError_t launch_bg_entropy(const Mesh &m, const Geo &G, const PhysParams &P, const double *Q0, const double *TQ,
                             float *out, float *gout, hipStream_t s) {
#define C_(n) launch_bg_entropy_t<n>(m, G, P, Q0, TQ, out, gout, s)
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
