// Mixed-precision SD kernels (gfx950): FP64 state and SSP-RK3 accumulation,
// FP32 interpolation, fluxes and derivatives on perturbations about a
// hydrostatic background at rest (Q0 with zero momentum).
//
// Split of the residual (exact algebra; only rounding differs):
//   R(Q) = R0 + dR,  R0 = R(Q0) computed once in FP64 (stored FP32), and
//   dR = R(Q) - R(Q0) evaluated from P = Q - Q0 without cancellation:
//   * gradients are linear: grad Q = grad Q0 + grad P, each from its own
//     BR1 common values (the wall state enters in perturbation form);
//   * inviscid:  mass m'.S, momentum m'(m'.S)/rho + p'S,
//                energy (gamma E0 + E' + p')(m'.S)/rho,
//                p' = (gamma-1)(E' - |m'|^2/(2 rho));
//   * Rusanov:   1/2 (dF_L + dF_R) - 1/2 |S| [lam (P_R - P_L) + (lam - lam0) dQ0],
//                lam - lam0 formed from the small quantities |u.n| + (c - c0)
//                and the background sound-speed jump;
//   * viscous:   tau(Q) (tau0 = 0), and the diffusive energy flux as
//                kappa/R [p' (gS0.S) + p ((gS - gS0).S)] + kappa_r terms, with
//                (gS - gS0).S written through grad P and the background
//                gradients, and gS0.S (the background entropy gradient along
//                S) computed in FP64 once;
//   * source:    M(P) (linear).
// FP32 rounding therefore scales with the perturbation, and the hydrostatic
// and isentropic cancellations of the background stay in FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"
#include "sd_common.hpp"

namespace chorus {

template <int N>
using OpsF = OpsT<float, N>;

// hardware reciprocal (1 ulp): every FP32 quantity here is
// perturbation-scaled, so this rounding is of the same order as the FP32
// arithmetic itself
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ---------------------------------------------------------------------------
// views
// ---------------------------------------------------------------------------
struct GeoF {
    const float *solgeo;   // [E][13][NP]
    const float *fluxgeo;  // [E][3][3][NFL]
    const int32_t *link;   // [E][6]
    const int32_t *info;   // [E][6]
    int64_t E;
    const float *rflux;    // [E][3][NFL] radius at the d-flux points
};

struct MixedBufs {
    const float *bg;    // [E][2][NP]    rho0, E0
    const float *dbg;   // [E][6][2][NF2] neighbour minus own background face trace (rho, E)
    const float *gS0;   // [E][3][NFL]   grad S0 . (|J| grad xi_d) at d-flux points
    const float *R0;    // [5][E][NP]    R(Q0)
    const float *gbg;   // [E][3][NP]    grad rho0 at the solution points (from FP64, once)
};

struct PhysF {
    float gm1, gam, R, cp, icp, GM, om, nu, kappa, kappa_r, RT_top;  // RT_top <= 0: off
    float kappa_r1, kappa_r2;                                    // kappa_r(r) = kappa_r + kappa_r1 r + kappa_r2 r^2
};

__device__ __forceinline__ PhysF physf_of(const PhysParams &P) {
    PhysF f;
    f.gm1 = (float)(P.gamma - 1.0);
    f.gam = (float)P.gamma;
    f.R = (float)P.R_gas;
    f.cp = (float)P.cp;
    f.icp = (float)(1.0 / P.cp);
    f.GM = (float)P.GM;
    f.om = (float)P.omega;
    f.nu = (float)P.nu;
    f.kappa = (float)P.kappa;
    f.kappa_r = (float)P.kappa_r;
    f.RT_top = (P.T_top > 0.0) ? (float)(P.R_gas * P.T_top) : -1.0f;
    f.kappa_r1 = (float)P.kappa_r1;
    f.kappa_r2 = (float)P.kappa_r2;
    return f;
}

// radiative-diffusivity variants of the flux pass: none, constant, radial
enum { KR_NONE = 0, KR_CONST = 1, KR_RADIAL = 2 };

// radiative diffusivity at a flux point from the value read with its
// geometry (the radius for KR_RADIAL)
template <int KR>
__device__ __forceinline__ float kr_of(const PhysF &F, float loaded) {
    if constexpr (KR == KR_RADIAL) return F.kappa_r + loaded * (F.kappa_r1 + loaded * F.kappa_r2);
    else return F.kappa_r;
}

// LDS field slots at solution points: perturbation (5), background (2)
enum { F_RP = 0, F_MX = 1, F_MY = 2, F_MZ = 3, F_EP = 4, F_R0 = 5, F_E0 = 6, NFIELD = 7 };
// gradient slots: field f, component c at slot 3 f + c (the perturbation
// fields and rho0; grad E0 enters only along S, through the background
// entropy gradient: see dflux_viscous)
constexpr int NGRAD = 3 * (F_R0 + 1);

// point state at a flux point: background and perturbation values and
// gradients (full gradient = background + perturbation)
struct PtState {
    float r0, E0, rp, m[3], Ep;          // values
    float gr0[3];                        // background density gradient
    float grp[3], gm[3][3], gEp[3];      // perturbation gradients
};

// ---------------------------------------------------------------------------
// pointwise perturbation physics
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dflux_inviscid(const PtState &s, const float S[3], const PhysF &F, float out[5]) {
    const float rho = s.r0 + s.rp, E = s.E0 + s.Ep;
    const float inv = rcp(rho);
    const float mS = s.m[0] * S[0] + s.m[1] * S[1] + s.m[2] * S[2];
    const float mm = s.m[0] * s.m[0] + s.m[1] * s.m[1] + s.m[2] * s.m[2];
    const float pp = F.gm1 * (s.Ep - 0.5f * mm * inv);
    const float uS = mS * inv;
    out[0] = mS;
    out[1] = s.m[0] * uS + pp * S[0];
    out[2] = s.m[1] * uS + pp * S[1];
    out[3] = s.m[2] * uS + pp * S[2];
    out[4] = (F.gam * E - F.gm1 * s.Ep + pp) * uS;
}

// (F_v(Q) - F_v(Q0)) . S given gS0S = grad S0 . S.  outer_wall / inner_wall
// select the wall forms (normal traction only; energy as interior at the
// outer wall, none at the inner wall where the prescribed flux is in R0).
// (kr: the radiative diffusivity at the point, used unless KR == KR_NONE)
template <int KR>
__device__ __forceinline__ void dflux_viscous(const PtState &s, const float S[3], float gS0S, const PhysF &F,
                                              float kr, int wall, float out[5]) {
    // with mu = rho nu and du_a/dx_c = (dm_a/dx_c - u_a drho/dx_c) / rho, the
    // stress along S needs the momentum gradient only through its
    // contractions with S: Y_a = sum_c dm_a/dx_c S_c (also in grad p' . S)
    // and Z_a = sum_b dm_b/dx_a S_b
    const float rho = s.r0 + s.rp, inv = rcp(rho);
    const float u[3] = {s.m[0] * inv, s.m[1] * inv, s.m[2] * inv};
    float grho[3];
    for (int c = 0; c < 3; ++c) grho[c] = s.gr0[c] + s.grp[c];
    const float gr0S = s.gr0[0] * S[0] + s.gr0[1] * S[1] + s.gr0[2] * S[2];
    const float grpS = s.grp[0] * S[0] + s.grp[1] * S[1] + s.grp[2] * S[2];
    const float grhoS = gr0S + grpS;
    const float uS = u[0] * S[0] + u[1] * S[1] + u[2] * S[2];
    const float ug = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
    float Y[3];
    for (int a = 0; a < 3; ++a) Y[a] = s.gm[a][0] * S[0] + s.gm[a][1] * S[1] + s.gm[a][2] * S[2];
    // (2/3) rho div u
    const float dv = (2.0f / 3.0f) * (s.gm[0][0] + s.gm[1][1] + s.gm[2][2] - ug);
    float tS[3];
    if (wall == 0) {
        for (int a = 0; a < 3; ++a) {
            const float Za = s.gm[0][a] * S[0] + s.gm[1][a] * S[1] + s.gm[2][a] * S[2];
            tS[a] = F.nu * (Y[a] + Za - u[a] * grhoS - uS * grho[a] - dv * S[a]);
        }
    } else {
        // normal traction: n . tau . n = mu (2 S.grad u.S / |S|^2 - 2/3 div u)
        const float A2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
        const float SY = S[0] * Y[0] + S[1] * Y[1] + S[2] * Y[2];
        const float tnn = F.nu * (2.0f * (SY - uS * grhoS) * rcp(A2) - dv);
        for (int a = 0; a < 3; ++a) tS[a] = tnn * S[a];
    }
    out[0] = 0.0f;
    out[1] = tS[0];
    out[2] = tS[1];
    out[3] = tS[2];
    if (wall == 1) {  // inner wall: stress free, no viscous work, energy flux in R0
        out[4] = 0.0f;
        return;
    }
    // p' and grad p' . S (m0 = 0, u0 = 0)
    const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const float pp = F.gm1 * (s.Ep - 0.5f * uu * rho);
    const float p0 = F.gm1 * s.E0, p = p0 + pp;
    const float gEpS = s.gEp[0] * S[0] + s.gEp[1] * S[1] + s.gEp[2] * S[2];
    const float gpS = F.gm1 * (gEpS - (u[0] * Y[0] + u[1] * Y[1] + u[2] * Y[2]) + 0.5f * uu * grhoS);
    // (grad S - grad S0).S / c_p with grad p0 . S / p0 = gamma (gS0S / c_p
    // + grad rho0 . S / rho0), the background entropy gradient's definition
    const float igp = rcp(F.gam * p), ir0 = rcp(s.r0);
    const float dgS = igp * (gpS - F.gam * pp * (gS0S * F.icp + gr0S * ir0)) - inv * (grpS - gr0S * s.rp * ir0);
    // rho T grad S . S - rho0 T0 grad S0 . S = (p' gS0S + p c_p dgS) / R
    const float iR = rcp(F.R);
    const float eS = F.kappa * (pp * gS0S + p * F.cp * dgS) * iR;
    // rho c_p grad T . S difference: c_p/R (grad p' . S - [p grad rho' . S / rho + grad rho0 . S (p/rho - p0/rho0)])
    float eT = 0.0f;
    if constexpr (KR != KR_NONE) {
        const float dpr = (pp * s.r0 - p0 * s.rp) * inv * ir0;
        eT = kr * F.cp * iR * (gpS - (p * grpS * inv + gr0S * dpr));
    }
    const float work = (wall == 0) ? (u[0] * tS[0] + u[1] * tS[1] + u[2] * tS[2]) : 0.0f;
    out[4] = work + eS + eT;
}

// ---------------------------------------------------------------------------
// element phases (generic N; items per thread fixed at compile time)
// ---------------------------------------------------------------------------
template <int N>
struct MixedLds {
    static constexpr int NP = N * N * N, NF2 = N * N, NFL = (N + 1) * N * N;
    float f[NFIELD][NP];          // perturbation + background fields
    float plo[5][NP];             // FP64 perturbation minus its FP32 value f[0..4] (stage update)
    float g[NGRAD][NP];           // gradients
    union {
        float cs[5][6][NF2];       // common values of the perturbation
        float ft[5][NFL];          // transformed flux of one direction, written after cs is consumed
    } u;
    int32_t lk[6], inf[6];        // neighbour element and info word per face
};

template <int N, int EPB, int NT>
struct Shape {
    static constexpr int NP = N * N * N, NF2 = N * N, NFL = (N + 1) * N * N;
    static constexpr int IT_SOL = (EPB * NP + NT - 1) / NT;
    static constexpr int IT_FACE = (EPB * 6 * NF2 + NT - 1) / NT;
    static constexpr int IT_FLUX = (EPB * 3 * NFL + NT - 1) / NT;
    static constexpr int NINTD = (N - 1) * N * N;     // interior flux points per element and direction
    static constexpr int IT_INTD = (EPB * NINTD + NT - 1) / NT;
    static constexpr int MB = 6 * 5 * NF2;             // mailbox floats per element
    static constexpr int DB = 6 * 2 * NF2;
};

// registers holding one thread's share of an element block's global inputs;
// everything is issued before the first use so that a block waits for
// memory once.  Items past the last element (or past the block's item
// count) load element 0's data through a clamped index: no load is
// predicated (a guarded load compiles to a branch that waits for it at
// once) and those items are never stored.
template <int N, int EPB, int NT>
struct Prologue {
    using Sh = Shape<N, EPB, NT>;
    double P[Sh::IT_SOL][5];
    float bg[Sh::IT_SOL][2];
    float gs[Sh::IT_SOL][9];
    float gb[Sh::IT_SOL][3];  // background density gradient
    // neighbour data at this thread's face items (face item it: el, f, pp):
    // perturbation trace, background jump
    float nq[Sh::IT_FACE][5], db[Sh::IT_FACE][2];
    int32_t lk, inf;
};

template <int N, int EPB, int NT>
__device__ __forceinline__ void prologue_load(const double *Pq, const MixedBufs &B, const GeoF &G,
                                              const float *__restrict__ TQ, int64_t e0, Prologue<N, EPB, NT> &R) {
    using Sh = Shape<N, EPB, NT>;
    constexpr int NP = Sh::NP, NF2 = Sh::NF2;
    const int64_t E = G.E;
    // issued in the order of first use, so that each phase waits only for
    // its own inputs: links, the LDS fields, the neighbour traces (common
    // values)
    {
        const int it = threadIdx.x;
        const bool okl = it < EPB * 6 && e0 + it / 6 < E;
        const int32_t lk = G.link[okl ? e0 * 6 + it : 0], inf = G.info[okl ? e0 * 6 + it : 0];
        R.lk = okl ? lk : -1;
        R.inf = okl ? inf : 0;
    }
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / NP, p = it % NP;
        const int64_t e = (it < EPB * NP && e0 + el < E) ? e0 + el : 0;
        for (int v = 0; v < 5; ++v) R.P[k][v] = Pq[((int64_t)v * E + e) * NP + p];
        R.bg[k][0] = B.bg[(e * 2 + 0) * NP + p];
        R.bg[k][1] = B.bg[(e * 2 + 1) * NP + p];
        for (int t = 0; t < 3; ++t) R.gb[k][t] = B.gbg[(e * 3 + t) * NP + p];
    }
#pragma unroll
    for (int k = 0; k < Sh::IT_FACE; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = (it < EPB * 6 * NF2 && e0 + el < E) ? e0 + el : 0;
        const int64_t base = e * 6 + f;
        for (int v = 0; v < 5; ++v) R.nq[k][v] = TQ[(base * 5 + v) * NF2 + pp];
        R.db[k][0] = B.dbg[(base * 2 + 0) * NF2 + pp];
        R.db[k][1] = B.dbg[(base * 2 + 1) * NF2 + pp];
    }
}

// the solution-point metrics (first used by the gradients)
template <int N, int EPB, int NT>
__device__ __forceinline__ void prologue_load_metrics(const GeoF &G, int64_t e0, Prologue<N, EPB, NT> &R) {
    using Sh = Shape<N, EPB, NT>;
    constexpr int NP = Sh::NP;
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / NP, p = it % NP;
        const int64_t e = (it < EPB * NP && e0 + el < G.E) ? e0 + el : 0;
        for (int t = 0; t < 9; ++t) R.gs[k][t] = G.solgeo[(e * 13 + t) * NP + p];
    }
}

// move the prologue registers into the element LDS
template <int N, int EPB, int NT>
__device__ __forceinline__ void prologue_store(const Prologue<N, EPB, NT> &R, MixedLds<N> *L) {
    using Sh = Shape<N, EPB, NT>;
    constexpr int NP = Sh::NP;
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        const int el = it / NP, p = it % NP;
        for (int v = 0; v < 5; ++v) {
            const float hi = (float)R.P[k][v];
            L[el].f[v][p] = hi;
            L[el].plo[v][p] = (float)(R.P[k][v] - (double)hi);
        }
        L[el].f[F_R0][p] = R.bg[k][0];
        L[el].f[F_E0][p] = R.bg[k][1];
        for (int c = 0; c < 3; ++c) L[el].g[3 * F_R0 + c][p] = R.gb[k][c];
    }
    if ((int)threadIdx.x < EPB * 6) {
        L[threadIdx.x / 6].lk[threadIdx.x % 6] = R.lk;
        L[threadIdx.x / 6].inf[threadIdx.x % 6] = R.inf;
    }
}

// interpolation of a field stored in LDS at flux point m of the line
// (base, st)
template <int N>
__device__ __forceinline__ float line_val(const OpsF<N> &op, const float *fld, int m, int base, int st) {
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b < N; ++b) s += op.I[m][b] * fld[base + b * st];
    return s;
}

// BR1 common values of the perturbation at the 6 N^2 face points (the
// background's gradients are computed once, in FP64, at set-up); the own
// face values of the 7 fields at the thread's face items are kept in fo when
// given: the face-flux phase reuses them
template <int N, int EPB, int NT>
__device__ __forceinline__ void common_values(const OpsF<N> &op, const GeoF &G, const PhysF &F, int64_t e0,
                                              MixedLds<N> *L, const Prologue<N, EPB, NT> &R,
                                              float (*fo)[NFIELD], const float (*Sf)[3]) {
    using Sh = Shape<N, EPB, NT>;
    constexpr int NF2 = N * N, NFL = (N + 1) * N * N;
#pragma unroll
    for (int k = 0; k < Sh::IT_FACE; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * 6 * NF2) break;
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        MixedLds<N> &l = L[el];
        const int t1 = pp % N, t2 = pp / N;
        const int d = f >> 1, m = (f & 1) ? N : 0, base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d);
        float pv[5];
        for (int v = 0; v < 5; ++v) pv[v] = line_val<N>(op, l.f[v], m, base, st);
        const float r0 = line_val<N>(op, l.f[F_R0], m, base, st), E0 = line_val<N>(op, l.f[F_E0], m, base, st);
        if (fo) {
            for (int v = 0; v < 5; ++v) fo[k][v] = pv[v];
            fo[k][F_R0] = r0;
            fo[k][F_E0] = E0;
        }
        const int32_t nb = l.lk[f], inf = l.inf[f];
        if (nb >= 0) {
            for (int v = 0; v < 5; ++v) l.u.cs[v][f][pp] = 0.5f * (pv[v] + R.nq[k][v]);
        } else {
            // wall state in perturbation form: rho' kept, normal momentum
            // removed, pressure kept (outer wall with T_top: p = rho R T_top)
            // (the normal projection is the same along +-S: the thread's
            // flux-point metric Sf serves)
            const bool outer = ((inf >> 6) - 1) == CHORUS_BC_OUTER;
            const float *S = Sf[k];
            const float A2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
            const float mn = (pv[1] * S[0] + pv[2] * S[1] + pv[3] * S[2]) * rcp(A2);
            float mb[3];
            for (int a = 0; a < 3; ++a) mb[a] = pv[1 + a] - mn * S[a];
            const float irho = rcp(r0 + pv[0]), igm1 = rcp(F.gm1);
            const float mm = pv[1] * pv[1] + pv[2] * pv[2] + pv[3] * pv[3];
            const float mbb = mb[0] * mb[0] + mb[1] * mb[1] + mb[2] * mb[2];
            float Eb;  // E_b - E0_b
            if (outer && F.RT_top > 0.0f) Eb = F.RT_top * pv[0] * igm1 + 0.5f * mbb * irho;
            else Eb = pv[4] + 0.5f * (mbb - mm) * irho;
            l.u.cs[0][f][pp] = pv[0];
            for (int a = 0; a < 3; ++a) l.u.cs[1 + a][f][pp] = mb[a];
            l.u.cs[4][f][pp] = Eb;
        }
    }
}

// gradients of the 5 perturbation fields at the solution points (those of
// the background are loaded)
template <int N, int EPB, int NT>
__device__ __forceinline__ void gradients(const OpsF<N> &op, const GeoF &G, int64_t e0, MixedLds<N> *L,
                                          const float (*gsol)[9]) {
    using Sh = Shape<N, EPB, NT>;
    constexpr int NP = N * N * N;
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        MixedLds<N> &l = L[el];
        const float *Gm = gsol[k];
        float dq[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int base = sol_of<N>(d, 0, t1, t2), st = stride_of<N>(d), pp = t1 + N * t2;
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                float s = op.D[a][0] * l.u.cs[v][2 * d][pp] + op.D[a][N] * l.u.cs[v][2 * d + 1][pp];
#pragma unroll
                for (int b = 0; b < N; ++b) s += op.B[a][b] * l.f[v][base + b * st];
                dq[d][v] = s;
            }
        }
#pragma unroll
        for (int v = 0; v < 5; ++v)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                l.g[3 * v + c][p] = Gm[c] * dq[0][v] + Gm[3 + c] * dq[1][v] + Gm[6 + c] * dq[2][v];
    }
}

// point state at the flux point m of the line (base, st); with vals given,
// the 7 field values are taken from there and only the gradients are
// interpolated
template <int N>
__device__ __forceinline__ void state_at(const OpsF<N> &op, const MixedLds<N> &l, int m, int base, int st,
                                         PtState &s, const float *vals = nullptr) {
    float w[N];
#pragma unroll
    for (int b = 0; b < N; ++b) w[b] = op.I[m][b];
    auto I = [&](const float *fld) {
        float t = 0.0f;
#pragma unroll
        for (int b = 0; b < N; ++b) t += w[b] * fld[base + b * st];
        return t;
    };
    if (vals) {
        s.rp = vals[F_RP];
        s.m[0] = vals[F_MX];
        s.m[1] = vals[F_MY];
        s.m[2] = vals[F_MZ];
        s.Ep = vals[F_EP];
        s.r0 = vals[F_R0];
        s.E0 = vals[F_E0];
    } else {
        s.rp = I(l.f[F_RP]);
        s.m[0] = I(l.f[F_MX]);
        s.m[1] = I(l.f[F_MY]);
        s.m[2] = I(l.f[F_MZ]);
        s.Ep = I(l.f[F_EP]);
        s.r0 = I(l.f[F_R0]);
        s.E0 = I(l.f[F_E0]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        s.grp[c] = I(l.g[3 * F_RP + c]);
        s.gm[0][c] = I(l.g[3 * F_MX + c]);
        s.gm[1][c] = I(l.g[3 * F_MY + c]);
        s.gm[2][c] = I(l.g[3 * F_MZ + c]);
        s.gEp[c] = I(l.g[3 * F_EP + c]);
        s.gr0[c] = I(l.g[3 * F_R0 + c]);
    }
}

// Own-side part of the common transformed flux difference at a face point,
// along the outward area vector So.  Interior face: the Rusanov flux of the
// own state s and the neighbour state (perturbation trace nq, background
// jump db) minus half of the own viscous flux fv (the neighbour's half is
// added by the lift pass from the neighbour's viscous trace).  Wall
// face: the complete wall flux (inviscid (0, p' So, 0); viscous wall form).
template <int KR>
__device__ __forceinline__ void face_flux_own(const PtState &s, const float nq[5], const float db[2], bool interior,
                                              bool outer, const float So[3], float gS0S, float kr,
                                              const float fv_in[5], const PhysF &F, float phi[5]) {
    if (interior) {
        PtState r = s;
        r.rp = nq[0];
        r.m[0] = nq[1];
        r.m[1] = nq[2];
        r.m[2] = nq[3];
        r.Ep = nq[4];
        const float dr0 = db[0], dE0 = db[1];
        r.r0 = s.r0 + dr0;
        r.E0 = s.E0 + dE0;
        float fL[5], fR[5];
        dflux_inviscid(s, So, F, fL);
        dflux_inviscid(r, So, F, fR);
        const float A = sqrtf(So[0] * So[0] + So[1] * So[1] + So[2] * So[2]), iA = rcp(A);
        // |u.n| + (c - c0) on each side; c^2 - c0^2 = gamma (p' rho0 - p0 rho') / (rho rho0)
        auto excess = [&](const PtState &q, float &c0) {
            const float inv = rcp(q.r0 + q.rp), ir0 = rcp(q.r0);
            const float un = fabsf((q.m[0] * So[0] + q.m[1] * So[1] + q.m[2] * So[2]) * iA * inv);
            const float mm = q.m[0] * q.m[0] + q.m[1] * q.m[1] + q.m[2] * q.m[2];
            const float pp_ = F.gm1 * (q.Ep - 0.5f * mm * inv), p0 = F.gm1 * q.E0;
            c0 = sqrtf(F.gam * p0 * ir0);
            const float dc2 = F.gam * (pp_ * q.r0 - p0 * q.rp) * inv * ir0;
            const float c = sqrtf(c0 * c0 + dc2);
            return un + dc2 * rcp(c + c0);
        };
        float c0L, c0R;
        const float eL = excess(s, c0L), eR = excess(r, c0R);
        // background sound-speed jump c0R - c0L from the FP64 background jump
        const float dc0 = F.gam * F.gm1 * (dE0 * s.r0 - s.E0 * dr0) * rcp(s.r0 * r.r0 * (c0L + c0R));
        const float dlam = fmaxf(eL, eR + dc0) - fmaxf(0.0f, dc0);
        const float lam0 = c0L + fmaxf(0.0f, dc0);
        const float hl = 0.5f * (lam0 + dlam) * A, hd = 0.5f * dlam * A;
        const float pR[5] = {r.rp, r.m[0], r.m[1], r.m[2], r.Ep};
        const float pL[5] = {s.rp, s.m[0], s.m[1], s.m[2], s.Ep};
        const float dq0[5] = {dr0, 0.0f, 0.0f, 0.0f, dE0};
        for (int v = 0; v < 5; ++v)
            phi[v] = 0.5f * (fL[v] + fR[v]) - hl * (pR[v] - pL[v]) - hd * dq0[v] - 0.5f * fv_in[v];
    } else {
        const float mm = s.m[0] * s.m[0] + s.m[1] * s.m[1] + s.m[2] * s.m[2];
        const float pp = F.gm1 * (s.Ep - 0.5f * mm * rcp(s.r0 + s.rp));
        float fv[5];
        dflux_viscous<KR>(s, So, gS0S, F, kr, outer ? 2 : 1, fv);
        phi[0] = 0.0f;
        for (int a = 0; a < 3; ++a) phi[1 + a] = pp * So[a] - fv[1 + a];
        phi[4] = -fv[4];
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// P = Q - Q0 (FP64) and the FP32 face traces of P
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_pert_begin(OpsF<N> opa, GeoF G, const double *__restrict__ Q,
                                                   const double *__restrict__ Q0, double *__restrict__ Pq,
                                                   float *__restrict__ TQ) {
    constexpr int NP = N * N * N, NF2 = N * N;
    __shared__ float sp[EPB][5][NP];
    __shared__ OpsF<N> op;
    ops_to_lds(opa, op);
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
        const int32_t nb = G.link[e * 6 + f];
        if (nb < 0) continue;
        const int64_t slot = mailbox_slot<N>(nb, G.info[e * 6 + f], pp);
        const int d = f >> 1, m = (f & 1) ? N : 0, base = sol_of<N>(d, 0, pp % N, pp / N), st = stride_of<N>(d);
        for (int v = 0; v < 5; ++v) TQ[slot + v * NF2] = line_val<N>(op, sp[el][v], m, base, st);
    }
}

// stage combination on P (see MixedStageArgs); mode 0 writes R0 + dR
using MixedStage = MixedStageArgs;

// ---------------------------------------------------------------------------
// flux pass + lift pass (the stage split used by the solver)
// ---------------------------------------------------------------------------
// Flux pass: every step that needs the gradients, once per stage.  Common
// values and gradients; at the face points the own viscous flux (pushed to
// the neighbour's viscous mailbox TV) and the own-side common flux (Rusanov
// minus half the own viscous flux, or the wall flux); at the interior flux
// points the transformed flux; the divergence of the flux polynomials with
// the own-side face fluxes at the line ends; the source.  The partial
// residual Rp = R0 - div/|J| - M, which lacks only the neighbours' viscous
// halves at interior interfaces, enters the stage combination here (FP64):
// Pout = c0 A + c1 (P + c2 Rp) (and Tout likewise), or Pout = Rp in
// residual mode; the lift pass adds the missing part in place.
template <int N, int EPB, int NT, int MINW, int KR>
__global__ __launch_bounds__(NT, MINW) void k_flux_mixed(OpsF<N> opa, GeoF G, MixedBufs B, PhysParams P,
                                                         const double *__restrict__ Pq, const float *__restrict__ TQ,
                                                         float *__restrict__ TV, MixedStage S_) {
    using Sh = Shape<N, EPB, NT>;
    constexpr int NP = Sh::NP, NF2 = Sh::NF2, NFL = Sh::NFL, NINTD = Sh::NINTD;
    __shared__ MixedLds<N> L[EPB];
    __shared__ OpsF<N> op;  // 1D operators (indexed per lane: LDS, not the argument segment)
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const PhysF F = physf_of(P);
    ops_to_lds(opa, op);
    // every global input of the element block, issued before the first wait
    // (unpredicated, clamped indices: see Prologue), in the order of first use
    Prologue<N, EPB, NT> R;
    prologue_load<N, EPB, NT>(Pq, B, G, TQ, e0, R);
    float Sf[Sh::IT_FACE][3], gSf[Sh::IT_FACE], krf[Sh::IT_FACE];
#pragma unroll
    for (int k = 0; k < Sh::IT_FACE; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = (it < EPB * 6 * NF2 && e0 + el < G.E) ? e0 + el : 0;
        const int d = f >> 1, fl = ((f & 1) ? N : 0) + (N + 1) * pp;
        // along +xi_d here; the face phase turns them outward
        for (int c = 0; c < 3; ++c) Sf[k][c] = G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
        gSf[k] = B.gS0[(e * 3 + d) * NFL + fl];
        krf[k] = (KR == KR_RADIAL) ? G.rflux[(e * 3 + d) * NFL + fl] : 0.0f;
    }
    prologue_load_metrics<N, EPB, NT>(G, e0, R);
    float Si[3][Sh::IT_INTD][3], gSi[3][Sh::IT_INTD], kri[3][Sh::IT_INTD];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < Sh::IT_INTD; ++k) {
            const int it = threadIdx.x + k * NT;
            const int el = it / NINTD, q = it % NINTD;
            const int fl = 1 + q % (N - 1) + (N + 1) * (q / (N - 1));
            const int64_t e = (it < EPB * NINTD && e0 + el < G.E) ? e0 + el : 0;
            for (int c = 0; c < 3; ++c) Si[d][k][c] = G.fluxgeo[((e * 3 + d) * 3 + c) * NFL + fl];
            gSi[d][k] = B.gS0[(e * 3 + d) * NFL + fl];
            kri[d][k] = (KR == KR_RADIAL) ? G.rflux[(e * 3 + d) * NFL + fl] : 0.0f;
        }
    prologue_store<N, EPB, NT>(R, L);
    __syncthreads();
    float fo[Sh::IT_FACE][NFIELD];
    common_values<N, EPB, NT>(op, G, F, e0, L, R, fo, Sf);
    __syncthreads();
    gradients<N, EPB, NT>(op, G, e0, L, R.gs);
    __syncthreads();
    // face points: own viscous flux to the neighbour, own-side common flux
    // kept in registers for the divergence
    float ffc[Sh::IT_FACE][5];
#pragma unroll
    for (int k = 0; k < Sh::IT_FACE; ++k) {
        const int it = threadIdx.x + k * NT;
        for (int v = 0; v < 5; ++v) ffc[k][v] = 0.0f;
        if (it >= EPB * 6 * NF2) break;
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        const int32_t nb = L[el].lk[f], inf = L[el].inf[f];
        const int d = f >> 1, m = (f & 1) ? N : 0, t1 = pp % N, t2 = pp / N;
        const float sg = (f & 1) ? 1.0f : -1.0f;
        const float So[3] = {sg * Sf[k][0], sg * Sf[k][1], sg * Sf[k][2]}, gSo = sg * gSf[k];
        float fv[5];
        PtState st;
        state_at<N>(op, L[el], m, sol_of<N>(d, 0, t1, t2), stride_of<N>(d), st, fo[k]);
        const float kr = kr_of<KR>(F, krf[k]);
        if (nb >= 0) {
            dflux_viscous<KR>(st, So, gSo, F, kr, 0, fv);
            // the viscous mass flux is zero: four components per point
            const int64_t slot = mailbox_slot<N, 4>(nb, inf, pp);
            for (int v = 1; v < 5; ++v) st_once(&TV[slot + (v - 1) * NF2], fv[v]);
        }
        face_flux_own<KR>(st, R.nq[k], R.db[k], nb >= 0, ((inf >> 6) - 1) == CHORUS_BC_OUTER, So, gSo, kr, fv,
                          F, ffc[k]);
    }
    // per direction d: transformed flux at the d-flux points, then its
    // derivative added to the divergence at the solution points
    float div[Sh::IT_SOL][5];
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k)
        for (int v = 0; v < 5; ++v) div[k][v] = 0.0f;
    // operands of the source and the stage combination, loaded before the
    // last divergence so that it covers their latency (every one before the
    // first store: the outputs may alias the inputs, and a load issued after
    // a store would wait for it); block-uniform bases, per-lane offsets
    // clamped to the last element
    float r0v[Sh::IT_SOL][5], gq[Sh::IT_SOL][4];
    double pst[Sh::IT_SOL][5], pb[Sh::IT_SOL][5];
    const bool rk = S_.mode != 0;
    const bool useA = rk && S_.c0 != 0.0, useT = rk && S_.Tout != nullptr, useB = useT && S_.d0 != 0.0;
    const int elmax = (G.E - 1 - e0 < EPB - 1) ? (int)(G.E - 1 - e0) : EPB - 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int k = 0; k < Sh::IT_INTD; ++k) {
            const int it = threadIdx.x + k * NT;
            if (it >= EPB * NINTD) break;
            const int el = it / NINTD, q = it % NINTD;
            const int m = 1 + q % (N - 1), tt = q / (N - 1), t1 = tt % N, t2 = tt / N;
            if (e0 + el >= G.E) continue;
            MixedLds<N> &l = L[el];
            PtState s;
            state_at<N>(op, l, m, sol_of<N>(d, 0, t1, t2), stride_of<N>(d), s);
            float fi[5], fv[5];
            dflux_inviscid(s, Si[d][k], F, fi);
            dflux_viscous<KR>(s, Si[d][k], gSi[d][k], F, kr_of<KR>(F, kri[d][k]), 0, fv);
            const int fl = m + (N + 1) * tt;
            for (int v = 0; v < 5; ++v) l.u.ft[v][fl] = fi[v] - fv[v];
        }
#pragma unroll
        for (int k = 0; k < Sh::IT_FACE; ++k) {
            const int it = threadIdx.x + k * NT;
            if (it >= EPB * 6 * NF2) break;
            const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
            if ((f >> 1) != d || e0 + el >= G.E) continue;
            MixedLds<N> &l = L[el];
            const int m = (f & 1) ? N : 0;
            const float sg = (f & 1) ? 1.0f : -1.0f;
            const int fl = m + (N + 1) * pp;
            for (int v = 0; v < 5; ++v) l.u.ft[v][fl] = sg * ffc[k][v];
        }
        __syncthreads();
        if (d == 2) {
            const float *sgb = G.solgeo + e0 * 13 * NP;
#pragma unroll
            for (int k = 0; k < Sh::IT_SOL; ++k) {
                const int it = threadIdx.x + k * NT;
                const int el = min(it / NP, elmax), p = it % NP;
                for (int c = 0; c < 4; ++c) gq[k][c] = ld_off(sgb, (uint32_t)((el * 13 + 9 + c) * NP + p));
                const uint32_t o = (uint32_t)(el * NP + p);
                for (int v = 0; v < 5; ++v) {
                    const int64_t vb = ((int64_t)v * G.E + e0) * NP;
                    r0v[k][v] = ld_off(B.R0 + vb, o);
                    pst[k][v] = useA ? ld_off(S_.A + vb, o) : 0.0;
                    pb[k][v] = useB ? ld_off(S_.B + vb, o) : 0.0;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < Sh::IT_SOL; ++k) {
            const int it = threadIdx.x + k * NT;
            if (it >= EPB * NP) break;
            const int el = it / NP, p = it % NP;
            if (e0 + el >= G.E) continue;
            const MixedLds<N> &l = L[el];
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int fb = (N + 1) * (t1 + N * t2);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                float sum = 0.0f;
#pragma unroll
                for (int mm = 0; mm <= N; ++mm) sum += op.D[a][mm] * l.u.ft[v][fb + mm];
                div[k][v] += sum;
            }
        }
        __syncthreads();
    }
    // source, background residual and stage combination (operands loaded
    // during the last direction's divergence)
#pragma unroll
    for (int k = 0; k < Sh::IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        const int el = it / NP, p = it % NP;
        if (el > elmax) continue;
        const MixedLds<N> &l = L[el];
        const float iJ = gq[k][0];
        const float g0 = F.GM * gq[k][1], g1 = F.GM * gq[k][2], g2 = F.GM * gq[k][3];
        const float rp = l.f[F_RP][p], mx = l.f[F_MX][p], my = l.f[F_MY][p], mz = l.f[F_MZ][p];
        float M[5];
        M[0] = 0.0f;
        M[1] = rp * g0 - 2.0f * F.om * my;
        M[2] = rp * g1 + 2.0f * F.om * mx;
        M[3] = rp * g2;
        M[4] = mx * g0 + my * g1 + mz * g2;
        const uint32_t o = (uint32_t)(el * NP + p);
        for (int v = 0; v < 5; ++v) {
            const int64_t vb = ((int64_t)v * G.E + e0) * NP;
            const double Rv = (double)r0v[k][v] + (double)(-div[k][v] * iJ - M[v]);
            if (!rk) {
                st_off(S_.Pout + vb, o, Rv);
                continue;
            }
            // the stage input from its FP32 value and FP32 remainder (48
            // significant bits: 2^-48 relative, far below the FP32 residual)
            const double pin = (double)l.f[v][p] + (double)l.plo[v][p];
            if (useT) st_off(S_.Tout + vb, o, S_.d0 * pb[k][v] + S_.d1 * (pin + S_.d2 * Rv));
            st_off(S_.Pout + vb, o, S_.c0 * pst[k][v] + S_.c1 * (pin + S_.c2 * Rv));
        }
    }
}

// Lift pass: the neighbours' viscous halves at the interior interface
// points enter the divergence through the end columns of the derivative
// matrix (D[a][0] at the lower, D[a][N] at the upper end of each line); the
// missing residual part -(1/|J|) * that lift is added in place to the
// outputs of the flux pass with their stage weights (Pout: c1 c2, Tout:
// d1 d2; residual mode: 1), and the FP32 face traces of the new P are
// pushed to the neighbours.
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_lift_mixed(OpsF<N> opa, GeoF G, const float *__restrict__ TV, MixedStage S_) {
    constexpr int NP = N * N * N, NF2 = N * N;
    constexpr int IT_MB = (EPB * 24 * NF2 + NT - 1) / NT, IT_SOL = (EPB * NP + NT - 1) / NT;
    __shared__ OpsF<N> op;
    ops_to_lds(opa, op);
    __shared__ float nv[EPB][6][4][NF2];  // neighbours' viscous momentum and energy flux, 0 on boundary faces
    __shared__ float sp[EPB][5][NP];      // new perturbation (FP32) for the traces
    __shared__ int32_t lk[EPB][6], inf[EPB][6];
    // blocks walk the elements from the last to the first: the flux pass
    // before ran from the first to the last, so the first blocks here read
    // its latest writes, which are still in the memory-side cache; the next
    // flux pass starts where this pass ends, for the same reason
    const int64_t e0 = (int64_t)(gridDim.x - 1 - blockIdx.x) * EPB;
    const bool useT = S_.mode != 0 && S_.Tout != nullptr;
    // every global input first: face links, the viscous mailbox (boundary
    // slots too: never written, selected away below), outputs of the flux
    // pass and 1/|J|
    int32_t rl = -1, ri = 0;
    {
        const bool okl = (int)threadIdx.x < EPB * 6 && e0 + threadIdx.x / 6 < G.E;
        const int32_t l = G.link[okl ? e0 * 6 + threadIdx.x : 0], i = G.info[okl ? e0 * 6 + threadIdx.x : 0];
        rl = okl ? l : -1;
        ri = okl ? i : 0;
    }
    // (unpredicated loads through clamped indices; items past the end are
    // never stored)
    float mb[IT_MB];
#pragma unroll
    for (int k = 0; k < IT_MB; ++k) {
        const int it = threadIdx.x + k * NT;
        const bool ok = it < EPB * 24 * NF2 && e0 + it / (24 * NF2) < G.E;
        mb[k] = ld_once(&TV[ok ? e0 * 24 * NF2 + it : 0]);
    }
    double po[IT_SOL][5], to[IT_SOL][5];
    float iJ[IT_SOL];
#pragma unroll
    for (int k = 0; k < IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        const int el = it / NP, p = it % NP;
        const int64_t e = (it < EPB * NP && e0 + el < G.E) ? e0 + el : 0;
        iJ[k] = ld_once(&G.solgeo[(e * 13 + 9) * NP + p]);
        for (int v = 0; v < 5; ++v) {
            const int64_t gi = ((int64_t)v * G.E + e) * NP + p;
            po[k][v] = S_.Pout[gi];
            to[k][v] = useT ? S_.Tout[gi] : 0.0;
        }
    }
    if ((int)threadIdx.x < EPB * 6) {
        lk[threadIdx.x / 6][threadIdx.x % 6] = rl;
        inf[threadIdx.x / 6][threadIdx.x % 6] = ri;
    }
    __syncthreads();
    // the mailbox slot of a boundary face is never written: select, do not
    // multiply by zero
#pragma unroll
    for (int k = 0; k < IT_MB; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * 24 * NF2) break;
        const int el = it / (24 * NF2), r = it % (24 * NF2), f = r / (4 * NF2);
        (&nv[el][0][0][0])[r] = (lk[el][f] >= 0) ? mb[k] : 0.0f;
    }
    __syncthreads();
    const double wP = (S_.mode == 0) ? 1.0 : S_.c1 * S_.c2, wT = S_.d1 * S_.d2;
#pragma unroll
    for (int k = 0; k < IT_SOL; ++k) {
        const int it = threadIdx.x + k * NT;
        if (it >= EPB * NP) break;
        const int el = it / NP, p = it % NP;
        const int64_t e = e0 + el;
        if (e >= G.E) continue;
        float corr[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int a, t1, t2;
            split_sol<N>(d, p, a, t1, t2);
            const int pp = t1 + N * t2;
            const float wl = -0.5f * op.D[a][0], wu = 0.5f * op.D[a][N];
#pragma unroll
            for (int v = 1; v < 5; ++v)
                corr[v] += wl * nv[el][2 * d][v - 1][pp] + wu * nv[el][2 * d + 1][v - 1][pp];
        }
        for (int v = 0; v < 5; ++v) {
            const int64_t gi = ((int64_t)v * G.E + e) * NP + p;
            const double x = -(double)(iJ[k] * corr[v]);
            const double pv = po[k][v] + wP * x;
            S_.Pout[gi] = pv;
            if (useT) S_.Tout[gi] = to[k][v] + wT * x;
            sp[el][v][p] = (float)pv;
        }
    }
    if (S_.mode == 0 || S_.TQout == nullptr) return;
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * 6 * NF2; it += NT) {
        const int el = it / (6 * NF2), r = it % (6 * NF2), f = r / NF2, pp = r % NF2;
        const int64_t e = e0 + el;
        const int32_t nb = lk[el][f];
        if (e >= G.E || nb < 0) continue;
        float *out = S_.TQout + mailbox_slot<N>(nb, inf[el][f], pp);
        const int d = f >> 1, m = (f & 1) ? N : 0, base = sol_of<N>(d, 0, pp % N, pp / N), st = stride_of<N>(d);
        for (int v = 0; v < 5; ++v) st_once(&out[v * NF2], line_val<N>(op, sp[el][v], m, base, st));
    }
}

// Q = Q0 + P
__global__ void k_pert_end(const double *__restrict__ Q0, const double *__restrict__ Pq, double *__restrict__ Q,
                           int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Q[i] = Q0[i] + Pq[i];
}

// background setup (FP64): rho0, E0 (FP32) at solution points; the jump of
// the background face traces across each interface (neighbour minus own,
// from the FP64 traces TQ0 of Q0, rounded to FP32); a flag if Q0 moves
template <int N, int EPB, int NT>
__global__ __launch_bounds__(NT) void k_bg_setup(Ops<N> opa, Geo G, const double *__restrict__ Q0,
                                                 const double *__restrict__ TQ0, float *__restrict__ bg,
                                                 float *__restrict__ dbg, int *__restrict__ flag) {
    constexpr int NP = N * N * N, NF2 = N * N;
    __shared__ double s0[EPB][2][NP];
    __shared__ Ops<N> op;
    ops_to_lds(opa, op);
    const int64_t e0 = (int64_t)blockIdx.x * EPB, E = G.E;
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
        const int32_t nb = G.link[e * 6 + f];
        for (int v = 0; v < 2; ++v) {
            double own = 0.0;
            for (int b = 0; b < N; ++b) own += op.I[m][b] * s0[el][v][base + b * st];
            double jump = 0.0;
            if (nb >= 0) {
                const int inf = G.info[e * 6 + f];
                const int pn = map_face_point<N>((inf >> 3) & 7, t1, t2);
                jump = TQ0[(((int64_t)nb * 6 + (inf & 7)) * 5 + (v == 0 ? 0 : 4)) * NF2 + pn] - own;
            }
            dbg[((e * 6 + f) * 2 + v) * NF2 + pp] = (float)jump;
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
// elements per block and threads of the element kernels (trace setup,
// background setup), and the minimum waves per SIMD of the flux pass
template <> struct CfgM<2> { static constexpr int EPB = 8, NT = 64, MINW = 2; };
template <> struct CfgM<3> { static constexpr int EPB = 2, NT = 64, MINW = 3; };
template <> struct CfgM<4> { static constexpr int EPB = 1, NT = 64, MINW = 4; };
template <> struct CfgM<5> { static constexpr int EPB = 1, NT = 128, MINW = 2; };
template <> struct CfgM<6> { static constexpr int EPB = 1, NT = 256, MINW = 1; };
// flux pass (elements per block, threads, minimum waves per SIMD) and lift
// pass (elements per block, threads)
template <int N> struct CfgF { static constexpr int EPB = CfgM<N>::EPB, NT = CfgM<N>::NT, MINW = CfgM<N>::MINW; };
template <int N> struct CfgL { static constexpr int EPB = CfgM<N>::EPB, NT = CfgM<N>::NT; };

static GeoF geof_of(const GeoM &g) {
    GeoF o;
    o.solgeo = g.solgeo32;
    o.fluxgeo = g.fluxgeo32;
    o.link = g.link;
    o.info = g.info;
    o.E = g.E;
    o.rflux = g.rflux32;
    return o;
}
static MixedBufs bufs_of(const GeoM &g) {
    MixedBufs b;
    b.bg = g.bg;
    b.dbg = g.dbg;
    b.gS0 = g.gS0;
    b.R0 = g.R0;
    b.gbg = g.gbg;
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
static hipError_t flux_mixed_t(const Mesh &m, const GeoM &g, const PhysParams &P, const double *Pq, const float *TQ,
                               float *TV, const MixedStageArgs &a, hipStream_t s) {
    constexpr int EPB = CfgF<N>::EPB, NT = CfgF<N>::NT, MINW = CfgF<N>::MINW;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    const MixedStage st = a;
    if (P.kappa_r1 != 0.0 || P.kappa_r2 != 0.0)
        hipLaunchKernelGGL((k_flux_mixed<N, EPB, NT, MINW, KR_RADIAL>), dim3(nb), dim3(NT), 0, s,
                           make_ops_t<float, N>(m.basis), geof_of(g), bufs_of(g), P, Pq, TQ, TV, st);
    else if (P.kappa_r != 0.0)
        hipLaunchKernelGGL((k_flux_mixed<N, EPB, NT, MINW, KR_CONST>), dim3(nb), dim3(NT), 0, s,
                           make_ops_t<float, N>(m.basis), geof_of(g), bufs_of(g), P, Pq, TQ, TV, st);
    else
        hipLaunchKernelGGL((k_flux_mixed<N, EPB, NT, MINW, KR_NONE>), dim3(nb), dim3(NT), 0, s,
                           make_ops_t<float, N>(m.basis), geof_of(g), bufs_of(g), P, Pq, TQ, TV, st);
    return hipGetLastError();
}
template <int N>
static hipError_t lift_mixed_t(const Mesh &m, const GeoM &g, const float *TV, const MixedStageArgs &a, hipStream_t s) {
    constexpr int EPB = CfgL<N>::EPB, NT = CfgL<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    const MixedStage st = a;
    hipLaunchKernelGGL((k_lift_mixed<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, make_ops_t<float, N>(m.basis),
                       geof_of(g), TV, st);
    return hipGetLastError();
}
template <int N>
static hipError_t bg_setup_t(const Mesh &m, const Geo &G, const double *Q0, const double *TQ0, float *bg, float *dbg,
                             int *flag, hipStream_t s) {
    constexpr int EPB = CfgM<N>::EPB, NT = CfgM<N>::NT;
    const unsigned nb = (unsigned)((m.E + EPB - 1) / EPB);
    hipLaunchKernelGGL((k_bg_setup<N, EPB, NT>), dim3(nb), dim3(NT), 0, s, make_ops_t<double, N>(m.basis), G, Q0,
                       TQ0, bg, dbg, flag);
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
hipError_t launch_flux_mixed(const Mesh &m, const GeoM &g, const PhysParams &P, const double *Pq, const float *TQ,
                             float *TV, const MixedStageArgs &a, hipStream_t s) {
#define C_(n) flux_mixed_t<n>(m, g, P, Pq, TQ, TV, a, s)
    CHORUS_DISPATCH_M(m.N, C_)
#undef C_
}
hipError_t launch_lift_mixed(const Mesh &m, const GeoM &g, const float *TV, const MixedStageArgs &a, hipStream_t s) {
#define C_(n) lift_mixed_t<n>(m, g, TV, a, s)
    CHORUS_DISPATCH_M(m.N, C_)
#undef C_
}
hipError_t launch_bg_setup(const Mesh &m, const Geo &G, const double *Q0, const double *TQ0, float *bg, float *dbg,
                           int *flag, hipStream_t s) {
#define C_(n) bg_setup_t<n>(m, G, Q0, TQ0, bg, dbg, flag, s)
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
