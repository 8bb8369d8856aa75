// Pointwise physics of the compressible Navier-Stokes system in a rotating
// frame (Section 2, Eqs. 1-9), written for one point and templated on the
// arithmetic type.  All "fluxes along S" take a non-normalised vector S and
// return (F, G, H) . S, which is linear in S, so the transformed flux
// |J| grad xi_d . (F, G, H) and interface normal fluxes share one routine.
// Every routine is written so that negating S negates the result exactly
// (the two sides of an interface evaluate the same common flux).
#pragma once

#include <hip/hip_runtime.h>

namespace chorus {

struct PhysParams {
    double gamma, R_gas, GM, omega, nu, kappa, kappa_r, T_top, F_bottom;
    double bc_state[5];
    double cp;  // gamma R / (gamma - 1)
    double kappa_r1, kappa_r2;  // kappa_r(r) = kappa_r + kappa_r1 r + kappa_r2 r^2
};

// radiative diffusivity at radius r
__host__ __device__ __forceinline__ double kappa_r_at(const PhysParams &P, double r) {
    return P.kappa_r + r * (P.kappa_r1 + r * P.kappa_r2);
}

template <typename T>
__device__ __forceinline__ T pressure_of(const T q[5], T gm1) {
    return gm1 * (q[4] - T(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

// inviscid flux along S: (rho u_S, rho u u_S + p S, (E + p) u_S)
template <typename T>
__device__ __forceinline__ void flux_inviscid(const T q[5], const T S[3], T gm1, T out[5]) {
    const T rho = q[0];
    const T inv = T(1) / rho;
    const T u0 = q[1] * inv, u1 = q[2] * inv, u2 = q[3] * inv;
    const T p = gm1 * (q[4] - T(0.5) * (q[1] * u0 + q[2] * u1 + q[3] * u2));
    const T un = u0 * S[0] + u1 * S[1] + u2 * S[2];
    out[0] = rho * un;
    out[1] = q[1] * un + p * S[0];
    out[2] = q[2] * un + p * S[1];
    out[3] = q[3] * un + p * S[2];
    out[4] = (q[4] + p) * un;
}

// primitive gradients from gradients of the conserved variables
// g[v][c] = dQ_v/dx_c: velocity gradient du[a][c], grad S (S = c_p ln(p^(1/g)/rho)),
// grad T (T = p/(rho R)); mu-independent.
template <typename T>
struct PrimGrad {
    T rho, u[3], p, Tmp, du[3][3], dS[3], dT[3];
};

template <typename T>
__device__ __forceinline__ void prim_grad(const T q[5], const T g[5][3], const PhysParams &P,
                                          PrimGrad<T> &o) {
    const T gm1 = T(P.gamma - 1.0), gam = T(P.gamma), R = T(P.R_gas), cp = T(P.cp);
    o.rho = q[0];
    const T inv = T(1) / o.rho;
    for (int a = 0; a < 3; ++a) o.u[a] = q[1 + a] * inv;
    o.p = gm1 * (q[4] - T(0.5) * (q[1] * o.u[0] + q[2] * o.u[1] + q[3] * o.u[2]));
    // one division each for 1/(rho R) and 1/(gamma p), reused below
    const T irR = T(1) / (o.rho * R), igp = T(1) / (gam * o.p);
    o.Tmp = o.p * irR;
    const T uu = o.u[0] * o.u[0] + o.u[1] * o.u[1] + o.u[2] * o.u[2];
    for (int c = 0; c < 3; ++c) {
        for (int a = 0; a < 3; ++a) o.du[a][c] = (g[1 + a][c] - o.u[a] * g[0][c]) * inv;
        const T dp = gm1 * (g[4][c] - (o.u[0] * g[1][c] + o.u[1] * g[2][c] + o.u[2] * g[3][c]) +
                            T(0.5) * uu * g[0][c]);
        o.dS[c] = cp * (dp * igp - g[0][c] * inv);
        o.dT[c] = (dp - R * o.Tmp * g[0][c]) * irR;
    }
}

// viscous flux along S: (0, tau.S, u.tau.S - f.S), tau = mu (grad u + grad u^T
// - 2/3 div u I), mu = rho nu, -f = kappa rho T grad S + kr rho c_p grad T
// (kr: the radiative diffusivity at the point).  With du_a/dx_c =
// (dm_a/dx_c - u_a drho/dx_c) / rho the gradients enter only through their
// contractions with S, gS_v = grad Q_v . S, and for the transposed stress
// Z_a = sum_b dm_b/dx_a S_b; with S = c_p ln(p^(1/gamma) / rho) and
// T = p / (rho R) the energy diffusion is (c_p / R) [kappa (grad p . S /
// gamma - p grad rho . S / rho) + kr (grad p . S - p grad rho . S / rho)],
// so 1/rho is the only reciprocal.
template <typename T>
__device__ __forceinline__ void flux_viscous(const T q[5], const T g[5][3], const T S[3],
                                             const PhysParams &P, T kr, T out[5]) {
    const T gm1 = T(P.gamma - 1.0), nu = T(P.nu);
    const T inv = T(1) / q[0];
    const T u[3] = {q[1] * inv, q[2] * inv, q[3] * inv};
    T gS[5];
    for (int v = 0; v < 5; ++v) gS[v] = g[v][0] * S[0] + g[v][1] * S[1] + g[v][2] * S[2];
    const T uS = u[0] * S[0] + u[1] * S[1] + u[2] * S[2];
    const T ug = u[0] * g[0][0] + u[1] * g[0][1] + u[2] * g[0][2];
    // (2/3) rho div u
    const T dv = T(2.0 / 3.0) * (g[1][0] + g[2][1] + g[3][2] - ug);
    T tS[3];
    for (int a = 0; a < 3; ++a) {
        const T Za = g[1][a] * S[0] + g[2][a] * S[1] + g[3][a] * S[2];
        tS[a] = nu * (gS[1 + a] + Za - u[a] * gS[0] - uS * g[0][a] - dv * S[a]);
    }
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T p = gm1 * (q[4] - T(0.5) * (q[1] * u[0] + q[2] * u[1] + q[3] * u[2]));
    const T dpS = gm1 * (gS[4] - (u[0] * gS[1] + u[1] * gS[2] + u[2] * gS[3]) + T(0.5) * uu * gS[0]);
    const T prS = p * inv * gS[0];
    out[0] = T(0);
    out[1] = tS[0];
    out[2] = tS[1];
    out[3] = tS[2];
    out[4] = u[0] * tS[0] + u[1] * tS[1] + u[2] * tS[2] +
             T(P.cp / P.R_gas) * (T(P.kappa) * (dpS * T(1.0 / P.gamma) - prS) + kr * (dpS - prS));
}

// Rusanov common flux along S (outward from the qL side), wave speed
// max(|u_L.n| + c_L, |u_R.n| + c_R), formed as max(|u_L.S| + c_L |S|, ...)
// (two square roots, no division by |S|)
template <typename T>
__device__ __forceinline__ void flux_rusanov(const T qL[5], const T qR[5], const T S[3],
                                             const PhysParams &P, T out[5]) {
    const T gm1 = T(P.gamma - 1.0), gam = T(P.gamma);
    T fL[5], fR[5];
    flux_inviscid(qL, S, gm1, fL);
    flux_inviscid(qR, S, gm1, fR);
    const T A2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
    const T iL = T(1) / qL[0], iR = T(1) / qR[0];
    const T unL = fabs((qL[1] * S[0] + qL[2] * S[1] + qL[3] * S[2]) * iL);
    const T unR = fabs((qR[1] * S[0] + qR[2] * S[1] + qR[3] * S[2]) * iR);
    const T pL = gm1 * (qL[4] - T(0.5) * (qL[1] * qL[1] + qL[2] * qL[2] + qL[3] * qL[3]) * iL);
    const T pR = gm1 * (qR[4] - T(0.5) * (qR[1] * qR[1] + qR[2] * qR[2] + qR[3] * qR[3]) * iR);
    const T cAL = sqrt(gam * pL * iL * A2);
    const T cAR = sqrt(gam * pR * iR * A2);
    const T lamA = T(0.5) * fmax(unL + cAL, unR + cAR);
    for (int v = 0; v < 5; ++v) out[v] = T(0.5) * (fL[v] + fR[v]) - lamA * (qR[v] - qL[v]);
}

// BR1 interface state on a wall (Section 5): normal momentum removed, pressure
// kept (outer wall with T_top > 0: p = rho R T_top)
template <typename T>
__device__ __forceinline__ void wall_state(const T q[5], const T S[3], bool outer, const PhysParams &P,
                                           T qb[5]) {
    const T gm1 = T(P.gamma - 1.0);
    const T A2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
    const T mn = (q[1] * S[0] + q[2] * S[1] + q[3] * S[2]) / A2;  // (m.n)/|S|
    T p = pressure_of(q, gm1);
    if (outer && P.T_top > 0.0) p = q[0] * T(P.R_gas) * T(P.T_top);
    qb[0] = q[0];
    for (int a = 0; a < 3; ++a) qb[1 + a] = q[1 + a] - mn * S[a];
    qb[4] = p / gm1 + T(0.5) * (qb[1] * qb[1] + qb[2] * qb[2] + qb[3] * qb[3]) / qb[0];
}

// total wall flux along the outward S: inviscid (0, p S, 0) with the interior
// p (V_r = 0); viscous: normal traction only (stress free), energy f.S =
// F_bottom |S| at the inner wall, interior diffusive flux at the outer wall
// (kr: the radiative diffusivity at the point)
template <typename T>
__device__ __forceinline__ void flux_wall(const T q[5], const T g[5][3], const T S[3], bool outer,
                                          const PhysParams &P, T kr, T out[5]) {
    PrimGrad<T> pg;
    prim_grad(q, g, P, pg);
    const T mu = pg.rho * T(P.nu);
    const T div = pg.du[0][0] + pg.du[1][1] + pg.du[2][2];
    const T A2 = S[0] * S[0] + S[1] * S[1] + S[2] * S[2];
    // n.tau.n = mu (2 n.grad u.n - 2/3 div)
    T ngn = T(0);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) ngn += S[a] * pg.du[a][b] * S[b];
    const T tnn = mu * (T(2) * ngn / A2 - T(2.0 / 3.0) * div);
    T ev;
    if (outer) {
        const T dSS = pg.dS[0] * S[0] + pg.dS[1] * S[1] + pg.dS[2] * S[2];
        const T dTS = pg.dT[0] * S[0] + pg.dT[1] * S[1] + pg.dT[2] * S[2];
        ev = T(P.kappa) * pg.rho * pg.Tmp * dSS + kr * pg.rho * T(P.cp) * dTS;
    } else {
        ev = T(P.F_bottom) * sqrt(A2);
    }
    out[0] = T(0);
    for (int a = 0; a < 3; ++a) out[1 + a] = (pg.p - tnn) * S[a];
    out[4] = -ev;
}

}  // namespace chorus
