"""CPU oracle of the almost-flux-balance background (Section 4.3) -- test
infrastructure only (tests, smoke and the benchmark's CPU leg may import it).

Polytrope of Section 4.2 with depth d = 1 and rho_c = p_c = 1 at the
mid-layer point chi = 1 (so T_c = 1 / R and GM = (n + 1) alpha):
    chi = c + alpha / r,  rho_a = chi^n,  p_a = chi^(n+1),  T_a = chi / R.
Target entropy gradient (Eq. target_entropy, with the overall sign that
makes the diffusive flux f = -kappa rho T grad S - kappa_r rho c_p grad T of
Section 2 carry the luminosity outward):
    Gamma = -(L / (4 pi r^2) + rho_a c_p kappa_r dT_a/dr) / (rho_a T_a kappa),
with kappa_r(r) = kappa_r + kappa_r1 r + kappa_r2 r^2 (constant unless the
quadratic terms are given: the solar case of Section 7.4).
State equations (Eq. state_equations), integrated from r_c (chi = 1) with
rho0 = p0 = 1 by scipy's DOP853 at tight tolerances:
    Gamma / c_p = -(rho0'/rho0 + g rho0 / (gamma p0)),  p0' = -rho0 g,
    g = GM / r^2.
"""
import math

import numpy as np


def polytrope_constants(beta, n_rho, poly_n):
    chi_o = (beta + 1.0) / (beta * math.exp(n_rho / poly_n) + 1.0)
    c = (2.0 * chi_o - beta - 1.0) / (1.0 - beta)
    alpha = (1.0 + beta) * (1.0 - chi_o) / (1.0 - beta) ** 2
    return chi_o, c, alpha


def target_gradient(r, beta, n_rho, luminosity, kappa, kappa_r=0.0, poly_n=1.5, gamma=5.0 / 3.0, R_gas=1.0,
                    kappa_r1=0.0, kappa_r2=0.0):
    _, c, alpha = polytrope_constants(beta, n_rho, poly_n)
    chi = c + alpha / r
    rho_a = chi ** poly_n
    T_a = chi / R_gas
    dT_a = -alpha / r ** 2 / R_gas
    cp = gamma * R_gas / (gamma - 1.0)
    kr = kappa_r + kappa_r1 * r + kappa_r2 * r * r
    return -(luminosity / (4.0 * math.pi * r ** 2) + rho_a * cp * kr * dT_a) / (rho_a * T_a * kappa)


def background(r, beta, n_rho, luminosity, kappa, kappa_r=0.0, poly_n=1.5, gamma=5.0 / 3.0, R_gas=1.0,
               kappa_r1=0.0, kappa_r2=0.0):
    """(rho0, p0) at the radii r (any shape)."""
    from scipy.integrate import solve_ivp
    _, c, alpha = polytrope_constants(beta, n_rho, poly_n)
    GM = (poly_n + 1.0) * alpha
    cp = gamma * R_gas / (gamma - 1.0)
    rc = alpha / (1.0 - c)

    def f(x, y):
        rho, p = y
        g = GM / x ** 2
        G = target_gradient(x, beta, n_rho, luminosity, kappa, kappa_r, poly_n, gamma, R_gas, kappa_r1, kappa_r2)
        return [-rho * (G / cp + g * rho / (gamma * p)), -rho * g]

    r = np.asarray(r, dtype=np.float64)
    out = np.zeros((2,) + r.shape)
    ri, ro = beta / (1.0 - beta), 1.0 / (1.0 - beta)
    for lo, hi, sel in ((rc, ro * (1 + 1e-12), r >= rc), (rc, ri * (1 - 1e-12), r < rc)):
        if not sel.any():
            continue
        sol = solve_ivp(f, (lo, hi), [1.0, 1.0], method="DOP853", rtol=1e-13, atol=1e-15, dense_output=True)
        out[:, sel] = sol.sol(r[sel])
    return out[0], out[1]
