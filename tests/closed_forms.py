"""Closed-form states and expected values shared by the oracle pins and their
GPU twins (test helpers; no spectral-difference arithmetic: every expected
value below is the continuous mathematics of Section 2 and Section 5
evaluated in closed form).

Walled slab (affine, periodic in y and z, walls on the two x-planes):
element integrals of the viscous part of the residual follow from the
discrete Gauss identity w^T D = e_N - e_0 (Section 3): the quadrature sum
over an element of the residual equals the sum over its faces of the common
flux at the face points times the face quadrature weights.  When every face
value the scheme forms is exact, an interior element integrates to the
continuous divergence theorem; a wall element differs by the wall flux the
boundary condition substitutes for the interior one.
"""
import math

import numpy as np

SLAB = dict(nx=4, ny=3, nz=3, lengths=(1.0, 0.8, 0.6))


def slab_columns(xyz, NP):
    """(column index along x, x0, x1, face area, element volume) per element
    of the walled slab."""
    nx, ny, nz = SLAB["nx"], SLAB["ny"], SLAB["nz"]
    L, Ly, Lz = SLAB["lengths"]
    hx = L / nx
    Af = (Ly / ny) * (Lz / nz)
    cx = xyz[0].reshape(-1, NP).mean(1)
    col = np.floor(cx / hx).astype(int)
    x0 = col * hx
    return col, x0, x0 + hx, Af, hx * Af


# --------------------------------------------------------------------------
# stress-free walls (Section 5): shear + dilatation vanishing at the walls
# --------------------------------------------------------------------------
TRACTION = dict(rho=1.3, p=2.0, nu=0.05, gamma=5.0 / 3.0, a=0.4, b=-0.3, c=0.7)


def traction_state(xyz):
    """u = (c x (L - x), a x, b x), uniform rho and p: the normal velocity
    vanishes on both walls, the viscous stress is linear in x with
    tau_xx = 4/3 mu c (L - 2x), tau_xy = mu a, tau_xz = mu b (mu = rho nu),
    so the wall traction has a normal and a tangential part."""
    t = TRACTION
    L = SLAB["lengths"][0]
    x = xyz[0]
    u = np.stack([t["c"] * x * (L - x), t["a"] * x, t["b"] * x])
    E = t["p"] / (t["gamma"] - 1) + 0.5 * t["rho"] * (u ** 2).sum(0)
    return np.concatenate([np.full((1, x.size), t["rho"]), t["rho"] * u, E[None]])


def traction_expected(xyz, NP, wall="stress_free"):
    """Element integrals [5][E] of the viscous residual R(nu) - R(0) with
    kappa = 0.  Momentum: the divergence of tau over the element, (-8/3 mu c
    V, 0, 0), plus on a wall element the substituted wall flux minus the
    interior traction through the wall.  Energy: the divergence of u.tau
    (its x-flux g(x) = 4/3 mu c^2 x (L - x)(L - 2x) + mu (a^2 + b^2) x)
    through the element's x-faces; on the walls the viscous work is
    dropped.  wall: 'stress_free' (Section 5: only the normal traction
    tau_nn n kept), 'full' (the interior traction) or 'none' (no viscous
    wall flux) -- the last two are the mistakes the pin must tell apart."""
    t = TRACTION
    L = SLAB["lengths"][0]
    mu = t["rho"] * t["nu"]
    a, b, c = t["a"], t["b"], t["c"]
    col, x0, x1, Af, V = slab_columns(xyz, NP)
    nx = SLAB["nx"]

    def g(x):
        return 4.0 / 3.0 * mu * c * c * x * (L - x) * (L - 2 * x) + mu * (a * a + b * b) * x

    out = np.zeros((5, col.size))
    out[1] = -8.0 / 3.0 * mu * c * V
    out[4] = Af * (g(x1) - g(x0))
    # interior traction through each wall (outward): x = 0, n = -x
    tS0 = -Af * np.array([4.0 / 3.0 * mu * c * L, mu * a, mu * b])
    wS0 = 0.0                                   # u = 0 on x = 0: no work
    # x = L, n = +x
    tSL = Af * np.array([-4.0 / 3.0 * mu * c * L, mu * a, mu * b])
    wSL = Af * g(L)
    for sel, tS, wS in ((col == 0, tS0, wS0), (col == nx - 1, tSL, wSL)):
        if wall == "stress_free":
            Fw = np.array([tS[0], 0.0, 0.0])    # normal traction only
            Fe = 0.0
        elif wall == "full":
            Fw, Fe = tS, wS
        else:
            Fw, Fe = np.zeros(3), 0.0
        out[1:4, sel] += (Fw - tS)[:, None]
        out[4, sel] += Fe - wS
    return out


# --------------------------------------------------------------------------
# wall energy fluxes (Section 5): conduction at rest
# --------------------------------------------------------------------------
CONDUCTION = dict(gamma=5.0 / 3.0, R_gas=1.0, r0=1.4, r1=-0.5, p0=2.0, p1=-0.6,
                  kappa=0.03, kappa_r=0.02, F_bottom=0.37)


def conduction_state(xyz):
    """At rest, rho = r0 + r1 x and p = p0 + p1 x (both linear, so every face
    trace and BR1 gradient is exact)."""
    t = CONDUCTION
    x = xyz[0]
    rho = t["r0"] + t["r1"] * x
    p = t["p0"] + t["p1"] * x
    z = np.zeros_like(x)
    return np.stack([rho, z, z, z, p / (t["gamma"] - 1)])


def conduction_T_top():
    t = CONDUCTION
    L = SLAB["lengths"][0]
    return (t["p0"] + t["p1"] * L) / (t["R_gas"] * (t["r0"] + t["r1"] * L))


def conduction_flux(x):
    """x-component of the viscous energy flux -f = kappa rho T dS/dx +
    kappa_r rho c_p dT/dx (Eq. 3 with f of Section 2) of the linear state."""
    t = CONDUCTION
    gam, R = t["gamma"], t["R_gas"]
    cp = gam * R / (gam - 1)
    rho = t["r0"] + t["r1"] * x
    p = t["p0"] + t["p1"] * x
    T = p / (R * rho)
    dS = cp * (t["p1"] / (gam * p) - t["r1"] / rho)
    dT = (t["p1"] - R * T * t["r1"]) / (R * rho)
    return t["kappa"] * rho * T * dS + t["kappa_r"] * rho * cp * dT


def conduction_expected(xyz, NP, outer="interior"):
    """Element integrals [E] of the energy part of R(kappa, kappa_r,
    F_bottom) - R(0) on the slab with the inner wall (tag 1) at x = 0 and the
    outer wall (tag 2) at x = L: the flux -f through the element's x-faces;
    the inner wall passes the prescribed F_bottom (heating), the outer wall
    the interior conductive flux ('interior', Section 5 with the wall
    temperature equal to the interior one).  outer='adiabatic' or
    'flipped' give the mistakes the pin must tell apart."""
    t = CONDUCTION
    L = SLAB["lengths"][0]
    col, x0, x1, Af, _ = slab_columns(xyz, NP)
    out = Af * (conduction_flux(x1) - conduction_flux(x0))
    w0 = col == 0
    out[w0] = Af * (conduction_flux(x1[w0]) + t["F_bottom"])
    wL = col == SLAB["nx"] - 1
    if outer == "adiabatic":
        out[wL] = -Af * conduction_flux(x0[wL])
    elif outer == "flipped":
        out[wL] = -Af * (conduction_flux(L) + conduction_flux(x0[wL]))
    return out


# --------------------------------------------------------------------------
# isentropic vortex (smooth exact Euler solution; design order, Section 3)
# --------------------------------------------------------------------------
VORTEX = dict(gamma=1.4, beta=5.0, uinf=(1.0, 0.5), length=10.0, amp=0.01, t_end=1.0, radius=3.0)


def vortex_state(xyz, t):
    """The isentropic vortex of strength beta centred at (L/2, L/2) + uinf t,
    advected by the uniform flow uinf (gas constant 1):
        du = -beta/(2 pi) (y - y0) e^{(1 - r^2)/2},  dv = beta/(2 pi) (x - x0) e^{(1 - r^2)/2},
        T = 1 - (gamma - 1) beta^2 / (8 gamma pi^2) e^{1 - r^2},  rho = T^{1/(gamma-1)},  p = rho T."""
    v = VORTEX
    gam, beta, L = v["gamma"], v["beta"], v["length"]
    x0 = 0.5 * L + v["uinf"][0] * t
    y0 = 0.5 * L + v["uinf"][1] * t
    dx, dy = xyz[0] - x0, xyz[1] - y0
    f = np.exp(0.5 * (1.0 - (dx * dx + dy * dy)))
    u = v["uinf"][0] - beta / (2 * math.pi) * dy * f
    w = v["uinf"][1] + beta / (2 * math.pi) * dx * f
    T = 1.0 - (gam - 1) * beta ** 2 / (8 * gam * math.pi ** 2) * f * f
    rho = T ** (1.0 / (gam - 1))
    p = rho * T
    z = np.zeros_like(rho)
    return np.stack([rho, rho * u, rho * w, z, p / (gam - 1) + 0.5 * rho * (u * u + w * w)])


def vortex_steps(N, n):
    """SSP-RK3 steps to t_end: dt = 0.25 h / (N |u + c|max) with h = L / n."""
    h = VORTEX["length"] / n
    return int(math.ceil(VORTEX["t_end"] / (0.25 * h / (N * 2.5))))


def vortex_errors(Q, xyz, wJ):
    """Per-variable L2 error at t_end over the disc of radius `radius` about
    the vortex centre (the state far out is the uniform flow; the vortex's
    exponential tail is not periodic, so the far field is left out)."""
    v = VORTEX
    ex = vortex_state(xyz, v["t_end"])
    c = (0.5 * v["length"] + v["uinf"][0] * v["t_end"], 0.5 * v["length"] + v["uinf"][1] * v["t_end"])
    w = wJ * (((xyz[0] - c[0]) ** 2 + (xyz[1] - c[1]) ** 2) < v["radius"] ** 2)
    Q = Q.reshape(5, -1)
    return np.array([math.sqrt((w * (Q[k] - ex[k]) ** 2).sum() / w.sum()) for k in range(5)])
