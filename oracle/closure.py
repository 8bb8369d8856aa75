"""CPU FP64 oracle of the learned subgrid closure (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the GPU library never does and shares no
code with it.

The paper names large-eddy simulation with subgrid modelling as the next
step of the code (Summary section) and already treats its entropy diffusion
as a parameterisation of unresolved motions (Section 2).  The closure here is
a pointwise network: at each solution point of an order-3 solve it maps the
resolved state and its BR1 gradients to a subgrid flux added to the total
flux.  Everything below is written from textbook definitions:

  * GELU, exact form x Phi(x) with Phi the standard normal CDF
    (Hendrycks & Gimpel 2016);
  * a multilayer perceptron 20 -> 64 -> 64 -> 15 with a mean-squared-error
    loss and its reverse-mode gradient;
  * Adam with bias correction (Kingma & Ba 2015, Algorithm 1);
  * bfloat16 = the upper 16 bits of an IEEE binary32, rounded to nearest
    even;
  * the subgrid flux of a filter G: tau = G(F(Q)) - F(G(Q)) with F the
    inviscid flux (the standard commutator definition of LES), and G the
    per-element L2 projection of |J| Q onto tensor polynomials of degree
    N_c - 1, divided by |J| at the coarse solution points (mass-preserving).

Parameter layout (FP32 in the library, float64 here), 6479 values:
  W1[64][20], b1[64], W2[64][64], b2[64], W3[15][64], b3[15]
  (z_j = sum_i W[j][i] x_i + b_j).
Normalisation, 70 values: x_mean[20], x_inv_std[20], y_mean[15], y_std[15];
raw features are (rho, rho u, rho v, rho w, E) and the 15 gradients
d(Q_v)/dx_c at index 5 + 3 v + c; outputs are indexed 3 v + c and mean the
Cartesian component c of the subgrid flux of variable v:
  tau[3 v + c] = y_mean + y_std * y.
"""
import math

import numpy as np

N_IN, N_HID, N_OUT = 20, 64, 15
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)  # 6479
N_NORM = 2 * N_IN + 2 * N_OUT  # 70


# ---------------------------------------------------------------------------
# activation
# ---------------------------------------------------------------------------
_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(x):
    """x Phi(x), Phi(x) = (1 + erf(x / sqrt 2)) / 2."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_prime(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x), phi the standard normal density."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + _erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
def unpack(params):
    params = np.asarray(params, dtype=np.float64)
    assert params.size == N_PARAM
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = params[o:o + n].reshape(shp)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


# ---------------------------------------------------------------------------
# network, loss and gradient (FP64)
# ---------------------------------------------------------------------------
def forward(params, X):
    """X [n][20] (normalised features) -> Y [n][15] and the activations."""
    P = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ P["W1"].T + P["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ P["W2"].T + P["b2"]
    H2 = gelu(Z2)
    Y = H2 @ P["W3"].T + P["b3"]
    return Y, (X, Z1, H1, Z2, H2)


def loss(params, X, T):
    """Mean over samples and outputs of (Y - T)^2."""
    Y, _ = forward(params, X)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def grad(params, X, T):
    """Gradient of loss() with respect to the parameter vector (chain rule
    through the three layers, the last one linear)."""
    P = unpack(params)
    Y, (X, Z1, H1, Z2, H2) = forward(params, X)
    T = np.asarray(T, dtype=np.float64)
    n = X.shape[0]
    dY = 2.0 * (Y - T) / (n * N_OUT)
    g = {"W3": dY.T @ H2, "b3": dY.sum(0)}
    dZ2 = (dY @ P["W3"]) * gelu_prime(Z2)
    g["W2"] = dZ2.T @ H1
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2 @ P["W2"]) * gelu_prime(Z1)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(0)
    return pack(g)


def adam_step(params, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) at step t >= 1;
    returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(params, X, T, batch_index, batch, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, step0=0, m=None, v=None):
    """Mini-batch Adam: iteration i uses the samples batch_index[i*batch:(i+1)*batch]
    (the index sequence is an input).  Returns (params, m, v, losses)."""
    params = np.array(params, dtype=np.float64)
    m = np.zeros_like(params) if m is None else np.array(m, dtype=np.float64)
    v = np.zeros_like(params) if v is None else np.array(v, dtype=np.float64)
    idx = np.asarray(batch_index).reshape(-1, batch)
    losses = []
    for i, ib in enumerate(idx):
        Xb, Tb = X[ib], T[ib]
        losses.append(loss(params, Xb, Tb))
        g = grad(params, Xb, Tb)
        params, m, v = adam_step(params, m, v, g, step0 + i + 1, lr, b1, b2, eps)
    return params, m, v, np.array(losses)


# ---------------------------------------------------------------------------
# bfloat16 inference as the fused kernel computes it
# ---------------------------------------------------------------------------
def to_bf16(x):
    """Round to float32, then to bfloat16 (nearest, ties to even); returned
    as float64 values."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def normalise(raw, norm):
    norm = np.asarray(norm, dtype=np.float64)
    return (np.asarray(raw, dtype=np.float64) - norm[0:20]) * norm[20:40]


def infer_bf16(params, norm, raw):
    """Subgrid flux [n][15] from raw features [n][20] with the precision
    steps of the BF16 kernel: normalised features, weights and hidden
    activations rounded to bfloat16; biases and sums exact (the kernel sums
    in FP32, this in FP64)."""
    P = unpack(params)
    norm = np.asarray(norm, dtype=np.float64)
    x = to_bf16(normalise(raw, norm))
    W1, W2, W3 = to_bf16(P["W1"]), to_bf16(P["W2"]), to_bf16(P["W3"])
    b1, b2, b3 = (np.float64(np.float32(b)) for b in (P["b1"], P["b2"], P["b3"]))
    h1 = to_bf16(gelu(x @ W1.T + b1))
    h2 = to_bf16(gelu(h1 @ W2.T + b2))
    y = h2 @ W3.T + b3
    return norm[40:55] + norm[55:70] * y


def infer_fp64(params, norm, raw):
    """The same network in FP64 throughout (no bfloat16 rounding)."""
    norm = np.asarray(norm, dtype=np.float64)
    y, _ = forward(params, normalise(raw, norm))
    return norm[40:55] + norm[55:70] * y


# ---------------------------------------------------------------------------
# features on an oracle mesh
# ---------------------------------------------------------------------------
def features(om, ph, Q):
    """Raw features [E N^3][20]: Q and its BR1 gradients at every solution
    point (sample index e N^3 + p)."""
    Q = np.asarray(Q, dtype=np.float64).reshape(5, om.E, om.np)
    G = om.gradients(ph, Q)
    return np.concatenate([Q.reshape(5, -1), G.reshape(15, -1)], axis=0).T.copy()


def sgs_field(om, ph, Q, params, norm, bf16=True):
    """Subgrid flux at the solution points as [15][E][N^3]."""
    f = infer_bf16 if bf16 else infer_fp64
    tau = f(params, norm, features(om, ph, Q))
    return tau.T.reshape(15, om.E, om.np).copy()


# ---------------------------------------------------------------------------
# filter and subgrid-flux targets
# ---------------------------------------------------------------------------
def _lagrange_matrix(nodes, x):
    """L[q][s] = h_s(x_q), the Lagrange basis on `nodes` evaluated at x."""
    nodes = np.asarray(nodes, dtype=np.float64)
    L = np.ones((len(x), len(nodes)))
    for s in range(len(nodes)):
        for t in range(len(nodes)):
            if t != s:
                L[:, s] *= (x - nodes[t]) / (nodes[s] - nodes[t])
    return L


def projection_1d(xs_fine, xs_coarse):
    """P[a][b]: values at the coarse solution points of the L2 projection on
    [0, 1] onto polynomials of degree < len(xs_coarse) of the interpolant of
    fine-point values.  Built by Gauss quadrature and the normal equations
    in the monomial basis."""
    nf, nc = len(xs_fine), len(xs_coarse)
    g, wq = np.polynomial.legendre.leggauss(nf + nc + 2)
    xq, wq = 0.5 * (g + 1.0), 0.5 * wq
    Hq = _lagrange_matrix(xs_fine, xq)                      # [q][b]
    Vq = np.vander(xq, nc, increasing=True)                 # [q][k]
    M = Vq.T @ (wq[:, None] * Vq)                           # Gram matrix
    rhs = Vq.T @ (wq[:, None] * Hq)                         # [k][b]
    coef = np.linalg.solve(M, rhs)
    Vc = np.vander(np.asarray(xs_coarse, dtype=np.float64), nc, increasing=True)
    return Vc @ coef


def filter_field(U, jac_fine, jac_coarse, Nf, Nc, xs_fine, xs_coarse):
    """G(U) = Pi(|J| U) / |J| per element: U [k][E][Nf^3] -> [k][E][Nc^3]."""
    P = projection_1d(xs_fine, xs_coarse)
    k = U.shape[0]
    E = U.shape[1]
    A = (np.asarray(U) * jac_fine.reshape(1, E, -1)).reshape(k, E, Nf, Nf, Nf)  # [.., kz, jy, ix]
    B = np.einsum("ai,vezyi->vezya", P, A)
    B = np.einsum("bj,vezja->vezba", P, B)
    B = np.einsum("ck,vekba->vecba", P, B)
    return B.reshape(k, E, Nc ** 3) / jac_coarse.reshape(1, E, -1)


def inviscid_flux_cartesian(Q, gamma):
    """F[3 v + c] = Cartesian component c of the inviscid flux of variable v."""
    rho, mx, my, mz, E = Q
    m = (mx, my, mz)
    p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho)
    F = np.zeros((15,) + rho.shape)
    for c in range(3):
        F[c] = m[c]
        for i in range(3):
            F[3 * (1 + i) + c] = m[i] * m[c] / rho + (p if i == c else 0.0)
        F[12 + c] = (E + p) * m[c] / rho
    return F


def sgs_target(Q_fine, jac_fine, jac_coarse, Nf, Nc, xs_fine, xs_coarse, gamma):
    """(G(Q), tau) with tau = G(F(Q)) - F(G(Q)) at the coarse points."""
    Qf = np.asarray(Q_fine, dtype=np.float64)
    Qbar = filter_field(Qf, jac_fine, jac_coarse, Nf, Nc, xs_fine, xs_coarse)
    Fbar = filter_field(inviscid_flux_cartesian(Qf, gamma), jac_fine, jac_coarse, Nf, Nc, xs_fine,
                        xs_coarse)
    tau = Fbar - inviscid_flux_cartesian(Qbar, gamma)
    tau[0:3] = 0.0  # the mass flux is linear in Q: G commutes with it
    return Qbar, tau
