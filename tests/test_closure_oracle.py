"""Pins of the closure oracle (oracle/closure.py and the subgrid-flux term of
the oracle residual) against closed forms, textbook identities and brute
force.  None of them compares the oracle with itself or with the GPU."""
import math

import numpy as np
import pytest

from chorus_inputs import box_mesh, cubed_sphere_shell, uniform_noise


@pytest.fixture(scope="module")
def cl(oracle_mod):
    from oracle import closure
    return closure


def _rand_params(cl, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, cl.N_PARAM)


# ---------------------------------------------------------------------------
# activation, bfloat16
# ---------------------------------------------------------------------------
def test_gelu_values(cl):
    # Phi(1) = 0.8413447460685429 (standard normal CDF table value)
    assert cl.gelu(0.0) == 0.0
    assert abs(cl.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(cl.gelu(-1.0) + 0.15865525393145707) < 1e-15
    x = np.linspace(-6, 6, 101)
    assert np.allclose(cl.gelu(x) - cl.gelu(-x), x, atol=1e-14)  # x Phi(x) + x Phi(-x) = x
    assert abs(cl.gelu(10.0) - 10.0) < 1e-20 + 1e-12
    h = 1e-5
    fd = (cl.gelu(x + h) - cl.gelu(x - h)) / (2 * h)
    assert np.allclose(cl.gelu_prime(x), fd, atol=1e-9)
    assert abs(cl.gelu_prime(0.0) - 0.5) < 1e-15


def test_bf16_rounding(cl):
    # 7 stored fraction bits: ulp(1) = 2^-7
    assert cl.to_bf16(1.0 + 2.0 ** -8) == 1.0                    # tie -> even
    assert cl.to_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6     # tie -> even (up)
    assert cl.to_bf16(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    assert cl.to_bf16(0.1) == 0.10009765625                      # 0x3DCD
    assert cl.to_bf16(-2.5) == -2.5
    x = np.random.default_rng(0).normal(size=1000)
    r = cl.to_bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * (1 + 1e-6))


# ---------------------------------------------------------------------------
# network orientation, gradient, Adam
# ---------------------------------------------------------------------------
def test_forward_orientation(cl):
    """A network built to compute known scalar compositions: layer 1 picks
    feature i into hidden unit j by W1[j][i], layer 2 is a permutation,
    layer 3 picks hidden units into outputs."""
    W1 = np.zeros((64, 20)); b1 = np.zeros(64)
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W3 = np.zeros((15, 64)); b3 = np.arange(15) * 0.01
    for j in range(20):
        W1[j, (7 * j) % 20] = 1.0 + 0.1 * j           # hidden j <- feature 7j mod 20
    perm = [(5 * j + 3) % 64 for j in range(64)]
    for j in range(64):
        W2[perm[j], j] = 1.0                         # hidden2[perm j] <- hidden1[j]
    for k in range(15):
        W3[k, perm[k]] = 2.0                         # output k <- hidden2[perm k]
    params = cl.pack(dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3))
    x = np.random.default_rng(1).normal(size=(3, 20))
    Y, _ = cl.forward(params, x)

    def g(t):
        return 0.5 * t * (1.0 + math.erf(t / math.sqrt(2.0)))
    for s in range(3):
        for k in range(15):
            want = 2.0 * g(g((1.0 + 0.1 * k) * x[s, (7 * k) % 20])) + 0.01 * k
            assert abs(Y[s, k] - want) < 1e-14


def test_gradient_matches_central_differences(cl):
    rng = np.random.default_rng(2)
    params = _rand_params(cl, 3)
    X = rng.normal(size=(7, 20))
    T = rng.normal(size=(7, 15))
    g = cl.grad(params, X, T)
    idx = rng.choice(cl.N_PARAM, 120, replace=False)
    # make sure every layer is sampled
    idx = np.concatenate([idx, [0, 1279, 1280, 1343, 1344, 5503, 5504, 6463, 6464, 6478]])
    h = 1e-6
    for i in idx:
        e = np.zeros(cl.N_PARAM); e[i] = h
        fd = (cl.loss(params + e, X, T) - cl.loss(params - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.abs(g).max()), (i, fd, g[i])


def test_adam_closed_forms(cl):
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-2, 1e-8
    # step 1: m_hat = g, v_hat = g^2 -> update -lr g / (|g| + eps)
    p1, m, v = cl.adam_step(p0, np.zeros(50), np.zeros(50), g, 1, lr=lr, eps=eps)
    assert np.allclose(p1 - p0, -lr * g / (np.abs(g) + eps), rtol=1e-13, atol=0)
    # constant gradient: the bias-corrected moments stay g and g^2
    p = p1
    for t in range(2, 6):
        pn, m, v = cl.adam_step(p, m, v, g, t, lr=lr, eps=eps)
        assert np.allclose(pn - p, -lr * g / (np.abs(g) + eps), rtol=1e-10, atol=0)
        p = pn


def test_training_fits_a_teacher(cl):
    """Targets made by a random network of the same shape are representable;
    mini-batch Adam must reduce the loss well below its start."""
    rng = np.random.default_rng(5)
    teacher = _rand_params(cl, 6, scale=0.25)
    X = rng.normal(size=(512, 20))
    T, _ = cl.forward(teacher, X)
    student = _rand_params(cl, 7, scale=0.2)
    order = np.concatenate([rng.permutation(512) for _ in range(40)])
    _, _, _, losses = cl.train(student, X, T, order[: 320 * 64], 64, lr=3e-3)
    assert losses[-10:].mean() < 0.15 * losses[:5].mean()


# ---------------------------------------------------------------------------
# filter and subgrid-flux targets
# ---------------------------------------------------------------------------
def _legendre_projection(xs_f, xs_c):
    """Independent construction: coefficients (2k+1) int f L_k with shifted
    Legendre polynomials (orthogonality), quadrature on 20 points."""
    g, w = np.polynomial.legendre.leggauss(20)
    x, w = 0.5 * (g + 1), 0.5 * w
    nf, nc = len(xs_f), len(xs_c)
    H = np.ones((20, nf))
    for s in range(nf):
        for t in range(nf):
            if t != s:
                H[:, s] *= (x - xs_f[t]) / (xs_f[s] - xs_f[t])
    P = np.zeros((nc, nf))
    for k in range(nc):
        Lk = np.polynomial.legendre.Legendre.basis(k)(2 * x - 1)
        ck = (2 * k + 1) * (w * Lk) @ H
        P += np.outer(np.polynomial.legendre.Legendre.basis(k)(2 * np.asarray(xs_c) - 1), ck)
    return P


@pytest.mark.parametrize("nf,nc", [(6, 3), (4, 3), (5, 2)])
def test_projection_1d(cl, oracle_mod, nf, nc):
    xs_f = oracle_mod.basis(nf)[0]
    xs_c = oracle_mod.basis(nc)[0]
    P = cl.projection_1d(xs_f, xs_c)
    assert np.allclose(P, _legendre_projection(xs_f, xs_c), atol=1e-13)
    # reproduces polynomials of degree < nc
    for k in range(nc):
        assert np.allclose(P @ xs_f ** k, xs_c ** k, atol=1e-13)


def test_filter_preserves_element_mass(cl, oracle_mod):
    m = cubed_sphere_shell(2, 1, 2.0, 3.0)
    of, oc = oracle_mod.OracleMesh(m, 6), oracle_mod.OracleMesh(m, 3)
    jf, jc = of.geometry()[0], oc.geometry()[0]
    _, wf = of.solpts()
    _, wc = oc.solpts()
    U = 1.0 + 0.3 * uniform_noise((2, of.n_solpts), 11)
    Ub = cl.filter_field(U.reshape(2, of.E, -1), jf, jc, 6, 3, oracle_mod.basis(6)[0], oracle_mod.basis(3)[0])
    mf = (U.reshape(2, of.E, -1) * wf.reshape(1, of.E, -1)).sum(-1)
    mc = (Ub * wc.reshape(1, oc.E, -1)).sum(-1)
    assert np.allclose(mf, mc, rtol=1e-13)


def test_sgs_target_structure(cl, oracle_mod):
    """tau vanishes for a uniform state on affine elements, its mass part
    is zero and its momentum part is symmetric (F_{m_i, c} = F_{m_c, i})."""
    m = box_mesh(2, 2, 2)
    of, oc = oracle_mod.OracleMesh(m, 6), oracle_mod.OracleMesh(m, 3)
    jf, jc = of.geometry()[0], oc.geometry()[0]
    xs6, xs3 = oracle_mod.basis(6)[0], oracle_mod.basis(3)[0]
    q = np.array([1.3, 0.2, -0.1, 0.3, 2.4])
    Qu = np.tile(q[:, None, None], (1, of.E, of.np))
    Qb, tau = cl.sgs_target(Qu, jf, jc, 6, 3, xs6, xs3, 5 / 3)
    assert np.allclose(Qb, np.tile(q[:, None, None], (1, oc.E, oc.np)), rtol=1e-13)
    assert np.abs(tau).max() < 1e-13
    xyz, _ = of.solpts()
    rng = np.random.default_rng(8)
    Q = Qu.copy()
    for v in range(5):
        Q[v] += 0.2 * np.sin(2 * np.pi * (rng.uniform(1, 3, 3) @ xyz + rng.uniform())).reshape(of.E, -1)
    _, tau = cl.sgs_target(Q, jf, jc, 6, 3, xs6, xs3, 5 / 3)
    assert np.abs(tau[0:3]).max() == 0.0
    assert np.abs(tau[3:12]).max() > 1e-4
    for i in range(3):
        for c in range(3):
            assert np.allclose(tau[3 * (1 + i) + c], tau[3 * (1 + c) + i], atol=1e-14)


# ---------------------------------------------------------------------------
# the subgrid flux in the oracle residual
# ---------------------------------------------------------------------------
def test_sgs_constant_flux_has_no_divergence(oracle_mod):
    """A uniform additional flux on a curved periodic box: its discrete
    divergence vanishes (free-stream property of the curl-form metrics)."""
    om = oracle_mod.OracleMesh(box_mesh(3, 3, 3, periodic=(True,) * 3, curve=0.03), 3)
    Q = np.tile(np.array([1.0, 0.1, 0.2, -0.1, 2.0])[:, None, None], (1, om.E, om.np))
    ph = oracle_mod.phys(nu=1e-2, kappa=1e-2)
    sgs = np.tile(np.linspace(-1, 1, 15)[:, None, None], (1, om.E, om.np))
    d = om.residual(ph, Q, sgs) - om.residual(ph, Q)
    assert np.abs(d).max() < 1e-12


def test_sgs_linear_flux_divergence_exact(oracle_mod):
    """tau_{v,c} = a_{v,c} x_c (degree 1): on the interior elements of an
    affine box the change of dQ/dt is exactly -sum_c a_{v,c}; the total
    change over a periodic box integrates to zero (telescoping faces)."""
    m = box_mesh(4, 4, 4, lengths=(1.0, 1.2, 0.8))
    om = oracle_mod.OracleMesh(m, 3)
    xyz, wJ = om.solpts()
    Q = np.tile(np.array([1.0, 0.1, 0.2, -0.1, 2.0])[:, None, None], (1, om.E, om.np))
    ph = oracle_mod.phys()
    a = np.random.default_rng(9).normal(size=(5, 3))
    sgs = np.zeros((15, om.n_solpts))
    for v in range(5):
        for c in range(3):
            sgs[3 * v + c] = a[v, c] * xyz[c]
    d = (om.residual(ph, Q, sgs) - om.residual(ph, Q)).reshape(5, 4, 4, 4, -1)  # [v][ez][ey][ex]
    inner = d[:, 1:3, 1:3, 1:3, :]
    for v in range(5):
        assert np.allclose(inner[v], -a[v].sum(), atol=1e-11)
    mp = box_mesh(3, 3, 3, periodic=(True,) * 3, curve=0.03)
    op = oracle_mod.OracleMesh(mp, 3)
    _, wJp = op.solpts()
    sg = uniform_noise((15, op.n_solpts), 12)
    dp = (op.residual(ph, Q[:, :op.E], sg) - op.residual(ph, Q[:, :op.E])).reshape(5, -1)
    for v in range(5):
        assert abs((dp[v] * wJp).sum()) < 1e-12 * np.abs(dp[v] * wJp).sum()
