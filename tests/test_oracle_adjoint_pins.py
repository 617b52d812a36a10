"""Pins of the oracle's discrete adjoint against the (pinned) forward oracle:
dot-product tests with central finite-difference Jacobian-vector products,
and the tau-sensitivity of a multi-step loss against finite differences."""
import numpy as np
import pytest

from paper_2301_01622_amd import inputs as I


@pytest.mark.parametrize("q", [19, 27])
def test_adjoint_dot_product(oracle, q):
    """<J v, w> = <v, J^T w> with J v by central differences (eps = 1e-6,
    truncation O(eps^2))."""
    shape = (4, 5, 6)
    M = I.random_moments(shape, seed=61)
    rng = np.random.default_rng(62)
    v = rng.standard_normal(M.shape)
    w = rng.standard_normal(M.shape)
    tau, eps = 0.67, 1e-6
    Jv = (oracle.moment_run(M + eps * v, q, tau, 1) - oracle.moment_run(M - eps * v, q, tau, 1)) / (2 * eps)
    JTw, _ = oracle.moment_adjoint_step(M, w, q, tau)
    lhs, rhs = np.sum(Jv * w), np.sum(v * JTw)
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)


@pytest.mark.parametrize("q", [19, 27])
def test_adjoint_omega_sensitivity(oracle, q):
    shape = (3, 4, 5)
    M = I.random_moments(shape, seed=63)
    w = np.random.default_rng(64).standard_normal(M.shape)
    tau, h = 0.7, 1e-6
    # d/domega <F(M; omega), w> by central differences in omega = 1/tau
    om = 1 / tau
    fp = oracle.moment_run(M, q, 1 / (om + h), 1)
    fm = oracle.moment_run(M, q, 1 / (om - h), 1)
    fd = np.sum((fp - fm) * w) / (2 * h)
    _, dom = oracle.moment_adjoint_step(M, w, q, tau)
    assert abs(fd - dom) <= 1e-7 * abs(fd)


def test_rollout_gradient_matches_finite_differences(oracle):
    """L = sum over nodes of (u_x(T) * pattern); gradient w.r.t. the initial
    velocity along a seeded solenoidal direction and w.r.t. tau."""
    q, n, T, tau = 19, 8, 12, 0.8
    rho, u0 = I.random_solenoidal_box(n, seed=65, umax=0.02)
    d = I.solenoidal((n, n, n), seed=66, umax=1.0)
    pattern = np.random.default_rng(67).standard_normal((n, n, n))

    def loss(u, t):
        M = oracle.moment_run(oracle.equilibrium_moments(rho, u), q, t, T)
        return np.sum(M[1] / M[0] * pattern), M

    L0, MT = loss(u0, tau)
    lam_T = np.zeros_like(MT)
    lam_T[0] = -MT[1] / MT[0] ** 2 * pattern
    lam_T[1] = pattern / MT[0]
    lam0, dL_dtau = oracle.moment_rollout_gradient(oracle.equilibrium_moments(rho, u0), lam_T, q, tau, T)
    # chain to u0 through M0 = (rho, rho u, rho/3 I + rho u u)
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    g_u = np.zeros_like(u0)
    for a in range(3):
        g_u[a] += rho * lam0[1 + a]
    for k, (a, b) in enumerate(pairs):
        g_u[a] += rho * u0[b] * lam0[4 + k]
        g_u[b] += rho * u0[a] * lam0[4 + k]
    h = 1e-4
    fd_u = (loss(u0 + h * d, tau)[0] - loss(u0 - h * d, tau)[0]) / (2 * h)
    assert abs(np.sum(g_u * d) - fd_u) <= 1e-6 * abs(fd_u)
    fd_tau = (loss(u0, tau + h)[0] - loss(u0, tau - h)[0]) / (2 * h)
    assert abs(dL_dtau - fd_tau) <= 1e-6 * abs(fd_tau)


def _cg_state(oracle, shape, seed):
    nz, ny, nx = shape
    r1, r2, u = I.droplets(shape, centres=[(nx * 0.3, ny * 0.45, nz * 0.5), (nx * 0.7, ny * 0.55, nz * 0.5)],
                           radius=min(shape) * 0.25, velocities=[(0.05, 0.0, 0.0), (-0.05, 0.0, 0.0)])
    H = oracle.equilibrium_moments2(r1, r2, u)
    H[5:] += 1e-3 * np.random.default_rng(seed).standard_normal(H[5:].shape)
    return np.ascontiguousarray(H)


@pytest.mark.parametrize("q", [19, 27])
def test_cg_adjoint_dot_product(oracle, q):
    """Two components: <J v, w> = <v, J^T w>, J v by central differences."""
    shape = (6, 7, 8)
    M = _cg_state(oracle, shape, 71)
    rng = np.random.default_rng(72)
    v = rng.standard_normal(M.shape)
    w = rng.standard_normal(M.shape)
    tau, sigma, beta, eps = 0.8, 0.01, 0.7, 1e-7
    A = oracle.sigma_to_A(sigma, tau)
    Jv = (oracle.cg_moment_run(M + eps * v, q, tau, A, beta, 1)
          - oracle.cg_moment_run(M - eps * v, q, tau, A, beta, 1)) / (2 * eps)
    JTw, _ = oracle.cg_adjoint_step(M, w, q, tau, sigma, beta)
    lhs, rhs = np.sum(Jv * w), np.sum(v * JTw)
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


def test_cg_adjoint_tau_sensitivity(oracle):
    """dL/dtau at fixed sigma (A = 9 sigma/(2 tau) moves with tau)."""
    q, shape = 19, (6, 7, 8)
    M = _cg_state(oracle, shape, 73)
    w = np.random.default_rng(74).standard_normal(M.shape)
    tau, sigma, beta, h = 0.8, 0.01, 0.7, 1e-6

    def F(t):
        return oracle.cg_moment_run(M, q, t, oracle.sigma_to_A(sigma, t), beta, 1)

    fd = np.sum((F(tau + h) - F(tau - h)) * w) / (2 * h)
    _, dt = oracle.cg_adjoint_step(M, w, q, tau, sigma, beta)
    assert abs(fd - dt) <= 1e-6 * abs(fd)


def test_cg_rollout_gradient_centroid_loss(oracle):
    """Droplet-centroid loss of the two-component configuration at small
    size: gradient w.r.t. the initial velocity (seeded solenoidal direction)
    and tau against central differences.  Two steps: with recolouring the
    linearised dynamics amplifies perturbations by orders of magnitude per
    few steps (measured, see the design notes), so finite differences over
    long horizons leave the linear regime."""
    q, n, T, tau, sigma, beta = 19, 16, 2, 0.8, 0.01, 0.7
    shape = (n, n, n)
    r1, r2, u0 = I.droplets(shape, centres=[(4.5, 7.0, 8.0), (11.5, 9.0, 8.0)], radius=3.0,
                            velocities=[(0.05, 0.0, 0.0), (-0.05, 0.0, 0.0)])
    d = I.solenoidal(shape, seed=75, umax=1.0)
    x = np.arange(n)[None, None, :] * np.ones(shape)
    left = x < n / 2

    def loss_and_grad_T(M):
        # L = sum_k |c_k - c_k*|^2 over the x-centroid of rho1 in each half
        L, g = 0.0, np.zeros_like(M)
        for mask, target in ((left, 4.5 + 2.0), (~left, 11.5 - 2.0)):
            m = M[0] * mask
            S, X = m.sum(), (m * x).sum()
            c = X / S
            L += (c - target) ** 2
            g[0] += 2 * (c - target) * mask * (x * S - X) / S ** 2
        return L, g

    def run(u, t):
        M0 = oracle.equilibrium_moments2(r1, r2, u)
        return oracle.cg_moment_run(M0, q, t, oracle.sigma_to_A(sigma, t), beta, T)

    L0, gT = loss_and_grad_T(run(u0, tau))
    M0 = oracle.equilibrium_moments2(r1, r2, u0)
    lam0, dL_dtau = oracle.cg_rollout_gradient(M0, gT, q, tau, sigma, beta, T)
    rho = r1 + r2
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    g_u = np.zeros_like(u0)
    for a in range(3):
        g_u[a] += rho * lam0[2 + a]
    for k, (a, b) in enumerate(pairs):
        g_u[a] += rho * u0[b] * lam0[5 + k]
        g_u[b] += rho * u0[a] * lam0[5 + k]
    h = 1e-6
    fd_u = (loss_and_grad_T(run(u0 + h * d, tau))[0] - loss_and_grad_T(run(u0 - h * d, tau))[0]) / (2 * h)
    assert abs(np.sum(g_u * d) - fd_u) <= 1e-5 * abs(fd_u)
    fd_t = (loss_and_grad_T(run(u0, tau + h))[0] - loss_and_grad_T(run(u0, tau - h))[0]) / (2 * h)
    assert abs(dL_dtau - fd_t) <= 1e-5 * abs(fd_t)


def test_cg_rollout_without_recolouring_long_horizon(oracle):
    """Without recolouring (beta = 0) the two-component adjoint stays well
    conditioned: 16 steps against central differences in a random direction."""
    q, n, T, tau, sigma = 19, 16, 16, 0.8, 0.01
    shape = (n, n, n)
    r1, r2, u0 = I.droplets(shape, centres=[(4.5, 7.0, 8.0), (11.5, 9.0, 8.0)], radius=3.0,
                            velocities=[(0.05, 0.0, 0.0), (-0.05, 0.0, 0.0)])
    M0 = oracle.equilibrium_moments2(r1, r2, u0)
    rng = np.random.default_rng(76)
    W = rng.standard_normal(M0.shape)
    v = rng.standard_normal(M0.shape)
    lam0, _ = oracle.cg_rollout_gradient(M0, W, q, tau, sigma, 0.0, T)
    A, h = oracle.sigma_to_A(sigma, tau), 1e-8
    fd = (np.sum(W * oracle.cg_moment_run(M0 + h * v, q, tau, A, 0.0, T))
          - np.sum(W * oracle.cg_moment_run(M0 - h * v, q, tau, A, 0.0, T))) / (2 * h)
    assert abs(np.sum(lam0 * v) - fd) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("species", [1, 2])
def test_equilibrium_adjoint_dot_product(oracle, species):
    """The oracle's chain through the equilibrium map M = (rho^k, rho u,
    rho c_s^2 I + rho u u) against central differences of the forward map:
    <J v, w> = <v, J^T w> for random directions v of (rho^k, u) and random
    moment weights w (the map is quadratic, so the central difference is
    exact up to rounding)."""
    shape = (3, 4, 5)
    rng = np.random.default_rng(71 + species)
    rho_k = 0.5 + rng.random((species,) + shape)
    u = 0.1 * rng.standard_normal((3,) + shape)
    v_rho = rng.standard_normal(rho_k.shape)
    v_u = rng.standard_normal(u.shape)
    w = rng.standard_normal((9 + species,) + shape)

    def fwd(r, uu):
        return oracle.equilibrium_moments(r[0], uu) if species == 1 else oracle.equilibrium_moments2(r[0], r[1], uu)

    eps = 1e-3

    def at(t):
        return fwd(rho_k + t * v_rho, u + t * v_u)

    Jv = (8 * (at(eps) - at(-eps)) - (at(2 * eps) - at(-2 * eps))) / (12 * eps)
    JTw = oracle.equilibrium_adjoint(rho_k[0] if species == 1 else rho_k, u, w)
    lhs = np.sum(Jv * w)
    rhs = np.sum(v_rho * JTw[:species]) + np.sum(v_u * JTw[species:])
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # a single component: dP_xy/du_x = rho u_y
    g = np.zeros_like(w)
    g[species + 6] = 1.0  # the Pxy weight
    JT = oracle.equilibrium_adjoint(rho_k[0] if species == 1 else rho_k, u, g)
    rho = rho_k.sum(0)
    np.testing.assert_allclose(JT[species], rho * u[1], rtol=1e-15)
    np.testing.assert_allclose(JT[species + 1], rho * u[0], rtol=1e-15)
    np.testing.assert_allclose(JT[species + 2], 0.0)
    np.testing.assert_allclose(JT[0], u[0] * u[1], rtol=1e-15)
