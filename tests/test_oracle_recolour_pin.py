"""Pin of the recolouring operator's magnitude in the two-component oracle.

The colour-gradient model (Sec. III.A) moves species 1 towards its own phase
by giving each moving population a share beta (rho1 rho2/rho) w_i (c_i.n)/|c_i|
on top of the share rho1/rho of the mixture population (the recolouring
reading of the oracle; n = G/D with the smoothed norm of the gradient of the
phase field phi, Sec. III.B).  Species and momentum conservation fix only the
operator's zero mass and its sign; this test fixes its size.

Setup: a flat interface, species-1 fraction a(s) varying along one axis s
only, total density 1, no velocity, equilibrium pressure tensor and no
surface tension (A = 0).  The mixture populations are then w_i at every node
before and after the step, so the mixture stays at rest and only rho1 moves.
Summing the pulled species-1 populations over the directions with the same
component c_s gives, with b = a (1 - a) and the exact fractions of the weights
(W0 = sum of w_i over c_s = 0 = 2/3, W1 = sum over c_s = +1 = 1/6, for both
lattices):

    a'(s) = W0 a(s) + W1 [a(s-1) + a(s+1)]
            + beta K [b(s-1) n(s-1) - b(s+1) n(s+1)],

    K = sum over c_s = +1 of w_i / |c_i|,
    n = g / sqrt(g^2 + eps^2),  g(s) = (phi(s+1) - phi(s-1)) / 2,  phi = 2a - 1,

the component of the colour gradient along s being
(1/c_s^2) (W1 phi(s+1) - W1 phi(s-1)) = g.  K is 1/18 + 4/(36 sqrt 2) for
D3Q19 and 2/27 + 4/(54 sqrt 2) + 4/(216 sqrt 3) for D3Q27, so a dropped 1/|c_i|,
a misplaced beta, a wrong weight or a mis-scaled gradient changes a' by far
more than the 1e-15 allowed.
"""
import math

import numpy as np
import pytest

EPS_G = 1e-3  # smoothing of the normal's norm (the oracle's reading)

K_BY_LATTICE = {
    19: 1.0 / 18.0 + 4.0 / (36.0 * math.sqrt(2.0)),
    27: 2.0 / 27.0 + 4.0 / (54.0 * math.sqrt(2.0)) + 4.0 / (216.0 * math.sqrt(3.0)),
}


def _profile(n, seed):
    """Species-1 fraction along the axis: two smooth interfaces (a slab of
    species 1) plus a small random ripple, values inside (0, 1)."""
    s = np.arange(n, dtype=np.float64)
    a = 0.5 * (np.tanh((s - 0.3 * n) / 1.7) - np.tanh((s - 0.7 * n) / 1.3))
    rng = np.random.default_rng(seed)
    a = 0.02 + 0.96 * a + 0.005 * rng.standard_normal(n)
    return np.clip(a, 0.01, 0.99)


def _closed_form(a, beta, K):
    phi = 2.0 * a - 1.0
    g = 0.5 * (np.roll(phi, -1) - np.roll(phi, 1))  # (phi(s+1) - phi(s-1)) / 2
    n = g / np.sqrt(g * g + EPS_G * EPS_G)
    b = a * (1.0 - a)
    bn = b * n
    left = np.roll(a, 1)    # a(s-1)
    right = np.roll(a, -1)  # a(s+1)
    return (2.0 / 3.0) * a + (1.0 / 6.0) * (left + right) + beta * K * (np.roll(bn, 1) - np.roll(bn, -1))


def _state(a, axis, shape):
    """Two-component public moments (rho1, rho2, j, P) with rho1 = a along
    `axis` (0 = x, 1 = y, 2 = z), rho = 1, u = 0, P = I/3."""
    nz, ny, nx = shape
    H = np.zeros((11, nz, ny, nx))
    view = [1, 1, 1]
    view[2 - axis] = a.size
    rho1 = np.broadcast_to(a.reshape(view), shape)
    H[0] = rho1
    H[1] = 1.0 - rho1
    H[5] = H[6] = H[7] = 1.0 / 3.0
    return H


def _line(field, axis):
    idx = [0, 0, 0]
    idx[2 - axis] = slice(None)
    return field[tuple(idx)]


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("beta", [0.7, 0.35])
def test_flat_interface_one_step_closed_form(oracle, q, axis, beta):
    n = 24
    a = _profile(n, seed=100 * q + 10 * axis + int(beta * 10))
    shape = [4, 5, 6]
    shape[2 - axis] = n
    H = _state(a, axis, tuple(shape))
    out = oracle.cg_moment_run(H, q, 0.8, 0.0, beta, 1)
    expect = _closed_form(a, beta, K_BY_LATTICE[q])
    # rho1 follows the closed form on every line along the axis
    rho1 = np.moveaxis(out[0], 2 - axis, -1).reshape(-1, n)
    assert np.abs(rho1 - expect[None, :]).max() <= 1e-15
    # the mixture stays at rest: rho = 1, j = 0, P = I/3
    assert np.abs(out[0] + out[1] - 1.0).max() <= 1e-15
    assert np.abs(out[2:5]).max() <= 1e-16
    assert np.abs(out[5:8] - 1.0 / 3.0).max() <= 1e-15
    assert np.abs(out[8:11]).max() <= 1e-16


@pytest.mark.parametrize("q", [19, 27])
def test_flat_interface_iterates_closed_form(oracle, q):
    """The mixture stays at rest, so the closed form applies step after step:
    five oracle steps equal five applications of it."""
    n = 20
    a = _profile(n, seed=q)
    H = _state(a, 0, (3, 3, n))
    out = oracle.cg_moment_run(H, q, 0.8, 0.0, 0.7, 5)
    expect = a.copy()
    for _ in range(5):
        expect = _closed_form(expect, 0.7, K_BY_LATTICE[q])
    assert np.abs(_line(out[0], 0) - expect).max() <= 1e-14


@pytest.mark.parametrize("q", [19, 27])
def test_closed_form_recolouring_sharpens(q):
    """Sanity of the closed form itself: without recolouring (beta = 0) it is
    a diffusion step that conserves mass; with recolouring the interface
    sharpens (the slab's profile moves away from 1/2 on both sides)."""
    a = _profile(32, seed=3)
    d0 = _closed_form(a, 0.0, K_BY_LATTICE[q])
    d1 = _closed_form(a, 0.7, K_BY_LATTICE[q])
    assert abs(d0.sum() - a.sum()) < 1e-13 and abs(d1.sum() - a.sum()) < 1e-13
    assert np.abs(d1 - 0.5).sum() > np.abs(d0 - 0.5).sum()
