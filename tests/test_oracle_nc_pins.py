"""Pins of the oracle's near-contact force (the LBNCI term of Sec. III.B,
under the readings stated in oracle/color_gradient.c) and of its Guo forcing.

* Two flat slabs of species 1 with sharp interfaces across a film of w nodes:
  the colour gradient at the four nodes next to the film is +-1 along x (the
  weights of the directions with c_x = 1 sum to 1/6, times 3 times the jump
  of 2), the probes along +-x cross the film at k = w (film nodes) and
  k = w + 1 (slab nodes), every other node has G = 0 or no film in reach;
  the force is (A_h/2) G there and zero elsewhere, so it points into each
  slab (repulsion).
* BGK with Guo's forcing on one node: the post-collision moments are the
  closed form rho' = rho, j' = j + F,
  P' = (1 - w) P + w (rho u* u* + rho c_s^2 I) + (1 - w/2)(u* F + F u*),
  u* = (j + F/2)/rho.
* A forced two-component step conserves both species' masses and changes
  the total momentum by exactly the total force (the colour-gradient
  operators carry no momentum).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore")

import oracle  # noqa: E402


def _slabs(nx, w, q=19):
    """phi (nz, ny, nx) = +1 on x in [3, 8] and [9 + w, 14 + w], -1 elsewhere."""
    phi = -np.ones((3, 3, nx))
    phi[:, :, 3:9] = 1.0
    phi[:, :, 9 + w:15 + w] = 1.0
    return phi


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("w", [1, 2, 3])
def test_film_between_flat_slabs(q, w):
    nx, Ah = 40, 0.02
    phi = _slabs(nx, w, q)
    F, h = oracle.nc_force(phi, q, Ah, hmax=4)
    b1, a2 = 8, 9 + w                      # last node of slab 1, first of slab 2
    expect_h = np.zeros(nx, dtype=int)
    expect_F = np.zeros(nx)
    # slab nodes next to the film: probes cross it at k = w + 1
    if w + 1 <= 4:
        expect_h[b1], expect_h[a2] = w + 1, w + 1
        expect_F[b1], expect_F[a2] = -0.5 * Ah, 0.5 * Ah
    # film nodes next to a slab (G = +-1 only if the film is at least 2 wide)
    if w >= 2:
        expect_h[b1 + 1], expect_h[a2 - 1] = w, w
        expect_F[b1 + 1], expect_F[a2 - 1] = -0.5 * Ah, 0.5 * Ah
    for z in range(3):
        for y in range(3):
            np.testing.assert_array_equal(h[z, y], expect_h)
            np.testing.assert_allclose(F[0, z, y], expect_F, rtol=1e-15, atol=1e-17)
    assert np.abs(F[1:]).max() == 0.0
    # the outer faces see a wide film only: no force there
    assert h[:, :, 3].max() == 0 and h[:, :, 14 + w].max() == 0


def test_probe_range_cutoff():
    phi = _slabs(40, 3)
    _, h4 = oracle.nc_force(phi, 19, 0.01, hmax=4)
    _, h3 = oracle.nc_force(phi, 19, 0.01, hmax=3)
    assert h4[0, 0, 8] == 4 and h3[0, 0, 8] == 0     # slab node: film of 3 needs 4 probes
    assert h3[0, 0, 9] == 3                          # film node: 3 probes


@pytest.mark.parametrize("q", [19, 27])
def test_guo_forcing_closed_form(q):
    rng = np.random.default_rng(4)
    tau = 0.83
    om = 1.0 / tau
    rho = 1.03
    j = rng.normal(0, 0.02, 3)
    A = rng.normal(0, 0.01, (3, 3))
    P = rho / 3 * np.eye(3) + np.outer(j, j) / rho + 0.5 * (A + A.T)
    F = rng.normal(0, 0.003, 3)
    f = oracle.forced_collide_node(q, tau, rho, j, P, F)
    c, _ = oracle.lattice(q)
    us = (j + 0.5 * F) / rho
    Pexp = (1 - om) * P + om * (rho * np.outer(us, us) + rho / 3 * np.eye(3)) \
        + (1 - 0.5 * om) * (np.outer(us, F) + np.outer(F, us))
    assert abs(f.sum() - rho) < 1e-14
    np.testing.assert_allclose(f @ c, j + F, rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", f, c, c), Pexp, rtol=0, atol=1e-14)


@pytest.mark.parametrize("q", [19, 27])
def test_forced_step_momentum_and_mass(q):
    """Two slabs with soft, unequal interfaces (so the forces do not cancel):
    one forced step changes sum j by exactly sum F and keeps both masses."""
    nx = 32
    x = np.arange(nx)
    prof = np.tanh((x - 4.0) / 1.5) - np.tanh((x - 12.0) / 1.5) + np.tanh((x - 15.0) / 2.5) \
        - np.tanh((x - 25.0) / 2.5) - 1.0
    phi = np.clip(prof, -0.98, 0.98)[None, None, :] * np.ones((4, 5, 1))
    rho = np.ones_like(phi)
    r1, r2 = 0.5 * (1 + phi) * rho, 0.5 * (1 - phi) * rho
    H = oracle.equilibrium_moments2(r1, r2, np.zeros((3,) + phi.shape))
    Ah, hmax, tau = 0.05, 5, 0.9
    F, h = oracle.nc_force(phi, q, Ah, hmax)
    assert h.max() > 0 and abs(F[0].sum()) > 1e-6
    H1 = oracle.cg_moment_run(H, q, tau, oracle.sigma_to_A(0.01, tau), 0.7, 1, Ah=Ah, hmax=hmax)
    for a in range(3):
        assert abs(H1[2 + a].sum() - H[2 + a].sum() - F[a].sum()) < 1e-12
    assert abs(H1[0].sum() - H[0].sum()) < 1e-11 and abs(H1[1].sum() - H[1].sum()) < 1e-11
    # the same step with populations gives the same result (both forced)
    f1, f2 = oracle.cg_populations_from_moments(H, q)
    g1, g2 = oracle.cg_population_run(f1, f2, q, tau, oracle.sigma_to_A(0.01, tau), 0.7, 1, regularize=True,
                                      Ah=Ah, hmax=hmax)
    Hp = oracle.cg_moments_from_populations(g1, g2, q)
    assert np.abs(Hp - H1).max() < 1e-13


def test_zero_strength_is_the_unforced_scheme():
    rng = np.random.default_rng(5)
    H = oracle.equilibrium_moments2(0.5 + 0.4 * rng.random((4, 5, 6)), 0.5 + 0.0 * rng.random((4, 5, 6)),
                                    0.01 * rng.standard_normal((3, 4, 5, 6)))
    a = oracle.cg_moment_run(H, 19, 0.8, 0.02, 0.7, 3)
    b = oracle.cg_moment_run(H, 19, 0.8, 0.02, 0.7, 3, Ah=0.0, hmax=4)
    np.testing.assert_array_equal(a, b)
