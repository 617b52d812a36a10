"""Seeded synthetic inputs: initial densities and velocities.

This module holds no lattice Boltzmann arithmetic.  It produces primitive
fields only (densities per species and a velocity field); both the GPU
library and the CPU oracle build their own moment states from them.  Random
draws use numpy's PCG64 with the stated seeds, so every workload is
reproducible bit for bit.

Array convention: scalar fields (nz, ny, nx), vector fields (3, nz, ny, nx),
float64, x fastest.

The paper's own workloads are droplet collisions in periodic boxes
(Sec. IV); no dataset is involved.  The generators below produce those
droplets plus the periodic flows used for closed-form checks and for
throughput: a two-dimensional Taylor-Green vortex, a random solenoidal
velocity field, and a shear wave with solenoidal noise.
"""
from __future__ import annotations

import numpy as np


def _grid(shape):
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    return x, y, z


def taylor_green_2d(n: int = 32, u0: float = 0.01, nz: int | None = None):
    """u = u0 (sin kx cos ky, -cos kx sin ky, 0), k = 2 pi / n, uniform density.

    Invariant along z; an exact incompressible Navier-Stokes solution whose
    amplitude decays as exp(-2 nu k^2 t).
    """
    shape = (nz or n, n, n)
    x, y, _ = _grid(shape)
    k = 2.0 * np.pi / n
    rho = np.ones(shape)
    u = np.zeros((3,) + shape)
    u[0] = u0 * np.sin(k * x) * np.cos(k * y) * np.ones(shape)
    u[1] = -u0 * np.cos(k * x) * np.sin(k * y) * np.ones(shape)
    return rho, u


def shear_wave(shape, u0: float, axis_u: int = 0, axis_k: int = 1, mode: int = 1, phase: float = 0.0):
    """u_{axis_u} = u0 sin(2 pi mode s / L + phase) along axis_k (x=0, y=1, z=2)."""
    x, y, z = _grid(shape)
    s = (x, y, z)[axis_k]
    L = shape[2 - axis_k]
    rho = np.ones(shape)
    u = np.zeros((3,) + shape)
    u[axis_u] = u0 * np.sin(2.0 * np.pi * mode * s / L + phase) * np.ones(shape)
    return rho, u


def solenoidal(shape, seed: int, umax: float, kmax: int = 4) -> np.ndarray:
    """Random divergence-free velocity u = curl(psi), psi a random vector
    potential on the integer Fourier modes 1 <= |n|_inf <= kmax, scaled so that
    max over nodes of |u| equals umax.

    The field is evaluated as a separable sum over the (2 kmax + 1)^3 modes,
    which keeps memory at a few copies of the output even for 512^3 boxes.
    """
    nz, ny, nx = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    m = np.arange(-kmax, kmax + 1)
    nm = m.size
    coef = rng.standard_normal((3, nm, nm, nm)) + 1j * rng.standard_normal((3, nm, nm, nm))
    mz, my, mx = np.meshgrid(m, m, m, indexing="ij")
    keep = np.maximum(np.maximum(np.abs(mx), np.abs(my)), np.abs(mz)) >= 1
    coef *= keep[None]
    kx = 2.0 * np.pi * mx / nx
    ky = 2.0 * np.pi * my / ny
    kz = 2.0 * np.pi * mz / nz
    # u_hat = i k x psi_hat
    uh = np.empty_like(coef)
    uh[0] = 1j * (ky * coef[2] - kz * coef[1])
    uh[1] = 1j * (kz * coef[0] - kx * coef[2])
    uh[2] = 1j * (kx * coef[1] - ky * coef[0])
    ez = np.exp(2j * np.pi * np.outer(np.arange(nz), m) / nz)  # (nz, nm)
    ey = np.exp(2j * np.pi * np.outer(np.arange(ny), m) / ny)
    ex = np.exp(2j * np.pi * np.outer(np.arange(nx), m) / nx)
    u = np.empty((3, nz, ny, nx))
    for a in range(3):
        t = np.tensordot(ez, uh[a], axes=([1], [0]))          # (nz, nm_y, nm_x)
        t = np.tensordot(t, ey, axes=([1], [1]))              # (nz, nm_x, ny)
        t = np.tensordot(t, ex, axes=([1], [1]))              # (nz, ny, nx)
        u[a] = t.real
    speed = np.sqrt((u * u).sum(axis=0)).max()
    u *= umax / speed
    return u


def random_solenoidal_box(n: int, seed: int, umax: float = 1e-3, kmax: int = 4):
    """Uniform density with a random solenoidal velocity (periodic n^3 box)."""
    shape = (n, n, n)
    return np.ones(shape), solenoidal(shape, seed, umax, kmax)


def shear_wave_with_noise(n: int, seed: int, u0: float = 0.01, noise: float = 1e-4, kmax: int = 4):
    """u_x = u0 sin(2 pi y / n) plus solenoidal noise of maximum norm `noise`."""
    shape = (n, n, n)
    rho, u = shear_wave(shape, u0, axis_u=0, axis_k=1)
    u += solenoidal(shape, seed, noise, kmax)
    return rho, u


def droplets(shape, centres, radius: float, velocities, width: float = 1.5):
    """Two-species droplets in a periodic box.

    Species 1 inside each sphere, species 2 outside:
    rho1 = sum_k 1/2 [1 - tanh((r_k - R)/width)], rho2 = 1 - rho1, with r_k the
    minimum-image distance to centre k.  Each drop moves with its velocity
    weighted by its own profile; the carrier fluid starts at rest.
    """
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    rho1 = np.zeros(shape)
    u = np.zeros((3,) + shape)
    for (cx, cy, cz), vel in zip(centres, velocities):
        dx = (x - cx + nx / 2.0) % nx - nx / 2.0
        dy = (y - cy + ny / 2.0) % ny - ny / 2.0
        dz = (z - cz + nz / 2.0) % nz - nz / 2.0
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        prof = 0.5 * (1.0 - np.tanh((r - radius) / width))
        rho1 += prof
        for a in range(3):
            u[a] += vel[a] * prof
    rho1 = np.clip(rho1, 0.0, 1.0)
    rho2 = 1.0 - rho1
    return rho1, rho2, u


def random_moments(shape, seed: int, drho: float = 0.02, dj: float = 0.02, dp: float = 0.01):
    """A random single-component moment state near rest, for identity checks:
    rho = 1 + drho N(0,1), j = dj N(0,1), P_aa = rho/3 + dp N(0,1),
    P_ab = dp N(0,1) (a != b).  Field order rho, jx, jy, jz, Pxx, Pyy, Pzz,
    Pxy, Pxz, Pyz.  The non-equilibrium part is generic (not small)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = np.empty((10,) + tuple(shape))
    H[0] = 1.0 + drho * rng.standard_normal(shape)
    H[1:4] = dj * rng.standard_normal((3,) + tuple(shape))
    H[4:7] = H[0] / 3.0 + dp * rng.standard_normal((3,) + tuple(shape))
    H[7:10] = dp * rng.standard_normal((3,) + tuple(shape))
    return H


# ---- the named workloads ---------------------------------------------------

SEED_C2 = 16220002
SEED_C4 = 16220004
SEED_C5 = 16220005


def droplet_collision_512(shape=(256, 256, 512)):
    """Two drops of radius 40 moving at +-0.05 along x, offset 0.5 R in y."""
    return droplets(shape, centres=[(176.0, 118.0, 128.0), (336.0, 138.0, 128.0)], radius=40.0,
                    velocities=[(0.05, 0.0, 0.0), (-0.05, 0.0, 0.0)])


def droplet_collision_128(shape=(128, 128, 128)):
    """Two drops of radius 20 moving at +-0.05 along x, offset 0.5 R in y."""
    return droplets(shape, centres=[(34.0, 59.0, 64.0), (94.0, 69.0, 64.0)], radius=20.0,
                    velocities=[(0.05, 0.0, 0.0), (-0.05, 0.0, 0.0)])


# The paper's validation collisions (Sec. IV): two drops of diameter 30 in a
# periodic 128^3 box, tau = 0.8, sigma = 0.01, beta = 0.7 (readings of the
# parameters the paper leaves to an external table; the impact parameter b
# in units of D, U_rel in units of the capillary velocity sigma/(rho nu),
# centres 38 apart along x).  A_h is the near-contact strength of the case.
PAPER_TAU, PAPER_SIGMA, PAPER_BETA, PAPER_HMAX = 0.8, 0.01, 0.7, 4
PAPER_CASES = {
    "off_axis": dict(b=0.85, u_rel=0.5, A_h=0.01),
    "head_on": dict(b=0.0, u_rel=0.25, A_h=0.01),
    "coalescence": dict(b=0.85, u_rel=0.5, A_h=0.0),
    "head_on_coalescence": dict(b=0.0, u_rel=0.25, A_h=0.0),
}


def paper_collision(case: str, n: int = 128):
    """(rho1, rho2, u) of a validation case on an n^3 box (drops of diameter
    30 n/128 moving at +-U_rel/2 along x, offset b D across the motion)."""
    c = PAPER_CASES[case]
    scale = n / 128.0
    D = 30.0 * scale
    u_cap = PAPER_SIGMA / (1.0 * (PAPER_TAU - 0.5) / 3.0)       # sigma / (rho nu)
    v = 0.5 * c["u_rel"] * u_cap
    dy = c["b"] * D
    cx, cy, cz = n / 2.0, n / 2.0, n / 2.0
    sep = 38.0 * scale
    centres = [(cx - sep / 2, cy - dy / 2, cz), (cx + sep / 2, cy + dy / 2, cz)]
    return droplets((n, n, n), centres=centres, radius=D / 2, velocities=[(v, 0, 0), (-v, 0, 0)])
