"""FP64 CPU oracle for the lattice Boltzmann scheme without populations.

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow implementation of the
paper's equations in C (``liboracle.so``, built by ``oracle/build.py``) plus
this thin numpy wrapper.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it.  It shares no code with the GPU library and
does not import it.

Array convention: a state is a float64 array of shape (nfields, nz, ny, nx),
C-contiguous, x fastest.  Single component: rho, jx, jy, jz, Pxx, Pyy, Pzz,
Pxy, Pxz, Pyz (j = rho u).  Two components: rho1, rho2, then the same nine.
Populations: (q, nz, ny, nx) in the oracle's own velocity ordering
(``lattice(q)``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CS2 = 1.0 / 3.0


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i, d, l = ctypes.c_int, ctypes.c_double, ctypes.c_long
        sigs = {
            "ora_lattice": (i, [i, ip, dp]),
            "ora_reconstruct": (i, [i, dp, dp]),
            "ora_collide_node": (i, [i, d, dp, dp]),
            "ora_project_node": (i, [i, dp, dp]),
            "ora_moment_run": (i, [i, i, i, i, d, i, dp]),
            "ora_populations_from_moments": (i, [i, l, dp, dp]),
            "ora_moments_from_populations": (i, [i, l, dp, dp]),
            "ora_population_run": (i, [i, i, i, i, d, i, i, dp]),
            "ora_cg_moment_run": (i, [i, i, i, i, d, d, d, d, i, i, dp]),
            "ora_cg_population_run": (i, [i, i, i, i, d, d, d, i, d, i, i, dp, dp]),
            "ora_nc_force": (i, [i, i, i, i, dp, d, i, dp, ip]),
            "ora_forced_collide_node": (i, [i, d, d, dp, dp, dp, dp]),
            "ora_moment_adjoint_step": (i, [i, i, i, i, d, dp, dp, dp, dp]),
            "ora_cg_adjoint_step": (i, [i, i, i, i, d, d, d, dp, dp, dp, dp]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed (rc={rc})")


# ---- lattice and single-node operators ----------------------------------------

def lattice(q: int):
    """Velocities c (q,3) int and weights w (q,) of the oracle's D3Q19/D3Q27."""
    c = np.zeros(q * 3, dtype=np.int32)
    w = np.zeros(q, dtype=np.float64)
    rc = _load().ora_lattice(q, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    if rc != q:
        raise ValueError(f"unsupported lattice D3Q{q}")
    return c.reshape(q, 3).astype(np.int64), w


def reconstruct(q: int, H10) -> np.ndarray:
    """Eq. 4 at one node: populations h_i from the 10 hydro-fields."""
    H = np.ascontiguousarray(H10, dtype=np.float64)
    h = np.zeros(q)
    _check(_load().ora_reconstruct(q, _dp(H), _dp(h)), "reconstruct")
    return h


def collide_node(q: int, tau: float, H10) -> np.ndarray:
    """Eq. 7 applied to the Eq. 4 reconstruction of one node."""
    H = np.ascontiguousarray(H10, dtype=np.float64)
    h = np.zeros(q)
    _check(_load().ora_collide_node(q, tau, _dp(H), _dp(h)), "collide_node")
    return h


def project_node(q: int, f) -> np.ndarray:
    """Eqs. 1-3 at one node: the 10 hydro-fields of q populations."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    H = np.zeros(10)
    _check(_load().ora_project_node(q, _dp(f), _dp(H)), "project_node")
    return H


# ---- initial states -------------------------------------------------------------

def equilibrium_moments(rho, u) -> np.ndarray:
    """Single-component state with zero non-equilibrium part: j = rho u,
    P = rho c_s^2 I + rho u u (second moment of Eq. 5)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    H = np.empty((10,) + rho.shape)
    H[0] = rho
    H[1:4] = rho * u
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for k, (a, b) in enumerate(pairs):
        H[4 + k] = rho * u[a] * u[b] + (rho * CS2 if a == b else 0.0)
    return np.ascontiguousarray(H)


def equilibrium_moments2(rho1, rho2, u) -> np.ndarray:
    """Two-component state (rho1, rho2, j, P) at equilibrium of the mixture."""
    rho1 = np.asarray(rho1, dtype=np.float64)
    rho2 = np.asarray(rho2, dtype=np.float64)
    H1 = equilibrium_moments(rho1 + rho2, u)
    return np.ascontiguousarray(np.concatenate([rho1[None], rho2[None], H1[1:]], axis=0))


def equilibrium_adjoint(rho_k, u, gM) -> np.ndarray:
    """Chain rule through the equilibrium map: given dL/dM of a state built by
    equilibrium_moments (one species, rho_k of shape (nz, ny, nx)) or
    equilibrium_moments2 (rho_k = (rho1, rho2)), returns dL/d(rho_k, u) with
    shape (species + 3, nz, ny, nx).  The map is M = (rho^k, rho u,
    rho c_s^2 I + rho u u); written term by term: rho enters j_a = rho u_a
    and P_ab = rho u_a u_b + rho c_s^2 delta_ab, and u_c enters j_c and every
    P_ab with a = c or b = c."""
    u = np.asarray(u, dtype=np.float64)
    gM = np.asarray(gM, dtype=np.float64)
    rho_k = np.asarray(rho_k, dtype=np.float64)
    species = 1 if rho_k.ndim == 3 else rho_k.shape[0]
    rho = rho_k if species == 1 else rho_k.sum(0)
    off = 1 if species == 1 else 2
    gj = gM[off:off + 3]
    gP = gM[off + 3:off + 9]
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    # d/drho of j and P at fixed u
    g_rho = np.zeros_like(rho)
    for a in range(3):
        g_rho += gj[a] * u[a]
    for k, (a, b) in enumerate(pairs):
        g_rho += gP[k] * (u[a] * u[b] + (CS2 if a == b else 0.0))
    # d/du_c of j and P at fixed rho
    g_u = np.zeros_like(u)
    for c in range(3):
        g_u[c] += rho * gj[c]
    for k, (a, b) in enumerate(pairs):
        # d(rho u_a u_b)/du_a = rho u_b and d/du_b = rho u_a (both when a = b)
        g_u[a] += gP[k] * rho * u[b]
        g_u[b] += gP[k] * rho * u[a]
    out = np.empty((species + 3,) + rho.shape)
    if species == 1:
        out[0] = gM[0] + g_rho
    else:
        out[0] = gM[0] + g_rho
        out[1] = gM[1] + g_rho
    out[species:] = g_u
    return out


def sigma_to_A(sigma: float, tau: float) -> float:
    """Perturbation amplitude for a surface tension sigma (sigma = 2 A tau / 9)."""
    return 9.0 * sigma / (2.0 * tau)


# ---- runs ---------------------------------------------------------------------------

def moment_run(H, q: int, tau: float, nsteps: int) -> np.ndarray:
    """Single-component scheme without populations: nsteps from state H."""
    H = np.array(H, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = H.shape
    assert H.shape[0] == 10
    _check(_load().ora_moment_run(q, nx, ny, nz, tau, nsteps, _dp(H)), "moment_run")
    return H


def populations_from_moments(H, q: int) -> np.ndarray:
    """f = R(H) (Eq. 4) at every node."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    f = np.zeros((q,) + H.shape[1:])
    _check(_load().ora_populations_from_moments(q, H[0].size, _dp(H), _dp(f)), "populations_from_moments")
    return f


def moments_from_populations(f, q: int) -> np.ndarray:
    """H = P f (Eqs. 1-3) at every node."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    H = np.zeros((10,) + f.shape[1:])
    _check(_load().ora_moments_from_populations(q, f[0].size, _dp(f), _dp(H)), "moments_from_populations")
    return H


def population_run(f, q: int, tau: float, nsteps: int, regularize: bool = False) -> np.ndarray:
    """Population-storing BGK (optionally regularized): nsteps from f."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = f.shape
    _check(_load().ora_population_run(q, nx, ny, nz, tau, int(regularize), nsteps, _dp(f)), "population_run")
    return f


def cg_moment_run(H, q: int, tau: float, A: float, beta: float, nsteps: int, Ah: float = 0.0,
                  hmax: int = 0) -> np.ndarray:
    """Two-component colour-gradient scheme without populations (with the
    near-contact force of strength Ah and probe range hmax if Ah != 0)."""
    H = np.array(H, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = H.shape
    assert H.shape[0] == 11
    _check(_load().ora_cg_moment_run(q, nx, ny, nz, tau, A, beta, Ah, hmax, nsteps, _dp(H)), "cg_moment_run")
    return H


def cg_population_run(f1, f2, q: int, tau: float, A: float, beta: float, nsteps: int,
                      regularize: bool = False, Ah: float = 0.0, hmax: int = 0):
    """Two-component colour-gradient scheme with populations (one set per species)."""
    f1 = np.array(f1, dtype=np.float64, order="C", copy=True)
    f2 = np.array(f2, dtype=np.float64, order="C", copy=True)
    _, nz, ny, nx = f1.shape
    _check(_load().ora_cg_population_run(q, nx, ny, nz, tau, A, beta, int(regularize), Ah, hmax, nsteps,
                                         _dp(f1), _dp(f2)), "cg_population_run")
    return f1, f2


def forced_collide_node(q: int, tau: float, rho: float, j, P, F) -> np.ndarray:
    """Post-collision populations of one node under body force F (BGK with
    Guo's forcing; no colour-gradient operators)."""
    j = np.ascontiguousarray(j, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(9)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(q)
    _check(_load().ora_forced_collide_node(q, tau, rho, _dp(j), _dp(P), _dp(F), _dp(out)), "forced_collide_node")
    return out


def nc_force(phi, q: int, Ah: float, hmax: int):
    """Near-contact force field F (3, nz, ny, nx) and film distance h (nz, ny,
    nx; 0 where none) from a phase field phi (nz, ny, nx)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    nz, ny, nx = phi.shape
    F = np.zeros((3,) + phi.shape)
    h = np.zeros(phi.shape, dtype=np.int32)
    _check(_load().ora_nc_force(q, nx, ny, nz, _dp(phi), Ah, hmax, _dp(F),
                                h.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), "nc_force")
    return F, h


def cg_populations_from_moments(H11, q: int):
    """Species populations (rho^k/rho) R(H) for a two-component moment state."""
    H11 = np.ascontiguousarray(H11, dtype=np.float64)
    rho = H11[0] + H11[1]
    Ht = np.ascontiguousarray(np.concatenate([rho[None], H11[2:]], axis=0))
    f = populations_from_moments(Ht, q)
    return np.ascontiguousarray(f * (H11[0] / rho)), np.ascontiguousarray(f * (H11[1] / rho))


def cg_moments_from_populations(f1, f2, q: int) -> np.ndarray:
    """Two-component moments (rho1, rho2, j, P) of species populations."""
    Ht = moments_from_populations(np.ascontiguousarray(f1 + f2), q)
    return np.ascontiguousarray(np.concatenate([f1.sum(0)[None], f2.sum(0)[None], Ht[1:]], axis=0))


# ---- discrete adjoint ---------------------------------------------------------------

def moment_adjoint_step(M, lam_next, q: int, tau: float):
    """Transposed Jacobian of one single-component step at state M applied to
    lam_next; returns (lam, dL/domega contribution of this step)."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
    assert M.shape == lam_next.shape and M.shape[0] == 10
    _, nz, ny, nx = M.shape
    lam = np.zeros_like(M)
    dom = ctypes.c_double(0.0)
    _check(_load().ora_moment_adjoint_step(q, nx, ny, nz, tau, _dp(M), _dp(lam_next), _dp(lam),
                                           ctypes.byref(dom)), "moment_adjoint_step")
    return lam, dom.value


def moment_rollout_gradient(M0, lam_T, q: int, tau: float, nsteps: int):
    """Gradient of a scalar loss L(M(T)) with respect to M(0) and tau, given
    lam_T = dL/dM(T): forward states kept in memory, then nsteps adjoint steps."""
    states = [np.ascontiguousarray(M0, dtype=np.float64)]
    for _ in range(nsteps - 1):
        states.append(moment_run(states[-1], q, tau, 1))
    lam = np.ascontiguousarray(lam_T, dtype=np.float64)
    dL_domega = 0.0
    for t in reversed(range(nsteps)):
        lam, dom = moment_adjoint_step(states[t], lam, q, tau)
        dL_domega += dom
    return lam, -dL_domega / (tau * tau)


def cg_adjoint_step(M, lam_next, q: int, tau: float, sigma: float, beta: float):
    """Transposed Jacobian of one two-component step (fixed sigma); returns
    (lam, dL/dtau contribution of this step)."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
    assert M.shape == lam_next.shape and M.shape[0] == 11
    _, nz, ny, nx = M.shape
    lam = np.zeros_like(M)
    dt = ctypes.c_double(0.0)
    _check(_load().ora_cg_adjoint_step(q, nx, ny, nz, tau, sigma_to_A(sigma, tau), beta, _dp(M), _dp(lam_next),
                                       _dp(lam), ctypes.byref(dt)), "cg_adjoint_step")
    return lam, dt.value


def cg_rollout_gradient(M0, lam_T, q: int, tau: float, sigma: float, beta: float, nsteps: int):
    """Gradient of L(M(T)) w.r.t. the two-component M(0) and tau (fixed sigma)."""
    A = sigma_to_A(sigma, tau)
    states = [np.ascontiguousarray(M0, dtype=np.float64)]
    for _ in range(nsteps - 1):
        states.append(cg_moment_run(states[-1], q, tau, A, beta, 1))
    lam = np.ascontiguousarray(lam_T, dtype=np.float64)
    dL_dtau = 0.0
    for t in reversed(range(nsteps)):
        lam, dt = cg_adjoint_step(states[t], lam, q, tau, sigma, beta)
        dL_dtau += dt
    return lam, dL_dtau
