"""Python handle on the C-ABI library: device memory and streams via PyTorch.

``LBM`` wraps one ``lbm_ctx``.  Moment tensors use the public layout of
include/lbm.h: shape (nfields, nz, ny, nx), x fastest, fields
(rho | rho1, rho2), jx, jy, jz, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz, with j = rho u.
Every computation runs in the library's HIP kernels; this module only passes
pointers, sizes and the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib

_STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


class LBM:
    """One periodic box advanced by the moment-only scheme (or, with
    scheme="population" / "population_aa", by the population-storing
    baselines with two copies / in place; split=True runs the moment scheme
    as the paper's split approach, a collision pass and a streaming pass)."""

    def __init__(self, shape, lattice: int = 19, tau: float = 0.8, species: int = 1, *,
                 scheme: str = "moment", storage: str = "f32", beta: float = 0.7, sigma: float = 0.01,
                 s_pi: float = 0.0, device: int = 0, stream: torch.cuda.Stream | None = None,
                 check_every: int = 0, split: bool = False, steps_per_sweep: int = 0, nc_A: float = 0.0,
                 nc_hmax: int = 0, state_buffers=None):
        lib = _lib.load()
        self.nx, self.ny, self.nz = (int(s) for s in shape)
        self.q, self.tau, self.species = int(lattice), float(tau), int(species)
        self.scheme, self.storage = scheme, storage
        self.split, self.steps_per_sweep = bool(split), int(steps_per_sweep)
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        opts = _lib.Opts()
        lib.lbm_default_opts(ctypes.byref(opts))
        opts.scheme = _lib.SCHEME[scheme]
        opts.storage = _lib.STORAGE[storage]
        opts.beta = beta
        opts.sigma = sigma
        opts.s_pi = s_pi
        opts.stream = ctypes.c_void_p(self.stream.cuda_stream)
        opts.device = device
        opts.check_every = check_every
        opts.split = int(bool(split))
        opts.steps_per_sweep = int(steps_per_sweep)
        opts.nc_A = float(nc_A)
        opts.nc_hmax = int(nc_hmax)
        if state_buffers is not None:
            # Caller-owned state copies (torch device tensors of at least
            # state_bytes_for() bytes each); kept alive with the context.
            bufs = list(state_buffers)
            nbytes = min(b.numel() * b.element_size() for b in bufs)
            for k, b in enumerate(bufs[:2]):
                assert b.is_cuda and b.is_contiguous()
                opts.state_buffers[k] = b.data_ptr()
            opts.state_buffer_bytes = nbytes
            self._state_buffers = bufs
        ctx = ctypes.c_void_p()
        rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(self.nx, self.ny, self.nz), self.q, self.tau,
                            self.species, ctypes.byref(opts))
        _lib.check(rc, None, "lbm_create")
        self._ctx = ctx
        self._lib = lib

    @staticmethod
    def state_bytes_for(shape, lattice: int = 19, species: int = 1, *, scheme: str = "moment",
                        storage: str = "f32", split: bool = False, steps_per_sweep: int = 0) -> int:
        """Bytes of one state copy a context of this setup uses (the size of
        each caller buffer passed as state_buffers)."""
        lib = _lib.load()
        opts = _lib.Opts()
        lib.lbm_default_opts(ctypes.byref(opts))
        opts.scheme = _lib.SCHEME[scheme]
        opts.storage = _lib.STORAGE[storage]
        opts.split = int(bool(split))
        opts.steps_per_sweep = int(steps_per_sweep)
        b = ctypes.c_int64()
        nx, ny, nz = (int(v) for v in shape)
        _lib.check(lib.lbm_state_bytes_for(_lib.Grid(nx, ny, nz), int(lattice), int(species), ctypes.byref(opts),
                                           ctypes.byref(b)), None, "state_bytes_for")
        return b.value

    # ---- properties -------------------------------------------------------
    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nfields(self) -> int:
        return 10 if self.species == 1 else 11

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    # ---- state ------------------------------------------------------------
    def _fields(self, t) -> _lib.Fields:
        if isinstance(t, torch.Tensor):
            assert t.is_contiguous() and t.dtype in (torch.float32, torch.float64)
            assert t.numel() % self.n_nodes == 0
            on_dev = 1 if t.is_cuda else 0
            return _lib.Fields(t.data_ptr(), self.n_nodes,
                               _lib.DTYPE_F64 if t.dtype == torch.float64 else _lib.DTYPE_F32, on_dev)
        a = t
        assert isinstance(a, np.ndarray) and a.flags.c_contiguous and a.dtype in (np.float32, np.float64)
        return _lib.Fields(a.ctypes.data, self.n_nodes,
                           _lib.DTYPE_F64 if a.dtype == np.float64 else _lib.DTYPE_F32, 0)

    def set_moments(self, M) -> None:
        """M: (nfields, nz, ny, nx) float32/float64, torch (any device) or numpy."""
        assert tuple(M.shape) == (self.nfields,) + self.shape, M.shape
        if isinstance(M, torch.Tensor) and M.is_cuda:
            M = M.contiguous()
        f = self._fields(M)
        _lib.check(self._lib.lbm_set_moments(self._ctx, ctypes.byref(f)), self._ctx, "set_moments")
        if isinstance(M, torch.Tensor) and M.is_cuda:
            self._keepalive = M  # the conversion may still be pending on the stream

    def set_equilibrium(self, rho, u) -> None:
        """rho: (nz,ny,nx) or (2,nz,ny,nx) for two species; u: (3,nz,ny,nx)."""
        if isinstance(rho, np.ndarray):
            prim = np.ascontiguousarray(np.concatenate([np.reshape(rho, (-1,) + self.shape), u], axis=0))
        else:
            prim = torch.cat([rho.reshape((-1,) + self.shape), u], dim=0).contiguous()
        assert prim.shape[0] == self.species + 3
        f = self._fields(prim)
        _lib.check(self._lib.lbm_set_equilibrium(self._ctx, ctypes.byref(f)), self._ctx, "set_equilibrium")
        if isinstance(prim, torch.Tensor) and prim.is_cuda:
            self._keepalive = prim  # the copy may still be pending on the stream

    def get_moments(self, dtype=torch.float64, device: str = "cuda") -> torch.Tensor:
        """Current (post-streaming) moments in the public layout."""
        dev = self.device if device == "cuda" else torch.device("cpu")
        out = torch.empty((self.nfields,) + self.shape, dtype=dtype, device=dev)
        if dev.type == "cpu":
            out = out.pin_memory() if torch.cuda.is_available() else out
        f = self._fields(out)
        _lib.check(self._lib.lbm_get_moments(self._ctx, ctypes.byref(f)), self._ctx, "get_moments")
        return out

    # ---- time stepping ---------------------------------------------------
    def step(self, n: int = 1) -> None:
        _lib.check(self._lib.lbm_step(self._ctx, int(n)), self._ctx, "step")

    def reduce(self) -> np.ndarray:
        """FP64 totals: sum rho (rho1), sum rho2, sum j."""
        out = (ctypes.c_double * 5)()
        _lib.check(self._lib.lbm_reduce(self._ctx, out), self._ctx, "reduce")
        return np.array(out[:])

    def memory_info(self):
        """(bytes of every stored state copy, minimum bytes moved per step)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _lib.check(self._lib.lbm_memory_info(self._ctx, ctypes.byref(a), ctypes.byref(b)), self._ctx)
        return a.value, b.value

    @property
    def state_bytes(self) -> int:
        """Bytes of one time level of the stored state."""
        b = ctypes.c_int64()
        _lib.check(self._lib.lbm_state_bytes(self._ctx, ctypes.byref(b)), self._ctx, "state_bytes")
        return b.value

    def new_checkpoint(self) -> torch.Tensor:
        """A device buffer able to hold one saved time level."""
        return torch.empty(self.state_bytes, dtype=torch.uint8, device=self.device)

    def save_state(self, buf: torch.Tensor) -> None:
        """Copies the current stored state into `buf` (device, state_bytes)."""
        assert buf.is_cuda and buf.numel() * buf.element_size() >= self.state_bytes
        _lib.check(self._lib.lbm_save_state(self._ctx, ctypes.c_void_p(buf.data_ptr())), self._ctx, "save_state")

    def load_state(self, buf: torch.Tensor) -> None:
        """Restores a state saved by save_state (same context shape/storage)."""
        assert buf.is_cuda and buf.numel() * buf.element_size() >= self.state_bytes
        _lib.check(self._lib.lbm_load_state(self._ctx, ctypes.c_void_p(buf.data_ptr())), self._ctx, "load_state")

    def step_state(self, src: torch.Tensor, dst: torch.Tensor) -> None:
        """One step from saved state `src` into buffer `dst` (both state_bytes)."""
        _lib.check(self._lib.lbm_step_state(self._ctx, ctypes.c_void_p(src.data_ptr()),
                                            ctypes.c_void_p(dst.data_ptr())), self._ctx, "step_state")

    def step_state2(self, src: torch.Tensor, mid: torch.Tensor, dst: torch.Tensor) -> None:
        """Two steps from saved state `src` in one pass: `mid` after the first,
        `dst` after the second (all state_bytes)."""
        _lib.check(self._lib.lbm_step_state2(self._ctx, ctypes.c_void_p(src.data_ptr()),
                                             ctypes.c_void_p(mid.data_ptr()), ctypes.c_void_p(dst.data_ptr())),
                   self._ctx, "step_state2")

    @property
    def sweeps(self) -> bool:
        """True if the context runs two-step sweeps (and has the two-step
        recompute and adjoint entry points)."""
        return int(self._lib.lbm_steps_per_sweep(self._ctx)) == 2

    @property
    def real_dtype(self):
        """Arithmetic type of the kernels (the co-state's element type)."""
        return torch.float64 if self.storage == "f64" else torch.float32

    def adjoint_step(self, state_t, lam_next, lam_out, dtau: float | None = None) -> float | None:
        """lam_out = (dM(t+1)/dM(t))^T lam_next at the state M(t) given as public
        moments; all three (nfields, nz, ny, nx) float32/float64, torch (host
        or device) or numpy.  Returns dtau + this step's dL/dtau if dtau is
        given (a float), else None."""
        for t in (state_t, lam_next, lam_out):
            assert tuple(t.shape) == (self.nfields,) + self.shape, t.shape
        fs, fl, fo = self._fields(state_t), self._fields(lam_next), self._fields(lam_out)
        acc = ctypes.c_double(0.0 if dtau is None else float(dtau))
        _lib.check(self._lib.lbm_adjoint_step(self._ctx, ctypes.byref(fs), ctypes.byref(fl), ctypes.byref(fo),
                                              ctypes.byref(acc) if dtau is not None else None),
                   self._ctx, "adjoint_step")
        return acc.value if dtau is not None else None

    # ---- the equilibrium map (initial fields -> initial moments) ------------
    def _prim_shape(self):
        return (self.species + 3,) + self.shape

    def equilibrium(self, prim, out=None):
        """Public moments (rho^k, rho u, rho c_s^2 I + rho u u) of the primitive
        fields prim = (rho | rho1, rho2, ux, uy, uz), shape (species+3, nz, ny,
        nx); the context's state is not touched."""
        assert tuple(prim.shape) == self._prim_shape(), prim.shape
        if out is None:
            out = torch.empty((self.nfields,) + self.shape, dtype=prim.dtype, device=prim.device)
        fi, fo = self._fields(prim), self._fields(out)
        _lib.check(self._lib.lbm_equilibrium_moments(self._ctx, ctypes.byref(fi), ctypes.byref(fo)), self._ctx,
                   "equilibrium_moments")
        return out

    def equilibrium_adjoint(self, prim, grad_moments, out=None):
        """Transpose of the Jacobian of equilibrium() at prim applied to a
        gradient with respect to the moments: dL/d(rho^k, u)."""
        assert tuple(prim.shape) == self._prim_shape(), prim.shape
        assert tuple(grad_moments.shape) == (self.nfields,) + self.shape, grad_moments.shape
        if out is None:
            out = torch.empty(self._prim_shape(), dtype=prim.dtype, device=prim.device)
        fp, fg, fo = self._fields(prim), self._fields(grad_moments), self._fields(out)
        _lib.check(self._lib.lbm_equilibrium_moments_adjoint(self._ctx, ctypes.byref(fp), ctypes.byref(fg),
                                                             ctypes.byref(fo)), self._ctx, "equilibrium_moments_adjoint")
        return out

    # ---- co-states in the stored layout -----------------------------------
    @property
    def costate_bytes(self) -> int:
        b = ctypes.c_int64()
        _lib.check(self._lib.lbm_costate_bytes(self._ctx, ctypes.byref(b)), self._ctx, "costate_bytes")
        return b.value

    def new_costate(self) -> torch.Tensor:
        """A zeroed device buffer for one co-state in the stored layout."""
        n = self.costate_bytes // torch.tensor([], dtype=self.real_dtype).element_size()
        return torch.zeros(n, dtype=self.real_dtype, device=self.device)

    def costate_to_stored(self, public: torch.Tensor, stored: torch.Tensor) -> None:
        assert public.dtype == self.real_dtype and public.is_contiguous() and public.is_cuda
        _lib.check(self._lib.lbm_costate_to_stored(self._ctx, ctypes.c_void_p(public.data_ptr()),
                                                   ctypes.c_void_p(stored.data_ptr())), self._ctx, "costate_to_stored")

    def costate_from_stored(self, stored: torch.Tensor, public: torch.Tensor) -> None:
        assert public.dtype == self.real_dtype and public.is_contiguous() and public.is_cuda
        _lib.check(self._lib.lbm_costate_from_stored(self._ctx, ctypes.c_void_p(stored.data_ptr()),
                                                     ctypes.c_void_p(public.data_ptr())), self._ctx,
                   "costate_from_stored")

    def adjoint_step_stored(self, state: torch.Tensor, lam_next: torch.Tensor, lam_out: torch.Tensor,
                            dtau_accum: torch.Tensor | None = None) -> None:
        """adjoint_step with both co-states in the stored layout (new_costate buffers)."""
        dptr = ctypes.c_void_p(dtau_accum.data_ptr()) if dtau_accum is not None else None
        _lib.check(self._lib.lbm_adjoint_step_stored(self._ctx, ctypes.c_void_p(state.data_ptr()),
                                                     ctypes.c_void_p(lam_next.data_ptr()),
                                                     ctypes.c_void_p(lam_out.data_ptr()), dptr), self._ctx,
                   "adjoint_step_stored")

    def adjoint_step2_stored(self, state_t1: torch.Tensor, state_t0: torch.Tensor, lam_next: torch.Tensor,
                             lam_out: torch.Tensor, dtau_accum: torch.Tensor | None = None) -> None:
        """Two adjoint steps in one pass (stored layout): lam_out =
        J(state_t0)^T J(state_t1)^T lam_next, state_t1 one step after state_t0."""
        dptr = ctypes.c_void_p(dtau_accum.data_ptr()) if dtau_accum is not None else None
        _lib.check(self._lib.lbm_adjoint_step2_stored(self._ctx, ctypes.c_void_p(state_t1.data_ptr()),
                                                      ctypes.c_void_p(state_t0.data_ptr()),
                                                      ctypes.c_void_p(lam_next.data_ptr()),
                                                      ctypes.c_void_p(lam_out.data_ptr()), dptr), self._ctx,
                   "adjoint_step2_stored")

    @property
    def steps_done(self) -> int:
        return int(self._lib.lbm_steps_done(self._ctx))

    def close(self) -> None:
        if getattr(self, "_ctx", None):
            self._lib.lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
