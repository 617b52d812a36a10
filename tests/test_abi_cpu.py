"""Host-side checks of the C-ABI library that need no GPU: it loads, it
exports every entry point include/lbm.h declares, and argument validation
rejects bad input before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2301_01622_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lbm_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    declared = _declared()
    assert {"lbm_create", "lbm_step", "lbm_get_moments", "lbm_set_moments", "lbm_reduce",
            "lbm_destroy"} <= declared
    for name in sorted(declared):
        assert hasattr(lib, name), name


def test_error_strings_and_null_safety():
    lib = _lib.load()
    for code in (_lib.LBM_OK, _lib.LBM_EINVAL, _lib.LBM_ENOMEM, _lib.LBM_EDEVICE, _lib.LBM_EUNSTABLE,
                 _lib.LBM_ESTATE, -99):
        assert lib.lbm_strerror(code)
    assert lib.lbm_last_error(None) == b""
    assert lib.lbm_destroy(None) == _lib.LBM_OK
    assert lib.lbm_steps_done(None) == -1


@pytest.mark.parametrize("grid,q,tau,species,scheme,storage", [
    ((2, 8, 8), 19, 0.8, 1, 0, 1),     # side < 3
    ((8, 8, 8), 15, 0.8, 1, 0, 1),     # unknown lattice
    ((8, 8, 8), 19, 0.5, 1, 0, 1),     # tau must exceed 1/2
    ((8, 8, 8), 19, float("nan"), 1, 0, 1),
    ((8, 8, 8), 19, 0.8, 3, 0, 1),     # species
    ((8, 8, 8), 19, 0.8, 1, 7, 1),     # scheme
    ((8, 8, 8), 19, 0.8, 1, 0, 9),     # storage
    ((8, 8, 8), 19, 0.8, 1, 1, 2),     # population scheme stores F32/F64 only
    ((8, 8, 8), 19, 0.8, 1, 2, 3),     # in-place population scheme: F32/F64 only
    ((8, 8, 8), 19, 0.8, 2, 2, 1),     # in-place population scheme: one species
])
def test_create_rejects_bad_arguments_before_device(grid, q, tau, species, scheme, storage):
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    opts.scheme, opts.storage = scheme, storage
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(*grid), q, tau, species, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value


@pytest.mark.parametrize("species,scheme,split", [
    (1, 0, 2),     # split is 0 or 1
    (2, 1, 1),     # split approach: moment scheme only (two species too)
    (1, 1, 1),     # split approach: moment scheme only
    (1, 2, 1),
])
def test_create_rejects_bad_split_before_device(species, scheme, split):
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    assert opts.split == 0
    opts.scheme, opts.split = scheme, split
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(8, 8, 8), 19, 0.8, species, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value


@pytest.mark.parametrize("species,scheme,storage,split,sweep", [
    (1, 0, 1, 0, 3),     # 0, 1 or 2
    (1, 0, 1, 0, -1),
    (1, 0, 0, 0, 2),     # two-step sweeps: not with FP64 storage
    (2, 0, 1, 0, 2),     # one species only
    (1, 1, 1, 0, 2),     # moment scheme only
    (1, 0, 1, 1, 2),     # fused step only
])
def test_create_rejects_bad_sweep_before_device(species, scheme, storage, split, sweep):
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    assert opts.steps_per_sweep == 0
    opts.scheme, opts.storage, opts.split, opts.steps_per_sweep = scheme, storage, split, sweep
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(8, 8, 8), 19, 0.8, species, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value


@pytest.mark.parametrize("species,A,hmax", [
    (1, 0.01, 4),            # two species only
    (2, 0.01, 0),            # 1 <= nc_hmax <= 32
    (2, 0.01, 33),
    (2, float("nan"), 4),
])
def test_create_rejects_bad_near_contact_before_device(species, A, hmax):
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    assert opts.nc_A == 0.0 and opts.nc_hmax == 0
    opts.nc_A, opts.nc_hmax = A, hmax
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(8, 8, 8), 19, 0.8, species, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value


def test_create_rejects_near_contact_beyond_its_launch_grid():
    """The force passes launch one block row per z-plane: more than 65535
    planes is refused at creation, not at the first step."""
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    opts.nc_A, opts.nc_hmax = 0.01, 4
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(3, 3, 65536), 19, 0.8, 2, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value


def test_two_step_sweeps_need_planes_below_2_gib():
    """A stored xy-plane of 8192 x 8192 FP32 nodes (10 fields, 2.5 GiB) is
    beyond the sweep's buffer range: asking for two-step sweeps is refused
    before any device work (the default then runs single steps)."""
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    opts.steps_per_sweep = 2
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(8192, 8192, 3), 19, 0.8, 1, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value


def test_two_species_moment_contexts_need_planes_below_2_gib():
    """The two-component moment step addresses one stored xy-plane of its 11
    fields per buffer descriptor: 4096 x 4096 FP32 nodes (0.69 GiB) are
    accepted by the validation (without a GPU the create then fails for want
    of a device), 8192 x 8192 (2.75 GiB) are refused before any device work."""
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(8192, 8192, 3), 19, 0.8, 2, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(4096, 4096, 3), 19, 0.8, 2, ctypes.byref(opts))
    assert rc != _lib.LBM_EINVAL
    if rc == 0:  # a GPU is present
        lib.lbm_destroy(ctx)


@pytest.mark.parametrize("species,scheme,storage,s_pi", [
    (1, 0, 1, 2.0),      # FP32 storage keeps S unscaled: only 0 or 1
    (1, 0, 0, 1024.0),   # FP64 likewise
    (2, 0, 1, 4.0),      # two species likewise
    (1, 1, 1, 8.0),      # population scheme: no stored S
    (1, 0, 2, 1000.0),   # 16-bit storage: a power of two only
    (1, 0, 3, 0.75),
    (1, 0, 2, -1.0),
    (1, 0, 2, float("inf")),
])
def test_create_rejects_s_pi_where_not_applied(species, scheme, storage, s_pi):
    """The scale of the stored S is applied by the kernels only for one
    species with 16-bit moment storage; any other value elsewhere would be
    silently read as unscaled, so creation refuses it before device work."""
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    assert opts.s_pi == 0.0
    opts.scheme, opts.storage, opts.s_pi = scheme, storage, s_pi
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(8, 8, 8), 19, 0.8, species, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value


@pytest.mark.parametrize("grid,q,species,scheme,storage,expect", [
    # moment scheme: blocked layout, nx and ny rounded up to 64 and 16
    ((64, 16, 4), 27, 1, 0, 1, 64 * 16 * 4 * 10 * 4),
    ((37, 23, 19), 19, 1, 0, 1, 64 * 32 * 19 * 10 * 4),
    ((37, 23, 19), 19, 2, 0, 0, 64 * 32 * 19 * 11 * 8),
    ((130, 17, 5), 27, 1, 0, 2, 192 * 32 * 5 * 10 * 2),
    # population schemes: q (two species 2q) arrays of N values
    ((37, 23, 19), 27, 1, 1, 1, 27 * 37 * 23 * 19 * 4),
    ((37, 23, 19), 19, 2, 1, 1, 38 * 37 * 23 * 19 * 4),
    ((37, 23, 19), 19, 1, 2, 0, 19 * 37 * 23 * 19 * 8),
])
def test_state_bytes_for_without_a_context(grid, q, species, scheme, storage, expect):
    """lbm_state_bytes_for: the size of one state copy of a setup (the size
    caller-owned state buffers need), computed on the host."""
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    assert not opts.state_buffers[0] and not opts.state_buffers[1] and opts.state_buffer_bytes == 0
    opts.scheme, opts.storage = scheme, storage
    b = ctypes.c_int64(-1)
    assert lib.lbm_state_bytes_for(_lib.Grid(*grid), q, species, ctypes.byref(opts), ctypes.byref(b)) == _lib.LBM_OK
    assert b.value == expect
    # the same validation as lbm_create
    assert lib.lbm_state_bytes_for(_lib.Grid(2, 8, 8), q, species, ctypes.byref(opts), ctypes.byref(b)) == \
        _lib.LBM_EINVAL
    assert lib.lbm_state_bytes_for(_lib.Grid(*grid), q, species, ctypes.byref(opts), None) == _lib.LBM_EINVAL


@pytest.mark.parametrize("which", ["one_missing", "same_twice", "too_small"])
def test_create_rejects_bad_state_buffers_before_device(which):
    """Caller-owned state buffers: both or none, distinct, and each at least
    lbm_state_bytes_for() bytes; refused before any device work (the
    pointers are never dereferenced on this path)."""
    lib = _lib.load()
    opts = _lib.Opts()
    lib.lbm_default_opts(ctypes.byref(opts))
    need = ctypes.c_int64()
    assert lib.lbm_state_bytes_for(_lib.Grid(8, 8, 8), 19, 1, ctypes.byref(opts), ctypes.byref(need)) == 0
    opts.state_buffers[0] = 0x1000
    opts.state_buffers[1] = {"one_missing": 0, "same_twice": 0x1000, "too_small": 0x2000}[which]
    opts.state_buffer_bytes = need.value - (1 if which == "too_small" else 0)
    ctx = ctypes.c_void_p(123)
    rc = lib.lbm_create(ctypes.byref(ctx), _lib.Grid(8, 8, 8), 19, 0.8, 1, ctypes.byref(opts))
    assert rc == _lib.LBM_EINVAL
    assert not ctx.value
