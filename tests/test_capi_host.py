"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/dgweno.h declares, and rejects invalid descriptors before any
device call (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgweno.h")
LIB = os.path.join(ROOT, "paper_2309_12019_amd", "libdgweno.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(dg_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdgweno.so is not built (python -m paper_2309_12019_amd.build)")
    from paper_2309_12019_amd import dgweno
    return dgweno.load(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("dg_init_mesh", "dg_project_ic", "dg_rhs", "dg_step", "dg_run"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2309_12019_amd import dgweno
    for name in declared():
        assert hasattr(lib, name), name
        assert name in dgweno.EXPORTS, name


def _desc(**kw):
    from paper_2309_12019_amd import dgweno
    d = dgweno.MeshDesc()
    dgweno.load().dg_default_desc(ctypes.byref(d))
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_default_desc(lib):
    d = _desc()
    assert (d.dim, d.nx, d.p, d.mode, d.q, d.b, d.w_nb, d.weno_eps, d.weno_pow, d.rk_order, d.bc_kind) == \
        (1, 64, 2, 2, 1.0, 0.0, 0.01, 1e-6, 2.0, 3, 0)


@pytest.mark.parametrize("bad", [
    dict(p=0), dict(p=5), dict(nx=0), dict(dim=3), dict(dim=2, ny=0),
    dict(dim=2, nx=4, ny=8),                  # non-square cells on the unit square
    dict(x1=0.0), dict(flux=7), dict(mode=9), dict(q=0.5), dict(b=1.5),
    dict(w_nb=0.6), dict(weno_eps=0.0), dict(weno_pow=-1.0), dict(lambda_override=-1.0),
    dict(vel_x=float("nan")), dict(rk_order=1), dict(rk_order=5), dict(zhao_theta=0.0),
    dict(bc_kind=2), dict(bc_kind=1, flux=1),                         # the exact exterior state is 2D
    dict(dim=2, nx=8, ny=8, flux=1, bc_kind=1),                       # ... on non-periodic boundaries
    dict(dim=2, nx=8, ny=8, flux=0, bc_kind=1, periodic_x=0, periodic_y=0),   # ... for Burgers
    dict(quad_vol=9), dict(quad_face=-1), dict(quad_proj=12), dict(cfl_mode=2), dict(check_finite=3),
    dict(device=-2),
])
def test_invalid_descriptors_rejected_on_host(lib, bad):
    d = _desc(**bad)
    h = ctypes.c_void_p(123)
    rc = lib.dg_init_mesh(ctypes.byref(d), ctypes.byref(h))
    assert rc == -1
    assert h.value is None
    assert len(lib.dg_last_error()) > 0


def test_batch_refuses_other_runge_kutta_orders_on_host(lib):
    """Batched runs implement the three-stage method only; the refusal comes
    from the host checks, before any device call."""
    from paper_2309_12019_amd import dgweno
    arr = (dgweno.MeshDesc * 2)(_desc(), _desc(rk_order=4))
    h = ctypes.c_void_p(123)
    rc = lib.dg_batch_create(arr, 2, ctypes.byref(h))
    assert rc == dgweno.DG_EUNSUPPORTED
    assert h.value is None
    assert "three-stage" in lib.dg_last_error().decode()


def test_null_arguments_rejected(lib):
    h = ctypes.c_void_p()
    assert lib.dg_init_mesh(None, ctypes.byref(h)) == -1
    assert lib.dg_rhs(None, None, None, None) == -1
    assert lib.dg_step(None, None, 0.1) == -1
    assert lib.dg_run(None, None, 0.1, 1) == -1
    assert lib.dg_project_ic(None, None, None) == -1
    assert lib.dg_sizes(None, None, None, None) == -1
    lib.dg_destroy(None)


@pytest.mark.parametrize("n,s", [(1, 0), (10, 0), (10, 2), (10, 9), (37, 3), (400, 20), (400, 400), (64, 6)])
def test_checkpoint_schedule_properties(lib, n, s):
    """Binomial checkpointing plan (host only): every step is reversed once, in
    order (checked inside the planner), no more than s slots are used, and
    enough slots remove all recomputation."""
    from paper_2309_12019_amd import dgweno
    st = dgweno.revolve_stats(n, s)
    assert st["adjoint_steps"] == n
    assert st["max_slot"] <= s
    assert st["forward_steps"] == (n - 1 if s > 0 else 0)
    if s >= n - 1:
        assert st["recomputed_steps"] == 0
    if s == 0:
        assert st["recomputed_steps"] == n * (n - 1) // 2


def test_checkpoint_recomputation_decreases_with_slots(lib):
    from paper_2309_12019_amd import dgweno
    rec = [dgweno.revolve_stats(200, s)["recomputed_steps"] for s in (1, 2, 4, 8, 16, 199)]
    assert all(a >= b for a, b in zip(rec, rec[1:])) and rec[-1] == 0
    # binomial bound: with s slots and t sweeps, C(s+t, s) steps are reversible
    # with at most t recomputations of each step
    assert dgweno.revolve_stats(200, 8)["recomputed_steps"] <= 3 * 200


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The product path has no CPU fallback: a missing library is an error."""
    from paper_2309_12019_amd import dgweno
    saved = dgweno._lib
    dgweno._lib = None
    try:
        with pytest.raises(ImportError):
            dgweno.load(str(tmp_path / "libdgweno_missing.so"))
    finally:
        dgweno._lib = saved


def test_product_code_does_not_import_the_oracle():
    """Only tests, the smoke check and the benchmark's CPU-baseline leg may
    use the oracle; the package itself never does."""
    pkg = os.path.join(ROOT, "paper_2309_12019_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            text = open(os.path.join(pkg, name)).read()
            assert not re.search(r"^\s*(import|from)\s+oracle", text, re.M), name


def test_static_step_checks_arguments_on_host(lib):
    """dg_step_static refuses bad arguments and problems beyond its static
    stage buffers (2^20 coefficients) before any device call."""
    U = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails on the host
    assert lib.dg_step_static(None, U, 0.1, 0.0) == -1
    assert lib.dg_step_static(ctypes.byref(_desc(p=0)), U, 0.1, 0.0) == -1
    assert lib.dg_step_static(ctypes.byref(_desc()), None, 0.1, 0.0) == -1
    assert lib.dg_step_static(ctypes.byref(_desc()), U, -0.1, 0.0) == -1
    assert lib.dg_step_static(ctypes.byref(_desc()), U, 0.1, float("inf")) == -1
    big = _desc(dim=2, nx=342, ny=342, p=2)          # 342^2 * 9 = 1,052,676 coefficients
    assert lib.dg_step_static(ctypes.byref(big), U, 0.1, 0.0) == -1
    assert b"exceed" in lib.dg_last_error()


@pytest.mark.parametrize("field,value", [("quad_vol", 5), ("quad_face", 2), ("quad_proj", 3)])
def test_quadrature_rules_that_are_not_built_are_refused_on_host(lib, field, value):
    """The rules are compile-time tables (p + 1 points for the linear flux of
    degree 2, projection p + 2): another count is valid but not built."""
    from paper_2309_12019_amd import dgweno
    d = _desc(**{field: value})
    h = ctypes.c_void_p(123)
    assert lib.dg_init_mesh(ctypes.byref(d), ctypes.byref(h)) == dgweno.DG_EUNSUPPORTED
    assert h.value is None
    assert b"not built" in lib.dg_last_error()


def test_built_quadrature_rules_named_explicitly_validate(lib):
    assert lib.dg_validate_desc(ctypes.byref(_desc(quad_vol=3, quad_face=3, quad_proj=4))) == 0
    assert lib.dg_validate_desc(ctypes.byref(_desc(dim=2, nx=8, ny=8, flux=1, quad_vol=4, quad_face=4))) == 0
    assert lib.dg_validate_desc(ctypes.byref(_desc(cfl_mode=1, check_finite=1, device=0))) == 0
