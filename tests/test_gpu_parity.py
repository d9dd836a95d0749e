"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Single-operator checks use meshes that span several workgroup tiles with a
ragged edge; run checks follow the SSP-RK3 step for 100 steps.  Tolerances:
one application of the operator <= 1e-12 relative L-inf (a few rounding
errors per term), 100 steps <= 1e-11 relative L-inf.
"""
import math
import sys

import numpy as np
import pytest
import torch

from helpers import SPREAD_CAP, oracle_for, oracle_initial, oracle_problem, run_bar
from paper_2309_12019_amd import inputs

pytestmark = pytest.mark.gpu


def _dg():
    from paper_2309_12019_amd import dgweno
    return dgweno


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def relinf(a, b):
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


def _mesh(kind, p, mode, n1=600, n2=(40, 36)):
    if kind == "adv1d":
        w = inputs.adv1d(n1, p, mode=mode)
    elif kind == "burgers1d":
        w = inputs.burgers1d(n1, p, mode=mode)
    elif kind == "rot2d":
        w = inputs.rot2d(n2[0], p, mode=mode, ny=n2[1])
        w.cy = 0.45  # keeps v.n single-signed on every face (y = 0.45 is a grid line)
    elif kind == "burgers2d":
        w = inputs.burgers2d(n2[0], p, mode=mode, ny=n2[1], steps=1)
    elif kind == "kpp2d":
        w = inputs.kpp2d(n2[0], p, mode=mode, steps=1, lam=0.0)   # lambda_e from F' (= 1)
    else:
        raise ValueError(kind)
    return w


def _state(w, O, seed):
    U = oracle_initial(w, O)
    rng = np.random.default_rng(seed)
    return U + 0.01 * torch.from_numpy(rng.standard_normal(U.shape)) * U.abs().max()


KINDS = ["adv1d", "burgers1d", "rot2d", "burgers2d", "kpp2d"]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_rhs_parity(kind, p, mode):
    _note(f"[rhs parity] {kind} p={p} mode={mode}")
    w = _mesh(kind, p, mode)
    O = oracle_for(w)
    U = _state(w, O, 11)
    Lo, go = O.rhs(U, with_gamma=True)
    g = _dg().DG.from_workload(w)
    Ud = U.cuda().contiguous()
    Lg, gg = g.rhs(Ud, with_gamma=True)
    torch.cuda.synchronize()
    assert relinf(Lg.cpu(), Lo) <= 1e-12
    assert float((gg.cpu() - go).abs().max()) <= 1e-12


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_projection_parity(kind, p):
    _note(f"[projection parity] {kind} p={p}")
    w = _mesh(kind, p, 2)
    w.ic = (lambda x: np.exp(np.sin(2 * np.pi * x))) if w.dim == 1 else \
        (lambda x, y: np.cos(3 * x - 2 * y) + x * y)
    O = oracle_for(w)
    Uo = oracle_initial(w, O)
    g = _dg().DG.from_workload(w)
    Ug = g.initial_state(w)
    torch.cuda.synchronize()
    assert relinf(Ug.cpu(), Uo) <= 1e-13


def _run_parity(w, U0, steps, tol=1e-11, O=None):
    """100-step parity at the bar of helpers.run_bar (1e-11 relative L-inf;
    for p = 4 WENO 10x the oracle's own one-ulp spread where larger, capped
    at helpers.SPREAD_CAP)."""
    O = O or oracle_for(w)
    ref = O.run(U0, w.dt(), steps)
    g = _dg().DG.from_workload(w)
    U = U0.cuda().contiguous()
    g.run(U, w.dt(), steps)
    torch.cuda.synchronize()
    err = relinf(U.cpu(), ref)
    bar, spread = run_bar(w, lambda V: O.run(V, w.dt(), steps), U0, ref=ref)
    bar = max(bar, tol)
    if spread is not None:
        _note(f"    oracle one-ulp spread = {spread:.3e}")
    _note(f"    rel Linf after {steps} steps = {err:.3e} (bar {bar:.1e})")
    assert err <= bar and bar <= SPREAD_CAP
    return U, ref


def test_config_1d_advection_100_steps():
    """1D u_t + u_x = 0, 64 cells, P2, sin(2 pi x) + square pulse, WENO, CFL 0.1."""
    _note("[run parity] adv1d 64 cells P2 WENO 100 steps")
    w = inputs.adv1d(64, 2, steps=100)
    O = oracle_for(w)
    _run_parity(w, oracle_initial(w, O), 100, O=O)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("kind", ["adv1d", "burgers1d"])
def test_1d_100_steps_ragged(kind, p):
    _note(f"[run parity] {kind} 300 cells P{p} WENO 100 steps")
    w = inputs.adv1d(300, p) if kind == "adv1d" else inputs.burgers1d(300, p)
    O = oracle_for(w)
    _run_parity(w, oracle_initial(w, O), 100, O=O)


@pytest.mark.parametrize("p", [2, 3])
def test_rotation_100_steps(p):
    """Solid-body rotation (hump + slotted cylinder), 48 x 40 cells, P2/P3."""
    _note(f"[run parity] rot2d 48x40 P{p} WENO 100 steps")
    w = inputs.rot2d(48, p, seed=3, ny=40)
    w.cy = 0.5  # 0.5 = 20 h is a grid line
    O = oracle_for(w)
    _run_parity(w, oracle_initial(w, O), 100, O=O)


@pytest.mark.parametrize("kind,p", [("adv1d", 3), ("rot2d", 2), ("burgers2d", 2)])
def test_zhao_sensor_100_steps(kind, p):
    """The sensor of Zhao et al. (Sec. 5.6) in place of eq. (sensor): 100 steps,
    including non-periodic boundaries (rotation) where m_e < 2d."""
    _note(f"[run parity] {kind} P{p} Zhao sensor, 100 steps")
    if kind == "adv1d":
        w = inputs.adv1d(300, p, mode=inputs.MODE_ZHAO)
    elif kind == "rot2d":
        w = inputs.rot2d(48, p, seed=3, ny=40, mode=inputs.MODE_ZHAO)
        w.cy = 0.5
    else:
        w = inputs.burgers2d(40, p, seed=0, mode=inputs.MODE_ZHAO)
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    if kind == "burgers2d":
        U0 = O.run(U0, w.dt(), w.steps)   # past the shock time, on the oracle
    _run_parity(w, U0, 100, O=O)


@pytest.mark.parametrize("mode", [inputs.MODE_LO, inputs.MODE_WENO])
def test_kpp_100_steps(mode):
    """The KPP flux of Sec. 5.5 (non-convex, sin/cos), 40 x 40 cells, P2,
    lambda_e = 2 as in the paper, 100 steps from the disc data (shocks and
    rarefactions from the first step)."""
    _note(f"[run parity] kpp2d 40x40 P2 mode={mode}, 100 steps")
    w = inputs.kpp2d(40, 2, mode=mode, steps=100)
    O = oracle_for(w)
    _run_parity(w, oracle_initial(w, O), 100, O=O)


@pytest.mark.parametrize("n", [37, 136, 184])
def test_kpp_split_kernel_at_each_wave_count(n):
    """The KPP kernel of 8x8 tiles runs 16, 8 or 4 waves per tile by the
    number of tiles per compute unit: 37^2 (25 ragged tiles), 136^2 (289 tiles,
    between one and two per compute unit on 256) and 184^2 (529 tiles).  At
    each size, p = 2 WENO: 3 steps and one operator bitwise equal on 8x8 and
    16x16 tiles, and the 8x8 operator against the oracle on the ragged mesh."""
    dgweno = _dg()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    tiles = ((n + 7) // 8) ** 2
    waves = 16 if tiles <= cus else 8 if tiles <= 2 * cus else 4
    _note(f"[kpp split] {n}^2 P2 WENO: {tiles} tiles of 8x8 on {cus} CUs -> {waves} waves per tile")
    w = inputs.kpp2d(n, 2, steps=3)
    g = dgweno.DG.from_workload(w)
    U0 = g.initial_state(w)
    gen = torch.Generator(device=U0.device).manual_seed(5)
    U0 = U0 + 0.02 * U0.abs().max() * torch.randn(U0.shape, generator=gen, device=U0.device, dtype=U0.dtype)
    outs = []
    for tile in ((8, 8), (16, 16)):
        g.set_tile(*tile)
        U = U0.clone()
        g.run(U, w.dt(), 3)
        L, gam = g.rhs(U0, with_gamma=True)
        outs.append((U, L, gam))
    torch.cuda.synchronize()
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    if n == 37:
        O = oracle_for(w)
        Lo, go = O.rhs(U0.cpu(), with_gamma=True)
        assert relinf(outs[0][1].cpu(), Lo) <= 1e-12
        assert float((outs[0][2].cpu() - go).abs().max()) <= 1e-12


def test_kpp_has_no_adjoint():
    dgweno = _dg()
    w = inputs.kpp2d(16, 2, steps=1)
    g = dgweno.DG.from_workload(w)
    U = g.initial_state(w)
    with pytest.raises(dgweno.DGError):
        g.rhs_vjp(U, U.clone())


def test_zhao_sensor_has_no_adjoint():
    dgweno = _dg()
    w = inputs.burgers2d(16, 2, mode=inputs.MODE_ZHAO, steps=1)
    g = dgweno.DG.from_workload(w)
    U = g.initial_state(w)
    with pytest.raises(dgweno.DGError):
        g.rhs_vjp(U, U.clone())
    with pytest.raises(dgweno.DGError):
        g.step_adjoint(U, w.dt(), U.clone())


def test_burgers2d_100_steps_after_shock():
    """2D Burgers with seeded Fourier data: the oracle first runs past the shock
    time, then both sides advance 100 steps from that state."""
    _note("[run parity] burgers2d 40x40 P2 WENO, 100 steps from a post-shock state")
    w = inputs.burgers2d(40, 2, seed=0)
    O = oracle_for(w)
    U0 = O.run(oracle_initial(w, O), w.dt(), w.steps)
    _run_parity(w, U0, 100, O=O)


@pytest.mark.parametrize("per", [(False, False), (True, False), (False, True)])
def test_burgers2d_shared_faces_at_constant_exterior_state(per):
    """2D P2 Burgers (the kernel that evaluates each face of a 16x16 tile
    once) on a ragged 37 x 29 mesh with a constant exterior state 0.3 on the
    non-periodic sides: 30 steps against the oracle, and bitwise the same as
    the 8x8 tile (per-cell faces) and the fused step kernel."""
    _note(f"[shared faces] burgers2d 37x29 P2, periodic {per}")
    w = inputs.burgers2d(37, 2, seed=4, ny=29, steps=30)
    w.periodic_x, w.periodic_y = per
    w.bc_value = 0.3
    O = oracle_for(w)
    U0 = _state(w, O, 11)
    ref = O.run(U0, w.dt(), 30)
    outs = []
    for tile, fused in (((16, 16), 0), ((8, 8), 0), (None, 1)):
        g = _dg().DG.from_workload(w)
        g.set_fused(fused)
        if tile:
            g.set_tile(*tile)
        U = U0.cuda().contiguous()
        g.run(U, w.dt(), 30)
        torch.cuda.synchronize()
        outs.append(U.cpu())
    err = relinf(outs[0], ref)
    _note(f"    rel Linf {err:.3e}")
    assert err <= 1e-11
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_run_equals_repeated_step_bitwise():
    _note("[determinism] dg_run vs dg_step")
    w = inputs.rot2d(40, 2, ny=36)
    g = _dg().DG.from_workload(w)
    U0 = g.initial_state(w)
    A = U0.clone()
    B = U0.clone()
    g.run(A, w.dt(), 70)          # one 64-step graph + 6 eager steps
    for _ in range(70):
        g.step(B, w.dt())
    torch.cuda.synchronize()
    assert torch.equal(A, B)
    C = U0.clone()
    g.run(C, w.dt(), 70)
    torch.cuda.synchronize()
    assert torch.equal(A, C)


@pytest.mark.parametrize("kind", ["rot2d", "burgers2d", "kpp2d", "adv1d"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tile_shape_independence(kind, p):
    """Per-cell arithmetic does not depend on the workgroup tile (one-wave 8x8
    and 64-cell tiles included; for the KPP flux the 8x8 tile is the kernel of
    four waves that evaluates the node fluxes apart from the cells), on a
    rough state that switches the sensor on and, for the rotation, with faces
    on which v.n changes sign (the centre of rotation off the grid lines),
    where the LLF flux takes the quadrature branch."""
    _note(f"[tiles] {kind} p={p}")
    w = _mesh(kind, p, 2, n1=1000, n2=(72, 40))
    if kind == "rot2d":
        w.cy = 0.4537
    g = _dg().DG.from_workload(w)
    g.set_fused(0)
    U0 = g.initial_state(w)
    gen = torch.Generator(device=U0.device).manual_seed(3)
    U0 = U0 + 0.02 * U0.abs().max() * torch.randn(U0.shape, generator=gen, device=U0.device, dtype=U0.dtype)
    outs = []
    tiles = [(256, 1), (64, 1)] if w.dim == 1 else [(16, 16), (8, 8)]
    for tx, ty in tiles:
        g.set_tile(tx, ty)
        for _ in range(2):
            U = U0.clone()
            g.run(U, w.dt(), 5)
            L = g.rhs(U)
            outs.append((U, L))
    torch.cuda.synchronize()
    for U, L in outs[1:]:
        assert torch.equal(U, outs[0][0]) and torch.equal(L, outs[0][1])


@pytest.mark.parametrize("kind", ["rot2d", "burgers2d"])
def test_one_wave_and_four_wave_tiles_at_a_larger_mesh(kind):
    """232^2 cells: 841 8x8 tiles, more than three per compute unit on 256,
    so 8x8 runs the one-wave tile kernel there (small meshes take the
    four-wave tile); 3 steps and one operator on 8x8 and 16x16 tiles, P2
    WENO on a rough state, bitwise equal."""
    _note(f"[tiles 232^2] {kind}")
    w = _mesh(kind, 2, 2, n2=(232, 232))
    if kind == "rot2d":
        w.cy = 0.4537
    g = _dg().DG.from_workload(w)
    g.set_fused(0)
    U0 = g.initial_state(w)
    gen = torch.Generator(device=U0.device).manual_seed(9)
    U0 = U0 + 0.02 * U0.abs().max() * torch.randn(U0.shape, generator=gen, device=U0.device, dtype=U0.dtype)
    outs = []
    for tile in ((8, 8), (16, 16)):
        g.set_tile(*tile)
        U = U0.clone()
        g.run(U, w.dt(), 3)
        outs.append((U, g.rhs(U0)))
    torch.cuda.synchronize()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_stable_dt_and_finite_check():
    _note("[stable dt]")
    w = inputs.burgers2d(48, 2, ny=40, steps=1)
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    g = _dg().DG.from_workload(w)
    U = U0.cuda().contiguous()
    dt = g.stable_dt(U, 0.1)
    lam = float(O.max_speed(U0).max())
    assert abs(dt - 0.1 * w.h / (5 * lam)) <= 1e-13 * dt
    assert g.count_nonfinite(U) == 0
    U[3, 2] = float("nan")
    U[7, 0] = float("inf")
    assert g.count_nonfinite(U) == 2


def test_run_reports_non_finite_states_with_check_finite():
    """check_finite: dg_run and dg_step count the non-finite entries of U once
    their steps are queued and return DG_ENONFINITE if there are any."""
    _note("[check_finite]")
    dgweno = _dg()
    w = inputs.burgers2d(40, 2, ny=36, steps=1)
    d = dgweno.desc_from_fields(w.fields())
    d.check_finite = 1
    g = dgweno.DG(d)
    U = g.initial_state(w)
    g.run(U, w.dt(), 3)            # finite: no error
    g.step(U, w.dt())
    U[5, 1] = float("nan")
    with pytest.raises(dgweno.DGError) as ex:
        g.run(U, w.dt(), 2)
    assert ex.value.code == dgweno.DG_ENONFINITE
    U[:] = 0.0
    U[7, 0] = float("inf")
    with pytest.raises(dgweno.DGError) as ex:
        g.step(U, w.dt())
    assert ex.value.code == dgweno.DG_ENONFINITE
    # without the flag the same run returns normally (the caller checks)
    g2 = dgweno.DG.from_workload(w)
    U2 = g2.initial_state(w)
    U2[5, 1] = float("nan")
    g2.run(U2, w.dt(), 2)
    torch.cuda.synchronize()
    assert g2.count_nonfinite(U2) > 0


def test_cfl_mode_and_named_quadrature_rules():
    """cfl_mode 1 (literal) gives (2p + 1) times the scaled step; naming the
    built quadrature rules explicitly changes nothing (bitwise)."""
    _note("[cfl_mode, quadrature fields]")
    dgweno = _dg()
    w = inputs.burgers2d(48, 2, ny=40, steps=1)
    d0 = dgweno.desc_from_fields(w.fields())
    d1 = dgweno.desc_from_fields(w.fields())
    d1.cfl_mode = 1
    d1.quad_vol, d1.quad_face, d1.quad_proj = 4, 4, 4
    g0, g1 = dgweno.DG(d0), dgweno.DG(d1)
    U0 = g0.initial_state(w)
    U1 = g1.initial_state(w)
    assert torch.equal(U0, U1)
    dt0, dt1 = g0.stable_dt(U0, 0.1), g1.stable_dt(U1, 0.1)
    assert abs(dt1 - 5 * dt0) <= 1e-15 * dt1
    g0.run(U0, dt0, 5)
    g1.run(U1, dt0, 5)
    torch.cuda.synchronize()
    assert torch.equal(U0, U1)


def test_invalid_arguments_through_the_binding():
    dgweno = _dg()
    w = inputs.adv1d(64, 2)
    g = dgweno.DG.from_workload(w)
    U = g.initial_state(w)
    with pytest.raises(dgweno.DGError):
        g.step(U, -1.0)
    with pytest.raises(dgweno.DGError):
        g.run(U, float("nan"), 3)
    with pytest.raises(dgweno.DGError):
        g.set_tile(100, 1)
    with pytest.raises(dgweno.DGError):
        g.set_tile(128, 1)
    with pytest.raises(ValueError):
        g.rhs(U.float())
