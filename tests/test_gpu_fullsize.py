"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (default tiles, fused stage kernel, graph-replayed runs).

The oracle cannot advance a 1024^2 mesh, so the comparisons are local: the
input state is the oracle's own L2 projection of the workload's initial data
plus a seeded perturbation of every coefficient (a generic, rough state that
switches the sensor on everywhere); the GPU applies the operator (dg_rhs) and
one SSP-RK3 step (dg_step) to the whole mesh, and at sampled cells the oracle
evaluates the same on a window of the input around the cell (radius 1 for the
operator, 3 for the step; the window oracle is pinned against the whole-mesh
oracle on small meshes).  Long GPU runs at full size are checked through
properties that hold at any size: finite values, gamma in [0, 1], and cell-mean
conservation on the periodic mesh.  The headline run (256^2 P2 rotation, 200
fused steps) is small enough for the oracle to follow whole."""
import sys

import numpy as np
import pytest
import torch

from helpers import oracle_for, oracle_initial, oracle_window
from paper_2309_12019_amd import inputs

pytestmark = pytest.mark.gpu

FULL = {
    "rot2d_256_p2": lambda: inputs.rot2d(256, 2, seed=0, steps=200),
    "rot2d_256_p3": lambda: inputs.rot2d(256, 3, seed=0, steps=200),
    "burgers2d_1024_p2": lambda: inputs.burgers2d(1024, 2, seed=0),
    "adv1d_64_p2": lambda: inputs.adv1d(64, 2, steps=100),
}


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dg():
    from paper_2309_12019_amd import dgweno
    return dgweno


def _samples(w, count, seed):
    """Seeded sample of cells: random cells plus the corners and edge midpoints."""
    rng = np.random.default_rng(seed)
    ny = w.ny if w.dim == 2 else 1
    pts = {(int(rng.integers(0, w.nx)), int(rng.integers(0, ny))) for _ in range(count)}
    for ix in (0, w.nx // 2, w.nx - 1):
        for iy in ((0, ny // 2, ny - 1) if w.dim == 2 else (0,)):
            pts.add((ix, iy))
    return sorted(pts)


def _input(w):
    O = oracle_for(w)
    U = oracle_initial(w, O)
    rng = np.random.default_rng(21)
    return U + 0.02 * torch.from_numpy(rng.standard_normal(U.shape)) * U.abs().max()


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_operator_and_step_at_sampled_cells(name):
    w = FULL[name]()
    _note(f"[full size] {name}: {w.ndof} DOFs, operator and one step at sampled cells")
    U = _input(w)
    g = _dg().DG.from_workload(w)
    Ud = U.cuda().contiguous()
    L, gam = g.rhs(Ud, with_gamma=True)
    S = Ud.clone()
    g.step(S, w.dt())
    torch.cuda.synchronize()
    L, gam, S = L.cpu(), gam.cpu(), S.cpu()
    Lscale, Sscale = float(L.abs().max()), float(S.abs().max())
    worst_L = worst_S = worst_g = 0.0
    for k, (ix, iy) in enumerate(_samples(w, 40, 5)):
        e = iy * w.nx + ix
        Ow, idx, c = oracle_window(w, ix, iy, 1)
        Lw, gw = Ow.rhs(U[idx], with_gamma=True)
        worst_L = max(worst_L, float((L[e] - Lw[c]).abs().max()) / Lscale)
        worst_g = max(worst_g, abs(float(gam[e] - gw[c])))
        if k % 2 == 0:
            Ow, idx, c = oracle_window(w, ix, iy, 3)
            Sw = Ow.step(U[idx], w.dt())
            worst_S = max(worst_S, float((S[e] - Sw[c]).abs().max()) / Sscale)
    _note(f"    operator {worst_L:.2e}, gamma {worst_g:.2e}, step {worst_S:.2e}")
    assert worst_L <= 1e-12 and worst_g <= 1e-12 and worst_S <= 1e-13


@pytest.mark.parametrize("name", ["burgers2d_1024_p2", "rot2d_256_p3"])
def test_full_size_run_invariants(name):
    """Whole workload runs on the GPU (Burgers: to 1.5 shock times): values
    stay finite, gamma stays in [0, 1], and on the periodic mesh the sum of
    cell means is conserved to rounding."""
    w = FULL[name]()
    _note(f"[full size] {name}: {w.steps} steps, invariants")
    g = _dg().DG.from_workload(w)
    U = g.initial_state(w)
    m0 = float(U[:, 0].sum())
    g.run(U, w.dt(), w.steps)
    _, gam = g.rhs(U, with_gamma=True)
    torch.cuda.synchronize()
    assert g.count_nonfinite(U) == 0
    assert float(gam.min()) >= 0.0 and float(gam.max()) <= 1.0
    m1 = float(U[:, 0].sum())
    scale = float(U[:, 0].abs().sum())
    if w.periodic_x and w.periodic_y:
        assert abs(m1 - m0) <= 1e-12 * scale
    else:
        # rotation with zero inflow: the data stay away from the boundary
        assert abs(m1 - m0) <= 1e-10 * scale


def test_full_size_adjoint_at_sampled_cells():
    """The adjoint at the adjoint benchmark's size (512^2 P2 Burgers, 32x8
    adjoint tiles, pass B sharing launches with pass A): J^T v of the operator
    and the adjoint of one SSP-RK3 step on the whole mesh, against the oracle's
    reverse mode on windows around sampled cells.  (J^T v)_e involves the
    operator on the face neighbours of e, each of which depends on its own face
    neighbours: a window of radius 2.  The step adjoint at e involves the step
    on cells within three face steps of e, each depending on cells within
    three more: radius 6."""
    w = inputs.burgers2d(512, 2, seed=0, steps=400)
    _note(f"[full size] adjoint burgers2d 512x512 p2: {w.ndof} DOFs, sampled cells")
    U = _input(w)
    rng = np.random.default_rng(33)
    v = torch.from_numpy(rng.standard_normal(U.shape))
    lam = torch.from_numpy(rng.standard_normal(U.shape))
    g = _dg().DG.from_workload(w)
    JTv = g.rhs_vjp(U.cuda().contiguous(), v.cuda().contiguous())
    lin = g.step_adjoint(U.cuda().contiguous(), w.dt(), lam.cuda().contiguous())
    torch.cuda.synchronize()
    JTv, lin = JTv.cpu(), lin.cpu()
    sJ, sS = float(JTv.abs().max()), float(lin.abs().max())
    worst_J = worst_S = 0.0
    for k, (ix, iy) in enumerate(_samples(w, 10, 8)):
        e = iy * w.nx + ix
        Ow, idx, c = oracle_window(w, ix, iy, 2)
        Ur = U[idx].clone().requires_grad_(True)
        (ref,) = torch.autograd.grad(Ow.rhs(Ur), Ur, v[idx])
        worst_J = max(worst_J, float((JTv[e] - ref[c]).abs().max()) / sJ)
        if k % 3 == 0:
            Ow, idx, c = oracle_window(w, ix, iy, 6)
            ref = Ow.step_vjp(U[idx], w.dt(), lam[idx])
            worst_S = max(worst_S, float((lin[e] - ref[c]).abs().max()) / sS)
    _note(f"    J^T v {worst_J:.2e}, step adjoint {worst_S:.2e}")
    assert worst_J <= 1e-11 and worst_S <= 1e-11


def test_headline_run_against_the_oracle_whole_mesh():
    """The headline benchmark run itself: 256^2 P2 rotation, 200 steps, the
    library's automatic path (the fused step kernel, graph replay), compared
    on the whole mesh with 200 oracle steps (about 40 s of host time)."""
    _note("[full size] rot2d_256_p2: 200 fused steps vs 200 oracle steps, whole mesh")
    w = FULL["rot2d_256_p2"]()
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    g = _dg().DG.from_workload(w)
    assert g.fused() and g.tile() == (16, 16)
    U = U0.cuda().contiguous()
    g.run(U, w.dt(), w.steps)
    torch.cuda.synchronize()
    ref = U0
    for k in range(w.steps):
        ref = O.step(ref, w.dt())
        if (k + 1) % 50 == 0:
            _note(f"    oracle step {k + 1}")
    err = float((U.cpu() - ref).abs().max() / ref.abs().max())
    _note(f"    rel Linf = {err:.3e}")
    assert err <= 1e-11
