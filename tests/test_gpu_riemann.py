"""The four-quadrant 2D Burgers problem of Sec. 5.4 on the GPU: the exterior
state on every boundary face is the exact solution in R^2 at the time of each
stage's input state (bc_kind RIEMANN).

Checked: one operator application at several times against the oracle
(<= 1e-12 relative L-inf), 100 steps of each SSP order from two start times
(<= 1e-11), the context's clock, the paths that take the constant exterior
state only refusing this one, and the paper's own size (128^2, P2, t = 0.5)
against the ranges of u_h printed for DG, LO and WENO
(tests/golden/burgers2d_riemann_ranges.json)."""
import json
import math
import os
import sys

import numpy as np
import pytest
import torch

from helpers import oracle_for, oracle_initial
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


def _state(w, O, seed, amp=0.01):
    U = oracle_initial(w, O)
    rng = np.random.default_rng(seed)
    return U + amp * torch.from_numpy(rng.standard_normal(U.shape)) * U.abs().max()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("mode", [inputs.MODE_DG, inputs.MODE_LO, inputs.MODE_WENO])
def test_rhs_parity_at_several_times(p, mode):
    """40^2 cells (2.5 tiles of 16 per side), a perturbed projection of the data."""
    _note(f"[riemann rhs] P{p} mode={mode}")
    w = inputs.burgers2d_riemann(40, p, mode=mode, steps=1)
    O = oracle_for(w)
    U = _state(w, O, 7)
    g = _dg().DG.from_workload(w)
    Ug = U.cuda().contiguous()
    for t in (0.0, 0.13, 0.37):
        ref, gref = O.rhs(U, with_gamma=True, t=t)
        g.set_time(t)
        got, gam = g.rhs(Ug, with_gamma=True)
        torch.cuda.synchronize()
        assert relinf(got.cpu(), ref) <= 1e-12, t
        assert (gam.cpu() - gref).abs().max() <= 1e-12


@pytest.mark.parametrize("k,t0", [(3, 0.0), (3, 0.2), (2, 0.1), (4, 0.0)])
def test_100_steps_parity(k, t0):
    _note(f"[riemann run] 40^2 P2 WENO, order {k}, from t = {t0}, 100 steps")
    w = inputs.burgers2d_riemann(40, 2, steps=100)
    w.rk_order = k
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    if t0 > 0.0:
        U0 = _state(w, O, 3)     # any state; the exterior state follows the clock
    ref = O.run(U0, w.dt(), 100, t0)
    g = _dg().DG.from_workload(w)
    assert not g.fused()
    g.set_time(t0)
    U = U0.cuda().contiguous()
    g.run(U, w.dt(), 60)
    for _ in range(40):
        g.step(U, w.dt())
    torch.cuda.synchronize()
    err = relinf(U.cpu(), ref)
    _note(f"    rel Linf = {err:.3e}")
    assert err <= 1e-11
    assert abs(g.time() - (t0 + 100 * w.dt())) <= 1e-15 * 100


def test_graph_replays_follow_the_clock():
    """dg_run replays captured graphs (64 steps, then the remainder) whose
    stages read their times from the context's device clock: two runs of 70
    steps (each one replay of the 64-step graph and one of 6) from t = 0.02
    against 140 oracle steps, and the clock after them."""
    _note("[riemann graphs] 40^2 P2 WENO, 2 x 70 steps from t = 0.02")
    w = inputs.burgers2d_riemann(40, 2, steps=140)
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    ref = O.run(U0, w.dt(), 140, 0.02)
    g = _dg().DG.from_workload(w)
    g.set_time(0.02)
    U = U0.cuda().contiguous()
    g.run(U, w.dt(), 70)
    g.run(U, w.dt(), 70)
    torch.cuda.synchronize()
    err = relinf(U.cpu(), ref)
    _note(f"    rel Linf = {err:.3e}")
    assert err <= 1e-11
    assert abs(g.time() - (0.02 + 140 * w.dt())) <= 1e-15 * 140


def test_refusals():
    dgweno = _dg()
    w = inputs.burgers2d_riemann(32, 2, steps=1)
    g = dgweno.DG.from_workload(w)
    U = g.initial_state(w)
    assert not g.fused()
    with pytest.raises(dgweno.DGError):
        g.set_fused(1)
    with pytest.raises(dgweno.DGError):
        g.rhs_vjp(U, U.clone())
    with pytest.raises(dgweno.DGError):
        g.step_adjoint(U, w.dt(), U.clone())
    with pytest.raises(dgweno.DGError):
        dgweno.Batch.from_workloads([w])


def test_papers_size_ranges_of_the_three_schemes():
    """128^2, P2, t = 0.5: u_h at the 3 x 3 Gauss points of every cell.  DG
    leaves the invariant set [-1, 0.8] (printed [-2.091, 1.691]); LO and WENO
    stay in it (printed [-1.000, 0.800] for both)."""
    dgweno = _dg()
    g_ = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "burgers2d_riemann_ranges.json")))
    lo0, hi0 = g_["invariant_set"]
    nodes = torch.tensor([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], dtype=torch.float64)
    P = torch.stack([torch.ones(3, dtype=torch.float64), nodes, 1.5 * nodes ** 2 - 0.5])   # P_a at the nodes
    V = torch.zeros(9, 9, dtype=torch.float64)
    for a in range(3):
        for b in range(3):
            for qx in range(3):
                for qy in range(3):
                    V[a + 3 * b, qx + 3 * qy] = P[a, qx] * P[b, qy]
    got = {}
    for mode, name in ((inputs.MODE_DG, "DG"), (inputs.MODE_LO, "LO"), (inputs.MODE_WENO, "WENO")):
        w = inputs.burgers2d_riemann(128, 2, mode=mode)
        dg = dgweno.DG.from_workload(w)
        U = dg.initial_state(w)
        n = int(math.ceil(0.5 / w.dt()))
        dg.run(U, 0.5 / n, n)
        torch.cuda.synchronize()
        assert abs(dg.time() - 0.5) < 1e-12
        assert dg.count_nonfinite(U) == 0
        vals = U.cpu() @ V
        got[name] = (float(vals.min()), float(vals.max()))
        _note(f"[burgers2d riemann 128^2 P2 t=0.5] {name}: u_h in [{got[name][0]:.4f}, {got[name][1]:.4f}] "
              f"(printed {g_['printed_range'][name]}), {n} steps")
    assert got["DG"][0] < lo0 - 0.2 and got["DG"][1] > hi0 + 0.2
    assert got["LO"][0] >= lo0 - 1e-3 and got["LO"][1] <= hi0 + 1e-3
    assert got["WENO"][0] >= lo0 - 1e-3 and got["WENO"][1] <= hi0 + 1e-3


@pytest.mark.parametrize("n,p", [(2, 1), (4, 3), (18, 2)])
def test_small_and_ragged_meshes(n, p):
    """2 x 2 cells (every cell on two boundaries), 4 x 4 P3 and 18 x 18 (one
    cell row past a 16 x 16 tile): 20 steps from t = 0.05 against the oracle."""
    _note(f"[riemann edge] {n}^2 P{p}")
    w = inputs.burgers2d_riemann(n, p, mode=inputs.MODE_WENO, steps=20)
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    ref = O.run(U0, w.dt(), 20, 0.05)
    g = _dg().DG.from_workload(w)
    g.set_time(0.05)
    U = U0.cuda().contiguous()
    g.run(U, w.dt(), 20)
    torch.cuda.synchronize()
    assert relinf(U.cpu(), ref) <= 1e-11


def test_papers_size_parity_20_steps():
    """The benchmark's four-quadrant workload (128^2, P2, WENO) from t = 0:
    20 steps of the whole mesh against the oracle."""
    _note("[riemann full size] 128^2 P2 WENO, 20 steps")
    w = inputs.burgers2d_riemann(128, 2, steps=20)
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    ref = O.run(U0, w.dt(), 20)
    g = _dg().DG.from_workload(w)
    U = U0.cuda().contiguous()
    g.run(U, w.dt(), 20)
    torch.cuda.synchronize()
    err = relinf(U.cpu(), ref)
    _note(f"    rel Linf = {err:.3e}")
    assert err <= 1e-11
