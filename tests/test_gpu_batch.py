"""Batched execution (dg_batch_*): every problem of a mixed batch must advance
exactly as it does alone (same per-cell arithmetic), whatever the schedule."""
import sys

import numpy as np
import pytest
import torch

from helpers import oracle_for, oracle_initial
from paper_2309_12019_amd import inputs

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dg():
    from paper_2309_12019_amd import dgweno
    return dgweno


def small_mix(seed=3, count=30, steps=8):
    """A seeded mix of the batch workload's problem types with sizes capped so
    the test is quick (1D up to 700 cells, 2D up to 40 x 40)."""
    ws = inputs.batch_mix(seed, count=count, steps=steps)
    for w in ws:
        if w.dim == 1:
            w.nx = min(w.nx, 700)
        else:
            n = min(w.nx, 40)
            w.nx = w.ny = n
            w.y1 = 1.0
    return ws


def _initial(ws, B, arena):
    dgweno = _dg()
    for w, v in zip(ws, B.views(arena)):
        g = dgweno.DG.from_workload(w)
        v.copy_(g.initial_state(w))
        g.close()
    torch.cuda.synchronize()


def _alone(ws, U0s, nsteps):
    dgweno = _dg()
    out = []
    for w, U0 in zip(ws, U0s):
        g = dgweno.DG.from_workload(w)
        U = U0.clone()
        g.run(U, w.dt(), nsteps)
        out.append(U)
    torch.cuda.synchronize()
    return out


def test_batch_equals_single_problem_runs():
    _note("[batch] mixed batch vs single-problem runs")
    ws = small_mix()
    B = _dg().Batch.from_workloads(ws)
    assert B.num_classes() > 4
    arena = B.empty()
    _initial(ws, B, arena)
    U0s = [v.clone() for v in B.views(arena)]
    dts = [w.dt() for w in ws]
    B.run(arena, dts, 8)
    torch.cuda.synchronize()
    ref = _alone(ws, U0s, 8)
    for w, v, r in zip(ws, B.views(arena), ref):
        assert torch.equal(v, r), w.name


def test_batch_schedule_and_tuner_do_not_change_results():
    _note("[batch] schedules")
    ws = small_mix(seed=5, count=20, steps=4)
    dgweno = _dg()
    B = dgweno.Batch.from_workloads(ws)
    arena = B.empty()
    _initial(ws, B, arena)
    U0 = arena.clone()
    dts = [w.dt() for w in ws]
    B.run(arena, dts, 4)
    torch.cuda.synchronize()
    ref = arena.clone()
    results = []
    for c in range(B.num_classes()):
        s = B.schedule(c)
        if s["dim"] == 1:
            B.set_schedule(c, 64, 1, 1, 2)
        else:
            B.set_schedule(c, 8, 8, 4, 1)
    for nb in (1, 3):
        B.set_branches(nb)
        arena.copy_(U0)
        B.run(arena, dts, 4)
        torch.cuda.synchronize()
        results.append(arena.clone())
    report = B.tune(U0.clone(), dts, reps=2)
    assert "class" in report and "branches" in report
    arena.copy_(U0)
    B.run(arena, dts, 4)
    torch.cuda.synchronize()
    results.append(arena.clone())
    arena.copy_(U0)
    B.run_sequential(arena, dts, 4)
    torch.cuda.synchronize()
    results.append(arena.clone())
    for r in results:
        assert torch.equal(r, ref)


@pytest.mark.parametrize("kind,p", [("adv1d", 3), ("burgers1d", 2), ("rot2d", 2)])
def test_batch_members_match_the_oracle(kind, p):
    _note(f"[batch] {kind} p={p} vs oracle inside a batch")
    if kind == "adv1d":
        target = inputs.adv1d(300, p, steps=20)
    elif kind == "burgers1d":
        target = inputs.burgers1d(257, p, steps=20)
    else:
        target = inputs.rot2d(40, p, seed=2, steps=20)
    ws = small_mix(seed=7, count=10, steps=20) + [target]
    B = _dg().Batch.from_workloads(ws)
    arena = B.empty()
    _initial(ws[:-1], B, arena)
    O = oracle_for(target)
    U0 = oracle_initial(target, O)
    B.views(arena)[-1].copy_(U0.cuda())
    B.run(arena, [w.dt() for w in ws], 20)
    torch.cuda.synchronize()
    ref = O.run(U0, target.dt(), 20)
    got = B.views(arena)[-1].cpu()
    assert float((got - ref).abs().max() / ref.abs().max()) <= 1e-11


def test_batch_argument_errors():
    dgweno = _dg()
    ws = small_mix(count=4)
    B = dgweno.Batch.from_workloads(ws)
    arena = B.empty()
    with pytest.raises(dgweno.DGError):
        B.run(arena, [0.0] * len(ws), 1)
    with pytest.raises(ValueError):
        B.run(arena, [1e-3] * (len(ws) + 1), 1)
    with pytest.raises(dgweno.DGError):
        B.set_schedule(0, 100, 1, 1, 0)
    with pytest.raises(dgweno.DGError):
        B.set_schedule(B.num_classes(), 256, 1, 1, 0)
    with pytest.raises(dgweno.DGError):
        B.set_branches(5)
    bad = dgweno.desc_from_fields(ws[0].fields())
    bad.p = 7
    with pytest.raises(dgweno.DGError):
        dgweno.Batch([bad])


@pytest.mark.parametrize("p", [2, 3, 4])
def test_batch_one_wave_tiles_match_single_runs(p):
    """2D rotation problems of one degree in a batch on 8x8 tiles (one wave
    per workgroup) advance exactly as alone, with
    the rotation centre off the grid lines (faces where v.n changes sign) and
    a rough state; the batch runs twice (a run-to-run difference would show a
    race or a stale register)."""
    _note(f"[batch] one-wave tiles p={p}")
    dgweno = _dg()
    ws = []
    for i, n in enumerate((40, 34, 23, 17)):
        w = inputs.rot2d(n, p, seed=11 + i, steps=4)
        w.cy = 0.4537
        ws.append(w)
    B = dgweno.Batch.from_workloads(ws)
    arena = B.empty()
    _initial(ws, B, arena)
    gen = torch.Generator(device=arena.device).manual_seed(5)
    arena += 0.02 * torch.randn(arena.shape, generator=gen, device=arena.device, dtype=arena.dtype)
    U0 = arena.clone()
    singles = []
    for w, v in zip(ws, B.views(U0)):
        g = dgweno.DG.from_workload(w)
        g.set_fused(0)
        U = v.clone()
        g.run(U, w.dt(), 4)
        singles.append(U)
    B.set_schedule(0, 8, 8, 1, 0)
    dts = [w.dt() for w in ws]
    for _ in range(2):
        arena.copy_(U0)
        B.run(arena, dts, 4)
        torch.cuda.synchronize()
        for w, v, r in zip(ws, B.views(arena), singles):
            assert torch.equal(v, r), w.name
