"""Work queued on a caller's stream other than the default one: graph-replayed
runs (fused and per-stage), one step and the step adjoint give the same bits
as on the default stream."""
import sys

import pytest
import torch

from paper_2309_12019_amd import inputs

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("fused", [-1, 0])
def test_side_stream_matches_default_stream(fused):
    from paper_2309_12019_amd import dgweno
    _note(f"[side stream] rot2d 64x64 P2, fused mode {fused}")
    w = inputs.rot2d(64, 2, seed=1, steps=20)
    g0 = dgweno.DG.from_workload(w)
    g0.set_fused(fused)
    U0 = g0.initial_state(w)
    ref = U0.clone()
    g0.run(ref, w.dt(), 20)
    g0.step(ref, w.dt())
    lam = torch.ones_like(U0) * 0.5
    ref_adj = g0.step_adjoint(ref, w.dt(), lam)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g1 = dgweno.DG.from_workload(w, stream=s)
        g1.set_fused(fused)
        U = U0.clone()
        g1.run(U, w.dt(), 20)
        g1.step(U, w.dt())
        adj = g1.step_adjoint(U, w.dt(), lam)
    s.synchronize()
    assert torch.equal(U, ref)
    assert torch.equal(adj, ref_adj)
