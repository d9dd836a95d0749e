"""Sec. 5.3 as printed: LeVeque's solid-body rotation with v = 2 pi (0.5 - y,
x - 0.5), a hump, a cone and a slotted cylinder, 128^2 cells, P2, one
revolution (t = 1).  The paper prints the range of u_h for DG, LO and WENO
(tests/golden/leveque_ranges.json); 100-step parity with the oracle first,
on a 40^2 mesh of the same problem."""
import json
import math
import os
import sys

import pytest
import torch

from helpers import oracle_for, oracle_initial
from paper_2309_12019_amd import inputs

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", [inputs.MODE_LO, inputs.MODE_WENO])
def test_100_steps_parity(mode):
    from paper_2309_12019_amd import dgweno
    _note(f"[leveque parity] 40^2 P2 mode={mode}")
    w = inputs.leveque2d(40, 2, mode=mode, steps=100)
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    ref = O.run(U0, w.dt(), 100)
    g = dgweno.DG.from_workload(w)
    U = U0.cuda().contiguous()
    g.run(U, w.dt(), 100)
    torch.cuda.synchronize()
    err = float((U.cpu() - ref).abs().max() / ref.abs().max())
    _note(f"    rel Linf = {err:.3e}")
    assert err <= 1e-11


def test_one_revolution_ranges_of_the_three_schemes():
    """DG over- and undershoots the data range [0, 1] (printed [-0.107,
    1.120]); LO stays in it and flattens the bodies (printed [0, 0.690]);
    WENO stays in it and keeps the peaks (printed [0, 1.000]).  u_h at the
    3 x 3 Gauss points of every cell."""
    from paper_2309_12019_amd import dgweno
    g_ = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "leveque_ranges.json")))
    nodes = torch.tensor([-math.sqrt(3 / 5), 0.0, math.sqrt(3 / 5)], dtype=torch.float64)
    P = torch.stack([torch.ones(3, dtype=torch.float64), nodes, 1.5 * nodes ** 2 - 0.5])
    V = torch.zeros(9, 9, dtype=torch.float64)
    for a in range(3):
        for b in range(3):
            for qx in range(3):
                for qy in range(3):
                    V[a + 3 * b, qx + 3 * qy] = P[a, qx] * P[b, qy]
    got = {}
    for mode, name in ((inputs.MODE_DG, "DG"), (inputs.MODE_LO, "LO"), (inputs.MODE_WENO, "WENO")):
        w = inputs.leveque2d(128, 2, mode=mode)
        g = dgweno.DG.from_workload(w)
        U = g.initial_state(w)
        n = int(math.ceil(1.0 / w.dt()))
        g.run(U, 1.0 / n, n)
        torch.cuda.synchronize()
        assert g.count_nonfinite(U) == 0
        vals = U.cpu() @ V
        got[name] = (float(vals.min()), float(vals.max()))
        _note(f"[leveque 128^2 P2 t=1] {name}: u_h in [{got[name][0]:.4f}, {got[name][1]:.4f}] "
              f"(printed {g_['printed_range'][name]}), {n} steps")
    pr = g_["printed_range"]
    assert got["DG"][0] < -0.05 and got["DG"][1] > 1.05
    assert got["LO"][0] >= -1e-3 and abs(got["LO"][1] - pr["LO"][1]) < 0.02
    assert got["WENO"][0] >= -1e-3 and abs(got["WENO"][1] - pr["WENO"][1]) < 1e-3
