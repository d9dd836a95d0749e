"""The window oracle used by the full-size GPU checks: on meshes small enough
for the whole-mesh oracle, the operator at a window's centre (radius 1) and
one SSP-RK3 step there (radius 3) equal the whole mesh's values, for
periodic, non-periodic and boundary cells."""
import numpy as np
import pytest
import torch

from helpers import oracle_for, oracle_initial, oracle_window
from paper_2309_12019_amd import inputs


def _cases():
    r = inputs.rot2d(12, 2, seed=1, ny=10)
    r.cy = 0.5 * 10 / 12
    b = inputs.burgers2d(11, 2, seed=2, ny=9, steps=1)
    a = inputs.adv1d(13, 3)
    u = inputs.burgers1d(9, 2)
    return [("rot2d", r), ("burgers2d", b), ("adv1d", a), ("burgers1d", u)]


@pytest.mark.parametrize("name,w", _cases())
def test_window_centre_equals_whole_mesh(name, w):
    O = oracle_for(w)
    U = oracle_initial(w, O)
    rng = np.random.default_rng(4)
    U = U + 0.05 * torch.from_numpy(rng.standard_normal(U.shape)) * U.abs().max()
    L = O.rhs(U)
    S = O.step(U, w.dt())
    ny = w.ny if w.dim == 2 else 1
    cells = [(ix, iy) for iy in range(ny) for ix in range(w.nx)]
    for ix, iy in cells:
        e = iy * w.nx + ix
        Ow, idx, c = oracle_window(w, ix, iy, 1)
        Lw = Ow.rhs(U[idx])
        assert torch.allclose(Lw[c], L[e], rtol=0, atol=1e-13 * float(L.abs().max())), (name, ix, iy)
        Ow, idx, c = oracle_window(w, ix, iy, 3)
        Sw = Ow.step(U[idx], w.dt())
        assert torch.allclose(Sw[c], S[e], rtol=0, atol=1e-13 * float(S.abs().max())), (name, ix, iy)
