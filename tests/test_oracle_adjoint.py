"""The oracle's discrete adjoint (reverse mode through eq. (ssp) and the whole
stabilised operator) against central finite differences of its forward map."""
import numpy as np
import pytest
import torch

from helpers import oracle_for, oracle_initial
from paper_2309_12019_amd import inputs


def _fd(f, U, v, delta):
    """Richardson-extrapolated central difference of f along v."""
    d1 = (f(U + delta * v) - f(U - delta * v)) / (2 * delta)
    d2 = (f(U + 0.5 * delta * v) - f(U - 0.5 * delta * v)) / delta
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("make", [
    lambda: inputs.burgers2d(5, 2, steps=1),
    lambda: inputs.rot2d(4, 3, ny=4),
    lambda: inputs.burgers1d(9, 3),
    lambda: inputs.adv1d(7, 2),
])
def test_step_vjp_matches_finite_differences(make):
    w = make()
    O = oracle_for(w)
    rng = np.random.default_rng(4)
    U = oracle_initial(w, O) + 0.05 * torch.from_numpy(rng.standard_normal((w.ncells, w.nloc)))
    lam = torch.from_numpy(rng.standard_normal((w.ncells, w.nloc)))
    dt = w.dt()
    g = O.step_vjp(U, dt, lam)
    for k in range(3):
        v = torch.from_numpy(rng.standard_normal((w.ncells, w.nloc)))
        fd = _fd(lambda X: float((lam * O.step(X, dt)).sum()), U, v, 1e-5)
        ad = float((g * v).sum())
        assert abs(fd - ad) <= 1e-7 * max(abs(ad), 1e-3)


def test_run_gradient_of_window_functional():
    w = inputs.burgers2d(8, 2, steps=1)
    O = oracle_for(w)
    U0 = oracle_initial(w, O)
    J = lambda U: O.window_functional(U, (0.25, 0.75), (0.25, 0.75))
    n = 3
    g = O.run_grad(U0, w.dt(), n, J)
    rng = np.random.default_rng(9)
    for _ in range(2):
        v = torch.from_numpy(rng.standard_normal(U0.shape))
        v /= v.norm()
        fd = _fd(lambda X: float(J(O.run(X, w.dt(), n))), U0, v, 1e-5)
        ad = float((g * v).sum())
        assert abs(fd - ad) <= 1e-7 * abs(ad)


def test_window_functional_gradient_closed_form():
    """J = int_W u^2: dJ/dc_i = 2 c_i int_K phi_i^2 on cells inside W, 0 outside."""
    w = inputs.burgers2d(8, 2, steps=1)
    O = oracle_for(w)
    U = oracle_initial(w, O).requires_grad_(True)
    (g,) = torch.autograd.grad(O.window_functional(U, (0.25, 0.75), (0.25, 0.75)), U)
    inside = ((O.xc > 0.25) & (O.xc < 0.75) & (O.yc > 0.25) & (O.yc < 0.75))
    expect = 2 * U.detach() * torch.diag(O.M)[None, :] * inside[:, None].to(torch.float64)
    assert torch.allclose(g, expect, rtol=1e-13, atol=1e-16)
