"""The plain C oracle (oracle/dgoracle.c), pinned before it is trusted.

It is checked (a) against the PyTorch oracle, an independent implementation
of the same readings that is itself pinned against the paper
(test_oracle_*.py), on small ragged meshes for every flux, degree, sensor mode
and SSP order; and (b) directly against what the paper and the mathematics
fix, with the test side's own numpy Legendre routines for projections and
errors: conservation of cell means on periodic meshes (Sec. 2), zero sensor
on data the HWENO reconstruction reproduces (Sec. 4), the zero mean row of
the dissipation (eq. astab), shift invariance of the sensor, gamma in [0, 1],
and rows of Table 1 (Sec. 5.1, linear advection, DG and LO columns) under
SSP-RK3 with a small step.  Results do not depend on the thread count.
"""
import json
import math
import os

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest
import torch

from helpers import oracle_for, oracle_initial, oracle_problem
from oracle import coracle
from paper_2309_12019_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def relinf(a, b):
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


def _mesh(kind, p, mode):
    if kind == "adv1d":
        return inputs.adv1d(37, p, mode=mode)
    if kind == "burgers1d":
        w = inputs.burgers1d(29, p, mode=mode)
        w.periodic_x = False      # inflow faces with the constant exterior state
        w.bc_value = 0.3
        return w
    if kind == "rot2d":
        return inputs.rot2d(13, p, mode=mode, ny=11)
    if kind == "burgers2d":
        return inputs.burgers2d(12, p, mode=mode, steps=5, ny=10)
    if kind == "kpp2d":
        return inputs.kpp2d(11, p, mode=mode, steps=5, lam=0.0)
    raise ValueError(kind)


def _rough(w, O, seed=1):
    U = oracle_initial(w, O)
    rng = np.random.default_rng(seed)
    return U + 0.05 * torch.from_numpy(rng.standard_normal(U.shape)) * U.abs().max()


@pytest.mark.parametrize("kind", ["adv1d", "burgers1d", "rot2d", "burgers2d", "kpp2d"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_c_oracle_matches_the_torch_oracle(kind, p, mode):
    """Operator, gamma_e and five SSP-RK3 steps on a rough state."""
    w = _mesh(kind, p, mode)
    O = oracle_for(w)
    C = coracle.COracle(oracle_problem(w))
    U = _rough(w, O)
    Lo, go = O.rhs(U, with_gamma=True)
    Lc, gc = C.rhs(U, with_gamma=True)
    assert relinf(Lc, Lo) <= 1e-13
    assert float((gc - go).abs().max()) <= 1e-13
    assert relinf(C.run(U, w.dt(), 5), O.run(U, w.dt(), 5)) <= 1e-13


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("kind", ["adv1d", "burgers2d", "kpp2d"])
def test_c_oracle_ssp_orders(order, kind):
    w = _mesh(kind, 3 if kind == "adv1d" else 2, inputs.MODE_WENO)
    w.rk_order = order
    O = oracle_for(w)
    C = coracle.COracle(oracle_problem(w))
    U = _rough(w, O)
    assert relinf(C.run(U, w.dt(), 5), O.run(U, w.dt(), 5)) <= 1e-13


# ---------------------------------------------------------------------------
# pins against the paper and the mathematics (numpy on the test side)
# ---------------------------------------------------------------------------
def _leg_coeffs_of(fun, xc, h, p, Q):
    """Legendre coefficients of the L2 projection of fun onto P_p on the cell
    [xc - h/2, xc + h/2], with numpy's Gauss rule of Q points."""
    xi, wq = npleg.leggauss(Q)
    vals = fun(xc[:, None] + 0.5 * h * xi[None, :])
    V = npleg.legvander(xi, p)                      # [Q, p+1]
    norms = 2.0 / (2 * np.arange(p + 1) + 1)
    return (vals * wq) @ V / norms


def _cell_poly_1d(a, xc, h, p):
    """Legendre coefficients, per cell, of the global polynomial sum_k a_k x^k
    (degree <= p) written in the cell's reference coordinate."""
    out = np.zeros((len(xc), p + 1))
    for e, x0 in enumerate(xc):
        # x = x0 + (h/2) xi: expand sum_k a_k (x0 + (h/2) xi)^k in powers of xi
        mono = np.zeros(p + 1)
        for k, ak in enumerate(a):
            for i in range(k + 1):
                mono[i] += ak * math.comb(k, i) * x0 ** (k - i) * (0.5 * h) ** i
        leg = npleg.poly2leg(mono)[: p + 1]
        out[e, : len(leg)] = leg
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("dim", [1, 2])
def test_reproduced_data_give_zero_sensor(dim, p):
    """Sec. 4: data the HWENO reconstruction reproduces (one global polynomial
    of degree <= p, plus an arbitrary constant per cell) have U* = U, so
    gamma_e = 0 on interior cells and the WENO operator equals the DG one."""
    rng = np.random.default_rng(p + 10 * dim)
    n = 9
    if dim == 1:
        w = inputs.adv1d(n, p, mode=inputs.MODE_WENO)
        w.periodic_x = False
        h = w.h
        xc = (np.arange(n) + 0.5) * h
        U = _cell_poly_1d(rng.standard_normal(p + 1), xc, h, p)
        U[:, 0] += rng.standard_normal(n)
        interior = np.arange(1, n - 1)
    else:
        w = inputs.rot2d(n, p, mode=inputs.MODE_WENO)
        h = w.h
        xc = (np.arange(n) + 0.5) * h
        ax = _cell_poly_1d(rng.standard_normal(p + 1), xc, h, p)   # q(x) = qx(x) qy(y)
        ay = _cell_poly_1d(rng.standard_normal(p + 1), xc, h, p)
        U = np.einsum("ia,jb->jiba", ax, ay).reshape(n * n, (p + 1) ** 2)  # cell = ix + n iy, mode a + (p+1) b
        U[:, 0] += rng.standard_normal(n * n)
        ii = np.arange(n * n)
        ix, iy = ii % n, ii // n
        interior = ii[(ix > 0) & (ix < n - 1) & (iy > 0) & (iy < n - 1)]
    U = torch.from_numpy(np.ascontiguousarray(U))
    C = coracle.COracle(oracle_problem(w))
    L, gam = C.rhs(U, with_gamma=True)
    assert float(gam[interior].abs().max()) <= 1e-13
    w.mode = inputs.MODE_DG
    Ld = coracle.COracle(oracle_problem(w)).rhs(U)
    assert relinf(L[interior], Ld[interior]) <= 1e-13


@pytest.mark.parametrize("kind", ["adv1d", "burgers2d", "kpp2d"])
def test_dissipation_has_a_zero_mean_row(kind):
    """Eq. (astab): int grad(1) . grad(u_h) = 0, so adding the dissipation
    (LO: gamma = 1 everywhere) leaves the cell-mean component of dU/dt
    unchanged (to rounding: the oracle inverts the mass matrix numerically,
    and its off-diagonal entries are zero only up to rounding)."""
    w = _mesh(kind, 3, inputs.MODE_LO)
    O = oracle_for(w)
    U = _rough(w, O)
    Llo = coracle.COracle(oracle_problem(w)).rhs(U)
    w.mode = inputs.MODE_DG
    Ldg = coracle.COracle(oracle_problem(w)).rhs(U)
    scale = float(Ldg.abs().max())
    assert float((Llo[:, 0] - Ldg[:, 0]).abs().max()) <= 1e-14 * scale
    assert float((Llo[:, 1:] - Ldg[:, 1:]).abs().max()) > 1e-3 * scale


@pytest.mark.parametrize("kind,p", [("adv1d", 2), ("burgers2d", 2), ("burgers2d", 4)])
def test_cell_means_are_conserved_on_periodic_meshes(kind, p):
    """Sec. 2: on a periodic mesh the LLF flux is single-valued on every face,
    so sum_e h^d c_e0 is constant over steps, with the sensor switched on."""
    w = _mesh(kind, p, inputs.MODE_WENO)
    O = oracle_for(w)
    U = _rough(w, O)
    C = coracle.COracle(oracle_problem(w))
    m0 = float(U[:, 0].sum())
    scale = float(U[:, 0].abs().sum())
    for _ in range(4):
        U = C.run(U, w.dt(), 5)
        assert abs(float(U[:, 0].sum()) - m0) <= 1e-14 * scale * 20


@pytest.mark.parametrize("kind", ["rot2d", "burgers2d"])
def test_sensor_is_shift_invariant_and_bounded(kind):
    """Eqs. (sensor)/(gensensor) see only derivatives: adding a constant to the
    data leaves gamma_e unchanged; gamma_e lies in [0, 1]."""
    w = _mesh(kind, 2, inputs.MODE_WENO)
    O = oracle_for(w)
    U = _rough(w, O)
    C = coracle.COracle(oracle_problem(w))
    _, g1 = C.rhs(U, with_gamma=True)
    V = U.clone()
    V[:, 0] += 3.7
    _, g2 = C.rhs(V, with_gamma=True)
    assert float((g1 - g2).abs().max()) <= 1e-13
    assert float(g1.min()) >= 0.0 and float(g1.max()) <= 1.0


def test_results_do_not_depend_on_the_thread_count():
    w = inputs.burgers2d(24, 3, steps=3)
    O = oracle_for(w)
    U = _rough(w, O)
    C = coracle.COracle(oracle_problem(w))
    nmax = coracle.max_threads()
    try:
        coracle.set_threads(1)
        a = C.run(U, w.dt(), 3)
        coracle.set_threads(max(2, nmax))
        b = C.run(U, w.dt(), 3)
    finally:
        coracle.set_threads(nmax)
    assert torch.equal(a, b)


TABLES = json.load(open(os.path.join(HERE, "golden", "paper_tables.json")))


def _table1(p, N, col):
    for r in TABLES["table1_advection"]["rows"]:
        if r["p"] == p and r["E_h"] == N:
            return r[col]
    raise KeyError((p, N))


@pytest.mark.parametrize("p,N,col,tol", [(1, 16, "LO", 0.02), (2, 32, "LO", 0.02), (3, 64, "LO", 0.02),
                                         (2, 16, "DG", 0.08), (3, 16, "DG", 0.08)])
def test_table1_rows_through_the_c_oracle(p, N, col, tol):
    """Table 1 (Sec. 5.1): u_t + u_x = 0 on periodic (0,1), u0 = cos(2 pi (x -
    0.5)), L1 error at t = 1.  SSP-RK3 with dt = 0.02 h / (2p+1) keeps the time
    error far below the tabulated errors; the projection and the L1 norm use
    numpy's Gauss-Legendre rules (p + 2 and p + 3 points)."""
    w = inputs.adv1d(N, p, mode=inputs.MODE_LO if col == "LO" else inputs.MODE_DG, cfl=0.02)
    h = w.h
    xc = (np.arange(N) + 0.5) * h
    U = torch.from_numpy(_leg_coeffs_of(inputs.cos_wave, xc, h, p, p + 2))
    C = coracle.COracle(oracle_problem(w))
    n = int(math.ceil(1.0 / w.dt()))
    U = C.run(U, 1.0 / n, n).numpy()
    xi, wq = npleg.leggauss(p + 3)
    uh = U @ npleg.legvander(xi, p).T
    exact = inputs.cos_wave(xc[:, None] + 0.5 * h * xi[None, :] - 1.0)
    err = float((np.abs(uh - exact) * wq).sum() * 0.5 * h)
    assert abs(err / _table1(p, N, col) - 1) < tol
