"""Pins of the 1D Euler oracle (Sec. 5.6: Euler equations, density-only
sensor, Sod's shock tube between reflecting walls)."""
import math

import numpy as np
import pytest
import torch

from oracle.dgoracle import MODE_DG, MODE_LO, MODE_WENO, MODE_ZHAO, gauss_legendre
from oracle.euler1d import EulerOracle, EulerProblem, conserved, flux, stable_dt, wave_speed
from exact_sod import _star, sod_density
from paper_2309_12019_amd import inputs

GAMMA = 1.4   # the heat capacity ratio of Sec. 5.6 (stated here, not taken from the oracle)


def _random_states(n, seed):
    rng = np.random.default_rng(seed)
    rho = torch.from_numpy(rng.uniform(0.1, 2.0, n))
    v = torch.from_numpy(rng.uniform(-2.0, 2.0, n))
    p = torch.from_numpy(rng.uniform(0.1, 3.0, n))
    return rho, v, p


def test_wave_speed_is_the_spectral_radius_of_the_flux_jacobian():
    """The eigenvalues of F'(U) (central differences) are v - c, v, v + c, so
    |v| + c is the spectral radius the LLF flux and lambda_e use."""
    rho, v, p = _random_states(50, 1)
    U = conserved(rho, v, p)[:, :, None]          # [n, 3, 1]
    h = 1e-6
    for i in range(U.shape[0]):
        J = np.zeros((3, 3))
        for k in range(3):
            e = torch.zeros_like(U[i:i + 1])
            e[0, k, 0] = h * max(1.0, abs(float(U[i, k, 0])))
            J[:, k] = ((flux(U[i:i + 1] + e) - flux(U[i:i + 1] - e)) / (2 * e[0, k, 0]))[0, :, 0].numpy()
        ev = np.sort(np.linalg.eigvals(J).real)
        c = math.sqrt(GAMMA * float(p[i]) / float(rho[i]))
        assert np.allclose(ev, [float(v[i]) - c, float(v[i]), float(v[i]) + c], atol=1e-6)
        assert abs(float(wave_speed(U[i:i + 1])[0, 0]) - (abs(float(v[i])) + c)) < 1e-13


@pytest.mark.parametrize("mode", [MODE_DG, MODE_LO, MODE_WENO, MODE_ZHAO])
def test_a_state_at_rest_between_walls_is_steady(mode):
    O = EulerOracle(EulerProblem(nx=12, p=2, mode=mode))
    U = torch.zeros(12, 3, 3, dtype=torch.float64)
    U[:, :, 0] = conserved(torch.tensor([0.7]), torch.tensor([0.0]), torch.tensor([0.4]))[0]
    assert O.rhs(U).abs().max() < 1e-13


@pytest.mark.parametrize("mode", [MODE_LO, MODE_WENO, MODE_DG])
def test_walls_conserve_mass_and_energy(mode):
    """At a wall the LLF flux of mass and energy vanishes for the mirror state,
    so the totals (cell means times h) stay fixed over a run."""
    w = inputs.sod1d(40, 2, mode=mode)
    O = EulerOracle(EulerProblem(nx=40, p=2, mode=mode))
    U = O.project(w.ic)
    tot0 = U[:, :, 0].sum(0) * O.h
    U = O.run(U, w.dt(), 60)
    tot = U[:, :, 0].sum(0) * O.h
    assert abs(float(tot[0] - tot0[0])) < 1e-13 and abs(float(tot[2] - tot0[2])) < 1e-13
    assert abs(float(tot[1] - tot0[1])) > 1e-6      # the walls do exert a force


def test_mirror_symmetry():
    """x -> 1 - x with v -> -v maps the operator onto itself."""
    O = EulerOracle(EulerProblem(nx=10, p=3, mode=MODE_WENO))
    rng = np.random.default_rng(4)
    U = O.project(inputs.sod_tube) + 0.005 * torch.from_numpy(rng.standard_normal((10, 3, 4)))
    assert torch.isfinite(O.rhs(U)).all()
    flip = torch.tensor([(-1.0) ** a for a in range(4)], dtype=torch.float64)
    sgn = torch.tensor([1.0, -1.0, 1.0], dtype=torch.float64)[:, None]

    def mirror(X):
        return X.flip(0) * flip * sgn

    assert torch.allclose(O.rhs(mirror(U)), mirror(O.rhs(U)), rtol=0, atol=1e-12)


def _brute_rhs(U, nx, p, gam, lam):
    """The weak form in physical coordinates: numpy Legendre polynomials of
    x on each cell, Gauss rules from numpy, mass and stiffness matrices by
    quadrature, walls by mirror states."""
    h = 1.0 / nx
    Q = p + 2
    xg, wg = np.polynomial.legendre.leggauss(Q)
    xe, we = np.polynomial.legendre.leggauss(p + 2)
    out = np.zeros_like(U)

    def phi(a, e, x, d=0):
        c = np.zeros(a + 1)
        c[a] = 1.0
        xi = (x - (e + 0.5) * h) * 2 / h
        return np.polynomial.legendre.legval(xi, np.polynomial.legendre.legder(c, d) if d else c) * (2 / h) ** d

    def state(e, x):
        return np.array([sum(U[e, k, a] * phi(a, e, x) for a in range(p + 1)) for k in range(3)])

    def F(u):
        rho, m, E = u
        v = m / rho
        pr = (GAMMA - 1) * (E - 0.5 * m * v)
        return np.array([m, m * v + pr, (E + pr) * v]), abs(v) + math.sqrt(GAMMA * pr / rho)

    for e in range(nx):
        x = (e + 0.5) * h + 0.5 * h * xg
        M = np.array([[np.sum(0.5 * h * we * phi(a, e, (e + 0.5) * h + 0.5 * h * xe) *
                              phi(b, e, (e + 0.5) * h + 0.5 * h * xe)) for b in range(p + 1)] for a in range(p + 1)])
        K = np.array([[np.sum(0.5 * h * we * phi(a, e, (e + 0.5) * h + 0.5 * h * xe, 1) *
                              phi(b, e, (e + 0.5) * h + 0.5 * h * xe, 1)) for b in range(p + 1)] for a in range(p + 1)])
        R = np.zeros((3, p + 1))
        for qi in range(Q):
            Fq, _ = F(state(e, x[qi]))
            for a in range(p + 1):
                R[:, a] += 0.5 * h * wg[qi] * Fq * phi(a, e, x[qi], 1)
        for side in (-1, 1):
            xf = (e + 0.5 + 0.5 * side) * h
            um = state(e, xf)
            nb = e + side
            up = state(nb, xf) if 0 <= nb < nx else um * np.array([1.0, -1.0, 1.0])
            Fm, sm = F(um)
            Fp, sp = F(up)
            H = 0.5 * side * (Fm + Fp) - 0.5 * max(sm, sp) * (up - um)
            for a in range(p + 1):
                R[:, a] -= H * phi(a, e, xf)
        nu = lam[e] * h / (2 * p)
        R -= gam[e] * nu * (U[e] @ K.T)
        out[e] = np.linalg.solve(M, R.T).T
    return out


@pytest.mark.parametrize("p,mode", [(1, MODE_LO), (2, MODE_WENO), (3, MODE_DG), (2, MODE_ZHAO)])
def test_operator_against_bruteforce(p, mode):
    nx = 6
    O = EulerOracle(EulerProblem(nx=nx, p=p, mode=mode))
    rng = np.random.default_rng(p)
    U = O.project(inputs.sod_tube) + 0.005 * torch.from_numpy(rng.standard_normal((nx, 3, p + 1)))
    L, gam = O.rhs(U, with_gamma=True)
    lam = O.max_speed(U)
    ref = _brute_rhs(U.numpy(), nx, p, gam.numpy(), lam.numpy())
    assert np.abs(L.numpy() - ref).max() <= 1e-11 * np.abs(ref).max()


# --- Sod's problem against its exact solution -----------------------------
def test_exact_sod_solution_satisfies_the_jump_conditions():
    """The star state: Rankine-Hugoniot across the right shock (mass, momentum,
    energy), the Riemann invariants across the left fan, p and v continuous at
    the contact."""
    g = GAMMA
    s = _star()
    ps, us, rrs, S = s["ps"], s["us"], s["rrs"], s["S"]
    Ur = np.array([0.125, 0.0, 0.1 / (g - 1)])
    Us = np.array([rrs, rrs * us, ps / (g - 1) + 0.5 * rrs * us * us])

    def Fx(U):
        rho, m, E = U
        v = m / rho
        pr = (g - 1) * (E - 0.5 * m * v)
        return np.array([m, m * v + pr, (E + pr) * v])

    assert np.allclose(Fx(Us) - Fx(Ur), S * (Us - Ur), rtol=0, atol=1e-12)
    # left fan: p / rho^g and v + 2c/(g-1) are constant through it
    rls = s["rls"]
    assert abs(ps / rls ** g - 1.0) < 1e-12
    cls = math.sqrt(g * ps / rls)
    assert abs(us + 2 * cls / (g - 1) - 2 * s["cl"] / (g - 1)) < 1e-12
    assert abs(cls - s["cls"]) < 1e-12


def _run_sod(n, mode, t=0.1):
    w = inputs.sod1d(n, 2, mode=mode)
    O = EulerOracle(EulerProblem(nx=n, p=2, mode=mode))
    U = O.project(w.ic)
    k = int(math.ceil(t / w.dt()))
    U = O.run(U, t / k, k)
    vals = O.evaluate(U, 4)[:, 0]              # density at 4 Gauss points per cell
    xq = O.S.nodes(4)[..., 0].numpy()
    _, wq = gauss_legendre(4)
    err = float((np.abs(vals.numpy() - sod_density(xq, t)) * wq.numpy() * 0.5 * O.h).sum())
    return err, float(vals.min()), float(vals.max())


def test_sod_errors_and_the_behaviour_of_the_three_schemes():
    """t = 0.1, P2: the LO and WENO density errors (L1, against the exact
    solution) fall under refinement, WENO is more accurate than LO, and DG
    over- and undershoots the data range [0.125, 1] while LO stays inside."""
    res = {(m, n): _run_sod(n, m) for m in (MODE_LO, MODE_WENO, MODE_DG) for n in (32, 64)}
    for m in (MODE_LO, MODE_WENO):
        assert res[(m, 64)][0] < 0.8 * res[(m, 32)][0]
    assert res[(MODE_WENO, 64)][0] < res[(MODE_LO, 64)][0]
    lo = res[(MODE_LO, 64)]
    assert lo[1] >= 0.125 - 1e-3 and lo[2] <= 1.0 + 1e-3
    dg = res[(MODE_DG, 64)]
    assert dg[1] < 0.125 - 1e-3 or dg[2] > 1.0 + 1e-3


def test_stable_dt_uses_the_largest_wave_speed():
    P = EulerProblem(nx=20, p=2)
    O = EulerOracle(P)
    U = O.project(inputs.sod_tube)
    dt = stable_dt(P, U, 0.5)
    assert abs(dt - 0.5 * (1 / 20) / (5 * math.sqrt(1.4))) < 1e-15
