"""Invariants the paper and the mathematics fix, checked on the oracle."""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

from helpers import oracle_for, oracle_initial, oracle_problem
from paper_2309_12019_amd import inputs


def linear_operator(O):
    """Matrix of the (linear) semi-discrete operator U -> dU/dt."""
    n = O.P.ncells * O.P.nloc
    I = torch.eye(n, dtype=torch.float64).reshape(n, O.P.ncells, O.P.nloc)
    return torch.stack([O.rhs(I[k]).reshape(-1) for k in range(n)], 1).numpy()


@pytest.mark.parametrize("make", [
    lambda: inputs.adv1d(24, 2),
    lambda: inputs.burgers1d(24, 3),
    lambda: inputs.burgers2d(8, 2, steps=1),
])
def test_mass_conservation_periodic(make):
    """Sec. 2: the LLF flux is conservative and the dissipation has a zero mean
    row, so int u_h is constant for periodic problems."""
    w = make()
    O = oracle_for(w)
    U = oracle_initial(w, O)
    m0 = O.mass(U)
    scale = O.mass(U.abs())
    for _ in range(10):
        U = O.step(U, w.dt())
    assert abs(O.mass(U) - m0) <= 1e-13 * scale


def test_dissipation_mean_row_is_zero():
    w = inputs.rot2d(6, 3, mode=inputs.MODE_LO)
    O = oracle_for(w)
    U = torch.from_numpy(np.random.default_rng(0).standard_normal((w.ncells, w.nloc)))
    assert torch.all(O.K[0] == 0) and torch.all(O.K[:, 0] == 0)
    s = O.dissipation(U)
    assert torch.all(s[:, 0] == 0)


@pytest.mark.parametrize("dim,p", [(1, 1), (1, 2), (1, 3), (1, 4), (2, 1), (2, 2), (2, 3)])
def test_reproduced_data_gives_zero_sensor(dim, p):
    """A global polynomial of degree <= p plus an arbitrary constant per cell is
    reproduced by every candidate, so U - U* has zero semi-norm and gamma = 0."""
    rng = np.random.default_rng(p)
    if dim == 1:
        w = inputs.adv1d(9, p)
        w.periodic_x = False
        coef = rng.standard_normal(p + 1)
        w.ic = lambda x: np.polynomial.polynomial.polyval(x, coef)
    else:
        w = inputs.rot2d(6, p)
        C = rng.standard_normal((p + 1, p + 1))
        w.ic = lambda x, y: np.polynomial.polynomial.polyval2d(x, y, C)
    O = oracle_for(w)
    U = oracle_initial(w, O)
    U[:, 0] += torch.from_numpy(rng.standard_normal(w.ncells))
    gam = O.sensor(U)
    assert float(gam.max()) < 1e-12
    wd = oracle_problem(w)
    wd.mode = inputs.MODE_DG
    Ld = type(O)(wd).rhs(U)
    Lw = O.rhs(U)
    assert float((Lw - Ld).abs().max()) <= 1e-13 * float(Ld.abs().max() + 1)


def test_sensor_range_and_constant_shift():
    w = inputs.rot2d(7, 2)
    O = oracle_for(w)
    U = torch.from_numpy(np.random.default_rng(5).standard_normal((w.ncells, w.nloc)))
    g = O.sensor(U)
    assert float(g.min()) >= 0.0 and float(g.max()) <= 1.0
    assert (g > 0).all() and (g < 1).any()
    U2 = U.clone()
    U2[:, 0] += 3.7
    assert torch.allclose(O.sensor(U2), g, rtol=1e-12, atol=1e-14)


def test_sensor_threshold_b():
    """eq. (gensensor): gamma^b equals gamma where the ratio reaches b, else 0."""
    w = inputs.adv1d(30, 2)
    O = oracle_for(w)
    U = oracle_initial(w, O)
    g0, det = O.sensor(U, details=True)
    b = float(det["ratio"].median())
    pb = oracle_problem(w)
    pb.b = b
    gb = type(O)(pb).sensor(U)
    keep = det["ratio"] >= b
    assert keep.any() and (~keep).any()
    assert torch.equal(gb[keep], g0[keep]) and torch.all(gb[~keep] == 0)


def test_sensor_q_exponent():
    w = inputs.adv1d(30, 2)
    O = oracle_for(w)
    U = oracle_initial(w, O)
    g1 = O.sensor(U)
    pq = oracle_problem(w)
    pq.q = 2.0
    g2 = type(O)(pq).sensor(U)
    assert torch.allclose(g2, g1 ** 2, rtol=1e-13, atol=1e-300)


def test_mirror_symmetry_1d():
    """Reflecting x -> -x maps c_a -> (-1)^a c_a and reverses the cells; the
    sensor is geometric, so gamma is reflected too; advection with v -> -v
    commutes with the reflection."""
    w = inputs.adv1d(17, 3)
    O = oracle_for(w)
    U = torch.from_numpy(np.random.default_rng(2).standard_normal((w.ncells, w.nloc)))
    sgn = torch.tensor([(-1.0) ** a for a in range(w.nloc)], dtype=torch.float64)
    R = U.flip(0) * sgn
    assert torch.allclose(O.sensor(R), O.sensor(U).flip(0), rtol=1e-12)
    wm = inputs.adv1d(17, 3)
    wm.vx = -1.0
    Om = oracle_for(wm)
    assert torch.allclose(Om.rhs(R), O.rhs(U).flip(0) * sgn, rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("mode", [inputs.MODE_DG, inputs.MODE_LO])
def test_ssp_rk3_is_the_cubic_taylor_polynomial(mode):
    """Eq. (ssp) applied to a linear operator A equals I + dtA + (dtA)^2/2 + (dtA)^3/6."""
    w = inputs.adv1d(12, 2, mode=mode)
    O = oracle_for(w)
    A = linear_operator(O)
    dt = 0.37 * w.h
    Z = dt * A
    S = np.eye(A.shape[0]) + Z + Z @ Z / 2 + Z @ Z @ Z / 6
    U = torch.from_numpy(np.random.default_rng(1).standard_normal((w.ncells, w.nloc)))
    got = O.step(U, dt).reshape(-1).numpy()
    assert np.allclose(got, S @ U.reshape(-1).numpy(), rtol=1e-13, atol=1e-13)


def test_ssp_rk3_third_order_in_time():
    w = inputs.adv1d(8, 1, mode=inputs.MODE_DG)
    O = oracle_for(w)
    A = linear_operator(O)
    U0 = oracle_initial(w, O)
    T = 0.25
    ref = scipy.linalg.expm(T * A) @ U0.reshape(-1).numpy()
    errs = []
    for n in (20, 40):
        errs.append(np.abs(O.run(U0, T / n, n).reshape(-1).numpy() - ref).max())
    assert 7.0 < errs[0] / errs[1] < 9.0


def _with_order(w, k):
    P = oracle_problem(w)
    P.rk_order = k
    return type(oracle_for(w))(P)


def _amplification_coefficients(O, k):
    """Coefficients c_j of the step's amplification polynomial R(z) = sum c_j z^j:
    for the linear DG operator the step maps an eigenvector v (eigenvalue lam)
    to R(dt lam) v, so R is fitted to its values at several dt."""
    A = linear_operator(O)
    lam, V = np.linalg.eig(A)
    j = int(np.argmax(np.abs(lam)))
    # R(dt lam_j) for several dt, from the step applied to the eigenvector
    zs, Rs = [], []
    v = V[:, j]
    for s in np.linspace(0.2, 1.0, 2 * k + 2):
        dt = s / abs(lam[j])
        out = (O.step(torch.from_numpy(v.real.copy()).reshape(O.P.ncells, O.P.nloc), dt).reshape(-1).numpy()
               + 1j * O.step(torch.from_numpy(v.imag.copy()).reshape(O.P.ncells, O.P.nloc), dt).reshape(-1).numpy())
        zs.append(dt * lam[j])
        Rs.append(np.vdot(v, out) / np.vdot(v, v))
    deg = {2: 2, 3: 3, 4: 5}[k]
    Vm = np.vander(np.array(zs), deg + 1, increasing=True)
    return np.linalg.lstsq(Vm, np.array(Rs), rcond=None)[0]


@pytest.mark.parametrize("k", [2, 3, 4])
def test_ssp_step_amplification_polynomial(k):
    """An SSP method of order k applied to a linear operator has the
    amplification polynomial of the Taylor series of exp(z) up to z^k: 1, 1,
    1/2, 1/6, 1/24 (order conditions).  The two-stage method is exactly
    1 + z + z^2/2; the five-stage fourth-order method has degree five."""
    w = inputs.adv1d(6, 1, mode=inputs.MODE_DG)
    c = _amplification_coefficients(_with_order(w, k), k)
    taylor = [1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0][: k + 1]
    assert np.allclose(c[: k + 1], taylor, rtol=0, atol=1e-9)
    if k == 2:
        assert abs(c[2] - 0.5) < 1e-9
    if k == 4:
        # five stages: the z^5 term is present and smaller than the Taylor 1/120
        assert 0.0 < c[5].real < 1.0 / 120.0


@pytest.mark.parametrize("k,lo,hi", [(2, 3.5, 4.5), (4, 14.0, 18.0)])
def test_ssp_orders_in_time(k, lo, hi):
    """Against the exact propagator exp(T A) of the linear DG operator, halving
    dt divides the error by 2^k."""
    w = inputs.adv1d(8, 1, mode=inputs.MODE_DG)
    O = _with_order(w, k)
    A = linear_operator(O)
    U0 = oracle_initial(w, O)
    T = 0.25
    ref = scipy.linalg.expm(T * A) @ U0.reshape(-1).numpy()
    errs = [np.abs(O.run(U0, T / n, n).reshape(-1).numpy() - ref).max() for n in (20, 40)]
    assert lo < errs[0] / errs[1] < hi


def test_ssp54_shu_osher_table_is_consistent_and_ssp():
    """The five-stage table: each row of alpha sums to one (consistency), all
    entries are non-negative (a convex combination of forward Euler steps),
    and the SSP coefficient min alpha/beta is the published 1.508."""
    O = _with_order(inputs.adv1d(4, 1), 4)
    ratios = []
    for ra, rb in zip(O.SSP54_ALPHA, O.SSP54_BETA):
        assert abs(sum(ra) - 1.0) < 1e-14
        assert min(ra) >= 0.0 and min(rb) >= 0.0
        ratios += [a / b for a, b in zip(ra, rb) if b > 0.0]
    assert abs(min(ratios) - 1.508) < 1e-3


def test_ssp_methods_conserve_mass():
    w = inputs.burgers1d(40, 2, mode=inputs.MODE_WENO)
    for k in (2, 4):
        O = _with_order(w, k)
        U = oracle_initial(w, O)
        m0 = float(U[:, 0].sum())
        U = O.run(U, w.dt(), 10)
        assert abs(float(U[:, 0].sum()) - m0) < 1e-12


@pytest.mark.parametrize("p,limit", [(1, 0.409), (2, 0.209), (3, 0.130), (4, 0.089)])
def test_dg_stability_limits(p, limit):
    """The upwind DG operator with SSP-RK3 is linearly stable up to the known
    Courant numbers dt |v| / h = 0.409, 0.209, 0.130, 0.089 (p = 1..4)."""
    w = inputs.adv1d(40, p, mode=inputs.MODE_DG)
    O = oracle_for(w)
    lam = np.linalg.eigvals(linear_operator(O)) * w.h

    def stable(c):
        z = c * lam
        return np.abs(1 + z + z * z / 2 + z ** 3 / 6).max() <= 1 + 1e-10

    lo, hi = 0.01, 1.0
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if stable(mid) else (lo, mid)
    assert abs(lo - limit) < 0.002


# --- the sensor of Zhao et al. (Sec. 5.6) ---------------------------------
def _zhao(w):
    pz = oracle_problem(w)
    pz.mode = inputs.MODE_ZHAO
    return type(oracle_for(w))(pz)


@pytest.mark.parametrize("dim,p", [(1, 1), (1, 2), (1, 4), (2, 2), (2, 3)])
def test_zhao_sensor_zero_on_reproduced_data(dim, p):
    """Data that every candidate reproduces (a global polynomial of degree <= p
    plus a constant per cell) give equal indicators, hence nonlinear weights
    equal to the linear ones and gamma^Z = 0."""
    rng = np.random.default_rng(10 + p)
    if dim == 1:
        w = inputs.adv1d(9, p)
        w.periodic_x = False
        coef = rng.standard_normal(p + 1)
        w.ic = lambda x: np.polynomial.polynomial.polyval(x, coef)
    else:
        w = inputs.rot2d(6, p)
        C = rng.standard_normal((p + 1, p + 1))
        w.ic = lambda x, y: np.polynomial.polynomial.polyval2d(x, y, C)
    O = _zhao(w)
    U = oracle_initial(w, O)
    U[:, 0] += torch.from_numpy(rng.standard_normal(w.ncells))
    assert float(O.gamma(U).abs().max()) < 1e-12


def test_zhao_sensor_reaches_one_when_a_neighbour_candidate_takes_all_weight():
    """The denominator is the largest value the numerator takes: all weight on
    the candidate with the smallest linear weight.  A constant left neighbour
    (indicator 0) next to a steep cell puts nearly all weight on that
    neighbour's candidate, so gamma^Z -> 1 (up to the eps of the weights)."""
    w = inputs.adv1d(3, 2)
    w.periodic_x = False
    O = _zhao(w)
    U = torch.tensor([[0.3, 0.0, 0.0], [0.0, 1.0, 0.5], [1.0, 1.0, 0.5]], dtype=torch.float64)
    g = O.gamma(U)
    assert abs(float(g[1]) - 1.0) <= 1e-9
    assert float(g.min()) >= 0.0 and float(g.max()) <= 1.0 + 1e-15


def test_zhao_sensor_range_shift_and_mirror():
    w = inputs.rot2d(7, 2)
    O = _zhao(w)
    U = torch.from_numpy(np.random.default_rng(6).standard_normal((w.ncells, w.nloc)))
    g = O.gamma(U)
    assert float(g.min()) >= 0.0 and float(g.max()) <= 1.0
    assert (g > 0).all()
    U2 = U.clone()
    U2[:, 0] += 3.7
    assert torch.allclose(O.gamma(U2), g, rtol=1e-12, atol=1e-14)
    w1 = inputs.adv1d(17, 3)
    O1 = _zhao(w1)
    V = torch.from_numpy(np.random.default_rng(7).standard_normal((w1.ncells, w1.nloc)))
    sgn = torch.tensor([(-1.0) ** a for a in range(w1.nloc)], dtype=torch.float64)
    assert torch.allclose(O1.gamma(V.flip(0) * sgn), O1.gamma(V).flip(0), rtol=1e-12)


def test_zhao_sensor_without_neighbours_is_zero():
    """A single cell on a non-periodic line has no candidate but its own: its
    weight is its linear weight and gamma^Z = 0 (the reading for the printed
    0/0)."""
    w = inputs.adv1d(1, 2)
    w.periodic_x = False
    O = _zhao(w)
    U = torch.tensor([[0.2, 0.7, -0.4]], dtype=torch.float64)
    assert float(O.gamma(U)[0]) == 0.0


def test_zhao_sensor_theta():
    """theta = 2 squares every deviation and the largest one in the denominator."""
    w = inputs.adv1d(30, 2)
    O = _zhao(w)
    U = oracle_initial(w, O)
    _, d = O.sensor(U, details=True)
    pz = oracle_problem(w)
    pz.mode, pz.theta = inputs.MODE_ZHAO, 2.0
    g2 = type(O)(pz).gamma(U)
    dev = ((d["omega"] / d["lin"] - 1.0) ** 2).sum(1)
    assert torch.allclose(g2, dev / ((1.0 / w.w_nb - 1.0) ** 2 + 2.0), rtol=1e-13, atol=1e-300)
