"""Pins of the oracle's one-dimensional building blocks against closed forms and
library routines (numpy.polynomial.legendre)."""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch
from numpy.polynomial import legendre as npleg

import oracle
from oracle.dgoracle import poly_deriv


@pytest.mark.parametrize("Q", range(1, 9))
def test_gauss_exact_to_degree_2Q_minus_1(Q):
    x, w = oracle.gauss_legendre(Q)
    for k in range(2 * Q):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(float((w * x ** k).sum()) - exact) < 1e-14
    # degree 2Q is not integrated exactly (the rule has exactly Q points)
    exact = 2.0 / (2 * Q + 1)
    assert abs(float((w * x ** (2 * Q)).sum()) - exact) > 1e-6
    xn, wn = npleg.leggauss(Q)
    assert np.allclose(x.numpy(), xn, atol=1e-15, rtol=0)
    assert np.allclose(w.numpy(), wn, atol=1e-15, rtol=0)


def test_legendre_closed_forms():
    F = Fraction
    assert oracle.legendre_poly(2) == [F(-1, 2), F(0), F(3, 2)]
    assert oracle.legendre_poly(3) == [F(0), F(-3, 2), F(0), F(5, 2)]
    assert oracle.legendre_poly(4) == [F(3, 8), F(0), F(-30, 8), F(0), F(35, 8)]
    for a in range(6):
        ref = npleg.leg2poly([0] * a + [1])
        got = [float(c) for c in oracle.legendre_poly(a)]
        assert np.allclose(got, ref, atol=1e-15)


@pytest.mark.parametrize("dim,p", [(1, 1), (1, 4), (2, 2), (2, 3)])
def test_basis_end_values_and_orthogonality(dim, p):
    B = oracle.Basis(dim, p)
    pts = torch.tensor([[1.0] * dim, [-1.0] * dim], dtype=torch.float64)
    V = B.eval(pts)
    for j, mode in enumerate(B.modes):
        assert V[0, j] == 1.0
        assert V[1, j] == (-1.0) ** sum(mode)
    ref, w = oracle.tensor_rule(dim, p + 1)
    E = B.eval(ref)
    M = (E.T * w) @ E
    diag = torch.tensor([math.prod(2.0 / (2 * a + 1) for a in mode) for mode in B.modes],
                        dtype=torch.float64)
    assert torch.allclose(M, torch.diag(diag), atol=1e-14, rtol=0)


def _prob(dim, p, **kw):
    n = 4
    return oracle.Problem(dim=dim, nx=n, ny=n if dim == 2 else 1, p=p, **kw)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_stiffness_1d_closed_form(p):
    """int phi_a' phi_b' dx = (2/h) S_ab, S_ab = m(m+1) (m = min(a,b)) for a+b even."""
    O = oracle.Oracle(_prob(1, p))
    for a in range(p + 1):
        for b in range(p + 1):
            m = min(a, b)
            S = m * (m + 1) if (a + b) % 2 == 0 else 0
            assert abs(float(O.K[a, b]) - 2.0 / O.h * S) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_stiffness_2d_tensor_form(p):
    """2D: int grad phi_i . grad phi_j = S (x) Mhat + Mhat (x) S (h-independent)."""
    O = oracle.Oracle(_prob(2, p))
    n = p + 1
    S = np.array([[min(a, b) * (min(a, b) + 1) if (a + b) % 2 == 0 else 0
                   for b in range(n)] for a in range(n)], dtype=float)
    Mh = np.diag([2.0 / (2 * a + 1) for a in range(n)])
    # j = a + n b  ->  Kronecker index (b, a)
    K = np.kron(Mh, S) + np.kron(S, Mh)
    assert np.allclose(O.K.numpy(), K, atol=1e-12)


def test_seminorm_1d_p2_closed_form():
    """1D, p=2: ||v||_e^2 = 4 c1^2 + 156 c2^2, independent of h."""
    for h_cells in (4, 37):
        O = oracle.Oracle(oracle.Problem(dim=1, nx=h_cells, p=2))
        C = torch.tensor([[0.3, -1.25, 0.7], [5.0, 0.0, 0.0], [0.0, 1.0, 0.0],
                          [0.0, 0.0, 1.0]], dtype=torch.float64)
        got = O.seminorm2(C)
        exp = 4 * C[:, 1] ** 2 + 156 * C[:, 2] ** 2
        assert torch.allclose(got, exp, rtol=1e-14, atol=1e-14)


def test_seminorm_2d_p1_closed_form():
    """2D, p=1, |k| = 1 only: v = c00 + c10 x + c01 y + c11 x y on [-1,1]^2:
    2^{2-2} int (c10 + c11 y)^2 + (c01 + c11 x)^2 = 4 c10^2 + 4 c01^2 + (8/3) c11^2."""
    O = oracle.Oracle(_prob(2, 1))
    C = torch.tensor([[0.1, 0.5, -0.25, 2.0]], dtype=torch.float64)  # j = a + 2b
    got = float(O.seminorm2(C)[0])
    exp = 4 * 0.5 ** 2 + 4 * 0.25 ** 2 + 8.0 / 3.0 * 2.0 ** 2
    assert abs(got - exp) < 1e-13


def test_continuation_matrix_integer_rows():
    """P_1(xi+2) = P_1 + 2,  P_2(xi+2) = P_2 + 6 P_1 + 6  (left neighbour seen
    from the cell), and the mirror image for the right neighbour."""
    O = oracle.Oracle(oracle.Problem(dim=1, nx=4, p=3))
    T = O.cont[(0, -1)]   # maps left-neighbour coefficients to own coefficients
    assert torch.allclose(T[:, 1], torch.tensor([2.0, 1.0, 0, 0], dtype=torch.float64), atol=1e-13)
    assert torch.allclose(T[:, 2], torch.tensor([6.0, 6.0, 1.0, 0], dtype=torch.float64), atol=1e-13)
    Tr = O.cont[(0, 1)]
    assert torch.allclose(Tr[:, 1], torch.tensor([-2.0, 1.0, 0, 0], dtype=torch.float64), atol=1e-13)
    assert torch.allclose(Tr[:, 2], torch.tensor([6.0, -6.0, 1.0, 0], dtype=torch.float64), atol=1e-13)
    # the continuation of P_3 reproduces P_3(xi + 2) exactly
    x = torch.linspace(-1, 1, 7, dtype=torch.float64)
    P3 = oracle.legendre_poly(3)
    lhs = sum(float(c) * (x + 2) ** i for i, c in enumerate(P3))
    B = oracle.Basis(1, 3).eval(x[:, None])
    assert torch.allclose(B @ T[:, 3], lhs, atol=1e-12)


def test_multi_indices():
    assert oracle.multi_indices(1, 3) == [(1,), (2,), (3,)]
    assert sorted(oracle.multi_indices(2, 2)) == sorted([(1, 0), (0, 1), (2, 0), (1, 1), (0, 2)])


def test_poly_deriv():
    F = Fraction
    assert poly_deriv([F(1), F(2), F(3)], 1) == [F(2), F(6)]
    assert poly_deriv([F(1), F(2), F(3)], 3) == [F(0)]


# ---------------------------------------------------------------------------
# Oracle.project and Oracle.l1_error against numpy's Legendre routines
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("dim", [1, 2])
def test_projection_reproduces_polynomials_of_degree_p(dim, p):
    """The L2 projection onto V_p (Sec. 2) is the identity on V_p: a global
    polynomial of degree <= p per axis comes back as its own Legendre
    coefficients on every cell (numpy's poly2leg of the polynomial written in
    the cell's reference coordinate)."""
    import numpy.polynomial.legendre as npleg
    import numpy.polynomial.polynomial as nppoly
    from oracle import Oracle, Problem
    rng = np.random.default_rng(10 * dim + p)
    n = 5
    prob = Problem(dim=dim, nx=n, ny=n if dim == 2 else 1, p=p, x0=-0.3, x1=0.7, y0=0.1, y1=1.1)
    O = Oracle(prob)
    ax = rng.standard_normal(p + 1)
    ay = rng.standard_normal(p + 1) if dim == 2 else None
    h = prob.h

    def cell_leg(a, c0):
        # sum_k a_k (c0 + (h/2) xi)^k in powers of xi, then Legendre
        mono = np.zeros(p + 1)
        for k, ak in enumerate(a):
            mono[: k + 1] += ak * nppoly.polypow([c0, 0.5 * h], k)[: k + 1]
        leg = np.zeros(p + 1)
        l_ = npleg.poly2leg(mono)
        leg[: len(l_)] = l_[: p + 1]
        return leg

    nodes = O.proj_nodes().numpy()
    if dim == 1:
        vals = nppoly.polyval(nodes[..., 0], ax)
    else:
        vals = nppoly.polyval(nodes[..., 0], ax) * nppoly.polyval(nodes[..., 1], ay)
    U = O.project(torch.from_numpy(vals)).numpy()
    for e in range(prob.ncells):
        ix, iy = e % n, e // n
        leg_x = cell_leg(ax, prob.x0 + (ix + 0.5) * h)
        if dim == 1:
            want = leg_x
        else:
            cy = cell_leg(ay, prob.y0 + (iy + 0.5) * h)
            want = np.outer(cy, leg_x).reshape(-1)        # j = a + (p+1) b
        assert np.allclose(U[e], want, rtol=1e-12, atol=1e-12)


def test_l1_error_of_known_fields():
    """l1_error integrates |u_h - u| with the node weights (h/2)^d w_q: for a
    state that is the constant c on every cell and exact values 0 it is
    |c| |Omega|; for u_h = x - x_c (a linear mode) it is the Q-point rule
    applied to |x - x_c| on every cell (numpy's Gauss rule)."""
    from oracle import Oracle, Problem
    O = Oracle(Problem(dim=2, nx=6, ny=6, p=2, x0=0.0, x1=1.5, y0=0.0, y1=1.5))
    U = torch.zeros(36, 9, dtype=torch.float64)
    U[:, 0] = -0.7
    assert abs(O.l1_error(U, torch.zeros(36, 16, dtype=torch.float64), 4) - 0.7 * 1.5 ** 2) < 1e-14
    O1 = Oracle(Problem(dim=1, nx=8, p=2))
    V = torch.zeros(8, 3, dtype=torch.float64)
    V[:, 1] = 0.5 * O1.h                 # u_h = (h/2) xi = x - x_c
    exact = torch.zeros(8, 6, dtype=torch.float64)
    # |xi| is not a polynomial: the 6-point rule integrates it only approximately
    xi, w = np.polynomial.legendre.leggauss(6)
    want = 8 * (0.5 * O1.h) ** 2 * float(np.sum(w * np.abs(xi)))
    assert abs(O1.l1_error(V, exact, 6) - want) < 1e-15
