"""CPU oracle for the dissipative-WENO-stabilised RKDG scheme.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
HIP library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code, tables or constants with the HIP library: Gauss rules,
Legendre polynomials, shifts and semi-norms are all derived here, from their
definitions, independently.

Paper: J. Vedral, "Dissipative WENO stabilization of high-order discontinuous
Galerkin methods for hyperbolic problems" (arXiv 2309.12019).

What is computed, in the paper's order and notation (all FP64, PyTorch CPU ops,
vectorised over cells only; no blocking, fusion or reordering):

* Fluxes: linear advection with a constant or rotating velocity, Burgers, and
  the non-convex KPP flux F(u) = (sin u, cos u) of Sec. 5.5 (2D).
* Sec. 2, eq. (weak2): the semi-discrete DG operator
      M dU/dt = R(U),
      R_i = int_K grad(phi_i) . F(U_h) dx - int_dK phi_i H(U^-, U^+, n) ds
  with the local Lax-Friedrichs flux H of Sec. 2 and the maximal wave speed
  s^+ = max_{w in [0,1]} |F'(w U^- + (1-w) U^+) . n|.
* Sec. 3, eqs. (lostab), (visc), (astab): the element-local dissipation
      s_i = gamma_e nu_e int_K grad(phi_i) . grad(U_h) dx,
      nu_e = lambda_e h_e / (2p),  lambda_e = ||F'(U_h)||_{L^inf(K_e)}.
  Mode DG uses gamma_e = 0, mode LO gamma_e = 1, mode WENO the sensor below,
  mode ZHAO the sensor of Zhao et al. that Sec. 5.6 compares with:
      gamma_e^Z = sum_l |omega_l / omega~_l - 1|^theta
                  / (|1 / min_l omega~_l - 1|^theta + m_e)
  over the candidates that exist, with the same HWENO weights.
* Sec. 4, eqs. (sensor), (gensensor) and the scaled Sobolev semi-norm:
      gamma_e = min(1, ||U - U*||_e / ||U||_e)^q   (0 below the threshold b),
      ||v||_e^2 = sum_{1<=|k|<=p} h^{2|k|-d} int_K |D^k v|^2 dx,
  with the Hermite-WENO reconstruction U* = sum_l omega_l U_l and the linear
  weights of Sec. 5 (omega~_0 = 1 - m_e w, omega~_l = w).
* Sec. 2, eq. (ssp): the three-stage SSP Runge-Kutta step; also the
  second-order and the five-stage fourth-order SSP methods (Sec. 5.1 uses SSP
  methods of order p + 1 for its convergence study).

Readings where the paper is silent (they are listed again, with reasons, in the
project's design notes):
* Candidates U_l: the polynomial of face neighbour l, continued into K_e and
  L2-projected onto V_p(K_e), with its mean replaced by the mean of U_h on K_e.
  The stencil is the face neighbours that exist (periodic wrap counts).
* Smoothness indicators beta_l = ||U_l||_e^2 (the same semi-norm); nonlinear
  weights alpha_l = omega~_l / (eps + beta_l)^r, omega_l = alpha_l / sum alpha.
* ||U - U*||_e = 0 gives ratio 0; ||U||_e = 0 < ||U - U*||_e gives ratio inf.
* lambda_e is the maximum of ||F'(u_h)||_2 over the volume Gauss nodes, unless
  an override is given (the paper fixes lambda_e by hand for one test).
* Basis: tensor Legendre polynomials on the reference cell [-1,1]^d; the
  method is basis-independent (Sec. 2).
* Non-periodic faces see a fixed exterior state through the same LLF flux;
  for the four-quadrant Burgers problem of Sec. 5.4 the exterior state is the
  exact solution in R^2 at the face Gauss points and at the time of the
  stage's input state (the paper sets its inflow data from the exact
  solution; here every boundary face uses it, inflow or not).  The exact
  solution comes from the Lax-Oleinik formula along the diagonal lines on
  which the problem is one-dimensional.
* Mode ZHAO: gamma_e = gamma_e^Z as printed (neither q nor the threshold b
  applies); min_l omega~_l runs over the candidates that exist; a cell with no
  face neighbour (m_e = 0) has gamma_e^Z = 0 (its only weight is its linear
  weight, and the printed quotient is 0/0).

Pins (tests/test_oracle_*.py): Gauss rules, Legendre polynomials, mass and
stiffness matrices and the semi-norm against closed forms; the operator, sensor
and wave speed against a brute-force evaluation of the integrals in physical
coordinates; conservation, zero sensor on reproduced data, symmetries; the
amplification polynomials of the three SSP methods (the Taylor coefficients of
exp up to their order), their orders in time against the exact propagator, and
the five-stage table's consistency and SSP coefficient 1.508; Table 1 and Table 2 of Sec. 5 (DG and LO
columns); the reverse mode against finite differences; the Zhao et al. sensor
is 0 on reproduced data, reaches 1 when one neighbour candidate takes all the
weight, lies in [0, 1] and is shift- and mirror-invariant; the KPP flux's
operator against the brute-force integrals (its LLF wave speed against a
search along the segment), and the three schemes on the KPP problem against
the solution ranges Sec. 5.5 prints; the exact solution of the
four-quadrant problem against its initial data, the integral conservation law
on boxes, the entropy condition, the invariant set [-1, 0.8] and a hand
derivation of its waves, and the operator with that exterior state against the
brute-force integrals.  The Hermite candidates
and nonlinear weights are a reading (the paper defers them to another
reference): against the paper's WENO columns they are parity unpinned, and only
the stated behaviour (optimal rates; WENO equal to DG with a threshold) is
checked.
"""

from __future__ import annotations

import dataclasses
import math
from fractions import Fraction
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

DTYPE = torch.float64

LINADV = 0   # F(u) = v(x) u, v(x) = (vx - omega (y - cy), vy + omega (x - cx))
BURGERS = 1  # F(u) = a u^2 / 2, a = (vx, vy)
KPP = 2      # F(u) = (sin u, cos u), the non-convex flux of Sec. 5.5 (2D)

MODE_DG, MODE_LO, MODE_WENO = 0, 1, 2   # labels of Sec. 5
MODE_ZHAO = 3   # the sensor of Zhao et al. that Sec. 5.6 compares with

BC_CONSTANT = 0   # non-periodic faces see the constant exterior state bc_value
BC_RIEMANN = 1    # ... see the exact solution of Sec. 5.4's four-quadrant problem

# Sec. 5.4: the initial states of the two-dimensional Burgers problem on the
# quadrants of the unit square (discontinuities on x = 1/2 and y = 1/2)
RIEMANN_NW, RIEMANN_NE, RIEMANN_SW, RIEMANN_SE = -0.2, -1.0, 0.5, 0.8


def burgers2d_riemann_exact(x, y, t: float) -> np.ndarray:
    """Entropy solution in R^2 of u_t + div(v u^2 / 2) = 0, v = (1, 1), from the
    four-quadrant data of Sec. 5.4, at points (x, y) and time t >= 0.

    With xi = x + y and c = x - y the equation reads u_t + (u^2)_xi = 0 on
    every line c = const, so each line carries a one-dimensional problem with
    the convex flux g(u) = u^2 and piecewise-constant data: south-west state
    for xi < 1 - |c|, then the south-east (c > 0) or north-west (c < 0)
    state, then the north-east state for xi > 1 + |c|.  Its entropy solution
    is the Lax-Oleinik formula (Evans, Partial Differential Equations,
    Sec. 3.4): u = (xi - y*) / (2t) where y* minimises
    U0(y) + (xi - y)^2 / (4t), U0 the integral of the data along the line
    (g* (q) = q^2 / 4 is the Legendre transform of g).  U0 is piecewise
    linear, so the minimiser is a break point or the stationary point
    y = xi - 2t u_k of one piece."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x, y = np.broadcast_arrays(x, y)
    if t <= 0.0:
        north = y > 0.5
        east = x > 0.5
        return np.where(north, np.where(east, RIEMANN_NE, RIEMANN_NW),
                        np.where(east, RIEMANN_SE, RIEMANN_SW))
    xi, c = x + y, x - y
    a, b = 1.0 - np.abs(c), 1.0 + np.abs(c)
    uA = np.full_like(xi, RIEMANN_SW)
    uB = np.where(c > 0.0, RIEMANN_SE, RIEMANN_NW)
    uC = np.full_like(xi, RIEMANN_NE)

    def U0(yy):
        return np.where(yy < a, uA * (yy - a),
                        np.where(yy <= b, uB * (yy - a), uB * (b - a) + uC * (yy - b)))

    inf = np.full_like(xi, np.inf)
    ys, vals = [], []
    for yy, ok in ((a, np.ones_like(xi, dtype=bool)), (b, np.ones_like(xi, dtype=bool)),
                   (xi - 2.0 * t * uA, xi - 2.0 * t * uA <= a),
                   (xi - 2.0 * t * uB, (xi - 2.0 * t * uB >= a) & (xi - 2.0 * t * uB <= b)),
                   (xi - 2.0 * t * uC, xi - 2.0 * t * uC >= b)):
        ys.append(yy)
        vals.append(np.where(ok, U0(yy) + (xi - yy) ** 2 / (4.0 * t), inf))
    best = np.argmin(np.stack(vals), axis=0)
    ystar = np.take_along_axis(np.stack(ys), best[None], axis=0)[0]
    # a stationary minimiser y* = xi - 2t u_k gives u = u_k: return the state
    # itself rather than (xi - y*)/(2t), which loses digits for small t
    return np.select([best == 2, best == 3, best == 4], [uA, uB, uC], (xi - ystar) / (2.0 * t))


# --------------------------------------------------------------------------
# Problem description
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """Scalar conservation law on a uniform Cartesian mesh of square cells.

    Sec. 2: U_t + div F(U) = 0 on Omega, U(.,0) = U_0; discretised with the
    broken space V_p (P_p in 1D, tensor Q_p in 2D).
    """
    dim: int = 1
    nx: int = 64
    ny: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    periodic_x: bool = True
    periodic_y: bool = True
    p: int = 2
    flux: int = LINADV
    vx: float = 1.0
    vy: float = 0.0
    omega: float = 0.0
    cx: float = 0.5
    cy: float = 0.5
    bc_value: float = 0.0
    bc_kind: int = BC_CONSTANT   # BC_RIEMANN: exterior state from the exact solution
    mode: int = MODE_WENO
    q: float = 1.0
    b: float = 0.0
    w_nb: float = 1e-2
    eps: float = 1e-6
    r: float = 2.0
    theta: float = 1.0   # exponent of the Zhao et al. sensor (mode MODE_ZHAO)
    rk_order: int = 3    # SSP Runge-Kutta order: 2, 3 (eq. ssp) or 4 (five stages)
    lambda_override: float = 0.0
    quad_vol: int = 0
    quad_face: int = 0
    quad_proj: int = 0

    # -- derived ---------------------------------------------------------
    @property
    def n1(self) -> int:
        return self.p + 1

    @property
    def nloc(self) -> int:
        return self.n1 ** self.dim

    @property
    def ncells(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)

    @property
    def h(self) -> float:
        return (self.x1 - self.x0) / self.nx

    def validate(self) -> None:
        if self.dim not in (1, 2):
            raise ValueError("dim must be 1 or 2")
        if not 1 <= self.p <= 4:
            raise ValueError("p must be in 1..4")
        if self.nx < 1 or (self.dim == 2 and self.ny < 1):
            raise ValueError("empty mesh")
        if self.dim == 2:
            hy = (self.y1 - self.y0) / self.ny
            if abs(hy - self.h) > 1e-12 * abs(self.h):
                raise ValueError("2D cells must be square")
        if self.flux == KPP and self.dim != 2:
            raise ValueError("the KPP flux is two-dimensional")
        if self.bc_kind == BC_RIEMANN and not (self.dim == 2 and self.flux == BURGERS):
            raise ValueError("the four-quadrant exterior state belongs to 2D Burgers")

    def qv(self) -> int:
        """Volume Gauss points per axis (exact for the polynomial part)."""
        if self.quad_vol:
            return self.quad_vol
        if self.flux == LINADV:
            return self.p + 1
        if self.flux == KPP:
            return self.p + 2
        if self.dim == 1:
            return -(-3 * self.p // 2)
        return -(-(3 * self.p + 1) // 2)

    def qf(self) -> int:
        if self.quad_face:
            return self.quad_face
        return self.qv()

    def qp(self) -> int:
        return self.quad_proj if self.quad_proj else self.p + 2


# --------------------------------------------------------------------------
# One-dimensional building blocks, from their definitions
# --------------------------------------------------------------------------
def legendre_poly(a: int) -> List[Fraction]:
    """Monomial coefficients of the Legendre polynomial P_a (Bonnet recursion
    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}), exact rationals."""
    prev, cur = [Fraction(1)], [Fraction(0), Fraction(1)]
    if a == 0:
        return prev
    for k in range(1, a):
        nxt = [Fraction(0)] * (k + 2)
        for i, c in enumerate(cur):
            nxt[i + 1] += Fraction(2 * k + 1, k + 1) * c
        for i, c in enumerate(prev):
            nxt[i] -= Fraction(k, k + 1) * c
        prev, cur = cur, nxt
    return cur


def poly_deriv(c: Sequence[Fraction], k: int = 1) -> List[Fraction]:
    c = list(c)
    for _ in range(k):
        c = [i * c[i] for i in range(1, len(c))] or [Fraction(0)]
    return c


def poly_eval(c: Sequence[Fraction], x: torch.Tensor) -> torch.Tensor:
    out = torch.zeros_like(x)
    for coef in reversed(c):
        out = out * x + float(coef)
    return out


def gauss_legendre(Q: int) -> Tuple[torch.Tensor, torch.Tensor]:
    """Gauss-Legendre nodes/weights on [-1,1]: roots of P_Q by Newton's
    method, weights 2 / ((1 - x^2) P_Q'(x)^2)."""
    xs, ws = [], []
    for i in range(Q):
        x = math.cos(math.pi * (i + 0.75) / (Q + 0.5))
        for _ in range(100):
            p0, p1 = 1.0, x
            for k in range(2, Q + 1):
                p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
            if Q == 1:
                p0, p1 = 1.0, x
            dp = Q * (x * p1 - p0) / (x * x - 1.0)
            dx = p1 / dp
            x -= dx
            if abs(dx) < 1e-17:
                break
        p0, p1 = 1.0, x
        for k in range(2, Q + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = Q * (x * p1 - p0) / (x * x - 1.0)
        xs.append(x)
        ws.append(2.0 / ((1.0 - x * x) * dp * dp))
    order = sorted(range(Q), key=lambda i: xs[i])
    return (torch.tensor([xs[i] for i in order], dtype=DTYPE),
            torch.tensor([ws[i] for i in order], dtype=DTYPE))


# --------------------------------------------------------------------------
# Basis on the reference cell [-1,1]^d
# --------------------------------------------------------------------------
class Basis:
    """phi_j(xi) = prod_i P_{a_i}(xi_i) with j = a_0 + (p+1) a_1 (x fastest)."""

    def __init__(self, dim: int, p: int):
        self.dim, self.p, self.n1 = dim, p, p + 1
        self.modes = [(j % self.n1, j // self.n1) if dim == 2 else (j,)
                      for j in range(self.n1 ** dim)]
        self.polys = [legendre_poly(a) for a in range(self.n1)]

    def eval(self, pts: torch.Tensor, k: Sequence[int] = None) -> torch.Tensor:
        """D^k phi_j at reference points pts [N, d] -> [N, nloc]."""
        if k is None:
            k = (0,) * self.dim
        cols = []
        for mode in self.modes:
            v = torch.ones(pts.shape[0], dtype=DTYPE)
            for ax in range(self.dim):
                v = v * poly_eval(poly_deriv(self.polys[mode[ax]], k[ax]), pts[:, ax])
            cols.append(v)
        return torch.stack(cols, dim=1)


def tensor_rule(dim: int, Q: int) -> Tuple[torch.Tensor, torch.Tensor]:
    """Tensor Gauss rule on [-1,1]^d: points [Q^d, d] (x fastest), weights."""
    x, w = gauss_legendre(Q)
    if dim == 1:
        return x[:, None].clone(), w.clone()
    X = x.repeat(Q)                 # x fastest
    Y = x.repeat_interleave(Q)
    W = w.repeat(Q) * w.repeat_interleave(Q)
    return torch.stack([X, Y], dim=1), W


def face_rule(dim: int, Q: int, axis: int, side: int):
    """Points on the face xi_axis = side of [-1,1]^d and their weights."""
    if dim == 1:
        return torch.tensor([[float(side)]], dtype=DTYPE), torch.ones(1, dtype=DTYPE)
    t, w = gauss_legendre(Q)
    pts = torch.empty(Q, 2, dtype=DTYPE)
    pts[:, axis] = float(side)
    pts[:, 1 - axis] = t
    return pts, w


def multi_indices(dim: int, p: int) -> List[Tuple[int, ...]]:
    """The index set 1 <= |k| <= p of the scaled Sobolev semi-norm (Sec. 4)."""
    if dim == 1:
        return [(k,) for k in range(1, p + 1)]
    return [(k1, s - k1) for s in range(1, p + 1) for k1 in range(s, -1, -1)]


# --------------------------------------------------------------------------
# The discretisation
# --------------------------------------------------------------------------
class Oracle:
    """Plain evaluation of the paper's semi-discrete operator and time step."""

    def __init__(self, prob: Problem):
        prob.validate()
        self.P = P = prob
        d, p = P.dim, P.p
        self.basis = B = Basis(d, p)
        h = P.h
        self.h = h
        self.J = (h / 2.0) ** d            # dx = J dxi
        self.Jf = (h / 2.0) ** (d - 1)     # ds = Jf ds_ref
        self.g = 2.0 / h                   # d/dx = g d/dxi

        # volume rule
        self.vpts, self.vw = tensor_rule(d, P.qv())
        self.V = B.eval(self.vpts)
        self.DV = [B.eval(self.vpts, tuple(1 if i == ax else 0 for i in range(d)))
                   for ax in range(d)]
        # faces: (axis, side) for side in (-1, +1)
        self.faces = [(ax, s) for ax in range(d) for s in (-1, 1)]
        self.fpts, self.fw, self.FV, self.FVopp = [], [], [], []
        for ax, s in self.faces:
            pts, w = face_rule(d, P.qf(), ax, s)
            opp = pts.clone()
            opp[:, ax] = -float(s)      # the same physical points seen from the neighbour
            self.fpts.append(pts)
            self.fw.append(w)
            self.FV.append(B.eval(pts))
            self.FVopp.append(B.eval(opp))

        # exact rule (p+1 points per axis) for mass, stiffness, projections of
        # continued neighbour polynomials and the semi-norm
        self.epts, self.ew = tensor_rule(d, p + 1)
        E = B.eval(self.epts)
        self.M = self.J * (E.T * self.ew) @ E                     # int phi_i phi_j dx
        self.Minv = torch.linalg.inv(self.M)
        DE = [B.eval(self.epts, tuple(1 if i == ax else 0 for i in range(d)))
              for ax in range(d)]
        self.K = sum(self.J * self.g ** 2 * (D.T * self.ew) @ D for D in DE)  # int grad.grad
        # continuation of the side-s neighbour along `axis` into this cell:
        # u_nb(xi - 2 s e_axis) projected onto V_p with the exact rule
        Mref = (E.T * self.ew) @ E
        self.cont = {}
        for ax, s in self.faces:
            shifted = self.epts.clone()
            shifted[:, ax] -= 2.0 * s
            Es = B.eval(shifted)
            self.cont[(ax, s)] = torch.linalg.solve(Mref, (E.T * self.ew) @ Es)
        # semi-norm: D^k phi at the exact nodes and the physical scale factors
        self.sn_terms = []
        for k in multi_indices(d, p):
            kk = sum(k)
            scale = h ** (2 * kk - d) * self.g ** (2 * kk) * self.J
            self.sn_terms.append((scale, B.eval(self.epts, k)))

        # mesh geometry and face-neighbour table (-1 = no neighbour)
        ny = P.ny if d == 2 else 1
        ix = torch.arange(P.nx).repeat(ny)
        iy = torch.arange(ny).repeat_interleave(P.nx)
        self.xc = P.x0 + (ix.to(DTYPE) + 0.5) * h
        self.yc = P.y0 + (iy.to(DTYPE) + 0.5) * h
        self.nbr = []
        for ax, s in self.faces:
            if ax == 0:
                jx, jy, n, per = ix + s, iy, P.nx, P.periodic_x
                j = jx
            else:
                jx, jy, n, per = ix, iy + s, ny, P.periodic_y
                j = jy
            if per:
                jx, jy = jx % P.nx, jy % ny
                idx = jx + P.nx * jy
            else:
                idx = torch.where((j >= 0) & (j < n), jx + P.nx * jy,
                                  torch.full_like(jx, -1))
            self.nbr.append(idx)

    # ------------------------------------------------------------------
    def phys(self, ref: torch.Tensor):
        """Physical coordinates [E, N] of reference points ref [N, d]."""
        x = self.xc[:, None] + 0.5 * self.h * ref[None, :, 0]
        if self.P.dim == 1:
            return x, None
        y = self.yc[:, None] + 0.5 * self.h * ref[None, :, 1]
        return x, y

    def velocity(self, x, y):
        """v(x) of the linear flux; (a_x, a_y) direction of the Burgers flux."""
        P = self.P
        if P.dim == 1:
            return (torch.full_like(x, P.vx),)
        vx = P.vx - P.omega * (y - P.cy)
        vy = P.vy + P.omega * (x - P.cx)
        return vx, vy

    def flux(self, u, x, y):
        """Components of F(u) at points."""
        P = self.P
        if P.flux == LINADV:
            return [v * u for v in self.velocity(x, y)]
        if P.flux == KPP:
            return [torch.sin(u), torch.cos(u)]
        a = (P.vx,) if P.dim == 1 else (P.vx, P.vy)
        return [ai * 0.5 * u * u for ai in a]

    def dflux(self, u, x, y):
        """Components of F'(u) at points."""
        P = self.P
        if P.flux == LINADV:
            return [v + 0.0 * u for v in self.velocity(x, y)]
        if P.flux == KPP:
            return [torch.cos(u), -torch.sin(u)]
        a = (P.vx,) if P.dim == 1 else (P.vx, P.vy)
        return [ai * u for ai in a]

    def llf(self, um, up, axis, side, x, y):
        """Local Lax-Friedrichs flux H(U^-, U^+, n), n = side * e_axis (Sec. 2).
        For the linear and Burgers fluxes F'(w U^- + (1-w) U^+) . n is affine
        in w, so the maximum of its modulus over [0,1] is attained at an end
        point.  For KPP it is |cos w| (x faces) or |sin w| (y faces) for w
        between the two states: 1 where that interval holds a point k pi (x)
        or pi/2 + k pi (y), else the larger end value (|cos| and |sin| fall
        and rise between consecutive such points)."""
        Fm = self.flux(um, x, y)[axis] * side
        Fp = self.flux(up, x, y)[axis] * side
        sm = torch.abs(self.dflux(um, x, y)[axis] * side)
        sp = torch.abs(self.dflux(up, x, y)[axis] * side)
        s_plus = torch.maximum(sm, sp)
        if self.P.flux == KPP:
            lo, hi = torch.minimum(um, up), torch.maximum(um, up)
            shift = 0.0 if axis == 0 else 0.5 * math.pi
            peak = torch.floor((hi - shift) / math.pi) >= torch.ceil((lo - shift) / math.pi)
            s_plus = torch.where(peak, torch.ones_like(s_plus), s_plus)
        return 0.5 * (Fm + Fp) - 0.5 * s_plus * (up - um)

    # ------------------------------------------------------------------
    def exterior(self, xf: torch.Tensor, yf: torch.Tensor, t: float) -> torch.Tensor:
        """The state outside a non-periodic boundary at the face points: the
        constant bc_value, or the exact solution at time t (Sec. 5.4 sets its
        inflow data from the exact solution; here every boundary face takes
        its values at the face Gauss points)."""
        if self.P.bc_kind == BC_RIEMANN:
            return torch.from_numpy(burgers2d_riemann_exact(xf.numpy(), yf.numpy(), t))
        return torch.full(xf.shape, self.P.bc_value, dtype=DTYPE)

    def galerkin_residual(self, U: torch.Tensor, t: float = 0.0) -> torch.Tensor:
        """R(U) of eq. (weak2) at time t (the time enters through the exterior
        state only): volume term minus face-flux term."""
        P, d = self.P, self.P.dim
        x, y = self.phys(self.vpts)
        uq = U @ self.V.T
        F = self.flux(uq, x, y)
        R = torch.zeros_like(U)
        for ax in range(d):
            R = R + self.J * self.g * (F[ax] * self.vw) @ self.DV[ax]
        for f, (ax, s) in enumerate(self.faces):
            xf, yf = self.phys(self.fpts[f])
            um = U @ self.FV[f].T
            nb = self.nbr[f]
            has = nb >= 0
            Unb = U[nb.clamp(min=0)]
            up_in = Unb @ self.FVopp[f].T
            up = torch.where(has[:, None], up_in, self.exterior(xf, yf, t).expand_as(up_in))
            H = self.llf(um, up, ax, s, xf, yf)
            R = R - self.Jf * (H * self.fw[f]) @ self.FV[f]
        return R

    def seminorm2(self, C: torch.Tensor) -> torch.Tensor:
        """||v||_e^2 for coefficient rows C [..., nloc] (Sec. 4)."""
        out = torch.zeros(C.shape[:-1], dtype=DTYPE)
        for scale, Dk in self.sn_terms:
            vals = C @ Dk.T
            out = out + scale * (vals * vals * self.ew).sum(-1)
        return out

    def candidates(self, U: torch.Tensor):
        """Hermite candidates U_l (l = 0 own, then one per face): [E, 1+2d, nloc]
        and a mask of which exist."""
        P = self.P
        cands, exists = [U], [torch.ones(U.shape[0], dtype=torch.bool)]
        for f, (ax, s) in enumerate(self.faces):
            nb = self.nbr[f]
            has = nb >= 0
            Cl = U[nb.clamp(min=0)] @ self.cont[(ax, s)].T
            Cl = torch.cat([U[:, :1], Cl[:, 1:]], dim=1)   # mean := own mean
            cands.append(Cl)
            exists.append(has)
        return torch.stack(cands, dim=1), torch.stack(exists, dim=1)

    def sensor(self, U: torch.Tensor, details: bool = False):
        """gamma_e of eqs. (sensor)/(gensensor) with the HWENO reconstruction."""
        P = self.P
        C, ex = self.candidates(U)
        m_e = ex[:, 1:].sum(1).to(DTYPE)
        lin = torch.full(ex.shape, P.w_nb, dtype=DTYPE)
        lin[:, 0] = 1.0 - m_e * P.w_nb
        beta = self.seminorm2(C)
        alpha = torch.where(ex, lin / (P.eps + beta) ** P.r, torch.zeros_like(beta))
        omega = alpha / alpha.sum(1, keepdim=True)
        Ustar = (omega[:, :, None] * C).sum(1)
        num2 = self.seminorm2(U - Ustar)
        den2 = beta[:, 0]
        one = torch.ones_like(num2)
        # square roots taken only of positive arguments (keeps reverse mode finite)
        num = torch.sqrt(torch.where(num2 > 0, num2, one))
        den = torch.sqrt(torch.where(den2 > 0, den2, one))
        ratio = torch.where(num2 > 0,
                            torch.where(den2 > 0, num / den, torch.full_like(num, math.inf)),
                            torch.zeros_like(num2))
        gam = torch.clamp(ratio, max=1.0) ** P.q
        gam = torch.where(ratio >= P.b, gam, torch.zeros_like(gam))
        if details:
            return gam, dict(beta=beta, omega=omega, ratio=ratio, Ustar=Ustar,
                             cands=C, exists=ex, lin=lin)
        return gam

    def zhao_sensor(self, U: torch.Tensor) -> torch.Tensor:
        """gamma_e^Z (Sec. 5.6, the sensor of Zhao et al.): the deviation of the
        nonlinear HWENO weights from the linear weights,
            sum_l |omega_l / omega~_l - 1|^theta / (|1 / min_l omega~_l - 1|^theta + m_e),
        sums and minimum over the candidates that exist; 0 where m_e = 0."""
        P = self.P
        _, d = self.sensor(U, details=True)
        omega, lin, ex = d["omega"], d["lin"], d["exists"]
        m_e = ex[:, 1:].sum(1).to(DTYPE)
        dev = torch.where(ex, torch.abs(omega / lin - 1.0) ** P.theta, torch.zeros_like(omega)).sum(1)
        lmin = torch.where(ex, lin, torch.full_like(lin, math.inf)).amin(1)
        den = torch.abs(1.0 / lmin - 1.0) ** P.theta + m_e
        return torch.where(m_e > 0, dev / torch.where(m_e > 0, den, torch.ones_like(den)), torch.zeros_like(dev))

    def gamma(self, U: torch.Tensor) -> torch.Tensor:
        P = self.P
        if P.mode == MODE_DG:
            return torch.zeros(U.shape[0], dtype=DTYPE)
        if P.mode == MODE_LO:
            return torch.ones(U.shape[0], dtype=DTYPE)
        if P.mode == MODE_ZHAO:
            return self.zhao_sensor(U)
        return self.sensor(U)

    def max_speed(self, U: torch.Tensor) -> torch.Tensor:
        """lambda_e = max over the volume nodes of ||F'(u_h)||_2 (eq. visc)."""
        P = self.P
        if P.lambda_override > 0:
            return torch.full((U.shape[0],), P.lambda_override, dtype=DTYPE)
        x, y = self.phys(self.vpts)
        dF = self.dflux(U @ self.V.T, x, y)
        if len(dF) == 1:
            return torch.abs(dF[0]).amax(dim=1)
        n2 = sum(c * c for c in dF)
        pos = n2 > 0
        return torch.where(pos, torch.sqrt(torch.where(pos, n2, torch.ones_like(n2))),
                           torch.zeros_like(n2)).amax(dim=1)

    def dissipation(self, U: torch.Tensor, gam=None) -> torch.Tensor:
        """s_i = gamma_e nu_e int grad(phi_i) . grad(U_h) (eqs. visc, astab)."""
        if gam is None:
            gam = self.gamma(U)
        nu = self.max_speed(U) * self.h / (2.0 * self.P.p)
        return (gam * nu)[:, None] * (U @ self.K.T)

    def rhs(self, U: torch.Tensor, with_gamma: bool = False, t: float = 0.0):
        """dU/dt = M^{-1} (R(U) - s(U)) at time t."""
        gam = self.gamma(U)
        L = (self.galerkin_residual(U, t) - self.dissipation(U, gam)) @ self.Minv.T
        return (L, gam) if with_gamma else L

    # Shu-Osher coefficients of the five-stage fourth-order SSP Runge-Kutta
    # method of Spiteri and Ruuth (as tabulated by Gottlieb, Ketcheson and Shu):
    # U_k = sum_j (alpha_kj U_j + beta_kj dt L(U_j)), rows k = 1..5 over j = 0..4
    SSP54_ALPHA = ((1.0,),
                   (0.444370493651235, 0.555629506348765),
                   (0.620101851488403, 0.0, 0.379898148511597),
                   (0.178079954393132, 0.0, 0.0, 0.821920045606868),
                   (0.0, 0.0, 0.517231671970585, 0.096059710526147, 0.386708617503269))
    SSP54_BETA = ((0.391752226571890,),
                  (0.0, 0.368410593050371),
                  (0.0, 0.0, 0.251891774271694),
                  (0.0, 0.0, 0.0, 0.544974750228521),
                  (0.0, 0.0, 0.0, 0.063692468666290, 0.226007483236906))

    def step(self, U: torch.Tensor, dt: float, t: float = 0.0) -> torch.Tensor:
        """One SSP Runge-Kutta step of the problem's order from time t: eq.
        (ssp), the optimal third-order method (the default); the second-order
        one; or the five-stage fourth-order one (Sec. 5.1 runs SSP methods of
        order p + 1 for its convergence study).  Each stage's operator is
        taken at the time of its input state, the same combination applied to
        t' = 1 (third order: t, t + dt, t + dt/2)."""
        k = self.P.rk_order
        if k == 2:
            U1 = U + dt * self.rhs(U, t=t)
            return 0.5 * U + 0.5 * U1 + 0.5 * dt * self.rhs(U1, t=t + dt)
        if k == 4:
            stages, times = [U], [t]
            Ls = [self.rhs(U, t=t)]
            for row_a, row_b in zip(self.SSP54_ALPHA, self.SSP54_BETA):
                Uk = sum(a * Uj for a, Uj in zip(row_a, stages) if a != 0.0)
                Uk = Uk + sum(b * dt * Lj for b, Lj in zip(row_b, Ls) if b != 0.0)
                tk = sum(a * tj for a, tj in zip(row_a, times)) + sum(row_b) * dt
                stages.append(Uk)
                times.append(tk)
                if len(stages) <= 5:
                    Ls.append(self.rhs(Uk, t=tk))
            return stages[-1]
        U1 = U + dt * self.rhs(U, t=t)
        U2 = 0.75 * U + 0.25 * U1 + 0.25 * dt * self.rhs(U1, t=t + dt)
        return U / 3.0 + (2.0 / 3.0) * U2 + (2.0 / 3.0) * dt * self.rhs(U2, t=t + 0.5 * dt)

    def run(self, U: torch.Tensor, dt: float, nsteps: int, t0: float = 0.0) -> torch.Tensor:
        """nsteps steps from time t0; step n starts at t0 + n dt."""
        for n in range(nsteps):
            U = self.step(U, dt, t0 + n * dt)
        return U

    # ------------------------------------------------------------------
    def nodes(self, Q: int) -> torch.Tensor:
        """Physical coordinates [E, Q^d, d] of the Q-point tensor Gauss nodes."""
        ref, _ = tensor_rule(self.P.dim, Q)
        x, y = self.phys(ref)
        return x[..., None] if y is None else torch.stack([x, y], dim=-1)

    def proj_nodes(self) -> torch.Tensor:
        return self.nodes(self.P.qp())

    def project(self, u_at_nodes: torch.Tensor, Q: Optional[int] = None) -> torch.Tensor:
        """L2 projection c = M^{-1} int phi u0 dx with the Q-point rule."""
        Q = Q or self.P.qp()
        ref, w = tensor_rule(self.P.dim, Q)
        Phi = self.basis.eval(ref)
        b = self.J * (u_at_nodes * w) @ Phi
        return b @ self.Minv.T

    def evaluate(self, U: torch.Tensor, Q: int):
        """u_h at the Q-point nodes of every cell, and the node weights (dx)."""
        ref, w = tensor_rule(self.P.dim, Q)
        return U @ self.basis.eval(ref).T, self.J * w

    def l1_error(self, U: torch.Tensor, exact_at_nodes: torch.Tensor, Q: int) -> float:
        uh, w = self.evaluate(U, Q)
        return float((torch.abs(uh - exact_at_nodes) * w).sum())

    def mass(self, U: torch.Tensor) -> float:
        """int u_h dx over the mesh."""
        uh, w = self.evaluate(U, self.P.p + 1)
        return float((uh * w).sum())

    def window_functional(self, U: torch.Tensor, wx: Tuple[float, float],
                          wy: Tuple[float, float]) -> torch.Tensor:
        """J(U) = int_W u_h^2 dx over an axis-aligned window W made of whole cells."""
        uh, w = self.evaluate(U, self.P.p + 1)
        inside = (self.xc > wx[0]) & (self.xc < wx[1])
        if self.P.dim == 2:
            inside = inside & (self.yc > wy[0]) & (self.yc < wy[1])
        return ((uh * uh * w).sum(1) * inside.to(DTYPE)).sum()

    # ------------------------------------------------------------------
    def step_vjp(self, U: torch.Tensor, dt: float, lam: torch.Tensor) -> torch.Tensor:
        """Discrete adjoint of one step: (d step / d U)^T lam, by reverse-mode
        differentiation of `step` (exact up to rounding)."""
        Ur = U.detach().clone().requires_grad_(True)
        out = self.step(Ur, dt)
        (g,) = torch.autograd.grad(out, Ur, lam)
        return g

    def run_grad(self, U0: torch.Tensor, dt: float, nsteps: int, objective) -> torch.Tensor:
        """Gradient of objective(U^N) with respect to U^0 (reverse mode)."""
        Ur = U0.detach().clone().requires_grad_(True)
        Jv = objective(self.run(Ur, dt, nsteps))
        (g,) = torch.autograd.grad(Jv, Ur)
        return g
