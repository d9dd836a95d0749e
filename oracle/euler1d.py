"""CPU oracle for the one-dimensional Euler equations of Sec. 5.6.

TEST INFRASTRUCTURE ONLY (like dgoracle, which it builds on): the plain
reference the HIP library's Euler path is checked against.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may use it.

What is computed (FP64, PyTorch CPU ops, vectorised over cells):

* Sec. 5.6: U = (rho, rho v, rho E), F(U) = (rho v, rho v^2 + p, (rho E + p) v),
  p = (gamma - 1) (rho E - rho v^2 / 2), gamma = 1.4.
* Sec. 2, eq. (weak2), component by component with the LLF flux
  H = (F(U^-) + F(U^+)) . n / 2 - s^+ (U^+ - U^-) / 2.
* Sec. 3, eqs. (visc), (astab): s_i = gamma_e nu_e int phi_i' U_h' dx for every
  component, nu_e = lambda_e h / (2p).
* Sec. 4 and Sec. 5.6: gamma_e from the density alone (the scalar sensor of
  eqs. (sensor)/(gensensor), or that of Zhao et al., applied to the density
  coefficients), the same gamma_e for all three components.
* eq. (ssp): the three-stage SSP Runge-Kutta step.

Readings where the paper is silent:
* s^+ = max(|v^-| + c^-, |v^+| + c^+), c = sqrt(gamma p / rho): the larger
  spectral radius of F'(U) at the two states (the scalar s^+ of Sec. 2 is the
  maximum of |F'| between the states; for the system the bound at the two
  states is taken).
* lambda_e = max over the volume Gauss nodes of |v| + c.
* Quadrature: p + 2 Gauss points (the flux is rational in U).
* Reflecting walls (Sod's tube of Sec. 5.6): the exterior state at a wall is
  the mirror state (rho, -rho v, rho E) through the same LLF flux; a wall is
  no face neighbour for the sensor's stencil.

Pins (tests/test_oracle_euler.py): the wave speed against the eigenvalues of
the flux Jacobian, a state at rest is steady, walls conserve mass and energy,
mirror symmetry, the operator against brute-force integrals in physical
coordinates, and the Sod problem against its exact solution (whose star state
is checked against the Rankine-Hugoniot conditions and the Riemann
invariants).
"""

from __future__ import annotations

import dataclasses

import torch

from .dgoracle import DTYPE, LINADV, MODE_WENO, Oracle, Problem

GAMMA = 1.4


@dataclasses.dataclass
class EulerProblem:
    nx: int = 128
    p: int = 2
    x0: float = 0.0
    x1: float = 1.0
    walls: bool = True          # reflecting walls at both ends (else periodic)
    mode: int = MODE_WENO       # sensor on the density: DG, LO, WENO, ZHAO
    q: float = 1.0
    b: float = 0.0
    w_nb: float = 1e-2
    eps: float = 1e-6
    r: float = 2.0
    theta: float = 1.0
    lambda_override: float = 0.0


def pressure(U: torch.Tensor) -> torch.Tensor:
    """p = (gamma - 1)(rho E - (rho v)^2 / (2 rho)); components on axis 1."""
    rho, m, E = U[:, 0], U[:, 1], U[:, 2]
    return (GAMMA - 1.0) * (E - 0.5 * m * m / rho)


def flux(U: torch.Tensor) -> torch.Tensor:
    """F(U) of Sec. 5.6 (components on axis 1)."""
    rho, m, E = U[:, 0], U[:, 1], U[:, 2]
    v = m / rho
    p = pressure(U)
    return torch.stack([m, m * v + p, (E + p) * v], dim=1)


def wave_speed(U: torch.Tensor) -> torch.Tensor:
    """|v| + c, c = sqrt(gamma p / rho)."""
    rho = U[:, 0]
    return torch.abs(U[:, 1] / rho) + torch.sqrt(GAMMA * pressure(U) / rho)


def conserved(rho, v, p):
    """(rho, rho v, rho E) from the primitive variables."""
    return torch.stack([rho, rho * v, p / (GAMMA - 1.0) + 0.5 * rho * v * v], dim=1)


class EulerOracle:
    """The semi-discrete Euler operator; U has shape [cells, 3, p + 1]."""

    def __init__(self, P: EulerProblem):
        self.P = P
        Q = P.p + 2
        sp = Problem(dim=1, nx=P.nx, x0=P.x0, x1=P.x1, periodic_x=not P.walls, p=P.p, flux=LINADV,
                     mode=P.mode, q=P.q, b=P.b, w_nb=P.w_nb, eps=P.eps, r=P.r, theta=P.theta,
                     quad_vol=Q, quad_face=Q)
        # basis, rules, mass and stiffness matrices, neighbour table, sensor
        self.S = Oracle(sp)
        self.h = self.S.h

    def max_speed(self, U: torch.Tensor) -> torch.Tensor:
        """lambda_e = max over the volume nodes of |v| + c (or the override)."""
        if self.P.lambda_override > 0:
            return torch.full((U.shape[0],), self.P.lambda_override, dtype=DTYPE)
        uq = U @ self.S.V.T                                   # [E, 3, Q]
        return wave_speed(uq).amax(dim=1)

    def llf(self, um: torch.Tensor, up: torch.Tensor, side: float) -> torch.Tensor:
        """H . n for the outward normal n = side, at face points [E, 3, 1]."""
        s = torch.maximum(wave_speed(um), wave_speed(up))[:, None]
        return 0.5 * side * (flux(um) + flux(up)) - 0.5 * s * (up - um)

    def galerkin_residual(self, U: torch.Tensor) -> torch.Tensor:
        S = self.S
        uq = U @ S.V.T
        R = S.J * S.g * (flux(uq) * S.vw) @ S.DV[0]
        for f, (ax, side) in enumerate(S.faces):
            um = U @ S.FV[f].T                                # [E, 3, 1]
            nb = S.nbr[f]
            has = nb >= 0
            up = U[nb.clamp(min=0)] @ S.FVopp[f].T
            wall = um * torch.tensor([1.0, -1.0, 1.0], dtype=DTYPE)[None, :, None]
            up = torch.where(has[:, None, None], up, wall)
            R = R - S.Jf * (self.llf(um, up, float(side)) * S.fw[f]) @ S.FV[f]
        return R

    def gamma(self, U: torch.Tensor) -> torch.Tensor:
        """gamma_e from the density coefficients (Sec. 5.6)."""
        return self.S.gamma(U[:, 0, :])

    def rhs(self, U: torch.Tensor, with_gamma: bool = False):
        gam = self.gamma(U)
        nu = self.max_speed(U) * self.h / (2.0 * self.P.p)
        diss = (gam * nu)[:, None, None] * (U @ self.S.K.T)
        L = (self.galerkin_residual(U) - diss) @ self.S.Minv.T
        return (L, gam) if with_gamma else L

    def step(self, U: torch.Tensor, dt: float) -> torch.Tensor:
        """Eq. (ssp)."""
        U1 = U + dt * self.rhs(U)
        U2 = 0.75 * U + 0.25 * U1 + 0.25 * dt * self.rhs(U1)
        return U / 3.0 + (2.0 / 3.0) * U2 + (2.0 / 3.0) * dt * self.rhs(U2)

    def run(self, U: torch.Tensor, dt: float, nsteps: int) -> torch.Tensor:
        for _ in range(nsteps):
            U = self.step(U, dt)
        return U

    def project(self, ic) -> torch.Tensor:
        """L2 projection of initial data ic(x) -> conserved variables stacked
        on the axis before the last ([E, 3, Qp] for x of shape [E, Qp])."""
        x = self.S.proj_nodes()[..., 0]
        C = torch.as_tensor(ic(x.numpy()), dtype=DTYPE)        # [E, 3, Qp]
        return torch.stack([self.S.project(C[:, k]) for k in range(3)], dim=1)

    def evaluate(self, U: torch.Tensor, Q: int):
        """Conserved variables at the Q Gauss points of every cell [E, 3, Q]."""
        vals = [self.S.evaluate(U[:, k], Q)[0] for k in range(3)]
        return torch.stack(vals, dim=1)


def stable_dt(prob: EulerProblem, U: torch.Tensor, cfl: float) -> float:
    """dt = CFL h / ((2p + 1) max(|v| + c)) over the volume nodes of U."""
    O = EulerOracle(prob)
    return cfl * O.h / ((2 * prob.p + 1) * float(O.max_speed(U).max()))


__all__ = ["EulerProblem", "EulerOracle", "GAMMA", "flux", "pressure", "wave_speed", "conserved",
           "stable_dt"]
