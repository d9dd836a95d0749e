"""Seeded synthetic workloads: problem descriptions and initial data.

This module holds no arithmetic of the method itself.  It describes problems
(mesh, degree, flux, sensor settings, time step, step count) and evaluates
initial data at whatever points a caller provides.  The HIP binding and the CPU
oracle both consume it; neither is imported here.

Workload shapes follow the paper's scalar test problems (Sec. 5): 1D linear
advection of a smooth wave plus a square pulse, solid-body rotation of a smooth
hump and a slotted cylinder, and inviscid Burgers with smooth data that steepens
into shocks.  Random centres, radii, Fourier modes and problem mixes are drawn
from numpy's default_rng(seed).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

LINADV, BURGERS, KPP = 0, 1, 2
EULER = 3   # the 1D Euler equations of Sec. 5.6 (three conserved variables per point)
MODE_DG, MODE_LO, MODE_WENO = 0, 1, 2
MODE_ZHAO = 3   # the sensor of Zhao et al. compared in Sec. 5.6
BC_CONSTANT, BC_RIEMANN = 0, 1   # exterior state: bc_value, or Sec. 5.4's exact solution


@dataclasses.dataclass
class Workload:
    name: str = "adv1d"
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
    bc_kind: int = BC_CONSTANT
    mode: int = MODE_WENO
    q: float = 1.0
    b: float = 0.0
    w_nb: float = 1e-2
    eps: float = 1e-6
    r: float = 2.0
    theta: float = 1.0                 # exponent of the Zhao et al. sensor (MODE_ZHAO)
    rk_order: int = 3                  # SSP Runge-Kutta order: 2, 3 or 4
    lambda_override: float = 0.0
    cfl: float = 0.1
    steps: int = 100
    ic: Optional[Callable] = None      # ic(x) in 1D, ic(x, y) in 2D (numpy)
    umax: float = 1.0                  # bound on |u0| used for the time step
    t_end: Optional[float] = None      # end time (steps follow from dt where set)
    dt_value: Optional[float] = None   # a time step set by the caller (with_dt)

    @property
    def h(self) -> float:
        return (self.x1 - self.x0) / self.nx

    @property
    def ncells(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)

    @property
    def nloc(self) -> int:
        """Coefficients per cell: (p+1)^dim, times 3 for the Euler system."""
        return (self.p + 1) ** self.dim * (3 if self.flux == EULER else 1)

    @property
    def ndof(self) -> int:
        return self.ncells * self.nloc

    def max_speed(self) -> float:
        """Upper bound of ||F'(u)||_2 over the domain for the initial data."""
        if self.flux == LINADV:
            if self.dim == 1:
                return abs(self.vx)
            far = max(math.hypot(x - self.cx, y - self.cy)
                      for x in (self.x0, self.x1) for y in (self.y0, self.y1))
            return math.hypot(abs(self.vx), abs(self.vy)) + abs(self.omega) * far
        if self.flux == KPP:
            # ||F'(u)||_2 = 1; a larger lambda override also bounds the step
            return max(1.0, self.lambda_override)
        if self.flux == EULER:
            return self.umax     # a stated bound on |v| + c over the run
        a = abs(self.vx) if self.dim == 1 else math.hypot(self.vx, self.vy)
        return a * self.umax

    def dt(self) -> float:
        """Fixed step: the caller's (with_dt), else dt = CFL h / ((2p+1) max
        speed) with the stated bound of max_speed."""
        if self.dt_value is not None:
            return self.dt_value
        return self.cfl * self.h / ((2 * self.p + 1) * self.max_speed())

    def with_dt(self, dt: float) -> "Workload":
        """Run with the time step dt (for instance CFL h / ((2p+1) lambda_max)
        of the projected initial state, as the library's dg_stable_dt gives
        it); a workload with an end time then takes ceil(t_end / dt) steps."""
        self.dt_value = float(dt)
        if self.t_end is not None:
            self.steps = int(math.ceil(self.t_end / self.dt_value))
        return self

    def fields(self) -> dict:
        """Plain field dictionary (everything but the initial-data callable)."""
        d = dataclasses.asdict(self)
        d.pop("ic")
        return d

    def eval_ic(self, pts):
        """Initial data at points pts [..., dim] (numpy array or torch tensor)."""
        if isinstance(pts, (list, tuple)) or (hasattr(pts, "dtype") and not hasattr(pts, "is_cuda")):
            pts = np.asarray(pts, dtype=np.float64)
        if self.dim == 1:
            return self.ic(pts[..., 0])
        return self.ic(pts[..., 0], pts[..., 1])


# ---------------------------------------------------------------------------
# initial data (numpy arrays, or torch tensors for evaluation on the device)
# ---------------------------------------------------------------------------
class _Ops:
    """The few array operations the initial data need, for numpy or torch."""

    def __init__(self, x):
        import sys
        torch = sys.modules.get("torch")
        self.t = torch is not None and isinstance(x, torch.Tensor)
        self.m = torch if self.t else np

    def where(self, c, a, b):
        if self.t:
            a = a if isinstance(a, self.m.Tensor) else self.m.full_like(c, a, dtype=self.m.float64)
            b = b if isinstance(b, self.m.Tensor) else self.m.full_like(c, b, dtype=self.m.float64)
        return self.m.where(c, a, b)

    def fl(self, c):
        return c.to(self.m.float64) if self.t else c.astype(np.float64)


def sin_plus_pulse(x):
    """sin(2 pi x) plus a unit square pulse on [0.3, 0.5]."""
    o = _Ops(x)
    return o.m.sin(2 * np.pi * x) + o.fl((x >= 0.3) & (x <= 0.5))


def cos_wave(x):
    """cos(2 pi (x - 0.5)), the smooth advection datum of Sec. 5.1."""
    return _Ops(x).m.cos(2 * np.pi * (x - 0.5))


def sin_wave(x):
    """sin(2 pi x), the Burgers datum of Sec. 5.2."""
    return _Ops(x).m.sin(2 * np.pi * x)


def square_and_bump(x):
    """Square wave on [0.15, 0.45] and a cos^2 bump on (0.55, 0.85) (Sec. 5.1)."""
    x = np.asarray(x)
    sq = ((x >= 0.15) & (x <= 0.45)).astype(np.float64)
    bump = np.where((x > 0.55) & (x < 0.85), np.cos(10 * np.pi / 3 * (x - 0.7)) ** 2, 0.0)
    return sq + bump


class HumpAndCylinder:
    """A smooth cosine hump and a slotted cylinder with seeded centres and radii.

    Hump: (1 + cos(pi rho / r)) / 4 for rho <= r.  Cylinder: height 1, a slot of
    half-width r/6 cut from the side facing the domain centre up to 2r/3 past
    the cylinder centre (the paper's shape, Sec. 5.3, scaled by r/0.15).
    Radii uniform in [0.1, 0.2]; centres at polar radius in [0.15, 0.48 - r]
    about (0.5, 0.5), non-overlapping (rejection sampling)."""

    def __init__(self, seed: int):
        rng = np.random.default_rng(seed)
        while True:
            shapes = []
            for _ in range(2):
                r = rng.uniform(0.1, 0.2)
                rad = rng.uniform(0.15, 0.48 - r)
                ang = rng.uniform(0.0, 2 * np.pi)
                shapes.append((0.5 + rad * np.cos(ang), 0.5 + rad * np.sin(ang), r))
            (x1, y1, r1), (x2, y2, r2) = shapes
            if math.hypot(x1 - x2, y1 - y2) > r1 + r2 + 1e-3:
                break
        self.hump, self.cyl = shapes

    def __call__(self, x, y):
        o = _Ops(x)
        m = o.m
        hx, hy, hr = self.hump
        rho = m.hypot(x - hx, y - hy)
        u = o.where(rho <= hr, 0.25 * (1 + m.cos(np.pi * rho / hr)), 0.0)
        cx, cy, cr = self.cyl
        ox, oy = cx - 0.5, cy - 0.5
        on = math.hypot(ox, oy)
        ex, ey = ox / on, oy / on                 # outward radial unit vector
        s = (x - cx) * ex + (y - cy) * ey         # along the radial direction
        t = -(x - cx) * ey + (y - cy) * ex        # across it
        inside = m.hypot(x - cx, y - cy) <= cr
        slot = (m.abs(t) < cr / 6) & (s < 2 * cr / 3)
        return u + o.fl(inside & ~slot)


def kpp_disc(x, y):
    """7 pi / 2 on the unit disc about the origin, pi / 4 outside (Sec. 5.5)."""
    o = _Ops(x)
    return o.where(x * x + y * y <= 1.0, 3.5 * np.pi, 0.25 * np.pi)


class FourierModes:
    """u0 = sum_j a_j cos(2 pi k_j . x + phi_j): 16 modes, integer wave vectors
    with 1 <= |k| <= 8 drawn uniformly, a_j ~ N(0,1)/|k_j|^2, phi_j ~ U[0, 2pi)."""

    def __init__(self, seed: int, nmodes: int = 16, kmax: int = 8, dim: int = 2):
        rng = np.random.default_rng(seed)
        if dim == 2:
            cand = [(i, j) for i in range(-kmax, kmax + 1) for j in range(-kmax, kmax + 1)
                    if 1 <= math.hypot(i, j) <= kmax]
        else:
            cand = [(i, 0) for i in range(-kmax, kmax + 1) if 1 <= abs(i) <= kmax]
        idx = rng.integers(0, len(cand), size=nmodes)
        self.k = np.array([cand[i] for i in idx], dtype=np.float64)
        kn = np.hypot(self.k[:, 0], self.k[:, 1])
        self.a = rng.standard_normal(nmodes) / kn ** 2
        self.phi = rng.uniform(0.0, 2 * np.pi, size=nmodes)
        self.dim = dim

    def __call__(self, x, y=None):
        o = _Ops(x)
        m = o.m
        y = m.zeros_like(x) if y is None else y
        out = m.zeros_like(x)
        for kx, ky, a, ph in zip(self.k[:, 0], self.k[:, 1], self.a, self.phi):
            out = out + a * m.cos(2 * np.pi * (kx * x + ky * y) + ph)
        return out

    def bound(self) -> float:
        return float(np.abs(self.a).sum())

    def shock_time(self, n: int = 1024) -> float:
        """t_c = 1 / max(-(d/dx + d/dy) u0) for u_t + (u^2/2)_x + (u^2/2)_y = 0,
        evaluated on an n x n sample."""
        g = (np.arange(n) + 0.5) / n
        X, Y = np.meshgrid(g, g, indexing="xy")
        arg = 2 * np.pi * (X[..., None] * self.k[:, 0] + Y[..., None] * self.k[:, 1]) + self.phi
        ksum = self.k[:, 0] + (self.k[:, 1] if self.dim == 2 else 0.0)
        du = (-self.a * 2 * np.pi * ksum * np.sin(arg)).sum(-1)
        return 1.0 / float(np.max(-du))


class ShockedFourier:
    """The Fourier data of FourierModes plus seeded jumps: four periodic
    square waves sq(n_m . x - c_m) (1 on the first half of each period, 0 on
    the second), n_m integer vectors with 1 <= |n_m|_inf <= 3, c_m ~ U[0, 1),
    heights ~ U[-1, 1] times the Fourier bound.  A periodic state with
    discontinuities along straight lines in several directions: where the
    state drops along (1, 1) they are shocks of the 2D Burgers flux, where it
    rises rarefactions, so a few steps from it have the structure of a state
    past the shock time."""

    def __init__(self, seed: int, njumps: int = 4):
        self.fm = FourierModes(seed)
        rng = np.random.default_rng(seed + 7919)
        self.n = []
        while len(self.n) < njumps:
            v = rng.integers(-3, 4, size=2)
            if v.any():
                self.n.append(v.astype(np.float64))
        self.c = rng.uniform(0.0, 1.0, size=njumps)
        self.h = rng.uniform(-1.0, 1.0, size=njumps) * self.fm.bound()

    def __call__(self, x, y):
        o = _Ops(x)
        u = self.fm(x, y)
        for (nx, ny), c, h in zip(self.n, self.c, self.h):
            s = nx * x + ny * y - c
            u = u + h * o.fl((s - o.m.floor(s)) < 0.5)
        return u

    def bound(self) -> float:
        return self.fm.bound() + float(np.abs(self.h).sum())


# ---------------------------------------------------------------------------
# the benchmark workloads
# ---------------------------------------------------------------------------
def adv1d(nx: int = 64, p: int = 2, mode: int = MODE_WENO, steps: int = 100,
          cfl: float = 0.1) -> Workload:
    """1D u_t + u_x = 0 on periodic [0,1], sin(2 pi x) + square pulse."""
    return Workload(name=f"adv1d_n{nx}_p{p}", dim=1, nx=nx, p=p, flux=LINADV, vx=1.0,
                    mode=mode, steps=steps, cfl=cfl, ic=sin_plus_pulse, umax=2.0)


def burgers1d(nx: int = 64, p: int = 2, mode: int = MODE_WENO, steps: int = 100,
              cfl: float = 0.1) -> Workload:
    """1D Burgers on periodic [0,1] with sin(2 pi x)."""
    return Workload(name=f"burgers1d_n{nx}_p{p}", dim=1, nx=nx, p=p, flux=BURGERS, vx=1.0,
                    mode=mode, steps=steps, cfl=cfl, ic=sin_wave, umax=1.0)


def rot2d(n: int = 256, p: int = 2, seed: int = 0, mode: int = MODE_WENO,
          steps: int = 200, cfl: float = 0.1, ny: Optional[int] = None) -> Workload:
    """Solid-body rotation v = (-(y-0.5), x-0.5) on [0,1] x [0, ny/n], zero
    inflow state on every boundary face, seeded hump + slotted cylinder."""
    ny = n if ny is None else ny
    return Workload(name=f"rot2d_{n}x{ny}_p{p}_s{seed}", dim=2, nx=n, ny=ny,
                    y1=ny / n, periodic_x=False, periodic_y=False, p=p, flux=LINADV,
                    vx=0.0, vy=0.0, omega=1.0, cx=0.5, cy=0.5, bc_value=0.0, mode=mode,
                    steps=steps, cfl=cfl, ic=HumpAndCylinder(seed), umax=1.0)


def leveque_rotation(x, y):
    """The three bodies of Sec. 5.3 (LeVeque's solid-body rotation): a smooth
    hump 1/4 + 1/4 cos(pi r / 0.15) about (0.25, 0.5), a cone 1 - r / 0.15
    about (0.5, 0.25), and a cylinder of height 1 about (0.5, 0.75) with a slot
    |x - 0.5| < 0.025 below y = 0.85; radius 0.15 each, 0 elsewhere."""
    o = _Ops(x)
    r_h = o.m.sqrt((x - 0.25) ** 2 + (y - 0.5) ** 2)
    r_c = o.m.sqrt((x - 0.5) ** 2 + (y - 0.25) ** 2)
    r_s = o.m.sqrt((x - 0.5) ** 2 + (y - 0.75) ** 2)
    hump = 0.25 + 0.25 * o.m.cos(np.pi * r_h / 0.15)
    cone = 1.0 - r_c / 0.15
    slot = (r_s <= 0.15) & ((o.m.abs(x - 0.5) >= 0.025) | (y >= 0.85))
    return o.where(r_h <= 0.15, hump, o.where(r_c <= 0.15, cone, o.fl(slot)))


def leveque2d(n: int = 128, p: int = 2, mode: int = MODE_WENO, steps: Optional[int] = None,
              cfl: float = 0.1, t_end: float = 1.0) -> Workload:
    """Sec. 5.3 as printed: v = 2 pi (0.5 - y, x - 0.5) on the unit square
    (one revolution per unit time), the three bodies of leveque_rotation,
    zero exterior state, n x n cells, run to t_end (the paper: 128^2, P2,
    t = 1)."""
    w = Workload(name=f"leveque2d_{n}_p{p}", dim=2, nx=n, ny=n, periodic_x=False, periodic_y=False,
                 p=p, flux=LINADV, vx=0.0, vy=0.0, omega=2.0 * np.pi, cx=0.5, cy=0.5, bc_value=0.0,
                 mode=mode, cfl=cfl, ic=leveque_rotation, umax=1.0)
    w.steps = steps if steps is not None else int(math.ceil(t_end / w.dt()))
    return w


def burgers2d(n: int = 1024, p: int = 2, seed: int = 0, mode: int = MODE_WENO,
              steps: Optional[int] = None, cfl: float = 0.1,
              t_end_factor: float = 1.5, ny: Optional[int] = None) -> Workload:
    """2D Burgers u_t + (u^2/2)_x + (u^2/2)_y = 0, periodic, seeded Fourier data.
    Without an explicit step count it runs to t_end_factor times the shock time."""
    ny = n if ny is None else ny
    fm = FourierModes(seed)
    w = Workload(name=f"burgers2d_{n}x{ny}_p{p}_s{seed}", dim=2, nx=n, ny=ny, y1=ny / n,
                 p=p, flux=BURGERS, vx=1.0, vy=1.0, mode=mode, cfl=cfl, ic=fm,
                 umax=fm.bound(), steps=1)
    if steps is None:
        w.t_end = t_end_factor * fm.shock_time()
        steps = int(math.ceil(w.t_end / w.dt()))
    w.steps = steps
    return w


def burgers2d_shocked(n: int = 1024, p: int = 2, seed: int = 0, mode: int = MODE_WENO,
                      steps: int = 100, cfl: float = 0.1) -> Workload:
    """2D Burgers as burgers2d, from the ShockedFourier state (the Fourier
    data with seeded jumps): a state with shocks at t = 0."""
    sf = ShockedFourier(seed)
    return Workload(name=f"burgers2d_shocked_{n}_p{p}_s{seed}", dim=2, nx=n, ny=n, p=p, flux=BURGERS,
                    vx=1.0, vy=1.0, mode=mode, cfl=cfl, ic=sf, umax=sf.bound(), steps=steps)


def batch_mix(seed: int = 0, count: int = 512, steps: int = 100) -> List[Workload]:
    """Independent problems: type uniform over {1D advection, 1D Burgers, 2D
    rotation}; 1D cells log-uniform in [64, 4096]; 2D side log-uniform in
    [32, 512]; degree uniform in 1..4."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = int(rng.integers(0, 3))
        p = int(rng.integers(1, 5))
        if kind < 2:
            n = int(round(math.exp(rng.uniform(math.log(64), math.log(4096)))))
            w = adv1d(n, p, steps=steps) if kind == 0 else burgers1d(n, p, steps=steps)
        else:
            n = int(round(math.exp(rng.uniform(math.log(32), math.log(512)))))
            w = rot2d(n, p, seed=seed * 100003 + i, steps=steps)
        w.name = f"b{i}_{w.name}"
        out.append(w)
    return out


def riemann_quadrants(x, y):
    """The four-quadrant data of Sec. 5.4 on the unit square: -0.2 (north-west),
    -1 (north-east), 0.5 (south-west), 0.8 (south-east)."""
    o = _Ops(x)
    north, east = y > 0.5, x > 0.5
    return o.where(north, o.where(east, -1.0, -0.2), o.where(east, 0.8, 0.5))


def sod_tube(x):
    """Sod's shock tube (Sec. 5.6) in conserved variables (rho, rho v, rho E),
    stacked on the axis before the last: (1, 0, 2.5) left of x = 1/2 (rho = 1,
    v = 0, p = 1), (0.125, 0, 0.25) right of it (rho = 0.125, v = 0, p = 0.1),
    gamma = 1.4."""
    o = _Ops(x)
    left = x < 0.5
    rho = o.where(left, 1.0, 0.125)
    m = o.where(left, 0.0, 0.0)
    E = o.where(left, 2.5, 0.25)
    return o.m.stack([rho, m, E], -2) if o.t else np.stack([rho, m, E], axis=-2)


def sod1d(n: int = 128, p: int = 2, mode: int = MODE_WENO, steps: Optional[int] = None,
          cfl: float = 0.1, t_end: float = 0.231) -> Workload:
    """Sod's shock tube of Sec. 5.6: the 1D Euler equations on (0, 1) between
    reflecting walls, n cells, run to t_end (the paper: 128 cells, P2,
    t = 0.231).  The step uses 2 as a bound on |v| + c over the run (the
    star region between the waves has |v| + c of about 1.93)."""
    w = Workload(name=f"sod1d_{n}_p{p}", dim=1, nx=n, periodic_x=False, p=p, flux=EULER,
                 vx=0.0, mode=mode, cfl=cfl, ic=sod_tube, umax=2.0)
    w.steps = steps if steps is not None else int(math.ceil(t_end / w.dt()))
    return w


def burgers2d_riemann(n: int = 128, p: int = 2, mode: int = MODE_WENO, steps: Optional[int] = None,
                      cfl: float = 0.1, t_end: float = 0.5) -> Workload:
    """The 2D Burgers problem of Sec. 5.4: u_t + div(v u^2/2) = 0, v = (1, 1),
    on the unit square with n x n cells, four-quadrant data, the exterior
    state on every boundary face from the exact solution in R^2, run to
    t_end (the paper: 128^2, P2, t = 0.5)."""
    w = Workload(name=f"burgers2d_riemann_{n}_p{p}", dim=2, nx=n, ny=n, periodic_x=False,
                 periodic_y=False, p=p, flux=BURGERS, vx=1.0, vy=1.0, bc_kind=BC_RIEMANN,
                 mode=mode, cfl=cfl, ic=riemann_quadrants, umax=1.0)
    w.steps = steps if steps is not None else int(math.ceil(t_end / w.dt()))
    return w


def kpp2d(n: int = 128, p: int = 2, mode: int = MODE_WENO, steps: Optional[int] = None,
          cfl: float = 0.1, lam: float = 2.0, t_end: float = 1.0) -> Workload:
    """The KPP problem of Sec. 5.5: u_t + div (sin u, cos u) = 0 on
    (-2, 2) x (-2.5, 1.5), n x n cells, lambda_e fixed at `lam` (the paper
    uses 2), the outer state pi/4 outside the mesh, run to t_end."""
    w = Workload(name=f"kpp2d_{n}_p{p}", dim=2, nx=n, ny=n, x0=-2.0, x1=2.0, y0=-2.5, y1=1.5,
                 periodic_x=False, periodic_y=False, p=p, flux=KPP, vx=0.0, vy=0.0,
                 bc_value=0.25 * np.pi, mode=mode, lambda_override=lam, cfl=cfl, ic=kpp_disc,
                 umax=3.5 * np.pi)
    w.steps = steps if steps is not None else int(math.ceil(t_end / w.dt()))
    return w
