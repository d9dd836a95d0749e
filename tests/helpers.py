"""Glue between the seeded workloads and the oracle (test-side only)."""
import numpy as np
import torch

import oracle
from paper_2309_12019_amd import inputs


def oracle_problem(w: inputs.Workload) -> oracle.Problem:
    f = w.fields()
    keep = {k: f[k] for k in oracle.Problem.__dataclass_fields__ if k in f}
    return oracle.Problem(**keep)


def oracle_for(w):
    return oracle.Oracle(oracle_problem(w))


def oracle_initial(w, O=None):
    """U^0 = L2 projection of the workload's initial data (oracle side)."""
    O = O or oracle_for(w)
    pts = O.proj_nodes().numpy()
    vals = torch.from_numpy(np.ascontiguousarray(w.eval_ic(pts)))
    return O.project(vals)


def oracle_window(w: inputs.Workload, ix: int, iy: int, radius: int):
    """An oracle on the window of cells within `radius` (max-norm) of cell
    (ix, iy): same flux, sensor and geometry (window origin at the window's
    first cell), never periodic; windows are clipped at non-periodic mesh
    boundaries, where the window's own boundary is then the mesh boundary.
    The operator at the window's centre depends only on the centre and its
    face neighbours, one SSP-RK3 step on cells within three face steps, so
    with radius 1 (operator) or 3 (step) the centre's value is the full
    mesh's.  Returns the oracle, the global cell index of every window cell
    (window order, x fastest) and the window index of the centre."""
    p = oracle_problem(w)
    h = p.h
    ny = w.ny if w.dim == 2 else 1

    def axis(i, n, per):
        if per:
            return [(i + d) % n for d in range(-radius, radius + 1)], radius
        lo, hi = max(0, i - radius), min(n - 1, i + radius)
        return list(range(lo, hi + 1)), i - lo

    xs, cx = axis(ix, w.nx, w.periodic_x)
    if w.dim == 2:
        ys, cy = axis(iy, ny, w.periodic_y)
    else:
        ys, cy = [0], 0
    # window geometry: the first window cell sits where its mesh cell sits
    # (periodic windows are unrolled from that cell on)
    x0 = w.x0 + (ix - cx) * h
    y0 = (w.y0 + (iy - cy) * h) if w.dim == 2 else p.y0
    p.nx = len(xs)
    p.x0, p.x1 = x0, x0 + len(xs) * h
    if w.dim == 2:
        p.ny = len(ys)
        p.y0, p.y1 = y0, y0 + len(ys) * h
    p.periodic_x = False
    p.periodic_y = False
    # a periodic axis keeps all face neighbours of the centre: the window
    # boundary is at least `radius` cells away from it
    cells = [yy * w.nx + xx for yy in ys for xx in xs]
    centre = cy * len(xs) + cx
    return oracle.Oracle(p), cells, centre


# Relative L-inf bar of 100-step parity runs (Sec. 2, eq. ssp, applied 100
# times).  Where the discrete map itself amplifies rounding beyond that (p = 4
# with the WENO sensor: c - c* cancels digits where the reconstruction nearly
# reproduces the data; long WENO runs over near-constant regions, where the
# sensor's ratio is a quotient of two rounding-level semi-norms; near
# discontinuities at p >= 3, where gamma_e of a nearly constant cell depends
# on a neighbour's highest mode through the continuation with gradients up to
# ~1e5), the bar is 10x the oracle's own spread under a one-ulp perturbation
# of its input (the larger of two perturbations) when that exceeds RUN_BAR,
# and never more than SPREAD_CAP.
RUN_BAR = 1e-11
SPREAD_CAP = 5e-8


def one_ulp_spread(run, U0, seeds=(0, 1), ref=None):
    """Spread of an oracle run against itself when its input is perturbed by
    about one unit in the last place (the larger over the seeded
    perturbations): run(U) -> U after the steps; ref = run(U0) if known."""
    b = run(U0) if ref is None else ref
    out = 0.0
    for seed in seeds:
        rng = np.random.default_rng(seed)
        U1 = U0 * (1 + 2.2e-16 * torch.from_numpy(rng.standard_normal(tuple(U0.shape))))
        out = max(out, float((run(U1) - b).abs().max() / b.abs().max()))
    return out


def run_bar(w, run, U0, measure=False, ref=None):
    """The bar for a multi-step comparison of workload w from U0 (and the
    measured spread, or None where the fixed bar applies).  The spread is
    measured for p = 4 WENO, and wherever a test asks for it; the caller
    asserts bar <= SPREAD_CAP after reporting."""
    if measure or (w.p == 4 and w.mode == inputs.MODE_WENO):
        spread = one_ulp_spread(run, U0, ref=ref)
        return max(RUN_BAR, 10 * spread), spread
    return RUN_BAR, None
