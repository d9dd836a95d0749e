"""FP64 operation counts of the oracle's operator, per cell and RK stage.

TEST INFRASTRUCTURE, like the rest of this package.  Counts the floating-point
operations the PyTorch oracle (dgoracle.Oracle) executes in one evaluation of
the stabilised operator dU/dt = M^-1 (R(U) - s(U)) (Sec. 2, eq. (weak2); Sec. 3,
eq. (astab); Sec. 4, eq. (sensor)), i.e. in one RK stage, on a periodic mesh
(every cell has all its face neighbours), divided by the number of cells.  The
count is taken from the operations themselves (a PyTorch dispatch mode), not
estimated:

* matrix products: 2 M N K (a multiply and an add per term);
* elementwise arithmetic, comparisons, abs, sqrt, pow, sin, cos, maximum,
  minimum, clamp: one per output element;
* reductions (sum, amax, amin): one per input element;
* not counted: copies, gathers, concatenation, views, fills, selections
  (torch.where) and type conversions.

The oracle evaluates the operator plainly (dense matrix products over all
basis functions and quadrature nodes, no sum factorisation, the constant
coefficient of the candidates included), so these counts bound what the
method needs from above; the benchmark quotes them beside the HIP kernel's
own executed count.

    python -m oracle.opcount     # writes oracle/opcounts.json
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch
from torch.utils._python_dispatch import TorchDispatchMode

from .dgoracle import BURGERS, KPP, LINADV, MODE_DG, MODE_LO, MODE_WENO, MODE_ZHAO, Oracle, Problem

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "opcounts.json")

_ELEMENTWISE = {"add", "sub", "mul", "div", "neg", "abs", "sqrt", "pow", "sin", "cos", "maximum", "minimum",
                "clamp", "gt", "ge", "lt", "le", "eq", "ne", "floor", "ceil", "rsub", "reciprocal", "exp", "log"}
_REDUCE = {"sum", "amax", "amin", "max", "min"}
_MATMUL = {"mm", "bmm", "addmm", "matmul"}


class _Counter(TorchDispatchMode):
    def __init__(self):
        super().__init__()
        self.ops = 0
        self.by_op = {}

    def __torch_dispatch__(self, func, types, args=(), kwargs=None):
        out = func(*args, **(kwargs or {}))
        name = func.overloadpacket.__name__.rstrip("_")
        n = 0
        if name in _MATMUL:
            a, b = args[-2], args[-1]
            k = a.shape[-1]
            n = 2 * k * out.numel()
        elif name in _ELEMENTWISE and isinstance(out, torch.Tensor) and out.is_floating_point() or \
                name in ("gt", "ge", "lt", "le", "eq", "ne"):
            n = out.numel() if isinstance(out, torch.Tensor) else 0
        elif name in _REDUCE:
            n = args[0].numel()
        if n:
            self.ops += n
            self.by_op[name] = self.by_op.get(name, 0) + n
        return out


def count(dim: int, p: int, flux: int, mode: int) -> dict:
    """Operations per cell of one operator evaluation (one RK stage)."""
    n = 8 if dim == 2 else 32
    prob = Problem(dim=dim, nx=n, ny=n if dim == 2 else 1, p=p, flux=flux, mode=mode,
                   vx=1.0, vy=1.0 if flux == BURGERS else 0.0, omega=1.0 if (flux == LINADV and dim == 2) else 0.0,
                   periodic_x=True, periodic_y=True)
    if flux == LINADV and dim == 2:
        prob.vx = prob.vy = 0.0
    O = Oracle(prob)
    rng = np.random.default_rng(0)
    U = torch.from_numpy(rng.standard_normal((prob.ncells, prob.nloc)))
    c = _Counter()
    with c:
        O.rhs(U)
    per_cell = c.ops / prob.ncells
    return {"ops_per_cell": per_cell, "ops_per_dof": per_cell / prob.nloc, "nloc": prob.nloc,
            "by_op_per_cell": {k: v / prob.ncells for k, v in sorted(c.by_op.items())}}


def key(dim, p, flux, mode) -> str:
    return f"{dim},{p},{flux},{mode}"


def main():
    table = {}
    for dim in (1, 2):
        for p in (1, 2, 3, 4):
            for flux in ((LINADV, BURGERS) if dim == 1 else (LINADV, BURGERS, KPP)):
                for mode in (MODE_DG, MODE_LO, MODE_WENO, MODE_ZHAO):
                    table[key(dim, p, flux, mode)] = count(dim, p, flux, mode)
    doc = {"what": "FP64 operations the PyTorch oracle executes per cell in one operator evaluation "
                   "(one RK stage) on a periodic mesh; key = 'dim,p,flux,mode' with flux 0 linear "
                   "advection, 1 Burgers, 2 KPP and mode 0 DG, 1 LO, 2 WENO, 3 Zhao",
           "written_by": "python -m oracle.opcount", "counts": table}
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    return OUT


if __name__ == "__main__":
    print(main())
