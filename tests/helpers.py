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
