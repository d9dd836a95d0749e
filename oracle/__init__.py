"""CPU oracle (test infrastructure only; see dgoracle's module docstring)."""
from .dgoracle import (Problem, Oracle, Basis, gauss_legendre, legendre_poly,  # noqa: F401
                       tensor_rule, multi_indices, LINADV, BURGERS,
                       MODE_DG, MODE_LO, MODE_WENO)
