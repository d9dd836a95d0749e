"""ctypes loader of the plain C oracle (oracle/dgoracle.c).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test suite, the
smoke check and the benchmark's CPU-baseline leg use it; the product never
does.  The C oracle computes what dgoracle.Oracle computes (same readings,
same layout U[cell][j]) with plain loops per cell, so that the largest
workloads can be followed whole for hundreds of steps.  It is pinned against
the PyTorch oracle and against the paper's invariants in
tests/test_oracle_c.py.

    python -m oracle.coracle     # build oracle/libdgoracle.so with gcc
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dgoracle.c")
LIB = os.path.join(HERE, "libdgoracle.so")
# x86-64-v3 (AVX2, FMA) runs on any host of this generation; the GPU hosts'
# CPUs are not this container's, so no -march=native
CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE"]


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("C oracle build failed:\n" + " ".join(cmd) + "\n" + p.stdout)
    os.replace(tmp, LIB)
    return LIB


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("per_x", ctypes.c_int), ("per_y", ctypes.c_int),
                ("p", ctypes.c_int), ("flux", ctypes.c_int),
                ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("omega", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("bc", ctypes.c_double),
                ("mode", ctypes.c_int), ("q", ctypes.c_double), ("b", ctypes.c_double),
                ("wnb", ctypes.c_double), ("eps", ctypes.c_double), ("r", ctypes.c_double),
                ("theta", ctypes.c_double), ("rk_order", ctypes.c_int),
                ("lam_over", ctypes.c_double), ("quad_vol", ctypes.c_int), ("quad_face", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()   # gcc is part of the image; the build takes seconds
        L = ctypes.CDLL(LIB)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(_Problem)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_rhs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]
        L.orc_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        L.orc_sizes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_int)]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


class COracle:
    """The C oracle for one problem (an oracle.Problem or any object with the
    same fields).  States are CPU float64 tensors [cells, nloc]."""

    def __init__(self, prob):
        if getattr(prob, "bc_kind", 0) != 0:
            raise ValueError("the C oracle has the constant exterior state only")
        P = _Problem(dim=prob.dim, nx=prob.nx, ny=prob.ny if prob.dim == 2 else 1,
                     x0=prob.x0, x1=prob.x1, y0=prob.y0, y1=prob.y1,
                     per_x=int(bool(prob.periodic_x)), per_y=int(bool(prob.periodic_y)),
                     p=prob.p, flux=prob.flux, vx=prob.vx, vy=prob.vy, omega=prob.omega,
                     cx=prob.cx, cy=prob.cy, bc=prob.bc_value, mode=prob.mode, q=prob.q, b=prob.b,
                     wnb=prob.w_nb, eps=prob.eps, r=prob.r, theta=prob.theta,
                     rk_order=prob.rk_order, lam_over=prob.lambda_override,
                     quad_vol=getattr(prob, "quad_vol", 0), quad_face=getattr(prob, "quad_face", 0))
        self._lib = lib()
        self._h = self._lib.orc_create(ctypes.byref(P))
        if not self._h:
            raise ValueError("the C oracle rejected the problem")
        n, nl = ctypes.c_long(), ctypes.c_int()
        self._lib.orc_sizes(self._h, ctypes.byref(n), ctypes.byref(nl))
        self.ncells, self.nloc = int(n.value), int(nl.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    def _state(self, U) -> torch.Tensor:
        U = torch.as_tensor(U, dtype=torch.float64)
        if U.device.type != "cpu" or tuple(U.shape) != (self.ncells, self.nloc):
            raise ValueError(f"state must be a CPU tensor [{self.ncells}, {self.nloc}]")
        return U.contiguous()

    def rhs(self, U, with_gamma: bool = False):
        """dU/dt = M^-1 (R(U) - s(U)) (and gamma_e)."""
        U = self._state(U)
        L = torch.empty_like(U)
        gam = torch.empty(self.ncells, dtype=torch.float64) if with_gamma else None
        self._lib.orc_rhs(self._h, U.data_ptr(), L.data_ptr(), gam.data_ptr() if with_gamma else None)
        return (L, gam) if with_gamma else L

    def step(self, U, dt: float) -> torch.Tensor:
        """One SSP Runge-Kutta step of the problem's order (a new tensor)."""
        out = self._state(U).clone()
        if self._lib.orc_step(self._h, out.data_ptr(), float(dt)):
            raise MemoryError("C oracle step")
        return out

    def run(self, U, dt: float, nsteps: int) -> torch.Tensor:
        out = self._state(U).clone()
        if self._lib.orc_run(self._h, out.data_ptr(), float(dt), int(nsteps)):
            raise MemoryError("C oracle run")
        return out


if __name__ == "__main__":
    print(build())
    sys.exit(0)
